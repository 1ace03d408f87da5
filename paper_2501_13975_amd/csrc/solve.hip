// solve.hip -- per-kernel local Newton solves and their application (Sec. 4.2).
//
// One thread per kernel reads its blocks (structure-of-arrays rows, coalesced)
// and solves, in the reduced coordinates of the primary camera:
//   position: Delta p = U Delta v, U an orthonormal basis of the plane normal to
//             the view direction r_k, (U^T H_p U) Delta v = -U^T g_p;
//   rotation: q(theta) = (cos(theta/2), sin(theta/2) r_k) q is the left rotation by
//             omega = theta r_k, so g_theta = r^T g_omega and H_theta = r^T H_omega r;
//   scaling:  Newton restricted to the row space of T = d lambda/d s (lambda the
//             eigenvalues of the primary 2D covariance), Delta s = T^T a;
//   opacity:  log barrier -alpha_s [ln sigma + ln(1 - sigma)];
//   colour:   per channel G = sum_v s_v Y(r_v) Y(r_v)^T, g = sum_v gamma_v Y(r_v).
// Every group is damped by the same rule: Cholesky of H + mu_j I,
// mu_j = mu0 10^j with mu0 = damp_rel |H|_F / sqrt(n) + damp_abs / (3 |I|), accepted
// when every pivot exceeds pivot_min (|H|_F / sqrt(n) + mu_j) and min/max pivot is at
// least pivot_min, else the
// scaled gradient step; the step is then clamped to the group's trust radius.
// The small systems are solved in double precision (the FP64 vector rate of
// gfx950 equals its unpacked FP32 rate, and this pass is bound by memory).  The colour system has rank at
// most V (number of views that see the kernel); when V < K it is solved in view
// space, (B B^T + mu S^-1) y = -S^-1 gamma, Delta = B^T y, which equals the
// damped K x K solve exactly and is far better conditioned.
#include <limits>
#include <mutex>

#include "gsn_internal.h"
#include "reduced.h"

namespace {

// Damped solve of a 1x1 or 2x2 symmetric system (H packed xx, xy, yy for n = 2) in precision T.
// *near (if given) is set when the accepted attempt passed its pivot tests by less than a factor
// of 10 or the gradient fallback was taken: the mixed form recomputes such systems in double.
template <class T>
__device__ int damped_small(int n, const T* H, const T* g, const gsn_solve_opts& o, T abs_scale, T* x,
                            bool* near = nullptr) {
    // scale of H: Frobenius norm / sqrt(n), invariant to the reduced basis
    const T ma = n == 1 ? fabs(H[0]) : sqrt(T(0.5) * (H[0] * H[0] + T(2) * H[1] * H[1] + H[2] * H[2]));
    T mu = (T)o.damp_rel * ma + (T)o.damp_abs * abs_scale;
    const T pmin = (T)o.pivot_min;
    for (int j = 0; j <= o.max_escalations; ++j) {
        // every pivot must exceed pivot_min times the size of H + mu I
        const T floor = pmin * (ma + mu);
        if (n == 1) {
            const T d = H[0] + mu;
            if (d > floor) {
                x[0] = -g[0] / d;
                if (near) *near = d < T(10) * floor;
                return j;
            }
        } else {
            const T a = H[0] + mu, b = H[1], c = H[2] + mu;
            if (a > floor) {
                const T l10 = b / a;
                const T d2 = c - l10 * b;
                if (d2 > floor && fmin(a, d2) >= pmin * fmax(a, d2)) {
                    // L D L^T with L = [[1, 0], [l10, 1]], D = diag(a, d2)
                    const T y0 = -g[0], y1 = -g[1] - l10 * y0;
                    x[1] = y1 / d2;
                    x[0] = (y0 - b * x[1]) / a;
                    if (near)
                        *near = fmin(a, d2) < T(10) * floor || fmin(a, d2) < T(10) * pmin * fmax(a, d2);
                    return j;
                }
            }
        }
        if (j < o.max_escalations) mu *= T(10);
    }
    const T den = ma + mu;
    for (int i = 0; i < n; ++i) x[i] = -g[i] / den;
    if (near) *near = true;
    return -1;
}

// Scales x onto the ball of the given radius when it lies outside; true when it did.
__device__ bool clamp_norm(int n, double* x, double radius) {
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += x[i] * x[i];
    nn = sqrt(nn);
    if (nn > radius && nn > 0.0) {
        for (int i = 0; i < n; ++i) x[i] *= radius / nn;
        return true;
    }
    return false;
}

// Events of one kernel's solve.  Bits 0-3: the system of position, rotation, scaling, opacity was
// accepted only after escalating the damping; bits 4-7: it fell back to the scaled gradient step;
// bits 8-11: the trust radius of position, rotation, scaling, colour (any channel) cut the step;
// bit 12: the kernel was solved; bit 13: a block or a step was not finite, so the kernel was
// skipped (zero step, decisions -3).  Bits 0-12 are counted while profiling (GSN_COUNT_SOLVE_*),
// bit 13 always (GSN_STAT_SKIPPED_NONFINITE).
constexpr int EV_ESC = 0, EV_FALLBACK = 4, EV_CLAMP = 8, EV_SOLVED = 12, EV_NONFINITE = 13;
constexpr int EV_PROFILED = GSN_SOLVE_EVENTS;  // bits counted while profiling
static_assert(GSN_COUNT_SOLVE_ESCALATED + GSN_SOLVE_EVENTS == GSN_COUNT_SOLVED + 1,
              "solve event bits 0-12 map onto the counters GSN_COUNT_SOLVE_ESCALATED .. GSN_COUNT_SOLVED");
__device__ __forceinline__ uint32_t decision_events(int group, int j) {
    return (j > 0 ? 1u << (EV_ESC + group) : 0u) | (j == -1 ? 1u << (EV_FALLBACK + group) : 0u);
}

// The overlap share of kernel k (with overlap_scale; else 1): omega = sum over its pixels in all
// views of (alpha T)^2 / sum of alpha T, clipped to [0, 1].  All kernels step at once, each step
// computed with the others fixed; where they overlap their steps add up in the shared pixels.
// omega <= H_kk / sum_j |H_kj| for the colour system (sum_j alpha_j T_j = 1 - T_final <= 1 at every
// pixel), a Gershgorin bound on that overshoot.  It multiplies the kernel's steps after the trust
// radii, so that overlapping kernels together move about as far as one kernel's radius allows.
// Vc: the view slots taken (the first Vc of the blocks' V), see view_slots.
template <class T, class RowFn>
__device__ __forceinline__ T overlap_share(RowFn B, int V, int Vc, const gsn_solve_opts& o) {
    if (!o.overlap_scale) return (T)1;
    T cov = (T)0;
    for (int v = 0; v < Vc; ++v) cov += (T)B(GSN_BLK_BASE + GSN_BLK_VIEW * v + 9);
    const T w2 = (T)B(GSN_BLK_BASE + GSN_BLK_VIEW * V);
    return cov > (T)0 ? fmin((T)1, fmax((T)0, w2 / cov)) : (T)0;
}

// The view slots a solve takes: all V of the blocks, or the first o.view_limit of them.
__host__ __device__ __forceinline__ int view_slots(int V, const gsn_solve_opts& o) {
    return o.view_limit > 0 && o.view_limit < V ? o.view_limit : V;
}

// Zero step and decisions -3 for a kernel skipped because of non-finite values.
__device__ __forceinline__ void skip_nonfinite(float* __restrict__ st, int32_t* __restrict__ fl, size_t N, int k,
                                               int NS) {
    for (int r = 0; r < NS; ++r) st[(size_t)r * N + k] = 0.f;
    for (int r = 0; r < 4; ++r) fl[(size_t)r * N + k] = -3;
    fl[4 * N + k] = 0;
}

// Adds a workgroup's solve events to the counters: the rare non-finite skips always, the others
// while profiling (per wave ballots summed in LDS, one atomic per counter and workgroup).
// Every thread of the workgroup calls it.
__device__ __forceinline__ void count_solve_events(uint32_t ev, unsigned long long* __restrict__ nonfinite,
                                                   unsigned long long* __restrict__ prof) {
    if ((ev >> EV_NONFINITE) & 1u) atomicAdd(nonfinite, 1ull);
    if (!prof) return;  // uniform across the launch
    __shared__ uint32_t cnt[EV_PROFILED];
    if (threadIdx.x < EV_PROFILED) cnt[threadIdx.x] = 0;
    __syncthreads();
#pragma unroll
    for (int b = 0; b < EV_PROFILED; ++b) {
        const uint64_t m = __ballot((ev >> b) & 1u);
        if (__lane_id() == 0 && m) atomicAdd(&cnt[b], (uint32_t)__popcll(m));
    }
    __syncthreads();
    // the workgroups add into GSN_SOLVE_SPREAD copies of the counters (summed by gsn_profile_read),
    // so that thousands of workgroups do not serialise on thirteen addresses
    unsigned long long* dst = prof + GSN_COUNT_N + (size_t)(blockIdx.x % GSN_SOLVE_SPREAD) * EV_PROFILED;
    if (threadIdx.x < EV_PROFILED && cnt[threadIdx.x])
        atomicAdd(&dst[threadIdx.x], (unsigned long long)cnt[threadIdx.x]);
}

// Cholesky solve of an m x m SPD system (m <= VM) held in a VM x VM register array (double).
// Loops run to the compile-time bound with guards, so the arrays stay in registers.
template <int VM, class T = double>
__device__ __forceinline__ bool chol_solve_v(int m, const T A[VM][VM], const T* b, T* x) {
    T L[VM][VM];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < VM; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            if (i < m) {
                T s = A[i][j];
#pragma unroll
                for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
                if (i == j) {
                    ok = ok && s > T(0);
                    L[i][i] = sqrt(fmax(s, std::numeric_limits<T>::min()));
                } else {
                    L[i][j] = s / L[j][j];
                }
            }
        }
    }
    T y[VM];
#pragma unroll
    for (int i = 0; i < VM; ++i) {
        if (i < m) {
            T s = b[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
            y[i] = s / L[i][i];
        }
    }
#pragma unroll
    for (int i = VM - 1; i >= 0; --i) {
        if (i < m) {
            T s = y[i];
#pragma unroll
            for (int k = i + 1; k < VM; ++k)
                if (k < m) s -= L[k][i] * x[k];
            x[i] = s / L[i][i];
        }
    }
    return ok;
}

// Colour step of one kernel, per channel, in view space (the system has rank at most the
// number of views nv that see the kernel):  with B the nv x K matrix of basis rows Y(r_v),
// S = diag(s_v) and gamma the per-view gradients, (B B^T + mu S^-1) y = -S^-1 gamma and
// Delta = B^T y, which equals the damped coefficient-space solve (B^T S B + mu I) Delta =
// -B^T gamma for every nv.  The basis rows are re-evaluated instead of stored.
template <int VM, class RowFn>
__device__ __forceinline__ bool colour_solve(int K, int V, RowFn B, const gsn_solve_opts& o, double frac,
                                             double omega, double abs_scale, float* __restrict__ st, size_t N,
                                             int k, int32_t* __restrict__ fl, double& chk) {
    int vb[VM];
    int nv = 0;
#pragma unroll
    for (int v = 0; v < VM; ++v) {
        vb[v] = 0;
        if (v < V && B(GSN_BLK_BASE + GSN_BLK_VIEW * v + 9) > 0.0) {
#pragma unroll
            for (int i = 0; i < VM; ++i)
                if (i == nv) vb[i] = GSN_BLK_BASE + GSN_BLK_VIEW * v;
            ++nv;
        }
    }
    fl[4 * N + k] = nv;
    // Gram matrix of the basis rows
    double Gm[VM][VM];
#pragma unroll
    for (int i = 0; i < VM; ++i)
#pragma unroll
        for (int j = 0; j < VM; ++j) Gm[i][j] = 0.0;
#pragma unroll
    for (int i = 0; i < VM; ++i) {
        if (i < nv) {
            double yi[16];
            sh_basis_dev<double>(K, B(vb[i] + 6), B(vb[i] + 7), B(vb[i] + 8), yi);
#pragma unroll
            for (int j = 0; j <= i; ++j) {
                if (j < nv) {
                    double d = 0.0;
                    sh_basis_visit<double>(K, B(vb[j] + 6), B(vb[j] + 7), B(vb[j] + 8),
                                           [&](int a, double yj) { d += yi[a] * yj; });
                    Gm[i][j] = d;
                    Gm[j][i] = d;
                }
            }
        }
    }
    double ych[3][VM];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
        for (int i = 0; i < VM; ++i) ych[ch][i] = 0.0;
        double smax = 0.0;
#pragma unroll
        for (int i = 0; i < VM; ++i)
            if (i < nv) smax = fmax(smax, fabs(B(vb[i] + 3 + ch)));
        if (!(smax > 0.0)) continue;
        double sv[VM], md = 0.0;  // md: mean diagonal of G = sum_v s_v Y Y^T
#pragma unroll
        for (int i = 0; i < VM; ++i) {
            sv[i] = 1.0;
            if (i < nv) {
                sv[i] = fmax(fabs(B(vb[i] + 3 + ch)), (double)o.sh_floor * smax);
                md += sv[i] * Gm[i][i];
            }
        }
        md /= (double)K;
        const double mu = (double)o.damp_sh * md + (double)o.damp_abs * abs_scale;
        double A[VM][VM], rhs[VM], y[VM];
#pragma unroll
        for (int i = 0; i < VM; ++i) {
#pragma unroll
            for (int j = 0; j < VM; ++j) A[i][j] = Gm[i][j] + (i == j ? mu / sv[i] : 0.0);
            rhs[i] = i < nv ? -B(vb[i] + ch) / sv[i] : 0.0;
        }
        if (chol_solve_v<VM, double>(nv, A, rhs, y)) {
#pragma unroll
            for (int i = 0; i < VM; ++i)
                if (i < nv) ych[ch][i] = y[i];
        }
    }
    // Delta_ch = B^T y_ch
    double dsh[3][16];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int a = 0; a < 16; ++a) dsh[ch][a] = 0.0;
#pragma unroll
    for (int i = 0; i < VM; ++i) {
        if (i < nv)
            sh_basis_visit<double>(K, B(vb[i] + 6), B(vb[i] + 7), B(vb[i] + 8), [&](int a, double ya) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dsh[ch][a] += ya * ych[ch][i];
            });
    }
    bool clamped = false;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        // trust radius on each channel's coefficient step
        double nn = 0.0;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            dsh[ch][a] *= frac;
            nn += dsh[ch][a] * dsh[ch][a];
        }
        nn = sqrt(nn);
        chk += nn * 0.0;
        const bool cut = nn > (double)o.trust_sh && nn > 0.0;
        clamped = clamped || cut;
        const double f = omega * (cut ? (double)o.trust_sh / nn : 1.0);
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a < K) st[(GSN_STEP_BASE + ch * K + a) * N + k] = (float)(dsh[ch][a] * f);
    }
    return clamped;
}

// The local solves of kernel k of one scene (all groups), writing its steps and decisions;
// returns the kernel's solve events (EV_*).
template <int VM>
__device__ __forceinline__ uint32_t solve_one(int k, const float* __restrict__ pos, const float* __restrict__ rot,
                                              const float* __restrict__ scale, const float* __restrict__ opac,
                                              int n, int K, const DevCam& c, float kappa,
                                              const float* __restrict__ blk, int V, const gsn_solve_opts& o,
                                              float* __restrict__ st, int32_t* __restrict__ fl) {
    const size_t N = (size_t)n;
    const int NS = GSN_STEP_BASE + 3 * K;
    if (!(blk[29 * N + k] > 0.f)) {
        for (int r = 0; r < NS; ++r) st[(size_t)r * N + k] = 0.f;
        for (int r = 0; r < 5; ++r) fl[(size_t)r * N + k] = -2;
        return 0u;
    }
    // chk stays 0 while every block entry the solve reads and every step component is finite
    // (x * 0 is NaN exactly for NaN and infinite x)
    double chk = 0.0;
    auto B = [&](int row) {
        const double v = (double)blk[(size_t)row * N + k];
        chk += v * 0.0;
        return v;
    };
    uint32_t ev = 1u << EV_SOLVED;
    const int Vc = view_slots(V, o);
    const double frac = (double)o.step_frac, omega = overlap_share<double>(B, V, Vc, o);
    const double abs_scale = 1.0 / (3.0 * (double)o.npix_primary);
    double s[3];
    for (int a = 0; a < 3; ++a) s[a] = scale[a * N + k];
    Reduced R;
    reduce_systems(pos, rot, scale, opac, n, k, c, kappa, B, o, abs_scale, R);
    for (int a = 0; a < 3; ++a) st[(4 + a) * N + k] = (float)R.r[a];
    // ---- position: Delta p = U Delta v
    {
        double dv[2];
        const int j = damped_small(2, R.Hp, R.gp, o, abs_scale, dv);
        fl[0 * N + k] = j;
        ev |= decision_events(0, j);
        for (int a = 0; a < 2; ++a) dv[a] *= frac;
        if (clamp_norm(2, dv, (double)o.trust_pos * fmax(s[0], fmax(s[1], s[2])))) ev |= 1u << (EV_CLAMP + 0);
        for (int a = 0; a < 3; ++a) {
            const double d = omega * (R.ux[a] * dv[0] + R.uy[a] * dv[1]);
            chk += d * 0.0;
            st[(size_t)a * N + k] = (float)d;
        }
    }
    // ---- rotation about r: omega = theta r
    {
        double th;
        const int j = damped_small(1, &R.Ht, &R.gt, o, abs_scale, &th);
        fl[1 * N + k] = j;
        ev |= decision_events(1, j);
        th *= frac;
        if (clamp_norm(1, &th, (double)o.trust_rot)) ev |= 1u << (EV_CLAMP + 1);
        chk += th * 0.0;
        st[3 * N + k] = (float)(omega * th);
    }
    // ---- scaling in the row space of d lambda / d s: Delta s = T^T a
    {
        double av[2];
        const int j = damped_small(2, R.Hs, R.gs, o, abs_scale, av);
        fl[2 * N + k] = j;
        ev |= decision_events(2, j);
        for (int a = 0; a < 2; ++a) av[a] *= frac;
        double dsv[3];
        for (int a = 0; a < 3; ++a) dsv[a] = R.T_[0][a] * av[0] + R.T_[1][a] * av[1];
        if (clamp_norm(3, dsv, (double)o.trust_scale * sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])))
            ev |= 1u << (EV_CLAMP + 2);
        for (int a = 0; a < 3; ++a) {
            chk += dsv[a] * 0.0;
            st[(7 + a) * N + k] = (float)(omega * dsv[a]);
        }
    }
    // ---- opacity with the log barrier
    {
        double ds;
        const int j = damped_small(1, &R.Ho, &R.go, o, abs_scale, &ds);
        fl[3 * N + k] = j;
        ev |= decision_events(3, j);
        chk += ds * 0.0;
        st[10 * N + k] = (float)(omega * (frac * ds));
    }
    // ---- colour, per channel
    if (colour_solve<VM>(K, Vc, B, o, frac, omega, abs_scale, st, N, k, fl, chk)) ev |= 1u << (EV_CLAMP + 3);
    if (!(chk == 0.0)) {
        skip_nonfinite(st, fl, N, k, NS);
        return 1u << EV_NONFINITE;
    }
    return ev;
}

// ---------------------------------------------------------------------------
// Mixed-precision form.  The colour Gram matrices B B^T (B: the basis rows Y(r_v) of the
// views that see a kernel) come from BF16 matrix-core products with FP32 accumulation: with
// Y = Y_hi + Y_lo (both BF16), G = Y_hi Y_hi^T + Y_hi Y_lo^T + Y_lo Y_hi^T, one correction
// of the BF16 rounding.  The reduced systems and all solves run in FP32; a position or
// rotation system whose pivots pass their tests by less than a factor of 10 (or that falls
// back to the gradient step) is solved again in FP64.
// ---------------------------------------------------------------------------
typedef short bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ short to_bf16(float x) {
    // round to nearest even (finite inputs)
    const uint32_t u = __float_as_uint(x);
    return (short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float from_bf16(short h) { return __uint_as_float(((uint32_t)(uint16_t)h) << 16); }

// Compacted list of the views that see kernel k (coverage > 0), at most 4.
__device__ __forceinline__ int active_views(const float* __restrict__ blk, size_t N, int k, int V, int vb[4]) {
    int nv = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        vb[v] = 0;
        if (v < V && blk[(size_t)(GSN_BLK_BASE + GSN_BLK_VIEW * v + 9) * N + k] > 0.f) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i == nv) vb[i] = GSN_BLK_BASE + GSN_BLK_VIEW * v;
            ++nv;
        }
    }
    return nv;
}

// One wave per 16 kernels, four 16x16x16 BF16 products per group of 4 kernels: row
// i = 4 q + v of the operand is the basis row of view v of kernel q, so the 4 x 4 diagonal
// blocks of Y Y^T are the kernels' Gram matrices.  With the operand layout of the instruction
// (lane l holds row l % 16, columns 4 (l / 16) .. + 3; the result lane l holds column l % 16,
// rows 4 (l / 16) .. + 3) the B operand of Y^T is the lane's own A operand.  The upper
// triangle of each Gram matrix is written to gram [10][n].
__global__ __launch_bounds__(256) void sh_gram_kernel(const float* __restrict__ blk, int n, int K, int V,
                                                       float* __restrict__ gram) {
    const int lane = __lane_id();
    const int wave = (int)(blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64);
    const size_t N = (size_t)n;
    const int row = lane % 16, q = row / 4, v = row % 4, c0 = 4 * (lane / 16);
#pragma unroll
    for (int grp = 0; grp < 4; ++grp) {
        const int base = wave * 16 + grp * 4;
        if (base >= n) break;  // uniform across the wave
        const int k = base + q;
        float y[4] = {0.f, 0.f, 0.f, 0.f};
        if (k < n) {
            int vb[4];
            const int nv = active_views(blk, N, k, V, vb);
            if (v < nv) {
                const float rx = blk[(size_t)(vb[v] + 6) * N + k], ry = blk[(size_t)(vb[v] + 7) * N + k],
                            rz = blk[(size_t)(vb[v] + 8) * N + k];
                sh_basis_visit<float>(K, rx, ry, rz, [&](int a, float ya) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        if (a == c0 + t) y[t] = ya;
                });
            }
        }
        bf16x4 hi, lo;
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            hi[t] = to_bf16(y[t]);
            lo[t] = to_bf16(y[t] - from_bf16(hi[t]));
        }
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hi, hi, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(hi, lo, acc, 0, 0, 0);
        acc = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(lo, hi, acc, 0, 0, 0);
        // result lane l holds column j = l % 16, rows 4 (l / 16) + r: a diagonal block when l / 16 == j / 4
        const int j = lane % 16, qr = lane / 16;
        const int kk = base + qr;
        if (qr == j / 4 && kk < n) {
            const int cj = j % 4;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                if (r <= cj) gram[(size_t)(r * 4 - (r * (r - 1)) / 2 + (cj - r)) * N + kk] = acc[r];
        }
    }
}

// Colour step of the mixed form (FP32), from the matrix-core Gram matrices.
template <class RowFn>
__device__ __forceinline__ bool colour_solve_mixed(int K, int V, RowFn B, const float* __restrict__ gram,
                                                   const gsn_solve_opts& o, float frac, float omega, float abs_scale,
                                                   float* __restrict__ st, size_t N, int k,
                                                   int32_t* __restrict__ fl, const float* __restrict__ blk,
                                                   float& chk) {
    int vb[4];
    const int nv = active_views(blk, N, k, V, vb);
    fl[4 * N + k] = nv;
    float Gm[4][4];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i; j < 4; ++j) {
            const float g = gram[(size_t)(i * 4 - (i * (i - 1)) / 2 + (j - i)) * N + k];
            Gm[i][j] = g;
            Gm[j][i] = g;
        }
    float ych[3][4];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
        for (int i = 0; i < 4; ++i) ych[ch][i] = 0.f;
        float smax = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
            if (i < nv) smax = fmaxf(smax, fabsf((float)B(vb[i] + 3 + ch)));
        if (!(smax > 0.f)) continue;
        float sv[4], md = 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            sv[i] = 1.f;
            if (i < nv) {
                sv[i] = fmaxf(fabsf((float)B(vb[i] + 3 + ch)), o.sh_floor * smax);
                md += sv[i] * Gm[i][i];
            }
        }
        md /= (float)K;
        const float mu = o.damp_sh * md + o.damp_abs * abs_scale;
        float A[4][4], rhs[4], y[4];
#pragma unroll
        for (int i = 0; i < 4; ++i) {
#pragma unroll
            for (int j = 0; j < 4; ++j) A[i][j] = Gm[i][j] + (i == j ? mu / sv[i] : 0.f);
            rhs[i] = i < nv ? -(float)B(vb[i] + ch) / sv[i] : 0.f;
        }
        if (chol_solve_v<4, float>(nv, A, rhs, y)) {
#pragma unroll
            for (int i = 0; i < 4; ++i)
                if (i < nv) ych[ch][i] = y[i];
        }
    }
    float dsh[3][16];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int a = 0; a < 16; ++a) dsh[ch][a] = 0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        if (i < nv)
            sh_basis_visit<float>(K, (float)B(vb[i] + 6), (float)B(vb[i] + 7), (float)B(vb[i] + 8), [&](int a, float ya) {
#pragma unroll
                for (int ch = 0; ch < 3; ++ch) dsh[ch][a] += ya * ych[ch][i];
            });
    }
    bool clamped = false;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        float nn = 0.f;
#pragma unroll
        for (int a = 0; a < 16; ++a) {
            dsh[ch][a] *= frac;
            nn += dsh[ch][a] * dsh[ch][a];
        }
        nn = sqrtf(nn);
        chk += nn * 0.f;
        const bool cut = nn > o.trust_sh && nn > 0.f;
        clamped = clamped || cut;
        const float f = omega * (cut ? o.trust_sh / nn : 1.f);
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a < K) st[(GSN_STEP_BASE + ch * K + a) * N + k] = dsh[ch][a] * f;
    }
    return clamped;
}

__device__ bool clamp_norm_f(int n, float* x, float radius) {
    float nn = 0.f;
    for (int i = 0; i < n; ++i) nn += x[i] * x[i];
    nn = sqrtf(nn);
    if (nn > radius && nn > 0.f) {
        for (int i = 0; i < n; ++i) x[i] *= radius / nn;
        return true;
    }
    return false;
}

// The local solves of kernel k in the mixed form; returns the kernel's solve events (EV_*).
__device__ __forceinline__ uint32_t solve_one_mixed(int k, const float* __restrict__ pos,
                                                    const float* __restrict__ rot, const float* __restrict__ scale,
                                                    const float* __restrict__ opac, int n, int K, const DevCam& c,
                                                    float kappa, const float* __restrict__ blk, int V,
                                                    const gsn_solve_opts& o, const float* __restrict__ gram,
                                                    float* __restrict__ st, int32_t* __restrict__ fl,
                                                    unsigned long long* __restrict__ n_fp64) {
    const size_t N = (size_t)n;
    const int NS = GSN_STEP_BASE + 3 * K;
    if (!(blk[29 * N + k] > 0.f)) {
        for (int r = 0; r < NS; ++r) st[(size_t)r * N + k] = 0.f;
        for (int r = 0; r < 5; ++r) fl[(size_t)r * N + k] = -2;
        return 0u;
    }
    // chk stays 0 while every block entry the solve reads and every step component is finite
    float chk = 0.f;
    auto Bf = [&](int row) {
        const float v = blk[(size_t)row * N + k];
        chk += v * 0.f;
        return v;
    };
    uint32_t ev = 1u << EV_SOLVED;
    const int Vc = view_slots(V, o);
    const float frac = o.step_frac, omega = overlap_share<float>(Bf, V, Vc, o);
    const float abs_scale = 1.0f / (3.0f * (float)o.npix_primary);
    float s[3];
    for (int a = 0; a < 3; ++a) s[a] = scale[a * N + k];
    ReducedT<float> R;
    reduce_systems(pos, rot, scale, opac, n, k, c, kappa, Bf, o, abs_scale, R);
    for (int a = 0; a < 3; ++a) st[(4 + a) * N + k] = R.r[a];
    bool redo_p = false, redo_r = false;
    // ---- position, rotation: FP32, and FP64 where the pivots flag ill-conditioning
    float dv[2], th;
    int jp = damped_small(2, R.Hp, R.gp, o, abs_scale, dv, &redo_p);
    int jr = damped_small(1, &R.Ht, &R.gt, o, abs_scale, &th, &redo_r);
    if (redo_p || redo_r) {
        auto Bd = [&](int row) { return (double)blk[(size_t)row * N + k]; };
        Reduced Rd;
        const double abs_d = 1.0 / (3.0 * (double)o.npix_primary);
        reduce_systems(pos, rot, scale, opac, n, k, c, kappa, Bd, o, abs_d, Rd);
        if (redo_p) {
            double d[2];
            jp = damped_small(2, Rd.Hp, Rd.gp, o, abs_d, d);
            dv[0] = (float)d[0];
            dv[1] = (float)d[1];
            for (int a = 0; a < 3; ++a) {
                R.ux[a] = (float)Rd.ux[a];
                R.uy[a] = (float)Rd.uy[a];
            }
        }
        if (redo_r) {
            double d;
            jr = damped_small(1, &Rd.Ht, &Rd.gt, o, abs_d, &d);
            th = (float)d;
        }
        if (n_fp64) atomicAdd(n_fp64, 1ull);
    }
    fl[0 * N + k] = jp;
    ev |= decision_events(0, jp);
    for (int a = 0; a < 2; ++a) dv[a] *= frac;
    if (clamp_norm_f(2, dv, o.trust_pos * fmaxf(s[0], fmaxf(s[1], s[2])))) ev |= 1u << (EV_CLAMP + 0);
    for (int a = 0; a < 3; ++a) {
        const float d = omega * (R.ux[a] * dv[0] + R.uy[a] * dv[1]);
        chk += d * 0.f;
        st[(size_t)a * N + k] = d;
    }
    fl[1 * N + k] = jr;
    ev |= decision_events(1, jr);
    th *= frac;
    if (clamp_norm_f(1, &th, o.trust_rot)) ev |= 1u << (EV_CLAMP + 1);
    chk += th * 0.f;
    st[3 * N + k] = omega * th;
    // ---- scaling and opacity in FP32
    {
        float av[2];
        const int j = damped_small(2, R.Hs, R.gs, o, abs_scale, av);
        fl[2 * N + k] = j;
        ev |= decision_events(2, j);
        for (int a = 0; a < 2; ++a) av[a] *= frac;
        float dsv[3];
        for (int a = 0; a < 3; ++a) dsv[a] = R.T_[0][a] * av[0] + R.T_[1][a] * av[1];
        if (clamp_norm_f(3, dsv, o.trust_scale * sqrtf(s[0] * s[0] + s[1] * s[1] + s[2] * s[2])))
            ev |= 1u << (EV_CLAMP + 2);
        for (int a = 0; a < 3; ++a) {
            chk += dsv[a] * 0.f;
            st[(7 + a) * N + k] = omega * dsv[a];
        }
    }
    {
        float ds;
        const int j = damped_small(1, &R.Ho, &R.go, o, abs_scale, &ds);
        fl[3 * N + k] = j;
        ev |= decision_events(3, j);
        chk += ds * 0.f;
        st[10 * N + k] = omega * (frac * ds);
    }
    if (colour_solve_mixed(K, Vc, Bf, gram, o, frac, omega, abs_scale, st, N, k, fl, blk, chk))
        ev |= 1u << (EV_CLAMP + 3);
    if (!(chk == 0.f)) {
        skip_nonfinite(st, fl, N, k, NS);
        return 1u << EV_NONFINITE;
    }
    return ev;
}

// The update of kernel k (kernels the solve skipped, decisions -2 or -3, are not passed here).
__device__ __forceinline__ void apply_one(float* __restrict__ pos, float* __restrict__ rot, float* __restrict__ scale,
                                          float* __restrict__ opac, float* __restrict__ sh, int n, int K,
                                          const float* __restrict__ st, const float* __restrict__ gscale,
                                          const gsn_solve_opts& o, uint32_t mask, int k, bool& bound) {
    const size_t N = (size_t)n;
    float a[5] = {1.f, 1.f, 1.f, 1.f, 1.f};
    if (gscale)
        for (int i = 0; i < 5; ++i) a[i] = gscale[i * N + k];
    if (mask & 1u)
        for (int c = 0; c < 3; ++c) pos[c * N + k] += a[0] * st[c * N + k];
    if (mask & 2u) {
        const float th = a[1] * st[3 * N + k];
        const float sh2 = sinf(0.5f * th);
        const float dq[4] = {cosf(0.5f * th), sh2 * st[4 * N + k], sh2 * st[5 * N + k], sh2 * st[6 * N + k]};
        float q[4], r[4];
        for (int c = 0; c < 4; ++c) q[c] = rot[c * N + k];
        qmul<float>(dq, q, r);
        const float il = 1.0f / sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        for (int c = 0; c < 4; ++c) rot[c * N + k] = r[c] * il;
    }
    if (mask & 4u)
        for (int c = 0; c < 3; ++c) {
            const float s = scale[c * N + k];
            scale[c * N + k] = fmaxf(s + a[2] * st[(7 + c) * N + k], o.scale_floor * s);
        }
    if (mask & 8u) {
        const float sg = opac[k];
        const float want = sg + a[3] * st[10 * N + k];
        const float moved = fminf(fmaxf(want, sg - o.opac_ftb * sg), sg + o.opac_ftb * (1.0f - sg));
        const float put = fminf(fmaxf(moved, o.opac_eps), 1.0f - o.opac_eps);
        bound = put != want;
        opac[k] = put;
    }
    if (mask & 16u) {
        // every coefficient's step and value loaded before any is stored (constant indices: the loads
        // are in flight together, which matters inside the solve's low-occupancy launch)
        constexpr int kMaxC = 48;  // 3 channels x 16 coefficients at degree 3
        float dv[kMaxC], sv[kMaxC];
#pragma unroll
        for (int i = 0; i < kMaxC; ++i)
            if (i < 3 * K) {
                dv[i] = st[(GSN_STEP_BASE + i) * N + k];
                sv[i] = sh[i * N + k];
            }
#pragma unroll
        for (int i = 0; i < kMaxC; ++i)
            if (i < 3 * K) sh[i * N + k] = sv[i] + a[4] * dv[i];
    }
}

// A solve with its update fused (ap.mask != 0): the thread that solved kernel k applies the groups
// of ap.mask of its step at once (as apply_kernel with no scales), reading back its own step and
// decisions; the opacity bound is counted as apply_kernel counts it.
__device__ __forceinline__ void fused_apply(const ApplyTo& ap, int n, int K, const float* __restrict__ st,
                                            const int32_t* __restrict__ fl, const gsn_solve_opts& o, int k,
                                            unsigned long long* __restrict__ prof) {
    bool bound = false;
    if (k < n && fl[k] >= -1) apply_one(ap.pos, ap.rot, ap.scale, ap.opac, ap.sh, n, K, st, nullptr, o, ap.mask, k, bound);
    if (prof) {  // uniform across the launch
        const uint64_t m = __ballot(bound);
        if (__lane_id() == 0 && m) atomicAdd(&prof[GSN_COUNT_OPAC_BOUND], (unsigned long long)__popcll(m));
    }
}

// pos, rot, scale and opac are not restrict-qualified here: with a fused update the same arrays are
// written through ap.
__global__ __launch_bounds__(128) void solve_mixed_kernel(const float* pos, const float* rot, const float* scale,
                                                           const float* opac, int n, int K, DevCam c,
                                                           float kappa, const float* __restrict__ blk, int V,
                                                           gsn_solve_opts o, const float* __restrict__ gram,
                                                           float* __restrict__ st, int32_t* __restrict__ fl,
                                                           unsigned long long* __restrict__ n_fp64,
                                                           unsigned long long* __restrict__ nonfinite,
                                                           unsigned long long* __restrict__ prof, ApplyTo ap) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t ev = 0;
    if (k < n) ev = solve_one_mixed(k, pos, rot, scale, opac, n, K, c, kappa, blk, V, o, gram, st, fl, n_fp64);
    count_solve_events(ev, nonfinite, prof);
    if (ap.mask) fused_apply(ap, n, K, st, fl, o, k, prof);  // uniform across the launch
}

template <int VM>
__global__ __launch_bounds__(128, 3) void solve_kernel(const float* pos, const float* rot, const float* scale,
                                                     const float* opac, int n, int K, DevCam c, float kappa,
                                                     const float* __restrict__ blk, int V, gsn_solve_opts o,
                                                     float* __restrict__ st, int32_t* __restrict__ fl,
                                                     unsigned long long* __restrict__ nonfinite,
                                                     unsigned long long* __restrict__ prof, ApplyTo ap) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t ev = 0;
    if (k < n) ev = solve_one<VM>(k, pos, rot, scale, opac, n, K, c, kappa, blk, V, o, st, fl);
    count_solve_events(ev, nonfinite, prof);
    if (ap.mask) fused_apply(ap, n, K, st, fl, o, k, prof);  // uniform across the launch
}

// Several scenes in one persistent launch: the threads of a grid sized to the device walk
// the concatenated kernel index space (scene s owns [first[s], first[s + 1])) in strides;
// each kernel's solve is the per-scene solve, so the results are identical.
template <int VM, int BLOCK>
__global__ __launch_bounds__(BLOCK, 3) void solve_batched_kernel(const SolveScene* __restrict__ scenes, int count,
                                                               long long total,
                                                               unsigned long long* __restrict__ nonfinite) {
    __shared__ long long s_first[GSN_SOLVE_MAX_SCENES + 1];
    for (int i = threadIdx.x; i <= count; i += blockDim.x) s_first[i] = i < count ? scenes[i].first : total;
    __syncthreads();
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long gi = (long long)blockIdx.x * blockDim.x + threadIdx.x; gi < total; gi += stride) {
        int lo = 0, hi = count - 1;  // last scene whose first index <= gi
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_first[mid] <= gi) lo = mid; else hi = mid - 1;
        }
        const SolveScene& sc = scenes[lo];
        const uint32_t ev = solve_one<VM>((int)(gi - s_first[lo]), sc.pos, sc.rot, sc.scale, sc.opac, sc.n, sc.K,
                                          sc.cam, sc.kappa, sc.blk, sc.V, sc.o, sc.st, sc.fl);
        if ((ev >> EV_NONFINITE) & 1u) atomicAdd(nonfinite, 1ull);
    }
}

__global__ __launch_bounds__(256) void apply_kernel(float* __restrict__ pos, float* __restrict__ rot,
                                                     float* __restrict__ scale, float* __restrict__ opac,
                                                     float* __restrict__ sh, int n, int K,
                                                     const float* __restrict__ st, const int32_t* __restrict__ fl,
                                                     const float* __restrict__ gscale, gsn_solve_opts o,
                                                     uint32_t mask, unsigned long long* __restrict__ prof) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    bool bound = false;  // the opacity step was cut by the fraction-to-boundary rule or the bounds
    if (k < n && fl[k] >= -1) apply_one(pos, rot, scale, opac, sh, n, K, st, gscale, o, mask, k, bound);
    if (prof) {  // uniform across the launch
        const uint64_t m = __ballot(bound);
        if (__lane_id() == 0 && m) atomicAdd(&prof[GSN_COUNT_OPAC_BOUND], (unsigned long long)__popcll(m));
    }
}

}  // namespace

// Scratch of gsn_local_newton_solve_noalloc: the mixed form's colour Gram matrices, [10][n] for
// n <= GSN_NOALLOC_MAX_N, one copy per device, held from the library's load to the end of the
// process.  Host code never passes this name to a kernel (on the host it is only a stand-in for
// the symbol): it uses the per-device address that solve_scratch_address returns.
static __device__ __align__(256) float scratch[10 * (size_t)GSN_NOALLOC_MAX_N];

hipError_t solve_scratch_address(int device, float** out) {
    // looked up once per device, with that device current, and kept for the process
    static std::mutex mu;
    static float* addr[GSN_MAX_DEVICES] = {};
    *out = nullptr;
    if (device < 0 || device >= GSN_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[device]) {
        int cur = 0;
        hipError_t e = hipGetDevice(&cur);
        if (e != hipSuccess) return e;
        if ((e = hipSetDevice(device)) != hipSuccess) return e;
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        const hipError_t e2 = hipSetDevice(cur);
        if (e != hipSuccess) return e;
        if (e2 != hipSuccess) return e2;
        if (!p) return hipErrorInvalidSymbol;
        addr[device] = static_cast<float*>(p);
    }
    *out = addr[device];
    return hipSuccess;
}

void launch_solve(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                  const gsn_solve_opts& o, const gsn_steps& st, unsigned long long* nonfinite,
                  unsigned long long* prof, const ApplyTo& ap, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    // the hot path has a primary and up to three secondaries: a 4-view kernel keeps its arrays in registers
    if (b.n_views <= 4)
        solve_kernel<4><<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                          b.d_data, b.n_views, o, st.d_data, st.d_flags, nonfinite,
                                                          prof, ap);
    else
        solve_kernel<9><<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                          b.d_data, b.n_views, o, st.d_data, st.d_flags, nonfinite,
                                                          prof, ap);
}

template <int BLOCK>
static void launch_batched_block(const SolveScene* d_scenes, int count, long long total, int max_views, int grid,
                                 unsigned long long* nonfinite, hipStream_t s) {
    if (max_views <= 4)
        solve_batched_kernel<4, BLOCK><<<grid, BLOCK, 0, s>>>(d_scenes, count, total, nonfinite);
    else
        solve_batched_kernel<9, BLOCK><<<grid, BLOCK, 0, s>>>(d_scenes, count, total, nonfinite);
}

int solve_view_slots(int V, const gsn_solve_opts& o) { return view_slots(V, o); }

void launch_sh_gram(const float* blk, int n, int K, int V, float* gram, hipStream_t s) {
    if (n == 0) return;
    const int waves = (n + 15) / 16;
    sh_gram_kernel<<<(waves + 3) / 4, 256, 0, s>>>(blk, n, K, V, gram);
}

void launch_solve_mixed(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                        const gsn_solve_opts& o, const float* gram, const gsn_steps& st, unsigned long long* nonfinite,
                        unsigned long long* prof, const ApplyTo& ap, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    unsigned long long* n_fp64 = prof ? prof + GSN_COUNT_FP64_SOLVES : nullptr;
    solve_mixed_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                         b.d_data, b.n_views, o, gram, st.d_data, st.d_flags, n_fp64,
                                                         nonfinite, prof, ap);
}

void launch_solve_batched(const SolveScene* d_scenes, int count, long long total, int max_views, int block,
                          int grid, unsigned long long* nonfinite, hipStream_t s) {
    if (total == 0) return;
    if (block == 64)
        launch_batched_block<64>(d_scenes, count, total, max_views, grid, nonfinite, s);
    else if (block == 256)
        launch_batched_block<256>(d_scenes, count, total, max_views, grid, nonfinite, s);
    else
        launch_batched_block<128>(d_scenes, count, total, max_views, grid, nonfinite, s);
}

void launch_apply(const gsn_gaussians& g, const gsn_steps& st, const gsn_solve_opts& o, const float* scale,
                  uint32_t mask, unsigned long long* prof, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    apply_kernel<<<(g.n + 255) / 256, 256, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.d_sh, g.n, K,
                                                   st.d_data, st.d_flags, scale, o, mask, prof);
}
