// solve.hip -- per-kernel local Newton solves and their application (Sec. 4.2).
//
// One thread per kernel reads its blocks (structure-of-arrays rows, coalesced)
// and solves, in the reduced coordinates of the primary camera:
//   position: Delta p = U Delta v, U an orthonormal basis of the plane normal to
//             the view direction r_k, (U^T H_p U) Delta v = -U^T g_p;
//   rotation: q(theta) = (cos(theta/2), sin(theta/2) r_k) q, with
//             dq/dtheta = (0, r_k)/2 q and d2q/dtheta2 = -q/4 at theta = 0;
//   scaling:  Newton restricted to the row space of T = d lambda/d s (lambda the
//             eigenvalues of the primary 2D covariance), Delta s = T^T a;
//   opacity:  log barrier -alpha_s [ln sigma + ln(1 - sigma)];
//   colour:   per channel G = sum_v s_v Y(r_v) Y(r_v)^T, g = sum_v gamma_v Y(r_v).
// Every group is damped by the same rule: Cholesky of H + mu_j I,
// mu_j = mu0 10^j, accepted when all pivots are positive and min/max pivot is at
// least pivot_min, else the scaled gradient step.  The colour system has rank at
// most V (number of views that see the kernel); when V < K it is solved in view
// space, (B B^T + mu S^-1) y = -S^-1 gamma, Delta = B^T y, which equals the
// damped K x K solve exactly and is far better conditioned.
#include "gsn_internal.h"

namespace {

constexpr int VMAX = 9;

// Damped solve of a 1x1 or 2x2 symmetric system (H packed xx, xy, yy for n = 2).
__device__ int damped_small(int n, const float* H, const float* g, const gsn_solve_opts& o, float abs_scale,
                            float* x) {
    const float md = n == 1 ? H[0] : 0.5f * (H[0] + H[2]);
    const float ma = n == 1 ? fabsf(H[0]) : 0.5f * (fabsf(H[0]) + fabsf(H[2]));
    float mu = o.damp_rel * fmaxf(md, 0.f) + o.damp_abs * abs_scale;
    for (int j = 0; j <= o.max_escalations; ++j) {
        if (n == 1) {
            const float d = H[0] + mu;
            if (d > 0.f) {
                x[0] = -g[0] / d;
                return j;
            }
        } else {
            const float a = H[0] + mu, b = H[1], c = H[2] + mu;
            if (a > 0.f) {
                const float l10 = b / a;
                const float d2 = c - l10 * b;
                if (d2 > 0.f && fminf(a, d2) >= o.pivot_min * fmaxf(a, d2)) {
                    // forward/back substitution with L = [[1, 0], [l10, 1]], D = diag(a, d2)
                    const float y0 = -g[0], y1 = -g[1] - l10 * y0;
                    x[1] = y1 / d2;
                    x[0] = (y0 - b * x[1]) / a;
                    return j;
                }
            }
        }
        if (j < o.max_escalations) mu *= 10.f;
    }
    const float den = ma + mu;
    for (int i = 0; i < n; ++i) x[i] = -g[i] / den;
    return -1;
}

// Cholesky solve of an m x m SPD system held in a VMAX x VMAX register array.
__device__ bool chol_solve_v(int m, float A[VMAX][VMAX], const float* b, float* x) {
    float L[VMAX][VMAX];
#pragma unroll
    for (int i = 0; i < VMAX; ++i) {
        if (i >= m) break;
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            float s = A[i][j];
#pragma unroll
            for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
            if (i == j) {
                if (!(s > 0.f)) return false;
                L[i][i] = sqrtf(s);
            } else {
                L[i][j] = s / L[j][j];
            }
        }
    }
    float y[VMAX];
#pragma unroll
    for (int i = 0; i < VMAX; ++i) {
        if (i >= m) break;
        float s = b[i];
#pragma unroll
        for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
        y[i] = s / L[i][i];
    }
#pragma unroll
    for (int i = VMAX - 1; i >= 0; --i) {
        if (i >= m) continue;
        float s = y[i];
#pragma unroll
        for (int k = i + 1; k < VMAX; ++k)
            if (k < m) s -= L[k][i] * x[k];
        x[i] = s / L[i][i];
    }
    return true;
}

__device__ __forceinline__ void qmul(const float a[4], const float b[4], float r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    r[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}

__global__ __launch_bounds__(128) void solve_kernel(const float* __restrict__ pos, const float* __restrict__ rot,
                                                     const float* __restrict__ scale, const float* __restrict__ opac,
                                                     int n, int K, DevCam c, float kappa,
                                                     const float* __restrict__ blk, int V, gsn_solve_opts o,
                                                     float* __restrict__ st, int32_t* __restrict__ fl) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    const int NS = GSN_STEP_BASE + 3 * K;
    auto B = [&](int row) { return blk[(size_t)row * N + k]; };
    if (!(B(34) > 0.f)) {
        for (int r = 0; r < NS; ++r) st[(size_t)r * N + k] = 0.f;
        for (int r = 0; r < 4; ++r) fl[(size_t)r * N + k] = -2;
        fl[4 * N + k] = -2;
        return;
    }
    const float abs_scale = 1.0f / (3.0f * (float)o.npix_primary);
    float p[3], q[4], s[3];
    for (int a = 0; a < 3; ++a) p[a] = pos[a * N + k];
    for (int a = 0; a < 4; ++a) q[a] = rot[a * N + k];
    for (int a = 0; a < 3; ++a) s[a] = scale[a * N + k];
    const float sig = opac[k];
    float r[3] = {p[0] - c.o[0], p[1] - c.o[1], p[2] - c.o[2]};
    {
        const float il = 1.0f / sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int a = 0; a < 3; ++a) r[a] *= il;
    }
    for (int a = 0; a < 3; ++a) st[(4 + a) * N + k] = r[a];
    // ---- position
    {
        float uy[3] = {-r[1] * r[0], 1.0f - r[1] * r[1], -r[1] * r[2]};
        float nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        if (nn < 1e-12f) {
            uy[0] = 1.0f - r[0] * r[0];
            uy[1] = -r[0] * r[1];
            uy[2] = -r[0] * r[2];
            nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        }
        const float inn = 1.0f / sqrtf(nn);
        for (int a = 0; a < 3; ++a) uy[a] *= inn;
        const float ux[3] = {r[1] * uy[2] - r[2] * uy[1], r[2] * uy[0] - r[0] * uy[2], r[0] * uy[1] - r[1] * uy[0]};
        const float Hp[3][3] = {{B(3), B(4), B(5)}, {B(4), B(6), B(7)}, {B(5), B(7), B(8)}};
        const float gp[3] = {B(0), B(1), B(2)};
        const float* U[2] = {ux, uy};
        float H2[3], g2[2], dv[2];
        for (int i = 0; i < 2; ++i) {
            g2[i] = U[i][0] * gp[0] + U[i][1] * gp[1] + U[i][2] * gp[2];
        }
        float HU[3][2];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 2; ++j) HU[a][j] = Hp[a][0] * U[j][0] + Hp[a][1] * U[j][1] + Hp[a][2] * U[j][2];
        H2[0] = ux[0] * HU[0][0] + ux[1] * HU[1][0] + ux[2] * HU[2][0];
        H2[1] = ux[0] * HU[0][1] + ux[1] * HU[1][1] + ux[2] * HU[2][1];
        H2[2] = uy[0] * HU[0][1] + uy[1] * HU[1][1] + uy[2] * HU[2][1];
        fl[0 * N + k] = damped_small(2, H2, g2, o, abs_scale, dv);
        for (int a = 0; a < 3; ++a) st[(size_t)a * N + k] = ux[a] * dv[0] + uy[a] * dv[1];
    }
    // ---- rotation about r
    {
        const float rq[4] = {0.f, 0.5f * r[0], 0.5f * r[1], 0.5f * r[2]};
        float t[4];
        qmul(rq, q, t);
        const float gq[4] = {B(9), B(10), B(11), B(12)};
        float Hq[4][4];
        int idx = 13;
        for (int a = 0; a < 4; ++a)
            for (int b = a; b < 4; ++b, ++idx) Hq[a][b] = Hq[b][a] = B(idx);
        float gt = 0.f, Ht = 0.f, gqq = 0.f;
        for (int a = 0; a < 4; ++a) {
            gt += gq[a] * t[a];
            gqq += gq[a] * q[a];
            for (int b = 0; b < 4; ++b) Ht += t[a] * Hq[a][b] * t[b];
        }
        Ht += -0.25f * gqq;
        float th;
        fl[1 * N + k] = damped_small(1, &Ht, &gt, o, abs_scale, &th);
        st[3 * N + k] = th;
    }
    // ---- scaling in the row space of d lambda / d s
    {
        float tf[3];
        for (int i = 0; i < 3; ++i) tf[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
        const float iz = 1.0f / tf[2];
        const float J00 = c.fx * iz, J02 = -c.fx * tf[0] * iz * iz, J11 = c.fy * iz, J12 = -c.fy * tf[1] * iz * iz;
        float M[2][3];
        for (int kk = 0; kk < 3; ++kk) {
            M[0][kk] = J00 * c.R[kk] + J02 * c.R[6 + kk];
            M[1][kk] = J11 * c.R[3 + kk] + J12 * c.R[6 + kk];
        }
        const float qn = 1.0f / sqrtf(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const float w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
        const float Rq[3][3] = {{1.f - 2.f * (y * y + z * z), 2.f * (x * y - w * z), 2.f * (x * z + w * y)},
                                {2.f * (x * y + w * z), 1.f - 2.f * (x * x + z * z), 2.f * (y * z - w * x)},
                                {2.f * (x * z - w * y), 2.f * (y * z + w * x), 1.f - 2.f * (x * x + y * y)}};
        float MR[2][3];
        for (int i = 0; i < 2; ++i)
            for (int a = 0; a < 3; ++a) MR[i][a] = M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a];
        float sxx = kappa, sxy = 0.f, syy = kappa;
        for (int a = 0; a < 3; ++a) {
            const float s2 = s[a] * s[a];
            sxx += MR[0][a] * MR[0][a] * s2;
            sxy += MR[0][a] * MR[1][a] * s2;
            syy += MR[1][a] * MR[1][a] * s2;
        }
        const float mid = 0.5f * (sxx + syy);
        const float rad = sqrtf(0.25f * (sxx - syy) * (sxx - syy) + sxy * sxy);
        const float l2 = mid + rad;
        float v2[2];
        if (sxx >= syy) {
            v2[0] = l2 - syy;
            v2[1] = sxy;
        } else {
            v2[0] = sxy;
            v2[1] = l2 - sxx;
        }
        float vn = sqrtf(v2[0] * v2[0] + v2[1] * v2[1]);
        if (vn == 0.f) {
            v2[0] = 1.f;
            v2[1] = 0.f;
            vn = 1.f;
        }
        v2[0] /= vn;
        v2[1] /= vn;
        const float v1[2] = {-v2[1], v2[0]};
        float Tm[2][3];
        for (int a = 0; a < 3; ++a) {
            const float e1 = v1[0] * MR[0][a] + v1[1] * MR[1][a];
            const float e2 = v2[0] * MR[0][a] + v2[1] * MR[1][a];
            Tm[0][a] = 2.f * s[a] * e1 * e1;
            Tm[1][a] = 2.f * s[a] * e2 * e2;
        }
        const float Hs[3][3] = {{B(26), B(27), B(28)}, {B(27), B(29), B(30)}, {B(28), B(30), B(31)}};
        const float gs[3] = {B(23), B(24), B(25)};
        float HT[3][2];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 2; ++j) HT[a][j] = Hs[a][0] * Tm[j][0] + Hs[a][1] * Tm[j][1] + Hs[a][2] * Tm[j][2];
        float H2[3], g2[2], av[2];
        for (int i = 0; i < 2; ++i) g2[i] = Tm[i][0] * gs[0] + Tm[i][1] * gs[1] + Tm[i][2] * gs[2];
        H2[0] = Tm[0][0] * HT[0][0] + Tm[0][1] * HT[1][0] + Tm[0][2] * HT[2][0];
        H2[1] = Tm[0][0] * HT[0][1] + Tm[0][1] * HT[1][1] + Tm[0][2] * HT[2][1];
        H2[2] = Tm[1][0] * HT[0][1] + Tm[1][1] * HT[1][1] + Tm[1][2] * HT[2][1];
        fl[2 * N + k] = damped_small(2, H2, g2, o, abs_scale, av);
        for (int a = 0; a < 3; ++a) st[(7 + a) * N + k] = Tm[0][a] * av[0] + Tm[1][a] * av[1];
    }
    // ---- opacity with the log barrier
    {
        const float as = o.barrier_beta * abs_scale;
        const float gB = as * (1.0f / (1.0f - sig) - 1.0f / sig);
        const float hB = as * (1.0f / (sig * sig) + 1.0f / ((1.0f - sig) * (1.0f - sig)));
        const float H1 = B(33) + hB, g1 = B(32) + gB;
        float ds;
        fl[3 * N + k] = damped_small(1, &H1, &g1, o, abs_scale, &ds);
        st[10 * N + k] = ds;
    }
    // ---- colour, per channel
    {
        int vidx[VMAX];
        int nv = 0;
        for (int v = 0; v < V && v < VMAX; ++v)
            if (B(GSN_BLK_BASE + GSN_BLK_VIEW * v + 9) > 0.f) vidx[nv++] = v;
        fl[4 * N + k] = nv;
        float Yv[VMAX][16];
        for (int i = 0; i < VMAX; ++i) {
            if (i >= nv) break;
            const int vb = GSN_BLK_BASE + GSN_BLK_VIEW * vidx[i];
            sh_basis_dev<float>(K, B(vb + 6), B(vb + 7), B(vb + 8), Yv[i]);
        }
        for (int ch = 0; ch < 3; ++ch) {
            float dsh[16];
            for (int i = 0; i < K; ++i) dsh[i] = 0.f;
            float smax = 0.f;
            for (int i = 0; i < nv; ++i) smax = fmaxf(smax, fabsf(B(GSN_BLK_BASE + GSN_BLK_VIEW * vidx[i] + 3 + ch)));
            if (smax > 0.f) {
                float sv[VMAX], gv[VMAX];
                float md = 0.f;  // mean diagonal of G = sum_v s_v Y Y^T
                for (int i = 0; i < VMAX; ++i) {
                    if (i >= nv) break;
                    const int vb = GSN_BLK_BASE + GSN_BLK_VIEW * vidx[i];
                    sv[i] = fmaxf(fabsf(B(vb + 3 + ch)), o.sh_floor * smax);
                    gv[i] = B(vb + ch);
                    float yy = 0.f;
                    for (int a = 0; a < K; ++a) yy += Yv[i][a] * Yv[i][a];
                    md += sv[i] * yy;
                }
                md /= (float)K;
                const float mu = o.damp_rel * md + o.damp_abs * abs_scale;
                float A[VMAX][VMAX], rhs[VMAX], y[VMAX];
                if (nv < K) {
                    // view space: (B B^T + mu S^-1) y = -S^-1 gamma, Delta = B^T y
                    for (int i = 0; i < VMAX; ++i) {
                        if (i >= nv) break;
                        for (int j = 0; j < VMAX; ++j) {
                            if (j >= nv) break;
                            float d = 0.f;
                            for (int a = 0; a < K; ++a) d += Yv[i][a] * Yv[j][a];
                            A[i][j] = d + (i == j ? mu / sv[i] : 0.f);
                        }
                        rhs[i] = -gv[i] / sv[i];
                    }
                    if (chol_solve_v(nv, A, rhs, y))
                        for (int a = 0; a < K; ++a) {
                            float acc = 0.f;
                            for (int i = 0; i < nv; ++i) acc += Yv[i][a] * y[i];
                            dsh[a] = acc;
                        }
                } else {
                    // coefficient space: (sum_v s_v Y Y^T + mu I) Delta = -sum_v gamma_v Y  (K <= nv <= VMAX)
                    for (int a = 0; a < VMAX; ++a) {
                        if (a >= K) break;
                        for (int b = 0; b < VMAX; ++b) {
                            if (b >= K) break;
                            float d = a == b ? mu : 0.f;
                            for (int i = 0; i < nv; ++i) d += sv[i] * Yv[i][a] * Yv[i][b];
                            A[a][b] = d;
                        }
                        float gg = 0.f;
                        for (int i = 0; i < nv; ++i) gg += gv[i] * Yv[i][a];
                        rhs[a] = -gg;
                    }
                    if (chol_solve_v(K, A, rhs, y))
                        for (int a = 0; a < K; ++a) dsh[a] = y[a];
                }
            }
            for (int a = 0; a < K; ++a) st[(GSN_STEP_BASE + ch * K + a) * N + k] = dsh[a];
        }
    }
}

__global__ __launch_bounds__(256) void apply_kernel(float* __restrict__ pos, float* __restrict__ rot,
                                                     float* __restrict__ scale, float* __restrict__ opac,
                                                     float* __restrict__ sh, int n, int K,
                                                     const float* __restrict__ st, const int32_t* __restrict__ fl,
                                                     gsn_solve_opts o, uint32_t mask) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    if (fl[k] == -2) return;
    if (mask & 1u)
        for (int a = 0; a < 3; ++a) pos[a * N + k] += st[a * N + k];
    if (mask & 2u) {
        const float th = st[3 * N + k];
        const float sh2 = sinf(0.5f * th);
        const float dq[4] = {cosf(0.5f * th), sh2 * st[4 * N + k], sh2 * st[5 * N + k], sh2 * st[6 * N + k]};
        float q[4], r[4];
        for (int a = 0; a < 4; ++a) q[a] = rot[a * N + k];
        qmul(dq, q, r);
        const float il = 1.0f / sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
        for (int a = 0; a < 4; ++a) rot[a * N + k] = r[a] * il;
    }
    if (mask & 4u)
        for (int a = 0; a < 3; ++a) {
            const float s = scale[a * N + k];
            scale[a * N + k] = fmaxf(s + st[(7 + a) * N + k], o.scale_floor * s);
        }
    if (mask & 8u) {
        const float sg = opac[k];
        opac[k] = fminf(fmaxf(sg + st[10 * N + k], sg - o.opac_ftb * sg), sg + o.opac_ftb * (1.0f - sg));
    }
    if (mask & 16u)
        for (int i = 0; i < 3 * K; ++i) sh[i * N + k] += st[(GSN_STEP_BASE + i) * N + k];
}

}  // namespace

void launch_solve(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                  const gsn_solve_opts& o, const gsn_steps& st, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    solve_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                   b.d_data, b.n_views, o, st.d_data, st.d_flags);
}

void launch_apply(const gsn_gaussians& g, const gsn_steps& st, const gsn_solve_opts& o, uint32_t mask,
                  hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    apply_kernel<<<(g.n + 255) / 256, 256, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.d_sh, g.n, K,
                                                   st.d_data, st.d_flags, o, mask);
}
