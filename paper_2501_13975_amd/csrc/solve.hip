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
#include "gsn_internal.h"

namespace {

// Damped solve of a 1x1 or 2x2 symmetric system (H packed xx, xy, yy for n = 2) in double.
__device__ int damped_small(int n, const double* H, const double* g, const gsn_solve_opts& o, double abs_scale,
                            double* x) {
    // scale of H: Frobenius norm / sqrt(n), invariant to the reduced basis
    const double ma = n == 1 ? fabs(H[0]) : sqrt(0.5 * (H[0] * H[0] + 2.0 * H[1] * H[1] + H[2] * H[2]));
    double mu = (double)o.damp_rel * ma + (double)o.damp_abs * abs_scale;
    for (int j = 0; j <= o.max_escalations; ++j) {
        // every pivot must exceed pivot_min times the size of H + mu I
        const double floor = (double)o.pivot_min * (ma + mu);
        if (n == 1) {
            const double d = H[0] + mu;
            if (d > floor) {
                x[0] = -g[0] / d;
                return j;
            }
        } else {
            const double a = H[0] + mu, b = H[1], c = H[2] + mu;
            if (a > floor) {
                const double l10 = b / a;
                const double d2 = c - l10 * b;
                if (d2 > floor && fmin(a, d2) >= (double)o.pivot_min * fmax(a, d2)) {
                    // L D L^T with L = [[1, 0], [l10, 1]], D = diag(a, d2)
                    const double y0 = -g[0], y1 = -g[1] - l10 * y0;
                    x[1] = y1 / d2;
                    x[0] = (y0 - b * x[1]) / a;
                    return j;
                }
            }
        }
        if (j < o.max_escalations) mu *= 10.0;
    }
    const double den = ma + mu;
    for (int i = 0; i < n; ++i) x[i] = -g[i] / den;
    return -1;
}

__device__ void clamp_norm(int n, double* x, double radius) {
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += x[i] * x[i];
    nn = sqrt(nn);
    if (nn > radius && nn > 0.0)
        for (int i = 0; i < n; ++i) x[i] *= radius / nn;
}

// Cholesky solve of an m x m SPD system (m <= VM) held in a VM x VM register array (double).
// Loops run to the compile-time bound with guards, so the arrays stay in registers.
template <int VM>
__device__ __forceinline__ bool chol_solve_v(int m, const double A[VM][VM], const double* b, double* x) {
    double L[VM][VM];
    bool ok = true;
#pragma unroll
    for (int i = 0; i < VM; ++i) {
#pragma unroll
        for (int j = 0; j <= i; ++j) {
            if (i < m) {
                double s = A[i][j];
#pragma unroll
                for (int k = 0; k < j; ++k) s -= L[i][k] * L[j][k];
                if (i == j) {
                    ok = ok && s > 0.0;
                    L[i][i] = sqrt(fmax(s, 1e-300));
                } else {
                    L[i][j] = s / L[j][j];
                }
            }
        }
    }
    double y[VM];
#pragma unroll
    for (int i = 0; i < VM; ++i) {
        if (i < m) {
            double s = b[i];
#pragma unroll
            for (int k = 0; k < i; ++k) s -= L[i][k] * y[k];
            y[i] = s / L[i][i];
        }
    }
#pragma unroll
    for (int i = VM - 1; i >= 0; --i) {
        if (i < m) {
            double s = y[i];
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
__device__ __forceinline__ void colour_solve(int K, int V, RowFn B, const gsn_solve_opts& o, double abs_scale,
                                             float* __restrict__ st, size_t N, int k, int32_t* __restrict__ fl) {
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
        const double mu = (double)o.damp_rel * md + (double)o.damp_abs * abs_scale;
        double A[VM][VM], rhs[VM], y[VM];
#pragma unroll
        for (int i = 0; i < VM; ++i) {
#pragma unroll
            for (int j = 0; j < VM; ++j) A[i][j] = Gm[i][j] + (i == j ? mu / sv[i] : 0.0);
            rhs[i] = i < nv ? -B(vb[i] + ch) / sv[i] : 0.0;
        }
        if (chol_solve_v<VM>(nv, A, rhs, y)) {
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
#pragma unroll
    for (int ch = 0; ch < 3; ++ch)
#pragma unroll
        for (int a = 0; a < 16; ++a)
            if (a < K) st[(GSN_STEP_BASE + ch * K + a) * N + k] = (float)dsh[ch][a];
}

template <class T>
__device__ __forceinline__ void qmul(const T a[4], const T b[4], T r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    r[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}

template <int VM>
__global__ __launch_bounds__(128) void solve_kernel(const float* __restrict__ pos, const float* __restrict__ rot,
                                                     const float* __restrict__ scale, const float* __restrict__ opac,
                                                     int n, int K, DevCam c, float kappa,
                                                     const float* __restrict__ blk, int V, gsn_solve_opts o,
                                                     float* __restrict__ st, int32_t* __restrict__ fl) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    const int NS = GSN_STEP_BASE + 3 * K;
    auto B = [&](int row) { return (double)blk[(size_t)row * N + k]; };
    if (!(B(29) > 0.0)) {
        for (int r = 0; r < NS; ++r) st[(size_t)r * N + k] = 0.f;
        for (int r = 0; r < 5; ++r) fl[(size_t)r * N + k] = -2;
        return;
    }
    const double abs_scale = 1.0 / (3.0 * (double)o.npix_primary);
    double p[3], q[4], s[3];
    for (int a = 0; a < 3; ++a) p[a] = pos[a * N + k];
    for (int a = 0; a < 4; ++a) q[a] = rot[a * N + k];
    for (int a = 0; a < 3; ++a) s[a] = scale[a * N + k];
    const double sig = opac[k];
    double r[3];
    {
        // camera centre -R^T t in double from the float camera
        double oc[3];
        for (int i = 0; i < 3; ++i)
            oc[i] = -((double)c.R[i] * c.t[0] + (double)c.R[3 + i] * c.t[1] + (double)c.R[6 + i] * c.t[2]);
        for (int a = 0; a < 3; ++a) r[a] = p[a] - oc[a];
        const double il = 1.0 / sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        for (int a = 0; a < 3; ++a) r[a] *= il;
    }
    for (int a = 0; a < 3; ++a) st[(4 + a) * N + k] = (float)r[a];
    // ---- position
    {
        double uy[3] = {-r[1] * r[0], 1.0 - r[1] * r[1], -r[1] * r[2]};
        double nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        if (nn < 1e-12) {
            uy[0] = 1.0 - r[0] * r[0];
            uy[1] = -r[0] * r[1];
            uy[2] = -r[0] * r[2];
            nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        }
        const double inn = 1.0 / sqrt(nn);
        for (int a = 0; a < 3; ++a) uy[a] *= inn;
        const double ux[3] = {r[1] * uy[2] - r[2] * uy[1], r[2] * uy[0] - r[0] * uy[2], r[0] * uy[1] - r[1] * uy[0]};
        const double Hp[3][3] = {{B(3), B(4), B(5)}, {B(4), B(6), B(7)}, {B(5), B(7), B(8)}};
        const double gp[3] = {B(0), B(1), B(2)};
        double HU[3][2];
        for (int a = 0; a < 3; ++a) {
            HU[a][0] = Hp[a][0] * ux[0] + Hp[a][1] * ux[1] + Hp[a][2] * ux[2];
            HU[a][1] = Hp[a][0] * uy[0] + Hp[a][1] * uy[1] + Hp[a][2] * uy[2];
        }
        double H2[3], g2[2], dv[2];
        g2[0] = ux[0] * gp[0] + ux[1] * gp[1] + ux[2] * gp[2];
        g2[1] = uy[0] * gp[0] + uy[1] * gp[1] + uy[2] * gp[2];
        H2[0] = ux[0] * HU[0][0] + ux[1] * HU[1][0] + ux[2] * HU[2][0];
        H2[1] = ux[0] * HU[0][1] + ux[1] * HU[1][1] + ux[2] * HU[2][1];
        H2[2] = uy[0] * HU[0][1] + uy[1] * HU[1][1] + uy[2] * HU[2][1];
        fl[0 * N + k] = damped_small(2, H2, g2, o, abs_scale, dv);
        clamp_norm(2, dv, (double)o.trust_pos * fmax(s[0], fmax(s[1], s[2])));
        for (int a = 0; a < 3; ++a) st[(size_t)a * N + k] = (float)(ux[a] * dv[0] + uy[a] * dv[1]);
    }
    // ---- rotation about r: omega = theta r
    {
        const double Hw[3][3] = {{B(12), B(13), B(14)}, {B(13), B(15), B(16)}, {B(14), B(16), B(17)}};
        double gt = 0.0, Ht = 0.0;
        for (int a = 0; a < 3; ++a) {
            gt += r[a] * B(9 + a);
            for (int b = 0; b < 3; ++b) Ht += r[a] * Hw[a][b] * r[b];
        }
        double th;
        fl[1 * N + k] = damped_small(1, &Ht, &gt, o, abs_scale, &th);
        clamp_norm(1, &th, (double)o.trust_rot);
        st[3 * N + k] = (float)th;
    }
    // ---- scaling in the row space of d lambda / d s (unit rows)
    {
        double tf[3];
        for (int i = 0; i < 3; ++i) tf[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
        const double iz = 1.0 / tf[2];
        const double J00 = c.fx * iz, J02 = -c.fx * tf[0] * iz * iz, J11 = c.fy * iz, J12 = -c.fy * tf[1] * iz * iz;
        double M[2][3];
        for (int kk = 0; kk < 3; ++kk) {
            M[0][kk] = J00 * c.R[kk] + J02 * c.R[6 + kk];
            M[1][kk] = J11 * c.R[3 + kk] + J12 * c.R[6 + kk];
        }
        const double qn = 1.0 / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const double w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
        const double Rq[3][3] = {{1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
                                 {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
                                 {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
        double MR[2][3];
        for (int i = 0; i < 2; ++i)
            for (int a = 0; a < 3; ++a) MR[i][a] = M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a];
        double sxx = kappa, sxy = 0.0, syy = kappa;
        for (int a = 0; a < 3; ++a) {
            const double s2 = s[a] * s[a];
            sxx += MR[0][a] * MR[0][a] * s2;
            sxy += MR[0][a] * MR[1][a] * s2;
            syy += MR[1][a] * MR[1][a] * s2;
        }
        const double mid = 0.5 * (sxx + syy);
        const double rad = sqrt(0.25 * (sxx - syy) * (sxx - syy) + sxy * sxy);
        const double l2 = mid + rad;
        double v2[2];
        if (sxx >= syy) {
            v2[0] = l2 - syy;
            v2[1] = sxy;
        } else {
            v2[0] = sxy;
            v2[1] = l2 - sxx;
        }
        double vn = sqrt(v2[0] * v2[0] + v2[1] * v2[1]);
        if (vn == 0.0) {
            v2[0] = 1.0;
            v2[1] = 0.0;
            vn = 1.0;
        }
        v2[0] /= vn;
        v2[1] /= vn;
        const double v1[2] = {-v2[1], v2[0]};
        double Tm[2][3];
        for (int a = 0; a < 3; ++a) {
            const double e1 = v1[0] * MR[0][a] + v1[1] * MR[1][a];
            const double e2 = v2[0] * MR[0][a] + v2[1] * MR[1][a];
            Tm[0][a] = 2.0 * s[a] * e1 * e1;
            Tm[1][a] = 2.0 * s[a] * e2 * e2;
        }
        // only the row space of T matters; unit rows keep the reduced system well scaled
        for (int i = 0; i < 2; ++i) {
            const double tn = sqrt(Tm[i][0] * Tm[i][0] + Tm[i][1] * Tm[i][1] + Tm[i][2] * Tm[i][2]);
            if (tn > 0.0)
                for (int a = 0; a < 3; ++a) Tm[i][a] /= tn;
        }
        const double Hs[3][3] = {{B(21), B(22), B(23)}, {B(22), B(24), B(25)}, {B(23), B(25), B(26)}};
        const double gs[3] = {B(18), B(19), B(20)};
        double HT[3][2];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 2; ++j) HT[a][j] = Hs[a][0] * Tm[j][0] + Hs[a][1] * Tm[j][1] + Hs[a][2] * Tm[j][2];
        double H2[3], g2[2], av[2];
        for (int i = 0; i < 2; ++i) g2[i] = Tm[i][0] * gs[0] + Tm[i][1] * gs[1] + Tm[i][2] * gs[2];
        H2[0] = Tm[0][0] * HT[0][0] + Tm[0][1] * HT[1][0] + Tm[0][2] * HT[2][0];
        H2[1] = Tm[0][0] * HT[0][1] + Tm[0][1] * HT[1][1] + Tm[0][2] * HT[2][1];
        H2[2] = Tm[1][0] * HT[0][1] + Tm[1][1] * HT[1][1] + Tm[1][2] * HT[2][1];
        fl[2 * N + k] = damped_small(2, H2, g2, o, abs_scale, av);
        double dsv[3];
        for (int a = 0; a < 3; ++a) dsv[a] = Tm[0][a] * av[0] + Tm[1][a] * av[1];
        clamp_norm(3, dsv, (double)o.trust_scale * sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
        for (int a = 0; a < 3; ++a) st[(7 + a) * N + k] = (float)dsv[a];
    }
    // ---- opacity with the log barrier
    {
        const double as = (double)o.barrier_beta * abs_scale;
        const double gB = as * (1.0 / (1.0 - sig) - 1.0 / sig);
        const double hB = as * (1.0 / (sig * sig) + 1.0 / ((1.0 - sig) * (1.0 - sig)));
        const double H1 = B(28) + hB, g1 = B(27) + gB;
        double ds;
        fl[3 * N + k] = damped_small(1, &H1, &g1, o, abs_scale, &ds);
        st[10 * N + k] = (float)ds;
    }
    // ---- colour, per channel
    colour_solve<VM>(K, V, B, o, abs_scale, st, N, k, fl);
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
        qmul<float>(dq, q, r);
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
    // the hot path has a primary and up to three secondaries: a 4-view kernel keeps its arrays in registers
    if (b.n_views <= 4)
        solve_kernel<4><<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                          b.d_data, b.n_views, o, st.d_data, st.d_flags);
    else
        solve_kernel<9><<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, K, cam, kappa,
                                                          b.d_data, b.n_views, o, st.d_data, st.d_flags);
}

void launch_apply(const gsn_gaussians& g, const gsn_steps& st, const gsn_solve_opts& o, uint32_t mask,
                  hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    apply_kernel<<<(g.n + 255) / 256, 256, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.d_sh, g.n, K,
                                                   st.d_data, st.d_flags, o, mask);
}
