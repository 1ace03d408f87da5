// reduced.h -- the reduced local systems of one kernel (Sec. 4.2, position, rotation,
// scaling and opacity paragraphs), built from its summed blocks in the primary camera's
// frame.  Shared by the solve and by the features of the learned step scale.
//   position: U = [u_x u_y] orthonormal in the plane normal to the view axis r,
//             H = U^T H_p U, g = U^T g_p (H packed xx, xy, yy);
//   rotation: the left rotation omega = theta r: H = r^T H_omega r, g = r . g_omega;
//   scaling:  the rows of T = d lambda / d s (lambda the eigenvalues of the primary's
//             2D covariance), normalised to unit length: H = T H_s T^T, g = T g_s;
//   opacity:  H_sigma + h_B, g_sigma + g_B with the log barrier
//             -alpha_s [ln sigma + ln(1 - sigma)], alpha_s = beta / (3 |I|).
#pragma once
#include "gsn_internal.h"

template <class T = double>
struct ReducedT {
    T r[3], ux[3], uy[3];
    T Hp[3], gp[2];
    T Ht, gt;
    T T_[2][3], Hs[3], gs[2];
    T Ho, go;
};
typedef ReducedT<double> Reduced;

// B(row) returns block row `row` of this kernel (rows as in the library's block layout).
// T is the working precision (double for the plain form, float for the mixed form).
template <class T, class RowFn>
__device__ __forceinline__ void reduce_systems(const float* __restrict__ pos, const float* __restrict__ rot,
                                               const float* __restrict__ scale, const float* __restrict__ opac,
                                               int n, int k, const DevCam& c, float kappa, RowFn B,
                                               const gsn_solve_opts& o, T abs_scale, ReducedT<T>& R) {
    const size_t N = (size_t)n;
    T p[3], q[4], s[3];
    for (int a = 0; a < 3; ++a) p[a] = pos[a * N + k];
    for (int a = 0; a < 4; ++a) q[a] = rot[a * N + k];
    for (int a = 0; a < 3; ++a) s[a] = scale[a * N + k];
    const T sig = opac[k];
    {
        // camera centre -R^T t in the working precision from the float camera
        T oc[3];
        for (int i = 0; i < 3; ++i)
            oc[i] = -((T)c.R[i] * c.t[0] + (T)c.R[3 + i] * c.t[1] + (T)c.R[6 + i] * c.t[2]);
        for (int a = 0; a < 3; ++a) R.r[a] = p[a] - oc[a];
        const T il = T(1.0) / sqrt(R.r[0] * R.r[0] + R.r[1] * R.r[1] + R.r[2] * R.r[2]);
        for (int a = 0; a < 3; ++a) R.r[a] *= il;
    }
    const T* r = R.r;
    // ---- position
    {
        T* uy = R.uy;
        uy[0] = -r[1] * r[0];
        uy[1] = T(1.0) - r[1] * r[1];
        uy[2] = -r[1] * r[2];
        T nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        if (nn < T(1e-12)) {
            uy[0] = T(1.0) - r[0] * r[0];
            uy[1] = -r[0] * r[1];
            uy[2] = -r[0] * r[2];
            nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        }
        const T inn = T(1.0) / sqrt(nn);
        for (int a = 0; a < 3; ++a) uy[a] *= inn;
        T* ux = R.ux;
        ux[0] = r[1] * uy[2] - r[2] * uy[1];
        ux[1] = r[2] * uy[0] - r[0] * uy[2];
        ux[2] = r[0] * uy[1] - r[1] * uy[0];
        const T Hp[3][3] = {{B(3), B(4), B(5)}, {B(4), B(6), B(7)}, {B(5), B(7), B(8)}};
        const T gp[3] = {B(0), B(1), B(2)};
        T HU[3][2];
        for (int a = 0; a < 3; ++a) {
            HU[a][0] = Hp[a][0] * ux[0] + Hp[a][1] * ux[1] + Hp[a][2] * ux[2];
            HU[a][1] = Hp[a][0] * uy[0] + Hp[a][1] * uy[1] + Hp[a][2] * uy[2];
        }
        R.gp[0] = ux[0] * gp[0] + ux[1] * gp[1] + ux[2] * gp[2];
        R.gp[1] = uy[0] * gp[0] + uy[1] * gp[1] + uy[2] * gp[2];
        R.Hp[0] = ux[0] * HU[0][0] + ux[1] * HU[1][0] + ux[2] * HU[2][0];
        R.Hp[1] = ux[0] * HU[0][1] + ux[1] * HU[1][1] + ux[2] * HU[2][1];
        R.Hp[2] = uy[0] * HU[0][1] + uy[1] * HU[1][1] + uy[2] * HU[2][1];
    }
    // ---- rotation about r
    {
        const T Hw[3][3] = {{B(12), B(13), B(14)}, {B(13), B(15), B(16)}, {B(14), B(16), B(17)}};
        R.gt = T(0.0);
        R.Ht = T(0.0);
        for (int a = 0; a < 3; ++a) {
            R.gt += r[a] * B(9 + a);
            for (int b = 0; b < 3; ++b) R.Ht += r[a] * Hw[a][b] * r[b];
        }
    }
    // ---- scaling
    {
        T tf[3];
        for (int i = 0; i < 3; ++i) tf[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
        const T iz = T(1.0) / tf[2];
        const T J00 = c.fx * iz, J02 = -c.fx * tf[0] * iz * iz, J11 = c.fy * iz, J12 = -c.fy * tf[1] * iz * iz;
        T M[2][3];
        for (int kk = 0; kk < 3; ++kk) {
            M[0][kk] = J00 * c.R[kk] + J02 * c.R[6 + kk];
            M[1][kk] = J11 * c.R[3 + kk] + J12 * c.R[6 + kk];
        }
        const T qn = T(1.0) / sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
        const T w = q[0] * qn, x = q[1] * qn, y = q[2] * qn, z = q[3] * qn;
        const T Rq[3][3] = {{T(1.0) - T(2.0) * (y * y + z * z), T(2.0) * (x * y - w * z), T(2.0) * (x * z + w * y)},
                                 {T(2.0) * (x * y + w * z), T(1.0) - T(2.0) * (x * x + z * z), T(2.0) * (y * z - w * x)},
                                 {T(2.0) * (x * z - w * y), T(2.0) * (y * z + w * x), T(1.0) - T(2.0) * (x * x + y * y)}};
        T MR[2][3];
        for (int i = 0; i < 2; ++i)
            for (int a = 0; a < 3; ++a) MR[i][a] = M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a];
        T sxx = kappa, sxy = T(0.0), syy = kappa;
        for (int a = 0; a < 3; ++a) {
            const T s2 = s[a] * s[a];
            sxx += MR[0][a] * MR[0][a] * s2;
            sxy += MR[0][a] * MR[1][a] * s2;
            syy += MR[1][a] * MR[1][a] * s2;
        }
        const T mid = T(0.5) * (sxx + syy);
        const T rad = sqrt(T(0.25) * (sxx - syy) * (sxx - syy) + sxy * sxy);
        const T l2 = mid + rad;
        T v2[2];
        if (sxx >= syy) {
            v2[0] = l2 - syy;
            v2[1] = sxy;
        } else {
            v2[0] = sxy;
            v2[1] = l2 - sxx;
        }
        T vn = sqrt(v2[0] * v2[0] + v2[1] * v2[1]);
        if (vn == T(0.0)) {
            v2[0] = T(1.0);
            v2[1] = T(0.0);
            vn = T(1.0);
        }
        v2[0] /= vn;
        v2[1] /= vn;
        const T v1[2] = {-v2[1], v2[0]};
        T (*Tm)[3] = R.T_;
        for (int a = 0; a < 3; ++a) {
            const T e1 = v1[0] * MR[0][a] + v1[1] * MR[1][a];
            const T e2 = v2[0] * MR[0][a] + v2[1] * MR[1][a];
            Tm[0][a] = T(2.0) * s[a] * e1 * e1;
            Tm[1][a] = T(2.0) * s[a] * e2 * e2;
        }
        // only the row space of T matters; unit rows keep the reduced system well scaled
        for (int i = 0; i < 2; ++i) {
            const T tn = sqrt(Tm[i][0] * Tm[i][0] + Tm[i][1] * Tm[i][1] + Tm[i][2] * Tm[i][2]);
            if (tn > T(0.0))
                for (int a = 0; a < 3; ++a) Tm[i][a] /= tn;
        }
        const T Hs[3][3] = {{B(21), B(22), B(23)}, {B(22), B(24), B(25)}, {B(23), B(25), B(26)}};
        const T gs[3] = {B(18), B(19), B(20)};
        T HT[3][2];
        for (int a = 0; a < 3; ++a)
            for (int j = 0; j < 2; ++j) HT[a][j] = Hs[a][0] * Tm[j][0] + Hs[a][1] * Tm[j][1] + Hs[a][2] * Tm[j][2];
        for (int i = 0; i < 2; ++i) R.gs[i] = Tm[i][0] * gs[0] + Tm[i][1] * gs[1] + Tm[i][2] * gs[2];
        R.Hs[0] = Tm[0][0] * HT[0][0] + Tm[0][1] * HT[1][0] + Tm[0][2] * HT[2][0];
        R.Hs[1] = Tm[0][0] * HT[0][1] + Tm[0][1] * HT[1][1] + Tm[0][2] * HT[2][1];
        R.Hs[2] = Tm[1][0] * HT[0][1] + Tm[1][1] * HT[1][1] + Tm[1][2] * HT[2][1];
    }
    // ---- opacity with the log barrier
    {
        const T as = (T)o.barrier_beta * abs_scale;
        const T gB = as * (T(1.0) / (T(1.0) - sig) - T(1.0) / sig);
        const T hB = as * (T(1.0) / (sig * sig) + T(1.0) / ((T(1.0) - sig) * (T(1.0) - sig)));
        R.Ho = B(28) + hB;
        R.go = B(27) + gB;
    }
}
