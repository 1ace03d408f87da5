// chain.h -- chain rule from projected-space statistics to attribute blocks.
// Host-and-device code: the same functions run in the reduce_chain kernel and in
// host-side precision studies.
//
// Per attribute group y, H_y = J^T H_z J + sum_i (g_z)_i d2 z_i/dy2 with J = dz/dy
// (eq. local_hessian_gradient applied to the projected quantities z), using
// second-order jets for z(y).  Sigma = A A^T + kappa I with A = J_persp W R S
// (Appendix A.3).  Position runs in single precision; scale and rotation run in
// double precision in the plain form, because the inverse Q = Sigma^{-1} of thin
// splats amplifies rounding by the squared condition number of Sigma (the mixed
// form runs them in single precision: templates on the working type Re).
#pragma once
#include "device_common.h"

struct KParams {
    float p[3], q[4], s[3];
    float fc, fs;  // principal frame of the splat in this view: e1 = (fc, fs), e2 = (-fs, fc)
};

// Rows of M rotated into the principal frame: M' = V^T M.
template <class TT>
GSN_HD inline void to_frame(TT M[2][3], float fc, float fs) {
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const TT m0 = M[0][k], m1 = M[1][k];
        M[0][k] = fc * m0 + fs * m1;
        M[1][k] = fc * m1 - fs * m0;
    }
}

// M = J_persp W: Jacobian of the perspective map at t = W p + t_c times the camera rotation.
template <class TT>
GSN_HD inline void persp_M(const TT t[3], const DevCam& c, TT M[2][3], TT& iz) {
    iz = jrecip(t[2]);
    const TT J00 = c.fx * iz, J11 = c.fy * iz;
    const TT J02 = -(c.fx * t[0]) * iz * iz, J12 = -(c.fy * t[1]) * iz * iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        M[0][k] = J00 * c.R[k] + J02 * c.R[6 + k];
        M[1][k] = J11 * c.R[3 + k] + J12 * c.R[6 + k];
    }
}

// Rotation matrix of the unit quaternion q/|q| = (w, x, y, z).
template <class T>
GSN_HD inline void quat_rot(const float q[4], T Rq[3][3]) {
    const T qn = sqrt((T)q[0] * q[0] + (T)q[1] * q[1] + (T)q[2] * q[2] + (T)q[3] * q[3]);
    const T w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    Rq[0][0] = T(1) - T(2) * (y * y + z * z);
    Rq[0][1] = T(2) * (x * y - w * z);
    Rq[0][2] = T(2) * (x * z + w * y);
    Rq[1][0] = T(2) * (x * y + w * z);
    Rq[1][1] = T(1) - T(2) * (x * x + z * z);
    Rq[1][2] = T(2) * (y * z - w * x);
    Rq[2][0] = T(2) * (x * z - w * y);
    Rq[2][1] = T(2) * (y * z + w * x);
    Rq[2][2] = T(1) - T(2) * (x * x + y * y);
}

// Q = Sigma^{-1} from A (2x3): Sigma = A A^T + kappa I.  The determinant is taken
// in the Cauchy-Binet form det(A A^T) = sum of squared 2x2 minors of A, plus
// kappa tr(A A^T) + kappa^2: a sum of non-negative terms, free of the
// cancellation of Sigma_xx Sigma_yy - Sigma_xy^2 for elongated splats.
template <class TT, class K>
GSN_HD inline void conic_from_A(const TT A[2][3], K kappa, TT Q[3]) {
    const TT sxx0 = A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2];
    const TT syy0 = A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2];
    const TT sxy = A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2];
    const TT m01 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const TT m02 = A[0][0] * A[1][2] - A[0][2] * A[1][0];
    const TT m12 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    const TT det = m01 * m01 + m02 * m02 + m12 * m12 + kappa * (sxx0 + syy0) + kappa * kappa;
    const TT sxx = sxx0 + kappa, syy = syy0 + kappa;
    const TT idet = jrecip(det);
    Q[0] = syy * idet;
    Q[1] = -(sxy * idet);
    Q[2] = sxx * idet;
}

// g_a = sum_i gz_i dz_i/dy_a;  H_ab = sum_ij Hz_ij dz_i/dy_a dz_j/dy_b + sum_i gz_i d2z_i/dy_a dy_b (packed).
// gn (local Gauss-Newton): the second sum, a loss gradient times curvature of z, is left out.
template <int N, int NZ, class T>
GSN_HD inline void chain_accumulate(const FJet<N, T>* zj, const T* gz, const T Hz[NZ][NZ], bool gn, T* g, T* H) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
        T acc = T(0);
#pragma unroll
        for (int i = 0; i < NZ; ++i) acc += gz[i] * zj[i].g[a];
        g[a] = acc;
    }
    T t[NZ][N];
#pragma unroll
    for (int i = 0; i < NZ; ++i)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            T acc = T(0);
#pragma unroll
            for (int j = 0; j < NZ; ++j) acc += Hz[i][j] * zj[j].g[b];
            t[i][b] = acc;
        }
    int idx = 0;
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a; b < N; ++b, ++idx) {
            T acc = T(0);
#pragma unroll
            for (int i = 0; i < NZ; ++i) acc += zj[i].g[a] * t[i][b];
            if (!gn) {
#pragma unroll
                for (int i = 0; i < NZ; ++i) acc += gz[i] * zj[i].h[idx];
            }
            H[idx] = acc;
        }
}

// Position: z = (pi', Q', c~) as functions of p (pi through the projection, Q through the
// perspective Jacobian, c~ through the view direction of the SH colour), in the
// splat's principal frame (pi' = V^T pi, Q' = (V^T M R S)(V^T M R S)^T + kappa I inverted).
// The kernel's SH coefficient (ch, i) is shk[(ch K + i) stride].
GSN_HD inline void chain_position(const KParams& kp, const float* shk, size_t stride, int K, const DevCam& c,
                                  float kappa, const float* z, bool gn, float* g, float* H) {
    typedef FJet<3> J;
    J p[3] = {J::var(kp.p[0], 0), J::var(kp.p[1], 1), J::var(kp.p[2], 2)};
    J t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
    J M[2][3], iz;
    persp_M(t, c, M, iz);
    to_frame(M, kp.fc, kp.fs);
    float Rq[3][3];
    quat_rot<float>(kp.q, Rq);
    J A[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a)
            A[i][a] = (M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a]) * kp.s[a];
    J zj[8];
    conic_from_A(A, kappa, zj + 2);
    {
        const J px = c.fx * t[0] * iz, py = c.fy * t[1] * iz;  // pi up to a constant offset
        zj[0] = kp.fc * px + kp.fs * py;
        zj[1] = kp.fc * py - kp.fs * px;
    }
    {
        const J d0 = p[0] - c.o[0], d1 = p[1] - c.o[1], d2 = p[2] - c.o[2];
        const J il = jrecip(jsqrt(d0 * d0 + d1 * d1 + d2 * d2));
        zj[5] = zj[6] = zj[7] = J(0.f);
        sh_basis_visit<J>(K, d0 * il, d1 * il, d2 * il, [&](int i, const J& y) {
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) zj[5 + ch] = zj[5 + ch] + shk[((size_t)ch * K + i) * stride] * y;
        });
    }
    // H_z over (pi_x, pi_y, Q_xx, Q_xy, Q_yy, c~_R, c~_G, c~_B)
    float Hz[8][8];
    int idx = 9;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j, ++idx) Hz[i][j] = Hz[j][i] = z[idx];
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) Hz[i][5 + ch] = Hz[5 + ch][i] = z[24 + i * 3 + ch];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b) Hz[5 + a][5 + b] = a == b ? z[39 + a] : 0.f;
    const float gz[8] = {z[0], z[1], z[2], z[3], z[4], z[6], z[7], z[8]};
    chain_accumulate<3, 8, float>(zj, gz, Hz, gn, g, H);
}

// Statistics of Q' = (Q'_11, Q'_12, Q'_22): entries 2..4 of the (pi', Q') block, kept in the
// double precision of the per-kernel sums (the rotation and scale Hessians cancel strongly).
template <class Re>
GSN_HD inline void q_stats(const double* __restrict__ z, Re gz[3], Re Hz[3][3]) {
    const int pk[3][3] = {{9 + 9, 9 + 10, 9 + 11}, {9 + 10, 9 + 12, 9 + 13}, {9 + 11, 9 + 13, 9 + 14}};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gz[i] = (Re)z[2 + i];
#pragma unroll
        for (int j = 0; j < 3; ++j) Hz[i][j] = (Re)z[pk[i][j]];
    }
}

// The same from the packed copy: zq[0..2] = statistics 2..4, zq[3..8] = statistics 18..23.
template <class Re>
GSN_HD inline void q_stats_packed(const double* __restrict__ zq, Re gz[3], Re Hz[3][3]) {
    const int pk[3][3] = {{3, 4, 5}, {4, 6, 7}, {5, 7, 8}};
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        gz[i] = (Re)zq[i];
#pragma unroll
        for (int j = 0; j < 3; ++j) Hz[i][j] = (Re)zq[pk[i][j]];
    }
}

// The six quantities of Sigma = A A^T + kappa I that the conic needs are bilinear in A,
// F(A) = B_f(A, A): the entries sxx, syy, sxy of A A^T and the three 2x2 minors of A
// (Cauchy-Binet).  B_f(X, Y) for f = 0..5:
template <int F, class Re>
GSN_HD inline Re conic_bilinear(const Re X[2][3], const Re Y[2][3]) {
    if (F == 0) return X[0][0] * Y[0][0] + X[0][1] * Y[0][1] + X[0][2] * Y[0][2];
    if (F == 1) return X[1][0] * Y[1][0] + X[1][1] * Y[1][1] + X[1][2] * Y[1][2];
    if (F == 2) return X[0][0] * Y[1][0] + X[0][1] * Y[1][1] + X[0][2] * Y[1][2];
    if (F == 3) return X[0][0] * Y[1][1] - X[0][1] * Y[1][0];
    if (F == 4) return X[0][0] * Y[1][2] - X[0][2] * Y[1][0];
    return X[0][1] * Y[1][2] - X[0][2] * Y[1][1];
}

// Second-order jet of F_f(A(y)) at y = 0 from A0 = A(0), D[i] = dA/dy_i and (if the map is
// not linear) E(i, j) = d2A/dy_i dy_j:
//   dF = B(D_i, A0) + B(A0, D_i),  d2F = B(D_i, D_j) + B(D_j, D_i) + B(E_ij, A0) + B(A0, E_ij).
template <int F, class Re, class EFn>
GSN_HD inline FJet<3, Re> bilinear_jet(const Re A0[2][3], const Re D[3][2][3], EFn E, bool quadratic) {
    FJet<3, Re> r;
    r.v = conic_bilinear<F>(A0, A0);
#pragma unroll
    for (int i = 0; i < 3; ++i) r.g[i] = conic_bilinear<F>(D[i], A0) + conic_bilinear<F>(A0, D[i]);
    int idx = 0;
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = i; j < 3; ++j, ++idx) {
            Re h = conic_bilinear<F>(D[i], D[j]) + conic_bilinear<F>(D[j], D[i]);
            if (quadratic) {
                Re Eij[2][3];
                E(i, j, Eij);
                h += conic_bilinear<F>(Eij, A0) + conic_bilinear<F>(A0, Eij);
            }
            r.h[idx] = h;
        }
    return r;
}

// Jets of the conic Q = Sigma^{-1} = (syy, -sxy, sxx) / det, det = sum of squared minors +
// kappa (sxx0 + syy0) + kappa^2 (the form of conic_from_A), with only scalar jets live.
template <class Re, class EFn>
GSN_HD inline void conic_jets(const Re A0[2][3], const Re D[3][2][3], EFn E, bool quadratic, Re kappa,
                              FJet<3, Re> Q[3]) {
    typedef FJet<3, Re> J;
    const J sxx0 = bilinear_jet<0>(A0, D, E, quadratic);
    const J syy0 = bilinear_jet<1>(A0, D, E, quadratic);
    J det = kappa * (sxx0 + syy0) + kappa * kappa;  // all in Re
    {
        const J m = bilinear_jet<3>(A0, D, E, quadratic);
        det = det + m * m;
    }
    {
        const J m = bilinear_jet<4>(A0, D, E, quadratic);
        det = det + m * m;
    }
    {
        const J m = bilinear_jet<5>(A0, D, E, quadratic);
        det = det + m * m;
    }
    const J idet = jrecip(det);
    const J sxy = bilinear_jet<2>(A0, D, E, quadratic);
    Q[0] = (syy0 + kappa) * idet;
    Q[1] = -(sxy * idet);
    Q[2] = (sxx0 + kappa) * idet;
}

// M' (rows of the perspective Jacobian times the camera rotation, in the splat's principal
// frame) and R(q) for one kernel, in the working precision Re.
template <class Re>
GSN_HD inline void frame_M_R(const KParams& kp, const DevCam& c, Re M[2][3], Re Rq[3][3]) {
    Re tf[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        tf[i] = (Re)c.R[3 * i] * kp.p[0] + (Re)c.R[3 * i + 1] * kp.p[1] + (Re)c.R[3 * i + 2] * kp.p[2] + c.t[i];
    Re iz;
    persp_M<Re>(tf, c, M, iz);
    to_frame(M, kp.fc, kp.fs);
    quat_rot<Re>(kp.q, Rq);
}

// Scale: A = M' R diag(s) is linear in s, dA/ds_a has the single column a of M' R.
template <class Re>
GSN_HD inline void chain_scale(const KParams& kp, const DevCam& c, float kappa, const Re gz[3],
                               const Re Hz[3][3], bool gn, Re* g, Re* H) {
    Re M[2][3], Rq[3][3];
    frame_M_R(kp, c, M, Rq);
    Re A0[2][3], D[3][2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int i = 0; i < 2; ++i) {
            const Re mr = M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a];
            A0[i][a] = mr * kp.s[a];
#pragma unroll
            for (int b = 0; b < 3; ++b) D[b][i][a] = b == a ? mr : Re(0);
        }
    FJet<3, Re> Q[3];
    conic_jets(A0, D, [](int, int, Re[2][3]) {}, false, (Re)kappa, Q);
    chain_accumulate<3, 3, Re>(Q, gz, Hz, gn, g, H);
}

// Rotation in the tangent space of left rotations: R(omega) = exp([omega]_x) R0, i.e.
// q(omega) = exp(omega/2) * q0.  With B0 = R0 diag(s) and A(omega) = M' R(omega) R0^T B0:
//   dA/domega_i = M' [e_i]_x B0,
//   d2A/domega_i domega_j = (1/2) (M' e_j)(e_i^T B0) + (1/2) (M' e_i)(e_j^T B0) - delta_ij M' B0
// (from [e_i]_x [e_j]_x = e_j e_i^T - delta_ij I).
template <class Re>
GSN_HD inline void chain_rotation(const KParams& kp, const DevCam& c, float kappa, const Re gz[3],
                                  const Re Hz[3][3], bool gn, Re* g, Re* H) {
    Re M[2][3], Rq[3][3];
    frame_M_R(kp, c, M, Rq);
    Re B0[3][3];
#pragma unroll
    for (int r = 0; r < 3; ++r)
#pragma unroll
        for (int a = 0; a < 3; ++a) B0[r][a] = Rq[r][a] * kp.s[a];
    Re A0[2][3], D[3][2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int a = 0; a < 3; ++a) A0[i][a] = M[i][0] * B0[0][a] + M[i][1] * B0[1][a] + M[i][2] * B0[2][a];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            // column a of [e_k]_x B0 = e_k x B0[:, a]
            const Re b0 = B0[0][a], b1 = B0[1][a], b2 = B0[2][a];
            const Re cx = k == 0 ? Re(0) : (k == 1 ? b2 : -b1);
            const Re cy = k == 0 ? -b2 : (k == 1 ? Re(0) : b0);
            const Re cz = k == 0 ? b1 : (k == 1 ? -b0 : Re(0));
#pragma unroll
            for (int i = 0; i < 2; ++i) D[k][i][a] = M[i][0] * cx + M[i][1] * cy + M[i][2] * cz;
        }
    auto E = [&](int i, int j, Re out[2][3]) {
#pragma unroll
        for (int r = 0; r < 2; ++r)
#pragma unroll
            for (int a = 0; a < 3; ++a)
                out[r][a] = Re(0.5) * (M[r][j] * B0[i][a] + M[r][i] * B0[j][a]) - (i == j ? A0[r][a] : Re(0));
    };
    FJet<3, Re> Q[3];
    conic_jets(A0, D, E, true, (Re)kappa, Q);
    chain_accumulate<3, 3, Re>(Q, gz, Hz, gn, g, H);
}
