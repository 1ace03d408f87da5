// gsn_oracle.cpp -- FP64 CPU oracle for the stochastic local-Newton 3DGS step
// of "3DGS^2: Near Second-order Converging 3D Gaussian Splatting" (arxiv 2501.13975).
//
// TEST INFRASTRUCTURE ONLY.  Nothing in the product path may call, link or load
// this file or the library built from it; only the tests, the smoke check and
// the bench's CPU-baseline leg do.  It shares no code with the HIP library.
//
// What it computes, in the paper's order and notation, written plainly and slowly:
//   * projection of each kernel (Sec. 3, eq. 3dgs; Appendix A.1-A.3): centre pi,
//     2D covariance Sigma (EWA), its inverse Q, view-dependent SH colour c~;
//   * the FP32 binning decisions (which tiles a kernel covers, its depth key),
//     evaluated op by op in single precision with no contraction so that a GPU
//     implementation can reproduce them bit for bit;
//   * per-pixel front-to-back alpha compositing (eq. 3dgs);
//   * the loss L = L2 + lambda * L_S with its per-pixel gradient and the
//     per-pixel diagonal of its Hessian (Sec. 4.2, L2 and SSIM derivatives);
//   * per-kernel gradients and Hessians of the loss with respect to each
//     attribute group (eq. local_hessian_gradient), taken by second-order
//     forward-mode jets through projection and compositing, one pixel at a
//     time, with the image Hessian kept diagonal per pixel as the paper does;
//   * the reduced-coordinate local Newton solves (position in the plane normal
//     to the view direction, rotation about the view axis, scaling in the
//     row space of d(lambda)/ds, opacity with a log barrier, SH colour) and
//     their application (Sec. 4.2, Position/Scaling/Rotation/Opacity/Color);
//   * camera KNN on the bounding sphere (Sec. 4.1) and the 2x box downsampling
//     of secondary targets (Sec. 4.3).
// Everything is double precision except the FP32 binning specification.

#include "jet.hpp"

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstring>
#include <limits>
#include <vector>

namespace {

// Option vector layout (double[O_COUNT]); the Python wrapper owns the defaults.
enum Opt {
    O_TILE = 0,      // tile edge in pixels
    O_ALPHA_MIN,     // skip a splat whose alpha is below this
    O_ALPHA_MAX,     // clamp alpha to at most this
    O_T_MIN,         // stop before transmittance would drop below this
    O_KAPPA,         // EWA low-pass dilation added to the 2D covariance diagonal
    O_RADIUS_SIGMA,  // splat radius in standard deviations of the major axis
    O_SMOOTH,        // 1 = brute force over all kernels, no tiles, thresholds, clamp or dilation
    O_BG_R, O_BG_G, O_BG_B,
    O_LAMBDA,        // SSIM weight lambda in L = L2 + lambda L_S
    O_BARRIER_BETA,  // opacity barrier weight alpha_sigma = beta / (3 |I|)
    O_DAMP_REL,      // damping mu0 = damp_rel * max(mean diag H, 0) + damp_abs / (3 |I|)
    O_DAMP_ABS,
    O_PIVOT_MIN,     // Cholesky accepted only if min pivot / max pivot >= this
    O_MAX_ESC,       // damping escalations mu_j = mu0 10^j, j = 0..max_esc
    O_SH_FLOOR,      // per-view SH curvature floor relative to the largest
    O_SCALE_FLOOR,   // s_new >= scale_floor * s
    O_OPAC_FTB,      // fraction-to-boundary factor for the opacity update
    O_NPIX_PRIMARY,  // |I| of the primary target (barrier and damping scales)
    O_TRUST_POS,     // |Delta p| <= trust_pos * max_a s_a
    O_TRUST_ROT,     // |theta| <= trust_rot (radians)
    O_TRUST_SCALE,   // |Delta s| <= trust_scale * |s|
    O_TRUST_SH,      // per channel |Delta c| <= trust_sh (SH coefficient vector)
    O_OPAC_EPS,      // applied opacity kept in [opac_eps, 1 - opac_eps]
    O_STEP_FRAC,     // every group's Newton step is multiplied by step_frac before the trust radii
    O_DAMP_SH,       // colour damping mu = damp_sh * mean diag(G) + damp_abs / (3 |I|)
    O_GAUSS_NEWTON,  // 1 = local Gauss-Newton blocks: H = sum_ch h_ch J_ch J_ch^T (no dL_ch d2c_ch term)
    O_OVERLAP,       // 1 = every kernel's steps scaled by its overlap share omega = sum (alpha T)^2 / sum alpha T
    O_COUNT
};

struct Cam {
    double R[9], t[3], fx, fy, cx, cy, znear;
    int W, H;
    double o[3];  // camera centre, -R^T t
};

Cam load_cam(const double* c) {
    Cam k;
    for (int i = 0; i < 9; ++i) k.R[i] = c[i];
    for (int i = 0; i < 3; ++i) k.t[i] = c[9 + i];
    k.fx = c[12]; k.fy = c[13]; k.cx = c[14]; k.cy = c[15];
    k.W = (int)c[16]; k.H = (int)c[17]; k.znear = c[18];
    for (int i = 0; i < 3; ++i)
        k.o[i] = -(k.R[i] * k.t[0] + k.R[3 + i] * k.t[1] + k.R[6 + i] * k.t[2]);
    return k;
}

struct Scene {
    const double *pos, *rot, *scale, *opac, *sh;
    int n, K;
};

// ---------------------------------------------------------------------------
// View-dependent colour basis (Appendix A.2): Y_i = B_i * Phi_i(r), with the
// polynomial basis Phi as the paper lists it and B_i the textbook real
// spherical-harmonic normalisation constants.
// ---------------------------------------------------------------------------
template <class T>
void sh_basis(int K, const T& x, const T& y, const T& z, T* Y) {
    const double PI = 3.14159265358979323846;
    Y[0] = T(0.5 / std::sqrt(PI));
    if (K <= 1) return;
    const double c1 = std::sqrt(3.0 / (4.0 * PI));
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (K <= 4) return;
    const double c2a = std::sqrt(15.0 / (4.0 * PI));
    const double c2b = std::sqrt(5.0 / (16.0 * PI));
    const double c2c = std::sqrt(15.0 / (16.0 * PI));
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = c2a * (x * y);
    Y[5] = c2a * (y * z);
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = c2a * (x * z);
    Y[8] = c2c * (xx - yy);
    if (K <= 9) return;
    const double c3a = std::sqrt(35.0 / (32.0 * PI));
    const double c3b = std::sqrt(105.0 / (4.0 * PI));
    const double c3c = std::sqrt(21.0 / (32.0 * PI));
    const double c3d = std::sqrt(7.0 / (16.0 * PI));
    const double c3e = std::sqrt(105.0 / (16.0 * PI));
    Y[9] = c3a * (y * (3.0 * xx - yy));
    Y[10] = c3b * (x * y * z);
    Y[11] = c3c * (y * (4.0 * zz - xx - yy));
    Y[12] = c3d * (z * (2.0 * zz - 3.0 * xx - 3.0 * yy));
    Y[13] = c3c * (x * (4.0 * zz - xx - yy));
    Y[14] = c3e * (z * (xx - yy));
    Y[15] = c3a * (x * (xx - 3.0 * yy));
}

// ---------------------------------------------------------------------------
// Projection of one kernel (Sec. 3; Appendix A.1 for pi, A.3 for Sigma).
// The camera is a pinhole with OpenCV axes; pi = (fx x/z + cx, fy y/z + cy).
// Sigma = J W R S S^T R^T W^T J^T + kappa I with J the local affine (EWA)
// Jacobian of the perspective map at the kernel centre.
// ---------------------------------------------------------------------------
template <class T>
struct Proj {
    T pi[2];
    T Q[3];   // Sigma^{-1}: (xx, xy, yy)
    T cov[3]; // Sigma: (xx, xy, yy)
    T ct[3];  // view-dependent colour c~
    T depth;
    bool ok;
};

template <class T>
Proj<T> project(const T p[3], const T q[4], const T s[3], const double* shk, int K,
                const Cam& c, double kappa) {
    Proj<T> P;
    P.ok = false;
    T t[3];
    for (int i = 0; i < 3; ++i)
        t[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
    P.depth = t[2];
    if (!(val(t[2]) > c.znear)) return P;
    // unit quaternion -> rotation matrix (Sec. 3)
    const T qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const T w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
    const T Rq[3][3] = {
        {1.0 - 2.0 * (y * y + z * z), 2.0 * (x * y - w * z), 2.0 * (x * z + w * y)},
        {2.0 * (x * y + w * z), 1.0 - 2.0 * (x * x + z * z), 2.0 * (y * z - w * x)},
        {2.0 * (x * z - w * y), 2.0 * (y * z + w * x), 1.0 - 2.0 * (x * x + y * y)}};
    // 3D covariance A = R S S^T R^T
    T S3[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            T acc = T(0.0);
            for (int a = 0; a < 3; ++a) acc = acc + Rq[i][a] * Rq[j][a] * (s[a] * s[a]);
            S3[i][j] = acc;
        }
    const T iz = recip(t[2]);
    const T J00 = c.fx * iz, J02 = -c.fx * t[0] * iz * iz;
    const T J11 = c.fy * iz, J12 = -c.fy * t[1] * iz * iz;
    T M[2][3];
    for (int k = 0; k < 3; ++k) {
        M[0][k] = J00 * c.R[k] + J02 * c.R[6 + k];
        M[1][k] = J11 * c.R[3 + k] + J12 * c.R[6 + k];
    }
    T cv[2][2];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            T acc = T(0.0);
            for (int i = 0; i < 3; ++i)
                for (int j = 0; j < 3; ++j) acc = acc + M[a][i] * S3[i][j] * M[b][j];
            cv[a][b] = acc;
        }
    P.cov[0] = cv[0][0] + kappa;
    P.cov[1] = cv[0][1];
    P.cov[2] = cv[1][1] + kappa;
    const T det = P.cov[0] * P.cov[2] - P.cov[1] * P.cov[1];
    if (!(val(det) > 0.0)) return P;
    P.Q[0] = P.cov[2] / det;
    P.Q[1] = -P.cov[1] / det;
    P.Q[2] = P.cov[0] / det;
    P.pi[0] = c.fx * t[0] * iz + c.cx;
    P.pi[1] = c.fy * t[1] * iz + c.cy;
    // view direction r_k from the camera centre to the kernel centre
    const T d0 = p[0] - c.o[0], d1 = p[1] - c.o[1], d2 = p[2] - c.o[2];
    const T dn = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
    const T rx = d0 / dn, ry = d1 / dn, rz = d2 / dn;
    T Y[16];
    sh_basis(K, rx, ry, rz, Y);
    for (int ch = 0; ch < 3; ++ch) {
        T acc = T(0.0);
        for (int i = 0; i < K; ++i) acc = acc + Y[i] * shk[ch * K + i];
        P.ct[ch] = acc;
    }
    P.ok = true;
    return P;
}

void gather_sh(const Scene& S, int k, double* shk) {
    for (int ch = 0; ch < 3; ++ch)
        for (int i = 0; i < S.K; ++i) shk[ch * S.K + i] = S.sh[((size_t)ch * S.K + i) * S.n + k];
}

Proj<double> project_value(const Scene& S, int k, const Cam& c, double kappa) {
    double p[3], q[4], s[3], shk[48];
    for (int a = 0; a < 3; ++a) p[a] = S.pos[(size_t)a * S.n + k];
    for (int a = 0; a < 4; ++a) q[a] = S.rot[(size_t)a * S.n + k];
    for (int a = 0; a < 3; ++a) s[a] = S.scale[(size_t)a * S.n + k];
    gather_sh(S, k, shk);
    return project<double>(p, q, s, shk, S.K, c, kappa);
}

// ---------------------------------------------------------------------------
// Per-pixel compositing (eq. 3dgs), front to back in list order.
// Standard mode adds the usual rasteriser extras: alpha clamped to alpha_max,
// splats with alpha < alpha_min skipped, and the pixel stopped before its
// transmittance would drop below T_min.  Smooth mode has none of these.
// ---------------------------------------------------------------------------
struct Rec {
    double px, py, q0, q1, q2, sig, c[3], depth;
    bool ok;
};

struct Added {
    int k;
    double alpha, T;  // alpha used and transmittance before this splat
    bool clamped;     // alpha was clamped to alpha_max
};

struct PixelOut {
    double C[3], Tfinal, margin;
    int ncontrib;
};

void composite_pixel(const Rec* rec, const int32_t* list, int64_t len, double x, double y,
                     const double* o, std::vector<Added>* added, PixelOut& out) {
    const bool smooth = o[O_SMOOTH] != 0.0;
    const double amin = o[O_ALPHA_MIN], amax = o[O_ALPHA_MAX], tmin = o[O_T_MIN];
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    double margin = std::numeric_limits<double>::infinity();
    int nc = 0;
    if (added) added->clear();
    for (int64_t j = 0; j < len; ++j) {
        const Rec& r = rec[list[j]];
        const double dx = r.px - x, dy = r.py - y;
        const double power = -0.5 * (r.q0 * dx * dx + r.q2 * dy * dy) - r.q1 * dx * dy;
        double a = r.sig * std::exp(power);
        bool clamped = false;
        if (!smooth) {
            margin = std::min(margin, std::fabs(a - amax) / amax);
            if (a > amax) {
                a = amax;
                clamped = true;
            }
            margin = std::min(margin, std::fabs(a - amin) / amin);
            if (a < amin) continue;
            const double Tn = T * (1.0 - a);
            margin = std::min(margin, std::fabs(Tn - tmin) / tmin);
            if (Tn < tmin) break;
        }
        for (int ch = 0; ch < 3; ++ch) C[ch] += a * T * r.c[ch];
        if (added) added->push_back({list[j], a, T, clamped});
        T *= 1.0 - a;
        nc = (int)j + 1;
    }
    for (int ch = 0; ch < 3; ++ch) out.C[ch] = C[ch] + T * o[O_BG_R + ch];
    out.Tfinal = T;
    out.margin = margin;
    out.ncontrib = nc;
}

// Depth-ordered list of every projected kernel (smooth mode), ties by id.
std::vector<int32_t> depth_order(const std::vector<Rec>& rec) {
    std::vector<int32_t> ids;
    for (int k = 0; k < (int)rec.size(); ++k)
        if (rec[k].ok) ids.push_back(k);
    std::stable_sort(ids.begin(), ids.end(),
                     [&](int32_t a, int32_t b) { return rec[a].depth < rec[b].depth; });
    return ids;
}

std::vector<Rec> project_all(const Scene& S, const Cam& c, const double* o) {
    const double kappa = o[O_SMOOTH] != 0.0 ? 0.0 : o[O_KAPPA];
    std::vector<Rec> rec(S.n);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < S.n; ++k) {
        Proj<double> P = project_value(S, k, c, kappa);
        Rec& r = rec[k];
        r.ok = P.ok;
        r.px = P.pi[0]; r.py = P.pi[1];
        r.q0 = P.Q[0]; r.q1 = P.Q[1]; r.q2 = P.Q[2];
        r.sig = S.opac[k];
        for (int ch = 0; ch < 3; ++ch) r.c[ch] = P.ct[ch];
        r.depth = P.depth;
    }
    return rec;
}

// ---------------------------------------------------------------------------
// Image-space loss (Sec. 4.2): L = L2 + lambda L_S with
//   L2  = 1/(6|I|) sum_pix sum_ch (c - c^t)^2,   dL2/dc = (c - c^t)/(3|I|),
//   L_S = 1/(3|I|) sum_pix sum_ch (1 - SSIM_ch(pix)),
// SSIM over an 11x11 Gaussian window (sigma 1.5, zero-padded borders) with
// C1 = 0.01^2, C2 = 0.03^2.  For each pixel the derivative of every window's
// SSIM with respect to that pixel's value is taken by the quotient rule in
// the paper's f0..f3 / g0..g3 notation and summed over the windows that
// contain the pixel; the Hessian is kept as its per-pixel diagonal.
// ---------------------------------------------------------------------------
void ssim_window(double w[11][11]) {
    double g[11], sum = 0.0;
    for (int i = 0; i < 11; ++i) {
        g[i] = std::exp(-((i - 5) * (i - 5)) / (2.0 * 1.5 * 1.5));
        sum += g[i];
    }
    for (int i = 0; i < 11; ++i)
        for (int j = 0; j < 11; ++j) w[i][j] = (g[i] / sum) * (g[j] / sum);
}

}  // namespace

extern "C" {

int orc_version() { return 1; }

// Basis values Y_0..Y_{K-1} at a unit direction r (K = 1, 4, 9 or 16).
void orc_sh_basis(int K, const double* r, double* out) { sh_basis<double>(K, r[0], r[1], r[2], out); }

// ---------------------------------------------------------------------------
// FP32 binning specification.  Every line is one IEEE single-precision
// operation evaluated left to right, with no fused multiply-add, correctly
// rounded division and square root.  Outputs per kernel: the bit pattern of
// the camera-space depth, the tile rectangle [x0, x1) x [y0, y1) and a
// visibility flag (in front of the near plane, positive-definite 2D
// covariance, non-empty rectangle).  cam32: R[9], t[3], fx, fy, cx, cy, W, H, znear.
// ---------------------------------------------------------------------------
void orc_project32(int n, const float* pos, const float* rot, const float* scale,
                   const float* cam, float kappa, float radius_sigma, int tile,
                   uint32_t* depth_bits, int32_t* rect, uint8_t* visible) {
    const int W = (int)cam[16], H = (int)cam[17];
    const int tiles_x = (W + tile - 1) / tile, tiles_y = (H + tile - 1) / tile;
    const float* R = cam;
    const float* tc = cam + 9;
    const float fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15], znear = cam[18];
    const float ftile = (float)tile;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        const float px = pos[k], py = pos[n + k], pz = pos[2 * n + k];
        rect[k] = rect[n + k] = rect[2 * n + k] = rect[3 * n + k] = 0;
        visible[k] = 0;
        const float tx = ((R[0] * px + R[1] * py) + R[2] * pz) + tc[0];
        const float ty = ((R[3] * px + R[4] * py) + R[5] * pz) + tc[1];
        const float tz = ((R[6] * px + R[7] * py) + R[8] * pz) + tc[2];
        uint32_t bits;
        std::memcpy(&bits, &tz, 4);
        depth_bits[k] = bits;
        if (!(tz > znear)) continue;
        const float qw = rot[k], qx = rot[n + k], qy = rot[2 * n + k], qz = rot[3 * n + k];
        const float nq = std::sqrt(((qw * qw + qx * qx) + qy * qy) + qz * qz);
        const float w = qw / nq, x = qx / nq, y = qy / nq, z = qz / nq;
        const float r[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                               {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                               {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
        const float s[3] = {scale[k], scale[n + k], scale[2 * n + k]};
        float m[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) m[i][j] = r[i][j] * s[j];
        float S[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) S[i][j] = (m[i][0] * m[j][0] + m[i][1] * m[j][1]) + m[i][2] * m[j][2];
        const float j00 = fx / tz;
        const float j02 = -(fx * tx) / (tz * tz);
        const float j11 = fy / tz;
        const float j12 = -(fy * ty) / (tz * tz);
        float a[2][3];
        for (int c = 0; c < 3; ++c) {
            a[0][c] = j00 * R[c] + j02 * R[6 + c];
            a[1][c] = j11 * R[3 + c] + j12 * R[6 + c];
        }
        float b[2][3];
        for (int i = 0; i < 2; ++i)
            for (int c = 0; c < 3; ++c) b[i][c] = (a[i][0] * S[0][c] + a[i][1] * S[1][c]) + a[i][2] * S[2][c];
        const float cxx = ((b[0][0] * a[0][0] + b[0][1] * a[0][1]) + b[0][2] * a[0][2]) + kappa;
        const float cxy = (b[0][0] * a[1][0] + b[0][1] * a[1][1]) + b[0][2] * a[1][2];
        const float cyy = ((b[1][0] * a[1][0] + b[1][1] * a[1][1]) + b[1][2] * a[1][2]) + kappa;
        const float det = cxx * cyy - cxy * cxy;
        if (!(det > 0.0f)) continue;
        const float mid = 0.5f * (cxx + cyy);
        const float lam = mid + std::sqrt(std::fmax(0.1f, mid * mid - det));
        const float radius = std::ceil(radius_sigma * std::sqrt(lam));
        const float u = (fx * tx) / tz + cx;
        const float v = (fy * ty) / tz + cy;
        const float x0 = std::fmin(std::fmax(std::floor((u - radius) / ftile), 0.0f), (float)tiles_x);
        const float x1 = std::fmin(std::fmax(std::floor((u + radius) / ftile) + 1.0f, 0.0f), (float)tiles_x);
        const float y0 = std::fmin(std::fmax(std::floor((v - radius) / ftile), 0.0f), (float)tiles_y);
        const float y1 = std::fmin(std::fmax(std::floor((v + radius) / ftile) + 1.0f, 0.0f), (float)tiles_y);
        const int ix0 = (int)x0, ix1 = (int)x1, iy0 = (int)y0, iy1 = (int)y1;
        if (ix1 <= ix0 || iy1 <= iy0) continue;
        rect[k] = ix0;
        rect[n + k] = iy0;
        rect[2 * n + k] = ix1;
        rect[3 * n + k] = iy1;
        visible[k] = 1;
    }
}

// Per-tile lists: for each tile, the visible kernels whose rectangle covers it,
// ordered by (depth bits, id).  Kernels are visited in that order and appended,
// so every list comes out sorted.  Call with ids == NULL to get the pair count.
int64_t orc_tile_lists(int n, const uint32_t* depth_bits, const int32_t* rect, const uint8_t* visible,
                       int tiles_x, int tiles_y, int64_t* tile_start, int32_t* ids) {
    const int ntiles = tiles_x * tiles_y;
    std::vector<int64_t> count(ntiles, 0);
    std::vector<int32_t> order;
    for (int k = 0; k < n; ++k)
        if (visible[k]) order.push_back(k);
    std::sort(order.begin(), order.end(), [&](int32_t a, int32_t b) {
        if (depth_bits[a] != depth_bits[b]) return depth_bits[a] < depth_bits[b];
        return a < b;
    });
    for (int32_t k : order)
        for (int ty = rect[n + k]; ty < rect[3 * n + k]; ++ty)
            for (int tx = rect[k]; tx < rect[2 * n + k]; ++tx) count[ty * tiles_x + tx]++;
    int64_t total = 0;
    for (int t = 0; t < ntiles; ++t) {
        if (tile_start) tile_start[t] = total;
        total += count[t];
    }
    if (tile_start) tile_start[ntiles] = total;
    if (!ids) return total;
    std::vector<int64_t> cur(tile_start, tile_start + ntiles);
    for (int32_t k : order)
        for (int ty = rect[n + k]; ty < rect[3 * n + k]; ++ty)
            for (int tx = rect[k]; tx < rect[2 * n + k]; ++tx) ids[cur[ty * tiles_x + tx]++] = k;
    return total;
}

// FP64 render.  Standard mode composites each pixel over its tile's list
// (tile_start/ids from orc_tile_lists); smooth mode (tile_start == NULL and
// O_SMOOTH set) composites every kernel in depth order with no thresholds.
// Outputs: img [3][H][W], Tfinal [H][W], ncontrib [H][W] (1 + index of the last
// list entry added), margin [H][W] (smallest relative distance of any
// threshold decision from its threshold; +inf in smooth mode).
int orc_render(int n, int K, const double* pos, const double* rot, const double* scale,
               const double* opac, const double* sh, const double* cam, const double* o,
               const int64_t* tile_start, const int32_t* ids, double* img, double* Tfinal,
               int32_t* ncontrib, double* margin) {
    const Scene S{pos, rot, scale, opac, sh, n, K};
    const Cam c = load_cam(cam);
    const std::vector<Rec> rec = project_all(S, c, o);
    const bool smooth = o[O_SMOOTH] != 0.0;
    std::vector<int32_t> all;
    if (smooth) all = depth_order(rec);
    const int tile = (int)o[O_TILE];
    const int tiles_x = (c.W + tile - 1) / tile;
    const size_t npx = (size_t)c.W * c.H;
#pragma omp parallel for schedule(dynamic, 16)
    for (int y = 0; y < c.H; ++y)
        for (int x = 0; x < c.W; ++x) {
            const int32_t* list;
            int64_t len;
            if (smooth) {
                list = all.data();
                len = (int64_t)all.size();
            } else {
                const int t = (y / tile) * tiles_x + (x / tile);
                list = ids + tile_start[t];
                len = tile_start[t + 1] - tile_start[t];
            }
            PixelOut po;
            composite_pixel(rec.data(), list, len, x, y, o, nullptr, po);
            const size_t i = (size_t)y * c.W + x;
            for (int ch = 0; ch < 3; ++ch) img[ch * npx + i] = po.C[ch];
            if (Tfinal) Tfinal[i] = po.Tfinal;
            if (ncontrib) ncontrib[i] = po.ncontrib;
            if (margin) margin[i] = po.margin;
        }
    return 0;
}

// Loss value and per-pixel derivative maps (see the comment above ssim_window).
// img, tgt: [3][H][W].  dL, hd: [3][H][W] (either may be NULL).  parts[0] = L2,
// parts[1] = L_S (so L = parts[0] + lambda parts[1]).
int orc_loss(int W, int H, const double* img, const double* tgt, double lambda, double* dL,
             double* hd, double* parts) {
    const double C1 = 0.01 * 0.01, C2 = 0.03 * 0.03;
    double w[11][11];
    ssim_window(w);
    const size_t npx = (size_t)W * H;
    const double norm = 1.0 / (3.0 * (double)npx);
    // window statistics at every centre: mu, mu^t, E[c^2], E[t^2], E[c t]
    std::vector<double> st(3 * npx * 5);
    // per-row partial sums, added in row order afterwards so the value is deterministic
    std::vector<double> row_l2(H, 0.0), row_ls(H, 0.0);
#pragma omp parallel for schedule(static)
    for (int b = 0; b < H; ++b)
        for (int a = 0; a < W; ++a)
            for (int ch = 0; ch < 3; ++ch) {
                const double* I = img + ch * npx;
                const double* T = tgt + ch * npx;
                double m1 = 0, m2 = 0, e11 = 0, e22 = 0, e12 = 0;
                for (int j = 0; j < 11; ++j)
                    for (int i = 0; i < 11; ++i) {
                        const int x = a + i - 5, y = b + j - 5;
                        if (x < 0 || y < 0 || x >= W || y >= H) continue;
                        const double cv = I[(size_t)y * W + x], tv = T[(size_t)y * W + x];
                        const double ww = w[j][i];
                        m1 += ww * cv;
                        m2 += ww * tv;
                        e11 += ww * cv * cv;
                        e22 += ww * tv * tv;
                        e12 += ww * cv * tv;
                    }
                double* q = &st[((size_t)ch * npx + (size_t)b * W + a) * 5];
                q[0] = m1; q[1] = m2; q[2] = e11; q[3] = e22; q[4] = e12;
                const double v1 = e11 - m1 * m1, v2 = e22 - m2 * m2, cov = e12 - m1 * m2;
                const double ssim = ((2 * m1 * m2 + C1) * (2 * cov + C2)) / ((m1 * m1 + m2 * m2 + C1) * (v1 + v2 + C2));
                row_ls[b] += 1.0 - ssim;
                const size_t i = (size_t)b * W + a;
                const double r = I[i] - T[i];
                row_l2[b] += r * r;
            }
    double l2 = 0.0, ls = 0.0;
    for (int b = 0; b < H; ++b) {
        l2 += row_l2[b];
        ls += row_ls[b];
    }
    if (parts) {
        parts[0] = l2 / (6.0 * (double)npx);
        parts[1] = ls * norm;
    }
    if (!dL && !hd) return 0;
#pragma omp parallel for schedule(static)
    for (int n_ = 0; n_ < H; ++n_)
        for (int m = 0; m < W; ++m)
            for (int ch = 0; ch < 3; ++ch) {
                const size_t pi = (size_t)n_ * W + m;
                const double cv = img[ch * npx + pi], tv = tgt[ch * npx + pi];
                double d1 = 0.0, d2 = 0.0;
                // windows centred at (a, b) containing pixel (m, n)
                for (int b = n_ - 5; b <= n_ + 5; ++b)
                    for (int a = m - 5; a <= m + 5; ++a) {
                        if (a < 0 || b < 0 || a >= W || b >= H) continue;
                        const double ww = w[n_ - b + 5][m - a + 5];
                        const double* q = &st[((size_t)ch * npx + (size_t)b * W + a) * 5];
                        const double mu = q[0], mut = q[1];
                        const double f0 = 2 * mu * mut + C1;
                        const double f1 = 2 * (q[4] - mu * mut) + C2;
                        const double f2 = mu * mu + mut * mut + C1;
                        const double f3 = (q[2] - mu * mu) + (q[3] - mut * mut) + C2;
                        const double F = (f0 * f1) / (f2 * f3);
                        const double g0 = 2 * ww * mut;
                        const double g1 = 2 * ww * (tv - mut);
                        const double g2 = 2 * ww * mu;
                        const double g3 = 2 * ww * (cv - mu);
                        // second derivatives of f0..f3 w.r.t. this pixel's value
                        const double h2 = 2 * ww * ww, h3 = 2 * ww * (1 - ww);
                        const double Sg = g0 / f0 + g1 / f1 - g2 / f2 - g3 / f3;
                        const double dS = -(g0 * g0) / (f0 * f0) - (g1 * g1) / (f1 * f1) -
                                          (h2 * f2 - g2 * g2) / (f2 * f2) - (h3 * f3 - g3 * g3) / (f3 * f3);
                        d1 += F * Sg;
                        d2 += F * (Sg * Sg + dS);
                    }
                // L_S uses 1 - SSIM, hence the minus signs
                const double gl2 = (cv - tv) * norm;
                if (dL) dL[ch * npx + pi] = gl2 - lambda * norm * d1;
                if (hd) hd[ch * npx + pi] = norm - lambda * norm * d2;
            }
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Per-kernel derivatives.  For one pixel and one kernel k that the pixel adds,
// the colour as a function of k's own attributes is (eq. 3dgs, other kernels
// and all threshold decisions held fixed)
//     c = P + T_k (alpha_k c~_k + (1 - alpha_k) A_k),
// where P is the colour of the splats in front of k, T_k the transmittance in
// front of k and A_k the normalised colour behind k (A of the last added splat
// is the background; A_j = alpha_{j+1} c~_{j+1} + (1 - alpha_{j+1}) A_{j+1}).
// alpha_k = sigma_k G_k(pi, Q) unless it was clamped, in which case it is the
// constant alpha_max.  Gradient and Hessian of the loss follow eq.
// local_hessian_gradient with the per-pixel diagonal image Hessian h:
//     g += sum_ch dL_ch dc_ch/dy,   H += sum_ch h_ch dc_ch/dy dc_ch/dy^T + dL_ch d2c_ch/dy2.
// The local Gauss-Newton variant (the cheaper Hessian the paper's discussion of
// the position-Hessian cost (Sec. 6) points to) keeps only the first term of H:
// the image Hessian pulled back by the first derivatives of the image.
// ---------------------------------------------------------------------------
namespace {

template <int N>
void pixel_accum(const Jet<N> pi[2], const Jet<N> Q[3], const Jet<N>& sig, const Jet<N> ct[3], double x,
                 double y, double T, const double A[3], bool clamped, double amax, const double dL[3],
                 const double hd[3], bool gauss_newton, double* g, double* H) {
    const Jet<N> dx = pi[0] - x, dy = pi[1] - y;
    const Jet<N> f = -0.5 * (Q[0] * dx * dx + Q[2] * dy * dy) - Q[1] * dx * dy;
    const Jet<N> a = clamped ? Jet<N>(amax) : sig * exp(f);
    for (int ch = 0; ch < 3; ++ch) {
        const Jet<N> c = T * (a * ct[ch] + (1.0 - a) * A[ch]);
        for (int i = 0; i < N; ++i) {
            g[i] += dL[ch] * c.g[i];
            for (int j = 0; j < N; ++j)
                H[i * N + j] += hd[ch] * c.g[i] * c.g[j] + (gauss_newton ? 0.0 : dL[ch] * c.h[i][j]);
        }
    }
}

template <int N>
void to_jets(const Proj<double>& P, Jet<N> pi[2], Jet<N> Q[3], Jet<N> ct[3]) {
    for (int i = 0; i < 2; ++i) pi[i] = Jet<N>(P.pi[i]);
    for (int i = 0; i < 3; ++i) Q[i] = Jet<N>(P.Q[i]);
    for (int i = 0; i < 3; ++i) ct[i] = Jet<N>(P.ct[i]);
}

// Visit every pixel that adds kernel k: fn(x, y, T, A[3], alpha, clamped, dL[3], hd[3]).
template <class Fn>
void for_each_pixel_of(int k, const std::vector<Rec>& rec, const Cam& c, const double* o,
                       const int64_t* tile_start, const int32_t* ids, const int32_t* rect, int n,
                       const std::vector<int32_t>& all, const double* dL, const double* hd, Fn fn) {
    const bool smooth = o[O_SMOOTH] != 0.0;
    const int tile = (int)o[O_TILE];
    const int tiles_x = (c.W + tile - 1) / tile;
    const size_t npx = (size_t)c.W * c.H;
    int x0 = 0, x1 = c.W, y0 = 0, y1 = c.H;
    if (!smooth) {
        x0 = rect[k] * tile;
        y0 = rect[n + k] * tile;
        x1 = std::min(c.W, rect[2 * n + k] * tile);
        y1 = std::min(c.H, rect[3 * n + k] * tile);
    }
    std::vector<Added> added;
    for (int y = y0; y < y1; ++y)
        for (int x = x0; x < x1; ++x) {
            const int32_t* list;
            int64_t len;
            if (smooth) {
                list = all.data();
                len = (int64_t)all.size();
            } else {
                const int t = (y / tile) * tiles_x + (x / tile);
                list = ids + tile_start[t];
                len = tile_start[t + 1] - tile_start[t];
            }
            PixelOut po;
            composite_pixel(rec.data(), list, len, x, y, o, &added, po);
            int m = -1;
            for (int i = 0; i < (int)added.size(); ++i)
                if (added[i].k == k) {
                    m = i;
                    break;
                }
            if (m < 0) continue;
            double A[3] = {o[O_BG_R], o[O_BG_G], o[O_BG_B]};
            for (int i = (int)added.size() - 1; i > m; --i) {
                const Rec& r = rec[added[i].k];
                for (int ch = 0; ch < 3; ++ch) A[ch] = added[i].alpha * r.c[ch] + (1.0 - added[i].alpha) * A[ch];
            }
            const size_t pix = (size_t)y * c.W + x;
            const double dl[3] = {dL[pix], dL[npx + pix], dL[2 * npx + pix]};
            const double hh[3] = {hd[pix], hd[npx + pix], hd[2 * npx + pix]};
            fn((double)x, (double)y, added[m].T, A, added[m].alpha, added[m].clamped, dl, hh);
        }
}

}  // namespace

extern "C" {

// Number of doubles per kernel written by orc_blocks.
enum {
    B_GP = 0, B_HP = 3, B_GW = 12, B_HW = 15, B_GS = 24, B_HS = 27, B_GO = 36, B_HO = 37,
    B_W = 38, B_GAM = 39, B_SC = 42, B_R = 45, B_W2 = 48, B_COUNT = 49
};
int orc_block_count() { return B_COUNT; }

// Per-kernel gradient and Hessian blocks of one view's loss for the kernels
// in sel (eq. local_hessian_gradient), with respect to position p (3x3),
// the left rotation vector omega of the orientation (3x3; q(omega) =
// exp(omega/2) q, so the paper's rotation by theta about r_k is omega = theta r_k),
// scale s (3x3) and opacity sigma (1x1),
// plus the colour statistics that determine the SH blocks: per channel
// gamma = dL/dc~ and s = sum_pix h (alpha T)^2 (so that the SH gradient is
// gamma Y(r) and the SH Hessian s Y(r) Y(r)^T, colour being linear in the
// coefficients), the view direction r, the coverage w = sum_pix alpha T and the sum of its
// squares sum_pix (alpha T)^2 (the overlap share of the kernel is their ratio).
// dL, hd: per-pixel loss derivative maps of this view ([3][H][W]).
// rect: from orc_project32 (standard mode).  out: [nsel][B_COUNT], row-major blocks.
int orc_blocks(int n, int K, const double* pos, const double* rot, const double* scale,
               const double* opac, const double* sh, const double* cam, const double* o,
               const int64_t* tile_start, const int32_t* ids, const int32_t* rect, const double* dL,
               const double* hd, int nsel, const int32_t* sel, double* out) {
    const Scene S{pos, rot, scale, opac, sh, n, K};
    const Cam c = load_cam(cam);
    const std::vector<Rec> rec = project_all(S, c, o);
    const bool smooth = o[O_SMOOTH] != 0.0;
    const double kappa = smooth ? 0.0 : o[O_KAPPA];
    const double amax = o[O_ALPHA_MAX];
    const bool gn = o[O_GAUSS_NEWTON] != 0.0;
    std::vector<int32_t> all;
    if (smooth) all = depth_order(rec);
#pragma omp parallel for schedule(dynamic, 1)
    for (int si = 0; si < nsel; ++si) {
        const int k = sel[si];
        double* B = out + (size_t)si * B_COUNT;
        std::fill(B, B + B_COUNT, 0.0);
        if (!rec[k].ok) continue;
        double p[3], q[4], s[3], shk[48];
        for (int a = 0; a < 3; ++a) p[a] = pos[(size_t)a * n + k];
        for (int a = 0; a < 4; ++a) q[a] = rot[(size_t)a * n + k];
        for (int a = 0; a < 3; ++a) s[a] = scale[(size_t)a * n + k];
        gather_sh(S, k, shk);
        const double sigv = opac[k];
        // jets of the projection with respect to each attribute group
        Jet<3> pj[3], pq[4], ps[3];
        for (int a = 0; a < 3; ++a) { pj[a] = Jet<3>::var(p[a], a); pq[a] = Jet<3>(q[a]); ps[a] = Jet<3>(s[a]); }
        pq[3] = Jet<3>(q[3]);
        const Proj<Jet<3>> PP = project<Jet<3>>(pj, pq, ps, shk, K, c, kappa);
        // q(omega) = exp(omega/2) q with exp(omega/2) = (1 - |omega|^2/8, omega/2) to second order
        Jet<3> wp[3], wq[4], ws[3];
        {
            const Jet<3> w0 = Jet<3>::var(0.0, 0), w1 = Jet<3>::var(0.0, 1), w2 = Jet<3>::var(0.0, 2);
            const Jet<3> e0 = 1.0 - (w0 * w0 + w1 * w1 + w2 * w2) / 8.0;
            const Jet<3> e1 = 0.5 * w0, e2 = 0.5 * w1, e3 = 0.5 * w2;
            wq[0] = e0 * q[0] - e1 * q[1] - e2 * q[2] - e3 * q[3];
            wq[1] = e0 * q[1] + e1 * q[0] + e2 * q[3] - e3 * q[2];
            wq[2] = e0 * q[2] + e2 * q[0] + e3 * q[1] - e1 * q[3];
            wq[3] = e0 * q[3] + e3 * q[0] + e1 * q[2] - e2 * q[1];
        }
        for (int a = 0; a < 3; ++a) { wp[a] = Jet<3>(p[a]); ws[a] = Jet<3>(s[a]); }
        const Proj<Jet<3>> PW = project<Jet<3>>(wp, wq, ws, shk, K, c, kappa);
        Jet<3> sp[3], sq[4], ss[3];
        for (int a = 0; a < 3; ++a) { sp[a] = Jet<3>(p[a]); ss[a] = Jet<3>::var(s[a], a); }
        for (int a = 0; a < 4; ++a) sq[a] = Jet<3>(q[a]);
        const Proj<Jet<3>> PS = project<Jet<3>>(sp, sq, ss, shk, K, c, kappa);
        const Proj<double> PV = project_value(S, k, c, kappa);
        Jet<1> opi[2], oQ[3], oct[3];
        to_jets<1>(PV, opi, oQ, oct);
        const Jet<1> osig = Jet<1>::var(sigv, 0);
        const Jet<3> sig3(sigv);
        // view direction
        double d[3], dn = 0;
        for (int a = 0; a < 3; ++a) { d[a] = p[a] - c.o[a]; dn += d[a] * d[a]; }
        dn = std::sqrt(dn);
        for (int a = 0; a < 3; ++a) B[B_R + a] = d[a] / dn;
        for_each_pixel_of(k, rec, c, o, tile_start, ids, rect, n, all, dL, hd,
                          [&](double x, double y, double T, const double* A, double alpha, bool clamped,
                              const double* dl, const double* hh) {
                              pixel_accum<3>(PP.pi, PP.Q, sig3, PP.ct, x, y, T, A, clamped, amax, dl, hh, gn,
                                             B + B_GP, B + B_HP);
                              pixel_accum<3>(PW.pi, PW.Q, sig3, PW.ct, x, y, T, A, clamped, amax, dl, hh, gn,
                                             B + B_GW, B + B_HW);
                              pixel_accum<3>(PS.pi, PS.Q, sig3, PS.ct, x, y, T, A, clamped, amax, dl, hh, gn,
                                             B + B_GS, B + B_HS);
                              pixel_accum<1>(opi, oQ, osig, oct, x, y, T, A, clamped, amax, dl, hh, gn,
                                             B + B_GO, B + B_HO);
                              // colour: dc_ch/dc~_ch = alpha T, and c is linear in c~
                              for (int ch = 0; ch < 3; ++ch) {
                                  B[B_GAM + ch] += dl[ch] * alpha * T;
                                  B[B_SC + ch] += hh[ch] * (alpha * T) * (alpha * T);
                              }
                              B[B_W] += alpha * T;
                              B[B_W2] += (alpha * T) * (alpha * T);
                          });
    }
    return 0;
}

// Per-kernel gradient (9) and Hessian (9x9) of one view's loss with respect to
// the kernel's projected quantities z = (pi_x, pi_y, Q_xx, Q_xy, Q_yy, sigma,
// c~_R, c~_G, c~_B), treated as independent (Q_xy enters d^T Q d twice), plus
// the coverage.  out: [nsel][9 + 81 + 1].
int orc_zstats(int n, int K, const double* pos, const double* rot, const double* scale,
               const double* opac, const double* sh, const double* cam, const double* o,
               const int64_t* tile_start, const int32_t* ids, const int32_t* rect, const double* dL,
               const double* hd, int nsel, const int32_t* sel, double* out) {
    const Scene S{pos, rot, scale, opac, sh, n, K};
    const Cam c = load_cam(cam);
    const std::vector<Rec> rec = project_all(S, c, o);
    const bool smooth = o[O_SMOOTH] != 0.0;
    const double amax = o[O_ALPHA_MAX];
    const bool gn = o[O_GAUSS_NEWTON] != 0.0;
    std::vector<int32_t> all;
    if (smooth) all = depth_order(rec);
    const int NZ = 9 + 81 + 1;
#pragma omp parallel for schedule(dynamic, 1)
    for (int si = 0; si < nsel; ++si) {
        const int k = sel[si];
        double* Z = out + (size_t)si * NZ;
        std::fill(Z, Z + NZ, 0.0);
        if (!rec[k].ok) continue;
        const Rec& r = rec[k];
        Jet<9> pi[2] = {Jet<9>::var(r.px, 0), Jet<9>::var(r.py, 1)};
        Jet<9> Q[3] = {Jet<9>::var(r.q0, 2), Jet<9>::var(r.q1, 3), Jet<9>::var(r.q2, 4)};
        Jet<9> sig = Jet<9>::var(r.sig, 5);
        Jet<9> ct[3] = {Jet<9>::var(r.c[0], 6), Jet<9>::var(r.c[1], 7), Jet<9>::var(r.c[2], 8)};
        for_each_pixel_of(k, rec, c, o, tile_start, ids, rect, n, all, dL, hd,
                          [&](double x, double y, double T, const double* A, double alpha, bool clamped,
                              const double* dl, const double* hh) {
                              pixel_accum<9>(pi, Q, sig, ct, x, y, T, A, clamped, amax, dl, hh, gn, Z, Z + 9);
                              Z[90] += alpha * T;
                          });
    }
    return 0;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Local Newton solves in the paper's reduced coordinates (Sec. 4.2), with the
// damping rule this implementation adopts where the paper specifies none:
// Cholesky of H + mu_j I, mu_j = mu0 10^j (j = 0..max_esc), mu0 = damp_rel |H|_F /
// sqrt(n) + damp_abs / (3 |I|), accepted when every pivot exceeds pivot_min
// (|H|_F / sqrt(n) + mu_j) and min/max pivot >= pivot_min; if every attempt fails the step is the scaled
// gradient -g / (|H|_F / sqrt(n) + mu_max).  The step is then clamped to the
// group's trust radius.
// ---------------------------------------------------------------------------
namespace {

// Cholesky solve of A x = b; fails unless every pivot exceeds `floor` and
// min/max pivot >= pivot_min.
bool cholesky_solve(int n, const double* A, const double* b, double pivot_min, double* x, double floor = 0.0) {
    double L[16 * 16];
    double dmin = std::numeric_limits<double>::infinity(), dmax = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = 0; j <= i; ++j) {
            double s = A[i * n + j];
            for (int k = 0; k < j; ++k) s -= L[i * n + k] * L[j * n + k];
            if (i == j) {
                if (!(s > floor)) return false;
                dmin = std::min(dmin, s);
                dmax = std::max(dmax, s);
                L[i * n + i] = std::sqrt(s);
            } else {
                L[i * n + j] = s / L[j * n + j];
            }
        }
    }
    if (dmin < pivot_min * dmax) return false;
    double y[16];
    for (int i = 0; i < n; ++i) {
        double s = b[i];
        for (int k = 0; k < i; ++k) s -= L[i * n + k] * y[k];
        y[i] = s / L[i * n + i];
    }
    for (int i = n - 1; i >= 0; --i) {
        double s = y[i];
        for (int k = i + 1; k < n; ++k) s -= L[k * n + i] * x[k];
        x[i] = s / L[i * n + i];
    }
    return true;
}

// Solves (H + mu I) x = -g by the damping rule; returns the escalation index j
// that succeeded, or -1 for the scaled-gradient fallback.  *cond receives the
// 2-norm condition number of the matrix that was solved (1 for the fallback).
int damped_solve(int n, const double* H, const double* g, const double* o, double* x, double* cond) {
    const double abs_scale = 1.0 / (3.0 * o[O_NPIX_PRIMARY]);
    // scale of H: Frobenius norm / sqrt(n) (invariant to the choice of reduced basis,
    // positive for indefinite H)
    double ma = 0.0;
    for (int i = 0; i < n * n; ++i) ma += H[i] * H[i];
    ma = std::sqrt(ma / n);
    const double mu0 = o[O_DAMP_REL] * ma + o[O_DAMP_ABS] * abs_scale;
    const int jmax = (int)o[O_MAX_ESC];
    double A[16 * 16], b[16];
    for (int i = 0; i < n; ++i) b[i] = -g[i];
    double mu = mu0;
    for (int j = 0; j <= jmax; ++j) {
        for (int i = 0; i < n * n; ++i) A[i] = H[i];
        for (int i = 0; i < n; ++i) A[i * n + i] += mu;
        // a pivot must also exceed pivot_min times the size of H + mu I, so that an
        // indefinite H shifted to (nearly) singular is not accepted
        if (cholesky_solve(n, A, b, o[O_PIVOT_MIN], x, o[O_PIVOT_MIN] * (ma + mu))) {
            *cond = 1.0;
            if (n == 2) {
                const double mid = 0.5 * (A[0] + A[3]), rad = std::sqrt(0.25 * (A[0] - A[3]) * (A[0] - A[3]) + A[1] * A[1]);
                *cond = (mid + rad) / (mid - rad);
            }
            return j;
        }
        if (j < jmax) mu *= 10.0;
    }
    const double den = ma + mu;
    for (int i = 0; i < n; ++i) x[i] = -g[i] / den;
    *cond = 1.0;
    return -1;
}

// Radial trust-region clamp: scales x so that |x| <= radius.
void clamp_norm(int n, double* x, double radius) {
    double nn = 0.0;
    for (int i = 0; i < n; ++i) nn += x[i] * x[i];
    nn = std::sqrt(nn);
    if (nn > radius && nn > 0.0)
        for (int i = 0; i < n; ++i) x[i] *= radius / nn;
}

void quat_mul(const double a[4], const double b[4], double r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    r[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}

}  // namespace

extern "C" {

// Summed-block layout consumed by orc_solve: per kernel
//   g_p 3 | H_p 9 | g_omega 3 | H_omega 9 | g_s 3 | H_s 9 | g_sig | H_sig | w_primary   (39)
// followed by V view records (gamma 3 | s 3 | r 3 | w 1).
// Step layout: dpos 3 | dtheta | axis 3 | dscale 3 | dopac | dsh [3][K]   (11 + 3K)
// Decisions [n][5]: escalation index for (position, rotation, scale, opacity),
// -1 = gradient fallback, -2 = kernel not visible in the primary (no step);
// the fifth entry is the number of views used by the colour solve.
// cond [n][4] (may be NULL): condition number of each group's solved matrix.
// Every step is then clamped to its group's trust radius.
enum { S_COUNT_BASE = 39, S_VIEW = 10, ST_DPOS = 0, ST_DTH = 3, ST_AXIS = 4, ST_DS = 7, ST_DO = 10, ST_DSH = 11 };

}  // extern "C"

namespace {

// The reduced local systems of one kernel (Sec. 4.2, position / rotation / scaling /
// opacity paragraphs) built from its summed blocks B in the primary camera's frame:
//   position: U = [u_x u_y] orthonormal in the plane normal to the view axis r,
//             H = U^T H_p U, g = U^T g_p;
//   rotation: the left rotation omega = theta r: H = r^T H_omega r, g = r . g_omega;
//   scaling:  the rows of T = d lambda / d s (unit length), H = T H_s T^T, g = T g_s;
//   opacity:  H_sigma + h_B, g_sigma + g_B with the log barrier.
struct Reduced {
    double r[3], ux[3], uy[3];
    double Hp[4], gp[2];
    double Ht, gt;
    double T2[2][3], Hs[4], gs[2];
    double Ho, go;
};

void reduce_systems(const double* B, const double p[3], const double q[4], const double s[3], double sig,
                    const Cam& c, double kappa, const double* o, double abs_scale, Reduced& R) {
    double rn = 0.0;
    for (int a = 0; a < 3; ++a) { R.r[a] = p[a] - c.o[a]; rn += R.r[a] * R.r[a]; }
    rn = std::sqrt(rn);
    for (int a = 0; a < 3; ++a) R.r[a] /= rn;
    const double* r = R.r;
    // position
    {
        double* uy = R.uy;
        uy[0] = -r[1] * r[0]; uy[1] = 1.0 - r[1] * r[1]; uy[2] = -r[1] * r[2];  // (I - r r^T) e_y
        double nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        if (nn < 1e-12) {
            uy[0] = 1.0 - r[0] * r[0]; uy[1] = -r[0] * r[1]; uy[2] = -r[0] * r[2];
            nn = uy[0] * uy[0] + uy[1] * uy[1] + uy[2] * uy[2];
        }
        nn = std::sqrt(nn);
        for (int a = 0; a < 3; ++a) uy[a] /= nn;
        double* ux = R.ux;
        ux[0] = r[1] * uy[2] - r[2] * uy[1]; ux[1] = r[2] * uy[0] - r[0] * uy[2]; ux[2] = r[0] * uy[1] - r[1] * uy[0];
        const double* U[2] = {ux, uy};
        for (int i = 0; i < 2; ++i) {
            R.gp[i] = 0.0;
            for (int a = 0; a < 3; ++a) R.gp[i] += U[i][a] * B[0 + a];
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += U[i][a] * B[3 + a * 3 + b] * U[j][b];
                R.Hp[i * 2 + j] = acc;
            }
        }
    }
    // rotation
    R.gt = 0.0;
    R.Ht = 0.0;
    for (int a = 0; a < 3; ++a) {
        R.gt += r[a] * B[12 + a];
        for (int b = 0; b < 3; ++b) R.Ht += r[a] * B[15 + a * 3 + b] * r[b];
    }
    // scaling
    {
        double sp[3] = {p[0], p[1], p[2]}, sq[4] = {q[0], q[1], q[2], q[3]}, ss[3] = {s[0], s[1], s[2]};
        double shk0[48] = {0};
        const Proj<double> P = project<double>(sp, sq, ss, shk0, 1, c, kappa);
        double (*T2)[3] = R.T2;
        for (int i = 0; i < 2; ++i)
            for (int a = 0; a < 3; ++a) T2[i][a] = 0.0;
        if (P.ok) {
            const double a_ = P.cov[0], b_ = P.cov[1], c_ = P.cov[2];
            const double mid = 0.5 * (a_ + c_), rad = std::sqrt(0.25 * (a_ - c_) * (a_ - c_) + b_ * b_);
            const double l2 = mid + rad;
            double v2[2];
            if (a_ >= c_) { v2[0] = l2 - c_; v2[1] = b_; } else { v2[0] = b_; v2[1] = l2 - a_; }
            double vn = std::sqrt(v2[0] * v2[0] + v2[1] * v2[1]);
            if (vn == 0.0) { v2[0] = 1.0; v2[1] = 0.0; vn = 1.0; }
            v2[0] /= vn; v2[1] /= vn;
            const double v1[2] = {-v2[1], v2[0]};
            // M = J W and the rotation of the kernel at the current state
            double t3[3];
            for (int i = 0; i < 3; ++i) t3[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
            const double iz = 1.0 / t3[2];
            const double J00 = c.fx * iz, J02 = -c.fx * t3[0] * iz * iz, J11 = c.fy * iz, J12 = -c.fy * t3[1] * iz * iz;
            double M[2][3];
            for (int kk = 0; kk < 3; ++kk) {
                M[0][kk] = J00 * c.R[kk] + J02 * c.R[6 + kk];
                M[1][kk] = J11 * c.R[3 + kk] + J12 * c.R[6 + kk];
            }
            const double qn = std::sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
            const double w = q[0] / qn, x = q[1] / qn, y = q[2] / qn, z = q[3] / qn;
            const double Rq[3][3] = {{1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)},
                                     {2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)},
                                     {2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)}};
            const double* vv[2] = {v1, v2};  // rows: lambda_min, lambda_max
            for (int i = 0; i < 2; ++i) {
                for (int a = 0; a < 3; ++a) {
                    double e = 0.0;  // v_i^T M R e_a
                    for (int b = 0; b < 2; ++b)
                        for (int kk = 0; kk < 3; ++kk) e += vv[i][b] * M[b][kk] * Rq[kk][a];
                    T2[i][a] = 2.0 * s[a] * e * e;
                }
                // only the row space of T matters; unit rows keep the reduced system well scaled
                const double tn = std::sqrt(T2[i][0] * T2[i][0] + T2[i][1] * T2[i][1] + T2[i][2] * T2[i][2]);
                if (tn > 0.0)
                    for (int a = 0; a < 3; ++a) T2[i][a] /= tn;
            }
        }
        for (int i = 0; i < 2; ++i) {
            R.gs[i] = 0.0;
            for (int a = 0; a < 3; ++a) R.gs[i] += T2[i][a] * B[24 + a];
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int a = 0; a < 3; ++a)
                    for (int b = 0; b < 3; ++b) acc += T2[i][a] * B[27 + a * 3 + b] * T2[j][b];
                R.Hs[i * 2 + j] = acc;
            }
        }
    }
    // opacity with the log barrier -alpha_s [ln sigma + ln(1 - sigma)]
    {
        const double as = o[O_BARRIER_BETA] * abs_scale;
        const double gB = as * (1.0 / (1.0 - sig) - 1.0 / sig);
        const double hB = as * (1.0 / (sig * sig) + 1.0 / ((1.0 - sig) * (1.0 - sig)));
        R.Ho = B[37] + hB;
        R.go = B[36] + gB;
    }
}

}  // namespace

extern "C" {

int orc_solve(int n, int K, const double* pos, const double* rot, const double* scale, const double* opac,
              const double* cam, const double* o, int V, const double* blocks, double* steps, int32_t* dec,
              double* cond) {
    const Cam c = load_cam(cam);
    // the summed blocks: base, V view slots, then the sum over views of sum_pix (alpha T)^2
    const int NB = S_COUNT_BASE + V * S_VIEW + 1, NS = 11 + 3 * K;
    const double kappa = o[O_SMOOTH] != 0.0 ? 0.0 : o[O_KAPPA];
    const double abs_scale = 1.0 / (3.0 * o[O_NPIX_PRIMARY]);
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        const double* B = blocks + (size_t)k * NB;
        double* st = steps + (size_t)k * NS;
        int32_t* dk = dec + (size_t)k * 5;
        double cnd[4] = {1.0, 1.0, 1.0, 1.0};
        std::fill(st, st + NS, 0.0);
        for (int i = 0; i < 5; ++i) dk[i] = -2;
        if (cond)
            for (int i = 0; i < 4; ++i) cond[(size_t)k * 4 + i] = 1.0;
        if (!(B[38] > 0.0)) continue;  // only kernels the primary target sees are trained
        double p[3], q[4], s[3];
        for (int a = 0; a < 3; ++a) p[a] = pos[(size_t)a * n + k];
        for (int a = 0; a < 4; ++a) q[a] = rot[(size_t)a * n + k];
        for (int a = 0; a < 3; ++a) s[a] = scale[(size_t)a * n + k];
        const double sig = opac[k];
        const double frac = o[O_STEP_FRAC];
        // overlap share (when asked for): every kernel's Newton step holds the other kernels fixed;
        // where several composite into the same pixels their steps add up there.  The share
        // omega = sum (alpha T)^2 / sum alpha T over the kernel's pixels in all views is at most its
        // Gershgorin ratio H_kk / sum_j |H_kj| for the colour system (sum_j alpha_j T_j = 1 - T_final
        // <= 1 at every pixel).  It multiplies the kernel's steps after the trust radii.
        double omega = 1.0;
        if (o[O_OVERLAP] != 0.0) {
            double cov = 0.0;
            for (int v = 0; v < V; ++v) cov += B[S_COUNT_BASE + v * S_VIEW + 9];
            const double w2 = B[S_COUNT_BASE + V * S_VIEW];
            omega = cov > 0.0 ? std::min(1.0, std::max(0.0, w2 / cov)) : 0.0;
        }
        Reduced R;
        reduce_systems(B, p, q, s, sig, c, kappa, o, abs_scale, R);
        for (int a = 0; a < 3; ++a) st[ST_AXIS + a] = R.r[a];
        // position: Delta p = U Delta v
        {
            double H2[4] = {R.Hp[0], R.Hp[1], R.Hp[2], R.Hp[3]}, dv[2];
            dk[0] = damped_solve(2, H2, R.gp, o, dv, &cnd[0]);
            for (int a = 0; a < 2; ++a) dv[a] *= frac;
            clamp_norm(2, dv, o[O_TRUST_POS] * std::max(s[0], std::max(s[1], s[2])));
            for (int a = 0; a < 3; ++a) st[ST_DPOS + a] = omega * (R.ux[a] * dv[0] + R.uy[a] * dv[1]);
        }
        // rotation: q(theta) = dq(theta) * q with dq = [cos(theta/2), sin(theta/2) r]
        {
            double th;
            dk[1] = damped_solve(1, &R.Ht, &R.gt, o, &th, &cnd[1]);
            th *= frac;
            clamp_norm(1, &th, o[O_TRUST_ROT]);
            st[ST_DTH] = omega * th;
        }
        // scaling: Delta s = T^T a
        {
            double av[2];
            dk[2] = damped_solve(2, R.Hs, R.gs, o, av, &cnd[2]);
            for (int a = 0; a < 2; ++a) av[a] *= frac;
            // the rows of T are unit but not orthogonal, so the clamp acts on Delta s itself
            double dsv[3];
            for (int a = 0; a < 3; ++a) dsv[a] = R.T2[0][a] * av[0] + R.T2[1][a] * av[1];
            clamp_norm(3, dsv, o[O_TRUST_SCALE] * std::sqrt(s[0] * s[0] + s[1] * s[1] + s[2] * s[2]));
            for (int a = 0; a < 3; ++a) st[ST_DS + a] = omega * dsv[a];
        }
        // opacity with the log barrier
        {
            double ds;
            dk[3] = damped_solve(1, &R.Ho, &R.go, o, &ds, &cnd[3]);
            st[ST_DO] = omega * (frac * ds);
        }
        // Colour: per channel, G = sum_v s~_v b_v b_v^T, g = sum_v gamma_v b_v, b_v = Y(r_v).
        {
            int nv = 0;
            for (int v = 0; v < V; ++v)
                if (B[S_COUNT_BASE + v * S_VIEW + 9] > 0.0) ++nv;
            dk[4] = nv;
            for (int ch = 0; ch < 3; ++ch) {
                double smax = 0.0;
                for (int v = 0; v < V; ++v) {
                    const double* vb = B + S_COUNT_BASE + v * S_VIEW;
                    if (vb[9] > 0.0) smax = std::max(smax, std::fabs(vb[3 + ch]));
                }
                if (!(smax > 0.0)) continue;
                double G[256] = {0}, gg[16] = {0}, Y[16];
                for (int v = 0; v < V; ++v) {
                    const double* vb = B + S_COUNT_BASE + v * S_VIEW;
                    if (!(vb[9] > 0.0)) continue;
                    sh_basis<double>(K, vb[6], vb[7], vb[8], Y);
                    const double sv = std::max(std::fabs(vb[3 + ch]), o[O_SH_FLOOR] * smax);
                    for (int i = 0; i < K; ++i) {
                        gg[i] += vb[ch] * Y[i];
                        for (int j = 0; j < K; ++j) G[i * K + j] += sv * Y[i] * Y[j];
                    }
                }
                double md = 0.0;
                for (int i = 0; i < K; ++i) md += G[i * K + i];
                md /= K;
                const double mu = o[O_DAMP_SH] * md + o[O_DAMP_ABS] * abs_scale;
                for (int i = 0; i < K; ++i) G[i * K + i] += mu;
                double x[16], b[16];
                for (int i = 0; i < K; ++i) b[i] = -gg[i];
                if (cholesky_solve(K, G, b, 0.0, x)) {
                    for (int i = 0; i < K; ++i) x[i] *= frac;
                    clamp_norm(K, x, o[O_TRUST_SH]);
                    for (int i = 0; i < K; ++i) st[ST_DSH + ch * K + i] = omega * x[i];
                }
            }
        }
        if (cond)
            for (int i = 0; i < 4; ++i) cond[(size_t)k * 4 + i] = cnd[i];
    }
    return 0;
}

// Features of the learned step scale (one 17-vector per kernel) from the summed blocks of
// the primary view alone, in the reduced coordinates of the solve, and the cached
// neighbouring-view residual.  With
// L(x) = log10(x + 1e-30) / 10:
//   0, 1  L(|lambda|) of the larger / smaller eigenvalue of the reduced position Hessian,
//   2     sign of its smaller eigenvalue (+1 when >= 0),
//   3, 4  L(|H_theta|), sign of H_theta,
//   5, 6  L(|lambda|) of the reduced scaling Hessian's eigenvalues (larger, smaller),
//   7     sign of its smaller eigenvalue,
//   8     L(|H_sigma + h_B|),
//   9     L(sum over channels of |s|, the primary view's colour Hessian diagonal),
//   10    L(primary coverage w),
//   11-14 L(|g|) of the reduced position, rotation, scaling and opacity gradients,
//   15    L(opacity),
//   16    L(resid[k]) (resid may be null: 0), the neighbouring-view residual of the kernel's
//         last full-rule sweep.
// ok[k] = 0 when the kernel is not visible in the primary view, else 1 when every L argument lies
// in [1e-30, 1e30] (so that no feature leaves [-3, 3]) and 2 when one does not.
int orc_features(int n, int K, const double* pos, const double* rot, const double* scale, const double* opac,
                 const double* cam, const double* o, int V, const double* blocks, const double* resid, double* feat,
                 uint8_t* ok) {
    const Cam c = load_cam(cam);
    const int NB = S_COUNT_BASE + V * S_VIEW + 1;
    const double kappa = o[O_SMOOTH] != 0.0 ? 0.0 : o[O_KAPPA];
    const double abs_scale = 1.0 / (3.0 * o[O_NPIX_PRIMARY]);
    (void)K;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        const double* B = blocks + (size_t)k * NB;
        double* f = feat + (size_t)k * 17;
        std::fill(f, f + 17, 0.0);
        ok[k] = 0;
        if (!(B[38] > 0.0)) continue;
        double p[3], q[4], s[3];
        for (int a = 0; a < 3; ++a) p[a] = pos[(size_t)a * n + k];
        for (int a = 0; a < 4; ++a) q[a] = rot[(size_t)a * n + k];
        for (int a = 0; a < 3; ++a) s[a] = scale[(size_t)a * n + k];
        Reduced R;
        reduce_systems(B, p, q, s, opac[k], c, kappa, o, abs_scale, R);
        bool in_range = true;
        auto L = [&](double x) {
            const double v = std::log10(x + 1e-30) / 10.0;
            if (!(v >= -3.0 && v <= 3.0)) in_range = false;
            return std::min(3.0, std::max(-3.0, v));
        };
        auto eig2 = [](const double* H, double& hi, double& lo) {
            const double mid = 0.5 * (H[0] + H[3]);
            const double rad = std::sqrt(0.25 * (H[0] - H[3]) * (H[0] - H[3]) + H[1] * H[1]);
            hi = mid + rad;
            lo = mid - rad;
        };
        double hi, lo;
        eig2(R.Hp, hi, lo);
        f[0] = L(std::fabs(hi));
        f[1] = L(std::fabs(lo));
        f[2] = lo >= 0.0 ? 1.0 : -1.0;
        f[3] = L(std::fabs(R.Ht));
        f[4] = R.Ht >= 0.0 ? 1.0 : -1.0;
        eig2(R.Hs, hi, lo);
        f[5] = L(std::fabs(hi));
        f[6] = L(std::fabs(lo));
        f[7] = lo >= 0.0 ? 1.0 : -1.0;
        f[8] = L(std::fabs(R.Ho));
        f[9] = L(std::fabs(B[S_COUNT_BASE + 3]) + std::fabs(B[S_COUNT_BASE + 4]) + std::fabs(B[S_COUNT_BASE + 5]));
        f[10] = L(B[38]);
        f[11] = L(std::sqrt(R.gp[0] * R.gp[0] + R.gp[1] * R.gp[1]));
        f[12] = L(std::fabs(R.gt));
        f[13] = L(std::sqrt(R.gs[0] * R.gs[0] + R.gs[1] * R.gs[1]));
        f[14] = L(std::fabs(R.go));
        f[15] = L(opac[k]);
        f[16] = L(resid ? resid[k] : 0.0);
        ok[k] = in_range ? 1 : 2;  // 0: not seen by the primary, 1: features in range, 2: seen, out of range
    }
    return 0;
}

// Applies the steps in the group order position, rotation, scaling, opacity,
// colour (bits 0..4 of group_mask).  Parameters are updated in place (FP64).
int orc_apply(int n, int K, double* pos, double* rot, double* scale, double* opac, double* sh,
              const double* o, const double* steps, const int32_t* dec, int group_mask) {
    const int NS = 11 + 3 * K;
#pragma omp parallel for schedule(static)
    for (int k = 0; k < n; ++k) {
        const double* st = steps + (size_t)k * NS;
        if (dec[(size_t)k * 5] == -2) continue;
        if (group_mask & 1)
            for (int a = 0; a < 3; ++a) pos[(size_t)a * n + k] += st[ST_DPOS + a];
        if (group_mask & 2) {
            const double th = st[ST_DTH];
            const double dq[4] = {std::cos(0.5 * th), std::sin(0.5 * th) * st[ST_AXIS],
                                  std::sin(0.5 * th) * st[ST_AXIS + 1], std::sin(0.5 * th) * st[ST_AXIS + 2]};
            double q[4], r[4];
            for (int a = 0; a < 4; ++a) q[a] = rot[(size_t)a * n + k];
            quat_mul(dq, q, r);
            const double rn = std::sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
            for (int a = 0; a < 4; ++a) rot[(size_t)a * n + k] = r[a] / rn;
        }
        if (group_mask & 4)
            for (int a = 0; a < 3; ++a) {
                const double s = scale[(size_t)a * n + k];
                scale[(size_t)a * n + k] = std::max(s + st[ST_DS + a], o[O_SCALE_FLOOR] * s);
            }
        if (group_mask & 8) {
            const double sg = opac[k], f = o[O_OPAC_FTB];
            const double moved = std::min(std::max(sg + st[ST_DO], sg - f * sg), sg + f * (1.0 - sg));
            opac[k] = std::min(std::max(moved, o[O_OPAC_EPS]), 1.0 - o[O_OPAC_EPS]);
        }
        if (group_mask & 16)
            for (int i = 0; i < 3 * K; ++i) sh[(size_t)i * n + k] += st[ST_DSH + i];
    }
    return 0;
}

// Camera KNN on the bounding sphere (Sec. 4.1): camera centres are projected
// radially onto a sphere about the scene centre and compared by great-circle
// distance (the radius only scales it).  Self excluded, ties by lower index.
int orc_knn(int ncam, const double* centers, const double* scene_center, int K, int32_t* out) {
    std::vector<double> u(3 * (size_t)ncam);
    for (int i = 0; i < ncam; ++i) {
        double d[3], nn = 0;
        for (int a = 0; a < 3; ++a) { d[a] = centers[3 * i + a] - scene_center[a]; nn += d[a] * d[a]; }
        nn = std::sqrt(nn);
        for (int a = 0; a < 3; ++a) u[3 * i + a] = d[a] / nn;
    }
    for (int i = 0; i < ncam; ++i) {
        std::vector<std::pair<double, int>> dist;
        for (int j = 0; j < ncam; ++j) {
            if (j == i) continue;
            double dot = u[3 * i] * u[3 * j] + u[3 * i + 1] * u[3 * j + 1] + u[3 * i + 2] * u[3 * j + 2];
            dot = std::min(1.0, std::max(-1.0, dot));
            dist.push_back({std::acos(dot), j});
        }
        std::sort(dist.begin(), dist.end());
        for (int k = 0; k < K; ++k) out[(size_t)i * K + k] = k < (int)dist.size() ? dist[k].second : -1;
    }
    return 0;
}

// FP64 projection of every kernel (for tests): out [n][12] =
// pi_x, pi_y, Sigma_xx, Sigma_xy, Sigma_yy, Q_xx, Q_xy, Q_yy, c~_R, c~_G, c~_B, depth; ok [n].
int orc_project64(int n, int K, const double* pos, const double* rot, const double* scale,
                  const double* opac, const double* sh, const double* cam, double kappa, double* out,
                  uint8_t* ok) {
    const Scene S{pos, rot, scale, opac, sh, n, K};
    const Cam c = load_cam(cam);
    for (int k = 0; k < n; ++k) {
        const Proj<double> P = project_value(S, k, c, kappa);
        double* r = out + (size_t)k * 12;
        r[0] = P.pi[0]; r[1] = P.pi[1];
        for (int i = 0; i < 3; ++i) { r[2 + i] = P.cov[i]; r[5 + i] = P.Q[i]; r[8 + i] = P.ct[i]; }
        r[11] = P.depth;
        ok[k] = P.ok ? 1 : 0;
    }
    return 0;
}

// Smooth-mode composite straight from projected records (for tests):
// rec [n][10] = pi_x, pi_y, Q_xx, Q_xy, Q_yy, sigma, c~_R, c~_G, c~_B, depth.
// Every record is composited at every pixel in depth order; img [3][H][W].
int orc_render_z(int n, const double* recs, int W, int H, const double* bg, double* img) {
    std::vector<Rec> rec(n);
    for (int k = 0; k < n; ++k) {
        const double* r = recs + (size_t)k * 10;
        rec[k] = Rec{r[0], r[1], r[2], r[3], r[4], r[5], {r[6], r[7], r[8]}, r[9], true};
    }
    const std::vector<int32_t> all = depth_order(rec);
    double o[O_COUNT] = {0};
    o[O_SMOOTH] = 1.0;
    o[O_BG_R] = bg[0]; o[O_BG_G] = bg[1]; o[O_BG_B] = bg[2];
    const size_t npx = (size_t)W * H;
    for (int y = 0; y < H; ++y)
        for (int x = 0; x < W; ++x) {
            PixelOut po;
            composite_pixel(rec.data(), all.data(), (int64_t)all.size(), x, y, o, nullptr, po);
            for (int ch = 0; ch < 3; ++ch) img[ch * npx + (size_t)y * W + x] = po.C[ch];
        }
    return 0;
}

// 2x2 box downsampling of a [3][H][W] image to [3][H/2][W/2] (secondary targets, Sec. 4.3).
void orc_downsample(int W, int H, const double* src, double* dst) {
    const int w2 = W / 2, h2 = H / 2;
    for (int ch = 0; ch < 3; ++ch)
        for (int y = 0; y < h2; ++y)
            for (int x = 0; x < w2; ++x) {
                const double* s = src + (size_t)ch * W * H;
                dst[((size_t)ch * h2 + y) * w2 + x] =
                    0.25 * (s[(size_t)(2 * y) * W + 2 * x] + s[(size_t)(2 * y) * W + 2 * x + 1] +
                            s[(size_t)(2 * y + 1) * W + 2 * x] + s[(size_t)(2 * y + 1) * W + 2 * x + 1]);
            }
}

}  // extern "C"
