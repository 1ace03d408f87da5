// device_common.h -- device helpers shared by the gfx950 kernels of libgsn.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#ifndef GSN_HD
#define GSN_HD __host__ __device__
#endif

#define GSN_TILE 16
#define GSN_BLOCK 256          // threads per tile workgroup (16 x 16 pixels, four wave64s)
#define GSN_NZ 48              // per-kernel projected-space statistics (44 used, then the sum of
                               // squared contribution weights, then zero padding), see backward.hip
#define GSN_ZCOV 43            // index of the coverage sum alpha T among the statistics
#define GSN_ZW2 44             // index of the sum of (alpha T)^2

// Kernel-space camera (floats) passed by value to kernels.
struct DevCam {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    float o[3];  // camera centre -R^T t
    int W, H, tiles_x, tiles_y;
    float znear;
};

struct DevRenderOpts {
    float alpha_min, alpha_max, T_min, kappa, radius_sigma;
    float bg[3];
};

// ----------------------------------------------------------------------------
// Splat records are kept in each splat's principal-axis frame: the eigenvectors
// of its 2D covariance, e1 = (c, s) and e2 = (-s, c), with eigenvalues
// lambda1 >= lambda2, so that the conic is Q' = diag(q1, q2), q_i = 1/lambda_i.
// Record (three float4 per kernel):
//   (mx, my, q1, q2), (c, s, sigma, colour_R), (colour_G, colour_B, mx_lo, my_lo),
// where the mean is mx + mx_lo, my + my_lo (a float pair carrying double precision).
// Working in this frame keeps the per-pixel derivative terms of thin splats
// well conditioned (in the image frame their conic derivatives are nearly
// collinear and rounding destroys the minor directions).
//
// Alpha of one splat at one pixel: alpha = min(alpha_max, sigma exp(-d'^T Q' d' / 2)),
// d' = V^T (m - x).  Forward and backward passes call this same function so
// that their skip and stop decisions agree exactly.
// ----------------------------------------------------------------------------
struct SplatEval {
    float G, alpha, d1, d2;  // d1, d2: offset from the pixel in the principal frame
    bool clamped;
};

__device__ __forceinline__ SplatEval eval_splat(const float4 a, const float4 b, const float4 c4, float px,
                                                float py, float amax) {
    SplatEval e;
    const float mx = a.x, my = a.y, q1 = a.z, q2 = a.w, c = b.x, s = b.y, sig = b.z;
    // mx - px is exact near the splat (Sterbenz), so the offset keeps the low word's precision
    const float dx = (mx - px) + c4.z, dy = (my - py) + c4.w;
    e.d1 = c * dx + s * dy;
    e.d2 = c * dy - s * dx;
    const float power = -0.5f * (q1 * e.d1 * e.d1 + q2 * e.d2 * e.d2);
    e.G = __expf(power);
    const float al = sig * e.G;
    e.clamped = al > amax;
    e.alpha = e.clamped ? amax : al;
    return e;
}

// Axis-aligned box (x_lo, x_hi, y_lo, y_hi), in pixel coordinates, that holds every
// pixel centre at which the splat can reach alpha >= alpha_min: the ellipse
// d'^T Q' d' <= 2 ln(sigma / alpha_min), widened by a relative 1e-3 and 0.02 px so
// that single-precision rounding of the per-pixel test can never reach outside it.
// A splat with sigma < alpha_min composites nowhere (empty box).  Used to skip list
// entries for a whole wave without changing any per-pixel decision.
__device__ __forceinline__ float4 splat_alpha_box(const float4 a, const float4 b, const float4 c4, float alpha_min) {
    const float sig = b.z;
    if (!(sig >= alpha_min)) return make_float4(1.f, -1.f, 1.f, -1.f);
    const float r2 = 2.0f * __logf(sig / alpha_min);
    const float c = b.x, s = b.y, i1 = 1.0f / a.z, i2 = 1.0f / a.w;
    const float ex = sqrtf(fmaxf(r2, 0.f) * (c * c * i1 + s * s * i2)) * 1.001f + 0.02f;
    const float ey = sqrtf(fmaxf(r2, 0.f) * (s * s * i1 + c * c * i2)) * 1.001f + 0.02f;
    const float mx = a.x + c4.z, my = a.y + c4.w;
    return make_float4(mx - ex, mx + ex, my - ey, my + ey);
}

// True when the box misses the pixel rows y0..y1 and columns x0..x1 (inclusive).
__device__ __forceinline__ bool box_misses(const float4 box, float x0, float x1, float y0, float y1) {
    return box.y < x0 || box.x > x1 || box.w < y0 || box.z > y1;
}

// True when no pixel centre of columns x0..x1, rows y0..y1 can reach alpha >= alpha_min: the
// minimum of the splat's quadratic form over the rectangle (its centre if inside, else the
// smallest of the four edges' minima, each at its clamped 1D minimiser, evaluated in the
// principal frame as the per-pixel test does) exceeds 2 ln(sigma / alpha_min) by more than a
// relative 1e-3 and 0.01 (far above single-precision rounding of the per-pixel test, and of
// the mean's two words added here).  Tighter than the bounding box for thin, rotated splats.
__device__ __forceinline__ bool ellipse_misses(const float4 a, const float4 b, const float4 c4, float alpha_min,
                                               float x0, float x1, float y0, float y1) {
    const float sig = b.z;
    if (!(sig >= alpha_min)) return true;
    const float r2 = 2.0f * __logf(sig / alpha_min);
    const float q1 = a.z, q2 = a.w, c = b.x, s = b.y;
    const float qxx = q1 * c * c + q2 * s * s, qyy = q1 * s * s + q2 * c * c, qxy = (q1 - q2) * c * s;
    const float mx = a.x + c4.z, my = a.y + c4.w;
    const float X0 = x0 - mx, X1 = x1 - mx, Y0 = y0 - my, Y1 = y1 - my;
    if (X0 <= 0.f && X1 >= 0.f && Y0 <= 0.f && Y1 >= 0.f) return false;
    auto q = [&](float X, float Y) {
        const float u1 = c * X + s * Y, u2 = c * Y - s * X;
        return q1 * u1 * u1 + q2 * u2 * u2;
    };
    const float m0 = q(X0, fminf(fmaxf(-qxy * X0 / qyy, Y0), Y1));
    const float m1 = q(X1, fminf(fmaxf(-qxy * X1 / qyy, Y0), Y1));
    const float m2 = q(fminf(fmaxf(-qxy * Y0 / qxx, X0), X1), Y0);
    const float m3 = q(fminf(fmaxf(-qxy * Y1 / qxx, X0), X1), Y1);
    return fminf(fminf(m0, m1), fminf(m2, m3)) > r2 * 1.001f + 0.01f;
}

// Principal frame of Sigma = A A^T + kappa I (A = J W R S, 2x3): eigenvalues from the
// trace and the Cauchy-Binet determinant (sum of squared 2x2 minors), the minor one as
// det / lambda1 so that neither cancels.
template <class T>
GSN_HD inline void principal_frame(const T A[2][3], T kappa, T& l1, T& l2, T& c, T& s) {
    const T sxx = A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2] + kappa;
    const T syy = A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2] + kappa;
    const T sxy = A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2];
    const T m01 = A[0][0] * A[1][1] - A[0][1] * A[1][0];
    const T m02 = A[0][0] * A[1][2] - A[0][2] * A[1][0];
    const T m12 = A[0][1] * A[1][2] - A[0][2] * A[1][1];
    const T det = m01 * m01 + m02 * m02 + m12 * m12 + kappa * (sxx + syy - kappa);
    const T half = T(0.5) * (sxx - syy);
    const T rad = sqrt(half * half + sxy * sxy);
    l1 = T(0.5) * (sxx + syy) + rad;
    l2 = det / l1;
    // eigenvector of l1: the better conditioned of (l1 - syy, sxy) and (sxy, l1 - sxx)
    T vx = l1 - syy, vy = sxy;
    if (fabs(sxy) + fabs(l1 - sxx) > fabs(vx) + fabs(vy)) {
        vx = sxy;
        vy = l1 - sxx;
    }
    const T vn = sqrt(vx * vx + vy * vy);
    if (vn > T(0)) {
        c = vx / vn;
        s = vy / vn;
    } else {
        c = T(1);
        s = T(0);
    }
}

// ----------------------------------------------------------------------------
// View-dependent colour basis Y_i = B_i Phi_i(r) (Appendix A.2 polynomials,
// real-SH normalisation constants), K = 1, 4, 9 or 16.
// ----------------------------------------------------------------------------
#define SH_C0 0.28209479177387814f
#define SH_C1 0.48860251190291992f
#define SH_C2A 1.09254843059207907f
#define SH_C2B 0.31539156525252005f
#define SH_C2C 0.54627421529603959f
#define SH_C3A 0.59004358992664352f
#define SH_C3B 2.89061144264055405f
#define SH_C3C 0.45704579946446573f
#define SH_C3D 0.37317633259011546f
#define SH_C3E 1.44530572132027737f

// Quaternion product r = a b, (w, x, y, z) order.
template <class T>
GSN_HD inline void qmul(const T a[4], const T b[4], T r[4]) {
    r[0] = a[0] * b[0] - a[1] * b[1] - a[2] * b[2] - a[3] * b[3];
    r[1] = a[0] * b[1] + b[0] * a[1] + a[2] * b[3] - a[3] * b[2];
    r[2] = a[0] * b[2] + b[0] * a[2] + a[3] * b[1] - a[1] * b[3];
    r[3] = a[0] * b[3] + b[0] * a[3] + a[1] * b[2] - a[2] * b[1];
}

// Visits (i, Y_i) for i < K in order, so that callers accumulate without holding an
// array of basis values (jets of 16 basis functions would not fit in registers).
template <class T, class F>
GSN_HD inline void sh_basis_visit(int K, const T& x, const T& y, const T& z, F f) {
    f(0, T(SH_C0));
    if (K <= 1) return;
    f(1, -SH_C1 * y);
    f(2, SH_C1 * z);
    f(3, -SH_C1 * x);
    if (K <= 4) return;
    const T xx = x * x, yy = y * y, zz = z * z;
    f(4, SH_C2A * (x * y));
    f(5, SH_C2A * (y * z));
    f(6, SH_C2B * (2.0f * zz - xx - yy));
    f(7, SH_C2A * (x * z));
    f(8, SH_C2C * (xx - yy));
    if (K <= 9) return;
    f(9, SH_C3A * (y * (3.0f * xx - yy)));
    f(10, SH_C3B * (x * y * z));
    f(11, SH_C3C * (y * (4.0f * zz - xx - yy)));
    f(12, SH_C3D * (z * (2.0f * zz - 3.0f * xx - 3.0f * yy)));
    f(13, SH_C3C * (x * (4.0f * zz - xx - yy)));
    f(14, SH_C3E * (z * (xx - yy)));
    f(15, SH_C3A * (x * (xx - 3.0f * yy)));
}

template <class T>
GSN_HD inline void sh_basis_dev(int K, const T& x, const T& y, const T& z, T* Y) {
    sh_basis_visit<T>(K, x, y, z, [&](int i, const T& v) { Y[i] = v; });
}

// ----------------------------------------------------------------------------
// Second-order forward-mode jets: value, gradient and the packed upper triangle
// of the Hessian with respect to N variables, in single or double precision.
// Used by the per-kernel chain rule (projected quantities as functions of
// position, rotation or scale).
// ----------------------------------------------------------------------------
template <int N, class T = float>
struct FJet {
    static constexpr int NH = N * (N + 1) / 2;
    T v;
    T g[N];
    T h[NH];
    GSN_HD FJet() : v(T(0)) {
#pragma unroll
        for (int i = 0; i < N; ++i) g[i] = T(0);
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = T(0);
    }
    GSN_HD FJet(T c) : v(c) {  // NOLINT
#pragma unroll
        for (int i = 0; i < N; ++i) g[i] = T(0);
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = T(0);
    }
    GSN_HD static FJet var(T x, int i) {
        FJet r(x);
        r.g[i] = T(1);
        return r;
    }
};

template <int N, class T>
GSN_HD inline FJet<N, T> operator+(const FJet<N, T>& a, const FJet<N, T>& b) {
    FJet<N, T> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N, T>::NH; ++i) r.h[i] = a.h[i] + b.h[i];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> operator-(const FJet<N, T>& a, const FJet<N, T>& b) {
    FJet<N, T> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N, T>::NH; ++i) r.h[i] = a.h[i] - b.h[i];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> operator-(const FJet<N, T>& a) {
    FJet<N, T> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = -a.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N, T>::NH; ++i) r.h[i] = -a.h[i];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> operator*(const FJet<N, T>& a, const FJet<N, T>& b) {
    FJet<N, T> r;
    r.v = a.v * b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] * b.v + a.v * b.g[i];
    int idx = 0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j, ++idx)
            r.h[idx] = a.h[idx] * b.v + a.v * b.h[idx] + a.g[i] * b.g[j] + a.g[j] * b.g[i];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> operator*(T c, const FJet<N, T>& a) {
    FJet<N, T> r;
    r.v = c * a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = c * a.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N, T>::NH; ++i) r.h[i] = c * a.h[i];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> operator*(const FJet<N, T>& a, T c) { return c * a; }
template <int N, class T>
GSN_HD inline FJet<N, T> operator+(const FJet<N, T>& a, T c) { FJet<N, T> r = a; r.v += c; return r; }
template <int N, class T>
GSN_HD inline FJet<N, T> operator-(const FJet<N, T>& a, T c) { FJet<N, T> r = a; r.v -= c; return r; }
template <int N, class T>
GSN_HD inline FJet<N, T> operator-(T c, const FJet<N, T>& a) { FJet<N, T> r = -a; r.v += c; return r; }
template <int N, class T>
GSN_HD inline FJet<N, T> operator+(T c, const FJet<N, T>& a) { return a + c; }

template <int N, class T>
GSN_HD inline FJet<N, T> compose(const FJet<N, T>& a, T f, T d1, T d2) {
    FJet<N, T> r;
    r.v = f;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = d1 * a.g[i];
    int idx = 0;
#pragma unroll
    for (int i = 0; i < N; ++i)
#pragma unroll
        for (int j = i; j < N; ++j, ++idx) r.h[idx] = d1 * a.h[idx] + d2 * a.g[i] * a.g[j];
    return r;
}
template <int N, class T>
GSN_HD inline FJet<N, T> jrecip(const FJet<N, T>& a) {
    const T x = a.v, ix = T(1) / x;
    return compose(a, ix, -ix * ix, T(2) * ix * ix * ix);
}
template <int N, class T>
GSN_HD inline FJet<N, T> jsqrt(const FJet<N, T>& a) {
    const T s = sqrt(a.v);
    return compose(a, s, T(0.5) / s, T(-0.25) / (s * a.v));
}
GSN_HD inline float jrecip(float x) { return 1.0f / x; }
GSN_HD inline float jsqrt(float x) { return sqrtf(x); }
GSN_HD inline double jrecip(double x) { return 1.0 / x; }
GSN_HD inline double jsqrt(double x) { return sqrt(x); }

GSN_HD inline int tri_index(int i, int j, int n) {
    // packed upper-triangle index of (i, j), i <= j, row by row
    return i * n - (i * (i - 1)) / 2 + (j - i);
}
