// device_common.h -- device helpers shared by the gfx950 kernels of libgsn.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define GSN_TILE 16
#define GSN_BLOCK 256          // threads per tile workgroup (16 x 16 pixels, four wave64s)
#define GSN_NZ 44              // per-kernel projected-space statistics, see backward.hip

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
// Alpha of one splat at one pixel: alpha = min(alpha_max, sigma exp(-d^T Q d / 2)).
// Forward and backward passes call this same function so that their skip and
// stop decisions agree exactly.
// ----------------------------------------------------------------------------
struct SplatEval {
    float G, alpha, dx, dy;
    bool clamped;
};

__device__ __forceinline__ SplatEval eval_splat(float mx, float my, float qxx, float qxy, float qyy,
                                                float sig, float px, float py, float amax) {
    SplatEval e;
    e.dx = mx - px;
    e.dy = my - py;
    const float power = -0.5f * (qxx * e.dx * e.dx + qyy * e.dy * e.dy) - qxy * e.dx * e.dy;
    e.G = __expf(power);
    const float a = sig * e.G;
    e.clamped = a > amax;
    e.alpha = e.clamped ? amax : a;
    return e;
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

template <class T>
__device__ __forceinline__ void sh_basis_dev(int K, const T& x, const T& y, const T& z, T* Y) {
    Y[0] = T(SH_C0);
    if (K <= 1) return;
    Y[1] = -SH_C1 * y;
    Y[2] = SH_C1 * z;
    Y[3] = -SH_C1 * x;
    if (K <= 4) return;
    const T xx = x * x, yy = y * y, zz = z * z;
    Y[4] = SH_C2A * (x * y);
    Y[5] = SH_C2A * (y * z);
    Y[6] = SH_C2B * (2.0f * zz - xx - yy);
    Y[7] = SH_C2A * (x * z);
    Y[8] = SH_C2C * (xx - yy);
    if (K <= 9) return;
    Y[9] = SH_C3A * (y * (3.0f * xx - yy));
    Y[10] = SH_C3B * (x * y * z);
    Y[11] = SH_C3C * (y * (4.0f * zz - xx - yy));
    Y[12] = SH_C3D * (z * (2.0f * zz - 3.0f * xx - 3.0f * yy));
    Y[13] = SH_C3C * (x * (4.0f * zz - xx - yy));
    Y[14] = SH_C3E * (z * (xx - yy));
    Y[15] = SH_C3A * (x * (xx - 3.0f * yy));
}

// ----------------------------------------------------------------------------
// Second-order forward-mode jets in single precision: value, gradient and the
// packed upper triangle of the Hessian with respect to N variables.  Used by
// the per-kernel chain rule (projected quantities as functions of position,
// rotation or scale).
// ----------------------------------------------------------------------------
template <int N>
struct FJet {
    static constexpr int NH = N * (N + 1) / 2;
    float v;
    float g[N];
    float h[NH];
    __device__ FJet() : v(0.f) {
#pragma unroll
        for (int i = 0; i < N; ++i) g[i] = 0.f;
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = 0.f;
    }
    __device__ FJet(float c) : v(c) {  // NOLINT
#pragma unroll
        for (int i = 0; i < N; ++i) g[i] = 0.f;
#pragma unroll
        for (int i = 0; i < NH; ++i) h[i] = 0.f;
    }
    __device__ static FJet var(float x, int i) {
        FJet r(x);
        r.g[i] = 1.f;
        return r;
    }
};

template <int N>
__device__ __forceinline__ FJet<N> operator+(const FJet<N>& a, const FJet<N>& b) {
    FJet<N> r;
    r.v = a.v + b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] + b.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N>::NH; ++i) r.h[i] = a.h[i] + b.h[i];
    return r;
}
template <int N>
__device__ __forceinline__ FJet<N> operator-(const FJet<N>& a, const FJet<N>& b) {
    FJet<N> r;
    r.v = a.v - b.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = a.g[i] - b.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N>::NH; ++i) r.h[i] = a.h[i] - b.h[i];
    return r;
}
template <int N>
__device__ __forceinline__ FJet<N> operator-(const FJet<N>& a) {
    FJet<N> r;
    r.v = -a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = -a.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N>::NH; ++i) r.h[i] = -a.h[i];
    return r;
}
template <int N>
__device__ __forceinline__ FJet<N> operator*(const FJet<N>& a, const FJet<N>& b) {
    FJet<N> r;
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
template <int N>
__device__ __forceinline__ FJet<N> operator*(float c, const FJet<N>& a) {
    FJet<N> r;
    r.v = c * a.v;
#pragma unroll
    for (int i = 0; i < N; ++i) r.g[i] = c * a.g[i];
#pragma unroll
    for (int i = 0; i < FJet<N>::NH; ++i) r.h[i] = c * a.h[i];
    return r;
}
template <int N>
__device__ __forceinline__ FJet<N> operator*(const FJet<N>& a, float c) { return c * a; }
template <int N>
__device__ __forceinline__ FJet<N> operator+(const FJet<N>& a, float c) { FJet<N> r = a; r.v += c; return r; }
template <int N>
__device__ __forceinline__ FJet<N> operator-(const FJet<N>& a, float c) { FJet<N> r = a; r.v -= c; return r; }
template <int N>
__device__ __forceinline__ FJet<N> operator-(float c, const FJet<N>& a) { FJet<N> r = -a; r.v += c; return r; }
template <int N>
__device__ __forceinline__ FJet<N> operator+(float c, const FJet<N>& a) { return a + c; }

template <int N>
__device__ __forceinline__ FJet<N> compose(const FJet<N>& a, float f, float d1, float d2) {
    FJet<N> r;
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
template <int N>
__device__ __forceinline__ FJet<N> jrecip(const FJet<N>& a) {
    const float x = a.v, ix = 1.0f / x;
    return compose(a, ix, -ix * ix, 2.0f * ix * ix * ix);
}
template <int N>
__device__ __forceinline__ FJet<N> jsqrt(const FJet<N>& a) {
    const float s = sqrtf(a.v);
    return compose(a, s, 0.5f / s, -0.25f / (s * a.v));
}
__device__ __forceinline__ float jrecip(float x) { return 1.0f / x; }
__device__ __forceinline__ float jsqrt(float x) { return sqrtf(x); }

__device__ __forceinline__ int tri_index(int i, int j, int n) {
    // packed upper-triangle index of (i, j), i <= j, row by row
    return i * n - (i * (i - 1)) / 2 + (j - i);
}
