// loss.hip -- per-pixel loss derivative maps (Sec. 4.2).
//
// L = L2 + lambda L_S with L2 = 1/(6|I|) sum (c - c^t)^2 and
// L_S = 1/(3|I|) sum_pix sum_ch (1 - SSIM), SSIM over an 11x11 Gaussian window
// (sigma 1.5, zero padding), C1 = 0.01^2, C2 = 0.03^2.  With the paper's f0..f3
// (f0 = 2 mu mu^t + C1, f1 = 2 cov + C2, f2 = mu^2 + mu^t^2 + C1,
// f3 = var + var^t + C2) the derivative of one window's SSIM F with respect to a
// pixel value c at window weight w is
//     dF = w (a0 + a1 c^t - a2 c) F,   a0 = 2mu^t/f0 - 2mu^t/f1 - 2mu/f2 + 2mu/f3,
//                                       a1 = 2/f1, a2 = 2/f3,
// and its exact second derivative is
//     d2F = w^2 F (b0 + bt c^t + bc c + bcc c^2 + btc c c^t) - 2 w F / f3
// with b0 = a0^2 - 4mu^t^2/f0^2 - 4mu^t^2/f1^2 - 2/f2 + 4mu^2/f2^2 + 2/f3 + 4mu^2/f3^2,
// bt = 2 a0 a1 + 8 mu^t/f1^2, bc = -2 a0 a2 - 8 mu/f3^2, bcc = 8/f3^2, btc = -8/(f1 f3).
// Summing over the windows that contain a pixel turns each window-centred
// coefficient map into a correlation with w (three maps) or w^2 (five maps).
//
// Pass 1 (one workgroup per 16x16 tile of window centres, its three channels in turn): moments
// by separable convolution through LDS, then the eight coefficient maps
// (computed in double and stored in single precision: their rounding moves dL
// and h by about 5e-8 of the maps' largest values) and the loss partial sums
// (double).  Pass 2 (32x32 tiles, one map at a time, the next map's halo tile
// read into registers meanwhile): the eight correlations in double and the
// per-pixel gradient dL and diagonal Hessian h.  Pass 3:
// double-precision reduction of the loss partials in a fixed order.
#include "gsn_internal.h"

namespace {

constexpr int T = 16, HALO = 5, R = T + 2 * HALO;  // 26
constexpr double kC1 = 0.01 * 0.01, kC2 = 0.03 * 0.03;

template <class Re>
__device__ __forceinline__ void window_weights(Re* g, Re* g2) {
    // normalised 1D Gaussian, sigma 1.5; the 2D window is the outer product (weights evaluated in
    // double, then rounded to the working type)
    if (threadIdx.x < 11) {
        double s = 0.0, v[11];
        for (int i = 0; i < 11; ++i) {
            v[i] = exp(-((double)((i - 5) * (i - 5))) / (2.0 * 1.5 * 1.5));
            s += v[i];
        }
        const double gi = v[threadIdx.x] / s;
        g[threadIdx.x] = (Re)gi;
        g2[threadIdx.x] = (Re)(gi * gi);
    }
}

template <class Re>
__global__ __launch_bounds__(256) void ssim_coef_kernel(const float* __restrict__ img, const float* __restrict__ tgt,
                                                         int W, int H, float* __restrict__ coef,
                                                         double* __restrict__ part) {
    __shared__ Re g[11], g2[11];
    __shared__ Re sc[R][R], st[R][R];
    __shared__ Re hs[5][R][T];
    __shared__ double red[2][4];
    const int x0 = blockIdx.x * T - HALO, y0 = blockIdx.y * T - HALO;
    const size_t np = (size_t)W * H;
    window_weights(g, g2);
    // the three channels one after another: the next channel's halo tiles of image and target are
    // loaded into registers while the current one is processed
    constexpr int NLD = (R * R + 255) / 256;  // 3 elements per thread and array
    float ld_c[NLD], ld_t[NLD];
    auto load = [&](int c) {
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + 256 * j;
            const int yy = i / R, xx = i % R, x = x0 + xx, y = y0 + yy;
            const bool in = i < R * R && x >= 0 && y >= 0 && x < W && y < H;
            const size_t at = in ? (size_t)c * np + (size_t)y * W + x : 0;
            ld_c[j] = in ? img[at] : 0.f;
            ld_t[j] = in ? tgt[at] : 0.f;
        }
    };
    load(0);
    for (int ch = 0; ch < 3; ++ch) {
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + 256 * j;
            if (i < R * R) {
                sc[i / R][i % R] = (Re)ld_c[j];
                st[i / R][i % R] = (Re)ld_t[j];
            }
        }
        __syncthreads();
        if (ch + 1 < 3) load(ch + 1);
        for (int i = threadIdx.x; i < R * T; i += 256) {
            const int yy = i / T, xx = i % T;
            Re a = 0, b = 0, c = 0, d = 0, e = 0;
#pragma unroll
            for (int k = 0; k < 11; ++k) {
                const Re u = sc[yy][xx + k], v = st[yy][xx + k], w = g[k];
                a += w * u;
                b += w * v;
                c += w * u * u;
                d += w * v * v;
                e += w * u * v;
            }
            hs[0][yy][xx] = a;
            hs[1][yy][xx] = b;
            hs[2][yy][xx] = c;
            hs[3][yy][xx] = d;
            hs[4][yy][xx] = e;
        }
        __syncthreads();
        const int lx = threadIdx.x % T, ly = threadIdx.x / T;
        const int x = blockIdx.x * T + lx, y = blockIdx.y * T + ly;
        double l2 = 0.0, ls = 0.0;  // loss partials in double in both forms
        if (x < W && y < H) {
            Re m[5] = {0, 0, 0, 0, 0};
#pragma unroll
            for (int k = 0; k < 11; ++k)
#pragma unroll
                for (int q = 0; q < 5; ++q) m[q] += g[k] * hs[q][ly + k][lx];
            // the quotient-rule coefficients in double in both forms: their terms in 1/f2 and 1/f3 cancel
            // to a small fraction of their size in flat regions, which single precision does not resolve
            const double mu = m[0], mut = m[1];
            const double f0 = 2.0 * mu * mut + kC1;
            const double f1 = 2.0 * ((double)m[4] - mu * mut) + kC2;
            const double f2 = mu * mu + mut * mut + kC1;
            const double f3 = ((double)m[2] - mu * mu) + ((double)m[3] - mut * mut) + kC2;
            const double F = (f0 * f1) / (f2 * f3);
            const double i0 = 1.0 / f0, i1 = 1.0 / f1, i2 = 1.0 / f2, i3 = 1.0 / f3;
            const double a0 = 2.0 * mut * i0 - 2.0 * mut * i1 - 2.0 * mu * i2 + 2.0 * mu * i3;
            const double a1 = 2.0 * i1, a2 = 2.0 * i3;
            const double b0 = a0 * a0 - 4.0 * mut * mut * i0 * i0 - 4.0 * mut * mut * i1 * i1 - 2.0 * i2 +
                              4.0 * mu * mu * i2 * i2 + 2.0 * i3 + 4.0 * mu * mu * i3 * i3;
            const double bt = 2.0 * a0 * a1 + 8.0 * mut * i1 * i1;
            const double bc = -2.0 * a0 * a2 - 8.0 * mu * i3 * i3;
            const double bcc = 8.0 * i3 * i3;
            const double btc = -8.0 * i1 * i3;
            const size_t pi = (size_t)y * W + x;
            float* cf = coef + (size_t)ch * 8 * np;
            cf[0 * np + pi] = (float)(F * a0);
            cf[1 * np + pi] = (float)(F * a1);
            cf[2 * np + pi] = (float)(F * a2);
            cf[3 * np + pi] = (float)(F * b0);
            cf[4 * np + pi] = (float)(F * bt);
            cf[5 * np + pi] = (float)(F * bc);
            cf[6 * np + pi] = (float)(F * bcc);
            cf[7 * np + pi] = (float)(F * btc);
            const double r = (double)sc[ly + HALO][lx + HALO] - (double)st[ly + HALO][lx + HALO];
            l2 = r * r;
            ls = 1.0 - (double)F;
        }
        // deterministic block reduction in double: a butterfly within each wave, then the four wave
        // sums in wave order
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) {
            l2 += __shfl_xor(l2, off, 64);
            ls += __shfl_xor(ls, off, 64);
        }
        if (__lane_id() == 0) {
            red[0][threadIdx.x / 64] = l2;
            red[1][threadIdx.x / 64] = ls;
        }
        __syncthreads();
        if (threadIdx.x == 0) {
            // the partials of (channel, tile row, tile column), as one workgroup per tile and channel
            const int nb = gridDim.x * gridDim.y * 3;
            const int b = (ch * gridDim.y + blockIdx.y) * gridDim.x + blockIdx.x;
            part[b] = ((red[0][0] + red[0][1]) + red[0][2]) + red[0][3];
            part[nb + b] = ((red[1][0] + red[1][1]) + red[1][2]) + red[1][3];
        }
        __syncthreads();  // the LDS tiles and sums are rewritten for the next channel
    }
}

// Pass 2 on 32 x 32 pixel tiles, one coefficient map at a time (the 42 x 42 halo tile of the map
// and its horizontal correlation in LDS): each thread owns four consecutive pixels of a column
// and folds each map's correlation into their derivatives; both correlation passes work on
// strips of four outputs that share their 14 inputs (a third of the LDS reads).  Halo reads are 1.7x the map instead of 2.6x with 16 x 16
// tiles, and the small LDS footprint keeps several workgroups per CU.
constexpr int T2 = 32, R2 = T2 + 2 * HALO;  // 42

template <class Re>
__global__ __launch_bounds__(256) void ssim_grad_kernel(const float* __restrict__ img, const float* __restrict__ tgt,
                                                         int W, int H, float lambda, const float* __restrict__ coef,
                                                         float* __restrict__ dL, float* __restrict__ hd) {
    __shared__ Re g[11], g2[11];
    __shared__ Re sm[R2][R2];
    __shared__ Re hs[R2][T2];
    const int ch = blockIdx.z;
    const int x0 = blockIdx.x * T2 - HALO, y0 = blockIdx.y * T2 - HALO;
    const size_t np = (size_t)W * H;
    const float* cf = coef + (size_t)ch * 8 * np;
    window_weights(g, g2);
    const int lx = threadIdx.x % T2, ly0 = 4 * (threadIdx.x / T2);  // rows ly0 .. ly0 + 3
    // d1 = v0 + t v1 - c v2 and d2 = v3 + t v4 + c v5 + c^2 v6 + c t v7 - v2 are linear in the
    // correlations v_q, so each map's correlation is folded in as soon as it is taken
    Re cv[4], tv[4], d1[4], d2[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = blockIdx.x * T2 + lx, y = blockIdx.y * T2 + ly0 + r;
        const bool in = x < W && y < H;
        const size_t pi = in ? (size_t)y * W + x : 0;
        cv[r] = in ? (Re)img[ch * np + pi] : Re(0.0);
        tv[r] = in ? (Re)tgt[ch * np + pi] : Re(0.0);
        d1[r] = d2[r] = Re(0.0);
    }
    // the halo tile of map q + 1 is loaded into registers while map q is correlated
    constexpr int NLD = (R2 * R2 + 255) / 256;  // 7 elements per thread
    float pre[NLD];
    auto load_map = [&](int q) {
        const float* map = cf + (size_t)q * np;
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + 256 * j;
            const int yy = i / R2, xx = i % R2, x = x0 + xx, y = y0 + yy;
            const bool in = i < R2 * R2 && x >= 0 && y >= 0 && x < W && y < H;
            pre[j] = in ? map[(size_t)y * W + x] : 0.f;
        }
    };
    load_map(0);
    for (int q = 0; q < 8; ++q) {
#pragma unroll
        for (int j = 0; j < NLD; ++j) {
            const int i = threadIdx.x + 256 * j;
            if (i < R2 * R2) sm[i / R2][i % R2] = (Re)pre[j];
        }
        __syncthreads();
        if (q + 1 < 8) load_map(q + 1);
        const Re* wq = q < 3 ? g : g2;
        // horizontal: strips of four outputs share their 14 inputs
        for (int i = threadIdx.x; i < R2 * (T2 / 4); i += 256) {
            const int yy = i / (T2 / 4), xs = 4 * (i % (T2 / 4));
            Re in14[14];
#pragma unroll
            for (int k = 0; k < 14; ++k) in14[k] = sm[yy][xs + k];
#pragma unroll
            for (int o = 0; o < 4; ++o) {
                Re a = Re(0.0);
#pragma unroll
                for (int k = 0; k < 11; ++k) a += wq[k] * in14[o + k];
                hs[yy][xs + o] = a;
            }
        }
        __syncthreads();
        // vertical: the thread's four rows share their 14 inputs
        Re col[14];
#pragma unroll
        for (int k = 0; k < 14; ++k) col[k] = hs[ly0 + k][lx];
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            Re a = Re(0.0);
#pragma unroll
            for (int k = 0; k < 11; ++k) a += wq[k] * col[r + k];
            const Re c = cv[r], t = tv[r];
            const Re k1 = q == 0 ? Re(1.0) : q == 1 ? t : q == 2 ? -c : Re(0.0);
            const Re k2 = q < 2 ? Re(0.0) : q == 2 ? -Re(1.0) : q == 3 ? Re(1.0) : q == 4 ? t : q == 5 ? c : q == 6 ? c * c : c * t;
            d1[r] += k1 * a;
            d2[r] += k2 * a;
        }
    }
    const Re norm = Re(1.0) / (Re(3.0) * (Re)np);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int x = blockIdx.x * T2 + lx, y = blockIdx.y * T2 + ly0 + r;
        if (x >= W || y >= H) continue;
        const size_t pi = (size_t)y * W + x;
        dL[ch * np + pi] = (float)((cv[r] - tv[r]) * norm - (Re)lambda * norm * d1[r]);
        hd[ch * np + pi] = (float)(norm - (Re)lambda * norm * d2[r]);
    }
}

// One workgroup of kReduceThreads: each thread sums its strided share of the partials with four
// independent accumulators (so that its loads are in flight together), then the workgroup adds the
// threads' sums in a fixed tree; the order depends only on nparts, so the value is deterministic.
constexpr int kReduceThreads = 1024;
__global__ __launch_bounds__(kReduceThreads) void loss_reduce_kernel(const double* __restrict__ part, int nparts,
                                                                      double npix, double* __restrict__ out) {
    __shared__ double red[2][kReduceThreads];
    const int t = threadIdx.x;
    double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
    int i = t;
    for (; i + 3 * kReduceThreads < nparts; i += 4 * kReduceThreads) {
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            a[u] += part[i + u * kReduceThreads];
            b[u] += part[nparts + i + u * kReduceThreads];
        }
    }
#pragma unroll
    for (int u = 0; u < 3; ++u)  // at most three left: i + 3 kReduceThreads >= nparts
        if (i + u * kReduceThreads < nparts) {
            a[u] += part[i + u * kReduceThreads];
            b[u] += part[nparts + i + u * kReduceThreads];
        }
    red[0][t] = (a[0] + a[1]) + (a[2] + a[3]);
    red[1][t] = (b[0] + b[1]) + (b[2] + b[3]);
    __syncthreads();
    for (int s = kReduceThreads / 2; s > 0; s >>= 1) {
        if (t < s) {
            red[0][t] += red[0][t + s];
            red[1][t] += red[1][t + s];
        }
        __syncthreads();
    }
    if (t == 0) {
        out[0] = red[0][0] / (6.0 * npix);
        out[1] = red[1][0] / (3.0 * npix);
    }
}

}  // namespace

void launch_loss_maps(const float* img, const float* tgt, int W, int H, float lambda, bool fp32, float* coef,
                      float* dL, float* hd, double* part, int* nparts, hipStream_t s) {
    dim3 grid((W + T - 1) / T, (H + T - 1) / T, 1);  // the three channels in each workgroup
    *nparts = (int)(grid.x * grid.y * 3);
    dim3 grid2((W + T2 - 1) / T2, (H + T2 - 1) / T2, 3);
    if (fp32) {
        ssim_coef_kernel<float><<<grid, 256, 0, s>>>(img, tgt, W, H, coef, part);
        ssim_grad_kernel<float><<<grid2, 256, 0, s>>>(img, tgt, W, H, lambda, coef, dL, hd);
    } else {
        ssim_coef_kernel<double><<<grid, 256, 0, s>>>(img, tgt, W, H, coef, part);
        ssim_grad_kernel<double><<<grid2, 256, 0, s>>>(img, tgt, W, H, lambda, coef, dL, hd);
    }
}

void launch_loss_reduce(const double* part, int nparts, int W, int H, double* out, hipStream_t s) {
    loss_reduce_kernel<<<1, kReduceThreads, 0, s>>>(part, nparts, (double)W * (double)H, out);
}
