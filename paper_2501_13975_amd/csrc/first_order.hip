// first_order.hip -- the first-order baseline on the same gradients as the Newton sweep.
//
// One thread per kernel.  The gradient is read from the blocks the sweep
// accumulated (position, left rotation vector, linear scale and opacity rows;
// the SH gradient of channel ch is the sum over views of gamma_{v,ch} Y(r_v),
// Sec. 4.2 colour paragraph), then one gradient-descent or Adam step (Kingma
// and Ba, 2015) is taken per attribute group with the Newton apply's parameter
// updates: rotation by the exponential map, scale >= scale_floor * s, opacity in
// [opac_eps, 1 - opac_eps].  Kernels the primary view does not see are left
// alone, moments included.  Moments are float [2][10 + 3K][n] (m then v),
// entries per kernel in the order position 3, omega 3, scale 3, opacity 1,
// colour [3][K]; coalesced across kernels.
#include "gsn_internal.h"

namespace {

__device__ __forceinline__ float fo_update(float g, float* m, float* v, size_t idx, const gsn_first_order_opts& fo,
                                           float c1, float c2, float lr) {
    if (!fo.adam) return lr * g;
    const float mm = fo.beta1 * m[idx] + (1.0f - fo.beta1) * g;
    const float vv = fo.beta2 * v[idx] + (1.0f - fo.beta2) * g * g;
    m[idx] = mm;
    v[idx] = vv;
    return lr * (mm * c1) / (sqrtf(vv * c2) + fo.eps);
}

__global__ __launch_bounds__(256) void first_order_kernel(float* __restrict__ pos, float* __restrict__ rot,
                                                          float* __restrict__ scale, float* __restrict__ opac,
                                                          float* __restrict__ sh, int n, int K,
                                                          const float* __restrict__ blk, int V,
                                                          gsn_first_order_opts fo, float c1, float c2,
                                                          float scale_floor, float opac_eps,
                                                          float* __restrict__ state, uint32_t mask) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    if (!(blk[29 * N + k] > 0.f)) return;  // not seen by the primary view
    const int F = 10 + 3 * K;
    float* m = state;
    float* v = state ? state + (size_t)F * N : nullptr;
    auto at = [&](int f) { return (size_t)f * N + k; };
    if (mask & 1u)
        for (int a = 0; a < 3; ++a) pos[a * N + k] -= fo_update(blk[a * N + k], m, v, at(a), fo, c1, c2, fo.lr[0]);
    if (mask & 2u) {
        float w[3];
        for (int a = 0; a < 3; ++a) w[a] = -fo_update(blk[(9 + a) * N + k], m, v, at(3 + a), fo, c1, c2, fo.lr[1]);
        const float th = sqrtf(w[0] * w[0] + w[1] * w[1] + w[2] * w[2]);
        if (th > 0.f) {
            const float sf = sinf(0.5f * th) / th;
            const float dq[4] = {cosf(0.5f * th), sf * w[0], sf * w[1], sf * w[2]};
            float q[4], r[4];
            for (int c = 0; c < 4; ++c) q[c] = rot[c * N + k];
            qmul<float>(dq, q, r);
            const float il = 1.0f / sqrtf(r[0] * r[0] + r[1] * r[1] + r[2] * r[2] + r[3] * r[3]);
            for (int c = 0; c < 4; ++c) rot[c * N + k] = r[c] * il;
        }
    }
    if (mask & 4u)
        for (int a = 0; a < 3; ++a) {
            const float s = scale[a * N + k];
            const float d = fo_update(blk[(18 + a) * N + k], m, v, at(6 + a), fo, c1, c2, fo.lr[2]);
            scale[a * N + k] = fmaxf(s - d, scale_floor * s);
        }
    if (mask & 8u) {
        const float d = fo_update(blk[27 * N + k], m, v, at(9), fo, c1, c2, fo.lr[3]);
        opac[k] = fminf(fmaxf(opac[k] - d, opac_eps), 1.0f - opac_eps);
    }
    if (mask & 16u) {
        float gc[3][16];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
            for (int i = 0; i < 16; ++i) gc[ch][i] = 0.f;
        for (int vw = 0; vw < V; ++vw) {
            const size_t b = GSN_BLK_BASE + (size_t)GSN_BLK_VIEW * vw;
            if (!(blk[(b + 9) * N + k] > 0.f)) continue;
            const float gam[3] = {blk[b * N + k], blk[(b + 1) * N + k], blk[(b + 2) * N + k]};
            sh_basis_visit<float>(K, blk[(b + 6) * N + k], blk[(b + 7) * N + k], blk[(b + 8) * N + k],
                                  [&](int i, float y) {
#pragma unroll
                                      for (int ch = 0; ch < 3; ++ch) gc[ch][i] += gam[ch] * y;
                                  });
        }
#pragma unroll
        for (int ch = 0; ch < 3; ++ch)
#pragma unroll
            for (int i = 0; i < 16; ++i)
                if (i < K)
                    sh[(ch * K + i) * N + k] -= fo_update(gc[ch][i], m, v, at(10 + ch * K + i), fo, c1, c2, fo.lr[4]);
    }
}

}  // namespace

void launch_first_order(const gsn_gaussians& g, const gsn_blocks& b, const gsn_first_order_opts& fo, float c1,
                        float c2, float scale_floor, float opac_eps, float* state, uint32_t mask, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    first_order_kernel<<<(g.n + 255) / 256, 256, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.d_sh, g.n, K,
                                                         b.d_data, b.n_views, fo, c1, c2, scale_floor, opac_eps,
                                                         state, mask);
}
