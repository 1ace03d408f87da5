// backward.hip -- per-kernel gradient and Hessian blocks (Sec. 4.2, eq. local_hessian_gradient).
//
// For a pixel and a splat k that the pixel adds, with the other splats and all
// skip/stop decisions held fixed, the colour is affine in k's opacity-weighted
// Gaussian alpha and in its colour c~ (eq. 3dgs):
//     c = P + T (alpha c~ + (1 - alpha) A),   A = (colour behind k) / (T (1 - alpha)).
// With alpha = sigma G(pi, Q), G = exp(f), f = -(d^T Q d)/2, d = pi - x:
//     dc/dalpha = a = T c~ - S/(1 - alpha) (S: colour behind k, = final colour minus
//                 the front-to-back sum up to and including k),
//     dc/dc~ = alpha T,  d2c/dalpha2 = 0,  d2c/dalpha dc~ = T,  d2c/dc~2 = 0.
// The per-kernel statistics over the projected variables, expressed in the
// splat's principal frame V = [e1 e2] (pi' = V^T pi, Q' = V^T Q V, so that
// Q' = diag(q1, q2) at the current state),
//     z = (pi'_1, pi'_2, Q'_11, Q'_12, Q'_22 | sigma | c~_R, c~_G, c~_B)
// (Q'_12 enters d'^T Q' d' twice) are, with u = df/d(pi', Q'), A1 = sum_ch dL_ch a_ch,
// A2 = sum_ch h_ch a_ch^2 (h: per-pixel diagonal image Hessian):
//     g_w  += A1 sigma G u          g_sigma += A1 G       g_c~ += dL alpha T
//     H_ww += (A2 sigma^2 G^2 + A1 sigma G) u u^T + A1 sigma G d2f
//     H_wc~ += sigma G T (h a alpha + dL) u   (per channel)
//     H_c~c~ += h (alpha T)^2 (diagonal)      H_sigma sigma += A2 G^2    w += alpha T
// (terms in w and sigma vanish where alpha was clamped).  These 44 numbers per
// kernel are everything the chain rule to position, rotation, scale, opacity
// and colour needs.
//
// raster_bwd: one 256-thread workgroup per tile re-traverses the tile's
// depth-ordered list front to back with the forward pass's decisions,
// computes each pixel's contribution to the 44 statistics of the current
// splat, reduces them across the wave by shuffles and across the four waves in
// LDS, and writes the tile's partial sum at the (tile, kernel) pair's slot.
// reduce_chain: one thread per kernel sums its pair slots in a fixed order (no
// atomics: results are deterministic), then applies the chain rule through the
// projection with second-order jets and adds the attribute blocks.
#include "gsn_internal.h"
#include "chain.h"

namespace {

constexpr int SB = 16;  // list entries reduced per LDS round

__device__ __forceinline__ float wave_sum(float v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(GSN_BLOCK) void raster_bwd_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const float4* __restrict__ rec,
    const uint2* __restrict__ rect, const uint32_t* __restrict__ pair_off, uint32_t n, DevCam cam, DevRenderOpts ro,
    const double* __restrict__ img64, const uint32_t* __restrict__ ncontrib, const float* __restrict__ dLm,
    const float* __restrict__ hdm, float* __restrict__ partial, uint8_t* __restrict__ flags) {
    __shared__ float4 s_a[GSN_BLOCK];
    __shared__ float4 s_b[GSN_BLOCK];
    __shared__ float2 s_c[GSN_BLOCK];
    __shared__ uint32_t s_slot[GSN_BLOCK];
    __shared__ float red[SB][GSN_BLOCK / 64][GSN_NZ];
    __shared__ uint32_t s_act[SB][GSN_BLOCK / 64];
    __shared__ uint32_t s_max;
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * GSN_TILE + (threadIdx.x % GSN_TILE);
    const int py = ty * GSN_TILE + (threadIdx.x / GSN_TILE);
    const bool inside = px < cam.W && py < cam.H;
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const uint2 rg = ranges[tile];
    const size_t np = (size_t)cam.W * cam.H, pi = (size_t)py * cam.W + px;
    double cf[3] = {0, 0, 0};
    float dl[3] = {0, 0, 0}, hh[3] = {0, 0, 0};
    uint32_t nc = 0;
    if (inside) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            cf[ch] = img64[ch * np + pi];
            dl[ch] = dLm[ch * np + pi];
            hh[ch] = hdm[ch * np + pi];
        }
        nc = ncontrib[pi];
    }
    if (threadIdx.x == 0) s_max = 0;
    __syncthreads();
    {
        uint32_t m = nc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
        if (lane == 0) atomicMax(&s_max, m);
    }
    __syncthreads();
    const uint32_t end = rg.x + s_max;
    // front-to-back sums in double, in the same order as the forward pass, so that the colour
    // behind a splat, S = c - sum(front..k), carries no cancellation error
    float T = 1.f;
    double Ca0 = 0.0, Ca1 = 0.0, Ca2 = 0.0;
    const float fpx = (float)px, fpy = (float)py;
    for (uint32_t base = rg.x; base < end; base += GSN_BLOCK) {
        const uint32_t e = base + threadIdx.x;
        if (e < end) {
            const uint32_t id = ids[e];
            s_a[threadIdx.x] = rec[id];
            s_b[threadIdx.x] = rec[n + id];
            const float4 c4 = rec[2 * (size_t)n + id];
            s_c[threadIdx.x] = make_float2(c4.x, c4.y);
            const uint2 rc = rect[id];
            const uint32_t x0 = rc.x & 0xffffu, y0 = rc.x >> 16, x1 = rc.y & 0xffffu;
            s_slot[threadIdx.x] = pair_off[id] + ((uint32_t)ty - y0) * (x1 - x0) + ((uint32_t)tx - x0);
        }
        __syncthreads();
        const int cnt = (int)min((uint32_t)GSN_BLOCK, end - base);
        for (int jb = 0; jb < cnt; jb += SB) {
            const int nj = min(SB, cnt - jb);
            for (int jj = 0; jj < nj; ++jj) {
                const int j = jb + jj;
                const uint32_t local = base + j - rg.x;
                float z[GSN_NZ];
#pragma unroll
                for (int f = 0; f < GSN_NZ; ++f) z[f] = 0.f;
                bool act = false;
                if (local < nc) {
                    const float4 a = s_a[j], b = s_b[j];
                    const float2 cc = s_c[j];
                    const float sig = b.z, q1 = a.z, q2 = a.w;
                    const float ct[3] = {b.w, cc.x, cc.y};
                    const SplatEval ev = eval_splat(a.x, a.y, q1, q2, b.x, b.y, sig, fpx, fpy, ro.alpha_max);
                    if (ev.alpha >= ro.alpha_min) {
                        act = true;
                        const float al = ev.alpha, wT = al * T;
                        const double wd = (double)wT;
                        Ca0 += wd * (double)ct[0];
                        Ca1 += wd * (double)ct[1];
                        Ca2 += wd * (double)ct[2];
                        const float inv = 1.0f / (1.0f - al);
                        const float av[3] = {T * ct[0] - (float)(cf[0] - Ca0) * inv,
                                             T * ct[1] - (float)(cf[1] - Ca1) * inv,
                                             T * ct[2] - (float)(cf[2] - Ca2) * inv};
                        const float A1 = dl[0] * av[0] + dl[1] * av[1] + dl[2] * av[2];
                        const float A2 = hh[0] * av[0] * av[0] + hh[1] * av[1] * av[1] + hh[2] * av[2] * av[2];
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) {
                            z[6 + ch] = dl[ch] * wT;
                            z[39 + ch] = hh[ch] * wT * wT;
                        }
                        z[43] = wT;
                        if (!ev.clamped) {
                            const float G = ev.G, dx = ev.d1, dy = ev.d2;
                            const float u[5] = {-q1 * dx, -q2 * dy, -0.5f * dx * dx, -dx * dy, -0.5f * dy * dy};
                            const float sG = sig * G;
                            const float k1 = A1 * sG;
                            const float k2 = A2 * sG * sG + k1;
#pragma unroll
                            for (int i = 0; i < 5; ++i) z[i] = k1 * u[i];
                            z[5] = A1 * G;
                            // H_ww: k2 u u^T + k1 d2f, d2f has -Q' on (pi', pi') and -d' on (pi', Q')
                            int idx = 9;
#pragma unroll
                            for (int i = 0; i < 5; ++i)
#pragma unroll
                                for (int jx = i; jx < 5; ++jx, ++idx) z[idx] = k2 * u[i] * u[jx];
                            z[9 + 0] -= k1 * q1;    // (pi'_1, pi'_1)
                            z[9 + 2] -= k1 * dx;    // (pi'_1, Q'_11)
                            z[9 + 3] -= k1 * dy;    // (pi'_1, Q'_12)
                            z[9 + 5] -= k1 * q2;    // (pi'_2, pi'_2)
                            z[9 + 7] -= k1 * dx;    // (pi'_2, Q'_12)
                            z[9 + 8] -= k1 * dy;    // (pi'_2, Q'_22)
#pragma unroll
                            for (int ch = 0; ch < 3; ++ch) {
                                const float bch = sG * T * (hh[ch] * av[ch] * al + dl[ch]);
#pragma unroll
                                for (int i = 0; i < 5; ++i) z[24 + i * 3 + ch] = bch * u[i];
                            }
                            z[42] = A2 * G * G;
                        }
                        T *= (1.0f - al);
                    }
                }
                const uint64_t any = __ballot(act);
                if (any) {
#pragma unroll
                    for (int f = 0; f < GSN_NZ; ++f) z[f] = wave_sum(z[f]);
                }
                // each wave owns its own LDS row: no barrier is needed inside this loop
                if (lane == 0) {
#pragma unroll
                    for (int f = 0; f < GSN_NZ; ++f) red[jj][wave][f] = any ? z[f] : 0.f;
                    s_act[jj][wave] = any ? 1u : 0u;
                }
            }
            __syncthreads();
            for (int idx = threadIdx.x; idx < nj * GSN_NZ; idx += GSN_BLOCK) {
                const int jj = idx / GSN_NZ, f = idx % GSN_NZ;
                if (!(s_act[jj][0] | s_act[jj][1] | s_act[jj][2] | s_act[jj][3])) continue;
                const float v = ((red[jj][0][f] + red[jj][1][f]) + red[jj][2][f]) + red[jj][3][f];
                const uint32_t slot = s_slot[jb + jj];
                partial[(size_t)slot * GSN_NZ + f] = v;
                if (f == 0) flags[slot] = 1;
            }
            __syncthreads();
        }
    }
}

__global__ __launch_bounds__(128) void reduce_chain_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale,
    const float* __restrict__ sh, int n, int K, const uint2* __restrict__ rect, const uint32_t* __restrict__ pair_off,
    const float* __restrict__ partial, const uint8_t* __restrict__ flags, const float4* __restrict__ rec, DevCam cam,
    float kappa, float weight, int slot, float* __restrict__ blk, float* __restrict__ zstats) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint2 rc = rect[k];
    const uint32_t nt = ((rc.y & 0xffffu) - (rc.x & 0xffffu)) * ((rc.y >> 16) - (rc.x >> 16));
    // the kernel's tile partials, summed in double in slot order
    double zd[GSN_NZ];
#pragma unroll
    for (int f = 0; f < GSN_NZ; ++f) zd[f] = 0.0;
    const uint32_t off = pair_off[k];
    for (uint32_t i = 0; i < nt; ++i) {
        const uint32_t sl = off + i;
        if (!flags[sl]) continue;
        const float4* pp = reinterpret_cast<const float4*>(partial + (size_t)sl * GSN_NZ);
#pragma unroll
        for (int f = 0; f < GSN_NZ / 4; ++f) {
            const float4 v = pp[f];
            zd[4 * f] += v.x;
            zd[4 * f + 1] += v.y;
            zd[4 * f + 2] += v.z;
            zd[4 * f + 3] += v.w;
        }
    }
    float z[GSN_NZ];
#pragma unroll
    for (int f = 0; f < GSN_NZ; ++f) z[f] = (float)zd[f];
    if (zstats) {
#pragma unroll
        for (int f = 0; f < GSN_NZ; ++f) zstats[(size_t)f * n + k] = z[f];
    }
    if (!(z[43] > 0.f)) return;
    KParams kp;
#pragma unroll
    for (int a = 0; a < 3; ++a) kp.p[a] = pos[(size_t)a * n + k];
#pragma unroll
    for (int a = 0; a < 4; ++a) kp.q[a] = rot[(size_t)a * n + k];
#pragma unroll
    for (int a = 0; a < 3; ++a) kp.s[a] = scale[(size_t)a * n + k];
    float shk[48];
    for (int i = 0; i < 3 * K; ++i) shk[i] = sh[(size_t)i * n + k];
    const float4 r1 = rec[(size_t)n + k];
    kp.fc = r1.x;
    kp.fs = r1.y;
    const size_t N = (size_t)n;
    {
        float g[3], H[6];
        chain_position(kp, shk, K, cam, kappa, z, g, H);
#pragma unroll
        for (int a = 0; a < 3; ++a) blk[a * N + k] += weight * g[a];
#pragma unroll
        for (int a = 0; a < 6; ++a) blk[(3 + a) * N + k] += weight * H[a];
    }
    {
        double g[3], H[6];
        chain_rotation(kp, cam, kappa, z, g, H);
#pragma unroll
        for (int a = 0; a < 3; ++a) blk[(9 + a) * N + k] += (float)(weight * g[a]);
#pragma unroll
        for (int a = 0; a < 6; ++a) blk[(12 + a) * N + k] += (float)(weight * H[a]);
        chain_scale(kp, cam, kappa, z, g, H);
#pragma unroll
        for (int a = 0; a < 3; ++a) blk[(18 + a) * N + k] += (float)(weight * g[a]);
#pragma unroll
        for (int a = 0; a < 6; ++a) blk[(21 + a) * N + k] += (float)(weight * H[a]);
    }
    blk[27 * N + k] += weight * z[5];
    blk[28 * N + k] += weight * z[42];
    if (slot == 0) blk[29 * N + k] = z[43];
    const size_t vb = GSN_BLK_BASE + (size_t)GSN_BLK_VIEW * slot;
    const float dx = kp.p[0] - cam.o[0], dy = kp.p[1] - cam.o[1], dz = kp.p[2] - cam.o[2];
    const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        blk[(vb + ch) * N + k] = weight * z[6 + ch];
        blk[(vb + 3 + ch) * N + k] = weight * z[39 + ch];
    }
    blk[(vb + 6) * N + k] = dx * il;
    blk[(vb + 7) * N + k] = dy * il;
    blk[(vb + 8) * N + k] = dz * il;
    blk[(vb + 9) * N + k] = z[43];
}

}  // namespace

void launch_raster_bwd(const gsn_frame& f, const float* dL, const float* hd, hipStream_t s) {
    const int tiles = f.tiles_x * f.tiles_y;
    raster_bwd_kernel<<<tiles, GSN_BLOCK, 0, s>>>(
        bp<uint2>(f.ranges), bp<uint32_t>(f.pv_a), bp<float4>(f.rec),
        bp<uint2>(f.rect), bp<uint32_t>(f.pair_off), (uint32_t)f.n, f.cam, f.ro, bp<double>(f.img64),
        bp<uint32_t>(f.ncontrib), dL, hd, bp<float>(f.partial), bp<uint8_t>(f.flags));
}

void launch_reduce_chain(const gsn_frame& f, const gsn_gaussians& g, float weight, int slot, const gsn_blocks& b,
                         float* zstats_out, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    reduce_chain_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(
        g.d_pos, g.d_rot, g.d_scale, g.d_sh, g.n, K, bp<uint2>(f.rect), bp<uint32_t>(f.pair_off),
        bp<float>(f.partial), bp<uint8_t>(f.flags), bp<float4>(f.rec), f.cam, f.ro.kappa, weight, slot, b.d_data,
        zstats_out);
}
