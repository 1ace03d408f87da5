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
//     H_c~c~ += h (alpha T)^2 (diagonal)      H_sigma sigma += A2 G^2    w += alpha T,
//     w2 += (alpha T)^2 (the kernel's overlap share is w2 / w)
// (terms in w and sigma vanish where alpha was clamped).  These 44 numbers per
// kernel are everything the chain rule to position, rotation, scale, opacity
// and colour needs.
//
// raster_bwd: one 256-thread workgroup per tile re-traverses the tile's
// depth-ordered list front to back with the forward pass's decisions, stages
// the contributing (pixel, splat) pairs of each round in LDS, and sums each
// splat's 44 statistics over its pairs (see raster_bwd_kernel); the tile's
// partial sum is written at the (tile, kernel) pair's slot.  Workgroups take the
// tiles with the longest composited prefixes (recorded by the forward pass) first.
// reduce_pairs: a wave per 16 kernels sums each flagged kernel's written pair slots in a fixed order
// (no atomics: results are deterministic); chain_pos / chain_rs: one thread per
// kernel applies the chain rule through the projection with second-order jets
// and adds the attribute blocks (position, opacity, colour / rotation, scale).
#include "gsn_internal.h"
#include "chain.h"

namespace {

constexpr int PMAX = 896;   // composited (pixel, entry) pairs staged per round
constexpr int BIG = 64;     // entries with more pairs are summed by LG lanes, others by SG
constexpr int SG = 8, LG = 32;
// statistics a pair adds to (0 .. GSN_ZW2); the rest of the GSN_NZ words are padding, kept zero
constexpr int kLiveZ = GSN_ZW2 + 1;
// The per-kernel sums the rotation and scale chain rule reads, kept in double: the conic gradient
// (statistics 2..4), its Hessian (18..23, packed upper triangle) and the coverage.
constexpr int kZq = 10, kZqCov = 9;
__device__ __forceinline__ int zq_slot(int f) {
    return (f >= 2 && f <= 4) ? f - 2 : (f >= 18 && f <= 23) ? f - 15 : f == GSN_ZCOV ? kZqCov : -1;
}

// Contribution of one active (pixel, splat) pair to the 44 statistics (see the header comment).
template <bool GN>
__device__ __forceinline__ void pair_terms(const float4 a, const float4 b, float G, float T, const float av[3],
                                           float dx, float dy, const float dl[3], const float hh[3], float amax,
                                           float* acc) {
    // adds the pair's 44 terms to acc (no 44-register temporary)
    const float sig = b.z, q1 = a.z, q2 = a.w;
    const float sGraw = sig * G;
    const bool clamped = sGraw > amax;
    const float al = clamped ? amax : sGraw;
    const float wT = al * T;
    const float A1 = dl[0] * av[0] + dl[1] * av[1] + dl[2] * av[2];
    const float A2 = hh[0] * av[0] * av[0] + hh[1] * av[1] * av[1] + hh[2] * av[2] * av[2];
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        acc[6 + ch] += dl[ch] * wT;
        acc[39 + ch] += hh[ch] * wT * wT;
    }
    acc[GSN_ZCOV] += wT;
    acc[GSN_ZW2] += wT * wT;
    if (clamped) return;
    const float u[5] = {-q1 * dx, -q2 * dy, -0.5f * dx * dx, -dx * dy, -0.5f * dy * dy};
    const float k1 = A1 * sGraw;
    // Gauss-Newton keeps only the h-weighted products of first derivatives: no k1 curvature terms
    const float k2 = GN ? A2 * sGraw * sGraw : A2 * sGraw * sGraw + k1;
#pragma unroll
    for (int i = 0; i < 5; ++i) acc[i] += k1 * u[i];
    acc[5] += A1 * G;
    // H_ww: k2 u u^T + k1 d2f, d2f has -Q' on (pi', pi') and -d' on (pi', Q')
    int idx = 9;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j, ++idx) {
            float t = k2 * u[i] * u[j];
            if (!GN) {
                if (idx == 9 + 0) t -= k1 * q1;  // (pi'_1, pi'_1)
                if (idx == 9 + 2) t -= k1 * dx;  // (pi'_1, Q'_11)
                if (idx == 9 + 3) t -= k1 * dy;  // (pi'_1, Q'_12)
                if (idx == 9 + 5) t -= k1 * q2;  // (pi'_2, pi'_2)
                if (idx == 9 + 7) t -= k1 * dx;  // (pi'_2, Q'_12)
                if (idx == 9 + 8) t -= k1 * dy;  // (pi'_2, Q'_22)
            }
            acc[idx] += t;
        }
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float bch = sGraw * T * (GN ? hh[ch] * av[ch] * al : hh[ch] * av[ch] * al + dl[ch]);
#pragma unroll
        for (int i = 0; i < 5; ++i) acc[24 + i * 3 + ch] += bch * u[i];
    }
    acc[42] += A2 * G * G;
}

// Cross-lane sums with DPP row operations (no LDS traffic): quad_sum leaves in every lane
// the sum over its group of 4 lanes, row_sum the sum over its row of 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, false));
}
__device__ __forceinline__ float quad_sum(float v) {
    v += dpp_mov<0xB1>(v);  // quad_perm [1, 0, 3, 2]
    v += dpp_mov<0x4E>(v);  // quad_perm [2, 3, 0, 1]
    return v;
}
__device__ __forceinline__ float row_sum(float v) {
    v = quad_sum(v);
    v += dpp_mov<0x141>(v);  // row_half_mirror: the other quad of the half row
    v += dpp_mov<0x140>(v);  // row_mirror: the other half of the row
    return v;
}
// Sum over aligned groups of G lanes (G = 4, 8, 16, 32 or 64): left in every lane of the group,
// except for G = 32, where it is in the group's second row (see group_writer).
template <int G>
__device__ __forceinline__ float group_sum(float v) {
    if (G == 4) return quad_sum(v);
    if (G == 8) return quad_sum(v) + dpp_mov<0x141>(quad_sum(v));
    if (G == 16) return row_sum(v);
    float r = row_sum(v);
    if (G == 32) {
        // row_bcast:15 adds the even row's total into the odd row: the group's total is in its second
        // row (lanes 16..31 of the group), the first row keeps its own total
        return r + __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(r), 0x142, 0xA, 0xF, false));
    }
    r += __shfl_xor(r, 16, 64);
    if (G == 64) r += __shfl_xor(r, 32, 64);
    return r;
}
// The lane of a G-lane group that holds the group's total after group_sum.
template <int G>
__device__ __forceinline__ constexpr int group_writer() { return G == 32 ? 16 : 0; }

// Adds the statistics of staged pair i (slot in LDS) of the splat (a, b, c4) to acc.
template <bool GN>
__device__ __forceinline__ void pair_stats(const float4 a, const float4 b, const float4 cl, const float4* s_pa,
                                           const float* s_pb, const uint8_t* s_pix, const float4* s_lm0,
                                           const float2* s_lm1, uint32_t i, int tx, int ty, float amax,
                                           float* acc) {
    const float4 pa = s_pa[i];
    const int p = s_pix[i];
    const float av[3] = {pa.z, pa.w, s_pb[i]};
    const float4 l0 = s_lm0[p];
    const float2 l1 = s_lm1[p];
    const float dl[3] = {l0.x, l0.y, l0.z};
    const float hh[3] = {l0.w, l1.x, l1.y};
    const float ddx = (a.x - (float)(tx * GSN_TILE + (p % GSN_TILE))) + cl.z;
    const float ddy = (a.y - (float)(ty * GSN_TILE + (p / GSN_TILE))) + cl.w;
    const float d1 = b.x * ddx + b.y * ddy, d2 = b.x * ddy - b.y * ddx;
    pair_terms<GN>(a, b, pa.y, pa.x, av, d1, d2, dl, hh, amax, acc);
}

__device__ __forceinline__ void write_partial(float* __restrict__ partial, uint8_t* __restrict__ flags, uint32_t slot,
                                              const float* acc) {
    float4* dst = reinterpret_cast<float4*>(partial + (size_t)slot * GSN_NZ);
#pragma unroll
    for (int f = 0; f < GSN_NZ / 4; ++f) dst[f] = make_float4(acc[4 * f], acc[4 * f + 1], acc[4 * f + 2], acc[4 * f + 3]);
    flags[slot] = 1;
}

// One workgroup per tile.  List entries are staged in LDS in batches of 256 (one per
// thread, with each entry's alpha-support box tested against the four 16 x 4 pixel
// bands of the tile's waves, giving each wave the ordered list of entries that may
// composite in it).  Per batch:
//  (a) a 256-bit mask of the entries every pixel composited (the forward pass's record
//      for the tile's first GSN_MASK_BATCHES batches; later batches evaluate the wave's
//      entries that come before the pixel's stopping entry again), and one ballot per
//      (entry, wave);
// then, in rounds that each take the longest run of entries whose composited
// (pixel, entry) pairs fit in LDS (usually the whole batch):
//  (b) a block scan over the (entry, wave) ballot counts gives every pair a slot;
//  (c) every pixel walks its composited entries front to back (transmittance,
//      colour behind the splat) and stores (T, G, a_R, a_G, a_B) in the pair's slot;
//  (d) for every entry with pairs, the 44 statistics are summed over its pairs in a
//      fixed order (SG lanes per entry, or LG for an entry with more than BIG pairs, handed
//      out to waves from a block-wide counter)
//      and the tile's partial sum is written at the (tile, kernel) pair's slot.
//      Only contributing pairs do the 44-term work.
// GN: local Gauss-Newton statistics (no loss-gradient times image-curvature terms).  CT: the type of
// the colour sums along the ray (double; float in the mixed form, from the single-precision image).
__device__ __forceinline__ uint32_t wave_max(uint32_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = max(v, (uint32_t)__shfl_xor((int)v, off, 64));
    return v;
}

template <bool GN, class CT, bool STEPS>
__global__ __launch_bounds__(GSN_BLOCK, 3) void raster_bwd_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids,
    const float4* __restrict__ rec, uint32_t n, DevCam cam, DevRenderOpts ro,
    const double* __restrict__ img64, const float* __restrict__ img, const uint32_t* __restrict__ ncontrib,
    const uint64_t* __restrict__ masks,
    const float* __restrict__ dLm, const float* __restrict__ hdm, float* __restrict__ partial,
    uint8_t* __restrict__ flags, uint8_t* __restrict__ kflag, unsigned long long* __restrict__ counts) {
    constexpr int NW = GSN_BLOCK / 64;
    __shared__ float4 r_a[GSN_BLOCK], r_b[GSN_BLOCK], r_c[GSN_BLOCK];
    __shared__ uint32_t r_slot[GSN_BLOCK], r_id[GSN_BLOCK];
    __shared__ uint8_t r_list[NW][GSN_BLOCK];
    __shared__ uint32_t r_cnt[NW][NW];  // [band][loader wave]
    __shared__ float4 s_lm0[GSN_BLOCK];  // per pixel: dL_R, dL_G, dL_B, h_R
    __shared__ float2 s_lm1[GSN_BLOCK];  // h_G, h_B
    __shared__ uint64_t s_mask[GSN_BLOCK][NW];
    __shared__ uint32_t s_off[GSN_BLOCK * NW + 1];
    __shared__ uint32_t s_wsum[NW];
    __shared__ uint8_t s_act[GSN_BLOCK], s_big[GSN_BLOCK];  // entries of the round with <= BIG / > BIG pairs
    __shared__ uint32_t s_nact[NW], s_nbig[NW], s_work;
    __shared__ float4 s_pa[PMAX];
    __shared__ float s_pb[PMAX];
    __shared__ uint8_t s_pix[PMAX];
    __shared__ uint32_t s_max;
    const int tid = threadIdx.x;
    const int tile = (int)order[blockIdx.x];
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * GSN_TILE + (tid % GSN_TILE);
    const int py = ty * GSN_TILE + (tid / GSN_TILE);
    const bool inside = px < cam.W && py < cam.H;
    const int lane = __lane_id(), wave = tid / 64;
    const float tx0 = (float)(tx * GSN_TILE), tx1 = tx0 + (float)(GSN_TILE - 1);
    const float ty0 = (float)(ty * GSN_TILE);
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint2 rg = ranges[tile];
    const size_t np = (size_t)cam.W * cam.H, pi = (size_t)py * cam.W + px;
    CT cf[3] = {CT(0), CT(0), CT(0)};
    uint32_t nc = 0;
    {
        float dlv[3], hv[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            dlv[ch] = inside ? dLm[ch * np + pi] : 0.f;
            hv[ch] = inside ? hdm[ch * np + pi] : 0.f;
            if (inside) cf[ch] = img64 ? (CT)img64[ch * np + pi] : (CT)img[ch * np + pi];
        }
        s_lm0[tid] = make_float4(dlv[0], dlv[1], dlv[2], hv[0]);
        s_lm1[tid] = make_float2(hv[1], hv[2]);
    }
    if (inside) nc = ncontrib[pi];
    if (tid == 0) s_max = 0;
    __syncthreads();
    {
        uint32_t m = nc;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
        if (lane == 0) atomicMax(&s_max, m);
    }
    __syncthreads();
    const uint32_t end = rg.x + s_max;
    float T = 1.f;
    CT Ca0 = CT(0), Ca1 = CT(0), Ca2 = CT(0);
    const float fpx = (float)px, fpy = (float)py;
    uint32_t n_eval = 0, n_act = 0, n_part = 0, n_stage = 0, n_steps = 0;  // n_steps: the wave's, in every lane
    // level-2 profiling: the wave's shader-clock cycles in staging and masks (a), the slot scan (b), the
    // per-pixel walk (c) and the per-entry sums (d)
    unsigned long long cyc[4] = {0ull, 0ull, 0ull, 0ull}, t_mark = STEPS ? clock64() : 0ull;
    auto lap = [&](int ph) {
        if (STEPS) {
            const unsigned long long now = clock64();
            cyc[ph] += now - t_mark;
            t_mark = now;
        }
    };
    for (uint32_t base = rg.x; base < end; base += GSN_BLOCK) {
        const int bcnt = (int)min((uint32_t)GSN_BLOCK, end - base);
        // stage the batch: one entry per thread, its slot and its band mask
#pragma unroll
        for (int w = 0; w < NW; ++w) s_mask[tid][w] = 0ull;
        uint32_t bandmask = 0;
        if (tid < bcnt) {
            ++n_stage;
            const uint32_t id = ids[base + tid];
            const float4* rp = rec + 4 * (size_t)id;  // the kernel's 64-byte record: one gather
            const float4 a = rp[0], b = rp[1], c4 = rp[2], d4 = rp[3];
            r_a[tid] = a;
            r_b[tid] = b;
            r_c[tid] = c4;
            const float4 box = splat_alpha_box(a, b, c4, ro.alpha_min);
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (!box_misses(box, tx0, tx1, ty0 + 4.f * w, ty0 + 4.f * w + 3.f) &&
                    !ellipse_misses(a, b, c4, ro.alpha_min, tx0, tx1, ty0 + 4.f * w, ty0 + 4.f * w + 3.f))
                    bandmask |= 1u << w;
            // the (tile, kernel) slot: the kernel's pair offset plus the tile's row-major place in its rectangle
            const uint32_t rx = __float_as_uint(d4.x), ry = __float_as_uint(d4.y), off = __float_as_uint(d4.z);
            const uint32_t x0 = rx & 0xffffu, y0 = rx >> 16, x1 = ry & 0xffffu;
            r_slot[tid] = off + ((uint32_t)ty - y0) * (x1 - x0) + ((uint32_t)tx - x0);
            r_id[tid] = id;
        }
        uint64_t bal[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            bal[w] = __ballot((bandmask >> w) & 1u);
            if (lane == 0) r_cnt[w][wave] = (uint32_t)__popcll(bal[w]);
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if ((bandmask >> w) & 1u) {
                uint32_t off = 0;
#pragma unroll
                for (int v = 0; v < NW; ++v) off += v < wave ? r_cnt[w][v] : 0u;
                r_list[w][off + (uint32_t)__popcll(bal[w] & lt_mask)] = (uint8_t)tid;
            }
        }
        uint32_t nl = 0;
#pragma unroll
        for (int v = 0; v < NW; ++v) nl += r_cnt[wave][v];
        __syncthreads();
        // (a) which of the batch's entries this pixel composited (256-bit mask, word by word): recorded
        // by the forward pass for the tile's first GSN_MASK_BATCHES batches, evaluated again after
        uint64_t bits[NW] = {0ull, 0ull, 0ull, 0ull};
        const uint32_t batch = (base - rg.x) / GSN_BLOCK;
        if (batch < (uint32_t)GSN_MASK_BATCHES) {
            // the forward pass's pixel-major words
            const uint64_t* mb = masks + ((size_t)tile * GSN_MASK_BATCHES + batch) * NW * GSN_BLOCK + tid;
#pragma unroll
            for (int w = 0; w < NW; ++w) bits[w] = mb[(size_t)w * GSN_BLOCK];
        } else {
            uint32_t i = 0;
            for (; i < nl; ++i) {
                const int j = r_list[wave][i];
                if (base + j - rg.x >= nc) break;
                ++n_eval;
                const SplatEval ev = eval_splat(r_a[j], r_b[j], r_c[j], fpx, fpy, ro.alpha_max);
                if (ev.alpha >= ro.alpha_min) {
#pragma unroll
                    for (int w = 0; w < NW; ++w)
                        if ((j >> 6) == w) bits[w] |= 1ull << (j & 63);
                }
            }
            if (STEPS) n_steps += wave_max(i < nl ? i + 1 : i);  // the breaking step counts
        }
        // per (entry, wave): the wave's pixels that composited the entry (the transpose of the pixels'
        // masks), one ballot per entry that some pixel of the wave composited
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            uint64_t any = bits[w];
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) any |= (uint64_t)__shfl_xor((unsigned long long)any, off, 64);
            while (any) {  // uniform across the wave
                const int jj = __ffsll((unsigned long long)any) - 1;
                any &= any - 1;
                const uint64_t m = __ballot((bits[w] >> jj) & 1ull);
                if (lane == 0) s_mask[w * 64 + jj][wave] = m;
            }
        }
        __syncthreads();
        lap(0);
        // (b) slots: block-wide exclusive scan of the batch's pair counts in (entry, wave) order, once per
        // batch; a round's slots are offsets from the scan at its first entry.  Thread t owns the four
        // cells of entry t.
        {
            {
                uint32_t c[NW], tot = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    c[w] = (uint32_t)__popcll(s_mask[tid][w]);
                    tot += c[w];
                }
                uint32_t v = tot;
#pragma unroll
                for (int d = 1; d < 64; d <<= 1) {
                    const uint32_t o = __shfl_up(v, d, 64);
                    if (lane >= d) v += o;
                }
                if (lane == 63) s_wsum[wave] = v;
                __syncthreads();
                uint32_t sb = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) sb += w < wave ? s_wsum[w] : 0u;
                uint32_t o = sb + v - tot;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    s_off[tid * NW + w] = o;
                    o += c[w];
                }
                if (tid == GSN_BLOCK - 1) s_off[GSN_BLOCK * NW] = o;
            }
            __syncthreads();
        }
        for (int r0 = 0; r0 < bcnt;) {
            // the round takes entries r0..r1-1: the largest r1 <= bcnt with s_off[r1 * NW] - s_off[r0 * NW]
            // <= PMAX (one entry has at most 256 pairs, so r1 > r0)
            const uint32_t rbase = s_off[r0 * NW];
            int lo = r0 + 1, hi = bcnt;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (s_off[mid * NW] - rbase <= (uint32_t)PMAX) lo = mid; else hi = mid - 1;
            }
            const int r1 = lo;
            lap(1);
            // (c) front to back over the pixel's composited entries r0..r1-1
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const int wlo = w * 64, whi = wlo + 64;
                if (r1 <= wlo || r0 >= whi) continue;
                uint64_t rem = bits[w];
                if (r0 > wlo) rem &= ~0ull << (r0 - wlo);
                if (r1 < whi) rem &= (1ull << (r1 - wlo)) - 1ull;
                if (STEPS) n_steps += wave_max((uint32_t)__popcll(rem));
                while (rem) {
                    const int j = wlo + __ffsll((unsigned long long)rem) - 1;
                    rem &= rem - 1;
                    ++n_act;
                    const float4 b = r_b[j], cc = r_c[j];
                    const SplatEval ev = eval_splat(r_a[j], b, cc, fpx, fpy, ro.alpha_max);
                    const float al = ev.alpha, wT = al * T;
                    const CT wd = (CT)wT;
                    Ca0 += wd * (CT)b.w;
                    Ca1 += wd * (CT)cc.x;
                    Ca2 += wd * (CT)cc.y;
                    // hardware reciprocal (within 1 ulp; the library's divisions are otherwise correctly
                    // rounded): only the pair terms use it, no decision depends on it
                    const float inv = __builtin_amdgcn_rcpf(1.0f - al);
                    const uint32_t slot =
                        s_off[j * NW + wave] - rbase + (uint32_t)__popcll(s_mask[j][wave] & lt_mask);
                    s_pa[slot] = make_float4(T, ev.G, T * b.w - (float)(cf[0] - Ca0) * inv,
                                             T * cc.x - (float)(cf[1] - Ca1) * inv);
                    s_pb[slot] = T * cc.y - (float)(cf[2] - Ca2) * inv;
                    s_pix[slot] = (uint8_t)tid;
                    T *= (1.0f - al);
                }
            }
            lap(2);
            // (d) per-entry sums.  Entries of the round with 1..BIG pairs go to groups of SG lanes, larger
            // ones to groups of LG; a group sums its entry's pairs lane-strided and then across its lanes
            // with DPP row operations, so every sum is taken in one fixed order.  Waves take the work
            // from a block-wide counter (large entries first), so they finish the round together.
            const uint32_t pc = (tid >= r0 && tid < r1) ? s_off[(tid + 1) * NW] - s_off[tid * NW] : 0u;
            const bool small = pc > 0 && pc <= (uint32_t)BIG, large = pc > (uint32_t)BIG;
            const uint64_t sbal = __ballot(small), lbal = __ballot(large);
            if (lane == 0) {
                s_nact[wave] = (uint32_t)__popcll(sbal);
                s_nbig[wave] = (uint32_t)__popcll(lbal);
            }
            if (tid == 0) s_work = 0;
            __syncthreads();
            uint32_t nsmall = 0, nlarge = 0;
            {
                uint32_t off = 0, offb = 0;
#pragma unroll
                for (int w = 0; w < NW; ++w) {
                    off += w < wave ? s_nact[w] : 0u;
                    offb += w < wave ? s_nbig[w] : 0u;
                    nsmall += s_nact[w];
                    nlarge += s_nbig[w];
                }
                if (small) s_act[off + (uint32_t)__popcll(sbal & lt_mask)] = (uint8_t)tid;
                if (large) s_big[offb + (uint32_t)__popcll(lbal & lt_mask)] = (uint8_t)tid;
            }
            __syncthreads();
            {
                // whole waves take work units from a block-wide counter, large entries first: a unit is
                // 64 / LG large entries (one per LG-lane group) or 64 / SG small ones (one per SG-lane group)
                constexpr uint32_t PL = 64 / LG, PS = 64 / SG;
                const uint32_t nlu = (nlarge + PL - 1) / PL, nsu = (nsmall + PS - 1) / PS;
                for (;;) {
                    uint32_t u = 0;
                    if (lane == 0) u = atomicAdd(&s_work, 1u);
                    u = (uint32_t)__shfl((int)u, 0, 64);
                    if (u >= nlu + nsu) break;  // uniform across the wave
                    float acc[GSN_NZ];
#pragma unroll
                    for (int f = 0; f < GSN_NZ; ++f) acc[f] = 0.f;
                    if (u < nlu) {
                        const int r = lane % LG;
                        const uint32_t k = u * PL + (uint32_t)(lane / LG);
                        int e = 0;
                        if (k < nlarge) {
                            e = s_big[k];
                            const uint32_t q0 = s_off[e * NW] - rbase, q1 = s_off[(e + 1) * NW] - rbase;
                            for (uint32_t i = q0 + r; i < q1; i += LG)
                                pair_stats<GN>(r_a[e], r_b[e], r_c[e], s_pa, s_pb, s_pix, s_lm0, s_lm1, i, tx, ty,
                                               ro.alpha_max, acc);
                        }
#pragma unroll
                        for (int f = 0; f < kLiveZ; ++f) acc[f] = group_sum<LG>(acc[f]);
                        if (k < nlarge && r == group_writer<LG>()) {
                            write_partial(partial, flags, r_slot[e], acc);
                            kflag[r_id[e]] = 1;
                            ++n_part;
                        }
                    } else {
                        const int r = lane % SG;
                        const uint32_t k = (u - nlu) * PS + (uint32_t)(lane / SG);
                        int e = 0;
                        if (k < nsmall) {
                            e = s_act[k];
                            const uint32_t q0 = s_off[e * NW] - rbase, q1 = s_off[(e + 1) * NW] - rbase;
                            for (uint32_t i = q0 + r; i < q1; i += SG)
                                pair_stats<GN>(r_a[e], r_b[e], r_c[e], s_pa, s_pb, s_pix, s_lm0, s_lm1, i, tx, ty,
                                               ro.alpha_max, acc);
                        }
#pragma unroll
                        for (int f = 0; f < kLiveZ; ++f) acc[f] = group_sum<SG>(acc[f]);
                        if (k < nsmall && r == group_writer<SG>()) {
                            write_partial(partial, flags, r_slot[e], acc);
                            kflag[r_id[e]] = 1;
                            ++n_part;
                        }
                    }
                }
            }
            r0 = r1;
            __syncthreads();
            lap(3);
        }
    }
    if (counts) {
        __shared__ unsigned long long s_cnt[9];
        if (tid < 9) s_cnt[tid] = 0;
        __syncthreads();
        if (STEPS && lane == 0)
            for (int ph = 0; ph < 4; ++ph) atomicAdd(&s_cnt[5 + ph], cyc[ph]);
        atomicAdd(&s_cnt[0], (unsigned long long)n_eval);
        atomicAdd(&s_cnt[1], (unsigned long long)n_act);
        atomicAdd(&s_cnt[2], (unsigned long long)n_part);
        atomicAdd(&s_cnt[3], (unsigned long long)n_stage);
        if (STEPS && lane == 0) atomicAdd(&s_cnt[4], (unsigned long long)n_steps);
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&counts[GSN_COUNT_BWD_EVALS], s_cnt[0]);
            atomicAdd(&counts[GSN_COUNT_BWD_ACTIVE], s_cnt[1]);
            atomicAdd(&counts[GSN_COUNT_PARTIALS], s_cnt[2]);
            atomicAdd(&counts[GSN_COUNT_BWD_STAGED], s_cnt[3]);
            atomicAdd(&counts[GSN_COUNT_BWD_WAVE_STEPS], s_cnt[4]);
            if (STEPS)
                for (int ph = 0; ph < 4; ++ph) atomicAdd(&counts[GSN_COUNT_BWD_CYCLES + ph], s_cnt[5 + ph]);
        }
    }
}

// One wave per kReduceKernels consecutive kernels.  Most kernels have no written slot in a view (their
// kernel flag is clear): for them only the coverage entry is written (zero), which the chain
// kernels test first.  The wave then takes its flagged kernels one after another: the kernel's
// (tile, kernel) slots are scanned 64 at a time, and lane f < 44 adds statistic f of every slot
// the backward pass wrote, in slot order and in double (deterministic, coalesced 176-byte reads
// per slot).  A wave per kernel would spend most of the launch starting waves that only read
// a clear flag.
// Kernels per wave of the pair reduction: the kernels a view reaches come in runs (the ids of a
// surface are contiguous), and a wave sums its flagged kernels one after another, so fewer kernels per
// wave spread a run's serial load latencies over more waves.
constexpr int kReduceKernels = 16;

template <class Acc>
__global__ __launch_bounds__(256) void reduce_pairs_kernel(int n, const uint2* __restrict__ rect,
                                                           const uint32_t* __restrict__ pair_off,
                                                           const float* __restrict__ partial,
                                                           const uint8_t* __restrict__ flags,
                                                           const uint8_t* __restrict__ kflag,
                                                           const float* __restrict__ primary_cov,
                                                           float* __restrict__ cov_out,
                                                           float* __restrict__ zf, double* __restrict__ zq) {
    const int lane = __lane_id();
    const int k0 = (blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64) * kReduceKernels;
    if (k0 >= n) return;
    // the wave's kReduceKernels kernels: those without partials (or, for a secondary view, not seen by
    // the primary) get a zero coverage, the others are summed one after another by the whole wave
    const int kl = k0 + lane;
    const bool mine = lane < kReduceKernels && kl < n;
    const bool has = mine && kflag[kl] != 0 && (!primary_cov || primary_cov[kl] > 0.f);
    if (mine && !has) {
        zf[(size_t)kl * GSN_NZ + GSN_ZCOV] = 0.f;
        zq[(size_t)kl * kZq + kZqCov] = 0.0;
    }
    // every lane reads its own kernel's slot range up front (one coalesced load instead of a
    // dependent load per kernel); the wave then takes each kernel's range from its lane
    uint32_t my_nt = 0, my_off = 0;
    if (has) {
        const uint2 rc = rect[kl];
        my_nt = ((rc.y & 0xffffu) - (rc.x & 0xffffu)) * ((rc.y >> 16) - (rc.x >> 16));
        my_off = pair_off[kl];
    }
    uint64_t todo = __ballot(has);
    while (todo) {  // uniform across the wave
        const int li = __ffsll((unsigned long long)todo) - 1;
        todo &= todo - 1;
        const int k = k0 + li;
        const uint32_t nt = (uint32_t)__shfl((int)my_nt, li, 64);
        const uint32_t off = (uint32_t)__shfl((int)my_off, li, 64);
        Acc acc = Acc(0);
        for (uint32_t base = 0; base < nt; base += 64) {
            const bool fl = base + lane < nt && flags[off + base + lane] != 0;
            uint64_t m = __ballot(fl);
            while (m) {  // up to eight written slots per step: their loads overlap, the adds keep slot order
                float v[8];
                int cntv = 0;
#pragma unroll
                for (int t = 0; t < 8; ++t) {
                    v[t] = 0.f;
                    if (m) {
                        const int i = __ffsll((unsigned long long)m) - 1;
                        m &= m - 1;
                        if (lane < GSN_NZ) v[t] = partial[(size_t)(off + base + i) * GSN_NZ + lane];
                        ++cntv;
                    }
                }
#pragma unroll
                for (int t = 0; t < 8; ++t)
                    if (t < cntv) acc += (Acc)v[t];
            }
        }
        // every statistic in single precision (192 contiguous bytes), and in double those the rotation and
        // scale chain rule reads (the plain form's conic statistics and coverage)
        if (lane < GSN_NZ) zf[(size_t)k * GSN_NZ + lane] = (float)(double)acc;
        const int q = zq_slot(lane);
        if (q >= 0) zq[(size_t)k * kZq + q] = (double)acc;
        // the primary view's coverage row of the blocks, which the secondary views' sums read
        if (cov_out && lane == GSN_ZCOV) cov_out[k] = (float)(double)acc;
    }
}

__device__ __forceinline__ void load_kparams(const float* __restrict__ pos, const float* __restrict__ rot,
                                             const float* __restrict__ scale, const float4* __restrict__ rec, int n,
                                             int k, KParams& kp) {
#pragma unroll
    for (int a = 0; a < 3; ++a) kp.p[a] = pos[(size_t)a * n + k];
#pragma unroll
    for (int a = 0; a < 4; ++a) kp.q[a] = rot[(size_t)a * n + k];
#pragma unroll
    for (int a = 0; a < 3; ++a) kp.s[a] = scale[(size_t)a * n + k];
    const float4 r1 = rec[4 * (size_t)k + 1];
    kp.fc = r1.x;
    kp.fs = r1.y;
}

// One thread per kernel: position, opacity and per-view colour blocks from the summed
// statistics (single precision), and the optional float copy of the statistics.
template <bool GN>
__global__ __launch_bounds__(128) void chain_pos_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale,
    const float* __restrict__ sh, int n, int K, const float* __restrict__ zf, const double* __restrict__ zq,
    const float4* __restrict__ rec,
    DevCam cam, float kappa, float weight, int slot, float* __restrict__ blk, float* __restrict__ sr,
    uint8_t* __restrict__ contrib, float* __restrict__ zstats) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double cov = zq[(size_t)k * kZq + kZqCov];
    const bool adds = cov > 0.0 && (float)cov > 0.f;
    contrib[k] = adds ? 1 : 0;
    if (!(cov > 0.0)) {  // no pixel of this view composited the kernel
        if (zstats) {
#pragma unroll
            for (int f = 0; f < GSN_NZ; ++f) zstats[(size_t)f * n + k] = 0.f;
        }
        return;
    }
    float z[GSN_NZ];
    {
        const float4* zp = reinterpret_cast<const float4*>(zf + (size_t)k * GSN_NZ);
#pragma unroll
        for (int f = 0; f < GSN_NZ / 4; ++f) {
            const float4 v = zp[f];
            z[4 * f] = v.x;
            z[4 * f + 1] = v.y;
            z[4 * f + 2] = v.z;
            z[4 * f + 3] = v.w;
        }
    }
    if (zstats) {
#pragma unroll
        for (int f = 0; f < GSN_NZ; ++f) zstats[(size_t)f * n + k] = z[f];
    }
    if (!adds) return;
    KParams kp;
    load_kparams(pos, rot, scale, rec, n, k, kp);
    const size_t N = (size_t)n;
    {
        float g[3], H[6];
        chain_position(kp, sh + k, N, K, cam, kappa, z, GN, g, H);
#pragma unroll
        for (int a = 0; a < 3; ++a) sr[a * N + k] = weight * g[a];
#pragma unroll
        for (int a = 0; a < 6; ++a) sr[(3 + a) * N + k] = weight * H[a];
    }
    sr[27 * N + k] = weight * z[5];
    sr[28 * N + k] = weight * z[42];
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
    blk[(vb + 9) * N + k] = z[GSN_ZCOV];
    // this view's share of the sum over the views of sum (alpha T)^2 (the overlap share's numerator)
    sr[(size_t)kSumOverlap * N + k] = weight * z[GSN_ZW2];
}

// One thread per kernel: rotation and scale blocks, in double from the double sums of the
// conic statistics (both Hessians cancel strongly for thin splats); Re = float in the mixed form.
template <bool GN, class Re>
__global__ __launch_bounds__(128) void chain_rs_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale, int n,
    const double* __restrict__ zq, const float4* __restrict__ rec, DevCam cam, float kappa, float weight,
    float* __restrict__ sr) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* zk = zq + (size_t)k * kZq;
    if (!(zk[kZqCov] > 0.0 && (float)zk[kZqCov] > 0.f)) return;  // the gate of chain_pos_kernel
    Re gq[3], Hq[3][3];
    q_stats_packed(zk, gq, Hq);
    KParams kp;
    load_kparams(pos, rot, scale, rec, n, k, kp);
    const size_t N = (size_t)n;
    Re g[3], H[6];
    chain_rotation(kp, cam, kappa, gq, Hq, GN, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) sr[(9 + a) * N + k] = (float)((Re)weight * g[a]);
#pragma unroll
    for (int a = 0; a < 6; ++a) sr[(12 + a) * N + k] = (float)((Re)weight * H[a]);
    chain_scale(kp, cam, kappa, gq, Hq, GN, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) sr[(18 + a) * N + k] = (float)((Re)weight * g[a]);
#pragma unroll
    for (int a = 0; a < 6; ++a) sr[(21 + a) * N + k] = (float)((Re)weight * H[a]);
}

// Adds the views' shares of the rows summed over the views (position, rotation, scaling, opacity,
// the overlap numerator) to the blocks, view after view in the order given, for the kernels each view
// reached: the same additions, in the same order, whether the views were accumulated one call at a
// time or together.
__global__ void sum_views_kernel(float* __restrict__ blk, int n, int V, SumViews sv) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    uint32_t mask = 0;
    for (int v = 0; v < sv.count; ++v) mask |= (sv.contrib[v][k] != 0 ? 1u : 0u) << v;
    if (!mask) return;
    // every row is loaded before any store (the views' rows and the blocks are separate arrays)
    constexpr int NR = kSumOverlap + 1;
    const size_t over = (size_t)GSN_BLK_BASE + (size_t)GSN_BLK_VIEW * V;
    float a[NR];
#pragma unroll
    for (int r = 0; r < NR; ++r) a[r] = blk[(r < kSumOverlap ? (size_t)r : over) * N + k];
    for (int v = 0; v < sv.count; ++v) {
        if (!((mask >> v) & 1u)) continue;
        const float* __restrict__ src = sv.rows[v];
        float t[NR];
#pragma unroll
        for (int r = 0; r < NR; ++r) t[r] = src[(size_t)r * N + k];
#pragma unroll
        for (int r = 0; r < NR; ++r) a[r] += t[r];
    }
#pragma unroll
    for (int r = 0; r < NR; ++r) blk[(r < kSumOverlap ? (size_t)r : over) * N + k] = a[r];
}

}  // namespace

template <bool STEPS>
static auto bwd_variant(bool gauss_newton, bool fp32) {
    return gauss_newton ? (fp32 ? raster_bwd_kernel<true, float, STEPS> : raster_bwd_kernel<true, double, STEPS>)
                        : (fp32 ? raster_bwd_kernel<false, float, STEPS> : raster_bwd_kernel<false, double, STEPS>);
}

void launch_raster_bwd(const gsn_frame& f, const float* dL, const float* hd, bool gauss_newton,
                       unsigned long long* counts, bool steps, hipStream_t s) {
    const int tiles = f.tiles_x * f.tiles_y;
    // the colour sums of the frame's render: double, or float in the mixed form
    auto kern = steps && counts ? bwd_variant<true>(gauss_newton, f.fp32) : bwd_variant<false>(gauss_newton, f.fp32);
    kern<<<tiles, GSN_BLOCK, 0, s>>>(
        bp<uint2>(f.ranges), bp<uint32_t>(f.bwd_order), f.list_ids, bp<float4>(f.rec),
        (uint32_t)f.n, f.cam, f.ro, f.fp32 ? nullptr : bp<double>(f.img64), bp<float>(f.img),
        bp<uint32_t>(f.ncontrib), bp<uint64_t>(f.masks), dL, hd, bp<float>(f.partial), bp<uint8_t>(f.flags),
        bp<uint8_t>(f.kflag), counts);
}

void launch_reduce_pairs(const gsn_frame& f, const gsn_gaussians& g, int slot, bool fp32, const gsn_blocks& b,
                         hipStream_t s) {
    if (g.n == 0) return;
    auto red_k = fp32 ? reduce_pairs_kernel<float> : reduce_pairs_kernel<double>;
    float* cov = b.d_data + (size_t)29 * g.n;
    red_k<<<(g.n + 4 * kReduceKernels - 1) / (4 * kReduceKernels), 256, 0, s>>>(g.n, bp<uint2>(f.rect), bp<uint32_t>(f.pair_off), bp<float>(f.partial),
                                            bp<uint8_t>(f.flags), bp<uint8_t>(f.kflag), slot > 0 ? cov : nullptr,
                                            slot == 0 ? cov : nullptr, bp<float>(f.zsum_f), bp<double>(f.zsum));
}

void launch_sum_views(const gsn_blocks& b, const SumViews& sv, hipStream_t s) {
    if (b.n > 0 && sv.count > 0) sum_views_kernel<<<(b.n + 255) / 256, 256, 0, s>>>(b.d_data, b.n, b.n_views, sv);
}

void launch_chain(const gsn_frame& f, const gsn_gaussians& g, float weight, int slot, bool gauss_newton, bool fp32,
                  const gsn_blocks& b, float* zstats_out, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    auto pos_k = gauss_newton ? chain_pos_kernel<true> : chain_pos_kernel<false>;
    auto rs_k = gauss_newton ? (fp32 ? chain_rs_kernel<true, float> : chain_rs_kernel<true, double>)
                             : (fp32 ? chain_rs_kernel<false, float> : chain_rs_kernel<false, double>);
    pos_k<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_sh, g.n, K, bp<float>(f.zsum_f),
                                            bp<double>(f.zsum),
                                            bp<float4>(f.rec), f.cam, f.ro.kappa, weight, slot, b.d_data,
                                            bp<float>(f.sumrows), bp<uint8_t>(f.contrib), zstats_out);
    rs_k<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.n, bp<double>(f.zsum), bp<float4>(f.rec),
                                           f.cam, f.ro.kappa, weight, bp<float>(f.sumrows));
}
