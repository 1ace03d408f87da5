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
// depth-ordered list front to back with the forward pass's decisions, stages
// the contributing (pixel, splat) pairs of each round in LDS, and sums each
// splat's 44 statistics over its pairs (see raster_bwd_kernel); the tile's
// partial sum is written at the (tile, kernel) pair's slot.
// reduce_pairs: one wave per kernel sums its pair slots in a fixed order (no
// atomics: results are deterministic); chain_pos / chain_rs: one thread per
// kernel applies the chain rule through the projection with second-order jets
// and adds the attribute blocks (position, opacity, colour / rotation, scale).
#include "gsn_internal.h"
#include "chain.h"

namespace {

constexpr int BS = 32;      // list entries examined per round
constexpr int PMAX = 2048;  // active (pixel, entry) pairs staged per round
constexpr int GRP = 8;      // threads that sum one entry's pairs

// Contribution of one active (pixel, splat) pair to the 44 statistics (see the header comment).
__device__ __forceinline__ void pair_terms(const float4 a, const float4 b, float G, float T, const float av[3],
                                           float dx, float dy, const float dl[3], const float hh[3], float amax,
                                           float* z) {
    const float sig = b.z, q1 = a.z, q2 = a.w;
    const float sGraw = sig * G;
    const bool clamped = sGraw > amax;
    const float al = clamped ? amax : sGraw;
    const float wT = al * T;
    const float A1 = dl[0] * av[0] + dl[1] * av[1] + dl[2] * av[2];
    const float A2 = hh[0] * av[0] * av[0] + hh[1] * av[1] * av[1] + hh[2] * av[2] * av[2];
#pragma unroll
    for (int f = 0; f < GSN_NZ; ++f) z[f] = 0.f;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        z[6 + ch] = dl[ch] * wT;
        z[39 + ch] = hh[ch] * wT * wT;
    }
    z[43] = wT;
    if (clamped) return;
    const float u[5] = {-q1 * dx, -q2 * dy, -0.5f * dx * dx, -dx * dy, -0.5f * dy * dy};
    const float k1 = A1 * sGraw;
    const float k2 = A2 * sGraw * sGraw + k1;
#pragma unroll
    for (int i = 0; i < 5; ++i) z[i] = k1 * u[i];
    z[5] = A1 * G;
    // H_ww: k2 u u^T + k1 d2f, d2f has -Q' on (pi', pi') and -d' on (pi', Q')
    int idx = 9;
#pragma unroll
    for (int i = 0; i < 5; ++i)
#pragma unroll
        for (int j = i; j < 5; ++j, ++idx) z[idx] = k2 * u[i] * u[j];
    z[9 + 0] -= k1 * q1;  // (pi'_1, pi'_1)
    z[9 + 2] -= k1 * dx;  // (pi'_1, Q'_11)
    z[9 + 3] -= k1 * dy;  // (pi'_1, Q'_12)
    z[9 + 5] -= k1 * q2;  // (pi'_2, pi'_2)
    z[9 + 7] -= k1 * dx;  // (pi'_2, Q'_12)
    z[9 + 8] -= k1 * dy;  // (pi'_2, Q'_22)
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        const float bch = sGraw * T * (hh[ch] * av[ch] * al + dl[ch]);
#pragma unroll
        for (int i = 0; i < 5; ++i) z[24 + i * 3 + ch] = bch * u[i];
    }
    z[42] = A2 * G * G;
}

// One workgroup per tile.  Each round examines up to BS list entries:
//  (a) every pixel evaluates which of them it composited (alpha >= alpha_min and
//      before its stopping entry) -> one ballot mask per (entry, wave);
//  (b) a scan over (entry, wave) gives every active (pixel, entry) pair a slot in
//      LDS; the round keeps the longest prefix of entries whose pairs fit;
//  (c) every pixel walks its active entries front to back (transmittance, colour
//      behind the splat) and stores (T, G, a_R, a_G, a_B) in the pair's slot;
//  (d) GRP threads per entry sum the 44 statistics over that entry's pairs in
//      double, in pixel order, and write the tile's partial sum at the
//      (tile, kernel) pair's slot.  Only contributing pairs do the 44-term work.
__global__ __launch_bounds__(GSN_BLOCK) void raster_bwd_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ ids, const float4* __restrict__ rec,
    const uint2* __restrict__ rect, const uint32_t* __restrict__ pair_off, uint32_t n, DevCam cam, DevRenderOpts ro,
    const double* __restrict__ img64, const uint32_t* __restrict__ ncontrib, const float* __restrict__ dLm,
    const float* __restrict__ hdm, float* __restrict__ partial, uint8_t* __restrict__ flags,
    unsigned long long* __restrict__ counts) {
    __shared__ float4 r_a[BS], r_b[BS];
    __shared__ float4 r_c[BS];
    __shared__ float4 r_box[BS];
    __shared__ uint32_t r_slot[BS];
    __shared__ float s_dl[3][GSN_BLOCK], s_h[3][GSN_BLOCK];
    __shared__ uint64_t s_mask[BS][GSN_BLOCK / 64];
    __shared__ uint32_t s_off[BS * (GSN_BLOCK / 64) + 1];
    __shared__ float4 s_pa[PMAX];
    __shared__ float s_pb[PMAX];
    __shared__ uint8_t s_pix[PMAX];
    __shared__ uint32_t s_max, s_J;
    const int tid = threadIdx.x;
    const int tile = blockIdx.x;
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * GSN_TILE + (tid % GSN_TILE);
    const int py = ty * GSN_TILE + (tid / GSN_TILE);
    const bool inside = px < cam.W && py < cam.H;
    const int lane = __lane_id(), wave = tid / 64;
    const float wx0 = (float)(tx * GSN_TILE), wx1 = wx0 + (float)(GSN_TILE - 1);
    const float wy0 = (float)(ty * GSN_TILE + wave * 4), wy1 = wy0 + 3.0f;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const uint2 rg = ranges[tile];
    const size_t np = (size_t)cam.W * cam.H, pi = (size_t)py * cam.W + px;
    double cf[3] = {0, 0, 0};
    uint32_t nc = 0;
#pragma unroll
    for (int ch = 0; ch < 3; ++ch) {
        s_dl[ch][tid] = inside ? dLm[ch * np + pi] : 0.f;
        s_h[ch][tid] = inside ? hdm[ch * np + pi] : 0.f;
        if (inside) cf[ch] = img64[ch * np + pi];
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
    double Ca0 = 0.0, Ca1 = 0.0, Ca2 = 0.0;
    const float fpx = (float)px, fpy = (float)py;
    uint32_t n_eval = 0, n_act = 0;
    for (uint32_t pos = rg.x; pos < end;) {
        const int cnt = (int)min((uint32_t)BS, end - pos);
        if (tid < cnt) {
            const uint32_t id = ids[pos + tid];
            r_a[tid] = rec[id];
            r_b[tid] = rec[n + id];
            r_c[tid] = rec[2 * (size_t)n + id];
            r_box[tid] = splat_alpha_box(r_a[tid], r_b[tid], r_c[tid], ro.alpha_min);
            const uint2 rc = rect[id];
            const uint32_t x0 = rc.x & 0xffffu, y0 = rc.x >> 16, x1 = rc.y & 0xffffu;
            r_slot[tid] = pair_off[id] + ((uint32_t)ty - y0) * (x1 - x0) + ((uint32_t)tx - x0);
        }
        __syncthreads();
        // (a) which of the round's entries this pixel composited
        uint32_t bits = 0;
        for (int j = 0; j < cnt; ++j) {
            if (pos + j - rg.x >= nc) break;
            if (box_misses(r_box[j], wx0, wx1, wy0, wy1)) continue;  // uniform across the wave
            ++n_eval;
            const SplatEval ev = eval_splat(r_a[j], r_b[j], r_c[j], fpx, fpy, ro.alpha_max);
            if (ev.alpha >= ro.alpha_min) bits |= 1u << j;
        }
        for (int j = 0; j < cnt; ++j) {
            const uint64_t m = __ballot((bits >> j) & 1u);
            if (lane == 0) s_mask[j][wave] = m;
        }
        __syncthreads();
        // (b) slots: exclusive scan of the pair counts in (entry, wave) order, by wave 0
        if (wave == 0) {
            const int e0 = 2 * lane, e1 = 2 * lane + 1;  // 128 (entry, wave) cells, two per lane
            const uint32_t c0 = (e0 / 4 < cnt) ? (uint32_t)__popcll(s_mask[e0 / 4][e0 % 4]) : 0u;
            const uint32_t c1 = (e1 / 4 < cnt) ? (uint32_t)__popcll(s_mask[e1 / 4][e1 % 4]) : 0u;
            uint32_t v = c0 + c1;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t o = __shfl_up(v, d, 64);
                if (lane >= d) v += o;
            }
            const uint32_t excl = v - (c0 + c1);
            s_off[e0] = excl;
            s_off[e1] = excl + c0;
            if (lane == 63) s_off[BS * 4] = v;
        }
        __syncthreads();
        if (tid == 0) {
            // longest prefix of entries whose pairs fit in PMAX (one entry has at most 256)
            int J = cnt;
            while (s_off[J * 4] > (uint32_t)PMAX) --J;
            s_J = (uint32_t)J;
        }
        __syncthreads();
        const int J = (int)s_J;
        // (c) front to back over the pixel's active entries of the prefix
        for (int j = 0; j < J; ++j) {
            if (pos + j - rg.x >= nc) break;
            if (!((bits >> j) & 1u)) continue;
            ++n_act;
            const float4 b = r_b[j], cc = r_c[j];
            const SplatEval ev = eval_splat(r_a[j], b, cc, fpx, fpy, ro.alpha_max);
            const float al = ev.alpha, wT = al * T;
            const double wd = (double)wT;
            Ca0 += wd * (double)b.w;
            Ca1 += wd * (double)cc.x;
            Ca2 += wd * (double)cc.y;
            const float inv = 1.0f / (1.0f - al);
            const uint32_t slot = s_off[j * 4 + wave] + (uint32_t)__popcll(s_mask[j][wave] & lt_mask);
            s_pa[slot] = make_float4(T, ev.G, T * b.w - (float)(cf[0] - Ca0) * inv, T * cc.x - (float)(cf[1] - Ca1) * inv);
            s_pb[slot] = T * cc.y - (float)(cf[2] - Ca2) * inv;
            s_pix[slot] = (uint8_t)tid;
            T *= (1.0f - al);
        }
        __syncthreads();
        // (d) GRP threads per entry accumulate its pairs in double, in pixel order
        {
            const int e = tid / GRP, r = tid % GRP;
            double acc[GSN_NZ];
#pragma unroll
            for (int f = 0; f < GSN_NZ; ++f) acc[f] = 0.0;
            uint32_t p0 = 0, p1 = 0;
            if (e < J) {
                p0 = s_off[e * 4];
                p1 = s_off[e * 4 + 4];
                const float4 a = r_a[e], b = r_b[e], cl = r_c[e];
                for (uint32_t i = p0 + r; i < p1; i += GRP) {
                    const float4 pa = s_pa[i];
                    const int p = s_pix[i];
                    const float av[3] = {pa.z, pa.w, s_pb[i]};
                    const float dl[3] = {s_dl[0][p], s_dl[1][p], s_dl[2][p]};
                    const float hh[3] = {s_h[0][p], s_h[1][p], s_h[2][p]};
                    const float ddx = (a.x - (float)(tx * GSN_TILE + (p % GSN_TILE))) + cl.z;
                    const float ddy = (a.y - (float)(ty * GSN_TILE + (p / GSN_TILE))) + cl.w;
                    const float d1 = b.x * ddx + b.y * ddy, d2 = b.x * ddy - b.y * ddx;
                    float z[GSN_NZ];
                    pair_terms(a, b, pa.y, pa.x, av, d1, d2, dl, hh, ro.alpha_max, z);
#pragma unroll
                    for (int f = 0; f < GSN_NZ; ++f) acc[f] += (double)z[f];
                }
            }
#pragma unroll
            for (int off = 1; off < GRP; off <<= 1)
#pragma unroll
                for (int f = 0; f < GSN_NZ; ++f) acc[f] += __shfl_xor(acc[f], off, 64);
            if (e < J && r == 0 && p1 > p0) {
                const uint32_t slot = r_slot[e];
                float4* dst = reinterpret_cast<float4*>(partial + (size_t)slot * GSN_NZ);
#pragma unroll
                for (int f = 0; f < GSN_NZ / 4; ++f)
                    dst[f] = make_float4((float)acc[4 * f], (float)acc[4 * f + 1], (float)acc[4 * f + 2],
                                         (float)acc[4 * f + 3]);
                flags[slot] = 1;
            }
        }
        __syncthreads();
        pos += (uint32_t)J;
    }
    if (counts) {
        __shared__ unsigned long long s_cnt[2];
        if (tid == 0) s_cnt[0] = s_cnt[1] = 0;
        __syncthreads();
        atomicAdd(&s_cnt[0], (unsigned long long)n_eval);
        atomicAdd(&s_cnt[1], (unsigned long long)n_act);
        __syncthreads();
        if (tid == 0) {
            atomicAdd(&counts[GSN_COUNT_BWD_EVALS], s_cnt[0]);
            atomicAdd(&counts[GSN_COUNT_BWD_ACTIVE], s_cnt[1]);
        }
    }
}

// One wave per kernel: the kernel's (tile, kernel) slots are scanned 64 at a time,
// and lane f < 44 adds statistic f of every slot the backward pass wrote, in slot
// order and in double (deterministic, coalesced 176-byte reads per slot).
__global__ __launch_bounds__(256) void reduce_pairs_kernel(int n, const uint2* __restrict__ rect,
                                                           const uint32_t* __restrict__ pair_off,
                                                           const float* __restrict__ partial,
                                                           const uint8_t* __restrict__ flags,
                                                           double* __restrict__ zsum) {
    const int k = blockIdx.x * (blockDim.x / 64) + threadIdx.x / 64;
    const int lane = __lane_id();
    if (k >= n) return;
    const uint2 rc = rect[k];
    const uint32_t nt = ((rc.y & 0xffffu) - (rc.x & 0xffffu)) * ((rc.y >> 16) - (rc.x >> 16));
    const uint32_t off = pair_off[k];
    double acc = 0.0;
    for (uint32_t base = 0; base < nt; base += 64) {
        const bool fl = base + lane < nt && flags[off + base + lane] != 0;
        uint64_t m = __ballot(fl);
        while (m) {
            const int i = __ffsll((unsigned long long)m) - 1;
            m &= m - 1;
            if (lane < GSN_NZ) acc += (double)partial[(size_t)(off + base + i) * GSN_NZ + lane];
        }
    }
    if (lane < GSN_NZ) zsum[(size_t)k * GSN_NZ + lane] = acc;
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
    const float4 r1 = rec[(size_t)n + k];
    kp.fc = r1.x;
    kp.fs = r1.y;
}

// One thread per kernel: position, opacity and per-view colour blocks from the summed
// statistics (single precision), and the optional float copy of the statistics.
__global__ __launch_bounds__(128) void chain_pos_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale,
    const float* __restrict__ sh, int n, int K, const double* __restrict__ zsum, const float4* __restrict__ rec,
    DevCam cam, float kappa, float weight, int slot, float* __restrict__ blk, float* __restrict__ zstats) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    float z[GSN_NZ];
    {
        const double2* zp = reinterpret_cast<const double2*>(zsum + (size_t)k * GSN_NZ);
#pragma unroll
        for (int f = 0; f < GSN_NZ / 2; ++f) {
            const double2 v = zp[f];
            z[2 * f] = (float)v.x;
            z[2 * f + 1] = (float)v.y;
        }
    }
    if (zstats) {
#pragma unroll
        for (int f = 0; f < GSN_NZ; ++f) zstats[(size_t)f * n + k] = z[f];
    }
    if (!(z[43] > 0.f)) return;
    KParams kp;
    load_kparams(pos, rot, scale, rec, n, k, kp);
    const size_t N = (size_t)n;
    {
        float g[3], H[6];
        chain_position(kp, sh + k, N, K, cam, kappa, z, g, H);
#pragma unroll
        for (int a = 0; a < 3; ++a) blk[a * N + k] += weight * g[a];
#pragma unroll
        for (int a = 0; a < 6; ++a) blk[(3 + a) * N + k] += weight * H[a];
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

// One thread per kernel: rotation and scale blocks, in double from the double sums of the
// conic statistics (both Hessians cancel strongly for thin splats).
__global__ __launch_bounds__(128) void chain_rs_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale, int n,
    const double* __restrict__ zsum, const float4* __restrict__ rec, DevCam cam, float kappa, float weight,
    float* __restrict__ blk) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const double* zk = zsum + (size_t)k * GSN_NZ;
    if (!(zk[43] > 0.0)) return;
    double gq[3], Hq[3][3];
    q_stats(zk, gq, Hq);
    KParams kp;
    load_kparams(pos, rot, scale, rec, n, k, kp);
    const size_t N = (size_t)n;
    double g[3], H[6];
    chain_rotation(kp, cam, kappa, gq, Hq, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) blk[(9 + a) * N + k] += (float)(weight * g[a]);
#pragma unroll
    for (int a = 0; a < 6; ++a) blk[(12 + a) * N + k] += (float)(weight * H[a]);
    chain_scale(kp, cam, kappa, gq, Hq, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) blk[(18 + a) * N + k] += (float)(weight * g[a]);
#pragma unroll
    for (int a = 0; a < 6; ++a) blk[(21 + a) * N + k] += (float)(weight * H[a]);
}

}  // namespace

void launch_raster_bwd(const gsn_frame& f, const float* dL, const float* hd, unsigned long long* counts, hipStream_t s) {
    const int tiles = f.tiles_x * f.tiles_y;
    raster_bwd_kernel<<<tiles, GSN_BLOCK, 0, s>>>(
        bp<uint2>(f.ranges), bp<uint32_t>(f.pv_a), bp<float4>(f.rec),
        bp<uint2>(f.rect), bp<uint32_t>(f.pair_off), (uint32_t)f.n, f.cam, f.ro, bp<double>(f.img64),
        bp<uint32_t>(f.ncontrib), dL, hd, bp<float>(f.partial), bp<uint8_t>(f.flags), counts);
}

void launch_reduce_chain(const gsn_frame& f, const gsn_gaussians& g, float weight, int slot, const gsn_blocks& b,
                         float* zstats_out, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    reduce_pairs_kernel<<<(g.n + 3) / 4, 256, 0, s>>>(g.n, bp<uint2>(f.rect), bp<uint32_t>(f.pair_off),
                                                      bp<float>(f.partial), bp<uint8_t>(f.flags),
                                                      bp<double>(f.zsum));
    chain_pos_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_sh, g.n, K,
                                                       bp<double>(f.zsum), bp<float4>(f.rec), f.cam, f.ro.kappa,
                                                       weight, slot, b.d_data, zstats_out);
    chain_rs_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.n, bp<double>(f.zsum),
                                                      bp<float4>(f.rec), f.cam, f.ro.kappa, weight, b.d_data);
}
