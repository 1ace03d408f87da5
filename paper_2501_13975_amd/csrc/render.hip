// render.hip -- projection, binning and forward compositing (Sec. 3, eq. 3dgs).
//
// Layout: one thread per kernel for projection; a global stable LSD radix sort
// of kernels by depth; (tile, kernel) pairs emitted in depth order and then
// stably radix-partitioned by tile id, so every tile's list comes out
// depth-ordered without a per-tile sort; one 256-thread workgroup (four
// wave64s) per 16x16 tile for compositing, splat records staged through LDS.
#include <algorithm>

#include "gsn_internal.h"
#include "chain.h"

namespace {

constexpr int kThreads = 256;

__global__ void fill_u32_kernel(uint32_t* p, uint32_t v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}
__global__ void fill_f32_kernel(float* p, float v, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

int grid_for(size_t n, int threads = kThreads, int cap = 65536) {
    size_t b = (n + threads - 1) / threads;
    if (b < 1) b = 1;
    if (b > (size_t)cap) b = cap;
    return (int)b;
}

// ---------------------------------------------------------------------------
// Binning decisions in single precision: one IEEE operation per step, left to
// right, no contraction, correctly rounded division and square root.  Any
// other implementation of the same sequence reproduces the depth key and the
// tile rectangle bit for bit.
// ---------------------------------------------------------------------------
struct BinOut {
    float tx, ty, tz, cxx, cxy, cyy, det, u, v;
    int x0, y0, x1, y1;
    bool vis;
};

__device__ __forceinline__ BinOut bin_spec(float px, float py, float pz, float qw, float qx, float qy, float qz,
                                        float s0, float s1, float s2, const DevCam& c, float kappa, float rsig) {
#pragma clang fp contract(off)
    BinOut b;
    b.vis = false;
    b.x0 = b.y0 = b.x1 = b.y1 = 0;
    const float* R = c.R;
    b.tx = ((R[0] * px + R[1] * py) + R[2] * pz) + c.t[0];
    b.ty = ((R[3] * px + R[4] * py) + R[5] * pz) + c.t[1];
    b.tz = ((R[6] * px + R[7] * py) + R[8] * pz) + c.t[2];
    if (!(b.tz > c.znear)) return b;
    const float nq = sqrtf(((qw * qw + qx * qx) + qy * qy) + qz * qz);
    const float w = ((qw) / (nq)), x = ((qx) / (nq)), y = ((qy) / (nq)), z = ((qz) / (nq));
    const float r[3][3] = {{1.0f - 2.0f * (y * y + z * z), 2.0f * (x * y - w * z), 2.0f * (x * z + w * y)},
                           {2.0f * (x * y + w * z), 1.0f - 2.0f * (x * x + z * z), 2.0f * (y * z - w * x)},
                           {2.0f * (x * z - w * y), 2.0f * (y * z + w * x), 1.0f - 2.0f * (x * x + y * y)}};
    const float s[3] = {s0, s1, s2};
    float m[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) m[i][j] = r[i][j] * s[j];
    float S[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) S[i][j] = (m[i][0] * m[j][0] + m[i][1] * m[j][1]) + m[i][2] * m[j][2];
    const float j00 = ((c.fx) / (b.tz));
    const float j02 = ((-(c.fx * b.tx)) / (b.tz * b.tz));
    const float j11 = ((c.fy) / (b.tz));
    const float j12 = ((-(c.fy * b.ty)) / (b.tz * b.tz));
    float a[2][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        a[0][k] = j00 * R[k] + j02 * R[6 + k];
        a[1][k] = j11 * R[3 + k] + j12 * R[6 + k];
    }
    float bb[2][3];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int k = 0; k < 3; ++k) bb[i][k] = (a[i][0] * S[0][k] + a[i][1] * S[1][k]) + a[i][2] * S[2][k];
    b.cxx = ((bb[0][0] * a[0][0] + bb[0][1] * a[0][1]) + bb[0][2] * a[0][2]) + kappa;
    b.cxy = (bb[0][0] * a[1][0] + bb[0][1] * a[1][1]) + bb[0][2] * a[1][2];
    b.cyy = ((bb[1][0] * a[1][0] + bb[1][1] * a[1][1]) + bb[1][2] * a[1][2]) + kappa;
    b.det = b.cxx * b.cyy - b.cxy * b.cxy;
    if (!(b.det > 0.0f)) return b;
    const float mid = 0.5f * (b.cxx + b.cyy);
    const float lam = mid + sqrtf(fmaxf(0.1f, mid * mid - b.det));
    const float radius = ceilf(rsig * sqrtf(lam));
    b.u = ((c.fx * b.tx) / (b.tz)) + c.cx;
    b.v = ((c.fy * b.ty) / (b.tz)) + c.cy;
    const float ft = (float)GSN_TILE;
    const float x0 = fminf(fmaxf(floorf(((b.u - radius) / (ft))), 0.0f), (float)c.tiles_x);
    const float x1 = fminf(fmaxf(floorf(((b.u + radius) / (ft))) + 1.0f, 0.0f), (float)c.tiles_x);
    const float y0 = fminf(fmaxf(floorf(((b.v - radius) / (ft))), 0.0f), (float)c.tiles_y);
    const float y1 = fminf(fmaxf(floorf(((b.v + radius) / (ft))) + 1.0f, 0.0f), (float)c.tiles_y);
    b.x0 = (int)x0;
    b.x1 = (int)x1;
    b.y0 = (int)y0;
    b.y1 = (int)y1;
    b.vis = (b.x1 > b.x0) && (b.y1 > b.y0);
    return b;
}

// One thread per kernel: binning decisions, conic, view-dependent colour.
__global__ __launch_bounds__(kThreads) void preprocess_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale,
    const float* __restrict__ opac, const float* __restrict__ sh, int n, int K, DevCam cam, DevRenderOpts ro,
    float4* __restrict__ rec, uint2* __restrict__ rect, uint32_t* __restrict__ depth_key,
    uint32_t* __restrict__ ids, uint32_t* __restrict__ ntiles, unsigned long long* __restrict__ culled) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const float px = pos[k], py = pos[n + k], pz = pos[2 * n + k];
    const float qw = rot[k], qx = rot[n + k], qy = rot[2 * n + k], qz = rot[3 * n + k];
    const float s0 = scale[k], s1 = scale[n + k], s2 = scale[2 * n + k], sig = opac[k];
    // a NaN or infinite attribute culls the kernel (x * 0 is NaN exactly for those x)
    const bool finite = ((((px * 0.f + py * 0.f) + (pz * 0.f + qw * 0.f)) + ((qx * 0.f + qy * 0.f) + (qz * 0.f + s0 * 0.f))) +
                         ((s1 * 0.f + s2 * 0.f) + sig * 0.f)) == 0.f;
    ids[k] = (uint32_t)k;
    BinOut b;
    b.vis = false;
    if (finite) b = bin_spec(px, py, pz, qw, qx, qy, qz, s0, s1, s2, cam, ro.kappa, ro.radius_sigma);
    else atomicAdd(culled, 1ull);
    auto cull = [&]() {
        depth_key[k] = 0xffffffffu;
        ntiles[k] = 0;
        rect[k] = make_uint2(0, 0);
    };
    if (!b.vis) {
        cull();
        return;
    }
    depth_key[k] = __float_as_uint(b.tz);
    ntiles[k] = (uint32_t)((b.x1 - b.x0) * (b.y1 - b.y0));
    const uint2 rk = make_uint2((uint32_t)b.x0 | ((uint32_t)b.y0 << 16), (uint32_t)b.x1 | ((uint32_t)b.y1 << 16));
    rect[k] = rk;
    // Compositing record in the splat's principal frame (see device_common.h), evaluated in
    // double from the float attributes: the mean is kept as a float pair (hi + lo) because the
    // single-precision pixel coordinate of a mean (ulp 1.2e-4 at x = 1920) would shift a thin
    // splat's Gaussian across its minor axis by a visible fraction of its width.
    double tf[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        tf[i] = (double)cam.R[3 * i] * px + (double)cam.R[3 * i + 1] * py + (double)cam.R[3 * i + 2] * pz +
                (double)cam.t[i];
    double M[2][3], iz;
    persp_M<double>(tf, cam, M, iz);
    double Rq[3][3];
    {
        const float q[4] = {rot[k], rot[n + k], rot[2 * n + k], rot[3 * n + k]};
        quat_rot<double>(q, Rq);
    }
    double A[2][3];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double sa = scale[(size_t)a * n + k];
#pragma unroll
        for (int i = 0; i < 2; ++i) A[i][a] = (M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a]) * sa;
    }
    double l1, l2, fc, fs;
    principal_frame<double>(A, (double)ro.kappa, l1, l2, fc, fs);
    const double mu = (double)cam.fx * tf[0] * iz + (double)cam.cx;
    const double mv = (double)cam.fy * tf[1] * iz + (double)cam.cy;
    const float mu_hi = (float)mu, mv_hi = (float)mv;
    const double dx = (double)px - cam.o[0], dy = (double)py - cam.o[1], dz = (double)pz - cam.o[2];
    const double il = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
    double acc[3] = {0.0, 0.0, 0.0};
    sh_basis_visit<double>(K, dx * il, dy * il, dz * il, [&](int i, double y) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) acc[ch] += y * (double)sh[((size_t)ch * K + i) * n + k];
    });
    const float col[3] = {(float)acc[0], (float)acc[1], (float)acc[2]};
    if (!(((col[0] * 0.f + col[1] * 0.f) + col[2] * 0.f) == 0.f)) {  // a non-finite colour in this view
        cull();
        atomicAdd(culled, 1ull);
        return;
    }
    // one 64-byte record per kernel: a list entry's record is one gather (the pair offset is filled
    // in by pair_off_kernel after the depth sort)
    float4* r = rec + 4 * (size_t)k;
    r[0] = make_float4(mu_hi, mv_hi, (float)(1.0 / l1), (float)(1.0 / l2));
    r[1] = make_float4((float)fc, (float)fs, opac[k], col[0]);
    r[2] = make_float4(col[1], col[2], (float)(mu - (double)mu_hi), (float)(mv - (double)mv_hi));
    r[3] = make_float4(__uint_as_float(rk.x), __uint_as_float(rk.y), 0.f, 0.f);
}

// ---------------------------------------------------------------------------
// Device-wide exclusive scan (u32): per-block totals, a recursive scan of the
// totals, then a block-local scan with the block's offset added.
// ---------------------------------------------------------------------------
constexpr int kScanItems = 8;
constexpr int kScanTile = kThreads * kScanItems;

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t o = __shfl_up(v, d, 64);
        if (lane >= d) v += o;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the block total in *total.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* total) {
    __shared__ uint32_t wsum[kThreads / 64];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const uint32_t inc = wave_incl_scan(v);
    if (lane == 63) wsum[wave] = inc;
    __syncthreads();
    uint32_t off = 0, tot = 0;
#pragma unroll
    for (int w = 0; w < kThreads / 64; ++w) {
        if (w < wave) off += wsum[w];
        tot += wsum[w];
    }
    __syncthreads();
    *total = tot;
    return off + inc - v;
}

__global__ __launch_bounds__(kThreads) void scan_reduce_kernel(const uint32_t* __restrict__ in, uint32_t n,
                                                                uint32_t* __restrict__ block_sums) {
    const size_t base = (size_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t idx = base + (size_t)i * kThreads + threadIdx.x;
        if (idx < n) s += in[idx];
    }
    uint32_t tot;
    block_excl_scan(s, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// The block's tile passes through LDS so that the global loads and stores are coalesced (thread t
// scans items 8t .. 8t + 7 of the tile, read and written as two 16-byte words).
__global__ __launch_bounds__(kThreads) void scan_apply_kernel(const uint32_t* __restrict__ in,
                                                               uint32_t* __restrict__ out, uint32_t n,
                                                               const uint32_t* __restrict__ block_off,
                                                               uint32_t* __restrict__ d_total) {
    static_assert(kScanItems == 8, "two 16-byte LDS words per thread");
    __shared__ uint4 tile4[kScanTile / 4];
    uint32_t* tile = reinterpret_cast<uint32_t*>(tile4);
    const size_t base = (size_t)blockIdx.x * kScanTile;
    const int tid = threadIdx.x;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t idx = base + (size_t)i * kThreads + tid;
        tile[i * kThreads + tid] = idx < n ? in[idx] : 0u;
    }
    __syncthreads();
    const uint4 w0 = tile4[2 * tid], w1 = tile4[2 * tid + 1];
    const uint32_t v[kScanItems] = {w0.x, w0.y, w0.z, w0.w, w1.x, w1.y, w1.z, w1.w};
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) s += v[i];
    uint32_t tot;
    uint32_t off = block_excl_scan(s, &tot) + (block_off ? block_off[blockIdx.x] : 0u);
    uint32_t o[kScanItems];
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        o[i] = off;
        off += v[i];
    }
    tile4[2 * tid] = make_uint4(o[0], o[1], o[2], o[3]);
    tile4[2 * tid + 1] = make_uint4(o[4], o[5], o[6], o[7]);
    if (d_total && blockIdx.x == gridDim.x - 1 && tid == kThreads - 1) *d_total = off;
    __syncthreads();
#pragma unroll
    for (int i = 0; i < kScanItems; ++i) {
        const size_t idx = base + (size_t)i * kThreads + tid;
        if (idx < n) out[idx] = tile[i * kThreads + tid];
    }
}

hipError_t scan_rec(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total, uint32_t* tmp,
                    size_t tmp_words, hipStream_t s) {
    const uint32_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb <= 1) {
        scan_apply_kernel<<<1, kThreads, 0, s>>>(in, out, n, nullptr, d_total);
        return hipGetLastError();
    }
    if ((size_t)2 * nb > tmp_words) return hipErrorInvalidValue;
    uint32_t* sums = tmp;
    uint32_t* offs = tmp + nb;
    scan_reduce_kernel<<<nb, kThreads, 0, s>>>(in, n, sums);
    hipError_t e = scan_rec(sums, offs, nb, nullptr, tmp + 2 * nb, tmp_words - 2 * nb, s);
    if (e != hipSuccess) return e;
    scan_apply_kernel<<<nb, kThreads, 0, s>>>(in, out, n, offs, d_total);
    return hipGetLastError();
}

size_t scan_tmp_words(uint32_t n) {
    size_t words = 0;
    uint32_t m = n;
    while (m > (uint32_t)kScanTile) {
        const uint32_t nb = (m + kScanTile - 1) / kScanTile;
        words += 2 * (size_t)nb;
        m = nb;
    }
    return words + 16;
}

// ---------------------------------------------------------------------------
// Stable LSD radix sort, 8-bit digits, 4096 keys per workgroup per pass:
// histogram per workgroup -> exclusive scan over (digit, workgroup) ->
// stable scatter.  Within a workgroup the keys are ranked in order: each
// wave finds its lanes with equal digit by ballots over the digit bits.
// ---------------------------------------------------------------------------
// Keys per thread of one pass: 16 for the pair passes (tens of millions of keys), 4 for the depth
// sort of the kernels (about a million keys: 4x the workgroups, so the chip is filled).
constexpr int kRsItems = 16, kRsItemsSmall = 4;
constexpr uint32_t kRsSmallN = 1u << 22;
__host__ __device__ inline uint32_t radix_tile(uint32_t n) {
    return (uint32_t)kThreads * (n <= kRsSmallN ? kRsItemsSmall : kRsItems);
}

// Key counts n_cap (the launch's size) or, when d_n is given, min(*d_n, n_cap) read on the device.
__device__ __forceinline__ uint32_t live_count(uint32_t n_cap, const uint32_t* __restrict__ d_n) {
    return d_n ? min(*d_n, n_cap) : n_cap;
}

template <int ITEMS>
__global__ __launch_bounds__(kThreads) void radix_hist_kernel(const uint32_t* __restrict__ keys, uint32_t n_cap,
                                                               const uint32_t* __restrict__ d_n, int shift,
                                                               uint32_t nb, uint32_t* __restrict__ hist) {
    constexpr int TILE = kThreads * ITEMS;
    const uint32_t n = live_count(n_cap, d_n);
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const size_t base = (size_t)blockIdx.x * TILE;
    const int lane = __lane_id();
    // a wave holds 64 consecutive keys; runs of equal digits (the pair keys of one splat's tiles
    // share their high digit) are counted by the run's first lane with one atomic
#pragma unroll 4
    for (int i = 0; i < ITEMS; ++i) {
        const size_t idx = base + (size_t)i * kThreads + threadIdx.x;
        const bool valid = idx < n;
        const uint32_t d = valid ? (keys[idx] >> shift) & 255u : 256u;
        const uint32_t prev = (uint32_t)__shfl_up((int)d, 1, 64);
        const uint64_t heads = __ballot(lane == 0 || d != prev);
        const uint64_t later = lane == 63 ? 0ull : heads >> (lane + 1);
        const uint32_t len = later ? (uint32_t)__ffsll((unsigned long long)later) : (uint32_t)(64 - lane);
        if (valid && ((heads >> lane) & 1ull)) atomicAdd(&cnt[d], len);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of one digit's counts over the workgroups of a pass (one workgroup per digit,
// kScanTile counts per step with a running carry), and the digit's total.  The scatter adds
// the exclusive prefix of the 256 digit totals itself, so a pass is three launches.
__global__ __launch_bounds__(kThreads) void radix_colscan_kernel(const uint32_t* __restrict__ hist, uint32_t nb,
                                                                  uint32_t* __restrict__ offs,
                                                                  uint32_t* __restrict__ dtot) {
    const size_t row = (size_t)blockIdx.x * nb;
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < nb; b0 += kScanTile) {  // uniform across the block
        const uint32_t i0 = b0 + threadIdx.x * kScanItems;
        uint32_t v[kScanItems], sum = 0;
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            v[i] = i0 + i < nb ? hist[row + i0 + i] : 0u;
            sum += v[i];
        }
        uint32_t tot;
        uint32_t off = carry + block_excl_scan(sum, &tot);
#pragma unroll
        for (int i = 0; i < kScanItems; ++i) {
            if (i0 + i < nb) offs[row + i0 + i] = off;
            off += v[i];
        }
        carry += tot;
    }
    if (threadIdx.x == 0) dtot[blockIdx.x] = carry;
}

// Stable scatter of one 8-bit digit pass.  Each wave owns a contiguous quarter of the tile (16
// rows of 64 items, kept in registers) and ranks it without block barriers: equal-digit peers
// by ballots over the digit bits, per-wave digit counts, then a block scan over (digit, wave)
// gives every wave the position of its first item of each digit.  Items are placed in LDS in
// digit order and written out by LDS position, so that consecutive threads write consecutive
// addresses of one digit's run (coalesced).
template <int ITEMS>
__global__ __launch_bounds__(kThreads) void radix_scatter_kernel(
    const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint32_t n_cap,
    const uint32_t* __restrict__ d_n, int shift, uint32_t nb, const uint32_t* __restrict__ offs,
    const uint32_t* __restrict__ dtot, uint32_t* __restrict__ kout, uint32_t* __restrict__ vout) {
    constexpr int NWV = kThreads / 64;
    constexpr int TILE = kThreads * ITEMS;
    const uint32_t n = live_count(n_cap, d_n);
    if ((size_t)blockIdx.x * TILE >= n) return;  // uniform: a workgroup past the live keys has nothing to place
    __shared__ uint32_t base_d[256], lstart[256];
    __shared__ uint32_t wpos[NWV][256];
    __shared__ uint32_t wsum[NWV];
    __shared__ uint2 skv[TILE];  // (key, value)
    const int tid = threadIdx.x, lane = __lane_id(), wave = tid / 64;
    {
        // global start of digit tid: the totals of the smaller digits, then this workgroup's offset
        uint32_t tot;
        base_d[tid] = block_excl_scan(dtot[tid], &tot) + offs[(size_t)tid * nb + blockIdx.x];
    }
#pragma unroll
    for (int w = 0; w < NWV; ++w) wpos[w][tid] = 0;
    __syncthreads();
    const uint64_t lt_mask = (lane == 0) ? 0ull : ((~0ull) >> (64 - lane));
    const size_t base = (size_t)blockIdx.x * TILE;
    const size_t wbase = base + (size_t)wave * 64 * ITEMS;
    uint32_t key[ITEMS], val[ITEMS];
    uint64_t peers[ITEMS];
    // (1) the wave's items, their equal-digit peers, and the wave's count of each digit
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const size_t idx = wbase + (size_t)it * 64 + lane;
        const bool valid = idx < n;
        key[it] = valid ? kin[idx] : 0u;
        val[it] = valid ? vin[idx] : 0u;
        const uint32_t d = (key[it] >> shift) & 255u;
        uint64_t pm = __ballot(valid);
        if (!valid) pm = 0ull;
#pragma unroll
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t m = __ballot(bit);
            pm &= bit ? m : ~m;
        }
        peers[it] = pm;
        if (valid && __popcll(pm & lt_mask) == 0) wpos[wave][d] += (uint32_t)__popcll(pm);
    }
    __syncthreads();
    // (2) block-local start of each digit, and of each (digit, wave) run
    {
        uint32_t c[NWV], tot = 0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) {
            c[w] = wpos[w][tid];
            tot += c[w];
        }
        uint32_t v = tot;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t o = __shfl_up(v, dd, 64);
            if (lane >= dd) v += o;
        }
        if (lane == 63) wsum[wave] = v;
        __syncthreads();
        uint32_t sb = 0;
#pragma unroll
        for (int w = 0; w < NWV; ++w) sb += w < wave ? wsum[w] : 0u;
        uint32_t o = sb + v - tot;
        lstart[tid] = o;
#pragma unroll
        for (int w = 0; w < NWV; ++w) {
            wpos[w][tid] = o;
            o += c[w];
        }
    }
    __syncthreads();
    // (3) place the wave's items in order (row by row, lane by lane within a digit)
#pragma unroll
    for (int it = 0; it < ITEMS; ++it) {
        const uint64_t pm = peers[it];
        if (pm == 0ull) continue;  // invalid lane
        const uint32_t d = (key[it] >> shift) & 255u;
        const uint32_t rank = (uint32_t)__popcll(pm & lt_mask);
        const uint32_t pos = wpos[wave][d] + rank;
        skv[pos] = make_uint2(key[it], val[it]);
        if (rank == 0) wpos[wave][d] = pos + (uint32_t)__popcll(pm);
    }
    __syncthreads();
    const uint32_t cnt = (uint32_t)min((size_t)TILE, (size_t)n - base);
    for (uint32_t j = tid; j < cnt; j += kThreads) {
        const uint2 kv = skv[j];
        const uint32_t d = (kv.x >> shift) & 255u;
        const uint32_t gpos = base_d[d] + (j - lstart[d]);
        kout[gpos] = kv.x;
        vout[gpos] = kv.y;
    }
}

// The pair count of a render against the frame's capacity: d_pairs[0] holds the scanned total;
// d_pairs[1] receives the live count, the total when it fits and 0 (render nothing) when it does
// not, in which case the overflow and the count needed are recorded.  One thread.
__global__ void pair_capacity_kernel(uint32_t* __restrict__ d_pairs, uint32_t cap,
                                     unsigned long long* __restrict__ stats, unsigned long long* __restrict__ prof) {
    const uint32_t total = d_pairs[0];
    const bool fits = total <= cap;
    d_pairs[1] = fits ? total : 0u;
    if (!fits) {
        atomicAdd(&stats[GSN_STAT_PAIR_OVERFLOW], 1ull);
        atomicMax(&stats[GSN_STAT_PAIRS_NEEDED], (unsigned long long)total);
    }
    if (prof && fits) atomicAdd(&prof[GSN_COUNT_PAIRS], (unsigned long long)total);
}

// p[0 .. ceil(*d_count / per_word)) = v, at most cap words (a fill sized on the device).
__global__ void fill_u32_dev_kernel(uint32_t* __restrict__ p, uint32_t v, const uint32_t* __restrict__ d_count,
                                    uint32_t per_word, size_t cap) {
    const size_t n = min(cap, ((size_t)*d_count + per_word - 1) / per_word);
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) p[i] = v;
}

// dst[0 .. min(*d_count, cap)) = src[...] (u32).
__global__ void copy_u32_dev_kernel(uint32_t* __restrict__ dst, const uint32_t* __restrict__ src,
                                    const uint32_t* __restrict__ d_count, size_t cap) {
    const size_t n = d_count ? min(cap, (size_t)*d_count) : cap;
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (; i < n; i += stride) dst[i] = src[i];
}

__global__ void records_out_kernel(const float4* __restrict__ rec, int n, float4* __restrict__ out) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
#pragma unroll
    for (int j = 0; j < 3; ++j) out[(size_t)j * n + k] = rec[4 * (size_t)k + j];
}

__global__ void gather_u32_kernel(const uint32_t* __restrict__ src, const uint32_t* __restrict__ idx,
                                  uint32_t* __restrict__ dst, uint32_t n) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[idx[i]];
}

// One thread per depth rank: writes the kernel's (tile, id) pairs, row-major
// over its rectangle, at its scanned offset.
// Each kernel's slot range: pair_off[id] = offsets[depth rank], kernel r (depth rank) owning the
// slots [offsets[r], offsets[r] + ntiles) of its (tile, kernel) pairs in row-major tile order.  The
// offset is also stored in the kernel's record (word 14), next to its tile rectangle.
__global__ void pair_off_kernel(const uint32_t* __restrict__ sorted_ids, const uint32_t* __restrict__ offsets,
                                uint32_t n, uint32_t* __restrict__ pair_off, uint32_t* __restrict__ rec_words) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const uint32_t id = sorted_ids[r], o0 = offsets[r];
    pair_off[id] = o0;
    rec_words[16 * (size_t)id + 14] = o0;
}

// ---------------------------------------------------------------------------
// Per-tile lists by two-level binning.  The tiles are grouped into super-tiles of kSuper x kSuper
// tiles.  (1) Each kernel, in depth order, emits one membership (super-tile, kernel) per super-tile
// its tile rectangle meets, and a stable radix partition by super-tile leaves each super-tile's
// members in depth order (a few memberships per kernel, against tens of (tile, kernel) pairs).
// (2) A super-tile's members are cut into segments of kSegment, one wave each.  The wave counts
// its entries per tile (lane j holds tile j's count), and one exclusive scan over the counts laid
// out super-tile by super-tile, tile by tile within it and segment by segment within a tile, gives
// every segment's place in every tile's list.  The wave then writes its entries in member order: for
// each tile a ballot over the wave ranks the members that cover it, so each list comes out in depth
// order, identical to a stable partition of all pairs by tile, and its run is written coalesced.
// The lists are stored super-tile after super-tile; ranges index them.
// ---------------------------------------------------------------------------
constexpr int kSuper = 8, kSuperTiles = kSuper * kSuper;
constexpr int kSegment = 512;

__device__ __forceinline__ void rect_bounds(uint2 rc, uint32_t& x0, uint32_t& y0, uint32_t& x1, uint32_t& y1) {
    x0 = rc.x & 0xffffu;
    y0 = rc.x >> 16;
    x1 = rc.y & 0xffffu;
    y1 = rc.y >> 16;
}

// nsup[r]: the number of super-tiles the tile rectangle of depth rank r meets (0 for an empty one).
__global__ void super_count_kernel(const uint32_t* __restrict__ sorted_ids, const uint2* __restrict__ rect,
                                   uint32_t n, uint32_t* __restrict__ nsup) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    uint32_t x0, y0, x1, y1;
    rect_bounds(rect[sorted_ids[r]], x0, y0, x1, y1);
    nsup[r] = (x1 > x0 && y1 > y0) ? ((x1 - 1) / kSuper - x0 / kSuper + 1) * ((y1 - 1) / kSuper - y0 / kSuper + 1) : 0u;
}

// The live membership count: the scanned total, or 0 when the render's pairs did not fit (d_total[1]
// is then 0 while d_total[0] is not).  Memberships never outnumber pairs (each meets at least one
// tile), so a live count fits the pair buffers.  One thread.
__global__ void member_live_kernel(uint32_t* __restrict__ d_total) {
    d_total[3] = (d_total[1] == 0u && d_total[0] != 0u) ? 0u : d_total[2];
}

// A membership's key: the super-tile id (row-major) in the low 16 bits, which the partition sorts
// on, and above them the kernel's rectangle clipped to the super-tile in its local tile coordinates
// (lx0, ly0, lx1 - 1, ly1 - 1, 3 bits each), so that the segment passes need no gather by kernel id.
__device__ __forceinline__ uint32_t member_key(uint32_t st, uint32_t lx0, uint32_t ly0, uint32_t lx1, uint32_t ly1) {
    return st | (lx0 << 16) | (ly0 << 19) | ((lx1 - 1) << 22) | ((ly1 - 1) << 25);
}
__device__ __forceinline__ void member_rect(uint32_t key, uint32_t& lx0, uint32_t& ly0, uint32_t& lx1, uint32_t& ly1) {
    lx0 = (key >> 16) & 7u;
    ly0 = (key >> 19) & 7u;
    lx1 = ((key >> 22) & 7u) + 1;
    ly1 = ((key >> 25) & 7u) + 1;
}

// Memberships of depth rank r at moffs[r]: keys as member_key, values = kernel id.
__global__ void super_emit_kernel(const uint32_t* __restrict__ sorted_ids, const uint2* __restrict__ rect,
                                  const uint32_t* __restrict__ moffs, uint32_t n, const uint32_t* __restrict__ d_total,
                                  uint32_t sup_x, uint32_t* __restrict__ keys, uint32_t* __restrict__ vals) {
    const uint32_t r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || d_total[3] == 0u) return;
    const uint32_t id = sorted_ids[r];
    uint32_t x0, y0, x1, y1;
    rect_bounds(rect[id], x0, y0, x1, y1);
    if (x1 <= x0 || y1 <= y0) return;
    uint32_t m = moffs[r];
    for (uint32_t sy = y0 / kSuper; sy <= (y1 - 1) / kSuper; ++sy)
        for (uint32_t sx = x0 / kSuper; sx <= (x1 - 1) / kSuper; ++sx) {
            const uint32_t ox = sx * kSuper, oy = sy * kSuper;
            keys[m] = member_key(sy * sup_x + sx, max(x0, ox) - ox, max(y0, oy) - oy, min(x1, ox + kSuper) - ox,
                                 min(y1, oy + kSuper) - oy);
            vals[m] = id;
            ++m;
        }
}

// seg_base[st]: the first segment of super-tile st (exclusive scan of ceil(members / kSegment)),
// seg_base[n_super] the number of segments.  One workgroup of kThreads.
__global__ __launch_bounds__(kThreads) void segment_scan_kernel(const uint2* __restrict__ sranges, uint32_t n_super,
                                                                 uint32_t* __restrict__ seg_base) {
    uint32_t carry = 0;
    for (uint32_t b0 = 0; b0 < n_super; b0 += kThreads) {  // uniform across the workgroup
        const uint32_t st = b0 + threadIdx.x;
        uint32_t c = 0;
        if (st < n_super) {
            const uint2 sr = sranges[st];
            c = (sr.y - sr.x + kSegment - 1) / kSegment;
        }
        uint32_t tot;
        const uint32_t off = block_excl_scan(c, &tot);
        if (st < n_super) seg_base[st] = carry + off;
        carry += tot;
    }
    if (threadIdx.x == 0) seg_base[n_super] = carry;
}

// Segment b's super-tile (the last st with seg_base[st] <= b), its member range and the segments
// [b0, b1) of that super-tile.  False past the last segment.
__device__ __forceinline__ bool segment_of(uint32_t b, const uint32_t* __restrict__ seg_base, uint32_t n_super,
                                           const uint2* __restrict__ sranges, uint32_t& st, uint32_t& m0,
                                           uint32_t& m1, uint32_t& b0, uint32_t& b1) {
    if (b >= seg_base[n_super]) return false;
    uint32_t lo = 0, hi = n_super - 1;
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (seg_base[mid] <= b) lo = mid; else hi = mid - 1;
    }
    st = lo;
    b0 = seg_base[st];
    b1 = seg_base[st + 1];
    const uint2 sr = sranges[st];
    m0 = sr.x + (b - b0) * (uint32_t)kSegment;
    m1 = min(sr.y, m0 + (uint32_t)kSegment);
    return true;
}

// Place of (segment b, local tile j) in the count and offset arrays: the super-tile's block starts at
// kSuperTiles * b0 and holds its tiles one after another, each with its segments in order.
__device__ __forceinline__ size_t count_index(uint32_t b, uint32_t j, uint32_t b0, uint32_t b1) {
    return (size_t)kSuperTiles * b0 + (size_t)j * (b1 - b0) + (b - b0);
}

// One wave per segment: counts of its entries per local tile (COUNT), or its entries written into the
// tile lists at the scanned offsets, in member order (!COUNT).  Waves of a workgroup are independent.
template <bool COUNT>
__global__ __launch_bounds__(kThreads) void segment_tiles_kernel(const uint32_t* __restrict__ mkeys,
                                                                  const uint32_t* __restrict__ mvals,
                                                                  const uint2* __restrict__ sranges,
                                                                  const uint32_t* __restrict__ seg_base,
                                                                  uint32_t n_super, uint32_t* __restrict__ counts,
                                                                  const uint32_t* __restrict__ offs,
                                                                  uint32_t* __restrict__ ids) {
    const int lane = __lane_id();
    const uint32_t b = blockIdx.x * (kThreads / 64) + threadIdx.x / 64;
    uint32_t st, m0, m1, b0, b1;
    if (!segment_of(b, seg_base, n_super, sranges, st, m0, m1, b0, b1)) return;  // uniform across the wave
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const size_t ci = count_index(b, (uint32_t)lane, b0, b1);
    uint32_t run = COUNT ? 0u : offs[ci];  // lane j: tile j's count, or its next place in the list
    for (uint32_t base = m0; base < m1; base += 64) {  // uniform across the wave
        const uint32_t m = base + (uint32_t)lane;
        uint32_t id = 0, lx0 = 0, ly0 = 0, lx1 = 0, ly1 = 0;
        if (m < m1) {
            if (!COUNT) id = mvals[m];
            member_rect(mkeys[m], lx0, ly0, lx1, ly1);
        }
        for (uint32_t ly = 0; ly < (uint32_t)kSuper; ++ly) {
            const bool row = ly >= ly0 && ly < ly1;
            if (__ballot(row) == 0ull) continue;  // no member of this batch covers the row
#pragma unroll
            for (uint32_t lx = 0; lx < (uint32_t)kSuper; ++lx) {
                const uint32_t j = ly * kSuper + lx;
                const bool c = row && lx >= lx0 && lx < lx1;
                const uint64_t bal = __ballot(c);
                if (!COUNT) {
                    // tile j's next place, read from lane j (j is uniform across the wave)
                    const uint32_t at = (uint32_t)__builtin_amdgcn_readlane((int)run, (int)j);
                    if (c) ids[at + (uint32_t)__popcll(bal & lt_mask)] = id;
                }
                if ((uint32_t)lane == j) run += (uint32_t)__popcll(bal);
            }
        }
    }
    if (COUNT) counts[ci] = run;
}

// Per tile: its range in the lists (the offset of its super-tile's first segment, and the last
// segment's offset plus count); (0, 0) for a tile whose super-tile has no members.
__global__ void tile_list_ranges_kernel(const uint32_t* __restrict__ seg_base, uint32_t tiles_x, uint32_t tiles,
                                        uint32_t sup_x, const uint32_t* __restrict__ counts,
                                        const uint32_t* __restrict__ offs, uint2* __restrict__ ranges) {
    const uint32_t t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const uint32_t tx = t % tiles_x, ty = t / tiles_x;
    const uint32_t st = (ty / kSuper) * sup_x + tx / kSuper, j = (ty % kSuper) * kSuper + tx % kSuper;
    const uint32_t b0 = seg_base[st], b1 = seg_base[st + 1];
    if (b1 == b0) {
        ranges[t] = make_uint2(0u, 0u);
        return;
    }
    const size_t first = count_index(b0, j, b0, b1), last = count_index(b1 - 1, j, b0, b1);
    ranges[t] = make_uint2(offs[first], offs[last] + counts[last]);
}

// [start, end) of each key's run in keys sorted on their bits `mask` (live count *d_count; grid-stride,
// so the grid need not cover the capacity).
__global__ void key_ranges_kernel(const uint32_t* __restrict__ keys, const uint32_t* __restrict__ d_count,
                                  uint32_t mask, uint2* __restrict__ ranges) {
    const uint32_t count = *d_count;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < count; i += gridDim.x * blockDim.x) {
        const uint32_t k = keys[i] & mask;
        if (i == 0 || (keys[i - 1] & mask) != k) ranges[k].x = i;
        if (i == count - 1 || (keys[i + 1] & mask) != k) ranges[k].y = i + 1;
    }
}

// One workgroup: tiles bucketed by list length (four buckets per octave) and written out longest
// bucket first, so that the raster passes start their longest tiles first and the short ones fill
// the end of the launch.  The order within a bucket is whatever the LDS atomics give: every tile is
// computed independently, so results do not depend on it.
constexpr int kOrderBuckets = 1 + 32 * 4;
__device__ __forceinline__ int length_bucket(uint32_t len) {
    if (len == 0) return 0;
    const int lz = 31 - __clz((int)len);
    const uint32_t frac = lz >= 2 ? (len >> (lz - 2)) & 3u : (len << (2 - lz)) & 3u;
    return 1 + 4 * lz + (int)frac;
}

__global__ __launch_bounds__(1024) void tile_order_kernel(const uint2* __restrict__ ranges,
                                                          const uint32_t* __restrict__ lens, int tiles,
                                                          uint32_t* __restrict__ order) {
    auto length = [&](int i) -> uint32_t {
        if (lens) return lens[i];
        const uint2 r = ranges[i];
        return r.y - r.x;
    };
    __shared__ uint32_t cnt[kOrderBuckets];
    for (int b = threadIdx.x; b < kOrderBuckets; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    for (int i = threadIdx.x; i < tiles; i += blockDim.x) atomicAdd(&cnt[length_bucket(length(i))], 1u);
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t acc = 0;
        for (int b = kOrderBuckets - 1; b >= 0; --b) {
            const uint32_t c = cnt[b];
            cnt[b] = acc;
            acc += c;
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < tiles; i += blockDim.x) order[atomicAdd(&cnt[length_bucket(length(i))], 1u)] = (uint32_t)i;
}

// ---------------------------------------------------------------------------
// Forward compositing, one workgroup per tile, one thread per pixel.  Records are
// staged in LDS in batches of 256 list entries; each wave (a band of 16 x 4 pixels)
// gets the ordered list of the batch's entries whose alpha-support box meets its
// band, so a wave only steps through entries that can composite in it.
// ---------------------------------------------------------------------------
// Six waves per SIMD (at most 80 VGPRs, no spills; six workgroups' LDS fit in a CU).  CT: the type
// of the colour sums (double; float in the mixed form, which then writes no double image).
template <class CT, bool STEPS>
__global__ __launch_bounds__(GSN_BLOCK, 6) void raster_fwd_kernel(
    const uint2* __restrict__ ranges, const uint32_t* __restrict__ order, const uint32_t* __restrict__ ids, const float4* __restrict__ rec, uint32_t n,
    DevCam cam, DevRenderOpts ro, float* __restrict__ img, double* __restrict__ img64, float* __restrict__ Tfin,
    uint32_t* __restrict__ ncontrib, uint64_t* __restrict__ masks, uint32_t* __restrict__ tile_len,
    unsigned long long* __restrict__ counts) {
    constexpr int NW = GSN_BLOCK / 64;
    static_assert(NW == 4, "the composited-entry words below assume four waves");
    __shared__ float4 s_a[GSN_BLOCK];
    __shared__ float4 s_b[GSN_BLOCK];
    __shared__ float4 s_c[GSN_BLOCK];
    __shared__ uint8_t s_list[NW][GSN_BLOCK];
    __shared__ uint32_t s_cnt[NW][NW];  // [band][loader wave]
    const int tile = (int)order[blockIdx.x];
    const int tx = tile % cam.tiles_x, ty = tile / cam.tiles_x;
    const int px = tx * GSN_TILE + (threadIdx.x % GSN_TILE);
    const int py = ty * GSN_TILE + (threadIdx.x / GSN_TILE);
    const bool inside = px < cam.W && py < cam.H;
    const uint2 rg = ranges[tile];
    const int lane = __lane_id(), wave = threadIdx.x / 64;
    const uint64_t lt_mask = lane == 0 ? 0ull : (~0ull >> (64 - lane));
    const float tx0 = (float)(tx * GSN_TILE), tx1 = tx0 + (float)(GSN_TILE - 1);
    const float ty0 = (float)(ty * GSN_TILE);
    // colour accumulated in CT: the backward pass subtracts partial sums from it
    float T = 1.0f;
    CT C0 = CT(0), C1 = CT(0), C2 = CT(0);
    uint32_t last = 0;
    bool done = !inside;
    const float fpx = (float)px, fpy = (float)py;
    uint32_t evals = 0, staged = 0;
    uint32_t wsteps = 0;  // the wave's steps: the longest walk over its lanes, batch after batch
    // each thread's entry of the next batch is loaded while the current batch is composited
    float4 na = make_float4(0.f, 0.f, 0.f, 0.f), nb = na, nc = na;
    bool nvalid = rg.x + threadIdx.x < rg.y;
    if (nvalid) {
        const float4* r = rec + 4 * (size_t)ids[rg.x + threadIdx.x];
        na = r[0];
        nb = r[1];
        nc = r[2];
    }
    for (uint32_t base = rg.x; base < rg.y; base += GSN_BLOCK) {
        if (__syncthreads_count(done) == GSN_BLOCK) break;
        const float4 a = na, b = nb, c4 = nc;
        const bool valid = nvalid;
        {
            const uint32_t e2 = base + GSN_BLOCK + threadIdx.x;
            nvalid = e2 < rg.y;
            if (nvalid) {
                const float4* r = rec + 4 * (size_t)ids[e2];
                na = r[0];
                nb = r[1];
                nc = r[2];
            }
        }
        uint32_t bandmask = 0;
        if (valid) {
            ++staged;
            s_a[threadIdx.x] = a;
            s_b[threadIdx.x] = b;
            s_c[threadIdx.x] = c4;
            const float4 box = splat_alpha_box(a, b, c4, ro.alpha_min);
#pragma unroll
            for (int w = 0; w < NW; ++w)
                if (!box_misses(box, tx0, tx1, ty0 + 4.f * w, ty0 + 4.f * w + 3.f) &&
                    !ellipse_misses(a, b, c4, ro.alpha_min, tx0, tx1, ty0 + 4.f * w, ty0 + 4.f * w + 3.f))
                    bandmask |= 1u << w;
        }
        uint64_t bal[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            bal[w] = __ballot((bandmask >> w) & 1u);
            if (lane == 0) s_cnt[w][wave] = (uint32_t)__popcll(bal[w]);
        }
        __syncthreads();
#pragma unroll
        for (int w = 0; w < NW; ++w) {
            if ((bandmask >> w) & 1u) {
                uint32_t off = 0;
#pragma unroll
                for (int v = 0; v < NW; ++v) off += v < wave ? s_cnt[w][v] : 0u;
                s_list[w][off + (uint32_t)__popcll(bal[w] & lt_mask)] = (uint8_t)threadIdx.x;
            }
        }
        __syncthreads();
        uint32_t nl = 0;
#pragma unroll
        for (int v = 0; v < NW; ++v) nl += s_cnt[wave][v];
        uint64_t bits[NW];
#pragma unroll
        for (int w = 0; w < NW; ++w) bits[w] = 0ull;
        uint32_t i = 0;
        for (; i < nl && !done; ++i) {
            // the wave's lanes walk its band list together: the entry is the same in every lane
            const int j = __builtin_amdgcn_readfirstlane((int)s_list[wave][i]);
            const float4 a = s_a[j], b = s_b[j], cc = s_c[j];
            const SplatEval ev = eval_splat(a, b, cc, fpx, fpy, ro.alpha_max);
            ++evals;
            bool comp = ev.alpha >= ro.alpha_min;
            const float Tn = T * (1.0f - ev.alpha);
            if (comp && Tn < ro.T_min) {  // stop before the entry that would cross T_min
                done = true;
                comp = false;
            }
            if (comp) {
                const CT w = (CT)(ev.alpha * T);
                C0 += w * (CT)b.w;
                C1 += w * (CT)cc.x;
                C2 += w * (CT)cc.y;
                T = Tn;
                last = base + j + 1 - rg.x;
                // word and bit are uniform across the wave: the selects are scalar, the ors plain
                const uint64_t bit = 1ull << (j & 63);
                const int q = j >> 6;
#pragma unroll
                for (int w = 0; w < NW; ++w) bits[w] |= q == w ? bit : 0ull;
            }
        }
        if (STEPS) {  // the wave walks as far as its longest lane
            uint32_t m = i;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
            wsteps += m;
        }
        const uint32_t batch = (base - rg.x) / GSN_BLOCK;
        if (masks && batch < (uint32_t)GSN_MASK_BATCHES) {
            // pixel-major words [w][pixel] (the backward pass rebuilds the per-(entry, wave) words from them)
            uint64_t* mb = masks + ((size_t)tile * GSN_MASK_BATCHES + batch) * NW * GSN_BLOCK + threadIdx.x;
#pragma unroll
            for (int w = 0; w < NW; ++w) mb[(size_t)w * GSN_BLOCK] = bits[w];
        }
    }
    {
        // the tile's composited prefix (the longest over its pixels): the backward pass's work
        uint32_t m = last;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off, 64));
        __shared__ uint32_t s_len;
        if (threadIdx.x == 0) s_len = 0;
        __syncthreads();
        if (lane == 0) atomicMax(&s_len, m);
        __syncthreads();
        if (threadIdx.x == 0) tile_len[tile] = s_len;
    }
    if (counts) {
        __shared__ unsigned long long s_evals, s_staged, s_steps;
        if (threadIdx.x == 0) s_evals = s_staged = s_steps = 0;
        __syncthreads();
        atomicAdd(&s_evals, (unsigned long long)evals);
        atomicAdd(&s_staged, (unsigned long long)staged);
        if (STEPS && lane == 0) atomicAdd(&s_steps, (unsigned long long)wsteps);
        __syncthreads();
        if (threadIdx.x == 0) {
            atomicAdd(&counts[GSN_COUNT_FWD_EVALS], s_evals);
            atomicAdd(&counts[GSN_COUNT_FWD_STAGED], s_staged);
            atomicAdd(&counts[GSN_COUNT_FWD_WAVE_STEPS], s_steps);
        }
    }
    if (inside) {
        const size_t np = (size_t)cam.W * cam.H, pi = (size_t)py * cam.W + px;
        const CT c0 = C0 + (CT)(T * ro.bg[0]), c1 = C1 + (CT)(T * ro.bg[1]), c2 = C2 + (CT)(T * ro.bg[2]);
        img[pi] = (float)c0;
        img[np + pi] = (float)c1;
        img[2 * np + pi] = (float)c2;
        if (img64) {
            img64[pi] = (double)c0;
            img64[np + pi] = (double)c1;
            img64[2 * np + pi] = (double)c2;
        }
        Tfin[pi] = T;
        ncontrib[pi] = last;
    }
}

__global__ void downsample2x_kernel(const float* __restrict__ src, int W, int H, float* __restrict__ dst) {
    const int w2 = W / 2, h2 = H / 2;
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)3 * w2 * h2) return;
    const int x = (int)(i % w2), y = (int)((i / w2) % h2), ch = (int)(i / ((size_t)w2 * h2));
    const float* s = src + (size_t)ch * W * H;
    const float a = s[(size_t)(2 * y) * W + 2 * x], b = s[(size_t)(2 * y) * W + 2 * x + 1];
    const float c = s[(size_t)(2 * y + 1) * W + 2 * x], d = s[(size_t)(2 * y + 1) * W + 2 * x + 1];
    dst[i] = 0.25f * (((a + b) + c) + d);
}

// Mean of the kernel positions in double, one workgroup: thread t sums kernels t, t + 1024, ...
// in order, then a fixed-shape tree in LDS (the result does not depend on timing).
__global__ __launch_bounds__(1024) void scene_center_kernel(const float* __restrict__ pos, int n,
                                                             double* __restrict__ out) {
    __shared__ double s[3][1024];
    double a[3] = {0.0, 0.0, 0.0};
    for (int k = threadIdx.x; k < n; k += 1024)
#pragma unroll
        for (int c = 0; c < 3; ++c) a[c] += (double)pos[(size_t)c * n + k];
#pragma unroll
    for (int c = 0; c < 3; ++c) s[c][threadIdx.x] = a[c];
    __syncthreads();
    for (int w = 512; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w)
#pragma unroll
            for (int c = 0; c < 3; ++c) s[c][threadIdx.x] += s[c][threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x < 3) out[threadIdx.x] = n > 0 ? s[threadIdx.x][0] / (double)n : 0.0;
}

}  // namespace

// ------------------------------------------------------------------ launchers
void launch_scene_center(const float* pos, int n, double* out, hipStream_t s) {
    scene_center_kernel<<<1, 1024, 0, s>>>(pos, n, out);
}

void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s) {
    if (n) fill_u32_kernel<<<grid_for(n), kThreads, 0, s>>>(p, v, n);
}
void launch_fill_f32(float* p, float v, size_t n, hipStream_t s) {
    if (n) fill_f32_kernel<<<grid_for(n), kThreads, 0, s>>>(p, v, n);
}

void launch_preprocess(const gsn_gaussians& g, const DevCam& cam, const DevRenderOpts& ro, float4* rec,
                       uint2* rect, uint32_t* depth_key, uint32_t* ids, uint32_t* ntiles, unsigned long long* culled,
                       hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    preprocess_kernel<<<(g.n + kThreads - 1) / kThreads, kThreads, 0, s>>>(
        g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.d_sh, g.n, K, cam, ro, rec, rect, depth_key, ids, ntiles, culled);
}

size_t scan_tmp_bytes(uint32_t n) {
    const size_t hist_words = (size_t)256 * ((n + radix_tile(n) - 1) / radix_tile(n));
    return 4 * std::max(scan_tmp_words(n), scan_tmp_words((uint32_t)hist_words));
}

hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total, DevBuf& scan_tmp,
                              hipStream_t s) {
    const size_t words = scan_tmp_words(n);
    hipError_t e = buf_reserve(scan_tmp, words * 4);
    if (e != hipSuccess) return e;
    return scan_rec(in, out, n, d_total, bp<uint32_t>(scan_tmp), words, s);
}

hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n, const uint32_t* d_n,
                            int bit_lo, int bit_hi, DevBuf& hist, hipStream_t s, uint32_t** k_res, uint32_t** v_res) {
    if (n == 0) return hipSuccess;
    const uint32_t tile = radix_tile(n), nb = (n + tile - 1) / tile;
    const bool small = n <= kRsSmallN;
    if (hist.bytes < radix_hist_bytes(n)) return hipErrorInvalidValue;  // reserved by the caller
    uint32_t* h = bp<uint32_t>(hist);
    uint32_t* o = h + (size_t)256 * nb;
    uint32_t* dt = o + (size_t)256 * nb;
    int passes = 0;
    uint32_t *ka = k0, *va = v0, *kb = k1, *vb = v1;
    for (int shift = bit_lo; shift < bit_hi; shift += 8, ++passes) {
        if (small) radix_hist_kernel<kRsItemsSmall><<<nb, kThreads, 0, s>>>(ka, n, d_n, shift, nb, h);
        else radix_hist_kernel<kRsItems><<<nb, kThreads, 0, s>>>(ka, n, d_n, shift, nb, h);
        radix_colscan_kernel<<<256, kThreads, 0, s>>>(h, nb, o, dt);
        if (small)
            radix_scatter_kernel<kRsItemsSmall><<<nb, kThreads, 0, s>>>(ka, va, n, d_n, shift, nb, o, dt, kb, vb);
        else
            radix_scatter_kernel<kRsItems><<<nb, kThreads, 0, s>>>(ka, va, n, d_n, shift, nb, o, dt, kb, vb);
        uint32_t* t = ka; ka = kb; kb = t;
        t = va; va = vb; vb = t;
    }
    if (k_res && v_res) {  // the caller takes the result where the passes left it
        *k_res = ka;
        *v_res = va;
        return hipGetLastError();
    }
    if (passes & 1) {
        // the result is in the second buffers: copy the live keys back with kernels (no copy nodes when a
        // caller captures the stream)
        if (d_n) {
            copy_u32_dev_kernel<<<grid_for(n), kThreads, 0, s>>>(k0, ka, d_n, n);
            copy_u32_dev_kernel<<<grid_for(n), kThreads, 0, s>>>(v0, va, d_n, n);
        } else {
            launch_copy_u32(k0, ka, n, s);
            launch_copy_u32(v0, va, n, s);
        }
    }
    return hipGetLastError();
}

void launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, uint32_t n, hipStream_t s) {
    if (n) gather_u32_kernel<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(src, idx, dst, n);
}

size_t radix_hist_bytes(uint32_t n) {
    const size_t nb = ((size_t)n + radix_tile(n) - 1) / radix_tile(n);
    return ((size_t)256 * nb * 2 + 256) * 4;
}

void launch_pair_off(const uint32_t* sorted_ids, const uint32_t* offsets, uint32_t n, uint32_t* pair_off, float4* rec,
                     hipStream_t s) {
    if (n)
        pair_off_kernel<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(sorted_ids, offsets, n, pair_off,
                                                                           reinterpret_cast<uint32_t*>(rec));
}

uint32_t super_tiles_x(int tiles_x) { return (uint32_t)((tiles_x + kSuper - 1) / kSuper); }
uint32_t super_tiles(int tiles_x, int tiles_y) { return super_tiles_x(tiles_x) * (uint32_t)((tiles_y + kSuper - 1) / kSuper); }
// segments are at most ceil(members / kSegment) per super-tile, members at most pairs
size_t max_segments(size_t cap_pairs, int tiles_x, int tiles_y) {
    return (cap_pairs + kSegment - 1) / kSegment + super_tiles(tiles_x, tiles_y);
}
size_t segment_words(size_t cap_pairs, int tiles_x, int tiles_y) {
    return max_segments(cap_pairs, tiles_x, tiles_y) * kSuperTiles;
}

hipError_t build_tile_lists(const uint32_t* sorted_ids, const uint2* rect, uint32_t n, uint32_t* d_total, uint32_t cap,
                            int tiles_x, int tiles_y, const TileListBufs& bb, DevBuf& hist, DevBuf& scan_tmp,
                            uint32_t** ids_out, hipStream_t s) {
    const uint32_t tiles = (uint32_t)tiles_x * (uint32_t)tiles_y;
    const uint32_t sup_x = super_tiles_x(tiles_x), n_super = super_tiles(tiles_x, tiles_y);
    const uint32_t ng = (n + kThreads - 1) / kThreads;
    if (n == 0 || cap == 0) {
        launch_fill_u32(reinterpret_cast<uint32_t*>(bb.ranges), 0u, 2 * (size_t)tiles, s);
        *ids_out = bb.mv;
        return hipGetLastError();
    }
    // (1) memberships in depth order, partitioned by super-tile
    launch_fill_u32(reinterpret_cast<uint32_t*>(bb.sranges), 0u, 2 * (size_t)n_super, s);
    super_count_kernel<<<ng, kThreads, 0, s>>>(sorted_ids, rect, n, bb.nsup);
    hipError_t e = exclusive_scan_u32(bb.nsup, bb.moffs, n, d_total + 2, scan_tmp, s);
    if (e != hipSuccess) return e;
    member_live_kernel<<<1, 1, 0, s>>>(d_total);
    super_emit_kernel<<<ng, kThreads, 0, s>>>(sorted_ids, rect, bb.moffs, n, d_total, sup_x, bb.mk, bb.mv);
    int bits = 1;
    // at most 16: the image limits (at most 2^28 pixels, 65535 tiles a side) keep n_super below 2^15
    while ((1u << bits) < n_super) ++bits;
    uint32_t *mk = bb.mk, *mv = bb.mv;
    e = radix_sort_pairs(bb.mk, bb.mv, bb.mk2, bb.mv2, cap, d_total + 3, 0, bits, hist, s, &mk, &mv);
    if (e != hipSuccess) return e;
    key_ranges_kernel<<<grid_for(cap, kThreads, 4096), kThreads, 0, s>>>(mk, d_total + 3, 0xffffu, bb.sranges);
    // the tile lists go to whichever values buffer the sorted members do not occupy
    *ids_out = mv == bb.mv ? bb.mv2 : bb.mv;
    // (2) segments: counts per tile, one scan, then the lists
    segment_scan_kernel<<<1, kThreads, 0, s>>>(bb.sranges, n_super, bb.seg_base);
    const size_t words = segment_words(cap, tiles_x, tiles_y);
    const uint32_t nwg = (uint32_t)((max_segments(cap, tiles_x, tiles_y) + kThreads / 64 - 1) / (kThreads / 64));
    segment_tiles_kernel<true><<<nwg, kThreads, 0, s>>>(mk, mv, bb.sranges, bb.seg_base, n_super, bb.counts, nullptr,
                                                         nullptr);
    // the scan runs over the capacity: entries past the live segments are never read
    e = exclusive_scan_u32(bb.counts, bb.offs, (uint32_t)words, d_total + 4, scan_tmp, s);
    if (e != hipSuccess) return e;
    tile_list_ranges_kernel<<<(tiles + kThreads - 1) / kThreads, kThreads, 0, s>>>(bb.seg_base, (uint32_t)tiles_x,
                                                                                   tiles, sup_x, bb.counts, bb.offs,
                                                                                   bb.ranges);
    segment_tiles_kernel<false><<<nwg, kThreads, 0, s>>>(mk, mv, bb.sranges, bb.seg_base, n_super, nullptr, bb.offs,
                                                          *ids_out);
    return hipGetLastError();
}


void launch_pair_capacity(uint32_t* d_pairs, uint32_t cap, unsigned long long* stats, unsigned long long* prof,
                          hipStream_t s) {
    pair_capacity_kernel<<<1, 1, 0, s>>>(d_pairs, cap, stats, prof);
}

void launch_fill_u32_dev(uint32_t* p, uint32_t v, const uint32_t* d_count, uint32_t per_word, size_t cap,
                         hipStream_t s) {
    if (cap) fill_u32_dev_kernel<<<grid_for(cap), kThreads, 0, s>>>(p, v, d_count, per_word, cap);
}

void launch_records_out(const float4* rec, int n, float4* out, hipStream_t s) {
    if (n > 0) records_out_kernel<<<(n + kThreads - 1) / kThreads, kThreads, 0, s>>>(rec, n, out);
}

void launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t s) {
    if (n) copy_u32_dev_kernel<<<grid_for(n), kThreads, 0, s>>>(dst, src, nullptr, n);
}

void launch_tile_order(const uint2* ranges, const uint32_t* lens, int tiles, uint32_t* order, hipStream_t s) {
    if (tiles > 0) tile_order_kernel<<<1, 1024, 0, s>>>(ranges, lens, tiles, order);
}

void launch_raster_fwd(const uint2* ranges, const uint32_t* order, const uint32_t* ids, const float4* rec, uint32_t n, const DevCam& cam,
                       const DevRenderOpts& ro, bool fp32, float* img, double* img64, float* Tfin, uint32_t* ncontrib,
                       uint64_t* masks, uint32_t* tile_len, unsigned long long* counts, bool steps, hipStream_t s) {
    const int tiles = cam.tiles_x * cam.tiles_y;
    steps = steps && counts;
    auto kern = fp32 ? (steps ? raster_fwd_kernel<float, true> : raster_fwd_kernel<float, false>)
                     : (steps ? raster_fwd_kernel<double, true> : raster_fwd_kernel<double, false>);
    kern<<<tiles, GSN_BLOCK, 0, s>>>(ranges, order, ids, rec, n, cam, ro, img, fp32 ? nullptr : img64, Tfin, ncontrib,
                                     masks, tile_len, counts);
}

void launch_downsample2x(const float* src, int W, int H, float* dst, hipStream_t s) {
    const size_t n = (size_t)3 * (W / 2) * (H / 2);
    if (n) downsample2x_kernel<<<(unsigned)((n + kThreads - 1) / kThreads), kThreads, 0, s>>>(src, W, H, dst);
}
