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
// The per-kernel statistics over the projected variables
//     z = (pi_x, pi_y, Q_xx, Q_xy, Q_yy | sigma | c~_R, c~_G, c~_B)
// (Q_xy enters d^T Q d twice) are, with u = df/d(pi, Q), A1 = sum_ch dL_ch a_ch,
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
    const float* __restrict__ img, const uint32_t* __restrict__ ncontrib, const float* __restrict__ dLm,
    const float* __restrict__ hdm, float* __restrict__ partial, uint8_t* __restrict__ flags) {
    __shared__ float4 s_a[GSN_BLOCK];
    __shared__ float4 s_b[GSN_BLOCK];
    __shared__ float s_c[GSN_BLOCK];
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
    float cf[3] = {0, 0, 0}, dl[3] = {0, 0, 0}, hh[3] = {0, 0, 0};
    uint32_t nc = 0;
    if (inside) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            cf[ch] = img[ch * np + pi];
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
    float T = 1.f, Ca0 = 0.f, Ca1 = 0.f, Ca2 = 0.f;
    const float fpx = (float)px, fpy = (float)py;
    for (uint32_t base = rg.x; base < end; base += GSN_BLOCK) {
        const uint32_t e = base + threadIdx.x;
        if (e < end) {
            const uint32_t id = ids[e];
            s_a[threadIdx.x] = rec[id];
            s_b[threadIdx.x] = rec[n + id];
            s_c[threadIdx.x] = rec[2 * (size_t)n + id].x;
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
                    const float sig = b.y;
                    const float ct[3] = {b.z, b.w, s_c[j]};
                    const SplatEval ev = eval_splat(a.x, a.y, a.z, a.w, b.x, sig, fpx, fpy, ro.alpha_max);
                    if (ev.alpha >= ro.alpha_min) {
                        act = true;
                        const float al = ev.alpha, wT = al * T;
                        Ca0 += wT * ct[0];
                        Ca1 += wT * ct[1];
                        Ca2 += wT * ct[2];
                        const float inv = 1.0f / (1.0f - al);
                        const float av[3] = {T * ct[0] - (cf[0] - Ca0) * inv, T * ct[1] - (cf[1] - Ca1) * inv,
                                             T * ct[2] - (cf[2] - Ca2) * inv};
                        const float A1 = dl[0] * av[0] + dl[1] * av[1] + dl[2] * av[2];
                        const float A2 = hh[0] * av[0] * av[0] + hh[1] * av[1] * av[1] + hh[2] * av[2] * av[2];
#pragma unroll
                        for (int ch = 0; ch < 3; ++ch) {
                            z[6 + ch] = dl[ch] * wT;
                            z[39 + ch] = hh[ch] * wT * wT;
                        }
                        z[43] = wT;
                        if (!ev.clamped) {
                            const float G = ev.G, dx = ev.dx, dy = ev.dy;
                            const float u[5] = {-(a.z * dx + a.w * dy), -(a.w * dx + b.x * dy), -0.5f * dx * dx,
                                                -dx * dy, -0.5f * dy * dy};
                            const float sG = sig * G;
                            const float k1 = A1 * sG;
                            const float k2 = A2 * sG * sG + k1;
#pragma unroll
                            for (int i = 0; i < 5; ++i) z[i] = k1 * u[i];
                            z[5] = A1 * G;
                            // H_ww: k2 u u^T + k1 d2f, d2f has -Q on (pi, pi) and -d on (pi, Q)
                            int idx = 9;
#pragma unroll
                            for (int i = 0; i < 5; ++i)
#pragma unroll
                                for (int jx = i; jx < 5; ++jx, ++idx) z[idx] = k2 * u[i] * u[jx];
                            z[9 + 0] -= k1 * a.z;   // (pi_x, pi_x)
                            z[9 + 1] -= k1 * a.w;   // (pi_x, pi_y)
                            z[9 + 2] -= k1 * dx;    // (pi_x, Q_xx)
                            z[9 + 3] -= k1 * dy;    // (pi_x, Q_xy)
                            z[9 + 5] -= k1 * b.x;   // (pi_y, pi_y)
                            z[9 + 7] -= k1 * dx;    // (pi_y, Q_xy)
                            z[9 + 8] -= k1 * dy;    // (pi_y, Q_yy)
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

// ---------------------------------------------------------------------------
// Chain rule through the projection (Sec. 3; Appendix A.1-A.3): per attribute
// group y, H_y = J^T H_z J + sum_i (g_z)_i d2 z_i / dy2 with J = dz/dy, using
// jets for z(y).  Sigma = A A^T + kappa I with A = J_persp W R(q/|q|) diag(s).
// ---------------------------------------------------------------------------
struct KParams {
    float p[3], q[4], s[3];
};

// Jacobian of the perspective map at t = W p + t_c times the camera rotation (M = J W).
template <class TT>
__device__ __forceinline__ void persp_M(const TT t[3], const DevCam& c, TT M[2][3], TT& iz) {
    iz = jrecip(t[2]);
    const TT J00 = c.fx * iz, J11 = c.fy * iz;
    const TT J02 = -(c.fx * t[0]) * iz * iz, J12 = -(c.fy * t[1]) * iz * iz;
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        M[0][k] = J00 * c.R[k] + J02 * c.R[6 + k];
        M[1][k] = J11 * c.R[3 + k] + J12 * c.R[6 + k];
    }
}

template <class TT>
__device__ __forceinline__ void quat_rot(const TT q[4], TT Rq[3][3]) {
    const TT qn = jsqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const TT iq = jrecip(qn);
    const TT w = q[0] * iq, x = q[1] * iq, y = q[2] * iq, z = q[3] * iq;
    Rq[0][0] = 1.0f - 2.0f * (y * y + z * z);
    Rq[0][1] = 2.0f * (x * y - w * z);
    Rq[0][2] = 2.0f * (x * z + w * y);
    Rq[1][0] = 2.0f * (x * y + w * z);
    Rq[1][1] = 1.0f - 2.0f * (x * x + z * z);
    Rq[1][2] = 2.0f * (y * z - w * x);
    Rq[2][0] = 2.0f * (x * z - w * y);
    Rq[2][1] = 2.0f * (y * z + w * x);
    Rq[2][2] = 1.0f - 2.0f * (x * x + y * y);
}

// Q = Sigma^{-1} from A (2x3): Sigma = A A^T + kappa I.
template <class TT>
__device__ __forceinline__ void conic_from_A(const TT A[2][3], float kappa, TT Q[3]) {
    const TT sxx = A[0][0] * A[0][0] + A[0][1] * A[0][1] + A[0][2] * A[0][2] + kappa;
    const TT sxy = A[0][0] * A[1][0] + A[0][1] * A[1][1] + A[0][2] * A[1][2];
    const TT syy = A[1][0] * A[1][0] + A[1][1] * A[1][1] + A[1][2] * A[1][2] + kappa;
    const TT idet = jrecip(sxx * syy - sxy * sxy);
    Q[0] = syy * idet;
    Q[1] = -(sxy * idet);
    Q[2] = sxx * idet;
}

// Accumulates g and packed H of group y from z-jets: H = sum_ij Hz_ij dz_i dz_j^T + sum_i gz_i d2z_i.
template <int N, int NZ>
__device__ __forceinline__ void chain_accumulate(const FJet<N>* zj, const float* gz, const float Hz[NZ][NZ],
                                                 float* g, float* H) {
#pragma unroll
    for (int a = 0; a < N; ++a) {
        float acc = 0.f;
#pragma unroll
        for (int i = 0; i < NZ; ++i) acc += gz[i] * zj[i].g[a];
        g[a] = acc;
    }
    float t[NZ][N];
#pragma unroll
    for (int i = 0; i < NZ; ++i)
#pragma unroll
        for (int b = 0; b < N; ++b) {
            float acc = 0.f;
#pragma unroll
            for (int j = 0; j < NZ; ++j) acc += Hz[i][j] * zj[j].g[b];
            t[i][b] = acc;
        }
    int idx = 0;
#pragma unroll
    for (int a = 0; a < N; ++a)
#pragma unroll
        for (int b = a; b < N; ++b, ++idx) {
            float acc = 0.f;
#pragma unroll
            for (int i = 0; i < NZ; ++i) acc += zj[i].g[a] * t[i][b] + gz[i] * zj[i].h[idx];
            H[idx] = acc;
        }
}

__device__ void chain_position(const KParams& kp, const float* shk, int K, const DevCam& c, float kappa,
                               const float* z, float* g, float* H) {
    typedef FJet<3> J;
    J p[3] = {J::var(kp.p[0], 0), J::var(kp.p[1], 1), J::var(kp.p[2], 2)};
    J t[3];
#pragma unroll
    for (int i = 0; i < 3; ++i) t[i] = c.R[3 * i] * p[0] + c.R[3 * i + 1] * p[1] + c.R[3 * i + 2] * p[2] + c.t[i];
    J M[2][3], iz;
    persp_M(t, c, M, iz);
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
    zj[0] = c.fx * t[0] * iz + c.cx;
    zj[1] = c.fy * t[1] * iz + c.cy;
    {
        const J d0 = p[0] - c.o[0], d1 = p[1] - c.o[1], d2 = p[2] - c.o[2];
        const J il = jrecip(jsqrt(d0 * d0 + d1 * d1 + d2 * d2));
        J Y[16];
        sh_basis_dev<J>(K, d0 * il, d1 * il, d2 * il, Y);
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            J acc(0.f);
            for (int i = 0; i < K; ++i) acc = acc + shk[ch * K + i] * Y[i];
            zj[5 + ch] = acc;
        }
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
    chain_accumulate<3, 8>(zj, gz, Hz, g, H);
}

template <int N>
__device__ void chain_shape(const KParams& kp, const DevCam& c, float kappa, const float* z, bool rotation, float* g,
                            float* H) {
    typedef FJet<N> J;
    float tf[3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
        tf[i] = c.R[3 * i] * kp.p[0] + c.R[3 * i + 1] * kp.p[1] + c.R[3 * i + 2] * kp.p[2] + c.t[i];
    float M[2][3], iz;
    persp_M<float>(tf, c, M, iz);
    J A[2][3];
    if (rotation) {
        J q[4];
#pragma unroll
        for (int a = 0; a < 4; ++a) q[a] = a < N ? J::var(kp.q[a], a < N ? a : 0) : J(kp.q[a]);
        J Rq[3][3];
        quat_rot<J>(q, Rq);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a) A[i][a] = (M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a]) * kp.s[a];
    } else {
        float Rq[3][3];
        quat_rot<float>(kp.q, Rq);
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const J sv = J::var(kp.s[a], a < N ? a : 0);
                A[i][a] = (M[i][0] * Rq[0][a] + M[i][1] * Rq[1][a] + M[i][2] * Rq[2][a]) * sv;
            }
    }
    J Q[3];
    conic_from_A(A, kappa, Q);
    float Hz[3][3];
    // (Q_xx, Q_xy, Q_yy) are entries 2..4 of the (pi, Q) block
    const int pk[3][3] = {{9 + 9, 9 + 10, 9 + 11}, {9 + 10, 9 + 12, 9 + 13}, {9 + 11, 9 + 13, 9 + 14}};
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Hz[i][j] = z[pk[i][j]];
    const float gz[3] = {z[2], z[3], z[4]};
    chain_accumulate<N, 3>(Q, gz, Hz, g, H);
}

__global__ __launch_bounds__(128) void reduce_chain_kernel(
    const float* __restrict__ pos, const float* __restrict__ rot, const float* __restrict__ scale,
    const float* __restrict__ sh, int n, int K, const uint2* __restrict__ rect, const uint32_t* __restrict__ pair_off,
    const float* __restrict__ partial, const uint8_t* __restrict__ flags, DevCam cam, float kappa, float weight,
    int slot, float* __restrict__ blk, float* __restrict__ zstats) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const uint2 rc = rect[k];
    const uint32_t nt = ((rc.y & 0xffffu) - (rc.x & 0xffffu)) * ((rc.y >> 16) - (rc.x >> 16));
    float z[GSN_NZ];
#pragma unroll
    for (int f = 0; f < GSN_NZ; ++f) z[f] = 0.f;
    const uint32_t off = pair_off[k];
    for (uint32_t i = 0; i < nt; ++i) {
        const uint32_t sl = off + i;
        if (!flags[sl]) continue;
        const float4* pp = reinterpret_cast<const float4*>(partial + (size_t)sl * GSN_NZ);
#pragma unroll
        for (int f = 0; f < GSN_NZ / 4; ++f) {
            const float4 v = pp[f];
            z[4 * f] += v.x;
            z[4 * f + 1] += v.y;
            z[4 * f + 2] += v.z;
            z[4 * f + 3] += v.w;
        }
    }
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
    float g[4], H[10];
    const size_t N = (size_t)n;
    chain_position(kp, shk, K, cam, kappa, z, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) blk[a * N + k] += weight * g[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) blk[(3 + a) * N + k] += weight * H[a];
    chain_shape<4>(kp, cam, kappa, z, true, g, H);
#pragma unroll
    for (int a = 0; a < 4; ++a) blk[(9 + a) * N + k] += weight * g[a];
#pragma unroll
    for (int a = 0; a < 10; ++a) blk[(13 + a) * N + k] += weight * H[a];
    chain_shape<3>(kp, cam, kappa, z, false, g, H);
#pragma unroll
    for (int a = 0; a < 3; ++a) blk[(23 + a) * N + k] += weight * g[a];
#pragma unroll
    for (int a = 0; a < 6; ++a) blk[(26 + a) * N + k] += weight * H[a];
    blk[32 * N + k] += weight * z[5];
    blk[33 * N + k] += weight * z[42];
    if (slot == 0) blk[34 * N + k] = z[43];
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
        bp<uint2>(f.rect), bp<uint32_t>(f.pair_off), (uint32_t)f.n, f.cam, f.ro, bp<float>(f.img),
        bp<uint32_t>(f.ncontrib), dL, hd, bp<float>(f.partial), bp<uint8_t>(f.flags));
}

void launch_reduce_chain(const gsn_frame& f, const gsn_gaussians& g, float weight, int slot, const gsn_blocks& b,
                         float* zstats_out, hipStream_t s) {
    if (g.n == 0) return;
    const int K = (g.sh_degree + 1) * (g.sh_degree + 1);
    reduce_chain_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(
        g.d_pos, g.d_rot, g.d_scale, g.d_sh, g.n, K, bp<uint2>(f.rect), bp<uint32_t>(f.pair_off),
        bp<float>(f.partial), bp<uint8_t>(f.flags), f.cam, f.ro.kappa, weight, slot, b.d_data, zstats_out);
}
