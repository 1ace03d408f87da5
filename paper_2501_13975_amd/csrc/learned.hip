// learned.hip -- the learned per-kernel step scale: features, labels, and the
// 17 -> 32 -> 5 network (inference and Adam training).
//
// The overshoot control of Sec. 4.3 (eq. tildel) adds the blocks of the |N_t|
// nearest training views to the primary's.  The learned form replaces those
// views on most sweeps by a network that predicts, per kernel and attribute
// group, how much of the primary-only Newton step the full rule would keep; it
// is trained on sweeps that run the full rule.
//
// features_kernel: one thread per kernel, the reduced systems of the solve built
//   from the primary view's blocks alone (reduced.h), 16 log-scaled summaries, and
//   the neighbouring-view residual cached from the kernel's last full-rule sweep.
// labels_kernel:   alpha_eff = <Delta_aug, Delta_prim> / |Delta_prim|^2 per group.
// mlp_infer_kernel: one thread per kernel, FP16 weights staged in LDS, FP32
//   accumulation, alpha = 1.5 sigmoid(W2 relu(W1 f + b1) + b2).
// mlp_grad_kernel / mlp_adam_kernel: per-block gradient partials over 128
//   samples (fixed summation order), then one workgroup sums the partials in
//   block order, divides by the number of labelled entries and takes one Adam
//   step on the FP32 master weights, refreshing the FP16 copy.
#include "gsn_internal.h"
#include "reduced.h"
#include <hip/hip_fp16.h>

namespace {

constexpr int NI = GSN_MLP_IN, NH = GSN_MLP_HID, NO = GSN_MLP_OUT, NP = GSN_MLP_PARAMS;
constexpr int OFF_B1 = NH * NI, OFF_W2 = OFF_B1 + NH, OFF_B2 = OFF_W2 + NO * NH;
constexpr int GRAD_SAMPLES = 128;

__device__ __forceinline__ float feat_log(double x, bool& in_range) {
    const double v = log10(x + 1e-30) / 10.0;
    if (!(v >= -3.0 && v <= 3.0)) in_range = false;
    return (float)fmin(3.0, fmax(-3.0, v));
}

__device__ __forceinline__ void eig2(const double H[3], double& hi, double& lo) {
    const double mid = 0.5 * (H[0] + H[2]);
    const double rad = sqrt(0.25 * (H[0] - H[2]) * (H[0] - H[2]) + H[1] * H[1]);
    hi = mid + rad;
    lo = mid - rad;
}

__global__ __launch_bounds__(128) void features_kernel(const float* __restrict__ pos, const float* __restrict__ rot,
                                                        const float* __restrict__ scale,
                                                        const float* __restrict__ opac, int n, DevCam c,
                                                        float kappa, const float* __restrict__ blk,
                                                        gsn_solve_opts o, const float* __restrict__ resid,
                                                        float* __restrict__ feat, uint8_t* __restrict__ ok) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    auto B = [&](int row) { return (double)blk[(size_t)row * N + k]; };
    float f[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) f[i] = 0.f;
    const bool vis = B(29) > 0.0;
    bool in_range = vis;
    if (vis) {
        const double abs_scale = 1.0 / (3.0 * (double)o.npix_primary);
        Reduced R;
        reduce_systems(pos, rot, scale, opac, n, k, c, kappa, B, o, abs_scale, R);
        double hi, lo;
        eig2(R.Hp, hi, lo);
        f[0] = feat_log(fabs(hi), in_range);
        f[1] = feat_log(fabs(lo), in_range);
        f[2] = lo >= 0.0 ? 1.f : -1.f;
        f[3] = feat_log(fabs(R.Ht), in_range);
        f[4] = R.Ht >= 0.0 ? 1.f : -1.f;
        eig2(R.Hs, hi, lo);
        f[5] = feat_log(fabs(hi), in_range);
        f[6] = feat_log(fabs(lo), in_range);
        f[7] = lo >= 0.0 ? 1.f : -1.f;
        f[8] = feat_log(fabs(R.Ho), in_range);
        f[9] = feat_log(fabs(B(GSN_BLK_BASE + 3)) + fabs(B(GSN_BLK_BASE + 4)) + fabs(B(GSN_BLK_BASE + 5)), in_range);
        f[10] = feat_log(B(29), in_range);
        f[11] = feat_log(sqrt(R.gp[0] * R.gp[0] + R.gp[1] * R.gp[1]), in_range);
        f[12] = feat_log(fabs(R.gt), in_range);
        f[13] = feat_log(sqrt(R.gs[0] * R.gs[0] + R.gs[1] * R.gs[1]), in_range);
        f[14] = feat_log(fabs(R.go), in_range);
        f[15] = feat_log((double)opac[k], in_range);
        f[16] = feat_log(resid ? (double)resid[k] : 0.0, in_range);
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) feat[(size_t)i * N + k] = f[i];
    ok[k] = !vis ? GSN_FEAT_HIDDEN : in_range ? GSN_FEAT_OK : GSN_FEAT_OUT_OF_RANGE;
}

// Neighbouring-view residual of every kernel covered by the primary and a secondary view.
__global__ __launch_bounds__(256) void neighbour_residual_kernel(const float* __restrict__ blk, int n, int V,
                                                                  float* __restrict__ resid) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    if (!(blk[29 * N + k] > 0.f)) return;
    auto gnorm = [&](int v) {
        const size_t b = GSN_BLK_BASE + (size_t)GSN_BLK_VIEW * v;
        const double x = blk[b * N + k], y = blk[(b + 1) * N + k], z = blk[(b + 2) * N + k];
        return sqrt(x * x + y * y + z * z);
    };
    double sec = 0.0;
    bool seen = false;
    for (int v = 1; v < V; ++v) {
        if (blk[(GSN_BLK_BASE + (size_t)GSN_BLK_VIEW * v + 9) * N + k] > 0.f) {
            sec += gnorm(v);
            seen = true;
        }
    }
    if (seen) resid[k] = (float)(sec / (gnorm(0) + 1e-30));
}

constexpr int LABEL_BLOCK = 256;

// Labels of every kernel, and per workgroup the sums of mask |alpha - label| and of the mask
// (part[2 b], part[2 b + 1]) when alpha is given.
__global__ __launch_bounds__(LABEL_BLOCK) void labels_kernel(int n, int K, const float* __restrict__ sp,
                                                              const int32_t* __restrict__ fp,
                                                              const float* __restrict__ sa,
                                                              const uint8_t* __restrict__ ok,
                                                              const float* __restrict__ alpha,
                                                              float* __restrict__ label, float* __restrict__ mask,
                                                              double* __restrict__ part) {
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    double err = 0.0, cnt = 0.0;
    if (k < n) {
        const size_t N = (size_t)n;
        // a kernel the solve stepped (decisions >= -1) whose features were in range
        const bool use = fp[k] >= -1 && (!ok || ok[k] == GSN_FEAT_OK);
        const int lo[NO] = {0, 3, 7, 10, GSN_STEP_BASE};
        const int hi[NO] = {3, 4, 10, 11, GSN_STEP_BASE + 3 * K};
#pragma unroll
        for (int gi = 0; gi < NO; ++gi) {
            double pp = 0.0, ap = 0.0;
            for (int r = lo[gi]; r < hi[gi]; ++r) {
                const double p = sp[(size_t)r * N + k], a = sa[(size_t)r * N + k];
                pp += p * p;
                ap += a * p;
            }
            const bool good = use && pp > 1e-30;
            const float lab = good ? (float)fmin(1.5, fmax(0.0, ap / pp)) : 0.f;
            label[(size_t)gi * N + k] = lab;
            mask[(size_t)gi * N + k] = good ? 1.f : 0.f;
            if (good && alpha) {
                err += fabs((double)alpha[(size_t)gi * N + k] - (double)lab);
                cnt += 1.0;
            }
        }
    }
    if (!part) return;  // uniform across the launch
    __shared__ double s_e[LABEL_BLOCK], s_c[LABEL_BLOCK];
    s_e[threadIdx.x] = err;
    s_c[threadIdx.x] = cnt;
    __syncthreads();
    for (int w = LABEL_BLOCK / 2; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            s_e[threadIdx.x] += s_e[threadIdx.x + w];
            s_c[threadIdx.x] += s_c[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s_e[0];
        part[2 * blockIdx.x + 1] = s_c[0];
    }
}

// Deterministic sums of the rows of a [rows][cols] array of per-block partials: the rows are cut into
// kSlices contiguous ranges, and out[s][c] = the sum over range s of in[r][c] in a fixed order (each of
// the workgroup's four waves takes every fourth row, the waves' sums are added in wave order); the
// consumer adds the kSlices slice sums in order.  Grid (ceil(cols / 64), kSlices), 256 threads.  One
// thread per column summing thousands of partials one after another was latency-bound (6 ms for the
// network's gradient at 1M kernels).
constexpr int kSlices = 64;
template <class T>
__global__ __launch_bounds__(256) void column_slices_kernel(const T* __restrict__ in, int rows, int cols,
                                                             double* __restrict__ out) {
    __shared__ double s_w[4][64];
    const int lane = __lane_id(), w = threadIdx.x / 64;
    const int c = blockIdx.x * 64 + lane;
    const int chunk = (rows + kSlices - 1) / kSlices;
    const int r0 = blockIdx.y * chunk, r1 = min(rows, r0 + chunk);
    double a = 0.0;
    if (c < cols)
        for (int r = r0 + w; r < r1; r += 4) a += (double)in[(size_t)r * cols + c];
    s_w[w][lane] = a;
    __syncthreads();
    if (w == 0 && c < cols) out[(size_t)blockIdx.y * cols + c] = ((s_w[0][lane] + s_w[1][lane]) + s_w[2][lane]) + s_w[3][lane];
}

// out[0] += the sum of the label errors, out[1] += that of the mask, from the slice sums of part.
__global__ void label_error_sum_kernel(const double* __restrict__ slices, double* __restrict__ out) {
    const int t = threadIdx.x;
    if (t >= 2) return;
    double a = 0.0;
    for (int sl = 0; sl < kSlices; ++sl) a += slices[2 * sl + t];
    out[t] += a;
}

__global__ __launch_bounds__(256) void mlp_infer_kernel(const __half* __restrict__ wh, int n,
                                                         const float* __restrict__ feat,
                                                         const uint8_t* __restrict__ ok, float* __restrict__ out,
                                                         uint32_t* __restrict__ n_out_of_range) {
    __shared__ float w[NP];
    for (int i = threadIdx.x; i < NP; i += blockDim.x) w[i] = __half2float(wh[i]);
    __syncthreads();
    const int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    const size_t N = (size_t)n;
    float f[NI];
#pragma unroll
    for (int i = 0; i < NI; ++i) f[i] = feat[(size_t)i * N + k];
    float z2[NO];
#pragma unroll
    for (int g = 0; g < NO; ++g) z2[g] = w[OFF_B2 + g];
    for (int j = 0; j < NH; ++j) {
        float z = w[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NI; ++i) z += w[j * NI + i] * f[i];
        const float h = fmaxf(z, 0.f);
#pragma unroll
        for (int g = 0; g < NO; ++g) z2[g] += w[OFF_W2 + g * NH + j] * h;
    }
    const bool use = ok[k] == GSN_FEAT_OK;
#pragma unroll
    for (int g = 0; g < NO; ++g) out[(size_t)g * N + k] = use ? 1.5f / (1.f + expf(-z2[g])) : 0.f;
    if (n_out_of_range && ok[k] == GSN_FEAT_OUT_OF_RANGE) atomicAdd(n_out_of_range, 1u);
}

// Per-block gradient partials (not yet divided by the number of labelled entries): part[b][p],
// and per-block sums of the squared masked residuals and of the mask in double.
__global__ __launch_bounds__(GRAD_SAMPLES) void mlp_grad_kernel(const float* __restrict__ wf, int n,
                                                                 const float* __restrict__ feat,
                                                                 const float* __restrict__ label,
                                                                 const float* __restrict__ mask,
                                                                 float* __restrict__ part,
                                                                 double* __restrict__ stat) {
    __shared__ float w[NP];
    __shared__ float sF[GRAD_SAMPLES][NI], sH[GRAD_SAMPLES][NH], sD1[GRAD_SAMPLES][NH];
    __shared__ float sD2[GRAD_SAMPLES][NO];
    __shared__ double sL[GRAD_SAMPLES], sM[GRAD_SAMPLES];
    const int t = threadIdx.x;
    for (int i = t; i < NP; i += GRAD_SAMPLES) w[i] = wf[i];
    __syncthreads();
    const int k = blockIdx.x * GRAD_SAMPLES + t;
    const size_t N = (size_t)n;
    float f[NI], z1[NH], d2[NO];
    double ls = 0.0, ms = 0.0;
#pragma unroll
    for (int i = 0; i < NI; ++i) f[i] = k < n ? feat[(size_t)i * N + k] : 0.f;
    float z2[NO];
#pragma unroll
    for (int g = 0; g < NO; ++g) z2[g] = w[OFF_B2 + g];
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float z = w[OFF_B1 + j];
#pragma unroll
        for (int i = 0; i < NI; ++i) z += w[j * NI + i] * f[i];
        z1[j] = z;
        const float h = fmaxf(z, 0.f);
        sH[t][j] = h;
#pragma unroll
        for (int g = 0; g < NO; ++g) z2[g] += w[OFF_W2 + g * NH + j] * h;
    }
#pragma unroll
    for (int g = 0; g < NO; ++g) {
        const float sg = 1.f / (1.f + expf(-z2[g]));
        const float m = k < n ? mask[(size_t)g * N + k] : 0.f;
        const float r = k < n ? (1.5f * sg - label[(size_t)g * N + k]) * m : 0.f;
        ls += (double)r * (double)r;
        ms += (double)m;
        d2[g] = 2.f * r * 1.5f * sg * (1.f - sg);
        sD2[t][g] = d2[g];
    }
#pragma unroll
    for (int j = 0; j < NH; ++j) {
        float dh = 0.f;
#pragma unroll
        for (int g = 0; g < NO; ++g) dh += w[OFF_W2 + g * NH + j] * d2[g];
        sD1[t][j] = z1[j] > 0.f ? dh : 0.f;
    }
#pragma unroll
    for (int i = 0; i < NI; ++i) sF[t][i] = f[i];
    sL[t] = ls;
    sM[t] = ms;
    __syncthreads();
    float* pb = part + (size_t)blockIdx.x * NP;
    for (int p = t; p < NP; p += GRAD_SAMPLES) {
        float acc = 0.f;
        if (p < OFF_B1) {
            const int j = p / NI, i = p % NI;
            for (int s = 0; s < GRAD_SAMPLES; ++s) acc += sD1[s][j] * sF[s][i];
        } else if (p < OFF_W2) {
            const int j = p - OFF_B1;
            for (int s = 0; s < GRAD_SAMPLES; ++s) acc += sD1[s][j];
        } else if (p < OFF_B2) {
            const int g = (p - OFF_W2) / NH, j = (p - OFF_W2) % NH;
            for (int s = 0; s < GRAD_SAMPLES; ++s) acc += sD2[s][g] * sH[s][j];
        } else {
            const int g = p - OFF_B2;
            for (int s = 0; s < GRAD_SAMPLES; ++s) acc += sD2[s][g];
        }
        pb[p] = acc;
    }
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int s = 0; s < GRAD_SAMPLES; ++s) {
            a += sL[s];
            b += sM[s];
        }
        stat[2 * blockIdx.x] = a;
        stat[2 * blockIdx.x + 1] = b;
    }
}

// One workgroup: sums the partials in block order, divides by the labelled count, takes one
// Adam step (step number t) and refreshes the FP16 copy; writes the loss before the step.
__global__ __launch_bounds__(256) void mlp_adam_kernel(float* __restrict__ wf, float* __restrict__ m,
                                                        float* __restrict__ v, __half* __restrict__ wh,
                                                        const double* __restrict__ grad_slices,
                                                        const double* __restrict__ stat_slices, int t,
                                                        float lr, float b1, float b2, float eps,
                                                        float* __restrict__ grad_out, double* __restrict__ loss) {
    __shared__ double s_cnt, s_loss;
    if (threadIdx.x == 0) {
        double a = 0.0, c = 0.0;
        for (int sl = 0; sl < kSlices; ++sl) {
            a += stat_slices[2 * sl];
            c += stat_slices[2 * sl + 1];
        }
        s_cnt = fmax(c, 1.0);
        s_loss = a;
    }
    __syncthreads();
    const double cnt = s_cnt;
    if (threadIdx.x == 0 && loss) loss[0] = s_loss / cnt;
    const double c1 = 1.0 - pow((double)b1, (double)t), c2 = 1.0 - pow((double)b2, (double)t);
    for (int p = threadIdx.x; p < NP; p += blockDim.x) {
        double gsum = 0.0;
        for (int sl = 0; sl < kSlices; ++sl) gsum += grad_slices[(size_t)sl * NP + p];
        const float g = (float)(gsum / cnt);
        if (grad_out) grad_out[p] = g;
        const float mm = b1 * m[p] + (1.f - b1) * g;
        const float vv = b2 * v[p] + (1.f - b2) * g * g;
        m[p] = mm;
        v[p] = vv;
        const float w = wf[p] - lr * (float)((double)mm / c1) / (sqrtf((float)((double)vv / c2)) + eps);
        wf[p] = w;
        wh[p] = __float2half(w);
    }
}

__global__ void mlp_reset_kernel(const float* __restrict__ wf, float* __restrict__ m, float* __restrict__ v,
                                 __half* __restrict__ wh) {
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= NP) return;
    m[p] = 0.f;
    v[p] = 0.f;
    wh[p] = __float2half(wf[p]);
}

}  // namespace

void launch_features(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                     const gsn_solve_opts& o, const float* resid, float* feat, uint8_t* ok, hipStream_t s) {
    if (g.n == 0) return;
    features_kernel<<<(g.n + 127) / 128, 128, 0, s>>>(g.d_pos, g.d_rot, g.d_scale, g.d_opac, g.n, cam, kappa,
                                                      b.d_data, o, resid, feat, ok);
}

void launch_neighbour_residual(const gsn_blocks& b, float* resid, hipStream_t s) {
    if (b.n == 0) return;
    neighbour_residual_kernel<<<(b.n + 255) / 256, 256, 0, s>>>(b.d_data, b.n, b.n_views, resid);
}

int label_blocks(int n) { return (n + LABEL_BLOCK - 1) / LABEL_BLOCK; }

void launch_labels(int n, int K, const float* sp, const int32_t* fp, const float* sa, const uint8_t* ok,
                   const float* alpha, float* label, float* mask, double* part, double* err, hipStream_t s) {
    if (n == 0) return;
    const int nb = label_blocks(n);
    labels_kernel<<<nb, LABEL_BLOCK, 0, s>>>(n, K, sp, fp, sa, ok, alpha, label, mask, alpha && err ? part : nullptr);
    if (alpha && err) {
        double* slices = part + 2 * (size_t)nb;
        column_slices_kernel<double><<<dim3(1, kSlices), 256, 0, s>>>(part, nb, 2, slices);
        label_error_sum_kernel<<<1, 64, 0, s>>>(slices, err);
    }
}

size_t label_part_words(int n) { return 2 * (size_t)std::max(label_blocks(n), 1) + 2 * (size_t)kSlices; }
size_t mlp_stat_words(int n) {
    return 2 * (size_t)std::max(mlp_grad_blocks(n), 1) + (size_t)kSlices * (GSN_MLP_PARAMS + 2);
}

void launch_mlp_infer(const uint16_t* wh, int n, const float* feat, const uint8_t* ok, float* out,
                      uint32_t* n_out_of_range, hipStream_t s) {
    if (n == 0) return;
    mlp_infer_kernel<<<(n + 255) / 256, 256, 0, s>>>(reinterpret_cast<const __half*>(wh), n, feat, ok, out,
                                                     n_out_of_range);
}

int mlp_grad_blocks(int n) { return (n + GRAD_SAMPLES - 1) / GRAD_SAMPLES; }

void launch_mlp_train(gsn_mlp& mlp, int n, const float* feat, const float* label, const float* mask, float* part,
                      double* stat, const gsn_adam_opts& a, float* grad_out, double* loss, hipStream_t s) {
    const int nb = std::max(mlp_grad_blocks(n), 1);
    if (n > 0) mlp_grad_kernel<<<nb, GRAD_SAMPLES, 0, s>>>(mlp.d_params, n, feat, label, mask, part, stat);
    // stat holds [nb][2] partials, then the slice sums of the gradient [kSlices][NP] and of stat [kSlices][2]
    double* gslices = stat + 2 * (size_t)nb;
    double* sslices = gslices + (size_t)kSlices * NP;
    const int rows = n > 0 ? nb : 0;
    column_slices_kernel<float><<<dim3((NP + 63) / 64, kSlices), 256, 0, s>>>(part, rows, NP, gslices);
    column_slices_kernel<double><<<dim3(1, kSlices), 256, 0, s>>>(stat, rows, 2, sslices);
    mlp_adam_kernel<<<1, 256, 0, s>>>(mlp.d_params, mlp.d_m, mlp.d_v, reinterpret_cast<__half*>(mlp.d_half), gslices,
                                      sslices, mlp.step, a.lr, a.beta1, a.beta2, a.eps, grad_out, loss);
}

void launch_mlp_reset(gsn_mlp& mlp, hipStream_t s) {
    mlp_reset_kernel<<<(GSN_MLP_PARAMS + 255) / 256, 256, 0, s>>>(mlp.d_params, mlp.d_m, mlp.d_v,
                                                                  reinterpret_cast<__half*>(mlp.d_half));
}
