// gsn_internal.h -- host-side declarations shared by the translation units of libgsn.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/gsn.h"
#include "device_common.h"

// Device buffer that only grows.
struct DevBuf {
    void* p = nullptr;
    size_t bytes = 0;
};
hipError_t buf_reserve(DevBuf& b, size_t bytes);
void buf_free(DevBuf& b);
template <class T>
T* bp(const DevBuf& b) { return static_cast<T*>(b.p); }

// The forward raster records, for the first GSN_MASK_BATCHES staged batches of each tile's
// list, which entries every pixel composited; the backward raster reads these masks instead of
// evaluating the batch again (later batches are evaluated).
constexpr int GSN_MASK_BATCHES = 8;

struct gsn_frame {
    bool rendered = false;
    int n = 0, K = 0, W = 0, H = 0, tiles_x = 0, tiles_y = 0;
    // pair count of the last render when known on the host (growing mode), -1 in reserved mode
    // (then it lives only in total[1] on the device)
    int64_t pairs = 0;
    // reserved mode (gsn_frame_reserve): capacities the buffers were sized for; cap_pairs == 0 means
    // growing mode (buffers sized from the pair count read back after the depth sort)
    int64_t cap_pairs = 0;
    int cap_n = 0, cap_W = 0, cap_H = 0;
    // mixed form: the colour sums along each ray in single precision (no double image)
    bool fp32 = false;
    DevCam cam{};
    DevRenderOpts ro{};
    // per kernel
    DevBuf rec;         // float4 [n][4], one 64-byte record per kernel: (mx, my, q1, q2), (c, s, sigma, R),
                        // (G, B, mx_lo, my_lo), (rect x0 | y0 << 16, rect x1 | y1 << 16, pair offset, 0)
    DevBuf rect;        // uint2 [n]: (x0 | y0 << 16, x1 | y1 << 16)
    DevBuf depth_key;   // u32 [n], 0xffffffff when culled
    DevBuf ntiles;      // u32 [n]
    DevBuf ids_a, ids_b, keys_a, keys_b;  // u32 [n] sort ping-pong
    DevBuf offsets;     // u32 [n + 1] pair offset by depth rank
    DevBuf pair_off;    // u32 [n] pair offset by kernel id
    DevBuf nsup, moffs; // u32 [n] super-tile memberships by depth rank, and their offsets
    // per pair: the super-tile memberships (key, id) and their sort buffers; the tile lists are
    // written into the values buffer the sorted memberships do not occupy (list_ids)
    DevBuf pk_a, pv_a, pk_b, pv_b;
    uint32_t* list_ids = nullptr;  // u32 [pairs]: kernel ids of the tile lists, ranges index it
    // per super-tile / segment
    DevBuf sranges;     // uint2 [super-tiles]: member range
    DevBuf seg_base;    // u32 [super-tiles + 1]: first segment
    DevBuf seg_counts, seg_offs;  // u32 [segments x 64]: entries per (segment, tile), and their places in the lists
    DevBuf partial;     // float [pairs][GSN_NZ]
    DevBuf flags;       // u8 [pairs], partial written
    DevBuf kflag;       // u8 [n], some partial of the kernel written
    // per tile / pixel
    DevBuf ranges;      // uint2 [tiles]
    DevBuf tile_order;  // u32 [tiles]: launch order of the forward raster, longest lists first
    DevBuf tile_len;    // u32 [tiles]: composited prefix of each tile's list (longest over its pixels)
    DevBuf bwd_order;   // u32 [tiles]: launch order of the backward raster, longest prefixes first
    DevBuf img;         // float [3][H][W]
    DevBuf img64;       // double [3][H][W], the same colour before rounding
    DevBuf Tfin;        // float [H][W]
    DevBuf ncontrib;    // u32 [H][W]
    DevBuf masks;       // u64 [tiles][GSN_MASK_BATCHES][4][256]: composited (pixel, entry) pairs of each
                        // staged batch of 256 list entries, per pixel (bit j of word w: entry 64 w + j of
                        // the batch)
    DevBuf dL, hd;      // float [3][H][W] loss maps
    DevBuf coef;        // float [3][8][H][W] SSIM coefficient maps (computed in double, stored rounded)
    DevBuf zsum_f;      // float [n][GSN_NZ] per-kernel sums of the pair partials
    DevBuf zsum;        // double [n][10]: of those, the ones the rotation and scale chain rule reads
    DevBuf sumrows;     // float [kSumOverlap + 1][n]: this view's shares of the rows summed over the views
    DevBuf contrib;     // u8 [n]: the kernel has shares in sumrows (the view reached it)
    DevBuf zstats;      // float [GSN_NZ][n], optional debug copy
    DevBuf loss_part;   // double [2][nblocks]
    // sort / scan scratch; total: u32 [0] scanned pair total, [1] live pair count of the render,
    // [2] scanned membership total, [3] live membership count, [4] scanned tile-list total
    DevBuf hist, scan_tmp, total;
    uint32_t* h_total = nullptr;  // pinned host word
};

struct ProfRec {
    int stage;
    hipEvent_t start, stop;
};

struct gsn_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    std::string err;
    // measurement (gsn_profile_enable)
    bool prof = false;
    bool prof_steps = false;  // level 2: the raster passes also count their wave steps
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> pool;
    unsigned long long* d_counts = nullptr;  // GSN_COUNT_N device counters
    // GSN_STAT_N device counters read and cleared by gsn_sync_status (always gathered)
    unsigned long long* d_stats = nullptr;
    // gradient partials of gsn_mlp_train_step, error partials of gsn_step_labels
    DevBuf mlp_part, mlp_stat, label_part;
    // batched solve: scene table and the tuned launch shape (0 = not tuned)
    DevBuf solve_table;
    int solve_block = 0, solve_grid = 0;
    // colour Gram matrices of the mixed form
    DevBuf gram;
    // this device's fixed scratch array of gsn_local_newton_solve_noalloc ([10][GSN_NOALLOC_MAX_N] floats)
    float* noalloc_gram = nullptr;
    // graph capture (gsn_capture_begin / end): the calls between them are recorded on cap_stream,
    // the library's own stream, in place of the caller's
    bool capturing = false, capture_failed = false;
    hipStream_t cap_stream = nullptr, user_stream = nullptr;
    // gsn_accumulate_views: the context's stream and three of the library's own take the views in
    // turn (the side streams forked from and joined back into the context's stream; four streams in
    // all, as many as the device gives a process hardware queues), and the events that order them
    static constexpr int kSide = 3, kMaxViews = 9;
    hipStream_t side[kSide] = {};
    hipEvent_t ev_fork = nullptr, ev_join[kSide] = {}, ev_chain[kMaxViews] = {};
};

struct gsn_graph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    DevBuf table;
    int stage = GSN_STAGE_SOLVE;  // profiler stage of a replay, -1: not timed (a captured sweep)
};

// Brackets one stage with events when profiling is on.
struct StageTimer {
    gsn_ctx* ctx;
    int idx = -1;
    StageTimer(gsn_ctx* c, int stage);
    ~StageTimer();
};
inline unsigned long long* prof_counts(const gsn_ctx* c) { return c->prof ? c->d_counts : nullptr; }
// The profile counter array holds GSN_COUNT_N counters, then GSN_SOLVE_SPREAD copies of the
// GSN_SOLVE_EVENTS solve counters (GSN_COUNT_SOLVE_ESCALATED onwards) that gsn_profile_read sums.
#define GSN_SOLVE_EVENTS 13
#define GSN_SOLVE_SPREAD 64
constexpr int GSN_PROF_WORDS = GSN_COUNT_N + GSN_SOLVE_SPREAD * GSN_SOLVE_EVENTS;

// ---- launchers (render.hip)
void launch_fill_u32(uint32_t* p, uint32_t v, size_t n, hipStream_t s);
void launch_fill_f32(float* p, float v, size_t n, hipStream_t s);
// culled: device counter of kernels culled for non-finite attributes or colour
void launch_preprocess(const gsn_gaussians& g, const DevCam& cam, const DevRenderOpts& ro, float4* rec,
                       uint2* rect, uint32_t* depth_key, uint32_t* ids, uint32_t* ntiles, unsigned long long* culled,
                       hipStream_t s);
// stable LSD radix sort of (key, val) pairs on bits [bit_lo, bit_hi); result lands in (k0, v0).  The
// launches are sized for n keys; with d_n, only the first min(*d_n, n) keys (read on the device) are
// sorted.  hist must hold radix_hist_bytes(n) bytes.
// With k_res and v_res the result is left where the passes put it and returned there (no copy back).
hipError_t radix_sort_pairs(uint32_t* k0, uint32_t* v0, uint32_t* k1, uint32_t* v1, uint32_t n, const uint32_t* d_n,
                            int bit_lo, int bit_hi, DevBuf& hist, hipStream_t s, uint32_t** k_res = nullptr,
                            uint32_t** v_res = nullptr);
void launch_copy_u32(uint32_t* dst, const uint32_t* src, size_t n, hipStream_t s);
// d_pairs[1] = d_pairs[0] when it is at most cap, else 0 with the overflow recorded in stats
void launch_pair_capacity(uint32_t* d_pairs, uint32_t cap, unsigned long long* stats, unsigned long long* prof,
                          hipStream_t s);
// p[0 .. ceil(*d_count / per_word)) = v, at most cap words
void launch_fill_u32_dev(uint32_t* p, uint32_t v, const uint32_t* d_count, uint32_t per_word, size_t cap,
                         hipStream_t s);
// bytes of scan scratch for scanning up to n values (and the 256 x blocks radix histograms of n keys)
size_t scan_tmp_bytes(uint32_t n);
// exclusive scan of n u32 values into out; *d_total receives the sum
hipError_t exclusive_scan_u32(const uint32_t* in, uint32_t* out, uint32_t n, uint32_t* d_total,
                              DevBuf& scan_tmp, hipStream_t s);
void launch_gather_u32(const uint32_t* src, const uint32_t* idx, uint32_t* dst, uint32_t n, hipStream_t s);
// each kernel's (tile, kernel) slot offset by id, also into its record
void launch_pair_off(const uint32_t* sorted_ids, const uint32_t* offsets, uint32_t n, uint32_t* pair_off, float4* rec,
                     hipStream_t s);
// buffers of the two-level tile binning
struct TileListBufs {
    uint32_t *nsup, *moffs;           // [n]
    uint32_t *mk, *mv, *mk2, *mv2;    // [cap pairs]
    uint2* sranges;                   // [super-tiles]
    uint32_t* seg_base;               // [super-tiles + 1]
    uint32_t *counts, *offs;          // [segment_words]
    uint2* ranges;                    // [tiles]
};
uint32_t super_tiles(int tiles_x, int tiles_y);
// words of the per-(segment, tile) count and offset arrays for cap_pairs pairs
size_t segment_words(size_t cap_pairs, int tiles_x, int tiles_y);
// per-tile lists of the kernels whose tile rectangle covers each tile, in depth order (sorted_ids),
// for the live pair count d_total[1] (launches sized for cap pairs); *ids_out receives the list
// buffer (one of mv, mv2) that ranges index
hipError_t build_tile_lists(const uint32_t* sorted_ids, const uint2* rect, uint32_t n, uint32_t* d_total, uint32_t cap,
                            int tiles_x, int tiles_y, const TileListBufs& bufs, DevBuf& hist, DevBuf& scan_tmp,
                            uint32_t** ids_out, hipStream_t s);
// the projected records [n][4] as the public layout [3][n] (gsn_frame_records)
void launch_records_out(const float4* rec, int n, float4* out, hipStream_t s);
size_t radix_hist_bytes(uint32_t n);
// tiles ordered by a length, longest first (coarse: four buckets per octave, any order within one): the
// list lengths of ranges when lens is null, else lens
void launch_tile_order(const uint2* ranges, const uint32_t* lens, int tiles, uint32_t* order, hipStream_t s);
void launch_raster_fwd(const uint2* ranges, const uint32_t* order, const uint32_t* ids, const float4* rec, uint32_t n, const DevCam& cam,
                       const DevRenderOpts& ro, bool fp32, float* img, double* img64, float* Tfin, uint32_t* ncontrib,
                       uint64_t* masks, uint32_t* tile_len, unsigned long long* counts, bool steps, hipStream_t s);
void launch_downsample2x(const float* src, int W, int H, float* dst, hipStream_t s);
void launch_scene_center(const float* pos, int n, double* out, hipStream_t s);

// ---- launchers (loss.hip)
void launch_loss_maps(const float* img, const float* tgt, int W, int H, float lambda, bool fp32, float* coef,
                      float* dL, float* hd, double* part, int* nparts, hipStream_t s);
void launch_loss_reduce(const double* part, int nparts, int W, int H, double* out, hipStream_t s);

// ---- launchers (backward.hip)
void launch_raster_bwd(const gsn_frame& f, const float* dL, const float* hd, bool gauss_newton,
                       unsigned long long* counts, bool steps, hipStream_t s);
// Rows of the blocks summed over the views: 0..28 (position, rotation, scaling, opacity), then the
// overlap numerator (row kSumOverlap of a frame's sumrows, row GSN_BLK_BASE + GSN_BLK_VIEW V of the blocks).
constexpr int kSumOverlap = 29;
struct SumViews {
    int count;
    const float* rows[9];
    const uint8_t* contrib[9];
};
// adds the views' shares (sumrows of each frame, in the order given) to the blocks
void launch_sum_views(const gsn_blocks& b, const SumViews& sv, hipStream_t s);
// per-kernel sums of a view's (tile, kernel) partials (a secondary slot reads the primary coverage row,
// the primary's writes it)
void launch_reduce_pairs(const gsn_frame& f, const gsn_gaussians& g, int slot, bool fp32, const gsn_blocks& b,
                         hipStream_t s);
// the chain rule from those sums into the blocks (adds to the rows summed over the views)
void launch_chain(const gsn_frame& f, const gsn_gaussians& g, float weight, int slot, bool gauss_newton, bool fp32,
                  const gsn_blocks& b, float* zstats_out, hipStream_t s);

// ---- launchers (solve.hip)
// nonfinite: device counter of kernels skipped for non-finite blocks or steps (always counted);
// prof: the profile counters (solve events, GSN_COUNT_SOLVE_*), or NULL when not profiling
// The update a solve launch applies as it goes (mask 0: none; else the parameter groups of mask, as
// gsn_apply_step with no scales).
struct ApplyTo {
    float* pos = nullptr;
    float* rot = nullptr;
    float* scale = nullptr;
    float* opac = nullptr;
    float* sh = nullptr;
    uint32_t mask = 0;
};
void launch_solve(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                  const gsn_solve_opts& o, const gsn_steps& st, unsigned long long* nonfinite,
                  unsigned long long* prof, const ApplyTo& ap, hipStream_t s);
void launch_apply(const gsn_gaussians& g, const gsn_steps& st, const gsn_solve_opts& o, const float* scale,
                  uint32_t mask, unsigned long long* prof, hipStream_t s);
void launch_first_order(const gsn_gaussians& g, const gsn_blocks& b, const gsn_first_order_opts& fo, float c1,
                        float c2, float scale_floor, float opac_eps, float* state, uint32_t mask, hipStream_t s);
// One scene of a batched solve (device-side table entry).
#define GSN_SOLVE_MAX_SCENES 64
#define GSN_SOLVE_MAX_BLOCK 256
struct SolveScene {
    const float *pos, *rot, *scale, *opac;
    int n, K, V;
    DevCam cam;
    float kappa;
    const float* blk;
    gsn_solve_opts o;
    float* st;
    int32_t* fl;
    long long first;  // index of the scene's first kernel in the concatenated index space
};
void launch_solve_batched(const SolveScene* d_scenes, int count, long long total, int max_views, int block,
                          int grid, unsigned long long* nonfinite, hipStream_t s);
// the view slots a solve with options o takes of blocks with V slots
int solve_view_slots(int V, const gsn_solve_opts& o);
void launch_sh_gram(const float* blk, int n, int K, int V, float* gram, hipStream_t s);
// Devices whose no-allocation scratch address is cached.
#define GSN_MAX_DEVICES 64
// Device address of the fixed scratch array of gsn_local_newton_solve_noalloc on `device`
// (looked up once per device with hipGetSymbolAddress, then cached).
hipError_t solve_scratch_address(int device, float** out);
void launch_solve_mixed(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                        const gsn_solve_opts& o, const float* gram, const gsn_steps& st, unsigned long long* nonfinite,
                        unsigned long long* prof, const ApplyTo& ap, hipStream_t s);
void launch_features(const gsn_gaussians& g, const DevCam& cam, float kappa, const gsn_blocks& b,
                     const gsn_solve_opts& o, const float* resid, float* feat, uint8_t* ok, hipStream_t s);
void launch_neighbour_residual(const gsn_blocks& b, float* resid, hipStream_t s);
int label_blocks(int n);
// words (double) of the label and training scratch: the per-block partials and their slice sums
size_t label_part_words(int n);
size_t mlp_stat_words(int n);
// part: double [2][label_blocks(n)] scratch, used when alpha and err are given (err[0..1] +=)
void launch_labels(int n, int K, const float* sp, const int32_t* fp, const float* sa, const uint8_t* ok,
                   const float* alpha, float* label, float* mask, double* part, double* err, hipStream_t s);
void launch_mlp_infer(const uint16_t* wh, int n, const float* feat, const uint8_t* ok, float* out,
                      uint32_t* n_out_of_range, hipStream_t s);
int mlp_grad_blocks(int n);
void launch_mlp_train(gsn_mlp& mlp, int n, const float* feat, const float* label, const float* mask, float* part,
                      double* stat, const gsn_adam_opts& a, float* grad_out, double* loss, hipStream_t s);
void launch_mlp_reset(gsn_mlp& mlp, hipStream_t s);
