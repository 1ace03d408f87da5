/*
 * gsn.h -- C ABI of the MI355X (gfx950) stochastic local-Newton 3DGS step.
 *
 * Method: "3DGS^2: Near Second-order Converging 3D Gaussian Splatting"
 * (arxiv 2501.13975).  For one training image the library renders the image
 * from the Gaussian kernels (Sec. 3, eq. 3dgs), assembles each kernel's
 * gradient and small Hessian blocks of the image loss per attribute group
 * (Sec. 4.2, eq. local_hessian_gradient), adds the same blocks from the
 * secondary targets (Sec. 4.3, eq. tildel), solves the per-kernel local
 * Newton systems (eq. local_newton) and applies the steps.
 *
 * Conventions shared by every call
 *  - Pointers named d_* are DEVICE pointers on the context's device, owned by
 *    the caller; the library never frees them.  Host pointers are named h_*.
 *  - Arrays are structure-of-arrays, row per field: a "[F][N]" array holds
 *    field f of kernel k at index f * N + k.  float is IEEE binary32.
 *  - Every call is asynchronous on the context's HIP stream and returns a
 *    gsn_status; results are valid after the stream is synchronised.
 *    gsn_render synchronises the stream once to learn the number of (tile,
 *    kernel) pairs it must sort, unless the frame has a reserved pair
 *    capacity (gsn_frame_reserve): then the count stays on the device and the
 *    call never waits, so that a whole sweep can be captured in a HIP graph.
 *  - Numeric issues do not fail a call: kernels with a non-finite attribute are
 *    culled by gsn_render, kernels whose blocks or steps are not finite are
 *    skipped by the solve (zero step), and both are counted; gsn_sync_status
 *    reports them (GSN_E_NUMERIC) together with pair-capacity overflows.
 *  - Invalid arguments are reported before any work is launched
 *    (GSN_E_INVALID, GSN_E_SHAPE); gsn_last_error() gives a message.
 *  - A context is used from one host thread at a time.
 */
#ifndef GSN_H
#define GSN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GSN_OK = 0,
    GSN_E_INVALID = -1,  /* null pointer, bad option value, unknown handle */
    GSN_E_SHAPE = -2,    /* sizes inconsistent with each other or with the frame */
    GSN_E_CAPACITY = -3, /* a size exceeds what the call supports */
    GSN_E_HIP = -4,      /* a HIP runtime call failed (message has the HIP error) */
    GSN_E_NOMEM = -5,    /* device allocation of internal scratch failed */
    GSN_E_NUMERIC = -6   /* NaN or Inf met since the last gsn_sync_status: the affected kernels were
                            skipped, not updated (returned by gsn_sync_status only) */
} gsn_status;

typedef struct gsn_ctx gsn_ctx;
typedef struct gsn_frame gsn_frame;

/* Gaussian kernels (Sec. 3): position p, unit quaternion q = (w, x, y, z),
 * linear scale s > 0, opacity sigma in (0, 1), SH colour coefficients.
 * d_pos [3][n], d_rot [4][n], d_scale [3][n], d_opac [n],
 * d_sh [3][K][n] with K = (sh_degree + 1)^2, sh_degree in 0..3. */
typedef struct {
    float *d_pos, *d_rot, *d_scale, *d_opac, *d_sh;
    int32_t n;
    int32_t sh_degree;
} gsn_gaussians;

/* Pinhole camera, world -> camera rigid transform with OpenCV axes
 * (x right, y down, z forward); pixel centres at integer coordinates.
 * R is row-major. */
typedef struct {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
    float znear;
} gsn_camera;

/* Rasteriser options.  tile must be 16.  alpha = min(alpha_max, sigma G);
 * splats with alpha < alpha_min are skipped; a pixel stops before its
 * transmittance would drop below T_min; kappa is added to the diagonal of the
 * 2D covariance; a splat covers the tiles within radius_sigma standard
 * deviations of its major axis; bg is the background colour. */
typedef struct {
    int32_t tile;
    float alpha_min, alpha_max, T_min, kappa, radius_sigma;
    float bg[3];
    /* 0: the colour sums along each ray in double (the backward pass takes the colour behind each
     * splat as the final minus the partial colour); 1: single precision (no double image is kept;
     * that difference then loses enough to move position and rotation steps by ~1e-4 relative). */
    int32_t precision;
} gsn_render_opts;

/* Loss options (Sec. 4.2): L = L2 + lambda_ssim * L_S, with an 11x11 Gaussian
 * SSIM window (sigma 1.5).  weight multiplies this view's gradient and
 * Hessian before they are added to the blocks (1 for every target, Sec. 4.3).
 * gauss_newton nonzero: local Gauss-Newton blocks, H = sum over pixels and
 * channels of h dc/dy dc/dy^T; the terms of eq. local_hessian_gradient that
 * multiply the loss gradient by second derivatives of the image (through the
 * splat's alpha and through the projection) are left out, as the paper's
 * discussion of the position-Hessian cost suggests (Sec. 6).  Gradients, the
 * opacity and colour blocks (the image is linear in both) are unchanged;
 * the other blocks are positive semidefinite wherever h >= 0. */
typedef struct {
    float lambda_ssim;
    float weight;
    int32_t keep_zstats; /* nonzero: keep this view's per-kernel projected-space
                            statistics in the frame for gsn_frame_zstats */
    int32_t gauss_newton;
    /* 0: SSIM window sums and correlations, the per-kernel sums of the statistics and the rotation
     * and scale chain rule in double; 1: mixed form, all of these in single precision.  The SSIM
     * quotient-rule coefficients and the loss value are computed in double in both forms. */
    int32_t precision;
} gsn_loss_opts;

/* Solve options.  Damping: Cholesky of H + mu_j I, mu_j = mu0 10^j for
 * j = 0..max_escalations with mu0 = damp_rel * |H|_F / sqrt(n) +
 * damp_abs / (3 |I|); accepted when every pivot exceeds
 * pivot_min (|H|_F / sqrt(n) + mu_j) and min/max pivot >= pivot_min;
 * otherwise the scaled gradient step.  Steps are
 * then clamped to trust radii: |Delta p| <= trust_pos * max(s),
 * |theta| <= trust_rot, |Delta s| <= trust_scale * |s|, per colour channel
 * |Delta c| <= trust_sh (Euclidean norm of the SH coefficient step), and the
 * applied opacity is kept in [opac_eps, 1 - opac_eps].  Before the trust radii
 * every step is multiplied by step_frac (1 is the paper's unit Newton step).  The small systems are
 * solved in double precision.
 * Opacity barrier weight alpha_sigma = barrier_beta / (3 |I|), |I| =
 * npix_primary.  sh_floor: per-view colour curvature floor relative to the
 * largest.  scale_floor: s_new >= scale_floor * s.  opac_ftb:
 * fraction-to-boundary factor of the opacity update.  kappa: the 2D
 * covariance dilation the primary target was rendered with (the scaling
 * solve differentiates that covariance's eigenvalues). */
typedef struct {
    float damp_rel, damp_abs, pivot_min;
    int32_t max_escalations;
    float barrier_beta, sh_floor, scale_floor, opac_ftb;
    int32_t npix_primary;
    float kappa;
    float trust_pos, trust_rot, trust_scale, trust_sh, opac_eps, step_frac;
    float damp_sh;  /* colour damping relative to the mean diagonal of the colour Gram matrix */
    /* 0: plain form (reduced systems and solves in FP64); 1: mixed form (n_views <= 4):
     * colour Gram matrices from BF16 matrix-core products with one BF16 correction of the
     * basis rounding and FP32 accumulation, reduced systems and solves in FP32, and FP64
     * again for position or rotation systems whose pivots pass their tests by less than a
     * factor of 10 (counted as GSN_COUNT_FP64_SOLVES while profiling). */
    int32_t precision;
    /* 0: every kernel takes the paper's Newton step (times step_frac).  1: each kernel's steps,
     * after the trust radii, are multiplied by its overlap share omega = sum (alpha T)^2 / sum
     * alpha T over its pixels in all views of the blocks (in (0, 1]; 1 for a kernel alone on its
     * pixels).  The steps of all
     * kernels are taken at once, each computed with the others held fixed (the blocks are the
     * diagonal of the full Hessian); where kernels overlap, their steps add up in the shared pixels
     * and overshoot.  omega is at most the Gershgorin ratio H_kk / sum_j |H_kj| of the colour system
     * (sum_j alpha_j T_j = 1 - T_final <= 1 at every pixel), which bounds that overshoot. */
    int32_t overlap_scale;
    /* 0: the colour solve and the overlap share take every view slot of the blocks; k > 0: only the
     * first k (with k = 1, the primary-only step of a sweep whose secondary views are already in the
     * blocks' slots but whose shares of the summed rows are not yet added, gsn_add_view_shares). */
    int32_t view_limit;
} gsn_solve_opts;

/* Per-kernel gradient/Hessian blocks, summed over the views added so far.
 * d_data is a device array of gsn_blocks_floats(n, n_views) floats laid out
 * [GSN_BLK_BASE + GSN_BLK_VIEW * n_views + 1][n]:
 *   rows 0..2 g_p, 3..8 H_p (xx xy xz yy yz zz); rows 9..11 g_omega and 12..17
 *   H_omega for the rotation, parametrised by the left rotation vector omega
 *   (q <- exp(omega/2) q, so the paper's rotation angle about r_k is omega =
 *   theta r_k); 18..20 g_s, 21..26 H_s; 27 g_sigma, 28 H_sigma; 29 coverage of
 *   the primary target (sum of alpha T); then per view slot v at 30 + 10 v:
 *   gamma (dL/dc~, 3), s (sum h (alpha T)^2, 3), view direction r (3),
 *   coverage (1); and last, row 30 + 10 n_views: the sum over the views added
 *   of sum (alpha T)^2 over the kernel's pixels (with the view coverages, the
 *   kernel's overlap share, gsn_solve_opts.overlap_scale). */
#define GSN_BLK_BASE 30
#define GSN_BLK_VIEW 10
typedef struct {
    float* d_data;
    int32_t n;
    int32_t n_views;
} gsn_blocks;

/* Newton steps, d_data [GSN_STEP_BASE + 3K][n]: rows 0..2 Delta p, 3 theta
 * (rotation angle about the axis), 4..6 rotation axis r_k, 7..9 Delta s,
 * 10 Delta sigma, 11.. Delta SH [3][K].  d_flags [5][n] int32: escalation
 * index per group (position, rotation, scaling, opacity), -1 for the
 * gradient fallback, -2 when the kernel is not seen by the primary target
 * (no step), -3 when a block entry or step component was not finite (no
 * step); row 4 holds the number of views the colour solve used. */
#define GSN_STEP_BASE 11
typedef struct {
    float* d_data;
    int32_t* d_flags;
    int32_t n;
    int32_t sh_degree;
} gsn_steps;

/* ---------------------------------------------------------------- context */

/* Creates a context on HIP device `device` issuing work on `hip_stream`
 * (a hipStream_t; NULL means the null stream).  *out receives the handle. */
gsn_status gsn_create(gsn_ctx** out, int32_t device, void* hip_stream);
/* Frees the context and all frames and scratch it owns.  NULL is a no-op. */
gsn_status gsn_destroy(gsn_ctx* ctx);
/* Message of the last failed call on this context ("" if none).  Owned by the context. */
const char* gsn_last_error(const gsn_ctx* ctx);
/* Switches the stream used by later calls. */
gsn_status gsn_set_stream(gsn_ctx* ctx, void* hip_stream);

/* A frame holds one rendered view: projected kernels, the depth-ordered
 * per-tile lists, the image and per-pixel compositing state that
 * gsn_accumulate_hessian needs.  Owned by the context. */
gsn_status gsn_frame_create(gsn_ctx* ctx, gsn_frame** out);
gsn_status gsn_frame_destroy(gsn_ctx* ctx, gsn_frame* frame);

/* --------------------------------------------------------------- the step */

/* Renders the image of `g` seen by `cam` (Sec. 3, eq. 3dgs) into `frame`:
 * projection of every kernel (EWA 2D covariance, view-dependent SH colour,
 * Appendix A.1-A.3), binning into 16x16 tiles, a global depth sort and a
 * stable partition by tile, and front-to-back alpha compositing per pixel.
 * The tile rectangles and depth keys are computed in single precision with
 * a fixed operation order and no contraction.  d_rgb_out [3][H][W] and
 * d_T_out [H][W] receive copies of the image and final transmittance when
 * not NULL (opts->precision selects the colour sums' precision for this frame and
 * its gsn_accumulate_hessian).  Kernels with a NaN or infinite attribute, or whose colour in this
 * view is not finite, are culled (not drawn) and counted (GSN_STAT_CULLED_NONFINITE).
 * A frame in reserved mode (gsn_frame_reserve) is rendered without any allocation
 * or host wait.  Errors: GSN_E_INVALID (null handle or arrays, tile != 16,
 * sh_degree outside 0..3, precision not 0 or 1), GSN_E_SHAPE (n < 0, image size <= 0),
 * GSN_E_CAPACITY (reserved frame smaller than n or the image). */
gsn_status gsn_render(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* cam,
                      const gsn_render_opts* opts, gsn_frame* frame, float* d_rgb_out,
                      float* d_T_out);

/* Adds to `blocks` the gradient and Hessian blocks of the loss of the image
 * in `frame` against d_target [3][H][W] (Sec. 4.2, eq. local_hessian_gradient
 * with the per-pixel diagonal image Hessian of L2 + lambda SSIM), for every
 * kernel and attribute group, and writes this view's colour statistics into
 * view slot `view_slot` (0 = primary target, 1.. = secondary targets, Sec.
 * 4.3).  `g` must be the kernels the frame was rendered from.  Slot 0 also
 * sets the primary coverage row; accumulate slot 0 first in a sweep: the
 * secondary slots add blocks only for kernels the primary covers (the only
 * kernels a sweep updates), the others keep what gsn_blocks_zero left.  d_loss_out (device double[2], may be NULL)
 * receives (L2, L_S) of this view.  Blocks are accumulated with a fixed
 * reduction order (no atomics), so results are deterministic.
 * Errors: GSN_E_SHAPE (n differs from the frame's, view_slot outside
 * 0..n_views-1), GSN_E_INVALID (frame never rendered, null pointers). */
gsn_status gsn_accumulate_hessian(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_frame* frame,
                                  const float* d_target, const gsn_loss_opts* opts,
                                  int32_t view_slot, gsn_blocks* blocks, double* d_loss_out);

/* The views of one sweep (Sec. 4.3: the primary target and its secondary targets) rendered and
 * accumulated together: for i = 0..n_views-1, gsn_render of cams[i] into frames[i] followed by
 * gsn_accumulate_hessian of d_targets[i] into slot first_slot + i, with results identical bit
 * for bit to those calls made one after another.  The views take in turn the context's stream and
 * three streams of the library's own (default priority), forked from the context's stream and
 * joined back into it before the call returns, so that a view's projection, sort, rasters and loss
 * maps overlap the others'; each view's shares of the rows summed over the views are kept in its
 * frame and added to the blocks after the join, in view order (the blocks equal those of the calls
 * made one after another, bit for bit), and a secondary slot's per-kernel sums wait for the
 * primary's coverage row when slot 0 is among the views.  With the profiler on (gsn_profile_enable) the views run one after another
 * on the context's stream.  The frames must be distinct; reserved frames (gsn_frame_reserve)
 * keep the call free of host waits and let it be captured (gsn_capture_begin).
 * cams [n_views], frames [n_views], d_targets [n_views] (device [3][H][W] each, at each camera's
 * size) are caller-owned; d_loss_out (device double [n_views][2], may be NULL) receives (L2, L_S)
 * per view.  add_shares = 0 leaves the views' shares of the rows summed over the views in the
 * frames, for gsn_add_view_shares (the slot rows and the primary's coverage row are written in both
 * cases).  Errors: those of gsn_render and gsn_accumulate_hessian (part of the other views'
 * work may have been issued; the blocks are then incomplete), GSN_E_SHAPE (n_views < 1 or above 9, slots outside the blocks'
 * 0..n_views-1), GSN_E_INVALID (null arrays or entries, a frame given twice), GSN_E_HIP. */
gsn_status gsn_accumulate_views(gsn_ctx* ctx, const gsn_gaussians* g, int32_t n_views, int32_t first_slot,
                                const gsn_camera* cams, gsn_frame* const* frames,
                                const float* const* d_targets, const gsn_render_opts* ropts,
                                const gsn_loss_opts* lopts, gsn_blocks* blocks, double* d_loss_out,
                                int32_t add_shares);

/* The views' shares of the rows summed over the views (position, rotation, scaling, opacity and the
 * overlap numerator; each frame keeps its view's shares from its accumulation) added to `blocks` in
 * the order of frames[]: with gsn_accumulate_views(..., add_shares = 0) a caller adds the primary's
 * share, solves the primary-only step (gsn_solve_opts.view_limit = 1), then adds the secondaries'
 * (the learned form's full-rule sweep, Sec. 4.3), with the blocks of one gsn_accumulate_views call
 * at the end.  frames [n_views] must hold views accumulated into these blocks since they were last
 * rendered.  Errors: GSN_E_INVALID (null handles, a frame with no accumulated view of this size),
 * GSN_E_SHAPE (n_views outside 0..9). */
gsn_status gsn_add_view_shares(gsn_ctx* ctx, gsn_blocks* blocks, int32_t n_views, gsn_frame* const* frames);

/* Solves every kernel's local Newton systems (eq. local_newton) in the
 * paper's reduced coordinates relative to the primary camera: position in
 * the plane normal to the view direction r_k, rotation angle about r_k,
 * scale in the row space of d(lambda)/ds (eigenvalues of the primary 2D
 * covariance), opacity with a log barrier, SH colour per channel from the
 * per-view statistics (Sec. 4.2, Position/Scaling/Rotation/Opacity/Color
 * solve).  Kernels the primary target does not see get no step (decisions -2); kernels with a
 * non-finite step component, or a non-finite block entry among those their solve reads, get a
 * zero step (decisions -3) and are counted (GSN_STAT_SKIPPED_NONFINITE).
 * Errors: GSN_E_SHAPE (blocks.n or steps.n != g->n, sh_degree mismatch). */
gsn_status gsn_local_newton_solve(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                                  const gsn_blocks* blocks, const gsn_solve_opts* opts,
                                  gsn_steps* steps);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc): gsn_local_newton_solve with the same arguments and
 * results, and no allocation of any kind.  Its only scratch, the mixed form's colour Gram
 * matrices (10 floats per kernel, precision = 1), lives in a fixed array of
 * 10 * GSN_NOALLOC_MAX_N floats (40 MiB) that every device holds from the library's load until
 * the process ends; the plain form uses none.  All calls on one device share that array, so calls
 * that overlap on one device (other streams or contexts) race; calls on one stream are ordered.
 * Nothing is timed by gsn_profile_enable.  Errors: as gsn_local_newton_solve, and GSN_E_CAPACITY
 * when n > GSN_NOALLOC_MAX_N. */
#define GSN_NOALLOC_MAX_N (1 << 20)
gsn_status gsn_local_newton_solve_noalloc(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                                          const gsn_blocks* blocks, const gsn_solve_opts* opts,
                                          gsn_steps* steps);

/* Applies the steps in place, for the groups in group_mask (bit 0 position,
 * 1 rotation, 2 scaling, 3 opacity, 4 colour): p += Delta p; q <- dq(theta) q
 * renormalised with dq = (cos(theta/2), sin(theta/2) r_k); s <- max(s + Delta s,
 * scale_floor s); sigma <- sigma + Delta sigma clipped to the fraction
 * opac_ftb of the way to 0 or 1; SH += Delta SH (Sec. 4.2).
 * d_scale: NULL, or device float [5][n] multiplying each kernel's step of each
 * group (position, rotation, scaling, opacity, colour) before it is applied
 * (the learned step scale, see gsn_mlp_infer).
 * Errors: GSN_E_SHAPE (steps.n != g->n). */
gsn_status gsn_apply_step(gsn_ctx* ctx, gsn_gaussians* g, const gsn_steps* steps,
                          const gsn_solve_opts* opts, const float* d_scale, uint32_t group_mask);

/* gsn_local_newton_solve followed by gsn_apply_step(g, steps, opts, NULL, group_mask) in one
 * launch: the thread that solves a kernel applies its step at once (a sweep's solve and update,
 * Sec. 4.2), so the parameters are read and written in the same pass.  steps receive the solved
 * steps and decisions as with gsn_local_newton_solve; g's parameters end as after the two calls,
 * bit for bit.  Errors: as gsn_local_newton_solve, and GSN_E_INVALID for group_mask bits above 4. */
gsn_status gsn_solve_apply(gsn_ctx* ctx, gsn_gaussians* g, const gsn_camera* primary,
                           const gsn_blocks* blocks, const gsn_solve_opts* opts, gsn_steps* steps,
                           uint32_t group_mask);

/* First-order baseline on the same gradients (the comparison behind the paper's
 * claims of fewer iterations than first-order training, Sec. 1 and Sec. 5).
 * lr: learning rates of the groups position, rotation (left rotation vector,
 * radians), scaling (linear scale), opacity, colour (SH coefficients).
 * adam = 0: gradient descent x <- x - lr g.  adam = 1: Adam (Kingma and Ba,
 * 2015) with moments beta1, beta2, eps and bias corrections for step count
 * step >= 1. */
typedef struct {
    float lr[5];
    float beta1, beta2, eps;
    int32_t adam;
    int32_t step;
} gsn_first_order_opts;

/* One first-order step for every kernel the primary view sees (blocks row 29 >
 * 0), from the gradients in `blocks` (the SH gradient of channel ch is the sum
 * over view slots of gamma_ch Y(r), with the basis of Sec. 4.2's colour
 * paragraph), for the groups in group_mask (bits as gsn_apply_step).  Updates
 * as gsn_apply_step: q <- exp(omega/2) q renormalised for the rotation step
 * omega = -lr u; s <- max(s - lr u, scale_floor s); sigma clipped to
 * [opac_eps, 1 - opac_eps] (scale_floor and opac_eps from `opts`).
 * d_state: device float [2][10 + 3K][n] (first then second moments; entries
 * per kernel position 3, omega 3, scale 3, opacity 1, colour [3][K]), owned by
 * the caller and zeroed by it before step 1; may be NULL when adam = 0.
 * Errors: GSN_E_SHAPE (blocks.n != g->n), GSN_E_INVALID (null state with
 * adam = 1, step < 1, negative learning rate, beta outside [0, 1)). */
gsn_status gsn_first_order_step(gsn_ctx* ctx, gsn_gaussians* g, const gsn_blocks* blocks,
                                const gsn_solve_opts* opts, const gsn_first_order_opts* fo, float* d_state,
                                uint32_t group_mask);

/* The colour Gram matrices of the mixed form: for every kernel, B B^T over the
 * views that see it (coverage > 0, at most 4, in slot order), B the rows of the
 * SH basis Y(r_v) (Appendix A.2), from BF16 matrix-core products with FP32
 * accumulation; upper triangle written to d_out (device float [10][n], entry
 * (i, j), i <= j, at row 4 i - i (i - 1) / 2 + j - i).  Errors: GSN_E_SHAPE
 * (n_views > 4). */
gsn_status gsn_sh_gram(gsn_ctx* ctx, const gsn_blocks* blocks, int32_t sh_degree, float* d_out);

/* ------------------------------------------------- batched solve
 * The local Newton solves of several scenes (Sec. 4.2, eq. local_newton) in
 * one persistent launch: a grid sized to the device walks the concatenated
 * kernel index space of all scenes, every kernel solving all of its groups
 * (sizes 1, 2 reduced, 3 and the per-channel colour systems) exactly as
 * gsn_local_newton_solve does, so the results are identical to per-scene
 * calls (plain form: opts.precision must be 0).  Each item's pointers are
 * borrowed for the call (the graph form below keeps them). */
typedef struct {
    const gsn_gaussians* g;
    const gsn_camera* primary;
    const gsn_blocks* blocks;
    const gsn_solve_opts* opts;
    gsn_steps* steps;
} gsn_solve_item;
/* Errors: GSN_E_INVALID (count < 1 or > 64, null pointers), GSN_E_SHAPE and
 * GSN_E_CAPACITY as for gsn_local_newton_solve, per item. */
gsn_status gsn_solve_batched(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count);
/* Launch-shape autotuner of the batched solve: times block sizes {64, 128,
 * 256} and grids of {1, 2, 4, 8, 16} workgroups per compute unit or one thread
 * per kernel on the
 * given items (the solves run, and rerun, on the real buffers), keeps the
 * fastest for later gsn_solve_batched and graph calls on this context and
 * returns it (h_block, h_grid may be NULL).  Synchronises the stream. */
gsn_status gsn_solve_tune(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count, int32_t* h_block,
                          int32_t* h_grid);
/* A HIP graph holding one batched solve of the given items: the scene table is
 * copied to device memory owned by the graph and the launch is captured on a
 * stream of the library's own; gsn_graph_launch replays it on the context's
 * stream (the items' buffers must stay valid and keep their sizes). */
typedef struct gsn_graph gsn_graph;
gsn_status gsn_solve_graph_create(gsn_ctx* ctx, const gsn_solve_item* items, int32_t count, gsn_graph** out);
gsn_status gsn_graph_launch(gsn_ctx* ctx, gsn_graph* graph);
gsn_status gsn_graph_destroy(gsn_ctx* ctx, gsn_graph* graph);
/* Records the calls made on the context between gsn_capture_begin and gsn_capture_end into a HIP
 * graph instead of running them (a whole sweep: gsn_blocks_zero, the renders and accumulations of
 * its views, the solve and the apply), so that gsn_graph_launch replays them with one launch and
 * no host work.  The recorded calls keep their arguments: device buffers, cameras and options are those of the
 * capture, and every buffer must keep its size.  Frames rendered under capture must be reserved
 * (gsn_frame_reserve) and every buffer the calls use must already have its size (run the same
 * calls once before capturing); a call that would allocate or wait fails, and gsn_capture_end then
 * returns an error and no graph.  Calls that read results back to the host (gsn_profile_read,
 * gsn_sync_status, frame introspection) are refused while capturing.  begin synchronises the
 * context's stream; the graph is replayed on the context's stream.  Replays are stage-timed as a
 * whole only (not per stage).  Errors: GSN_E_INVALID (already / not capturing, a call failed
 * under capture), GSN_E_HIP. */
gsn_status gsn_capture_begin(gsn_ctx* ctx);
gsn_status gsn_capture_end(gsn_ctx* ctx, gsn_graph** out);

/* ------------------------------------------------- learned step scale
 * The overshoot control of Sec. 4.3 (eq. tildel) adds the blocks of the
 * |N_t| nearest training views to the primary's.  The learned form predicts,
 * per kernel and group, the scale alpha that the full rule applies along the
 * primary-only step, so that most sweeps render only the primary view:
 *   features (gsn_step_features) from the primary view's blocks alone,
 *   network 17 -> 32 (ReLU) -> 5, alpha = 1.5 sigmoid(.) (gsn_mlp_infer),
 *   labels alpha_eff = <Delta_aug, Delta_prim> / |Delta_prim|^2 clipped to
 *   [0, 1.5] from a sweep that runs the full rule (gsn_step_labels),
 *   training by mean squared error and Adam (gsn_mlp_train_step). */
#define GSN_MLP_IN 17
#define GSN_MLP_HID 32
#define GSN_MLP_OUT 5
#define GSN_MLP_PARAMS 741
/* Network state, device buffers owned by the caller: d_params float [741]
 * master weights laid out W1 [32][17] row-major, b1 [32], W2 [5][32]
 * row-major, b2 [5]; d_m, d_v float [741] Adam moments; d_half fp16 [741]
 * inference copy; step: Adam steps taken (advanced by gsn_mlp_train_step). */
typedef struct {
    float* d_params;
    float* d_m;
    float* d_v;
    uint16_t* d_half;
    int32_t step;
} gsn_mlp;
typedef struct {
    float lr, beta1, beta2, eps;
} gsn_adam_opts;

/* Feature status of a kernel (gsn_step_features, d_ok). */
#define GSN_FEAT_HIDDEN 0        /* not seen by the primary target: no step */
#define GSN_FEAT_OK 1            /* features in range: the network's scale applies */
#define GSN_FEAT_OUT_OF_RANGE 2  /* seen, but a feature left [-3, 3]: the network is not trusted and the
                                    kernel needs the full overshoot rule (gsn_mlp_infer counts it) */
/* Features of every kernel (device float [17][n], layout feature-major) from
 * blocks holding only the primary view (slot 0), in the reduced coordinates of
 * gsn_local_newton_solve, and the residual the neighbouring views left at the
 * kernel.  With L(x) = log10(x + 1e-30) / 10 clipped to [-3, 3]:
 * 0, 1 L(|lambda|) of the reduced position Hessian's larger / smaller
 * eigenvalue; 2 sign of the smaller; 3, 4 L(|H_theta|), sign; 5, 6, 7 the same
 * for the reduced scaling Hessian; 8 L(|H_sigma + h_B|); 9 L(sum of |s| of the
 * primary's colour Hessian diagonal); 10 L(primary coverage); 11-14 L(|g|) of
 * the reduced position, rotation, scaling and opacity gradients; 15 L(opacity);
 * 16 L(d_resid[k]), the neighbouring-view residual cached by
 * gsn_neighbour_residual (d_resid may be NULL: 0).
 * d_ok (device u8 [n]) receives GSN_FEAT_HIDDEN, GSN_FEAT_OK or GSN_FEAT_OUT_OF_RANGE.
 * Errors: GSN_E_SHAPE. */
gsn_status gsn_step_features(gsn_ctx* ctx, const gsn_gaussians* g, const gsn_camera* primary,
                             const gsn_blocks* blocks, const gsn_solve_opts* opts, const float* d_resid,
                             float* d_feat, uint8_t* d_ok);
/* The residual the neighbouring views (the secondary targets of Sec. 4.3) leave at each kernel,
 * from blocks that hold them (a sweep that runs the full rule): for every kernel the primary
 * sees and at least one secondary view covers, d_resid[k] = sum over the secondary slots v >= 1
 * that cover it of |gamma_v| / (|gamma_0| + 1e-30), gamma_v the view's colour gradient (3
 * channels, Euclidean norm); other kernels keep their value (the cache of their last visit).
 * d_resid: device float [n].  Errors: GSN_E_SHAPE (n_views < 2), GSN_E_INVALID. */
gsn_status gsn_neighbour_residual(gsn_ctx* ctx, const gsn_blocks* blocks, float* d_resid);
/* Labels from the primary-only steps (prim) and the full-rule steps (aug) of
 * the same sweep: d_label, d_mask device float [5][n]; the mask is 1 where the
 * solve stepped the kernel (decisions >= -1), its features were in range
 * (d_ok[k] == GSN_FEAT_OK; d_ok may be NULL) and |Delta_prim|^2 > 1e-30 for the group.
 * With d_alpha (the network's scales [5][n] for the same kernels, may be NULL) and
 * d_err (device double [2], may be NULL), d_err[0] += sum of mask |alpha - label|
 * and d_err[1] += sum of mask, summed in a fixed order (the error of the network
 * against the overshoot rule it replaces). */
gsn_status gsn_step_labels(gsn_ctx* ctx, const gsn_steps* prim, const gsn_steps* aug, const uint8_t* d_ok,
                           const float* d_alpha, float* d_label, float* d_mask, double* d_err);
/* Zeroes the Adam moments and the step count and refreshes the fp16 copy from
 * the master weights. */
gsn_status gsn_mlp_reset(gsn_ctx* ctx, gsn_mlp* mlp);
/* alpha (device float [5][n]) for every kernel from its features, with the
 * fp16 weights and FP32 accumulation; kernels whose d_ok[k] is not GSN_FEAT_OK
 * get 0.  d_out_of_range (device u32, may be NULL) += the number of kernels with
 * d_ok[k] == GSN_FEAT_OUT_OF_RANGE: a caller that finds it nonzero runs the full
 * overshoot rule for the sweep (the fallback of the learned form). */
gsn_status gsn_mlp_infer(gsn_ctx* ctx, const gsn_mlp* mlp, int32_t n, const float* d_feat,
                         const uint8_t* d_ok, float* d_alpha, uint32_t* d_out_of_range);
/* One Adam step on the mean squared error over the entries with mask 1
 * (features [17][n], labels and mask [5][n]); writes the loss before the step
 * to d_loss (device double, may be NULL) and the gradient to d_grad (device
 * float [741], may be NULL).  Gradient partials are summed in a fixed order:
 * results are deterministic.  Errors: GSN_E_INVALID (n < 0, null buffers). */
gsn_status gsn_mlp_train_step(gsn_ctx* ctx, gsn_mlp* mlp, int32_t n, const float* d_feat, const float* d_label,
                              const float* d_mask, const gsn_adam_opts* adam, double* d_loss, float* d_grad);

/* ---------------------------------------------------------------- helpers */

/* Number of floats of a blocks array for n kernels and n_views view slots:
 * (GSN_BLK_BASE + GSN_BLK_VIEW * n_views + 1) * n. */
int64_t gsn_blocks_floats(int32_t n, int32_t n_views);
/* Zeroes a blocks array (asynchronously, with a fill kernel). */
gsn_status gsn_blocks_zero(gsn_ctx* ctx, gsn_blocks* blocks);
/* Number of floats of a steps array for n kernels and SH degree. */
int64_t gsn_steps_floats(int32_t n, int32_t sh_degree);

/* Secondary targets are downsampled (Sec. 4.3): d_dst [3][H/2][W/2] is the
 * 2x2 box mean of d_src [3][H][W].  Errors: GSN_E_SHAPE (W or H < 2). */
gsn_status gsn_downsample2x(gsn_ctx* ctx, const float* d_src, int32_t width, int32_t height,
                            float* d_dst);

/* Camera of a secondary target (Sec. 4.3): the target is the 2x2 box mean of
 * the full-resolution image (gsn_downsample2x), so a half-resolution pixel
 * centre u' lies at the full-resolution coordinate 2 u' + 0.5.  On the host:
 * *out = *cam with fx/2, fy/2, cx' = (cx + 0.5)/2 - 0.5, cy' likewise (evaluated
 * in double from the float inputs, rounded to float), width/2, height/2
 * (rounded down).  out may equal cam.  Errors: GSN_E_INVALID (null pointers),
 * GSN_E_SHAPE (width or height < 2). */
gsn_status gsn_camera_half(const gsn_camera* cam, gsn_camera* out);

/* Centre of the scene for the camera KNN (Sec. 4.1): the mean of the kernel
 * positions, summed in double in a fixed order on the device (deterministic);
 * d_out: device double [3].  Errors: GSN_E_INVALID (null pointers), as
 * gsn_render for the kernels. */
gsn_status gsn_scene_center(gsn_ctx* ctx, const gsn_gaussians* g, double* d_out);

/* Camera KNN on the bounding sphere (Sec. 4.1), on the host: camera centres
 * h_centers [ncam][3] are projected radially onto a sphere about
 * h_scene_center and ranked by great-circle distance; h_out [ncam][k]
 * receives the k nearest other cameras (ties by lower index).
 * Errors: GSN_E_INVALID (k < 1 or k >= ncam). */
gsn_status gsn_camera_knn(const double* h_centers, int32_t ncam, const double* h_scene_center,
                          int32_t k, int32_t* h_out);

/* Frame introspection for tests and profiling (host values, synchronous on the
 * context's stream): number of (tile, kernel) pairs of the last render, and
 * copies of its per-tile ranges (uint32 [2][tiles]) and sorted kernel ids
 * (uint32 [pairs]) into device buffers.  Any pointer may be NULL. */
gsn_status gsn_frame_info(gsn_ctx* ctx, const gsn_frame* frame, int64_t* h_pairs, int32_t* h_tiles_x,
                          int32_t* h_tiles_y);
gsn_status gsn_frame_lists(gsn_ctx* ctx, const gsn_frame* frame, uint32_t* d_ranges, uint32_t* d_ids,
                           uint32_t* d_depth_bits, int32_t* d_rect, uint32_t* d_ncontrib);
/* Per-kernel projected-space statistics of the last gsn_accumulate_hessian on
 * this frame that ran with keep_zstats (float [48][n]), in each kernel's
 * principal frame (pi' = V^T pi, Q' = V^T Q V, V from gsn_frame_records):
 * gradient w.r.t. (pi'_1, pi'_2, Q'_11, Q'_12, Q'_22) (5), sigma (1), c~ (3);
 * Hessian block over (pi', Q') (15, upper triangle), its cross block with c~
 * (5 x 3), the c~ diagonal (3), the sigma-sigma entry (1) and the coverage
 * sum alpha T (1), then the sum of (alpha T)^2 (1) and 3 zeros. */
gsn_status gsn_frame_zstats(gsn_ctx* ctx, const gsn_frame* frame, float* d_out);
/* Copy of the projected kernels of the last render (float [12][n]): image
 * position, high word (2), conic in the principal frame q1 = 1/lambda1,
 * q2 = 1/lambda2 (2), principal axis (cos, sin) (2), opacity (1), view-dependent
 * colour (3), image position, low word (2): the position is the sum of the two
 * words (evaluated in double, kept as a float pair).
 * The per-kernel statistics of gsn_frame_zstats are expressed in this
 * principal frame. */
gsn_status gsn_frame_records(gsn_ctx* ctx, const gsn_frame* frame, float* d_out);
/* Copies of the per-pixel loss gradient dL/dc and diagonal Hessian d2L/dc2
 * ([3][H][W] floats each) of the last gsn_accumulate_hessian on this frame. */
gsn_status gsn_frame_loss_maps(gsn_ctx* ctx, const gsn_frame* frame, float* d_dL, float* d_h);

/* ------------------------------------------------- status without host waits
 * The calls of a sweep never wait for the device when every frame has a reserved capacity, so a
 * caller can queue (or capture in a HIP graph) many sweeps and check their outcome once.  What
 * the device met meanwhile is counted in the context and read by gsn_sync_status. */

/* Reserves a frame's device memory for views of at most width x height pixels with n kernels and at
 * most max_pairs (tile, kernel) pairs, and switches the frame to reserved mode: gsn_render then
 * allocates nothing and no longer reads the pair count back to the host.  A render whose pairs
 * exceed max_pairs draws no kernel (its image is the background, its lists are empty, and its
 * gsn_accumulate_hessian adds nothing), counts GSN_STAT_PAIR_OVERFLOW and records the pair count it
 * needed; reserve again with a larger max_pairs to render such views.  max_pairs = 0 returns the
 * frame to growing mode (the render sizes its buffers from the count it reads back).  Synchronises
 * the stream.  Errors: GSN_E_INVALID (null handles), GSN_E_SHAPE (n < 0, image size <= 0,
 * max_pairs < 0), GSN_E_CAPACITY (max_pairs >= 2^31), GSN_E_NOMEM. */
gsn_status gsn_frame_reserve(gsn_ctx* ctx, gsn_frame* frame, int32_t n, int32_t width, int32_t height,
                             int64_t max_pairs);

/* Counters of gsn_sync_status. */
typedef enum {
    GSN_STAT_CULLED_NONFINITE = 0,  /* kernels gsn_render culled (per render): a position, rotation, scale
                                       or opacity, or the view-dependent colour, was NaN or infinite */
    GSN_STAT_SKIPPED_NONFINITE = 1, /* kernels a solve skipped (zero step, decisions -3) because a block
                                       entry or a step component was NaN or infinite */
    GSN_STAT_PAIR_OVERFLOW = 2,     /* renders of reserved frames whose pairs exceeded the capacity */
    GSN_STAT_PAIRS_NEEDED = 3,      /* the largest pair count such a render needed */
    GSN_STAT_N = 4
} gsn_stat;

/* Synchronises the context's stream, copies the counters gathered since the last call (or since
 * gsn_create) into h_stats[GSN_STAT_N] (may be NULL) and clears them.  Returns GSN_E_CAPACITY when
 * a reserved render overflowed, else GSN_E_NUMERIC when a non-finite value was met (the kernels
 * concerned were culled or skipped, not updated), else GSN_OK; gsn_last_error describes it. */
gsn_status gsn_sync_status(gsn_ctx* ctx, int64_t* h_stats);

/* ------------------------------------------------------------ measurement */

/* Stages timed by the profiler. */
typedef enum {
    GSN_STAGE_PROJECT = 0,     /* per-kernel projection and binning decisions */
    GSN_STAGE_SORT = 1,        /* depth sort, pair emission, tile partition, ranges */
    GSN_STAGE_RASTER_FWD = 2,  /* forward compositing */
    GSN_STAGE_LOSS = 3,        /* loss value and per-pixel derivative maps */
    GSN_STAGE_RASTER_BWD = 4,  /* backward compositing and per-tile statistics */
    GSN_STAGE_CHAIN = 5,       /* per-kernel reduction and chain rule */
    GSN_STAGE_SOLVE = 6,       /* local Newton solves */
    GSN_STAGE_APPLY = 7,       /* parameter update */
    GSN_STAGE_COUNT = 8
} gsn_stage;

/* Work counters gathered while profiling. */
typedef enum {
    GSN_COUNT_FWD_EVALS = 0,   /* (pixel, list entry) evaluations in the forward pass */
    GSN_COUNT_BWD_EVALS = 1,   /* (pixel, list entry) evaluations in the backward pass */
    GSN_COUNT_BWD_ACTIVE = 2,  /* of which contributed (alpha >= alpha_min) */
    GSN_COUNT_PAIRS = 3,       /* (tile, kernel) pairs binned */
    GSN_COUNT_PARTIALS = 4,    /* (tile, kernel) partial statistics written by the backward pass */
    GSN_COUNT_FWD_STAGED = 5,  /* list entries the forward pass staged (read) before its tiles finished */
    GSN_COUNT_FP64_SOLVES = 6, /* kernels whose position or rotation system the mixed form re-solved in FP64 */
    GSN_COUNT_BWD_STAGED = 7,  /* list entries the backward pass staged (read): each tile's composited prefix */
    /* Solve decisions (gsn_local_newton_solve), per group g = 0 position, 1 rotation, 2 scaling,
     * 3 opacity: the damped system was accepted only after escalating mu (j > 0), or every attempt
     * failed and the scaled gradient step was taken (j = -1); and per g = 0 position, 1 rotation,
     * 2 scaling, 3 colour (any channel) the trust radius cut the step. */
    GSN_COUNT_SOLVE_ESCALATED = 8,  /* + g */
    GSN_COUNT_SOLVE_FALLBACK = 12,  /* + g */
    GSN_COUNT_SOLVE_CLAMPED = 16,   /* + g */
    GSN_COUNT_SOLVED = 20,          /* kernels solved (visible in the primary, finite blocks and steps) */
    GSN_COUNT_OPAC_BOUND = 21,      /* gsn_apply_step: opacity steps cut by the fraction-to-boundary rule
                                       or the bounds [opac_eps, 1 - opac_eps] */
    /* Wave steps of the raster passes' per-pixel loops (one per entry a wave's pixels visit
     * together): against the per-pixel counts above they give the share of lanes at work.
     * Counted only at profiling level 2 (gsn_profile_enable), whose raster passes take longer. */
    GSN_COUNT_FWD_WAVE_STEPS = 22,  /* forward: entries of the band lists the wave walked */
    GSN_COUNT_BWD_WAVE_STEPS = 23,  /* backward: composited entries the wave walked, and entries evaluated
                                       again past the recorded batches */
    /* Shader-clock cycles the backward raster's waves spent (level 2): + 0 staging the batch and its
     * composited-entry masks, + 1 the slot scan, + 2 the per-pixel walk, + 3 the per-entry sums. */
    GSN_COUNT_BWD_CYCLES = 24,
    GSN_COUNT_N = 28
} gsn_counter;

/* Turns stage timing on (on = 1, or 2 to count the raster passes' wave steps too) or off (0)
 * and clears what was accumulated.  While on, every stage is bracketed by HIP events on the
 * context's stream (a few microseconds of overhead per stage) and the raster passes count their
 * work. */
gsn_status gsn_profile_enable(gsn_ctx* ctx, int32_t on);
/* Synchronises the stream and returns, per stage, the summed event time in
 * milliseconds (h_ms[GSN_STAGE_COUNT]) and the number of timed launches
 * (h_launches[GSN_STAGE_COUNT]), and the work counters
 * (h_counts[GSN_COUNT_N]).  Any pointer may be NULL. */
gsn_status gsn_profile_read(gsn_ctx* ctx, double* h_ms, int64_t* h_launches, int64_t* h_counts);

#ifdef __cplusplus
}
#endif
#endif /* GSN_H */
