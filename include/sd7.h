/*
 * sd7.h -- C ABI of lib7dgs.so, the MI355X (gfx950) render path of 7D
 * Gaussian Splatting (7DGS).
 *
 * The path (Sec. 4.2 and Sec. 4.4 of the paper):
 *   sd7_slice        condition every 7D Gaussian (position, time, direction)
 *                    on the observed time t and view direction d: conditional
 *                    mean (eq. cond_mean), covariance (eq. cond_cov) and
 *                    opacity alpha_cond = alpha f_temp f_dir (eq. temp_mod,
 *                    eq. dir_mod); Algorithm 1 steps 3-6, with the adaptive
 *                    refinement of steps 1-2 taken as the identity ("w/o AGR").
 *   sd7_project      standard perspective (EWA) projection of each conditional
 *                    3D Gaussian to a 2D Gaussian, culling, footprint, depth,
 *                    and the degree-3 SH colour (Sec. 3, eq. 2; Sec. 4.1).
 *   sd7_bin          depth sort of the kept Gaussians, per-tile lists of
 *                    (tile, Gaussian) pairs in (depth, index) order.
 *   sd7_rasterize    depth-aware, opacity-blended front-to-back compositing
 *                    of each 16x16 pixel tile (Sec. 4.4).
 *   sd7_rasterize_backward, sd7_project_backward, sd7_slice_backward
 *                    the reverse pass of the three compute stages
 *                    (differentiable rasterization, Sec. 4.4).
 *
 * Constants the paper leaves open, fixed here: tiles of 16x16 pixels;
 * alpha = min(0.99, alpha_cond exp(-q/2)); a Gaussian is skipped at a pixel
 * when alpha < 1/255 (FP32 value); compositing stops before the Gaussian
 * that would bring transmittance below 1e-4; near plane z = 0.2; 0.3 px^2
 * added to the 2D covariance diagonal; the EWA Jacobian is evaluated at
 * view-ray ratios clamped to 1.3x the half field of view; depth is the
 * camera-space z; ties go to the smaller Gaussian index; colour =
 * max(0, 0.5 + SH(dir)) with dir the unit vector from the camera centre to
 * the conditional mean (world space); pixel (i, j) has centre (i+0.5, j+0.5).
 *
 * BATCHES.  Every entry point takes an array of nf frames (1 <= nf <=
 * SD7_MAX_FRAMES).  A frame is one (scene, view) render request; frames of
 * one call may use different scenes and resolutions.  All frames of a call
 * are processed by the same kernel launches; no frame's result depends on
 * the others (a frame renders bit-identically alone and in any batch), except
 * that the pair arena is shared: frames that do not fit are flagged
 * SD7_FLAG_PAIR_OVERFLOW and render as background.
 *
 * MEMORY.  The caller owns all memory.  Scene arrays, frame outputs and the
 * workspace are device pointers; frame descriptors are host memory, read
 * during the call only.  The library never allocates or frees device memory.
 * All intermediate arrays live in one caller-allocated workspace whose size
 * and layout sd7_plan() computes from the frames and a pair capacity; the
 * layout is part of this ABI (see sd7_layout) so callers may inspect every
 * intermediate.  The same (frames, nf, workspace) must be passed to all stage
 * calls of one render, in order: slice, project, bin, rasterize, then (for
 * training) rasterize_backward, project_backward, slice_backward.
 *
 * ASYNCHRONY.  Calls enqueue work on the given HIP stream (NULL = the null
 * stream) and return without waiting, except where stated.  Host-side
 * argument errors return synchronously and enqueue nothing.
 *
 * ERRORS.  Every call returns SD7_OK (0) or a negative sd7_status;
 * sd7_last_error() gives a message (per host thread).  Conditions found on
 * the device go to the per-frame flags word in the workspace (sd7_layout.
 * off_counts, word SD7_CNT_FLAGS of each frame).  No exception or abort
 * crosses the ABI.
 *
 * THREADS.  A context may be used from several host threads on different
 * streams with disjoint workspaces.
 */
#ifndef SD7_H
#define SD7_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t sd7_status;
#define SD7_OK 0
#define SD7_EINVAL (-1)     /* bad argument (null pointer, size out of range, ...) */
#define SD7_EHIP (-2)       /* a HIP runtime call failed */
#define SD7_EWORKSPACE (-3) /* workspace smaller than sd7_plan() requires */
#define SD7_ENOMEM (-4)     /* host allocation failed */

#define SD7_MAX_FRAMES 64
#define SD7_TILE 16
#define SD7_MAX_DIM 16384
#define SD7_PAIR_ROUND 2048 /* a frame's share of the pair arena is a multiple of this */

/* per-frame device flags (bitmask) */
#define SD7_FLAG_NONPOS_DIAG 1u   /* some L has a diagonal entry <= 0 (Gaussian culled) */
#define SD7_FLAG_NONFINITE 2u     /* a non-finite conditional statistic (Gaussian culled) */
#define SD7_FLAG_PAIR_OVERFLOW 4u /* the pair arena was too small: frame not rasterized */
#define SD7_FLAG_SORT_STALL 8u    /* a depth-sort work tile gave up waiting for the counts of an
                                     earlier one (never expected; the frame's output is not valid) */

/* per-frame device counters: SD7_CNT_WORDS uint32 words per frame */
#define SD7_CNT_KEPT 0      /* Gaussians that survive culling */
#define SD7_CNT_PAIRS 1     /* (tile, Gaussian) pairs of the frame */
#define SD7_CNT_PAIR_BASE 2 /* first arena slot of the frame's pairs */
#define SD7_CNT_FLAGS 3     /* SD7_FLAG_* bits */
#define SD7_CNT_NEEDED 4    /* pairs the frame needs, written by sd7_bin whether or not they
                               fit (on SD7_FLAG_PAIR_OVERFLOW: the share a re-run must give it) */
#define SD7_CNT_WORDS 16    /* words 5..15 are internal scratch of sd7_bin */

typedef struct sd7_ctx sd7_ctx;
typedef void* sd7_stream; /* a hipStream_t */

/* A scene of n 7D Gaussians (Sec. 4.1), device memory, FP32 structure of
 * arrays, read only (agr optional):
 *   mu_p [3][n]  spatial mean          mu_t [n]      temporal mean
 *   mu_d [3][n]  directional mean      alpha [n]     opacity in (0, 1)
 *   L   [28][n]  Cholesky factor of the 7x7 covariance Sigma = L L^T, lower
 *                triangle packed row-major: entry (i, j), i >= j, in plane
 *                i*(i+1)/2 + j; dimension order (x, y, z, t, dx, dy, dz).
 *                Diagonal entries must be positive (the caller's activation).
 *   sh  [48][n]  SH coefficients, plane 3*k + channel, k = l*l + l + m.
 *   agr [SD7_AGR_WEIGHTS]  adaptive Gaussian refinement (Sec. 4.3), or NULL
 *                for the variant without it.  Four two-layer MLPs, in the
 *                order mu_p, mu_t, mu_d, L, each stored as W1[64][27]
 *                (row-major), b1[64], W2[C_out][64], b2[C_out] with C_out =
 *                3, 1, 3, 28.  The input is f = mu_p, mu_t, mu_d, gamma(t)
 *                with gamma(t) = sin(2^k pi t), cos(2^k pi t), k = 0..9,
 *                interleaved; the hidden activation is ReLU; each output is
 *                added to its parameter (the L output in the packing above)
 *                before the slice.  The reverse calls do not support it. */
#define SD7_AGR_WEIGHTS 9443
typedef struct {
    const float* mu_p;
    const float* mu_t;
    const float* mu_d;
    const float* L;
    const float* alpha;
    const float* sh;
    int64_t n;
    const float* agr;
} sd7_scene;

/* A pinhole view at time t (host memory, by value).  R_wc is the row-major
 * world-to-camera rotation (camera axes x right, y down, z forward); c the
 * camera centre; (fx, fy, cx, cy) the intrinsics in pixels; d the view
 * direction the Gaussians are conditioned on (Algorithm 1 takes one d);
 * bg the background colour.  d_per_gaussian = 1 conditions Gaussian i on
 * its own direction unit(mu_p,i - c) instead of d (mu_p after refinement
 * when the scene has AGR weights). */
typedef struct {
    float R_wc[9];
    float c[3];
    float fx, fy, cx, cy;
    int32_t W, H;
    float t;
    float d[3];
    float lambda_t, lambda_d;
    float bg[3];
    int32_t d_per_gaussian;
} sd7_view;

/* Gradient outputs of one frame (device, overwritten by the backward):
 * same shapes as the scene arrays; alpha is the activated opacity.  lambda
 * (optional, NULL to skip) receives dL/dlambda_t and dL/dlambda_d of the
 * frame's view, added with atomics: the caller zeroes it. */
typedef struct {
    float* mu_p;
    float* mu_t;
    float* mu_d;
    float* L;
    float* alpha;
    float* sh;
    float* lambda;
} sd7_scene_grad;

/* One render request. */
typedef struct {
    sd7_scene scene;
    sd7_view view;
    float* image;            /* out [3][H][W]: C + T_final * bg */
    float* final_T;          /* out [H][W]: transmittance after compositing */
    uint32_t* last;          /* out [H][W]: tile-list entries the pixel consumed: those before
                                the one that stopped it, else the whole list */
    const float* dL_dimage;  /* in  [3][H][W]: backward only (may be NULL otherwise) */
    sd7_scene_grad grad;     /* out: backward only (may be NULL otherwise) */
    uint32_t* ncontrib;      /* optional out [H][W]: splats that contributed to the pixel;
                                NULL: not counted (the count costs one add per test) */
    uint32_t outputs;        /* SD7_OUT_* bits: intermediates to keep in the workspace */
} sd7_frame;

/* sd7_frame.outputs: sd7_slice_project and sd7_render write a frame's sliced
 * statistics (off_mu_c, off_cov_c, off_alpha_c) only when the frame asks for
 * them with SD7_OUT_SLICED or has gradient buffers (grad.L non-NULL: a
 * reverse pass will read them); sd7_slice always writes them.  A render
 * without them writes 40 bytes less per (Gaussian, frame). */
#define SD7_OUT_SLICED 1u

/* Workspace layout.  Every offset is in bytes from the workspace base and a
 * multiple of 256.  Per-Gaussian arrays hold the frames back to back: frame f
 * owns Gaussians [g0[f], g0[f] + n_f) with g0 the running sum of n; a
 * k-plane array stores frame f's planes at element k_planes*g0[f] + k*n_f.
 *   off_counts   uint32 [nf][SD7_CNT_WORDS]    per-frame counters and flags
 *   off_mu_c     float  [3 planes]             conditional mean
 *   off_cov_c    float  [6 planes]             conditional covariance (xx,xy,xz,yy,yz,zz)
 *   off_alpha_c  float  [1 plane]              conditional opacity
 *   off_splat    float  [Ntot][12]             per kept Gaussian (AoS; culled: not written): u, v, A, B, C, lo,
 *                                              r, g, b, 16 C, alpha_c, depth where
 *                                              (A, B, C) = -log2(e) (a/2, b, c/2) for the
 *                                              conic q = a dx^2 + 2b dx dy + c dy^2 and
 *                                              lo = log2(alpha_c), so that
 *                                              alpha_c e^{-q/2} = 2^(A dx^2 + B dx dy + C dy^2 + lo)
 *   off_rect     uint32 [Ntot][4]              kept Gaussians' tile footprint: the tile box (x0 | y0 << 16,
 *                                              x1 | y1 << 16; x1, y1 exclusive), then row
 *                                              trims: word 2 for box rows 0..3, word 3 for
 *                                              rows m..m+3 (m = h - 4 if the box has h > 8
 *                                              rows, else 4), one byte per row, low nibble =
 *                                              tiles dropped at the row's left end, high
 *                                              nibble = at its right end; other rows whole.
 *                                              Row r then spans tiles [x0 + lo, x1 - hi).
 *                                              A dropped tile holds no pixel where the
 *                                              splat reaches alpha >= 1/255.
 *   off_depth_key uint32 [Ntot]                float bits of depth; 0xFFFFFFFF = culled
 *   off_order    uint32 [Ntot]                 frame-local indices of kept Gaussians in
 *                                              (depth, index) order; entries >= kept unused
 *   off_pair_g   uint32 [capacity]             the pair arena: frame-local Gaussian index of
 *                                              every (tile, Gaussian) pair, grouped by tile
 *                                              (row-major tile ids ty*tiles_x+tx) and in
 *                                              (depth, index) order within a tile; frame f
 *                                              from arena slot counts[f][SD7_CNT_PAIR_BASE]
 *   off_ranges   uint32 [Ttot][2]              per tile [begin, end) arena slots (the tile of
 *                                              slot i is the tile whose range holds i); frame
 *                                              f's tiles start at the running sum of tile counts
 *   off_d_splat  float  [9 planes]             backward: dL/d(u, v, a, b, c, opacity, r, g, b)
 *   off_d_mu_c, off_d_cov_c, off_d_alpha_c     backward: dL/d of the slice outputs
 */
typedef struct {
    size_t bytes;
    int32_t nframes;
    int32_t tile_sort_passes;
    int64_t n_total;
    int64_t tiles_total;
    int64_t pair_capacity;
    size_t off_table;
    size_t off_counts;
    size_t off_mu_c, off_cov_c, off_alpha_c;
    size_t off_splat, off_rect, off_depth_key;
    size_t off_order;
    size_t off_pair_g;
    size_t off_ranges;
    size_t off_d_splat, off_d_mu_c, off_d_cov_c, off_d_alpha_c;
    size_t off_scratch; /* sort and scan temporaries; no stable meaning */
    int64_t g0[SD7_MAX_FRAMES];
    int64_t tile0[SD7_MAX_FRAMES];
} sd7_layout;

/* Context on HIP device `device`.  *out is set on success.  With the
 * environment variable SD7_PROFILE set (to anything but "0") when the context
 * is created, every stage the context runs (each stage call, and the three
 * stages inside sd7_render and sd7_render_static; not captured graphs) is
 * timed between two HIP events on its stream; sd7_profile_read returns the
 * totals.  The event pool (256 pairs) is made here, so timing allocates
 * nothing later; when every pair is in flight the oldest is waited for. */
sd7_status sd7_create(int device, sd7_ctx** out);
void sd7_destroy(sd7_ctx* ctx);

/* Per-stage GPU time of a context created with SD7_PROFILE set (Sec. 4.4's
 * stages: slice, project, slice_project, bin, rasterize and the three reverse
 * stages).  name: a static string; calls: stage runs; total_ms / max_ms: sum
 * and largest of their event-to-event times. */
typedef struct {
    const char* name;
    uint64_t calls;
    double total_ms;
    double max_ms;
} sd7_stage_time;

/* Host only; blocks until every timed stage has run.  Writes up to `max`
 * entries, one per stage that ran at least once, in pipeline order, and sets
 * *count to the number written (0 for a context without SD7_PROFILE).
 * reset != 0 clears the totals afterwards.  SD7_EINVAL for a NULL ctx or
 * count, a negative max, or a NULL out with max > 0. */
sd7_status sd7_profile_read(sd7_ctx* ctx, sd7_stage_time* out, int max, int* count, int reset);

/* Densification helper (Algorithm 1's optional step; Sec. 4.4): for n
 * symmetric 3x3 covariances cov[6][n] (packed xx, xy, xz, yy, yz, zz, e.g.
 * the sliced Sigma_cond planes of a workspace), Sigma = R diag(S^2) R^T with
 * scale[3][n] = S in descending order (square roots of the eigenvalues, 0
 * for negative ones) and rot[9][n] = R row-major (plane 3*row + col), its
 * columns the eigenvectors and det R = +1 (the last column negated when the
 * decomposition gives -1).  FP64 inside.  Device arrays; asynchronous. */
sd7_status sd7_cov_decompose(sd7_ctx* ctx, int64_t n, const float* cov, float* scale, float* rot,
                             sd7_stream stream);
/* Temporal split test of densification (Sec. 4.4): out[i] = 1 where
 * |(Sigma_xt, Sigma_yt, Sigma_zt)| > 0.05 * extent and
 * sqrt(Sigma_t) / time_span > 0.25 for Sigma = L L^T of the scene (the
 * paper's thresholds; extent is the scene's spatial extent, time_span the
 * length of the time range), else 0.  FP64 inside.  out: device, n bytes. */
sd7_status sd7_split_test(sd7_ctx* ctx, const sd7_scene* scene, float extent, float time_span,
                          uint8_t* out, sd7_stream stream);

/* ---- training-side helpers (Sec. 4.4: the 3DGS optimizer, pruning at the
 * raised opacity floor tau_min) ------------------------------------------ */

/* Mutable per-Gaussian arrays in the scene's shapes: parameters, or one of
 * Adam's moment sets (device, FP32). */
typedef struct {
    float* mu_p;
    float* mu_t;
    float* mu_d;
    float* L;
    float* alpha;
    float* sh;
} sd7_arrays;

typedef struct {
    float lr[6];               /* learning rate per group: mu_p, mu_t, mu_d, L, alpha, sh */
    float beta1, beta2, eps;   /* Adam */
    int32_t step;              /* 1 on the first step (bias correction) */
    float alpha_lo, alpha_hi;  /* the (activated) opacity is kept in [alpha_lo, alpha_hi] */
    float diag_min;            /* L's diagonal entries are kept >= diag_min */
} sd7_adam;

/* One Adam step over every parameter value of n Gaussians, in place:
 * m = b1 m + (1 - b1) g, v = b2 v + (1 - b2) g^2,
 * p -= lr / (1 - b1^step) * m / (sqrt(v) / sqrt(1 - b2^step) + eps), then
 * the opacity and L's diagonal are projected onto their bounds.  m, v start
 * at zero (the caller's).  grad: the backward's gradient arrays (lambda
 * unused).  Asynchronous; SD7_EINVAL on NULL arrays, step < 1 or bad betas. */
sd7_status sd7_adam_step(sd7_ctx* ctx, int64_t n, const sd7_arrays* params, const sd7_scene_grad* grad,
                         const sd7_arrays* m, const sd7_arrays* v, const sd7_adam* cfg,
                         sd7_stream stream);

/* Pruning in two calls, with a caller workspace of sd7_prune_workspace_size(n)
 * bytes (256-byte aligned).  sd7_prune_count marks the Gaussians with
 * alpha >= tau and writes their number to *d_kept (device); the caller then
 * allocates arrays for that many Gaussians and sd7_prune_apply copies, for
 * each of narrays arrays of planes[j] planes ([planes][n] -> [planes][n_kept]),
 * the kept Gaussians in their order (at most 32 arrays, e.g. a scene's six
 * parameter arrays and Adam's moments); with n_kept = 0 it copies nothing
 * and the array pointers may be NULL.  The workspace must hold the state of
 * the count call with the same alpha.  Asynchronous. */
size_t sd7_prune_workspace_size(int64_t n);
sd7_status sd7_prune_count(sd7_ctx* ctx, int64_t n, const float* alpha, float tau, void* ws,
                           size_t ws_bytes, uint32_t* d_kept, sd7_stream stream);
sd7_status sd7_prune_apply(sd7_ctx* ctx, int64_t n, int64_t n_kept, const float* const* src,
                           float* const* dst, const int32_t* planes, int narrays, const void* ws,
                           size_t ws_bytes, sd7_stream stream);

/* Message of the last failing call on this host thread ("" if none). */
const char* sd7_last_error(void);

/* Host only.  Workspace size and layout for these frames and a pair arena of
 * `pair_capacity` (tile, Gaussian) pairs shared by all frames (each frame's
 * share is rounded up to a multiple of SD7_PAIR_ROUND pairs).  Checks the frames:
 * 1 <= nf <= SD7_MAX_FRAMES, 0 <= n < 2^31, 1 <= W, H <= SD7_MAX_DIM, total
 * Gaussians and tiles < 2^31, pair_capacity < 2^31, non-null scene arrays
 * when n > 0, non-null image/final_T/last.  Returns SD7_EINVAL otherwise. */
sd7_status sd7_plan(const sd7_frame* frames, int nf, int64_t pair_capacity, sd7_layout* out);

/* Stage calls.  `ws`/`ws_bytes`: the workspace (device); `pair_capacity` must
 * equal the value given to sd7_plan.  SD7_EWORKSPACE if ws_bytes is too small. */

/* Sec. 4.2: writes mu_c, cov_c, alpha_c; zeroes the counters. */
sd7_status sd7_slice(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                     void* ws, size_t ws_bytes, sd7_stream stream);
/* Sec. 4.4 projection: writes depth_key, the KEPT counters and, for kept
 * Gaussians, splat and rect. */
sd7_status sd7_project(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                       void* ws, size_t ws_bytes, sd7_stream stream);
/* sd7_slice followed by sd7_project in one pass (Sec. 4.2, Sec. 4.4): frames
 * of the call that share a scene (the same six parameter arrays and n) are
 * sliced together, the view-independent part of each Gaussian's slice formed
 * once.  Outputs are bitwise those of the two separate calls. */
sd7_status sd7_slice_project(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                             void* ws, size_t ws_bytes, sd7_stream stream);
/* Depth sort of the kept Gaussians, then the tile lists: writes order,
 * pair_g, ranges and the PAIRS / PAIR_BASE counters; sets
 * SD7_FLAG_PAIR_OVERFLOW for frames whose pairs do not fit.  Tile lists are
 * built by counting (per chunk of depth-sorted Gaussians, how many boxes cover
 * each tile) and placement by groups of 8 x 8 tiles walking the depth order;
 * calls with a frame of more than 32768 tiles use a stable radix sort of
 * (tile, Gaussian) pairs instead.  Both give the same arena contents. */
sd7_status sd7_bin(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                   void* ws, size_t ws_bytes, sd7_stream stream);
/* Front-to-back compositing into each frame's image, final_T and last. */
sd7_status sd7_rasterize(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                         void* ws, size_t ws_bytes, sd7_stream stream);
/* slice + project + bin + rasterize in one call. */
sd7_status sd7_render(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                      void* ws, size_t ws_bytes, sd7_stream stream);

/* Replayed renders (Sec. 4.4 render path as one HIP graph).  A request loop
 * that renders frames of the same sizes again and again (one frame per call,
 * say) spends most of a small frame's time launching its ~30 kernels.
 * sd7_graph_create captures the kernel launches of sd7_render for these
 * frames, this pair capacity and this workspace (which the graph keeps
 * using: it must outlive the graph) into one HIP graph; nothing is launched
 * at creation.  sd7_graph_launch uploads the frames' descriptors to the
 * workspace and replays the graph on `stream`: views, scene arrays and
 * output pointers may differ from the captured frames, but the number of
 * frames, each frame's Gaussian count and resolution, whether it counts
 * contributors or carries AGR weights, and which frames share a scene (the
 * same arrays) must not (SD7_EINVAL otherwise).  The
 * outputs are bitwise those of sd7_render.  Launches of one graph share its
 * workspace: on different streams they must be ordered by the caller.
 * sd7_graph_destroy frees the graph (not the workspace). */
typedef struct sd7_graph sd7_graph;
sd7_status sd7_graph_create(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity, void* ws,
                            size_t ws_bytes, sd7_graph** out);
sd7_status sd7_graph_launch(sd7_graph* graph, const sd7_frame* frames, int nf, sd7_stream stream);
void sd7_graph_destroy(sd7_graph* graph);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, serving loops that must not call hipMalloc, harnesses that forbid
 * it.  sd7_render over a workspace the library owns instead of one the caller
 * passes: one static array of SD7_STATIC_WS_BYTES per device, held from the
 * library's load until the process ends.  For scale, one 200,000-Gaussian
 * 800x800 frame with a 1.5M-pair arena needs 53 MiB.  Frames whose sd7_plan()
 * size exceeds it are refused with SD7_EWORKSPACE before anything is enqueued.
 * The caller still owns the scene arrays and the frames' outputs; the call
 * allocates nothing.  counts_out (device, nf x SD7_CNT_WORDS uint32 words, or
 * NULL) receives the frames' counters and flags when the render ends, e.g.
 * whether the pair arena overflowed.  Every call on one device shares that
 * device's array and finds the previous call's intermediates in it (the
 * render clears what it needs cleared): calls that overlap on one device, from
 * any stream, thread or context, race, and the caller must serialize them.
 * Outputs are bitwise those of sd7_render with the same frames and capacity. */
#define SD7_STATIC_WS_BYTES 67108864u /* 64 MiB */
sd7_status sd7_render_static(sd7_ctx* ctx, const sd7_frame* frames, int nf, int64_t pair_capacity,
                             uint32_t* counts_out, sd7_stream stream);

/* Reverse of the compositing (Sec. 4.4, differentiable rasterization): each
 * pixel walks the list entries it consumed back to front from its final_T,
 * recomputing transmittance and the colour behind each entry (no per-pixel
 * list state is stored).  Reads each frame's dL_dimage, final_T, last and the
 * bins; writes d_splat (zeroed first, then accumulated). */
sd7_status sd7_rasterize_backward(sd7_ctx* ctx, const sd7_frame* frames, int nf,
                                  int64_t pair_capacity, void* ws, size_t ws_bytes,
                                  sd7_stream stream);
/* Reverse of the projection and SH colour: reads d_splat, writes d_mu_c,
 * d_cov_c, d_alpha_c and each frame's grad.sh. */
sd7_status sd7_project_backward(sd7_ctx* ctx, const sd7_frame* frames, int nf,
                                int64_t pair_capacity, void* ws, size_t ws_bytes,
                                sd7_stream stream);
/* Reverse of the slice (FP64 inside): reads d_mu_c, d_cov_c, d_alpha_c and
 * writes each frame's grad.mu_p, mu_t, mu_d, L, alpha.  Frames of one call
 * must not share gradient buffers. */
sd7_status sd7_slice_backward(sd7_ctx* ctx, const sd7_frame* frames, int nf,
                              int64_t pair_capacity, void* ws, size_t ws_bytes,
                              sd7_stream stream);

/* Blocks until the stream is idle and copies the nf x SD7_CNT_WORDS counters
 * to host memory `out`. */
sd7_status sd7_read_counts(sd7_ctx* ctx, int nf, const void* ws, uint32_t* out,
                           sd7_stream stream);

#ifdef __cplusplus
}
#endif
#endif /* SD7_H */
