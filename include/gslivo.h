/*
 * gslivo.h — C ABI of the MI355X (gfx950) Gaussian-splatting hot path of
 * GS-LIVO (arXiv 2501.08672): projection, tile binning with a radix sort,
 * front-to-back alpha compositing, and the photometric backward pass to the
 * Gaussians and to each camera's SE(3) pose.
 *
 * Conventions for every entry point
 *   - Device pointers are caller-owned device memory on the context's device;
 *     host pointers are read during the call only.  The library never
 *     allocates or frees device memory in these calls.
 *   - Work is enqueued on the caller's stream (`hipStream_t` passed as void*,
 *     NULL = the null stream) with no host synchronisation, so it can be
 *     recorded into a HIP graph.  Results are valid once the stream reaches
 *     them.
 *   - Return value: GSL_OK (0) or a negative GSL_E* code; nothing is thrown
 *     across the ABI.  gsl_last_error() describes the last failure on the
 *     calling thread.  Argument errors are detected on the host before any
 *     launch; a capacity overflow is detected on the device and reported
 *     through the `d_status` word of gsl_bins.
 *   - Floating-point arrays are float32 unless stated.  Gaussian parameters
 *     are SoA, component-major: mean[3][N], scale[3][N], quat[4][N],
 *     opacity[N], color[3][N].
 *   - Images of a camera set are packed: camera c occupies the planar block
 *     image[3][H_c][W_c] starting at float offset 3 * P_c, with
 *     P_c = sum_{j<c} W_j H_j; per-pixel arrays (T_final, n_walk) start at P_c.
 */
#ifndef GSLIVO_H
#define GSLIVO_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GSL_ABI_VERSION 3

#ifndef GSL_API
#define GSL_API __attribute__((visibility("default")))
#endif

enum {
    GSL_OK = 0,
    GSL_EINVAL = -1,    /* null pointer, bad size or option */
    GSL_ENOTSUP = -2,   /* tile size not in {8, 16, 32}, too many cameras */
    GSL_ECAPACITY = -3, /* instance count K exceeds capacity_K (device status) */
    GSL_EHIP = -4,      /* a HIP runtime call failed */
    GSL_ESTATE = -5     /* context/device mismatch */
};

#define GSL_MAX_CAMERAS 1024

typedef struct gsl_ctx gsl_ctx;

/* Pinhole camera.  p_C = R_cw p_W + t_cw; x right, y down, z forward.
 * Pixel (u, v) covers [u, u+1) x [v, v+1); its centre is (u + 0.5, v + 0.5). */
typedef struct {
    float fx, fy, cx, cy;
    int32_t width, height;
    float R_cw[9]; /* row-major world -> camera rotation */
    float t_cw[3];
} gsl_camera;

/* Rendering constants.  alpha_max and T_min are the alpha clamp and the
 * transmittance cutoff; the others are readings of what the paper leaves
 * open (gsl_default_opts fills them). */
typedef struct {
    float near_z;    /* cull a Gaussian whose camera depth is <= near_z (0.2 m) */
    float eps2d;     /* dilation added to the diagonal of Sigma2D (0.3 px^2) */
    float alpha_min; /* skip a Gaussian whose alpha at a pixel is < alpha_min (1/255) */
    float alpha_max; /* alpha = min(alpha_max, sigma G) (0.99) */
    float T_min;     /* stop before a Gaussian that would take T below T_min (1e-4) */
    float bg[3];     /* background colour (0) */
    float guard;     /* cull when the 2D mean lies beyond guard*W / guard*H outside the image (0.15) */
    int32_t tile;    /* tile edge in pixels: 8, 16 or 32 */
    int32_t chunk;   /* splats the fused window kernel stages in LDS per chunk: 64, 128 or
                      * 256; 0 = the one gsl_window_tune chose for these shapes, else 256
                      * at tile 32 and 64 at tiles 16 and 8 (gsl_default_opts: 0) */
} gsl_opts;

/* Gaussians of the window (SoA, component-major, device).
 *
 * View-dependent colour (the map's spherical-harmonic coefficients, Sec.
 * II-B): with sh_degree D in 1..3 the colour of Gaussian i seen from a camera
 * centred at o is c = color_i + sum_k sh_k,i B_k(u), u = (mean_i - o) /
 * |mean_i - o| in world coordinates, where B_k are the real orthonormal
 * harmonics of degrees 1..D (order l = 1..D, m = -l..l; Cartesian forms
 * without the Condon-Shortley sign: B_1 = c1 (y, z, x), ...) divided by
 * Y_00 = 1 / (2 sqrt(pi)), so the degree-0 coefficient is `color` itself.
 * K = (D + 1)^2 - 1 coefficients per channel, stored sh[(k * 3 + ch) * N + i].
 * No clamp.  sh_degree 0 (sh may be NULL): the colour is `color`. */
typedef struct {
    const float *mean;    /* [3][N] world position (m) */
    const float *scale;   /* [3][N] per-axis standard deviation (m), activated */
    const float *quat;    /* [4][N] rotation (w, x, y, z), any non-zero length */
    const float *opacity; /* [N] in (0, 1), activated */
    const float *color;   /* [3][N] degree-0 RGB */
    int32_t N;
    int32_t sh_degree;    /* 0..3 */
    const float *sh;      /* [K][3][N] higher-order SH coefficients (sh_degree > 0) */
} gsl_gaussians;

/* One projected Gaussian in one camera (48 bytes, 16-byte aligned).  The 2D
 * Gaussian is G(x) = exp(-1/2 |L (x - mu)|^2) with L = [[l11, l12], [0, l22]]
 * the upper Cholesky factor of Sigma2D^{-1}.  A culled splat has depth 0 and
 * an empty bbox (x0 > x1).  bbox is the inclusive pixel rectangle outside of
 * which alpha < alpha_min for certain. */
typedef struct {
    float mx, my;
    float l11, l12;
    float l22, opacity;
    float r, g;
    float b, depth;
    int16_t x0, y0, x1, y1;
} gsl_splat;

/* Output of gsl_project for C cameras x N Gaussians (device). */
/* Binning record of one projected Gaussian in one camera (32 bytes, 32-byte
 * aligned): the splat's mean and conic factor as in gsl_splat, kq such that
 * alpha >= alpha_min only inside the ellipse |L (x - mu)|^2 <= kq
 * (kq = 2 ln(opacity / alpha_min) + 0.01), and the same bbox.  gsl_project
 * writes it; gsl_bin_sort reads it in depth order, so its size is what that
 * gather moves. */
typedef struct {
    float mx, my;
    float l11, l12;
    float l22, kq;
    int16_t x0, y0, x1, y1;
} gsl_binrec;

typedef struct {
    gsl_splat *splats;      /* [C][N] */
    int32_t *tiles_touched; /* [C][N] number of tiles the alpha_min ellipse reaches */
    gsl_binrec *binrecs;    /* [C][N], 32-byte aligned */
    uint32_t *depth_keys;   /* [C][N] bits of the float depth (0xFFFFFFFF when culled): the depth-sort key */
} gsl_proj;

/* Tile bins (device).  After gsl_bin_sort, instances [0, K) are ordered by
 * (global tile id, depth, Gaussian index); ranges[t] = {start, end} of tile t
 * (end == start when empty).  The global tile id of camera c's tile
 * (tx, ty) is tile_offset_c + ty * tiles_x_c + tx, where tiles_x_c =
 * ceil(W_c / tile) and tile_offset_c counts the tiles of cameras before c. */
typedef struct {
    uint32_t *tile_ids;  /* [capacity_K] */
    uint32_t *gauss_ids; /* [capacity_K] low 28 bits: Gaussian index i of the instance;
                            top 4 bits: the tile parts the splat can reach: for
                            32x32 tiles the 16x16 quadrants (bit 2 * row half +
                            column half), for 16x16 tiles the quarter-row bands
                            (bit q: rows [4q, 4q + 4)), for 8x8 tiles 0 */
    uint32_t *ranges;    /* [T_total][2] */
    int64_t *d_K;        /* device scalar: instance count K (even when K > capacity) */
    int32_t *d_status;   /* device scalar: GSL_OK or GSL_ECAPACITY */
    int64_t capacity_K;
} gsl_bins;

/* Gradient outputs (device).  g_pose is float64 [C][6]: (dphi, dt) of a left
 * perturbation T_CW <- Exp(dphi, dt) T_CW of each camera.  Any pointer may be
 * NULL to skip that output except g2d-dependent ones noted per call. */
typedef struct {
    float *g_mean;    /* [3][N] */
    float *g_scale;   /* [3][N] */
    float *g_quat;    /* [4][N] */
    float *g_opacity; /* [N] */
    float *g_color;   /* [3][N] */
    double *g_pose;   /* [C][6] */
    float *g_sh;      /* [K][3][N], with SH colour (sh_degree > 0) */
} gsl_grads;

/* ---- context ---------------------------------------------------------- */

/* Creates a context bound to HIP device `device` (made current by the call). */
GSL_API int gsl_create(gsl_ctx **out, int device);
GSL_API int gsl_destroy(gsl_ctx *ctx);
/* Message of the last failure on this thread ("" if none).  Owned by the library. */
GSL_API const char *gsl_last_error(void);
GSL_API void gsl_default_opts(gsl_opts *opts);

/* Number of tiles and pixels of a camera set at opts->tile (host only). */
GSL_API int gsl_layout(const gsl_camera *cams, int32_t C, int32_t tile, int64_t *T_total, int64_t *P_total);

/* Bytes of device workspace the calls below need for these shapes (host
 * only; ctx is not used and may be NULL). */
GSL_API int gsl_workspace_size(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                       int64_t capacity_K, size_t *bytes);

/* ---- the four steps --------------------------------------------------- */

/* Projection (Sec. II-B, eqs. equ:3dgs, equ:q, equ:spat): for each camera c
 * and Gaussian i, Sigma3D = R(q) diag(s)^2 R(q)^T, p_C = R_cw p_W + t_cw,
 * mean2d = pinhole(p_C), Sigma2D = J R_cw Sigma3D R_cw^T J^T + eps2d I with J
 * the pinhole Jacobian at p_C.  Culls z <= near_z, means outside the guard
 * band and opacity < alpha_min.  Arithmetic is float64; the stored splat is
 * rounded to float32.  `workspace` receives the camera table used by the
 * later calls of the same camera set. */
GSL_API int gsl_project(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                gsl_proj *out, void *workspace, size_t workspace_bytes, void *stream);

/* Tile binning and sorting (Sec. II-C, the tile-based depth sorting of the
 * Gaussians in the GPU rasteriser; the front-to-back order eq. eq:raster
 * composites in): orders the Gaussians of every camera by depth
 * (32-bit float key, ties by index), emits one instance per overlapped tile
 * and sorts the instances by tile with a stable LSD radix sort, so the
 * instance order equals a sort by the 64-bit key (tile << 32 | depth bits)
 * with ties by index.  A Gaussian is binned into the tiles whose pixel-centre
 * rectangle its alpha_min ellipse reaches (a superset of every pixel where
 * alpha >= alpha_min, so the image does not depend on the tile size); N must
 * be below 2^28.  Writes K and, when K > capacity_K, GSL_ECAPACITY to
 * *d_status (then no instance is emitted and every tile's range is empty,
 * so a render of these bins draws nothing; call again with more capacity). */
GSL_API int gsl_bin_sort(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                 const gsl_proj *proj, gsl_bins *bins, void *workspace, size_t workspace_bytes, void *stream);

/* Forward compositing (eq. eq:raster): for every pixel walks its tile's list
 * front to back, alpha = min(alpha_max, opacity G), skips alpha < alpha_min,
 * stops before T (1 - alpha) < T_min, C += alpha T c.  Writes the packed
 * image (C + T bg), T_final and n_walk (the list position after the last
 * contributor: the backward pass starts there). */
GSL_API int gsl_render_fwd(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                   const gsl_proj *proj, const gsl_bins *bins, float *image, float *T_final, uint32_t *n_walk,
                   void *workspace, size_t workspace_bytes, void *stream);

/* Backward pass (eq. eq:gaussian_optimization, Appendix A): given
 * dL_dimage (packed like the image), the forward's T_final and n_walk,
 * walks each tile in reverse recovering T from T_final, accumulates the 2D
 * gradients per (camera, Gaussian), then chains them in float64 to the 3D
 * parameters (summed over cameras) and to each camera's pose.  Outputs are
 * overwritten unless accumulate != 0. */
GSL_API int gsl_render_bwd(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                   const gsl_proj *proj, const gsl_bins *bins, const float *T_final, const uint32_t *n_walk,
                   const float *dL_dimage, int accumulate, gsl_grads *grads, void *workspace,
                   size_t workspace_bytes, void *stream);

/* gsl_render_bwd without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc).  Same arguments, results and error
 * behaviour as gsl_render_bwd; its scratch memory (the camera table, the
 * per-(camera, Gaussian) 2D gradients, 36 B each, and the per-block pose
 * partials) lives in a file-scope device array of 160 MiB per GPU, created
 * with the library's code object and held until the process ends.  Shapes
 * whose scratch exceeds it (about C * N <= 4.6M records) are rejected with
 * GSL_EINVAL before any launch; GSL_EHIP when the array's address could not
 * be obtained at gsl_create.  The call allocates nothing.  Every call on one
 * GPU shares that GPU's array and clears what it accumulates into at its
 * start: calls that overlap on one GPU (other streams, other threads or
 * contexts) race and must be serialised by the caller. */
GSL_API int gsl_render_bwd_noalloc(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C,
                                   const gsl_opts *opts, const gsl_proj *proj, const gsl_bins *bins,
                                   const float *T_final, const uint32_t *n_walk, const float *dL_dimage,
                                   int accumulate, gsl_grads *grads, void *stream);

/* Work counts of the compositing on these bins (for throughput accounting):
 * d_counts[0] = (pixel, Gaussian) pairs the forward walk evaluates, up to
 * and including the one that stops it; d_counts[1] = contributing pairs;
 * d_counts[2] = pairs the backward walk evaluates (per pixel, the list
 * positions up to its last contributor whose splat reaches the pixel's row
 * band).
 * d_counts is device uint64[3], overwritten. */
GSL_API int gsl_render_stats(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                             const gsl_proj *proj, const gsl_bins *bins, uint64_t *d_counts, void *workspace,
                             size_t workspace_bytes, void *stream);

/* ---- the batched window ------------------------------------------------ */

enum { GSL_LOSS_L1 = 1, GSL_LOSS_L2 = 2 };

/* One optimisation pass over the sliding window of keyframes (Sec. II-C: the
 * window's Gaussians are optimised on the GPU against its keyframes; Sec.
 * III-B: 10 such passes per frame, see gsl_window_optimize), the photometric
 * loss of eq. eq:gaussian_optimization and its gradient: project, bin_sort, then
 * one fused launch over all (camera, tile) items that composites,
 * forms the per-pixel loss gradient against `target` (packed like the image;
 * L1: mean absolute error per frame summed over frames, L2: 1/2 sum of
 * squares), and walks back, then the projection adjoint.  Writes the loss to
 * *d_loss (device float64) and the gradients (overwritten); image may be NULL.
 * The fused launch uses the kernel variant (persistent work queue or one
 * workgroup per item; items in tile order or longest list first) that
 * gsl_window_tune chose for these shapes, else the default.  With
 * use_graph != 0 the sequence is recorded once into a HIP graph per (camera
 * sizes, Gaussian count, buffers, options, variant, loss) and replayed on
 * later calls with the same arguments; the camera table (poses and
 * intrinsics) is uploaded on the stream before each launch, so new poses of
 * the same cameras replay the cached graph. */
GSL_API int gsl_window_step(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                    const float *target, int loss, gsl_proj *proj, gsl_bins *bins, float *image,
                    double *d_loss, gsl_grads *grads, void *workspace, size_t workspace_bytes,
                    int use_graph, void *stream);

/* Pins the fused-kernel variant and LDS chunk depth gsl_window_step uses
 * for these shapes (what gsl_window_tune would store): variant bit 0
 * persistent work queue, bit 1 longest list first, 4 = contiguous tile runs
 * per XCD (0..4 are valid); chunk 64, 128 or 256, or 0 for the tile size's
 * default. */
GSL_API int gsl_window_variant(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, int32_t tile,
                               int32_t variant, int32_t chunk);

/* Measurement aid for the roofline of the compositing kernels, not an
 * operation of the method: runs a kernel of independent dependency chains on
 * every CU (eight waves per SIMD) and writes the wave64 VALU instructions it
 * issued per CU per 2.4-GHz cycle.  mode 0: FP32 fused multiply-add; 1: FP32
 * multiply + v_exp_f32; 2: unsigned integer min + FP32 add; 3: FP32 add;
 * 4: FP32 multiply.  d_sink: one
 * float of device memory the kernel could write (it never does).  Waits for
 * the device (default stream).  GSL_EINVAL for a NULL pointer, a mode outside
 * [0, 4] or host memory; GSL_EHIP when the launch or its timing fails. */
GSL_API int gsl_valu_probe(gsl_ctx *ctx, int32_t mode, float *d_sink, double *insts_per_cu_cycle);

/* Forward render of a window (the compositing of Sec. II-B, eq. raster, over
 * tile lists built as in Sec. II-C) as one unit: gsl_project, gsl_bin_sort
 * and gsl_render_fwd of all C cameras, the same kernels in the same order, so
 * proj, bins, image, T_final and n_walk are bit-identical to those three
 * calls'.  Buffers, layouts and workspace as for those calls (the workspace
 * must satisfy gsl_workspace_size).  With use_graph the launches are recorded
 * once per shape (camera sizes, N, tile, every pointer and the options; not
 * the poses or intrinsics: the camera table is uploaded on the stream before
 * each launch) into a HIP graph held by the context and replayed.  Errors as
 * for the three calls; GSL_EHIP when recording or launching the graph
 * fails. */
GSL_API int gsl_window_render(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C,
                              const gsl_opts *opts, gsl_proj *proj, gsl_bins *bins, float *image, float *T_final,
                              uint32_t *n_walk, void *workspace, size_t workspace_bytes, int use_graph,
                              void *stream);

/* Number of HIP graphs the context holds (window steps and optimisation
 * loops recorded so far, at most 65 before the cache is flushed). */
GSL_API int gsl_graph_count(gsl_ctx *ctx, int64_t *count);

/* Profiling hook: while enabled, every window step records HIP events on its
 * stream between its stages (a graph step launches a graph captured for
 * profiling, cached beside the plain one, whose event-record nodes are these
 * events).  gsl_profile_read waits for the last profiled step and writes up
 * to n milliseconds:
 * [0] upload + project, [1] bin_sort, [2] the fused render launch,
 * [3] loss reduction + projection adjoint, [4] the whole step. */
GSL_API int gsl_profile(gsl_ctx *ctx, int enable);
GSL_API int gsl_profile_read(gsl_ctx *ctx, float *ms, int32_t n);

/* Autotuner for gsl_window_step: times every tile size in {8, 16, 32}, every
 * LDS chunk depth in {64, 128, 256} and every fused-kernel variant on the
 * given window (eager launches on `stream`, synchronising it), keeps the
 * fastest (variant, chunk) per tile size in the context and writes the
 * fastest tile size to opts_inout->tile (opts_inout->chunk is left as it
 * is; 0 uses the tuned chunk).  The
 * buffers must be sized for tile 8 (the largest T_total) and enough
 * capacity_K for every tile size; times_ms (may be NULL) receives up to
 * `ntimes` measured milliseconds in the order tried: tiles 8, 16, 32; per
 * tile the chunks 64, 128, 256; per chunk the five variants 0..4 (45 in
 * all). */
GSL_API int gsl_window_tune(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, gsl_opts *opts_inout,
                    const float *target, int loss, gsl_proj *proj, gsl_bins *bins, double *d_loss,
                    gsl_grads *grads, void *workspace, size_t workspace_bytes, float *times_ms, int32_t ntimes,
                    void *stream);

/* ---- Adam over the map parameters ----------------------------------------- */

/* The map is refined with Adam (Sec. II-B, eq. eq:gaussian_optimization).
 * The optimiser keeps raw parameters: 14 rows of N floats at a row stride ld:
 * mean (3), log-scale (3), quaternion (4), opacity logit (1), colour (3), then
 * with SH colour the 3K higher-order coefficients.  The
 * renderer takes the activated values (scale = exp(log-scale), opacity =
 * sigmoid(logit), the rest unchanged), which the optimiser writes into the
 * arrays of a gsl_gaussians (its pointers are written through). */
typedef struct {
    float lr[5];  /* learning rates: mean, log-scale, quaternion, opacity logit, colour */
    float beta1, beta2, eps;
    float lr_sh;  /* learning rate of the higher-order SH coefficients */
} gsl_adam;

typedef struct {
    float *raw;      /* [14 + 3K][ld] raw parameters: row r of Gaussian i at raw[r * ld + i] */
    float *m, *v;    /* [14 + 3K][ld] first and second moments (zero before the first step) */
    int32_t *d_step; /* device: steps taken (0 before the first step), advanced by each step */
    int32_t N;       /* Gaussians in the window */
    int32_t ld;      /* row stride in floats, >= N (0: N).  A window kept at a fixed
                      * capacity (gsl_window_compact) uses its capacity here. */
    int32_t sh_degree; /* rows 14 .. 14 + 3K - 1 are the SH coefficients in the
                        * gsl_gaussians.sh order (identity activation); must equal
                        * the activated Gaussians' sh_degree */
} gsl_adam_state;

/* Starting point of the optimisation of the map parameters (Sec. II-B):
 * raw <- the inverse activation of act (log-scale = ln(scale), opacity
 * logit = ln(o / (1 - o)); mean, quaternion, colour and SH rows as they are),
 * m = v = 0 and *d_step = 0, in float32 on the device.  act.N and
 * act.sh_degree must equal the state's; scales must be > 0 and opacities in
 * (0, 1) (otherwise the raw value is not finite).  d_step must not be NULL. */
GSL_API int gsl_adam_init(gsl_ctx *ctx, const gsl_gaussians *act, gsl_adam_state *st, void *stream);

/* act <- activation(raw).  No optimiser step. */
GSL_API int gsl_adam_activate(gsl_ctx *ctx, const gsl_adam_state *st, gsl_gaussians *act, void *stream);

/* One Adam step at step number t = *d_step + 1: the gradients of the
 * activated values (grads, as gsl_render_bwd / gsl_window_step write them)
 * are chained to the raw rows, m <- b1 m + (1 - b1) g,
 * v <- b2 v + (1 - b2) g^2, raw <- raw - lr (m / (1 - b1^t)) /
 * (sqrt(v / (1 - b2^t)) + eps); then act <- activation(raw) and *d_step += 1. */
GSL_API int gsl_adam_step(gsl_ctx *ctx, gsl_adam_state *st, const gsl_adam *hp, const gsl_grads *grads,
                          gsl_gaussians *act, void *stream);

/* `iters` optimisation iterations of the window (the paper runs 10 per
 * keyframe): each is gsl_window_step on act followed by gsl_adam_step, the
 * loss of iteration k going to d_losses[k] (device float64 [iters]).  act must
 * hold activation(raw) on entry (gsl_adam_activate).  With use_graph != 0 the
 * whole sequence is recorded once into a HIP graph per (shapes, buffers,
 * options, Adam hyper-parameters, iters) and replayed; as for
 * gsl_window_step, the camera table is uploaded before each launch. */
GSL_API int gsl_window_optimize(gsl_ctx *ctx, gsl_adam_state *st, const gsl_adam *hp, gsl_gaussians *act,
                                const gsl_camera *cams, int32_t C, const gsl_opts *opts, const float *target,
                                int loss, gsl_proj *proj, gsl_bins *bins, double *d_losses, gsl_grads *grads,
                                int32_t iters, void *workspace, size_t workspace_bytes, int use_graph,
                                void *stream);

/* Initial colour of new Gaussians (Sec. II-B, eq. c(mu_I)): each mean
 * (device float mean[a * mean_ld + i], a = 0..2) is projected into the
 * camera in float64; the colour is the bilinear interpolation of the image
 * (device float, planar [3][H][W]) there.  Pixel (c, r) has its centre at
 * (c + 1/2, r + 1/2); the projected point minus 1/2 is clamped to the range
 * of the centres and the four surrounding pixels are weighted by the areas
 * of the opposite sub-rectangles.  Writes color[ch * color_ld + i] for the
 * means in front of opts->near_z that project into [0, W) x [0, H) and
 * valid[i] (may be NULL) = 1 for those, 0 otherwise (colour untouched).
 * The higher-order SH coefficients of new Gaussians start at zero. */
GSL_API int gsl_color_init(gsl_ctx *ctx, const float *mean, int64_t mean_ld, int32_t n, const gsl_camera *cam,
                           const float *image, const gsl_opts *opts, float *color, int64_t color_ld,
                           uint8_t *valid, void *stream);

/* ---- sliding-window maintenance ------------------------------------------ */

/* The window of Gaussians is kept contiguous on the device and updated
 * incrementally from frame to frame (Sec. II-C, Steps 1-4).  Each Gaussian
 * carries the 64-bit key of the root voxel it belongs to (Sec. II-A, eq.
 * HashKey): with i = floor(p / v_s) per axis, computed in float64,
 *   key = ((ix + 2^20) << 42) | ((iy + 2^20) << 21) | (iz + 2^20),
 * defined for indices in [-2^20, 2^20).  Its parameters are R rows of 4-byte
 * words at a row stride ld (a capacity): row r of Gaussian i at
 * rows[r * ld + i].  Raw parameters and Adam moments allocated as one
 * [3 (14 + 3K)][ld] block (raw, m, v of a gsl_adam_state with that ld; 42
 * rows without SH colour) are moved by one call. */

/* keys[i] <- the voxel key of point i, whose coordinates are
 * xyz[i * point_stride + a * axis_stride], a = 0, 1, 2 (device float; [P][3]
 * interleaved: strides 3, 1; component-major [3][P] like gsl_gaussians.mean:
 * strides 1, P).  A point without a key (non-finite, or an index outside
 * [-2^20, 2^20)) gets 0xFFFFFFFFFFFFFFFF, which no window Gaussian may carry
 * and stay in the window.  For keying new Gaussians at insertion. */
GSL_API int gsl_voxel_keys(gsl_ctx *ctx, const float *xyz, int32_t P, int64_t point_stride, int64_t axis_stride,
                           float voxel_size, uint64_t *keys, void *stream);

/* Workspace bytes for gsl_window_classify / gsl_window_compact with a window
 * of n Gaussians and a frame of P points (P <= 2^28): a hash table of 16 B
 * per slot (the smallest power of two >= max(1024, 2P)), 12 B per point,
 * 12 B per window Gaussian and the scan partials.  The workspace must be
 * 256-byte aligned. */
GSL_API int gsl_window_workspace_size(int32_t n, int32_t P, size_t *bytes);

/* Steps 1 and 3.  points: device float [P][3] world coordinates of the
 * current LiDAR frame (interleaved x, y, z); voxel_size v_s > 0; keys: device
 * uint64 [n] of the window.  The field of view is the set of keys of the
 * frame's points (points without a key are ignored).  Writes, on the device:
 *   counts  int32[2]: D, the window Gaussians whose key is not in the field
 *           of view (DELETE), and A, the keys of the frame that no window
 *           Gaussian carries (ADD);
 *   add_keys uint64[P] (may be NULL): entries [0, A) are the ADD keys, each
 *           once, in the order of their first point.
 * The workspace keeps the classification for gsl_window_compact; it must not
 * be reused before that call has been enqueued. */
GSL_API int gsl_window_classify(gsl_ctx *ctx, const float *points, int32_t P, float voxel_size,
                                const uint64_t *keys, int32_t n, int32_t *counts, uint64_t *add_keys,
                                void *workspace, size_t workspace_bytes, void *stream);

/* Steps 2 and 4, in place, after gsl_window_classify on the same workspace
 * with the same n.  keys: device uint64[ld]; rows: device float [R][ld]
 * (R may be 0: keys only).  D is the DELETE count that call wrote (read back
 * by the caller).  In stream order:
 *   1. the DELETE Gaussians are gathered, in window order, into
 *      evicted_keys uint64[D] and evicted_rows float[R][D] (row stride D);
 *      either may be NULL (not written);
 *   2. with n' = n - D, the k-th DELETE slot below n' receives the k-th kept
 *      Gaussian of [n', n) (keys and rows); kept Gaussians below n' keep
 *      their slot;
 *   3. the A new Gaussians add_keys uint64[A], add_rows float[R][A] (row
 *      stride A) are written to slots [n', n' + A).
 * Afterwards the window holds n - D + A Gaussians.  Host checks: n - D + A <=
 * ld, 0 <= D <= n.  If n or D differ from what the classification found on
 * the device, nothing is written and *status (device int32, may be NULL)
 * is set to 1; otherwise to 0. */
GSL_API int gsl_window_compact(gsl_ctx *ctx, uint64_t *keys, float *rows, int32_t R, int64_t ld, int32_t n,
                               int32_t D, const uint64_t *add_keys, const float *add_rows, int32_t A,
                               uint64_t *evicted_keys, float *evicted_rows, const void *workspace,
                               size_t workspace_bytes, int32_t *status, void *stream);

enum { GSL_D2H = 0, GSL_H2D = 1 };

/* Moves `count` Gaussians of the window update between the device and pinned
 * host memory (Sec. II-C: the Gaussians that leave the window go back to the
 * global map in host RAM, those that enter come from it): count uint64 keys
 * and R rows of 4-byte words, row r of Gaussian i at rows[r * ld + i], with
 * the source's and the destination's row strides src_ld and dst_ld
 * (>= count).  Asynchronous copies on the stream: one for the keys, one
 * strided 2D copy for the rows.  dir GSL_D2H: sources in device memory,
 * destinations in pinned host memory; GSL_H2D the reverse.  Keys or rows may
 * be NULL on both sides (not moved).  GSL_EINVAL when a host-side buffer is
 * not pinned (hipHostMalloc, or a pinned torch tensor) or a device-side one
 * is not device memory, so that no copy silently goes through a pageable
 * staging path.  Host buffers must stay untouched until the stream reaches
 * the copies. */
GSL_API int gsl_window_transfer(gsl_ctx *ctx, int dir, const uint64_t *src_keys, const float *src_rows,
                                int64_t src_ld, uint64_t *dst_keys, float *dst_rows, int64_t dst_ld, int32_t R,
                                int32_t count, void *stream);

/* ---- pose Jacobians for the IESKF visual update -------------------------- */

/* Workspace bytes for gsl_pose_jacobian: the bytes gsl_workspace_size gives
 * for the same arguments, plus 160 B per (camera, Gaussian) record for its
 * twist tangents (those of the 2D mean and conic, and of the colour when it
 * is view-dependent) and 224 B per tile for the per-tile partial sums (host
 * only; ctx is not used and may be NULL). */
GSL_API int gsl_pose_jacobian_workspace_size(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N,
                                             const gsl_opts *opts, int64_t capacity_K, size_t *bytes);

/* Photometric measurement model of the visual update (Sec. II-D, eq.
 * eq:minimization; Appendix A): the Jacobian of the rendered colour with
 * respect to each camera's twist xi = (dphi, dt) of the left perturbation
 * T_CW <- Exp(xi) T_CW, by forward-mode differentiation through the
 * projection (eqs. eqn:grad_meani_rcw ... eqn:grad_covi_tcw) and the same
 * front-to-back walk as gsl_render_fwd (same contributors; the thresholds
 * are held fixed).  With SH colour (sh_degree > 0) the colours' own
 * dependence on the camera centre (the translation of the twist) is
 * included.  Needs gsl_project and gsl_bin_sort outputs for these
 * Gaussians and cameras.  Device outputs, each may be NULL:
 *   image  float[3 * P_total]  the rendered colour, packed as gsl_render_fwd;
 *   jac    float[18 * P_total] plane 6 * ch + j holds dI_ch/dxi_j of every
 *          pixel in the packed pixel order (plane stride P_total);
 *   HtH    double[C][36], Htz double[C][6], zz double[C]: per camera the sums
 *          over its pixels p and channels of w_p h h^T, w_p h z and w_p z^2,
 *          where h = dI_ch/dxi (6), z = I_ch - target_ch, and w_p = weight[p]
 *          (device float[P_total], R^-1 of the pixel) or 1 when weight is
 *          NULL.  These need target (packed like the image).
 * The workspace must hold gsl_pose_jacobian_workspace_size bytes.
 * Stream-ordered, no host synchronisation. */
GSL_API int gsl_pose_jacobian(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C,
                              const gsl_opts *opts, const gsl_proj *proj, const gsl_bins *bins, const float *target,
                              const float *weight, float *image, float *jac, double *HtH, double *Htz, double *zz,
                              void *workspace, size_t workspace_bytes, void *stream);

/* Host helpers (plain double arrays in host memory, row-major; no device
 * work).  gsl_imu_to_camera_twist writes A (6x6) with xi_cam = A xi_imu to
 * first order, from the perturbation model of Appendix A (eq.
 * eq:perturbation): (T(xi_cam) T_CW)^-1 T_CI = T_WI [+] xi_imu, the IMU
 * pose perturbed as (R_WI Exp(dphi), t_WI + dt); so dphi_cam = -R_CI dphi_imu
 * and dt_cam = t_CI^ dphi_cam - R_CW dt_imu.  H_imu = H_cam A. */
GSL_API int gsl_imu_to_camera_twist(const double R_CI[9], const double t_CI[3], const double R_CW[9], double A[36]);

/* One IESKF update of a 6-dof pose from its normal equations (Appendix A):
 * K = (H^T R^-1 H + P^-1)^-1 H^T R^-1,
 * delta = -K z - (I - K H) dx_prior,  P_post = (I - K H) P,
 * with dx_prior = x_hat [-] x_bar (NULL: zero, the first iteration) and the
 * Jacobian of [-] taken as the identity.  HtRH, P, P_post are 6x6, HtRz,
 * delta 6-vectors.  GSL_EINVAL when P or H^T R^-1 H + P^-1 is singular. */
GSL_API int gsl_ieskf_pose_update(const double HtRH[36], const double HtRz[6], const double P[36],
                                  const double dx_prior[6], double delta[6], double P_post[36]);

/* The visual update of the IMU pose from one camera's photometric normal
 * equations (Sec. II-D, eq. eq:minimization; Appendix A): with A from
 * gsl_imu_to_camera_twist the measurement Jacobian in the IMU twist is
 * H_imu = H_cam A, and with the noise R = noise_var I the update of
 * gsl_ieskf_pose_update takes H_imu^T R^-1 H_imu = A^T (H_cam^T H_cam) A /
 * noise_var and H_imu^T R^-1 z = A^T (H_cam^T z) / noise_var.  HtH_cam and
 * Htz_cam are a camera's HtH and Htz as gsl_pose_jacobian writes them (any
 * per-pixel weights already applied), copied to the host; the other
 * arguments as for gsl_ieskf_pose_update.  GSL_EINVAL for a NULL argument,
 * noise_var not finite and > 0, or a singular system. */
GSL_API int gsl_ieskf_visual_update(const double HtH_cam[36], const double Htz_cam[6], const double A[36],
                                    double noise_var, const double P[36], const double dx_prior[6], double delta[6],
                                    double P_post[36]);

#ifdef __cplusplus
}
#endif
#endif /* GSLIVO_H */
