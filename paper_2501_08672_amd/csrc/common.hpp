// Internal declarations shared by the HIP translation units of libgslivo.
// Device-side layouts, wave64 helpers and the host launchers that api.cpp calls.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "gslivo.h"

namespace gsl {

constexpr int kWave = 64;

// Camera as the kernels see it: intrinsics, pose, and its place in the packed
// tile and pixel layouts of the camera set.
struct DevCam {
    float fx, fy, cx, cy;
    int32_t W, H;
    float R[9];
    float t[3];
    int32_t tiles_x, tiles_y;
    int32_t tile_offset;  // first global tile id of this camera
    int32_t pad;
    int64_t pix_offset;   // first pixel of this camera in the packed layout
};
static_assert(sizeof(DevCam) == 96, "DevCam layout");
static_assert(sizeof(gsl_binrec) == 32, "gsl_binrec layout");

// Constants of one call, passed by value.
struct DevOpts {
    float near_z, eps2d, alpha_min, alpha_max, T_min;
    float bg[3];
    float guard;
    int32_t tile;
};

// Per-(camera, Gaussian) 2D gradient record: d/d(mx, my), d/d(A, B, C) of the
// conic, d/d opacity, d/d(r, g, b).  AoS so the atomics of one instance touch
// one cache line.
constexpr int kG2 = 9;

// ---------------------------------------------------------------- binning rule
// Threshold of the alpha_min ellipse, |L d|^2 <= kq, with a margin of 0.01 on
// top of 2 ln(sigma / alpha_min) that covers the float32 evaluation of the
// power in the renderer.  The projection computes it once per record, in
// float32 (the hardware base-2 logarithm, a few ulps: far inside the margin),
// and stores it in the binning record that counting and emission both read.
__device__ __forceinline__ float ellipse_k(float opacity, float alpha_min)
{
    constexpr float kTwoLn2 = 1.3862943611198906f;
    return fmaf(kTwoLn2, __builtin_amdgcn_logf(opacity / alpha_min), 0.01f);
}

// Does the ellipse |L (x - mu)|^2 <= kq reach a rectangle [x0, x1] x [y0, y1]
// of pixel centres?  The minimum of the convex quadratic over the rectangle
// is 0 when mu lies inside; otherwise it lies on an edge that faces mu (the
// segment from any other boundary point to mu would cross such an edge at a
// lower value), so at most one vertical and one horizontal edge are
// evaluated, each in closed form: on x = const the minimiser is dy = kv dx,
// on y = const it is dx = kh dy, clamped to the edge.  The projection-side
// count and the emit kernel both call this, so the instance count matches
// the instances written exactly.
struct EllipseTest {
    float mx, my, l11, l12, l22, kq;
    float kv;  // -(l11 l12) / (l12^2 + l22^2)
    float kh;  // -l12 / l11
};

__device__ __forceinline__ EllipseTest ellipse_test(const gsl_binrec &s)
{
    EllipseTest e;
    e.mx = s.mx;
    e.my = s.my;
    e.l11 = s.l11;
    e.l12 = s.l12;
    e.l22 = s.l22;
    e.kq = s.kq;
    const float cc = s.l12 * s.l12 + s.l22 * s.l22;
    e.kv = -(s.l11 * s.l12) / cc;
    e.kh = -s.l12 / s.l11;
    return e;
}

__device__ __forceinline__ bool ellipse_hits_rect(const EllipseTest &e, float x0, float x1, float y0, float y1)
{
    const bool in_x = e.mx >= x0 && e.mx <= x1, in_y = e.my >= y0 && e.my <= y1;
    if (in_x && in_y) return true;
    // The clamp of the unconstrained minimiser to the edge is a median of
    // three (the edge's ends are ordered), one v_med3_f32; the quadratic form
    // takes two fused multiply-adds.
    float best = 3.0e38f;
    if (!in_x) {  // the vertical edge facing mu
        const float dx = (e.mx < x0 ? x0 : x1) - e.mx;
        const float dy = __builtin_amdgcn_fmed3f(e.kv * dx, y0 - e.my, y1 - e.my);
        const float u = fmaf(e.l12, dy, e.l11 * dx), w = e.l22 * dy;
        best = fmaf(u, u, w * w);
    }
    if (!in_y) {  // the horizontal edge facing mu
        const float dy = (e.my < y0 ? y0 : y1) - e.my;
        const float dx = __builtin_amdgcn_fmed3f(e.kh * dy, x0 - e.mx, x1 - e.mx);
        const float u = fmaf(e.l12, dy, e.l11 * dx), w = e.l22 * dy;
        best = fminf(best, fmaf(u, u, w * w));
    }
    return best <= e.kq;
}

// Pixel-centre rectangle of tile (tx, ty) clipped to a W x H image.
__device__ __forceinline__ void tile_rect(int tx, int ty, int T, int W, int H, float &x0, float &x1, float &y0,
                                          float &y1)
{
    x0 = (float)(tx * T) + 0.5f;
    x1 = (float)min((tx + 1) * T, W) - 0.5f;
    y0 = (float)(ty * T) + 0.5f;
    y1 = (float)min((ty + 1) * T, H) - 0.5f;
}

// Instance payload: the Gaussian index in the low 28 bits and, in the top 4
// bits, which parts of the tile the alpha_min ellipse reaches (32x32 tiles:
// the 16x16 quadrants, bit 2 * row half + column half; 16x16 tiles: the
// quarter-row bands of 4 rows; 8x8 tiles: none).
constexpr uint32_t kGidBits = 28;
constexpr uint32_t kGidMask = (1u << kGidBits) - 1u;

// ---------------------------------------------------------------- host-side
struct Layout {
    int32_t C = 0, N = 0;
    int64_t M = 0;          // C * N projection records
    int64_t T_total = 0;    // tiles of all cameras
    int64_t P_total = 0;    // pixels of all cameras
    int32_t tile = 16;
    int32_t tile_bits = 1;  // bits needed for a global tile id
};

// Workspace regions (byte offsets from the workspace base).
struct WsLayout {
    size_t cams = 0;        // DevCam[C]
    size_t dkey = 0, dval = 0, dkey2 = 0, dval2 = 0;  // depth sort, u32[M] each
    size_t counts = 0;      // u32[M] tiles of the depth-ordered records
    size_t offsets = 0;     // u32[M] exclusive scan of counts
    size_t ikey2 = 0, ival2 = 0;  // u32[capacity] ping-pong for the tile sort
    size_t hist = 0;        // u32[256 * max_blocks] digit histograms
    size_t hist_off = 0;    // u32[256 * max_blocks] scanned histograms
    size_t partial = 0;     // u64[...] scan partial sums
    size_t rs_totals = 0;   // u32[256] per-digit totals of a radix pass
    size_t g2d = 0;         // float[C][N][kG2]
    size_t pose_part = 0;   // double[C][6][pose_blocks]
    size_t pose_part_sh = 0;  // the same for the SH colour's camera-centre term
    size_t loss_part = 0;   // double[T_total]
    size_t order = 0;       // u32[T_total] work order of the fused kernel
    size_t big = 0;         // u32[M] list of records spanning more than kBigTiles tiles
    size_t misc = 0;        // small scalars: work-queue counter (byte 0), kept-record count (byte 64),
                            // big-record list length (byte 128)
    size_t total = 0;
    int64_t sort_blocks = 0;
    int64_t scan_partials = 0;
    int32_t pose_blocks = 0;
};

// noalloc.hip: the file-scope scratch array of gsl_render_bwd_noalloc (bytes
// per GPU) and its device address on `device` (which must be current; looked
// up once per device and cached).
constexpr size_t kStaticScratchBytes = (size_t)160 << 20;
constexpr int kMaxScratchDevices = 64;
hipError_t static_scratch_address(int device, void **ptr);

// Radix sort / scan geometry
constexpr int kSortThreads = 512;
constexpr int kSortItems = 8;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 4;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kPoseThreads = 256;

// optim.hip: Adam over raw parameters [14][ld]; with update == false only the
// activated values are written.  g / act: mean, scale, quaternion, opacity,
// colour and SH arrays in the gsl_gaussians layout (row stride N).
void launch_adam(const float *const g[6], float *const act[6], float *raw, float *m, float *v, const int32_t *d_step,
                 const float lr[6], float beta1, float beta2, float eps, int N, int sh_degree, int64_t ld,
                 bool update, hipStream_t s);
// raw <- inverse activation of act (same layouts), m = v = 0, *d_step = 0.
void launch_adam_init(const float *const act[6], float *raw, float *m, float *v, int32_t *d_step, int N,
                      int sh_degree, int64_t ld, hipStream_t s);

// window.hip: maintenance of the sliding window (hash set of the frame's
// voxel keys, DELETE / ADD classification, in-place compaction).
struct WinWs {
    void *table = nullptr;      // 16-byte slots
    uint64_t slots = 0;         // power of two, >= 2 P
    int64_t *hdr = nullptr;     // D, A, n, P of the last classification, a marker
    uint32_t *pslot = nullptr;  // [P] slot of each point's key
    uint32_t *addf = nullptr, *arank = nullptr;  // [P]
    uint32_t *del = nullptr, *drank = nullptr, *evpos = nullptr;  // [n]
    uint64_t *partial = nullptr;  // scan partial sums
};
uint64_t window_table_slots(int64_t P);
// key of point i from xyz[i * ps + a * as], a = 0..2 (~0 where it has none)
void launch_voxel_keys(const float *xyz, int64_t P, int64_t ps, int64_t as, float voxel_size, uint64_t *keys,
                       hipStream_t s);
void launch_window_classify(const float *pts, int64_t P, float voxel_size, const uint64_t *keys, int64_t n,
                            const WinWs &w, int32_t *counts, uint64_t *add_keys, hipStream_t s);
void launch_window_compact(uint64_t *keys, float *rows, int R, int64_t ld, int64_t n, int64_t D,
                           const uint64_t *add_keys, const float *add_rows, int64_t A, uint64_t *evicted_keys,
                           float *evicted_rows, const WinWs &w, int32_t *status, hipStream_t s);

// ---------------------------------------------------------------- launchers
// project.hip
void launch_upload_cams(DevCam *d_cams, const DevCam *h_cams, int C, hipStream_t s);
void launch_project(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                    gsl_splat *splats, gsl_binrec *binrecs, uint32_t *depth_keys, int32_t *tiles_touched,
                    uint32_t *big_list, uint32_t *big_n, hipStream_t s, float *g2d_zero = nullptr,
                    uint32_t *queue_zero = nullptr);
void launch_project_bwd(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                        const float *g2d, const gsl_grads &out, int accumulate, double *pose_part,
                        int pose_blocks, hipStream_t s);
// Per-record derivatives of the 2D mean and conic along the camera twist,
// kTangent floats per record (records that reach no tile are not written).
constexpr int kTangent = 32;
// With a view-dependent colour the record also holds dc/d(dt) (3 channels x
// 3 translation directions) at floats 30..38: 40 floats.
constexpr int kTangentSH = 40;
void launch_project_tangent(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                            const int32_t *tiles_touched, float *tangent, hipStream_t s);

// sort.hip
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
// exclusive scan of n u32 counts (n known on the host) into u32 offsets; the
// 64-bit total goes to *d_total.  With d_n (device), counts at or beyond *d_n
// are taken as 0 (they are not read; every position still gets its offset).
void launch_scan_u32(const uint32_t *counts, uint32_t *offsets, int64_t n, uint64_t *partial, int64_t *d_total,
                     hipStream_t s, const int64_t *d_n = nullptr);
// Extra inputs and outputs of the depth sort, folded into its first and last
// passes: the first pass reads record j's key from first_keys[j], drops it
// when first_tiles[j] == 0 and takes j as its value; the last pass also
// writes counts_out[p] = gather_tiles[value] at every output position p < kept.
// When the record indices leave at least four high bits free, the values
// carry the tile count there from the first pass (a count that does not fit
// is marked all-ones and gathered), so the last pass gathers almost nothing.
struct DepthSortIO {
    const uint32_t *first_keys;
    const int32_t *first_tiles;
    const int32_t *gather_tiles;
    uint32_t *counts_out;
    uint32_t *zero_word = nullptr;  // cleared by the first pass's histogram kernel (may be null)
    // single-workgroup sorts (radix_one_block) also write the exclusive scan of
    // counts_out (positions at or beyond the kept count get the total) and
    // the total; the caller then skips its own scan
    uint32_t *offsets_out = nullptr;
    int64_t *d_total = nullptr;
};
// Up to this many keys one workgroup sorts them through all passes in LDS in
// one launch (and, for the depth sort, scans the tile counts): at these sizes
// the three launches per pass of the multi-block sort cost more than the work.
constexpr int64_t kOneBlockSortKeys = 16384;
inline bool radix_one_block(int64_t n_max) { return n_max > 0 && n_max <= kOneBlockSortKeys; }
// Stable LSD radix sort of (key, val) pairs over bits [0, bits) in as few
// passes of at most 8 bits as cover them; n_max bounds the grid, d_n (may be
// null) holds the live count on the device.  Returns 1 when the result is in
// keys2/vals2, 0 when in keys/vals.  With d_kept, keys 0xffffffff are dropped
// by the first pass and the number kept is written to *d_kept (later passes
// sort only those).  For n_max <= kOneBlockSortKeys one workgroup runs every
// pass (and, with io->offsets_out, the scan of the counts) in one launch; it
// then also writes the per-key-value ranges [first, one past last) of the
// sorted keys into ranges[2 * T_total] when ranges is given (keys >= T_total
// ignored), which the caller need not compute.
int launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, int64_t n_max,
                      const int64_t *d_n, int bits, uint32_t *hist, uint32_t *hist_off, uint32_t *totals,
                      hipStream_t s, int64_t *d_kept = nullptr, const DepthSortIO *io = nullptr,
                      uint32_t *ranges = nullptr, int64_t T_total = 0);
// tiles_touched of every (camera, Gaussian) record under the binning rule
// the records k_project put on the big-record list (tiles_touched of each)
void launch_count_big(const gsl_binrec *binrecs, const DevCam *cams, const Layout &L, int32_t *tiles_touched,
                      uint32_t *big_list, uint32_t *big_n, hipStream_t s);
// instances of the depth-ordered records; *big_n must be zero on entry (the
// depth sort's first histogram pass clears it through DepthSortIO::zero_word)
void launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *counts, const gsl_binrec *binrecs,
                 const DevCam *cams, const Layout &L, const int64_t *d_K, int64_t capacity, uint32_t *tile_ids,
                 uint32_t *gauss_ids, int32_t *d_status, uint32_t *big_list, uint32_t *big_n, const int64_t *d_V,
                 hipStream_t s);
void launch_ranges(const uint32_t *tile_ids, const int64_t *d_K, int64_t capacity, int64_t T_total,
                   uint32_t *ranges, hipStream_t s);

// render.hip
struct RenderArgs {
    const DevCam *cams;
    int32_t C, N;
    DevOpts o;
    const gsl_splat *splats;
    const uint32_t *gauss_ids;
    const uint32_t *ranges;
    int64_t T_total;
    // forward outputs / backward inputs
    float *image;
    float *T_final;
    uint32_t *n_walk;
    const float *dL_dimage;
    // fused loss
    const float *target;
    int32_t loss;
    double *loss_part;
    // backward output
    float *g2d;
    // persistent work queue
    const uint32_t *order;
    uint32_t *queue;
    // pose Jacobian (forward mode)
    const float *tangent;   // [M][kTangent], or [M][kTangentSH] with sh_colour
    int sh_colour;          // the tangents carry colour derivatives
    const float *weight;    // per-pixel R^-1 weight or NULL (1)
    int64_t P_total;        // pixels of all cameras (plane stride of jac)
    float *jac;             // [18][P_total] dI_ch/dxi_j planes (plane 6 ch + j) or NULL
    double *nrm_part;       // [T_total][kNrm] per-item normal-equation sums
};
// per item: H^T R^-1 H (21, upper triangle row by row), H^T R^-1 z (6), z^T R^-1 z
constexpr int kNrm = 28;
void launch_render_jvp(const RenderArgs &a, hipStream_t s);
// Per-camera sums of the item partials: HtH [C][36] (full), Htz [C][6], zz [C]; each may be NULL.
void launch_normal_reduce(const double *nrm_part, const DevCam *cams, int C, double *HtH, double *Htz, double *zz,
                          hipStream_t s);
void launch_render_fwd(const RenderArgs &a, hipStream_t s);
void launch_render_bwd(const RenderArgs &a, hipStream_t s);
// variant bit 0: persistent work queue (else one workgroup per item);
// bit 1: items in a.order (heaviest first) rather than tile order;
// bit 2: one workgroup per item with contiguous runs of tiles per XCD
// (variants 0..4 are the distinct ones)
constexpr int kVariants = 5;
// chunk: splats staged in LDS per chunk (64, 128 or 256)
void launch_render_fused(const RenderArgs &a, int variant, int chunk, int num_cus, hipStream_t s);
void launch_order_by_length(const uint32_t *ranges, int64_t T, uint32_t *order, hipStream_t s);
// counts[3] (device, accumulated): forward pairs evaluated, contributors, backward pairs
void launch_render_count(const RenderArgs &a, unsigned long long *counts, hipStream_t s);
void launch_reduce_f64(const double *part, int64_t n, double *out, hipStream_t s);
// sh.hip: bilinear colour of new Gaussians from a camera image
void launch_color_init(const float *mean, int64_t mean_ld, int n, const gsl_camera &c, float near_z,
                       const float *image, float *color, int64_t color_ld, uint8_t *valid, hipStream_t s);
// sums pose_part (and pose_part2 when not null), [C][6][blocks] each
void launch_pose_reduce(const double *pose_part, const double *pose_part2, int blocks, int C, double *g_pose,
                        int accumulate, hipStream_t s);
// adjoint of the SH colour (no-op at sh_degree 0): g_sh written or
// accumulated, the view-direction term added to g_mean, pose dt partials
void launch_sh_bwd(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const float *g2d, float *g_sh,
                   float *g_mean, int accumulate, double *pose_part, int pose_blocks, hipStream_t s);

// probe.hip: wave64 VALU instructions per CU and 2.4-GHz cycle of an
// instruction kind (0 FMA, 1 multiply + exp2, 2 integer min + add) over the
// whole chip; 0 on success
int run_valu_probe(int mode, int num_cus, float *sink, double *rate);

}  // namespace gsl
