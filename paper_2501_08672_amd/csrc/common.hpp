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
// power in the renderer.  Computed in float64 and rounded once, so every
// kernel that needs it gets the same float.
__device__ __forceinline__ float ellipse_k(float opacity, float alpha_min)
{
    return (float)(2.0 * log((double)opacity / (double)alpha_min) + 0.01);
}

// Does the ellipse |L (x - mu)|^2 <= kq reach the rectangle [x0, x1] x [y0, y1]
// of pixel centres?  The minimum of the convex quadratic over the rectangle is
// at mu when mu lies inside, else on one of its edges, where it has a closed
// form.  The projection kernel (counting) and the emit kernel (writing) both
// call this, so the instance count matches the instances written exactly.
__device__ __forceinline__ bool ellipse_hits_rect(float mx, float my, float l11, float l12, float l22, float kq,
                                                  float x0, float x1, float y0, float y1)
{
    if (mx >= x0 && mx <= x1 && my >= y0 && my <= y1) return true;
    const float dx0 = x0 - mx, dx1 = x1 - mx, dy0 = y0 - my, dy1 = y1 - my;
    const float cc = l12 * l12 + l22 * l22;
    float best = 3.0e38f;
    // vertical edges: dx fixed, dy free in [dy0, dy1]
    for (int e = 0; e < 2; e++) {
        const float dx = e ? dx1 : dx0;
        const float a = l11 * dx;
        const float dy = fminf(fmaxf(-(a * l12) / cc, dy0), dy1);
        const float u = a + l12 * dy, w = l22 * dy;
        best = fminf(best, u * u + w * w);
    }
    // horizontal edges: dy fixed, dx free in [dx0, dx1]
    for (int e = 0; e < 2; e++) {
        const float dy = e ? dy1 : dy0;
        const float b = l12 * dy, w = l22 * dy;
        const float dx = fminf(fmaxf(-b / l11, dx0), dx1);
        const float u = l11 * dx + b;
        best = fminf(best, u * u + w * w);
    }
    return best <= kq;
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
// bits, which quarter-row bands of the tile the alpha_min ellipse reaches
// (bit q: rows [q*T/4, (q+1)*T/4) of the tile).
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
    size_t g2d = 0;         // float[C][N][kG2]
    size_t pose_part = 0;   // double[pose_blocks][C][6]
    size_t loss_part = 0;   // double[T_total]
    size_t order = 0;       // u32[T_total] work order of the fused kernel
    size_t misc = 0;        // small scalars: queue counter, internal K
    size_t total = 0;
    int64_t sort_blocks = 0;
    int64_t scan_partials = 0;
    int32_t pose_blocks = 0;
};

// Radix sort / scan geometry
constexpr int kSortThreads = 256;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortThreads * kSortItems;  // keys per block
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanTile = kScanThreads * kScanItems;
constexpr int kPoseThreads = 256;

// ---------------------------------------------------------------- launchers
// project.hip
void launch_upload_cams(DevCam *d_cams, const DevCam *h_cams, int C, hipStream_t s);
void launch_project(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                    gsl_splat *splats, int32_t *tiles_touched, hipStream_t s);
void launch_project_bwd(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                        const float *g2d, const gsl_grads &out, int accumulate, double *pose_part,
                        int pose_blocks, hipStream_t s);

// sort.hip
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t n, hipStream_t s);
void launch_fill_f32(float *p, float v, int64_t n, hipStream_t s);
void launch_fill_f64(double *p, double v, int64_t n, hipStream_t s);
// exclusive scan of n u32 counts (n known on the host) into u32 offsets; the
// 64-bit total goes to *d_total.
void launch_scan_u32(const uint32_t *counts, uint32_t *offsets, int64_t n, uint64_t *partial, int64_t *d_total,
                     hipStream_t s);
// stable LSD radix sort of (key, val) pairs over bits [0, bits); n_max bounds
// the grid, d_n (may be null) holds the live count on the device.  Returns the
// buffer index (0: keys/vals, 1: keys2/vals2) that holds the result.
int launch_radix_sort(uint32_t *keys, uint32_t *vals, uint32_t *keys2, uint32_t *vals2, int64_t n_max,
                      const int64_t *d_n, int bits, uint32_t *hist, uint32_t *hist_off, uint64_t *partial,
                      hipStream_t s);
void launch_depth_keys(const gsl_splat *splats, const int32_t *tiles, int64_t M, uint32_t *keys, uint32_t *vals,
                       hipStream_t s);
void launch_gather_counts(const uint32_t *order, const int32_t *tiles, int64_t M, uint32_t *counts,
                          hipStream_t s);
// tiles_touched of every (camera, Gaussian) record under the binning rule
void launch_count_tiles(const gsl_splat *splats, const DevCam *cams, const Layout &L, float alpha_min,
                        int32_t *tiles_touched, hipStream_t s);
void launch_emit(const uint32_t *order, const uint32_t *offsets, const uint32_t *counts, const gsl_splat *splats,
                 const DevCam *cams, const Layout &L, float alpha_min, const int64_t *d_K, int64_t capacity,
                 uint32_t *tile_ids, uint32_t *gauss_ids, int32_t *d_status, hipStream_t s);
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
};
void launch_render_fwd(const RenderArgs &a, hipStream_t s);
void launch_render_bwd(const RenderArgs &a, hipStream_t s);
// variant bit 0: persistent work queue (else one workgroup per item);
// bit 1: items in a.order (heaviest first) rather than tile order
constexpr int kVariants = 4;
void launch_render_fused(const RenderArgs &a, int variant, int num_cus, hipStream_t s);
void launch_order_by_length(const uint32_t *ranges, int64_t T, uint32_t *order, hipStream_t s);
// counts[3] (device, accumulated): forward pairs evaluated, contributors, backward pairs
void launch_render_count(const RenderArgs &a, unsigned long long *counts, hipStream_t s);
void launch_reduce_f64(const double *part, int64_t n, double *out, hipStream_t s);
void launch_pose_reduce(const double *pose_part, int blocks, int C, double *g_pose, int accumulate,
                        hipStream_t s);

}  // namespace gsl
