// Host side of the C ABI declared in gslivo.h: argument checks, the packed
// tile/pixel layout of a camera set, the workspace carve-up, the launch
// sequence of each step, HIP-graph capture of the window step and the
// autotuner that picks tile size and fused-kernel variant.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.hpp"
#include "gslivo.h"

using namespace gsl;

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int check_hip(hipError_t e, const char *what)
{
    if (e != hipSuccess) return fail(GSL_EHIP, "%s: %s", what, hipGetErrorString(e));
    return GSL_OK;
}

int check_launch(const char *what)
{
    return check_hip(hipGetLastError(), what);
}

#define GSL_TRY(x)                \
    do {                          \
        int _rc = (x);            \
        if (_rc != GSL_OK) return _rc; \
    } while (0)

size_t align_up(size_t v, size_t a = 256) { return (v + a - 1) / a * a; }

int ceil_log2(int64_t v)
{
    int b = 0;
    while (((int64_t)1 << b) < v) b++;
    return b < 1 ? 1 : b;
}

// Signature of a window used to key graphs and tuning results.
struct VariantKey {
    std::vector<int64_t> v;
    bool operator<(const VariantKey &o) const { return v < o.v; }
};

struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
};

}  // namespace

// Stages of a window step timed by the profiling hook.
enum { kStProject, kStBinSort, kStRender, kStProjectBwd, kStages };

struct gsl_ctx {
    int device = 0;
    int num_cus = 256;
    hipStream_t cap_stream = nullptr;
    bool profile = false;
    hipEvent_t ev[kStages + 1] = {};
    bool ev_recorded = false;
    std::mutex mu;
    std::map<VariantKey, int> variant;  // (window shapes, tile) -> fused variant | chunk << 8
    std::map<VariantKey, GraphEntry> graphs;
    void *scratch = nullptr;                   // device address of the static scratch array
    hipError_t scratch_err = hipErrorNotReady;  // why it is NULL
};

namespace {

int check_opts(const gsl_opts *o)
{
    if (!o) return fail(GSL_EINVAL, "opts is NULL");
    if (o->tile != 8 && o->tile != 16 && o->tile != 32)
        return fail(GSL_ENOTSUP, "tile size %d not in {8, 16, 32}", o->tile);
    if (!(o->alpha_min > 0.f) || !(o->alpha_max > o->alpha_min) || !(o->alpha_max < 1.f))
        return fail(GSL_EINVAL, "need 0 < alpha_min < alpha_max < 1");
    if (!(o->T_min > 0.f) || !(o->T_min < 1.f)) return fail(GSL_EINVAL, "need 0 < T_min < 1");
    if (!(o->near_z > 0.f)) return fail(GSL_EINVAL, "need near_z > 0");
    if (!(o->eps2d >= 0.f)) return fail(GSL_EINVAL, "need eps2d >= 0");
    if (!(o->guard >= 0.f)) return fail(GSL_EINVAL, "need guard >= 0");
    if (o->chunk != 0 && o->chunk != 64 && o->chunk != 128 && o->chunk != 256)
        return fail(GSL_EINVAL, "chunk %d not in {0, 64, 128, 256}", o->chunk);
    return GSL_OK;
}

DevOpts dev_opts(const gsl_opts *o)
{
    DevOpts d;
    d.near_z = o->near_z;
    d.eps2d = o->eps2d;
    d.alpha_min = o->alpha_min;
    d.alpha_max = o->alpha_max;
    d.T_min = o->T_min;
    for (int k = 0; k < 3; k++) d.bg[k] = o->bg[k];
    d.guard = o->guard;
    d.tile = o->tile;
    return d;
}

int make_layout(const gsl_camera *cams, int32_t C, int32_t N, int32_t tile, Layout &L, std::vector<DevCam> *dc)
{
    if (!cams) return fail(GSL_EINVAL, "cams is NULL");
    if (C < 1 || C > GSL_MAX_CAMERAS) return fail(GSL_ENOTSUP, "camera count %d not in [1, %d]", C, GSL_MAX_CAMERAS);
    if (N < 0) return fail(GSL_EINVAL, "negative Gaussian count");
    if (N > (int32_t)kGidMask) return fail(GSL_EINVAL, "N = %d exceeds 2^28 - 1", N);
    if (tile != 8 && tile != 16 && tile != 32) return fail(GSL_ENOTSUP, "tile size %d not in {8, 16, 32}", tile);
    L.C = C;
    L.N = N;
    L.M = (int64_t)C * N;
    if (L.M > 0xffffffffll) return fail(GSL_EINVAL, "C*N = %lld exceeds 2^32-1", (long long)L.M);
    L.tile = tile;
    int64_t T = 0, P = 0;
    if (dc) dc->resize(C);
    for (int c = 0; c < C; c++) {
        const gsl_camera &k = cams[c];
        if (k.width < 1 || k.height < 1 || k.width > 32767 || k.height > 32767)
            return fail(GSL_EINVAL, "camera %d size %dx%d out of range", c, k.width, k.height);
        if (!(k.fx > 0.f) || !(k.fy > 0.f)) return fail(GSL_EINVAL, "camera %d focal length must be > 0", c);
        const int tx = (k.width + tile - 1) / tile, ty = (k.height + tile - 1) / tile;
        if (dc) {
            DevCam &d = (*dc)[c];
            d.fx = k.fx; d.fy = k.fy; d.cx = k.cx; d.cy = k.cy;
            d.W = k.width; d.H = k.height;
            for (int j = 0; j < 9; j++) d.R[j] = k.R_cw[j];
            for (int j = 0; j < 3; j++) d.t[j] = k.t_cw[j];
            d.tiles_x = tx; d.tiles_y = ty;
            d.tile_offset = (int32_t)T;
            d.pad = 0;
            d.pix_offset = P;
        }
        T += (int64_t)tx * ty;
        P += (int64_t)k.width * k.height;
    }
    if (T > 0x7fffffffll) return fail(GSL_EINVAL, "too many tiles");
    L.T_total = T;
    L.P_total = P;
    L.tile_bits = ceil_log2(T);
    return GSL_OK;
}

WsLayout ws_layout(const Layout &L, int64_t capacity)
{
    WsLayout w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    const int64_t M = L.M;
    w.cams = take(sizeof(DevCam) * (size_t)L.C);
    w.dkey = take(4 * (size_t)M);
    w.dval = take(4 * (size_t)M);
    w.dkey2 = take(4 * (size_t)M);
    w.dval2 = take(4 * (size_t)M);
    w.counts = take(4 * (size_t)M);
    w.offsets = take(4 * (size_t)M);
    w.ikey2 = take(4 * (size_t)capacity);
    w.ival2 = take(4 * (size_t)capacity);
    const int64_t nb = (std::max<int64_t>(M, capacity) + kSortTile - 1) / kSortTile;
    w.sort_blocks = nb;
    w.hist = take(4 * (size_t)(256 * nb + 1));
    w.hist_off = take(4 * (size_t)(256 * nb + 1));
    const int64_t scan_n = std::max<int64_t>(256 * nb, M);
    w.scan_partials = (scan_n + kScanTile - 1) / kScanTile + 1;
    w.partial = take(8 * (size_t)w.scan_partials);
    w.rs_totals = take(4 * 256);
    w.g2d = take(4 * (size_t)M * kG2);
    w.pose_blocks = (int32_t)((L.N + kPoseThreads - 1) / kPoseThreads);
    w.pose_part = take(8 * (size_t)std::max<int64_t>(1, (int64_t)w.pose_blocks * L.C * 6));
    w.pose_part_sh = take(8 * (size_t)std::max<int64_t>(1, (int64_t)w.pose_blocks * L.C * 6));
    w.loss_part = take(8 * (size_t)std::max<int64_t>(1, L.T_total));
    w.order = take(4 * (size_t)std::max<int64_t>(1, L.T_total));
    w.big = take(4 * (size_t)std::max<int64_t>(1, M));
    w.misc = take(256);
    w.total = o;
    return w;
}

template <typename T>
T *at(void *ws, size_t off)
{
    return reinterpret_cast<T *>(static_cast<char *>(ws) + off);
}

struct Prepared {
    Layout L;
    WsLayout W;
    std::vector<DevCam> dc;
    DevOpts o;
};

int check_device(const gsl_ctx *ctx)
{
    int cur = -1;
    GSL_TRY(check_hip(hipGetDevice(&cur), "hipGetDevice"));
    if (cur != ctx->device) return fail(GSL_ESTATE, "current device %d is not the context's device %d", cur, ctx->device);
    return GSL_OK;
}

int prepare(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts, int64_t capacity,
            void *ws, size_t ws_bytes, Prepared &p)
{
    if (!ctx) return fail(GSL_EINVAL, "ctx is NULL");
    GSL_TRY(check_opts(opts));
    if (capacity < 0 || capacity > 0xffffffffll) return fail(GSL_EINVAL, "capacity_K out of range");
    GSL_TRY(make_layout(cams, C, N, opts->tile, p.L, &p.dc));
    p.W = ws_layout(p.L, capacity);
    p.o = dev_opts(opts);
    if (!ws) return fail(GSL_EINVAL, "workspace is NULL");
    if (ws_bytes < p.W.total)
        return fail(GSL_EINVAL, "workspace too small: %zu < %zu bytes", ws_bytes, p.W.total);
    return check_device(ctx);
}

// Scratch regions of the backward pass alone (camera table, 2D gradients,
// pose partials), for gsl_render_bwd_noalloc.
WsLayout bwd_scratch_layout(const Layout &L)
{
    WsLayout w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    w.cams = take(sizeof(DevCam) * (size_t)L.C);
    w.g2d = take(4 * (size_t)L.M * kG2);
    w.pose_blocks = (int32_t)((L.N + kPoseThreads - 1) / kPoseThreads);
    w.pose_part = take(8 * (size_t)std::max<int64_t>(1, (int64_t)w.pose_blocks * L.C * 6));
    w.pose_part_sh = take(8 * (size_t)std::max<int64_t>(1, (int64_t)w.pose_blocks * L.C * 6));
    w.loss_part = take(8);
    w.order = take(4);
    w.misc = take(256);
    w.total = o;
    return w;
}

int check_gauss(const gsl_gaussians *g, bool need_all)
{
    if (!g) return fail(GSL_EINVAL, "gaussians is NULL");
    if (g->N < 0) return fail(GSL_EINVAL, "negative Gaussian count");
    if (g->N > 0 && (!g->mean || !g->scale || !g->quat || (need_all && (!g->opacity || !g->color))))
        return fail(GSL_EINVAL, "Gaussian parameter pointer is NULL");
    if (g->sh_degree < 0 || g->sh_degree > 3) return fail(GSL_EINVAL, "sh_degree %d not in [0, 3]", g->sh_degree);
    if (g->sh_degree > 0 && g->N > 0 && need_all && !g->sh) return fail(GSL_EINVAL, "sh is NULL");
    return GSL_OK;
}

int check_proj(const gsl_proj *p, const Layout &L)
{
    if (!p) return fail(GSL_EINVAL, "proj is NULL");
    if (L.M > 0 && (!p->splats || !p->tiles_touched || !p->binrecs || !p->depth_keys))
        return fail(GSL_EINVAL, "proj buffer is NULL");
    if (reinterpret_cast<uintptr_t>(p->binrecs) % 32 != 0) return fail(GSL_EINVAL, "binrecs not 32-byte aligned");
    return GSL_OK;
}

int check_bins(const gsl_bins *b)
{
    if (!b) return fail(GSL_EINVAL, "bins is NULL");
    if (!b->ranges || !b->d_K || !b->d_status) return fail(GSL_EINVAL, "bins buffer is NULL");
    if (b->capacity_K > 0 && (!b->tile_ids || !b->gauss_ids)) return fail(GSL_EINVAL, "bins instance buffer is NULL");
    return GSL_OK;
}

// ---- step bodies (enqueue only) ----

void do_upload(const Prepared &p, void *ws, hipStream_t s)
{
    launch_upload_cams(at<DevCam>(ws, p.W.cams), p.dc.data(), p.L.C, s);
}

// With clear_g2d (the fused window step) the projection also clears the
// 2D-gradient records the compositing kernel accumulates into.
void do_project(const Prepared &p, const gsl_gaussians *g, gsl_proj *out, void *ws, hipStream_t s,
                bool clear_g2d = false)
{
    launch_project(*g, at<DevCam>(ws, p.W.cams), p.L, p.o, out->splats, out->binrecs, out->depth_keys,
                   out->tiles_touched,
                   at<uint32_t>(ws, p.W.big), at<uint32_t>(ws, p.W.misc + 128), s,
                   clear_g2d ? at<float>(ws, p.W.g2d) : nullptr, clear_g2d ? at<uint32_t>(ws, p.W.misc) : nullptr);
}

void do_bin_sort(const Prepared &p, const gsl_proj *proj, gsl_bins *bins, void *ws, hipStream_t s)
{
    const Layout &L = p.L;
    const WsLayout &W = p.W;
    uint32_t *dkey = at<uint32_t>(ws, W.dkey), *dval = at<uint32_t>(ws, W.dval);
    uint32_t *dkey2 = at<uint32_t>(ws, W.dkey2), *dval2 = at<uint32_t>(ws, W.dval2);
    uint32_t *hist = at<uint32_t>(ws, W.hist), *hist_off = at<uint32_t>(ws, W.hist_off);
    uint64_t *partial = at<uint64_t>(ws, W.partial);
    // 1. depth order of the records that reach a tile (ties by record index =
    // Gaussian index per camera); the first pass reads the projection's depth
    // keys and tile counts directly and drops the records that reach no tile,
    // the last pass also writes each kept record's tile count in depth order
    // (positions beyond the kept records are never read)
    int64_t *d_V = at<int64_t>(ws, W.misc + 64);
    uint32_t *counts = at<uint32_t>(ws, W.counts), *offsets = at<uint32_t>(ws, W.offsets);
    uint32_t *totals = at<uint32_t>(ws, W.rs_totals);
    DepthSortIO io;
    io.first_keys = proj->depth_keys;
    io.first_tiles = proj->tiles_touched;
    io.gather_tiles = proj->tiles_touched;
    io.counts_out = counts;
    io.zero_word = at<uint32_t>(ws, W.misc + 128);  // the emit's big-record counter
    // 2. instance offsets in that order (a one-workgroup sort scans them itself)
    io.offsets_out = offsets;
    io.d_total = bins->d_K;
    int where = launch_radix_sort(dkey, dval, dkey2, dval2, L.M, nullptr, 32, hist, hist_off, totals, s, d_V, &io);
    const uint32_t *order = where ? dval2 : dval;
    if (!radix_one_block(L.M)) launch_scan_u32(counts, offsets, L.M, partial, bins->d_K, s, d_V);
    // 3. emit and sort by tile; the pass count decides which buffer is emitted
    // into (a one-workgroup sort writes the other buffer, as one pass does)
    const int passes = L.tile_bits <= 0 ? 0 : radix_one_block(bins->capacity_K) ? 1 : (L.tile_bits + 7) / 8;
    uint32_t *ek = bins->tile_ids, *ev = bins->gauss_ids;
    uint32_t *ak = at<uint32_t>(ws, W.ikey2), *av = at<uint32_t>(ws, W.ival2);
    if (passes & 1) std::swap(ek, ak), std::swap(ev, av);
    launch_emit(order, offsets, counts, proj->binrecs, at<DevCam>(ws, W.cams), L, bins->d_K, bins->capacity_K, ek, ev,
                bins->d_status, at<uint32_t>(ws, W.big), at<uint32_t>(ws, W.misc + 128), d_V, s);
    // 4. per-tile ranges (a one-workgroup tile sort writes them itself)
    const bool one = L.tile_bits > 0 && radix_one_block(bins->capacity_K);
    launch_radix_sort(ek, ev, ak, av, bins->capacity_K, bins->d_K, L.tile_bits, hist, hist_off, totals, s, nullptr,
                      nullptr, one ? bins->ranges : nullptr, L.T_total);
    if (!one) launch_ranges(bins->tile_ids, bins->d_K, bins->capacity_K, L.T_total, bins->ranges, s);
}

RenderArgs render_args(const Prepared &p, const gsl_proj *proj, const gsl_bins *bins, void *ws)
{
    RenderArgs a;
    memset(&a, 0, sizeof a);
    a.cams = at<DevCam>(ws, p.W.cams);
    a.C = p.L.C;
    a.N = p.L.N;
    a.o = p.o;
    a.splats = proj->splats;
    a.gauss_ids = bins->gauss_ids;
    a.ranges = bins->ranges;
    a.T_total = p.L.T_total;
    a.g2d = at<float>(ws, p.W.g2d);
    a.loss_part = at<double>(ws, p.W.loss_part);
    a.queue = at<uint32_t>(ws, p.W.misc);
    return a;
}

void do_project_bwd(const Prepared &p, const gsl_gaussians *g, gsl_grads *grads, int accumulate, void *ws,
                    hipStream_t s)
{
    double *pose_part = at<double>(ws, p.W.pose_part);
    double *pose_part_sh = g->sh_degree > 0 ? at<double>(ws, p.W.pose_part_sh) : nullptr;
    launch_project_bwd(*g, at<DevCam>(ws, p.W.cams), p.L, p.o, at<float>(ws, p.W.g2d), *grads, accumulate,
                       pose_part, p.W.pose_blocks, s);
    launch_sh_bwd(*g, at<DevCam>(ws, p.W.cams), p.L, at<float>(ws, p.W.g2d), grads->g_sh, grads->g_mean, accumulate,
                  pose_part_sh, p.W.pose_blocks, s);
    if (grads->g_pose) {
        if (p.L.N == 0) {
            if (!accumulate) launch_fill_f64(grads->g_pose, 0.0, 6 * (int64_t)p.L.C, s);
        } else {
            launch_pose_reduce(pose_part, pose_part_sh, p.W.pose_blocks, p.L.C, grads->g_pose, accumulate, s);
        }
    }
}

// Enqueues the raster adjoint and the projection adjoint.  Everything of the
// scratch memory the kernels accumulate into is cleared here first: the 2D
// gradients by a fill kernel, the pose partials by the adjoint that writes
// every one of them.
void do_render_bwd(const Prepared &p, const gsl_gaussians *g, const gsl_proj *proj, const gsl_bins *bins,
                   const float *T_final, const uint32_t *n_walk, const float *dL_dimage, int accumulate,
                   gsl_grads *grads, void *ws, hipStream_t s)
{
    do_upload(p, ws, s);
    launch_fill_f32(at<float>(ws, p.W.g2d), 0.f, p.L.M * kG2, s);
    RenderArgs a = render_args(p, proj, bins, ws);
    a.T_final = const_cast<float *>(T_final);
    a.n_walk = const_cast<uint32_t *>(n_walk);
    a.dL_dimage = dL_dimage;
    launch_render_bwd(a, s);
    do_project_bwd(p, g, grads, accumulate, ws, s);
}

// Enqueues one window step.  With `timed`, HIP events are recorded on the
// stream between the stages (never while capturing a graph).
void do_window(gsl_ctx *ctx, const Prepared &p, const gsl_gaussians *g, const float *target, int loss,
               gsl_proj *proj, gsl_bins *bins, float *image, double *d_loss, gsl_grads *grads, void *ws, int variant,
               hipStream_t s, bool timed = false, bool upload = true)
{
    auto mark = [&](int k) {
        if (timed) (void)hipEventRecord(ctx->ev[k], s);
    };
    mark(kStProject);
    if (upload) do_upload(p, ws, s);
    // the projection also clears the 2D-gradient records and the persistent
    // kernel's work counter (with no records it launches nothing: fill here)
    do_project(p, g, proj, ws, s, true);
    mark(kStBinSort);
    do_bin_sort(p, proj, bins, ws, s);
    if (p.L.M == 0) launch_fill_u32(at<uint32_t>(ws, p.W.misc), 0u, 1, s);
    RenderArgs a = render_args(p, proj, bins, ws);
    a.image = image;
    a.target = target;
    a.loss = loss;
    if (variant & 2) {  // bit 1 of the variant: longest list first
        uint32_t *order = at<uint32_t>(ws, p.W.order);
        launch_order_by_length(bins->ranges, p.L.T_total, order, s);
        a.order = order;
    }
    mark(kStRender);
    launch_render_fused(a, variant & 0xff, variant >> 8, ctx->num_cus, s);
    mark(kStProjectBwd);
    launch_reduce_f64(at<double>(ws, p.W.loss_part), p.L.T_total, d_loss, s);
    do_project_bwd(p, g, grads, 0, ws, s);
    mark(kStages);
    if (timed) ctx->ev_recorded = true;
}

// LDS chunk depth a tile size uses unless tuned or set: one staged splat per
// lane of the workgroup.
int default_chunk(int tile) { return tile == 32 ? 256 : 64; }

VariantKey window_key(const Layout &L, const gsl_camera *cams);

// Fused-kernel launch configuration of a window, variant | chunk << 8: the
// tuned one for these shapes (else variant 0 and the tile's default chunk),
// with opts->chunk, when set, in place of the chunk.
int fused_config(gsl_ctx *ctx, const VariantKey &vk, const gsl_opts *opts)
{
    int cfg = default_chunk(opts->tile) << 8;
    {
        std::lock_guard<std::mutex> lk(ctx->mu);
        auto it = ctx->variant.find(vk);
        if (it != ctx->variant.end()) cfg = it->second;
    }
    if (opts->chunk) cfg = (cfg & 0xff) | (opts->chunk << 8);
    return cfg;
}

VariantKey window_key(const Layout &L, const gsl_camera *cams)
{
    VariantKey k;
    k.v = {L.C, L.N, L.tile};
    for (int c = 0; c < L.C; c++) {
        k.v.push_back(cams[c].width);
        k.v.push_back(cams[c].height);
    }
    return k;
}

// Records the work `enqueue(stream)` launches into a HIP graph cached under
// `key` (first call) and launches the graph on `s`.
template <typename F>
int graph_run(gsl_ctx *ctx, const VariantKey &key, hipStream_t s, F &&enqueue)
{
    std::lock_guard<std::mutex> lk(ctx->mu);
    auto it = ctx->graphs.find(key);
    if (it == ctx->graphs.end()) {
        GraphEntry e;
        hipStream_t cs = ctx->cap_stream;
        GSL_TRY(check_hip(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture"));
        enqueue(cs);
        hipError_t le = hipGetLastError();
        hipError_t ce = hipStreamEndCapture(cs, &e.graph);
        if (le != hipSuccess) return fail(GSL_EHIP, "launch during capture: %s", hipGetErrorString(le));
        GSL_TRY(check_hip(ce, "hipStreamEndCapture"));
        hipError_t ie = hipGraphInstantiate(&e.exec, e.graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            (void)hipGraphDestroy(e.graph);
            return fail(GSL_EHIP, "hipGraphInstantiate: %s", hipGetErrorString(ie));
        }
        if (ctx->graphs.size() > 64) {  // bound the cache
            for (auto &kv : ctx->graphs) {
                (void)hipGraphExecDestroy(kv.second.exec);
                (void)hipGraphDestroy(kv.second.graph);
            }
            ctx->graphs.clear();
        }
        it = ctx->graphs.emplace(key, e).first;
    }
    return check_hip(hipGraphLaunch(it->second.exec, s), "hipGraphLaunch");
}

// Graph key of a window pass: shapes (camera sizes are in vk), variant, loss,
// every pointer and the options.  Poses and intrinsics are not part of it:
// the graphs read the camera table from the workspace, which the caller
// uploads on the stream before each launch, so a new keyframe pose replays
// the same graph.
VariantKey window_graph_key(const VariantKey &vk, int variant, int loss, const gsl_gaussians *g, const float *target,
                            const gsl_proj *proj, const gsl_bins *bins, const float *image, const double *d_loss,
                            const gsl_grads *grads, const void *workspace, const gsl_opts *opts)
{
    VariantKey gk = vk;
    gk.v.push_back(variant);
    gk.v.push_back(loss);
    auto ptr = [&](const void *q) { gk.v.push_back((int64_t)(uintptr_t)q); };
    ptr(g->mean); ptr(g->scale); ptr(g->quat); ptr(g->opacity); ptr(g->color); ptr(g->sh);
    gk.v.push_back(g->sh_degree);
    ptr(target); ptr(proj->splats); ptr(proj->tiles_touched); ptr(proj->binrecs); ptr(proj->depth_keys);
    ptr(bins->tile_ids); ptr(bins->gauss_ids); ptr(bins->ranges); ptr(bins->d_K); ptr(bins->d_status);
    gk.v.push_back(bins->capacity_K);
    ptr(image); ptr(d_loss); ptr(grads->g_mean); ptr(grads->g_scale); ptr(grads->g_quat);
    ptr(grads->g_opacity); ptr(grads->g_color); ptr(grads->g_pose); ptr(grads->g_sh); ptr(workspace);
    const int32_t *ow = reinterpret_cast<const int32_t *>(opts);
    for (size_t k = 0; k < sizeof(gsl_opts) / 4; k++) gk.v.push_back(ow[k]);
    return gk;
}

int check_adam(const gsl_adam_state *st, const gsl_adam *hp)
{
    if (!st) return fail(GSL_EINVAL, "adam state is NULL");
    if (st->N < 0) return fail(GSL_EINVAL, "negative Gaussian count");
    if (st->N > 0 && (!st->raw || !st->m || !st->v || !st->d_step)) return fail(GSL_EINVAL, "adam buffer is NULL");
    if (st->ld != 0 && st->ld < st->N) return fail(GSL_EINVAL, "adam row stride %d < N %d", st->ld, st->N);
    if (st->sh_degree < 0 || st->sh_degree > 3) return fail(GSL_EINVAL, "sh_degree %d not in [0, 3]", st->sh_degree);
    if (hp) {
        if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f) || !(hp->beta2 >= 0.f && hp->beta2 < 1.f))
            return fail(GSL_EINVAL, "need 0 <= beta < 1");
        if (!(hp->eps > 0.f)) return fail(GSL_EINVAL, "need eps > 0");
        for (int k = 0; k < 5; k++)
            if (!(hp->lr[k] >= 0.f)) return fail(GSL_EINVAL, "learning rates must be >= 0");
        if (!(hp->lr_sh >= 0.f)) return fail(GSL_EINVAL, "learning rates must be >= 0");
    }
    return GSL_OK;
}

int64_t adam_ld(const gsl_adam_state *st) { return st->ld ? st->ld : st->N; }

void act_arrays(gsl_gaussians *act, float *out[6])
{
    out[0] = const_cast<float *>(act->mean);
    out[1] = const_cast<float *>(act->scale);
    out[2] = const_cast<float *>(act->quat);
    out[3] = const_cast<float *>(act->opacity);
    out[4] = const_cast<float *>(act->color);
    out[5] = const_cast<float *>(act->sh);
}

void do_adam(gsl_adam_state *st, const gsl_adam *hp, const gsl_grads *grads, gsl_gaussians *act, hipStream_t s)
{
    const float *g[6] = {grads->g_mean, grads->g_scale, grads->g_quat, grads->g_opacity, grads->g_color,
                         grads->g_sh};
    float *a[6];
    act_arrays(act, a);
    const float lr[6] = {hp->lr[0], hp->lr[1], hp->lr[2], hp->lr[3], hp->lr[4], hp->lr_sh};
    launch_adam(g, a, st->raw, st->m, st->v, st->d_step, lr, hp->beta1, hp->beta2, hp->eps, st->N, st->sh_degree,
                adam_ld(st), true, s);
}

// The optimiser state and the activated Gaussians describe the same window.
int check_adam_act(const gsl_adam_state *st, const gsl_gaussians *act, const gsl_grads *grads)
{
    if (act->N != st->N) return fail(GSL_EINVAL, "act.N %d != state N %d", act->N, st->N);
    if (act->sh_degree != st->sh_degree)
        return fail(GSL_EINVAL, "act.sh_degree %d != state sh_degree %d", act->sh_degree, st->sh_degree);
    if (grads && st->N > 0 &&
        (!grads->g_mean || !grads->g_scale || !grads->g_quat || !grads->g_opacity || !grads->g_color ||
         (st->sh_degree > 0 && !grads->g_sh)))
        return fail(GSL_EINVAL, "gradient buffer is NULL");
    return GSL_OK;
}

// Bytes gsl_pose_jacobian needs past the common workspace: per-record
// tangents, then per-item normal-equation partials.
size_t jvp_tangent_bytes(const Layout &L) { return align_up(4 * (size_t)kTangentSH * (size_t)L.M); }
size_t jvp_extra_bytes(const Layout &L)
{
    return jvp_tangent_bytes(L) + align_up(8 * (size_t)kNrm * (size_t)std::max<int64_t>(1, L.T_total));
}

// In-place Gauss-Jordan inverse of a 6x6 row-major matrix with partial
// pivoting; false when a pivot vanishes.
bool invert6(const double *A, double *X)
{
    double M[6][12];
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 12; c++) M[r][c] = c < 6 ? A[6 * r + c] : (c - 6 == r ? 1.0 : 0.0);
    for (int k = 0; k < 6; k++) {
        int piv = k;
        for (int r = k + 1; r < 6; r++)
            if (std::fabs(M[r][k]) > std::fabs(M[piv][k])) piv = r;
        if (!(std::fabs(M[piv][k]) > 0.0) || !std::isfinite(M[piv][k])) return false;
        if (piv != k)
            for (int c = 0; c < 12; c++) std::swap(M[k][c], M[piv][c]);
        const double inv = 1.0 / M[k][k];
        for (int c = 0; c < 12; c++) M[k][c] *= inv;
        for (int r = 0; r < 6; r++) {
            if (r == k) continue;
            const double f = M[r][k];
            if (f != 0.0)
                for (int c = 0; c < 12; c++) M[r][c] -= f * M[k][c];
        }
    }
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) X[6 * r + c] = M[r][6 + c];
    return true;
}

// Window-maintenance workspace: the header and the per-Gaussian arrays come
// first (their offsets depend on n only, so gsl_window_compact can find them
// without P), then the scan partials, the per-point arrays and the table.
constexpr int64_t kWinMaxPoints = (int64_t)1 << 28;

struct WinLayout {
    size_t hdr = 0, del = 0, drank = 0, evpos = 0, compact_end = 0;
    size_t partial = 0, pslot = 0, addf = 0, arank = 0, table = 0, total = 0;
    uint64_t slots = 0;
};

WinLayout win_layout(int64_t n, int64_t P)
{
    WinLayout w;
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t at = o;
        o = align_up(o + bytes);
        return at;
    };
    w.hdr = take(64);
    w.del = take(4 * (size_t)n);
    w.drank = take(4 * (size_t)n);
    w.evpos = take(4 * (size_t)n);
    w.compact_end = o;
    const int64_t nb = (std::max(n, P) + kScanTile - 1) / kScanTile;
    w.partial = take(8 * (size_t)std::max<int64_t>(nb, 1));
    w.pslot = take(4 * (size_t)P);
    w.addf = take(4 * (size_t)P);
    w.arank = take(4 * (size_t)P);
    w.slots = window_table_slots(P);
    w.table = take(16 * (size_t)w.slots);
    w.total = o;
    return w;
}

WinWs win_ws(void *ws, const WinLayout &l)
{
    char *b = static_cast<char *>(ws);
    WinWs w;
    w.hdr = reinterpret_cast<int64_t *>(b + l.hdr);
    w.del = reinterpret_cast<uint32_t *>(b + l.del);
    w.drank = reinterpret_cast<uint32_t *>(b + l.drank);
    w.evpos = reinterpret_cast<uint32_t *>(b + l.evpos);
    if (l.total) {
        w.partial = reinterpret_cast<uint64_t *>(b + l.partial);
        w.pslot = reinterpret_cast<uint32_t *>(b + l.pslot);
        w.addf = reinterpret_cast<uint32_t *>(b + l.addf);
        w.arank = reinterpret_cast<uint32_t *>(b + l.arank);
        w.table = b + l.table;
        w.slots = l.slots;
    }
    return w;
}

int check_device(gsl_ctx *ctx)
{
    int cur = -1;
    GSL_TRY(check_hip(hipGetDevice(&cur), "hipGetDevice"));
    if (cur != ctx->device) return fail(GSL_ESTATE, "current device %d is not the context's device %d", cur, ctx->device);
    return GSL_OK;
}

}  // namespace

// =====================================================================
extern "C" {

const char *gsl_last_error(void) { return g_err.c_str(); }

void gsl_default_opts(gsl_opts *o)
{
    if (!o) return;
    o->near_z = 0.2f;
    o->eps2d = 0.3f;
    o->alpha_min = 1.0f / 255.0f;
    o->alpha_max = 0.99f;
    o->T_min = 1e-4f;
    o->bg[0] = o->bg[1] = o->bg[2] = 0.f;
    o->guard = 0.15f;
    o->tile = 16;
    o->chunk = 0;
}

int gsl_create(gsl_ctx **out, int device)
{
    if (!out) return fail(GSL_EINVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    GSL_TRY(check_hip(hipGetDeviceCount(&n), "hipGetDeviceCount"));
    if (device < 0 || device >= n) return fail(GSL_EINVAL, "device %d not in [0, %d)", device, n);
    GSL_TRY(check_hip(hipSetDevice(device), "hipSetDevice"));
    gsl_ctx *c = new gsl_ctx();
    c->device = device;
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && cus > 0)
        c->num_cus = cus;
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        delete c;
        return fail(GSL_EHIP, "hipStreamCreateWithFlags failed");
    }
    // device address of the static scratch array (gsl_render_bwd_noalloc);
    // a failure here only disables that entry point
    c->scratch_err = static_scratch_address(device, &c->scratch);
    if (c->scratch_err != hipSuccess) c->scratch = nullptr;
    *out = c;
    g_err.clear();
    return GSL_OK;
}

int gsl_destroy(gsl_ctx *ctx)
{
    if (!ctx) return GSL_OK;
    (void)hipSetDevice(ctx->device);
    for (auto &kv : ctx->graphs) {
        if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
        if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
    }
    if (ctx->cap_stream) (void)hipStreamDestroy(ctx->cap_stream);
    for (auto &e : ctx->ev)
        if (e) (void)hipEventDestroy(e);
    delete ctx;
    return GSL_OK;
}

int gsl_layout(const gsl_camera *cams, int32_t C, int32_t tile, int64_t *T_total, int64_t *P_total)
{
    Layout L;
    GSL_TRY(make_layout(cams, C, 0, tile, L, nullptr));
    if (T_total) *T_total = L.T_total;
    if (P_total) *P_total = L.P_total;
    return GSL_OK;
}

int gsl_workspace_size(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                       int64_t capacity_K, size_t *bytes)
{
    (void)ctx;  // sizes depend on the shapes only
    if (!bytes) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_opts(opts));
    if (capacity_K < 0 || capacity_K > 0xffffffffll) return fail(GSL_EINVAL, "capacity_K out of range");
    Layout L;
    GSL_TRY(make_layout(cams, C, N, opts->tile, L, nullptr));
    *bytes = ws_layout(L, capacity_K).total;
    return GSL_OK;
}

int gsl_project(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                gsl_proj *out, void *workspace, size_t workspace_bytes, void *stream)
{
    GSL_TRY(check_gauss(g, true));
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, g->N, opts, 0, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(out, p.L));
    hipStream_t s = (hipStream_t)stream;
    do_upload(p, workspace, s);
    do_project(p, g, out, workspace, s);
    return check_launch("gsl_project");
}

int gsl_bin_sort(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                 const gsl_proj *proj, gsl_bins *bins, void *workspace, size_t workspace_bytes, void *stream)
{
    GSL_TRY(check_bins(bins));
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    hipStream_t s = (hipStream_t)stream;
    do_upload(p, workspace, s);
    do_bin_sort(p, proj, bins, workspace, s);
    return check_launch("gsl_bin_sort");
}

int gsl_render_fwd(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                   const gsl_proj *proj, const gsl_bins *bins, float *image, float *T_final, uint32_t *n_walk,
                   void *workspace, size_t workspace_bytes, void *stream)
{
    GSL_TRY(check_bins(bins));
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    if (!image || !T_final || !n_walk) return fail(GSL_EINVAL, "output buffer is NULL");
    hipStream_t s = (hipStream_t)stream;
    do_upload(p, workspace, s);
    RenderArgs a = render_args(p, proj, bins, workspace);
    a.image = image;
    a.T_final = T_final;
    a.n_walk = n_walk;
    launch_render_fwd(a, s);
    return check_launch("gsl_render_fwd");
}

int gsl_render_stats(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, const gsl_opts *opts,
                     const gsl_proj *proj, const gsl_bins *bins, uint64_t *d_counts, void *workspace,
                     size_t workspace_bytes, void *stream)
{
    GSL_TRY(check_bins(bins));
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    if (!d_counts) return fail(GSL_EINVAL, "d_counts is NULL");
    hipStream_t s = (hipStream_t)stream;
    do_upload(p, workspace, s);
    launch_fill_f64(reinterpret_cast<double *>(d_counts), 0.0, 3, s);  // all-zero bits
    RenderArgs a = render_args(p, proj, bins, workspace);
    launch_render_count(a, reinterpret_cast<unsigned long long *>(d_counts), s);
    return check_launch("gsl_render_stats");
}

int gsl_render_bwd(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                   const gsl_proj *proj, const gsl_bins *bins, const float *T_final, const uint32_t *n_walk,
                   const float *dL_dimage, int accumulate, gsl_grads *grads, void *workspace, size_t workspace_bytes,
                   void *stream)
{
    GSL_TRY(check_gauss(g, false));
    GSL_TRY(check_bins(bins));
    if (!grads) return fail(GSL_EINVAL, "grads is NULL");
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, g->N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    if (!T_final || !n_walk || !dL_dimage) return fail(GSL_EINVAL, "input buffer is NULL");
    do_render_bwd(p, g, proj, bins, T_final, n_walk, dL_dimage, accumulate, grads, workspace, (hipStream_t)stream);
    return check_launch("gsl_render_bwd");
}

int gsl_render_bwd_noalloc(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C,
                           const gsl_opts *opts, const gsl_proj *proj, const gsl_bins *bins, const float *T_final,
                           const uint32_t *n_walk, const float *dL_dimage, int accumulate, gsl_grads *grads,
                           void *stream)
{
    if (!ctx) return fail(GSL_EINVAL, "ctx is NULL");
    GSL_TRY(check_gauss(g, false));
    GSL_TRY(check_bins(bins));
    if (!grads) return fail(GSL_EINVAL, "grads is NULL");
    GSL_TRY(check_opts(opts));
    Prepared p;
    GSL_TRY(make_layout(cams, C, g->N, opts->tile, p.L, &p.dc));
    p.W = bwd_scratch_layout(p.L);
    p.o = dev_opts(opts);
    if (p.W.total > kStaticScratchBytes)
        return fail(GSL_EINVAL, "%d cameras x %d Gaussians need %zu bytes of scratch; the static array holds %zu",
                    C, g->N, p.W.total, kStaticScratchBytes);
    GSL_TRY(check_proj(proj, p.L));
    if (!T_final || !n_walk || !dL_dimage) return fail(GSL_EINVAL, "input buffer is NULL");
    GSL_TRY(check_device(ctx));
    if (!ctx->scratch)
        return fail(GSL_EHIP, "static scratch array unavailable: %s", hipGetErrorString(ctx->scratch_err));
    do_render_bwd(p, g, proj, bins, T_final, n_walk, dL_dimage, accumulate, grads, ctx->scratch, (hipStream_t)stream);
    return check_launch("gsl_render_bwd_noalloc");
}

int gsl_window_step(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                    const float *target, int loss, gsl_proj *proj, gsl_bins *bins, float *image, double *d_loss,
                    gsl_grads *grads, void *workspace, size_t workspace_bytes, int use_graph, void *stream)
{
    GSL_TRY(check_gauss(g, true));
    GSL_TRY(check_bins(bins));
    if (!grads || !target || !d_loss) return fail(GSL_EINVAL, "NULL argument");
    if (loss != GSL_LOSS_L1 && loss != GSL_LOSS_L2) return fail(GSL_EINVAL, "unknown loss %d", loss);
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, g->N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    hipStream_t s = (hipStream_t)stream;
    const VariantKey vk = window_key(p.L, cams);
    const int variant = fused_config(ctx, vk, opts);
    if (!use_graph) {
        do_window(ctx, p, g, target, loss, proj, bins, image, d_loss, grads, workspace, variant, s, ctx->profile);
        return check_launch("gsl_window_step");
    }
    VariantKey gk = window_graph_key(vk, variant, loss, g, target, proj, bins, image, d_loss, grads, workspace, opts);
    // a profiled step is its own graph, with the stage events as event-record nodes
    const bool timed = ctx->profile;
    gk.v.push_back(timed ? 1 : 0);
    do_upload(p, workspace, s);
    const int rc = graph_run(ctx, gk, s, [&](hipStream_t cs) {
        do_window(ctx, p, g, target, loss, proj, bins, image, d_loss, grads, workspace, variant, cs, timed, false);
    });
    if (rc == GSL_OK && timed) ctx->ev_recorded = true;  // also when the graph came from the cache
    return rc;
}

int gsl_window_render(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                      gsl_proj *proj, gsl_bins *bins, float *image, float *T_final, uint32_t *n_walk,
                      void *workspace, size_t workspace_bytes, int use_graph, void *stream)
{
    GSL_TRY(check_gauss(g, true));
    GSL_TRY(check_bins(bins));
    if (!image || !T_final || !n_walk) return fail(GSL_EINVAL, "output buffer is NULL");
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, g->N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    hipStream_t s = (hipStream_t)stream;
    // the kernels of gsl_project, gsl_bin_sort and gsl_render_fwd, in order
    auto body = [&](hipStream_t cs) {
        do_project(p, g, proj, workspace, cs);
        do_bin_sort(p, proj, bins, workspace, cs);
        RenderArgs a = render_args(p, proj, bins, workspace);
        a.image = image;
        a.T_final = T_final;
        a.n_walk = n_walk;
        launch_render_fwd(a, cs);
    };
    do_upload(p, workspace, s);  // the camera table, outside the graph (poses are not in the key)
    if (!use_graph) {
        body(s);
        return check_launch("gsl_window_render");
    }
    VariantKey gk = window_key(p.L, cams);
    gk.v.push_back(-2);  // forward-render graphs (window-step keys continue with a variant >= 0)
    auto ptr = [&](const void *q) { gk.v.push_back((int64_t)(uintptr_t)q); };
    ptr(g->mean); ptr(g->scale); ptr(g->quat); ptr(g->opacity); ptr(g->color); ptr(g->sh);
    gk.v.push_back(g->sh_degree);
    ptr(proj->splats); ptr(proj->tiles_touched); ptr(proj->binrecs); ptr(proj->depth_keys);
    ptr(bins->tile_ids); ptr(bins->gauss_ids); ptr(bins->ranges); ptr(bins->d_K); ptr(bins->d_status);
    gk.v.push_back(bins->capacity_K);
    ptr(image); ptr(T_final); ptr(n_walk); ptr(workspace);
    const int32_t *ow = reinterpret_cast<const int32_t *>(opts);
    for (size_t k = 0; k < sizeof(gsl_opts) / 4; k++) gk.v.push_back(ow[k]);
    return graph_run(ctx, gk, s, body);
}

int gsl_graph_count(gsl_ctx *ctx, int64_t *count)
{
    if (!ctx || !count) return fail(GSL_EINVAL, "NULL argument");
    std::lock_guard<std::mutex> lk(ctx->mu);
    *count = (int64_t)ctx->graphs.size();
    return GSL_OK;
}

int gsl_window_variant(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N, int32_t tile, int32_t variant,
                       int32_t chunk)
{
    if (!ctx) return fail(GSL_EINVAL, "ctx is NULL");
    if (variant < 0 || variant >= kVariants) return fail(GSL_EINVAL, "variant %d not in [0, %d)", variant, kVariants);
    if (chunk != 0 && chunk != 64 && chunk != 128 && chunk != 256)
        return fail(GSL_EINVAL, "chunk %d not in {0, 64, 128, 256}", chunk);
    Layout L;
    GSL_TRY(make_layout(cams, C, N, tile, L, nullptr));
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->variant[window_key(L, cams)] = variant | ((chunk ? chunk : default_chunk(tile)) << 8);
    return GSL_OK;
}

int gsl_profile(gsl_ctx *ctx, int enable)
{
    if (!ctx) return fail(GSL_EINVAL, "ctx is NULL");
    if (enable && !ctx->ev[0])
        for (auto &e : ctx->ev) GSL_TRY(check_hip(hipEventCreate(&e), "hipEventCreate"));
    ctx->profile = enable != 0;
    ctx->ev_recorded = false;
    return GSL_OK;
}

int gsl_profile_read(gsl_ctx *ctx, float *ms, int32_t n)
{
    if (!ctx || !ms) return fail(GSL_EINVAL, "NULL argument");
    if (!ctx->ev_recorded) return fail(GSL_ESTATE, "no profiled window step has been enqueued");
    GSL_TRY(check_hip(hipEventSynchronize(ctx->ev[kStages]), "hipEventSynchronize"));
    for (int k = 0; k < kStages && k < n; k++)
        GSL_TRY(check_hip(hipEventElapsedTime(&ms[k], ctx->ev[k], ctx->ev[k + 1]), "hipEventElapsedTime"));
    if (n > kStages) GSL_TRY(check_hip(hipEventElapsedTime(&ms[kStages], ctx->ev[0], ctx->ev[kStages]),
                                       "hipEventElapsedTime"));
    return GSL_OK;
}

int gsl_window_tune(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, gsl_opts *opts_inout,
                    const float *target, int loss, gsl_proj *proj, gsl_bins *bins, double *d_loss, gsl_grads *grads,
                    void *workspace, size_t workspace_bytes, float *times_ms, int32_t ntimes, void *stream)
{
    GSL_TRY(check_gauss(g, true));
    GSL_TRY(check_bins(bins));
    if (!grads || !target || !d_loss || !opts_inout) return fail(GSL_EINVAL, "NULL argument");
    if (loss != GSL_LOSS_L1 && loss != GSL_LOSS_L2) return fail(GSL_EINVAL, "unknown loss %d", loss);
    hipStream_t s = (hipStream_t)stream;
    hipEvent_t e0, e1;
    GSL_TRY(check_hip(hipEventCreate(&e0), "hipEventCreate"));
    GSL_TRY(check_hip(hipEventCreate(&e1), "hipEventCreate"));
    const int tiles[3] = {8, 16, 32};
    float best_all = 1e30f;
    int best_tile = opts_inout->tile;
    int k = 0;
    int rc = GSL_OK;
    for (int ti = 0; ti < 3 && rc == GSL_OK; ti++) {
        gsl_opts o = *opts_inout;
        o.tile = tiles[ti];
        Prepared p;
        rc = prepare(ctx, cams, C, g->N, &o, bins->capacity_K, workspace, workspace_bytes, p);
        if (rc != GSL_OK) break;
        rc = check_proj(proj, p.L);
        if (rc != GSL_OK) break;
        float best = 1e30f;
        int best_v = 0;
        for (int cv = 0; cv < 3 * kVariants; cv++) {
            const int variant = (cv % kVariants) | ((64 << (cv / kVariants)) << 8);
            // one untimed run, then check the capacity status
            do_window(ctx, p, g, target, loss, proj, bins, nullptr, d_loss, grads, workspace, variant, s);
            int32_t status = 0;
            (void)hipMemcpyAsync(&status, bins->d_status, 4, hipMemcpyDeviceToHost, s);
            if ((rc = check_hip(hipStreamSynchronize(s), "tune sync")) != GSL_OK) break;
            if (status != GSL_OK) {
                rc = fail(GSL_ECAPACITY, "capacity_K too small for tile %d", tiles[ti]);
                break;
            }
            // the status read left the GPU idle, and its clock takes some ten
            // steps to come back: time only after untimed steps
            for (int r = 0; r < 6; r++)
                do_window(ctx, p, g, target, loss, proj, bins, nullptr, d_loss, grads, workspace, variant, s);
            const int reps = 8;
            (void)hipEventRecord(e0, s);
            for (int r = 0; r < reps; r++)
                do_window(ctx, p, g, target, loss, proj, bins, nullptr, d_loss, grads, workspace, variant, s);
            (void)hipEventRecord(e1, s);
            if ((rc = check_hip(hipEventSynchronize(e1), "tune event")) != GSL_OK) break;
            float ms = 0;
            (void)hipEventElapsedTime(&ms, e0, e1);
            ms /= reps;
            if (times_ms && k < ntimes) times_ms[k] = ms;
            k++;
            if (ms < best) {
                best = ms;
                best_v = variant;
            }
        }
        if (rc != GSL_OK) break;
        {
            std::lock_guard<std::mutex> lk(ctx->mu);
            ctx->variant[window_key(p.L, cams)] = best_v;
        }
        if (best < best_all) {
            best_all = best;
            best_tile = tiles[ti];
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc != GSL_OK) return rc;
    opts_inout->tile = best_tile;
    return check_launch("gsl_window_tune");
}

int gsl_adam_activate(gsl_ctx *ctx, const gsl_adam_state *st, gsl_gaussians *act, void *stream)
{
    if (!ctx || !act) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_adam(st, nullptr));
    GSL_TRY(check_adam_act(st, act, nullptr));
    GSL_TRY(check_gauss(act, true));
    float *a[6];
    act_arrays(act, a);
    launch_adam(nullptr, a, st->raw, nullptr, nullptr, nullptr, nullptr, 0.f, 0.f, 1.f, st->N, st->sh_degree,
                adam_ld(st), false, (hipStream_t)stream);
    return check_launch("gsl_adam_activate");
}

int gsl_adam_init(gsl_ctx *ctx, const gsl_gaussians *act, gsl_adam_state *st, void *stream)
{
    if (!ctx || !act) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_adam(st, nullptr));
    if (!st->d_step) return fail(GSL_EINVAL, "adam step counter is NULL");
    GSL_TRY(check_adam_act(st, act, nullptr));
    GSL_TRY(check_gauss(act, true));
    const float *a[6] = {act->mean, act->scale, act->quat, act->opacity, act->color, act->sh};
    launch_adam_init(a, st->raw, st->m, st->v, st->d_step, st->N, st->sh_degree, adam_ld(st), (hipStream_t)stream);
    return check_launch("gsl_adam_init");
}

int gsl_adam_step(gsl_ctx *ctx, gsl_adam_state *st, const gsl_adam *hp, const gsl_grads *grads, gsl_gaussians *act,
                  void *stream)
{
    if (!ctx || !act || !hp || !grads) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_adam(st, hp));
    GSL_TRY(check_adam_act(st, act, grads));
    GSL_TRY(check_gauss(act, true));
    do_adam(st, hp, grads, act, (hipStream_t)stream);
    return check_launch("gsl_adam_step");
}

int gsl_window_optimize(gsl_ctx *ctx, gsl_adam_state *st, const gsl_adam *hp, gsl_gaussians *act,
                        const gsl_camera *cams, int32_t C, const gsl_opts *opts, const float *target, int loss,
                        gsl_proj *proj, gsl_bins *bins, double *d_losses, gsl_grads *grads, int32_t iters,
                        void *workspace, size_t workspace_bytes, int use_graph, void *stream)
{
    if (!act || !hp) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_adam(st, hp));
    GSL_TRY(check_gauss(act, true));
    GSL_TRY(check_bins(bins));
    if (!grads || !target || !d_losses) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_adam_act(st, act, grads));
    if (!grads->g_mean || !grads->g_scale || !grads->g_quat || !grads->g_opacity || !grads->g_color)
        return fail(GSL_EINVAL, "gradient buffer is NULL");
    if (loss != GSL_LOSS_L1 && loss != GSL_LOSS_L2) return fail(GSL_EINVAL, "unknown loss %d", loss);
    if (iters < 1 || iters > 1000) return fail(GSL_EINVAL, "iters %d not in [1, 1000]", iters);
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, act->N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    hipStream_t s = (hipStream_t)stream;
    const VariantKey vk = window_key(p.L, cams);
    const int variant = fused_config(ctx, vk, opts);
    // the camera table is uploaded once; the iterations read it from the workspace
    do_upload(p, workspace, s);
    auto enqueue = [&](hipStream_t q) {
        for (int k = 0; k < iters; k++) {
            do_window(ctx, p, act, target, loss, proj, bins, nullptr, d_losses + k, grads, workspace, variant, q,
                      false, false);
            do_adam(st, hp, grads, act, q);
        }
    };
    if (!use_graph) {
        enqueue(s);
        return check_launch("gsl_window_optimize");
    }
    VariantKey gk = window_graph_key(vk, variant, loss, act, target, proj, bins, nullptr, d_losses, grads,
                                     workspace, opts);
    gk.v.push_back(-1);  // a separator from the single-step keys
    gk.v.push_back(iters);
    for (const void *q : {(const void *)st->raw, (const void *)st->m, (const void *)st->v, (const void *)st->d_step})
        gk.v.push_back((int64_t)(uintptr_t)q);
    gk.v.push_back(adam_ld(st));
    gk.v.push_back(st->sh_degree);
    const int32_t *hw = reinterpret_cast<const int32_t *>(hp);
    for (size_t k = 0; k < sizeof(gsl_adam) / 4; k++) gk.v.push_back(hw[k]);
    return graph_run(ctx, gk, s, enqueue);
}

int gsl_window_workspace_size(int32_t n, int32_t P, size_t *bytes)
{
    if (!bytes) return fail(GSL_EINVAL, "NULL argument");
    if (n < 0 || P < 0 || P > kWinMaxPoints) return fail(GSL_EINVAL, "need n >= 0 and 0 <= P <= 2^28");
    *bytes = win_layout(n, P).total;
    return GSL_OK;
}

int gsl_color_init(gsl_ctx *ctx, const float *mean, int64_t mean_ld, int32_t n, const gsl_camera *cam,
                   const float *image, const gsl_opts *opts, float *color, int64_t color_ld, uint8_t *valid,
                   void *stream)
{
    if (!ctx || !cam) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_opts(opts));
    if (n < 0) return fail(GSL_EINVAL, "negative count");
    if (n > 0 && (!mean || !image || !color)) return fail(GSL_EINVAL, "NULL argument");
    if (mean_ld < n || color_ld < n) return fail(GSL_EINVAL, "row strides must be >= n");
    if (cam->width <= 0 || cam->height <= 0) return fail(GSL_EINVAL, "empty image");
    GSL_TRY(check_device(ctx));
    launch_color_init(mean, mean_ld, n, *cam, opts->near_z, image, color, color_ld, valid, (hipStream_t)stream);
    return check_launch("gsl_color_init");
}

int gsl_voxel_keys(gsl_ctx *ctx, const float *xyz, int32_t P, int64_t point_stride, int64_t axis_stride,
                   float voxel_size, uint64_t *keys, void *stream)
{
    if (!ctx) return fail(GSL_EINVAL, "NULL argument");
    if (P < 0) return fail(GSL_EINVAL, "negative point count");
    if (P > 0 && (!xyz || !keys)) return fail(GSL_EINVAL, "NULL argument");
    if (point_stride < 0 || axis_stride < 0) return fail(GSL_EINVAL, "negative stride");
    if (!(voxel_size > 0.f) || !std::isfinite(voxel_size)) return fail(GSL_EINVAL, "voxel_size must be finite and > 0");
    GSL_TRY(check_device(ctx));
    launch_voxel_keys(xyz, P, point_stride, axis_stride, voxel_size, keys, (hipStream_t)stream);
    return check_launch("gsl_voxel_keys");
}

int gsl_window_classify(gsl_ctx *ctx, const float *points, int32_t P, float voxel_size, const uint64_t *keys,
                        int32_t n, int32_t *counts, uint64_t *add_keys, void *workspace, size_t workspace_bytes,
                        void *stream)
{
    if (!ctx || !counts || !workspace) return fail(GSL_EINVAL, "NULL argument");
    if (n < 0 || P < 0 || P > kWinMaxPoints) return fail(GSL_EINVAL, "need n >= 0 and 0 <= P <= 2^28");
    if (P > 0 && !points) return fail(GSL_EINVAL, "points is NULL");
    if (n > 0 && !keys) return fail(GSL_EINVAL, "keys is NULL");
    if (!(voxel_size > 0.f) || !std::isfinite(voxel_size)) return fail(GSL_EINVAL, "voxel_size must be finite and > 0");
    if ((uintptr_t)workspace % 256) return fail(GSL_EINVAL, "workspace must be 256-byte aligned");
    const WinLayout l = win_layout(n, P);
    if (workspace_bytes < l.total)
        return fail(GSL_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes, l.total);
    GSL_TRY(check_device(ctx));
    launch_window_classify(points, P, voxel_size, keys, n, win_ws(workspace, l), counts, add_keys,
                           (hipStream_t)stream);
    return check_launch("gsl_window_classify");
}

int gsl_window_compact(gsl_ctx *ctx, uint64_t *keys, float *rows, int32_t R, int64_t ld, int32_t n, int32_t D,
                       const uint64_t *add_keys, const float *add_rows, int32_t A, uint64_t *evicted_keys,
                       float *evicted_rows, const void *workspace, size_t workspace_bytes, int32_t *status,
                       void *stream)
{
    if (!ctx || !workspace) return fail(GSL_EINVAL, "NULL argument");
    if (R < 0 || n < 0 || A < 0) return fail(GSL_EINVAL, "negative size");
    if (D < 0 || D > n) return fail(GSL_EINVAL, "D %d not in [0, n = %d]", D, n);
    if (ld < (int64_t)n || (int64_t)n - D + A > ld)
        return fail(GSL_EINVAL, "row stride %lld too small for n = %d, n - D + A = %lld", (long long)ld, n,
                    (long long)n - D + A);
    if ((n > 0 || A > 0) && !keys) return fail(GSL_EINVAL, "keys is NULL");
    if (R > 0 && (n > 0 || A > 0) && !rows) return fail(GSL_EINVAL, "rows is NULL");
    if (A > 0 && (!add_keys || (R > 0 && !add_rows))) return fail(GSL_EINVAL, "added Gaussians are NULL");
    if ((uintptr_t)workspace % 256) return fail(GSL_EINVAL, "workspace must be 256-byte aligned");
    WinLayout l = win_layout(n, 0);
    if (workspace_bytes < l.compact_end)
        return fail(GSL_EINVAL, "workspace too small: %zu < %zu bytes", workspace_bytes, l.compact_end);
    l.total = 0;  // only the header and the per-Gaussian arrays are used
    GSL_TRY(check_device(ctx));
    launch_window_compact(keys, rows, R, ld, n, D, add_keys, add_rows, A, evicted_keys, evicted_rows,
                          win_ws(const_cast<void *>(workspace), l), status, (hipStream_t)stream);
    return check_launch("gsl_window_compact");
}

namespace {

// Is p (not NULL) memory of the wanted kind: pinned host memory, or device
// memory?  Pageable host memory reports no attributes or an unregistered
// type.
bool is_memory(const void *p, bool host)
{
    hipPointerAttribute_t at;
    if (hipPointerGetAttributes(&at, p) != hipSuccess) {
        (void)hipGetLastError();  // clear the error the query left for pageable memory
        return false;
    }
    return host ? at.type == hipMemoryTypeHost : at.type == hipMemoryTypeDevice;
}

}  // namespace

int gsl_window_transfer(gsl_ctx *ctx, int dir, const uint64_t *src_keys, const float *src_rows, int64_t src_ld,
                        uint64_t *dst_keys, float *dst_rows, int64_t dst_ld, int32_t R, int32_t count, void *stream)
{
    if (!ctx) return fail(GSL_EINVAL, "ctx is NULL");
    if (dir != GSL_D2H && dir != GSL_H2D) return fail(GSL_EINVAL, "direction %d is not GSL_D2H or GSL_H2D", dir);
    if (R < 0 || count < 0) return fail(GSL_EINVAL, "negative size");
    if (!src_keys != !dst_keys) return fail(GSL_EINVAL, "keys: source and destination must both be given or both NULL");
    if (!src_rows != !dst_rows) return fail(GSL_EINVAL, "rows: source and destination must both be given or both NULL");
    const bool rows = src_rows && R > 0;
    if (rows && (src_ld < count || dst_ld < count)) return fail(GSL_EINVAL, "row strides must be >= count");
    if (count == 0) return GSL_OK;
    GSL_TRY(check_device(ctx));
    const bool src_host = dir == GSL_H2D;
    const void *srcs[2] = {src_keys, rows ? (const void *)src_rows : nullptr};
    const void *dsts[2] = {dst_keys, rows ? (const void *)dst_rows : nullptr};
    for (int k = 0; k < 2; k++) {
        if (srcs[k] && !is_memory(srcs[k], src_host))
            return fail(GSL_EINVAL, "source %s is not %s", k ? "rows" : "keys", src_host ? "pinned host memory" : "device memory");
        if (dsts[k] && !is_memory(dsts[k], !src_host))
            return fail(GSL_EINVAL, "destination %s is not %s", k ? "rows" : "keys",
                        src_host ? "device memory" : "pinned host memory");
    }
    hipStream_t s = (hipStream_t)stream;
    const hipMemcpyKind kind = src_host ? hipMemcpyHostToDevice : hipMemcpyDeviceToHost;
    if (src_keys) GSL_TRY(check_hip(hipMemcpyAsync(dst_keys, src_keys, 8 * (size_t)count, kind, s), "hipMemcpyAsync"));
    if (rows)
        GSL_TRY(check_hip(hipMemcpy2DAsync(dst_rows, 4 * (size_t)dst_ld, src_rows, 4 * (size_t)src_ld, 4 * (size_t)count,
                                           (size_t)R, kind, s),
                          "hipMemcpy2DAsync"));
    return GSL_OK;
}

int gsl_pose_jacobian_workspace_size(gsl_ctx *ctx, const gsl_camera *cams, int32_t C, int32_t N,
                                     const gsl_opts *opts, int64_t capacity_K, size_t *bytes)
{
    (void)ctx;  // sizes depend on the shapes only
    if (!bytes) return fail(GSL_EINVAL, "NULL argument");
    GSL_TRY(check_opts(opts));
    if (capacity_K < 0 || capacity_K > 0xffffffffll) return fail(GSL_EINVAL, "capacity_K out of range");
    Layout L;
    GSL_TRY(make_layout(cams, C, N, opts->tile, L, nullptr));
    *bytes = ws_layout(L, capacity_K).total + jvp_extra_bytes(L);
    return GSL_OK;
}

int gsl_pose_jacobian(gsl_ctx *ctx, const gsl_gaussians *g, const gsl_camera *cams, int32_t C, const gsl_opts *opts,
                      const gsl_proj *proj, const gsl_bins *bins, const float *target, const float *weight,
                      float *image, float *jac, double *HtH, double *Htz, double *zz, void *workspace,
                      size_t workspace_bytes, void *stream)
{
    GSL_TRY(check_gauss(g, false));
    if (g->sh_degree > 0 && g->N > 0 && !g->sh) return fail(GSL_EINVAL, "sh is NULL");
    GSL_TRY(check_bins(bins));
    Prepared p;
    GSL_TRY(prepare(ctx, cams, C, g->N, opts, bins->capacity_K, workspace, workspace_bytes, p));
    GSL_TRY(check_proj(proj, p.L));
    const size_t need = p.W.total + jvp_extra_bytes(p.L);
    if (workspace_bytes < need)
        return fail(GSL_EINVAL, "workspace too small for the pose Jacobian: %zu < %zu bytes", workspace_bytes, need);
    const bool normal = HtH || Htz || zz;
    if (normal && !target) return fail(GSL_EINVAL, "the normal equations need the target image");
    hipStream_t s = (hipStream_t)stream;
    do_upload(p, workspace, s);
    float *tangent = at<float>(workspace, p.W.total);
    double *part = at<double>(workspace, p.W.total + jvp_tangent_bytes(p.L));
    launch_project_tangent(*g, at<DevCam>(workspace, p.W.cams), p.L, p.o, proj->tiles_touched, tangent, s);
    RenderArgs a = render_args(p, proj, bins, workspace);
    a.image = image;
    a.target = normal ? target : nullptr;
    a.weight = weight;
    a.jac = jac;
    a.tangent = tangent;
    a.sh_colour = g->sh_degree > 0;
    a.P_total = p.L.P_total;
    a.nrm_part = normal ? part : nullptr;
    launch_render_jvp(a, s);
    if (normal) launch_normal_reduce(part, at<DevCam>(workspace, p.W.cams), p.L.C, HtH, Htz, zz, s);
    return check_launch("gsl_pose_jacobian");
}

int gsl_imu_to_camera_twist(const double R_CI[9], const double t_CI[3], const double R_CW[9], double A[36])
{
    if (!R_CI || !t_CI || !R_CW || !A) return fail(GSL_EINVAL, "NULL argument");
    for (int k = 0; k < 36; k++) A[k] = 0.0;
    // dphi_cam = -R_CI dphi_imu
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) A[6 * r + c] = -R_CI[3 * r + c];
    // dt_cam = t_CI^ dphi_cam - R_CW dt_imu = -(t_CI^ R_CI) dphi_imu - R_CW dt_imu
    const double tx[9] = {0.0, -t_CI[2], t_CI[1], t_CI[2], 0.0, -t_CI[0], -t_CI[1], t_CI[0], 0.0};
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double v = 0.0;
            for (int k = 0; k < 3; k++) v += tx[3 * r + k] * R_CI[3 * k + c];
            A[6 * (3 + r) + c] = -v;
            A[6 * (3 + r) + 3 + c] = -R_CW[3 * r + c];
        }
    return GSL_OK;
}

int gsl_ieskf_pose_update(const double HtRH[36], const double HtRz[6], const double P[36], const double dx_prior[6],
                          double delta[6], double P_post[36])
{
    if (!HtRH || !HtRz || !P || !delta || !P_post) return fail(GSL_EINVAL, "NULL argument");
    double Pinv[36], S[36], Sinv[36], KH[36], IKH[36];
    if (!invert6(P, Pinv)) return fail(GSL_EINVAL, "prior covariance is singular");
    for (int k = 0; k < 36; k++) S[k] = HtRH[k] + Pinv[k];
    if (!invert6(S, Sinv)) return fail(GSL_EINVAL, "H^T R^-1 H + P^-1 is singular");
    // K H = S^-1 H^T R^-1 H,  K z = S^-1 H^T R^-1 z
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) {
            double v = 0.0;
            for (int k = 0; k < 6; k++) v += Sinv[6 * r + k] * HtRH[6 * k + c];
            KH[6 * r + c] = v;
            IKH[6 * r + c] = (r == c ? 1.0 : 0.0) - v;
        }
    for (int r = 0; r < 6; r++) {
        double kz = 0.0, px = 0.0;
        for (int k = 0; k < 6; k++) {
            kz += Sinv[6 * r + k] * HtRz[k];
            if (dx_prior) px += IKH[6 * r + k] * dx_prior[k];
        }
        delta[r] = -kz - px;
    }
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) {
            double v = 0.0;
            for (int k = 0; k < 6; k++) v += IKH[6 * r + k] * P[6 * k + c];
            P_post[6 * r + c] = v;
        }
    return GSL_OK;
}

int gsl_ieskf_visual_update(const double HtH_cam[36], const double Htz_cam[6], const double A[36], double noise_var,
                            const double P[36], const double dx_prior[6], double delta[6], double P_post[36])
{
    if (!HtH_cam || !Htz_cam || !A) return fail(GSL_EINVAL, "NULL argument");
    if (!(noise_var > 0.0) || !std::isfinite(noise_var)) return fail(GSL_EINVAL, "noise variance must be finite and > 0");
    // H_imu = H_cam A:  H_imu^T R^-1 H_imu = A^T (H_cam^T H_cam) A / var,  H_imu^T R^-1 z = A^T (H_cam^T z) / var
    double HA[36], HtRH[36], HtRz[6];
    for (int r = 0; r < 6; r++)
        for (int c = 0; c < 6; c++) {
            double v = 0.0;
            for (int k = 0; k < 6; k++) v += HtH_cam[6 * r + k] * A[6 * k + c];
            HA[6 * r + c] = v;
        }
    for (int r = 0; r < 6; r++) {
        for (int c = 0; c < 6; c++) {
            double v = 0.0;
            for (int k = 0; k < 6; k++) v += A[6 * k + r] * HA[6 * k + c];
            HtRH[6 * r + c] = v / noise_var;
        }
        double z = 0.0;
        for (int k = 0; k < 6; k++) z += A[6 * k + r] * Htz_cam[k];
        HtRz[r] = z / noise_var;
    }
    return gsl_ieskf_pose_update(HtRH, HtRz, P, dx_prior, delta, P_post);
}

int gsl_valu_probe(gsl_ctx *ctx, int32_t mode, float *d_sink, double *insts_per_cu_cycle)
{
    if (!ctx || !d_sink || !insts_per_cu_cycle) return fail(GSL_EINVAL, "NULL argument");
    if (mode < 0 || mode > 4) return fail(GSL_EINVAL, "probe mode %d not in [0, 4]", mode);
    GSL_TRY(check_device(ctx));
    if (!is_memory(d_sink, false)) return fail(GSL_EINVAL, "d_sink is not device memory");
    if (run_valu_probe(mode, ctx->num_cus, d_sink, insts_per_cu_cycle) != 0)
        return fail(GSL_EHIP, "probe launch or timing failed");
    return check_launch("gsl_valu_probe");
}

}  // extern "C"
