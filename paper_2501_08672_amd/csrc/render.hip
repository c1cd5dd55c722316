// Front-to-back alpha compositing (eq. eq:raster) and its hand-written
// adjoint (eq. eq:gaussian_optimization), per (camera, tile) work item.
//
// One workgroup owns one tile of TS x TS pixels, one lane per pixel.  The
// tile's depth-ordered instance list is staged through LDS in chunks of up to
// TS*TS splats (48 B each, loaded as three float4 by one lane per splat) and
// every lane walks the chunk from LDS with broadcast reads.  A per-workgroup
// vote ends the walk once every pixel is done.
//
// Per pixel (centre x = (u + 0.5, v + 0.5)):
//   power = -1/2 |L (x - mu)|^2,  alpha = min(alpha_max, sigma exp(power))
//   alpha < alpha_min          -> skip
//   T (1 - alpha) < T_min      -> stop before this Gaussian
//   C += alpha T c,  T *= 1 - alpha
//
// The backward pass stores nothing beyond T_final and the walk length per
// pixel: it walks the same list from the back, recovers T before each
// contributor by dividing by (1 - alpha), and carries the suffix
// S = sum_{j>k} c_j alpha_j T_j + T_final bg, so that
//   dI/dc_k = alpha_k T_k,  dI/dalpha_k = T_k c_k - S / (1 - alpha_k).
// The nine 2D gradients of a Gaussian are summed over the 64 lanes of a wave
// (skipped when no lane contributed) and added with one float atomic per
// value per wave into the per-(camera, Gaussian) record.
//
// The fused kernel runs forward, the per-pixel loss gradient against a target
// image (L1 or L2, local to the pixel) and the backward walk in one pass over
// each item, keeping T, the walk length and the colour in registers.  Its
// persistent variant launches a few workgroups per CU that pull items from an
// atomic counter.
#include "common.hpp"

namespace gsl {

namespace {

constexpr float kLog2e = 1.4426950408889634f;

__device__ __forceinline__ float exp_fast(float x) { return __builtin_amdgcn_exp2f(x * kLog2e); }
__device__ __forceinline__ float rcp_fast(float x) { return __builtin_amdgcn_rcpf(x); }

__device__ __forceinline__ int find_cam(const DevCam *__restrict__ cams, int C, int t)
{
    int lo = 0, hi = C - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (cams[mid].tile_offset <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

struct TileInfo {
    int c;
    int W, H;
    int px, py;
    bool inside;
    uint32_t rs, re;
    int64_t pix;       // packed pixel index of this lane
    int64_t plane0;    // float offset of this camera's image
    int64_t npix;      // W * H
};

template <int TS>
__device__ __forceinline__ TileInfo tile_info(const RenderArgs &a, int t)
{
    TileInfo ti;
    ti.c = find_cam(a.cams, a.C, t);
    const DevCam &cam = a.cams[ti.c];
    ti.W = cam.W;
    ti.H = cam.H;
    const int local = t - cam.tile_offset;
    const int ty = local / cam.tiles_x, tx = local - ty * cam.tiles_x;
    ti.px = tx * TS + (int)(threadIdx.x % TS);
    ti.py = ty * TS + (int)(threadIdx.x / TS);
    ti.inside = ti.px < ti.W && ti.py < ti.H;
    ti.rs = a.ranges[2 * (int64_t)t];
    ti.re = a.ranges[2 * (int64_t)t + 1];
    ti.npix = (int64_t)ti.W * ti.H;
    ti.pix = cam.pix_offset + (int64_t)ti.py * ti.W + ti.px;
    ti.plane0 = 3 * cam.pix_offset;
    return ti;
}

template <int BS>
struct Stage {
    float4 p0[BS];  // mx, my, l11, l12
    float4 p1[BS];  // l22, opacity, r, g
    float p2[BS];   // b
    uint32_t gid[BS];
};

template <int BS>
__device__ __forceinline__ void stage_load(Stage<BS> &st, const RenderArgs &a, const gsl_splat *__restrict__ rec,
                                           uint32_t k, uint32_t end)
{
    if (k < end) {
        const uint32_t gid = a.gauss_ids[k];
        const float4 *r4 = reinterpret_cast<const float4 *>(rec + gid);
        st.p0[threadIdx.x] = r4[0];
        st.p1[threadIdx.x] = r4[1];
        st.p2[threadIdx.x] = r4[2].x;
        st.gid[threadIdx.x] = gid;
    }
}

struct PixState {
    float T;
    float C0, C1, C2;
    uint32_t nwalk;
};

// Forward walk over the tile list; every lane of the workgroup must call it.
template <int TS>
__device__ __forceinline__ PixState fwd_walk(const RenderArgs &a, const TileInfo &ti, Stage<TS * TS> &st)
{
    constexpr int BS = TS * TS;
    const gsl_splat *rec = a.splats + (int64_t)ti.c * a.N;
    const float fx = ti.px + 0.5f, fy = ti.py + 0.5f;
    const float amin = a.o.alpha_min, amax = a.o.alpha_max, Tmin = a.o.T_min;
    PixState ps{1.f, 0.f, 0.f, 0.f, 0u};
    bool done = !ti.inside;
    for (uint32_t start = ti.rs; start < ti.re; start += BS) {
        if (__syncthreads_count(done) == BS) break;
        stage_load<BS>(st, a, rec, start + threadIdx.x, ti.re);
        __syncthreads();
        const int cnt = (int)min((uint32_t)BS, ti.re - start);
        for (int j = 0; !done && j < cnt; j++) {
            const float4 p0 = st.p0[j];
            const float4 p1 = st.p1[j];
            const float dx = fx - p0.x, dy = fy - p0.y;
            const float t1 = p0.z * dx + p0.w * dy, t2 = p1.x * dy;
            const float alpha = fminf(amax, p1.y * exp_fast(-0.5f * (t1 * t1 + t2 * t2)));
            if (alpha < amin) continue;
            const float Tn = ps.T * (1.f - alpha);
            if (Tn < Tmin) {
                done = true;
                break;
            }
            const float w = alpha * ps.T;
            ps.C0 += w * p1.z;
            ps.C1 += w * p1.w;
            ps.C2 += w * st.p2[j];
            ps.T = Tn;
            ps.nwalk = start + (uint32_t)j + 1u - ti.rs;
        }
    }
    return ps;
}

__device__ __forceinline__ float wave_sum(float v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// Backward walk.  T is the final transmittance, v the cotangent of the pixel.
template <int TS>
__device__ __forceinline__ void bwd_walk(const RenderArgs &a, const TileInfo &ti, Stage<TS * TS> &st, float T,
                                         uint32_t nwalk, float v0, float v1, float v2, uint32_t *s_max)
{
    constexpr int BS = TS * TS;
    const gsl_splat *rec = a.splats + (int64_t)ti.c * a.N;
    float *g2d = a.g2d + (int64_t)ti.c * a.N * kG2;
    const float fx = ti.px + 0.5f, fy = ti.py + 0.5f;
    const float amin = a.o.alpha_min, amax = a.o.alpha_max;
    const int lane = threadIdx.x & (kWave - 1);
    float S0 = T * a.o.bg[0], S1 = T * a.o.bg[1], S2 = T * a.o.bg[2];
    if (!ti.inside) nwalk = 0;
    if (nwalk > ti.re - ti.rs) nwalk = ti.re - ti.rs;  // never walk past the tile's list
    __syncthreads();
    if (threadIdx.x == 0) *s_max = 0;
    __syncthreads();
    if (nwalk) atomicMax(s_max, nwalk);
    __syncthreads();
    const uint32_t maxn = *s_max;
    const int64_t lo = ti.rs;
    for (int64_t end = lo + maxn; end > lo; end -= BS) {
        const int64_t start = end - BS > lo ? end - BS : lo;
        __syncthreads();
        stage_load<BS>(st, a, rec, (uint32_t)(start + threadIdx.x), (uint32_t)end);
        __syncthreads();
        for (int j = (int)(end - start) - 1; j >= 0; j--) {
            const uint32_t pos = (uint32_t)(start - lo) + (uint32_t)j;
            float g[kG2];
#pragma unroll
            for (int f = 0; f < kG2; f++) g[f] = 0.f;
            bool contrib = false;
            if (pos < nwalk) {
                const float4 p0 = st.p0[j];
                const float4 p1 = st.p1[j];
                const float dx = fx - p0.x, dy = fy - p0.y;
                const float t1 = p0.z * dx + p0.w * dy, t2 = p1.x * dy;
                const float G = exp_fast(-0.5f * (t1 * t1 + t2 * t2));
                const float s = p1.y * G;
                const float alpha = fminf(amax, s);
                if (alpha >= amin) {
                    contrib = true;
                    const float r = rcp_fast(1.f - alpha);
                    T = T * r;  // transmittance before this Gaussian
                    const float w = alpha * T;
                    const float c0 = p1.z, c1 = p1.w, c2 = st.p2[j];
                    g[6] = w * v0;
                    g[7] = w * v1;
                    g[8] = w * v2;
                    const float ga = v0 * (T * c0 - S0 * r) + v1 * (T * c1 - S1 * r) + v2 * (T * c2 - S2 * r);
                    S0 += c0 * w;
                    S1 += c1 * w;
                    S2 += c2 * w;
                    if (s < amax) {
                        g[5] = G * ga;
                        const float gp = s * ga;
                        g[0] = gp * (p0.z * t1);
                        g[1] = gp * (p0.w * t1 + p1.x * t2);
                        g[2] = -0.5f * gp * dx * dx;
                        g[3] = -gp * dx * dy;
                        g[4] = -0.5f * gp * dy * dy;
                    }
                }
            }
            if (__ballot(contrib) != 0ull) {
#pragma unroll
                for (int f = 0; f < kG2; f++) g[f] = wave_sum(g[f]);
                if (lane == 0) {
                    float *dst = g2d + (int64_t)st.gid[j] * kG2;
#pragma unroll
                    for (int f = 0; f < kG2; f++)
                        if (g[f] != 0.f) unsafeAtomicAdd(dst + f, g[f]);
                }
            }
        }
    }
}

template <int TS>
__global__ __launch_bounds__(TS *TS) void k_render_fwd(RenderArgs a)
{
    __shared__ Stage<TS * TS> st;
    const TileInfo ti = tile_info<TS>(a, (int)blockIdx.x);
    const PixState ps = fwd_walk<TS>(a, ti, st);
    if (!ti.inside) return;
    const int64_t off = (int64_t)ti.py * ti.W + ti.px;
    a.image[ti.plane0 + off] = ps.C0 + ps.T * a.o.bg[0];
    a.image[ti.plane0 + ti.npix + off] = ps.C1 + ps.T * a.o.bg[1];
    a.image[ti.plane0 + 2 * ti.npix + off] = ps.C2 + ps.T * a.o.bg[2];
    a.T_final[ti.pix] = ps.T;
    a.n_walk[ti.pix] = ps.nwalk;
}

template <int TS>
__global__ __launch_bounds__(TS *TS) void k_render_bwd(RenderArgs a)
{
    __shared__ Stage<TS * TS> st;
    __shared__ uint32_t s_max;
    const TileInfo ti = tile_info<TS>(a, (int)blockIdx.x);
    float T = 1.f, v0 = 0.f, v1 = 0.f, v2 = 0.f;
    uint32_t nw = 0;
    if (ti.inside) {
        const int64_t off = (int64_t)ti.py * ti.W + ti.px;
        T = a.T_final[ti.pix];
        nw = a.n_walk[ti.pix];
        v0 = a.dL_dimage[ti.plane0 + off];
        v1 = a.dL_dimage[ti.plane0 + ti.npix + off];
        v2 = a.dL_dimage[ti.plane0 + 2 * ti.npix + off];
    }
    bwd_walk<TS>(a, ti, st, T, nw, v0, v1, v2, &s_max);
}

// Forward, per-pixel loss and its gradient, backward for one item.
template <int TS>
__device__ __forceinline__ void fused_item(const RenderArgs &a, int t, Stage<TS * TS> &st, uint32_t *s_max,
                                           float *s_loss)
{
    constexpr int BS = TS * TS;
    const TileInfo ti = tile_info<TS>(a, t);
    const PixState ps = fwd_walk<TS>(a, ti, st);
    float v0 = 0.f, v1 = 0.f, v2 = 0.f, lpix = 0.f;
    if (ti.inside) {
        const int64_t off = (int64_t)ti.py * ti.W + ti.px;
        const float I0 = ps.C0 + ps.T * a.o.bg[0];
        const float I1 = ps.C1 + ps.T * a.o.bg[1];
        const float I2 = ps.C2 + ps.T * a.o.bg[2];
        if (a.image) {
            a.image[ti.plane0 + off] = I0;
            a.image[ti.plane0 + ti.npix + off] = I1;
            a.image[ti.plane0 + 2 * ti.npix + off] = I2;
        }
        const float r0 = I0 - a.target[ti.plane0 + off];
        const float r1 = I1 - a.target[ti.plane0 + ti.npix + off];
        const float r2 = I2 - a.target[ti.plane0 + 2 * ti.npix + off];
        if (a.loss == GSL_LOSS_L1) {
            const float inv = 1.f / (3.f * (float)ti.npix);
            auto sgn = [](float x) { return x > 0.f ? 1.f : (x < 0.f ? -1.f : 0.f); };
            v0 = sgn(r0) * inv;
            v1 = sgn(r1) * inv;
            v2 = sgn(r2) * inv;
            lpix = (fabsf(r0) + fabsf(r1) + fabsf(r2)) * inv;
        } else {
            v0 = r0;
            v1 = r1;
            v2 = r2;
            lpix = 0.5f * (r0 * r0 + r1 * r1 + r2 * r2);
        }
    }
    // per-item loss partial
    float ls = wave_sum(lpix);
    if ((threadIdx.x & (kWave - 1)) == 0) s_loss[threadIdx.x / kWave] = ls;
    __syncthreads();
    if (threadIdx.x == 0) {
        double tot = 0;
        for (int w = 0; w < (BS + kWave - 1) / kWave; w++) tot += s_loss[w];
        a.loss_part[t] = tot;
    }
    bwd_walk<TS>(a, ti, st, ps.T, ps.nwalk, v0, v1, v2, s_max);
}

template <int TS>
__global__ __launch_bounds__(TS *TS) void k_render_fused(RenderArgs a)
{
    __shared__ Stage<TS * TS> st;
    __shared__ uint32_t s_max;
    __shared__ float s_loss[(TS * TS + kWave - 1) / kWave];
    const int t = a.order ? (int)a.order[blockIdx.x] : (int)blockIdx.x;
    fused_item<TS>(a, t, st, &s_max, s_loss);
}

template <int TS>
__global__ __launch_bounds__(TS *TS) void k_render_fused_persistent(RenderArgs a)
{
    __shared__ Stage<TS * TS> st;
    __shared__ uint32_t s_max;
    __shared__ uint32_t s_item;
    __shared__ float s_loss[(TS * TS + kWave - 1) / kWave];
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0) s_item = atomicAdd(a.queue, 1u);
        __syncthreads();
        const uint32_t item = s_item;
        if (item >= (uint32_t)a.T_total) break;
        const int t = a.order ? (int)a.order[item] : (int)item;
        fused_item<TS>(a, t, st, &s_max, s_loss);
    }
}

__global__ __launch_bounds__(256) void k_reduce_f64(const double *__restrict__ part, int64_t n, double *__restrict__ out)
{
    __shared__ double s[256 / kWave];
    double acc = 0;
    for (int64_t k = threadIdx.x; k < n; k += 256) acc += part[k];
    for (int off = 32; off > 0; off >>= 1) acc += __shfl_xor(acc, off, kWave);
    if ((threadIdx.x & 63) == 0) s[threadIdx.x / kWave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0;
        for (int w = 0; w < 256 / kWave; w++) t += s[w];
        *out = t;
    }
}

template <int TS>
void launch_fwd_t(const RenderArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_render_fwd<TS>, dim3((unsigned)a.T_total), dim3(TS * TS), 0, s, a);
}
template <int TS>
void launch_bwd_t(const RenderArgs &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_render_bwd<TS>, dim3((unsigned)a.T_total), dim3(TS * TS), 0, s, a);
}
template <int TS>
void launch_fused_t(const RenderArgs &a, int variant, int num_cus, hipStream_t s)
{
    if (variant == 1) {
        const int per_cu = TS == 8 ? 8 : (TS == 16 ? 4 : 1);
        int64_t g = (int64_t)num_cus * per_cu;
        if (g > a.T_total) g = a.T_total;
        hipLaunchKernelGGL(k_render_fused_persistent<TS>, dim3((unsigned)g), dim3(TS * TS), 0, s, a);
    } else {
        hipLaunchKernelGGL(k_render_fused<TS>, dim3((unsigned)a.T_total), dim3(TS * TS), 0, s, a);
    }
}

}  // namespace

void launch_render_fwd(const RenderArgs &a, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_fwd_t<8>(a, s); break;
    case 16: launch_fwd_t<16>(a, s); break;
    default: launch_fwd_t<32>(a, s); break;
    }
}

void launch_render_bwd(const RenderArgs &a, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_bwd_t<8>(a, s); break;
    case 16: launch_bwd_t<16>(a, s); break;
    default: launch_bwd_t<32>(a, s); break;
    }
}

void launch_render_fused(const RenderArgs &a, int variant, int num_cus, hipStream_t s)
{
    if (a.T_total == 0) return;
    switch (a.o.tile) {
    case 8: launch_fused_t<8>(a, variant, num_cus, s); break;
    case 16: launch_fused_t<16>(a, variant, num_cus, s); break;
    default: launch_fused_t<32>(a, variant, num_cus, s); break;
    }
}

void launch_reduce_f64(const double *part, int64_t n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_reduce_f64, dim3(1), dim3(256), 0, s, part, n, out);
}

}  // namespace gsl
