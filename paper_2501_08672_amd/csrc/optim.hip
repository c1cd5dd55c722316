// Adam over the map parameters (Sec. II-B: the Gaussian map is refined with
// the Adam optimiser on the photometric loss of eq. eq:gaussian_optimization).
//
// The optimiser owns the raw parameters, 14 rows of N floats at a row stride
// ld (a window kept at a fixed capacity uses the capacity): mean (3),
// log-scale (3), quaternion (4), opacity logit (1), colour (3), then the 3K
// higher-order SH coefficients of a view-dependent colour; the renderer
// takes the activated values, scale = exp(log-scale) and opacity =
// sigmoid(logit), the other rows unchanged.  One lane per Gaussian: the
// gradients of the activated values are chained to the raw rows, the moments
// and the raw values are updated, and the new activated values are written
// for the next pass.  The step count lives in device memory and is advanced by
// a second one-lane kernel, so a captured graph of several iterations (or its
// replays) uses the right bias corrections.
#include "sh.hpp"

namespace gsl {

namespace {

struct AdamArgs {
    const float *g[6];      // gradients of the activated mean, scale, quaternion, opacity, colour, SH
    float *act[6];          // activated outputs, same layout
    float *raw, *m, *v;     // [14 + 3K][ld]
    const int32_t *d_step;  // steps taken so far
    float lr[6];
    float beta1, beta2, eps;
    int N;
    int rows;               // 14 + 3K
    int64_t ld;
    bool update;            // false: only write the activated values of raw
};

constexpr int kBaseRows = 14;
constexpr int kMaxRows = kBaseRows + 3 * kShMaxK;
constexpr int kRowGroup[14] = {0, 0, 0, 1, 1, 1, 2, 2, 2, 2, 3, 4, 4, 4};
constexpr int kRowInGroup[14] = {0, 1, 2, 0, 1, 2, 0, 1, 2, 3, 0, 0, 1, 2};
__host__ __device__ constexpr int row_group(int r) { return r < kBaseRows ? kRowGroup[r] : 5; }
__host__ __device__ constexpr int row_in_group(int r) { return r < kBaseRows ? kRowInGroup[r] : r - kBaseRows; }

__global__ __launch_bounds__(256) void k_adam(AdamArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int64_t N = a.N, ld = a.ld;
    float bc1 = 1.f, bc2 = 1.f;
    if (a.update) {
        const float t = (float)(*a.d_step + 1);
        bc1 = 1.f - powf(a.beta1, t);
        bc2 = 1.f - powf(a.beta2, t);
    }
#pragma unroll
    for (int r = 0; r < kMaxRows; r++) {
        if (r >= a.rows) break;
        const int grp = row_group(r), k = row_in_group(r);
        float x = a.raw[r * ld + i];
        if (a.update) {
            float g = a.g[grp][k * N + i];
            if (grp == 1) {
                g *= expf(x);  // d exp(u) / du
            } else if (grp == 3) {
                const float s = 1.f / (1.f + expf(-x));
                g *= s * (1.f - s);  // d sigmoid(u) / du
            }
            const float m = fmaf(a.beta1, a.m[r * ld + i], (1.f - a.beta1) * g);
            const float v = fmaf(a.beta2, a.v[r * ld + i], (1.f - a.beta2) * g * g);
            a.m[r * ld + i] = m;
            a.v[r * ld + i] = v;
            x -= a.lr[grp] * (m / bc1) / (sqrtf(v / bc2) + a.eps);
            a.raw[r * ld + i] = x;
        }
        float y = x;
        if (grp == 1) y = expf(x);
        else if (grp == 3) y = 1.f / (1.f + expf(-x));
        a.act[grp][k * N + i] = y;
    }
}

__global__ void k_step_advance(int32_t *d_step) { *d_step += 1; }

// Starting point of the optimisation: raw <- inverse activation of the
// activated parameters (log-scale = ln s, opacity logit = ln(o / (1 - o)),
// the other rows as they are), both moments zero.
__global__ __launch_bounds__(256) void k_adam_init(AdamArgs a)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.N) return;
    const int64_t N = a.N, ld = a.ld;
#pragma unroll
    for (int r = 0; r < kMaxRows; r++) {
        if (r >= a.rows) break;
        const int grp = row_group(r), k = row_in_group(r);
        const float y = a.g[grp][k * N + i];
        float x = y;
        if (grp == 1) x = logf(y);
        else if (grp == 3) x = logf(y / (1.f - y));
        a.raw[r * ld + i] = x;
        a.m[r * ld + i] = 0.f;
        a.v[r * ld + i] = 0.f;
    }
}

__global__ void k_step_reset(int32_t *d_step) { *d_step = 0; }

}  // namespace

void launch_adam(const float *const g[6], float *const act[6], float *raw, float *m, float *v, const int32_t *d_step,
                 const float lr[6], float beta1, float beta2, float eps, int N, int sh_degree, int64_t ld,
                 bool update, hipStream_t s)
{
    if (N == 0) return;
    AdamArgs a;
    for (int k = 0; k < 6; k++) {
        a.g[k] = g ? g[k] : nullptr;
        a.act[k] = act[k];
        a.lr[k] = lr ? lr[k] : 0.f;
    }
    a.rows = kBaseRows + 3 * sh_count(sh_degree);
    a.raw = raw;
    a.m = m;
    a.v = v;
    a.d_step = d_step;
    a.beta1 = beta1;
    a.beta2 = beta2;
    a.eps = eps;
    a.N = N;
    a.ld = ld;
    a.update = update;
    hipLaunchKernelGGL(k_adam, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a);
    if (update) hipLaunchKernelGGL(k_step_advance, dim3(1), dim3(1), 0, s, const_cast<int32_t *>(d_step));
}

void launch_adam_init(const float *const act[6], float *raw, float *m, float *v, int32_t *d_step, int N,
                      int sh_degree, int64_t ld, hipStream_t s)
{
    hipLaunchKernelGGL(k_step_reset, dim3(1), dim3(1), 0, s, d_step);
    if (N == 0) return;
    AdamArgs a = {};
    for (int k = 0; k < 6; k++) a.g[k] = act[k];
    a.rows = kBaseRows + 3 * sh_count(sh_degree);
    a.raw = raw;
    a.m = m;
    a.v = v;
    a.N = N;
    a.ld = ld;
    hipLaunchKernelGGL(k_adam_init, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, a);
}

}  // namespace gsl
