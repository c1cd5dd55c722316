// Colour initialisation of new Gaussians (Sec. II-B: the degree-0 colour is
// the bilinear interpolation of the camera image at the projected mean; the
// higher orders start at zero).  One lane per Gaussian; projection in
// float64 like the renderer's.
#include "sh.hpp"

namespace gsl {

namespace {

struct InitCam {
    double fx, fy, cx, cy;
    double R[9], t[3];
    int W, H;
};

__global__ __launch_bounds__(256) void k_color_init(const float *__restrict__ mean, int64_t mean_ld, int n,
                                                    InitCam cam, double near_z, const float *__restrict__ image,
                                                    float *__restrict__ color, int64_t color_ld,
                                                    uint8_t *__restrict__ valid)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double px = mean[i], py = mean[mean_ld + i], pz = mean[2 * mean_ld + i];
    const double x = cam.R[0] * px + cam.R[1] * py + cam.R[2] * pz + cam.t[0];
    const double y = cam.R[3] * px + cam.R[4] * py + cam.R[5] * pz + cam.t[1];
    const double z = cam.R[6] * px + cam.R[7] * py + cam.R[8] * pz + cam.t[2];
    bool ok = z > near_z;
    double u = 0, v = 0;
    if (ok) {
        u = cam.fx * x / z + cam.cx;
        v = cam.fy * y / z + cam.cy;
        ok = u >= 0.0 && u < (double)cam.W && v >= 0.0 && v < (double)cam.H;
    }
    if (valid) valid[i] = ok ? 1 : 0;
    if (!ok) return;
    // pixel (c, r) has its centre at (c + 1/2, r + 1/2): clamp to the centres
    const double sx = fmin(fmax(u - 0.5, 0.0), (double)cam.W - 1.0);
    const double sy = fmin(fmax(v - 0.5, 0.0), (double)cam.H - 1.0);
    const int i0 = min((int)floor(sx), max(cam.W - 2, 0));
    const int j0 = min((int)floor(sy), max(cam.H - 2, 0));
    const double a = sx - i0, b = sy - j0;
    const int i1 = min(i0 + 1, cam.W - 1), j1 = min(j0 + 1, cam.H - 1);
    const int64_t plane = (int64_t)cam.W * cam.H;
    for (int ch = 0; ch < 3; ch++) {
        const float *im = image + ch * plane;
        const double c = (1.0 - a) * (1.0 - b) * im[(int64_t)j0 * cam.W + i0] + a * (1.0 - b) * im[(int64_t)j0 * cam.W + i1] +
                         (1.0 - a) * b * im[(int64_t)j1 * cam.W + i0] + a * b * im[(int64_t)j1 * cam.W + i1];
        color[ch * color_ld + i] = (float)c;
    }
}

}  // namespace

void launch_color_init(const float *mean, int64_t mean_ld, int n, const gsl_camera &c, float near_z,
                       const float *image, float *color, int64_t color_ld, uint8_t *valid, hipStream_t s)
{
    if (n == 0) return;
    InitCam ic;
    ic.fx = c.fx;
    ic.fy = c.fy;
    ic.cx = c.cx;
    ic.cy = c.cy;
    for (int k = 0; k < 9; k++) ic.R[k] = c.R_cw[k];
    for (int k = 0; k < 3; k++) ic.t[k] = c.t_cw[k];
    ic.W = c.width;
    ic.H = c.height;
    hipLaunchKernelGGL(k_color_init, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, mean, mean_ld, n, ic,
                       (double)near_z, image, color, color_ld, valid);
}

}  // namespace gsl
