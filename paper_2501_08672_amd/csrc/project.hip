// Projection of 3D Gaussians into the cameras of a window and its adjoint.
//
// Forward (Sec. II-B, eqs. equ:3dgs, equ:q, equ:spat): one lane per
// (camera, Gaussian).  The arithmetic is float64 (CDNA4 issues it at the
// rate of non-packed float32), so the float32 splat it stores carries a
// correctly rounded mean and conic factor even for the thin, grazing
// surfels a LiDAR map produces.
//
// Sigma2D is formed as P P^T + eps I with P = (J W) R diag(s), the product of
// the pinhole Jacobian J, the camera rotation W = R_cw and the Gaussian's
// rotation and scale, which equals (J W) Sigma3D (J W)^T.  The conic is
// stored as its upper Cholesky factor L (Sigma2D^{-1} = L^T L) so the
// renderer evaluates |L d|^2 as a sum of two squares.
//
// Backward (Appendix A): one lane per Gaussian looping over the cameras,
// chaining the per-(camera, Gaussian) 2D gradients to mean, scale,
// quaternion, opacity and colour (summed in registers across cameras, so no
// atomics) and, per camera, to the twist (dphi, dt) of a left perturbation of
// T_CW: dL/ddt = sum_i dL/dp_C,i and dL/ddphi = sum_i p_C,i x dL/dp_C,i plus
// the term of Sigma2D's dependence on W.  Per-workgroup pose partials are
// summed by a second kernel, so the pose gradient is deterministic.
#include "binning.hpp"
#include "sh.hpp"

namespace gsl {

namespace {

struct CamBatch {
    DevCam cams[16];
    DevCam *dst;
    int n;
};

__global__ void k_upload_cams(CamBatch b)
{
    int i = threadIdx.x;
    if (i < b.n) b.dst[i] = b.cams[i];
}

// Everything the forward computes for one (camera, Gaussian), kept for the
// backward, which recomputes it instead of storing it.
struct Proj {
    double x, y, z;     // camera-frame mean
    double W[9];        // camera rotation
    double Rg[9];       // Gaussian rotation (normalised quaternion)
    double qn[4], qlen;
    double s[3];
    double M[6];        // J W, 2 x 3
    double P[6];        // J W Rg diag(s), 2 x 3
    double a, b, c;     // Sigma2D = [[a, b], [b, c]] including eps
    double det;
    double mx, my;
};

// The projection's arithmetic (quat_rot, load_gauss, project_cam) may fuse
// multiplies and adds: every kernel inlines these same functions, so the
// projection, its adjoint and the pose tangents still see one projection.
__device__ __forceinline__ void quat_rot(const double q[4], double R[9])
{
#pragma clang fp contract(fast)
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

// The camera-independent part of a Gaussian: world mean, normalised
// quaternion and its rotation, scale.
struct GaussLocal {
    double px, py, pz;
    double qn[4], qlen;
    double Rg[9];
    double s[3];
};

// LEN: also the quaternion's length (the adjoint needs it); without it the
// normalisation takes one reciprocal square root.
template <bool LEN = true>
__device__ __forceinline__ void load_gauss(const float *__restrict__ mean, const float *__restrict__ scale,
                                           const float *__restrict__ quat, int N, int i, GaussLocal &gl)
{
#pragma clang fp contract(fast)
    gl.px = mean[i];
    gl.py = mean[N + i];
    gl.pz = mean[2 * N + i];
    double q[4] = {quat[i], quat[N + i], quat[2 * N + i], quat[3 * N + i]};
    const double qq = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    gl.qlen = LEN ? sqrt(qq) : 0.0;
    const double il = LEN ? 1.0 / gl.qlen : rsqrt(qq);
    for (int k = 0; k < 4; k++) gl.qn[k] = q[k] * il;
    quat_rot(gl.qn, gl.Rg);
    gl.s[0] = scale[i];
    gl.s[1] = scale[N + i];
    gl.s[2] = scale[2 * N + i];
}

// Returns false when the Gaussian is behind the near plane (only x, y, z are
// valid then).
__device__ __forceinline__ bool project_cam(const GaussLocal &gl, const DevCam &cam, float eps2d, float near_z,
                                            Proj &p)
{
#pragma clang fp contract(fast)
    const double px = gl.px, py = gl.py, pz = gl.pz;
    for (int k = 0; k < 9; k++) p.W[k] = cam.R[k];
    p.x = p.W[0] * px + p.W[1] * py + p.W[2] * pz + (double)cam.t[0];
    p.y = p.W[3] * px + p.W[4] * py + p.W[5] * pz + (double)cam.t[1];
    p.z = p.W[6] * px + p.W[7] * py + p.W[8] * pz + (double)cam.t[2];
    if (!(p.z > (double)near_z)) return false;
    const double iz = 1.0 / p.z;
    const double fx = cam.fx, fy = cam.fy;
    p.mx = fx * p.x * iz + (double)cam.cx;
    p.my = fy * p.y * iz + (double)cam.cy;
    // J W: rows (fx/z) (W0 - x/z W2) and (fy/z) (W1 - y/z W2)
    const double ux = p.x * iz, uy = p.y * iz;
    for (int k = 0; k < 3; k++) {
        p.M[k] = fx * iz * (p.W[k] - ux * p.W[6 + k]);
        p.M[3 + k] = fy * iz * (p.W[3 + k] - uy * p.W[6 + k]);
    }
    p.qlen = gl.qlen;
    for (int k = 0; k < 4; k++) p.qn[k] = gl.qn[k];
    for (int k = 0; k < 9; k++) p.Rg[k] = gl.Rg[k];
    for (int k = 0; k < 3; k++) p.s[k] = gl.s[k];
    for (int r = 0; r < 2; r++)
        for (int k = 0; k < 3; k++) {
            const double mr = p.M[3 * r] * p.Rg[k] + p.M[3 * r + 1] * p.Rg[3 + k] + p.M[3 * r + 2] * p.Rg[6 + k];
            p.P[3 * r + k] = mr * p.s[k];
        }
    p.a = p.P[0] * p.P[0] + p.P[1] * p.P[1] + p.P[2] * p.P[2] + (double)eps2d;
    p.b = p.P[0] * p.P[3] + p.P[1] * p.P[4] + p.P[2] * p.P[5];
    p.c = p.P[3] * p.P[3] + p.P[4] * p.P[4] + p.P[5] * p.P[5] + (double)eps2d;
    p.det = p.a * p.c - p.b * p.b;
    return true;
}

template <bool LEN = true>
__device__ __forceinline__ bool compute_proj(const float *__restrict__ mean, const float *__restrict__ scale,
                                             const float *__restrict__ quat, int N, int i, const DevCam &cam,
                                             float eps2d, float near_z, Proj &p)
{
    GaussLocal gl;
    load_gauss<LEN>(mean, scale, quat, N, i, gl);
    return project_cam(gl, cam, eps2d, near_z, p);
}

// Also counts the tiles each splat's alpha_min ellipse reaches (tiles_touched)
// with the binning walk of the emission, from the record still in registers;
// records spanning more than kBigTiles tiles go to big_list for a second kernel.
template <bool SH>
__global__ __launch_bounds__(256) void k_project(const float *__restrict__ mean, const float *__restrict__ scale,
                                                 const float *__restrict__ quat,
                                                 const float *__restrict__ opacity,
                                                 const float *__restrict__ color,
                                                 const float *__restrict__ sh, int shd, int N, int64_t M,
                                                 const DevCam *__restrict__ cams, DevOpts o,
                                                 gsl_splat *__restrict__ out, gsl_binrec *__restrict__ bout,
                                                 uint32_t *__restrict__ kout, int32_t *__restrict__ tiles,
                                                 uint32_t *__restrict__ big_list, uint32_t *__restrict__ big_n,
                                                 float *__restrict__ g2d_zero, uint32_t *__restrict__ queue_zero)
{
    if (queue_zero && blockIdx.x == 0 && threadIdx.x == 0) *queue_zero = 0u;
    __shared__ RecTiles rec[256];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    // with g2d_zero (the fused window step): clear the 2D-gradient records of
    // this workgroup's records, one contiguous block written coalesced, in
    // place of a separate fill before the compositing kernel
    if (g2d_zero) {
        const int64_t base = (int64_t)blockIdx.x * blockDim.x * kG2, end = M * kG2;
#pragma unroll
        for (int q = 0; q < kG2; q++) {
            const int64_t k = base + (int64_t)q * blockDim.x + threadIdx.x;
            if (k < end) g2d_zero[k] = 0.f;
        }
    }
    uint32_t nt = 0;
    bool big = false;
    int c = 0;
    gsl_binrec br;
    if (m < M) {
        c = (int)(m / N);
        const int i = (int)(m - (int64_t)c * N);
        const DevCam cam = cams[c];

        gsl_splat sp;
        sp.mx = sp.my = sp.l11 = sp.l12 = sp.l22 = 0.f;
        sp.opacity = opacity[i];
        sp.r = color[i];
        sp.g = color[N + i];
        sp.b = color[2 * N + i];
        sp.depth = 0.f;
        sp.x0 = 0; sp.y0 = 0; sp.x1 = -1; sp.y1 = -1;

        Proj p;
        float kq = 0.f;  // the binning threshold of the record
        bool kept = compute_proj<false>(mean, scale, quat, N, i, cam, o.eps2d, o.near_z, p);
        if (kept) {
            const double W = cam.W, H = cam.H, g = o.guard;
            if (p.mx < -g * W || p.mx > (1.0 + g) * W || p.my < -g * H || p.my > (1.0 + g) * H) kept = false;
            if (!(p.det > 0.0)) kept = false;
            const double sigma = sp.opacity;
            if (!(sigma >= (double)o.alpha_min)) kept = false;
            if (kept) {
                // |L d|^2 <= kq  <=>  sigma G(d) >= alpha_min (up to kq's margin);
                // the bbox of that ellipse is |dx| <= sqrt(kq a), |dy| <= sqrt(kq c),
                // widened by 0.01 px (far more than the float32 square roots' error)
                kq = ellipse_k(sp.opacity, o.alpha_min);
                const double hx = (double)sqrtf(kq * (float)p.a) + 0.01;
                const double hy = (double)sqrtf(kq * (float)p.c) + 0.01;
                double x0 = ceil(p.mx - hx - 0.5), x1 = floor(p.mx + hx - 0.5);
                double y0 = ceil(p.my - hy - 0.5), y1 = floor(p.my + hy - 0.5);
                x0 = fmax(x0, 0.0); y0 = fmax(y0, 0.0);
                x1 = fmin(x1, W - 1.0); y1 = fmin(y1, H - 1.0);
                if (x0 > x1 || y0 > y1) {
                    kept = false;
                } else {
                    const int ix0 = (int)x0, ix1 = (int)x1, iy0 = (int)y0, iy1 = (int)y1;
                    sp.x0 = (int16_t)ix0; sp.x1 = (int16_t)ix1;
                    sp.y0 = (int16_t)iy0; sp.y1 = (int16_t)iy1;
                    // L = [[sqrt(c/det), -b/sqrt(c det)], [0, 1/sqrt(c)]]: two
                    // square roots and one division
                    const double sc = sqrt(p.c), sd = sqrt(p.det);
                    const double rcd = 1.0 / (sc * sd);
                    const double l22 = sd * rcd;
                    const double l11 = p.c * rcd;
                    const double l12 = -p.b * rcd;
                    sp.mx = (float)p.mx;
                    sp.my = (float)p.my;
                    sp.l11 = (float)l11;
                    sp.l12 = (float)l12;
                    sp.l22 = (float)l22;
                    sp.depth = (float)p.z;
                    if (SH) {
                        // view-dependent colour from the camera centre
                        double u[3];
                        view_dir(cam, mean[i], mean[N + i], mean[2 * N + i], u);
                        const int K = sh_count(shd);
                        double rgb[3] = {sp.r, sp.g, sp.b};
#pragma unroll
                        for (int k = 0; k < kShMaxK; k++) {
                            if (k < K) {
                                const double bk = sh_b(k, u[0], u[1], u[2]);
                                for (int ch = 0; ch < 3; ch++)
                                    rgb[ch] += bk * (double)sh[((int64_t)k * 3 + ch) * N + i];
                            }
                        }
                        sp.r = (float)rgb[0];
                        sp.g = (float)rgb[1];
                        sp.b = (float)rgb[2];
                    }
                }
            }
        }
        out[m] = sp;
        br.mx = sp.mx;
        br.my = sp.my;
        br.l11 = sp.l11;
        br.l12 = sp.l12;
        br.l22 = sp.l22;
        br.kq = kept ? kq : 0.f;
        br.x0 = sp.x0;
        br.y0 = sp.y0;
        br.x1 = sp.x1;
        br.y1 = sp.y1;
        bout[m] = br;
        kout[m] = kept ? __float_as_uint(sp.depth) : 0xffffffffu;
        nt = (uint32_t)bbox_tiles(br, o.tile);
        if (nt > kBigTiles) {
            push_big(big_list, big_n, (uint32_t)m);
            big = true;
            nt = 0;
        }
    }
    const uint32_t incl = (uint32_t)wave_incl_scan_u64(nt, lane), excl = incl - nt;
    const int wave0 = threadIdx.x & ~(kWave - 1);
    const int slot = rec_slot(nt, lane);
    if (nt) rec_fill(rec[wave0 + slot], br, cams[c], o.tile, 0, 0, 0, excl);
    const uint32_t total = __shfl(incl, kWave - 1, kWave);
    __syncthreads();
    const uint32_t n = expand_tiles<false>(rec + wave0, lane, excl, incl, total, o.tile, nullptr, nullptr);
    if (m < M && !big) tiles[m] = (int32_t)n;
}

// ------------------------------------------------------------------ pose tangents

// Derivatives of one splat's 2D mean and conic along the six twist
// directions (dphi, dt) of the left perturbation T_CW <- Exp(dphi, dt) T_CW
// (Sec. II-D and Appendix A, the chains of eqs. eqn:grad_meani_rcw ...
// eqn:grad_covi_tcw taken forward): to first order p_C moves by
// dphi x p_C + dt and W by dphi^ W.  With M = J W and P = M Rg diag(s),
//   dmu = J dp_C,  dM = dJ(dp_C) W + J dW,  dP = dM Rg diag(s),
//   dSigma2D = dP P^T + P dP^T,  dconic = -conic dSigma2D conic.
// Record m gets kTangent floats: dmx[6], dmy[6], dA[6], dB[6], dC[6] of the
// conic (A, B, C) = Sigma2D^{-1}, then two unused.  Only records that reach a
// tile are written (no other record is ever read).
template <bool SH>
__global__ __launch_bounds__(256) void k_project_tangent(const float *__restrict__ mean,
                                                         const float *__restrict__ scale,
                                                         const float *__restrict__ quat,
                                                         const float *__restrict__ sh, int shd, int N, int64_t M,
                                                         const DevCam *__restrict__ cams, DevOpts o,
                                                         const int32_t *__restrict__ tiles_touched,
                                                         float *__restrict__ tangent)
{
    constexpr int STRIDE = SH ? kTangentSH : kTangent;
    const int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (m >= M || tiles_touched[m] <= 0) return;
    const int c = (int)(m / N);
    const int i = (int)(m - (int64_t)c * N);
    const DevCam cam = cams[c];
    Proj p;
    if (!compute_proj(mean, scale, quat, N, i, cam, o.eps2d, o.near_z, p)) return;
    const double iz = 1.0 / p.z, fx = cam.fx, fy = cam.fy;
    const double J00 = fx * iz, J02 = -fx * p.x * iz * iz, J11 = fy * iz, J12 = -fy * p.y * iz * iz;
    const double id = 1.0 / p.det;
    const double QA = p.c * id, QB = -p.b * id, QC = p.a * id;
    float *out = tangent + m * STRIDE;
    for (int k = 0; k < 6; k++) {
        double dp[3] = {0.0, 0.0, 0.0};
        double E[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};  // [e]x for a rotation direction
        if (k < 3) {
            const double e0 = k == 0, e1 = k == 1, e2 = k == 2;
            dp[0] = e1 * p.z - e2 * p.y;
            dp[1] = e2 * p.x - e0 * p.z;
            dp[2] = e0 * p.y - e1 * p.x;
            E[1] = -e2; E[2] = e1; E[3] = e2; E[5] = -e0; E[6] = -e1; E[7] = e0;
        } else {
            dp[k - 3] = 1.0;
        }
        out[k] = (float)(J00 * dp[0] + J02 * dp[2]);
        out[6 + k] = (float)(J11 * dp[1] + J12 * dp[2]);
        const double dz = dp[2];
        const double dJ00 = -fx * dz * iz * iz, dJ11 = -fy * dz * iz * iz;
        const double dJ02 = -fx * (dp[0] * iz * iz - 2.0 * p.x * dz * iz * iz * iz);
        const double dJ12 = -fy * (dp[1] * iz * iz - 2.0 * p.y * dz * iz * iz * iz);
        // dW = E W;  dM = dJ W + J E W
        double EW[9];
        for (int r = 0; r < 3; r++)
            for (int q = 0; q < 3; q++)
                EW[3 * r + q] = E[3 * r] * p.W[q] + E[3 * r + 1] * p.W[3 + q] + E[3 * r + 2] * p.W[6 + q];
        double dM[6];
        for (int q = 0; q < 3; q++) {
            dM[q] = dJ00 * p.W[q] + dJ02 * p.W[6 + q] + J00 * EW[q] + J02 * EW[6 + q];
            dM[3 + q] = dJ11 * p.W[3 + q] + dJ12 * p.W[6 + q] + J11 * EW[3 + q] + J12 * EW[6 + q];
        }
        double dP[6];
        for (int r = 0; r < 2; r++)
            for (int q = 0; q < 3; q++)
                dP[3 * r + q] = (dM[3 * r] * p.Rg[q] + dM[3 * r + 1] * p.Rg[3 + q] + dM[3 * r + 2] * p.Rg[6 + q]) *
                                p.s[q];
        const double da = 2.0 * (dP[0] * p.P[0] + dP[1] * p.P[1] + dP[2] * p.P[2]);
        const double db = dP[0] * p.P[3] + dP[1] * p.P[4] + dP[2] * p.P[5] + p.P[0] * dP[3] + p.P[1] * dP[4] +
                          p.P[2] * dP[5];
        const double dc = 2.0 * (dP[3] * p.P[3] + dP[4] * p.P[4] + dP[5] * p.P[5]);
        // dQ = -Q dS Q with Q = [[QA, QB], [QB, QC]], dS = [[da, db], [db, dc]]
        const double t00 = QA * da + QB * db, t01 = QA * db + QB * dc;
        const double t10 = QB * da + QC * db, t11 = QB * db + QC * dc;
        out[12 + k] = (float)(-(t00 * QA + t01 * QB));
        out[18 + k] = (float)(-(t00 * QB + t01 * QC));
        out[24 + k] = (float)(-(t10 * QB + t11 * QC));
    }
    if (!SH) {
        out[30] = 0.f;
        out[31] = 0.f;
        return;
    }
    // colour along the twist: a rotation keeps the camera centre; dt moves
    // the view vector d = mu - o by R^T dt, so dc/ddt = dc/du (I - u u^T) / r R^T
    double u[3];
    const double r = view_dir(cam, mean[i], mean[N + i], mean[2 * N + i], u);
    const int K = sh_count(shd);
    double du[3][3] = {{0, 0, 0}, {0, 0, 0}, {0, 0, 0}};  // [channel][axis]
#pragma unroll
    for (int k = 0; k < kShMaxK; k++) {
        if (k < K) {
            double dx, dy, dz;
            sh_db(k, u[0], u[1], u[2], dx, dy, dz);
            for (int ch = 0; ch < 3; ch++) {
                const double w = sh[((int64_t)k * 3 + ch) * N + i];
                du[ch][0] += w * dx;
                du[ch][1] += w * dy;
                du[ch][2] += w * dz;
            }
        }
    }
    const double ir = 1.0 / r;
    for (int ch = 0; ch < 3; ch++) {
        const double ug = u[0] * du[ch][0] + u[1] * du[ch][1] + u[2] * du[ch][2];
        double dd[3];
        for (int a = 0; a < 3; a++) dd[a] = (du[ch][a] - u[a] * ug) * ir;
        for (int j = 0; j < 3; j++)
            out[30 + 3 * ch + j] = (float)(p.W[3 * j] * dd[0] + p.W[3 * j + 1] * dd[1] + p.W[3 * j + 2] * dd[2]);
    }
    out[39] = 0.f;
}

// ------------------------------------------------------------------ backward

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

// One DPP move of a double (both halves with the same control; rows the
// masks leave out read 0).
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, ROWS, 0xF, false);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, ROWS, 0xF, false);
    return __hiloint2double(hi, lo);
}

// Sum of a wave's doubles in a fixed order, by DPP moves (no LDS round
// trips): the total lands in lane 63.
__device__ __forceinline__ double dpp_sum63_f64(double v)
{
    v += dpp_f64<0xB1, 0xF>(v);   // quad [1,0,3,2]
    v += dpp_f64<0x4E, 0xF>(v);   // quad [2,3,0,1]
    v += dpp_f64<0x141, 0xF>(v);  // row_half_mirror
    v += dpp_f64<0x140, 0xF>(v);  // row_mirror
    v += dpp_f64<0x142, 0xA>(v);  // row_bcast:15
    v += dpp_f64<0x143, 0xC>(v);  // row_bcast:31
    return v;
}

__global__ __launch_bounds__(kPoseThreads) void k_project_bwd(
    const float *__restrict__ mean, const float *__restrict__ scale, const float *__restrict__ quat, int N, int C,
    const DevCam *__restrict__ cams, DevOpts o, const float *__restrict__ g2d, gsl_grads out, int accumulate,
    double *__restrict__ pose_part)
{
    __shared__ double s_red[kPoseThreads / kWave][6];
    const int i = blockIdx.x * kPoseThreads + threadIdx.x;
    const bool valid = i < N;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;

    double gm[3] = {0, 0, 0}, gs[3] = {0, 0, 0}, gq[4] = {0, 0, 0, 0}, gop = 0, gc[3] = {0, 0, 0};
    GaussLocal gl;  // once per Gaussian, not per camera
    double iql = 0.0;
    if (valid) {
        load_gauss(mean, scale, quat, N, i, gl);
        iql = 1.0 / gl.qlen;
    }
    // the next camera's 2D gradients are loaded while this camera's are chained
    float g2n[kG2];
    for (int k = 0; k < kG2; k++) g2n[k] = valid && C > 0 ? g2d[(int64_t)i * kG2 + k] : 0.f;
    for (int c = 0; c < C; c++) {
        double pose[6] = {0, 0, 0, 0, 0, 0};
        bool any = false;
        float g2[kG2];
        for (int k = 0; k < kG2; k++) {
            g2[k] = g2n[k];
            any |= g2[k] != 0.f;
        }
        if (valid && c + 1 < C) {
            const float *src = g2d + ((int64_t)(c + 1) * N + i) * kG2;
            for (int k = 0; k < kG2; k++) g2n[k] = src[k];
        }
        if (any) {
            // The chain rule below may fuse its multiplies and adds, as the
            // projection it recomputes does (gradients need no bit-level
            // agreement with anything but themselves).
#pragma clang fp contract(fast)
            const DevCam cam = cams[c];
            Proj p;
            project_cam(gl, cam, o.eps2d, o.near_z, p);
            gop += g2[5];
            gc[0] += g2[6]; gc[1] += g2[7]; gc[2] += g2[8];
            // conic (A, B, C) = Sigma2D^{-1};  dL/dSigma2D = -Q Gq Q with
            // Gq = [[gA, gB/2], [gB/2, gC]]
            const double id = 1.0 / p.det;
            const double QA = p.c * id, QB = -p.b * id, QC = p.a * id;
            const double gA = g2[2], gB = 0.5 * (double)g2[3], gC = g2[4];
            // T = Q Gq
            const double t00 = QA * gA + QB * gB, t01 = QA * gB + QB * gC;
            const double t10 = QB * gA + QC * gB, t11 = QB * gB + QC * gC;
            const double S00 = -(t00 * QA + t01 * QB);
            const double S01 = -(t00 * QB + t01 * QC);
            const double S11 = -(t10 * QB + t11 * QC);
            // Sigma2D = P P^T + eps I:  dL/dP = 2 S P
            double GP[6];
            for (int k = 0; k < 3; k++) {
                GP[k] = 2.0 * (S00 * p.P[k] + S01 * p.P[3 + k]);
                GP[3 + k] = 2.0 * (S01 * p.P[k] + S11 * p.P[3 + k]);
            }
            // P = M Rg diag(s):  dL/dM = GP diag(s) Rg^T,  dL/d(Rg diag s) = M^T GP
            double GM[6];
            for (int r = 0; r < 2; r++)
                for (int j = 0; j < 3; j++) {
                    double acc = 0;
                    for (int k = 0; k < 3; k++) acc += GP[3 * r + k] * p.s[k] * p.Rg[3 * j + k];
                    GM[3 * r + j] = acc;
                }
            double GRg[9];
            for (int j = 0; j < 3; j++)
                for (int k = 0; k < 3; k++) {
                    const double gn = p.M[j] * GP[k] + p.M[3 + j] * GP[3 + k];
                    GRg[3 * j + k] = gn * p.s[k];
                    gs[k] += gn * p.Rg[3 * j + k];
                }
            // Rg from the normalised quaternion
            {
                const double w = p.qn[0], x = p.qn[1], y = p.qn[2], z = p.qn[3];
                const double *G = GRg;
                double dw = 2.0 * (-z * G[1] + y * G[2] + z * G[3] - x * G[5] - y * G[6] + x * G[7]);
                double dx = 2.0 * (y * G[1] + z * G[2] + y * G[3] - 2.0 * x * G[4] - w * G[5] + z * G[6] + w * G[7] -
                                   2.0 * x * G[8]);
                double dy = 2.0 * (-2.0 * y * G[0] + x * G[1] + w * G[2] + x * G[3] + z * G[5] - w * G[6] + z * G[7] -
                                   2.0 * y * G[8]);
                double dz = 2.0 * (-2.0 * z * G[0] - w * G[1] + x * G[2] + w * G[3] - 2.0 * z * G[4] + y * G[5] +
                                   x * G[6] + y * G[7]);
                const double dot = dw * w + dx * x + dy * y + dz * z;
                const double il = iql;
                gq[0] += (dw - w * dot) * il;
                gq[1] += (dx - x * dot) * il;
                gq[2] += (dy - y * dot) * il;
                gq[3] += (dz - z * dot) * il;
            }
            // M = J W:  dL/dJ = GM W^T,  dL/dW (through Sigma2D) = J^T GM
            const double iz = 1.0 / p.z, fx = cam.fx, fy = cam.fy;
            const double J00 = fx * iz, J02 = -fx * p.x * iz * iz, J11 = fy * iz, J12 = -fy * p.y * iz * iz;
            double GJ[6];
            for (int r = 0; r < 2; r++)
                for (int j = 0; j < 3; j++)
                    GJ[3 * r + j] = GM[3 * r] * p.W[3 * j] + GM[3 * r + 1] * p.W[3 * j + 1] +
                                    GM[3 * r + 2] * p.W[3 * j + 2];
            double GW[9];
            for (int k = 0; k < 3; k++) {
                GW[k] = J00 * GM[k];
                GW[3 + k] = J11 * GM[3 + k];
                GW[6 + k] = J02 * GM[k] + J12 * GM[3 + k];
            }
            // dL/dp_C: through mean2d (Jacobian J) and through J(p_C)
            const double gmx = g2[0], gmy = g2[1];
            const double iz2 = iz * iz, iz3 = iz2 * iz;
            double gpx = J00 * gmx + GJ[2] * (-fx * iz2);
            double gpy = J11 * gmy + GJ[5] * (-fy * iz2);
            double gpz = J02 * gmx + J12 * gmy + GJ[0] * (-fx * iz2) + GJ[2] * (2.0 * fx * p.x * iz3) +
                         GJ[4] * (-fy * iz2) + GJ[5] * (2.0 * fy * p.y * iz3);
            // p_C = W p_W + t
            gm[0] += p.W[0] * gpx + p.W[3] * gpy + p.W[6] * gpz;
            gm[1] += p.W[1] * gpx + p.W[4] * gpy + p.W[7] * gpz;
            gm[2] += p.W[2] * gpx + p.W[5] * gpy + p.W[8] * gpz;
            // left twist: p_C <- p_C + dphi x p_C + dt,  W <- W + dphi^ W
            // X = GW W^T;  the W term is (X21 - X12, X02 - X20, X10 - X01)
            double X[9];
            for (int r = 0; r < 3; r++)
                for (int j = 0; j < 3; j++)
                    X[3 * r + j] = GW[3 * r] * p.W[3 * j] + GW[3 * r + 1] * p.W[3 * j + 1] +
                                   GW[3 * r + 2] * p.W[3 * j + 2];
            pose[0] = p.y * gpz - p.z * gpy + (X[7] - X[5]);
            pose[1] = p.z * gpx - p.x * gpz + (X[2] - X[6]);
            pose[2] = p.x * gpy - p.y * gpx + (X[3] - X[1]);
            pose[3] = gpx;
            pose[4] = gpy;
            pose[5] = gpz;
        }
        // per-camera block partial of the pose gradient (skipped when no lane
        // of the workgroup sees this camera)
        if (__syncthreads_or(any)) {
            for (int k = 0; k < 6; k++) {
                const double v = dpp_sum63_f64(pose[k]);
                if (lane == kWave - 1) s_red[wv][k] = v;
            }
            __syncthreads();
            if (threadIdx.x < 6) {
                double v = 0;
                for (int w = 0; w < kPoseThreads / kWave; w++) v += s_red[w][threadIdx.x];
                pose_part[((int64_t)c * 6 + threadIdx.x) * gridDim.x + blockIdx.x] = v;
            }
            __syncthreads();
        } else if (threadIdx.x < 6) {
            pose_part[((int64_t)c * 6 + threadIdx.x) * gridDim.x + blockIdx.x] = 0.0;
        }
    }
    if (!valid) return;
    auto put = [&](float *dst, int64_t idx, double v) {
        if (!dst) return;
        if (accumulate) dst[idx] += (float)v;
        else dst[idx] = (float)v;
    };
    for (int k = 0; k < 3; k++) {
        put(out.g_mean, (int64_t)k * N + i, gm[k]);
        put(out.g_scale, (int64_t)k * N + i, gs[k]);
        put(out.g_color, (int64_t)k * N + i, gc[k]);
    }
    for (int k = 0; k < 4; k++) put(out.g_quat, (int64_t)k * N + i, gq[k]);
    put(out.g_opacity, i, gop);
}

// Adjoint of the view-dependent colour (SH degree > 0), after k_project_bwd:
// one lane per Gaussian looping over the cameras.  From the colour gradient
// g_c of each (camera, Gaussian) record: dL/dsh_k = sum_c g_c B_k(u_c); the
// colour's dependence on the view direction u = (mu - o) / r adds
// (I - u u^T) g_u / r to the mean gradient, with g_u = sum_ch g_c,ch
// sum_k sh_k,ch dB_k/du; the camera centre o = -R^T t moves by -R^T dt under
// the left twist (a rotation leaves it in place), so the twist's dt gets
// R (I - u u^T) g_u / r, written as per-workgroup partials (the dphi slots
// zero) for the pose reduction.
__global__ __launch_bounds__(kPoseThreads) void k_sh_bwd(const float *__restrict__ mean, const float *__restrict__ sh,
                                                         int shd, int N, int C, const DevCam *__restrict__ cams,
                                                         const float *__restrict__ g2d, float *__restrict__ g_sh,
                                                         float *__restrict__ g_mean, int accumulate,
                                                         double *__restrict__ pose_part)
{
    __shared__ double s_red[kPoseThreads / kWave][3];
    const int i = blockIdx.x * kPoseThreads + threadIdx.x;
    const bool valid = i < N;
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const int K = sh_count(shd);
    float acc[3 * kShMaxK];
#pragma unroll
    for (int k = 0; k < 3 * kShMaxK; k++) acc[k] = 0.f;
    double gm[3] = {0, 0, 0};
    double px = 0, py = 0, pz = 0;
    if (valid) {
        px = mean[i];
        py = mean[N + i];
        pz = mean[2 * N + i];
    }
    // the next camera's colour gradient is loaded while this camera's is chained
    float gcn[3] = {0.f, 0.f, 0.f};
    if (valid && C > 0)
        for (int k = 0; k < 3; k++) gcn[k] = g2d[(int64_t)i * kG2 + 6 + k];
    for (int c = 0; c < C; c++) {
        double gt[3] = {0, 0, 0};
        const float gc[3] = {gcn[0], gcn[1], gcn[2]};
        if (valid && c + 1 < C) {
            const float *src = g2d + ((int64_t)(c + 1) * N + i) * kG2 + 6;
            gcn[0] = src[0];
            gcn[1] = src[1];
            gcn[2] = src[2];
        }
        const bool any = gc[0] != 0.f || gc[1] != 0.f || gc[2] != 0.f;
        if (any) {
            const DevCam cam = cams[c];
            double u[3];
            const double r = view_dir(cam, px, py, pz, u);
            double gu[3] = {0, 0, 0};
#pragma unroll
            for (int k = 0; k < kShMaxK; k++) {
                if (k < K) {
                    const double bk = sh_b(k, u[0], u[1], u[2]);
                    double dx, dy, dz;
                    sh_db(k, u[0], u[1], u[2], dx, dy, dz);
                    double w = 0;
                    for (int ch = 0; ch < 3; ch++) {
                        acc[3 * k + ch] += (float)((double)gc[ch] * bk);
                        w += (double)gc[ch] * (double)sh[((int64_t)k * 3 + ch) * N + i];
                    }
                    gu[0] += w * dx;
                    gu[1] += w * dy;
                    gu[2] += w * dz;
                }
            }
            const double ug = u[0] * gu[0] + u[1] * gu[1] + u[2] * gu[2];
            const double ir = 1.0 / r;
            double gd[3];
            for (int j = 0; j < 3; j++) {
                gd[j] = (gu[j] - u[j] * ug) * ir;
                gm[j] += gd[j];
            }
            for (int j = 0; j < 3; j++)
                gt[j] = cam.R[3 * j] * gd[0] + cam.R[3 * j + 1] * gd[1] + cam.R[3 * j + 2] * gd[2];
        }
        if (__syncthreads_or(any)) {
            for (int k = 0; k < 3; k++) {
                const double v = dpp_sum63_f64(gt[k]);
                if (lane == kWave - 1) s_red[wv][k] = v;
            }
            __syncthreads();
            if (threadIdx.x < 6) {
                double v = 0;
                if (threadIdx.x >= 3)
                    for (int w = 0; w < kPoseThreads / kWave; w++) v += s_red[w][threadIdx.x - 3];
                pose_part[((int64_t)c * 6 + threadIdx.x) * gridDim.x + blockIdx.x] = v;
            }
            __syncthreads();
        } else if (threadIdx.x < 6) {
            pose_part[((int64_t)c * 6 + threadIdx.x) * gridDim.x + blockIdx.x] = 0.0;
        }
    }
    if (!valid) return;
    if (g_mean)
        for (int k = 0; k < 3; k++) g_mean[(int64_t)k * N + i] += (float)gm[k];
    if (g_sh) {
#pragma unroll
        for (int k = 0; k < 3 * kShMaxK; k++) {
            if (k < 3 * K) {
                float *dst = g_sh + (int64_t)k * N + i;
                if (accumulate) *dst += acc[k];
                else *dst = acc[k];
            }
        }
    }
}

// Sums the per-workgroup pose partials (and a second set, when given).
__global__ __launch_bounds__(256) void k_pose_reduce(const double *__restrict__ part,
                                                     const double *__restrict__ part2, int blocks, int C,
                                                     double *__restrict__ g_pose, int accumulate)
{
    // workgroup (c, k) sums the contiguous row part[c][k][0 .. blocks) (and
    // part2's) in a fixed order: the result does not depend on the run
    __shared__ double s_red[256 / kWave];
    const int c = blockIdx.x / 6, k = blockIdx.x - 6 * c;
    const double *row = part + ((int64_t)c * 6 + k) * blocks;
    const double *row2 = part2 ? part2 + ((int64_t)c * 6 + k) * blocks : nullptr;
    double acc = 0.0;
    int b = threadIdx.x;
    for (; b + 3 * 256 < blocks; b += 4 * 256) {  // four loads in flight, added in the same order
        double v[4], v2[4];
#pragma unroll
        for (int q = 0; q < 4; q++) {
            v[q] = row[b + q * 256];
            v2[q] = row2 ? row2[b + q * 256] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 4; q++) {
            acc += v[q];
            if (row2) acc += v2[q];
        }
    }
    for (; b < blocks; b += 256) {
        acc += row[b];
        if (row2) acc += row2[b];
    }
    const int lane = threadIdx.x & (kWave - 1), wv = threadIdx.x / kWave;
    const double w = wave_sum_f64(acc);
    if (lane == 0) s_red[wv] = w;
    __syncthreads();
    if (threadIdx.x == 0) {
        double v = 0;
        for (int q = 0; q < 256 / kWave; q++) v += s_red[q];
        if (accumulate) g_pose[c * 6 + k] += v;
        else g_pose[c * 6 + k] = v;
    }
}

}  // namespace

void launch_upload_cams(DevCam *d_cams, const DevCam *h_cams, int C, hipStream_t s)
{
    for (int b = 0; b < C; b += 16) {
        CamBatch cb;
        cb.n = C - b < 16 ? C - b : 16;
        cb.dst = d_cams + b;
        for (int k = 0; k < cb.n; k++) cb.cams[k] = h_cams[b + k];
        hipLaunchKernelGGL(k_upload_cams, dim3(1), dim3(64), 0, s, cb);
    }
}

void launch_project(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                    gsl_splat *splats, gsl_binrec *binrecs, uint32_t *depth_keys, int32_t *tiles_touched,
                    uint32_t *big_list, uint32_t *big_n, hipStream_t s, float *g2d_zero, uint32_t *queue_zero)
{
    if (L.M == 0) return;
    const int64_t blocks = (L.M + 255) / 256;
    launch_fill_u32(big_n, 0u, 1, s);
    if (g.sh_degree > 0)
        hipLaunchKernelGGL(k_project<true>, dim3((unsigned)blocks), dim3(256), 0, s, g.mean, g.scale, g.quat,
                           g.opacity, g.color, g.sh, g.sh_degree, g.N, L.M, cams, o, splats, binrecs, depth_keys,
                           tiles_touched, big_list, big_n, g2d_zero, queue_zero);
    else
        hipLaunchKernelGGL(k_project<false>, dim3((unsigned)blocks), dim3(256), 0, s, g.mean, g.scale, g.quat,
                           g.opacity, g.color, g.sh, 0, g.N, L.M, cams, o, splats, binrecs, depth_keys,
                           tiles_touched, big_list, big_n, g2d_zero, queue_zero);
    launch_count_big(binrecs, cams, L, tiles_touched, big_list, big_n, s);
}

void launch_project_tangent(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                            const int32_t *tiles_touched, float *tangent, hipStream_t s)
{
    if (L.M == 0) return;
    const int64_t blocks = (L.M + 255) / 256;
    if (g.sh_degree > 0)
        hipLaunchKernelGGL(k_project_tangent<true>, dim3((unsigned)blocks), dim3(256), 0, s, g.mean, g.scale, g.quat,
                           g.sh, g.sh_degree, g.N, L.M, cams, o, tiles_touched, tangent);
    else
        hipLaunchKernelGGL(k_project_tangent<false>, dim3((unsigned)blocks), dim3(256), 0, s, g.mean, g.scale,
                           g.quat, g.sh, 0, g.N, L.M, cams, o, tiles_touched, tangent);
}

void launch_project_bwd(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const DevOpts &o,
                        const float *g2d, const gsl_grads &out, int accumulate, double *pose_part,
                        int pose_blocks, hipStream_t s)
{
    if (L.N == 0 || pose_blocks == 0) return;
    hipLaunchKernelGGL(k_project_bwd, dim3(pose_blocks), dim3(kPoseThreads), 0, s, g.mean, g.scale, g.quat, g.N,
                       L.C, cams, o, g2d, out, accumulate, pose_part);
}

void launch_pose_reduce(const double *pose_part, const double *pose_part2, int blocks, int C, double *g_pose,
                        int accumulate, hipStream_t s)
{
    if (!g_pose || C == 0) return;
    hipLaunchKernelGGL(k_pose_reduce, dim3(6 * C), dim3(256), 0, s, pose_part, pose_part2, blocks, C, g_pose,
                       accumulate);
}

void launch_sh_bwd(const gsl_gaussians &g, const DevCam *cams, const Layout &L, const float *g2d, float *g_sh,
                   float *g_mean, int accumulate, double *pose_part, int pose_blocks, hipStream_t s)
{
    if (L.N == 0 || pose_blocks == 0 || g.sh_degree <= 0) return;
    hipLaunchKernelGGL(k_sh_bwd, dim3(pose_blocks), dim3(kPoseThreads), 0, s, g.mean, g.sh, g.sh_degree, g.N, L.C,
                       cams, g2d, g_sh, g_mean, accumulate, pose_part);
}

}  // namespace gsl
