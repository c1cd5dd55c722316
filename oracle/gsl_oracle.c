/*
 * FP64 CPU oracle for differentiable 3D Gaussian splatting (GS-LIVO,
 * arXiv 2501.08672, Sec. II-B and Appendix A).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain definition that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or helper with the GPU library.
 *
 * What it computes, in the paper's order:
 *   projection   Sigma3D = (R S)(R S)^T                       (eq. equ:3dgs)
 *                q = pi(T_CW p_W)                             (eq. equ:q)
 *                Sigma2D = (J W) Sigma3D (J W)^T + eps I      (eq. equ:spat, W = R_CW)
 *   compositing  I(x) = sum_i c_i a_i prod_{j<i} (1 - a_j),
 *                a_i = min(a_max, sigma_i G_i(x))             (eq. eq:raster)
 *                every term evaluated at the pixel centre x; Gaussians in
 *                ascending (camera depth, index) order; a Gaussian with
 *                a_i < a_min is skipped; the walk stops before the first
 *                Gaussian that would bring the transmittance below T_min.
 *   backward     the exact adjoint of that function for a linear functional
 *                L = sum_p <v_p, I_p> (any loss enters through v = dL/dI),
 *                chained to means, scales, quaternions, opacities, colours
 *                (eq. eq:gaussian_optimization) and to a left perturbation
 *                T_CW <- Exp(dphi, dt) T_CW of the camera pose (Appendix A,
 *                eq. eq:perturbation; eqs. eqn:grad_meani_rcw ... eqn:grad_covi_tcw).
 *
 * Everything is double precision.  The only non-double decision is the depth
 * order: Gaussians are ordered by their depth rounded to float, ties broken
 * by index, which is the order a 32-bit depth key gives.
 *
 * Ambiguity flags: a pixel whose result hinges on a threshold decision that
 * FP32 arithmetic may take the other way is flagged.  A flip of the a_min
 * decision (or of a cull decision on its border) at transmittance T moves the
 * pixel by at most 2 a T (max |c| + max |bg|) — the Gaussian's own term and the
 * rescaling of the rest of the walk by (1 - a) — and the relative error of T
 * by a.  Such flips are left unflagged while their summed bound stays within
 * amb_ignore, their T effect being added to the transmittance bound; beyond
 * that the pixel is flagged AMB_VALUE.  AMB_VALUE also marks T(1 - a) within
 * the accumulated bound of T_min at a Gaussian whose weight a T exceeds T_min
 * (the pixel may change by a whole contribution).  AMB_TCUT: the same cutoff ambiguity at a Gaussian with
 * a T <= T_min (the walk may stop one Gaussian earlier or later; that
 * Gaussian and everything after it weigh at most about 2 T_min, so the pixel
 * changes by at most 2.01 T_min (max c + bg)).  AMB_GRAD: a contributor whose
 * sigma*G lies within the bound of a_max, where the clamp switches the alpha
 * gradient on or off.  The bound is first order in the FP32 unit
 * roundoff u = 2^-24: the rounding of the 2D mean and of the conic factor,
 * the evaluation of the quadratic form, exp and the products, times the
 * safety factor amb_rel; for T it accumulates a (dalpha)/(1 - a) per
 * contributor.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double fx, fy, cx, cy;
    int32_t width, height;
    double R[9]; /* world -> camera rotation, row-major */
    double t[3]; /* world -> camera translation */
} orc_camera;

typedef struct {
    double near_z;    /* cull when camera depth <= near_z */
    double eps2d;     /* isotropic dilation added to Sigma2D (px^2) */
    double alpha_min; /* skip a Gaussian whose alpha is below this */
    double alpha_max; /* clamp on alpha */
    double T_min;     /* transmittance cutoff */
    double bg[3];     /* background colour */
    double guard;     /* cull when the 2D mean is beyond guard*W (guard*H) outside the image */
    double amb_rel;   /* safety factor on the FP32 error bound used by the ambiguity flags */
    double amb_ignore; /* pixel deviation budget for alpha-threshold flips left unflagged */
} orc_opts;

enum { ORC_KEPT = 1, ORC_BORDER = 2 };
enum { AMB_VALUE = 1, AMB_GRAD = 2, AMB_TCUT = 4 };

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                      */
/* ------------------------------------------------------------------------ */

/* unit quaternion (w, x, y, z) -> rotation matrix, row-major */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* C = A B with A (m x k), B (k x n), row-major */
static void matmul(const double *A, const double *B, double *C, int m, int k, int n)
{
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) {
            double s = 0;
            for (int l = 0; l < k; l++) s += A[i * k + l] * B[l * n + j];
            C[i * n + j] = s;
        }
}

/* B = A^T with A (m x n) */
static void transpose(const double *A, double *B, int m, int n)
{
    for (int i = 0; i < m; i++)
        for (int j = 0; j < n; j++) B[j * m + i] = A[i * n + j];
}

/* ------------------------------------------------------------------------ */
/* projection of one Gaussian into one camera                               */
/* ------------------------------------------------------------------------ */

typedef struct {
    double qn[4];      /* normalised quaternion */
    double qnorm;      /* |q| */
    double R[9];       /* rotation of the Gaussian */
    double S3[9];      /* Sigma3D (world) */
    double pC[3];      /* mean in the camera frame */
    double J[6];       /* 2x3 pinhole Jacobian at pC */
    double M3[9];      /* W Sigma3D W^T */
    double mu[2];      /* 2D mean */
    double S2[3];      /* Sigma2D: xx, xy, yy (including eps) */
    double Q[3];       /* conic = Sigma2D^{-1}: A, B, C */
    int status;        /* ORC_KEPT | ORC_BORDER */
} proj_t;

static void project_one(const double *mean, const double *scale, const double *quat,
                        const orc_camera *cam, const orc_opts *o, proj_t *p)
{
    /* rotation from the normalised quaternion; Sigma3D = R S S^T R^T (eq. equ:3dgs) */
    double n = sqrt(quat[0] * quat[0] + quat[1] * quat[1] + quat[2] * quat[2] + quat[3] * quat[3]);
    p->qnorm = n;
    for (int k = 0; k < 4; k++) p->qn[k] = quat[k] / n;
    quat_to_rot(p->qn, p->R);
    double RS[9], RSt[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) RS[r * 3 + c] = p->R[r * 3 + c] * scale[c];
    transpose(RS, RSt, 3, 3);
    matmul(RS, RSt, p->S3, 3, 3, 3);

    /* camera-frame mean: T_CW p_W (eq. equ:q) */
    const double *W = cam->R;
    for (int r = 0; r < 3; r++)
        p->pC[r] = W[r * 3 + 0] * mean[0] + W[r * 3 + 1] * mean[1] + W[r * 3 + 2] * mean[2] + cam->t[r];
    double x = p->pC[0], y = p->pC[1], z = p->pC[2];
    int kept = 1, border = 0;
    const double tiny = 1e-9;
    if (z <= o->near_z) kept = 0;
    if (fabs(z - o->near_z) <= tiny * o->near_z) border = 1;
    if (z <= 0) { /* behind the camera: nothing below is defined */
        p->status = 0;
        return;
    }
    /* pinhole projection and its Jacobian */
    p->mu[0] = cam->fx * x / z + cam->cx;
    p->mu[1] = cam->fy * y / z + cam->cy;
    p->J[0] = cam->fx / z; p->J[1] = 0;              p->J[2] = -cam->fx * x / (z * z);
    p->J[3] = 0;           p->J[4] = cam->fy / z;    p->J[5] = -cam->fy * y / (z * z);
    double lo_x = -o->guard * cam->width, hi_x = (1 + o->guard) * cam->width;
    double lo_y = -o->guard * cam->height, hi_y = (1 + o->guard) * cam->height;
    if (p->mu[0] < lo_x || p->mu[0] > hi_x || p->mu[1] < lo_y || p->mu[1] > hi_y) kept = 0;
    double bx = tiny * (1 + cam->width), by = tiny * (1 + cam->height);
    if (fabs(p->mu[0] - lo_x) <= bx || fabs(p->mu[0] - hi_x) <= bx ||
        fabs(p->mu[1] - lo_y) <= by || fabs(p->mu[1] - hi_y) <= by)
        border = 1;

    /* Sigma2D = J W Sigma3D W^T J^T + eps I (eq. equ:spat) */
    double Wt[9], WS[9], JM[6], Jt[6], S2full[4];
    transpose(W, Wt, 3, 3);
    matmul(W, p->S3, WS, 3, 3, 3);
    matmul(WS, Wt, p->M3, 3, 3, 3);
    matmul(p->J, p->M3, JM, 2, 3, 3);
    transpose(p->J, Jt, 2, 3);
    matmul(JM, Jt, S2full, 2, 3, 2);
    p->S2[0] = S2full[0] + o->eps2d;
    p->S2[1] = S2full[1];
    p->S2[2] = S2full[3] + o->eps2d;
    double det = p->S2[0] * p->S2[2] - p->S2[1] * p->S2[1];
    if (det <= 0) {
        kept = 0;
        det = 1; /* keep Q finite; the Gaussian is culled */
    }
    p->Q[0] = p->S2[2] / det;
    p->Q[1] = -p->S2[1] / det;
    p->Q[2] = p->S2[0] / det;
    p->status = (kept ? ORC_KEPT : 0) | (border ? ORC_BORDER : 0);
}

int orc_project(int64_t N, const double *mean, const double *scale, const double *quat,
                const orc_camera *cam, const orc_opts *o,
                double *p_cam, double *mean2d, double *cov2d, double *conic, int32_t *status)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) {
        proj_t p;
        memset(&p, 0, sizeof p);
        project_one(mean + 3 * i, scale + 3 * i, quat + 4 * i, cam, o, &p);
        if (p_cam) memcpy(p_cam + 3 * i, p.pC, sizeof p.pC);
        if (mean2d) memcpy(mean2d + 2 * i, p.mu, sizeof p.mu);
        if (cov2d) memcpy(cov2d + 3 * i, p.S2, sizeof p.S2);
        if (conic) memcpy(conic + 3 * i, p.Q, sizeof p.Q);
        if (status) status[i] = p.status;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* depth order                                                              */
/* ------------------------------------------------------------------------ */

typedef struct {
    float zf;
    int64_t id;
} order_t;

static int cmp_order(const void *a, const void *b)
{
    const order_t *x = (const order_t *)a, *y = (const order_t *)b;
    if (x->zf < y->zf) return -1;
    if (x->zf > y->zf) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* Projects every Gaussian and returns those kept or on a cull border, in
 * ascending (float depth, index) order. */
/* max |colour| + max |bg|: bounds how much one Gaussian's presence can move a pixel */
static double colour_bound(int64_t N, const double *color, const orc_opts *o)
{
    double cm = 0.0, bm = 0.0;
    for (int64_t k = 0; k < 3 * N; k++) cm = fmax(cm, fabs(color[k]));
    for (int ch = 0; ch < 3; ch++) bm = fmax(bm, fabs(o->bg[ch]));
    return cm + bm;
}

static int64_t build_order(int64_t N, const double *mean, const double *scale, const double *quat,
                           const orc_camera *cam, const orc_opts *o, proj_t **proj_out, int64_t **order_out)
{
    proj_t *proj = (proj_t *)calloc((size_t)N, sizeof(proj_t));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++) project_one(mean + 3 * i, scale + 3 * i, quat + 4 * i, cam, o, &proj[i]);
    int64_t M = 0;
    for (int64_t i = 0; i < N; i++)
        if (proj[i].status) M++;
    order_t *ord = (order_t *)malloc(sizeof(order_t) * (size_t)(M > 0 ? M : 1));
    M = 0;
    for (int64_t i = 0; i < N; i++)
        if (proj[i].status) {
            ord[M].zf = (float)proj[i].pC[2];
            ord[M].id = i;
            M++;
        }
    qsort(ord, (size_t)M, sizeof(order_t), cmp_order);
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(M > 0 ? M : 1));
    for (int64_t k = 0; k < M; k++) order[k] = ord[k].id;
    free(ord);
    *proj_out = proj;
    *order_out = order;
    return M;
}

/* ------------------------------------------------------------------------ */
/* per-pixel compositing (eq. eq:raster)                                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int64_t id;
    double alpha, T, G, dx, dy;
    int clamped;
} contrib_t;

/* Walks the ordered Gaussians for the pixel centre (px, py).  Fills rgb,
 * returns the final transmittance; records contributors when `list` is set. */
static double composite_pixel(double px, double py, int64_t M, const int64_t *order, const proj_t *proj,
                              const double *opacity, const double *color, const orc_opts *o, double cb,
                              double rgb[3], int32_t *n_out, int64_t *last_out, int32_t *flags_out,
                              contrib_t *list)
{
    double T = 1.0, C[3] = {0, 0, 0};
    int32_t n = 0, flags = 0;
    int64_t last = -1;
    const double amb = o->amb_rel, u = 0x1p-24;
    double eT = 0.0;   /* relative FP32 error bound accumulated on T */
    double ign = 0.0;  /* summed deviation bound of the a_min flips left unflagged */
    /* a flip of the a_min decision for a Gaussian of value s at transmittance T */
#define ORC_ALPHA_FLIP(s_)                                   \
    do {                                                     \
        const double eff_ = 2.0 * (s_) * T * cb;             \
        if (ign + eff_ <= o->amb_ignore) {                   \
            ign += eff_;                                     \
            eT += (s_);                                      \
        } else {                                             \
            flags |= AMB_VALUE;                              \
        }                                                    \
    } while (0)
    for (int64_t k = 0; k < M; k++) {
        int64_t i = order[k];
        const proj_t *p = &proj[i];
        double dx = px - p->mu[0], dy = py - p->mu[1];
        double power = -0.5 * (p->Q[0] * dx * dx + 2.0 * p->Q[1] * dx * dy + p->Q[2] * dy * dy);
        double G = exp(power);
        double s = opacity[i] * G;
        /* first-order relative error bound of an FP32 evaluation of s */
        double gx = p->Q[0] * dx + p->Q[1] * dy, gy = p->Q[1] * dx + p->Q[2] * dy;
        double sa = sqrt(p->Q[0]);
        double t1 = fabs(sa * dx + p->Q[1] / sa * dy), e1 = sa * fabs(dx) + fabs(p->Q[1]) / sa * fabs(dy);
        double ds = amb * u *
                    (16.0 + 4.0 * fabs(power) + 2.0 * (fabs(gx) * (fabs(p->mu[0]) + fabs(dx)) +
                                                       fabs(gy) * (fabs(p->mu[1]) + fabs(dy))) +
                     2.0 * t1 * e1);
        if (!(p->status & ORC_KEPT)) { /* on a cull border only: it may be kept in FP32 */
            if (s >= o->alpha_min * (1 - ds)) ORC_ALPHA_FLIP(s < o->alpha_max ? s : o->alpha_max);
            continue;
        }
        if (p->status & ORC_BORDER)
            if (s >= o->alpha_min * (1 - ds)) ORC_ALPHA_FLIP(s < o->alpha_max ? s : o->alpha_max);
        if (fabs(s - o->alpha_min) <= ds * o->alpha_min) ORC_ALPHA_FLIP(s);
        double a = s < o->alpha_max ? s : o->alpha_max;
        if (a < o->alpha_min) continue;
        if (fabs(s - o->alpha_max) <= ds * o->alpha_max) flags |= AMB_GRAD;
        double Tn = T * (1.0 - a);
        double da = s < o->alpha_max ? a * ds / (1.0 - a) : 0.0;
        if (fabs(Tn - o->T_min) <= o->T_min * (eT + da + amb * 4.0 * u))
            flags |= a * T <= o->T_min ? AMB_TCUT : AMB_VALUE;
        if (Tn < o->T_min) break;
        eT += da + amb * 4.0 * u;
        for (int ch = 0; ch < 3; ch++) C[ch] += a * T * color[3 * i + ch];
        if (list) {
            list[n].id = i;
            list[n].alpha = a;
            list[n].T = T;
            list[n].G = G;
            list[n].dx = dx;
            list[n].dy = dy;
            list[n].clamped = s >= o->alpha_max;
        }
        T = Tn;
        n++;
        last = i;
    }
#undef ORC_ALPHA_FLIP
    for (int ch = 0; ch < 3; ch++) rgb[ch] = C[ch] + T * o->bg[ch];
    if (n_out) *n_out = n;
    if (last_out) *last_out = last;
    if (flags_out) *flags_out = flags;
    return T;
}

int orc_render_fwd(int64_t N, const double *mean, const double *scale, const double *quat,
                   const double *opacity, const double *color, const orc_camera *cam, const orc_opts *o,
                   int64_t npix, const int32_t *pix, double *rgb, double *T_final, int32_t *n_contrib,
                   int64_t *last_id, int32_t *flags)
{
    proj_t *proj;
    int64_t *order;
    int64_t M = build_order(N, mean, scale, quat, cam, o, &proj, &order);
    const double cb = colour_bound(N, color, o);
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t p = 0; p < npix; p++) {
        double px = pix[2 * p] + 0.5, py = pix[2 * p + 1] + 0.5;
        double c[3];
        int32_t n, f;
        int64_t last;
        double T = composite_pixel(px, py, M, order, proj, opacity, color, o, cb, c, &n, &last, &f, NULL);
        rgb[3 * p] = c[0]; rgb[3 * p + 1] = c[1]; rgb[3 * p + 2] = c[2];
        if (T_final) T_final[p] = T;
        if (n_contrib) n_contrib[p] = n;
        if (last_id) last_id[p] = last;
        if (flags) flags[p] = f;
    }
    free(proj);
    free(order);
    return 0;
}

/* Contributor trace of one pixel, for the brute-force tests: ids, alphas and
 * transmittances before each contributor.  Returns the contributor count. */
int32_t orc_pixel_trace(int64_t N, const double *mean, const double *scale, const double *quat,
                        const double *opacity, const double *color, const orc_camera *cam, const orc_opts *o,
                        int32_t u, int32_t v, int32_t cap, int64_t *ids, double *alphas, double *Ts)
{
    proj_t *proj;
    int64_t *order;
    int64_t M = build_order(N, mean, scale, quat, cam, o, &proj, &order);
    contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)(M > 0 ? M : 1));
    double c[3];
    int32_t n;
    composite_pixel(u + 0.5, v + 0.5, M, order, proj, opacity, color, o, colour_bound(N, color, o), c, &n, NULL,
                    NULL, list);
    for (int32_t k = 0; k < n && k < cap; k++) {
        ids[k] = list[k].id;
        alphas[k] = list[k].alpha;
        Ts[k] = list[k].T;
    }
    free(list);
    free(proj);
    free(order);
    return n;
}

/* ------------------------------------------------------------------------ */
/* backward                                                                 */
/* ------------------------------------------------------------------------ */

/* per-(camera, Gaussian) 2D gradient: mean2d (2), conic A B C (3), opacity, colour (3) */
#define G2D 9

/* Adjoint of the pixel walk for the cotangent v (3 channels).  Accumulates
 * into the 2D gradient rows of `acc`. */
static void pixel_adjoint(double px, double py, const double v[3], int64_t M, const int64_t *order,
                          const proj_t *proj, const double *opacity, const double *color, const orc_opts *o,
                          contrib_t *list, double *acc)
{
    double rgb[3];
    int32_t n;
    double Tf = composite_pixel(px, py, M, order, proj, opacity, color, o, 0.0, rgb, &n, NULL, NULL, list);
    /* S = sum_{j > k} c_j a_j T_j + T_final bg, built from the back */
    double S[3] = {Tf * o->bg[0], Tf * o->bg[1], Tf * o->bg[2]};
    for (int32_t k = n - 1; k >= 0; k--) {
        const contrib_t *e = &list[k];
        int64_t i = e->id;
        const double *c = color + 3 * i;
        double *g = acc + G2D * i;
        /* dI/dc_k = a_k T_k */
        for (int ch = 0; ch < 3; ch++) g[6 + ch] += e->alpha * e->T * v[ch];
        /* dI/da_k = T_k c_k - S_k / (1 - a_k) */
        double ga = 0;
        for (int ch = 0; ch < 3; ch++) ga += v[ch] * (e->T * c[ch] - S[ch] / (1.0 - e->alpha));
        for (int ch = 0; ch < 3; ch++) S[ch] += c[ch] * e->alpha * e->T;
        if (e->clamped) continue; /* a = a_max does not depend on sigma or G */
        /* a = sigma G, G = exp(power) */
        g[5] += e->G * ga;
        double gpow = opacity[i] * e->G * ga;
        const double *Q = proj[i].Q;
        double dx = e->dx, dy = e->dy;
        /* power = -1/2 d^T Q d, d = x - mu:  dpower/dmu = Q d */
        g[0] += gpow * (Q[0] * dx + Q[1] * dy);
        g[1] += gpow * (Q[1] * dx + Q[2] * dy);
        /* dpower/dA = -dx^2/2, dpower/dB = -dx dy, dpower/dC = -dy^2/2 */
        g[2] += gpow * (-0.5 * dx * dx);
        g[3] += gpow * (-dx * dy);
        g[4] += gpow * (-0.5 * dy * dy);
    }
}

/* Chains one Gaussian's 2D gradient to its 3D parameters and to the pose
 * accumulators (dL/dW total, dL/dt). */
static void chain_to_3d(const proj_t *p, const double *g2, const double *mean, const double *scale,
                        const orc_camera *cam, double *g_mean, double *g_scale, double *g_quat,
                        double GW[9], double gt[3])
{
    const double *W = cam->R;
    double x = p->pC[0], y = p->pC[1], z = p->pC[2];
    /* conic -> Sigma2D: dL/dSigma = -Q G_Q Q with G_Q the symmetric gradient */
    double Qm[4] = {p->Q[0], p->Q[1], p->Q[1], p->Q[2]};
    double GQ[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    double T1[4], GS2[4];
    matmul(Qm, GQ, T1, 2, 2, 2);
    matmul(T1, Qm, GS2, 2, 2, 2);
    for (int k = 0; k < 4; k++) GS2[k] = -GS2[k];
    /* Sigma2D = J M3 J^T with M3 = W Sigma3 W^T */
    double Jt[6], GJ[6], tmp23[6], GM3[9], tmp32[6];
    transpose(p->J, Jt, 2, 3);
    matmul(GS2, p->J, tmp23, 2, 2, 3);   /* G J */
    matmul(tmp23, p->M3, GJ, 2, 3, 3);   /* G J M3 */
    for (int k = 0; k < 6; k++) GJ[k] *= 2.0;
    matmul(Jt, GS2, tmp32, 3, 2, 2);     /* J^T G */
    matmul(tmp32, p->J, GM3, 3, 2, 3);   /* J^T G J */
    /* M3 = W S3 W^T:  dL/dS3 = W^T GM3 W,  dL/dW = 2 GM3 W S3 */
    double Wt[9], t9[9], GS3[9], GWs[9];
    transpose(W, Wt, 3, 3);
    matmul(Wt, GM3, t9, 3, 3, 3);
    matmul(t9, W, GS3, 3, 3, 3);
    matmul(GM3, W, t9, 3, 3, 3);
    matmul(t9, p->S3, GWs, 3, 3, 3);
    for (int k = 0; k < 9; k++) GWs[k] *= 2.0;
    /* dL/dp_C from the 2D mean (dmu/dp_C = J) and from J(p_C) */
    double gp[3];
    gp[0] = p->J[0] * g2[0] + p->J[3] * g2[1];
    gp[1] = p->J[1] * g2[0] + p->J[4] * g2[1];
    gp[2] = p->J[2] * g2[0] + p->J[5] * g2[1];
    double fx = cam->fx, fy = cam->fy;
    /* J00 = fx/z, J02 = -fx x/z^2, J11 = fy/z, J12 = -fy y/z^2 */
    gp[0] += GJ[2] * (-fx / (z * z));
    gp[1] += GJ[5] * (-fy / (z * z));
    gp[2] += GJ[0] * (-fx / (z * z)) + GJ[2] * (2.0 * fx * x / (z * z * z)) + GJ[4] * (-fy / (z * z)) +
             GJ[5] * (2.0 * fy * y / (z * z * z));
    /* p_C = W p_W + t */
    for (int c = 0; c < 3; c++) g_mean[c] += W[0 * 3 + c] * gp[0] + W[1 * 3 + c] * gp[1] + W[2 * 3 + c] * gp[2];
    for (int r = 0; r < 3; r++) {
        gt[r] += gp[r];
        for (int c = 0; c < 3; c++) GW[r * 3 + c] += gp[r] * mean[c] + GWs[r * 3 + c];
    }
    /* S3 = Nm Nm^T with Nm = R diag(s):  dL/dNm = 2 GS3 Nm */
    double Nm[9], GN[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) Nm[r * 3 + c] = p->R[r * 3 + c] * scale[c];
    matmul(GS3, Nm, GN, 3, 3, 3);
    for (int k = 0; k < 9; k++) GN[k] *= 2.0;
    double GR[9];
    for (int c = 0; c < 3; c++) {
        double gs = 0;
        for (int r = 0; r < 3; r++) {
            gs += p->R[r * 3 + c] * GN[r * 3 + c];
            GR[r * 3 + c] = GN[r * 3 + c] * scale[c];
        }
        g_scale[c] += gs;
    }
    /* R(q) for the normalised q: derivative of each entry with respect to w, x, y, z */
    double w = p->qn[0], qx = p->qn[1], qy = p->qn[2], qz = p->qn[3];
    double dRw[9] = {0, -2 * qz, 2 * qy, 2 * qz, 0, -2 * qx, -2 * qy, 2 * qx, 0};
    double dRx[9] = {0, 2 * qy, 2 * qz, 2 * qy, -4 * qx, -2 * w, 2 * qz, 2 * w, -4 * qx};
    double dRy[9] = {-4 * qy, 2 * qx, 2 * w, 2 * qx, 0, 2 * qz, -2 * w, 2 * qz, -4 * qy};
    double dRz[9] = {-4 * qz, -2 * w, 2 * qx, 2 * w, -4 * qz, 2 * qy, 2 * qx, 2 * qy, 0};
    double gq[4] = {0, 0, 0, 0};
    for (int k = 0; k < 9; k++) {
        gq[0] += GR[k] * dRw[k];
        gq[1] += GR[k] * dRx[k];
        gq[2] += GR[k] * dRy[k];
        gq[3] += GR[k] * dRz[k];
    }
    /* through q_hat = q / |q| */
    double dot = gq[0] * p->qn[0] + gq[1] * p->qn[1] + gq[2] * p->qn[2] + gq[3] * p->qn[3];
    for (int k = 0; k < 4; k++) g_quat[k] += (gq[k] - p->qn[k] * dot) / p->qnorm;
}

/* Gradient of L = sum_p <v_p, I_p> over the listed pixels of one camera.
 * All outputs are accumulated (+=): g_mean, g_scale, g_color (N x 3),
 * g_quat (N x 4), g_opac (N), g_pose (6: dphi then dt, left perturbation of
 * T_CW) and, when not NULL, g2d (N x 9: mean2d, conic A B C, opacity, colour). */
int orc_render_bwd(int64_t N, const double *mean, const double *scale, const double *quat,
                   const double *opacity, const double *color, const orc_camera *cam, const orc_opts *o,
                   int64_t npix, const int32_t *pix, const double *v,
                   double *g_mean, double *g_scale, double *g_quat, double *g_opac, double *g_color,
                   double *g_pose, double *g2d)
{
    proj_t *proj;
    int64_t *order;
    int64_t M = build_order(N, mean, scale, quat, cam, o, &proj, &order);
    double *acc = (double *)calloc((size_t)N * G2D, sizeof(double));
    #pragma omp parallel
    {
        double *loc = (double *)calloc((size_t)N * G2D, sizeof(double));
        contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)(M > 0 ? M : 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; p++) {
            const double *vp = v + 3 * p;
            if (vp[0] == 0 && vp[1] == 0 && vp[2] == 0) continue;
            pixel_adjoint(pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5, vp, M, order, proj, opacity, color, o, list, loc);
        }
        #pragma omp critical
        for (int64_t k = 0; k < N * G2D; k++) acc[k] += loc[k];
        free(list);
        free(loc);
    }
    double GW[9] = {0}, gt[3] = {0};
    for (int64_t i = 0; i < N; i++) {
        const double *g2 = acc + G2D * i;
        int any = 0;
        for (int k = 0; k < G2D; k++) any |= g2[k] != 0;
        if (!any) continue;
        if (g2d)
            for (int k = 0; k < G2D; k++) g2d[G2D * i + k] += g2[k];
        g_opac[i] += g2[5];
        for (int ch = 0; ch < 3; ch++) g_color[3 * i + ch] += g2[6 + ch];
        chain_to_3d(&proj[i], g2, mean + 3 * i, scale + 3 * i, cam, g_mean + 3 * i, g_scale + 3 * i,
                    g_quat + 4 * i, GW, gt);
    }
    /* left perturbation W <- (I + dphi^) W, t <- (I + dphi^) t + dt:
     * dL/ddphi = vee of (GW W^T) + t x gt, dL/ddt = gt */
    double Wt[9], X[9];
    transpose(cam->R, Wt, 3, 3);
    matmul(GW, Wt, X, 3, 3, 3);
    const double *t = cam->t;
    g_pose[0] += X[7] - X[5] + (t[1] * gt[2] - t[2] * gt[1]);
    g_pose[1] += X[2] - X[6] + (t[2] * gt[0] - t[0] * gt[2]);
    g_pose[2] += X[3] - X[1] + (t[0] * gt[1] - t[1] * gt[0]);
    g_pose[3] += gt[0];
    g_pose[4] += gt[1];
    g_pose[5] += gt[2];
    free(acc);
    free(proj);
    free(order);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* forward-mode derivative with respect to the camera twist                 */
/* ------------------------------------------------------------------------ */

/* Derivatives of one Gaussian's 2D mean and conic along the six twist
 * directions (dphi_x, dphi_y, dphi_z, dt_x, dt_y, dt_z) of the left
 * perturbation T_CW <- Exp(dphi, dt) T_CW, to first order
 * p_C <- p_C + dphi x p_C + dt and W <- W + dphi^ W (the chains of eqs.
 * eqn:grad_meani_rcw ... eqn:grad_covi_tcw, taken forward).  dmu[2][6] and
 * dQ[3][6] (rows A, B, C of the conic), row-major. */
static void project_tangent(const proj_t *p, const orc_camera *cam, double dmu[12], double dQ[18])
{
    const double x = p->pC[0], y = p->pC[1], z = p->pC[2];
    const double fx = cam->fx, fy = cam->fy;
    const double Qm[4] = {p->Q[0], p->Q[1], p->Q[1], p->Q[2]};
    double Jt[6];
    transpose(p->J, Jt, 2, 3);
    for (int k = 0; k < 6; k++) {
        double e[3] = {0, 0, 0}, dp[3] = {0, 0, 0};
        if (k < 3) { /* rotation about axis k: dp = e x p_C */
            e[k] = 1;
            dp[0] = e[1] * z - e[2] * y;
            dp[1] = e[2] * x - e[0] * z;
            dp[2] = e[0] * y - e[1] * x;
        } else { /* translation along axis k - 3 */
            dp[k - 3] = 1;
        }
        /* mu = (fx x / z + cx, fy y / z + cy):  dmu = J dp */
        dmu[k] = p->J[0] * dp[0] + p->J[1] * dp[1] + p->J[2] * dp[2];
        dmu[6 + k] = p->J[3] * dp[0] + p->J[4] * dp[1] + p->J[5] * dp[2];
        /* J(p_C) moves with p_C */
        double dJ[6] = {-fx * dp[2] / (z * z), 0, -fx * (dp[0] / (z * z) - 2 * x * dp[2] / (z * z * z)),
                        0, -fy * dp[2] / (z * z), -fy * (dp[1] / (z * z) - 2 * y * dp[2] / (z * z * z))};
        /* M3 = W Sigma3 W^T with dW = E W, E = [e]x:  dM3 = E M3 - M3 E */
        double dM3[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (k < 3) {
            double E[9] = {0, -e[2], e[1], e[2], 0, -e[0], -e[1], e[0], 0}, A1[9], A2[9];
            matmul(E, p->M3, A1, 3, 3, 3);
            matmul(p->M3, E, A2, 3, 3, 3);
            for (int m = 0; m < 9; m++) dM3[m] = A1[m] - A2[m];
        }
        /* Sigma2D = J M3 J^T + eps I:  dSigma2D = dJ M3 J^T + J dM3 J^T + J M3 dJ^T */
        double dJt[6], t23[6], Sa[4], Sb[4], Sc[4], dS[4];
        transpose(dJ, dJt, 2, 3);
        matmul(dJ, p->M3, t23, 2, 3, 3);
        matmul(t23, Jt, Sa, 2, 3, 2);
        matmul(p->J, dM3, t23, 2, 3, 3);
        matmul(t23, Jt, Sb, 2, 3, 2);
        matmul(p->J, p->M3, t23, 2, 3, 3);
        matmul(t23, dJt, Sc, 2, 3, 2);
        for (int m = 0; m < 4; m++) dS[m] = Sa[m] + Sb[m] + Sc[m];
        /* Q = Sigma2D^{-1}:  dQ = -Q dSigma2D Q */
        double T1[4], T2[4];
        matmul(Qm, dS, T1, 2, 2, 2);
        matmul(T1, Qm, T2, 2, 2, 2);
        dQ[k] = -T2[0];
        dQ[6 + k] = -T2[1];
        dQ[12 + k] = -T2[3];
    }
}

/* dI/dxi of one pixel (jac[3][6], channel-major), with the contributor set
 * held fixed: along the walk T_{k+1} = T_k (1 - a_k), so
 * dT_{k+1} = dT_k (1 - a_k) - T_k da_k and the pixel gains
 * c_k (T_k da_k + a_k dT_k), plus a_k T_k dc_k when the colour itself
 * depends on the pose (dcol_all, N x 3 x 6, may be NULL); the background
 * adds bg dT_final.  A clamped alpha has da = 0; otherwise da = a dpower with
 * dpower = (Q d) . dmu - 1/2 d^T dQ d, d = x - mu. */
static void pixel_tangent(double px, double py, int64_t M, const int64_t *order, const proj_t *proj,
                          const double *opacity, const double *color, const orc_opts *o, const double *dmu_all,
                          const double *dQ_all, const double *dcol_all, contrib_t *list, double rgb[3],
                          double jac[18])
{
    int32_t n;
    composite_pixel(px, py, M, order, proj, opacity, color, o, 0.0, rgb, &n, NULL, NULL, list);
    double dT[6] = {0, 0, 0, 0, 0, 0};
    for (int m = 0; m < 18; m++) jac[m] = 0;
    for (int32_t k = 0; k < n; k++) {
        const contrib_t *e = &list[k];
        const int64_t i = e->id;
        const double *c = color + 3 * i, *Q = proj[i].Q;
        const double *dmu = dmu_all + 12 * i, *dQ = dQ_all + 18 * i;
        const double dx = e->dx, dy = e->dy;
        double da[6] = {0, 0, 0, 0, 0, 0};
        if (!e->clamped) {
            const double gx = Q[0] * dx + Q[1] * dy, gy = Q[1] * dx + Q[2] * dy;
            for (int j = 0; j < 6; j++) {
                double dpow = gx * dmu[j] + gy * dmu[6 + j] -
                              0.5 * (dQ[j] * dx * dx + 2.0 * dQ[6 + j] * dx * dy + dQ[12 + j] * dy * dy);
                da[j] = e->alpha * dpow;
            }
        }
        for (int j = 0; j < 6; j++) {
            for (int ch = 0; ch < 3; ch++) {
                jac[6 * ch + j] += c[ch] * (e->T * da[j] + e->alpha * dT[j]);
                if (dcol_all) jac[6 * ch + j] += e->alpha * e->T * dcol_all[18 * i + 6 * ch + j];
            }
            dT[j] = dT[j] * (1.0 - e->alpha) - e->T * da[j];
        }
    }
    for (int ch = 0; ch < 3; ch++)
        for (int j = 0; j < 6; j++) jac[6 * ch + j] += o->bg[ch] * dT[j];
}

/* Per-pixel Jacobian of the rendered colour with respect to the camera twist
 * (dphi, dt) of the left perturbation of T_CW, for the listed pixels:
 * jac (npix x 3 x 6), and the colour itself in rgb (npix x 3).  dcol
 * (N x 3 x 6, may be NULL) is the derivative of each Gaussian's colour with
 * respect to the twist (a view-dependent colour). */
int orc_render_jvp(int64_t N, const double *mean, const double *scale, const double *quat,
                   const double *opacity, const double *color, const double *dcol, const orc_camera *cam,
                   const orc_opts *o, int64_t npix, const int32_t *pix, double *rgb, double *jac)
{
    proj_t *proj;
    int64_t *order;
    int64_t M = build_order(N, mean, scale, quat, cam, o, &proj, &order);
    double *dmu = (double *)calloc((size_t)(N > 0 ? N : 1) * 12, sizeof(double));
    double *dQ = (double *)calloc((size_t)(N > 0 ? N : 1) * 18, sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < N; i++)
        if (proj[i].status & ORC_KEPT) project_tangent(&proj[i], cam, dmu + 12 * i, dQ + 18 * i);
    #pragma omp parallel
    {
        contrib_t *list = (contrib_t *)malloc(sizeof(contrib_t) * (size_t)(M > 0 ? M : 1));
        #pragma omp for schedule(dynamic, 16)
        for (int64_t p = 0; p < npix; p++)
            pixel_tangent(pix[2 * p] + 0.5, pix[2 * p + 1] + 0.5, M, order, proj, opacity, color, o, dmu, dQ, dcol,
                          list, rgb + 3 * p, jac + 18 * p);
        free(list);
    }
    free(dmu);
    free(dQ);
    free(proj);
    free(order);
    return 0;
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
