/*
 * FP64 CPU oracle for the sensitivity pass and sensitivity sampling of
 * "Provable Pruning for Efficient 3D Gaussian Splatting via Coresets".
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * HIP path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product library never
 * links or calls it, and it shares no code, header or constant with the HIP
 * sources.
 *
 * What it computes (paper section / equation cited at each function):
 *   - projection of each Gaussian into each view (Section 3, rendering query
 *     and scalar rendering function: kernel k, attenuation rho = alpha k,
 *     front-to-back order by view depth);
 *   - per-ray compositing: prefix transmittance T, contribution a = c rho T,
 *     render A = sum a  (Section 3, scalar rendering function);
 *   - importance a/A and sensitivity s = max over rays (Section 3.2, Eq. sen),
 *     rays with A = 0 skipped (Section 3.2);
 *   - sampling m i.i.d. indices with p proportional to s and weights
 *     n_i / (m p_i) (Algorithm 1, steps 4-5; proof of Theorem 2);
 *   - objectives: full A, fixed relaxation A^th_w, true reduced render A_w,
 *     validity count and log-transmittance gap (Section 3, pruned scene;
 *     Section 3.3, Definition 2 and Assumption 1).
 *
 * Conventions the paper leaves open are fixed as follows (each is a reading,
 * not a statement of the paper):
 *   - k is the unnormalised peak-1 Gaussian of the local-affine (EWA)
 *     projection of Sigma, truncated to the Mahalanobis ellipse d^2 <= r^2
 *     (r = 3 by default; the appendix's 3-sigma footprint), boundary included;
 *   - the 2D covariance gets an isotropic dilation delta (pixels^2);
 *   - Gaussians with camera depth z <= z_near are absent from the view;
 *   - order: ascending float32-rounded camera depth, ties by index;
 *   - pixel centres at (px + 1/2, py + 1/2); OpenCV camera axes;
 *   - colour: real SH (degree <= 3) evaluated at the direction from the
 *     camera centre to the mean, plus 1/2, clamped at 0; the per-ray query
 *     sums the three channels (mode 0), or uses colour 1 (mode 1, the
 *     paper's "nocolor" variant);
 *   - Sigma = R(q) diag(exp(2 l)) R(q)^T with q normalised.
 *
 * Parity unpinned (the paper fixes none of these): dilation value, SH basis
 * sign convention, pixel-centre offset, field-of-view axis.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int32_t sh_degree;
    const float *mean;      /* [3][n] */
    const float *log_scale; /* [3][n] */
    const float *quat;      /* [4][n] w x y z */
    const float *opacity;   /* [n] */
    const float *sh;        /* [(deg+1)^2][3][n] */
} ora_scene;

typedef struct {
    int32_t n_views;
    const double *world_to_cam; /* [V][12] row-major [R|t] */
    const double *intrinsics;   /* [V][4] fx fy cx cy */
    const int32_t *size;        /* [V][2] width height */
} ora_views;

typedef struct {
    double footprint_sigma; /* r */
    double dilation;        /* delta, px^2 */
    double z_near;
    double share_floor;     /* only used to count "live" pairs */
    double ambiguity_beta;  /* relative band around d^2 = r^2 that flags a pair */
    int32_t query_mode;     /* 0: RGB sum, 1: colour 1 (nocolor), 2: L2 of the RGB sum, 3: per channel */
    int32_t n_threads;
} ora_params;

/* Per (view, Gaussian) projection result. */
typedef struct {
    int present;        /* z > z_near */
    double z;           /* camera depth */
    float key;          /* float32 rounding of z (order key) */
    int key_ambiguous;  /* z within 2^-40 z of a float32 rounding midpoint */
    double mx, my;      /* projected mean, pixels */
    double cov[3];      /* Sigma_2d: xx, xy, yy (with dilation) */
    double conic[3];    /* inverse of Sigma_2d: xx, xy, yy */
    double rgb[3];      /* clamped colour per channel */
    double cbar;        /* colour factor of the query: sum of channels (mode 0), 1 (mode 1),
                           sum of squared channels (mode 2), largest channel (mode 3) */
    double alpha;
    double rx, ry;      /* half extents of the r-ellipse */
} ora_proj;

/* ------------------------------------------------------------------------ */
/* Real spherical harmonics, orthonormal on the unit sphere, degree <= 3.
 * Index k = l^2 + l + m.  (x, y, z) must be a unit vector. */
void ora_sh_basis(double x, double y, double z, double *Y)
{
    const double pi = 3.14159265358979323846;
    Y[0] = 0.5 * sqrt(1.0 / pi);
    Y[1] = sqrt(3.0 / (4.0 * pi)) * y;
    Y[2] = sqrt(3.0 / (4.0 * pi)) * z;
    Y[3] = sqrt(3.0 / (4.0 * pi)) * x;
    Y[4] = 0.5 * sqrt(15.0 / pi) * x * y;
    Y[5] = 0.5 * sqrt(15.0 / pi) * y * z;
    Y[6] = 0.25 * sqrt(5.0 / pi) * (3.0 * z * z - 1.0);
    Y[7] = 0.5 * sqrt(15.0 / pi) * x * z;
    Y[8] = 0.25 * sqrt(15.0 / pi) * (x * x - y * y);
    Y[9] = 0.25 * sqrt(35.0 / (2.0 * pi)) * y * (3.0 * x * x - y * y);
    Y[10] = 0.5 * sqrt(105.0 / pi) * x * y * z;
    Y[11] = 0.25 * sqrt(21.0 / (2.0 * pi)) * y * (5.0 * z * z - 1.0);
    Y[12] = 0.25 * sqrt(7.0 / pi) * z * (5.0 * z * z - 3.0);
    Y[13] = 0.25 * sqrt(21.0 / (2.0 * pi)) * x * (5.0 * z * z - 1.0);
    Y[14] = 0.25 * sqrt(105.0 / pi) * z * (x * x - y * y);
    Y[15] = 0.25 * sqrt(35.0 / (2.0 * pi)) * x * (x * x - 3.0 * y * y);
}

/* Is z within 2^-40 z of a point where float32 rounding changes? */
static int key_is_ambiguous(double z)
{
    float f = (float)z;
    float up = nextafterf(f, INFINITY);
    float dn = nextafterf(f, -INFINITY);
    double mid_up = 0.5 * ((double)f + (double)up);
    double mid_dn = 0.5 * ((double)f + (double)dn);
    double band = ldexp(fabs(z), -40);
    return fabs(z - mid_up) <= band || fabs(z - mid_dn) <= band;
}

/* Projection of Gaussian i into view v (Section 3: camera map p -> R p + t,
 * projected kernel; local-affine projection of Sigma). */
void ora_project_one(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                     int32_t v, int64_t i, ora_proj *o)
{
    const int64_t n = g->n;
    const double *P = vw->world_to_cam + 12 * (int64_t)v;
    const double fx = vw->intrinsics[4 * v + 0], fy = vw->intrinsics[4 * v + 1];
    const double cx = vw->intrinsics[4 * v + 2], cy = vw->intrinsics[4 * v + 3];
    double mu[3] = {g->mean[i], g->mean[n + i], g->mean[2 * n + i]};
    double p[3];
    for (int r = 0; r < 3; ++r)
        p[r] = P[4 * r + 0] * mu[0] + P[4 * r + 1] * mu[1] + P[4 * r + 2] * mu[2] + P[4 * r + 3];
    memset(o, 0, sizeof(*o));
    o->z = p[2];
    o->present = p[2] > prm->z_near;
    o->alpha = g->opacity[i];
    if (!o->present) return;
    const double x = p[0], y = p[1], z = p[2];
    o->key = (float)z;
    o->key_ambiguous = key_is_ambiguous(z);

    /* Rotation of the normalised quaternion (w, x, y, z). */
    double qw = g->quat[i], qx = g->quat[n + i], qy = g->quat[2 * n + i], qz = g->quat[3 * n + i];
    double qn = sqrt(qw * qw + qx * qx + qy * qy + qz * qz);
    qw /= qn; qx /= qn; qy /= qn; qz /= qn;
    double Rq[3][3] = {
        {1 - 2 * (qy * qy + qz * qz), 2 * (qx * qy - qw * qz), 2 * (qx * qz + qw * qy)},
        {2 * (qx * qy + qw * qz), 1 - 2 * (qx * qx + qz * qz), 2 * (qy * qz - qw * qx)},
        {2 * (qx * qz - qw * qy), 2 * (qy * qz + qw * qx), 1 - 2 * (qx * qx + qy * qy)}};
    double sc[3] = {exp(g->log_scale[i]), exp(g->log_scale[n + i]), exp(g->log_scale[2 * n + i])};

    /* Jacobian of (x, y, z) -> (fx x / z + cx, fy y / z + cy). */
    double J[2][3] = {{fx / z, 0.0, -fx * x / (z * z)}, {0.0, fy / z, -fy * y / (z * z)}};
    double Rv[3][3];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) Rv[r][c] = P[4 * r + c];
    /* M = J Rv Rq diag(sc) */
    double JR[2][3], M[2][3];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += J[r][k] * Rv[k][c];
            JR[r][c] = acc;
        }
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < 3; ++k) acc += JR[r][k] * Rq[k][c];
            M[r][c] = acc * sc[c];
        }
    double sxx = 0, sxy = 0, syy = 0;
    for (int k = 0; k < 3; ++k) {
        sxx += M[0][k] * M[0][k];
        sxy += M[0][k] * M[1][k];
        syy += M[1][k] * M[1][k];
    }
    sxx += prm->dilation;
    syy += prm->dilation;
    o->cov[0] = sxx; o->cov[1] = sxy; o->cov[2] = syy;
    double det = sxx * syy - sxy * sxy;
    o->conic[0] = syy / det;
    o->conic[1] = -sxy / det;
    o->conic[2] = sxx / det;
    o->mx = fx * x / z + cx;
    o->my = fy * y / z + cy;
    o->rx = prm->footprint_sigma * sqrt(sxx);
    o->ry = prm->footprint_sigma * sqrt(syy);

    /* View-dependent colour: SH at the unit direction camera centre -> mean. */
    double cam[3];
    for (int c = 0; c < 3; ++c)
        cam[c] = -(P[0 * 4 + c] * P[3] + P[1 * 4 + c] * P[7] + P[2 * 4 + c] * P[11]);
    double d[3] = {mu[0] - cam[0], mu[1] - cam[1], mu[2] - cam[2]};
    double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    double Y[16];
    ora_sh_basis(d[0] / dn, d[1] / dn, d[2] / dn, Y);
    int K = (g->sh_degree + 1) * (g->sh_degree + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < K; ++k) acc += Y[k] * (double)g->sh[((int64_t)k * 3 + ch) * n + i];
        acc += 0.5;
        o->rgb[ch] = acc > 0.0 ? acc : 0.0;
    }
    if (prm->query_mode == 1) o->cbar = 1.0;
    else if (prm->query_mode == 2) o->cbar = o->rgb[0] * o->rgb[0] + o->rgb[1] * o->rgb[1] + o->rgb[2] * o->rgb[2];
    else if (prm->query_mode == 3) o->cbar = fmax(o->rgb[0], fmax(o->rgb[1], o->rgb[2]));
    else o->cbar = o->rgb[0] + o->rgb[1] + o->rgb[2];
}

/* Query variants (Section 3.5, additional variants, and Algorithm 1's
 * per-channel queries).  Each ray holds nq queries: one for the pixel-level
 * objectives, three (R, G, B) per channel.  A Gaussian's contributions to
 * them at a pair with attenuation rho and prefix transmittance T:
 *   mode 0 (L1, RGB sum):  a = (c_R + c_G + c_B) rho T
 *   mode 1 (nocolor):      a = rho T
 *   mode 2 (L2):           a = (c_R^2 + c_G^2 + c_B^2) rho^2 T^2, the three
 *                          channels' squared contributions summed into one
 *                          pixel objective
 *   mode 3 (per channel):  a_k = c_k rho T for k = R, G, B.
 * Each query's objective A is the sum of its contributions over the ray.   */
static int n_queries(const ora_params *prm) { return prm->query_mode == 3 ? 3 : 1; }

static void pair_contrib(const ora_params *prm, const ora_proj *o, double rho, double T, double *a)
{
    if (prm->query_mode == 3) {
        for (int k = 0; k < 3; ++k) a[k] = o->rgb[k] * rho * T;
    } else if (prm->query_mode == 2) {
        a[0] = o->cbar * (rho * T) * (rho * T);
    } else {
        a[0] = o->cbar * rho * T;
    }
}

/* Largest contribution any later Gaussian of the ray can make to one of its
 * queries (rho <= 1): c_max T, or c_max T^2 for the L2 objective.          */
static double later_bound(const ora_params *prm, double cbar_max, double T)
{
    return prm->query_mode == 2 ? cbar_max * T * T : cbar_max * T;
}

/* Batched projection for tests: fills arrays of length V*n (view-major). */
void ora_project(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                 int32_t *present, double *z, float *key, int32_t *key_amb, double *mean2d /*[V*n][2]*/,
                 double *cov /*[V*n][3]*/, double *conic /*[V*n][3]*/, double *rgb /*[V*n][3]*/,
                 double *cbar, double *radius /*[V*n][2]*/)
{
    for (int32_t v = 0; v < vw->n_views; ++v)
        for (int64_t i = 0; i < g->n; ++i) {
            ora_proj o;
            ora_project_one(g, vw, prm, v, i, &o);
            int64_t j = (int64_t)v * g->n + i;
            present[j] = o.present;
            z[j] = o.z;
            key[j] = o.key;
            key_amb[j] = o.key_ambiguous;
            mean2d[2 * j] = o.mx; mean2d[2 * j + 1] = o.my;
            for (int c = 0; c < 3; ++c) {
                cov[3 * j + c] = o.cov[c];
                conic[3 * j + c] = o.conic[c];
                rgb[3 * j + c] = o.rgb[c];
            }
            cbar[j] = o.cbar;
            radius[2 * j] = o.rx; radius[2 * j + 1] = o.ry;
        }
}

/* ------------------------------------------------------------------------ */
/* Front-to-back order (Section 3: order induced by view depths).           */
typedef struct { float key; int64_t idx; } ora_order;

static int order_cmp(const void *a, const void *b)
{
    const ora_order *x = (const ora_order *)a, *y = (const ora_order *)b;
    if (x->key < y->key) return -1;
    if (x->key > y->key) return 1;
    return (x->idx > y->idx) - (x->idx < y->idx);
}

typedef struct {
    ora_proj *proj;   /* [n] projections for this view */
    ora_order *order; /* present Gaussians in front-to-back order */
    int64_t n_present;
    double cbar_max;  /* largest query colour among present Gaussians */
} ora_view_setup;

static void setup_view(const ora_scene *g, const ora_views *vw, const ora_params *prm, int32_t v,
                       ora_view_setup *s)
{
    s->proj = (ora_proj *)malloc(sizeof(ora_proj) * (size_t)g->n);
    s->order = (ora_order *)malloc(sizeof(ora_order) * (size_t)g->n);
    s->n_present = 0;
    s->cbar_max = 0.0;
    for (int64_t i = 0; i < g->n; ++i) {
        ora_project_one(g, vw, prm, v, i, &s->proj[i]);
        if (s->proj[i].present) {
            s->order[s->n_present].key = s->proj[i].key;
            s->order[s->n_present].idx = i;
            s->n_present++;
            if (s->proj[i].cbar > s->cbar_max) s->cbar_max = s->proj[i].cbar;
        }
    }
    qsort(s->order, (size_t)s->n_present, sizeof(ora_order), order_cmp);
}

static void free_view(ora_view_setup *s)
{
    free(s->proj);
    free(s->order);
}

/* Pixel range [lo, hi] whose centres can lie inside the ellipse (conservative). */
static void pixel_range(double m, double r, int32_t extent, int32_t *lo, int32_t *hi)
{
    double a = floor(m - r - 0.5) - 1.0, b = ceil(m + r - 0.5) + 1.0;
    if (a < 0) a = 0;
    if (b > extent - 1) b = extent - 1;
    *lo = (int32_t)a;
    *hi = (int32_t)b;
}

static inline int ray_selected(const uint32_t *mask, int64_t ray)
{
    return mask == NULL || ((mask[ray >> 5] >> (ray & 31)) & 1u);
}

/* ------------------------------------------------------------------------ */
/* Sensitivity (Section 3.2, Eq. sen): for every ray q with A(q) > 0,
 * s_i = max_q a_i(q) / A(q).  Every ray is composited front to back: the
 * Gaussians of the view are visited in order and each one updates the rays
 * inside its ellipse, so each ray sees its Gaussians in order.              */
typedef struct {
    const ora_scene *g;
    const ora_views *vw;
    const ora_params *prm;
    const uint32_t *ray_mask;
    int32_t view;
    int64_t ray_base;       /* global index of the view's first ray */
    int32_t band_rows;
    int32_t n_threads, tid;
    ora_view_setup *setup;
    /* outputs */
    double *A;            /* [rays] (nullable) */
    uint8_t *ray_flag;    /* [rays] (nullable) */
    double *s_thread;     /* this worker's private max array [n] */
    int64_t pairs, live_pairs, rays_positive;
} sens_worker;

/* Threads split the Gaussians of one view for projection. */
static void *project_worker_main(void *arg)
{
    sens_worker *w = (sens_worker *)arg;
    ora_view_setup *S = w->setup;
    for (int64_t i = w->tid; i < w->g->n; i += w->n_threads)
        ora_project_one(w->g, w->vw, w->prm, w->view, i, &S->proj[i]);
    return NULL;
}

/* Threads take bands of rows of one view, round robin. */
static void *sens_worker_main(void *arg)
{
    sens_worker *w = (sens_worker *)arg;
    const double r2 = w->prm->footprint_sigma * w->prm->footprint_sigma;
    const double beta = w->prm->ambiguity_beta;
    const int32_t v = w->view;
    const int32_t W = w->vw->size[2 * v], H = w->vw->size[2 * v + 1];
    ora_view_setup *S = w->setup;
    for (int32_t y0 = w->tid * w->band_rows; y0 < H; y0 += w->n_threads * w->band_rows) {
        const int32_t y1 = y0 + w->band_rows < H ? y0 + w->band_rows : H; /* exclusive */
        const int64_t npix = (int64_t)(y1 - y0) * W;
        const int64_t base = w->ray_base + (int64_t)y0 * W;
        const int nq = n_queries(w->prm);
        double *T = (double *)malloc(sizeof(double) * (size_t)npix);
        double *A = (double *)calloc((size_t)(npix * nq), sizeof(double));   /* [pixel][query] */
        uint8_t *sel = (uint8_t *)malloc((size_t)npix);
        uint8_t *flag = (uint8_t *)calloc((size_t)npix, 1);
        uint8_t row_on[16] = {0};
        int any = 0;
        for (int64_t p = 0; p < npix; ++p) {
            sel[p] = (uint8_t)ray_selected(w->ray_mask, base + p);
            row_on[p / W] |= sel[p];
            any |= sel[p];
            T[p] = 1.0;
        }
        if (any) {
            /* Pass 1: T and A for every selected ray of the band. */
            for (int64_t k = 0; k < S->n_present; ++k) {
                const ora_proj *o = &S->proj[S->order[k].idx];
                int32_t ylo, yhi, xlo, xhi;
                pixel_range(o->my, o->ry, H, &ylo, &yhi);
                if (yhi < y0 || ylo >= y1) continue;
                if (ylo < y0) ylo = y0;
                if (yhi > y1 - 1) yhi = y1 - 1;
                pixel_range(o->mx, o->rx, W, &xlo, &xhi);
                for (int32_t py = ylo; py <= yhi; ++py) {
                    if (!row_on[py - y0]) continue;
                    for (int32_t px = xlo; px <= xhi; ++px) {
                        int64_t p = (int64_t)(py - y0) * W + px;
                        if (!sel[p]) continue;
                        double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                        double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                        if (fabs(d2 - r2) <= beta * r2 || (o->key_ambiguous && d2 <= r2 * (1.0 + beta)))
                            flag[p] = 1;
                        if (d2 > r2) continue;
                        double rho = o->alpha * exp(-0.5 * d2), a[3];
                        pair_contrib(w->prm, o, rho, T[p], a);
                        for (int q = 0; q < nq; ++q) A[p * nq + q] += a[q];
                        T[p] *= (1.0 - rho);
                    }
                }
            }
            /* Pass 2: shares a/A on the queries with A > 0; running maxima.
             * A ray counts as positive if one of its queries is.            */
            uint8_t *pos = (uint8_t *)calloc((size_t)npix, 1);
            double *Amin = (double *)malloc(sizeof(double) * (size_t)npix);
            for (int64_t p = 0; p < npix; ++p) {
                T[p] = 1.0;
                Amin[p] = A[p * nq];
                for (int q = 0; q < nq; ++q) {
                    if (A[p * nq + q] > 0.0) pos[p] = 1;
                    if (A[p * nq + q] < Amin[p]) Amin[p] = A[p * nq + q];
                }
                if (sel[p] && pos[p]) w->rays_positive++;
            }
            for (int64_t k = 0; k < S->n_present; ++k) {
                const int64_t i = S->order[k].idx;
                const ora_proj *o = &S->proj[i];
                int32_t ylo, yhi, xlo, xhi;
                pixel_range(o->my, o->ry, H, &ylo, &yhi);
                if (yhi < y0 || ylo >= y1) continue;
                if (ylo < y0) ylo = y0;
                if (yhi > y1 - 1) yhi = y1 - 1;
                pixel_range(o->mx, o->rx, W, &xlo, &xhi);
                for (int32_t py = ylo; py <= yhi; ++py) {
                    if (!row_on[py - y0]) continue;
                    for (int32_t px = xlo; px <= xhi; ++px) {
                        int64_t p = (int64_t)(py - y0) * W + px;
                        if (!sel[p] || !pos[p]) continue;
                        double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                        double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                        if (d2 > r2) continue;
                        double rho = o->alpha * exp(-0.5 * d2), a[3];
                        pair_contrib(w->prm, o, rho, T[p], a);
                        for (int q = 0; q < nq; ++q) {
                            if (!(A[p * nq + q] > 0.0)) continue;
                            double share = a[q] / A[p * nq + q];
                            if (share > w->s_thread[i]) w->s_thread[i] = share;
                        }
                        w->pairs++;
                        /* live: some query of the ray could still receive a
                         * contribution of at least floor times its objective */
                        if (later_bound(w->prm, S->cbar_max, T[p]) >= w->prm->share_floor * Amin[p]) w->live_pairs++;
                        T[p] *= (1.0 - rho);
                    }
                }
            }
            free(pos); free(Amin);
        }
        for (int64_t p = 0; p < npix; ++p) {
            for (int q = 0; q < nq; ++q)
                if (w->A) w->A[(base + p) * nq + q] = sel[p] ? A[p * nq + q] : 0.0;
            if (w->ray_flag) w->ray_flag[base + p] = flag[p];
        }
        free(T); free(A); free(sel); free(flag);
    }
    return NULL;
}

/* Projection of one view with n_threads threads, then the depth order of the
 * present Gaussians whose pixel range meets a row band that holds a selected
 * ray (band_used[b] for rows [16 b, 16 b + 16)); the order of that subset is
 * the full order restricted to it, so skipping the others changes nothing. */
static void setup_view_threaded(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                                int32_t v, int nt, const uint8_t *band_used, ora_view_setup *s)
{
    s->proj = (ora_proj *)malloc(sizeof(ora_proj) * (size_t)g->n);
    s->order = (ora_order *)malloc(sizeof(ora_order) * (size_t)g->n);
    sens_worker *ws = (sens_worker *)calloc((size_t)nt, sizeof(sens_worker));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
    for (int t = 0; t < nt; ++t) {
        ws[t].g = g; ws[t].vw = vw; ws[t].prm = prm; ws[t].view = v;
        ws[t].n_threads = nt; ws[t].tid = t; ws[t].setup = s;
        pthread_create(&th[t], NULL, project_worker_main, &ws[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    free(ws); free(th);
    s->n_present = 0;
    s->cbar_max = 0.0;
    const int32_t H = vw->size[2 * v + 1];
    for (int64_t i = 0; i < g->n; ++i)
        if (s->proj[i].present) {
            int32_t ylo, yhi, use = 0;
            pixel_range(s->proj[i].my, s->proj[i].ry, H, &ylo, &yhi);
            if (s->proj[i].cbar > s->cbar_max) s->cbar_max = s->proj[i].cbar;
            for (int32_t b = ylo / 16; b <= yhi / 16 && !use; ++b) use = band_used[b];
            if (!use) continue;
            s->order[s->n_present].key = s->proj[i].key;
            s->order[s->n_present].idx = i;
            s->n_present++;
        }
    qsort(s->order, (size_t)s->n_present, sizeof(ora_order), order_cmp);
}

/* s: [n] out.  A: [rays][nq] out (nullable; nq = 3 per channel, else 1),
 * every query's objective, 0 on unselected rays.
 * ray_flag: [rays] out (nullable), 1 where some candidate pair lies within the
 * ambiguity band of the cutoff or has an ambiguous order key.
 * counters: [3] out = pairs with d^2 <= r^2 on selected rays with A > 0,
 * the subset still "live" (T c_max >= floor A), and the number of such rays.
 * Views are processed one after another; threads split each view's rows.   */
int ora_sensitivity(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                    const uint32_t *ray_mask, double *s, double *A, uint8_t *ray_flag, int64_t *counters)
{
    const int32_t V = vw->n_views;
    const int nt = prm->n_threads > 0 ? prm->n_threads : 1;
    sens_worker *ws = (sens_worker *)calloc((size_t)nt, sizeof(sens_worker));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
    for (int t = 0; t < nt; ++t) ws[t].s_thread = (double *)calloc((size_t)g->n, sizeof(double));
    int64_t ray_base = 0;
    for (int32_t v = 0; v < V; ++v) {
        const int64_t nrays = (int64_t)vw->size[2 * v] * vw->size[2 * v + 1];
        /* skip views with no selected ray; note which row bands hold one */
        const int32_t W = vw->size[2 * v], H = vw->size[2 * v + 1];
        uint8_t *band_used = (uint8_t *)calloc((size_t)(H / 16 + 1), 1);
        int any = 0;
        for (int32_t y = 0; y < H; ++y) {
            int row_any = ray_mask == NULL;
            for (int32_t x = 0; x < W && !row_any; ++x) row_any = ray_selected(ray_mask, ray_base + (int64_t)y * W + x);
            if (row_any) { band_used[y / 16] = 1; any = 1; }
        }
        if (!any) {
            for (int64_t p = 0; p < nrays; ++p) {
                for (int q = 0; q < n_queries(prm); ++q)
                    if (A) A[(ray_base + p) * n_queries(prm) + q] = 0.0;
                if (ray_flag) ray_flag[ray_base + p] = 0;
            }
            ray_base += nrays;
            free(band_used);
            continue;
        }
        ora_view_setup S;
        setup_view_threaded(g, vw, prm, v, nt, band_used, &S);
        free(band_used);
        for (int t = 0; t < nt; ++t) {
            sens_worker *w = &ws[t];
            w->g = g; w->vw = vw; w->prm = prm; w->ray_mask = ray_mask; w->view = v;
            w->ray_base = ray_base; w->band_rows = 16; w->n_threads = nt; w->tid = t;
            w->setup = &S; w->A = A; w->ray_flag = ray_flag;
            pthread_create(&th[t], NULL, sens_worker_main, w);
        }
        for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
        free_view(&S);
        ray_base += nrays;
    }
    int64_t c0 = 0, c1 = 0, c2 = 0;
    for (int64_t i = 0; i < g->n; ++i) s[i] = 0.0;
    for (int t = 0; t < nt; ++t) {
        for (int64_t i = 0; i < g->n; ++i)
            if (ws[t].s_thread[i] > s[i]) s[i] = ws[t].s_thread[i];
        c0 += ws[t].pairs; c1 += ws[t].live_pairs; c2 += ws[t].rays_positive;
        free(ws[t].s_thread);
    }
    if (counters) { counters[0] = c0; counters[1] = c1; counters[2] = c2; }
    free(ws); free(th);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* ------------------------------------------------------------------------ */
/* Aggregated sensitivities (Section 3.5, per-tile, per-image and per-scene
 * queries).  A query Q is a set of rays; a Gaussian's contribution to it is
 * a_i(Q) = sum over q in Q of a_i(q), the query objective is A(Q) = sum over
 * q in Q of A(q), and s_i = max over queries with A(Q) > 0 of a_i(Q) / A(Q).
 * level 1: Q = the rays of one 16x16 pixel tile of one view (ragged at the
 * right and bottom edges); level 2: Q = the rays of one view; level 3: one
 * query holding every ray.  Only rays selected by the mask belong to queries.
 * The 16-row bands the threads take are tile rows, so a band holds whole
 * tiles: after a Gaussian's visit the band knows its contribution to each
 * tile of the row.                                                          */
typedef struct {
    const ora_scene *g;
    const ora_views *vw;
    const ora_params *prm;
    const uint32_t *ray_mask;
    int32_t view, level;
    int64_t ray_base;
    int32_t n_threads, tid;
    ora_view_setup *setup;
    double *s_thread;   /* level 1: this worker's max over its tiles [n] */
    double *num;        /* levels 2, 3: this worker's sum of a_i over its rays [n] */
    double den;         /* levels 2, 3: this worker's sum of A over its rays */
} agg_worker;

static void *agg_worker_main(void *arg)
{
    agg_worker *w = (agg_worker *)arg;
    const double r2 = w->prm->footprint_sigma * w->prm->footprint_sigma;
    const int32_t v = w->view;
    const int32_t W = w->vw->size[2 * v], H = w->vw->size[2 * v + 1];
    const int32_t tiles_x = (W + 15) / 16;
    ora_view_setup *S = w->setup;
    double *tile_sum = (double *)calloc((size_t)tiles_x, sizeof(double));
    double *tile_A = (double *)malloc(sizeof(double) * (size_t)tiles_x);
    for (int32_t y0 = w->tid * 16; y0 < H; y0 += w->n_threads * 16) {
        const int32_t y1 = y0 + 16 < H ? y0 + 16 : H;
        const int64_t npix = (int64_t)(y1 - y0) * W;
        const int64_t base = w->ray_base + (int64_t)y0 * W;
        double *T = (double *)malloc(sizeof(double) * (size_t)npix);
        double *A = (double *)calloc((size_t)npix, sizeof(double));
        uint8_t *sel = (uint8_t *)malloc((size_t)npix);
        int any = 0;
        for (int64_t p = 0; p < npix; ++p) {
            sel[p] = (uint8_t)ray_selected(w->ray_mask, base + p);
            any |= sel[p];
            T[p] = 1.0;
        }
        if (any) {
            /* A(q) for every selected ray of the band, front to back */
            for (int64_t k = 0; k < S->n_present; ++k) {
                const ora_proj *o = &S->proj[S->order[k].idx];
                int32_t ylo, yhi, xlo, xhi;
                pixel_range(o->my, o->ry, H, &ylo, &yhi);
                if (yhi < y0 || ylo >= y1) continue;
                if (ylo < y0) ylo = y0;
                if (yhi > y1 - 1) yhi = y1 - 1;
                pixel_range(o->mx, o->rx, W, &xlo, &xhi);
                for (int32_t py = ylo; py <= yhi; ++py)
                    for (int32_t px = xlo; px <= xhi; ++px) {
                        int64_t p = (int64_t)(py - y0) * W + px;
                        if (!sel[p]) continue;
                        double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                        double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                        if (d2 > r2) continue;
                        double rho = o->alpha * exp(-0.5 * d2), a;
                        pair_contrib(w->prm, o, rho, T[p], &a);
                        A[p] += a;
                        T[p] *= (1.0 - rho);
                    }
            }
            /* query objectives: per tile of the row, or summed into den */
            for (int32_t tx = 0; tx < tiles_x; ++tx) tile_A[tx] = 0.0;
            for (int64_t p = 0; p < npix; ++p) {
                T[p] = 1.0;
                if (!sel[p]) continue;
                if (w->level == 1) tile_A[(p % W) / 16] += A[p];
                else w->den += A[p];
            }
            /* contributions a_i(q) summed over each query's rays */
            for (int64_t k = 0; k < S->n_present; ++k) {
                const int64_t i = S->order[k].idx;
                const ora_proj *o = &S->proj[i];
                int32_t ylo, yhi, xlo, xhi;
                pixel_range(o->my, o->ry, H, &ylo, &yhi);
                if (yhi < y0 || ylo >= y1) continue;
                if (ylo < y0) ylo = y0;
                if (yhi > y1 - 1) yhi = y1 - 1;
                pixel_range(o->mx, o->rx, W, &xlo, &xhi);
                for (int32_t py = ylo; py <= yhi; ++py)
                    for (int32_t px = xlo; px <= xhi; ++px) {
                        int64_t p = (int64_t)(py - y0) * W + px;
                        if (!sel[p]) continue;
                        double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                        double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                        if (d2 > r2) continue;
                        double rho = o->alpha * exp(-0.5 * d2), a;
                        pair_contrib(w->prm, o, rho, T[p], &a);
                        if (w->level == 1) tile_sum[px / 16] += a;
                        else w->num[i] += a;
                        T[p] *= (1.0 - rho);
                    }
                if (w->level == 1)
                    for (int32_t tx = xlo / 16; tx <= xhi / 16; ++tx) {
                        if (tile_A[tx] > 0.0) {
                            double share = tile_sum[tx] / tile_A[tx];
                            if (share > w->s_thread[i]) w->s_thread[i] = share;
                        }
                        tile_sum[tx] = 0.0;
                    }
            }
        }
        free(T); free(A); free(sel);
    }
    free(tile_sum); free(tile_A);
    return NULL;
}

/* s: [n] out, the aggregated sensitivities of `level` (1 tile, 2 image,
 * 3 scene).  Views one after another; threads split each view's tile rows;
 * per-image and per-scene sums are merged in thread order.                  */
int ora_sensitivity_agg(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                        const uint32_t *ray_mask, int32_t level, double *s)
{
    if (level < 1 || level > 3) return 1;
    /* an aggregated query sums its rays' channels (Section 3.5), so the
     * per-channel mode has no aggregated form of its own */
    if (n_queries(prm) != 1) return 2;
    const int32_t V = vw->n_views;
    const int nt = prm->n_threads > 0 ? prm->n_threads : 1;
    agg_worker *ws = (agg_worker *)calloc((size_t)nt, sizeof(agg_worker));
    pthread_t *th = (pthread_t *)malloc(sizeof(pthread_t) * (size_t)nt);
    double *num = (double *)calloc((size_t)g->n, sizeof(double));   /* scene level */
    double den = 0.0;
    for (int t = 0; t < nt; ++t) {
        ws[t].s_thread = (double *)calloc((size_t)g->n, sizeof(double));
        ws[t].num = (double *)calloc((size_t)g->n, sizeof(double));
    }
    for (int64_t i = 0; i < g->n; ++i) s[i] = 0.0;
    int64_t ray_base = 0;
    for (int32_t v = 0; v < V; ++v) {
        const int32_t W = vw->size[2 * v], H = vw->size[2 * v + 1];
        const int64_t nrays = (int64_t)W * H;
        uint8_t *band_used = (uint8_t *)calloc((size_t)(H / 16 + 1), 1);
        int any = 0;
        for (int32_t y = 0; y < H; ++y) {
            int row_any = ray_mask == NULL;
            for (int32_t x = 0; x < W && !row_any; ++x) row_any = ray_selected(ray_mask, ray_base + (int64_t)y * W + x);
            if (row_any) { band_used[y / 16] = 1; any = 1; }
        }
        if (any) {
            ora_view_setup S;
            setup_view_threaded(g, vw, prm, v, nt, band_used, &S);
            for (int t = 0; t < nt; ++t) {
                agg_worker *w = &ws[t];
                w->g = g; w->vw = vw; w->prm = prm; w->ray_mask = ray_mask; w->view = v; w->level = level;
                w->ray_base = ray_base; w->n_threads = nt; w->tid = t; w->setup = &S; w->den = 0.0;
                pthread_create(&th[t], NULL, agg_worker_main, w);
            }
            for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
            free_view(&S);
            if (level >= 2) {
                /* the view's sums, thread by thread */
                double dv = 0.0;
                for (int t = 0; t < nt; ++t) dv += ws[t].den;
                for (int64_t i = 0; i < g->n; ++i) {
                    double nv = 0.0;
                    for (int t = 0; t < nt; ++t) { nv += ws[t].num[i]; ws[t].num[i] = 0.0; }
                    if (level == 2) {
                        if (dv > 0.0 && nv / dv > s[i]) s[i] = nv / dv;
                    } else {
                        num[i] += nv;
                    }
                }
                den += dv;
            }
        }
        free(band_used);
        ray_base += nrays;
    }
    if (level == 1)
        for (int t = 0; t < nt; ++t)
            for (int64_t i = 0; i < g->n; ++i)
                if (ws[t].s_thread[i] > s[i]) s[i] = ws[t].s_thread[i];
    if (level == 3 && den > 0.0)
        for (int64_t i = 0; i < g->n; ++i) s[i] = num[i] / den;
    for (int t = 0; t < nt; ++t) { free(ws[t].s_thread); free(ws[t].num); }
    free(ws); free(th); free(num);
    return 0;
}

/* Objectives (Section 3): full render A, fixed relaxation
 * A^th_w = sum_i w_i a_i (full-scene transmittance), true reduced render
 * A_w = sum_i w_i c_i rho_i T_w,i with T_w,i = prod_{j before i} (1 - w_j rho_j).
 * The nocolor and L2 variants replace a_i by their contribution (with T_w
 * in place of T for the reduced render); per-channel queries are rejected.
 * Validity (Definition 2): pairs with w_i rho_i >= 1 are counted.
 * Log-transmittance gap (Assumption 1): gamma = max |log T - log T_w| over
 * contributing pairs (rho > 0) of retained Gaussians (w > 0), on rays where
 * every factor 1 - w rho stays positive.  log T and log T_w are kept as sums
 * of log(1 - rho_j) and log(1 - w_j rho_j), which equal the logs of the
 * products but do not underflow on long rays.                                */
int ora_objective(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                  const uint32_t *ray_mask, const double *w,
                  double *A_full, double *A_fixed, double *A_true, /* [rays] each, nullable */
                  double *view_sums /* [V][3] nullable */, int64_t *n_invalid, double *gamma)
{
    /* one objective per ray: the per-channel mode has three */
    if (n_queries(prm) != 1) return 2;
    const int32_t V = vw->n_views;
    const double r2 = prm->footprint_sigma * prm->footprint_sigma;
    int64_t ray0 = 0, invalid = 0;
    double gam = 0.0;
    for (int32_t v = 0; v < V; ++v) {
        const int32_t W = vw->size[2 * v], H = vw->size[2 * v + 1];
        const int64_t npix = (int64_t)W * H;
        ora_view_setup S;
        setup_view(g, vw, prm, v, &S);
        double *T = (double *)malloc(sizeof(double) * (size_t)npix);
        double *Tw = (double *)malloc(sizeof(double) * (size_t)npix);
        double *Af = (double *)calloc((size_t)npix, sizeof(double));
        double *Ax = (double *)calloc((size_t)npix, sizeof(double));
        double *At = (double *)calloc((size_t)npix, sizeof(double));
        double *gq = (double *)calloc((size_t)npix, sizeof(double));
        double *LT = (double *)calloc((size_t)npix, sizeof(double));  /* log T as a sum */
        double *LTw = (double *)calloc((size_t)npix, sizeof(double)); /* log T_w as a sum */
        uint8_t *bad = (uint8_t *)calloc((size_t)npix, 1);
        for (int64_t p = 0; p < npix; ++p) { T[p] = 1.0; Tw[p] = 1.0; }
        for (int64_t k = 0; k < S.n_present; ++k) {
            const int64_t i = S.order[k].idx;
            const ora_proj *o = &S.proj[i];
            int32_t ylo, yhi, xlo, xhi;
            pixel_range(o->my, o->ry, H, &ylo, &yhi);
            pixel_range(o->mx, o->rx, W, &xlo, &xhi);
            const double wi = w ? w[i] : 1.0;
            for (int32_t py = ylo; py <= yhi; ++py)
                for (int32_t px = xlo; px <= xhi; ++px) {
                    int64_t p = (int64_t)py * W + px;
                    if (!ray_selected(ray_mask, ray0 + p)) continue;
                    double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                    double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                    if (d2 > r2) continue;
                    double rho = o->alpha * exp(-0.5 * d2), a, aw;
                    pair_contrib(prm, o, rho, T[p], &a);
                    Af[p] += a;
                    Ax[p] += wi * a;
                    if (wi > 0.0) {
                        /* the reduced render: the same contribution with the
                         * retained scene's transmittance T_w */
                        pair_contrib(prm, o, rho, Tw[p], &aw);
                        At[p] += wi * aw;
                        if (!bad[p] && rho > 0.0) {
                            double gap = fabs(LT[p] - LTw[p]);
                            if (gap > gq[p]) gq[p] = gap;
                        }
                        if (wi * rho >= 1.0) { invalid++; bad[p] = 1; }
                        if (!bad[p]) LTw[p] += log1p(-wi * rho);
                        Tw[p] *= (1.0 - wi * rho);
                    }
                    LT[p] += log1p(-rho);
                    T[p] *= (1.0 - rho);
                }
        }
        double sf = 0, sx = 0, st = 0;
        for (int64_t p = 0; p < npix; ++p) {
            int on = ray_selected(ray_mask, ray0 + p) && Af[p] > 0.0;
            if (A_full) A_full[ray0 + p] = on ? Af[p] : 0.0;
            if (A_fixed) A_fixed[ray0 + p] = on ? Ax[p] : 0.0;
            if (A_true) A_true[ray0 + p] = on ? At[p] : 0.0;
            if (on) {
                sf += Af[p]; sx += Ax[p]; st += At[p];
                if (!bad[p] && gq[p] > gam) gam = gq[p];
            }
        }
        if (view_sums) { view_sums[3 * v] = sf; view_sums[3 * v + 1] = sx; view_sums[3 * v + 2] = st; }
        free(T); free(Tw); free(Af); free(Ax); free(At); free(gq); free(LT); free(LTw); free(bad);
        free_view(&S);
        ray0 += npix;
    }
    if (n_invalid) *n_invalid = invalid;
    if (gamma) *gamma = gam;
    return 0;
}

/* Rounding scale of the true reduced render (test infrastructure: it sets
 * the FP32 tolerance of A_w, it is not part of the method).  A relative error
 * d in rho_j moves the factor 1 - w_j rho_j by a relative
 * w_j rho_j d / |1 - w_j rho_j|, and with it T_w of every later pair of the
 * ray; per ray, to first order in d,
 *   |dA_w| <= d E,  E = sum_i |w_i a_i^w| k (1 + sum_{j before i} (1 + w_j rho_j) / |1 - w_j rho_j|),
 * with a_i^w the pair's contribution under T_w and k its degree in (rho_i,
 * T_w): 2 for the L2 objective, else 1.  A factor that is exactly 0 makes
 * E infinite.  Rays outside the mask or with A = 0 get 0.                 */
int ora_objective_true_scale(const ora_scene *g, const ora_views *vw, const ora_params *prm,
                             const uint32_t *ray_mask, const double *w, double *E /* [rays] */)
{
    if (n_queries(prm) != 1) return 2;
    const int32_t V = vw->n_views;
    const double r2 = prm->footprint_sigma * prm->footprint_sigma;
    const double kT = prm->query_mode == 2 ? 2.0 : 1.0;
    int64_t ray0 = 0;
    for (int32_t v = 0; v < V; ++v) {
        const int32_t W = vw->size[2 * v], H = vw->size[2 * v + 1];
        const int64_t npix = (int64_t)W * H;
        ora_view_setup S;
        setup_view(g, vw, prm, v, &S);
        double *T = (double *)malloc(sizeof(double) * (size_t)npix);
        double *Tw = (double *)malloc(sizeof(double) * (size_t)npix);
        double *Af = (double *)calloc((size_t)npix, sizeof(double));
        double *K = (double *)calloc((size_t)npix, sizeof(double));
        double *Es = (double *)calloc((size_t)npix, sizeof(double));
        for (int64_t p = 0; p < npix; ++p) { T[p] = 1.0; Tw[p] = 1.0; }
        for (int64_t k = 0; k < S.n_present; ++k) {
            const int64_t i = S.order[k].idx;
            const ora_proj *o = &S.proj[i];
            int32_t ylo, yhi, xlo, xhi;
            pixel_range(o->my, o->ry, H, &ylo, &yhi);
            pixel_range(o->mx, o->rx, W, &xlo, &xhi);
            const double wi = w ? w[i] : 1.0;
            for (int32_t py = ylo; py <= yhi; ++py)
                for (int32_t px = xlo; px <= xhi; ++px) {
                    int64_t p = (int64_t)py * W + px;
                    if (!ray_selected(ray_mask, ray0 + p)) continue;
                    double dx = (px + 0.5) - o->mx, dy = (py + 0.5) - o->my;
                    double d2 = o->conic[0] * dx * dx + 2.0 * o->conic[1] * dx * dy + o->conic[2] * dy * dy;
                    if (d2 > r2) continue;
                    double rho = o->alpha * exp(-0.5 * d2), a, aw;
                    pair_contrib(prm, o, rho, T[p], &a);
                    Af[p] += a;
                    T[p] *= (1.0 - rho);
                    if (wi > 0.0) {
                        pair_contrib(prm, o, rho, Tw[p], &aw);
                        Es[p] += fabs(wi * aw) * kT * (1.0 + K[p]);
                        const double f = 1.0 - wi * rho;
                        K[p] += (1.0 + fabs(wi * rho)) / fabs(f);
                        Tw[p] *= f;
                    }
                }
        }
        for (int64_t p = 0; p < npix; ++p) {
            const int on = ray_selected(ray_mask, ray0 + p) && Af[p] > 0.0;
            E[ray0 + p] = on ? Es[p] : 0.0;
        }
        free(T); free(Tw); free(Af); free(K); free(Es);
        free_view(&S);
        ray0 += npix;
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC 2011): 10 rounds of the Philox S-P network on a
 * 4x32-bit counter with a 2x32-bit key bumped by the Weyl constants.        */
void ora_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * c2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t n0 = hi1 ^ c1 ^ k0;
        uint32_t n1 = lo1;
        uint32_t n2 = hi0 ^ c3 ^ k1;
        uint32_t n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* Integer target of one draw: floor(u Q / 2^128) for the 128-bit value
 * u = x0 + 2^32 x1 + 2^64 x2 + 2^96 x3, computed exactly. */
uint64_t ora_draw_target(const uint32_t x[4], uint64_t Q)
{
    unsigned __int128 u_lo = ((unsigned __int128)x[1] << 32) | x[0];
    unsigned __int128 u_hi = ((unsigned __int128)x[3] << 32) | x[2];
    unsigned __int128 lo_prod = u_lo * Q;              /* < 2^128 */
    unsigned __int128 hi_prod = u_hi * Q;              /* < 2^128 */
    unsigned __int128 mid = hi_prod + (lo_prod >> 64); /* = floor(u Q / 2^64) < 2^128 */
    return (uint64_t)(mid >> 64);
}

/* Sensitivity sampling (Algorithm 1, steps 3-5; proof of Theorem 2).
 * p_i is realised exactly as q_i / Q with q_i = ceil(s_i 2^40) (0 iff s_i = 0)
 * and Q = sum q_i; draw t maps the 128-bit Philox output u to the integer
 * target floor(u Q / 2^128) and picks the first i whose inclusive prefix sum
 * exceeds it.  Weights w_i = n_i Q / (m q_i) for drawn i, 0 otherwise.
 * Returns 0, or 4 if every s_i is 0, or 1 on bad arguments.                 */
int ora_sample(const float *s, int64_t n, int64_t m, uint64_t seed,
               uint32_t *counts, double *weights, int64_t *support, uint64_t *Q_out)
{
    if (n < 1 || m < 1) return 1;
    /* A sensitivity is a largest share (Eq. sen), so it lies in [0, 1]; the
     * float32 value of a share can exceed 1 by a few ulps, so values up to
     * 1 + 2^-10 are accepted.  With n <= 2^24 - 2^16 such values keep
     * Q = sum ceil(s 2^40) below 2^64.  Anything else (NaN included) is
     * rejected with every output zeroed. */
    for (int64_t i = 0; i < n; ++i)
        if (!(s[i] >= 0.0f && s[i] <= 1.0009765625f) || n > ((int64_t)1 << 24) - ((int64_t)1 << 16)) {
            for (int64_t j = 0; j < n; ++j) { counts[j] = 0; weights[j] = 0.0; }
            *support = 0;
            if (Q_out) *Q_out = 0;
            return 5;
        }
    uint64_t *q = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t *C = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)n);
    uint64_t acc = 0;
    for (int64_t i = 0; i < n; ++i) {
        double x = ldexp((double)s[i], 40);
        q[i] = s[i] > 0.0f ? (uint64_t)ceil(x) : 0u;
        acc += q[i];
        C[i] = acc;
        counts[i] = 0;
        weights[i] = 0.0;
    }
    const uint64_t Q = acc;
    if (Q_out) *Q_out = Q;
    if (Q == 0) {
        *support = 0;
        free(q); free(C);
        return 4;
    }
    const uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t t = 0; t < m; ++t) {
        uint32_t ctr[4] = {(uint32_t)t, (uint32_t)((uint64_t)t >> 32), 0u, 0u}, x[4];
        ora_philox4x32_10(ctr, key, x);
        uint64_t target = ora_draw_target(x, Q);
        /* first i with C[i] > target */
        int64_t lo = 0, hi = n - 1;
        while (lo < hi) {
            int64_t mididx = lo + (hi - lo) / 2;
            if (C[mididx] > target) hi = mididx; else lo = mididx + 1;
        }
        counts[lo]++;
    }
    int64_t sup = 0;
    for (int64_t i = 0; i < n; ++i)
        if (counts[i] > 0) {
            double num = (double)counts[i] * (double)Q;
            double den = (double)m * (double)q[i];
            weights[i] = num / den;
            sup++;
        }
    *support = sup;
    free(q); free(C);
    return 0;
}

/* ------------------------------------------------------------------------
 * Neighbourhood of each mean for the learned sampling proposal (features of
 * the proposal network; the paper has no learned part, so this follows the
 * feature definition the library documents, not a passage of the paper).
 *
 * For every Gaussian i, its k nearest other means by brute force over every
 * j != i.  The squared distance is a float32 value computed in this order,
 * each operation rounded to float32:  (dx*dx + dy*dy) + dz*dz  with
 * dx = float(x_j - x_i) etc.  Neighbours are ordered by (squared distance,
 * index), so ties go to the smaller index.  The decision which points are
 * neighbours is therefore taken in float32 on both sides; the features built
 * from the neighbours are then evaluated in FP64 by the Python layer.
 * idx [n][k]: neighbour indices (0xFFFFFFFF when fewer than k others exist);
 * d2 [n][k]: their float32 squared distances (+inf for missing ones).
 */
typedef struct {
    const float *mean;
    int64_t n;
    int k;
    int64_t i0, i1;
    uint32_t *idx;
    float *d2;
} knn_job;

static void *knn_worker(void *arg)
{
    knn_job *J = (knn_job *)arg;
    const int64_t n = J->n;
    const float *X = J->mean, *Y = J->mean + n, *Z = J->mean + 2 * n;
    for (int64_t i = J->i0; i < J->i1; ++i) {
        uint32_t *bi = J->idx + i * J->k;
        float *bd = J->d2 + i * J->k;
        for (int t = 0; t < J->k; ++t) { bi[t] = 0xFFFFFFFFu; bd[t] = INFINITY; }
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            volatile float dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            volatile float xx = dx * dx, yy = dy * dy, zz = dz * dz;
            volatile float s = xx + yy;
            const float d = s + zz;
            /* insert (d, j) into the sorted list if it precedes the last */
            const int last = J->k - 1;
            if (!(d < bd[last] || (d == bd[last] && (uint32_t)j < bi[last]))) continue;
            int t = last;
            while (t > 0 && (d < bd[t - 1] || (d == bd[t - 1] && (uint32_t)j < bi[t - 1]))) {
                bd[t] = bd[t - 1];
                bi[t] = bi[t - 1];
                --t;
            }
            bd[t] = d;
            bi[t] = (uint32_t)j;
        }
    }
    return NULL;
}

int ora_knn(const float *mean, int64_t n, int k, int n_threads, uint32_t *idx, float *d2)
{
    if (n < 1 || k < 1) return 1;
    int nt = n_threads < 1 ? 1 : n_threads;
    if (nt > 64) nt = 64;
    pthread_t th[64];
    knn_job jobs[64];
    for (int t = 0; t < nt; ++t) {
        jobs[t].mean = mean;
        jobs[t].n = n;
        jobs[t].k = k;
        jobs[t].i0 = n * t / nt;
        jobs[t].i1 = n * (t + 1) / nt;
        jobs[t].idx = idx;
        jobs[t].d2 = d2;
        pthread_create(&th[t], NULL, knn_worker, &jobs[t]);
    }
    for (int t = 0; t < nt; ++t) pthread_join(th[t], NULL);
    return 0;
}
