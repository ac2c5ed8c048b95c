/*
 * swgs_oracle.c -- plain, slow FP64 CPU oracle for the sliding-window
 * Gaussian-splatting hot path (SwinGS, arXiv 2409.07759).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the tests, the smoke check and the CPU-baseline leg of
 * the bench use it.  It shares no code, header or constant table with the HIP
 * library: every formula here is written out from the paper (and, where the
 * paper defers to prior 3DGS work, from the readings listed in the design doc).
 *
 * Conventions (all arrays caller-owned, host memory):
 *   params  double[F*S]  planar rows: row r of slot i at params[r*S + i].
 *           rows 0-2 mean, 3-5 log-scale, 6-9 quaternion (w,x,y,z),
 *           10 opacity logit, 11+3k+ch SH coefficient k of channel ch.
 *   cam     double[16]   world->camera R (row-major 9), t (3), fx, fy, cx, cy.
 *   rec     double[S*REC] per-slot screen-space record of one view (below).
 *   images  planar [3][H][W]; pixel (x, y) has its centre at (x+0.5, y+0.5).
 *
 * Parity: every function here is pinned by tests/test_oracle_*.py against
 * closed forms, brute force, finite differences or library routines.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Threads for the per-slot and per-pixel loops (OpenMP).  The library
 * starts single-threaded; the CPU-baseline timing raises it.  Loops over
 * slots and pixels write disjoint outputs, so the thread count changes no
 * result, except the order in which the adjoint sums pixel contributions
 * into a slot's record gradient (with more than one thread: per-thread
 * partial sums, added in thread order). */
static int g_threads = 1;
void orc_set_threads(int n) { g_threads = n > 0 ? n : 1; }
int orc_get_threads(void) { return g_threads; }

/* Per-slot record of one view, as doubles. */
enum {
    R_U = 0, R_V, R_A, R_B, R_C, R_OPA, R_RED, R_GRN, R_BLU, R_DEPTH,
    R_COVA, R_COVB, R_COVC, R_HX, R_HY, R_MARGIN, REC
};

/* ------------------------------------------------------------------------
 * Philox4x32-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as
 * easy as 1, 2, 3", SC'11): ten rounds of two 32x32->64 multiplies with the
 * published multipliers, the key bumped by the published Weyl constants
 * between rounds.
 * ---------------------------------------------------------------------- */
void orc_philox4x32_10(const uint32_t ctr_in[4], const uint32_t key_in[2], uint32_t out[4])
{
    uint32_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint32_t k0 = key_in[0], k1 = key_in[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)c0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)c2;
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

/* ------------------------------------------------------------------------
 * Real spherical-harmonic basis up to degree 3 at a unit direction, in the
 * sign/order convention of the original 3DGS renderer that the paper uses
 * (Sec. 2.1; view-dependent colour degree from Sec. 8.1).  Normalisations
 * are written as their closed forms.
 * ---------------------------------------------------------------------- */
static double sh_k(int k)
{
    const double pi = 3.14159265358979323846;
    const double r = 1.0 / sqrt(pi);
    switch (k) {
    case 0: return 0.5 * r;                         /* 1/(2 sqrt(pi))        */
    case 1: return 0.5 * sqrt(3.0) * r;             /* sqrt(3)/(2 sqrt(pi))  */
    case 2: return 0.5 * sqrt(15.0) * r;            /* xy, yz, xz            */
    case 3: return 0.25 * sqrt(5.0) * r;            /* 2z^2-x^2-y^2          */
    case 4: return 0.25 * sqrt(15.0) * r;           /* x^2-y^2               */
    case 5: return 0.25 * sqrt(17.5) * r;           /* y(3x^2-y^2), x(x^2-3y^2) */
    case 6: return 0.5 * sqrt(105.0) * r;           /* xyz                   */
    case 7: return 0.25 * sqrt(10.5) * r;           /* y(4z^2-x^2-y^2), x(..) */
    case 8: return 0.25 * sqrt(7.0) * r;            /* z(2z^2-3x^2-3y^2)     */
    case 9: return 0.25 * sqrt(105.0) * r;          /* z(x^2-y^2)            */
    }
    return 0.0;
}

/* Y[k] and, if dY != NULL, dY[3k..3k+2] = d Y_k / d(x,y,z) treating x, y, z
 * as independent (the caller projects onto the sphere). */
void orc_sh_basis(int deg, const double d[3], double *Y, double *dY)
{
    double x = d[0], y = d[1], z = d[2];
    double g[16][3];
    memset(g, 0, sizeof g);
    Y[0] = sh_k(0);
    if (deg >= 1) {
        double c1 = sh_k(1);
        Y[1] = -c1 * y;  g[1][1] = -c1;
        Y[2] =  c1 * z;  g[2][2] =  c1;
        Y[3] = -c1 * x;  g[3][0] = -c1;
    }
    if (deg >= 2) {
        double a = sh_k(2), b = sh_k(3), c = sh_k(4);
        Y[4] =  a * x * y;                 g[4][0] = a * y; g[4][1] = a * x;
        Y[5] = -a * y * z;                 g[5][1] = -a * z; g[5][2] = -a * y;
        Y[6] =  b * (2 * z * z - x * x - y * y);
        g[6][0] = -2 * b * x; g[6][1] = -2 * b * y; g[6][2] = 4 * b * z;
        Y[7] = -a * x * z;                 g[7][0] = -a * z; g[7][2] = -a * x;
        Y[8] =  c * (x * x - y * y);       g[8][0] = 2 * c * x; g[8][1] = -2 * c * y;
    }
    if (deg >= 3) {
        double e = sh_k(5), f = sh_k(6), h = sh_k(7), m = sh_k(8), n = sh_k(9);
        double xx = x * x, yy = y * y, zz = z * z;
        Y[9]  = -e * y * (3 * xx - yy);
        g[9][0] = -e * 6 * x * y; g[9][1] = -e * (3 * xx - 3 * yy);
        Y[10] =  f * x * y * z;
        g[10][0] = f * y * z; g[10][1] = f * x * z; g[10][2] = f * x * y;
        Y[11] = -h * y * (4 * zz - xx - yy);
        g[11][0] = h * 2 * x * y; g[11][1] = -h * (4 * zz - xx - 3 * yy); g[11][2] = -h * 8 * y * z;
        Y[12] =  m * z * (2 * zz - 3 * xx - 3 * yy);
        g[12][0] = -m * 6 * x * z; g[12][1] = -m * 6 * y * z; g[12][2] = m * (6 * zz - 3 * xx - 3 * yy);
        Y[13] = -h * x * (4 * zz - xx - yy);
        g[13][0] = -h * (4 * zz - 3 * xx - yy); g[13][1] = h * 2 * x * y; g[13][2] = -h * 8 * x * z;
        Y[14] =  n * z * (xx - yy);
        g[14][0] = n * 2 * x * z; g[14][1] = -n * 2 * y * z; g[14][2] = n * (xx - yy);
        Y[15] = -e * x * (xx - 3 * yy);
        g[15][0] = -e * (3 * xx - 3 * yy); g[15][1] = e * 6 * x * y;
    }
    if (dY) {
        int nk = (deg + 1) * (deg + 1);
        for (int k = 0; k < nk; ++k)
            for (int j = 0; j < 3; ++j) dY[3 * k + j] = g[k][j];
    }
}

/* ------------------------------------------------------------------------
 * Small dense helpers (3x3 row-major).
 * ---------------------------------------------------------------------- */
static void quat_to_rot(const double q[4], double R[9])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

static double margin_rel(double value, double threshold)
{
    double s = fabs(threshold) > 1e-300 ? fabs(threshold) : 1.0;
    return fabs(value - threshold) / s;
}

/* distance of z to the nearest integer, relative to max(|z|, 1) */
static double margin_floor(double z)
{
    double d = fabs(z - nearbyint(z));
    double s = fabs(z) > 1.0 ? fabs(z) : 1.0;
    return d / s;
}

/* relative distance of z to the nearest FP32 rounding boundary.  A value
 * lying exactly on a boundary comes from an exact FP64 computation (an
 * inexact one lands there with probability ~2^-28), which any correct
 * implementation reproduces and rounds the same way (ties to even), so it
 * is not a near-decision. */
static double margin_f32(double z)
{
    float f = (float)z;
    double fd = (double)f;
    float up = nextafterf(f, INFINITY), dn = nextafterf(f, -INFINITY);
    double mid_up = 0.5 * (fd + (double)up), mid_dn = 0.5 * (fd + (double)dn);
    double d = fmin(fabs(z - mid_up), fabs(z - mid_dn));
    if (d == 0.0) return INFINITY;
    return d / (fabs(z) > 1e-300 ? fabs(z) : 1.0);
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }
static double softplus(double x) { return x > 0 ? x + log1p(exp(-x)) : log1p(exp(x)); }

/* ------------------------------------------------------------------------
 * Lifespan gate (Sec. 4.2: a Gaussian takes part in rendering a frame only
 * if start <= frame < expire; Algorithm 1's two filters).
 * ---------------------------------------------------------------------- */
int orc_active(int32_t start, int32_t expire, int frame)
{
    return start <= frame && frame < expire;
}

/* ------------------------------------------------------------------------
 * Screen-space record of slot i in one view (Eqs. 1-3 and Sec. 2.1: the 3D
 * Gaussian with covariance R S S^T R^T (Eq. 2) is replaced by its 2D
 * projection; the projection itself is the EWA first-order approximation of
 * the perspective map, a reading).  Returns 1 if the slot is visible.
 * rect[4] = tile range x0, y0, x1, y1 (half-open) for tiles of tw x th.
 * ---------------------------------------------------------------------- */
int orc_preprocess_one(const double *params, int64_t S, int64_t i, int deg,
                       const double cam[16], int W, int H, int tw, int th,
                       double *rec, int32_t *rect)
{
    const double *R = cam, *t = cam + 9;
    double fx = cam[12], fy = cam[13], cx = cam[14], cy = cam[15];
    double mu[3] = {params[0 * S + i], params[1 * S + i], params[2 * S + i]};
    double margin = INFINITY;
    for (int k = 0; k < REC; ++k) rec[k] = 0.0;
    rect[0] = rect[1] = rect[2] = rect[3] = 0;

    /* camera-space position; cull at the near plane z <= 0.2 */
    double p[3];
    for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + t[r];
    margin = fmin(margin, margin_rel(p[2], 0.2));
    if (p[2] <= 0.2) { rec[R_MARGIN] = margin; return 0; }

    /* projected mean (pinhole) */
    double u = fx * p[0] / p[2] + cx;
    double v = fy * p[1] / p[2] + cy;

    /* 3D covariance Sigma = M M^T, M = Rq diag(exp(s))  (Eq. 2) */
    double q[4] = {params[6 * S + i], params[7 * S + i], params[8 * S + i], params[9 * S + i]};
    double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) q[k] /= qn;
    double Rq[9];
    quat_to_rot(q, Rq);
    double sc[3] = {exp(params[3 * S + i]), exp(params[4 * S + i]), exp(params[5 * S + i])};
    double M[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
    double Sig[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += M[3 * r + k] * M[3 * c + k];
            Sig[3 * r + c] = acc;
        }

    /* Jacobian of the perspective map at the (FoV-clamped) camera point */
    double limx = 1.3 * (0.5 * W / fx), limy = 1.3 * (0.5 * H / fy);
    double txr = p[0] / p[2], tyr = p[1] / p[2];
    margin = fmin(margin, fmin(margin_rel(fabs(txr), limx), margin_rel(fabs(tyr), limy)));
    double tx = txr < -limx ? -limx : (txr > limx ? limx : txr);
    double ty = tyr < -limy ? -limy : (tyr > limy ? limy : tyr);
    double J[6] = {fx / p[2], 0.0, -fx * tx / p[2],
                   0.0, fy / p[2], -fy * ty / p[2]};
    /* T = J R_view (2x3); cov2 = T Sigma T^T + 0.3 I */
    double T[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = J[3 * r] * R[c] + J[3 * r + 1] * R[3 + c] + J[3 * r + 2] * R[6 + c];
    double ST0[3], ST1[3];
    for (int r = 0; r < 3; ++r) {
        ST0[r] = Sig[3 * r] * T[0] + Sig[3 * r + 1] * T[1] + Sig[3 * r + 2] * T[2];
        ST1[r] = Sig[3 * r] * T[3] + Sig[3 * r + 1] * T[4] + Sig[3 * r + 2] * T[5];
    }
    double ca = T[0] * ST0[0] + T[1] * ST0[1] + T[2] * ST0[2] + 0.3;
    double cb = T[0] * ST1[0] + T[1] * ST1[1] + T[2] * ST1[2];
    double cc = T[3] * ST1[0] + T[4] * ST1[1] + T[5] * ST1[2] + 0.3;
    double det = ca * cc - cb * cb;
    if (det <= 0.0) { rec[R_MARGIN] = margin; return 0; }
    double A = cc / det, B = -cb / det, C = ca / det;

    /* opacity and the exact support {alpha >= 1/255}: Q <= 2 ln(255 o) */
    double o = sigmoid(params[10 * S + i]);
    margin = fmin(margin, margin_rel(255.0 * o, 1.0));
    if (255.0 * o <= 1.0) { rec[R_MARGIN] = margin; return 0; }
    double kappa = 2.0 * log(255.0 * o);
    double hx = sqrt(kappa * ca), hy = sqrt(kappa * cc);

    /* tile range with a one-pixel pad, clipped to the grid */
    int ntx = (W + tw - 1) / tw, nty = (H + th - 1) / th;
    double zx0 = (u - hx - 1.0) / tw, zx1 = (u + hx + 1.0) / tw;
    double zy0 = (v - hy - 1.0) / th, zy1 = (v + hy + 1.0) / th;
    margin = fmin(margin, fmin(fmin(margin_floor(zx0), margin_floor(zx1)),
                               fmin(margin_floor(zy0), margin_floor(zy1))));
    double fx0 = floor(zx0), fx1 = floor(zx1) + 1.0, fy0 = floor(zy0), fy1 = floor(zy1) + 1.0;
    int x0 = fx0 < 0 ? 0 : (fx0 > ntx ? ntx : (int)fx0);
    int x1 = fx1 < 0 ? 0 : (fx1 > ntx ? ntx : (int)fx1);
    int y0 = fy0 < 0 ? 0 : (fy0 > nty ? nty : (int)fy0);
    int y1 = fy1 < 0 ? 0 : (fy1 > nty ? nty : (int)fy1);
    if (x0 >= x1 || y0 >= y1) { rec[R_MARGIN] = margin; return 0; }

    /* view-dependent colour: SH at the unit direction from the camera centre */
    double campos[3];
    for (int c = 0; c < 3; ++c) campos[c] = -(R[c] * t[0] + R[3 + c] * t[1] + R[6 + c] * t[2]);
    double dir[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
    double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int c = 0; c < 3; ++c) dir[c] /= dn;
    double Y[16];
    orc_sh_basis(deg, dir, Y, NULL);
    int nk = (deg + 1) * (deg + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += Y[k] * params[(11 + 3 * k + ch) * S + i];
        double val = acc + 0.5;
        rec[R_RED + ch] = val > 0.0 ? val : 0.0;
    }

    /* depth key: camera-space z rounded to FP32 */
    margin = fmin(margin, margin_f32(p[2]));
    rec[R_U] = u; rec[R_V] = v;
    rec[R_A] = A; rec[R_B] = B; rec[R_C] = C;
    rec[R_OPA] = o;
    rec[R_DEPTH] = (double)(float)p[2];
    rec[R_COVA] = ca; rec[R_COVB] = cb; rec[R_COVC] = cc;
    rec[R_HX] = hx; rec[R_HY] = hy;
    rec[R_MARGIN] = margin;
    rect[0] = x0; rect[1] = y0; rect[2] = x1; rect[3] = y1;
    return 1;
}

/* All slots of one view: visible[i], rec[i*REC..], rect[4i..]. Slots that
 * fail the lifespan gate are invisible. */
void orc_preprocess(const double *params, int64_t S, int deg,
                    const int32_t *start, const int32_t *expire, int frame,
                    const double cam[16], int W, int H, int tw, int th,
                    int32_t *visible, double *rec, int32_t *rect)
{
#pragma omp parallel for schedule(dynamic, 256) num_threads(g_threads)
    for (int64_t i = 0; i < S; ++i) {
        if (!orc_active(start[i], expire[i], frame)) {
            visible[i] = 0;
            for (int k = 0; k < REC; ++k) rec[i * REC + k] = 0.0;
            rec[i * REC + R_MARGIN] = INFINITY;
            rect[4 * i] = rect[4 * i + 1] = rect[4 * i + 2] = rect[4 * i + 3] = 0;
            continue;
        }
        visible[i] = orc_preprocess_one(params, S, i, deg, cam, W, H, tw, th,
                                        rec + i * REC, rect + 4 * i);
    }
}

/* ------------------------------------------------------------------------
 * Depth order: "close to far" (Sec. 2.1), i.e. ascending FP32 camera z,
 * ties broken by ascending slot.
 * ---------------------------------------------------------------------- */
static const double *g_sort_rec;
static int cmp_depth(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    double da = g_sort_rec[a * REC + R_DEPTH], db = g_sort_rec[b * REC + R_DEPTH];
    if (da < db) return -1;
    if (da > db) return 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

int64_t orc_depth_order(int64_t S, const int32_t *visible, const double *rec, int64_t *order)
{
    int64_t n = 0;
    for (int64_t i = 0; i < S; ++i)
        if (visible[i]) order[n++] = i;
    g_sort_rec = rec;
    qsort(order, (size_t)n, sizeof(int64_t), cmp_depth);
    return n;
}

/* ------------------------------------------------------------------------
 * Per-pixel blend (Eq. 3): walk all visible Gaussians in depth order;
 * alpha = min(0.99, o * exp(-Q/2)), skip alpha < 1/255, stop before the
 * transmittance would fall below 1e-4; C = sum c alpha T + T_final * bg.
 * Writes rgb, T_final, contributor count and the smallest relative margin
 * of any skip/stop decision (dmargin) and of the 0.99 clamp (cmargin).
 * ---------------------------------------------------------------------- */
static void blend_pixel(int64_t n, const int64_t *order, const double *rec,
                        double px, double py, const double bg[3],
                        double out[3], double *T_out, int32_t *ncontrib,
                        double *dmargin, double *cmargin)
{
    double T = 1.0, C[3] = {0, 0, 0};
    double dm = INFINITY, cm = INFINITY;
    int cnt = 0;
    for (int64_t k = 0; k < n; ++k) {
        const double *r = rec + order[k] * REC;
        double dx = px - r[R_U], dy = py - r[R_V];
        double Q = r[R_A] * dx * dx + 2.0 * r[R_B] * dx * dy + r[R_C] * dy * dy;
        double og = r[R_OPA] * exp(-0.5 * Q);
        cm = fmin(cm, margin_rel(og, 0.99));
        double alpha = og < 0.99 ? og : 0.99;
        dm = fmin(dm, margin_rel(alpha, 1.0 / 255.0));
        if (alpha < 1.0 / 255.0) continue;
        double Tn = T * (1.0 - alpha);
        dm = fmin(dm, margin_rel(Tn, 1e-4));
        if (Tn < 1e-4) break;
        for (int c = 0; c < 3; ++c) C[c] += r[R_RED + c] * alpha * T;
        T = Tn;
        ++cnt;
    }
    for (int c = 0; c < 3; ++c) out[c] = C[c] + T * bg[c];
    *T_out = T;
    *ncontrib = cnt;
    *dmargin = dm;
    *cmargin = cm;
}

/* Render a list of pixels (pix[j] = y*W + x), or all pixels when pix is
 * NULL.  out_rgb is [3][npix]. */
void orc_render(int64_t S, const int32_t *visible, const double *rec,
                int W, int H, const double bg[3], int64_t npix, const int64_t *pix,
                double *out_rgb, double *out_T, int32_t *out_n,
                double *out_dmargin, double *out_cmargin)
{
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    int64_t n = orc_depth_order(S, visible, rec, order);
    int64_t np = pix ? npix : (int64_t)W * H;
#pragma omp parallel for schedule(dynamic, 64) num_threads(g_threads)
    for (int64_t j = 0; j < np; ++j) {
        int64_t id = pix ? pix[j] : j;
        double px = (double)(id % W) + 0.5, py = (double)(id / W) + 0.5;
        double c[3];
        blend_pixel(n, order, rec, px, py, bg, c, &out_T[j], &out_n[j],
                    &out_dmargin[j], &out_cmargin[j]);
        for (int ch = 0; ch < 3; ++ch) out_rgb[ch * np + j] = c[ch];
    }
    free(order);
}

/* ------------------------------------------------------------------------
 * Adjoint of the blend for one view (Algorithm 1's backward through Eq. 3).
 * For each pixel the forward walk stores every contributor's alpha and
 * prefix transmittance T_k; the backward walk keeps, from the back,
 *   U = colour behind k as seen from just behind k   (U <- c a + (1-a) U)
 *   Rr = product of (1 - a_j) over contributors behind k
 * so that dC/da_k = T_k (c_k - U - Rr bg) without any division.
 * drec[i*9..] accumulates d/d(u, v, A, B, C, o, r, g, b) of slot i.
 * ---------------------------------------------------------------------- */
void orc_blend_backward_pixels(int64_t S, const int32_t *visible, const double *rec,
                               int W, int H, const double bg[3], const double *dLdC,
                               int64_t npix, const int64_t *pix, double *drec);

void orc_blend_backward(int64_t S, const int32_t *visible, const double *rec,
                        int W, int H, const double bg[3], const double *dLdC,
                        double *drec)
{
    orc_blend_backward_pixels(S, visible, rec, W, H, bg, dLdC, -1, NULL, drec);
}

/* Adjoint of one pixel: the forward walk stores its contributors (who, al,
 * Tk: scratch of n entries), the backward walk accumulates into drec. */
static void adjoint_pixel(int64_t n, const int64_t *order, const double *rec, double px, double py,
                          const double bg[3], const double g[3], int64_t *who, double *al, double *Tk,
                          double *drec)
{
    /* forward walk, storing contributors */
    double T = 1.0;
    int64_t m = 0;
    for (int64_t k = 0; k < n; ++k) {
        const double *r = rec + order[k] * REC;
        double dx = px - r[R_U], dy = py - r[R_V];
        double Q = r[R_A] * dx * dx + 2.0 * r[R_B] * dx * dy + r[R_C] * dy * dy;
        double og = r[R_OPA] * exp(-0.5 * Q);
        double alpha = og < 0.99 ? og : 0.99;
        if (alpha < 1.0 / 255.0) continue;
        double Tn = T * (1.0 - alpha);
        if (Tn < 1e-4) break;
        who[m] = order[k]; al[m] = alpha; Tk[m] = T; ++m;
        T = Tn;
    }
    /* backward walk */
    double U[3] = {0, 0, 0}, Rr = 1.0;
    for (int64_t j = m - 1; j >= 0; --j) {
        int64_t i = who[j];
        const double *r = rec + i * REC;
        double a = al[j], Tj = Tk[j];
        double dalpha = 0.0;
        for (int c = 0; c < 3; ++c) {
            dalpha += g[c] * Tj * (r[R_RED + c] - U[c] - Rr * bg[c]);
            drec[i * 9 + 6 + c] += g[c] * a * Tj;
        }
        for (int c = 0; c < 3; ++c) U[c] = r[R_RED + c] * a + (1.0 - a) * U[c];
        Rr *= (1.0 - a);
        double dx = px - r[R_U], dy = py - r[R_V];
        double Q = r[R_A] * dx * dx + 2.0 * r[R_B] * dx * dy + r[R_C] * dy * dy;
        double G = exp(-0.5 * Q);
        if (r[R_OPA] * G >= 0.99) continue;   /* clamped: alpha is constant */
        /* alpha = o G, G = exp(-Q/2) */
        drec[i * 9 + 5] += dalpha * G;
        double dQ = -0.5 * r[R_OPA] * G * dalpha;
        drec[i * 9 + 2] += dQ * dx * dx;
        drec[i * 9 + 3] += dQ * 2.0 * dx * dy;
        drec[i * 9 + 4] += dQ * dy * dy;
        /* dQ/ddx = 2(A dx + B dy); ddx/du = -1 */
        drec[i * 9 + 0] += -dQ * 2.0 * (r[R_A] * dx + r[R_B] * dy);
        drec[i * 9 + 1] += -dQ * 2.0 * (r[R_B] * dx + r[R_C] * dy);
    }
}

/* Same over a list of pixels (pix[j] = y*W + x, dLdC[3][npix]) or, when pix
 * is NULL, over the whole image (dLdC[3][W*H]).  Pixels are summed in
 * ascending order into drec (one thread), or into per-thread partials that
 * are then added in thread order. */
void orc_blend_backward_pixels(int64_t S, const int32_t *visible, const double *rec,
                               int W, int H, const double bg[3], const double *dLdC,
                               int64_t npix, const int64_t *pix, double *drec)
{
    int64_t *order = (int64_t *)malloc(sizeof(int64_t) * (size_t)(S > 0 ? S : 1));
    int64_t n = orc_depth_order(S, visible, rec, order);
    const size_t nn = (size_t)(n > 0 ? n : 1);
    int64_t P = pix ? npix : (int64_t)W * H;
    const int nt = g_threads;
    double *part = nt > 1 ? (double *)calloc((size_t)nt * (size_t)S * 9, sizeof(double)) : NULL;
#pragma omp parallel num_threads(nt)
    {
        const int tid = omp_get_thread_num();
        int64_t *who = (int64_t *)malloc(sizeof(int64_t) * nn);
        double *al = (double *)malloc(sizeof(double) * nn);
        double *Tk = (double *)malloc(sizeof(double) * nn);
        double *acc = part ? part + (size_t)tid * (size_t)S * 9 : drec;
#pragma omp for schedule(dynamic, 16)
        for (int64_t j = 0; j < P; ++j) {
            int64_t pid = pix ? pix[j] : j;
            double px = (double)(pid % W) + 0.5, py = (double)(pid / W) + 0.5;
            double g[3] = {dLdC[j], dLdC[P + j], dLdC[2 * P + j]};
            adjoint_pixel(n, order, rec, px, py, bg, g, who, al, Tk, acc);
        }
        free(who); free(al); free(Tk);
    }
    if (part) {
        for (int t = 0; t < nt; ++t) {
            const double *pt = part + (size_t)t * (size_t)S * 9;
            for (size_t k = 0; k < (size_t)S * 9; ++k) drec[k] += pt[k];
        }
        free(part);
    }
    free(order);
}

/* ------------------------------------------------------------------------
 * Adjoint of the per-slot preprocess for one view: from the record
 * gradient d(u, v, A, B, C, o, r, g, b) to the parameter gradient
 * (accumulated into dparams, planar rows like params).
 * ---------------------------------------------------------------------- */
void orc_preprocess_backward_one(const double *params, int64_t S, int64_t i, int deg,
                                 const double cam[16], int W, int H,
                                 const double dr[9], double *dparams)
{
    const double *R = cam, *t = cam + 9;
    double fx = cam[12], fy = cam[13];
    double mu[3] = {params[0 * S + i], params[1 * S + i], params[2 * S + i]};
    double p[3];
    for (int r = 0; r < 3; ++r) p[r] = R[3 * r] * mu[0] + R[3 * r + 1] * mu[1] + R[3 * r + 2] * mu[2] + t[r];

    /* ---- recompute the forward intermediates ---- */
    double qraw[4] = {params[6 * S + i], params[7 * S + i], params[8 * S + i], params[9 * S + i]};
    double qn = sqrt(qraw[0] * qraw[0] + qraw[1] * qraw[1] + qraw[2] * qraw[2] + qraw[3] * qraw[3]);
    double q[4];
    for (int k = 0; k < 4; ++k) q[k] = qraw[k] / qn;
    double Rq[9];
    quat_to_rot(q, Rq);
    double sc[3] = {exp(params[3 * S + i]), exp(params[4 * S + i]), exp(params[5 * S + i])};
    double M[9], Sig[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) M[3 * r + c] = Rq[3 * r + c] * sc[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += M[3 * r + k] * M[3 * c + k];
            Sig[3 * r + c] = acc;
        }
    double limx = 1.3 * (0.5 * W / fx), limy = 1.3 * (0.5 * H / fy);
    double txr = p[0] / p[2], tyr = p[1] / p[2];
    int clx = (txr < -limx || txr > limx), cly = (tyr < -limy || tyr > limy);
    double tx = txr < -limx ? -limx : (txr > limx ? limx : txr);
    double ty = tyr < -limy ? -limy : (tyr > limy ? limy : tyr);
    double J[6] = {fx / p[2], 0.0, -fx * tx / p[2], 0.0, fy / p[2], -fy * ty / p[2]};
    double T[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            T[3 * r + c] = J[3 * r] * R[c] + J[3 * r + 1] * R[3 + c] + J[3 * r + 2] * R[6 + c];
    double ST0[3], ST1[3];
    for (int r = 0; r < 3; ++r) {
        ST0[r] = Sig[3 * r] * T[0] + Sig[3 * r + 1] * T[1] + Sig[3 * r + 2] * T[2];
        ST1[r] = Sig[3 * r] * T[3] + Sig[3 * r + 1] * T[4] + Sig[3 * r + 2] * T[5];
    }
    double ca = T[0] * ST0[0] + T[1] * ST0[1] + T[2] * ST0[2] + 0.3;
    double cb = T[0] * ST1[0] + T[1] * ST1[1] + T[2] * ST1[2];
    double cc = T[3] * ST1[0] + T[4] * ST1[1] + T[5] * ST1[2] + 0.3;
    double det = ca * cc - cb * cb;
    double o = sigmoid(params[10 * S + i]);

    double dmu[3] = {0, 0, 0}, dp[3] = {0, 0, 0};

    /* ---- colour: rgb = max(0, sum_k Y_k f_k + 0.5) ---- */
    double campos[3];
    for (int c = 0; c < 3; ++c) campos[c] = -(R[c] * t[0] + R[3 + c] * t[1] + R[6 + c] * t[2]);
    double dir[3] = {mu[0] - campos[0], mu[1] - campos[1], mu[2] - campos[2]};
    double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    double dh[3] = {dir[0] / dn, dir[1] / dn, dir[2] / dn};
    double Y[16], dY[48];
    orc_sh_basis(deg, dh, Y, dY);
    int nk = (deg + 1) * (deg + 1);
    double ddh[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += Y[k] * params[(11 + 3 * k + ch) * S + i];
        if (acc + 0.5 <= 0.0) continue;            /* clamped channel */
        double g = dr[6 + ch];
        for (int k = 0; k < nk; ++k) {
            dparams[(11 + 3 * k + ch) * S + i] += Y[k] * g;
            double f = params[(11 + 3 * k + ch) * S + i] * g;
            for (int j = 0; j < 3; ++j) ddh[j] += f * dY[3 * k + j];
        }
    }
    /* dh = dir/|dir|: d dir = (I - dh dh^T) ddh / |dir| */
    double dd = ddh[0] * dh[0] + ddh[1] * dh[1] + ddh[2] * dh[2];
    for (int j = 0; j < 3; ++j) dmu[j] += (ddh[j] - dh[j] * dd) / dn;

    /* ---- opacity o = sigmoid(logit) ---- */
    dparams[10 * S + i] += dr[5] * o * (1.0 - o);

    /* ---- conic (A, B, C) = (c, -b, a)/det ---- */
    double dA = dr[2], dB = dr[3], dC = dr[4];
    double i2 = 1.0 / (det * det);
    double dca = (-cc * cc * dA + cb * cc * dB - cb * cb * dC) * i2;
    double dcb = (2.0 * cb * cc * dA - (ca * cc + cb * cb) * dB + 2.0 * ca * cb * dC) * i2;
    double dcc = (-cb * cb * dA + ca * cb * dB - ca * ca * dC) * i2;

    /* ---- cov2 = T Sigma T^T (+0.3 I): a = T0 S T0, b = T0 S T1, c = T1 S T1 ---- */
    double Gm[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c)
            Gm[3 * r + c] = dca * T[r] * T[c] + dcb * T[r] * T[3 + c] + dcc * T[3 + r] * T[3 + c];
    double dT[6];
    for (int c = 0; c < 3; ++c) {
        dT[c] = 2.0 * dca * ST0[c] + dcb * ST1[c];
        dT[3 + c] = dcb * ST0[c] + 2.0 * dcc * ST1[c];
    }
    /* T = J R_view: dJ = dT R_view^T */
    double dJ[6];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c)
            dJ[3 * r + c] = dT[3 * r] * R[3 * c] + dT[3 * r + 1] * R[3 * c + 1] + dT[3 * r + 2] * R[3 * c + 2];
    double z = p[2], z2 = z * z;
    dp[2] += dJ[0] * (-fx / z2) + dJ[2] * (fx * tx / z2) + dJ[4] * (-fy / z2) + dJ[5] * (fy * ty / z2);
    double dtx = dJ[2] * (-fx / z), dty = dJ[5] * (-fy / z);
    if (!clx) { dp[0] += dtx / z; dp[2] += -dtx * p[0] / z2; }
    if (!cly) { dp[1] += dty / z; dp[2] += -dty * p[1] / z2; }

    /* ---- mean2D ---- */
    dp[0] += dr[0] * fx / z;
    dp[2] += -dr[0] * fx * p[0] / z2;
    dp[1] += dr[1] * fy / z;
    dp[2] += -dr[1] * fy * p[1] / z2;

    /* ---- p = R_view mu + t ---- */
    for (int j = 0; j < 3; ++j) dmu[j] += R[j] * dp[0] + R[3 + j] * dp[1] + R[6 + j] * dp[2];
    for (int j = 0; j < 3; ++j) dparams[j * S + i] += dmu[j];

    /* ---- Sigma = M M^T: dM = (G + G^T) M ---- */
    double dM[9];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += (Gm[3 * r + k] + Gm[3 * k + r]) * M[3 * k + c];
            dM[3 * r + c] = acc;
        }
    /* M = Rq diag(sc) */
    double dRq[9];
    for (int c = 0; c < 3; ++c) {
        double ds = 0;
        for (int r = 0; r < 3; ++r) {
            dRq[3 * r + c] = dM[3 * r + c] * sc[c];
            ds += dM[3 * r + c] * Rq[3 * r + c];
        }
        dparams[(3 + c) * S + i] += ds * sc[c];
    }
    /* Rq(q) for unit q = (w, x, y, z) */
    double w = q[0], x = q[1], y = q[2], zq = q[3];
    double dq[4];
    dq[0] = 2 * (-zq * dRq[1] + y * dRq[2] + zq * dRq[3] - x * dRq[5] - y * dRq[6] + x * dRq[7]);
    dq[1] = 2 * (y * dRq[1] + zq * dRq[2] + y * dRq[3] - 2 * x * dRq[4] - w * dRq[5]
                 + zq * dRq[6] + w * dRq[7] - 2 * x * dRq[8]);
    dq[2] = 2 * (-2 * y * dRq[0] + x * dRq[1] + w * dRq[2] + x * dRq[3] + zq * dRq[5]
                 - w * dRq[6] + zq * dRq[7] - 2 * y * dRq[8]);
    dq[3] = 2 * (-2 * zq * dRq[0] - w * dRq[1] + x * dRq[2] + w * dRq[3] - 2 * zq * dRq[4]
                 + y * dRq[5] + x * dRq[6] + y * dRq[7]);
    /* q = qraw/|qraw| */
    double qd = dq[0] * q[0] + dq[1] * q[1] + dq[2] * q[2] + dq[3] * q[3];
    for (int k = 0; k < 4; ++k) dparams[(6 + k) * S + i] += (dq[k] - q[k] * qd) / qn;
}

/* The adjoint preprocess of every visible slot i < n (each writes its own
 * parameter column). */
void orc_preprocess_backward_many(const double *params, int64_t S, int deg, const double cam[16], int W, int H,
                                  const int32_t *visible, int64_t n, const double *drec, double *dparams)
{
#pragma omp parallel for schedule(dynamic, 256) num_threads(g_threads)
    for (int64_t i = 0; i < n; ++i)
        if (visible[i]) orc_preprocess_backward_one(params, S, i, deg, cam, W, H, drec + 9 * i, dparams);
}

/* Whole-view adjoint: dparams += d/dparams of sum(dLdC * image), for the
 * slots visible in this view that are not frozen (slot < n_opt). */
void orc_view_backward(const double *params, int64_t S, int deg,
                       const int32_t *start, const int32_t *expire, int frame,
                       const double cam[16], int W, int H, const double bg[3],
                       int64_t n_opt, const double *dLdC, double *dparams, double *drec_out)
{
    int32_t *vis = (int32_t *)malloc(sizeof(int32_t) * (size_t)S);
    double *rec = (double *)malloc(sizeof(double) * (size_t)S * REC);
    int32_t *rect = (int32_t *)malloc(sizeof(int32_t) * (size_t)S * 4);
    double *drec = drec_out ? drec_out : (double *)malloc(sizeof(double) * (size_t)S * 9);
    if (!drec_out) memset(drec, 0, sizeof(double) * (size_t)S * 9);
    orc_preprocess(params, S, deg, start, expire, frame, cam, W, H, 16, 16, vis, rec, rect);
    orc_blend_backward(S, vis, rec, W, H, bg, dLdC, drec);
    orc_preprocess_backward_many(params, S, deg, cam, W, H, vis, n_opt < S ? n_opt : S, drec, dparams);
    free(vis); free(rec); free(rect);
    if (!drec_out) free(drec);
}

/* ------------------------------------------------------------------------
 * Relocation of dead Gaussians (Sec. 3.2 and Algorithm 1: low-opacity
 * Gaussians are moved onto alive ones sampled in proportion to opacity;
 * the moved and the sampled Gaussians are then rescaled so that the sum of
 * their contributions stays approximately that of the source).
 *
 * in_A[i] != 0 marks the optimisable active slots (i < n_opt).  Dead:
 * logit < fl32(ln(0.005/0.995)).  Alive weights: floor(sigmoid(logit) 2^24)
 * in FP64.  Draw j: r = Philox(key=seed, ctr=(j, step lo, step hi, 0x52454C4F))
 * as r = out0 | out1 << 32; u = floor(r W / 2^64); source = first alive slot
 * whose inclusive prefix weight exceeds u.  The j-th dead slot (ascending)
 * receives source j.  N_s = 1 + copies of s, capped at n_max.  New opacity
 * 1-(1-o)^(1/N); new scale = scale * o / S_N(o'), with S_N the double
 * binomial sum of the 3DGS-MCMC relocation rule.  Mean, rotation and SH are
 * copied; Adam moments of sources and copies are zeroed.
 * Returns the number of dead slots; dst/src hold the pairs in order.
 * ---------------------------------------------------------------------- */
static double binom(int n, int k)
{
    double r = 1.0;
    for (int j = 1; j <= k; ++j) r = r * (double)(n - k + j) / (double)j;
    return r;
}

double orc_reloc_SN(int N, double a)
{
    double s = 0.0;
    for (int i = 1; i <= N; ++i)
        for (int k = 0; k <= i - 1; ++k)
            s += binom(i - 1, k) * ((k & 1) ? -1.0 : 1.0) * pow(a, (double)(k + 1)) / sqrt((double)(k + 1));
    return s;
}

int64_t orc_relocate(int64_t S, int64_t n_opt, int F, double *params, double *adam_m, double *adam_v,
                     const uint8_t *in_A, uint64_t seed, uint64_t step, int n_max,
                     int32_t *dst, int32_t *src, double *wmargin)
{
    const double Lstar = (double)(float)log(0.005 / 0.995);
    uint64_t *pref = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(n_opt > 0 ? n_opt : 1));
    int64_t *alive = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_opt > 0 ? n_opt : 1));
    int64_t na = 0, nd = 0;
    uint64_t W = 0;
    double wm = INFINITY;
    for (int64_t i = 0; i < n_opt; ++i) {
        if (!in_A[i]) continue;
        double lg = params[10 * S + i];
        if (lg < Lstar) { dst[nd++] = (int32_t)i; continue; }
        double sw = sigmoid(lg) * 16777216.0;
        double fl = floor(sw);
        double fr = sw - fl;
        wm = fmin(wm, fmin(fr, 1.0 - fr) / (sw > 1.0 ? sw : 1.0));
        W += (uint64_t)fl;
        alive[na] = i;
        pref[na] = W;
        ++na;
    }
    if (wmargin) *wmargin = wm;
    if (nd == 0 || na == 0 || W == 0) { free(pref); free(alive); return 0; }
    int32_t *cnt = (int32_t *)calloc((size_t)n_opt, sizeof(int32_t));
    uint32_t key[2] = {(uint32_t)seed, (uint32_t)(seed >> 32)};
    for (int64_t j = 0; j < nd; ++j) {
        uint32_t ctr[4] = {(uint32_t)j, (uint32_t)step, (uint32_t)(step >> 32), 0x52454C4Fu};
        uint32_t o4[4];
        orc_philox4x32_10(ctr, key, o4);
        uint64_t r = (uint64_t)o4[0] | ((uint64_t)o4[1] << 32);
        uint64_t u = (uint64_t)(((unsigned __int128)r * (unsigned __int128)W) >> 64);
        /* first alive index whose inclusive prefix exceeds u (linear scan) */
        int64_t a = 0;
        while (pref[a] <= u) ++a;
        src[j] = (int32_t)alive[a];
        cnt[alive[a]] += 1;
    }
    /* new opacity / scale of each source, computed from the source's
     * parameters before anything is written */
    double *newlogit = (double *)malloc(sizeof(double) * (size_t)n_opt);
    double *dscale = (double *)malloc(sizeof(double) * (size_t)n_opt);
    for (int64_t i = 0; i < n_opt; ++i) {
        if (!cnt[i]) continue;
        int N = 1 + cnt[i];
        if (N > n_max) N = n_max;
        /* 1 - o' = (1 - o)^(1/N), evaluated in log space:
         * ln(1 - o) = -softplus(logit), ln(o) = -softplus(-logit) */
        double lg = params[10 * S + i];
        double l1m = -softplus(lg) / (double)N;       /* ln(1 - o') */
        double on = -expm1(l1m);                      /* o'         */
        newlogit[i] = log(on) - l1m;
        dscale[i] = -softplus(-lg) - log(orc_reloc_SN(N, on));
    }
    for (int64_t j = 0; j < nd; ++j) {
        int64_t d = dst[j], s = src[j];
        for (int r = 0; r < F; ++r) params[r * S + d] = params[r * S + s];
        params[10 * S + d] = newlogit[s];
        for (int c = 0; c < 3; ++c) params[(3 + c) * S + d] = params[(3 + c) * S + s] + dscale[s];
        for (int r = 0; r < F; ++r) { adam_m[r * n_opt + d] = 0.0; adam_v[r * n_opt + d] = 0.0; }
    }
    for (int64_t s = 0; s < n_opt; ++s) {
        if (!cnt[s]) continue;
        params[10 * S + s] = newlogit[s];
        for (int c = 0; c < 3; ++c) params[(3 + c) * S + s] += dscale[s];
        for (int r = 0; r < F; ++r) { adam_m[r * n_opt + s] = 0.0; adam_v[r * n_opt + s] = 0.0; }
    }
    free(cnt); free(newlogit); free(dscale); free(pref); free(alive);
    return nd;
}
