/*
 * FP64 reference ("oracle") for one view of the Gaussian-splatting training
 * step.  TEST INFRASTRUCTURE ONLY: it is called by the test-suite, by the
 * package smoke check and by the CPU-baseline leg of the benchmark, never by
 * the product path.  It shares no code with the GPU implementation.
 *
 * What it computes, per the paper's preliminaries (Sec. 3.1):
 *   - Eq. 1: a 3D Gaussian exp(-1/2 (p-u)^T Sigma^-1 (p-u)) with
 *     Sigma = R S S^T R^T, R from the quaternion q, S = diag(exp(log-scale)).
 *   - the projection X^proj (not spelled out in the paper; read as the EWA
 *     local-affine projection: Sigma' = J W Sigma W^T J^T + dilation * I).
 *   - alpha = o * X^proj(p) with o = sigmoid(logit), clamped to alpha_max,
 *     kept when alpha >= alpha_min.
 *   - Eq. 2: C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j), front to back in
 *     (depth, index) order, stopping before the first Gaussian that would
 *     push the transmittance below T_min; background added with the final T.
 *   - colour c from the real spherical harmonics f, evaluated at the view
 *     direction, plus 0.5 and clamped at zero.
 *
 * Every pixel is evaluated against every Gaussian (no tiles, no bounding
 * boxes): the rasterizer's result is a per-pixel definition.  Reverse mode
 * keeps each pixel's list with its transmittances and walks it back to front,
 * then applies the chain rule through the projection to the raw parameters.
 *
 * Build: gcc -O2 -fno-fast-math -ffp-contract=off -fopenmp -shared -fPIC.
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>
#include <omp.h>

#define NPLANE(d) (11 + 3 * ((d) + 1) * ((d) + 1))

typedef struct {
    double R[9];   /* world -> camera rotation, row major */
    double t[3];
    double fx, fy, cx, cy;
    int W, H;
} orc_cam;

typedef struct {
    double near_z;     /* cull when camera depth <= near_z */
    double alpha_min;  /* keep when alpha >= alpha_min */
    double alpha_max;  /* alpha = min(alpha_max, o G) */
    double T_min;      /* stop before T would drop below T_min */
    double dilation;   /* added to the diagonal of the 2D covariance */
    double jac_clip;   /* clamp of x/z, y/z in units of the half field of view */
    double bg[3];
} orc_cfg;

/* per-pixel flags: a decision taken within rounding distance of a threshold */
enum {
    F_ALPHA_MIN = 1,   /* alpha close to alpha_min */
    F_T_MIN = 2,       /* T(1-alpha) close to T_min */
    F_DEPTH_TIE = 4,   /* two kept Gaussians with nearly equal depth */
    F_ALPHA_MAX = 8,   /* o G close to alpha_max (gradient kink) */
    F_NEAR = 16,       /* a Gaussian close to the near plane is visible here */
    F_COLOUR = 32,     /* kept Gaussian whose colour clamp is nearly active */
    F_CLIP = 64        /* kept Gaussian whose Jacobian clamp is nearly active */
};

/* ------------------------------------------------------------------ */
/* small linear algebra                                                 */

static void mat3_mul(const double *a, const double *b, double *c) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            c[3 * i + j] = s;
        }
}

static void mat3_transpose(const double *a, double *b) {
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) b[3 * j + i] = a[3 * i + j];
}

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_rot(const double *q, double *R) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* dR/dq_k for the same map, k = 0..3 (w, x, y, z) */
static void quat_rot_grad(const double *q, double dR[4][9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    double dw[9] = {0, -2 * z, 2 * y, 2 * z, 0, -2 * x, -2 * y, 2 * x, 0};
    double dx[9] = {0, 2 * y, 2 * z, 2 * y, -4 * x, -2 * w, 2 * z, 2 * w, -4 * x};
    double dy[9] = {-4 * y, 2 * x, 2 * w, 2 * x, 0, 2 * z, -2 * w, 2 * z, -4 * y};
    double dz[9] = {-4 * z, -2 * w, 2 * x, 2 * w, -4 * z, 2 * y, 2 * x, 2 * y, 0};
    memcpy(dR[0], dw, sizeof dw);
    memcpy(dR[1], dx, sizeof dx);
    memcpy(dR[2], dy, sizeof dy);
    memcpy(dR[3], dz, sizeof dz);
}

/* ------------------------------------------------------------------ */
/* real spherical harmonics, degree <= 3                                */
/*
 * Orthonormal real harmonics with the Condon-Shortley phase kept in the
 * associated Legendre function, m ordered -l..l, index k = l*l + l + m:
 *   Y_l0  = N_l^0 P_l(z)
 *   Y_lm  = sqrt2 N_l^m P_l^m(z) cos(m phi)     (m > 0)
 *   Y_l-m = sqrt2 N_l^m P_l^m(z) sin(m phi)     (m > 0)
 * with P_l^m(z) = (-1)^m (1-z^2)^{m/2} d^m P_l/dz^m and
 * N_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!).  On the unit sphere
 * (1-z^2)^{m/2} cos(m phi) = Re (x + i y)^m and the sine part is Im, so each
 * harmonic is a polynomial in (x, y, z): evaluated and differentiated as such.
 */
static double leg[4][4];          /* leg[l][p]: coefficient of z^p in P_l */
static int leg_ready = 0;

static void legendre_init(void) {
    if (leg_ready) return;
    memset(leg, 0, sizeof leg);
    leg[0][0] = 1;
    leg[1][1] = 1;
    for (int l = 1; l < 3; l++)               /* (l+1) P_{l+1} = (2l+1) z P_l - l P_{l-1} */
        for (int p = 0; p < 4; p++) {
            double v = -l * leg[l - 1][p];
            if (p > 0) v += (2 * l + 1) * leg[l][p - 1];
            leg[l + 1][p] = v / (l + 1);
        }
    leg_ready = 1;
}

/* m-th derivative of P_l at z */
static double legendre_deriv(int l, int m, double z) {
    double s = 0;
    for (int p = m; p <= l; p++) {
        double c = leg[l][p];
        for (int r = 0; r < m; r++) c *= (p - r);
        s += c * pow(z, p - m);
    }
    return s;
}

static double factorial(int n) { double f = 1; for (int i = 2; i <= n; i++) f *= i; return f; }

/* (x + i y)^m as (re, im) */
static void cpow_xy(double x, double y, int m, double *re, double *im) {
    double a = 1, b = 0;
    for (int i = 0; i < m; i++) { double t = a * x - b * y; b = a * y + b * x; a = t; }
    *re = a; *im = b;
}

/* Y[k] and, when dY != NULL, dY[k][0..2] = partial derivatives in x, y, z */
static void sh_eval(int deg, const double *d, double *Y, double (*dY)[3]) {
    legendre_init();
    double x = d[0], y = d[1], z = d[2];
    for (int l = 0; l <= deg; l++) {
        for (int m = -l; m <= l; m++) {
            int am = m < 0 ? -m : m;
            int k = l * l + l + m;
            double N = sqrt((2 * l + 1) / (4 * M_PI) * factorial(l - am) / factorial(l + am));
            double pre = (am == 0) ? N : sqrt(2.0) * N * ((am & 1) ? -1.0 : 1.0);
            double D = legendre_deriv(l, am, z);
            double D1 = (am + 1 <= l) ? legendre_deriv(l, am + 1, z) : 0.0;
            double re, im, re1 = 0, im1 = 0;
            cpow_xy(x, y, am, &re, &im);
            if (am > 0) cpow_xy(x, y, am - 1, &re1, &im1);
            double ang = (m >= 0) ? re : im;
            Y[k] = pre * D * ang;
            if (dY) {
                /* d/dx (x+iy)^m = m (x+iy)^{m-1};  d/dy = i m (x+iy)^{m-1} */
                double dax, day;
                if (m >= 0) { dax = am * re1; day = -am * im1; }
                else        { dax = am * im1; day = am * re1; }
                dY[k][0] = pre * D * dax;
                dY[k][1] = pre * D * day;
                dY[k][2] = pre * D1 * ang;
            }
        }
    }
}

/* ------------------------------------------------------------------ */
/* projection of one Gaussian into one view                             */

typedef struct {
    int valid;           /* passes the near-plane and opacity culls */
    double qn[4], qlen;  /* normalised quaternion and |q| */
    double s[3];         /* exp(log-scale) */
    double Rq[9];        /* rotation of the Gaussian */
    double Sig[9];       /* 3D covariance */
    double t[3];         /* camera-space mean */
    double rx, ry;       /* clamped x/z and y/z */
    int clx, cly;        /* clamp active */
    double J[6];         /* 2x3 Jacobian */
    double Tm[6];        /* J W (2x3) */
    double S2[3];        /* 2D covariance (xx, xy, yy) incl. dilation */
    double A[3];         /* conic (a, b, c) = inverse of S2 */
    double m[2];         /* pixel-space mean */
    double o;            /* opacity */
    double dir[3], vlen; /* view direction, |u - centre| */
    double Y[16];
    double raw[3];       /* SH sum before offset and clamp */
    double col[3];
    double near_gap, clip_gap, col_gap;
    double lmax;      /* largest eigenvalue of the conic */
    double dm;        /* bound on an FP32 evaluation's error in the pixel-space mean */
    double cabs[3];   /* sum of |terms| of the colour (SH terms and the 0.5 offset) */
} proj_t;

static void project_one(int deg, const double *P, long stride, long i, const orc_cam *cam,
                        const orc_cfg *cfg, proj_t *g) {
    double u[3], q[4], ls[3];
    for (int k = 0; k < 3; k++) u[k] = P[(0 + k) * stride + i];
    for (int k = 0; k < 4; k++) q[k] = P[(3 + k) * stride + i];
    for (int k = 0; k < 3; k++) ls[k] = P[(7 + k) * stride + i];
    double logit = P[10 * stride + i];

    g->qlen = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; k++) g->qn[k] = q[k] / g->qlen;
    for (int k = 0; k < 3; k++) g->s[k] = exp(ls[k]);
    quat_rot(g->qn, g->Rq);
    double M[9], MT[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[3 * r + c] = g->Rq[3 * r + c] * g->s[c];
    mat3_transpose(M, MT);
    mat3_mul(M, MT, g->Sig);

    const double *W = cam->R;
    for (int r = 0; r < 3; r++)
        g->t[r] = W[3 * r] * u[0] + W[3 * r + 1] * u[1] + W[3 * r + 2] * u[2] + cam->t[r];
    double tz = g->t[2];
    g->near_gap = fabs(tz / cfg->near_z - 1.0);
    g->o = 1.0 / (1.0 + exp(-logit));
    g->valid = (tz > cfg->near_z) && (g->o >= cfg->alpha_min);
    if (tz <= 0) { g->valid = 0; return; }

    g->m[0] = cam->fx * g->t[0] / tz + cam->cx;
    g->m[1] = cam->fy * g->t[1] / tz + cam->cy;
    double limx = cfg->jac_clip * 0.5 * cam->W / cam->fx;
    double limy = cfg->jac_clip * 0.5 * cam->H / cam->fy;
    double ux = g->t[0] / tz, uy = g->t[1] / tz;
    g->clx = (ux < -limx || ux > limx);
    g->cly = (uy < -limy || uy > limy);
    g->rx = ux < -limx ? -limx : (ux > limx ? limx : ux);
    g->ry = uy < -limy ? -limy : (uy > limy ? limy : uy);
    g->clip_gap = fmin(fabs(fabs(ux) / limx - 1.0), fabs(fabs(uy) / limy - 1.0));
    g->J[0] = cam->fx / tz; g->J[1] = 0; g->J[2] = -cam->fx * g->rx / tz;
    g->J[3] = 0; g->J[4] = cam->fy / tz; g->J[5] = -cam->fy * g->ry / tz;
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += g->J[3 * r + k] * W[3 * k + c];
            g->Tm[3 * r + c] = s;
        }
    /* S2 = Tm Sig Tm^T + dilation I */
    double TS[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += g->Tm[3 * r + k] * g->Sig[3 * k + c];
            TS[3 * r + c] = s;
        }
    double S2f[4];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += TS[3 * r + k] * g->Tm[3 * c + k];
            S2f[2 * r + c] = s;
        }
    g->S2[0] = S2f[0] + cfg->dilation;
    g->S2[1] = 0.5 * (S2f[1] + S2f[2]);
    g->S2[2] = S2f[3] + cfg->dilation;
    double det = g->S2[0] * g->S2[2] - g->S2[1] * g->S2[1];
    g->A[0] = g->S2[2] / det;
    g->A[1] = -g->S2[1] / det;
    g->A[2] = g->S2[0] / det;

    /* Inputs of the rounding bounds (alpha_rel_err below): an FP32
     * evaluation places the mean to within a few roundings of its pixel
     * coordinates, taken as 2 * 2^-24 (|m_x| + |m_y|). */
    g->lmax = 0.5 * (g->A[0] + g->A[2]) +
              sqrt(0.25 * (g->A[0] - g->A[2]) * (g->A[0] - g->A[2]) + g->A[1] * g->A[1]);
    g->dm = 2.0 * 0x1p-24 * (fabs(g->m[0]) + fabs(g->m[1]));

    double cc[3];
    mat3_transpose(W, MT);
    for (int r = 0; r < 3; r++)
        cc[r] = -(MT[3 * r] * cam->t[0] + MT[3 * r + 1] * cam->t[1] + MT[3 * r + 2] * cam->t[2]);
    double v[3] = {u[0] - cc[0], u[1] - cc[1], u[2] - cc[2]};
    g->vlen = sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]);
    for (int k = 0; k < 3; k++) g->dir[k] = v[k] / g->vlen;
    sh_eval(deg, g->dir, g->Y, NULL);
    int nk = (deg + 1) * (deg + 1);
    g->col_gap = 1e300;
    for (int ch = 0; ch < 3; ch++) {
        double s = 0, sa = 0.5;
        for (int k = 0; k < nk; k++) {
            s += g->Y[k] * P[(11 + 3 * k + ch) * stride + i];
            sa += fabs(g->Y[k] * P[(11 + 3 * k + ch) * stride + i]);
        }
        g->raw[ch] = s;
        g->cabs[ch] = sa;
        g->col[ch] = s + 0.5 > 0 ? s + 0.5 : 0.0;
        g->col_gap = fmin(g->col_gap, fabs(s + 0.5));
    }
}

/* ------------------------------------------------------------------ */
/* per-pixel compositing                                                */

typedef struct { double depth; long idx; double alpha; double araw; double G; double dx, dy, rerr; } hit_t;

static int hit_cmp(const void *a, const void *b) {
    const hit_t *x = a, *y = b;
    if (x->depth < y->depth) return -1;
    if (x->depth > y->depth) return 1;
    return (x->idx < y->idx) ? -1 : (x->idx > y->idx);
}

#define U32 0x1p-24   /* FP32 unit roundoff */

/* First-order bound on the relative error of alpha = o exp(-e/2) at a pixel
 * whose exponent is e, when it is evaluated in FP32.  The mean's pixel
 * position is off by up to dm; a shift d of the offset changes
 * e = delta^T A delta by up to 2 sqrt(lambda_max e) |d|, hence alpha by
 * sqrt(lambda_max e) |d| relative.  The conic, the exponent, exp and the
 * opacity add a few roundings each, relative to e and to 1. */
static double alpha_rel_err(const proj_t *G, double e) {
    return sqrt(G->lmax * e) * G->dm + U32 * (8.0 + 8.0 * e);
}

/* Gather, sort and composite one pixel; returns number of contributors.
 * T_before[j] holds the transmittance in front of list entry j.
 * err (optional, 4 doubles) receives first-order bounds on what an FP32
 * evaluation of the same pixel may differ by: err[0] relative to the final
 * T, err[1..3] absolute on the colour.  Each kept alpha carries
 * alpha_rel_err (zero when alpha_max clamps it); 1 - alpha_j then carries
 * alpha_j / (1 - alpha_j) times that, and each product and sum one more
 * rounding.  The same bounds widen the windows of the threshold decisions,
 * so that a decision an FP32 evaluation may take the other way is flagged. */
static int pixel_composite(const proj_t *g, long n, double px, double py, const orc_cfg *cfg,
                           hit_t *hits, double *T_before, double *rgb, double *T_out, int *flags,
                           double *err) {
    long nh = 0;
    int fl = 0;
    for (long i = 0; i < n; i++) {
        const proj_t *G = &g[i];
        if (G->t[2] <= 0) continue;
        if (!G->valid) {
            /* a Gaussian culled by the near plane but almost on it */
            if (G->near_gap < 1e-6 && G->o >= cfg->alpha_min) {
                double dx = px - G->m[0], dy = py - G->m[1];
                double e = G->A[0] * dx * dx + 2 * G->A[1] * dx * dy + G->A[2] * dy * dy;
                if (G->o * exp(-0.5 * e) >= cfg->alpha_min * (1 - 1e-4)) fl |= F_NEAR;
            }
            continue;
        }
        double dx = px - G->m[0], dy = py - G->m[1];
        double e = G->A[0] * dx * dx + 2 * G->A[1] * dx * dy + G->A[2] * dy * dy;
        double Gv = exp(-0.5 * e);
        double araw = G->o * Gv;
        double a = araw < cfg->alpha_max ? araw : cfg->alpha_max;
        if (fabs(a / cfg->alpha_min - 1.0) < fmax(1e-4, alpha_rel_err(G, e))) fl |= F_ALPHA_MIN;
        if (a < cfg->alpha_min) continue;
        if (G->near_gap < 1e-6) fl |= F_NEAR;
        hits[nh].depth = G->t[2];
        hits[nh].idx = i;
        hits[nh].alpha = a;
        hits[nh].araw = araw;
        hits[nh].G = Gv;
        hits[nh].dx = dx;
        hits[nh].dy = dy;
        hits[nh].rerr = alpha_rel_err(G, e);
        nh++;
    }
    qsort(hits, nh, sizeof(hit_t), hit_cmp);
    double T = 1.0;
    double C[3] = {0, 0, 0};
    double Trel = 0, Cerr[3] = {0, 0, 0};
    int nc = 0;
    for (long j = 0; j < nh; j++) {
        double a = hits[j].alpha;
        double Tn = T * (1 - a);
        const double ra = hits[j].araw < cfg->alpha_max ? hits[j].rerr : 0.0;
        const double Tnrel = Trel + a / (1 - a) * ra + 2 * U32;
        if (fabs(Tn / cfg->T_min - 1.0) < fmax(1e-4, Tnrel)) fl |= F_T_MIN;
        if (Tn < cfg->T_min) break;
        const proj_t *G = &g[hits[j].idx];
        if (fabs(hits[j].araw / cfg->alpha_max - 1.0) < fmax(1e-4, hits[j].rerr)) fl |= F_ALPHA_MAX;
        if (G->col_gap < 1e-6) fl |= F_COLOUR;
        if (G->clip_gap < 1e-6) fl |= F_CLIP;
        if (j > 0 && fabs(hits[j].depth - hits[j - 1].depth) < 1e-6 * hits[j].depth) fl |= F_DEPTH_TIE;
        T_before[j] = T;
        for (int ch = 0; ch < 3; ch++) {
            const double w = a * T;
            C[ch] += G->col[ch] * w;
            Cerr[ch] += w * (G->col[ch] * (ra + Trel + 3 * U32) + 8 * U32 * G->cabs[ch]) + U32 * C[ch];
        }
        T = Tn;
        Trel = Tnrel;
        nc++;
    }
    /* a tie between the last contributor and the next kept Gaussian matters too */
    if (nc < nh && nc > 0 && fabs(hits[nc].depth - hits[nc - 1].depth) < 1e-6 * hits[nc].depth) fl |= F_DEPTH_TIE;
    for (int ch = 0; ch < 3; ch++) rgb[ch] = C[ch] + T * cfg->bg[ch];
    if (err) {
        err[0] = Trel;
        for (int ch = 0; ch < 3; ch++) err[1 + ch] = Cerr[ch] + T * fabs(cfg->bg[ch]) * (Trel + 2 * U32) + U32 * fabs(rgb[ch]);
    }
    *T_out = T;
    *flags = fl;
    return nc;
}

static proj_t *project_all(int n, int deg, const double *P, long stride, const orc_cam *cam, const orc_cfg *cfg) {
    proj_t *g = (proj_t *)calloc((size_t)(n > 0 ? n : 1), sizeof(proj_t));
    legendre_init();
#pragma omp parallel for schedule(static)
    for (long i = 0; i < n; i++) project_one(deg, P, stride, i, cam, cfg, &g[i]);
    return g;
}

/* ------------------------------------------------------------------ */
/* exported entry points                                                */

#define ORC_PW 20
/* per-Gaussian projection output:
 * 0 valid, 1 mx, 2 my, 3 a, 4 b, 5 c, 6 depth, 7 opacity, 8..10 colour,
 * 11..13 S2 (xx, xy, yy), 14..16 camera-space mean, 17 clip gap,
 * 18 colour gap, 19 near gap */
int orc_project(int n, int deg, const double *P, long stride, const orc_cam *cam, const orc_cfg *cfg, double *out) {
    if (n < 0 || deg < 0 || deg > 3) return 1;
    proj_t *g = project_all(n, deg, P, stride, cam, cfg);
    for (long i = 0; i < n; i++) {
        double *o = out + ORC_PW * i;
        o[0] = g[i].valid;
        o[1] = g[i].m[0]; o[2] = g[i].m[1];
        o[3] = g[i].A[0]; o[4] = g[i].A[1]; o[5] = g[i].A[2];
        o[6] = g[i].t[2]; o[7] = g[i].o;
        for (int k = 0; k < 3; k++) o[8 + k] = g[i].col[k];
        for (int k = 0; k < 3; k++) o[11 + k] = g[i].S2[k];
        for (int k = 0; k < 3; k++) o[14 + k] = g[i].t[k];
        o[17] = g[i].clip_gap; o[18] = g[i].col_gap; o[19] = g[i].near_gap;
    }
    free(g);
    return 0;
}

/* Render the listed pixels (linear index y*W + x; NULL = every pixel). */
int orc_render(int n, int deg, const double *P, long stride, const orc_cam *cam, const orc_cfg *cfg,
               const long *pix, long npix, double *rgb, double *T, int *ncontrib, int *flags, double *err) {
    if (n < 0 || deg < 0 || deg > 3) return 1;
    long total = pix ? npix : (long)cam->W * cam->H;
    proj_t *g = project_all(n, deg, P, stride, cam, cfg);
#pragma omp parallel
    {
        hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * (size_t)(n > 0 ? n : 1));
        double *Tb = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(dynamic, 16)
        for (long k = 0; k < total; k++) {
            long p = pix ? pix[k] : k;
            double px = (p % cam->W) + 0.5, py = (p / cam->W) + 0.5;
            int fl;
            ncontrib[k] = pixel_composite(g, n, px, py, cfg, hits, Tb, rgb + 3 * k, T + k, &fl, err ? err + 4 * k : NULL);
            flags[k] = fl;
        }
        free(hits);
        free(Tb);
    }
    free(g);
    return 0;
}

/* per-Gaussian screen-space gradient accumulator */
typedef struct { double mx, my, a, b, c, o, col[3]; } sgrad_t;

/* Chain rule from the screen-space quantities of one Gaussian to its raw
 * parameters; adds into grad planes (stride = n). */
static void chain_to_params(int deg, const double *P, long stride, long i, const orc_cam *cam,
                            const proj_t *g, const sgrad_t *sg, double *grad, long gstride) {
    const double *W = cam->R;
    double gu[3] = {0, 0, 0};
    int nk = (deg + 1) * (deg + 1);

    /* opacity: o = sigmoid(logit) */
    grad[10 * gstride + i] += sg->o * g->o * (1 - g->o);

    /* colour: c = max(0, sum_k Y_k f_k + 0.5) */
    double Y[16], dY[16][3];
    sh_eval(deg, g->dir, Y, dY);
    double gdir[3] = {0, 0, 0};
    for (int ch = 0; ch < 3; ch++) {
        if (!(g->raw[ch] + 0.5 > 0)) continue;
        double gr = sg->col[ch];
        for (int k = 0; k < nk; k++) {
            grad[(11 + 3 * k + ch) * gstride + i] += Y[k] * gr;
            double f = P[(11 + 3 * k + ch) * stride + i];
            for (int a = 0; a < 3; a++) gdir[a] += f * gr * dY[k][a];
        }
    }
    /* dir = v / |v| with v = u - camera centre */
    double dd = gdir[0] * g->dir[0] + gdir[1] * g->dir[1] + gdir[2] * g->dir[2];
    for (int a = 0; a < 3; a++) gu[a] += (gdir[a] - g->dir[a] * dd) / g->vlen;

    /* conic -> 2D covariance: A = S2^{-1}, dL/dS2 = -A G_A A */
    double A[4] = {g->A[0], g->A[1], g->A[1], g->A[2]};
    double GA[4] = {sg->a, 0.5 * sg->b, 0.5 * sg->b, sg->c};
    double AG[4], GS[4];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) AG[2 * r + c] = A[2 * r] * GA[c] + A[2 * r + 1] * GA[2 + c];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) GS[2 * r + c] = -(AG[2 * r] * A[c] + AG[2 * r + 1] * A[2 + c]);

    /* S2 = Tm Sig Tm^T + dI:  dL/dSig = Tm^T GS Tm,  dL/dTm = 2 GS Tm Sig */
    double GSig[9], GT[6], GSTm[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) GSTm[3 * r + c] = GS[2 * r] * g->Tm[c] + GS[2 * r + 1] * g->Tm[3 + c];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) GSig[3 * r + c] = g->Tm[r] * GSTm[c] + g->Tm[3 + r] * GSTm[3 + c];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += GSTm[3 * r + k] * g->Sig[3 * k + c];
            GT[3 * r + c] = 2 * s;
        }
    /* Tm = J W: dL/dJ = GT W^T */
    double GJ[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += GT[3 * r + k] * W[3 * c + k];
            GJ[3 * r + c] = s;
        }
    /* J and mean2D as functions of the camera-space mean t */
    double tx = g->t[0], ty = g->t[1], tz = g->t[2];
    double fx = cam->fx, fy = cam->fy;
    double gt[3] = {0, 0, 0};
    double drx_dtx = g->clx ? 0 : 1 / tz, drx_dtz = g->clx ? 0 : -tx / (tz * tz);
    double dry_dty = g->cly ? 0 : 1 / tz, dry_dtz = g->cly ? 0 : -ty / (tz * tz);
    gt[2] += GJ[0] * (-fx / (tz * tz));
    gt[2] += GJ[2] * (fx * g->rx / (tz * tz) - fx / tz * drx_dtz);
    gt[0] += GJ[2] * (-fx / tz * drx_dtx);
    gt[2] += GJ[4] * (-fy / (tz * tz));
    gt[2] += GJ[5] * (fy * g->ry / (tz * tz) - fy / tz * dry_dtz);
    gt[1] += GJ[5] * (-fy / tz * dry_dty);
    gt[0] += sg->mx * fx / tz;
    gt[2] -= sg->mx * fx * tx / (tz * tz);
    gt[1] += sg->my * fy / tz;
    gt[2] -= sg->my * fy * ty / (tz * tz);
    /* t = W u + t_cw */
    for (int a = 0; a < 3; a++) gu[a] += W[a] * gt[0] + W[3 + a] * gt[1] + W[6 + a] * gt[2];
    for (int a = 0; a < 3; a++) grad[a * gstride + i] += gu[a];

    /* Sig = M M^T with M = Rq diag(s):  dL/dM = 2 GSig M */
    double M[9], GM[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M[3 * r + c] = g->Rq[3 * r + c] * g->s[c];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += GSig[3 * r + k] * M[3 * k + c];
            GM[3 * r + c] = 2 * s;
        }
    double GR[9];
    for (int c = 0; c < 3; c++) {
        double gs = 0;
        for (int r = 0; r < 3; r++) {
            gs += GM[3 * r + c] * g->Rq[3 * r + c];
            GR[3 * r + c] = GM[3 * r + c] * g->s[c];
        }
        grad[(7 + c) * gstride + i] += gs * g->s[c];   /* s = exp(log-scale) */
    }
    /* R(qn), qn = q / |q| */
    double dR[4][9], gqn[4];
    quat_rot_grad(g->qn, dR);
    for (int k = 0; k < 4; k++) {
        double s = 0;
        for (int e = 0; e < 9; e++) s += GR[e] * dR[k][e];
        gqn[k] = s;
    }
    double qd = 0;
    for (int k = 0; k < 4; k++) qd += gqn[k] * g->qn[k];
    for (int k = 0; k < 4; k++) grad[(3 + k) * gstride + i] += (gqn[k] - g->qn[k] * qd) / g->qlen;
}

/* Reverse mode of orc_render for a given dL/dC at the listed pixels.
 * grad: NPLANE(deg) planes of n doubles, accumulated into (+=).
 * sgrad_out (optional, n x 9): screen-space gradients
 * (mx, my, a, b, c, opacity, r, g, b) of this view. */
int orc_backward(int n, int deg, const double *P, long stride, const orc_cam *cam, const orc_cfg *cfg,
                 const long *pix, long npix, const double *dLdC, double *grad, double *sgrad_out) {
    if (n < 0 || deg < 0 || deg > 3) return 1;
    long total = pix ? npix : (long)cam->W * cam->H;
    proj_t *g = project_all(n, deg, P, stride, cam, cfg);
    int nth = omp_get_max_threads();
    sgrad_t *acc = (sgrad_t *)calloc((size_t)nth * (size_t)(n > 0 ? n : 1), sizeof(sgrad_t));
#pragma omp parallel
    {
        int tid = omp_get_thread_num();
        sgrad_t *my = acc + (size_t)tid * (size_t)(n > 0 ? n : 1);
        hit_t *hits = (hit_t *)malloc(sizeof(hit_t) * (size_t)(n > 0 ? n : 1));
        double *Tb = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
#pragma omp for schedule(static)
        for (long k = 0; k < total; k++) {
            const double *gc = dLdC + 3 * k;
            if (gc[0] == 0 && gc[1] == 0 && gc[2] == 0) continue;
            long p = pix ? pix[k] : k;
            double px = (p % cam->W) + 0.5, py = (p / cam->W) + 0.5;
            double rgb[3], Tf;
            int fl;
            int nc = pixel_composite(g, n, px, py, cfg, hits, Tb, rgb, &Tf, &fl, NULL);
            /* colour behind entry j, starting with the background */
            double S[3] = {Tf * cfg->bg[0], Tf * cfg->bg[1], Tf * cfg->bg[2]};
            for (int j = nc - 1; j >= 0; j--) {
                const hit_t *h = &hits[j];
                const proj_t *G = &g[h->idx];
                sgrad_t *sg = &my[h->idx];
                double a = h->alpha, Tj = Tb[j];
                double galpha = 0;
                for (int ch = 0; ch < 3; ch++) {
                    sg->col[ch] += gc[ch] * a * Tj;
                    galpha += gc[ch] * (G->col[ch] * Tj - S[ch] / (1 - a));
                    S[ch] += G->col[ch] * a * Tj;
                }
                if (h->araw < cfg->alpha_max) {
                    sg->o += galpha * h->G;
                    double ge = galpha * G->o * h->G * (-0.5);   /* dL/d(exponent quadratic) */
                    double dx = h->dx, dy = h->dy;
                    sg->a += ge * dx * dx;
                    sg->b += ge * 2 * dx * dy;
                    sg->c += ge * dy * dy;
                    sg->mx += ge * (-2) * (G->A[0] * dx + G->A[1] * dy);
                    sg->my += ge * (-2) * (G->A[1] * dx + G->A[2] * dy);
                }
            }
        }
        free(hits);
        free(Tb);
    }
    /* reduce thread accumulators in thread order, then chain rule */
    for (long i = 0; i < n; i++) {
        sgrad_t s;
        memset(&s, 0, sizeof s);
        for (int t = 0; t < nth; t++) {
            sgrad_t *a = &acc[(size_t)t * (size_t)n + i];
            s.mx += a->mx; s.my += a->my; s.a += a->a; s.b += a->b; s.c += a->c; s.o += a->o;
            for (int ch = 0; ch < 3; ch++) s.col[ch] += a->col[ch];
        }
        if (sgrad_out) {
            double *o = sgrad_out + 9 * i;
            o[0] = s.mx; o[1] = s.my; o[2] = s.a; o[3] = s.b; o[4] = s.c; o[5] = s.o;
            o[6] = s.col[0]; o[7] = s.col[1]; o[8] = s.col[2];
        }
        if (!g[i].valid) continue;
        chain_to_params(deg, P, stride, i, cam, &g[i], &s, grad, n);
    }
    free(acc);
    free(g);
    return 0;
}

/* Real SH basis at unit directions (for checks against a library routine). */
int orc_sh_basis(int deg, long n, const double *dirs, double *Y, double *dY) {
    for (long i = 0; i < n; i++) {
        double y[16], dy[16][3];
        sh_eval(deg, dirs + 3 * i, y, dy);
        int nk = (deg + 1) * (deg + 1);
        for (int k = 0; k < nk; k++) {
            Y[i * nk + k] = y[k];
            if (dY)
                for (int a = 0; a < 3; a++) dY[(i * nk + k) * 3 + a] = dy[k][a];
        }
    }
    return 0;
}

int orc_quat_rot(long n, const double *q, double *R) {
    for (long i = 0; i < n; i++) {
        double qn[4], l = 0;
        for (int k = 0; k < 4; k++) l += q[4 * i + k] * q[4 * i + k];
        l = sqrt(l);
        for (int k = 0; k < 4; k++) qn[k] = q[4 * i + k] / l;
        quat_rot(qn, R + 9 * i);
    }
    return 0;
}

int orc_num_threads(void) { return omp_get_max_threads(); }

/* threads of the following calls (timing of the oracle itself) */
void orc_set_threads(int n) { omp_set_num_threads(n > 0 ? n : 1); }
