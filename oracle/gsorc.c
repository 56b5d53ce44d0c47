/*
 * gsorc.c - FP64 CPU oracle for the differentiable Gaussian-splatting fit step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The product path
 * never calls it and shares no code with it.
 *
 * The paper (Method section, "Periphery Model Training") fits its peripheral
 * Gaussian model with a 3D Gaussian Splatting optimiser (Mini-Splatting2 with
 * Taming-3DGS techniques) and does not restate the rasterizer.  This oracle is
 * therefore the plain mathematical definition of that rasterizer:
 *
 *   - each 3D Gaussian is projected through the local affine approximation of
 *     the pinhole map (EWA splatting) to a 2D Gaussian with a 0.3 px^2 low-pass;
 *   - every pixel composites front to back over ALL Gaussians sorted by
 *     (fp32 camera depth, index), with no tiles: alpha = min(0.99, o e^power),
 *     skipped below 1/255, stopped before transmittance would drop below 1e-4;
 *   - the gradient is the exact derivative of that forward map (adjoint written
 *     out by the chain rule), with zero derivative through discrete decisions
 *     and active clamps;
 *   - the discrete stage (tile ids, sort order, ranges) is a nested loop plus
 *     qsort over (tile, fp32 depth bits, record) tuples; a record lists the
 *     tiles of each row of its box that its padded support ellipse reaches;
 *   - Adam is the bias-corrected form (the paper's continual refinement restarts
 *     it by discarding its state, Method section, last paragraph of
 *     "Periphery Model Training").
 *
 * Everything is float64.  Near-threshold decisions (alpha ~ 1/255, T ~ 1e-4,
 * depth ties within 4 fp32 ulps, box edges near an integer, clamps) are
 * reported through flag bits so tests can exclude them; a float32
 * implementation may legitimately decide those the other way.
 *
 * Camera record (27 doubles): R[9] row-major world->camera, t[3], campos[3],
 * fx, fy, cx, cy, tan_half_fov_x, tan_half_fov_y, znear, bg[3], width, height.
 * Parameters: planar [C][n], C = 11 + 3K, K = (deg+1)^2:
 *   mean(3) log-scale(3) quat wxyz(4) opacity-logit(1) sh[k][channel](3K).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_NREC 22
/* record fields */
enum { R_VALID, R_TZ, R_TX, R_TY, R_MX, R_MY, R_CA, R_CB, R_CC, R_O, R_CR, R_CG, R_CBL,
       R_SA, R_SB, R_SC, R_EX0, R_EX1, R_EY0, R_EY1, R_D32, R_COLRAW };

/* flag bits */
#define F_NEAR_ALPHA 1    /* o e^power within 1e-4 relative of 1/255 */
#define F_NEAR_STOP 2     /* T (1 - alpha) within 1e-4 relative of 1e-4 */
#define F_NEAR_TIE 4      /* two contributing Gaussians within 4 fp32 ulps of depth */
#define F_NEAR_CLAMP 8    /* o e^power within 1e-4 relative of the 0.99 clamp */
#define F_NEAR_CULL 16    /* record near a cull threshold */
#define F_NEAR_BOX 32     /* box edge near a rounding boundary that changes its tile */
#define F_NEAR_GRAD 64    /* colour or Jacobian clamp near its switch point */

#define C_R 0
#define C_T 9
#define C_CAMPOS 12
#define C_FX 15
#define C_FY 16
#define C_CX 17
#define C_CY 18
#define C_TANX 19
#define C_TANY 20
#define C_ZNEAR 21
#define C_BG 22
#define C_W 25
#define C_H 26

static const double ALPHA_MIN = 1.0 / 255.0;
static const double ALPHA_MAX = 0.99;
static const double T_STOP = 1e-4;
static const double LOWPASS = 0.3;
static const double JCLAMP = 1.3;
static const double BOX_REL = 1e-4;
static const double BOX_ABS = 1.0 / 64.0;

static int n_coeffs(int deg) { return (deg + 1) * (deg + 1); }


/* ---------------------------------------------------------------- SH basis */
/* Real spherical harmonics, orthonormal on the unit sphere, Condon-Shortley
 * phase, index k = l*l + l + m.  Constants are the closed-form normalisers. */
static void sh_basis(int deg, const double d[3], double Y[16], double dY[16][3]) {
    const double x = d[0], y = d[1], z = d[2];
    const double pi = acos(-1.0);
    const double c0 = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi);
    const double c20 = 0.25 * sqrt(5.0 / pi);
    const double c22 = 0.25 * sqrt(15.0 / pi);
    const double c33 = 0.25 * sqrt(35.0 / (2.0 * pi));
    const double c32 = 0.5 * sqrt(105.0 / pi);
    const double c31 = 0.25 * sqrt(21.0 / (2.0 * pi));
    const double c30 = 0.25 * sqrt(7.0 / pi);
    const double c32b = 0.25 * sqrt(105.0 / pi);
    memset(Y, 0, 16 * sizeof(double));
    if (dY) memset(dY, 0, 16 * 3 * sizeof(double));
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = -c1 * y; Y[2] = c1 * z; Y[3] = -c1 * x;
    if (dY) { dY[1][1] = -c1; dY[2][2] = c1; dY[3][0] = -c1; }
    if (deg < 2) return;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c20 * (2 * z * z - x * x - y * y);
    Y[7] = -c2a * x * z;
    Y[8] = c22 * (x * x - y * y);
    if (dY) {
        dY[4][0] = c2a * y; dY[4][1] = c2a * x;
        dY[5][1] = -c2a * z; dY[5][2] = -c2a * y;
        dY[6][0] = -2 * c20 * x; dY[6][1] = -2 * c20 * y; dY[6][2] = 4 * c20 * z;
        dY[7][0] = -c2a * z; dY[7][2] = -c2a * x;
        dY[8][0] = 2 * c22 * x; dY[8][1] = -2 * c22 * y;
    }
    if (deg < 3) return;
    Y[9] = -c33 * y * (3 * x * x - y * y);
    Y[10] = c32 * x * y * z;
    Y[11] = -c31 * y * (4 * z * z - x * x - y * y);
    Y[12] = c30 * z * (2 * z * z - 3 * x * x - 3 * y * y);
    Y[13] = -c31 * x * (4 * z * z - x * x - y * y);
    Y[14] = c32b * z * (x * x - y * y);
    Y[15] = -c33 * x * (x * x - 3 * y * y);
    if (dY) {
        dY[9][0] = -6 * c33 * x * y; dY[9][1] = -c33 * (3 * x * x - 3 * y * y);
        dY[10][0] = c32 * y * z; dY[10][1] = c32 * x * z; dY[10][2] = c32 * x * y;
        dY[11][0] = 2 * c31 * x * y; dY[11][1] = -c31 * (4 * z * z - x * x - 3 * y * y);
        dY[11][2] = -8 * c31 * y * z;
        dY[12][0] = -6 * c30 * x * z; dY[12][1] = -6 * c30 * y * z;
        dY[12][2] = c30 * (6 * z * z - 3 * x * x - 3 * y * y);
        dY[13][0] = -c31 * (4 * z * z - 3 * x * x - y * y); dY[13][1] = 2 * c31 * x * y;
        dY[13][2] = -8 * c31 * x * z;
        dY[14][0] = 2 * c32b * x * z; dY[14][1] = -2 * c32b * y * z;
        dY[14][2] = c32b * (x * x - y * y);
        dY[15][0] = -c33 * (3 * x * x - 3 * y * y); dY[15][1] = 6 * c33 * x * y;
    }
}

int orc_sh_basis(int deg, const double *dirs, int64_t n, double *out /* [n][16] */) {
    for (int64_t i = 0; i < n; i++) sh_basis(deg, dirs + 3 * i, out + 16 * i, NULL);
    return 0;
}

/* ------------------------------------------------------------ small linear algebra */
static void mat3_mul(const double *a, const double *b, double *c) { /* c = a b */
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) {
            double s = 0;
            for (int k = 0; k < 3; k++) s += a[3 * i + k] * b[3 * k + j];
            t[3 * i + j] = s;
        }
    memcpy(c, t, sizeof t);
}
static void mat3_transpose(const double *a, double *b) {
    double t[9];
    for (int i = 0; i < 3; i++)
        for (int j = 0; j < 3; j++) t[3 * j + i] = a[3 * i + j];
    memcpy(b, t, sizeof t);
}

/* rotation matrix of a unit quaternion (w, x, y, z) */
static void quat_rot(const double q[4], double R[9]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z); R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z); R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y); R[7] = 2 * (y * z + w * x); R[8] = 1 - 2 * (x * x + y * y);
}

/* d(loss)/d(q) from d(loss)/d(R), for R = quat_rot(q) with q treated as free */
static void quat_rot_vjp(const double q[4], const double dR[9], double dq[4]) {
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    dq[0] = 2 * (-z * dR[1] + y * dR[2] + z * dR[3] - x * dR[5] - y * dR[6] + x * dR[7]);
    dq[1] = 2 * (y * dR[1] + z * dR[2] + y * dR[3] - 2 * x * dR[4] - w * dR[5] + z * dR[6]
                 + w * dR[7] - 2 * x * dR[8]);
    dq[2] = 2 * (-2 * y * dR[0] + x * dR[1] + w * dR[2] + x * dR[3] + z * dR[5] - w * dR[6]
                 + z * dR[7] - 2 * y * dR[8]);
    dq[3] = 2 * (-2 * z * dR[0] - w * dR[1] + x * dR[2] + w * dR[3] - 2 * z * dR[4]
                 + y * dR[5] + x * dR[6] + y * dR[7]);
}

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* ------------------------------------------------------------- per-Gaussian state */
typedef struct {
    double mu[3], s[3], qn[4], qnorm, Rg[9], Sigma[9], o;
    double u[3], unorm, d[3]; /* direction from the camera centre */
    double t[3];
    int clampx, clampy;       /* Jacobian clamp sign (-1, 0, +1) */
    double J[6], M[6];        /* J (2x3), M = J W (2x3) */
    double sa, sb, sc, det;   /* Sigma' = [[sa, sb], [sb, sc]] (with low-pass) */
    double A, B, C;           /* conic */
    double mx, my;
    double Y[16], col_raw[3], col[3];
    int valid, flags;
} gstate;

static void load_gauss(const double *P, int64_t n, int64_t i, int deg, gstate *g) {
    for (int a = 0; a < 3; a++) {
        g->mu[a] = P[(0 + a) * n + i];
        g->s[a] = exp(P[(3 + a) * n + i]);
    }
    double q[4], qq = 0;
    for (int a = 0; a < 4; a++) { q[a] = P[(6 + a) * n + i]; qq += q[a] * q[a]; }
    g->qnorm = sqrt(qq);
    for (int a = 0; a < 4; a++) g->qn[a] = q[a] / g->qnorm;
    quat_rot(g->qn, g->Rg);
    /* Sigma = R diag(s^2) R^T */
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += g->Rg[3 * r + k] * g->s[k] * g->s[k] * g->Rg[3 * c + k];
            g->Sigma[3 * r + c] = acc;
        }
    g->o = sigmoid(P[10 * n + i]);
    (void)deg;
}

/* Projection of Gaussian i into camera cam (fills the per-view part of g). */
static void project_one(const double *P, int64_t n, int64_t i, int deg, const double *cam,
                        gstate *g) {
    load_gauss(P, n, i, deg, g);
    const double *W = cam + C_R, *tv = cam + C_T;
    g->flags = 0;
    g->valid = 1;
    for (int r = 0; r < 3; r++)
        g->t[r] = W[3 * r] * g->mu[0] + W[3 * r + 1] * g->mu[1] + W[3 * r + 2] * g->mu[2] + tv[r];
    const double znear = cam[C_ZNEAR];
    if (fabs(g->t[2] - znear) < 1e-6 * fmax(1.0, znear)) g->flags |= F_NEAR_CULL;
    if (g->t[2] <= znear) { g->valid = 0; return; }
    const double fx = cam[C_FX], fy = cam[C_FY], tz = g->t[2];
    const double limx = JCLAMP * cam[C_TANX], limy = JCLAMP * cam[C_TANY];
    double rx = g->t[0] / tz, ry = g->t[1] / tz;
    g->clampx = rx > limx ? 1 : (rx < -limx ? -1 : 0);
    g->clampy = ry > limy ? 1 : (ry < -limy ? -1 : 0);
    if (fabs(fabs(rx) - limx) < 1e-6 * limx || fabs(fabs(ry) - limy) < 1e-6 * limy)
        g->flags |= F_NEAR_GRAD;
    double txc = tz * (rx > limx ? limx : (rx < -limx ? -limx : rx));
    double tyc = tz * (ry > limy ? limy : (ry < -limy ? -limy : ry));
    g->J[0] = fx / tz; g->J[1] = 0; g->J[2] = -fx * txc / (tz * tz);
    g->J[3] = 0; g->J[4] = fy / tz; g->J[5] = -fy * tyc / (tz * tz);
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += g->J[3 * r + k] * W[3 * k + c];
            g->M[3 * r + c] = acc;
        }
    /* Sigma' = M Sigma M^T + 0.3 I */
    double S2[4];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++)
                for (int l = 0; l < 3; l++) acc += g->M[3 * r + k] * g->Sigma[3 * k + l] * g->M[3 * c + l];
            S2[2 * r + c] = acc;
        }
    g->sa = S2[0] + LOWPASS;
    g->sb = 0.5 * (S2[1] + S2[2]);
    g->sc = S2[3] + LOWPASS;
    g->det = g->sa * g->sc - g->sb * g->sb;
    if (g->det <= 1e-9 * g->sa * g->sc) g->flags |= F_NEAR_CULL;
    if (g->det <= 0) { g->valid = 0; return; }
    g->A = g->sc / g->det;
    g->B = -g->sb / g->det;
    g->C = g->sa / g->det;
    g->mx = fx * g->t[0] / tz + cam[C_CX];
    g->my = fy * g->t[1] / tz + cam[C_CY];
    if (fabs(g->o * 255.0 - 1.0) < 1e-5) g->flags |= F_NEAR_CULL;
    if (g->o < ALPHA_MIN) { g->valid = 0; return; }
    /* colour from SH along the viewing direction */
    double un = 0;
    for (int a = 0; a < 3; a++) { g->u[a] = g->mu[a] - cam[C_CAMPOS + a]; un += g->u[a] * g->u[a]; }
    g->unorm = sqrt(un);
    for (int a = 0; a < 3; a++) g->d[a] = g->u[a] / g->unorm;
    sh_basis(deg, g->d, g->Y, NULL);
    const int K = n_coeffs(deg);
    for (int ch = 0; ch < 3; ch++) {
        double acc = 0;
        for (int k = 0; k < K; k++) acc += P[(11 + 3 * k + ch) * n + i] * g->Y[k];
        g->col_raw[ch] = acc + 0.5;
        g->col[ch] = g->col_raw[ch] > 0 ? g->col_raw[ch] : 0.0;
        if (fabs(g->col_raw[ch]) < 1e-6) g->flags |= F_NEAR_GRAD;
    }
}

static void fill_record(const gstate *g, const double *cam, double *rec) {
    memset(rec, 0, ORC_NREC * sizeof(double));
    rec[R_VALID] = g->valid;
    rec[R_TZ] = g->t[2]; rec[R_TX] = g->t[0]; rec[R_TY] = g->t[1];
    if (!g->valid) return;
    rec[R_MX] = g->mx; rec[R_MY] = g->my;
    rec[R_CA] = g->A; rec[R_CB] = g->B; rec[R_CC] = g->C;
    rec[R_O] = g->o;
    rec[R_CR] = g->col[0]; rec[R_CG] = g->col[1]; rec[R_CBL] = g->col[2];
    rec[R_SA] = g->sa; rec[R_SB] = g->sb; rec[R_SC] = g->sc;
    /* support box: the exact AABB of the ellipse where o e^power >= 1/255,
     * padded by a relative and an absolute margin */
    const double k2 = 2.0 * log(255.0 * g->o);
    const double hx = sqrt(k2 * g->sa) * (1.0 + BOX_REL) + BOX_ABS;
    const double hy = sqrt(k2 * g->sc) * (1.0 + BOX_REL) + BOX_ABS;
    rec[R_EX0] = g->mx - hx - 0.5; rec[R_EX1] = g->mx + hx - 0.5;
    rec[R_EY0] = g->my - hy - 0.5; rec[R_EY1] = g->my + hy - 0.5;
    rec[R_D32] = (double)(float)g->t[2];
    (void)cam;
}

/* Per-view projection of all Gaussians: records [n][ORC_NREC], flags [n]. */
int orc_project(const double *P, int64_t n, int deg, const double *cam, double *rec,
                int32_t *flags) {
    if (deg < 0 || deg > 3 || n < 0) return 1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        gstate g;
        project_one(P, n, i, deg, cam, &g);
        fill_record(&g, cam, rec + ORC_NREC * i);
        flags[i] = g.flags;
    }
    return 0;
}

/* ----------------------------------------------------------------- depth order */
typedef struct { float d; int64_t i; } dkey;
static int cmp_dkey(const void *a, const void *b) {
    const dkey *x = a, *y = b;
    uint32_t bx, by;
    memcpy(&bx, &x->d, 4); memcpy(&by, &y->d, 4);
    if (bx != by) return bx < by ? -1 : 1;
    return x->i < y->i ? -1 : (x->i > y->i);
}

/* valid records sorted by (fp32 depth bit pattern, index); returns count */
static int64_t depth_order(const double *rec, int64_t n, int64_t *order) {
    dkey *k = malloc(sizeof(dkey) * (n > 0 ? n : 1));
    int64_t m = 0;
    for (int64_t i = 0; i < n; i++)
        if (rec[ORC_NREC * i + R_VALID] != 0) { k[m].d = (float)rec[ORC_NREC * i + R_TZ]; k[m].i = i; m++; }
    qsort(k, m, sizeof(dkey), cmp_dkey);
    for (int64_t j = 0; j < m; j++) order[j] = k[j].i;
    free(k);
    return m;
}

static uint32_t f32bits(double d) { float f = (float)d; uint32_t b; memcpy(&b, &f, 4); return b; }

/* ---------------------------------------------------------------- compositing */
typedef struct { int64_t i; double alpha, ae, T, power, dx, dy; int clamped; } contrib;

/* Front-to-back over all records in depth order at pixel centre (px, py).
 * Fills the contributor list (if non-NULL, capacity m) and returns the count. */
static int64_t composite_pixel(const double *rec, const int64_t *order, int64_t m, double px,
                               double py, const double *bg, double out[4], double *tfinal,
                               int64_t *last, int32_t *flags, contrib *list) {
    double T = 1.0, C[3] = {0, 0, 0};
    int64_t nc = 0, lst = -1;
    int32_t fl = 0;
    uint32_t prev_bits = 0;
    int have_prev = 0;
    for (int64_t j = 0; j < m; j++) {
        const int64_t i = order[j];
        const double *r = rec + ORC_NREC * i;
        const double dx = px - r[R_MX], dy = py - r[R_MY];
        const double power = -0.5 * (r[R_CA] * dx * dx + r[R_CC] * dy * dy) - r[R_CB] * dx * dy;
        if (power > 0) continue;
        const double ae = r[R_O] * exp(power);
        if (fabs(ae * 255.0 - 1.0) < 1e-4) fl |= F_NEAR_ALPHA;
        if (ae < ALPHA_MIN) continue;
        const double alpha = ae < ALPHA_MAX ? ae : ALPHA_MAX;
        if (fabs(ae / ALPHA_MAX - 1.0) < 1e-4) fl |= F_NEAR_CLAMP;
        const uint32_t bits = f32bits(r[R_TZ]);
        if (have_prev && bits - prev_bits <= 4u) fl |= F_NEAR_TIE;
        have_prev = 1;
        prev_bits = bits;
        const double Tn = T * (1.0 - alpha);
        if (fabs(Tn / T_STOP - 1.0) < 1e-4) fl |= F_NEAR_STOP;
        if (Tn < T_STOP) break;
        if (list) {
            contrib *c = &list[nc];
            c->i = i; c->alpha = alpha; c->ae = ae; c->T = T; c->power = power;
            c->dx = dx; c->dy = dy; c->clamped = ae > ALPHA_MAX;
        }
        C[0] += r[R_CR] * alpha * T;
        C[1] += r[R_CG] * alpha * T;
        C[2] += r[R_CBL] * alpha * T;
        T = Tn;
        lst = i;
        nc++;
    }
    for (int c = 0; c < 3; c++) out[c] = C[c] + T * bg[c];
    out[3] = 1.0 - T;
    *tfinal = T;
    *last = lst;
    *flags = fl;
    return nc;
}

static void pixel_xy(const double *cam, const int64_t *pix, int64_t k, double *px, double *py) {
    const int64_t w = (int64_t)cam[C_W];
    const int64_t id = pix ? pix[k] : k;
    *px = (double)(id % w) + 0.5;
    *py = (double)(id / w) + 0.5;
}

/* Render the listed pixels (linear ids y*W + x), or all pixels when pix == NULL.
 * rgba [4][npix], tfinal [npix], last [npix] (Gaussian index or -1),
 * ncontrib [npix], flags [npix]. */
int orc_render(const double *P, int64_t n, int deg, const double *cam, const int64_t *pix,
               int64_t npix, double *rgba, double *tfinal, int64_t *last, int64_t *ncontrib,
               int32_t *pflags) {
    if (deg < 0 || deg > 3) return 1;
    const int64_t total = (int64_t)cam[C_W] * (int64_t)cam[C_H];
    if (!pix) npix = total;
    double *rec = malloc(sizeof(double) * ORC_NREC * (n > 0 ? n : 1));
    int32_t *rf = malloc(sizeof(int32_t) * (n > 0 ? n : 1));
    int64_t *order = malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    orc_project(P, n, deg, cam, rec, rf);
    const int64_t m = depth_order(rec, n, order);
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t k = 0; k < npix; k++) {
        double px, py, out[4];
        pixel_xy(cam, pix, k, &px, &py);
        ncontrib[k] = composite_pixel(rec, order, m, px, py, cam + C_BG, out, &tfinal[k], &last[k],
                                      &pflags[k], NULL);
        for (int c = 0; c < 4; c++) rgba[c * npix + k] = out[c];
    }
    free(rec); free(rf); free(order);
    return 0;
}

/* ----------------------------------------------------------- projection adjoint */
/* Adds the parameter gradient of Gaussian i for one view, given the 2D gradient
 * g2 = (d mx, d my, d A, d B, d C, d o, d r, d g, d b).  dSigma accumulates the
 * covariance gradient so scale/rotation gradients can be formed once. */
static void project_vjp(const double *P, int64_t n, int64_t i, int deg, const double *cam,
                        const gstate *g, const double g2[9], double *G, double dSigma[9],
                        double *dopacity) {
    const double *W = cam + C_R;
    const double fx = cam[C_FX], fy = cam[C_FY], tz = g->t[2], tx = g->t[0], ty = g->t[1];
    /* conic = inverse(Sigma'): dSigma' = -Q dQ Q with dQ symmetric (B appears twice) */
    const double Q[4] = {g->A, g->B, g->B, g->C};
    const double dQ[4] = {g2[2], 0.5 * g2[3], 0.5 * g2[3], g2[4]};
    double tmp[4], dS2[4];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double acc = 0;
            for (int k = 0; k < 2; k++) acc += Q[2 * r + k] * dQ[2 * k + c];
            tmp[2 * r + c] = acc;
        }
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 2; c++) {
            double acc = 0;
            for (int k = 0; k < 2; k++) acc += tmp[2 * r + k] * Q[2 * k + c];
            dS2[2 * r + c] = -acc;
        }
    /* Sigma' = M Sigma M^T (+ 0.3 I): dSigma += M^T dS2 M; dM = 2 dS2 M Sigma */
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int a = 0; a < 2; a++)
                for (int b = 0; b < 2; b++) acc += g->M[3 * a + r] * dS2[2 * a + b] * g->M[3 * b + c];
            dSigma[3 * r + c] += acc;
        }
    double MS[6], dM[6], dJ[6];
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += g->M[3 * r + k] * g->Sigma[3 * k + c];
            MS[3 * r + c] = acc;
        }
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 2; k++) acc += dS2[2 * r + k] * MS[3 * k + c];
            dM[3 * r + c] = 2.0 * acc;
        }
    /* M = J W: dJ = dM W^T */
    for (int r = 0; r < 2; r++)
        for (int c = 0; c < 3; c++) {
            double acc = 0;
            for (int k = 0; k < 3; k++) acc += dM[3 * r + k] * W[3 * c + k];
            dJ[3 * r + c] = acc;
        }
    /* J entries as functions of t */
    double dt[3] = {0, 0, 0};
    dt[2] += -fx / (tz * tz) * dJ[0];
    dt[2] += -fy / (tz * tz) * dJ[4];
    const double limx = JCLAMP * cam[C_TANX], limy = JCLAMP * cam[C_TANY];
    if (g->clampx == 0) {
        dt[0] += -fx / (tz * tz) * dJ[2];
        dt[2] += 2.0 * fx * tx / (tz * tz * tz) * dJ[2];
    } else { /* J02 = -fx (+-limx) / tz */
        dt[2] += fx * (g->clampx * limx) / (tz * tz) * dJ[2];
    }
    if (g->clampy == 0) {
        dt[1] += -fy / (tz * tz) * dJ[5];
        dt[2] += 2.0 * fy * ty / (tz * tz * tz) * dJ[5];
    } else {
        dt[2] += fy * (g->clampy * limy) / (tz * tz) * dJ[5];
    }
    /* pixel mean: mx = fx tx / tz + cx */
    dt[0] += fx / tz * g2[0];
    dt[2] += -fx * tx / (tz * tz) * g2[0];
    dt[1] += fy / tz * g2[1];
    dt[2] += -fy * ty / (tz * tz) * g2[1];
    /* t = W mu + t_v */
    for (int a = 0; a < 3; a++)
        G[a * n + i] += W[a] * dt[0] + W[3 + a] * dt[1] + W[6 + a] * dt[2];
    *dopacity += g2[5];
    /* colour = max(0, sum_k sh_k Y_k(d) + 0.5) per channel */
    const int K = n_coeffs(deg);
    double Y[16], dY[16][3], dd[3] = {0, 0, 0};
    sh_basis(deg, g->d, Y, dY);
    for (int ch = 0; ch < 3; ch++) {
        if (!(g->col_raw[ch] > 0)) continue;
        const double dc = g2[6 + ch];
        for (int k = 0; k < K; k++) {
            G[(11 + 3 * k + ch) * n + i] += Y[k] * dc;
            const double shv = P[(11 + 3 * k + ch) * n + i];
            for (int a = 0; a < 3; a++) dd[a] += dc * shv * dY[k][a];
        }
    }
    /* d = u / |u|, u = mu - campos */
    const double ddot = dd[0] * g->d[0] + dd[1] * g->d[1] + dd[2] * g->d[2];
    for (int a = 0; a < 3; a++) G[a * n + i] += (dd[a] - g->d[a] * ddot) / g->unorm;
}

/* gradient through Sigma = R diag(s^2) R^T, s = exp(l), R = R(q / |q|) */
static void covariance_vjp(int64_t n, int64_t i, const gstate *g, const double dSigma[9],
                           double *G) {
    /* symmetrise (dSigma is the gradient w.r.t. a symmetric matrix) */
    double dS[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) dS[3 * r + c] = 0.5 * (dSigma[3 * r + c] + dSigma[3 * c + r]);
    /* M3 = R diag(s), Sigma = M3 M3^T: dM3 = 2 dS M3 */
    double M3[9], dM3[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) M3[3 * r + c] = g->Rg[3 * r + c] * g->s[c];
    mat3_mul(dS, M3, dM3);
    for (int k = 0; k < 9; k++) dM3[k] *= 2.0;
    double ds[3] = {0, 0, 0}, dR[9];
    for (int r = 0; r < 3; r++)
        for (int c = 0; c < 3; c++) {
            ds[c] += dM3[3 * r + c] * g->Rg[3 * r + c];
            dR[3 * r + c] = dM3[3 * r + c] * g->s[c];
        }
    for (int a = 0; a < 3; a++) G[(3 + a) * n + i] += ds[a] * g->s[a];
    double dqn[4];
    quat_rot_vjp(g->qn, dR, dqn);
    const double dot = dqn[0] * g->qn[0] + dqn[1] * g->qn[1] + dqn[2] * g->qn[2] + dqn[3] * g->qn[3];
    for (int a = 0; a < 4; a++) G[(6 + a) * n + i] += (dqn[a] - g->qn[a] * dot) / g->qnorm;
    (void)mat3_transpose;
}

/* Accumulate the per-Gaussian 2D gradient g2d [9][n] of one view for the listed
 * pixels given dL/dRGBA [4][npix]. */
static void composite_vjp(const double *rec, const int64_t *order, int64_t m, const double *cam,
                          const int64_t *pix, int64_t npix, const double *dl, int64_t n,
                          double *g2d) {
    int nthr = 1;
#ifdef _OPENMP
    nthr = omp_get_max_threads();
#endif
    double *acc = calloc((size_t)nthr * 9 * (size_t)(n > 0 ? n : 1), sizeof(double));
#pragma omp parallel
    {
        int tid = 0;
#ifdef _OPENMP
        tid = omp_get_thread_num();
#endif
        double *mine = acc + (size_t)tid * 9 * (size_t)n;
        contrib *list = malloc(sizeof(contrib) * (m > 0 ? m : 1));
        double *prefix = malloc(sizeof(double) * 3 * (m > 0 ? m : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t k = 0; k < npix; k++) {
            const double g[3] = {dl[0 * npix + k], dl[1 * npix + k], dl[2 * npix + k]};
            const double gA = dl[3 * npix + k];
            if (g[0] == 0 && g[1] == 0 && g[2] == 0 && gA == 0) continue;
            double px, py, out[4], Tf;
            int64_t lst;
            int32_t fl;
            pixel_xy(cam, pix, k, &px, &py);
            const int64_t nc = composite_pixel(rec, order, m, px, py, cam + C_BG, out, &Tf, &lst,
                                               &fl, list);
            /* inclusive prefix of colour * alpha * T */
            double run[3] = {0, 0, 0};
            for (int64_t j = 0; j < nc; j++) {
                const double *r = rec + ORC_NREC * list[j].i;
                const double w = list[j].alpha * list[j].T;
                run[0] += r[R_CR] * w; run[1] += r[R_CG] * w; run[2] += r[R_CBL] * w;
                prefix[3 * j] = run[0]; prefix[3 * j + 1] = run[1]; prefix[3 * j + 2] = run[2];
            }
            for (int64_t j = 0; j < nc; j++) {
                const contrib *c = &list[j];
                const double *r = rec + ORC_NREC * c->i;
                const double col[3] = {r[R_CR], r[R_CG], r[R_CBL]};
                /* colour behind this Gaussian: R_j = RGB - C_{<=j} */
                double gdotR = 0, gdotc = 0;
                for (int ch = 0; ch < 3; ch++) {
                    gdotR += g[ch] * (out[ch] - prefix[3 * j + ch]);
                    gdotc += g[ch] * col[ch];
                }
                const double oma = 1.0 - c->alpha;
                const double dalpha = c->T * gdotc - gdotR / oma + gA * Tf / oma;
                double *gi = mine;
                const int64_t i = c->i;
                for (int ch = 0; ch < 3; ch++) gi[(6 + ch) * n + i] += c->alpha * c->T * g[ch];
                if (c->clamped) continue;
                const double dpow = c->ae * dalpha;
                gi[5 * n + i] += exp(c->power) * dalpha;
                gi[2 * n + i] += -0.5 * c->dx * c->dx * dpow;
                gi[3 * n + i] += -c->dx * c->dy * dpow;
                gi[4 * n + i] += -0.5 * c->dy * c->dy * dpow;
                /* delta = p - mean */
                gi[0 * n + i] += (r[R_CA] * c->dx + r[R_CB] * c->dy) * dpow;
                gi[1 * n + i] += (r[R_CB] * c->dx + r[R_CC] * c->dy) * dpow;
            }
        }
        free(list);
        free(prefix);
    }
    for (int t = 0; t < nthr; t++)
        for (int64_t e = 0; e < 9 * n; e++) g2d[e] += acc[(size_t)t * 9 * (size_t)n + e];
    free(acc);
}

/* Gradient of sum_p <dl_p, rgba_p> w.r.t. the raw parameters for one view.
 * grads [C][n] and g2d [9][n] (may be NULL) are ACCUMULATED into. */
int orc_backward(const double *P, int64_t n, int deg, const double *cam, const int64_t *pix,
                 int64_t npix, const double *dl, double *grads, double *g2d_out) {
    if (deg < 0 || deg > 3) return 1;
    const int64_t total = (int64_t)cam[C_W] * (int64_t)cam[C_H];
    if (!pix) npix = total;
    const int64_t nn = n > 0 ? n : 1;
    double *rec = malloc(sizeof(double) * ORC_NREC * nn);
    int32_t *rf = malloc(sizeof(int32_t) * nn);
    int64_t *order = malloc(sizeof(int64_t) * nn);
    double *g2d = calloc(9 * (size_t)nn, sizeof(double));
    orc_project(P, n, deg, cam, rec, rf);
    const int64_t m = depth_order(rec, n, order);
    composite_vjp(rec, order, m, cam, pix, npix, dl, n, g2d);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++) {
        if (rec[ORC_NREC * i + R_VALID] == 0) continue;
        double g2[9];
        int any = 0;
        for (int f = 0; f < 9; f++) { g2[f] = g2d[f * n + i]; any |= g2[f] != 0; }
        if (!any) continue;
        gstate g;
        project_one(P, n, i, deg, cam, &g);
        double dSigma[9] = {0}, dop = 0;
        project_vjp(P, n, i, deg, cam, &g, g2, grads, dSigma, &dop);
        covariance_vjp(n, i, &g, dSigma, grads);
        grads[10 * n + i] += g.o * (1.0 - g.o) * dop;
    }
    if (g2d_out)
        for (int64_t e = 0; e < 9 * n; e++) g2d_out[e] += g2d[e];
    free(rec); free(rf); free(order); free(g2d);
    return 0;
}

/* ------------------------------------------------------------- discrete stage */
typedef struct { int64_t tile; uint32_t dbits; int64_t rec; } tkey;
static int cmp_tkey(const void *a, const void *b) {
    const tkey *x = a, *y = b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->dbits != y->dbits) return x->dbits < y->dbits ? -1 : 1;
    return x->rec < y->rec ? -1 : (x->rec > y->rec);
}

/* integer pixel box [x0, x1] from the real edges, clamped to the image */
static void int_box(double e0, double e1, int64_t size, int64_t *lo, int64_t *hi) {
    double a = ceil(e0), b = floor(e1);
    if (a < 0) a = 0;
    if (b > (double)(size - 1)) b = (double)(size - 1);
    *lo = (int64_t)a;
    *hi = (int64_t)b;
}

/* tile rectangle of an edge pair, or empty (returns 0) */
static int tile_rect(double e0, double e1, int64_t size, int tile, int64_t *t0, int64_t *t1) {
    int64_t lo, hi;
    if (!(e0 == e0) || !(e1 == e1)) return 0;
    if (e0 > 1e15 || e1 < -1e15) return 0;
    int_box(e0 < -1e15 ? -1e15 : e0, e1 > 1e15 ? 1e15 : e1, size, &lo, &hi);
    if (lo > hi) return 0;
    *t0 = lo / tile;
    *t1 = hi / tile;
    return 1;
}

/* Tile columns [*c0, *c1] of tile row ty that the padded support ellipse
 * reaches, or 0 when none.  The ellipse is q(d) = d^T Sigma'^-1 d <= Kp with
 * Kp = 2 ln(255 o) (1 + BOX_REL)^2, d the offset of a pixel centre from the
 * mean.  Over the row's pixel-centre band (rows ty T .. min(ty T + T, H) - 1)
 * its x extent is taken where the ellipse's boundary is rightmost (leftmost)
 * within the band, widened by BOX_ABS; the pixel columns whose centres lie in
 * that extent, clamped to the image and to the record's tile rectangle
 * [x0, x1], give the tiles.  `shift` moves both extents outward (> 0) or inward
 * (< 0), for the rounding flags. */
static int row_span(const double *r, int64_t ty, int tile, int64_t W, int64_t H, int64_t x0,
                    int64_t x1, double shift, int64_t *c0, int64_t *c1) {
    const double sa = r[R_SA], sb = r[R_SB], sc = r[R_SC];
    const double Kp = 2.0 * log(255.0 * r[R_O]) * (1.0 + BOX_REL) * (1.0 + BOX_REL);
    const int64_t ja = ty * tile, jb = (ty * tile + tile < H ? ty * tile + tile : H) - 1;
    const double ya = (double)ja + 0.5 - r[R_MY], yb = (double)jb + 0.5 - r[R_MY];
    const double ey = sqrt(Kp * sc);
    double lo = ya > -ey ? ya : -ey, hi = yb < ey ? yb : ey;
    if (lo > hi) lo = hi = (ya > ey ? ey : -ey);          /* band beside the ellipse: its tip */
    const double slope = sb / sc, wid = sa - sb * sb / sc;
    const double dyr = sb * sqrt(Kp / sa);                /* rows of the right- and leftmost points */
    const double d1 = dyr < lo ? lo : (dyr > hi ? hi : dyr);
    const double d2 = -dyr < lo ? lo : (-dyr > hi ? hi : -dyr);
    const double h1 = Kp - d1 * d1 / sc, h2 = Kp - d2 * d2 / sc;
    const double xr = slope * d1 + sqrt((h1 > 0 ? h1 : 0.0) * wid) + BOX_ABS + shift;
    const double xl = slope * d2 - sqrt((h2 > 0 ? h2 : 0.0) * wid) - BOX_ABS - shift;
    double a = ceil(r[R_MX] + xl - 0.5), b = floor(r[R_MX] + xr - 0.5);
    if (a < 0) a = 0;
    if (b > (double)(W - 1)) b = (double)(W - 1);
    if (a > b) return 0;
    int64_t t0 = (int64_t)a / tile, t1 = (int64_t)b / tile;
    if (t0 < x0) t0 = x0;
    if (t1 > x1) t1 = x1;
    if (t0 > t1) return 0;
    *c0 = t0;
    *c1 = t1;
    return 1;
}

/* Keys/values of all views ordered by (global tile, fp32 depth bits, record)
 * and the per-tile [start, end) ranges.  Records are r = v*n + i.  Returns the
 * key count in *m_out (keys beyond cap are counted but not written).
 * rflags [V*n] receives F_NEAR_BOX / F_NEAR_TIE / F_NEAR_CULL. */
int orc_discrete(const double *P, int64_t n, int deg, const double *cams, int nviews, int tile,
                 int64_t *keys, int64_t *vals, int64_t cap, int64_t *m_out, int64_t *ranges,
                 int32_t *rflags) {
    if (tile <= 0 || nviews <= 0) return 1;
    const int64_t nn = n > 0 ? n : 1;
    double *rec = malloc(sizeof(double) * ORC_NREC * nn);
    int32_t *rf = malloc(sizeof(int32_t) * nn);
    int64_t total_tiles = 0, count = 0, alloc = 1024;
    tkey *list = malloc(sizeof(tkey) * alloc);
    for (int v = 0; v < nviews; v++) {
        const double *cam = cams + 27 * v;
        const int64_t W = (int64_t)cam[C_W], H = (int64_t)cam[C_H];
        const int64_t tw = (W + tile - 1) / tile, th = (H + tile - 1) / tile;
        orc_project(P, n, deg, cam, rec, rf);
        for (int64_t i = 0; i < n; i++) {
            const double *r = rec + ORC_NREC * i;
            int32_t fl = rf[i] & F_NEAR_CULL;
            if (r[R_VALID] != 0) {
                /* a box edge is ambiguous if moving it by the margin changes the rect */
                const double mx = 2e-4 + 2e-6 * fabs(r[R_MX]), my = 2e-4 + 2e-6 * fabs(r[R_MY]);
                int64_t a0, a1, b0, b1, c0, c1, d0, d1;
                int ea = tile_rect(r[R_EX0] - mx, r[R_EX1] + mx, W, tile, &a0, &a1);
                int eb = tile_rect(r[R_EX0] + mx, r[R_EX1] - mx, W, tile, &b0, &b1);
                int ec = tile_rect(r[R_EY0] - my, r[R_EY1] + my, H, tile, &c0, &c1);
                int ed = tile_rect(r[R_EY0] + my, r[R_EY1] - my, H, tile, &d0, &d1);
                if (ea != eb || ec != ed || (ea && (a0 != b0 || a1 != b1))
                    || (ec && (c0 != d0 || c1 != d1)))
                    fl |= F_NEAR_BOX;
                int64_t x0, x1, y0, y1;
                if (tile_rect(r[R_EX0], r[R_EX1], W, tile, &x0, &x1)
                    && tile_rect(r[R_EY0], r[R_EY1], H, tile, &y0, &y1)) {
                    for (int64_t ty = y0; ty <= y1; ty++) {
                        /* the tiles of this row the support ellipse reaches */
                        int64_t s0 = x0, s1 = x1, p0, p1, q0, q1;
                        const double m = 2e-4 + 4e-6 * (fabs(r[R_MX]) + fabs(r[R_EX1] - r[R_EX0]));
                        const int in = row_span(r, ty, tile, W, H, x0, x1, 0.0, &s0, &s1);
                        const int out = row_span(r, ty, tile, W, H, x0, x1, m, &p0, &p1);
                        const int inw = row_span(r, ty, tile, W, H, x0, x1, -m, &q0, &q1);
                        if (out != inw || (out && (p0 != q0 || p1 != q1))) fl |= F_NEAR_BOX;
                        if (!in) continue;
                        for (int64_t tx = s0; tx <= s1; tx++) {
                            if (count == alloc) { alloc *= 2; list = realloc(list, sizeof(tkey) * alloc); }
                            list[count].tile = total_tiles + ty * tw + tx;
                            list[count].dbits = f32bits(r[R_TZ]);
                            list[count].rec = (int64_t)v * n + i;
                            count++;
                        }
                    }
                }
            }
            rflags[(int64_t)v * n + i] = fl;
        }
        total_tiles += tw * th;
    }
    qsort(list, count, sizeof(tkey), cmp_tkey);
    /* depth ties inside one tile */
    for (int64_t k = 1; k < count; k++)
        if (list[k].tile == list[k - 1].tile && list[k].dbits - list[k - 1].dbits <= 4u) {
            rflags[list[k].rec] |= F_NEAR_TIE;
            rflags[list[k - 1].rec] |= F_NEAR_TIE;
        }
    for (int64_t k = 0; k < count && k < cap; k++) { keys[k] = list[k].tile; vals[k] = list[k].rec; }
    /* ranges by lower bound: [lb(t), lb(t + 1)) */
    int64_t pos = 0;
    for (int64_t t = 0; t < total_tiles; t++) {
        ranges[2 * t] = pos;
        while (pos < count && list[pos].tile == t) pos++;
        ranges[2 * t + 1] = pos;
    }
    *m_out = count;
    free(list); free(rec); free(rf);
    return 0;
}

/* --------------------------------------------------------------- loss, Adam */
/* Fovea mask of pixel (x, y): its centre within `radius` of the gaze point,
 * inclusive (Method, "Periphery Model Training": the loss covers the fovea).
 * The test decides which entries the mean covers, an integer, so it is taken
 * in the compositing path's single precision: gaze and radius rounded to
 * float, then (x + 0.5 - gx)^2 + (y + 0.5 - gy)^2 <= radius^2 with every
 * operation rounded to float (no contraction; the build passes
 * -ffp-contract=off).  In double, a centre within a few float ulps of the
 * circle could land on the other side. */
static int in_fovea32(int64_t x, int64_t y, const double *gaze, double radius) {
    const float r = (float)radius;
    const float dx = ((float)x + 0.5f) - (float)gaze[0];
    const float dy = ((float)y + 0.5f) - (float)gaze[1];
    return dx * dx + dy * dy <= r * r;
}

/* Sum of |RGB - target| over the masked pixel-channels of one view and its
 * sign (written to dl [4][H*W], alpha channel zero).  Mask: in_fovea32;
 * gaze == NULL means no mask.  Returns the number of masked pixel-channels in
 * *count. */
double orc_loss_l1(const double *rgba, const double *target, int64_t w, int64_t h,
                   const double *gaze, double radius, double *dl, int64_t *count) {
    const int64_t npix = w * h;
    double sum = 0;
    int64_t cnt = 0;
    for (int64_t k = 0; k < npix; k++) {
        const int in = gaze ? in_fovea32(k % w, k / w, gaze, radius) : 1;
        dl[3 * npix + k] = 0;
        for (int c = 0; c < 3; c++) {
            const double d = rgba[c * npix + k] - target[c * npix + k];
            if (in) {
                sum += fabs(d);
                cnt++;
                dl[c * npix + k] = d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0);
            } else {
                dl[c * npix + k] = 0;
            }
        }
    }
    *count = cnt;
    return sum;
}

/* Alpha training with a background (Method, "Periphery Model Training": the
 * peripheral model is trained on alpha as well as colour, over randomised
 * backgrounds).  Reading: the target is RGBA, its colour premultiplied (an
 * emission-absorption render over black); prediction and target are both
 * composited over the view's background bg, i.e. the target becomes
 * target_rgb + (1 - target_alpha) bg while the prediction was rendered with
 * bg; the L1 covers R, G, B and, with alpha != 0, A.  Returns the sum of the
 * masked terms; *count = the number of masked entries; dl = their signs. */
double orc_loss_l1_rgba(const double *rgba, const double *target_rgba, const double *bg, int64_t w,
                        int64_t h, const double *gaze, double radius, int alpha, double *dl,
                        int64_t *count) {
    const int64_t npix = w * h;
    double sum = 0;
    int64_t cnt = 0;
    for (int64_t k = 0; k < npix; k++) {
        const int in = gaze ? in_fovea32(k % w, k / w, gaze, radius) : 1;
        const double ta = target_rgba[3 * npix + k];
        for (int c = 0; c < 4; c++) {
            double t = target_rgba[c * npix + k];
            if (c < 3 && bg) t += (1.0 - ta) * bg[c];
            const double d = rgba[c * npix + k] - t;
            if (in && (c < 3 || alpha)) {
                sum += fabs(d);
                cnt++;
                dl[c * npix + k] = d > 0 ? 1.0 : (d < 0 ? -1.0 : 0.0);
            } else {
                dl[c * npix + k] = 0;
            }
        }
    }
    *count = cnt;
    return sum;
}

/* One Adam step (t = step number, >= 1) on n elements, in place. */
void orc_adam(double *p, const double *g, double *m, double *v, int64_t n, double lr, double b1,
              double b2, double eps, int64_t t) {
    const double bc1 = 1.0 - pow(b1, (double)t), bc2 = 1.0 - pow(b2, (double)t);
    for (int64_t e = 0; e < n; e++) {
        m[e] = b1 * m[e] + (1.0 - b1) * g[e];
        v[e] = b2 * v[e] + (1.0 - b2) * g[e] * g[e];
        const double mh = m[e] / bc1, vh = v[e] / bc2;
        p[e] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------- first-hit point cloud */
/* Initial point cloud (Method, "Volumetric Path Tracing"): rays are cast at the
 * volume from several viewpoints, the first significant hit of each ray is
 * kept and coloured.  Each pixel-centre ray of each camera is marched through
 * the volume box [-1, 1]^3 in segments of length `step` from the box entry
 * (the last one shortened to the exit), each sampled at its midpoint: raw
 * value v trilinear in the grid (voxel centres at (idx + 1/2) 2/n - 1, zero
 * outside), density t = clamp((v - thr) / range, 0, 1), segment opacity
 * 1 - exp(-extinction t length).  The hit is the midpoint of the first
 * segment after which the accumulated opacity 1 - T reaches hit_alpha.  Its
 * colour is the emission-absorption colour (lo (1 - t) + hi t) of that
 * segment and the next color_steps - 1 segments (or up to the exit), composited
 * from opacity zero, divided by their accumulated opacity.
 * hit [R]: 1 / 0; pos [R][3]; col [R][3]; margin [R]: the smallest
 * |1 - T - hit_alpha| after any segment up to the decision (the whole ray
 * when there is no hit).  R = sum over views of width * height, rays in view,
 * row, column order. */
static double vol_sample(const uint16_t *vol, int n, const double p[3]) {
    double u[3], f[3];
    int64_t i0[3];
    for (int a = 0; a < 3; a++) {
        u[a] = (p[a] + 1.0) * 0.5 * n - 0.5;
        const double fl = floor(u[a]);
        i0[a] = (int64_t)fl;
        f[a] = u[a] - fl;
    }
    double acc = 0.0;
    for (int c = 0; c < 8; c++) {
        const int64_t i = i0[0] + (c >> 2 & 1), j = i0[1] + (c >> 1 & 1), k = i0[2] + (c & 1);
        if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) continue;
        const double w = ((c >> 2 & 1) ? f[0] : 1.0 - f[0]) * ((c >> 1 & 1) ? f[1] : 1.0 - f[1]) *
                         ((c & 1) ? f[2] : 1.0 - f[2]);
        acc += w * (double)vol[(i * n + j) * n + k];
    }
    return acc;
}

int orc_first_hits(const uint16_t *vol, int n, const double *cams, int nviews, double step,
                   double extinction, double thr, double range, const double *lo, const double *hi,
                   double hit_alpha, int color_steps, int32_t *hit, double *pos, double *col,
                   double *margin) {
    int64_t base = 0;
    for (int v = 0; v < nviews; v++) {
        const double *cam = cams + 27 * v;
        const int64_t W = (int64_t)cam[C_W], H = (int64_t)cam[C_H];
#pragma omp parallel for schedule(dynamic, 4)
        for (int64_t j = 0; j < H; j++)
            for (int64_t i = 0; i < W; i++) {
                const int64_t r = base + j * W + i;
                const double dc[3] = {((double)i + 0.5 - cam[C_CX]) / cam[C_FX],
                                      ((double)j + 0.5 - cam[C_CY]) / cam[C_FY], 1.0};
                double d[3], o[3], nn = 0.0;
                for (int a = 0; a < 3; a++) {   /* world direction R^T dc */
                    d[a] = cam[C_R + a] * dc[0] + cam[C_R + 3 + a] * dc[1] + cam[C_R + 6 + a] * dc[2];
                    nn += d[a] * d[a];
                    o[a] = cam[C_CAMPOS + a];
                }
                nn = sqrt(nn);
                double t0 = -INFINITY, t1 = INFINITY;
                for (int a = 0; a < 3; a++) {
                    d[a] /= nn;
                    double ta = (-1.0 - o[a]) / d[a], tb = (1.0 - o[a]) / d[a];
                    if (ta > tb) { const double x = ta; ta = tb; tb = x; }
                    if (ta > t0) t0 = ta;
                    if (tb < t1) t1 = tb;
                }
                if (t0 < 0.0) t0 = 0.0;
                hit[r] = 0;
                margin[r] = INFINITY;
                for (int a = 0; a < 3; a++) pos[3 * r + a] = col[3 * r + a] = 0.0;
                if (!(t1 > t0)) continue;
                double T = 1.0;
                int64_t khit = -1;
                for (int64_t k = 0;; k++) {
                    const double s0 = t0 + (double)k * step;
                    double s1 = s0 + step;
                    if (s1 > t1) s1 = t1;
                    if (!(s1 > s0)) break;
                    const double mid = 0.5 * (s0 + s1), p[3] = {o[0] + d[0] * mid, o[1] + d[1] * mid,
                                                                o[2] + d[2] * mid};
                    double t = (vol_sample(vol, n, p) - thr) / range;
                    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                    T *= exp(-extinction * t * (s1 - s0));
                    const double gap = fabs(1.0 - T - hit_alpha);
                    if (gap < margin[r]) margin[r] = gap;
                    if (1.0 - T >= hit_alpha) {
                        khit = k;
                        for (int a = 0; a < 3; a++) pos[3 * r + a] = p[a];
                        break;
                    }
                }
                if (khit < 0) continue;
                hit[r] = 1;
                double C[3] = {0.0, 0.0, 0.0}, Ts = 1.0;
                for (int64_t k = khit; k < khit + color_steps; k++) {
                    const double s0 = t0 + (double)k * step;
                    double s1 = s0 + step;
                    if (s1 > t1) s1 = t1;
                    if (!(s1 > s0)) break;
                    const double mid = 0.5 * (s0 + s1), p[3] = {o[0] + d[0] * mid, o[1] + d[1] * mid,
                                                                o[2] + d[2] * mid};
                    double t = (vol_sample(vol, n, p) - thr) / range;
                    t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
                    const double alpha = 1.0 - exp(-extinction * t * (s1 - s0));
                    for (int a = 0; a < 3; a++) C[a] += (lo[a] * (1.0 - t) + hi[a] * t) * alpha * Ts;
                    Ts *= 1.0 - alpha;
                }
                for (int a = 0; a < 3; a++) col[3 * r + a] = C[a] / (1.0 - Ts);
            }
        base += W * H;
    }
    return 0;
}

int orc_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
