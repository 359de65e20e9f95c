/*
 * megs_oracle.c -- plain FP64 CPU oracle for differentiable SG splatting.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing in the renderer's product path may call,
 * link or load this file; only the tests, the smoke check and the benchmark's
 * CPU-baseline leg do. It shares no code, header, table or constant generator
 * with the GPU library.
 *
 * What it computes (all in double precision, written for readability, not speed):
 *
 *  - Colour: the Spherical-Gaussian model of Sec. 3.2: one lobe is
 *    G(v; mu, s, a) = a * exp(s * (mu . v - 1)) (Eq. for an SG lobe) and the colour
 *    is c(v) = c0 + sum over lobes (Eq. for the view-dependent colour), with each
 *    lobe's amplitude gated by a soft lobe mask m_k = sigmoid(logit).
 *  - Compositing: C = sum_i c_i alpha_i prod_{j<i} (1 - alpha_j), with alpha_i the
 *    product of the primitive's opacity and its projected 2D Gaussian value at the
 *    pixel (Sec. 3.1, Preliminaries). The opacity is gated by a soft primitive mask.
 *  - The 3DGS conventions the paper builds on (Sec. 3.1 cites 3DGS; the paper prints
 *    none of them): EWA projection with a 0.3 pixel^2 dilation, alpha clamped to 0.99,
 *    fragments with alpha < 1/255 skipped, front-to-back termination before the
 *    transmittance would drop below 1e-4, near plane 0.2, Jacobian clamp at 1.3x the
 *    half field of view.
 *  - The tile/depth key table the paper names as part of the dynamic rendering memory
 *    (Sec. 1 and Appendix, evaluation details): key = tile << 32 | bits(float32 depth),
 *    value = record index, ordered by (key, value), with per-tile [start, end) ranges.
 *  - The exact derivative of the rendered image with respect to every raw parameter.
 *
 * Parity: pinned by the tests in tests/test_oracle_*.py (closed forms for the SG lobe and
 * its sphere mean, a single isotropic Gaussian's footprint, the two-Gaussian composite,
 * the empty scene, tiled == brute force, central finite differences, the O(n^2) direct
 * sum for the blend backward). The 3DGS constants above are conventions, not pins.
 */
#include <math.h>
#include <omp.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NEAR_BAND 2e-4 /* relative width of the "near a threshold" flag bands */

typedef struct {
    int64_t n;
    int32_t k;
    int32_t pad;
    const double *pos, *logscale, *quat, *op_logit, *pmask_logit;
    const double *base, *axis, *sharp, *amp, *lmask_logit;
    /* NULL: k lobes per Gaussian, planes axis/amp [k][3][n], sharp/lmask_logit [k][n].
     * Otherwise the lobes of Gaussian i are lobe_off[i] .. lobe_off[i + 1] - 1 (at most k) of
     * planes axis/amp [3][n_lobes], sharp/lmask_logit [n_lobes] (compressed rows). */
    const int32_t *lobe_off;
    int64_t n_lobes;
    /* NULL: SG colour. Otherwise the colour is max(0, sum_m Y_m(d) sh[m] + 1/2) per channel with
     * real spherical harmonics of degree <= sh_degree (3DGS's colour model, the paper's baseline
     * colour), coefficients sh[(sh_degree + 1)^2][3][n]; the SG planes are then unused. */
    const double *sh;
    int32_t sh_degree;
    int32_t pad2;
} oscene;

typedef struct {
    int32_t width, height;
    double fx, fy, cx, cy;
    double R[9], t[3];
    double znear;
    double bg[3];
} ocam;

/* constants of the 3DGS rasteriser conventions */
static const double DILATION = 0.3;
static const double ALPHA_MIN = 1.0 / 255.0;
static const double ALPHA_MAX = 0.99;
static const double T_MIN = 1e-4;
static const double FOV_CLAMP = 1.3;
static const double MAX_COORD = 1e7;

/* threads the OpenMP loops of this file use */
int32_t oracle_threads(void) { return omp_get_max_threads(); }

static double sigmoid(double x) { return 1.0 / (1.0 + exp(-x)); }

/* unit quaternion (w, x, y, z) to a row-major rotation matrix (textbook form) */
static void quat_to_rot(const double q[4], double R[9]) {
    double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1 - 2 * (y * y + z * z); R[1] = 2 * (x * y - w * z);     R[2] = 2 * (x * z + w * y);
    R[3] = 2 * (x * y + w * z);     R[4] = 1 - 2 * (x * x + z * z); R[5] = 2 * (y * z - w * x);
    R[6] = 2 * (x * z - w * y);     R[7] = 2 * (y * z + w * x);     R[8] = 1 - 2 * (x * x + y * y);
}

/* all intermediates of one Gaussian's projection into one view */
typedef struct {
    int valid;
    double s[3], qn, qh[4], Rq[9], M[9], S3[9];
    double t[3], u, v;
    double xi, eta; int xclamp, yclamp;
    double J[6], T[6];
    double A0, B0, C0, det0, det, conic[3];
    double o, mp, o_eff;
    double lmax, rho, cutoff; int radius;
    double campos[3], dvec[3], dlen, d[3];
    double rgb[3];
    double ax_len[8], muh[8][3], mk[8], ek[8], dot[8];
    double shY[16], shdY[16][3];
    int shclamp[3];
    int rect[4]; int ntiles;
} oproj;

static double P(const double *plane, int64_t n, int64_t row, int64_t i) { return plane[row * n + i]; }

/*
 * Real spherical harmonics of degree <= 3 at a unit direction d = (x, y, z), with their partial
 * derivatives in x, y, z (the polynomials extended off the sphere; the caller projects the
 * gradient onto the tangent plane). Orthonormal over the sphere; the sign convention is the one
 * of the 3DGS rasteriser's colour model (degree 1 ordered -y, z, -x).
 */
static void sh_basis(const double d[3], double Y[16], double dY[16][3]) {
    const double pi = acos(-1.0), x = d[0], y = d[1], z = d[2];
    const double a0 = 0.5 * sqrt(1.0 / pi), a1 = sqrt(3.0 / (4.0 * pi));
    const double b = 0.5 * sqrt(15.0 / pi), b6 = 0.25 * sqrt(5.0 / pi), b8 = 0.25 * sqrt(15.0 / pi);
    const double c9 = 0.25 * sqrt(35.0 / (2.0 * pi)), c10 = 0.5 * sqrt(105.0 / pi);
    const double c11 = 0.25 * sqrt(21.0 / (2.0 * pi)), c12 = 0.25 * sqrt(7.0 / pi), c14 = 0.25 * sqrt(105.0 / pi);
    const double xx = x * x, yy = y * y, zz = z * z;
    memset(dY, 0, 16 * 3 * sizeof(double));
    Y[0] = a0;
    Y[1] = -a1 * y;  dY[1][1] = -a1;
    Y[2] = a1 * z;   dY[2][2] = a1;
    Y[3] = -a1 * x;  dY[3][0] = -a1;
    Y[4] = b * x * y;               dY[4][0] = b * y;  dY[4][1] = b * x;
    Y[5] = -b * y * z;              dY[5][1] = -b * z; dY[5][2] = -b * y;
    Y[6] = b6 * (2 * zz - xx - yy); dY[6][0] = -2 * b6 * x; dY[6][1] = -2 * b6 * y; dY[6][2] = 4 * b6 * z;
    Y[7] = -b * x * z;              dY[7][0] = -b * z; dY[7][2] = -b * x;
    Y[8] = b8 * (xx - yy);          dY[8][0] = 2 * b8 * x; dY[8][1] = -2 * b8 * y;
    Y[9] = -c9 * y * (3 * xx - yy);
    dY[9][0] = -6 * c9 * x * y; dY[9][1] = -c9 * (3 * xx - 3 * yy);
    Y[10] = c10 * x * y * z;
    dY[10][0] = c10 * y * z; dY[10][1] = c10 * x * z; dY[10][2] = c10 * x * y;
    Y[11] = -c11 * y * (4 * zz - xx - yy);
    dY[11][0] = 2 * c11 * x * y; dY[11][1] = -c11 * (4 * zz - xx - 3 * yy); dY[11][2] = -8 * c11 * y * z;
    Y[12] = c12 * z * (2 * zz - 3 * xx - 3 * yy);
    dY[12][0] = -6 * c12 * x * z; dY[12][1] = -6 * c12 * y * z; dY[12][2] = c12 * (6 * zz - 3 * xx - 3 * yy);
    Y[13] = -c11 * x * (4 * zz - xx - yy);
    dY[13][0] = -c11 * (4 * zz - 3 * xx - yy); dY[13][1] = 2 * c11 * x * y; dY[13][2] = -8 * c11 * x * z;
    Y[14] = c14 * z * (xx - yy);
    dY[14][0] = 2 * c14 * x * z; dY[14][1] = -2 * c14 * y * z; dY[14][2] = c14 * (xx - yy);
    Y[15] = -c9 * x * (xx - 3 * yy);
    dY[15][0] = -c9 * (3 * xx - 3 * yy); dY[15][1] = 6 * c9 * x * y;
}

/* The basis and its derivatives at ndir unit directions: Y[ndir][16], dY[ndir][16][3]. */
void oracle_sh_basis(int64_t ndir, const double *dirs, double *Y, double *dY) {
    for (int64_t i = 0; i < ndir; ++i) sh_basis(dirs + 3 * i, Y + 16 * i, (double (*)[3])(dY + 48 * i));
}

/* Lobes of Gaussian i: their count (-1 when the compressed-row offsets are malformed) and the
 * element index of lobe l in a one-row plane (sharp, lobe mask) or of row c of a three-row
 * plane (axis, amplitude). */
static int lobe_count(const oscene *sc, int64_t i) {
    if (!sc->lobe_off) return sc->k;
    int64_t a = sc->lobe_off[i], b = sc->lobe_off[i + 1];
    if (a < 0 || b < a || b > sc->n_lobes || b - a > sc->k) return -1;
    return (int)(b - a);
}
static int64_t lobe1(const oscene *sc, int64_t i, int l) {
    return sc->lobe_off ? sc->lobe_off[i] + l : (int64_t)l * sc->n + i;
}
static int64_t lobe3(const oscene *sc, int64_t i, int l, int c) {
    return sc->lobe_off ? (int64_t)c * sc->n_lobes + sc->lobe_off[i] + l : ((int64_t)l * 3 + c) * sc->n + i;
}

/*
 * Tile selection inside the rectangle, written as its plain definition. With the conic C = [[a, b], [b, c]]
 * and Q(p) = (p - m)' C (p - m), a tile of the rectangle is listed exactly when the ellipse {Q <= k} meets
 * the box spanned by the centres of the tile's pixels that lie inside the image, that is when the minimum of Q
 * over that box is <= k. The level k = 2.004 ln(255 o) + 1e-4 sits slightly above 2 ln(255 o), the level of
 * alpha = 1/255 (alpha = o exp(-Q / 2)), so that FP32 rounding in a renderer cannot reach a pixel of an
 * unlisted tile. A conic that is not positive definite bounds nothing: every tile of the rectangle is listed.
 */
static double cutoff_level(double o) { return 2.004 * log(255.0 * o) + 1e-4; }

static double clampd(double x, double lo, double hi) { return x < lo ? lo : (x > hi ? hi : x); }

static double quad_form(double a, double b, double c, double dx, double dy) {
    return a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
}

/* positive definite conic (a > 0 and a c - b^2 > 0; the products of FP32 inputs are exact in FP64) */
static int conic_pd(double a, double b, double c) { return a > 0.0 && a * c - b * b > 0.0; }

/*
 * min of Q over the box [x0, x1] x [y0, y1] for a positive definite conic. Q is strictly convex, so the
 * minimum is 0 at the mean when the mean lies in the box; otherwise it lies on the box's boundary. On each
 * edge Q restricted to the edge is a convex parabola in the free coordinate, minimal at its vertex (for
 * x fixed: dy = -b dx / c; for y fixed: dx = -b dy / a) clamped to the edge.
 */
static double box_min_q(double u, double v, double a, double b, double c, double x0, double x1, double y0,
                        double y1) {
    if (u >= x0 && u <= x1 && v >= y0 && v <= y1) return 0.0;
    const double xs[2] = {x0, x1}, ys[2] = {y0, y1};
    double best = INFINITY;
    for (int e = 0; e < 2; ++e) {
        double dx = xs[e] - u;
        double dy = clampd(-b * dx / c, y0 - v, y1 - v);
        double q = quad_form(a, b, c, dx, dy);
        if (q < best) best = q;
        dy = ys[e] - v;
        dx = clampd(-b * dy / a, x0 - u, x1 - u);
        q = quad_form(a, b, c, dx, dy);
        if (q < best) best = q;
    }
    return best;
}

/* box_min_q for m problems: mean (u, v), conic [m][3], box [m][4] = x0, x1, y0, y1 -> out [m] (for the pins) */
void oracle_box_min(int64_t m, const double *u, const double *v, const double *conic, const double *box,
                    double *out) {
    for (int64_t i = 0; i < m; ++i) {
        const double *cn = conic + 3 * i, *b = box + 4 * i;
        out[i] = conic_pd(cn[0], cn[1], cn[2]) ? box_min_q(u[i], v[i], cn[0], cn[1], cn[2], b[0], b[1], b[2], b[3])
                                               : -INFINITY;
    }
}

/* pixel-centre box of tile (tx, ty) of edge `tile` in a w x h image: [x0, x1] x [y0, y1] */
static void tile_box(int tx, int ty, int tile, int w, int h, double box[4]) {
    int xe = (tx + 1) * tile < w ? (tx + 1) * tile : w;
    int ye = (ty + 1) * tile < h ? (ty + 1) * tile : h;
    box[0] = tx * tile + 0.5; box[1] = xe - 0.5;
    box[2] = ty * tile + 0.5; box[3] = ye - 0.5;
}

/* min of Q over tile (tx, ty)'s pixel-centre box; -INFINITY when the conic is not positive definite
 * (every tile listed) */
static double tile_q(double u, double v, const double cn[3], int tx, int ty, int tile, int w, int h) {
    if (!conic_pd(cn[0], cn[1], cn[2])) return -INFINITY;
    double box[4];
    tile_box(tx, ty, tile, w, h, box);
    return box_min_q(u, v, cn[0], cn[1], cn[2], box[0], box[1], box[2], box[3]);
}

/* Project Gaussian i into camera cam (tile edge tile). */
static void project_one(const oscene *sc, const ocam *cam, int tile, int64_t i, oproj *p) {
    int64_t n = sc->n;
    int k = lobe_count(sc, i);
    memset(p, 0, sizeof(*p));
    p->valid = 1;
    if (k < 0) { p->valid = 0; return; }
    double mu[3] = {P(sc->pos, n, 0, i), P(sc->pos, n, 1, i), P(sc->pos, n, 2, i)};
    for (int j = 0; j < 3; ++j) p->s[j] = exp(P(sc->logscale, n, j, i));
    double q[4];
    double qq = 0;
    for (int j = 0; j < 4; ++j) { q[j] = P(sc->quat, n, j, i); qq += q[j] * q[j]; }
    p->qn = sqrt(qq);
    if (!(p->qn > 0) || !isfinite(p->qn)) { p->valid = 0; return; }
    for (int j = 0; j < 4; ++j) p->qh[j] = q[j] / p->qn;
    quat_to_rot(p->qh, p->Rq);
    p->o = sigmoid(sc->op_logit[i]);
    p->mp = sc->pmask_logit ? sigmoid(sc->pmask_logit[i]) : 1.0;
    p->o_eff = p->o * p->mp;

    /* camera space */
    for (int r = 0; r < 3; ++r)
        p->t[r] = cam->R[3 * r] * mu[0] + cam->R[3 * r + 1] * mu[1] + cam->R[3 * r + 2] * mu[2] + cam->t[r];
    if (!(p->t[2] > cam->znear)) { p->valid = 0; return; }
    if (p->o_eff < ALPHA_MIN) { p->valid = 0; return; }
    double tx = p->t[0], ty = p->t[1], tz = p->t[2];
    p->u = cam->fx * tx / tz + cam->cx;
    p->v = cam->fy * ty / tz + cam->cy;

    /* 3D covariance S3 = M M^T, M = R(q) diag(s) */
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) p->M[3 * r + c] = p->Rq[3 * r + c] * p->s[c];
    for (int r = 0; r < 3; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += p->M[3 * r + m] * p->M[3 * c + m];
            p->S3[3 * r + c] = acc;
        }

    /* Jacobian of the perspective map at the clamped direction */
    double limx = FOV_CLAMP * (0.5 * cam->width) / cam->fx;
    double limy = FOV_CLAMP * (0.5 * cam->height) / cam->fy;
    double rx = tx / tz, ry = ty / tz;
    p->xi = rx; p->eta = ry;
    if (rx < -limx) { p->xi = -limx; p->xclamp = 1; }
    if (rx > limx) { p->xi = limx; p->xclamp = 1; }
    if (ry < -limy) { p->eta = -limy; p->yclamp = 1; }
    if (ry > limy) { p->eta = limy; p->yclamp = 1; }
    p->J[0] = cam->fx / tz; p->J[1] = 0; p->J[2] = -cam->fx * p->xi / tz;
    p->J[3] = 0; p->J[4] = cam->fy / tz; p->J[5] = -cam->fy * p->eta / tz;
    /* T = J W, W the camera rotation */
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 3; ++c) {
            double acc = 0;
            for (int m = 0; m < 3; ++m) acc += p->J[3 * r + m] * cam->R[3 * m + c];
            p->T[3 * r + c] = acc;
        }
    /* S2 = T S3 T^T */
    double S2[4];
    for (int r = 0; r < 2; ++r)
        for (int c = 0; c < 2; ++c) {
            double acc = 0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) acc += p->T[3 * r + a] * p->S3[3 * a + b] * p->T[3 * c + b];
            S2[2 * r + c] = acc;
        }
    p->A0 = S2[0]; p->B0 = 0.5 * (S2[1] + S2[2]); p->C0 = S2[3];

    /* dilation and the guarded determinant */
    double A = p->A0 + DILATION, B = p->B0, C = p->C0 + DILATION;
    p->det0 = p->A0 * p->C0 - p->B0 * p->B0;
    p->det = (p->det0 > 0 ? p->det0 : 0.0) + DILATION * (p->A0 + p->C0) + DILATION * DILATION;
    p->conic[0] = C / p->det;
    p->conic[1] = -B / p->det;
    p->conic[2] = A / p->det;

    /* opacity-aware radius: every pixel with alpha >= 1/255 lies within rho of the mean */
    double mid = 0.5 * (A + C);
    double disc = mid * mid - p->det;
    p->lmax = mid + sqrt(disc > 0 ? disc : 0.0);
    p->rho = sqrt(2.0 * log(255.0 * p->o_eff) * p->lmax);
    double r = ceil(p->rho);
    if (!isfinite(p->u) || !isfinite(p->v) || !isfinite(r) || fabs(p->u) > MAX_COORD ||
        fabs(p->v) > MAX_COORD || r > MAX_COORD) { p->valid = 0; return; }
    p->radius = (int)r;

    /* colour: view direction from the camera centre to the Gaussian */
    for (int a = 0; a < 3; ++a)
        p->campos[a] = -(cam->R[a] * cam->t[0] + cam->R[3 + a] * cam->t[1] + cam->R[6 + a] * cam->t[2]);
    double dd = 0;
    for (int a = 0; a < 3; ++a) { p->dvec[a] = mu[a] - p->campos[a]; dd += p->dvec[a] * p->dvec[a]; }
    p->dlen = sqrt(dd);
    for (int a = 0; a < 3; ++a) p->d[a] = p->dvec[a] / p->dlen;
    if (sc->sh) {
        const int nm = (sc->sh_degree + 1) * (sc->sh_degree + 1);
        sh_basis(p->d, p->shY, p->shdY);
        for (int c = 0; c < 3; ++c) {
            double acc = 0.5;
            for (int m = 0; m < nm; ++m) acc += p->shY[m] * sc->sh[((int64_t)m * 3 + c) * n + i];
            p->shclamp[c] = acc < 0.0;
            p->rgb[c] = acc < 0.0 ? 0.0 : acc;
        }
        k = 0;
    } else {
        for (int c = 0; c < 3; ++c) p->rgb[c] = P(sc->base, n, c, i);
    }
    for (int l = 0; l < k; ++l) {
        double ax[3], al = 0;
        for (int a = 0; a < 3; ++a) { ax[a] = sc->axis[lobe3(sc, i, l, a)]; al += ax[a] * ax[a]; }
        al = sqrt(al);
        if (!(al > 0) || !isfinite(al)) { p->valid = 0; return; }
        p->ax_len[l] = al;
        double dot = 0;
        for (int a = 0; a < 3; ++a) { p->muh[l][a] = ax[a] / al; dot += p->muh[l][a] * p->d[a]; }
        p->dot[l] = dot;
        double lam = sc->sharp[lobe1(sc, i, l)];
        p->mk[l] = sc->lmask_logit ? sigmoid(sc->lmask_logit[lobe1(sc, i, l)]) : 1.0;
        p->ek[l] = exp(lam * (dot - 1.0));
        for (int c = 0; c < 3; ++c)
            p->rgb[c] += p->mk[l] * sc->amp[lobe3(sc, i, l, c)] * p->ek[l];
    }
    for (int c = 0; c < 3; ++c)
        if (!isfinite(p->rgb[c])) { p->valid = 0; return; }

    /* the ellipse level bounding alpha >= 1/255 depends on the opacity only */
    p->cutoff = cutoff_level(p->o_eff);

    /* tile rectangle from pixel bounds floor(u) -/+ r, clipped to the image */
    int tiles_x = (cam->width + tile - 1) / tile, tiles_y = (cam->height + tile - 1) / tile;
    double x_lo = floor(p->u) - r, x_hi = floor(p->u) + r;
    double y_lo = floor(p->v) - r, y_hi = floor(p->v) + r;
    if (x_hi < 0 || y_hi < 0 || x_lo > cam->width - 1 || y_lo > cam->height - 1) { p->ntiles = 0; return; }
    if (x_lo < 0) x_lo = 0;
    if (y_lo < 0) y_lo = 0;
    if (x_hi > cam->width - 1) x_hi = cam->width - 1;
    if (y_hi > cam->height - 1) y_hi = cam->height - 1;
    p->rect[0] = (int)x_lo / tile; p->rect[1] = (int)x_hi / tile;
    p->rect[2] = (int)y_lo / tile; p->rect[3] = (int)y_hi / tile;
    (void)tiles_x; (void)tiles_y;
    p->ntiles = 0;
    for (int ty = p->rect[2]; ty <= p->rect[3]; ++ty)
        for (int tx = p->rect[0]; tx <= p->rect[1]; ++tx)
            if (tile_q(p->u, p->v, p->conic, tx, ty, tile, cam->width, cam->height) <= p->cutoff) ++p->ntiles;
}

/*
 * Records of all Gaussians in one view.
 * out_f: [n][11] = u, v, depth, conic a, b, c, o_eff, r, g, b, cutoff level
 * out_i: [n][7]  = valid, radius, tile x0, x1, y0, y1, ntiles (tiles of the rectangle reached)
 */
void oracle_project(const oscene *sc, const ocam *cam, int32_t tile, double *out_f, int32_t *out_i) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < sc->n; ++i) {
        oproj p;
        project_one(sc, cam, tile, i, &p);
        double *f = out_f + 11 * i;
        int32_t *g = out_i + 7 * i;
        f[0] = p.u; f[1] = p.v; f[2] = p.t[2];
        f[3] = p.conic[0]; f[4] = p.conic[1]; f[5] = p.conic[2];
        f[6] = p.o_eff; f[7] = p.rgb[0]; f[8] = p.rgb[1]; f[9] = p.rgb[2]; f[10] = p.cutoff;
        g[0] = p.valid; g[1] = p.radius;
        g[2] = p.rect[0]; g[3] = p.rect[1]; g[4] = p.rect[2]; g[5] = p.rect[3];
        g[6] = p.valid ? p.ntiles : 0;
    }
}

/* SG colour for one direction (for closed-form tests): rgb = base + sum m_k a_k e^{lam_k (mu_k.d - 1)} */
void oracle_sg_color(int32_t k, const double *base, const double *axis, const double *sharp,
                     const double *amp, const double *mask, const double *dir, double *rgb) {
    for (int c = 0; c < 3; ++c) rgb[c] = base[c];
    for (int l = 0; l < k; ++l) {
        double al = sqrt(axis[3 * l] * axis[3 * l] + axis[3 * l + 1] * axis[3 * l + 1] + axis[3 * l + 2] * axis[3 * l + 2]);
        double dot = (axis[3 * l] * dir[0] + axis[3 * l + 1] * dir[1] + axis[3 * l + 2] * dir[2]) / al;
        double e = exp(sharp[l] * (dot - 1.0));
        double m = mask ? mask[l] : 1.0;
        for (int c = 0; c < 3; ++c) rgb[c] += m * amp[3 * l + c] * e;
    }
}

/* the same for ndir directions dirs[ndir][3] -> rgb[ndir][3] */
void oracle_sg_color_many(int32_t k, const double *base, const double *axis, const double *sharp,
                          const double *amp, const double *mask, int64_t ndir, const double *dirs, double *rgb) {
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < ndir; ++i) oracle_sg_color(k, base, axis, sharp, amp, mask, dirs + 3 * i, rgb + 3 * i);
}

/* ---------------------------------------------------------------- keys ---- */

/*
 * Tile rectangle of one record, with the same integer arithmetic as project_one
 * (floor(u) -/+ r, clipped to the image). Returns the tile count.
 */
static int rect_of(double u, double v, int32_t r, int w, int h, int tile, int rect[4]) {
    double x_lo = floor(u) - r, x_hi = floor(u) + r;
    double y_lo = floor(v) - r, y_hi = floor(v) + r;
    if (x_hi < 0 || y_hi < 0 || x_lo > w - 1 || y_lo > h - 1) return 0;
    if (x_lo < 0) x_lo = 0;
    if (y_lo < 0) y_lo = 0;
    if (x_hi > w - 1) x_hi = w - 1;
    if (y_hi > h - 1) y_hi = h - 1;
    rect[0] = (int)x_lo / tile; rect[1] = (int)x_hi / tile;
    rect[2] = (int)y_lo / tile; rect[3] = (int)y_hi / tile;
    return (rect[1] - rect[0] + 1) * (rect[3] - rect[2] + 1);
}

/*
 * Candidate pairs of the key table over records of several views. Record g belongs to view rec_view[g];
 * view v has image size (w[v], h[v]) and its tiles are numbered from tile_off[v]. For every valid record
 * and every tile of its rectangle, q = the minimum of Q over the tile's pixel-centre box is compared with
 * the record's level k (cutoff[g]):
 *   state 1: listed, q <= k, and q is not within the band;
 *   state 2: |q - k| <= band * k: the decision lies within a relative band of the level, where a
 *            renderer evaluating the same definition in another rounding order may take either side.
 * Tiles with q > k outside the band are not returned. With band = 0 no pair has state 2.
 * When out_tile == NULL only the number of returned pairs is computed. out_tile: global tile id,
 * out_rec: record index, out_state: 1 or 2, in record order and row-major tile order per record.
 */
static int64_t record_candidates(int64_t g, const double *u, const double *v, const int32_t *radius,
                                 const double *conic, const double *cutoff, const int32_t *rec_view,
                                 const int32_t *w, const int32_t *h, const int64_t *tile_off, int tile, double band,
                                 int64_t *out_tile, uint32_t *out_rec, uint8_t *out_state) {
    int vv = rec_view[g];
    int rect[4];
    if (!rect_of(u[g], v[g], radius[g], w[vv], h[vv], tile, rect)) return 0;
    int tiles_x = (w[vv] + tile - 1) / tile;
    double k = cutoff[g];
    int64_t m = 0;
    for (int ty = rect[2]; ty <= rect[3]; ++ty)
        for (int tx = rect[0]; tx <= rect[1]; ++tx) {
            double q = tile_q(u[g], v[g], conic + 3 * g, tx, ty, tile, w[vv], h[vv]);
            int state = (band > 0.0 && fabs(q - k) <= band * k) ? 2 : (q <= k ? 1 : 0);
            if (!state) continue;
            if (out_tile) {
                out_tile[m] = tile_off[vv] + (int64_t)ty * tiles_x + tx;
                out_rec[m] = (uint32_t)g;
                out_state[m] = (uint8_t)state;
            }
            ++m;
        }
    return m;
}

int64_t oracle_tile_candidates(int64_t nrec, const double *u, const double *v, const int32_t *radius,
                               const double *conic, const double *cutoff, const int32_t *valid,
                               const int32_t *rec_view, const int32_t *w, const int32_t *h, const int64_t *tile_off,
                               int32_t tile, double band, int64_t *out_tile, uint32_t *out_rec, uint8_t *out_state) {
    int64_t *cnt = (int64_t *)calloc((size_t)(nrec > 0 ? nrec : 1) + 1, sizeof(int64_t));
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t g = 0; g < nrec; ++g)
        if (valid[g])
            cnt[g + 1] = record_candidates(g, u, v, radius, conic, cutoff, rec_view, w, h, tile_off, tile, band,
                                           NULL, NULL, NULL);
    for (int64_t g = 0; g < nrec; ++g) cnt[g + 1] += cnt[g];
    int64_t total = cnt[nrec];
    if (out_tile) {
        #pragma omp parallel for schedule(dynamic, 1024)
        for (int64_t g = 0; g < nrec; ++g)
            if (valid[g] && cnt[g + 1] > cnt[g])
                record_candidates(g, u, v, radius, conic, cutoff, rec_view, w, h, tile_off, tile, band,
                                  out_tile + cnt[g], out_rec + cnt[g], out_state + cnt[g]);
    }
    free(cnt);
    return total;
}

typedef struct { uint64_t key; uint32_t val; } okv;

static int cmp_kv(const void *a, const void *b) {
    const okv *x = (const okv *)a, *y = (const okv *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->val != y->val) return x->val < y->val ? -1 : 1;
    return 0;
}

/*
 * Orders (key, value) pairs by key, then value, in place, and writes the [start, end) of every tile
 * (key >> 32) into ranges[2 * total_tiles] ((0, 0) when the tile has no pair).
 */
void oracle_sort_pairs(int64_t count, uint64_t *keys, uint32_t *vals, int64_t total_tiles, uint32_t *ranges) {
    okv *kv = (okv *)malloc(sizeof(okv) * (size_t)(count > 0 ? count : 1));
    for (int64_t i = 0; i < count; ++i) { kv[i].key = keys[i]; kv[i].val = vals[i]; }
    qsort(kv, (size_t)count, sizeof(okv), cmp_kv);
    for (int64_t t = 0; t < 2 * total_tiles; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < count; ++i) {
        keys[i] = kv[i].key;
        vals[i] = kv[i].val;
        uint64_t t = kv[i].key >> 32;
        if (i == 0 || (kv[i - 1].key >> 32) != t) ranges[2 * t] = (uint32_t)i;
        if (i == count - 1 || (kv[i + 1].key >> 32) != t) ranges[2 * t + 1] = (uint32_t)(i + 1);
    }
    free(kv);
}

static uint32_t f32_bits(float f) { uint32_t b; memcpy(&b, &f, 4); return b; }

/*
 * The key table: key = global tile << 32 | bits(float32 depth), value = record index, for every listed
 * (tile, record) pair (the plain definition above, no band), ordered by (key, value), with per-tile
 * [start, end) ranges. When keys == NULL only the pair count is returned.
 */
int64_t oracle_pairs(int64_t nrec, const double *u, const double *v, const float *depth, const int32_t *radius,
                     const double *conic, const double *cutoff,
                     const int32_t *valid, const int32_t *rec_view, const int32_t *w, const int32_t *h,
                     const int64_t *tile_off, int32_t tile, int64_t total_tiles,
                     uint64_t *keys, uint32_t *vals, uint32_t *ranges) {
    int64_t count = oracle_tile_candidates(nrec, u, v, radius, conic, cutoff, valid, rec_view, w, h, tile_off, tile,
                                           0.0, NULL, NULL, NULL);
    if (!keys) return count;
    int64_t *tl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(count > 0 ? count : 1));
    uint8_t *st = (uint8_t *)malloc((size_t)(count > 0 ? count : 1));
    oracle_tile_candidates(nrec, u, v, radius, conic, cutoff, valid, rec_view, w, h, tile_off, tile, 0.0, tl, vals,
                           st);
    for (int64_t i = 0; i < count; ++i) keys[i] = ((uint64_t)tl[i] << 32) | f32_bits(depth[vals[i]]);
    free(tl);
    free(st);
    oracle_sort_pairs(count, keys, vals, total_tiles, ranges);
    return count;
}

/*
 * Sub-tile reach of listed pairs: for pair i (global tile tiles[i], record recs[i]), the 8 x 8 sub-tiles
 * of the tile (S = tile / 8 per edge; bit r S + c for sub-row r, sub-column c) whose pixel-centre boxes
 * inside the image the ellipse {Q <= k} meets. set[i]: sub-tiles with q <= k outside the relative band;
 * near[i]: sub-tiles with |q - k| <= band k. Sub-tiles with no pixel inside the image are in neither.
 * A conic that is not positive definite reaches every sub-tile with pixels.
 */
void oracle_subtile_flags(int64_t npairs, const int64_t *tiles, const uint32_t *recs, const double *u,
                          const double *v, const double *conic, const double *cutoff, const int32_t *rec_view,
                          int32_t nviews, const int32_t *w, const int32_t *h, const int64_t *tile_off, int32_t tile,
                          double band, uint32_t *set, uint32_t *near) {
    const int S = tile / 8;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < npairs; ++i) {
        uint32_t g = recs[i];
        int vv = rec_view[g];
        (void)nviews;
        int tiles_x = (w[vv] + tile - 1) / tile;
        int64_t lt = tiles[i] - tile_off[vv];
        int tx = (int)(lt % tiles_x), ty = (int)(lt / tiles_x);
        double k = cutoff[g];
        uint32_t s = 0, nb = 0;
        for (int r = 0; r < S; ++r)
            for (int c = 0; c < S; ++c) {
                int sx = tx * S + c, sy = ty * S + r;
                if (sx * 8 >= w[vv] || sy * 8 >= h[vv]) continue;
                double q = tile_q(u[g], v[g], conic + 3 * (int64_t)g, sx, sy, 8, w[vv], h[vv]);
                if (band > 0.0 && fabs(q - k) <= band * k) nb |= 1u << (r * S + c);
                else if (q <= k) s |= 1u << (r * S + c);
            }
        set[i] = s;
        near[i] = nb;
    }
}

/* --------------------------------------------------------------- blend ---- */

/* per-record data the compositor reads (FP64 copies of whatever records it is given) */
typedef struct {
    const double *u, *v, *conic, *o, *rgb; /* conic [n][3], rgb [n][3] */
} orecs;

static int near_rel(double x, double thr) { return fabs(x - thr) <= NEAR_BAND * thr; }

/* One fragment's alpha. Returns 0 when skipped (q > 0 or alpha < 1/255). */
static int frag_alpha(const orecs *rc, int64_t g, double px, double py, double *alpha, double *G,
                      int *clamped, double *dx, double *dy, int *flag) {
    *dx = px - rc->u[g];
    *dy = py - rc->v[g];
    const double *cn = rc->conic + 3 * g;
    double q = -0.5 * (cn[0] * (*dx) * (*dx) + cn[2] * (*dy) * (*dy)) - cn[1] * (*dx) * (*dy);
    if (q > 0) return 0;
    *G = exp(q);
    double a = rc->o[g] * (*G);
    *flag |= near_rel(a, ALPHA_MAX);
    *clamped = a > ALPHA_MAX;
    if (*clamped) a = ALPHA_MAX;
    *flag |= near_rel(a, ALPHA_MIN);
    *alpha = a;
    return a >= ALPHA_MIN;
}

/*
 * Composite one pixel over an ordered list of record indices (front to back).
 * Returns the number of list entries evaluated. Writes colour (with background),
 * final transmittance, last (1 + list position of the last included fragment)
 * and flag (1 when any decision lies within the threshold bands).
 */
static int64_t composite(const orecs *rc, const uint32_t *list, int64_t len, double px, double py,
                         const double bg[3], double out[3], double *T_out, int32_t *last_out, int *flag_out,
                         uint64_t *sig_out, double *weight_slots) {
    double T = 1.0, C[3] = {0, 0, 0};
    int32_t last = 0;
    int flag = 0;
    int64_t evaluated = 0;
    uint64_t sig = 0; /* decision signature: unsigned arithmetic, wrapping by definition */
    for (int64_t pos = 0; pos < len; ++pos) {
        ++evaluated;
        uint32_t g = list[pos];
        double alpha, G, dx, dy;
        int clamped;
        if (!frag_alpha(rc, g, px, py, &alpha, &G, &clamped, &dx, &dy, &flag)) continue;
        double Tn = T * (1.0 - alpha);
        flag |= near_rel(Tn, T_MIN);
        if (Tn < T_MIN) break;
        for (int c = 0; c < 3; ++c) C[c] += alpha * T * rc->rgb[3 * g + c];
        if (weight_slots) weight_slots[pos] += alpha * T;
        T = Tn;
        last = (int32_t)(pos + 1);
        sig = sig * 1000003u + (uint64_t)g * 2u + (uint64_t)clamped;
    }
    for (int c = 0; c < 3; ++c) out[c] = C[c] + T * bg[c];
    *T_out = T;
    *last_out = last;
    *flag_out = flag;
    if (sig_out) *sig_out = sig;
    return evaluated;
}

/*
 * Tiled forward blend of one view. vals/ranges are the view's slice of the sorted
 * key table (ranges indexed by the view-local tile, positions into vals).
 * image [3][h][w], T [h][w], last [h][w], flag [h][w], sig [h][w] (decision signature).
 * importance (nullable, [nrec]): adds each record's blending weights alpha * T summed over the
 * pixels -- the importance score of the Appendix's proximal-operator description -- through
 * per-pair slots summed in list order. npairs: length of vals (needed with importance).
 * Returns the number of (pixel, list entry) evaluations.
 */
int64_t oracle_blend(int32_t w, int32_t h, int32_t tile, const double *bg,
                     const double *u, const double *v, const double *conic, const double *o, const double *rgb,
                     const uint32_t *vals, const uint32_t *ranges,
                     double *image, double *T, int32_t *last, int32_t *flag, uint64_t *sig,
                     int64_t npairs, double *importance) {
    orecs rc = {u, v, conic, o, rgb};
    int tiles_x = (w + tile - 1) / tile, tiles_y = (h + tile - 1) / tile;
    int64_t total = 0;
    double *wslots = importance ? (double *)calloc((size_t)(npairs > 0 ? npairs : 1), sizeof(double)) : NULL;
    #pragma omp parallel for schedule(dynamic) reduction(+ : total)
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
        int tx = t % tiles_x, ty = t / tiles_x;
        uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
        for (int y = ty * tile; y < (ty + 1) * tile && y < h; ++y)
            for (int x = tx * tile; x < (tx + 1) * tile && x < w; ++x) {
                double out[3];
                int fl;
                int64_t p = (int64_t)y * w + x;
                total += composite(&rc, vals + s, (int64_t)e - s, x + 0.5, y + 0.5, bg, out, &T[p], &last[p], &fl,
                                   sig ? &sig[p] : NULL, wslots ? wslots + s : NULL);
                flag[p] = fl;
                for (int c = 0; c < 3; ++c) image[(int64_t)c * w * h + p] = out[c];
            }
    }
    if (wslots) {
        for (int64_t i = 0; i < npairs; ++i) importance[vals[i]] += wslots[i];
        free(wslots);
    }
    return total;
}

typedef struct { float d; uint32_t id; } odepth;
static int cmp_depth(const void *a, const void *b) {
    const odepth *x = (const odepth *)a, *y = (const odepth *)b;
    if (x->d != y->d) return x->d < y->d ? -1 : 1;
    return x->id < y->id ? -1 : (x->id > y->id);
}

/*
 * Brute force: every pixel composites all records of the view whose valid flag is set,
 * ordered by (float32 depth, index) -- no tiles, no rectangles.
 */
void oracle_bruteforce(int32_t w, int32_t h, const double *bg, int64_t nrec, const int32_t *valid,
                       const double *depth, const double *u, const double *v, const double *conic,
                       const double *o, const double *rgb, double *image, double *T, int32_t *last, int32_t *flag) {
    orecs rc = {u, v, conic, o, rgb};
    odepth *order = (odepth *)malloc(sizeof(odepth) * (size_t)(nrec > 0 ? nrec : 1));
    int64_t m = 0;
    for (int64_t g = 0; g < nrec; ++g)
        if (valid[g]) { order[m].d = (float)depth[g]; order[m].id = (uint32_t)g; ++m; }
    qsort(order, (size_t)m, sizeof(odepth), cmp_depth);
    uint32_t *list = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(m > 0 ? m : 1));
    for (int64_t i = 0; i < m; ++i) list[i] = order[i].id;
    #pragma omp parallel for schedule(dynamic)
    for (int y = 0; y < h; ++y)
        for (int x = 0; x < w; ++x) {
            double out[3];
            int fl;
            int32_t lst;
            int64_t p = (int64_t)y * w + x;
            composite(&rc, list, m, x + 0.5, y + 0.5, bg, out, &T[p], &lst, &fl, NULL, NULL);
            last[p] = lst;
            flag[p] = fl;
            for (int c = 0; c < 3; ++c) image[(int64_t)c * w * h + p] = out[c];
        }
    free(list);
    free(order);
}

/* ------------------------------------------------------- blend backward ---- */

/*
 * Gradient of L with respect to each record's 2D quantities for one view:
 * grad2d[g][9] = dL/d(u, v, conic a, b, c, o_eff, r, g, b), given dL/dimage
 * (dl [3][h][w]). Each pixel re-runs its own front-to-back pass (keeping the exact
 * transmittance in front of every included fragment), then walks the included
 * fragments back to front. direct != 0 evaluates dL/dalpha by the O(n^2) sum over
 * the fragments behind instead of the running background recursion.
 * Contributions go to per-pair slots (one per list position), summed per record
 * in list order afterwards, so the result does not depend on the thread count.
 * grad2d must hold nrec * 9 zeros on entry; contributions are added. grad2d_abs (nullable) receives
 * the sum of the absolute values of the same contributions (the scale against which the rounding
 * error of any summation order is measured).
 */
void oracle_blend_backward(int32_t w, int32_t h, int32_t tile, const double *bg,
                           const double *u, const double *v, const double *conic, const double *o, const double *rgb,
                           const uint32_t *vals, const uint32_t *ranges, int64_t npairs, const double *dl,
                           int32_t direct, double *grad2d, double *grad2d_abs) {
    orecs rc = {u, v, conic, o, rgb};
    int tiles_x = (w + tile - 1) / tile, tiles_y = (h + tile - 1) / tile;
    double *slots = (double *)calloc((size_t)(npairs > 0 ? npairs : 1) * 9, sizeof(double));
    double *aslots = (double *)calloc((size_t)(npairs > 0 ? npairs : 1) * 9, sizeof(double));
    #pragma omp parallel for schedule(dynamic)
    for (int t = 0; t < tiles_x * tiles_y; ++t) {
        int tx = t % tiles_x, ty = t / tiles_x;
        uint32_t s = ranges[2 * t], e = ranges[2 * t + 1];
        int64_t len = (int64_t)e - s;
        if (len <= 0) continue;
        int64_t *fpos = (int64_t *)malloc(sizeof(int64_t) * len);
        double *fa = (double *)malloc(sizeof(double) * len * 6); /* alpha, G, T_front, dx, dy, clamped */
        for (int y = ty * tile; y < (ty + 1) * tile && y < h; ++y)
            for (int x = tx * tile; x < (tx + 1) * tile && x < w; ++x) {
                int64_t p = (int64_t)y * w + x;
                double gp[3] = {dl[p], dl[(int64_t)w * h + p], dl[2 * (int64_t)w * h + p]};
                /* forward pass, remembering the included fragments */
                double T = 1.0;
                int64_t nf = 0;
                int flag = 0;
                for (int64_t pos = 0; pos < len; ++pos) {
                    uint32_t g = vals[s + pos];
                    double alpha, G, dx, dy;
                    int clamped;
                    if (!frag_alpha(&rc, g, x + 0.5, y + 0.5, &alpha, &G, &clamped, &dx, &dy, &flag)) continue;
                    double Tn = T * (1.0 - alpha);
                    if (Tn < T_MIN) break;
                    fpos[nf] = pos;
                    double *f = fa + 6 * nf;
                    f[0] = alpha; f[1] = G; f[2] = T; f[3] = dx; f[4] = dy; f[5] = clamped;
                    ++nf;
                    T = Tn;
                }
                double T_final = T;
                /* background seen behind each fragment, back to front */
                double Bk[3] = {bg[0], bg[1], bg[2]};
                for (int64_t j = nf - 1; j >= 0; --j) {
                    double *f = fa + 6 * j;
                    uint32_t g = vals[s + fpos[j]];
                    double alpha = f[0], G = f[1], Ti = f[2], dx = f[3], dy = f[4];
                    const double *c = rc.rgb + 3 * g;
                    double *slot = slots + 9 * (s + fpos[j]);
                    double *aslot = aslots + 9 * (s + fpos[j]);
                    for (int ch = 0; ch < 3; ++ch) {
                        slot[6 + ch] += alpha * Ti * gp[ch];
                        aslot[6 + ch] += fabs(alpha * Ti * gp[ch]);
                    }
                    double dalpha = 0;
                    if (!direct) {
                        for (int ch = 0; ch < 3; ++ch) dalpha += Ti * (c[ch] - Bk[ch]) * gp[ch];
                        for (int ch = 0; ch < 3; ++ch) Bk[ch] = alpha * c[ch] + (1.0 - alpha) * Bk[ch];
                    } else {
                        /* C = sum_i c_i a_i T_i + T_final bg; differentiate term by term */
                        double acc = 0;
                        for (int ch = 0; ch < 3; ++ch) acc += c[ch] * Ti * gp[ch];
                        for (int64_t m = j + 1; m < nf; ++m) {
                            const double *fm = fa + 6 * m;
                            const double *cm = rc.rgb + 3 * vals[s + fpos[m]];
                            for (int ch = 0; ch < 3; ++ch) acc -= cm[ch] * fm[0] * fm[2] / (1.0 - alpha) * gp[ch];
                        }
                        for (int ch = 0; ch < 3; ++ch) acc -= bg[ch] * T_final / (1.0 - alpha) * gp[ch];
                        dalpha = acc;
                    }
                    if (f[5] != 0) continue; /* alpha clamped at 0.99: no dependence on o_eff or q */
                    const double *cn = rc.conic + 3 * g;
                    double dq = dalpha * alpha;
                    double t9[6] = {dq * (cn[0] * dx + cn[1] * dy), dq * (cn[1] * dx + cn[2] * dy),
                                    dq * (-0.5 * dx * dx), dq * (-dx * dy), dq * (-0.5 * dy * dy), dalpha * G};
                    for (int c = 0; c < 6; ++c) {
                        slot[c] += t9[c];
                        aslot[c] += fabs(t9[c]);
                    }
                }
            }
        free(fpos);
        free(fa);
    }
    for (int64_t i = 0; i < npairs; ++i) {
        uint32_t g = vals[i];
        for (int c = 0; c < 9; ++c) grad2d[9 * (int64_t)g + c] += slots[9 * i + c];
        if (grad2d_abs)
            for (int c = 0; c < 9; ++c) grad2d_abs[9 * (int64_t)g + c] += aslots[9 * i + c];
    }
    free(slots);
    free(aslots);
}

/* -------------------------------------------------- projection backward ---- */

/*
 * Chain rule from one view's per-record 2D gradients grad2d[n][9] to the raw
 * parameters. Gradients are ADDED into the output planes (same shapes as the
 * scene planes; the mask planes may be NULL when the scene has no masks), so
 * calling once per view sums over views.
 */
typedef struct {
    double *pos, *logscale, *quat, *op_logit, *pmask_logit, *base, *axis, *sharp, *amp, *lmask_logit;
    double *sh;
} ograd;

void oracle_project_backward(const oscene *sc, const ocam *cam, int32_t tile, const double *grad2d, ograd *gr) {
    int64_t n = sc->n;
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; ++i) {
        oproj p;
        project_one(sc, cam, tile, i, &p);
        if (!p.valid) continue;
        const double *d2 = grad2d + 9 * i;
        double du = d2[0], dv = d2[1], da = d2[2], db = d2[3], dc = d2[4], dop = d2[5];
        const double *drgb = d2 + 6;

        /* colour */
        double gd[3] = {0, 0, 0};
        if (sc->sh) {
            const int nm = (sc->sh_degree + 1) * (sc->sh_degree + 1);
            for (int c = 0; c < 3; ++c) {
                if (p.shclamp[c]) continue;
                for (int m = 0; m < nm; ++m) {
                    gr->sh[((int64_t)m * 3 + c) * n + i] += p.shY[m] * drgb[c];
                    for (int a = 0; a < 3; ++a)
                        gd[a] += sc->sh[((int64_t)m * 3 + c) * n + i] * drgb[c] * p.shdY[m][a];
                }
            }
        } else {
            for (int c = 0; c < 3; ++c) gr->base[c * n + i] += drgb[c];
        }
        const int k = sc->sh ? 0 : lobe_count(sc, i);
        for (int l = 0; l < k; ++l) {
            double lam = sc->sharp[lobe1(sc, i, l)];
            double ip = 0;
            for (int c = 0; c < 3; ++c) ip += sc->amp[lobe3(sc, i, l, c)] * drgb[c];
            double wgt = p.mk[l] * p.ek[l];
            for (int c = 0; c < 3; ++c) gr->amp[lobe3(sc, i, l, c)] += wgt * drgb[c];
            gr->sharp[lobe1(sc, i, l)] += wgt * (p.dot[l] - 1.0) * ip;
            double gmu[3], md = 0;
            for (int a = 0; a < 3; ++a) { gmu[a] = wgt * lam * ip * p.d[a]; md += p.muh[l][a] * gmu[a]; }
            for (int a = 0; a < 3; ++a)
                gr->axis[lobe3(sc, i, l, a)] += (gmu[a] - p.muh[l][a] * md) / p.ax_len[l];
            for (int a = 0; a < 3; ++a) gd[a] += wgt * lam * ip * p.muh[l][a];
            if (gr->lmask_logit) gr->lmask_logit[lobe1(sc, i, l)] += p.mk[l] * (1.0 - p.mk[l]) * p.ek[l] * ip;
        }
        double gpos[3];
        {
            double dd = p.d[0] * gd[0] + p.d[1] * gd[1] + p.d[2] * gd[2];
            for (int a = 0; a < 3; ++a) gpos[a] = (gd[a] - p.d[a] * dd) / p.dlen;
        }

        /* opacity and primitive mask */
        gr->op_logit[i] += dop * p.mp * p.o * (1.0 - p.o);
        if (gr->pmask_logit) gr->pmask_logit[i] += dop * p.o * p.mp * (1.0 - p.mp);

        /* conic (a, b, c) = (C, -B, A) / det with A = A0 + h, C = C0 + h, B = B0 */
        double A = p.A0 + DILATION, B = p.B0, C = p.C0 + DILATION, det = p.det;
        double gdet = -(da * C - db * B + dc * A) / (det * det);
        double gA0 = dc / det, gC0 = da / det, gB0 = -db / det;
        if (p.det0 > 0) {
            gA0 += gdet * (p.C0 + DILATION);
            gC0 += gdet * (p.A0 + DILATION);
            gB0 += gdet * (-2.0 * p.B0);
        } else {
            gA0 += gdet * DILATION;
            gC0 += gdet * DILATION;
        }
        /* S2 = T S3 T^T with a symmetric gradient matrix G2 */
        double G2[4] = {gA0, 0.5 * gB0, 0.5 * gB0, gC0};
        double gS3[9], gT[6];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b) acc += p.T[3 * a + r] * G2[2 * a + b] * p.T[3 * b + c];
                gS3[3 * r + c] = acc;
            }
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 3; ++b) acc += G2[2 * r + a] * p.T[3 * a + b] * p.S3[3 * b + c];
                gT[3 * r + c] = 2.0 * acc;
            }
        /* T = J W */
        double gJ[6];
        for (int r = 0; r < 2; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += gT[3 * r + m] * cam->R[3 * c + m];
                gJ[3 * r + c] = acc;
            }
        double tx = p.t[0], ty = p.t[1], tz = p.t[2];
        double fx = cam->fx, fy = cam->fy;
        double gt[3] = {0, 0, 0};
        double dxi_dtx = p.xclamp ? 0.0 : 1.0 / tz, dxi_dtz = p.xclamp ? 0.0 : -tx / (tz * tz);
        double deta_dty = p.yclamp ? 0.0 : 1.0 / tz, deta_dtz = p.yclamp ? 0.0 : -ty / (tz * tz);
        /* J00 = fx/tz, J02 = -fx xi/tz, J11 = fy/tz, J12 = -fy eta/tz */
        gt[2] += gJ[0] * (-fx / (tz * tz));
        gt[2] += gJ[4] * (-fy / (tz * tz));
        gt[0] += gJ[2] * (-fx / tz) * dxi_dtx;
        gt[2] += gJ[2] * (fx * p.xi / (tz * tz) - fx / tz * dxi_dtz);
        gt[1] += gJ[5] * (-fy / tz) * deta_dty;
        gt[2] += gJ[5] * (fy * p.eta / (tz * tz) - fy / tz * deta_dtz);
        /* mean: u = fx tx/tz + cx, v = fy ty/tz + cy */
        gt[0] += du * fx / tz;
        gt[1] += dv * fy / tz;
        gt[2] += -du * fx * tx / (tz * tz) - dv * fy * ty / (tz * tz);
        /* t = W mu + t_c */
        for (int a = 0; a < 3; ++a)
            gpos[a] += cam->R[a] * gt[0] + cam->R[3 + a] * gt[1] + cam->R[6 + a] * gt[2];
        for (int a = 0; a < 3; ++a) gr->pos[a * n + i] += gpos[a];

        /* S3 = M M^T, M = R(q) diag(s) */
        double gM[9];
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                double acc = 0;
                for (int m = 0; m < 3; ++m) acc += (gS3[3 * r + m] + gS3[3 * m + r]) * p.M[3 * m + c];
                gM[3 * r + c] = acc;
            }
        double gR[9], gs[3] = {0, 0, 0};
        for (int r = 0; r < 3; ++r)
            for (int c = 0; c < 3; ++c) {
                gR[3 * r + c] = gM[3 * r + c] * p.s[c];
                gs[c] += gM[3 * r + c] * p.Rq[3 * r + c];
            }
        for (int c = 0; c < 3; ++c) gr->logscale[c * n + i] += gs[c] * p.s[c];
        /* derivative of the textbook rotation matrix with respect to (w, x, y, z) */
        double w = p.qh[0], x = p.qh[1], y = p.qh[2], z = p.qh[3];
        double gq[4];
        gq[0] = 2 * (-z * gR[1] + y * gR[2] + z * gR[3] - x * gR[5] - y * gR[6] + x * gR[7]);
        gq[1] = 2 * (y * gR[1] + z * gR[2] + y * gR[3] - 2 * x * gR[4] - w * gR[5] + z * gR[6] + w * gR[7] - 2 * x * gR[8]);
        gq[2] = 2 * (-2 * y * gR[0] + x * gR[1] + w * gR[2] + x * gR[3] + z * gR[5] - w * gR[6] + z * gR[7] - 2 * y * gR[8]);
        gq[3] = 2 * (-2 * z * gR[0] - w * gR[1] + x * gR[2] + w * gR[3] - 2 * z * gR[4] + y * gR[5] + x * gR[6] + y * gR[7]);
        double qd = 0;
        for (int a = 0; a < 4; ++a) qd += p.qh[a] * gq[a];
        for (int a = 0; a < 4; ++a) gr->quat[a * n + i] += (gq[a] - p.qh[a] * qd) / p.qn;
    }
}
