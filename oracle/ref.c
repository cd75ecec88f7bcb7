/*
 * CPU oracle for the Speedy-Splat forward rasterizer.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is a plain, slow, single-threaded
 * restatement of the method, used to check the GPU library.  Only the test
 * suite, the smoke check and the benchmark's CPU-baseline leg may load it.
 * It shares no code, header or constant with the GPU library.
 *
 * Build: gcc -O2 -std=c99 -ffp-contract=off -fno-fast-math -fPIC -shared.
 * Every floating-point operation below is one IEEE operation rounded once,
 * evaluated in the written order (no contraction into FMA).
 *
 * Stages and where the paper defines them (Speedy-Splat, arXiv 2412.00578):
 *   preprocess   Sec. 3.2.1 "Preprocessing": projection of the mean, the 3D
 *                covariance R S S^T R^T (Eq. for Sigma_3D), the EWA projection
 *                J W Sigma W^T J^T with the last row/column dropped, its
 *                inverse (the conic), and the view-dependent colour from SH.
 *   threshold    Sec. 4.1: alpha = 1/255 gives t = 2 log(255 sigma) and the
 *                ellipse a x^2 + 2 b x y + c y^2 = t (Eq. simplified_ellipse).
 *   3-sigma      Sec. 4.1, Eq. radius: r = ceil(3 sqrt(lambda_max)).
 *   SnugBox      Sec. 4.1.1, Eqs. ellipse_intersect and bbox_args, solved in
 *                closed form; edges converted to tiles by dividing by the tile
 *                size, rounding down and clipping to the image.
 *   AccuTile     Sec. 4.1.2 and Algorithm 1: per tile row (or column, whichever
 *                side of the SnugBox tile extent is shorter) the ellipse's
 *                extent is the SnugBox extremal point when it lies in the band,
 *                otherwise the extreme of the two band-boundary intersections.
 *   keys/sort    Sec. 3.2.2 "Sorting": key = tile index | depth, stable sort,
 *                per-tile ranges.
 *   blend        Sec. 3.2.3, Eqs. render_alpha, 2d_gaussian_scalar and
 *                contribution: alpha = sigma exp(-q/2), included when
 *                alpha >= 1/255 (tested as q <= t), front-to-back compositing.
 *
 * Readings where the paper is silent (pixel centres at +0.5, +0.3 dilation,
 * 0.2 near plane, the 1.3x field-of-view clamp in J, the 0.99 alpha clamp,
 * the 1e-4 transmittance stop, the 0.1 discriminant floor for lambda_max and
 * the floor-based tile conversion) are listed in the design notes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Independently typed constants (the GPU library exports its own copy). */
#define ORC_TILE 16
#define ORC_DILATION 0.3
#define ORC_FOV_CLAMP 1.3
#define ORC_DISC_FLOOR 0.1
#define ORC_ALPHA_MAX 0.99f
#define ORC_T_MIN 1e-4f

enum { MODE_3SIGMA = 0, MODE_SNUGBOX = 1, MODE_ACCUTILE = 2 };

/* Camera passed as 24 floats:
 * [0]=width [1]=height [2]=fx [3]=fy [4]=cx [5]=cy [6..14]=R (row-major)
 * [15..17]=t [18]=near [19..21]=background rgb [22,23] unused. */
typedef struct {
    int width, height, tiles_x, tiles_y;
    double fx, fy, cx, cy, R[9], t[3], near_z;
    float bg[3];
} orc_cam;

static void cam_unpack(const float *p, orc_cam *c)
{
    c->width = (int)p[0];
    c->height = (int)p[1];
    c->tiles_x = (c->width + ORC_TILE - 1) / ORC_TILE;
    c->tiles_y = (c->height + ORC_TILE - 1) / ORC_TILE;
    c->fx = p[2]; c->fy = p[3]; c->cx = p[4]; c->cy = p[5];
    for (int k = 0; k < 9; ++k) c->R[k] = p[6 + k];
    for (int k = 0; k < 3; ++k) c->t[k] = p[15 + k];
    c->near_z = p[18];
    for (int k = 0; k < 3; ++k) c->bg[k] = p[19 + k];
}

/* Real spherical harmonics up to degree 3, ordered (l, m = -l..l), with the
 * Condon-Shortley phase (the convention of the 3D-GS renderer the paper
 * builds on).  Values are the standard normalisation constants. */
static void sh_basis(double x, double y, double z, double *Y)
{
    const double c0 = 0.28209479177387814;
    const double c1 = 0.4886025119029199;
    const double c2a = 1.0925484305920792, c2b = 0.31539156525252005, c2c = 0.5462742152960396;
    const double c3a = 0.5900435899266435, c3b = 2.890611442640554, c3c = 0.4570457994644658;
    const double c3d = 0.3731763325901154, c3e = 1.445305721320277;
    double xx = x * x, yy = y * y, zz = z * z;
    Y[0] = c0;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    Y[4] = c2a * (x * y);
    Y[5] = -c2a * (y * z);
    Y[6] = c2b * (2.0 * zz - xx - yy);
    Y[7] = -c2a * (x * z);
    Y[8] = c2c * (xx - yy);
    Y[9] = -c3a * y * (3.0 * xx - yy);
    Y[10] = c3b * (x * y * z);
    Y[11] = -c3c * y * (4.0 * zz - xx - yy);
    Y[12] = c3d * z * (2.0 * zz - 3.0 * xx - 3.0 * yy);
    Y[13] = -c3c * x * (4.0 * zz - xx - yy);
    Y[14] = c3e * z * (xx - yy);
    Y[15] = -c3a * x * (xx - 3.0 * yy);
}

/* Exposed for the SH pin test: writes 16 basis values for direction (x,y,z). */
void orc_sh_basis(double x, double y, double z, double *out) { sh_basis(x, y, z, out); }

/*
 * Per-Gaussian record, FP64 over FP32 inputs, rounded once into FP32.
 * geom = (u, v, depth, t); conic = (a, b, c, sigma); rgb = (r, g, b, 0).
 * Returns 1 if the Gaussian survives, 0 if culled (record zeroed).
 */
static int record_one(const orc_cam *cam, const float *mean, const float *scale,
                      const float *quat, float opac, const float *sh, int sh_degree,
                      int sh_stride, int mode, float *geom, float *conic, float *rgb)
{
    memset(geom, 0, 4 * sizeof(float));
    memset(conic, 0, 4 * sizeof(float));
    memset(rgb, 0, 4 * sizeof(float));
    for (int k = 0; k < 3; ++k)
        if (!isfinite(mean[k]) || !isfinite(scale[k])) return 0;
    for (int k = 0; k < 4; ++k)
        if (!isfinite(quat[k])) return 0;
    if (!isfinite(opac) || !(opac > 0.0f)) return 0;

    /* camera space: p_c = R mu + t */
    const double *R = cam->R;
    double mx = mean[0], my = mean[1], mz = mean[2];
    double x = ((R[0] * mx + R[1] * my) + R[2] * mz) + cam->t[0];
    double y = ((R[3] * mx + R[4] * my) + R[5] * mz) + cam->t[1];
    double z = ((R[6] * mx + R[7] * my) + R[8] * mz) + cam->t[2];
    if (!(z > cam->near_z)) return 0;

    /* pinhole projection of the mean */
    double u = (cam->fx * x) / z + cam->cx;
    double v = (cam->fy * y) / z + cam->cy;

    /* rotation from the normalised quaternion (w, x, y, z) */
    double qw = quat[0], qx = quat[1], qy = quat[2], qz = quat[3];
    double nn = ((qw * qw + qx * qx) + qy * qy) + qz * qz;
    if (!(nn > 0.0)) return 0;
    double qn = sqrt(nn);
    qw = qw / qn; qx = qx / qn; qy = qy / qn; qz = qz / qn;
    double Rq[9];
    Rq[0] = 1.0 - 2.0 * (qy * qy + qz * qz);
    Rq[1] = 2.0 * (qx * qy - qw * qz);
    Rq[2] = 2.0 * (qx * qz + qw * qy);
    Rq[3] = 2.0 * (qx * qy + qw * qz);
    Rq[4] = 1.0 - 2.0 * (qx * qx + qz * qz);
    Rq[5] = 2.0 * (qy * qz - qw * qx);
    Rq[6] = 2.0 * (qx * qz - qw * qy);
    Rq[7] = 2.0 * (qy * qz + qw * qx);
    Rq[8] = 1.0 - 2.0 * (qx * qx + qy * qy);

    /* Sigma_3D = (R S)(R S)^T */
    double M[9], S3[9];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) M[3 * i + j] = Rq[3 * i + j] * (double)scale[j];
    for (int i = 0; i < 3; ++i)
        for (int k = 0; k < 3; ++k)
            S3[3 * i + k] = (M[3 * i] * M[3 * k] + M[3 * i + 1] * M[3 * k + 1]) +
                            M[3 * i + 2] * M[3 * k + 2];

    /* EWA: Jacobian of the projection at the (field-of-view clamped) mean */
    double limx = ORC_FOV_CLAMP * ((0.5 * cam->width) / cam->fx);
    double limy = ORC_FOV_CLAMP * ((0.5 * cam->height) / cam->fy);
    double txz = x / z, tyz = y / z;
    if (txz < -limx) txz = -limx;
    if (txz > limx) txz = limx;
    if (tyz < -limy) tyz = -limy;
    if (tyz > limy) tyz = limy;
    double J00 = cam->fx / z, J02 = -(cam->fx * txz) / z;
    double J11 = cam->fy / z, J12 = -(cam->fy * tyz) / z;
    double T[6];
    for (int j = 0; j < 3; ++j) {
        T[j] = J00 * R[j] + J02 * R[6 + j];
        T[3 + j] = J11 * R[3 + j] + J12 * R[6 + j];
    }
    double V[6];
    for (int i = 0; i < 2; ++i)
        for (int k = 0; k < 3; ++k)
            V[3 * i + k] = (T[3 * i] * S3[k] + T[3 * i + 1] * S3[3 + k]) + T[3 * i + 2] * S3[6 + k];
    double s00 = (V[0] * T[0] + V[1] * T[1]) + V[2] * T[2];
    double s01 = (V[0] * T[3] + V[1] * T[4]) + V[2] * T[5];
    double s11 = (V[3] * T[3] + V[4] * T[4]) + V[5] * T[5];
    double A = s00 + ORC_DILATION, B = s01, C = s11 + ORC_DILATION;
    double D = A * C - B * B;
    if (!(D > 0.0)) return 0;

    /* conic = Sigma_2D^{-1} and threshold t = 2 log(255 sigma) */
    float ca = (float)(C / D), cb = (float)(-B / D), cc = (float)(A / D);
    float tt = (float)(2.0 * log(255.0 * (double)opac));
    if (mode != MODE_3SIGMA && !(tt > 0.0f)) return 0;

    /* view-dependent colour: SH at the unit direction from the camera centre */
    double cpx = -((R[0] * cam->t[0] + R[3] * cam->t[1]) + R[6] * cam->t[2]);
    double cpy = -((R[1] * cam->t[0] + R[4] * cam->t[1]) + R[7] * cam->t[2]);
    double cpz = -((R[2] * cam->t[0] + R[5] * cam->t[1]) + R[8] * cam->t[2]);
    double dx = mx - cpx, dy = my - cpy, dz = mz - cpz;
    double dn = sqrt(dx * dx + dy * dy + dz * dz);
    double Y[16];
    sh_basis(dx / dn, dy / dn, dz / dn, Y);
    int nb = (sh_degree + 1) * (sh_degree + 1);
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < nb; ++k) acc += Y[k] * (double)sh[3 * k + ch];
        acc += 0.5;
        rgb[ch] = (float)(acc > 0.0 ? acc : 0.0);
    }
    (void)sh_stride;
    geom[0] = (float)u; geom[1] = (float)v; geom[2] = (float)z; geom[3] = tt;
    conic[0] = ca; conic[1] = cb; conic[2] = cc; conic[3] = opac;
    return 1;
}

/* ----------------------------------------------------------------------------
 * Tile geometry on the stored FP32 record (FP64 arithmetic).
 * ------------------------------------------------------------------------- */

/* Convert an interval edge to a tile index: divide by the tile size, round
 * down, clip to the image.  lo-edges clip into [0, n], hi-edges into [-1, n-1],
 * so an interval entirely outside the image becomes empty (lo > hi). */
static int tile_lo(double x, int n)
{
    double f = floor(x / ORC_TILE);
    if (f < 0.0) f = 0.0;
    if (f > (double)n) f = (double)n;
    return (int)f;
}

static int tile_hi(double x, int n)
{
    double f = floor(x / ORC_TILE);
    if (f < -1.0) f = -1.0;
    if (f > (double)(n - 1)) f = (double)(n - 1);
    return (int)f;
}

typedef struct {
    double u, v, a, b, c, t, det, hx, hy;
    double box[4];      /* pixel-space extent x0, x1, y0, y1 of the mode */
    int x0, x1, y0, y1; /* inclusive tile rect; empty if x0 > x1 or y0 > y1 */
} orc_ellipse;

/* Returns 0 when the record cannot touch any tile. */
static int ellipse_setup(const float *geom, const float *conic, int mode, int tx_n, int ty_n,
                         orc_ellipse *e)
{
    e->u = geom[0]; e->v = geom[1]; e->t = geom[3];
    e->a = conic[0]; e->b = conic[1]; e->c = conic[2];
    e->det = e->a * e->c - e->b * e->b;
    if (!(e->det > 0.0)) return 0;
    double xl, xh, yl, yh;
    if (mode == MODE_3SIGMA) {
        /* largest eigenvalue of the record ellipse's covariance (conic^{-1}) */
        double sxx = e->c / e->det, syy = e->a / e->det;
        double mid = 0.5 * (sxx + syy);
        double disc = mid * mid - 1.0 / e->det;
        if (disc < ORC_DISC_FLOOR) disc = ORC_DISC_FLOOR;
        double lam = mid + sqrt(disc);
        double r = ceil(3.0 * sqrt(lam));
        xl = e->u - r; xh = e->u + r; yl = e->v - r; yh = e->v + r;
    } else {
        if (!(e->t > 0.0)) return 0;
        /* SnugBox half-extents: sqrt(t * Sxx), sqrt(t * Syy) */
        e->hx = sqrt((e->t * e->c) / e->det);
        e->hy = sqrt((e->t * e->a) / e->det);
        xl = e->u - e->hx; xh = e->u + e->hx; yl = e->v - e->hy; yh = e->v + e->hy;
    }
    e->box[0] = xl; e->box[1] = xh; e->box[2] = yl; e->box[3] = yh;
    e->x0 = tile_lo(xl, tx_n); e->x1 = tile_hi(xh, tx_n);
    e->y0 = tile_lo(yl, ty_n); e->y1 = tile_hi(yh, ty_n);
    return (e->x0 <= e->x1 && e->y0 <= e->y1);
}

/* x-range of the ellipse on the horizontal line y = Y (left/right roots). */
static void row_roots(const orc_ellipse *e, double Y, double *xl, double *xr)
{
    double dy = Y - e->v;
    double rad = e->t * e->a - (e->det * dy) * dy;
    double s = sqrt(rad > 0.0 ? rad : 0.0);
    double bd = e->b * dy;
    *xl = e->u + (-bd - s) / e->a;
    *xr = e->u + (-bd + s) / e->a;
}

/* y-range of the ellipse on the vertical line x = X (Eq. ellipse_intersect). */
static void col_roots(const orc_ellipse *e, double X, double *yt, double *yb)
{
    double dx = X - e->u;
    double rad = e->t * e->c - (e->det * dx) * dx;
    double s = sqrt(rad > 0.0 ? rad : 0.0);
    double bd = e->b * dx;
    *yt = e->v + (-bd - s) / e->c;
    *yb = e->v + (-bd + s) / e->c;
}

/*
 * Enumerate the tiles of one record in emission order, writing tile ids
 * (ty * tiles_x + tx) to out[] when out is non-NULL.  Returns the count.
 * 3-sigma and SnugBox: the rectangle, row by row.  AccuTile: row by row when
 * the rectangle has no more rows than columns, otherwise column by column.
 */
int64_t orc_tile_list(const float *geom, const float *conic, int mode, int tx_n, int ty_n,
                      uint32_t *out)
{
    orc_ellipse e;
    if (!ellipse_setup(geom, conic, mode, tx_n, ty_n, &e)) return 0;
    int64_t n = 0;
    if (mode != MODE_ACCUTILE) {
        for (int ty = e.y0; ty <= e.y1; ++ty)
            for (int tx = e.x0; tx <= e.x1; ++tx) {
                if (out) out[n] = (uint32_t)(ty * tx_n + tx);
                ++n;
            }
        return n;
    }
    int nrows = e.y1 - e.y0 + 1, ncols = e.x1 - e.x0 + 1;
    if (nrows <= ncols) {
        /* y of the leftmost / rightmost points of the ellipse */
        double k = (e.b / e.c) * e.hx;
        double y_left = e.v + k, y_right = e.v - k;
        double box_b = e.v - e.hy, box_t = e.v + e.hy;
        for (int ty = e.y0; ty <= e.y1; ++ty) {
            double ylo = 16.0 * ty, yhi = 16.0 * ty + 16.0;
            if (ylo < box_b) ylo = box_b;
            if (yhi > box_t) yhi = box_t;
            double l0, r0, l1, r1;
            row_roots(&e, ylo, &l0, &r0);
            row_roots(&e, yhi, &l1, &r1);
            double left = (ylo <= y_left && y_left <= yhi) ? e.u - e.hx : (l0 < l1 ? l0 : l1);
            double right = (ylo <= y_right && y_right <= yhi) ? e.u + e.hx : (r0 > r1 ? r0 : r1);
            int lo = tile_lo(left, tx_n), hi = tile_hi(right, tx_n);
            if (lo < e.x0) lo = e.x0;
            if (hi > e.x1) hi = e.x1;
            for (int tx = lo; tx <= hi; ++tx) {
                if (out) out[n] = (uint32_t)(ty * tx_n + tx);
                ++n;
            }
        }
    } else {
        double m = (e.b / e.a) * e.hy;
        double x_top = e.u + m, x_bot = e.u - m;   /* x of the min-y / max-y points */
        double box_l = e.u - e.hx, box_r = e.u + e.hx;
        for (int tx = e.x0; tx <= e.x1; ++tx) {
            double xlo = 16.0 * tx, xhi = 16.0 * tx + 16.0;
            if (xlo < box_l) xlo = box_l;
            if (xhi > box_r) xhi = box_r;
            double t0, b0, t1, b1;
            col_roots(&e, xlo, &t0, &b0);
            col_roots(&e, xhi, &t1, &b1);
            double top = (xlo <= x_top && x_top <= xhi) ? e.v - e.hy : (t0 < t1 ? t0 : t1);
            double bot = (xlo <= x_bot && x_bot <= xhi) ? e.v + e.hy : (b0 > b1 ? b0 : b1);
            int lo = tile_lo(top, ty_n), hi = tile_hi(bot, ty_n);
            if (lo < e.y0) lo = e.y0;
            if (hi > e.y1) hi = e.y1;
            for (int ty = lo; ty <= hi; ++ty) {
                if (out) out[n] = (uint32_t)(ty * tx_n + tx);
                ++n;
            }
        }
    }
    return n;
}

/* Inclusive tile rectangle of a record for a mode (for tests); returns 0 if empty. */
int orc_tile_rect(const float *geom, const float *conic, int mode, int tx_n, int ty_n,
                  int32_t *rect4)
{
    orc_ellipse e;
    int ok = ellipse_setup(geom, conic, mode, tx_n, ty_n, &e);
    rect4[0] = ok ? e.x0 : 0; rect4[1] = ok ? e.y0 : 0;
    rect4[2] = ok ? e.x1 : -1; rect4[3] = ok ? e.y1 : -1;
    return ok;
}

/* Preprocess all Gaussians: records (with the colour of every surviving
 * record) and tile counts.  Returns the visible count. */
int64_t orc_preprocess(const float *campack, int64_t n, int sh_degree, int sh_stride,
                       const float *means, const float *scales, const float *quats,
                       const float *opacity, const float *sh, int mode,
                       float *geom, float *conic, float *rgb, uint32_t *counts)
{
    orc_cam cam;
    cam_unpack(campack, &cam);
    int64_t visible = 0;
    for (int64_t i = 0; i < n; ++i) {
        float *g = geom + 4 * i, *q = conic + 4 * i, *c = rgb + 4 * i;
        int ok = record_one(&cam, means + 3 * i, scales + 3 * i, quats + 4 * i, opacity[i],
                            sh + (int64_t)3 * sh_stride * i, sh_degree, sh_stride, mode,
                            g, q, c);
        counts[i] = ok ? (uint32_t)orc_tile_list(g, q, mode, cam.tiles_x, cam.tiles_y, NULL) : 0u;
        visible += ok;
    }
    return visible;
}

/* Emit (key, value) pairs: Gaussians in index order, tiles in enumeration
 * order.  key = tile_id << 32 | bits(depth).  Returns the number written. */
int64_t orc_emit(int64_t n, const float *geom, const float *conic, int mode, int tx_n, int ty_n,
                 uint64_t *keys, uint32_t *values)
{
    int64_t p = 0;
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)tx_n * (size_t)ty_n);
    for (int64_t i = 0; i < n; ++i) {
        int64_t m = orc_tile_list(geom + 4 * i, conic + 4 * i, mode, tx_n, ty_n, tmp);
        uint32_t dbits;
        memcpy(&dbits, &geom[4 * i + 2], 4);
        for (int64_t k = 0; k < m; ++k) {
            keys[p] = ((uint64_t)tmp[k] << 32) | (uint64_t)dbits;
            values[p] = (uint32_t)i;
            ++p;
        }
    }
    free(tmp);
    return p;
}

/* Sort pairs by (key, value): the result of a stable sort by key when the
 * input is in value order. */
typedef struct { uint64_t k; uint32_t v; } orc_pair;

static int pair_cmp(const void *pa, const void *pb)
{
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    if (a->k != b->k) return a->k < b->k ? -1 : 1;
    if (a->v != b->v) return a->v < b->v ? -1 : 1;
    return 0;
}

void orc_sort(int64_t p, uint64_t *keys, uint32_t *values)
{
    orc_pair *tmp = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(p > 0 ? p : 1));
    for (int64_t i = 0; i < p; ++i) { tmp[i].k = keys[i]; tmp[i].v = values[i]; }
    qsort(tmp, (size_t)p, sizeof(orc_pair), pair_cmp);
    for (int64_t i = 0; i < p; ++i) { keys[i] = tmp[i].k; values[i] = tmp[i].v; }
    free(tmp);
}

/* Per-tile [start, end) of the sorted keys; an empty tile gets
 * start = end = the position of the first key of a later tile. */
void orc_ranges(int64_t p, const uint64_t *keys, int64_t n_tiles, uint32_t *ranges)
{
    int64_t pos = 0;
    for (int64_t tile = 0; tile < n_tiles; ++tile) {
        while (pos < p && (int64_t)(keys[pos] >> 32) < tile) ++pos;
        int64_t start = pos;
        while (pos < p && (int64_t)(keys[pos] >> 32) == tile) ++pos;
        ranges[2 * tile] = (uint32_t)start;
        ranges[2 * tile + 1] = (uint32_t)pos;
    }
}

/*
 * Blend one tile front to back.  For each pixel centre (px + 0.5, py + 0.5),
 * with dx, dy its offsets from the record's centre (one FP64 subtraction
 * each), the quadratic form q = (a dx^2 + c dy^2) + 2b dx dy of the stored
 * record is evaluated in FP64 and a Gaussian is included when q <= t
 * (alpha >= 1/255): the same inequality, on the same record and in the same
 * precision, as the tile geometry, so a pixel is included only where its
 * tile was assigned.  alpha = min(0.99, sigma exp(-q/2)) in FP32 from q
 * rounded to FP32; the walk stops before a Gaussian that would take the
 * transmittance below 1e-4; colours accumulate in FP32.  Output planar [3,H,W].
 *
 * ambig[] (optional) marks the pixels where another faithful implementation
 * may decide differently:
 *  - inclusion: any FP64 evaluation of q with at most four roundings per term
 *    lies within gamma_4 * S of the exact q (S = |a| dx^2 + |c| dy^2 +
 *    2 |b dx dy|, gamma_4 = 4v / (1 - 4v), v = 2^-53); a pair whose q lies
 *    within twice that of t is flagged.
 *  - stop: the relative error of T that another faithful alpha can cause is
 *    tracked as err.  alpha may differ by 16 FP32 ulp through exp and, where
 *    two FP64 values of q round to neighbouring FP32 values, by half an ulp of
 *    q times q; each alpha not clamped on both sides adds that relative error
 *    times alpha / (1 - alpha), and a stop test within T_MIN * (err + 4 ulp)
 *    of the threshold is flagged.
 * n_contrib (optional) counts the Gaussians blended into each pixel.
 */
static void blend_tile(const orc_cam *cam, int tx, int ty, const uint32_t *ranges,
                       const uint32_t *values, const float *geom, const float *conic,
                       const float *rgb, float *img, float *t_final, uint32_t *n_last,
                       uint32_t *n_eval, uint32_t *n_contrib, uint8_t *ambig)
{
    int tile = ty * cam->tiles_x + tx;
    uint32_t start = ranges[2 * tile], end = ranges[2 * tile + 1];
    int64_t hw = (int64_t)cam->width * cam->height;
    for (int py = ty * ORC_TILE; py < ty * ORC_TILE + ORC_TILE && py < cam->height; ++py)
        for (int px = tx * ORC_TILE; px < tx * ORC_TILE + ORC_TILE && px < cam->width; ++px) {
            float T = 1.0f, C[3] = {0.0f, 0.0f, 0.0f};
            uint32_t last = 0, evals = end - start, contrib = 0;
            int amb = 0;
            double err = 0.0;
            const double ulp = ldexp(1.0, -24), v = ldexp(1.0, -53);
            const double gam_q = 2.0 * (4.0 * v / (1.0 - 4.0 * v));
            double fx = (double)px + 0.5, fy = (double)py + 0.5;
            for (uint32_t j = start; j < end; ++j) {
                uint32_t i = values[j];
                const float *g = geom + 4 * (int64_t)i, *q = conic + 4 * (int64_t)i;
                double dx = fx - (double)g[0], dy = fy - (double)g[1];
                double a = q[0], b = q[1], c = q[2], t = g[3];
                double q64 = (a * dx * dx + c * dy * dy) + 2.0 * b * dx * dy;
                double mag = fabs(a) * dx * dx + fabs(c) * dy * dy + 2.0 * fabs(b * dx * dy);
                if (fabs(q64 - t) <= gam_q * mag + 0x1p-1000) amb = 1;
                if (!(q64 <= t)) continue;
                float qq = (float)q64;
                float raw = q[3] * expf(-0.5f * qq);
                float al = raw > ORC_ALPHA_MAX ? ORC_ALPHA_MAX : raw;
                float tn = T * (1.0f - al);
                double rel_al = 16.0 * ulp + 0.5 * ulp * fabs((double)qq);
                if ((double)raw <= (double)ORC_ALPHA_MAX * (1.0 + 2.0 * rel_al))
                    err += rel_al * (double)al / (1.0 - (double)al);
                if (fabs((double)tn - (double)ORC_T_MIN) <= (double)ORC_T_MIN * (err + 4.0 * ulp))
                    amb = 1;
                if (tn < ORC_T_MIN) {
                    evals = j - start + 1;
                    break;
                }
                float w = al * T;
                const float *col = rgb + 4 * (int64_t)i;
                C[0] = C[0] + col[0] * w;
                C[1] = C[1] + col[1] * w;
                C[2] = C[2] + col[2] * w;
                T = tn;
                last = j - start + 1;
                ++contrib;
            }
            int64_t pix = (int64_t)py * cam->width + px;
            for (int ch = 0; ch < 3; ++ch) img[ch * hw + pix] = C[ch] + T * cam->bg[ch];
            if (t_final) t_final[pix] = T;
            if (n_last) n_last[pix] = last;
            if (n_eval) n_eval[pix] = evals;
            if (n_contrib) n_contrib[pix] = contrib;
            if (ambig) ambig[pix] = (uint8_t)amb;
        }
}

/* Blend the listed tiles (tile ids), or every tile when n_list < 0. */
void orc_blend(const float *campack, const uint32_t *ranges, const uint32_t *values,
               const float *geom, const float *conic, const float *rgb,
               int64_t n_list, const int32_t *tile_list,
               float *img, float *t_final, uint32_t *n_last, uint32_t *n_eval,
               uint32_t *n_contrib, uint8_t *ambig)
{
    orc_cam cam;
    cam_unpack(campack, &cam);
    if (n_list < 0) {
        for (int ty = 0; ty < cam.tiles_y; ++ty)
            for (int tx = 0; tx < cam.tiles_x; ++tx)
                blend_tile(&cam, tx, ty, ranges, values, geom, conic, rgb, img, t_final, n_last,
                           n_eval, n_contrib, ambig);
    } else {
        for (int64_t k = 0; k < n_list; ++k) {
            int tile = tile_list[k];
            blend_tile(&cam, tile % cam.tiles_x, tile / cam.tiles_x, ranges, values, geom, conic,
                       rgb, img, t_final, n_last, n_eval, n_contrib, ambig);
        }
    }
}

/*
 * Brute-force reference (FP64), no tiles: every pixel in `pix` walks every
 * record in (depth bits, index) order given by `order`, with the same
 * inclusion, clamp and stop rules.  When rect_mode >= 0, a record is only
 * considered at pixels whose tile lies in its tile rectangle for that mode
 * (the 3-sigma restricted reference); rect_mode < 0 considers every record.
 * ambig[k] is set when an inclusion or stop decision lay in its rounding band
 * (inclusion: |q - t| within 16 FP64 ulp of the magnitude of q's terms, which
 * covers two FP64 evaluations of q in different orders; stop: a relative 1e-3
 * of the threshold).  Output rgb[k*3 + ch].
 */
void orc_brute_pixels(const float *campack, int64_t n, const float *geom, const float *conic,
                      const float *rgb, const int64_t *order, int64_t n_order, int rect_mode,
                      int64_t n_pix, const int32_t *pix, double *out, uint8_t *ambig)
{
    orc_cam cam;
    cam_unpack(campack, &cam);
    int32_t *rects = NULL;
    if (rect_mode >= 0) {
        rects = (int32_t *)malloc(sizeof(int32_t) * 4 * (size_t)(n > 0 ? n : 1));
        for (int64_t i = 0; i < n; ++i)
            orc_tile_rect(geom + 4 * i, conic + 4 * i, rect_mode, cam.tiles_x, cam.tiles_y,
                          rects + 4 * i);
    }
    const double gam = 16.0 * ldexp(1.0, -53);
    for (int64_t k = 0; k < n_pix; ++k) {
        int px = pix[2 * k], py = pix[2 * k + 1];
        int tx = px / ORC_TILE, ty = py / ORC_TILE;
        double T = 1.0, C[3] = {0.0, 0.0, 0.0};
        int amb = 0;
        double fx = px + 0.5, fy = py + 0.5;
        for (int64_t o = 0; o < n_order; ++o) {
            int64_t i = order[o];
            if (rects) {
                const int32_t *r = rects + 4 * i;
                if (tx < r[0] || tx > r[2] || ty < r[1] || ty > r[3]) continue;
            }
            const float *g = geom + 4 * i, *q = conic + 4 * i;
            double a = q[0], b = q[1], c = q[2], t = g[3];
            if (a == 0.0 && b == 0.0 && c == 0.0) continue; /* culled record */
            double dx = fx - g[0], dy = fy - g[1];
            double qq = a * dx * dx + 2.0 * b * dx * dy + c * dy * dy;
            double mag = fabs(a) * dx * dx + 2.0 * fabs(b * dx * dy) + fabs(c) * dy * dy;
            if (fabs(qq - t) <= gam * (mag + fabs(t))) amb = 1;
            if (!(qq <= t)) continue;
            double al = (double)q[3] * exp(-0.5 * qq);
            if (al > 0.99) al = 0.99;
            double tn = T * (1.0 - al);
            if (fabs(tn - 1e-4) <= 1e-3 * 1e-4) amb = 1;
            if (tn < 1e-4) break;
            const float *col = rgb + 4 * i;
            for (int ch = 0; ch < 3; ++ch) C[ch] += col[ch] * al * T;
            T = tn;
        }
        for (int ch = 0; ch < 3; ++ch) out[3 * k + ch] = C[ch] + T * cam.bg[ch];
        if (ambig) ambig[k] = (uint8_t)amb;
    }
    free(rects);
}

/* Pixel-space extent [x0, x1, y0, y1] of a record for a mode (3-sigma square
 * or SnugBox box, before the tile conversion); returns 0 if none. */
int orc_extent(const float *geom, const float *conic, int mode, double *out4)
{
    orc_ellipse e;
    e.box[0] = e.box[1] = e.box[2] = e.box[3] = 0.0;
    ellipse_setup(geom, conic, mode, 1 << 20, 1 << 20, &e);
    if (!(e.det > 0.0) || (mode != MODE_3SIGMA && !(e.t > 0.0))) return 0;
    for (int k = 0; k < 4; ++k) out4[k] = e.box[k];
    return 1;
}
