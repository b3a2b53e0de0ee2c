/*
 * linprim_oracle.c -- FP64 CPU reference ("oracle") of the differentiable
 * tile rasterizer for transparent octahedra and tetrahedra of
 * LinPrim (von Luetzow & Niessner, arXiv 2501.16312).
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; only the test-suite, the smoke check and the CPU-baseline
 * leg of the benchmark use it.  It shares no code, header or constant table
 * with the HIP implementation.  It is plain and slow on purpose: every step
 * follows the paper's description in the paper's order, in double precision,
 * with no blocking or fusion beyond what the paper itself states (tiling and
 * a global sort, Sec. 3.2).
 *
 * Readings of the paper where it is silent (each documented with the build):
 *   - quaternion (w,x,y,z), normalised by the rotation formula itself;
 *   - tetrahedron basis: (1,1,1),(1,-1,-1),(-1,1,-1),(-1,-1,1) over sqrt(3);
 *   - ray space: the EWA map x -> (fx*x/z+cx, fy*y/z+cy, |x|) linearised at
 *     the primitive centre (the third coordinate is the Euclidean distance);
 *   - pixel centres at (i+1/2, j+1/2); the pixel rectangle of a primitive is
 *     the set of pixel centres inside its projected bounding box;
 *   - sort key = float32 bits of the centre's camera z, ties by index;
 *   - opacity o = min(1 - exp(-sigma * chord), 0.99);
 *   - compositing stops after the primitive that brings the transmittance
 *     to 1e-3 or below;
 *   - no gradient through min(d) of Eq. 1 (App. G);
 *   - exact variant (the appendix on the ray-space approximation): the same
 *     pipeline without ray space; each pixel ray leaves the camera centre and
 *     the chord is the Euclidean length of its segment inside the camera-space
 *     primitive; the bounding box is that of the perspective-projected
 *     corners, and a primitive with a corner at or in front of the near plane
 *     is culled (its projection is undefined there).
 *
 * The binning quantities (pixel rectangle, tile rectangle, depth key) are
 * integer decisions.  They are computed in double precision with a fixed
 * left-to-right evaluation order and no fused multiply-add, so that any other
 * implementation that evaluates the same expressions in IEEE double reaches
 * the same integers.  Build with -ffp-contract=off.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OCTA 0
#define ORC_TETRA 1
#define ORC_MAX_VIEWS 256

/* Eq. 1: density normaliser uses 0.99 * alpha. */
#define ORC_ALPHA_SCALE 0.99
/* Sec. 3.2 "Compositing": stop once cumulative opacity reaches 0.999. */
#define ORC_T_STOP 1e-3
/* Opacity clamp (keeps 1/(1-o) finite in the backward pass). */
#define ORC_O_MAX 0.99
/* 1/sqrt(3) as a decimal literal (parsed to the nearest double). */
#define ORC_INV_SQRT3 0.57735026918962576451

/* Conditioning thresholds of the parity contract: a decision within these
 * margins may go either way in float32 (see step_ill and orc_backward). */
#define ORC_ILL_T 1e-6
#define ORC_ILL_O 1e-6
#define ORC_ILL_BARY 1e-5
#define ORC_ILL_RGB 1e-6
/* float32 evaluation errors of a primitive's opacities, weighted as they
 * enter its opacity and SH gradients, above this fraction of those
 * gradients (under a third of the gradient tolerance, with its floor)
 * flag the primitive: e.g. chords that graze its edge are known only to a
 * few digits in float32 */
#define ORC_ILL_REL 3e-4

typedef struct {
    double Rw[3][3], tw[3];
    double fx, fy, cx, cy;
    int W, H;
    double near_z;
    int tiles_x, tiles_y;
    int64_t tile_base;
    int64_t pix_base;
} orc_view;

typedef struct {
    int valid;
    int rect[4];     /* i0, j0, i1, j1 (inclusive) */
    int trect[4];    /* tile x0, y0, x1, y1 (inclusive) */
    int64_t tiles;   /* tiles touched */
    uint32_t key;    /* float32 bits of camera-space centre z */
    double tc[3];    /* camera-space centre */
    double c[3];     /* ray-space centre */
    double a[4][3];  /* ray-space offsets: octahedron a0..a2, tetrahedron a0..a3 */
    double oc[4][3]; /* camera-space offsets from the centre to the axes / corners */
    double vc[6][3]; /* camera-space corners (exact variant) */
    double sigma;
    double rgb[3];
    double raw[3];   /* colour before the clamp at zero */
    double radius;   /* half the larger side of the projected bounding box (pixels) */
} orc_prep;

typedef struct {
    int type, deg, K, nd;
    int exact;               /* 0: EWA ray space (Sec. 3.2); 1: pixel rays in camera space (App. "Ray Space Approximation") */
    int aa;                  /* 2D anti-aliasing filter (App. "Anti-Aliasing"), ray space only */
    int64_t n;
    double *means, *quats, *dists, *opac, *sh;
    int n_views, tile;
    orc_view views[ORC_MAX_VIEWS];
    orc_prep *prep;          /* [n_views][n] */
    int64_t n_pairs;
    uint64_t *keys;
    uint32_t *vals;
    int64_t n_tiles_total;
    int64_t *rlo, *rhi;
    double *sgrad;           /* [n_views][n][2] dL/d(projected centre) of the last backward */
} orc_scene;

/* ------------------------------------------------------------------------ */
/* Spherical harmonics (Sec. 3.1, "same approach described in 3DGS"):       */
/* real orthonormal SH up to degree 3, Condon-Shortley phase kept for odd m, */
/* ordered l = 0..3, m = -l..l.  Constants from their closed forms.         */
/* ------------------------------------------------------------------------ */
void orc_sh_basis(int deg, const double d[3], double Y[16])
{
    const double pi = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    const double c0 = 0.5 * sqrt(1.0 / pi);
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    for (int k = 0; k < 16; ++k) Y[k] = 0.0;
    Y[0] = c0;
    if (deg < 1) return;
    Y[1] = -c1 * y;
    Y[2] = c1 * z;
    Y[3] = -c1 * x;
    if (deg < 2) return;
    Y[4] = c2a * x * y;
    Y[5] = -c2a * y * z;
    Y[6] = c2b * (2.0 * z * z - x * x - y * y);
    Y[7] = -c2a * x * z;
    Y[8] = c2c * (x * x - y * y);
    if (deg < 3) return;
    Y[9] = -c3a * y * (3.0 * x * x - y * y);
    Y[10] = c3b * x * y * z;
    Y[11] = -c3c * y * (4.0 * z * z - x * x - y * y);
    Y[12] = c3d * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    Y[13] = -c3c * x * (4.0 * z * z - x * x - y * y);
    Y[14] = c3e * z * (x * x - y * y);
    Y[15] = -c3a * x * (x * x - 3.0 * y * y);
}

/* Partial derivatives dY_k/d(x,y,z) of the polynomials above, treating the
 * three direction components as independent variables. */
static void sh_basis_grad(int deg, const double d[3], double G[16][3])
{
    const double pi = 3.14159265358979323846;
    const double x = d[0], y = d[1], z = d[2];
    const double c1 = sqrt(3.0 / (4.0 * pi));
    const double c2a = 0.5 * sqrt(15.0 / pi), c2b = 0.25 * sqrt(5.0 / pi), c2c = 0.25 * sqrt(15.0 / pi);
    const double c3a = 0.25 * sqrt(35.0 / (2.0 * pi)), c3b = 0.5 * sqrt(105.0 / pi);
    const double c3c = 0.25 * sqrt(21.0 / (2.0 * pi)), c3d = 0.25 * sqrt(7.0 / pi);
    const double c3e = 0.25 * sqrt(105.0 / pi);
    memset(G, 0, sizeof(double) * 48);
    if (deg < 1) return;
    G[1][1] = -c1;
    G[2][2] = c1;
    G[3][0] = -c1;
    if (deg < 2) return;
    G[4][0] = c2a * y;  G[4][1] = c2a * x;
    G[5][1] = -c2a * z; G[5][2] = -c2a * y;
    G[6][0] = -2.0 * c2b * x; G[6][1] = -2.0 * c2b * y; G[6][2] = 4.0 * c2b * z;
    G[7][0] = -c2a * z; G[7][2] = -c2a * x;
    G[8][0] = 2.0 * c2c * x; G[8][1] = -2.0 * c2c * y;
    if (deg < 3) return;
    G[9][0] = -c3a * 6.0 * x * y;
    G[9][1] = -c3a * (3.0 * x * x - 3.0 * y * y);
    G[10][0] = c3b * y * z; G[10][1] = c3b * x * z; G[10][2] = c3b * x * y;
    G[11][0] = -c3c * y * (-2.0 * x);
    G[11][1] = -c3c * (4.0 * z * z - x * x - 3.0 * y * y);
    G[11][2] = -c3c * y * 8.0 * z;
    G[12][0] = c3d * z * (-6.0 * x);
    G[12][1] = c3d * z * (-6.0 * y);
    G[12][2] = c3d * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    G[13][0] = -c3c * (4.0 * z * z - 3.0 * x * x - y * y);
    G[13][1] = -c3c * x * (-2.0 * y);
    G[13][2] = -c3c * x * 8.0 * z;
    G[14][0] = c3e * z * 2.0 * x; G[14][1] = -c3e * z * 2.0 * y; G[14][2] = c3e * (x * x - y * y);
    G[15][0] = -c3a * (3.0 * x * x - 3.0 * y * y);
    G[15][1] = -c3a * x * (-6.0 * y);
}

/* ------------------------------------------------------------------------ */
/* Geometry of one primitive (Sec. 3.1).                                    */
/* ------------------------------------------------------------------------ */

/* Rotation of the unit quaternion q/|q|, written with s = 2/|q|^2 so that no
 * square root is needed.  Returns 0 for a zero or non-finite quaternion. */
static int quat_rotation(const double *q, double R[3][3])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    const double n2 = w * w + x * x + y * y + z * z;
    if (!(n2 > 0.0) || !isfinite(n2)) return 0;
    const double s = 2.0 / n2;
    R[0][0] = 1.0 - s * (y * y + z * z);
    R[0][1] = s * (x * y - w * z);
    R[0][2] = s * (x * z + w * y);
    R[1][0] = s * (x * y + w * z);
    R[1][1] = 1.0 - s * (x * x + z * z);
    R[1][2] = s * (y * z - w * x);
    R[2][0] = s * (x * z - w * y);
    R[2][1] = s * (y * z + w * x);
    R[2][2] = 1.0 - s * (x * x + y * y);
    return 1;
}

/* Tetrahedron basis directions (before the 1/sqrt(3) scale). */
static const double TET_B[4][3] = {{1, 1, 1}, {1, -1, -1}, {-1, 1, -1}, {-1, -1, 1}};

/* World-space offsets from the centre to the corners: octahedron: the three
 * rotated axes scaled by their distances (corners mu +/- o_k); tetrahedron:
 * the four rotated basis directions scaled by their distances (corners
 * mu + o_i). */
static void world_offsets(int type, const double R[3][3], const double *d, double o[4][3])
{
    if (type == ORC_OCTA) {
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) o[k][r] = R[r][k] * d[k];
    } else {
        for (int i = 0; i < 4; ++i) {
            const double g = d[i] * ORC_INV_SQRT3;
            for (int r = 0; r < 3; ++r)
                o[i][r] = (TET_B[i][0] * R[r][0] + TET_B[i][1] * R[r][1] + TET_B[i][2] * R[r][2]) * g;
        }
    }
}

static void mat3_vec(const double M[3][3], const double v[3], double out[3])
{
    for (int r = 0; r < 3; ++r) out[r] = M[r][0] * v[0] + M[r][1] * v[1] + M[r][2] * v[2];
}

static void mat3T_vec(const double M[3][3], const double v[3], double out[3])
{
    for (int c = 0; c < 3; ++c) out[c] = M[0][c] * v[0] + M[1][c] * v[1] + M[2][c] * v[2];
}

/* EWA ray-space Jacobian at camera-space point t (Zwicker et al.), with the
 * viewport scale folded into the first two rows. */
static void ray_jacobian(const orc_view *V, const double t[3], double J[3][3])
{
    const double iz = 1.0 / t[2];
    const double px = V->fx * t[0] * iz, py = V->fy * t[1] * iz;
    const double l = sqrt(t[0] * t[0] + t[1] * t[1] + t[2] * t[2]);
    J[0][0] = V->fx * iz; J[0][1] = 0.0; J[0][2] = -(px * iz);
    J[1][0] = 0.0; J[1][1] = V->fy * iz; J[1][2] = -(py * iz);
    J[2][0] = t[0] / l; J[2][1] = t[1] / l; J[2][2] = t[2] / l;
}

/* The 2D anti-aliasing filter (appendix "Anti-Aliasing", filter size in
 * App. G): the corners that lie on the tiling box move outward, parallel to
 * the screen, so that the box grows by the filter size of 0.1 pixel per
 * axis.  An octahedron's ray-space axis vector a_k carries the two mirrored
 * corners c +/- a_k, so it moves by half the size (each side of the box by
 * 0.05), as App. G states; a tetrahedron's extreme corners move by the same
 * half size each, so both kinds grow by the same 0.1 per axis.  A corner on
 * two sides of the box moves along both axes.  The selection is piecewise
 * constant, so gradients pass through unchanged. */
#define ORC_AA_SIZE 0.1
static void antialias_shift(int type, double a[4][3])
{
    for (int ax = 0; ax < 2; ++ax) {
        if (type == ORC_OCTA) {
            double ext = 0.0;
            for (int k = 0; k < 3; ++k) if (fabs(a[k][ax]) > ext) ext = fabs(a[k][ax]);
            double shift[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < 3; ++k)
                if (fabs(a[k][ax]) == ext) shift[k] = copysign(0.5 * ORC_AA_SIZE, a[k][ax]);
            for (int k = 0; k < 3; ++k) a[k][ax] += shift[k];
        } else {
            double lo = a[0][ax], hi = a[0][ax];
            for (int i = 1; i < 4; ++i) {
                if (a[i][ax] < lo) lo = a[i][ax];
                if (a[i][ax] > hi) hi = a[i][ax];
            }
            double shift[4] = {0.0, 0.0, 0.0, 0.0};
            for (int i = 0; i < 4; ++i) {
                if (a[i][ax] == lo) shift[i] -= 0.5 * ORC_AA_SIZE;
                if (a[i][ax] == hi) shift[i] += 0.5 * ORC_AA_SIZE;
            }
            for (int i = 0; i < 4; ++i) a[i][ax] += shift[i];
        }
    }
}

/* Sec. 3.2 "Preprocessing": build the primitive, transform it to the camera,
 * colour it from the viewing direction, project it into ray space and bound
 * it on screen. */
static void preprocess_one(const orc_scene *S, const orc_view *V, int64_t n, orc_prep *P)
{
    memset(P, 0, sizeof(*P));
    const double *mu = S->means + 3 * n;
    const double *d = S->dists + S->nd * n;
    const double alpha = S->opac[n];
    double R[3][3];
    if (!quat_rotation(S->quats + 4 * n, R)) return;
    for (int k = 0; k < S->nd; ++k)
        if (!(d[k] > 0.0) || !isfinite(d[k])) return;
    if (!isfinite(mu[0]) || !isfinite(mu[1]) || !isfinite(mu[2])) return;
    if (!(alpha >= 0.0 && alpha <= 1.0)) return;

    /* world -> camera */
    double tc[3];
    for (int r = 0; r < 3; ++r)
        tc[r] = V->Rw[r][0] * mu[0] + V->Rw[r][1] * mu[1] + V->Rw[r][2] * mu[2] + V->tw[r];
    if (!(tc[2] > V->near_z)) return;

    double o[4][3], oc[4][3];
    world_offsets(S->type, R, d, o);
    const int na = (S->type == ORC_OCTA) ? 3 : 4;
    for (int k = 0; k < na; ++k) mat3_vec(V->Rw, o[k], oc[k]);
    memcpy(P->oc, oc, sizeof(oc));

    /* ray space: centre c = phi(tc), offsets a_k = J(tc) * oc_k */
    const double iz = 1.0 / tc[2];
    const double px = V->fx * tc[0] * iz, py = V->fy * tc[1] * iz;
    const double cxp = px + V->cx, cyp = py + V->cy;
    const double J00 = V->fx * iz, J02 = -(px * iz), J11 = V->fy * iz, J12 = -(py * iz);
    const double l = sqrt(tc[0] * tc[0] + tc[1] * tc[1] + tc[2] * tc[2]);
    P->tc[0] = tc[0]; P->tc[1] = tc[1]; P->tc[2] = tc[2];
    P->c[0] = cxp; P->c[1] = cyp; P->c[2] = l;
    for (int k = 0; k < na; ++k) {
        P->a[k][0] = J00 * oc[k][0] + J02 * oc[k][2];
        P->a[k][1] = J11 * oc[k][1] + J12 * oc[k][2];
        P->a[k][2] = tc[0] / l * oc[k][0] + tc[1] / l * oc[k][1] + tc[2] / l * oc[k][2];
    }
    if (S->aa) antialias_shift(S->type, P->a);
    double xmin = INFINITY, xmax = -INFINITY, ymin = INFINITY, ymax = -INFINITY;
    for (int k = 0; k < na; ++k) {
        const double ax = P->a[k][0], ay = P->a[k][1];
        /* corners: c + a_k, and for the octahedron also c - a_k */
        const double xs[2] = {cxp + ax, cxp - ax}, ys[2] = {cyp + ay, cyp - ay};
        const int nsign = (S->type == ORC_OCTA) ? 2 : 1;
        for (int s = 0; s < nsign; ++s) {
            if (xs[s] < xmin) xmin = xs[s];
            if (xs[s] > xmax) xmax = xs[s];
            if (ys[s] < ymin) ymin = ys[s];
            if (ys[s] > ymax) ymax = ys[s];
        }
    }
    if (S->exact) {
        /* Without the ray-space approximation the footprint is the
         * perspective projection of the corners themselves.  A corner at or
         * behind the near plane has no projection, so such a primitive is
         * culled; otherwise every point of it lies in front of the camera and
         * each pixel ray meets it at positive depth only. */
        const int nc = (S->type == ORC_OCTA) ? 6 : 4;
        for (int k = 0; k < nc; ++k)
            for (int r = 0; r < 3; ++r) {
                if (S->type == ORC_OCTA)
                    P->vc[k][r] = (k & 1) ? tc[r] - oc[k >> 1][r] : tc[r] + oc[k >> 1][r];
                else
                    P->vc[k][r] = tc[r] + oc[k][r];
            }
        xmin = INFINITY; xmax = -INFINITY; ymin = INFINITY; ymax = -INFINITY;
        for (int k = 0; k < nc; ++k) {
            if (!(P->vc[k][2] > V->near_z)) return;
            const double xp = V->fx * P->vc[k][0] / P->vc[k][2] + V->cx;
            const double yp = V->fy * P->vc[k][1] / P->vc[k][2] + V->cy;
            if (xp < xmin) xmin = xp;
            if (xp > xmax) xmax = xp;
            if (yp < ymin) ymin = yp;
            if (yp > ymax) ymax = yp;
        }
    }
    if (!isfinite(xmin) || !isfinite(xmax) || !isfinite(ymin) || !isfinite(ymax)) return;
    P->radius = 0.5 * fmax(xmax - xmin, ymax - ymin);

    /* projected bounding box -> pixel rectangle (centres inside the box) */
    double fi0 = ceil(xmin - 0.5), fi1 = floor(xmax - 0.5);
    double fj0 = ceil(ymin - 0.5), fj1 = floor(ymax - 0.5);
    if (fi0 < 0.0) fi0 = 0.0;
    if (fj0 < 0.0) fj0 = 0.0;
    if (fi1 > (double)(V->W - 1)) fi1 = (double)(V->W - 1);
    if (fj1 > (double)(V->H - 1)) fj1 = (double)(V->H - 1);
    if (fi0 > fi1 || fj0 > fj1) return;
    P->rect[0] = (int)fi0; P->rect[1] = (int)fj0; P->rect[2] = (int)fi1; P->rect[3] = (int)fj1;
    const int T = S->tile;
    P->trect[0] = P->rect[0] / T; P->trect[1] = P->rect[1] / T;
    P->trect[2] = P->rect[2] / T; P->trect[3] = P->rect[3] / T;
    P->tiles = (int64_t)(P->trect[2] - P->trect[0] + 1) * (int64_t)(P->trect[3] - P->trect[1] + 1);
    const float zf = (float)tc[2];
    memcpy(&P->key, &zf, 4);

    /* Eq. 1: density from opacity and the smallest distance */
    double dmin = d[0];
    for (int k = 1; k < S->nd; ++k) if (d[k] < dmin) dmin = d[k];
    P->sigma = -log(1.0 - ORC_ALPHA_SCALE * alpha) / (2.0 * dmin);

    /* view-dependent colour from the SH (degree S->deg) */
    double cam[3], dir[3], Y[16];
    mat3T_vec(V->Rw, V->tw, cam);
    for (int k = 0; k < 3; ++k) dir[k] = mu[k] + cam[k];   /* mu - (-Rw^T t) */
    const double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
    for (int k = 0; k < 3; ++k) dir[k] /= dn;
    orc_sh_basis(S->deg, dir, Y);
    const double *sh = S->sh + (int64_t)48 * n;
    for (int ch = 0; ch < 3; ++ch) {
        double acc = 0.0;
        for (int k = 0; k < S->K; ++k) acc += sh[3 * k + ch] * Y[k];
        P->raw[ch] = acc + 0.5;
        P->rgb[ch] = P->raw[ch] > 0.0 ? P->raw[ch] : 0.0;
    }
    P->valid = 1;
}

/* ------------------------------------------------------------------------ */
/* Ray-triangle intersection (Sec. 3.2 "Rasterization", Moeller-Trumbore).  */
/* Pixel rays in ray space start at (rx, ry, 0) and run along +z.           */
/* ------------------------------------------------------------------------ */
typedef struct {
    int hit;
    double t, u, v, det;
} orc_hit;

static orc_hit mtia(const double V0[3], const double V1[3], const double V2[3], double rx, double ry)
{
    orc_hit H = {0, 0, 0, 0, 0};
    const double e1[3] = {V1[0] - V0[0], V1[1] - V0[1], V1[2] - V0[2]};
    const double e2[3] = {V2[0] - V0[0], V2[1] - V0[1], V2[2] - V0[2]};
    const double h[3] = {-e2[1], e2[0], 0.0};                 /* D x e2, D = (0,0,1) */
    const double a = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
    if (a == 0.0) return H;
    const double f = 1.0 / a;
    const double s[3] = {rx - V0[0], ry - V0[1], -V0[2]};
    const double u = f * (s[0] * h[0] + s[1] * h[1] + s[2] * h[2]);
    if (u < 0.0 || u > 1.0) return H;
    const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    const double v = f * q[2];                                /* D . q */
    if (v < 0.0 || u + v > 1.0) return H;
    H.hit = 1;
    H.t = f * (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]);
    H.u = u; H.v = v; H.det = a;
    return H;
}

/* App. E: derivatives of the intersection depth i with respect to the three
 * ray-space triangle corners.  dV[j][k] = d i / d V_j[k].  The paper prints
 * the V0 barycentric derivatives; those for V1 and V2 are derived the same
 * way from the Moeller-Trumbore expressions. */
static void mtia_depth_grad(const double V0[3], const double V1[3], const double V2[3],
                            double rx, double ry, const orc_hit *H, double dV[3][3])
{
    const double d = H->det, u = H->u, v = H->v;
    const double s[2] = {rx - V0[0], ry - V0[1]};
    const double e1[2] = {V1[0] - V0[0], V1[1] - V0[1]};
    const double e2[2] = {V2[0] - V0[0], V2[1] - V0[1]};
    double du[3][2], dv[3][2];
    /* corner 0, as printed in App. E */
    du[0][0] = ((V2[1] - ry) - u * (V2[1] - V1[1])) / d;
    du[0][1] = ((rx - V2[0]) - u * (V1[0] - V2[0])) / d;
    dv[0][0] = ((ry - V1[1]) - v * (V2[1] - V1[1])) / d;
    dv[0][1] = ((V1[0] - rx) - v * (V1[0] - V2[0])) / d;
    /* corner 1: only e1 depends on V1 */
    du[1][0] = u * e2[1] / d;
    du[1][1] = -u * e2[0] / d;
    dv[1][0] = (-s[1] + v * e2[1]) / d;
    dv[1][1] = (s[0] - v * e2[0]) / d;
    /* corner 2: only e2 depends on V2 */
    du[2][0] = (s[1] - u * e1[1]) / d;
    du[2][1] = (-s[0] + u * e1[0]) / d;
    dv[2][0] = -v * e1[1] / d;
    dv[2][1] = v * e1[0] / d;
    const double w[3] = {1.0 - u - v, u, v};
    for (int j = 0; j < 3; ++j) {
        for (int k = 0; k < 2; ++k)
            dV[j][k] = -(du[j][k] + dv[j][k]) * V0[2] + du[j][k] * V1[2] + dv[j][k] * V2[2];
        dV[j][2] = w[j];
    }
}

/* Faces of a primitive as corner index triples into the corner list:
 * octahedron corners (c+a0, c-a0, c+a1, c-a1, c+a2, c-a2), face f uses sign
 * bits of f for the x, y, z axes; tetrahedron corners c+a_i, face f is made
 * of the three corners other than f. */
static int prim_faces(int type, int F[8][3])
{
    if (type == ORC_OCTA) {
        for (int f = 0; f < 8; ++f) {
            F[f][0] = 0 + ((f >> 0) & 1);
            F[f][1] = 2 + ((f >> 1) & 1);
            F[f][2] = 4 + ((f >> 2) & 1);
        }
        return 8;
    }
    for (int f = 0; f < 4; ++f) {
        int m = 0;
        for (int i = 0; i < 4; ++i) if (i != f) F[f][m++] = i;
    }
    return 4;
}

static int prim_corners(int type, const orc_prep *P, double Vc[6][3])
{
    if (type == ORC_OCTA) {
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) {
                Vc[2 * k][r] = P->c[r] + P->a[k][r];
                Vc[2 * k + 1][r] = P->c[r] - P->a[k][r];
            }
        return 6;
    }
    for (int i = 0; i < 4; ++i)
        for (int r = 0; r < 3; ++r) Vc[i][r] = P->c[r] + P->a[i][r];
    return 4;
}

typedef struct {
    double delta;          /* chord length i2 - i1 (0 if fewer than two hits) */
    int nhit;
    int f_in, f_out;       /* entry / exit face index (first in face order on ties) */
    orc_hit h_in, h_out;
} orc_chord_t;

/* Chord through the primitive along the pixel ray by per-face MTIA: the
 * entry depth i1 is the smallest and the exit depth i2 the largest hit. */
static orc_chord_t chord_mtia(int type, const orc_prep *P, double rx, double ry)
{
    orc_chord_t C;
    memset(&C, 0, sizeof(C));
    C.f_in = C.f_out = -1;
    double Vc[6][3];
    int F[8][3];
    prim_corners(type, P, Vc);
    const int nf = prim_faces(type, F);
    for (int f = 0; f < nf; ++f) {
        orc_hit H = mtia(Vc[F[f][0]], Vc[F[f][1]], Vc[F[f][2]], rx, ry);
        if (!H.hit) continue;
        if (C.nhit == 0 || H.t < C.h_in.t) { C.h_in = H; C.f_in = f; }
        if (C.nhit == 0 || H.t > C.h_out.t) { C.h_out = H; C.f_out = f; }
        C.nhit++;
    }
    C.delta = (C.nhit >= 1) ? (C.h_out.t - C.h_in.t) : 0.0;
    return C;
}

/* Independent chord formulation used only to cross-check chord_mtia:
 * octahedron: points c + M s with |s|_1 <= 1; along the ray s(z) = s0 + z m and
 * the chord is the measure of {z : sum_k |s0_k + z m_k| <= 1}, found from the
 * breakpoints of the piecewise-linear convex function.
 * tetrahedron: barycentric coordinates are affine in z; clip the interval
 * where all four are non-negative (Cyrus-Beck). */
static int solve3(const double A[3][3], const double b[3], double x[3])
{
    double M[3][4];
    for (int r = 0; r < 3; ++r) { for (int c = 0; c < 3; ++c) M[r][c] = A[r][c]; M[r][3] = b[r]; }
    for (int c = 0; c < 3; ++c) {
        int p = c;
        for (int r = c + 1; r < 3; ++r) if (fabs(M[r][c]) > fabs(M[p][c])) p = r;
        if (M[p][c] == 0.0) return 0;
        if (p != c) for (int k = 0; k < 4; ++k) { double t = M[c][k]; M[c][k] = M[p][k]; M[p][k] = t; }
        for (int r = 0; r < 3; ++r) {
            if (r == c) continue;
            const double f = M[r][c] / M[c][c];
            for (int k = c; k < 4; ++k) M[r][k] -= f * M[c][k];
        }
    }
    for (int r = 0; r < 3; ++r) x[r] = M[r][3] / M[r][r];
    return 1;
}

static double l1_of(const double s0[3], const double m[3], double z)
{
    return fabs(s0[0] + z * m[0]) + fabs(s0[1] + z * m[1]) + fabs(s0[2] + z * m[2]);
}

/* Length of the interval of z where |s0 + z m|_1 <= 1 (a convex piecewise
 * linear function): from its smallest breakpoint value walk outwards to the
 * two crossings of 1. */
static double l1_chord(const double s0[3], const double m[3])
{
    double bp[3];
    int nb = 0;
    for (int k = 0; k < 3; ++k) if (m[k] != 0.0) bp[nb++] = -s0[k] / m[k];
    /* sort breakpoints */
    for (int i = 0; i < nb; ++i)
        for (int j = i + 1; j < nb; ++j) if (bp[j] < bp[i]) { double t = bp[i]; bp[i] = bp[j]; bp[j] = t; }
    int best = 0;
    for (int i = 1; i < nb; ++i) if (l1_of(s0, m, bp[i]) < l1_of(s0, m, bp[best])) best = i;
    const double zb = bp[best], fb = l1_of(s0, m, zb);
    if (fb > 1.0) return 0.0;
    /* walk right from the minimum to the crossing f = 1 */
    double hi;
    {
        double z0 = zb, f0 = fb;
        int i = best + 1;
        for (;;) {
            if (i < nb) {
                const double f1 = l1_of(s0, m, bp[i]);
                if (f1 > 1.0) { hi = z0 + (1.0 - f0) * (bp[i] - z0) / (f1 - f0); break; }
                z0 = bp[i]; f0 = f1; ++i;
            } else {
                const double slope = fabs(m[0]) + fabs(m[1]) + fabs(m[2]);
                hi = z0 + (1.0 - f0) / slope;
                break;
            }
        }
    }
    double lo;
    {
        double z0 = zb, f0 = fb;
        int i = best - 1;
        for (;;) {
            if (i >= 0) {
                const double f1 = l1_of(s0, m, bp[i]);
                if (f1 > 1.0) { lo = z0 - (1.0 - f0) * (z0 - bp[i]) / (f1 - f0); break; }
                z0 = bp[i]; f0 = f1; --i;
            } else {
                const double slope = fabs(m[0]) + fabs(m[1]) + fabs(m[2]);
                lo = z0 - (1.0 - f0) / slope;
                break;
            }
        }
    }
    return hi - lo;
}

/* Length of the interval of z where every barycentric coordinate
 * lam0_i + z lam1_i is non-negative (Cyrus-Beck). */
static double bary_chord(const double lam0[4], const double lam1[4])
{
    double zlo = -INFINITY, zhi = INFINITY;
    for (int i = 0; i < 4; ++i) {
        if (lam1[i] > 0.0) { const double z = -lam0[i] / lam1[i]; if (z > zlo) zlo = z; }
        else if (lam1[i] < 0.0) { const double z = -lam0[i] / lam1[i]; if (z < zhi) zhi = z; }
        else if (lam0[i] < 0.0) return 0.0;
    }
    return (zhi > zlo) ? (zhi - zlo) : 0.0;
}

/* Interval length along the line p0 + z dir through the primitive with
 * centre c and offsets a (octahedron: c + [a0 a1 a2] s, |s|_1 <= 1;
 * tetrahedron: corners c + a_i). */
static double clip_line(int type, const double c[3], const double a[4][3], const double b0[3],
                        const double dir[3])
{
    if (type == ORC_OCTA) {
        double M[3][3];
        for (int r = 0; r < 3; ++r) for (int k = 0; k < 3; ++k) M[r][k] = a[k][r];
        double s0[3], m[3];
        if (!solve3(M, b0, s0) || !solve3(M, dir, m)) return 0.0;
        return l1_chord(s0, m);
    }
    /* corners V_i = c + a_i; barycentrics lambda solve sum_i lambda_i V_i = X,
     * sum_i lambda_i = 1.  Use lambda_1..3 from the 3x3 system with V_0 as
     * origin, lambda_0 = 1 - sum.  b0 is the line origin relative to c. */
    double E[3][3];
    for (int r = 0; r < 3; ++r) for (int k = 0; k < 3; ++k) E[r][k] = a[k + 1][r] - a[0][r];
    const double rel[3] = {b0[0] - a[0][0], b0[1] - a[0][1], b0[2] - a[0][2]};
    double l0[3], l1[3];
    if (!solve3(E, rel, l0) || !solve3(E, dir, l1)) return 0.0;
    const double lam0[4] = {1.0 - l0[0] - l0[1] - l0[2], l0[0], l0[1], l0[2]};
    const double lam1[4] = {-l1[0] - l1[1] - l1[2], l1[0], l1[1], l1[2]};
    (void)c;
    return bary_chord(lam0, lam1);
}

static double chord_clip(int type, const orc_prep *P, double rx, double ry)
{
    const double ez[3] = {0.0, 0.0, 1.0};
    if (type == ORC_OCTA) {
        const double b0[3] = {rx - P->c[0], ry - P->c[1], 0.0};
        return clip_line(type, P->c, P->a, b0, ez);
    }
    const double b0[3] = {rx - P->c[0], ry - P->c[1], -P->c[2]};
    return clip_line(type, P->c, P->a, b0, ez);
}

/* ------------------------------------------------------------------------ */
/* Exact variant (appendix "Ray Space Approximation"): no affine ray space.  */
/* The pixel ray leaves the camera centre along                              */
/* D = ((px - cx) / fx, (py - cy) / fy, 1) and crosses the camera-space      */
/* primitive; the chord is the Euclidean length of the segment inside it.    */
/* ------------------------------------------------------------------------ */
static void pixel_ray(const orc_view *V, double px, double py, double D[3])
{
    D[0] = (px - V->cx) / V->fx;
    D[1] = (py - V->cy) / V->fy;
    D[2] = 1.0;
}

static double norm3(const double v[3]) { return sqrt(v[0] * v[0] + v[1] * v[1] + v[2] * v[2]); }

/* Moeller-Trumbore for the ray t D (t real) from the camera centre; the hit
 * parameter t is also the hit's camera z because D_z = 1. */
static orc_hit mtia_ray(const double V0[3], const double V1[3], const double V2[3], const double D[3])
{
    orc_hit H = {0, 0, 0, 0, 0};
    const double e1[3] = {V1[0] - V0[0], V1[1] - V0[1], V1[2] - V0[2]};
    const double e2[3] = {V2[0] - V0[0], V2[1] - V0[1], V2[2] - V0[2]};
    const double h[3] = {D[1] * e2[2] - D[2] * e2[1], D[2] * e2[0] - D[0] * e2[2], D[0] * e2[1] - D[1] * e2[0]};
    const double a = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
    if (a == 0.0) return H;
    const double f = 1.0 / a;
    const double s[3] = {-V0[0], -V0[1], -V0[2]};              /* ray origin (0,0,0) - V0 */
    const double u = f * (s[0] * h[0] + s[1] * h[1] + s[2] * h[2]);
    if (u < 0.0 || u > 1.0) return H;
    const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
    const double v = f * (D[0] * q[0] + D[1] * q[1] + D[2] * q[2]);
    if (v < 0.0 || u + v > 1.0) return H;
    H.hit = 1;
    H.t = f * (e2[0] * q[0] + e2[1] * q[1] + e2[2] * q[2]);
    H.u = u; H.v = v; H.det = a;
    return H;
}

static orc_chord_t chord_mtia_exact(int type, const orc_prep *P, const double D[3])
{
    orc_chord_t C;
    memset(&C, 0, sizeof(C));
    C.f_in = C.f_out = -1;
    int F[8][3];
    const int nf = prim_faces(type, F);
    for (int f = 0; f < nf; ++f) {
        orc_hit H = mtia_ray(P->vc[F[f][0]], P->vc[F[f][1]], P->vc[F[f][2]], D);
        if (!H.hit) continue;
        if (C.nhit == 0 || H.t < C.h_in.t) { C.h_in = H; C.f_in = f; }
        if (C.nhit == 0 || H.t > C.h_out.t) { C.h_out = H; C.f_out = f; }
        C.nhit++;
    }
    C.delta = (C.nhit >= 1) ? (C.h_out.t - C.h_in.t) * norm3(D) : 0.0;
    return C;
}

/* How far the pixel ray passes inside (> 0) or outside (< 0) the nearest
 * face, in barycentric units: the largest over the faces of
 * min(u, v, 1 - u - v), with the Moeller-Trumbore algebra of the two chord
 * routines but without their early exits.  Ray space: origin (rx, ry, 0),
 * direction +z; exact variant (D != NULL): origin 0, direction D. */
static double bary_margin(int type, const orc_prep *P, double rx, double ry, const double *D)
{
    double Vc[6][3];
    int F[8][3];
    const double dz[3] = {0.0, 0.0, 1.0};
    const double *dir = D ? D : dz;
    const double org[3] = {D ? 0.0 : rx, D ? 0.0 : ry, 0.0};
    if (D) memcpy(Vc, P->vc, sizeof(Vc));
    else prim_corners(type, P, Vc);
    const int nf = prim_faces(type, F);
    double best = -HUGE_VAL;
    for (int f = 0; f < nf; ++f) {
        const double *V0 = Vc[F[f][0]], *V1 = Vc[F[f][1]], *V2 = Vc[F[f][2]];
        const double e1[3] = {V1[0] - V0[0], V1[1] - V0[1], V1[2] - V0[2]};
        const double e2[3] = {V2[0] - V0[0], V2[1] - V0[1], V2[2] - V0[2]};
        const double h[3] = {dir[1] * e2[2] - dir[2] * e2[1], dir[2] * e2[0] - dir[0] * e2[2],
                             dir[0] * e2[1] - dir[1] * e2[0]};
        const double a = e1[0] * h[0] + e1[1] * h[1] + e1[2] * h[2];
        if (a == 0.0) continue;
        const double s[3] = {org[0] - V0[0], org[1] - V0[1], org[2] - V0[2]};
        const double u = (s[0] * h[0] + s[1] * h[1] + s[2] * h[2]) / a;
        const double q[3] = {s[1] * e1[2] - s[2] * e1[1], s[2] * e1[0] - s[0] * e1[2], s[0] * e1[1] - s[1] * e1[0]};
        const double v = (dir[0] * q[0] + dir[1] * q[1] + dir[2] * q[2]) / a;
        const double b = fmin(fmin(u, v), 1.0 - u - v);
        if (b > best) best = b;
    }
    return best;
}

/* Independent formulation of the exact chord: the same clipping as
 * chord_clip along the line t D in camera space. */
static double chord_clip_exact(int type, const orc_prep *P, const double D[3])
{
    const double b0[3] = {-P->tc[0], -P->tc[1], -P->tc[2]};
    return clip_line(type, P->tc, P->oc, b0, D) * norm3(D);
}

/* App. E's rule for a general ray direction: moving corner j of the hit
 * triangle by dV moves the hit parameter by w_j (n . dV) / (n . D), with w
 * the hit's barycentric weights (1 - u - v, u, v) and n the face normal. */
static void mtia_ray_grad(const double V0[3], const double V1[3], const double V2[3], const double D[3],
                          const orc_hit *H, double dV[3][3])
{
    const double e1[3] = {V1[0] - V0[0], V1[1] - V0[1], V1[2] - V0[2]};
    const double e2[3] = {V2[0] - V0[0], V2[1] - V0[1], V2[2] - V0[2]};
    const double n[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
    const double nd = n[0] * D[0] + n[1] * D[1] + n[2] * D[2];
    const double w[3] = {1.0 - H->u - H->v, H->u, H->v};
    for (int j = 0; j < 3; ++j)
        for (int r = 0; r < 3; ++r) dV[j][r] = w[j] * n[r] / nd;
}

/* ------------------------------------------------------------------------ */
/* Scene object and the ctypes-facing API.                                  */
/* ------------------------------------------------------------------------ */
void *orc_new(int type, int sh_degree, int64_t n, const double *means, const double *quats,
              const double *dists, const double *opacity, const double *sh)
{
    if ((type != ORC_OCTA && type != ORC_TETRA) || sh_degree < 0 || sh_degree > 3 || n < 0) return NULL;
    orc_scene *S = (orc_scene *)calloc(1, sizeof(orc_scene));
    S->type = type;
    S->deg = sh_degree;
    S->K = (sh_degree + 1) * (sh_degree + 1);
    S->nd = (type == ORC_OCTA) ? 3 : 4;
    S->n = n;
    const size_t nn = (size_t)(n > 0 ? n : 1);
    S->means = (double *)malloc(sizeof(double) * 3 * nn);
    S->quats = (double *)malloc(sizeof(double) * 4 * nn);
    S->dists = (double *)malloc(sizeof(double) * S->nd * nn);
    S->opac = (double *)malloc(sizeof(double) * nn);
    S->sh = (double *)malloc(sizeof(double) * 48 * nn);
    memcpy(S->means, means, sizeof(double) * 3 * n);
    memcpy(S->quats, quats, sizeof(double) * 4 * n);
    memcpy(S->dists, dists, sizeof(double) * S->nd * n);
    memcpy(S->opac, opacity, sizeof(double) * n);
    memcpy(S->sh, sh, sizeof(double) * 48 * n);
    return S;
}

static void free_views(orc_scene *S)
{
    free(S->prep); S->prep = NULL;
    free(S->keys); S->keys = NULL;
    free(S->vals); S->vals = NULL;
    free(S->rlo); S->rlo = NULL;
    free(S->sgrad); S->sgrad = NULL;
    free(S->rhi); S->rhi = NULL;
    S->n_pairs = 0;
}

void orc_free(void *h)
{
    orc_scene *S = (orc_scene *)h;
    if (!S) return;
    free_views(S);
    free(S->means); free(S->quats); free(S->dists); free(S->opac); free(S->sh);
    free(S);
}

/* cams: n_views rows of 20 doubles:
 * [Rw (9, row-major) interleaved with t as a 3x4 row-major matrix (12)],
 * fx, fy, cx, cy, W, H, near, (unused). */
int orc_set_views(void *h, int n_views, const double *cams, int tile)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || n_views < 1 || n_views > ORC_MAX_VIEWS || tile < 1) return -1;
    free_views(S);
    S->n_views = n_views;
    S->tile = tile;
    int64_t tb = 0, pb = 0;
    for (int v = 0; v < n_views; ++v) {
        const double *c = cams + 20 * v;
        orc_view *V = &S->views[v];
        for (int r = 0; r < 3; ++r) {
            for (int k = 0; k < 3; ++k) V->Rw[r][k] = c[4 * r + k];
            V->tw[r] = c[4 * r + 3];
        }
        V->fx = c[12]; V->fy = c[13]; V->cx = c[14]; V->cy = c[15];
        V->W = (int)c[16]; V->H = (int)c[17]; V->near_z = c[18];
        if (V->W < 1 || V->H < 1) return -1;
        V->tiles_x = (V->W + tile - 1) / tile;
        V->tiles_y = (V->H + tile - 1) / tile;
        V->tile_base = tb;
        V->pix_base = pb;
        tb += (int64_t)V->tiles_x * V->tiles_y;
        pb += (int64_t)V->W * V->H;
    }
    S->n_tiles_total = tb;
    S->prep = (orc_prep *)calloc((size_t)n_views * (size_t)(S->n > 0 ? S->n : 1), sizeof(orc_prep));
    return 0;
}

/* Selects the 2D anti-aliasing filter for the following orc_preprocess
 * (ray space only). */
int orc_set_antialias(void *h, int aa)
{
    orc_scene *S = (orc_scene *)h;
    if (!S) return -1;
    S->aa = aa ? 1 : 0;
    return 0;
}

/* Selects the chord model for the following orc_preprocess: 0 = EWA ray
 * space (Sec. 3.2), 1 = exact pixel rays in camera space. */
int orc_set_exact(void *h, int exact)
{
    orc_scene *S = (orc_scene *)h;
    if (!S) return -1;
    S->exact = exact ? 1 : 0;
    return 0;
}

int orc_preprocess(void *h)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep) return -1;
    for (int v = 0; v < S->n_views; ++v) {
        orc_prep *Pv = S->prep + (int64_t)v * S->n;
#pragma omp parallel for schedule(static)
        for (int64_t n = 0; n < S->n; ++n) preprocess_one(S, &S->views[v], n, Pv + n);
    }
    return 0;
}

/* Copy per-primitive results of one view out.  Culled primitives have
 * rect = (-1,-1,-1,-1), tiles = 0, key = 0. */
int orc_get_prep(void *h, int v, int32_t *rect, int64_t *tiles, uint32_t *key, double *tc,
                 double *c, double *a, double *sigma, double *rgb, double *raw)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || v < 0 || v >= S->n_views) return -1;
    const orc_prep *Pv = S->prep + (int64_t)v * S->n;
    for (int64_t n = 0; n < S->n; ++n) {
        const orc_prep *P = Pv + n;
        for (int k = 0; k < 4; ++k) rect[4 * n + k] = P->valid ? P->rect[k] : -1;
        tiles[n] = P->valid ? P->tiles : 0;
        key[n] = P->valid ? P->key : 0;
        for (int k = 0; k < 3; ++k) {
            tc[3 * n + k] = P->tc[k];
            c[3 * n + k] = P->c[k];
            rgb[3 * n + k] = P->rgb[k];
            raw[3 * n + k] = P->raw[k];
        }
        for (int k = 0; k < 12; ++k) a[12 * n + k] = P->a[k / 3][k % 3];
        sigma[n] = P->sigma;
    }
    return 0;
}

/* Sec. 3.2 "Global Sorting and Tiling": one (key, value) pair per primitive
 * and tile it touches, key = global tile id << 32 | depth bits, value =
 * primitive index; pairs are emitted view by view, primitive by primitive,
 * tiles in row-major order, and sorted by key with ties kept in emission
 * order. */
typedef struct { uint64_t key; uint64_t seq; uint32_t val; } orc_pair;

static int cmp_pair(const void *pa, const void *pb)
{
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    if (a->key != b->key) return a->key < b->key ? -1 : 1;
    if (a->seq != b->seq) return a->seq < b->seq ? -1 : 1;
    return 0;
}

int orc_sort(void *h)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep) return -1;
    int64_t np = 0;
    for (int v = 0; v < S->n_views; ++v)
        for (int64_t n = 0; n < S->n; ++n) {
            const orc_prep *P = S->prep + (int64_t)v * S->n + n;
            if (P->valid) np += P->tiles;
        }
    orc_pair *pairs = (orc_pair *)malloc(sizeof(orc_pair) * (size_t)(np > 0 ? np : 1));
    int64_t e = 0;
    for (int v = 0; v < S->n_views; ++v) {
        const orc_view *V = &S->views[v];
        for (int64_t n = 0; n < S->n; ++n) {
            const orc_prep *P = S->prep + (int64_t)v * S->n + n;
            if (!P->valid) continue;
            for (int ty = P->trect[1]; ty <= P->trect[3]; ++ty)
                for (int tx = P->trect[0]; tx <= P->trect[2]; ++tx) {
                    const uint64_t g = (uint64_t)(V->tile_base + (int64_t)ty * V->tiles_x + tx);
                    pairs[e].key = (g << 32) | (uint64_t)P->key;
                    pairs[e].seq = (uint64_t)e;
                    pairs[e].val = (uint32_t)n;
                    ++e;
                }
        }
    }
    qsort(pairs, (size_t)np, sizeof(orc_pair), cmp_pair);
    free(S->keys); free(S->vals); free(S->rlo); free(S->rhi);
    S->n_pairs = np;
    S->keys = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(np > 0 ? np : 1));
    S->vals = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)(np > 0 ? np : 1));
    for (int64_t i = 0; i < np; ++i) { S->keys[i] = pairs[i].key; S->vals[i] = pairs[i].val; }
    free(pairs);
    S->rlo = (int64_t *)malloc(sizeof(int64_t) * (size_t)S->n_tiles_total);
    S->rhi = (int64_t *)malloc(sizeof(int64_t) * (size_t)S->n_tiles_total);
    for (int64_t t = 0; t < S->n_tiles_total; ++t) { S->rlo[t] = 0; S->rhi[t] = 0; }
    for (int64_t i = 0; i < np; ++i) {
        const int64_t g = (int64_t)(S->keys[i] >> 32);
        if (i == 0 || (int64_t)(S->keys[i - 1] >> 32) != g) S->rlo[g] = i;
        S->rhi[g] = i + 1;
    }
    return 0;
}

int64_t orc_num_pairs(void *h) { return h ? ((orc_scene *)h)->n_pairs : -1; }
int64_t orc_num_tiles(void *h) { return h ? ((orc_scene *)h)->n_tiles_total : -1; }

int orc_get_sort(void *h, uint64_t *keys, uint32_t *vals, int64_t *ranges)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->keys) return -1;
    memcpy(keys, S->keys, sizeof(uint64_t) * (size_t)S->n_pairs);
    memcpy(vals, S->vals, sizeof(uint32_t) * (size_t)S->n_pairs);
    for (int64_t t = 0; t < S->n_tiles_total; ++t) { ranges[2 * t] = S->rlo[t]; ranges[2 * t + 1] = S->rhi[t]; }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Per-pixel compositing (Sec. 3.2 "Rasterization" and "Compositing").      */
/* ------------------------------------------------------------------------ */
typedef struct {
    int64_t pos;       /* position in the tile list (or -1 in brute force) */
    int64_t prim;
    double delta, e, o, T;   /* T = transmittance in front of this primitive */
    int clamped;
    orc_chord_t ch;
} orc_step;

typedef struct {
    double rgb[3], T;
    int64_t last;
    int64_t iterated, evaluated, intersected;
    int ill;           /* ORC_BIT_* flags of the pixel's steps and decisions */
    double cond;       /* float32 error estimate of the pixel's value (sum of T_k est_k) */
    int64_t amb_k;     /* list index of the first step ending within 1e-6 of the threshold, or -1 */
    int64_t amb_hits;  /* evaluated primitives whose hit-or-miss decision is ambiguous */
    double depth;      /* depth of the primitive where cumulative opacity first exceeds 0.5 (0: never) */
    int depth_ill;     /* a step leaves T within 1e-6 of 0.5 (the crossing may move in float32) */
} orc_pix;

/* Appendix "Depth and Surface Reconstruction": a pixel's depth is the
 * distance along its viewing ray to the first primitive at which the
 * cumulative opacity 1 - T exceeds 0.5, i.e. to that primitive's entry hit.
 * In ray space the third coordinate is the distance from the camera (the
 * affine map of Sec. 3.2), so the distance is the entry hit's ray-space
 * depth; without the ray-space approximation it is the entry parameter
 * along the pixel ray D times |D|. */
#define ORC_DEPTH_T 0.5

static int in_rect(const orc_prep *P, int i, int j)
{
    return i >= P->rect[0] && i <= P->rect[2] && j >= P->rect[1] && j <= P->rect[3];
}

/* Conditioning flags of the parity contract: a float32 evaluation of the
 * same arithmetic may legitimately take a different discrete decision.
 *   bit 0: the pixel's value may differ beyond rounding (a step ends within
 *          1e-6 of the termination threshold, or an opacity sits within 1e-6
 *          of the clamp);
 *   bit 1: a primitive's own gradient may switch form (an active face within
 *          1e-5 barycentric of an edge, or the clamp);
 *   bit 2: a hit-or-miss decision may flip (the ray passes within 1e-5
 *          barycentric of the primitive's silhouette), which moves the last
 *          blended position and the intersected count but not the value
 *          beyond rounding (the chord vanishes there);
 *   bit 3: termination may move to a neighbouring step (subset of bit 0). */
#define ORC_BIT_VALUE 1
#define ORC_BIT_GRAD 2
#define ORC_BIT_HIT 4
#define ORC_BIT_TERM 8
/* bit 4 (a subset of bit 0): the float32 error estimate of the pixel's value
 * (the transmittance-weighted sum of its steps' opacity estimates) exceeds
 * the image tolerance, ORC_ILL_F32 */
#define ORC_BIT_F32 16
#define ORC_ILL_F32 1e-5

/* Flags of one blended step.  It also estimates the float32 error of the
 * step's opacity, from its active faces evaluated over the primitive's pixel
 * rectangle about the rectangle's centre: err_o (if not NULL) receives the
 * estimate, and cond (if not NULL) accumulates it weighted by the
 * transmittance in front of the step, a first-order bound on the error it
 * carries into the pixel's colour and transmittance. */
static int step_ill(int type, const orc_prep *P, const orc_step *st, double Tafter, double *cond,
                    const orc_view *V, const double *D, double *err_o)
{
    int ill = 0;
    if (fabs(Tafter - ORC_T_STOP) <= ORC_ILL_T) ill |= ORC_BIT_VALUE | ORC_BIT_TERM;
    if (fabs((1.0 - st->e) - ORC_O_MAX) <= ORC_ILL_O) ill |= ORC_BIT_VALUE | ORC_BIT_GRAD;
    const orc_hit *hs[2] = {&st->ch.h_in, &st->ch.h_out};
    double bmax = 0.0;
    for (int s = 0; s < 2; ++s) {
        const double b = fmin(fmin(hs[s]->u, hs[s]->v), 1.0 - hs[s]->u - hs[s]->v);
        if (b < ORC_ILL_BARY) ill |= ORC_BIT_GRAD;
        if (s == 0 || b > bmax) bmax = b;
    }
    /* both hits on an edge: the ray grazes the silhouette */
    if (bmax < ORC_ILL_BARY) ill |= ORC_BIT_HIT;
    int F[8][3];
    prim_faces(type, F);
    const int fs[2] = {st->ch.f_in, st->ch.f_out};
    /* half-extents of the pixel rectangle about its centre */
    const double hw = 0.5 * (double)(P->rect[2] - P->rect[0]), hh = 0.5 * (double)(P->rect[3] - P->rect[1]);
    double est = 0.0;
    if (D) {
        /* exact variant: the face plane in normal form about the primitive's
         * centre t_c, n.(X - t_c) = 1, meets the pixel ray X = z_c (1 + tau) D
         * at tau = (u + 1) / (c - u) with u = n.(t_c - z_c D), c = n.t_c;
         * u, evaluated in float32 about the rectangle's centre, errs by about
         * 2^-23 (|du/dx| hw + |du/dy| hh + |u at the centre|) and c by
         * 2^-23 |c|; tau and the chord z_c |D| (tau_out - tau_in) follow */
        const double zc = P->tc[2];
        double Dc[3];
        pixel_ray(V, 0.5 * (double)(P->rect[0] + P->rect[2]) + 0.5, 0.5 * (double)(P->rect[1] + P->rect[3]) + 0.5,
                  Dc);
        double err = 0.0;
        for (int s = 0; s < 2; ++s) {
            const double *A = P->vc[F[fs[s]][0]], *B = P->vc[F[fs[s]][1]], *C = P->vc[F[fs[s]][2]];
            double nv[3] = {(B[1] - A[1]) * (C[2] - A[2]) - (B[2] - A[2]) * (C[1] - A[1]),
                            (B[2] - A[2]) * (C[0] - A[0]) - (B[0] - A[0]) * (C[2] - A[2]),
                            (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0])};
            const double lev = nv[0] * (A[0] - P->tc[0]) + nv[1] * (A[1] - P->tc[1]) + nv[2] * (A[2] - P->tc[2]);
            if (lev == 0.0) continue;
            for (int r = 0; r < 3; ++r) nv[r] /= lev;
            const double c = nv[0] * P->tc[0] + nv[1] * P->tc[1] + nv[2] * P->tc[2];
            const double u = c - zc * (nv[0] * D[0] + nv[1] * D[1] + nv[2] * D[2]);
            const double uc = c - zc * (nv[0] * Dc[0] + nv[1] * Dc[1] + nv[2] * Dc[2]);
            const double den = c - u;
            if (den == 0.0) continue;
            const double du = fabs(zc * nv[0] / V->fx) * hw + fabs(zc * nv[1] / V->fy) * hh + fabs(uc);
            err += (fabs(c + 1.0) * du + fabs(u + 1.0) * fabs(c)) / (den * den);
        }
        est = P->sigma * st->e * zc * norm3(D) * err * 1.1920928955078125e-7;
    } else {
        /* a face plane z = z0 + a (x - xc) + b (y - yc) about the rectangle's
         * centre (xc, yc), evaluated in float32 over the rectangle, errs by
         * about 2^-23 (|a| hw + |b| hh + |z0 - l|) in depth (its coefficients
         * and its arithmetic rounded relative to the largest term); this
         * moves the opacity by sigma * e times that */
        double Vc[6][3], terms = 0.0;
        prim_corners(type, P, Vc);
        const double xc = 0.5 * (double)(P->rect[0] + P->rect[2]) + 0.5;
        const double yc = 0.5 * (double)(P->rect[1] + P->rect[3]) + 0.5;
        for (int s = 0; s < 2; ++s) {
            const double *A = Vc[F[fs[s]][0]], *B = Vc[F[fs[s]][1]], *C = Vc[F[fs[s]][2]];
            const double n0 = (B[1] - A[1]) * (C[2] - A[2]) - (B[2] - A[2]) * (C[1] - A[1]);
            const double n1 = (B[2] - A[2]) * (C[0] - A[0]) - (B[0] - A[0]) * (C[2] - A[2]);
            const double n2 = (B[0] - A[0]) * (C[1] - A[1]) - (B[1] - A[1]) * (C[0] - A[0]);
            if (n2 == 0.0) continue;
            const double a = -n0 / n2, b = -n1 / n2;
            const double z0 = A[2] + a * (xc - A[0]) + b * (yc - A[1]) - P->c[2];
            terms += fabs(a) * hw + fabs(b) * hh + fabs(z0);
        }
        est = P->sigma * st->e * terms * 1.1920928955078125e-7;
    }
    if (err_o) *err_o = est;
    if (cond) *cond += st->T * est;
    return ill;
}

/* Composite one pixel along an ordered list of primitives.  If steps != NULL
 * the blended steps are recorded (for the backward pass). */
static void composite(const orc_scene *S, int v, const int64_t *list, const int64_t *pos, int64_t len,
                      int i, int j, const double bg[3], int use_clip, orc_pix *out,
                      orc_step *steps, int64_t *nsteps, int64_t last_default, int64_t *amb, int64_t *namb)
{
    const orc_prep *Pv = S->prep + (int64_t)v * S->n;
    const double rx = i + 0.5, ry = j + 0.5;
    double D[3];
    pixel_ray(&S->views[v], rx, ry, D);
    double T = 1.0, C[3] = {0.0, 0.0, 0.0};
    int64_t last = last_default, it = 0, ev = 0, hit = 0, ns = 0, amb_k = -1, amb_hits = 0, na = 0;
    int ill = 0, depth_ill = 0;
    double cond = 0.0, depth = 0.0;
    for (int64_t k = 0; k < len; ++k) {
        ++it;
        const orc_prep *P = Pv + list[k];
        if (!in_rect(P, i, j)) continue;
        ++ev;
        orc_chord_t ch;
        double delta;
        if (use_clip) {
            memset(&ch, 0, sizeof(ch));
            delta = S->exact ? chord_clip_exact(S->type, P, D) : chord_clip(S->type, P, rx, ry);
        } else {
            ch = S->exact ? chord_mtia_exact(S->type, P, D) : chord_mtia(S->type, P, rx, ry);
            delta = ch.delta;
        }
        if (!(delta > 0.0)) {
            /* a miss that grazes the silhouette may be a hit in float32 */
            if (!use_clip && bary_margin(S->type, P, rx, ry, S->exact ? D : NULL) > -ORC_ILL_BARY) {
                ill |= ORC_BIT_HIT;
                ++amb_hits;
                if (amb) amb[na++] = list[k];
            }
            continue;
        }
        ++hit;
        const double e = exp(-P->sigma * delta);
        double o = 1.0 - e;
        int clamped = 0;
        if (o > ORC_O_MAX) { o = ORC_O_MAX; clamped = 1; }
        orc_step st;
        st.pos = pos ? pos[k] : -1;
        st.prim = list[k];
        st.delta = delta; st.e = e; st.o = o; st.T = T; st.clamped = clamped; st.ch = ch;
        for (int c = 0; c < 3; ++c) C[c] += T * o * P->rgb[c];
        const double Tbefore = T;
        T = T * (1.0 - o);
        if (Tbefore >= ORC_DEPTH_T && T < ORC_DEPTH_T)
            depth = S->exact ? ch.h_in.t * norm3(D) : ch.h_in.t;
        if (fabs(T - ORC_DEPTH_T) <= ORC_ILL_T) depth_ill = 1;
        if (!use_clip) {
            const int sill = step_ill(S->type, P, &st, T, &cond, &S->views[v], S->exact ? D : NULL, NULL);
            if ((sill & ORC_BIT_TERM) && amb_k < 0) amb_k = k;
            if (sill & ORC_BIT_HIT) ++amb_hits;
            ill |= sill;
        }
        if (steps) steps[ns] = st;
        ++ns;
        last = pos ? pos[k] + 1 : k + 1;
        if (T <= ORC_T_STOP) break;
    }
    if (cond > ORC_ILL_F32) ill |= ORC_BIT_VALUE | ORC_BIT_F32;
    for (int c = 0; c < 3; ++c) out->rgb[c] = C[c] + T * bg[c];
    out->T = T;
    out->last = last;
    out->depth = depth;
    out->depth_ill = depth_ill;
    out->iterated = it; out->evaluated = ev; out->intersected = hit;
    out->ill = ill;
    out->cond = cond;
    out->amb_k = amb_k;
    out->amb_hits = amb_hits;
    if (nsteps) *nsteps = ns;
    if (namb) *namb = na;
}

/* Build the per-pixel list: tiled (the sorted tile list, as the paper's
 * renderer walks it) or brute force (every primitive whose pixel rectangle
 * contains the pixel, ordered by (depth key, index)). */
static int cmp_keyidx(const void *pa, const void *pb)
{
    const uint64_t a = *(const uint64_t *)pa, b = *(const uint64_t *)pb;
    return (a > b) - (a < b);
}

static int64_t pixel_list(const orc_scene *S, int v, int i, int j, int brute, int64_t **list, int64_t **pos,
                          int64_t *cap, int64_t *start)
{
    const orc_view *V = &S->views[v];
    if (!brute) {
        const int64_t g = V->tile_base + (int64_t)(j / S->tile) * V->tiles_x + (i / S->tile);
        const int64_t lo = S->rlo[g], hi = S->rhi[g];
        const int64_t len = hi - lo;
        if (len > *cap) {
            *cap = len;
            *list = (int64_t *)realloc(*list, sizeof(int64_t) * (size_t)len);
            *pos = (int64_t *)realloc(*pos, sizeof(int64_t) * (size_t)len);
        }
        for (int64_t k = 0; k < len; ++k) { (*list)[k] = S->vals[lo + k]; (*pos)[k] = lo + k; }
        *start = lo;
        return len;
    }
    const orc_prep *Pv = S->prep + (int64_t)v * S->n;
    int64_t len = 0;
    for (int64_t n = 0; n < S->n; ++n) if (Pv[n].valid && in_rect(Pv + n, i, j)) ++len;
    if (len > *cap) {
        *cap = len;
        *list = (int64_t *)realloc(*list, sizeof(int64_t) * (size_t)len);
        *pos = (int64_t *)realloc(*pos, sizeof(int64_t) * (size_t)len);
    }
    /* depth keys are 32-bit and indices below 2^32: sort packed (key, index) */
    uint64_t *kk = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)(len > 0 ? len : 1));
    int64_t m = 0;
    for (int64_t n = 0; n < S->n; ++n)
        if (Pv[n].valid && in_rect(Pv + n, i, j)) kk[m++] = ((uint64_t)Pv[n].key << 32) | (uint64_t)n;
    qsort(kk, (size_t)len, sizeof(uint64_t), cmp_keyidx);
    for (int64_t k = 0; k < len; ++k) { (*list)[k] = (int64_t)(kk[k] & 0xffffffffull); (*pos)[k] = -1; }
    free(kk);
    *start = 0;
    return len;
}

/* Render every view.  mode 0: tiled walk with MTIA chords (the paper's
 * pipeline); mode 1: brute-force lists with MTIA chords; mode 2: tiled walk
 * with the independent clipping chord.  Outputs are packed view by view:
 * rgb [3,H,W], T [H,W], last [H,W] (one past the tile-list position of the
 * last blended primitive, or the tile's list start), ill [H,W], cond [H,W].
 * counts[6*v + 0..5] = iterated, evaluated, intersected, frustum, hit-or-miss
 * decisions that may flip in float32, pixels whose termination may move. */
static int render_rows(orc_scene *S, int mode, const double *bg, double *rgb, double *T, int64_t *last,
                       uint8_t *ill, double *cond, int64_t *counts, int band_j0, int band_j1);

int orc_render(void *h, int mode, const double *bg, double *rgb, double *T, int64_t *last,
               uint8_t *ill, double *cond, int64_t *counts)
{
    return render_rows((orc_scene *)h, mode, bg, rgb, T, last, ill, cond, counts, 0, 1 << 30);
}

/* orc_render restricted to the rows [j0, j1) of every view (the other
 * pixels of the outputs are left untouched); used to time a bounded
 * sample of a large workload. */
int orc_render_band(void *h, int mode, const double *bg, double *rgb, double *T, int64_t *last,
                    uint8_t *ill, double *cond, int64_t *counts, int j0, int j1)
{
    return render_rows((orc_scene *)h, mode, bg, rgb, T, last, ill, cond, counts, j0, j1);
}

static int render_rows(orc_scene *S, int mode, const double *bg, double *rgb, double *T, int64_t *last,
                       uint8_t *ill, double *cond, int64_t *counts, int band_j0, int band_j1)
{
    if (!S || !S->prep || (mode != 1 && !S->rlo)) return -1;
    const int brute = (mode == 1), clip = (mode == 2);
    int64_t rgb_base = 0;
    for (int v = 0; v < S->n_views; ++v) {
        const orc_view *V = &S->views[v];
        const int64_t HW = (int64_t)V->W * V->H;
        int64_t it = 0, ev = 0, hit = 0, fr = 0, ah = 0, at = 0;
        for (int64_t n = 0; n < S->n; ++n) fr += S->prep[(int64_t)v * S->n + n].valid;
#pragma omp parallel reduction(+ : it, ev, hit, ah, at)
        {
            int64_t *list = NULL, *pos = NULL, cap = 0, start = 0;
            const int jlo = band_j0 > 0 ? band_j0 : 0;
            const int jhi = band_j1 < V->H ? band_j1 : V->H;
#pragma omp for schedule(dynamic, 1)
            for (int j = jlo; j < jhi; ++j) {
                for (int i = 0; i < V->W; ++i) {
                    const int64_t len = pixel_list(S, v, i, j, brute, &list, &pos, &cap, &start);
                    orc_pix px;
                    composite(S, v, list, brute ? NULL : pos, len, i, j, bg + 3 * v, clip, &px, NULL, NULL, start, NULL, NULL);
                    const int64_t p = (int64_t)j * V->W + i;
                    for (int c = 0; c < 3; ++c) rgb[rgb_base + c * HW + p] = px.rgb[c];
                    T[V->pix_base + p] = px.T;
                    last[V->pix_base + p] = px.last;
                    ill[V->pix_base + p] = (uint8_t)px.ill;
                    cond[V->pix_base + p] = px.cond;
                    it += px.iterated; ev += px.evaluated; hit += px.intersected;
                    ah += px.amb_hits; at += (px.amb_k >= 0);
                }
            }
            free(list);
            free(pos);
        }
        int64_t *cv = counts + 6 * v;
        cv[0] = it; cv[1] = ev; cv[2] = hit; cv[3] = fr; cv[4] = ah; cv[5] = at;
        rgb_base += 3 * HW;
    }
    return 0;
}

/* Depth map of every view (tiled walk), packed like T; depth_ill[p] = 1
 * where the crossing of 0.5 may move under float32 evaluation (a step ends
 * within 1e-6 of it) or the pixel's value is ill-conditioned. */
int orc_render_depth(void *h, const double *bg, double *depth, uint8_t *depth_ill)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep || !S->rlo) return -1;
    for (int v = 0; v < S->n_views; ++v) {
        const orc_view *V = &S->views[v];
#pragma omp parallel
        {
            int64_t *list = NULL, *pos = NULL, cap = 0, start = 0;
#pragma omp for schedule(dynamic, 1)
            for (int j = 0; j < V->H; ++j)
                for (int i = 0; i < V->W; ++i) {
                    const int64_t len = pixel_list(S, v, i, j, 0, &list, &pos, &cap, &start);
                    orc_pix px;
                    composite(S, v, list, pos, len, i, j, bg + 3 * v, 0, &px, NULL, NULL, start, NULL, NULL);
                    const int64_t p = V->pix_base + (int64_t)j * V->W + i;
                    depth[p] = px.depth;
                    depth_ill[p] = (uint8_t)(px.depth_ill || (px.ill & 1));
                }
            free(list);
            free(pos);
        }
    }
    return 0;
}

/* Render selected pixels of one view by brute force (for sampled checks on
 * scenes too large to render whole on the CPU).  pix: npix (i, j) pairs. */
int orc_render_pixels(void *h, int v, int64_t npix, const int32_t *pix, const double *bg,
                      double *rgb, double *T, uint8_t *ill, int64_t *evaluated, double *cond)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep || v < 0 || v >= S->n_views) return -1;
#pragma omp parallel
    {
        int64_t *list = NULL, *pos = NULL, cap = 0, start = 0;
#pragma omp for schedule(dynamic, 4)
        for (int64_t q = 0; q < npix; ++q) {
            const int i = pix[2 * q], j = pix[2 * q + 1];
            const int64_t len = pixel_list(S, v, i, j, 1, &list, &pos, &cap, &start);
            orc_pix px;
            composite(S, v, list, NULL, len, i, j, bg, 0, &px, NULL, NULL, 0, NULL, NULL);
            for (int c = 0; c < 3; ++c) rgb[3 * q + c] = px.rgb[c];
            T[q] = px.T;
            ill[q] = (uint8_t)px.ill;
            evaluated[q] = px.evaluated;
            cond[q] = px.cond;
        }
        free(list);
        free(pos);
    }
    return 0;
}

/* Chord of one primitive at one pixel centre (ray-space line through the
 * pixel centre (px, py)).  method 0: MTIA; 1: clipping. */
double orc_chord(void *h, int v, int64_t n, double px, double py, int method)
{
    orc_scene *S = (orc_scene *)h;
    const orc_prep *P = S->prep + (int64_t)v * S->n + n;
    if (!P->valid) return 0.0;
    if (S->exact) {
        double D[3];
        pixel_ray(&S->views[v], px, py, D);
        return method == 0 ? chord_mtia_exact(S->type, P, D).delta : chord_clip_exact(S->type, P, D);
    }
    return method == 0 ? chord_mtia(S->type, P, px, py).delta : chord_clip(S->type, P, px, py);
}

/* One exact-variant ray hit and its corner derivatives, for tests:
 * V: 9 doubles (three camera-space corners), D: ray direction;
 * out: hit, t, u, v, det, dt/dV (9). */
void orc_mtia_ray(const double *V, const double *D, double *out)
{
    orc_hit H = mtia_ray(V, V + 3, V + 6, D);
    out[0] = H.hit; out[1] = H.t; out[2] = H.u; out[3] = H.v; out[4] = H.det;
    double dV[3][3];
    memset(dV, 0, sizeof(dV));
    if (H.hit) mtia_ray_grad(V, V + 3, V + 6, D, &H, dV);
    for (int k = 0; k < 9; ++k) out[5 + k] = dV[k / 3][k % 3];
}

/* One MTIA evaluation and its App. E depth derivatives, for tests:
 * V: 9 doubles (three corners); out: hit, t, u, v, det, dV (9). */
void orc_mtia(const double *V, double rx, double ry, double *out)
{
    orc_hit H = mtia(V, V + 3, V + 6, rx, ry);
    out[0] = H.hit; out[1] = H.t; out[2] = H.u; out[3] = H.v; out[4] = H.det;
    double dV[3][3];
    memset(dV, 0, sizeof(dV));
    if (H.hit) mtia_depth_grad(V, V + 3, V + 6, rx, ry, &H, dV);
    for (int k = 0; k < 9; ++k) out[5 + k] = dV[k / 3][k % 3];
}

/* ------------------------------------------------------------------------ */
/* Backward pass (Sec. 3.4 "Rasterization/Preprocessing Backpropagation",   */
/* App. E).                                                                 */
/* ------------------------------------------------------------------------ */
typedef struct {
    double gV[6][3];   /* dL/d ray-space corner */
    double grgb[3];
    double gsigma;
    double err[3];     /* per channel, sum over steps of |g_c| T est(o): float32 error scale of grgb */
    double err_sigma;  /* sum over steps of |dL/do| |1 - sigma chord| est(o) / sigma: that of gsigma */
    int ill;
} orc_pgrad;

/* Blend backward for one pixel: walks the recorded steps from the last one
 * to the first with the colour accumulated behind each step, and pushes the
 * depth gradients of the entry and exit hits onto the ray-space corners. */
static int pixel_backward(const orc_scene *S, int v, int i, int j, const orc_step *st, int64_t ns,
                          double Tfinal, const double bg[3], const double g[3], orc_pgrad *G)
{
    const orc_prep *Pv = S->prep + (int64_t)v * S->n;
    const double rx = i + 0.5, ry = j + 0.5;
    double D[3];
    pixel_ray(&S->views[v], rx, ry, D);
    const double nD = norm3(D);
    double behind[3];
    int ill = 0;
    for (int c = 0; c < 3; ++c) behind[c] = Tfinal * bg[c];
    int F[8][3];
    prim_faces(S->type, F);
    for (int64_t k = ns - 1; k >= 0; --k) {
        const orc_step *s = st + k;
        const orc_prep *P = Pv + s->prim;
        orc_pgrad *pg = G + s->prim;
        double dLdo = 0.0;
        for (int c = 0; c < 3; ++c) {
            pg->grgb[c] += g[c] * s->T * s->o;
            dLdo += g[c] * (s->T * P->rgb[c] - behind[c] / (1.0 - s->o));
        }
        for (int c = 0; c < 3; ++c) behind[c] += s->T * s->o * P->rgb[c];
        const double Tafter = s->T * (1.0 - s->o);
        double est = 0.0;
        const int sill = step_ill(S->type, P, s, Tafter, NULL, &S->views[v], S->exact ? D : NULL, &est);
        if (sill & (ORC_BIT_GRAD | ORC_BIT_HIT)) pg->ill = 1;
        for (int c = 0; c < 3; ++c) pg->err[c] += fabs(g[c]) * s->T * est;
        ill |= sill;
        if (s->clamped) continue;
        /* App. E: o = 1 - exp(-sigma (i2 - i1)) */
        const double dLdDelta = dLdo * P->sigma * s->e;
        pg->gsigma += dLdo * s->delta * s->e;
        /* a chord error d moves delta e by e (1 - sigma delta) d, and est = sigma e d */
        if (P->sigma > 0.0) pg->err_sigma += fabs(dLdo) * fabs(1.0 - P->sigma * s->delta) * est / P->sigma;
        const int fs[2] = {s->ch.f_in, s->ch.f_out};
        const orc_hit *hs[2] = {&s->ch.h_in, &s->ch.h_out};
        const double sgn[2] = {-1.0, 1.0};
        if (S->exact) {
            /* chord = |D| (t_out - t_in); gradients onto camera-space corners */
            for (int q = 0; q < 2; ++q) {
                const int *tri = F[fs[q]];
                double dV[3][3];
                mtia_ray_grad(P->vc[tri[0]], P->vc[tri[1]], P->vc[tri[2]], D, hs[q], dV);
                for (int m = 0; m < 3; ++m)
                    for (int r = 0; r < 3; ++r) pg->gV[tri[m]][r] += sgn[q] * dLdDelta * nD * dV[m][r];
            }
            continue;
        }
        double Vc[6][3];
        prim_corners(S->type, P, Vc);
        for (int q = 0; q < 2; ++q) {
            const int *tri = F[fs[q]];
            double dV[3][3];
            mtia_depth_grad(Vc[tri[0]], Vc[tri[1]], Vc[tri[2]], rx, ry, hs[q], dV);
            for (int m = 0; m < 3; ++m)
                for (int r = 0; r < 3; ++r) pg->gV[tri[m]][r] += sgn[q] * dLdDelta * dV[m][r];
        }
    }
    return ill;
}

/* Preprocessing backward for one primitive in one view: ray space ->
 * camera -> world, then onto the rotation, distances, opacity and SH. */
static void prim_backward(const orc_scene *S, const orc_view *V, int64_t n, const orc_prep *P,
                          const orc_pgrad *pg, double *gm, double *gq, double *gd, double *go, double *gsh,
                          double *esh)
{
    const double *mu = S->means + 3 * n;
    const double *d = S->dists + S->nd * n;
    const double *q = S->quats + 4 * n;
    const double alpha = S->opac[n];
    const int na = (S->type == ORC_OCTA) ? 3 : 4;

    /* corners -> ray-space centre and offsets ("gradients to opposite
     * corners are negated" for octahedra, App. E) */
    double gc[3] = {0, 0, 0}, ga[4][3];
    memset(ga, 0, sizeof(ga));
    if (S->type == ORC_OCTA) {
        for (int k = 0; k < 3; ++k)
            for (int r = 0; r < 3; ++r) {
                gc[r] += pg->gV[2 * k][r] + pg->gV[2 * k + 1][r];
                ga[k][r] = pg->gV[2 * k][r] - pg->gV[2 * k + 1][r];
            }
    } else {
        for (int k = 0; k < 4; ++k)
            for (int r = 0; r < 3; ++r) { gc[r] += pg->gV[k][r]; ga[k][r] = pg->gV[k][r]; }
    }

    /* recompute the forward intermediates */
    double R[3][3];
    quat_rotation(q, R);
    double o[4][3], oc[4][3];
    world_offsets(S->type, R, d, o);
    for (int k = 0; k < na; ++k) mat3_vec(V->Rw, o[k], oc[k]);
    const double *t = P->tc;
    double J[3][3];
    ray_jacobian(V, t, J);
    const double x = t[0], y = t[1], z = t[2];
    const double l = sqrt(x * x + y * y + z * z);

    double gt[3];
    double goc[4][3];
    if (S->exact) {
        /* the corners are camera-space points: centre t, offsets oc_k */
        for (int r = 0; r < 3; ++r) gt[r] = gc[r];
        for (int k = 0; k < na; ++k)
            for (int r = 0; r < 3; ++r) goc[k][r] = ga[k][r];
    } else {
        /* c = phi(t), d phi / d t = J */
        mat3T_vec(J, gc, gt);
        /* a_k = J(t) oc_k */
        for (int k = 0; k < na; ++k) {
            mat3T_vec(J, ga[k], goc[k]);
            const double *w = oc[k];
            const double tw = x * w[0] + y * w[1] + z * w[2];
            const double l3 = l * l * l;
            const double fx = V->fx, fy = V->fy;
            /* d(J w)/dx, d(J w)/dy, d(J w)/dz (columns) */
            const double dJw[3][3] = {
                {-fx * w[2] / (z * z), 0.0, -fx * w[0] / (z * z) + 2.0 * fx * x * w[2] / (z * z * z)},
                {0.0, -fy * w[2] / (z * z), -fy * w[1] / (z * z) + 2.0 * fy * y * w[2] / (z * z * z)},
                {w[0] / l - tw * x / l3, w[1] / l - tw * y / l3, w[2] / l - tw * z / l3}};
            for (int c = 0; c < 3; ++c)
                gt[c] += dJw[0][c] * ga[k][0] + dJw[1][c] * ga[k][1] + dJw[2][c] * ga[k][2];
        }
    }
    /* camera -> world */
    double gmu[3], go_w[4][3];
    mat3T_vec(V->Rw, gt, gmu);
    for (int k = 0; k < na; ++k) mat3T_vec(V->Rw, goc[k], go_w[k]);
    /* offsets -> rotation and distances */
    double gR[3][3];
    memset(gR, 0, sizeof(gR));
    if (S->type == ORC_OCTA) {
        for (int k = 0; k < 3; ++k) {
            double dd = 0.0;
            for (int r = 0; r < 3; ++r) { gR[r][k] += go_w[k][r] * d[k]; dd += go_w[k][r] * R[r][k]; }
            gd[k] += dd;
        }
    } else {
        for (int i = 0; i < 4; ++i) {
            const double g = d[i] * ORC_INV_SQRT3;
            double dd = 0.0;
            for (int r = 0; r < 3; ++r) {
                const double rb = TET_B[i][0] * R[r][0] + TET_B[i][1] * R[r][1] + TET_B[i][2] * R[r][2];
                for (int c = 0; c < 3; ++c) gR[r][c] += go_w[i][r] * TET_B[i][c] * g;
                dd += go_w[i][r] * rb * ORC_INV_SQRT3;
            }
            gd[i] += dd;
        }
    }
    /* rotation -> quaternion: R = I + s K(q), s = 2 / |q|^2 */
    {
        const double w = q[0], qx = q[1], qy = q[2], qz = q[3];
        const double n2 = w * w + qx * qx + qy * qy + qz * qz;
        const double s = 2.0 / n2;
        const double K[3][3] = {{-(qy * qy + qz * qz), qx * qy - w * qz, qx * qz + w * qy},
                                {qx * qy + w * qz, -(qx * qx + qz * qz), qy * qz - w * qx},
                                {qx * qz - w * qy, qy * qz + w * qx, -(qx * qx + qy * qy)}};
        /* dK/dq_m for m = w, x, y, z */
        const double dK[4][3][3] = {
            {{0, -qz, qy}, {qz, 0, -qx}, {-qy, qx, 0}},
            {{0, qy, qz}, {qy, -2 * qx, -w}, {qz, w, -2 * qx}},
            {{-2 * qy, qx, w}, {qx, 0, qz}, {-w, qz, -2 * qy}},
            {{-2 * qz, -w, qx}, {w, -2 * qz, qy}, {qx, qy, 0}}};
        double gK = 0.0;
        for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) gK += gR[r][c] * K[r][c];
        for (int m = 0; m < 4; ++m) {
            double acc = -s * s * q[m] * gK;
            for (int r = 0; r < 3; ++r) for (int c = 0; c < 3; ++c) acc += s * gR[r][c] * dK[m][r][c];
            gq[m] += acc;
        }
    }
    /* Eq. 1 with min(d) held constant (App. G) */
    {
        double dmin = d[0];
        for (int k = 1; k < S->nd; ++k) if (d[k] < dmin) dmin = d[k];
        go[0] += pg->gsigma * ORC_ALPHA_SCALE / ((1.0 - ORC_ALPHA_SCALE * alpha) * 2.0 * dmin);
    }
    /* colour -> SH and viewing direction */
    {
        double cam[3], dir[3], Y[16], G[16][3];
        mat3T_vec(V->Rw, V->tw, cam);
        for (int k = 0; k < 3; ++k) dir[k] = mu[k] + cam[k];
        const double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        for (int k = 0; k < 3; ++k) dir[k] /= dn;
        orc_sh_basis(S->deg, dir, Y);
        sh_basis_grad(S->deg, dir, G);
        const double *sh = S->sh + (int64_t)48 * n;
        double gdir[3] = {0, 0, 0};
        for (int ch = 0; ch < 3; ++ch) {
            if (!(P->raw[ch] > 0.0)) continue;
            const double gr = pg->grgb[ch];
            for (int k = 0; k < S->K; ++k) {
                gsh[3 * k + ch] += gr * Y[k];
                esh[3 * k + ch] += pg->err[ch] * fabs(Y[k]);
                for (int r = 0; r < 3; ++r) gdir[r] += gr * sh[3 * k + ch] * G[k][r];
            }
        }
        const double dot = gdir[0] * dir[0] + gdir[1] * dir[1] + gdir[2] * dir[2];
        for (int r = 0; r < 3; ++r) gmu[r] += (gdir[r] - dot * dir[r]) / dn;
    }
    for (int r = 0; r < 3; ++r) gm[r] += gmu[r];
}

/* Full backward: grad_rgb packed like orc_render's rgb.  Pixels whose three
 * gradient channels are all zero are skipped.  Outputs (overwritten):
 * parameter gradients summed over views, and prim_ill[n]: bit 0 if a pixel
 * with a non-zero gradient reached primitive n through a step whose discrete
 * decisions may differ in float32 (an active face near an edge, the clamp,
 * a silhouette graze or near miss, an ambiguous termination at or in front
 * of it) or its colour sits at the clamp; bit 1 if the float32 error
 * estimate of its opacity or SH gradient exceeds ORC_ILL_REL of it. */
int orc_backward(void *h, const double *bg, const double *grad_rgb, double *gm, double *gq,
                 double *gd, double *go, double *gsh, uint8_t *prim_ill)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep || !S->rlo) return -1;
    const int64_t n = S->n;
    memset(gm, 0, sizeof(double) * 3 * n);
    memset(gq, 0, sizeof(double) * 4 * n);
    memset(gd, 0, sizeof(double) * S->nd * n);
    memset(go, 0, sizeof(double) * n);
    memset(gsh, 0, sizeof(double) * 48 * n);
    memset(prim_ill, 0, (size_t)n);
    int nthreads = 1;
#ifdef _OPENMP
    nthreads = omp_get_max_threads();
#endif
    free(S->sgrad);
    S->sgrad = (double *)calloc((size_t)S->n_views * (size_t)(n > 0 ? n : 1) * 2, sizeof(double));
    orc_pgrad *acc = (orc_pgrad *)malloc(sizeof(orc_pgrad) * (size_t)(n > 0 ? n : 1));
    double *err_alpha = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    double *err_sh = (double *)calloc((size_t)48 * (size_t)(n > 0 ? n : 1), sizeof(double));
    orc_pgrad *tacc = (orc_pgrad *)calloc((size_t)nthreads * (size_t)(n > 0 ? n : 1), sizeof(orc_pgrad));
    int64_t rgb_base = 0;
    for (int v = 0; v < S->n_views; ++v) {
        const orc_view *V = &S->views[v];
        const int64_t HW = (int64_t)V->W * V->H;
        memset(tacc, 0, sizeof(orc_pgrad) * (size_t)nthreads * (size_t)n);
#pragma omp parallel
        {
            int tid = 0;
#ifdef _OPENMP
            tid = omp_get_thread_num();
#endif
            orc_pgrad *G = tacc + (int64_t)tid * n;
            int64_t *list = NULL, *pos = NULL, cap = 0, start = 0;
            orc_step *steps = NULL;
            int64_t *amb = NULL;
            int64_t scap = 0;
#pragma omp for schedule(static)
            for (int j = 0; j < V->H; ++j) {
                for (int i = 0; i < V->W; ++i) {
                    const int64_t p = (int64_t)j * V->W + i;
                    const double g[3] = {grad_rgb[rgb_base + p], grad_rgb[rgb_base + HW + p],
                                         grad_rgb[rgb_base + 2 * HW + p]};
                    if (g[0] == 0.0 && g[1] == 0.0 && g[2] == 0.0) continue;
                    const int64_t len = pixel_list(S, v, i, j, 0, &list, &pos, &cap, &start);
                    if (len > scap) {
                        scap = len;
                        steps = (orc_step *)realloc(steps, sizeof(orc_step) * (size_t)len);
                        amb = (int64_t *)realloc(amb, sizeof(int64_t) * (size_t)len);
                    }
                    orc_pix px;
                    int64_t ns = 0, na = 0;
                    composite(S, v, list, pos, len, i, j, bg + 3 * v, 0, &px, steps, &ns, start, amb, &na);
                    pixel_backward(S, v, i, j, steps, ns, px.T, bg + 3 * v, g, G);
                    /* a miss that grazes the silhouette may be a hit in
                     * float32, with a gradient of its own */
                    for (int64_t a = 0; a < na; ++a) G[amb[a]].ill = 1;
                    /* termination may move by a step in float32: the crossing
                     * primitive and every one behind it may blend or not */
                    if (px.amb_k >= 0) {
                        const orc_prep *Pv = S->prep + (int64_t)v * n;
                        for (int64_t k = px.amb_k; k < len; ++k)
                            if (in_rect(Pv + list[k], i, j)) G[list[k]].ill = 1;
                    }
                }
            }
            free(list); free(pos); free(steps); free(amb);
        }
        /* reduce the per-thread buffers in thread order */
        memset(acc, 0, sizeof(orc_pgrad) * (size_t)n);
        for (int t = 0; t < nthreads; ++t) {
            const orc_pgrad *G = tacc + (int64_t)t * n;
            for (int64_t m = 0; m < n; ++m) {
                for (int k = 0; k < 6; ++k) for (int r = 0; r < 3; ++r) acc[m].gV[k][r] += G[m].gV[k][r];
                for (int c = 0; c < 3; ++c) acc[m].grgb[c] += G[m].grgb[c];
                acc[m].gsigma += G[m].gsigma;
                for (int c = 0; c < 3; ++c) acc[m].err[c] += G[m].err[c];
                acc[m].err_sigma += G[m].err_sigma;
                acc[m].ill |= G[m].ill;
            }
        }
        const orc_prep *Pv = S->prep + (int64_t)v * n;
#pragma omp parallel for schedule(static)
        for (int64_t m = 0; m < n; ++m) {
            double *sg = S->sgrad + 2 * ((int64_t)v * n + m);
            sg[0] = sg[1] = 0.0;
            if (!Pv[m].valid) continue;
            /* Sec. 3.4 "Adaptive Population Control": the view-space positional
             * gradient, dL/d(ray-space centre x, y) with the offsets held
             * fixed, i.e. the sum of the corner gradients (ray space only) */
            if (!S->exact) {
                const int nc = (S->type == ORC_OCTA) ? 6 : 4;
                for (int k = 0; k < nc; ++k) { sg[0] += acc[m].gV[k][0]; sg[1] += acc[m].gV[k][1]; }
            }
            if (acc[m].ill) prim_ill[m] |= 1;
            for (int c = 0; c < 3; ++c)
                if (fabs(Pv[m].raw[c]) <= ORC_ILL_RGB && acc[m].grgb[c] != 0.0) prim_ill[m] |= 1;
            prim_backward(S, V, m, Pv + m, acc + m, gm + 3 * m, gq + 4 * m, gd + S->nd * m, go + m,
                          gsh + 48 * m, err_sh + 48 * m);
            /* the opacity gradient's share: dsigma/dalpha (R14) times that of gsigma */
            const double *dm = S->dists + S->nd * m;
            double dmin = dm[0];
            for (int k = 1; k < S->nd; ++k) dmin = fmin(dmin, dm[k]);
            err_alpha[m] += acc[m].err_sigma * ORC_ALPHA_SCALE / ((1.0 - ORC_ALPHA_SCALE * S->opac[m]) * 2.0 * dmin);
        }
        rgb_base += 3 * HW;
    }
    /* opacity and SH gradients whose float32 error estimate exceeds
     * ORC_ILL_REL of max(|gradient|, 1e-2 rms of that tensor over the
     * primitives the gradient reaches), the form of the parity tolerance */
    double ss = 0.0, ssh = 0.0;
    int64_t cnt = 0;
    for (int64_t m = 0; m < n; ++m)
        if (go[m] != 0.0) {
            ss += go[m] * go[m];
            for (int k = 0; k < 3 * S->K; ++k) ssh += gsh[48 * m + k] * gsh[48 * m + k];
            ++cnt;
        }
    const double floor_a = cnt ? 1e-2 * sqrt(ss / (double)cnt) : 0.0;
    const double floor_sh = cnt ? 1e-2 * sqrt(ssh / ((double)cnt * 3 * S->K)) : 0.0;
    for (int64_t m = 0; m < n; ++m) {
        if (err_alpha[m] > ORC_ILL_REL * fmax(fabs(go[m]), floor_a)) prim_ill[m] |= 2;
        for (int k = 0; k < 3 * S->K; ++k)
            if (err_sh[48 * m + k] > ORC_ILL_REL * fmax(fabs(gsh[48 * m + k]), floor_sh)) prim_ill[m] |= 2;
    }
    free(err_alpha);
    free(err_sh);
    free(acc);
    free(tacc);
    return 0;
}

/* Per (view, primitive) screen-space statistics of the last orc_backward:
 * sgrad [n_views][n][2] = dL/d(projected centre, pixels), radius
 * [n_views][n] = half the larger side of the projected box, visible
 * [n_views][n] = 1 where the primitive touches a tile. */
int orc_get_stats(void *h, double *sgrad, double *radius, uint8_t *visible)
{
    orc_scene *S = (orc_scene *)h;
    if (!S || !S->prep || !S->sgrad) return -1;
    const int64_t vn = (int64_t)S->n_views * S->n;
    memcpy(sgrad, S->sgrad, sizeof(double) * 2 * (size_t)vn);
    for (int64_t k = 0; k < vn; ++k) {
        radius[k] = S->prep[k].valid ? S->prep[k].radius : 0.0;
        visible[k] = (uint8_t)S->prep[k].valid;
    }
    return 0;
}

/* Threads of the OpenMP regions that follow (used to time the oracle on
 * one core and on all cores). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
