/*
 * HPMC reference oracle -- TEST INFRASTRUCTURE ONLY (see hpmc_oracle.h).
 *
 * Plain serial FP64 C, built with -O2 -ffp-contract=off -fno-fast-math so
 * that every expression below is evaluated exactly in the written order with
 * IEEE round-to-nearest and no fused multiply-add.  The paper's steps are
 * followed in its order:
 *   - Metropolis for hard shapes: pick a particle, propose a small move,
 *     reject on any overlap (Sec. 2.1);
 *   - cell list with cells no narrower than d_max, searching the own cell and
 *     its neighbours +-1 per axis (Sec. 2.2.1);
 *   - overlap checks in the local frame of particle A, position plus
 *     orientation per particle, support function of the Minkowski difference
 *     (Sec. 2.3, Eqs. 1-2);
 *   - hash-keyed random streams per trial move (Sec. 2.5);
 *   - checkerboard: one trial move per non-empty active cell, moves that
 *     leave the active region are rejected, a random translation (here: of
 *     the grid) per step (Sec. 2.5.1, 2.5.2).
 * Where the paper is silent, the readings stated in the design notes are
 * used: even n >= 4, uniform random occupant per cell, fixed colour order,
 * Philox4x32-10 counters, ascending-tag cell order, touching is not overlap.
 */
#include "hpmc_oracle.h"

/*
 * ORACLE_PLANT_* switches each compile in one deliberate, plausible mistake.
 * Only the test suite's sensitivity checks build with one defined, to show
 * that some pin fails when the oracle is wrong.  The normal build defines
 * none of them.
 */

#include <math.h>
#include <stdlib.h>
#include <string.h>

/*
 * ORACLE_COUNT_OPS builds a variant that counts algorithmic events of the
 * sweep (moves by kind, candidate pairs, separating-axis set-ups and axes
 * evaluated, XenoCollide set-ups, support evaluations and iterations,
 * swept-polygon distance set-ups and point-segment tests), all
 * with early exit, for the benchmark's work-per-move figure.  The normal
 * build compiles EVENT() to nothing.
 */
enum { EV_TRANSLATE, EV_ROTATE2, EV_ROTATE3, EV_CAND2, EV_CAND3, EV_SAT_SETUP, EV_SAT_AXIS,
       EV_SAT_FRAME_B, EV_MPR_SETUP, EV_MPR_SUPPORT, EV_MPR_ITER, EV_SEG_SETUP, EV_SEG_TEST,
       EV_COUNT };
#ifdef ORACLE_COUNT_OPS
static int64_t or_events[EV_COUNT];
int64_t *or_event_counts(void) { return or_events; }
int32_t or_n_events(void) { return EV_COUNT; }
#define EVENT(k) (or_events[(k)] += 1)
#else
#define EVENT(k) ((void)0)
#endif

/* ------------------------------------------------------------------------ */
/* Random numbers: Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11).       */
/* Counter-based, so every trial move has its own independent stream,       */
/* the role the paper gives its hash-based generator (Sec. 2.5).            */
/* ------------------------------------------------------------------------ */

static void mulhilo32(uint32_t a, uint32_t b, uint32_t *hi, uint32_t *lo)
{
    uint64_t p = (uint64_t)a * (uint64_t)b;
    *hi = (uint32_t)(p >> 32);
    *lo = (uint32_t)p;
}

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    const uint32_t M0 = 0xD2511F53u, M1 = 0xCD9E8D57u;
    const uint32_t W0 = 0x9E3779B9u, W1 = 0xBB67AE85u;
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
#ifdef ORACLE_PLANT_PHILOX_9_ROUNDS
    for (int round = 0; round < 9; ++round) {
#else
    for (int round = 0; round < 10; ++round) {
#endif
        if (round > 0) {
            k0 += W0;
            k1 += W1;
        }
        uint32_t hi0, lo0, hi1, lo1;
        mulhilo32(M0, x0, &hi0, &lo0);
        mulhilo32(M1, x2, &hi1, &lo1);
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* Uniform in (0,1): (w + 1/2) / 2^32, exact in binary64. */
void or_philox4x32_10_many(const uint32_t *ctr, int64_t n, const uint32_t key[2], uint32_t *out)
{
    for (int64_t i = 0; i < n; ++i)
        or_philox4x32_10(ctr + 4 * i, key, out + 4 * i);
}

double or_u01(uint32_t w)
{
#ifdef ORACLE_PLANT_U01_NO_HALF
    return (double)w * 0x1p-32;
#endif
    return ((double)w + 0.5) * 0x1p-32;
}

/* Index in [0, n): floor(w * n / 2^32). */
uint32_t or_index(uint32_t w, uint32_t n)
{
    return (uint32_t)(((uint64_t)w * (uint64_t)n) >> 32);
}

enum { PURPOSE_SHIFT = 1, PURPOSE_SELECT = 2, PURPOSE_MOVE = 3,
       PURPOSE_SERIAL_SELECT = 5, PURPOSE_SERIAL_MOVE = 6 };

/* Counter (sweep, purpose<<28 | select, id, replica), key = seed. */
static void draw(uint64_t seed, uint32_t t, uint32_t purpose, uint32_t select,
                 uint32_t id, uint32_t replica, uint32_t out[4])
{
    uint32_t ctr[4] = { t, (purpose << 28) | select, id, replica };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    or_philox4x32_10(ctr, key, out);
}

/* ------------------------------------------------------------------------ */
/* sin / cos of a small rotation angle: Taylor polynomials through delta^15  */
/* and delta^16, Horner in delta^2, coefficients 1/k! rounded to binary64.   */
/* ------------------------------------------------------------------------ */

static double inv_factorial(int k)
{
    double f = 1.0;
    for (int i = 2; i <= k; ++i)
        f = f * (double)i; /* exact for k <= 18 */
    return 1.0 / f;
}

void or_sincos(double delta, double *c, double *s)
{
    double x2 = delta * delta;
    /* sin: sum_{k=0..7} (-1)^k delta^(2k+1) / (2k+1)!, innermost term first */
    double ps = -inv_factorial(15);
    for (int k = 6; k >= 0; --k) {
        double coef = (k % 2 == 1) ? -inv_factorial(2 * k + 1) : inv_factorial(2 * k + 1);
#ifdef ORACLE_PLANT_SINCOS_DROP_TERM
        if (k == 4)
            coef = 0.0;
#endif
        ps = ps * x2;
        ps = ps + coef;
    }
    *s = delta * ps;
    /* cos: sum_{k=0..8} (-1)^k delta^(2k) / (2k)! */
    double pc = inv_factorial(16);
    for (int k = 7; k >= 0; --k) {
        double coef = (k % 2 == 1) ? -inv_factorial(2 * k) : inv_factorial(2 * k);
        pc = pc * x2;
        pc = pc + coef;
    }
    *c = pc;
}

/* ------------------------------------------------------------------------ */
/* Shapes (Sec. 2.3): geometry given once per type in the particle frame.   */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dim, kind, nv;
    double v[OR_MAXV][3];
    double nrm[OR_MAXV][2];               /* polygon outward edge normals */
    double pmin[OR_MAXV], pmax[OR_MAXV];  /* own projections onto them */
    double R, dmax, circ2, tol2;
    double sweep;  /* sweep radius of a spheropolygon / -polyhedron, 0 otherwise */
} shape_t;

static int setup_shape(const or_species *sp, shape_t *sh)
{
    memset(sh, 0, sizeof(*sh));
    sh->dim = sp->dim;
    sh->kind = sp->shape;
    if (sp->shape == OR_DISK) {
        if (sp->dim != 2 || !(sp->diameter > 0.0) || sp->sweep_radius != 0.0)
            return OR_ERR_INVALID_ARG;
        sh->R = sp->diameter * 0.5;
    } else {
        int want_dim = sp->shape == OR_POLYGON ? 2 : 3;
        if (sp->shape != OR_POLYGON && sp->shape != OR_POLYHEDRON)
            return OR_ERR_INVALID_ARG;
        if (sp->dim != want_dim || sp->verts == NULL)
            return OR_ERR_INVALID_ARG;
        if (!(sp->sweep_radius >= 0.0) || !isfinite(sp->sweep_radius))
            return OR_ERR_INVALID_ARG;
        sh->sweep = sp->sweep_radius;
        int min_verts = sh->sweep > 0.0 ? 1 : want_dim + 1;
        if (sp->n_verts < min_verts || sp->n_verts > OR_MAXV)
            return OR_ERR_INVALID_ARG;
        sh->nv = sp->n_verts;
        double rmax = 0.0;
        for (int k = 0; k < sh->nv; ++k) {
            double r2 = 0.0;
            for (int a = 0; a < sh->dim; ++a) {
                sh->v[k][a] = sp->verts[k * sh->dim + a];
                r2 = r2 + sh->v[k][a] * sh->v[k][a];
            }
            double r = sqrt(r2);
            if (r > rmax)
                rmax = r;
        }
        /* one ulp up so that every vertex (and, for a spheropolyhedron,
         * every point within the sweep radius of one) lies inside */
        sh->R = nextafter(rmax + sh->sweep, INFINITY);
        if (sp->shape == OR_POLYGON) {
            /* a swept core of one or two vertices (a point, a segment) has
             * no turn to check; its edge k -> k+1 normals still serve the
             * separating-axis test of the cores */
            for (int k = 0; k < sh->nv; ++k) {
                int k1 = (k + 1) % sh->nv, k2 = (k + 2) % sh->nv;
                double ex = sh->v[k1][0] - sh->v[k][0];
                double ey = sh->v[k1][1] - sh->v[k][1];
                double fx = sh->v[k2][0] - sh->v[k1][0];
                double fy = sh->v[k2][1] - sh->v[k1][1];
                if (sh->nv >= 3 && !(ex * fy - ey * fx > 0.0))
                    return OR_ERR_INVALID_ARG; /* not strictly convex CCW */
                sh->nrm[k][0] = ey;
                sh->nrm[k][1] = -ex;
            }
            for (int k = 0; k < sh->nv; ++k) {
                double lo = 0.0, hi = 0.0;
                for (int j = 0; j < sh->nv; ++j) {
                    double p = sh->nrm[k][0] * sh->v[j][0] + sh->nrm[k][1] * sh->v[j][1];
                    if (j == 0 || p < lo) lo = p;
                    if (j == 0 || p > hi) hi = p;
                }
                sh->pmin[k] = lo;
                sh->pmax[k] = hi;
            }
        }
    }
    sh->dmax = sh->R + sh->R;
    sh->circ2 = sh->dmax * sh->dmax;
    double tol = 1e-12 * sh->dmax;
    sh->tol2 = tol * tol;
    if (!(sp->d >= 0.0) || !(sp->a >= 0.0) || !(sp->p_rot >= 0.0) || !(sp->p_rot <= 1.0))
        return OR_ERR_INVALID_ARG;
    if (sp->shape == OR_DISK && sp->p_rot != 0.0)
        return OR_ERR_INVALID_ARG;
    return OR_OK;
}

int or_shape_info(const or_species *sp, double out[4])
{
    shape_t sh;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    out[0] = sh.R;
    out[1] = sh.dmax;
    out[2] = sh.circ2;
    out[3] = sh.tol2;
    return OR_OK;
}

/* ------------------------------------------------------------------------ */
/* Overlap tests (Sec. 2.3).  A is at the origin of its own frame; B sits at */
/* t with relative orientation z (2D) or rotation matrix M (3D).             */
/* ------------------------------------------------------------------------ */

/* Convex polygons by separating axes: every edge normal of A (in A's frame)
 * and of B (in B's frame) is tried; an axis separates when the projection
 * intervals do not overlap, touching counting as separated. */
static int overlap_polygon(const shape_t *sh, const double r[2], const double qa[2],
                           const double qb[2])
{
    double cA = qa[0], sA = qa[1], cB = qb[0], sB = qb[1];
    /* relative orientation z = conj(zA) zB and B's centre in A's frame */
    EVENT(EV_SAT_SETUP);
    double zc = cA * cB + sA * sB;
    double zs = cA * sB - sA * cB;
    double tx = cA * r[0] + sA * r[1];
#ifdef ORACLE_PLANT_SAT_SIGN
    double ty = cA * r[1] + sA * r[0];
#else
    double ty = cA * r[1] - sA * r[0];
#endif

    /* axes of A, in A's frame: B's vertices mapped into A's frame */
    double bx[OR_MAXV], by[OR_MAXV];
    for (int j = 0; j < sh->nv; ++j) {
        bx[j] = (zc * sh->v[j][0] - zs * sh->v[j][1]) + tx;
        by[j] = (zs * sh->v[j][0] + zc * sh->v[j][1]) + ty;
    }
    for (int k = 0; k < sh->nv; ++k) {
        double lo = 0.0, hi = 0.0;
        for (int j = 0; j < sh->nv; ++j) {
            double p = sh->nrm[k][0] * bx[j] + sh->nrm[k][1] * by[j];
            if (j == 0)
                EVENT(EV_SAT_AXIS);
            if (j == 0 || p < lo) lo = p;
            if (j == 0 || p > hi) hi = p;
        }
        if (sh->pmax[k] <= lo || hi <= sh->pmin[k])
            return 0;
    }
#ifdef ORACLE_PLANT_SAT_A_AXES_ONLY
    return 1;
#endif
    /* axes of B, in B's frame: A's vertices mapped into B's frame */
    double ax[OR_MAXV], ay[OR_MAXV];
    EVENT(EV_SAT_FRAME_B);
    for (int j = 0; j < sh->nv; ++j) {
        double ux = sh->v[j][0] - tx;
        double uy = sh->v[j][1] - ty;
        ax[j] = zc * ux + zs * uy;
        ay[j] = zc * uy - zs * ux;
    }
    for (int k = 0; k < sh->nv; ++k) {
        double lo = 0.0, hi = 0.0;
        for (int j = 0; j < sh->nv; ++j) {
            double p = sh->nrm[k][0] * ax[j] + sh->nrm[k][1] * ay[j];
            if (j == 0)
                EVENT(EV_SAT_AXIS);
            if (j == 0 || p < lo) lo = p;
            if (j == 0 || p > hi) hi = p;
        }
        if (hi <= sh->pmin[k] || sh->pmax[k] <= lo)
            return 0;
    }
    return 1;
}

/* Spheropolygons (swept convex polygons, Sec. 2.3): the particle is every
 * point within the sweep radius s of its core polygon, so two overlap when
 * their cores overlap or pass closer than s + s.  Two convex cores that do
 * not meet are closest at a vertex of one and an edge of the other; a core of
 * one or two vertices is a point or a segment, covered by its "edges"
 * k -> k+1 all the same.  Point p is closer than r (r2 = r^2) to the
 * segment a-b exactly when the nearest point of the segment is: the end a
 * (projection parameter c1 <= 0), the end b (c1 >= |b - a|^2 = c2), or the
 * foot of the perpendicular, at squared distance cross^2 / c2. */
static int point_segment_close(double px, double py, double ax, double ay, double bx, double by,
                               double r2)
{
    EVENT(EV_SEG_TEST);
    double ex = bx - ax, ey = by - ay;
    double wx = px - ax, wy = py - ay;
    double c1 = wx * ex + wy * ey;
    if (c1 <= 0.0)
        return wx * wx + wy * wy < r2;
    double c2 = ex * ex + ey * ey;
    if (c1 >= c2) {
        double dx = px - bx, dy = py - by;
        return dx * dx + dy * dy < r2;
    }
    double cr = ex * wy - ey * wx;
    return cr * cr < r2 * c2;
}

/* Cores closer than s + s, measured in A's frame: A's vertices against B's
 * edges, then B's vertices against A's edges. */
static int polygon_cores_close(const shape_t *sh, const double r[2], const double qa[2],
                               const double qb[2])
{
    double cA = qa[0], sA = qa[1], cB = qb[0], sB = qb[1];
    EVENT(EV_SEG_SETUP);
    double zc = cA * cB + sA * sB;
    double zs = cA * sB - sA * cB;
    double tx = cA * r[0] + sA * r[1];
    double ty = cA * r[1] - sA * r[0];
#ifdef ORACLE_PLANT_SWEEP_ONE_SIDED
    double reach = sh->sweep;
#else
    double reach = sh->sweep + sh->sweep;
#endif
    double r2 = reach * reach;
    double bx[OR_MAXV], by[OR_MAXV];
    for (int j = 0; j < sh->nv; ++j) {
        bx[j] = (zc * sh->v[j][0] - zs * sh->v[j][1]) + tx;
        by[j] = (zs * sh->v[j][0] + zc * sh->v[j][1]) + ty;
    }
    for (int j = 0; j < sh->nv; ++j)
        for (int k = 0; k < sh->nv; ++k) {
            int k1 = (k + 1) % sh->nv;
            if (point_segment_close(sh->v[j][0], sh->v[j][1], bx[k], by[k], bx[k1], by[k1], r2))
                return 1;
        }
#ifdef ORACLE_PLANT_SWEPT_ONE_WAY
    return 0;
#endif
    for (int j = 0; j < sh->nv; ++j)
        for (int k = 0; k < sh->nv; ++k) {
            int k1 = (k + 1) % sh->nv;
            if (point_segment_close(bx[j], by[j], sh->v[k][0], sh->v[k][1], sh->v[k1][0],
                                    sh->v[k1][1], r2))
                return 1;
        }
    return 0;
}

/* Hamilton product p (x) q, each component summed left to right. */
static void quat_mul(const double p[4], const double q[4], double out[4])
{
    out[0] = ((p[0] * q[0] - p[1] * q[1]) - p[2] * q[2]) - p[3] * q[3];
    out[1] = ((p[0] * q[1] + p[1] * q[0]) + p[2] * q[3]) - p[3] * q[2];
    out[2] = ((p[0] * q[2] - p[1] * q[3]) + p[2] * q[0]) + p[3] * q[1];
    out[3] = ((p[0] * q[3] + p[1] * q[2]) - p[2] * q[1]) + p[3] * q[0];
}

/* Rotation matrix of a unit quaternion (w, x, y, z). */
static void quat_to_matrix(const double q[4], double m[3][3])
{
    double w = q[0], x = q[1], y = q[2], z = q[3];
    m[0][0] = 1.0 - 2.0 * (y * y + z * z);
    m[0][1] = 2.0 * (x * y - w * z);
    m[0][2] = 2.0 * (x * z + w * y);
    m[1][0] = 2.0 * (x * y + w * z);
    m[1][1] = 1.0 - 2.0 * (x * x + z * z);
    m[1][2] = 2.0 * (y * z - w * x);
    m[2][0] = 2.0 * (x * z - w * y);
    m[2][1] = 2.0 * (y * z + w * x);
    m[2][2] = 1.0 - 2.0 * (x * x + y * y);
}

static double dot3(const double a[3], const double b[3])
{
    return (a[0] * b[0] + a[1] * b[1]) + a[2] * b[2];
}

static void cross3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[1] * b[2] - a[2] * b[1];
    out[1] = a[2] * b[0] - a[0] * b[2];
    out[2] = a[0] * b[1] - a[1] * b[0];
}

static void sub3(const double a[3], const double b[3], double out[3])
{
    out[0] = a[0] - b[0];
    out[1] = a[1] - b[1];
    out[2] = a[2] - b[2];
}

typedef struct {
    const shape_t *sh;
    double m[3][3]; /* B frame -> A frame */
    double t[3];    /* B's centre in A's frame */
} mink_t;

/* Support point of the Minkowski difference B - A in direction n, in A's
 * frame: S_{B-A}(n) = M S_B(M^T n) + t - S_A(-n) (Eq. 2 with the centre
 * offset expressed in A's frame).  S_X(n) is the first vertex attaining the
 * largest n . v.  A spheropolyhedron of sweep radius s is its hull plus a
 * ball of radius s, whose support adds s n/|n|; both particles share s, so
 * the difference gains (s + s) n/|n| (skipped for n = 0). */
static void support(const mink_t *mk, const double n[3], double out[3])
{
    const shape_t *sh = mk->sh;
    double nb[3];
    EVENT(EV_MPR_SUPPORT);
    for (int a = 0; a < 3; ++a)
#ifdef ORACLE_PLANT_MPR_TRANSPOSE
        nb[a] = (mk->m[a][0] * n[0] + mk->m[a][1] * n[1]) + mk->m[a][2] * n[2];
#else
        nb[a] = (mk->m[0][a] * n[0] + mk->m[1][a] * n[1]) + mk->m[2][a] * n[2];
#endif
    int kb = 0;
    double best = dot3(nb, sh->v[0]);
    for (int k = 1; k < sh->nv; ++k) {
        double p = dot3(nb, sh->v[k]);
        if (p > best) { best = p; kb = k; }
    }
    double na[3] = { -n[0], -n[1], -n[2] };
    int ka = 0;
    best = dot3(na, sh->v[0]);
    for (int k = 1; k < sh->nv; ++k) {
        double p = dot3(na, sh->v[k]);
        if (p > best) { best = p; ka = k; }
    }
    for (int a = 0; a < 3; ++a) {
        double sb = ((mk->m[a][0] * sh->v[kb][0] + mk->m[a][1] * sh->v[kb][1])
                     + mk->m[a][2] * sh->v[kb][2]) + mk->t[a];
        out[a] = sb - sh->v[ka][a];
    }
    double nn = dot3(n, n);
    if (sh->sweep > 0.0 && nn > 0.0) {
#ifdef ORACLE_PLANT_SWEEP_ONE_SIDED
        double s = sh->sweep / sqrt(nn);
#else
        double s = (sh->sweep + sh->sweep) / sqrt(nn);
#endif
        for (int a = 0; a < 3; ++a)
            out[a] = out[a] + s * n[a];
    }
}

#define MPR_MAX_ITER 1024

static int is_zero3(const double v[3])
{
    return v[0] == 0.0 && v[1] == 0.0 && v[2] == 0.0;
}

/* XenoCollide / minkowski portal refinement (Jacobs 2008; Snethen): does the
 * Minkowski difference D = B - A contain the origin?  v0 = t is an interior
 * point of D.  Portal discovery finds a triangle (v1, v2, v3) of support
 * points through which the ray from v0 to the origin passes; refinement
 * pushes the portal out to the boundary of D until the origin is either
 * behind the portal (overlap) or beyond a support plane (no overlap). */
static int overlap_polyhedron(const shape_t *sh, const double r[3], const double qa[4],
                              const double qb[4])
{
    mink_t mk;
    mk.sh = sh;
    EVENT(EV_MPR_SETUP);
    double qac[4] = { qa[0], -qa[1], -qa[2], -qa[3] };
    double q[4], ma[3][3];
    quat_mul(qac, qb, q);
    quat_to_matrix(q, mk.m);
    quat_to_matrix(qa, ma);
    for (int a = 0; a < 3; ++a)
        mk.t[a] = (ma[0][a] * r[0] + ma[1][a] * r[1]) + ma[2][a] * r[2];

    double v0[3] = { mk.t[0], mk.t[1], mk.t[2] };
    if (is_zero3(v0))
        return 1; /* coincident centres */

    double n[3], v1[3], v2[3], v3[3], v4[3], e1[3], e2[3], tmp[3];
    n[0] = -v0[0]; n[1] = -v0[1]; n[2] = -v0[2];
    support(&mk, n, v1);
    if (dot3(v1, n) <= 0.0)
        return 0;

    cross3(v1, v0, n);
    if (is_zero3(n))
        return 1; /* origin on the segment v0 -> v1 */
    support(&mk, n, v2);
    if (dot3(v2, n) <= 0.0)
        return 0;

    /* portal normal, oriented so that it points from v0 towards the origin */
    sub3(v1, v0, e1);
    sub3(v2, v0, e2);
    cross3(e1, e2, n);
    if (dot3(n, v0) > 0.0) {
        double s[3] = { v1[0], v1[1], v1[2] };
        v1[0] = v2[0]; v1[1] = v2[1]; v1[2] = v2[2];
        v2[0] = s[0]; v2[1] = s[1]; v2[2] = s[2];
        n[0] = -n[0]; n[1] = -n[1]; n[2] = -n[2];
    }

    /* portal discovery */
    int iter = 0;
    for (;;) {
        if (++iter > MPR_MAX_ITER)
            return 1; /* cap reached: conservative */
        EVENT(EV_MPR_ITER);
        support(&mk, n, v3);
        if (dot3(v3, n) <= 0.0)
            return 0;
        /* origin outside the cone face (v0, v1, v3): drop v2 */
        cross3(v1, v3, tmp);
        if (dot3(tmp, v0) < 0.0) {
            v2[0] = v3[0]; v2[1] = v3[1]; v2[2] = v3[2];
            sub3(v1, v0, e1);
            sub3(v3, v0, e2);
            cross3(e1, e2, n);
            continue;
        }
        /* origin outside the cone face (v0, v3, v2): drop v1 */
        cross3(v3, v2, tmp);
        if (dot3(tmp, v0) < 0.0) {
            v1[0] = v3[0]; v1[1] = v3[1]; v1[2] = v3[2];
            sub3(v3, v0, e1);
            sub3(v2, v0, e2);
            cross3(e1, e2, n);
            continue;
        }
        break;
    }

    /* portal refinement */
    for (;;) {
        if (++iter > MPR_MAX_ITER)
            return 1;
        EVENT(EV_MPR_ITER);
        sub3(v2, v1, e1);
        sub3(v3, v1, e2);
        cross3(e1, e2, n);
        if (dot3(n, v1) >= 0.0)
            return 1; /* origin behind the portal: inside D */
        support(&mk, n, v4);
        if (dot3(v4, n) <= 0.0)
            return 0; /* support plane separates the origin */
        sub3(v4, v3, tmp);
        double gap = dot3(tmp, n);
        if (gap <= 0.0 || gap * gap <= sh->tol2 * dot3(n, n))
            return 0; /* portal converged onto the boundary, origin beyond */
        /* keep the sub-triangle of (v1, v2, v3) split at v4 that the ray
         * from v0 through the origin crosses */
        cross3(v4, v0, tmp);
        if (dot3(v1, tmp) > 0.0) {
#ifdef ORACLE_PLANT_MPR_PORTAL
            if (dot3(v2, tmp) <= 0.0) {
#else
            if (dot3(v2, tmp) > 0.0) {
#endif
                v1[0] = v4[0]; v1[1] = v4[1]; v1[2] = v4[2];
            } else {
                v3[0] = v4[0]; v3[1] = v4[1]; v3[2] = v4[2];
            }
        } else {
            if (dot3(v3, tmp) > 0.0) {
                v2[0] = v4[0]; v2[1] = v4[1]; v2[2] = v4[2];
            } else {
                v1[0] = v4[0]; v1[1] = v4[1]; v1[2] = v4[2];
            }
        }
    }
}

static double norm2(const double *r, int dim)
{
    double s = r[0] * r[0] + r[1] * r[1];
    if (dim == 3)
        s = s + r[2] * r[2];
    return s;
}

static int full_test(const shape_t *sh, const double *r, const double *qa, const double *qb)
{
    if (sh->kind == OR_DISK)
        return norm2(r, 2) < sh->circ2;
    if (sh->kind == OR_POLYGON) {
        if (overlap_polygon(sh, r, qa, qb))
            return 1;
        return sh->sweep > 0.0 && polygon_cores_close(sh, r, qa, qb);
    }
    return overlap_polyhedron(sh, r, qa, qb);
}

static int pair_overlaps(const shape_t *sh, const double *r, const double *qa, const double *qb)
{
    if (!(norm2(r, sh->dim) < sh->circ2))
        return 0;
    return full_test(sh, r, qa, qb);
}

int or_overlap_full(const or_species *sp, const double *r, const double *qa, const double *qb)
{
    shape_t sh;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    return full_test(&sh, r, qa, qb);
}

int or_pair_overlaps(const or_species *sp, const double *r, const double *qa, const double *qb)
{
    shape_t sh;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    return pair_overlaps(&sh, r, qa, qb);
}

/* ------------------------------------------------------------------------ */
/* Cell grid (Sec. 2.2.1) and checkerboard (Sec. 2.5.2).                    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int dim, n, ncells, ncolours, rounds;
    double L, w, inv_w, inv_L;
} grid_t;

static int make_grid(const shape_t *sh, int32_t N, double L, int32_t rounds_req, grid_t *g)
{
    if (!(L > 0.0) || N < 0)
        return OR_ERR_INVALID_ARG;
    /* cells at least d_max wide (with a 2^-30 relative guard), an even
     * number per side so that same-coloured cells never touch across the
     * periodic boundary, and at least 4 per side */
    double nf = L / (sh->dmax * (1.0 + 0x1p-30));
    if (nf > 65536.0)
        return OR_ERR_INVALID_ARG;
    int n = (int)nf;
    n -= n & 1;
    if (n < 4)
        return OR_ERR_BOX_TOO_SMALL;
    if (sh->dim == 3 && n > 1024)
        return OR_ERR_INVALID_ARG;
    g->dim = sh->dim;
    g->n = n;
    g->L = L;
    g->w = L / (double)n;
    g->inv_w = (double)n / L;
    g->inv_L = 1.0 / L;
    g->ncells = sh->dim == 2 ? n * n : n * n * n;
    g->ncolours = 1 << sh->dim;
    if (rounds_req > 0) {
        g->rounds = rounds_req;
    } else {
        int r = (N + g->ncells / 2) / g->ncells; /* round(N / cells) */
        g->rounds = r < 1 ? 1 : r;
    }
    return OR_OK;
}

int or_grid(const or_species *sp, int32_t N, double L, int32_t *n, double *w, int32_t *rounds)
{
    shape_t sh;
    grid_t g;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    rc = make_grid(&sh, N, L, sp->rounds, &g);
    if (rc) return rc;
    *n = g.n;
    *w = g.w;
    *rounds = g.rounds;
    return OR_OK;
}

/* Cell coordinate of x along one axis of a grid shifted by s in (0, w). */
static int cell_coord(const grid_t *g, double x, double s)
{
    double y = x - s;
    if (y < 0.0)
        y = y + g->L;
    int j = (int)(y * g->inv_w);
    if (j > g->n - 1)
        j = g->n - 1;
    return j;
}

static int cell_linear(const grid_t *g, const int *c)
{
    if (g->dim == 2)
        return c[0] + g->n * c[1];
    return c[0] + g->n * (c[1] + g->n * c[2]);
}

static void cell_coords(const grid_t *g, int lin, int *c)
{
    c[0] = lin % g->n;
    c[1] = (lin / g->n) % g->n;
    if (g->dim == 3)
        c[2] = lin / (g->n * g->n);
}

static int cell_colour(const grid_t *g, const int *c)
{
    int k = (c[0] & 1) + 2 * (c[1] & 1);
    if (g->dim == 3)
        k += 4 * (c[2] & 1);
    return k;
}

/* Periodic wrap of a coordinate displaced by less than L. */
static double wrap(double x, double L)
{
    double y = x;
    if (x >= L)
        y = x - L;
    else if (x < 0.0)
        y = x + L;
    if (y >= L)
        y = 0.0;
    return y;
}

static double min_image(const grid_t *g, double r)
{
#ifdef ORACLE_PLANT_NO_MIN_IMAGE
    return r;
#endif
    return r - g->L * rint(r * g->inv_L);
}

typedef struct {
    int *count, *start, *members, *cell_of, *fill;
} cells_t;

static int cells_alloc(cells_t *cl, const grid_t *g, int N)
{
    cl->count = (int *)calloc((size_t)g->ncells, sizeof(int));
    cl->start = (int *)calloc((size_t)g->ncells + 1, sizeof(int));
    cl->members = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    cl->cell_of = (int *)calloc((size_t)(N > 0 ? N : 1), sizeof(int));
    cl->fill = (int *)calloc((size_t)g->ncells, sizeof(int));
    return cl->count && cl->start && cl->members && cl->cell_of && cl->fill ? OR_OK
                                                                            : OR_ERR_INVALID_ARG;
}

static void cells_free(cells_t *cl)
{
    free(cl->count);
    free(cl->start);
    free(cl->members);
    free(cl->cell_of);
    free(cl->fill);
}

/* Bucket sort of all particles into the grid shifted by s; each cell lists
 * its occupants in ascending tag order. */
static void cells_build(cells_t *cl, const grid_t *g, int N, const double *pos, const double *s)
{
    memset(cl->count, 0, sizeof(int) * (size_t)g->ncells);
    for (int i = 0; i < N; ++i) {
        int c[3] = { 0, 0, 0 };
        for (int a = 0; a < g->dim; ++a)
            c[a] = cell_coord(g, pos[a * N + i], s[a]);
        cl->cell_of[i] = cell_linear(g, c);
        cl->count[cl->cell_of[i]] += 1;
    }
    cl->start[0] = 0;
    for (int c = 0; c < g->ncells; ++c)
        cl->start[c + 1] = cl->start[c] + cl->count[c];
    memset(cl->fill, 0, sizeof(int) * (size_t)g->ncells);
    for (int i = 0; i < N; ++i) {
        int c = cl->cell_of[i];
        cl->members[cl->start[c] + cl->fill[c]] = i;
        cl->fill[c] += 1;
    }
}

static void load_orient(const shape_t *sh, int N, const double *orient, int i, double *q)
{
    if (sh->kind == OR_POLYGON) {
        q[0] = orient[i];
        q[1] = orient[N + i];
    } else if (sh->kind == OR_POLYHEDRON) {
        for (int k = 0; k < 4; ++k)
            q[k] = orient[k * N + i];
    }
}

static void store_orient(const shape_t *sh, int N, double *orient, int i, const double *q)
{
    if (sh->kind == OR_POLYGON) {
        orient[i] = q[0];
        orient[N + i] = q[1];
    } else if (sh->kind == OR_POLYHEDRON) {
        for (int k = 0; k < 4; ++k)
            orient[k * N + i] = q[k];
    }
}

/* Trial move r + dr or q . dq (Sec. 2.1 step 2) from one Philox block m:
 * m[0] decides translation vs rotation, m[1..dim] give the components. */
static int propose(const or_species *sp, const shape_t *sh, const grid_t *g, const uint32_t m[4],
                   const double *x, const double *q, double *xn, double *qn)
{
    int rotate = sp->p_rot > 0.0 && or_u01(m[0]) < sp->p_rot;
    for (int a = 0; a < sh->dim; ++a)
        xn[a] = x[a];
    for (int k = 0; k < 4; ++k)
        qn[k] = q[k];
    if (!rotate) {
        EVENT(EV_TRANSLATE);
        for (int a = 0; a < sh->dim; ++a) {
            double u = 2.0 * or_u01(m[1 + a]) - 1.0;
            xn[a] = wrap(x[a] + sp->d * u, g->L);
        }
    } else if (sh->kind == OR_POLYGON) {
        EVENT(EV_ROTATE2);
        double delta = sp->a * (2.0 * or_u01(m[1]) - 1.0);
        double cd, sd;
        or_sincos(delta, &cd, &sd);
        qn[0] = q[0] * cd - q[1] * sd;
        qn[1] = q[1] * cd + q[0] * sd;
    } else {
        EVENT(EV_ROTATE3);
        double dq[4] = { 1.0, 0.0, 0.0, 0.0 };
        for (int a = 0; a < 3; ++a)
            dq[1 + a] = sp->a * (2.0 * or_u01(m[1 + a]) - 1.0);
        double p[4];
#ifdef ORACLE_PLANT_LEFT_ROTATION
        quat_mul(dq, q, p);
#else
        quat_mul(q, dq, p);
#endif
        double nrm = sqrt(((p[0] * p[0] + p[1] * p[1]) + p[2] * p[2]) + p[3] * p[3]);
        for (int k = 0; k < 4; ++k)
            qn[k] = p[k] / nrm;
    }
    return rotate;
}

/* Does a trial configuration (xn, qn) of particle i overlap any particle of
 * the 3^dim cells around cell c (Sec. 2.2.1)? */
static int trial_overlaps(const shape_t *sh, const grid_t *g, const cells_t *cl, int N,
                          const double *pos, const double *orient, int i, int c,
                          const double *xn, const double *qn)
{
    int cc[3] = { 0, 0, 0 };
    cell_coords(g, c, cc);
    int o2lo = g->dim == 3 ? -1 : 0, o2hi = g->dim == 3 ? 1 : 0;
    for (int o2 = o2lo; o2 <= o2hi; ++o2)
        for (int o1 = -1; o1 <= 1; ++o1)
            for (int o0 = -1; o0 <= 1; ++o0) {
                int nb[3] = { (cc[0] + o0 + g->n) % g->n, (cc[1] + o1 + g->n) % g->n, 0 };
                if (g->dim == 3)
                    nb[2] = (cc[2] + o2 + g->n) % g->n;
                int cn = cell_linear(g, nb);
                for (int p = cl->start[cn]; p < cl->start[cn + 1]; ++p) {
                    int k = cl->members[p];
                    if (k == i)
                        continue;
                    EVENT(g->dim == 2 ? EV_CAND2 : EV_CAND3);
                    double r[3] = { 0.0, 0.0, 0.0 }, qk[4];
                    for (int a = 0; a < g->dim; ++a)
                        r[a] = min_image(g, pos[a * N + k] - xn[a]);
                    load_orient(sh, N, orient, k, qk);
                    if (pair_overlaps(sh, r, qn, qk))
                        return 1; /* early exit on the first overlap (Sec. 2.1) */
                }
            }
    return 0;
}

int or_sweep(const or_species *sp, int32_t N, double L, double *pos, double *orient,
             uint64_t seed, uint32_t replica, uint64_t t0, uint64_t n_sweeps, int64_t *stats)
{
    shape_t sh;
    grid_t g;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    rc = make_grid(&sh, N, L, sp->rounds, &g);
    if (rc) return rc;
    if (t0 + n_sweeps > 0x100000000ull || t0 + n_sweeps < t0)
        return OR_ERR_SWEEP_OVERFLOW;
    if ((uint64_t)g.rounds * (uint64_t)g.ncolours >= (1ull << 28))
        return OR_ERR_INVALID_ARG;
    cells_t cl;
    if (cells_alloc(&cl, &g, N)) {
        cells_free(&cl);
        return OR_ERR_INVALID_ARG;
    }
    for (uint64_t sw = 0; sw < n_sweeps; ++sw) {
        uint32_t t = (uint32_t)(t0 + sw);
        /* random grid shift in (0, w)^dim: the analogue of translating all
         * particles by one random vector per step (Sec. 2.5.1) */
        uint32_t sh_words[4];
        draw(seed, t, PURPOSE_SHIFT, 0, 0, replica, sh_words);
        double s[3];
        for (int a = 0; a < g.dim; ++a)
            s[a] = g.w * or_u01(sh_words[a]);
        cells_build(&cl, &g, N, pos, s);

        for (int rnd = 0; rnd < g.rounds; ++rnd)
            for (int colour = 0; colour < g.ncolours; ++colour) {
                uint32_t select = (uint32_t)(rnd * g.ncolours + colour);
                for (int c = 0; c < g.ncells; ++c) {
                    int cc[3] = { 0, 0, 0 };
                    cell_coords(&g, c, cc);
                    if (cell_colour(&g, cc) != colour || cl.count[c] == 0)
                        continue;
                    /* one trial move per non-empty active cell (Sec. 2.5.2):
                     * a uniformly chosen occupant */
                    uint32_t wsel[4];
                    draw(seed, t, PURPOSE_SELECT, select, (uint32_t)c, replica, wsel);
                    int i = cl.members[cl.start[c] + (int)or_index(wsel[0], (uint32_t)cl.count[c])];
                    uint32_t m[4];
                    draw(seed, t, PURPOSE_MOVE, select, (uint32_t)i, replica, m);
                    double x[3] = { 0, 0, 0 }, q[4] = { 1, 0, 0, 0 }, xn[3], qn[4];
                    for (int a = 0; a < g.dim; ++a)
                        x[a] = pos[a * N + i];
                    load_orient(&sh, N, orient, i, q);
                    stats[OR_ST_ATTEMPTED] += 1;
                    int rotate = propose(sp, &sh, &g, m, x, q, xn, qn);
                    if (rotate)
                        stats[OR_ST_ATTEMPTED_ROT] += 1;
                    /* a trial position outside the active cell is rejected */
                    int leaves = 0;
                    for (int a = 0; a < g.dim; ++a)
                        if (cell_coord(&g, xn[a], s[a]) != cc[a])
                            leaves = 1;
#ifdef ORACLE_PLANT_NO_CELL_RULE
                    leaves = 0;
#endif
                    if (leaves) {
                        stats[OR_ST_CELL_REJECT] += 1;
                        continue;
                    }
                    if (trial_overlaps(&sh, &g, &cl, N, pos, orient, i, c, xn, qn)) {
                        stats[OR_ST_OVERLAP_REJECT] += 1;
                        continue;
                    }
                    for (int a = 0; a < g.dim; ++a)
                        pos[a * N + i] = xn[a];
                    store_orient(&sh, N, orient, i, qn);
                    stats[OR_ST_ACCEPT] += 1;
                }
            }
    }
    cells_free(&cl);
    return OR_OK;
}

int or_pair_histogram(int32_t dim, int32_t N, double L, const double *pos,
                      const double *edges2, int32_t n_bins, int64_t *out)
{
    if ((dim != 2 && dim != 3) || N < 0 || !(L > 0.0) || n_bins < 1 || !edges2 || !out)
        return OR_ERR_INVALID_ARG;
    for (int b = 0; b < n_bins; ++b)
        if (!(edges2[b] < edges2[b + 1]))
            return OR_ERR_INVALID_ARG;
    grid_t g;
    memset(&g, 0, sizeof(g));
    g.L = L;
    g.inv_L = 1.0 / L;
    for (int b = 0; b < n_bins; ++b)
        out[b] = 0;
    for (int i = 0; i < N; ++i)
        for (int k = i + 1; k < N; ++k) {
            double r[3] = { 0.0, 0.0, 0.0 };
            for (int a = 0; a < dim; ++a)
                r[a] = min_image(&g, pos[a * N + k] - pos[a * N + i]);
            double r2 = r[0] * r[0] + r[1] * r[1];
            if (dim == 3)
                r2 = r2 + r[2] * r[2];
            for (int b = 0; b < n_bins; ++b)
                if (edges2[b] <= r2 && r2 < edges2[b + 1])
                    ++out[b];
        }
    return OR_OK;
}

int or_scale_positions(int32_t dim, int32_t N, double L, double L_new, double *pos)
{
    if ((dim != 2 && dim != 3) || N < 0 || !(L > 0.0) || !(L_new > 0.0) || !pos)
        return OR_ERR_INVALID_ARG;
    double k = L_new / L;
    for (int a = 0; a < dim; ++a)
        for (int i = 0; i < N; ++i)
            pos[a * N + i] = wrap(pos[a * N + i] * k, L_new);
    return OR_OK;
}

int or_scale_counts(const or_species *sp, int32_t N, double L, const double *pos,
                    const double *orient, const double *s, int32_t n_s, int64_t *out)
{
    shape_t sh;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    if (N < 0 || !(L > 0.0) || n_s < 1 || !s || !out || !pos)
        return OR_ERR_INVALID_ARG;
    for (int b = 0; b < n_s; ++b)
        if (!(s[b] >= 0.0 && s[b] < 1.0) || (b > 0 && !(s[b - 1] < s[b])))
            return OR_ERR_INVALID_ARG;
    grid_t g;
    memset(&g, 0, sizeof(g));
    g.L = L;
    g.inv_L = 1.0 / L;
    for (int b = 0; b < n_s; ++b)
        out[b] = 0;
    for (int i = 0; i < N; ++i) {
        double qi[4] = { 1, 0, 0, 0 };
        load_orient(&sh, N, orient, i, qi);
        for (int k = i + 1; k < N; ++k) {
            double r[3] = { 0.0, 0.0, 0.0 }, qk[4] = { 1, 0, 0, 0 };
            for (int a = 0; a < sh.dim; ++a)
                r[a] = min_image(&g, pos[a * N + k] - pos[a * N + i]);
            load_orient(&sh, N, orient, k, qk);
            for (int b = 0; b < n_s; ++b) {
                double f = 1.0 - s[b];
                double rs[3] = { r[0] * f, r[1] * f, r[2] * f };
                out[b] += pair_overlaps(&sh, rs, qi, qk);
            }
        }
    }
    return OR_OK;
}

int64_t or_count_overlaps(const or_species *sp, int32_t N, double L, const double *pos,
                          const double *orient)
{
    shape_t sh;
    grid_t g;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    rc = make_grid(&sh, N, L, sp->rounds, &g);
    if (rc) return rc;
    cells_t cl;
    if (cells_alloc(&cl, &g, N)) {
        cells_free(&cl);
        return OR_ERR_INVALID_ARG;
    }
    double s[3] = { 0.0, 0.0, 0.0 };
    cells_build(&cl, &g, N, pos, s);
    int64_t total = 0;
    for (int i = 0; i < N; ++i) {
        int cc[3] = { 0, 0, 0 };
        cell_coords(&g, cl.cell_of[i], cc);
        double qi[4] = { 1, 0, 0, 0 };
        load_orient(&sh, N, orient, i, qi);
        int o2lo = g.dim == 3 ? -1 : 0, o2hi = g.dim == 3 ? 1 : 0;
        for (int o2 = o2lo; o2 <= o2hi; ++o2)
            for (int o1 = -1; o1 <= 1; ++o1)
                for (int o0 = -1; o0 <= 1; ++o0) {
                    int nb[3] = { (cc[0] + o0 + g.n) % g.n, (cc[1] + o1 + g.n) % g.n, 0 };
                    if (g.dim == 3)
                        nb[2] = (cc[2] + o2 + g.n) % g.n;
                    int cn = cell_linear(&g, nb);
                    for (int p = cl.start[cn]; p < cl.start[cn + 1]; ++p) {
                        int k = cl.members[p];
#ifdef ORACLE_PLANT_COUNT_OWN_CELL_ONLY
                        if (o0 != 0 || o1 != 0 || o2 != 0)
                            continue;
#endif
                        if (k <= i)
                            continue;
                        double r[3] = { 0.0, 0.0, 0.0 }, qk[4] = { 1, 0, 0, 0 };
                        for (int a = 0; a < g.dim; ++a)
                            r[a] = min_image(&g, pos[a * N + k] - pos[a * N + i]);
                        load_orient(&sh, N, orient, k, qk);
                        total += pair_overlaps(&sh, r, qi, qk);
                    }
                }
    }
    cells_free(&cl);
    return total;
}

int or_serial_metropolis(const or_species *sp, int32_t N, double L, double *pos,
                         double *orient, uint64_t seed, uint64_t move0, uint64_t n_moves,
                         int64_t *stats)
{
    shape_t sh;
    grid_t g;
    int rc = setup_shape(sp, &sh);
    if (rc) return rc;
    rc = make_grid(&sh, N, L, sp->rounds, &g);
    if (rc) return rc;
    if (N < 2)
        return OR_ERR_INVALID_ARG;
    for (uint64_t mv = move0; mv < move0 + n_moves; ++mv) {
        uint32_t lo = (uint32_t)mv, hi = (uint32_t)(mv >> 32) & 0x0FFFFFFFu;
        uint32_t wsel[4], m[4];
        /* 1. select a particle at random (Sec. 2.1) */
        draw(seed, lo, PURPOSE_SERIAL_SELECT, hi, 0, 0, wsel);
        int i = (int)or_index(wsel[0], (uint32_t)N);
        /* 2. small random trial move */
        draw(seed, lo, PURPOSE_SERIAL_MOVE, hi, 0, 0, m);
        double x[3] = { 0, 0, 0 }, q[4] = { 1, 0, 0, 0 }, xn[3], qn[4];
        for (int a = 0; a < g.dim; ++a)
            x[a] = pos[a * N + i];
        load_orient(&sh, N, orient, i, q);
        stats[OR_ST_ATTEMPTED] += 1;
        if (propose(sp, &sh, &g, m, x, q, xn, qn))
            stats[OR_ST_ATTEMPTED_ROT] += 1;
        /* 3. check against all other particles */
        int hit = 0;
        for (int k = 0; k < N && !hit; ++k) {
            if (k == i)
                continue;
            double r[3] = { 0.0, 0.0, 0.0 }, qk[4] = { 1, 0, 0, 0 };
            for (int a = 0; a < g.dim; ++a)
                r[a] = min_image(&g, pos[a * N + k] - xn[a]);
            load_orient(&sh, N, orient, k, qk);
            hit = pair_overlaps(&sh, r, qn, qk);
        }
        /* 4. reject on overlap, else accept */
        if (hit) {
            stats[OR_ST_OVERLAP_REJECT] += 1;
            continue;
        }
        for (int a = 0; a < g.dim; ++a)
            pos[a * N + i] = xn[a];
        store_orient(&sh, N, orient, i, qn);
        stats[OR_ST_ACCEPT] += 1;
    }
    return OR_OK;
}
