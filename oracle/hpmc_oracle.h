/*
 * HPMC reference oracle -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, serial FP64 CPU implementation of the checkerboard-parallel
 * hard-shape Metropolis sweep of Anderson, Irrgang and Glotzer, "Scalable
 * Metropolis Monte Carlo for simulation of hard shapes" (HPMC).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or helper with the GPU library.
 *
 * Layouts (all caller-owned host memory):
 *   pos    : structure of arrays, pos[a*N + i] is coordinate a of particle i,
 *            a < dim, particles in canonical (tag) order, values in [0, L).
 *   orient : 2D polygons: orient[i] = c_i, orient[N + i] = s_i (unit complex);
 *            3D polyhedra: orient[k*N + i], k = 0..3 -> quaternion (w,x,y,z);
 *            disks: unused (may be NULL).
 *   verts  : n_verts rows of dim doubles, particle frame; polygons CCW.
 *
 * Return codes: 0 on success, negative on error (see OR_ERR_*).
 */
#ifndef HPMC_ORACLE_H
#define HPMC_ORACLE_H

#include <stdint.h>

#define OR_DISK 0
#define OR_POLYGON 1
#define OR_POLYHEDRON 2

#define OR_OK 0
#define OR_ERR_INVALID_ARG (-1)
#define OR_ERR_BOX_TOO_SMALL (-2)
#define OR_ERR_SWEEP_OVERFLOW (-6)

#define OR_MAXV 64

/* Counters of one sweep call; index order of the int64 stats array. */
#define OR_ST_ATTEMPTED 0
#define OR_ST_ATTEMPTED_ROT 1
#define OR_ST_CELL_REJECT 2
#define OR_ST_OVERLAP_REJECT 3
#define OR_ST_ACCEPT 4
#define OR_NSTATS 5

typedef struct {
    int32_t dim;          /* 2 or 3 */
    int32_t shape;        /* OR_DISK, OR_POLYGON, OR_POLYHEDRON */
    int32_t n_verts;      /* polygons / polyhedra */
    const double *verts;  /* n_verts x dim, particle frame */
    double diameter;      /* disks */
    double d;             /* translation half width */
    double a;             /* rotation size */
    double p_rot;         /* probability that a move is a rotation */
    int32_t rounds;       /* colour rounds per sweep, 0 = automatic */
    double sweep_radius;  /* polygons and polyhedra: the shape is every point
                             within this distance of the convex hull of verts
                             (a spheropolygon / spheropolyhedron, Sec. 2.3);
                             0 = the hull itself.  With sweep_radius > 0,
                             1..OR_MAXV vertices (one vertex: a disk or
                             sphere, two: a stadium or spherocylinder). */
} or_species;

void or_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4]);
/* n counters (4 words each, consecutive) under one key, for bulk checks. */
void or_philox4x32_10_many(const uint32_t *ctr, int64_t n, const uint32_t key[2], uint32_t *out);
double or_u01(uint32_t w);
uint32_t or_index(uint32_t w, uint32_t n);
void or_sincos(double delta, double *c, double *s);

/* out[0] = R (circumradius), out[1] = d_max, out[2] = circumsphere threshold
 * (R+R)^2, out[3] = squared XenoCollide tolerance. */
int or_shape_info(const or_species *sp, double out[4]);

/* n (even cells per side), w, rounds per sweep. */
int or_grid(const or_species *sp, int32_t N, double L, int32_t *n, double *w,
            int32_t *rounds);

/* Full overlap test of B against A in A's frame; r = min-image r_B - r_A
 * (world frame, dim values), qa/qb = orientations (2 or 4 values, unused
 * for disks).  Returns 1 (overlap), 0 (no overlap) or a negative error. */
int or_overlap_full(const or_species *sp, const double *r, const double *qa,
                    const double *qb);

/* Circumsphere test AND full test: the exact predicate of a pair. */
int or_pair_overlaps(const or_species *sp, const double *r, const double *qa,
                     const double *qb);

/* Number of unordered overlapping pairs (i < k) of one system. */
int64_t or_count_overlaps(const or_species *sp, int32_t N, double L,
                          const double *pos, const double *orient);

/* Histogram of pair separations, the sampling behind the pressure check of
 * Sec. 4 (contact value of g(r)): out[b] = number of unordered pairs i < k
 * with edges2[b] <= r^2 < edges2[b+1], r the minimum-image separation of
 * particle k from particle i, r^2 = (x^2 + y^2) (+ z^2).  edges2: n_bins + 1
 * ascending squared distances.  Every pair is visited (no cell list). */
int or_pair_histogram(int32_t dim, int32_t N, double L, const double *pos,
                      const double *edges2, int32_t n_bins, int64_t *out);

/* Compressions behind the volume-perturbation pressure of Sec. 4: out[b] =
 * number of unordered pairs i < k that overlap (circumsphere test, then the
 * full test) once their minimum-image separation r is replaced by r (1 - s[b])
 * with orientations unchanged, i.e. after the box is shrunk by the scale
 * factor s[b].  s: n_s strictly ascending values in [0, 1).  Every pair is
 * visited (no cell list). */
int or_scale_counts(const or_species *sp, int32_t N, double L, const double *pos,
                    const double *orient, const double *s, int32_t n_s, int64_t *out);

/* Isotropic box change of an NPT volume move (Sec. 1 names the NPT
 * ensemble): every coordinate x in [0, L) becomes x * (L_new / L), wrapped
 * into [0, L_new) (x' >= L_new gives x' - L_new, and 0 if still >= L_new).
 * The scale factor is one binary64 division, each coordinate one product. */
int or_scale_positions(int32_t dim, int32_t N, double L, double L_new, double *pos);

/* n_sweeps checkerboard sweeps of one system, sweep counter t0, t0+1, ...
 * Updates pos / orient in place and ADDS to stats[OR_NSTATS]. */
int or_sweep(const or_species *sp, int32_t N, double L, double *pos,
             double *orient, uint64_t seed, uint32_t replica, uint64_t t0,
             uint64_t n_sweeps, int64_t *stats);

/* Serial one-move-at-a-time Metropolis (statistical reference only):
 * n_moves moves, each on a particle chosen uniformly from all N, overlap
 * checks against all other particles.  Adds to stats (no cell rejects). */
int or_serial_metropolis(const or_species *sp, int32_t N, double L,
                         double *pos, double *orient, uint64_t seed,
                         uint64_t move0, uint64_t n_moves, int64_t *stats);

#endif
