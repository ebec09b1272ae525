/*
 * hpmc.h -- C ABI of the MI355X (gfx950) checkerboard hard-shape Monte Carlo
 * library (libhpmc.so).
 *
 * The library runs the checkerboard-parallel Metropolis sweep of hard shapes
 * of Anderson, Irrgang and Glotzer, "Scalable Metropolis Monte Carlo for
 * simulation of hard shapes" (HPMC):
 *   - Metropolis for hard particles: select a particle, propose a small
 *     translation r + dr or rotation q . dq, reject it if the trial shape
 *     overlaps any other particle, otherwise accept (Sec. 2.1);
 *   - a cell list whose cells are at least d_max wide, searched over the own
 *     cell and its neighbours +-1 per axis (Sec. 2.2.1);
 *   - overlap checks in the frame of one particle, positions in FP64 and
 *     orientations as unit complex numbers / quaternions (Sec. 2.3, Eqs. 1-2);
 *   - one trial move per non-empty active cell of a 2^dim-colour checkerboard,
 *     moves leaving their cell rejected, a random offset per sweep
 *     (Sec. 2.5.1-2.5.2), random numbers from a counter-based stream per move
 *     (Sec. 2.5).
 * One sweep is N trial moves (Sec. 2): rounds x 2^dim colour passes, each
 * making one move in every non-empty cell of that colour.
 *
 * Memory: every device buffer is owned by the caller (the Python binding
 * allocates them with PyTorch) and must stay alive until hpmc_destroy().
 * The library never allocates device memory: all scratch lives in the
 * caller's workspace.  Host arrays passed to hpmc_init are copied.
 *
 * Streams and threads: a state is bound to one HIP stream (passed as void*,
 * NULL = the default stream) and is not thread safe.  Distinct states on
 * distinct streams are independent.  hpmc_sweep is asynchronous; calls that
 * return data to the host synchronise the stream.  A batch of several shape
 * kinds on the persistent path runs the kinds' launches on private streams
 * of the state, forked from and joined back to its stream, so work enqueued
 * on that stream afterwards still sees every sweep complete.
 *
 * Errors: every call returns HPMC_OK (0) or a negative HPMC_ERR_* code and
 * never throws.  Device faults surface at the next synchronising call.
 */
#ifndef HPMC_H
#define HPMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HPMC_OK 0
#define HPMC_ERR_INVALID_ARG (-1)         /* malformed arguments or shape */
#define HPMC_ERR_BOX_TOO_SMALL (-2)       /* fewer than 4 cells per side */
#define HPMC_ERR_INITIAL_OVERLAP (-3)     /* hpmc_init found overlapping pairs */
#define HPMC_ERR_WORKSPACE_TOO_SMALL (-4) /* workspace_bytes below requirement */
#define HPMC_ERR_HIP (-5)                 /* a HIP runtime call failed */
#define HPMC_ERR_SWEEP_OVERFLOW (-6)      /* sweep counter would reach 2^32 */
#define HPMC_ERR_UNSUPPORTED (-7)         /* valid request the library does not support */
#define HPMC_ERR_CELL_OVERFLOW (-8)       /* a persistent 2D cell list outgrew its ghost-column
                                             slots: only a state with overlaps written into
                                             the caller's arrays can do that; the sweeps
                                             stopped without moving a particle */

/* The persistent path launches one kernel per this many sweeps (a call of
 * n sweeps: n / 64 such launches, then one launch of the n % 64 left). */
#define HPMC_PERSISTENT_SWEEPS_PER_LAUNCH 64

/* Largest rotation size a (radians) of a polygon species.  The 2D move
 * rotates the unit complex orientation by cos/sin polynomials truncated after
 * the delta^16 / delta^15 terms and never renormalises it; below this bound
 * the first dropped term (delta^17 / 17!) is under 2^-53, so |z| drifts only
 * by rounding.  Larger a: HPMC_ERR_INVALID_ARG. */
#define HPMC_MAX_POLYGON_ROTATION 0.75

/* hpmc_init_args.flags */
#define HPMC_FLAG_NO_GRAPH 1 /* launch kernels directly instead of replaying a hipGraph */
/* How the full overlap tests of a colour pass are scheduled (Sec. 2.5.3).  The
 * default is the block work queue, kept per wave64 in LDS.  The two flags
 * below select the variants the paper measured it against; they exist for
 * comparison, give the same trajectory (only pair_tests differ), run on the
 * GRID path only (PERSISTENT with either flag: HPMC_ERR_UNSUPPORTED; AUTO
 * then means GRID) and are mutually exclusive (HPMC_ERR_INVALID_ARG).
 *   REGISTER_QUEUE: each lane pre-filters its candidates up to its first hit;
 *     the wave then runs the full tests of all lanes holding one.
 *   GLOBAL_QUEUE: three kernels per pass (propose and pre-filter into a queue
 *     in the workspace, test every queued pair, apply); no early exit; the
 *     workspace grows by about 64 bytes per particle and 60 per cell. */
#define HPMC_FLAG_REGISTER_QUEUE 2
#define HPMC_FLAG_GLOBAL_QUEUE 4

/* Opaque host-side handle of one set of replicas. */
typedef struct hpmc_state hpmc_state;

typedef enum { HPMC_DISK = 0, HPMC_POLYGON = 1, HPMC_POLYHEDRON = 2 } hpmc_shape;

/* FP64: every overlap decision in binary64, in the pinned operation order.
 * MIXED: overlap tests in binary32 with a rigorous forward-error margin; a
 * pair whose binary32 result falls inside the margin is re-evaluated in
 * binary64, so every decision equals the FP64 decision (the paper's mixed
 * mode, Sec. 2.3, trusts binary32 outright; this one does not). */
typedef enum { HPMC_FP64 = 0, HPMC_MIXED = 1 } hpmc_precision;

/* GRID: one kernel per colour pass over a cell list in global memory, for
 * large systems.  PERSISTENT: one work-group per replica runs whole sweeps
 * with the cell list in LDS (small systems and batches).  AUTO picks. */
typedef enum { HPMC_PATH_AUTO = 0, HPMC_PATH_GRID = 1, HPMC_PATH_PERSISTENT = 2 } hpmc_path;

/* One particle type (all particles of a replica share it), the parameters of
 * the paper's job script (Fig. 1): vertices in the particle frame, move
 * sizes d and a. */
typedef struct {
    int32_t dim;          /* 2 (disk, polygon) or 3 (polyhedron) */
    int32_t shape;        /* hpmc_shape */
    int32_t n_verts;      /* polygon: 3..8 (CCW, strictly convex), or 1..8 with
                             sweep_radius > 0; polyhedron: 4..64, or 1..64 with
                             sweep_radius > 0 */
    const double *verts;  /* host, n_verts x dim row-major; NULL for disks */
    double diameter;      /* disks */
    double d;             /* translation: each component uniform in [-d, d] */
    double a;             /* rotation: 2D angle uniform in [-a, a], a at most
                             HPMC_MAX_POLYGON_ROTATION; 3D dq = (1, v),
                             v uniform in [-a, a]^3, renormalised */
    double p_rot;         /* probability that a move is a rotation (0 for disks) */
    int32_t rounds;       /* colour rounds per sweep; 0 = max(1, round(N / cells)) */
    double sweep_radius;  /* polygons and polyhedra: the particle is every point
                             within this distance of the vertices' convex hull
                             (a spheropolygon or spheropolyhedron, Sec. 2.3;
                             one vertex gives a disk / sphere, two a stadium /
                             spherocylinder); 0 for the hull itself and for
                             disks.  Swept shapes are always tested in binary64
                             (spheropolygons: the cores overlap or pass closer
                             than twice the radius; spheropolyhedra:
                             XenoCollide); spheropolygons need the wave queue. */
} hpmc_species;

typedef struct {
    int32_t n_replicas;            /* >= 1 independent systems */
    const hpmc_species *species;   /* host, n_replicas entries */
    const int32_t *N;              /* host, particles per replica (1 .. 2^26 - 1) */
    const double *L;               /* host, periodic box side per replica */
    int32_t precision;             /* hpmc_precision */
    int32_t path;                  /* hpmc_path */
    /* Device, caller-owned, canonical particle order, replicas concatenated.
     * pos: replica r occupies dim_r * N_r doubles, coordinate a of particle i
     *      at [a * N_r + i], all values in [0, L_r).
     * orient: replica r occupies k_r * N_r doubles (k = 0 disk, 2 polygon
     *      (c, s), 4 polyhedron (w, x, y, z)), component k of particle i at
     *      [k * N_r + i]; may be NULL when every replica is a disk. */
    double *pos;
    double *orient;
    void *workspace;               /* device, caller-owned, 256-byte aligned */
    size_t workspace_bytes;
    void *stream;                  /* hipStream_t or NULL */
    int32_t flags;                 /* HPMC_FLAG_* */
    const double *L_max;           /* host, per replica: largest box side that
                                      hpmc_scale_box may set (>= L; the cell
                                      lists are sized for it); NULL = L */
} hpmc_init_args;

/* Per-replica counters since init or the last hpmc_reset_stats. */
typedef struct {
    uint64_t attempted;      /* trial moves, including cell-boundary rejects */
    uint64_t attempted_rot;  /* of which rotations */
    uint64_t cell_reject;    /* trial position left the active cell */
    uint64_t overlap_reject; /* trial shape overlapped a neighbour */
    uint64_t accept;
    uint64_t pair_tests;     /* full (non-circumsphere) overlap tests run */
    uint64_t pair_fp64;      /* of which decided in binary64 (all, in FP64 mode;
                                the re-checked ones, in MIXED mode) */
    uint64_t sweeps;         /* sweeps completed */
} hpmc_stats;

/* Workspace size for these arguments (pos/orient/workspace may be NULL). */
int hpmc_workspace_bytes(const hpmc_init_args *args, size_t *out_bytes);

/* Validate, build the shape tables and grids, copy them to the workspace and
 * count overlaps of the initial state (HPMC_ERR_INITIAL_OVERLAP if any).
 * Synchronises the stream.  On success *out owns a host handle. */
int hpmc_init(hpmc_state **out, const hpmc_init_args *args);

/* n_sweeps sweeps of every replica with Philox key = seed and sweep counter
 * t, t+1, ... continuing from the state's counter (so two calls of a and b
 * sweeps equal one call of a + b).  Asynchronous on the state's stream. */
int hpmc_sweep(hpmc_state *st, uint64_t n_sweeps, uint64_t seed);

/* Time the launch configurations this state can use over trial_sweeps
 * sweeps each, keep the fastest, and restore positions, orientations,
 * counters and the sweep counter exactly.  The trajectory does not depend
 * on the configuration.  Three stages, each keeping the fastest so far:
 *   1. grid path: lanes per active cell 1, 2, 4, ..., 64 (1 .. 8 with the
 *      register queue, 1 with the global queue); persistent path: the LDS
 *      residency level (0: particle data in global memory, 1: positions in
 *      LDS, 2: positions and orientations, 3: both, without the binary32
 *      cell-sorted copy); with HPMC_MIXED and polyhedra also the binary64
 *      XenoCollide walk (its decisions equal the certified binary32 walk's);
 *   2. the queue depth (wave queue only): a wave drains its queued full
 *      tests once 64, 32 or 16 wait;
 *   3. persistent path: the work-group size, the default (enough lanes for
 *      one 64-cell tile per wave), half or a quarter of it (at least 64).
 * Synchronising.  *out_config (may be NULL) receives the chosen
 * configuration: lanes per cell or residency level in bits 0-7, 0x100 for
 * the binary64 walk, the queue depth code (0: 64, 1: 32, 2: 16) in bits 9-10
 * and the work-group size code (0: default, 1: half, 2: quarter) in bits
 * 11-12. */
int hpmc_autotune(hpmc_state *st, uint32_t trial_sweeps, int32_t *out_config);

/* Apply a launch configuration in the encoding hpmc_autotune returns, e.g. one
 * found by an earlier autotuning run of the same kind of system.  Any listed
 * configuration gives the same trajectory.  Synchronising.  Returns
 * HPMC_ERR_INVALID_ARG for a configuration this state cannot use. */
int hpmc_set_config(hpmc_state *st, int32_t config);

/* Box change of an NPT volume move (Sec. 1: the paper runs NVT and NPT
 * ensembles): every coordinate of replica r becomes x * (L_new / L) (one
 * binary64 division for the factor, one product per coordinate), wrapped into
 * [0, L_new) (x' >= L_new gives x' - L_new, and 0 if still >= L_new); the
 * replica's grid is rebuilt for L_new (largest even n with cells at least
 * d_max wide) and *overlaps (host, may be NULL) receives the number of
 * overlapping pairs of the scaled state.  The replica's previous positions
 * and box are kept until its next hpmc_scale_box or hpmc_restore_box, or
 * any hpmc_autotune of the state.  HPMC_ERR_INVALID_ARG for L_new <= 0 or above the replica's
 * L_max, HPMC_ERR_BOX_TOO_SMALL below 4 cells per side (nothing changes then).
 * Orientations are unchanged.  Synchronising. */
int hpmc_scale_box(hpmc_state *st, int32_t replica, double L_new, uint64_t *overlaps);

/* Undo the last hpmc_scale_box of replica r exactly (positions and box), as
 * after a rejected volume move.  HPMC_ERR_INVALID_ARG when there is nothing
 * to undo.  Synchronising. */
int hpmc_restore_box(hpmc_state *st, int32_t replica);

/* One isotropic volume move of replica r in the isobaric ensemble (Sec. 1:
 * the paper samples NVT and NPT; the move is the textbook one for hard
 * particles).  With V = L^dim (pow) and the caller's uniforms u1, u2 in
 * [0, 1): dV = delta_v (2 u1 - 1), V' = V + dV, L' = V'^(1/dim) (pow).  The
 * move is rejected, leaving the replica unchanged, when V' <= 0, L' > L_max,
 * the box L' has fewer than 4 cells per side, or dV < 0 and the scaled state
 * (hpmc_scale_box) has an overlapping pair; otherwise it is accepted iff
 * arg >= 0 or u2 < exp(arg), arg = -beta_p dV + N log(V' / V) (beta_p =
 * pressure / kT).  *accepted (host) receives 1 or 0 and *L_after (host, may
 * be NULL) the box side afterwards.  An accepted move leaves the previous box
 * restorable with hpmc_restore_box.  HPMC_ERR_INVALID_ARG for u1 or u2
 * outside [0, 1), a non-finite beta_p or a negative or non-finite delta_v.
 * Synchronising. */
int hpmc_volume_move(hpmc_state *st, int32_t replica, double u1, double u2, double beta_p,
                     double delta_v, int32_t *accepted, double *L_after);

/* Volume-perturbation counts of one replica, the sampling behind the
 * pressure of particles with shape (Sec. 4): out[b] = number of unordered
 * pairs i < k that overlap (circumsphere test, then the full binary64 test)
 * once their minimum-image separation r is replaced by r (1 - scales[b]) --
 * the box shrunk by that factor -- with orientations unchanged.  scales:
 * host, n_scales (1..64) strictly ascending values in [0, 1); out: host,
 * n_scales counts.  HPMC_ERR_UNSUPPORTED when 2R / (1 - scales[n_scales - 1])
 * exceeds two cell widths (or one, with fewer than 5 cells per side).
 * Synchronising; the state is unchanged. */
int hpmc_scale_counts(hpmc_state *st, int32_t replica, const double *scales, int32_t n_scales,
                      uint64_t *out);

/* Histogram of pair separations of one replica, the sampling behind the
 * pressure check of Sec. 4 (the contact value of g(r) for disks, Table 1):
 * out[b] = number of unordered pairs i < k with
 * edges2[b] <= r^2 < edges2[b + 1], r the minimum-image centre separation in
 * binary64 (x^2 + y^2 (+ z^2), the circumsphere test's expression).
 * edges2: host, n_bins + 1 strictly increasing squared distances, edges2[0]
 * >= 0, 1 <= n_bins <= 64, edges2[n_bins] below (2 w)^2 with w the cell
 * width (below w^2 when the grid has fewer than 5 cells per side), else
 * HPMC_ERR_UNSUPPORTED.  out: host, n_bins counts.  Reads the caller's
 * position array; synchronising. */
int hpmc_pair_histogram(hpmc_state *st, int32_t replica, const double *edges2, int32_t n_bins,
                        uint64_t *out);

/* Unordered overlapping pairs per replica under the exact FP64 predicate
 * (circumsphere test and full test, the paper's system-level check, Sec. 4).
 * out_per_replica: host, n_replicas entries.  Synchronising. */
int hpmc_count_overlaps(hpmc_state *st, uint64_t *out_per_replica);

/* Counters per replica.  out_per_replica: host, n_replicas entries.
 * Synchronising.  HPMC_ERR_CELL_OVERFLOW (counters still filled in) when a
 * persistent sweep since the last reset stopped on a cell-list overflow. */
int hpmc_get_stats(hpmc_state *st, hpmc_stats *out_per_replica);
int hpmc_reset_stats(hpmc_state *st);

/* Make the caller's pos / orient arrays current (the state works on them in
 * place, so this only synchronises the stream). */
int hpmc_sync_to_canonical(hpmc_state *st);

/* Sweep counter, for checkpoint and resume. */
int hpmc_get_sweep(hpmc_state *st, uint64_t *out_t);
int hpmc_set_sweep(hpmc_state *st, uint64_t t);

/* Cells per side, rounds per sweep and path chosen for replica r. */
int hpmc_replica_info(hpmc_state *st, int32_t r, int32_t *cells_per_side, int32_t *rounds,
                      int32_t *path);

/* 1 if sweeps replay a captured hipGraph, 0 if kernels are launched directly. */
int hpmc_uses_graph(hpmc_state *st);

/* Sweeps run since hpmc_init by replaying the captured hipGraph (the rest ran
 * as direct launches: HPMC_FLAG_NO_GRAPH, or a failed capture or replay). */
int hpmc_graph_sweeps(hpmc_state *st, uint64_t *out);

/* Per-wave phase clock of a trace build (compiled with -DHPMC_TRACE; the
 * normal build returns HPMC_ERR_UNSUPPORTED).  out (host, n >= 24 words)
 * receives, for the persistent batch kernel and then the grid path's colour
 * pass, the shader-clock cycles that all their waves together spent in each
 * of 11 phases -- cell-list build, trial move, pre-filter scan, queued full
 * tests, write-back, waiting at the barrier after a pass, other, and the
 * persistent kernel's in-LDS build split into counting, prefix sum, scatter
 * and in-cell ordering (its first phase then holds only the clearing of the
 * counts) -- followed by the number of waves, summed over every launch since
 * the last reset.  The device is synchronised first; reset != 0 clears the
 * totals. */
int hpmc_phase_trace(uint64_t *out, int32_t n, int32_t reset);

/* The hipError_t of the last failed HIP call of this state (0 if none); with
 * st = NULL, that of the last hpmc_init that failed in a HIP call. */
int hpmc_last_hip_error(hpmc_state *st);

void hpmc_destroy(hpmc_state *st);
const char *hpmc_strerror(int code);

/* Bytes of the library's own device scratch, used by hpmc_sweep_static. */
#define HPMC_STATIC_SCRATCH_BYTES (64u << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid hipMalloc): hpmc_init +
 * hpmc_set_sweep(t0) + hpmc_sweep(n_sweeps, seed) + hpmc_get_stats in one
 * call that allocates nothing.  The tables, cell lists and counters live in
 * a static device array of HPMC_STATIC_SCRATCH_BYTES (64 MiB) that each GPU
 * the library runs on holds until the process ends; the caller still passes
 * pos / orient (device, updated in place, the hpmc_init layout).
 * args->workspace must be NULL and workspace_bytes 0 (else
 * HPMC_ERR_INVALID_ARG); HPMC_FLAG_NO_GRAPH is implied (kernels launch
 * directly on args->stream, the launches of several shape kinds one after
 * another); the register and global queue flags give HPMC_ERR_UNSUPPORTED.
 * A batch whose workspace (without the autotuning and box-move snapshots)
 * exceeds the scratch gives HPMC_ERR_WORKSPACE_TOO_SMALL before any device
 * work.  Positions must lie in [0, L) and orientations be finite
 * (HPMC_ERR_INVALID_ARG otherwise); the initial state is not checked for
 * overlaps.  The trajectory equals the hpmc_init / hpmc_sweep one bit for
 * bit.  out_per_replica (host, may be NULL) receives the counters of these
 * sweeps; *hip_error (may be NULL) the hipError_t of a failed HIP call, else
 * 0.  Synchronising.  Every call on one GPU shares that GPU's scratch and
 * overwrites it: calls that overlap in time on one GPU (other host threads
 * or streams) race and must be serialised by the caller. */
int hpmc_sweep_static(const hpmc_init_args *args, uint64_t t0, uint64_t n_sweeps, uint64_t seed,
                      hpmc_stats *out_per_replica, int32_t *hip_error);

#ifdef __cplusplus
}
#endif

#endif /* HPMC_H */
