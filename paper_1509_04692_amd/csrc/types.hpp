// Tables shared by the host side of the library and its kernels.
#pragma once

#include <cstdint>

namespace hpmc {

constexpr int kMaxPolyVerts = 8;     // polygons: 3..8 vertices
constexpr int kMaxPolyhedronVerts = 64;
constexpr int kMaxHistBins = 64;     // pair-separation histogram

// kSpheropolygon: a polygon species with a sweep radius (its own kernels:
// binary64 tests only); the public API names it a polygon with
// sweep_radius > 0.
enum Kind : int32_t { kDisk = 0, kPolygon = 1, kPolyhedron = 2, kSpheropolygon = 3 };
constexpr int kNumKinds = 4;

// Orientation components per particle: none (disks), a unit complex number
// (2D shapes), a unit quaternion (polyhedra).
constexpr int orient_comps(int kind) { return kind == kDisk ? 0 : (kind == kPolyhedron ? 4 : 2); }

// Bytes per particle of the cell-sorted binary32 coordinate copy.
constexpr int xs_bytes(int dim) { return dim == 3 ? 16 : 8; }

// Counters kept per replica in the workspace (u64 each), same order as
// hpmc_stats minus the host-side sweep count.
enum Stat : int { kAttempted = 0, kAttemptedRot, kCellReject, kOverlapReject, kAccept,
                  kPairTests, kPairFp64, kCellOverflow, kNumStats };

// The counters of a replica are kept in kStatStripes copies, one 64-byte line
// each; a work-group adds into stripe blockIdx % kStatStripes, so that
// thousands of work-groups of one pass do not serialise on one line.  Readers
// sum the stripes.
constexpr int kStatStripes = 64;
constexpr int kStatStride = 8;  // u64 per stripe (kNumStats used)
constexpr int kStatsPerReplica = kStatStripes * kStatStride;

// One particle type, built on the host at init.  Vertex coordinates are
// stored per axis so that a uniform loop over vertices reads scalars.
struct alignas(16) SpeciesDev {
    int32_t kind, dim, nv, pad0;
    double R;        // circumradius, rounded up one ulp
    double circ2;    // circumsphere threshold (R + R)^2
    double tol2;     // squared XenoCollide tolerance
    double d, a, p_rot;
    double sweep;    // sweep radius of a spheropolygon / -polyhedron, 0 otherwise
    double vx[kMaxPolyhedronVerts], vy[kMaxPolyhedronVerts], vz[kMaxPolyhedronVerts];
    double nx[kMaxPolyVerts], ny[kMaxPolyVerts];      // polygon outward edge normals
    double pmin[kMaxPolyVerts], pmax[kMaxPolyVerts];  // own projections onto them
    // binary32 copies for the mixed-precision filters
    float vx32[kMaxPolyhedronVerts], vy32[kMaxPolyhedronVerts], vz32[kMaxPolyhedronVerts];
    float nx32[kMaxPolyVerts], ny32[kMaxPolyVerts];
    float pmin32[kMaxPolyVerts], pmax32[kMaxPolyVerts];
    float sat_margin_scale;  // forward-error bound factor of the polygon filter
    float R32;               // circumradius rounded up to binary32
    float tol32;             // XenoCollide tolerance rounded up to binary32
    int32_t mpr32_ok;        // binary32 XenoCollide allowed (R within its range)
    int32_t regular;         // polygon symmetric under rotation by 2 pi / nv (to the margin)
    float sat_margin_regular;  // margin of the symmetric-polygon filter
    float pad2[2];
};

// Sweep counter, Philox key and the length of a persistent launch, read by
// the kernels from device memory so that one captured sweep (grid path) or
// chunk (persistent path) can be replayed for any call: set once per
// hpmc_sweep call (n changed again before a shorter last chunk), t advanced
// by n by a kernel at the end of every sweep or chunk.
struct alignas(16) Clock {
    uint32_t t, k0, k1;
    uint32_t n;  // sweeps per persistent launch (1 on the grid path)
};

// One replica (independent system) and its grid.
struct alignas(16) SysDev {
    double L, inv_L, w, inv_w;
    int32_t n, dim, N, rounds;
    int32_t ncells, species, replica, path;
    int64_t pos_off, orient_off;  // element offsets into the caller's arrays
    // this replica's slice of the global cell list: count/start entries from
    // cell_off (ncells + 1 of them), per-particle entries (cell_of, slot_of,
    // members, sorted coordinates) from slot_off, scan partials from part_off
    int64_t cell_off, slot_off, part_off;
    // Threshold of the binary32 circumsphere pre-filter on the cell-sorted
    // coordinate copy: every pair whose binary64 |r|^2 is below circ2 has a
    // binary32 |r|^2 below scan_t2 (bound derived on the host).
    float scan_t2;
    // queued full tests at which a wave drains its queue (16, 32 or 64; the
    // autotuner's queue depth)
    uint32_t drain_at;
    // persistent 2D path: LDS slots reserved for the ghost copies of the two
    // edge columns of the cell list (0: no ghost columns)
    int32_t ghost_cap;
};

// Phases of the per-wave clock of a trace build (HPMC_TRACE): cell-list
// build, trial move, pre-filter scan, queued full tests, write-back, waiting
// at the work-group barrier after a pass, everything else (loads, loop
// overhead); then the steps of the persistent kernel's in-LDS build, each up
// to the barrier that ends it: counting per cell, the prefix sum of the
// counts, the scatter, the ascending-tag order within each cell (its kPhBuild
// is then the clearing of the counts alone).  Kernels traced: the persistent
// batch kernel and the grid path's colour pass.
enum Phase : int { kPhBuild = 0, kPhPropose, kPhScan, kPhDrain, kPhWrite, kPhBarrier, kPhOther,
                   kPhCount, kPhPrefix, kPhScatter, kPhSort, kNumPhases };
enum TracedKernel : int { kTraceBatch = 0, kTraceUpdate = 1, kTraceKernels = 2 };
// Per traced kernel: kNumPhases cycle totals, then the number of waves.
constexpr int kTraceWords = kTraceKernels * (kNumPhases + 1);

// Floats per particle reserved for the cell-sorted coordinates of any
// replica in the global cell list (float2 in 2D, float4 in 3D).
constexpr int kXsStride = 4;

}  // namespace hpmc
