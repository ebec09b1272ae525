// Host-side view of the workspace and the kernel launchers.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "types.hpp"

namespace hpmc {

constexpr int kBatchBlock = 1024;  // most lanes of a persistent work-group (16 waves)
constexpr int kBatchOwn = 4;       // particles per lane the persistent build keeps in registers

// Lanes of a persistent work-group for replicas of at most n_max particles
// and n_act_max active cells per colour: one 64-cell tile per wave covers a
// pass, and every particle of the cell-list build stays in registers; a
// multiple of 64 from 64 to kBatchBlock.  Smaller replicas take fewer lanes,
// so more of their work-groups share a compute unit.
inline int persistent_block(int64_t n_act_max, int64_t n_max) {
    int64_t need = n_act_max > (n_max + kBatchOwn - 1) / kBatchOwn ? n_act_max
                                                                   : (n_max + kBatchOwn - 1) / kBatchOwn;
    need = (need + 63) / 64 * 64;
    return need < 64 ? 64 : (need > kBatchBlock ? kBatchBlock : (int)need);
}

constexpr int64_t kGqPerSlot = 8;  // queue entries reserved per particle (2^dim, dim <= 3)

// Global-queue variant of a colour pass: trial state of every active cell and
// the queue of pair tests in global memory (allocated only when selected).
struct GlobalQueue {
    double* trial;      // 7 x cell_total: x, y, z, q0 .. q3 of each active cell
    uint32_t* meta;     // 3 x cell_total: moving tag, its slot, bits (1 live, 2 rotated, 4 translated)
    uint32_t* flag;     // cell_total: an overlap was found
    uint2* entries;     // per replica 2^dim N entries from kGqPerSlot slot_off: (active index, slot)
    uint32_t* count;    // queued entries per replica (zero between passes)
    int64_t cell_total; // sum over replicas of ncells + 1
};

struct Workspace {
    SpeciesDev* species;              // one per replica
    SysDev* sys;                      // one per replica
    unsigned long long* stats;        // n_replicas x kStatStripes x kStatStride
    unsigned long long* overlap_out;  // n_replicas
    // global-memory cell lists, one slice per replica (offsets in SysDev)
    uint32_t* count;    // ncells + 1 per replica
    uint32_t* start;    // ncells + 1 per replica
    uint32_t* cell_of;  // N per replica
    uint32_t* slot_of;  // N per replica
    uint32_t* members;  // N per replica
    float* xs;          // kXsStride floats per particle: cell-sorted binary32 coordinates
    double* hist_edges;             // kMaxHistBins + 1 squared bin edges
    unsigned long long* hist_out;   // kMaxHistBins pair counts
    uint32_t* partial;  // scan tiles, per replica
    int32_t* batch_list;  // replica indices of the launch groups, grouped by kind
    int32_t* ident;       // 0 .. n_replicas - 1 (single-replica launches)
    Clock* clock;         // sweep counter and key read by the kernels
    double* backup_pos;   // autotuning snapshot of the caller's arrays
    double* backup_ori;
    unsigned long long* backup_stats;
    GlobalQueue gq;       // null pointers unless the global queue is selected
};

// How the full overlap tests of a pass are scheduled (grid path).
enum QueueMode : int32_t { kQueueWave = 0, kQueueRegister = 1, kQueueGlobal = 2 };

struct ReplicaHost {
    int32_t kind, dim, N, n, ncells, rounds, path;
    int32_t ncells_cap;      // cells allocated for this replica (grid of its largest box)
    double L, L_max;         // current box side, largest allowed (NPT box moves)
    int32_t lanes_per_cell;  // grid path: lanes per active cell (1, 2, 4, ..., 64)
    int32_t ghost_cap;       // persistent 2D path: ghost-column slots (0: none)
    int32_t n_cap;           // cells per side of the largest box (L_max)
    int32_t nv;              // polygon vertex count (compile-time fast path for 5)
    int64_t pos_off, orient_off;
};

// Replicas of one shape kind launched together: the persistent path (one
// work-group per replica) and the grid path (blockIdx.y selects the replica).
struct BatchGroup {
    int32_t kind, first, count;
    int32_t resident;  // persistent: 0 none, 1 positions, 2 positions + orientations in LDS,
                       // 3 the same without the binary32 cell-sorted copy
    int32_t fits;      // bit lv set when residency level lv fits in LDS
    int32_t ghost;     // bit lv set when level lv keeps ghost edge columns
    int32_t nv;        // common polygon vertex count, 0 when mixed or not a polygon
    size_t lds_bytes;
    size_t need[4];    // dynamic LDS per residency level
    // grid path: largest replica of the group and the lanes per active cell
    int32_t dim, lanes, rounds_max;
    int64_t n_max, nc_max, n_act_max;
    int32_t block = kBatchBlock;       // persistent: lanes per work-group
    int32_t block_base = kBatchBlock;  // the size persistent_block chose
};

constexpr int kScanTile = 2048;  // cells per scan work-group (256 lanes x 8)
// Replicas up to this size build their cell list in one work-group (LDS
// histogram of at most kSmallBuildCells cells).
constexpr int64_t kSmallBuildN = 8192;
constexpr int kSmallBuildCells = 16000;  // 64 KB of LDS with the scan scratch

// Cell lists of the replicas list[0 .. count) in global memory (one launch
// per step, blockIdx.y picks the replica; all of dimension dim, at most
// n_max particles and nc_max cells): shifted grid of sweep t when shifted !=
// 0, the unshifted grid otherwise.
hipError_t build_cells(const Workspace& ws, const int32_t* list, int count, int dim, int64_t n_max,
                       int64_t nc_max, const double* pos, int shifted, hipStream_t stream);
// The same for replica r alone.
hipError_t build_cells_one(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                           int shifted, hipStream_t stream);

// Device clock: set {t, key, sweeps per persistent launch n}; set n alone;
// advance t by n.
hipError_t set_clock(const Workspace& ws, uint32_t t, uint32_t k0, uint32_t k1, uint32_t n,
                     hipStream_t stream);
hipError_t set_chunk(const Workspace& ws, uint32_t n, hipStream_t stream);
hipError_t advance_clock(const Workspace& ws, hipStream_t stream);

// All colour passes of sweep t for the replicas of a grid-path group on
// their global cell lists.
hipError_t grid_passes(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                       int precision, int queue, hipStream_t stream);

// Whole sweeps of the replicas of one batch group, one work-group each; the
// number of sweeps is the device clock's n.
// prepare = true only raises the kernel's dynamic-LDS limit (call before
// launching or capturing).
hipError_t persistent_sweeps(const Workspace& ws, const BatchGroup& g, double* pos,
                             double* orient, int precision, bool prepare, hipStream_t stream);

// Overlapping pairs of replica r (after build_cells with shifted = 0), added
// to ws.overlap_out[r].
hipError_t count_pairs(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                       const double* orient, hipStream_t stream);

// Invalid particles of replica r (coordinate outside [0, L), non-finite
// orientation) added to ws.overlap_out[r].
// Pair-separation histogram of replica r (edges already in ws.hist_edges).
hipError_t pair_histogram(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                          int n_bins, int reach, hipStream_t stream);
hipError_t validate_state(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                          const double* orient, hipStream_t stream);
// Volume-perturbation counts of replica r (scale factors already in
// ws.hist_edges, cell list unshifted), written to ws.hist_out[0 .. n_s).
hipError_t scale_counts(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                        const double* orient, int n_s, int reach, hipStream_t stream);

hipError_t fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t stream);
// n coordinates x -> x k wrapped into [0, L_new) (NPT box change).
hipError_t scale_box(double* pos, int64_t n, double k, double L_new, hipStream_t stream);

// Trace build (HPMC_TRACE): copy the kTraceWords phase totals to out (host)
// after synchronising the device, and clear them when reset; otherwise
// hipErrorNotSupported.
hipError_t read_phase_trace(unsigned long long* out, bool reset);

constexpr int kResidencyLevels = 4;

// Dynamic LDS of a persistent work-group of `block` lanes for a replica of
// this kind, precision, cell count (n per side) and N at residency level
// res; ghost_cap > 0: with that many ghost-column slots (2D, res <= 2).
size_t persistent_lds_bytes(int kind, int precision, int ncells, int n, int N, int res, int block,
                            int ghost_cap);

}  // namespace hpmc
