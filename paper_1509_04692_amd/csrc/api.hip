// C ABI of libhpmc: argument validation, shape tables, grids, workspace
// layout and the sweep / count schedules.  No device allocation happens
// here: every device buffer belongs to the caller.
#include "../../include/hpmc.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <atomic>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "launch.hpp"
#include "mpr32.hpp"
#include "overlap32.hpp"
#include "types.hpp"

using namespace hpmc;

// Device memory of hpmc_sweep_static, the entry point that allocates
// nothing: every workspace region of its call lives here.  Each GPU the
// library runs on holds its own copy until the process ends.  Host code never
// passes this name to a kernel or a copy (on the host it is a stand-in, not a
// device address): it uses the per-device address from hipGetSymbolAddress.
__device__ __align__(256) unsigned char scratch[HPMC_STATIC_SCRATCH_BYTES];

struct hpmc_state {
    int n_replicas = 0;
    int precision = HPMC_FP64;
    int walk64 = 0;  // MIXED: polyhedra walk in binary64 (autotuned; same results)
    int path = HPMC_PATH_GRID;
    int queue = kQueueWave;  // grid path: how full tests are scheduled
    hipStream_t stream = nullptr;
    double* pos = nullptr;
    double* orient = nullptr;
    Workspace ws{};
    std::vector<ReplicaHost> rep;
    std::vector<SysDev> sys;
    std::vector<SpeciesDev> spc;
    std::vector<BatchGroup> groups;
    uint64_t t = 0;
    uint64_t sweeps_done = 0;
    int last_hip = 0;
    int flags = 0;
    size_t pos_total = 0, ori_total = 0;  // doubles in the caller's arrays
    hipStream_t cap_stream = nullptr;     // private stream used only for capture
    // persistent path with several launch groups: private streams that run
    // the groups after the first beside it, forked from and joined back to
    // the stream a sweep is enqueued on
    std::vector<hipStream_t> side;
    std::vector<hipEvent_t> side_done;
    hipEvent_t fork = nullptr;
    std::vector<hpmc_species> spec_host;  // species as given (vertex pointer cleared)
    std::vector<int32_t> list;            // host copy of the launch groups' replica list
    std::vector<SysDev> sys_saved;        // box before the last hpmc_scale_box, per replica
    std::vector<ReplicaHost> rep_saved;
    std::vector<uint8_t> box_saved;
    hipGraphExec_t graph = nullptr;       // one sweep (grid) / one chunk (persistent)
    uint64_t graph_sweeps = 0;            // sweeps run by replaying `graph` since init
};

namespace {

constexpr uint64_t kSweepLimit = 1ull << 32;
constexpr size_t kAlign = 256;
// LDS per work-group available to the persistent path (gfx950: 160 KiB;
// the device attribute is queried at init).
// LDS per work-group of the current device; gfx950's 160 KiB when no device
// can be queried (workspace sizing on a host without a GPU).
size_t device_lds_limit() {
    constexpr size_t kGfx950Lds = 160 * 1024;
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess) return kGfx950Lds;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
        return kGfx950Lds;
    return (size_t)v;
}
constexpr uint32_t kPersistentChunk = HPMC_PERSISTENT_SWEEPS_PER_LAUNCH;

size_t align_up(size_t x) { return (x + kAlign - 1) & ~(kAlign - 1); }

int check_hip(hpmc_state* st, hipError_t e) {
    if (e == hipSuccess) return HPMC_OK;
    if (st) st->last_hip = (int)e;
    return HPMC_ERR_HIP;
}

// Per-type tables (Sec. 2.3: geometry given once per type, particle frame).
int build_species(const hpmc_species& s, SpeciesDev& P) {
    std::memset(&P, 0, sizeof(P));
    P.kind = s.shape;
    P.dim = s.dim;
    if (!(s.d >= 0.0) || !(s.a >= 0.0) || !(s.p_rot >= 0.0) || !(s.p_rot <= 1.0))
        return HPMC_ERR_INVALID_ARG;
    // the 2D rotation's sine and cosine are truncated series, and the unit
    // complex orientation is never renormalised: angles are bounded so that
    // the first dropped term stays below binary64 rounding (Sec. 2.1 move)
    if (s.shape == HPMC_POLYGON && !(s.a <= HPMC_MAX_POLYGON_ROTATION)) return HPMC_ERR_INVALID_ARG;
    if (s.rounds < 0) return HPMC_ERR_INVALID_ARG;
    if (!(s.sweep_radius >= 0.0) || !std::isfinite(s.sweep_radius)) return HPMC_ERR_INVALID_ARG;
    if (s.sweep_radius > 0.0 && s.shape == HPMC_DISK) return HPMC_ERR_INVALID_ARG;
    P.sweep = s.sweep_radius;
    if (s.shape == HPMC_POLYGON && P.sweep > 0.0) P.kind = kSpheropolygon;
    if (s.shape == HPMC_DISK) {
        if (s.dim != 2 || !(s.diameter > 0.0) || s.p_rot != 0.0) return HPMC_ERR_INVALID_ARG;
        P.R = s.diameter * 0.5;
    } else if (s.shape == HPMC_POLYGON || s.shape == HPMC_POLYHEDRON) {
        const int want_dim = s.shape == HPMC_POLYGON ? 2 : 3;
        const int maxv = s.shape == HPMC_POLYGON ? kMaxPolyVerts : kMaxPolyhedronVerts;
        if (s.dim != want_dim || s.verts == nullptr) return HPMC_ERR_INVALID_ARG;
        const int minv = P.sweep > 0.0 ? 1 : want_dim + 1;
        if (s.n_verts < minv || s.n_verts > maxv) return HPMC_ERR_INVALID_ARG;
        P.nv = s.n_verts;
        double rmax = 0.0;
        for (int k = 0; k < P.nv; ++k) {
            const double x = s.verts[k * s.dim], y = s.verts[k * s.dim + 1];
            const double z = s.dim == 3 ? s.verts[k * s.dim + 2] : 0.0;
            if (!std::isfinite(x) || !std::isfinite(y) || !std::isfinite(z)) return HPMC_ERR_INVALID_ARG;
            P.vx[k] = x;
            P.vy[k] = y;
            P.vz[k] = z;
            double r2 = x * x + y * y;
            if (s.dim == 3) r2 = r2 + z * z;
            const double r = std::sqrt(r2);
            if (r > rmax) rmax = r;
        }
        // every vertex, and every point within the sweep radius of one, inside
        P.R = std::nextafter(rmax + P.sweep, INFINITY);
        if (s.shape == HPMC_POLYGON && !fill_polygon_tables(P)) return HPMC_ERR_INVALID_ARG;
    } else {
        return HPMC_ERR_INVALID_ARG;
    }
    const double dmax = P.R + P.R;
    P.circ2 = dmax * dmax;
    const double tol = 1e-12 * dmax;
    P.tol2 = tol * tol;
    if (s.shape == HPMC_POLYHEDRON) fill_mpr32_tables(P, tol);
    if (P.sweep > 0.0) P.mpr32_ok = 0;  // the binary32 walk has no bound for the swept term
    P.d = s.d;
    P.a = s.a;
    P.p_rot = s.p_rot;
    return HPMC_OK;
}

// Threshold of the binary32 circumsphere pre-filter.  The scan compares
// |r32|^2 with it, where each component of r32 is a binary32 grid coordinate
// (|y| <= L, cast from binary64) minus a binary32 reference point
// (|ref| <= L + w).  Per axis r32 is within
//   e = u32 (2L + 3w) + u64 (2L + 3w)
// of the exact separation (two casts, one subtraction of a result below 2w +
// 2R, and the binary64 roundings of the grid coordinates and of the min-image
// separation), so a pair with binary64 |r|^2 < circ2 has |r| < sqrt(circ2)
// (1 + 2 u64) and |r32| < that + sqrt(dim) e; three binary32 roundings of the
// square sum add a factor (1 + u32)^3.  The bound is doubled and rounded up.
float scan_threshold(double circ2, double L, double w, int dim) {
    const double u32 = 0x1p-24, u64 = 0x1p-53;
    const double e = 2.0 * (u32 + u64) * (2.0 * L + 3.0 * w);
    const double rho = std::sqrt(circ2) * (1.0 + 4.0 * u64) + std::sqrt((double)dim) * e;
    const double t = rho * rho * (1.0 + 8.0 * u32);
    float f = (float)t;
    if ((double)f < t) f = std::nextafter(f, INFINITY);
    return f;
}

// Grid of Sec. 2.2.1 with the checkerboard constraint: the largest even n
// with cells at least d_max (times 1 + 2^-30) wide, n >= 4.
int build_grid(const hpmc_species& s, const SpeciesDev& P, int32_t N, double L, SysDev& S,
               ReplicaHost& rh) {
    if (!(L > 0.0) || !std::isfinite(L) || N < 1) return HPMC_ERR_INVALID_ARG;
    if (N >= (1 << 26)) return HPMC_ERR_UNSUPPORTED;  // queue entries hold 26-bit slots
    const double dmax = P.R + P.R;
    const double nf = L / (dmax * (1.0 + 0x1p-30));
    if (nf > 65536.0) return HPMC_ERR_UNSUPPORTED;
    int n = (int)nf;
    n -= n & 1;
    if (n < 4) return HPMC_ERR_BOX_TOO_SMALL;
    if (s.dim == 3 && n > 1024) return HPMC_ERR_UNSUPPORTED;
    if (!(s.d < L)) return HPMC_ERR_INVALID_ARG;
    std::memset(&S, 0, sizeof(S));
    S.L = L;
    S.inv_L = 1.0 / L;
    S.w = L / (double)n;
    S.inv_w = (double)n / L;
    S.n = n;
    S.dim = s.dim;
    S.N = N;
    const int64_t ncells = s.dim == 2 ? (int64_t)n * n : (int64_t)n * n * n;
    if (ncells > (int64_t)1 << 30) return HPMC_ERR_UNSUPPORTED;
    S.ncells = (int32_t)ncells;
    if (s.rounds > 0) {
        S.rounds = s.rounds;
    } else {
        const int64_t r = ((int64_t)N + ncells / 2) / ncells;
        S.rounds = r < 1 ? 1 : (int32_t)r;
    }
    if ((int64_t)S.rounds * (1 << s.dim) >= ((int64_t)1 << 28)) return HPMC_ERR_INVALID_ARG;
    S.scan_t2 = scan_threshold(P.circ2, L, S.w, s.dim);
    S.drain_at = 64;
    rh.kind = P.kind;
    rh.dim = s.dim;
    rh.N = N;
    rh.n = n;
    rh.ncells = S.ncells;
    rh.rounds = S.rounds;
    rh.L = L;
    return HPMC_OK;
}

struct Layout {
    size_t species, sys, stats, overlap, count, start, cell_of, slot_of, members, xs, hist_edges,
        hist_out, partial, list, ident,
        clock, backup_pos, backup_ori, backup_stats, gq_trial, gq_meta, gq_flag, gq_entries,
        gq_count, total;
    int64_t cell_total;
    size_t pos_total, ori_total;
};

// hipError_t of the last hpmc_init that failed in a HIP call (the state it
// was building is gone by then).
std::atomic<int> g_last_init_hip{0};

// Highest residency level at most lv whose LDS fits the group.
int highest_fit(const BatchGroup& g, int lv) {
    for (; lv > 0; --lv)
        if (g.fits & (1 << lv)) return lv;
    return 0;
}

// Ghost-column slots a persistent 2D replica needs at most: the particles of
// two columns of cells.  Particles that do not overlap have disjoint
// inscribed disks of radius r_in, and the disks of the particles centred in
// one cell (width w < 1.5 d_max, as n >= 4 is the largest even count with
// w >= d_max) lie in a square of side w + 2 r_in, so a cell holds at most
// (w + 2 r_in)^2 / (pi r_in^2) of them.  0 (no ghost columns) for 3D kinds,
// for shapes whose centre is not inside them, and where the slots would
// exceed the 16-bit cell list.
int ghost_capacity(const SpeciesDev& P, int N, int n_cap) {
    if (P.kind == kPolyhedron) return 0;
    double r_in = 0.0;
    if (P.kind == kDisk) {
        r_in = P.R;
    } else {
        if (P.nv >= 3) {
            r_in = INFINITY;
            for (int k = 0; k < P.nv; ++k)
                r_in = std::fmin(r_in, P.pmax[k] / std::sqrt(P.nx[k] * P.nx[k] + P.ny[k] * P.ny[k]));
            if (!(r_in > 0.0)) r_in = 0.0;
        }
        r_in += P.sweep;
    }
    if (!(r_in > 0.0)) return 0;
    const double w = 1.5 * (P.R + P.R) * (1.0 + 1e-9);
    const double per_cell = std::floor((w + 2.0 * r_in) * (w + 2.0 * r_in) / (3.141592653589793 * r_in * r_in)) + 1.0;
    const double cap = std::fmin((double)N, 2.0 * (double)n_cap * per_cell);
    if ((double)N + cap > 65535.0) return 0;
    return (int)cap;
}

// Dynamic LDS per residency level for the replicas of group g at `block`
// lanes, the levels that fit, and those that keep ghost edge columns (2D
// kinds at levels 0-2, wherever every replica has a ghost capacity and the
// larger layout fits).
void group_lds_levels(BatchGroup& g, const std::vector<int32_t>& list, const std::vector<ReplicaHost>& rep,
                      int precision, int block, size_t limit) {
    size_t plain[kResidencyLevels] = {}, ghost[kResidencyLevels] = {};
    bool all_ghost = true;
    for (int j = g.first; j < g.first + g.count; ++j) {
        const ReplicaHost& h = rep[list[j]];
        all_ghost &= h.ghost_cap > 0;
        for (int lv = 0; lv < kResidencyLevels; ++lv) {
            plain[lv] = std::max(plain[lv], persistent_lds_bytes(g.kind, precision, h.ncells_cap, h.n_cap, h.N,
                                                                 lv, block, 0));
            if (lv <= 2 && h.ghost_cap > 0)
                ghost[lv] = std::max(ghost[lv], persistent_lds_bytes(g.kind, precision, h.ncells_cap, h.n_cap,
                                                                     h.N, lv, block, h.ghost_cap));
        }
    }
    g.fits = 1;
    g.ghost = 0;
    for (int lv = 0; lv < kResidencyLevels; ++lv) {
        g.need[lv] = plain[lv];
        if (lv <= 2 && all_ghost && g.kind != kPolyhedron && ghost[lv] <= limit) {
            g.need[lv] = ghost[lv];
            g.ghost |= 1 << lv;
        }
        // disks have no orientations, so their level 2 is level 1
        if (lv >= 1 && g.need[lv] <= limit && !(g.kind == kDisk && lv == 2)) g.fits |= 1 << lv;
    }
}

// Queue mode from hpmc_init_args.flags; -1 when both variants are asked for.
int queue_mode(int32_t flags) {
    const bool reg = (flags & HPMC_FLAG_REGISTER_QUEUE) != 0, glob = (flags & HPMC_FLAG_GLOBAL_QUEUE) != 0;
    if (reg && glob) return -1;
    return glob ? kQueueGlobal : (reg ? kQueueRegister : kQueueWave);
}

// Lanes per active cell on the grid path: enough waves to cover the chip
// (256 CUs x 8 waves) when a pass has few active cells.
int choose_lanes_per_cell(int64_t n_act) {
    const int64_t target_waves = 256 * 8;
    int g = 1;
    while (g < 8 && n_act * g / 64 < target_waves) g *= 2;
    return g;
}

// backups = false leaves out the snapshot buffers of autotuning and box moves.
int plan(const hpmc_init_args* a, std::vector<ReplicaHost>& rep, std::vector<SysDev>& sys,
         std::vector<SpeciesDev>& spc, Layout& lay, int& path, std::vector<BatchGroup>& groups,
         std::vector<int32_t>& list, size_t lds_limit, bool backups = true) {
    if (a == nullptr || a->n_replicas < 1 || a->species == nullptr || a->N == nullptr ||
        a->L == nullptr)
        return HPMC_ERR_INVALID_ARG;
    if (a->precision != HPMC_FP64 && a->precision != HPMC_MIXED) return HPMC_ERR_INVALID_ARG;
    if (a->path < HPMC_PATH_AUTO || a->path > HPMC_PATH_PERSISTENT) return HPMC_ERR_INVALID_ARG;
    const int queue = queue_mode(a->flags);
    if (queue < 0) return HPMC_ERR_INVALID_ARG;
    if (queue != kQueueWave && a->path == HPMC_PATH_PERSISTENT) return HPMC_ERR_UNSUPPORTED;
    const int R = a->n_replicas;
    rep.assign(R, ReplicaHost{});
    sys.assign(R, SysDev{});
    spc.assign(R, SpeciesDev{});
    int64_t pos_off = 0, ori_off = 0;
    int64_t cell_total = 0, slot_total = 0, part_total = 0;
    bool fits_lds = true;
    for (int r = 0; r < R; ++r) {
        int rc = build_species(a->species[r], spc[r]);
        if (rc) return rc;
        // swept polygons run the wave queue only
        if (spc[r].kind == kSpheropolygon && queue != kQueueWave) return HPMC_ERR_UNSUPPORTED;
        rc = build_grid(a->species[r], spc[r], a->N[r], a->L[r], sys[r], rep[r]);
        if (rc) return rc;
        // cell lists are sized for the largest box a volume move may reach
        const double L_max = a->L_max ? a->L_max[r] : a->L[r];
        if (!(L_max >= a->L[r]) || !std::isfinite(L_max)) return HPMC_ERR_INVALID_ARG;
        SysDev smax;
        ReplicaHost hmax;
        rc = build_grid(a->species[r], spc[r], a->N[r], L_max, smax, hmax);
        if (rc) return rc;
        rep[r].ncells_cap = std::max(smax.ncells, sys[r].ncells);
        rep[r].n_cap = std::max(hmax.n, rep[r].n);
        rep[r].L_max = L_max;
        sys[r].species = r;
        sys[r].replica = r;
        sys[r].pos_off = pos_off;
        sys[r].orient_off = ori_off;
        rep[r].pos_off = pos_off;
        rep[r].orient_off = ori_off;
        const int ncomp = orient_comps(spc[r].kind);
        pos_off += (int64_t)sys[r].dim * sys[r].N;
        ori_off += (int64_t)ncomp * sys[r].N;
        // this replica's slice of the global cell lists
        sys[r].cell_off = cell_total;
        sys[r].slot_off = slot_total;
        sys[r].part_off = part_total;
        cell_total += (int64_t)rep[r].ncells_cap + 1;
        slot_total += sys[r].N;
        part_total += ((int64_t)rep[r].ncells_cap + kScanTile - 1) / kScanTile;
        const size_t lb = persistent_lds_bytes(spc[r].kind, a->precision, rep[r].ncells_cap, rep[r].n_cap,
                                               sys[r].N, 0, kBatchBlock, 0);
        if (sys[r].N > 65535 || lb > lds_limit) fits_lds = false;
        const int half = sys[r].n / 2;
        const int64_t n_act = sys[r].dim == 3 ? (int64_t)half * half * half : (int64_t)half * half;
        rep[r].lanes_per_cell = choose_lanes_per_cell(n_act);
        rep[r].nv = spc[r].nv;
    }
    if (a->path == HPMC_PATH_PERSISTENT && !fits_lds) return HPMC_ERR_UNSUPPORTED;
    if (a->path == HPMC_PATH_AUTO)
        path = (fits_lds && R > 1 && queue == kQueueWave) ? HPMC_PATH_PERSISTENT : HPMC_PATH_GRID;
    else
        path = a->path;
    for (int r = 0; r < R; ++r) {
        sys[r].path = path;
        rep[r].path = path;
        const int cap = path == HPMC_PATH_PERSISTENT ? ghost_capacity(spc[r], sys[r].N, rep[r].n_cap) : 0;
        sys[r].ghost_cap = cap;
        rep[r].ghost_cap = cap;
    }
    // persistent path: one launch per shape kind; positions held in LDS when
    // every replica of the kind fits
    groups.clear();
    list.clear();
    if (path == HPMC_PATH_PERSISTENT) {
        // kinds with the costlier overlap test first: their launch is captured
        // first and takes the compute units first, and the cheaper kinds'
        // work-groups fill in as they free up
        constexpr int kCostOrder[kNumKinds] = {kPolyhedron, kSpheropolygon, kPolygon, kDisk};
        for (const int kind : kCostOrder) {
            BatchGroup g{};
            g.kind = kind;
            g.first = (int32_t)list.size();
            g.nv = -1;
            int64_t n_max = 0, n_act_max = 0;
            for (int r = 0; r < R; ++r) {
                if (spc[r].kind != kind) continue;
                const int64_t half = sys[r].n / 2;
                n_max = std::max<int64_t>(n_max, sys[r].N);
                n_act_max = std::max<int64_t>(n_act_max, sys[r].dim == 3 ? half * half * half : half * half);
            }
            g.block = persistent_block(n_act_max, n_max);
            g.block_base = g.block;
            for (int r = 0; r < R; ++r) {
                if (spc[r].kind != kind) continue;
                list.push_back(r);
                g.count++;
                g.nv = (g.nv == -1 || g.nv == spc[r].nv) ? spc[r].nv : 0;
            }
            if (g.count == 0) continue;
            // largest replicas first: work-groups start in list order, so the
            // longest ones do not wait behind short ones for a compute unit
            std::stable_sort(list.begin() + g.first, list.end(),
                             [&](int32_t x, int32_t y) { return sys[x].N > sys[y].N; });
            // levels whose LDS fits (level 0 always)
            group_lds_levels(g, list, rep, a->precision, g.block, lds_limit);
            // before autotuning: the binary32 copy kept when it fits (level
            // 2, else 1), level 3 only when neither fits
            g.resident = highest_fit(g, 2);
            if (g.resident == 0 && (g.fits & 8)) g.resident = 3;
            g.lds_bytes = g.need[g.resident];
            if (g.nv < 0) g.nv = 0;
            groups.push_back(g);
        }
    } else {
        // grid path: one launch per step for all replicas of a kind
        for (int kind = 0; kind < kNumKinds; ++kind) {
            BatchGroup g{};
            g.kind = kind;
            g.first = (int32_t)list.size();
            g.nv = -1;
            g.lanes = 1;
            int64_t n_act_total = 0;
            for (int r = 0; r < R; ++r) {
                if (spc[r].kind != kind) continue;
                list.push_back(r);
                g.count++;
                g.nv = (g.nv == -1 || g.nv == spc[r].nv) ? spc[r].nv : 0;
                g.dim = sys[r].dim;
                const int half = sys[r].n / 2;
                const int64_t n_act = sys[r].dim == 3 ? (int64_t)half * half * half : (int64_t)half * half;
                g.rounds_max = std::max<int32_t>(g.rounds_max, sys[r].rounds);
                g.n_max = std::max<int64_t>(g.n_max, sys[r].N);
                g.nc_max = std::max<int64_t>(g.nc_max, sys[r].ncells);
                g.n_act_max = std::max<int64_t>(g.n_act_max, n_act);
                n_act_total += n_act;
            }
            if (g.count == 0) continue;
            if (g.nv < 0) g.nv = 0;
            g.lanes = choose_lanes_per_cell(n_act_total);
            for (int r : list)
                if (spc[r].kind == kind) rep[r].lanes_per_cell = g.lanes;
            groups.push_back(g);
        }
    }
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off = align_up(off + bytes);
        return o;
    };
    lay.species = take(sizeof(SpeciesDev) * R);
    lay.sys = take(sizeof(SysDev) * R);
    lay.stats = take(sizeof(unsigned long long) * kStatsPerReplica * R);
    lay.overlap = take(sizeof(unsigned long long) * R);
    lay.count = take(4 * (size_t)cell_total);
    lay.start = take(4 * (size_t)cell_total);
    lay.cell_of = take(4 * (size_t)slot_total);
    lay.slot_of = take(4 * (size_t)slot_total);
    lay.members = take(4 * (size_t)slot_total);
    lay.xs = take(sizeof(float) * kXsStride * (size_t)slot_total);
    lay.hist_edges = take(sizeof(double) * (kMaxHistBins + 1));
    lay.hist_out = take(sizeof(unsigned long long) * kMaxHistBins);
    lay.partial = take(4 * (size_t)(part_total > 0 ? part_total : 1));
    lay.list = take(4 * (size_t)R);
    lay.ident = take(4 * (size_t)R);
    lay.clock = take(sizeof(Clock));
    lay.pos_total = (size_t)pos_off;
    lay.ori_total = (size_t)ori_off;
    lay.backup_pos = take(backups ? 8 * (size_t)pos_off : 0);
    lay.backup_ori = take(backups ? 8 * (size_t)(ori_off > 0 ? ori_off : 1) : 0);
    lay.backup_stats = take(backups ? sizeof(unsigned long long) * kStatsPerReplica * R : 0);
    const bool gq = queue == kQueueGlobal;
    lay.cell_total = cell_total;
    lay.gq_trial = take(gq ? 8 * 7 * (size_t)cell_total : 0);
    lay.gq_meta = take(gq ? 4 * 3 * (size_t)cell_total : 0);
    lay.gq_flag = take(gq ? 4 * (size_t)cell_total : 0);
    lay.gq_entries = take(gq ? 8 * (size_t)kGqPerSlot * (size_t)slot_total : 0);
    lay.gq_count = take(gq ? 8 * (size_t)R : 0);
    lay.total = off;
    return HPMC_OK;
}

int count_all(hpmc_state* st, uint64_t* out) {
    int rc = check_hip(st, fill_u64(st->ws.overlap_out, 0ull, st->n_replicas, st->stream));
    if (rc) return rc;
    for (int r = 0; r < st->n_replicas; ++r) {
        rc = check_hip(st, build_cells_one(st->ws, st->rep[r], r, st->pos, 0, st->stream));
        if (rc) return rc;
        rc = check_hip(st, count_pairs(st->ws, st->rep[r], r, st->pos, st->orient, st->stream));
        if (rc) return rc;
    }
    rc = check_hip(st, hipMemcpyAsync(out, st->ws.overlap_out, sizeof(uint64_t) * st->n_replicas,
                                      hipMemcpyDeviceToHost, st->stream));
    if (rc) return rc;
    return check_hip(st, hipStreamSynchronize(st->stream));
}

// Precision of a group's kernels: MIXED polyhedra may take the binary64
// walk when the autotuner found it faster (the decisions are the same);
// swept polygons have binary64 tests only.
int group_precision(const hpmc_state* st, const BatchGroup& g) {
    if (g.kind == kSpheropolygon) return HPMC_FP64;
    return (g.kind == kPolyhedron && st->walk64) ? HPMC_FP64 : st->precision;
}

// One sweep (grid path) or the device clock's n sweeps (persistent path) of
// every replica on stream s, ending with the device clock advanced by n.
int enqueue_sweeps(hpmc_state* st, hipStream_t s) {
    int rc = HPMC_OK;
    if (st->path == HPMC_PATH_PERSISTENT) {
        // the groups (one per shape kind) share no replica, so with side
        // streams they run concurrently: the compute units that the small
        // replicas of one kind leave idle take work of another kind
        const size_t ng = st->groups.size();
        const bool fork = ng > 1 && st->side.size() + 1 == ng;
        // the groups are captured in their order (costliest kind first)
        size_t forked = 0;  // side streams that wait on the fork event
        if (fork) rc = check_hip(st, hipEventRecord(st->fork, s));
        for (size_t k = 0; !rc && k < (fork ? 1 : ng); ++k) {
            const BatchGroup& g = st->groups[k];
            rc = check_hip(st, persistent_sweeps(st->ws, g, st->pos, st->orient, group_precision(st, g),
                                                 false, s));
        }
        for (size_t k = 1; fork && !rc && k < ng; ++k) {
            rc = check_hip(st, hipStreamWaitEvent(st->side[k - 1], st->fork, 0));
            if (rc) break;
            forked = k;
            const BatchGroup& g = st->groups[k];
            rc = check_hip(st, persistent_sweeps(st->ws, g, st->pos, st->orient, group_precision(st, g),
                                                 false, st->side[k - 1]));
        }
        // every forked stream joins back, also after a failed launch
        for (size_t k = 1; k <= forked; ++k) {
            int rj = check_hip(st, hipEventRecord(st->side_done[k - 1], st->side[k - 1]));
            if (!rj) rj = check_hip(st, hipStreamWaitEvent(s, st->side_done[k - 1], 0));
            if (!rc) rc = rj;
        }
        if (rc) return rc;
        return check_hip(st, advance_clock(st->ws, s));
    }
    for (const BatchGroup& g : st->groups) {
        if (rc) break;
        rc = check_hip(st, build_cells(st->ws, st->ws.batch_list + g.first, g.count, g.dim, g.n_max,
                                       g.nc_max, st->pos, 1, s));
        if (!rc)
            rc = check_hip(st, grid_passes(st->ws, g, st->pos, st->orient, group_precision(st, g),
                                           st->queue, s));
    }
    if (!rc) rc = check_hip(st, advance_clock(st->ws, s));
    return rc;
}

uint32_t sweep_unit(const hpmc_state* st) {
    return st->path == HPMC_PATH_PERSISTENT ? kPersistentChunk : 1u;
}

void drop_graph(hpmc_state* st) {
    if (st->graph) (void)hipGraphExecDestroy(st->graph);
    st->graph = nullptr;
}

void drop_side_streams(hpmc_state* st) {
    for (hipStream_t q : st->side) (void)hipStreamDestroy(q);
    for (hipEvent_t e : st->side_done) (void)hipEventDestroy(e);
    if (st->fork) (void)hipEventDestroy(st->fork);
    st->side.clear();
    st->side_done.clear();
    st->fork = nullptr;
}

// Side streams (default priority) and events of a persistent state with
// more than one launch group.  Failure leaves the groups on one stream, one
// after another (not an error).
void make_side_streams(hpmc_state* st) {
    drop_side_streams(st);
    if (st->path != HPMC_PATH_PERSISTENT || st->groups.size() < 2) return;
    bool ok = hipEventCreateWithFlags(&st->fork, hipEventDisableTiming) == hipSuccess;
    if (!ok) st->fork = nullptr;
    for (size_t k = 1; ok && k < st->groups.size(); ++k) {
        hipStream_t q = nullptr;
        hipEvent_t e = nullptr;
        ok = hipStreamCreateWithFlags(&q, hipStreamNonBlocking) == hipSuccess;
        if (ok) st->side.push_back(q);
        ok = ok && hipEventCreateWithFlags(&e, hipEventDisableTiming) == hipSuccess;
        if (ok) st->side_done.push_back(e);
    }
    if (!ok) {
        drop_side_streams(st);
        (void)hipGetLastError();
    }
}

// Capture one sweep unit into a hipGraph on the private stream.  Failure
// leaves the state in direct-launch mode (not an error).
void capture_graph(hpmc_state* st) {
    drop_graph(st);
    if (st->flags & HPMC_FLAG_NO_GRAPH) return;
    if (st->cap_stream == nullptr &&
        hipStreamCreateWithFlags(&st->cap_stream, hipStreamNonBlocking) != hipSuccess) {
        st->cap_stream = nullptr;
        (void)hipGetLastError();
        return;
    }
    hipGraph_t g = nullptr;
    if (hipStreamBeginCapture(st->cap_stream, hipStreamCaptureModeThreadLocal) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    const int last = st->last_hip;
    const int rc = enqueue_sweeps(st, st->cap_stream);
    const hipError_t ec = hipStreamEndCapture(st->cap_stream, &g);
    st->last_hip = last;
    if (rc == HPMC_OK && ec == hipSuccess && g != nullptr) {
        hipGraphExec_t ex = nullptr;
        if (hipGraphInstantiate(&ex, g, nullptr, nullptr, 0) == hipSuccess) st->graph = ex;
    }
    if (g) (void)hipGraphDestroy(g);
    (void)hipGetLastError();
}

// Launch configurations of a state, one int:
//   bits 0-7   lanes per active cell (grid) or LDS residency level (persistent)
//   bit  8     MIXED polyhedra take the binary64 walk
//   bits 9-10  queue depth: drain at 64 (0), 32 (1) or 16 (2) queued tests
//   bits 11-12 persistent work-group size: the default (0), half (1) or a
//              quarter (2) of it, at least 64 lanes
constexpr int kWalk64 = 0x100;
constexpr int kDrainShift = 9, kBlockShift = 11;
constexpr uint32_t kDrainAt[3] = {64u, 32u, 16u};

int drain_code(int cfg) { return (cfg >> kDrainShift) & 3; }
int block_code(int cfg) { return (cfg >> kBlockShift) & 3; }

// Lanes of a persistent group under a block code: the default size halved
// `code` times, rounded down to whole waves (0 below one wave).
int group_block(const BatchGroup& g, int code) {
    const int b = (g.block_base >> code) / 64 * 64;
    return b >= 64 ? b : 0;
}

// LDS per residency level and the levels that fit, for the group's replicas
// at `block` lanes.
void group_lds(const hpmc_state* st, BatchGroup& g, int block) {
    group_lds_levels(g, st->list, st->rep, st->precision, block, device_lds_limit());
}

// Lanes-per-cell or residency choices (with the walk bit) of the first
// tuning stage.
std::vector<int> base_candidates(const hpmc_state* st) {
    std::vector<int> cands;
    if (st->path == HPMC_PATH_PERSISTENT) {
        int any = 0;
        for (const BatchGroup& g : st->groups) any |= g.fits;
        for (int lv = kResidencyLevels - 1; lv >= 0; --lv)
            if (any & (1 << lv)) cands.push_back(lv);
    } else if (st->queue == kQueueGlobal) {
        cands = {1};  // one lane per cell or queued pair: nothing to choose but the walk
    } else if (st->queue == kQueueWave) {
        cands = {1, 2, 4, 8, 16, 32, 64};
    } else {
        cands = {1, 2, 4, 8};
    }
    bool poly_mixed = false;
    for (const BatchGroup& g : st->groups) poly_mixed |= g.kind == kPolyhedron && st->precision == HPMC_MIXED;
    if (poly_mixed) {
        const size_t n0 = cands.size();
        for (size_t i = 0; i < n0; ++i) cands.push_back(cands[i] | kWalk64);
    }
    return cands;
}

// A configuration this state can use: a base candidate, a queue depth the
// wave queue has (the register and global queues have none), and a
// work-group size every persistent group can take.
bool config_valid(const hpmc_state* st, int cfg) {
    if (cfg < 0 || (cfg >> 13) != 0) return false;
    const std::vector<int> base = base_candidates(st);
    if (std::find(base.begin(), base.end(), cfg & 0x1ff) == base.end()) return false;
    const int dc = drain_code(cfg), bc = block_code(cfg);
    if (dc > 2 || (dc != 0 && st->queue != kQueueWave)) return false;
    if (bc > 2 || (bc != 0 && st->path != HPMC_PATH_PERSISTENT)) return false;
    for (const BatchGroup& g : st->groups)
        if (st->path == HPMC_PATH_PERSISTENT && group_block(g, bc) == 0) return false;
    return true;
}

// Switch to configuration cfg and re-capture the sweep graph.
int apply_config(hpmc_state* st, int cfg) {
    if (!config_valid(st, cfg)) return HPMC_ERR_INVALID_ARG;
    const int c = cfg & 0xff;
    st->walk64 = (cfg & kWalk64) ? 1 : 0;
    const uint32_t drain_at = kDrainAt[drain_code(cfg)];
    bool sys_changed = false;
    for (SysDev& S : st->sys) {
        sys_changed |= S.drain_at != drain_at;
        S.drain_at = drain_at;
    }
    if (sys_changed) {
        int rc = check_hip(st, hipMemcpyAsync(st->ws.sys, st->sys.data(), sizeof(SysDev) * st->n_replicas,
                                              hipMemcpyHostToDevice, st->stream));
        if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
        if (rc) return rc;
    }
    if (st->path == HPMC_PATH_PERSISTENT) {
        for (BatchGroup& g : st->groups) {
            g.block = group_block(g, block_code(cfg));
            group_lds(st, g, g.block);
            g.resident = highest_fit(g, c);
            g.lds_bytes = g.need[g.resident];
            const int rc = check_hip(st, persistent_sweeps(st->ws, g, st->pos, st->orient,
                                                           group_precision(st, g), true, st->stream));
            if (rc) return rc;
        }
    } else {
        for (ReplicaHost& rh : st->rep) rh.lanes_per_cell = c;
        for (BatchGroup& g : st->groups) g.lanes = c;
    }
    capture_graph(st);
    return HPMC_OK;
}

// Grid-path launch sizes of each group after a replica's box changed.
void refresh_grid_groups(hpmc_state* st) {
    if (st->path != HPMC_PATH_GRID) return;
    for (BatchGroup& g : st->groups) {
        g.rounds_max = 0;
        g.nc_max = 0;
        g.n_act_max = 0;
        for (int j = g.first; j < g.first + g.count; ++j) {
            const SysDev& S = st->sys[st->list[j]];
            const int half = S.n / 2;
            const int64_t n_act = S.dim == 3 ? (int64_t)half * half * half : (int64_t)half * half;
            g.rounds_max = std::max<int32_t>(g.rounds_max, S.rounds);
            g.nc_max = std::max<int64_t>(g.nc_max, S.ncells);
            g.n_act_max = std::max<int64_t>(g.n_act_max, n_act);
        }
    }
}

// Replace replica r's box description (host and device).  The kernels read
// the descriptor from device memory, so the captured sweep stays valid
// unless a launch size changed; only then is it captured again.
int set_replica_box(hpmc_state* st, int r, const SysDev& S, const ReplicaHost& rh) {
    st->sys[r] = S;
    st->rep[r] = rh;
    int rc = check_hip(st, hipMemcpyAsync(st->ws.sys + r, &st->sys[r], sizeof(SysDev),
                                          hipMemcpyHostToDevice, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    std::vector<BatchGroup> before = st->groups;
    refresh_grid_groups(st);
    bool same = before.size() == st->groups.size();
    for (size_t i = 0; same && i < before.size(); ++i)
        same = before[i].rounds_max == st->groups[i].rounds_max &&
               before[i].nc_max == st->groups[i].nc_max && before[i].n_act_max == st->groups[i].n_act_max;
    if (!rc && !same) capture_graph(st);
    return rc;
}

int run_sweeps(hpmc_state* st, uint64_t n_sweeps, uint32_t k0, uint32_t k1) {
    // a persistent launch runs the clock's n sweeps: whole chunks first, then
    // the shorter remainder through the same captured launch
    const uint32_t unit = sweep_unit(st);
    const uint32_t first = n_sweeps < unit ? (uint32_t)n_sweeps : unit;
    int rc = check_hip(st, set_clock(st->ws, (uint32_t)st->t, k0, k1, first, st->stream));
    uint64_t done = 0;
    while (!rc && done < n_sweeps) {
        const uint32_t len = n_sweeps - done < unit ? (uint32_t)(n_sweeps - done) : unit;
        if (len != first) rc = check_hip(st, set_chunk(st->ws, len, st->stream));
        if (rc) break;
        if (st->graph) {
            const hipError_t e = hipGraphLaunch(st->graph, st->stream);
            if (e != hipSuccess) {  // fall back to direct launches from here on
                (void)hipGetLastError();
                drop_graph(st);
                st->flags |= HPMC_FLAG_NO_GRAPH;
                continue;
            }
            st->graph_sweeps += len;
        } else {
            rc = enqueue_sweeps(st, st->stream);
        }
        done += len;
    }
    return rc;
}


// Device address of `scratch` on the current device: looked up once per
// device, with that device current, and kept.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

int static_scratch(void** out, int* hip_error) {
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) {
        *hip_error = (int)e;
        return HPMC_ERR_HIP;
    }
    if (dev < 0 || dev >= kMaxDevices) return HPMC_ERR_UNSUPPORTED;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (g_scratch_ptr[dev] == nullptr) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || p == nullptr) {
            *hip_error = (int)e;
            return HPMC_ERR_HIP;
        }
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return HPMC_OK;
}

// The caller's particle buffers: positions always, orientations unless every
// replica is a disk.
int check_buffers(const hpmc_init_args* args, const std::vector<SpeciesDev>& spc) {
    if (args->pos == nullptr) return HPMC_ERR_INVALID_ARG;
    if (args->orient == nullptr)
        for (const auto& sp : spc)
            if (sp.kind != kDisk) return HPMC_ERR_INVALID_ARG;
    return HPMC_OK;
}

// Point the state at the caller's arrays and carve its workspace (base) by
// the layout.
void bind_workspace(hpmc_state* st, const hpmc_init_args* args, const Layout& lay,
                    const std::vector<int32_t>& list, char* base) {
    st->n_replicas = args->n_replicas;
    st->precision = args->precision;
    st->stream = (hipStream_t)args->stream;
    st->pos = args->pos;
    st->orient = args->orient ? args->orient : args->pos;  // never dereferenced for disks
    st->ws.species = (SpeciesDev*)(base + lay.species);
    st->ws.sys = (SysDev*)(base + lay.sys);
    st->ws.stats = (unsigned long long*)(base + lay.stats);
    st->ws.overlap_out = (unsigned long long*)(base + lay.overlap);
    st->ws.count = (uint32_t*)(base + lay.count);
    st->ws.start = (uint32_t*)(base + lay.start);
    st->ws.cell_of = (uint32_t*)(base + lay.cell_of);
    st->ws.slot_of = (uint32_t*)(base + lay.slot_of);
    st->ws.members = (uint32_t*)(base + lay.members);
    st->ws.xs = (float*)(base + lay.xs);
    st->ws.hist_edges = (double*)(base + lay.hist_edges);
    st->ws.hist_out = (unsigned long long*)(base + lay.hist_out);
    st->ws.partial = (uint32_t*)(base + lay.partial);
    st->ws.batch_list = (int32_t*)(base + lay.list);
    st->ws.ident = (int32_t*)(base + lay.ident);
    st->ws.clock = (Clock*)(base + lay.clock);
    st->ws.backup_pos = (double*)(base + lay.backup_pos);
    st->ws.backup_ori = (double*)(base + lay.backup_ori);
    st->ws.backup_stats = (unsigned long long*)(base + lay.backup_stats);
    st->pos_total = lay.pos_total;
    st->ori_total = lay.ori_total;
    st->flags = args->flags;
    st->queue = queue_mode(args->flags);
    st->list = list;
    st->spec_host.assign(args->species, args->species + args->n_replicas);
    for (hpmc_species& sp : st->spec_host) sp.verts = nullptr;  // not kept by the caller
    st->sys_saved.assign(st->n_replicas, SysDev{});
    st->rep_saved.assign(st->n_replicas, ReplicaHost{});
    st->box_saved.assign(st->n_replicas, 0);
    if (st->queue == kQueueGlobal) {
        GlobalQueue& q = st->ws.gq;
        q.trial = (double*)(base + lay.gq_trial);
        q.meta = (uint32_t*)(base + lay.gq_meta);
        q.flag = (uint32_t*)(base + lay.gq_flag);
        q.entries = (uint2*)(base + lay.gq_entries);
        q.count = (uint32_t*)(base + lay.gq_count);
        q.cell_total = lay.cell_total;
    }
}

// Copy the shape, grid and launch tables to the workspace, clear what the
// kernels expect to start at zero (counters, cell histograms, queue
// lengths), raise the persistent kernels' LDS limit, and check that every
// position lies in [0, L) and every orientation is finite (before any cell
// lookup).  Synchronises the stream.
int upload_and_validate(hpmc_state* st, const Layout& lay) {
    int rc = check_hip(st, hipMemcpyAsync(st->ws.species, st->spc.data(),
                                          sizeof(SpeciesDev) * st->n_replicas, hipMemcpyHostToDevice,
                                          st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(st->ws.sys, st->sys.data(), sizeof(SysDev) * st->n_replicas,
                                          hipMemcpyHostToDevice, st->stream));
    if (!rc && !st->list.empty())
        rc = check_hip(st, hipMemcpyAsync(st->ws.batch_list, st->list.data(),
                                          sizeof(int32_t) * st->list.size(), hipMemcpyHostToDevice,
                                          st->stream));
    std::vector<int32_t> ident(st->n_replicas);
    for (int r = 0; r < st->n_replicas; ++r) ident[r] = r;
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(st->ws.ident, ident.data(), sizeof(int32_t) * ident.size(),
                                          hipMemcpyHostToDevice, st->stream));
    if (!rc)
        rc = check_hip(st, fill_u64(st->ws.stats, 0ull, (size_t)kStatsPerReplica * st->n_replicas,
                                    st->stream));
    if (!rc) rc = check_hip(st, set_clock(st->ws, 0u, 0u, 0u, 1u, st->stream));
    if (!rc)  // cell histograms start at zero; every build leaves them so
        rc = check_hip(st, fill_u64((unsigned long long*)st->ws.count, 0ull,
                                    ((size_t)lay.cell_total + 1) / 2, st->stream));
    if (!rc && st->queue == kQueueGlobal)  // queue lengths start at zero; each pass leaves them so
        rc = check_hip(st, fill_u64((unsigned long long*)st->ws.gq.count, 0ull, (size_t)st->n_replicas,
                                    st->stream));
    if (st->path == HPMC_PATH_PERSISTENT)
        for (const BatchGroup& g : st->groups)
            if (!rc) rc = check_hip(st, persistent_sweeps(st->ws, g, st->pos, st->orient, group_precision(st, g),
                                                          true, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    if (rc) return rc;
    std::vector<uint64_t> bad(st->n_replicas, 0);
    rc = check_hip(st, fill_u64(st->ws.overlap_out, 0ull, st->n_replicas, st->stream));
    for (int r = 0; r < st->n_replicas && !rc; ++r)
        rc = check_hip(st, validate_state(st->ws, st->rep[r], r, st->pos, st->orient, st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(bad.data(), st->ws.overlap_out, sizeof(uint64_t) * st->n_replicas,
                                          hipMemcpyDeviceToHost, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    if (!rc)
        for (uint64_t b : bad)
            if (b != 0) rc = HPMC_ERR_INVALID_ARG;
    return rc;
}

}  // namespace

extern "C" {

int hpmc_workspace_bytes(const hpmc_init_args* args, size_t* out_bytes) {
    if (out_bytes == nullptr) return HPMC_ERR_INVALID_ARG;
    std::vector<ReplicaHost> rep;
    std::vector<SysDev> sys;
    std::vector<SpeciesDev> spc;
    Layout lay{};
    int path = 0;
    std::vector<BatchGroup> groups;
    std::vector<int32_t> list;
    const int rc = plan(args, rep, sys, spc, lay, path, groups, list, device_lds_limit());
    if (rc) return rc;
    *out_bytes = lay.total;
    return HPMC_OK;
}

int hpmc_init(hpmc_state** out, const hpmc_init_args* args) {
    if (out == nullptr) return HPMC_ERR_INVALID_ARG;
    *out = nullptr;
    hpmc_state* st = new (std::nothrow) hpmc_state();
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    Layout lay{};
    std::vector<int32_t> list;
    int rc = plan(args, st->rep, st->sys, st->spc, lay, st->path, st->groups, list,
                  device_lds_limit());
    if (rc == HPMC_OK) rc = check_buffers(args, st->spc);
    if (rc == HPMC_OK && args->workspace == nullptr) rc = HPMC_ERR_INVALID_ARG;
    if (rc == HPMC_OK && ((uintptr_t)args->workspace % kAlign) != 0) rc = HPMC_ERR_INVALID_ARG;
    if (rc == HPMC_OK && args->workspace_bytes < lay.total) rc = HPMC_ERR_WORKSPACE_TOO_SMALL;
    if (rc) {
        delete st;
        return rc;
    }
    bind_workspace(st, args, lay, list, (char*)args->workspace);
    rc = upload_and_validate(st, lay);
    if (!rc) {
        std::vector<uint64_t> counts(st->n_replicas, 0);
        rc = count_all(st, counts.data());
        if (!rc)
            for (uint64_t c : counts)
                if (c != 0) rc = HPMC_ERR_INITIAL_OVERLAP;
    }
    if (!rc) make_side_streams(st);
    if (!rc) capture_graph(st);
    if (rc) {
        g_last_init_hip.store(st->last_hip);
        hpmc_destroy(st);
        return rc;
    }
    *out = st;
    return HPMC_OK;
}

int hpmc_sweep_static(const hpmc_init_args* args, uint64_t t0, uint64_t n_sweeps, uint64_t seed,
                      hpmc_stats* out_per_replica, int32_t* hip_error) {
    if (hip_error) *hip_error = 0;
    if (args == nullptr) return HPMC_ERR_INVALID_ARG;
    if (t0 >= kSweepLimit || n_sweeps > kSweepLimit - t0) return HPMC_ERR_SWEEP_OVERFLOW;
    hpmc_state st;
    Layout lay{};
    std::vector<int32_t> list;
    int rc = plan(args, st.rep, st.sys, st.spc, lay, st.path, st.groups, list, device_lds_limit(),
                  false);
    if (rc) return rc;
    rc = check_buffers(args, st.spc);
    if (!rc && (args->workspace != nullptr || args->workspace_bytes != 0)) rc = HPMC_ERR_INVALID_ARG;
    if (!rc && queue_mode(args->flags) != kQueueWave) rc = HPMC_ERR_UNSUPPORTED;
    if (!rc && lay.total > (size_t)HPMC_STATIC_SCRATCH_BYTES) rc = HPMC_ERR_WORKSPACE_TOO_SMALL;
    if (rc) return rc;
    void* base = nullptr;
    int hip = 0;
    rc = static_scratch(&base, &hip);
    if (rc) {
        if (hip_error) *hip_error = hip;
        return rc;
    }
    bind_workspace(&st, args, lay, list, (char*)base);
    st.flags |= HPMC_FLAG_NO_GRAPH;  // direct launches: no graph, no side streams
    rc = upload_and_validate(&st, lay);
    st.t = t0;
    if (!rc && n_sweeps) rc = run_sweeps(&st, n_sweeps, (uint32_t)seed, (uint32_t)(seed >> 32));
    st.sweeps_done = n_sweeps;
    if (!rc && out_per_replica) rc = hpmc_get_stats(&st, out_per_replica);
    if (!rc) rc = check_hip(&st, hipStreamSynchronize(st.stream));
    if (hip_error) *hip_error = st.last_hip;
    return rc;
}

int hpmc_sweep(hpmc_state* st, uint64_t n_sweeps, uint64_t seed) {
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    if (n_sweeps == 0) return HPMC_OK;
    if (n_sweeps > kSweepLimit || st->t + n_sweeps > kSweepLimit) return HPMC_ERR_SWEEP_OVERFLOW;
    const int rc = run_sweeps(st, n_sweeps, (uint32_t)seed, (uint32_t)(seed >> 32));
    if (rc) return rc;
    st->t += n_sweeps;
    st->sweeps_done += n_sweeps;
    return HPMC_OK;
}

int hpmc_count_overlaps(hpmc_state* st, uint64_t* out_per_replica) {
    if (st == nullptr || out_per_replica == nullptr) return HPMC_ERR_INVALID_ARG;
    return count_all(st, out_per_replica);
}

int hpmc_pair_histogram(hpmc_state* st, int32_t replica, const double* edges2, int32_t n_bins,
                        uint64_t* out) {
    if (st == nullptr || edges2 == nullptr || out == nullptr) return HPMC_ERR_INVALID_ARG;
    if (replica < 0 || replica >= st->n_replicas || n_bins < 1 || n_bins > kMaxHistBins)
        return HPMC_ERR_INVALID_ARG;
    if (!(edges2[0] >= 0.0)) return HPMC_ERR_INVALID_ARG;
    for (int b = 0; b < n_bins; ++b)
        if (!(edges2[b] < edges2[b + 1]) || !std::isfinite(edges2[b + 1])) return HPMC_ERR_INVALID_ARG;
    // pairs closer than reach cell widths lie within `reach` cells of each other
    const ReplicaHost& rh = st->rep[replica];
    const double w = st->sys[replica].w;
    const double guard = 1.0 - 0x1p-30;
    int reach = 0;
    if (edges2[n_bins] <= w * w * guard)
        reach = 1;
    else if (edges2[n_bins] <= 4.0 * w * w * guard && rh.n >= 5)
        reach = 2;
    else
        return HPMC_ERR_UNSUPPORTED;
    int rc = check_hip(st, hipMemcpyAsync(st->ws.hist_edges, edges2, sizeof(double) * (n_bins + 1),
                                          hipMemcpyHostToDevice, st->stream));
    if (!rc) rc = check_hip(st, build_cells_one(st->ws, rh, replica, st->pos, 0, st->stream));
    if (!rc) rc = check_hip(st, pair_histogram(st->ws, rh, replica, st->pos, n_bins, reach, st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(out, st->ws.hist_out, sizeof(uint64_t) * n_bins,
                                          hipMemcpyDeviceToHost, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    return rc;
}

int hpmc_scale_box(hpmc_state* st, int32_t replica, double L_new, uint64_t* overlaps) {
    if (st == nullptr || replica < 0 || replica >= st->n_replicas) return HPMC_ERR_INVALID_ARG;
    const int r = replica;
    if (!(L_new > 0.0) || !std::isfinite(L_new) || L_new > st->rep[r].L_max)
        return HPMC_ERR_INVALID_ARG;
    SysDev S = st->sys[r];
    ReplicaHost rh = st->rep[r];
    int rc = build_grid(st->spec_host[r], st->spc[r], rh.N, L_new, S, rh);
    if (rc) return rc;
    if (rh.ncells > st->rep[r].ncells_cap) return HPMC_ERR_INVALID_ARG;
    // keep what build_grid does not know: offsets, indices, launch settings
    const SysDev& old = st->sys[r];
    S.species = old.species;
    S.replica = old.replica;
    S.path = old.path;
    S.pos_off = old.pos_off;
    S.orient_off = old.orient_off;
    S.cell_off = old.cell_off;
    S.slot_off = old.slot_off;
    S.part_off = old.part_off;
    S.drain_at = old.drain_at;
    S.ghost_cap = old.ghost_cap;
    const ReplicaHost& oh = st->rep[r];
    rh.path = oh.path;
    rh.lanes_per_cell = oh.lanes_per_cell;
    rh.ghost_cap = oh.ghost_cap;
    rh.n_cap = oh.n_cap;
    rh.nv = oh.nv;
    rh.pos_off = oh.pos_off;
    rh.orient_off = oh.orient_off;
    rh.ncells_cap = oh.ncells_cap;
    rh.L_max = oh.L_max;
    const int64_t nval = (int64_t)rh.dim * rh.N;
    double* p = st->pos + oh.pos_off;
    rc = check_hip(st, hipMemcpyAsync(st->ws.backup_pos + oh.pos_off, p, 8 * (size_t)nval,
                                      hipMemcpyDeviceToDevice, st->stream));
    if (!rc) rc = check_hip(st, scale_box(p, nval, L_new / old.L, L_new, st->stream));
    if (rc) return rc;
    st->sys_saved[r] = st->sys[r];
    st->rep_saved[r] = st->rep[r];
    st->box_saved[r] = 1;
    rc = set_replica_box(st, r, S, rh);
    if (rc || overlaps == nullptr) return rc;
    rc = check_hip(st, fill_u64(st->ws.overlap_out, 0ull, st->n_replicas, st->stream));
    if (!rc) rc = check_hip(st, build_cells_one(st->ws, st->rep[r], r, st->pos, 0, st->stream));
    if (!rc) rc = check_hip(st, count_pairs(st->ws, st->rep[r], r, st->pos, st->orient, st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(overlaps, st->ws.overlap_out + r, sizeof(uint64_t),
                                          hipMemcpyDeviceToHost, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    return rc;
}

int hpmc_restore_box(hpmc_state* st, int32_t replica) {
    if (st == nullptr || replica < 0 || replica >= st->n_replicas || !st->box_saved[replica])
        return HPMC_ERR_INVALID_ARG;
    const int r = replica;
    const ReplicaHost& rh = st->rep_saved[r];
    const int64_t nval = (int64_t)rh.dim * rh.N;
    int rc = check_hip(st, hipMemcpyAsync(st->pos + rh.pos_off, st->ws.backup_pos + rh.pos_off,
                                          8 * (size_t)nval, hipMemcpyDeviceToDevice, st->stream));
    if (rc) return rc;
    st->box_saved[r] = 0;
    return set_replica_box(st, r, st->sys_saved[r], st->rep_saved[r]);
}

int hpmc_scale_counts(hpmc_state* st, int32_t replica, const double* scales, int32_t n_scales,
                      uint64_t* out) {
    if (st == nullptr || scales == nullptr || out == nullptr) return HPMC_ERR_INVALID_ARG;
    if (replica < 0 || replica >= st->n_replicas || n_scales < 1 || n_scales > kMaxHistBins)
        return HPMC_ERR_INVALID_ARG;
    for (int b = 0; b < n_scales; ++b)
        if (!(scales[b] >= 0.0 && scales[b] < 1.0) || (b > 0 && !(scales[b - 1] < scales[b])))
            return HPMC_ERR_INVALID_ARG;
    // a pair can overlap at the largest compression only if |r| < 2R / f_min;
    // such pairs lie within `reach` cells of each other
    const ReplicaHost& rh = st->rep[replica];
    const double w = st->sys[replica].w, f_min = 1.0 - scales[n_scales - 1];
    const double circ2 = st->spc[replica].circ2, guard = 1.0 - 0x1p-30;
    int reach = 0;
    if (circ2 <= w * w * f_min * f_min * guard)
        reach = 1;
    else if (circ2 <= 4.0 * w * w * f_min * f_min * guard && rh.n >= 5)
        reach = 2;
    else
        return HPMC_ERR_UNSUPPORTED;
    int rc = check_hip(st, hipMemcpyAsync(st->ws.hist_edges, scales, sizeof(double) * n_scales,
                                          hipMemcpyHostToDevice, st->stream));
    if (!rc) rc = check_hip(st, build_cells_one(st->ws, rh, replica, st->pos, 0, st->stream));
    if (!rc)
        rc = check_hip(st, scale_counts(st->ws, rh, replica, st->pos, st->orient, n_scales, reach,
                                        st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(out, st->ws.hist_out, sizeof(uint64_t) * n_scales,
                                          hipMemcpyDeviceToHost, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    return rc;
}

int hpmc_get_stats(hpmc_state* st, hpmc_stats* out) {
    if (st == nullptr || out == nullptr) return HPMC_ERR_INVALID_ARG;
    std::vector<unsigned long long> raw((size_t)kStatsPerReplica * st->n_replicas);
    int rc = check_hip(st, hipMemcpyAsync(raw.data(), st->ws.stats, raw.size() * sizeof(raw[0]),
                                          hipMemcpyDeviceToHost, st->stream));
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    if (rc) return rc;
    for (int r = 0; r < st->n_replicas; ++r) {
        unsigned long long v[kNumStats] = {};
        for (int s = 0; s < kStatStripes; ++s)
            for (int k = 0; k < kNumStats; ++k)
                v[k] += raw[((size_t)r * kStatStripes + s) * kStatStride + k];
        out[r].attempted = v[kAttempted];
        out[r].attempted_rot = v[kAttemptedRot];
        out[r].cell_reject = v[kCellReject];
        out[r].overlap_reject = v[kOverlapReject];
        out[r].accept = v[kAccept];
        out[r].pair_tests = v[kPairTests];
        out[r].pair_fp64 = v[kPairFp64];
        out[r].sweeps = st->sweeps_done;
        if (v[kCellOverflow]) rc = HPMC_ERR_CELL_OVERFLOW;
    }
    return rc;
}

int hpmc_reset_stats(hpmc_state* st) {
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    st->sweeps_done = 0;
    return check_hip(st, fill_u64(st->ws.stats, 0ull, (size_t)kStatsPerReplica * st->n_replicas,
                                  st->stream));
}

int hpmc_sync_to_canonical(hpmc_state* st) {
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    return check_hip(st, hipStreamSynchronize(st->stream));
}

int hpmc_get_sweep(hpmc_state* st, uint64_t* out_t) {
    if (st == nullptr || out_t == nullptr) return HPMC_ERR_INVALID_ARG;
    *out_t = st->t;
    return HPMC_OK;
}

int hpmc_set_sweep(hpmc_state* st, uint64_t t) {
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    if (t >= kSweepLimit) return HPMC_ERR_SWEEP_OVERFLOW;
    st->t = t;
    return HPMC_OK;
}

int hpmc_replica_info(hpmc_state* st, int32_t r, int32_t* cells_per_side, int32_t* rounds,
                      int32_t* path) {
    if (st == nullptr || r < 0 || r >= st->n_replicas) return HPMC_ERR_INVALID_ARG;
    if (cells_per_side) *cells_per_side = st->rep[r].n;
    if (rounds) *rounds = st->rep[r].rounds;
    if (path) *path = st->path;
    return HPMC_OK;
}

int hpmc_last_hip_error(hpmc_state* st) { return st ? st->last_hip : g_last_init_hip.load(); }

void hpmc_destroy(hpmc_state* st) {
    if (st == nullptr) return;
    (void)hipStreamSynchronize(st->stream);
    drop_graph(st);
    drop_side_streams(st);
    if (st->cap_stream) (void)hipStreamDestroy(st->cap_stream);
    delete st;
}

int hpmc_uses_graph(hpmc_state* st) { return (st && st->graph) ? 1 : 0; }

int hpmc_phase_trace(uint64_t* out, int32_t n, int32_t reset) {
    if (out == nullptr || n < kTraceWords) return HPMC_ERR_INVALID_ARG;
    const hipError_t e = read_phase_trace((unsigned long long*)out, reset != 0);
    if (e == hipErrorNotSupported) return HPMC_ERR_UNSUPPORTED;
    return e == hipSuccess ? HPMC_OK : HPMC_ERR_HIP;
}

int hpmc_graph_sweeps(hpmc_state* st, uint64_t* out) {
    if (st == nullptr || out == nullptr) return HPMC_ERR_INVALID_ARG;
    *out = st->graph_sweeps;
    return HPMC_OK;
}

int hpmc_volume_move(hpmc_state* st, int32_t replica, double u1, double u2, double beta_p,
                     double delta_v, int32_t* accepted, double* L_after) {
    if (st == nullptr || accepted == nullptr || replica < 0 || replica >= st->n_replicas)
        return HPMC_ERR_INVALID_ARG;
    if (!(u1 >= 0.0 && u1 < 1.0) || !(u2 >= 0.0 && u2 < 1.0) || !std::isfinite(beta_p) ||
        !(delta_v >= 0.0) || !std::isfinite(delta_v))
        return HPMC_ERR_INVALID_ARG;
    const int r = replica;
    const ReplicaHost& rh = st->rep[r];
    *accepted = 0;
    const double L = rh.L;
    if (L_after) *L_after = L;
    // trial volume V' = V + delta_v (2 u1 - 1) and side V'^(1/dim)
    const double V = std::pow(L, (double)rh.dim);
    const double dV = delta_v * (2.0 * u1 - 1.0);
    const double V2 = V + dV;
    if (!(V2 > 0.0)) return HPMC_OK;
    const double L2 = std::pow(V2, 1.0 / (double)rh.dim);
    if (L2 > rh.L_max) return HPMC_OK;
    // scaled state; only a compression can create an overlap (the overlap
    // region of two convex shapes is a convex set of separations containing
    // 0, so r outside it keeps k r outside for k >= 1)
    uint64_t ov = 0;
    int rc = hpmc_scale_box(st, r, L2, dV < 0.0 ? &ov : nullptr);
    if (rc == HPMC_ERR_BOX_TOO_SMALL) return HPMC_OK;
    if (rc) return rc;
    // Metropolis test of the isobaric volume move, min(1, exp(arg)); with
    // u2 < 1 every arg >= 0 accepts, which also keeps exp from overflowing
    const double arg = -beta_p * dV + (double)rh.N * std::log(V2 / V);
    const bool ok = !(dV < 0.0 && ov > 0) && (arg >= 0.0 || u2 < std::exp(arg));
    if (!ok) return hpmc_restore_box(st, r);
    *accepted = 1;
    if (L_after) *L_after = L2;
    return HPMC_OK;
}

int hpmc_autotune(hpmc_state* st, uint32_t trial_sweeps, int32_t* out_config) {
    if (st == nullptr || trial_sweeps == 0) return HPMC_ERR_INVALID_ARG;
    std::fill(st->box_saved.begin(), st->box_saved.end(), 0);  // its snapshot reuses that buffer
    const size_t nstat = (size_t)kStatsPerReplica * st->n_replicas;
    // snapshot the caller's state
    int rc = check_hip(st, hipMemcpyAsync(st->ws.backup_pos, st->pos, 8 * st->pos_total,
                                          hipMemcpyDeviceToDevice, st->stream));
    if (!rc && st->ori_total)
        rc = check_hip(st, hipMemcpyAsync(st->ws.backup_ori, st->orient, 8 * st->ori_total,
                                          hipMemcpyDeviceToDevice, st->stream));
    if (!rc)
        rc = check_hip(st, hipMemcpyAsync(st->ws.backup_stats, st->ws.stats, 8 * nstat,
                                          hipMemcpyDeviceToDevice, st->stream));
    if (rc) return rc;
    // three stages, each keeping the fastest: lanes per cell or LDS
    // residency (and the walk), then the queue depth, then (persistent) the
    // work-group size
    std::vector<int> cands = base_candidates(st);
    auto apply = [&](int cfg) { (void)apply_config(st, cfg); };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (!rc) rc = check_hip(st, hipEventCreate(&e0));
    if (!rc) rc = check_hip(st, hipEventCreate(&e1));
    float best_ms = 0.f;
    int best = cands.empty() ? 0 : cands[0];
    bool first = true;
    for (int stage = 0; stage < 3 && !rc; ++stage) {
        if (stage == 1) {
            cands.clear();
            for (int dc = 1; dc <= 2; ++dc) cands.push_back(best | (dc << kDrainShift));
        } else if (stage == 2) {
            cands.clear();
            for (int bc = 1; bc <= 2; ++bc) cands.push_back(best | (bc << kBlockShift));
        }
    for (size_t ci = 0; ci < cands.size() && !rc; ++ci) {
        if (!config_valid(st, cands[ci])) continue;
        apply(cands[ci]);
        rc = run_sweeps(st, 1, 0xA5A5u, 0x5A5Au);  // warm-up
        if (!rc) rc = check_hip(st, hipEventRecord(e0, st->stream));
        if (!rc) rc = run_sweeps(st, trial_sweeps, 0xA5A5u, 0x5A5Au);
        if (!rc) rc = check_hip(st, hipEventRecord(e1, st->stream));
        if (!rc) rc = check_hip(st, hipEventSynchronize(e1));
        float ms = 0.f;
        if (!rc) rc = check_hip(st, hipEventElapsedTime(&ms, e0, e1));
        if (!rc && (first || ms < best_ms)) {
            best_ms = ms;
            best = cands[ci];
            first = false;
        }
        // restore the snapshot after every trial
        if (!rc)
            rc = check_hip(st, hipMemcpyAsync(st->pos, st->ws.backup_pos, 8 * st->pos_total,
                                              hipMemcpyDeviceToDevice, st->stream));
        if (!rc && st->ori_total)
            rc = check_hip(st, hipMemcpyAsync(st->orient, st->ws.backup_ori, 8 * st->ori_total,
                                              hipMemcpyDeviceToDevice, st->stream));
        if (!rc)
            rc = check_hip(st, hipMemcpyAsync(st->ws.stats, st->ws.backup_stats, 8 * nstat,
                                              hipMemcpyDeviceToDevice, st->stream));
    }
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    if (!rc) apply(best);
    if (!rc) rc = check_hip(st, hipStreamSynchronize(st->stream));
    if (!rc && out_config) *out_config = best;
    return rc;
}

int hpmc_set_config(hpmc_state* st, int32_t config) {
    if (st == nullptr) return HPMC_ERR_INVALID_ARG;
    int rc = check_hip(st, hipStreamSynchronize(st->stream));
    if (!rc) rc = apply_config(st, config);
    return rc;
}

const char* hpmc_strerror(int code) {
    switch (code) {
        case HPMC_OK: return "ok";
        case HPMC_ERR_INVALID_ARG: return "invalid argument";
        case HPMC_ERR_BOX_TOO_SMALL: return "box too small: fewer than 4 cells per side";
        case HPMC_ERR_INITIAL_OVERLAP: return "initial configuration has overlapping particles";
        case HPMC_ERR_WORKSPACE_TOO_SMALL: return "workspace too small";
        case HPMC_ERR_HIP: return "HIP runtime error";
        case HPMC_ERR_SWEEP_OVERFLOW: return "sweep counter would exceed 2^32";
        case HPMC_ERR_UNSUPPORTED: return "unsupported configuration";
        case HPMC_ERR_CELL_OVERFLOW: return "cell list overflow (overlapping state)";
        default: return "unknown error";
    }
}

}  // extern "C"
