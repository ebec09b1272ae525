// One colour pass over a tile of active cells, executed by one wave64.
//
// The paper's block queue (Sec. 2.5.3) restricted to a wave, so that no
// work-group barrier is needed inside a pass:
//   1. the leader lane of each group of G lanes proposes the trial move of
//      its cell (uniform occupant, Philox stream, translation or rotation,
//      reject when it leaves the cell) and broadcasts it to its group;
//   2. the group's lanes scan the 3^dim neighbour cells in a strided fashion
//      and only run a binary32 circumsphere pre-filter on a cell-sorted copy
//      of the grid coordinates; hits are compacted with a wave ballot and
//      prefix count into an LDS ring of (owner lane, neighbour slot);
//   3. whenever 64 entries are queued, every lane takes one entry and runs
//      the binary64 circumsphere test and then the full overlap test; an
//      overlap sets the owner cell's flag, and flagged cells queue no further
//      work (early exit);
//   4. leaders of unflagged live cells write the move back.
// The accept decision is the OR over all neighbours, so it does not depend on
// the order in which the tests run.
#pragma once

#include <type_traits>

#include "device_common.hpp"
#include "overlap32.hpp"
#include "overlap64.hpp"
#include "types.hpp"

namespace hpmc {

template <int KIND>
struct Traits {
    static constexpr int dim = KIND == kPolyhedron ? 3 : 2;
    static constexpr int ncomp = orient_comps(KIND);
    static constexpr int nbrs = KIND == kPolyhedron ? 27 : 9;
};

// Shapes turned by a unit complex number (Sec. 2.1's 2D rotation move).
template <int KIND>
constexpr bool kPlanarTurn = KIND == kPolygon || KIND == kSpheropolygon;

// Per-lane counters, named fields (an array indexed on two branches gets its
// increments merged through a selected address and lands in scratch).
struct Counters {
    uint32_t attempted, attempted_rot, cell_reject, overlap_reject, accept, pair_tests, pair_fp64;
};

__device__ __forceinline__ void flush_one(uint32_t v, unsigned long long* p) {
    const uint32_t s = wave_sum(v);
    if (__lane_id() == 0 && s != 0) atomicAdd(p, (unsigned long long)s);
}

// The stripe of replica r's counters that this work-group adds into.
__device__ __forceinline__ unsigned long long* stat_stripe(unsigned long long* stats, int r) {
    return stats + ((size_t)r * kStatStripes + blockIdx.x % kStatStripes) * kStatStride;
}

// One 64-bit atomic per wave and counter.  Every lane of the wave must call.
__device__ __forceinline__ void flush(const Counters& c, unsigned long long* stats) {
    flush_one(c.attempted, stats + kAttempted);
    flush_one(c.attempted_rot, stats + kAttemptedRot);
    flush_one(c.cell_reject, stats + kCellReject);
    flush_one(c.overlap_reject, stats + kOverlapReject);
    flush_one(c.accept, stats + kAccept);
    flush_one(c.pair_tests, stats + kPairTests);
    flush_one(c.pair_fp64, stats + kPairFp64);
}

// One 64-bit atomic per work-group and counter: the waves' sums meet in LDS
// (lds: at least 4 x kNumStats words, free to overwrite).  Every thread of
// the work-group must call (contains barriers); at most 16 waves.
__device__ __forceinline__ void flush_block(const Counters& c, uint32_t* lds, unsigned long long* stats) {
    const uint32_t v[kNumStats] = {c.attempted, c.attempted_rot, c.cell_reject, c.overlap_reject,
                                   c.accept, c.pair_tests, c.pair_fp64};
    const int wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    uint32_t s[kNumStats];
#pragma unroll
    for (int k = 0; k < kNumStats; ++k) s[k] = wave_sum(v[k]);
    __syncthreads();
    if (__lane_id() == 0) {
#pragma unroll
        for (int k = 0; k < kNumStats; ++k) lds[wave * kNumStats + k] = s[k];
    }
    __syncthreads();
    if ((int)threadIdx.x < kNumStats) {
        unsigned long long t = 0;
        for (int w = 0; w < nwaves; ++w) t += lds[w * kNumStats + threadIdx.x];
        if (t) atomicAdd(stats + threadIdx.x, t);
    }
}

// Per-wave phase clock.  In a trace build (HPMC_TRACE) mark<PH>() adds the
// shader cycles since the previous mark to phase PH (all lanes hold the same
// wave-uniform values); flush() adds a wave's totals and 1 to the wave count
// of its kernel's record.  In a normal build every call is empty.
#ifdef HPMC_TRACE
struct PhaseClock {
    unsigned long long acc[kNumPhases];
    unsigned long long last;
    __device__ __forceinline__ void start() {
#pragma unroll
        for (int k = 0; k < kNumPhases; ++k) acc[k] = 0ull;
        last = (unsigned long long)clock64();
    }
    template <int PH>
    __device__ __forceinline__ void mark() {
        const unsigned long long now = (unsigned long long)clock64();
        acc[PH] += now - last;
        last = now;
    }
    __device__ __forceinline__ void flush(unsigned long long* rec) const {
        if (__lane_id() == 0) {
#pragma unroll
            for (int k = 0; k < kNumPhases; ++k) atomicAdd(rec + k, acc[k]);
            atomicAdd(rec + kNumPhases, 1ull);
        }
    }
};
#else
struct PhaseClock {
    __device__ __forceinline__ void start() {}
    template <int PH>
    __device__ __forceinline__ void mark() {}
    __device__ __forceinline__ void flush(unsigned long long*) const {}
};
#endif

__device__ __forceinline__ void wave_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

// ---------------------------------------------------------------------------
// Views of particle positions (tag order, structure of arrays) and of the
// cell list.
// ---------------------------------------------------------------------------
struct PosView {
    double* p;  // global or LDS
    int N;
    __device__ __forceinline__ double get(int a, uint32_t k) const { return p[a * N + k]; }
    __device__ __forceinline__ void set(int a, uint32_t k, double v) const { p[a * N + k] = v; }
};

struct GlobalCells {
    static constexpr bool ghost = false;
    const uint32_t* __restrict__ start;
    const uint32_t* __restrict__ members;
    // storage index of cell cc (linear index c)
    __device__ __forceinline__ uint32_t index(const int (&)[3], uint32_t c, int) const { return c; }
    __device__ __forceinline__ uint32_t begin(uint32_t c) const { return start[c]; }
    __device__ __forceinline__ uint32_t end(uint32_t c) const { return start[c + 1]; }
    __device__ __forceinline__ uint32_t member(uint32_t p) const { return members[p]; }
};

// LDS cell list: inclusive ends[ncells] and members (16-bit tags).
struct LdsCells {
    static constexpr bool ghost = false;
    const uint16_t* ends;
    const uint16_t* members;
    __device__ __forceinline__ uint32_t index(const int (&)[3], uint32_t c, int) const { return c; }
    __device__ __forceinline__ uint32_t begin(uint32_t c) const { return c ? ends[c - 1] : 0u; }
    __device__ __forceinline__ uint32_t end(uint32_t c) const { return ends[c]; }
    __device__ __forceinline__ uint32_t member(uint32_t p) const { return members[p]; }
};

// LDS cell list of a 2D grid with ghost edge columns: every row of n cells
// is stored as n + 2, the first a copy of the row's last cell and the last a
// copy of its first, their binary32 coordinates shifted by -L and +L.  The
// cells x - 1 .. x + 1 of any row are then one contiguous slot range, with
// no periodic wrap along x.  Storage index of cell (x, y): x + 1 + (n + 2) y.
struct LdsGhostCells {
    static constexpr bool ghost = true;
    const uint16_t* ends;
    const uint16_t* members;
    __device__ __forceinline__ uint32_t index(const int (&cc)[3], uint32_t, int n) const {
        return (uint32_t)(cc[0] + 1 + (n + 2) * cc[1]);
    }
    __device__ __forceinline__ uint32_t begin(uint32_t c) const { return c ? ends[c - 1] : 0u; }
    __device__ __forceinline__ uint32_t end(uint32_t c) const { return ends[c]; }
    __device__ __forceinline__ uint32_t member(uint32_t p) const { return members[p]; }
};

// Cell-sorted binary32 copy of the grid coordinates: slot p of the cell list
// holds the shifted-frame coordinates of its member (2D float2, 3D float4).
// Only the pre-filter reads it; every decision uses the binary64 state.
template <int D>
struct XsView {
    float* p;
    __device__ __forceinline__ void load(uint32_t s, float (&v)[3]) const {
        if constexpr (D == 2) {
            const float2 f = reinterpret_cast<const float2*>(p)[s];
            v[0] = f.x;
            v[1] = f.y;
            v[2] = 0.0f;
        } else {
            const float4 f = reinterpret_cast<const float4*>(p)[s];
            v[0] = f.x;
            v[1] = f.y;
            v[2] = f.z;
        }
    }
    __device__ __forceinline__ void store(uint32_t s, const double (&y)[3]) const {
        if constexpr (D == 2)
            reinterpret_cast<float2*>(p)[s] = make_float2((float)y[0], (float)y[1]);
        else
            reinterpret_cast<float4*>(p)[s] = make_float4((float)y[0], (float)y[1], (float)y[2], 0.0f);
    }
    __device__ __forceinline__ void store(uint32_t s, const float (&v)[3]) const {
        if constexpr (D == 2)
            reinterpret_cast<float2*>(p)[s] = make_float2(v[0], v[1]);
        else
            reinterpret_cast<float4*>(p)[s] = make_float4(v[0], v[1], v[2], 0.0f);
    }
};

// The same binary32 shifted-frame coordinates computed on the fly from the
// binary64 positions (tag order, LDS) through the cell list's members, for
// work-groups that keep positions and orientations in LDS and have no room
// for the copy: the values equal the copy's bit for bit (one binary64
// subtraction and wrap, then the cast), so the pre-filter decides the same.
// Stores are dropped: the positions themselves are the state.
template <int D>
struct PosXsView {
    const uint16_t* mem;
    const double* p;
    int N;
    double s0, s1, s2, L;
    __device__ __forceinline__ void load(uint32_t s, float (&v)[3]) const {
        const uint32_t k = mem[s];
        v[0] = (float)grid_coord(p[k], s0, L);
        v[1] = (float)grid_coord(p[N + k], s1, L);
        v[2] = D == 3 ? (float)grid_coord(p[2 * N + k], s2, L) : 0.0f;
    }
    template <class T>
    __device__ __forceinline__ void store(uint32_t, const T&) const {}
};

template <int KIND>
__device__ __forceinline__ void load_orient(const double* __restrict__ ori, int N, uint32_t i,
                                            double (&q)[4]) {
    q[0] = 1.0;
    q[1] = q[2] = q[3] = 0.0;
    if constexpr (kPlanarTurn<KIND>) {
        q[0] = ori[i];
        q[1] = ori[N + i];
    } else if constexpr (KIND == kPolyhedron) {
        q[0] = ori[i];
        q[1] = ori[N + i];
        q[2] = ori[2 * N + i];
        q[3] = ori[3 * N + i];
    }
}

// Full overlap test of a pair that passed the circumsphere test.
template <int KIND, int PREC, int NV>
__device__ __forceinline__ bool full_test(const SpeciesDev& P, const double (&r)[3],
                                          const double (&qi)[4], const double (&qk)[4],
                                          Counters& ct) {
    if constexpr (KIND == kDisk) {
        return true;
    } else if constexpr (KIND == kSpheropolygon) {
        ct.pair_tests++;
        ct.pair_fp64++;
        return spheropolygon_overlap64(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1]);
    } else if constexpr (KIND == kPolygon) {
        ct.pair_tests++;
        if constexpr (PREC == 1) {
            const int d = P.regular ? polygon_overlap32_regular<NV>(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1])
                                    : polygon_overlap32<NV>(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1]);
            if (d != kUncertain) return d == kOverlap;
        }
        ct.pair_fp64++;
        return polygon_overlap64<NV>(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1]);
    } else {
        ct.pair_tests++;
        if constexpr (PREC == 1) {
            const int d = polyhedron_overlap_mixed(P, V3{r[0], r[1], r[2]}, Quat{qi[0], qi[1], qi[2], qi[3]},
                                                   Quat{qk[0], qk[1], qk[2], qk[3]});
            ct.pair_fp64 += (uint32_t)(d >> 1);
            return (d & 1) != 0;
        }
        ct.pair_fp64++;
        return polyhedron_overlap64(P, V3{r[0], r[1], r[2]}, Quat{qi[0], qi[1], qi[2], qi[3]},
                                    Quat{qk[0], qk[1], qk[2], qk[3]});
    }
}

__device__ __forceinline__ void grid_shift(const SysDev& S, uint32_t t, uint32_t k0, uint32_t k1,
                                           int shifted, double (&sh)[3]) {
    sh[0] = sh[1] = sh[2] = 0.0;
    if (shifted) {
        const uint4 w = draw(t, kShift, 0u, 0u, (uint32_t)S.replica, k0, k1);
        sh[0] = S.w * u01(w.x);
        sh[1] = S.w * u01(w.y);
        sh[2] = S.w * u01(w.z);
    }
}

template <int D, class POS>
__device__ __forceinline__ void particle_grid(const SysDev& S, const POS& pos, uint32_t i,
                                              const double (&sh)[3], double (&y)[3]) {
    y[2] = 0.0;
#pragma unroll
    for (int a = 0; a < D; ++a) y[a] = grid_coord(pos.get(a, i), sh[a], S.L);
}

template <int D>
__device__ __forceinline__ uint32_t cell_of_grid(const SysDev& S, const double (&y)[3]) {
    const int n = S.n;
    const int cx = cell_of_coord(y[0], S.inv_w, n);
    const int cy = cell_of_coord(y[1], S.inv_w, n);
    const int cz = D == 3 ? cell_of_coord(y[2], S.inv_w, n) : 0;
    return (uint32_t)(cx + n * (cy + n * cz));
}

template <int D, class POS>
__device__ __forceinline__ uint32_t particle_cell(const SysDev& S, const POS& pos, uint32_t i,
                                                  const double (&sh)[3]) {
    double y[3];
    particle_grid<D>(S, pos, i, sh, y);
    return cell_of_grid<D>(S, y);
}

// floor(a / m) for 0 <= a < 2^30 through a binary64 reciprocal (within one
// of the quotient, then corrected): cheaper than an integer division.
__device__ __forceinline__ int div_floor(int a, int m, double inv_m) {
    int q = (int)((double)a * inv_m);
    q -= q * m > a ? 1 : 0;
    q += (q + 1) * m <= a ? 1 : 0;
    return q;
}

// Cell of active index a in colour `colour`: the active cells of a colour
// are every other cell along each axis, offset by the colour's bits.  The
// index runs fastest along x, or along y when Y_FIRST (consecutive lanes then
// share an x column, so few waves hold a cell at the periodic x edge).
template <bool Y_FIRST = false>
__device__ __forceinline__ void active_cell(const SysDev& S, int D, uint32_t colour, int a,
                                            double inv_half, int (&cc)[3], uint32_t& c) {
    const int half = S.n / 2;
    const int q1 = div_floor(a, half, inv_half);
    const int q2 = D == 3 ? div_floor(q1, half, inv_half) : 0;
    const int fast = a - q1 * half, mid = q1 - q2 * half;
    cc[0] = 2 * (Y_FIRST ? mid : fast) + (int)(colour & 1u);
    cc[1] = 2 * (Y_FIRST ? fast : mid) + (int)((colour >> 1) & 1u);
    cc[2] = D == 3 ? 2 * q2 + (int)((colour >> 2) & 1u) : 0;
    c = (uint32_t)(cc[0] + S.n * (cc[1] + S.n * cc[2]));
}

__device__ __forceinline__ int wrap_cell(int x, int n) {
    x += x < 0 ? n : 0;
    return x - (x >= n ? n : 0);
}

// Linear index of neighbour j (0 .. 3^dim - 1) of cell cc.
template <int D>
__device__ __forceinline__ uint32_t neighbour_cell(const int (&cc)[3], int j, int n) {
    const int x = wrap_cell(cc[0] + (j % 3) - 1, n);
    const int y = wrap_cell(cc[1] + ((j / 3) % 3) - 1, n);
    const int z = D == 3 ? wrap_cell(cc[2] + (j / 9) - 1, n) : 0;
    return (uint32_t)(x + n * (y + n * z));
}

// The 3^dim neighbour cells of cell cc, as member ranges of the cell-sorted
// list: the three cells of a neighbour row (fixed y, z) are consecutive in
// the linear cell index, so each row is one contiguous range -- except at the
// periodic edge, where the wrapped cell is a second range.  Range ri:
// row ri / 2 (dy = row % 3 - 1, dz = row / 3 - 1), segment ri % 2 (0: main,
// 1: wrapped cell or empty).  ref is the trial point in the frame of the
// range's periodic image: a neighbour across the edge at 0 holds coordinates
// near L, so its separation is y_k - (y_n + L), and the other way round.
template <int D>
struct Neighbourhood {
    static constexpr int ranges = D == 3 ? 18 : 6;
};

// Neighbour slot range ri of cell cc for the pre-filter, with the reference
// point (the trial position, shifted by +-L where the range wraps).  Plain
// lists: per row an in-row range (ri even) and the x-wrapped cell (ri odd,
// empty unless cc sits at an x edge).  Ghost lists (2D): one range per row.
template <int D, class CELLS>
__device__ __forceinline__ void neighbour_range(const CELLS& cl, const int (&cc)[3], int n, int ri,
                                                double L, const double (&yn)[3], uint32_t& b,
                                                uint32_t& e, float (&ref)[3]) {
    if constexpr (CELLS::ghost) {
        static_assert(D == 2, "ghost edge columns are a 2D layout");
        const int yy = cc[1] + ri - 1;
        const int y = wrap_cell(yy, n);
        ref[0] = (float)yn[0];
        ref[1] = (float)(yy < 0 ? yn[1] + L : (yy >= n ? yn[1] - L : yn[1]));
        ref[2] = 0.0f;
        const uint32_t base = (uint32_t)((n + 2) * y + cc[0]);  // storage index of x - 1
        b = cl.begin(base);
        e = cl.end(base + 2u);
        return;
    }
    const int row = ri >> 1;
    const int yy = cc[1] + (row % 3) - 1;
    const int zz = D == 3 ? cc[2] + (row / 3) - 1 : 0;
    const int y = wrap_cell(yy, n);
    const int z = D == 3 ? wrap_cell(zz, n) : 0;
    ref[1] = (float)(yy < 0 ? yn[1] + L : (yy >= n ? yn[1] - L : yn[1]));
    ref[2] = D == 3 ? (float)(zz < 0 ? yn[2] + L : (zz >= n ? yn[2] - L : yn[2])) : 0.0f;
    const int base = n * (y + n * z);
    int x0, x1;
    if ((ri & 1) == 0) {
        x0 = cc[0] > 0 ? cc[0] - 1 : 0;
        x1 = cc[0] < n - 1 ? cc[0] + 1 : n - 1;
        ref[0] = (float)yn[0];
    } else if (cc[0] == 0) {
        x0 = x1 = n - 1;
        ref[0] = (float)(yn[0] + L);
    } else if (cc[0] == n - 1) {
        x0 = x1 = 0;
        ref[0] = (float)(yn[0] - L);
    } else {
        b = e = 0;
        ref[0] = 0.0f;
        return;
    }
    b = cl.begin((uint32_t)(base + x0));
    e = cl.end((uint32_t)(base + x1));
}

// Candidates a lane of the wave-queue scan loads at once from a cell list in
// global memory (a 3D neighbour range holds about three times as many as a
// 2D one); one from LDS, whose latency is short.  Scans of a global list
// also queue the member tag with each hit, so the drain needs no lookup.
template <int D, bool GLOBAL>
constexpr int kScanUnroll = GLOBAL ? (D == 3 ? 4 : 2) : 1;
template <class CELLS>
constexpr bool kGlobalList = std::is_same<CELLS, GlobalCells>::value;

// Per-wave LDS scratch: one flag per group (cell) of the tile, a 128-entry
// ring of queued pair tests, and a second ring for the two-stage binary64
// polygon drain.
struct WaveScratch {
    uint32_t* flag;  // 64 entries
    uint32_t* q;     // 128 entries: owner lane << 26 | neighbour tag (global cell
                     // list) or slot (LDS cell list)
    uint32_t* q2;    // 128 entries: polygon pairs left after their first half of axes
};
constexpr int kQueueWords = 128;
constexpr int kFlagWords = 64;
constexpr int kWaveScratchWords = 2 * kQueueWords + kFlagWords;
// Words a wave needs: the second ring only for binary64 polygons.
__host__ __device__ constexpr int wave_scratch_words(int kind, int prec) {
    return kind == kPolygon && prec == 0 ? kWaveScratchWords : kFlagWords + kQueueWords;
}
__device__ __forceinline__ WaveScratch wave_scratch(uint32_t* base) {
    return WaveScratch{base, base + kFlagWords, base + kFlagWords + kQueueWords};
}
constexpr uint32_t kTagMask = (1u << 26) - 1u;

// How a pass hands the full overlap tests to lanes: the per-wave LDS queue
// (the paper's block queue), or the register queue it improves on.
enum QueueKind : int { kWaveQueue = 0, kRegisterQueue = 1 };

// ---------------------------------------------------------------------------
// Drain n (<= 64) queued pair tests: lane L takes entry L, fetches the owner
// cell's trial state from the owner lane, runs the binary64 circumsphere test
// (the pre-filter only narrows the candidates) and then the full test.  All
// lanes must call (contains cross-lane shuffles).
// ---------------------------------------------------------------------------
template <int KIND, int PREC, int G, int NV, class POS, class CELLS>
__device__ __forceinline__ void drain(const SysDev& S, const SpeciesDev& P, const POS& pos,
                                      const double* __restrict__ ori, const CELLS& cl,
                                      const double (&xn)[3], const double (&qn)[4], uint32_t n,
                                      WaveScratch ws, Counters& ct) {
    constexpr int D = Traits<KIND>::dim;
    const uint32_t lane = __lane_id();
    wave_sync();
    const uint32_t e = lane < n ? ws.q[lane] : 0u;
    const int owner = lane < n ? (int)(e >> 26) : (int)lane;
    double tx[3], tq[4];
#pragma unroll
    for (int a = 0; a < 3; ++a) tx[a] = a < D ? __shfl(xn[a], owner, 64) : 0.0;
#pragma unroll
    for (int c = 0; c < 4; ++c) tq[c] = c < Traits<KIND>::ncomp ? __shfl(qn[c], owner, 64) : qn[c];
    if (lane < n && ws.flag[owner / G] == 0u) {
        const uint32_t k = kGlobalList<CELLS> ? e & kTagMask : cl.member(e & kTagMask);
        // the neighbour's orientation is loaded with its position (one
        // memory latency for both), before the circumsphere test needs it
        double qk[4];
        load_orient<KIND>(ori, S.N, k, qk);
        double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < D; ++a) r[a] = min_image(pos.get(a, k) - tx[a], S.L, S.inv_L);
        double r2 = r[0] * r[0] + r[1] * r[1];
        if constexpr (D == 3) r2 = r2 + r[2] * r[2];
        if (r2 < P.circ2) {
            if (full_test<KIND, PREC, NV>(P, r, tq, qk, ct)) ws.flag[owner / G] = 1u;
        }
    }
    wave_sync();
}

// Binary64 polygons drain in two stages so that a drain's lanes run similar
// work (the binary32 filter's halves are too cheap to pay for the second
// queue, so the mixed path keeps one stage):
// stage 1 runs the binary64 circumsphere test and the first half of the
// separating axes (A's normals); pairs that half cannot separate go to a
// second queue, whose drain runs the other half (B's normals).  The result
// is the OR over both halves, as in the one-stage test.  Stage 1 returns the
// new length of the second queue.  All lanes must call.
template <int PREC, int G, int NV, class POS, class CELLS>
__device__ __forceinline__ uint32_t drain_polygon1(const SysDev& S, const SpeciesDev& P, const POS& pos,
                                                   const double* __restrict__ ori, const CELLS& cl,
                                                   const double (&xn)[3], const double (&qn)[4],
                                                   uint32_t n, WaveScratch ws, uint32_t queued2,
                                                   Counters& ct) {
    const uint32_t lane = __lane_id();
    wave_sync();
    const uint32_t e = lane < n ? ws.q[lane] : 0u;
    const int owner = lane < n ? (int)(e >> 26) : (int)lane;
    const double tx = __shfl(xn[0], owner, 64), ty = __shfl(xn[1], owner, 64);
    const double tc = __shfl(qn[0], owner, 64), ts = __shfl(qn[1], owner, 64);
    bool push = false;
    if (lane < n && ws.flag[owner / G] == 0u) {
        const uint32_t k = kGlobalList<CELLS> ? e & kTagMask : cl.member(e & kTagMask);
        const double rx = min_image(pos.get(0, k) - tx, S.L, S.inv_L);
        const double ry = min_image(pos.get(1, k) - ty, S.L, S.inv_L);
        if (rx * rx + ry * ry < P.circ2) {
            ct.pair_tests++;
            const double kc = ori[k], ks = ori[S.N + k];
            if constexpr (PREC == 1) {
                const int h = polygon_half32<NV, 0>(P, rx, ry, tc, ts, kc, ks);
                if (h == kHalfUnsure) {
                    ct.pair_fp64++;
                    if (polygon_overlap64<NV>(P, rx, ry, tc, ts, kc, ks)) ws.flag[owner / G] = 1u;
                }
                push = h == kHalfOverlaps;
            } else {
                ct.pair_fp64++;
                push = !polygon_half_separated64<NV, 0>(P, rx, ry, tc, ts, kc, ks);
            }
        }
    }
    const uint64_t pm = wave_ballot(push);
    if (push) ws.q2[queued2 + lanes_below(pm)] = e;
    wave_sync();
    return queued2 + (uint32_t)__builtin_popcountll(pm);
}

template <int PREC, int G, int NV, class POS, class CELLS>
__device__ __forceinline__ void drain_polygon2(const SysDev& S, const SpeciesDev& P, const POS& pos,
                                               const double* __restrict__ ori, const CELLS& cl,
                                               const double (&xn)[3], const double (&qn)[4], uint32_t n,
                                               WaveScratch ws, Counters& ct) {
    const uint32_t lane = __lane_id();
    wave_sync();
    const uint32_t e = lane < n ? ws.q2[lane] : 0u;
    const int owner = lane < n ? (int)(e >> 26) : (int)lane;
    const double tx = __shfl(xn[0], owner, 64), ty = __shfl(xn[1], owner, 64);
    const double tc = __shfl(qn[0], owner, 64), ts = __shfl(qn[1], owner, 64);
    if (lane < n && ws.flag[owner / G] == 0u) {
        const uint32_t k = kGlobalList<CELLS> ? e & kTagMask : cl.member(e & kTagMask);
        const double rx = min_image(pos.get(0, k) - tx, S.L, S.inv_L);
        const double ry = min_image(pos.get(1, k) - ty, S.L, S.inv_L);
        const double kc = ori[k], ks = ori[S.N + k];
        bool overlap;
        if constexpr (PREC == 1) {
            const int h = polygon_half32<NV, 1>(P, rx, ry, tc, ts, kc, ks);
            if (h == kHalfUnsure) {
                ct.pair_fp64++;
                overlap = polygon_overlap64<NV>(P, rx, ry, tc, ts, kc, ks);
            } else {
                overlap = h == kHalfOverlaps;
            }
        } else {
            overlap = !polygon_half_separated64<NV, 1>(P, rx, ry, tc, ts, kc, ks);
        }
        if (overlap) ws.flag[owner / G] = 1u;
    }
    wave_sync();
}

// Keep queue entries [from, from + count) as entries [0, count).
__device__ __forceinline__ void compact_queue(uint32_t* q, uint32_t from, uint32_t count) {
    const uint32_t lane = __lane_id();
    const uint32_t v = lane < count ? q[from + lane] : 0u;
    wave_sync();
    if (lane < count) q[lane] = v;
    wave_sync();
}

// Trial move of active cell a (index within its colour): uniform occupant
// (Philox SELECT keyed on the cell), translation or rotation (Philox MOVE
// keyed on the tag), periodic wrap, and the rule that a translation must
// stay in the cell.  Sets live when the cell is non-empty and the trial
// stays in it.  YF: active cells indexed y first (2D).
template <int KIND, bool YF = false, class POS, class CELLS>
__device__ __forceinline__ void propose(const SysDev& S, const SpeciesDev& P, const POS& pos,
                                        const double* __restrict__ ori, const CELLS& cl,
                                        uint32_t colour, uint32_t select, uint32_t t, uint32_t k0,
                                        uint32_t k1, const double (&sh)[3], int a, int (&cc)[3],
                                        uint32_t& c, uint32_t& i, uint32_t& pi, bool& live,
                                        double (&xn)[3], double (&qn)[4], bool& c_rot,
                                        bool& c_moved, Counters& ct) {
    constexpr int D = Traits<KIND>::dim;
    const int n = S.n;
    active_cell<YF && D == 2>(S, D, colour, a, 1.0 / (double)(n / 2), cc, c);
    const uint32_t ci = cl.index(cc, c, n);  // storage index (c unless ghost columns)
    const uint32_t beg = cl.begin(ci), fin = cl.end(ci);
    if (beg != fin) {
        ct.attempted++;
        const uint4 wsel = draw(t, kSelect, select, c, S.replica, k0, k1);
        pi = beg + index_below(wsel.x, fin - beg);
        i = cl.member(pi);
        const uint4 m = draw(t, kMove, select, i, S.replica, k0, k1);
#pragma unroll
        for (int ax = 0; ax < D; ++ax) xn[ax] = pos.get(ax, i);
        load_orient<KIND>(ori, S.N, i, qn);
        const bool rotate = KIND != kDisk && P.p_rot > 0.0 && u01(m.x) < P.p_rot;
        live = true;
        c_rot = rotate;
        c_moved = !rotate;
        if (!rotate) {
            const uint32_t mw[3] = {m.y, m.z, m.w};
#pragma unroll
            for (int ax = 0; ax < D; ++ax) {
                xn[ax] = wrap_periodic(xn[ax] + P.d * (2.0 * u01(mw[ax]) - 1.0), S.L);
                live &= cell_coord(xn[ax], sh[ax], S.L, S.inv_w, n) == cc[ax];
            }
        } else {
            if constexpr (kPlanarTurn<KIND>) {
                const double delta = P.a * (2.0 * u01(m.y) - 1.0);
                double cd, sd;
                small_angle_sincos(delta, cd, sd);
                const double c0 = qn[0], s0 = qn[1];
                qn[0] = c0 * cd - s0 * sd;
                qn[1] = s0 * cd + c0 * sd;
            } else if constexpr (KIND == kPolyhedron) {
                const Quat dq{1.0, P.a * (2.0 * u01(m.y) - 1.0), P.a * (2.0 * u01(m.z) - 1.0),
                              P.a * (2.0 * u01(m.w) - 1.0)};
                const Quat p = qmul(Quat{qn[0], qn[1], qn[2], qn[3]}, dq);
                const double nrm = sqrt(((p.w * p.w + p.x * p.x) + p.y * p.y) + p.z * p.z);
                qn[0] = p.w / nrm;
                qn[1] = p.x / nrm;
                qn[2] = p.y / nrm;
                qn[3] = p.z / nrm;
            }
        }
    }
}

// One wave's share of a colour pass: active cells a0 + lane / G below a_end
// (at most 64 / G of them).
// PARK: the sorted copy is in LDS and the moving particle's slot is parked
// at infinity during its own scan (else the scan tests the slot).
// YF: active cells indexed y first (work-groups with their state in LDS).
template <int KIND, int PREC, int G, int NV, bool PARK, int Q = kWaveQueue, bool YF = PARK,
          class POS, class CELLS, class XSV>
__device__ __forceinline__ void pass_tile(const SysDev& S, const SpeciesDev& P, const POS& pos,
                                          double* __restrict__ ori, const CELLS& cl,
                                          const XSV& xs, uint32_t colour,
                                          uint32_t select, uint32_t t, uint32_t k0, uint32_t k1,
                                          const double (&sh)[3], int a0, int a_end, WaveScratch ws,
                                          Counters& ct, PhaseClock& pc) {
    constexpr int D = Traits<KIND>::dim;
    pc.mark<kPhOther>();
    const int lane = (int)__lane_id();
    const int grp = lane / G, sub = lane % G;
    const int leader = grp * G;
    const int a = a0 + grp;
    const int n = S.n, N = S.N;

    // ---- 1. propose (group leaders)
    int cc[3] = {0, 0, 0};
    uint32_t c = 0, i = 0, pi = 0;  // active cell, moving tag, its slot in the cell list
    bool live = false;
    double xn[3] = {0.0, 0.0, 0.0};
    double qn[4] = {1.0, 0.0, 0.0, 0.0};
    bool c_rot = false, c_moved = false;  // rotation attempted / translation attempted
    // LDS-resident 2D tiles (YF) index y first: data locality does not matter
    // there, and most waves then skip the x-wrapped ranges (in 3D a wave
    // spans several x columns, so nearly every wave holds an edge)
    if (sub == 0 && a < a_end)
        propose<KIND, YF>(S, P, pos, ori, cl, colour, select, t, k0, k1, sh, a, cc, c, i, pi, live, xn, qn,
                          c_rot, c_moved, ct);
    ct.attempted_rot += (sub == 0 && a < a_end && c_rot) ? 1u : 0u;
    ct.cell_reject += (sub == 0 && a < a_end && c_moved && !live) ? 1u : 0u;
    // the moving particle's own slot is parked at infinity for the scan (no
    // candidate is closer), so the loop needs no self test
    float own[3] = {0.0f, 0.0f, 0.0f};
    if (PARK && sub == 0 && live) {
        xs.load(pi, own);
        const float far[3] = {INFINITY, INFINITY, INFINITY};
        xs.store(pi, far);
    }
    if (lane < 64 / G) ws.flag[lane] = 0u;
    if constexpr (G > 1) {
        live = __shfl((int)live, leader, 64) != 0;
        if constexpr (!PARK) pi = (uint32_t)__shfl((int)pi, leader, 64);
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            cc[ax] = __shfl(cc[ax], leader, 64);
            if (ax < D) xn[ax] = __shfl(xn[ax], leader, 64);
        }
    }
    double yn[3] = {0.0, 0.0, 0.0};  // trial point in the shifted frame
#pragma unroll
    for (int ax = 0; ax < D; ++ax) yn[ax] = grid_coord(xn[ax], sh[ax], S.L);
    wave_sync();
    pc.mark<kPhPropose>();

    if constexpr (Q == kWaveQueue) {
        // ---- 2 + 3. binary32 circumsphere pre-filter over the neighbour ranges
        // (lane `sub` of a group takes ranges sub, sub + G, ...), queued exact
        // tests.  The outer loop over ranges is uniform; each inner loop runs to
        // the longest range of the wave.
        constexpr int NR = CELLS::ghost ? 3 : Neighbourhood<D>::ranges;
        constexpr int NK = (NR + G - 1) / G;
        constexpr bool TAGQ = kGlobalList<CELLS>;
        constexpr int U = kScanUnroll<D, TAGQ>;
        const float t2 = S.scan_t2;
        // queue depth: a drain starts once this many tests wait (at most 64,
        // so at most 127 entries are ever queued)
        const uint32_t drain_at = S.drain_at;
        bool flagged = false;  // this lane's cell already has an overlap (register copy)
        uint32_t queued = 0;   // wave-uniform
        uint32_t queued2 = 0;  // wave-uniform, polygons only
        // with one lane per cell, the x-wrapped (odd) ranges are empty unless a
        // live cell of the wave sits at the periodic x edge: skip them then
        const bool x_edge = G > 1 || CELLS::ghost || wave_ballot(live && (cc[0] == 0 || cc[0] == n - 1)) != 0ull;
        for (int kr = 0; kr < NK; ++kr) {
            if (G == 1 && !CELLS::ghost && (kr & 1) && !x_edge) continue;
            const int ri = sub + kr * G;
            uint32_t p = 0, e = 0;
            float ref[3] = {0.0f, 0.0f, 0.0f};
            if (live && !flagged && ri < NR) neighbour_range<D>(cl, cc, n, ri, S.L, yn, p, e, ref);
            for (;;) {
                if (wave_ballot(p < e) == 0ull) break;
                // U candidates per lane at a time: their loads are issued
                // together so that one memory latency covers them; each is
                // then tested and queued in slot order.  Each predicate is a
                // single compare so that its ballot is the compare's lane mask:
                // an idle lane's distance is infinite, a flagged lane's range
                // ends at the candidate where the flag was seen.
                uint32_t sl[U], tg[U];
                float v[U][3];
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    sl[u] = p + u < e ? p + u : 0u;  // idle lanes read slot 0 (always valid)
                    xs.load(sl[u], v[u]);
                    tg[u] = TAGQ ? cl.member(sl[u]) : sl[u];
                }
#pragma unroll
                for (int u = 0; u < U; ++u) {
                    const bool work = p + (uint32_t)u < e;
                    const float rx = v[u][0] - ref[0], ry = v[u][1] - ref[1];
                    float r2 = fmaf(ry, ry, rx * rx);
                    if constexpr (D == 3) {
                        const float rz = v[u][2] - ref[2];
                        r2 = fmaf(rz, rz, r2);
                    }
                    r2 = (work && (PARK || sl[u] != pi)) ? r2 : INFINITY;
                    const bool hit = r2 < t2;
                    const uint64_t hm = wave_ballot(hit);
                    if (hit) ws.q[queued + lanes_below(hm)] = ((uint32_t)leader << 26) | tg[u];  // tag or slot
                    queued += (uint32_t)__builtin_popcountll(hm);
                    if (queued >= drain_at) {
                        // up to one entry per lane; the rest stays queued
                        const uint32_t m = queued < 64u ? queued : 64u;
                        pc.mark<kPhScan>();
                        if constexpr (KIND == kPolygon && PREC == 0) {
                            queued2 = drain_polygon1<PREC, G, NV>(S, P, pos, ori, cl, xn, qn, m, ws, queued2, ct);
                        } else {
                            drain<KIND, PREC, G, NV>(S, P, pos, ori, cl, xn, qn, m, ws, ct);
                        }
                        queued -= m;
                        compact_queue(ws.q, m, queued);
                        if constexpr (KIND == kPolygon && PREC == 0) {
                            if (queued2 >= 64u) {
                                drain_polygon2<PREC, G, NV>(S, P, pos, ori, cl, xn, qn, 64u, ws, ct);
                                queued2 -= 64u;
                                compact_queue(ws.q2, 64u, queued2);
                            }
                        }
                        flagged = ws.flag[grp] != 0u;
                        const uint32_t stop = p + (uint32_t)u + 1u;
                        e = flagged && stop < e ? stop : e;
                        pc.mark<kPhDrain>();
                    }
                }
                p = p + (uint32_t)U < e ? p + (uint32_t)U : e;
            }
        }
        pc.mark<kPhScan>();
        if constexpr (KIND == kPolygon && PREC == 0) {
            if (queued) queued2 = drain_polygon1<PREC, G, NV>(S, P, pos, ori, cl, xn, qn, queued, ws, queued2, ct);
            while (queued2) {
                const uint32_t m = queued2 < 64u ? queued2 : 64u;
                drain_polygon2<PREC, G, NV>(S, P, pos, ori, cl, xn, qn, m, ws, ct);
                queued2 -= m;
                if (queued2) compact_queue(ws.q2, 64u, queued2);
            }
        } else {
            if (queued) drain<KIND, PREC, G, NV>(S, P, pos, ori, cl, xn, qn, queued, ws, ct);
        }
        pc.mark<kPhDrain>();
    } else {
        // ---- 2 + 3, register queue (the paper's first variant): each lane
        // runs the pre-filter over its ranges and stops at its first hit; the
        // wave then runs the full tests of all lanes that hold a hit, on the
        // lane's own trial state, and the scan resumes where it stopped.
        if constexpr (G > 1) {
#pragma unroll
            for (int c4 = 0; c4 < 4; ++c4) qn[c4] = __shfl(qn[c4], leader, 64);
        }
        constexpr int NR = CELLS::ghost ? 3 : Neighbourhood<D>::ranges;
        constexpr int NK = (NR + G - 1) / G;
        const float t2 = S.scan_t2;
        bool flagged = false;
        for (int kr = 0; kr < NK; ++kr) {
            const int ri = sub + kr * G;
            uint32_t p = 0, e = 0;
            float ref[3] = {0.0f, 0.0f, 0.0f};
            if (live && !flagged && ri < NR) neighbour_range<D>(cl, cc, n, ri, S.L, yn, p, e, ref);
            for (;;) {
                uint32_t hit = 0xffffffffu;
                while (p < e) {
                    const uint32_t slot = p++;
                    float v[3];
                    xs.load(slot, v);
                    const float rx = v[0] - ref[0], ry = v[1] - ref[1];
                    float r2 = fmaf(ry, ry, rx * rx);
                    if constexpr (D == 3) {
                        const float rz = v[2] - ref[2];
                        r2 = fmaf(rz, rz, r2);
                    }
                    if (r2 < t2 && (PARK || slot != pi)) {
                        hit = slot;
                        break;
                    }
                }
                const bool has = hit != 0xffffffffu;
                if (wave_ballot(has) == 0ull) break;
                if (has) {
                    const uint32_t k = cl.member(hit);
                    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) r[ax] = min_image(pos.get(ax, k) - xn[ax], S.L, S.inv_L);
                    double r2 = r[0] * r[0] + r[1] * r[1];
                    if constexpr (D == 3) r2 = r2 + r[2] * r[2];
                    if (r2 < P.circ2) {
                        double qk[4];
                        load_orient<KIND>(ori, S.N, k, qk);
                        if (full_test<KIND, PREC, NV>(P, r, qn, qk, ct)) ws.flag[grp] = 1u;
                    }
                }
                wave_sync();
                flagged = ws.flag[grp] != 0u;
                e = flagged ? p : e;
            }
        }
        pc.mark<kPhScan>();
    }

    // ---- 4. write back (counters updated arithmetically, not per branch)
    const bool rejected = live && ws.flag[grp] != 0u;
    ct.overlap_reject += (sub == 0 && rejected) ? 1u : 0u;
    ct.accept += (sub == 0 && live && !rejected) ? 1u : 0u;
    if (sub == 0 && live) {
        if (!rejected && c_moved) {
            xs.store(pi, yn);
            if constexpr (CELLS::ghost) {
                // the ghost copy of an edge-column particle follows it: same
                // offset in the copy of its cell, x shifted by +L (copy after
                // the row's last cell) or -L (before its first)
                if (cc[0] == 0 || cc[0] == n - 1) {
                    const uint32_t ci = cl.index(cc, c, n);
                    const uint32_t gi = cc[0] == 0 ? ci + (uint32_t)n : ci - (uint32_t)n;
                    const double gy[3] = {cc[0] == 0 ? yn[0] + S.L : yn[0] - S.L, yn[1], yn[2]};
                    xs.store(pi - cl.begin(ci) + cl.begin(gi), gy);
                }
            }
        } else if (PARK) {
            xs.store(pi, own);
        }
        // only what the move changed
        if (!rejected && c_moved) {
#pragma unroll
            for (int ax = 0; ax < D; ++ax) pos.set(ax, i, xn[ax]);
        }
        if (!rejected && c_rot) {
            if constexpr (kPlanarTurn<KIND>) {
                ori[i] = qn[0];
                ori[N + i] = qn[1];
            } else if constexpr (KIND == kPolyhedron) {
                ori[i] = qn[0];
                ori[N + i] = qn[1];
                ori[2 * N + i] = qn[2];
                ori[3 * N + i] = qn[3];
            }
        }
    }
    wave_sync();
    pc.mark<kPhWrite>();
}

}  // namespace hpmc
