// Kernels of the checkerboard sweep for gfx950 (wave64).
//
// Grid path (large systems): per sweep a counting sort builds the cell list
// of the shifted grid in global memory (assign + histogram, scan, scatter,
// per-cell ascending-tag order), then one kernel per colour pass makes one
// trial move in every non-empty active cell (Sec. 2.5.2).
//
// Persistent path (small systems, batches of replicas): one work-group owns a
// replica and runs whole sweeps; its cell list lives in LDS and the colour
// passes are separated by work-group barriers, so no grid-wide
// synchronisation is needed.
#include "device_common.hpp"
#include "launch.hpp"
#include "overlap32.hpp"
#include "overlap64.hpp"

namespace hpmc {

template <int KIND>
struct Traits {
    static constexpr int dim = KIND == kPolyhedron ? 3 : 2;
    static constexpr int ncomp = KIND == kDisk ? 0 : (KIND == kPolygon ? 2 : 4);
};

struct Counters {
    uint32_t v[kNumStats];
};

// One 64-bit atomic per wave and counter.  Every lane of the wave must call.
__device__ __forceinline__ void flush(const Counters& c, unsigned long long* stats) {
#pragma unroll
    for (int k = 0; k < kNumStats; ++k) {
        const uint32_t s = wave_sum(c.v[k]);
        if (__lane_id() == 0 && s != 0) atomicAdd(stats + k, (unsigned long long)s);
    }
}

// ---------------------------------------------------------------------------
// Cell-list views: global (start[ncells + 1], members u32) and LDS
// (inclusive ends[ncells], members u16).
// ---------------------------------------------------------------------------
struct GlobalCells {
    const uint32_t* __restrict__ start;
    const uint32_t* __restrict__ members;
    __device__ __forceinline__ uint32_t begin(uint32_t c) const { return start[c]; }
    __device__ __forceinline__ uint32_t end(uint32_t c) const { return start[c + 1]; }
    __device__ __forceinline__ uint32_t member(uint32_t p) const { return members[p]; }
};

struct LdsCells {
    const uint32_t* ends;
    const uint16_t* members;
    __device__ __forceinline__ uint32_t begin(uint32_t c) const { return c ? ends[c - 1] : 0u; }
    __device__ __forceinline__ uint32_t end(uint32_t c) const { return ends[c]; }
    __device__ __forceinline__ uint32_t member(uint32_t p) const { return members[p]; }
};

template <int KIND>
__device__ __forceinline__ void load_orient(const double* __restrict__ ori, int N, uint32_t i,
                                            double (&q)[4]) {
    q[0] = 1.0;
    q[1] = q[2] = q[3] = 0.0;
    if constexpr (KIND == kPolygon) {
        q[0] = ori[i];
        q[1] = ori[N + i];
    } else if constexpr (KIND == kPolyhedron) {
        q[0] = ori[i];
        q[1] = ori[N + i];
        q[2] = ori[2 * N + i];
        q[3] = ori[3 * N + i];
    }
}

// Full overlap test of a pair that passed the circumsphere test; for disks
// that test is the whole predicate.
template <int KIND, int PREC>
__device__ __forceinline__ bool full_test(const SpeciesDev& P, const double (&r)[3],
                                          const double (&qi)[4], const double (&qk)[4],
                                          Counters& ct) {
    if constexpr (KIND == kDisk) {
        return true;
    } else if constexpr (KIND == kPolygon) {
        ct.v[kPairTests]++;
        if constexpr (PREC == 1) {
            const int d = polygon_overlap32(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1]);
            if (d != kUncertain) return d == kOverlap;
        }
        ct.v[kPairFp64]++;
        return polygon_overlap64(P, r[0], r[1], qi[0], qi[1], qk[0], qk[1]);
    } else {
        ct.v[kPairTests]++;
        ct.v[kPairFp64]++;
        return polyhedron_overlap64(P, V3{r[0], r[1], r[2]}, Quat{qi[0], qi[1], qi[2], qi[3]},
                                    Quat{qk[0], qk[1], qk[2], qk[3]});
    }
}

// ---------------------------------------------------------------------------
// One trial move in cell c (coordinates cc) of the grid shifted by sh:
// uniform occupant, Philox move stream keyed on its tag, translation or
// rotation, reject if it leaves the cell, reject on the first overlap with
// an occupant of the 3^dim cells around c, otherwise write back (Sec. 2.1,
// Sec. 2.5.2).
// ---------------------------------------------------------------------------
template <int KIND, int PREC, class CL>
__device__ __forceinline__ void trial_move(const SysDev& S, const SpeciesDev& P,
                                           double* __restrict__ pos, double* __restrict__ ori,
                                           const CL& cl, uint32_t c, const int (&cc)[3],
                                           uint32_t select, uint32_t t, uint32_t k0, uint32_t k1,
                                           const double (&sh)[3], Counters& ct) {
    constexpr int D = Traits<KIND>::dim;
    const uint32_t beg = cl.begin(c), fin = cl.end(c);
    if (beg == fin) return;
    ct.v[kAttempted]++;
    const uint4 ws = draw(t, kSelect, select, c, S.replica, k0, k1);
    const uint32_t i = cl.member(beg + index_below(ws.x, fin - beg));
    const uint4 m = draw(t, kMove, select, i, S.replica, k0, k1);
    const int N = S.N;

    double xn[3] = {0.0, 0.0, 0.0};
#pragma unroll
    for (int a = 0; a < D; ++a) xn[a] = pos[a * N + i];
    double qn[4];
    load_orient<KIND>(ori, N, i, qn);

    const bool rotate = KIND != kDisk && P.p_rot > 0.0 && u01(m.x) < P.p_rot;
    if (!rotate) {
        const uint32_t mw[3] = {m.y, m.z, m.w};
        bool leaves = false;
#pragma unroll
        for (int a = 0; a < D; ++a) {
            xn[a] = wrap_periodic(xn[a] + P.d * (2.0 * u01(mw[a]) - 1.0), S.L);
            leaves |= cell_coord(xn[a], sh[a], S.L, S.inv_w, S.n) != cc[a];
        }
        if (leaves) {
            ct.v[kCellReject]++;
            return;
        }
    } else {
        ct.v[kAttemptedRot]++;
        if constexpr (KIND == kPolygon) {
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

    const int n = S.n;
    bool hit = false;
    constexpr int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
    for (int oz = zlo; oz <= zhi && !hit; ++oz) {
        int z = cc[2] + oz;
        z += z < 0 ? n : 0;
        z -= z >= n ? n : 0;
        for (int oy = -1; oy <= 1 && !hit; ++oy) {
            int y = cc[1] + oy;
            y += y < 0 ? n : 0;
            y -= y >= n ? n : 0;
            for (int ox = -1; ox <= 1 && !hit; ++ox) {
                int x = cc[0] + ox;
                x += x < 0 ? n : 0;
                x -= x >= n ? n : 0;
                const uint32_t cn = (uint32_t)(x + n * (y + n * z));
                const uint32_t e = cl.end(cn);
                for (uint32_t p = cl.begin(cn); p < e; ++p) {
                    const uint32_t k = cl.member(p);
                    if (k == i) continue;
                    double r[3] = {0.0, 0.0, 0.0};
#pragma unroll
                    for (int a = 0; a < D; ++a) r[a] = min_image(pos[a * N + k] - xn[a], S.L, S.inv_L);
                    double r2 = r[0] * r[0] + r[1] * r[1];
                    if constexpr (D == 3) r2 = r2 + r[2] * r[2];
                    if (!(r2 < P.circ2)) continue;
                    double qk[4];
                    load_orient<KIND>(ori, N, k, qk);
                    if (full_test<KIND, PREC>(P, r, qn, qk, ct)) {
                        hit = true;
                        break;
                    }
                }
            }
        }
    }
    if (hit) {
        ct.v[kOverlapReject]++;
        return;
    }
#pragma unroll
    for (int a = 0; a < D; ++a) pos[a * N + i] = xn[a];
    if constexpr (KIND == kPolygon) {
        ori[i] = qn[0];
        ori[N + i] = qn[1];
    } else if constexpr (KIND == kPolyhedron) {
        ori[i] = qn[0];
        ori[N + i] = qn[1];
        ori[2 * N + i] = qn[2];
        ori[3 * N + i] = qn[3];
    }
    ct.v[kAccept]++;
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

template <int D>
__device__ __forceinline__ uint32_t particle_cell(const SysDev& S, const double* __restrict__ pos,
                                                  int i, const double (&sh)[3]) {
    const int N = S.N, n = S.n;
    const int cx = cell_coord(pos[i], sh[0], S.L, S.inv_w, n);
    const int cy = cell_coord(pos[N + i], sh[1], S.L, S.inv_w, n);
    int cz = 0;
    if constexpr (D == 3) cz = cell_coord(pos[2 * N + i], sh[2], S.L, S.inv_w, n);
    return (uint32_t)(cx + n * (cy + n * cz));
}

__device__ __forceinline__ void active_cell(const SysDev& S, int D, uint32_t colour, int a,
                                            int (&cc)[3], uint32_t& c) {
    const int half = S.n / 2;
    cc[0] = 2 * (a % half) + (int)(colour & 1u);
    cc[1] = 2 * ((a / half) % half) + (int)((colour >> 1) & 1u);
    cc[2] = D == 3 ? 2 * (a / (half * half)) + (int)((colour >> 2) & 1u) : 0;
    c = (uint32_t)(cc[0] + S.n * (cc[1] + S.n * cc[2]));
}

// ---------------------------------------------------------------------------
// Work-group scans (blockDim.x a multiple of 64, at most 1024).
// ---------------------------------------------------------------------------
__device__ __forceinline__ uint32_t wave_inclusive_scan(uint32_t v) {
    const int lane = __lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(v, d, 64);
        if (lane >= d) v += y;
    }
    return v;
}

// Exclusive prefix of v over the work-group; total of all v in *total.
// sm must hold 16 words.  Contains barriers: all threads must call.
__device__ __forceinline__ uint32_t block_exclusive_scan(uint32_t v, uint32_t* sm, uint32_t& total) {
    const int lane = __lane_id(), wave = threadIdx.x >> 6, nwaves = blockDim.x >> 6;
    const uint32_t inc = wave_inclusive_scan(v);
    __syncthreads();
    if (lane == 63) sm[wave] = inc;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < nwaves; ++w) {
        const uint32_t s = sm[w];
        before += w < wave ? s : 0u;
        tot += s;
    }
    total = tot;
    return before + inc - v;
}

// ---------------------------------------------------------------------------
// Grid path: global cell list.
// ---------------------------------------------------------------------------
__global__ void k_fill_u32(uint32_t* __restrict__ p, uint32_t v, int n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_u64(unsigned long long* __restrict__ p, unsigned long long v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <int D>
__global__ void __launch_bounds__(256) k_assign(const SysDev* __restrict__ sys, int r,
                                                const double* __restrict__ pos_base, uint32_t t,
                                                uint32_t k0, uint32_t k1, int shifted,
                                                uint32_t* __restrict__ count,
                                                uint32_t* __restrict__ cell_of,
                                                uint32_t* __restrict__ slot_of) {
    const SysDev S = sys[r];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    double sh[3];
    grid_shift(S, t, k0, k1, shifted, sh);
    const uint32_t c = particle_cell<D>(S, pos_base + S.pos_off, i, sh);
    cell_of[i] = c;
    slot_of[i] = atomicAdd(count + c, 1u);
}

// Counts particles of replica r with a coordinate outside [0, L) or a
// non-finite orientation component (rejected by hpmc_init).
template <int NCOMP>
__global__ void __launch_bounds__(256) k_validate(const SysDev* __restrict__ sys, int r,
                                                  const double* __restrict__ pos_base,
                                                  const double* __restrict__ ori_base,
                                                  unsigned long long* __restrict__ out) {
    const SysDev S = sys[r];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t bad = 0;
    if (i < S.N) {
        const double* pos = pos_base + S.pos_off;
        for (int a = 0; a < S.dim; ++a) {
            const double x = pos[a * S.N + i];
            bad |= !(x >= 0.0 && x < S.L) ? 1u : 0u;
        }
        const double* ori = ori_base + S.orient_off;
        for (int k = 0; k < NCOMP; ++k) bad |= !isfinite(ori[k * S.N + i]) ? 1u : 0u;
    }
    const uint32_t s = wave_sum(bad);
    if (__lane_id() == 0 && s) atomicAdd(out + r, (unsigned long long)s);
}

// Tile sums of the cell histogram (kScanTile cells per 256-lane work-group).
__global__ void __launch_bounds__(256) k_scan_tiles(const uint32_t* __restrict__ count, int nc,
                                                    uint32_t* __restrict__ partial) {
    __shared__ uint32_t sm[16];
    const int base = blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += base + j < nc ? count[base + j] : 0u;
    uint32_t total;
    block_exclusive_scan(s, sm, total);
    if (threadIdx.x == 0) partial[blockIdx.x] = total;
}

// Exclusive scan of the tile sums in place (one work-group).
__global__ void __launch_bounds__(256) k_scan_partials(uint32_t* __restrict__ partial, int ntiles) {
    __shared__ uint32_t sm[16];
    uint32_t carry = 0;
    for (int base = 0; base < ntiles; base += blockDim.x) {
        const int j = base + threadIdx.x;
        const uint32_t v = j < ntiles ? partial[j] : 0u;
        uint32_t total;
        const uint32_t ex = block_exclusive_scan(v, sm, total);
        if (j < ntiles) partial[j] = carry + ex;
        carry += total;
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_scan_apply(const uint32_t* __restrict__ count, int nc,
                                                    const uint32_t* __restrict__ partial,
                                                    uint32_t* __restrict__ start, uint32_t N) {
    __shared__ uint32_t sm[16];
    const int base = blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = base + j < nc ? count[base + j] : 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sm, total) + partial[blockIdx.x];
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (base + j < nc) start[base + j] = run;
        run += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) start[nc] = N;
}

__global__ void __launch_bounds__(256) k_scatter(const uint32_t* __restrict__ cell_of,
                                                 const uint32_t* __restrict__ slot_of,
                                                 const uint32_t* __restrict__ start,
                                                 uint32_t* __restrict__ members, int N) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) members[start[cell_of[i]] + slot_of[i]] = (uint32_t)i;
}

// Occupants of each cell in ascending tag order (atomics scatter them in
// arbitrary order; cells hold a handful, so insertion sort).
__global__ void __launch_bounds__(256) k_sort_cells(const uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ members, int nc) {
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= nc) return;
    const uint32_t b = start[c], e = start[c + 1];
    for (uint32_t p = b + 1; p < e; ++p) {
        const uint32_t v = members[p];
        uint32_t q = p;
        while (q > b && members[q - 1] > v) {
            members[q] = members[q - 1];
            --q;
        }
        members[q] = v;
    }
}

template <int KIND, int PREC>
__global__ void __launch_bounds__(256) k_update(const SysDev* __restrict__ sys,
                                                const SpeciesDev* __restrict__ spc, int r,
                                                double* __restrict__ pos_base,
                                                double* __restrict__ ori_base,
                                                const uint32_t* __restrict__ start,
                                                const uint32_t* __restrict__ members,
                                                uint32_t colour, uint32_t select, uint32_t t,
                                                uint32_t k0, uint32_t k1,
                                                unsigned long long* __restrict__ stats) {
    constexpr int D = Traits<KIND>::dim;
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    Counters ct = {};
    const int half = S.n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    const int a = blockIdx.x * blockDim.x + threadIdx.x;
    if (a < n_act) {
        double sh[3];
        grid_shift(S, t, k0, k1, 1, sh);
        int cc[3];
        uint32_t c;
        active_cell(S, D, colour, a, cc, c);
        GlobalCells cl{start, members};
        trial_move<KIND, PREC>(S, P, pos_base + S.pos_off, ori_base + S.orient_off, cl, c, cc,
                               select, t, k0, k1, sh, ct);
    }
    flush(ct, stats + (size_t)r * kNumStats);
}

template <int KIND>
__global__ void __launch_bounds__(256) k_count(const SysDev* __restrict__ sys,
                                               const SpeciesDev* __restrict__ spc, int r,
                                               const double* __restrict__ pos_base,
                                               const double* __restrict__ ori_base,
                                               const uint32_t* __restrict__ start,
                                               const uint32_t* __restrict__ members,
                                               const uint32_t* __restrict__ cell_of,
                                               unsigned long long* __restrict__ out) {
    constexpr int D = Traits<KIND>::dim;
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    const double* pos = pos_base + S.pos_off;
    const double* ori = ori_base + S.orient_off;
    const int N = S.N, n = S.n;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t found = 0;
    Counters dummy = {};
    if (i < N) {
        const uint32_t c = cell_of[i];
        const int cc[3] = {(int)(c % (uint32_t)n), (int)((c / (uint32_t)n) % (uint32_t)n),
                           (int)(c / ((uint32_t)n * (uint32_t)n))};
        double xi[3] = {0.0, 0.0, 0.0}, qi[4];
#pragma unroll
        for (int a = 0; a < D; ++a) xi[a] = pos[a * N + i];
        load_orient<KIND>(ori, N, (uint32_t)i, qi);
        constexpr int zlo = D == 3 ? -1 : 0, zhi = D == 3 ? 1 : 0;
        for (int oz = zlo; oz <= zhi; ++oz)
            for (int oy = -1; oy <= 1; ++oy)
                for (int ox = -1; ox <= 1; ++ox) {
                    const int x = (cc[0] + ox + n) % n, y = (cc[1] + oy + n) % n,
                              z = D == 3 ? (cc[2] + oz + n) % n : 0;
                    const uint32_t cn = (uint32_t)(x + n * (y + n * z));
                    for (uint32_t p = start[cn]; p < start[cn + 1]; ++p) {
                        const uint32_t k = members[p];
                        if (k <= (uint32_t)i) continue;
                        double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
                        for (int a = 0; a < D; ++a) rr[a] = min_image(pos[a * N + k] - xi[a], S.L, S.inv_L);
                        double r2 = rr[0] * rr[0] + rr[1] * rr[1];
                        if constexpr (D == 3) r2 = r2 + rr[2] * rr[2];
                        if (!(r2 < P.circ2)) continue;
                        double qk[4];
                        load_orient<KIND>(ori, N, k, qk);
                        found += full_test<KIND, 0>(P, rr, qi, qk, dummy) ? 1u : 0u;
                    }
                }
    }
    const uint32_t s = wave_sum(found);
    if (__lane_id() == 0 && s) atomicAdd(out + r, (unsigned long long)s);
}

// ---------------------------------------------------------------------------
// Persistent path: whole sweeps per work-group, cell list in LDS.
// LDS: ends[ncells] u32, 16 scan words, members[N] u16.
// ---------------------------------------------------------------------------
template <int KIND, int PREC>
__device__ void persistent_body(const SysDev& S, const SpeciesDev& P, double* __restrict__ pos,
                                double* __restrict__ ori, uint32_t* ends, uint32_t* sm,
                                uint16_t* mem, uint32_t t0, uint32_t n_sweeps, uint32_t k0,
                                uint32_t k1, Counters& ct) {
    constexpr int D = Traits<KIND>::dim;
    const int tid = threadIdx.x, B = blockDim.x;
    const int N = S.N, nc = S.ncells;
    const int half = S.n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    const int chunk = (nc + B - 1) / B;
    for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
        const uint32_t t = t0 + sw;
        double sh[3];
        grid_shift(S, t, k0, k1, 1, sh);
        // counting sort of the shifted grid into LDS
        for (int c = tid; c < nc; c += B) ends[c] = 0u;
        __syncthreads();
        for (int i = tid; i < N; i += B) atomicAdd(ends + particle_cell<D>(S, pos, i, sh), 1u);
        __syncthreads();
        {
            const int c0 = tid * chunk, c1 = min(nc, c0 + chunk);
            uint32_t s = 0;
            for (int c = c0; c < c1; ++c) s += ends[c];
            uint32_t total;
            uint32_t run = block_exclusive_scan(s, sm, total);
            for (int c = c0; c < c1; ++c) {
                const uint32_t v = ends[c];
                ends[c] = run;
                run += v;
            }
        }
        __syncthreads();
        for (int i = tid; i < N; i += B) {
            const uint32_t p = atomicAdd(ends + particle_cell<D>(S, pos, i, sh), 1u);
            mem[p] = (uint16_t)i;
        }
        __syncthreads();
        for (int c = tid; c < nc; c += B) {
            const uint32_t b = c ? ends[c - 1] : 0u, e = ends[c];
            for (uint32_t p = b + 1; p < e; ++p) {
                const uint16_t v = mem[p];
                uint32_t q = p;
                while (q > b && mem[q - 1] > v) {
                    mem[q] = mem[q - 1];
                    --q;
                }
                mem[q] = v;
            }
        }
        __syncthreads();
        const LdsCells cl{ends, mem};
        const uint32_t ncol = 1u << D;
        for (int rnd = 0; rnd < S.rounds; ++rnd) {
            for (uint32_t colour = 0; colour < ncol; ++colour) {
                const uint32_t select = (uint32_t)rnd * ncol + colour;
                for (int a = tid; a < n_act; a += B) {
                    int cc[3];
                    uint32_t c;
                    active_cell(S, D, colour, a, cc, c);
                    trial_move<KIND, PREC>(S, P, pos, ori, cl, c, cc, select, t, k0, k1, sh, ct);
                }
                __syncthreads();
            }
        }
    }
}

template <int PREC>
__global__ void __launch_bounds__(256) k_persistent(const SysDev* __restrict__ sys,
                                                    const SpeciesDev* __restrict__ spc,
                                                    double* __restrict__ pos_base,
                                                    double* __restrict__ ori_base,
                                                    unsigned long long* __restrict__ stats,
                                                    uint32_t t0, uint32_t n_sweeps, uint32_t k0,
                                                    uint32_t k1) {
    extern __shared__ uint32_t lds[];
    const int r = blockIdx.x;
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    uint32_t* ends = lds;
    uint32_t* sm = lds + S.ncells;
    uint16_t* mem = reinterpret_cast<uint16_t*>(sm + 16);
    double* pos = pos_base + S.pos_off;
    double* ori = ori_base + S.orient_off;
    Counters ct = {};
    const int kind = P.kind;
    if (kind == kDisk)
        persistent_body<kDisk, PREC>(S, P, pos, ori, ends, sm, mem, t0, n_sweeps, k0, k1, ct);
    else if (kind == kPolygon)
        persistent_body<kPolygon, PREC>(S, P, pos, ori, ends, sm, mem, t0, n_sweeps, k0, k1, ct);
    else
        persistent_body<kPolyhedron, PREC>(S, P, pos, ori, ends, sm, mem, t0, n_sweeps, k0, k1, ct);
    flush(ct, stats + (size_t)r * kNumStats);
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static inline int blocks_for(long n, int b) { return (int)((n + b - 1) / b); }

size_t persistent_lds_bytes(int ncells, int N) {
    return (size_t)ncells * 4 + 16 * 4 + (size_t)((N + 1) & ~1) * 2;
}

hipError_t fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    k_fill_u64<<<blocks_for((long)n, 256), 256, 0, stream>>>(p, v, n);
    return hipGetLastError();
}

hipError_t build_cells(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                       uint32_t t, uint32_t k0, uint32_t k1, int shifted, hipStream_t stream) {
    const int nc = rh.ncells, N = rh.N;
    const int ntiles = blocks_for(nc, kScanTile);
    k_fill_u32<<<blocks_for(nc, 256), 256, 0, stream>>>(ws.count, 0u, nc);
    if (rh.dim == 3)
        k_assign<3><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, t, k0, k1, shifted,
                                                             ws.count, ws.cell_of, ws.slot_of);
    else
        k_assign<2><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, t, k0, k1, shifted,
                                                             ws.count, ws.cell_of, ws.slot_of);
    k_scan_tiles<<<ntiles, 256, 0, stream>>>(ws.count, nc, ws.partial);
    k_scan_partials<<<1, 256, 0, stream>>>(ws.partial, ntiles);
    k_scan_apply<<<ntiles, 256, 0, stream>>>(ws.count, nc, ws.partial, ws.start, (uint32_t)N);
    k_scatter<<<blocks_for(N, 256), 256, 0, stream>>>(ws.cell_of, ws.slot_of, ws.start,
                                                       ws.members, N);
    k_sort_cells<<<blocks_for(nc, 256), 256, 0, stream>>>(ws.start, ws.members, nc);
    return hipGetLastError();
}

template <int KIND, int PREC>
static void launch_passes(const Workspace& ws, const ReplicaHost& rh, int r, double* pos,
                          double* orient, uint32_t t, uint32_t k0, uint32_t k1,
                          hipStream_t stream) {
    const int half = rh.n / 2;
    const long n_act = rh.dim == 3 ? (long)half * half * half : (long)half * half;
    const uint32_t ncol = 1u << rh.dim;
    for (int rnd = 0; rnd < rh.rounds; ++rnd)
        for (uint32_t colour = 0; colour < ncol; ++colour)
            k_update<KIND, PREC><<<blocks_for(n_act, 256), 256, 0, stream>>>(
                ws.sys, ws.species, r, pos, orient, ws.start, ws.members, colour,
                (uint32_t)rnd * ncol + colour, t, k0, k1, ws.stats);
}

hipError_t grid_passes(const Workspace& ws, const ReplicaHost& rh, int r, double* pos,
                       double* orient, int precision, uint32_t t, uint32_t k0, uint32_t k1,
                       hipStream_t stream) {
    if (rh.kind == kDisk)
        launch_passes<kDisk, 0>(ws, rh, r, pos, orient, t, k0, k1, stream);
    else if (rh.kind == kPolygon && precision == 1)
        launch_passes<kPolygon, 1>(ws, rh, r, pos, orient, t, k0, k1, stream);
    else if (rh.kind == kPolygon)
        launch_passes<kPolygon, 0>(ws, rh, r, pos, orient, t, k0, k1, stream);
    else
        launch_passes<kPolyhedron, 0>(ws, rh, r, pos, orient, t, k0, k1, stream);
    return hipGetLastError();
}

hipError_t persistent_sweeps(const Workspace& ws, int n_replicas, size_t lds_bytes, double* pos,
                             double* orient, int precision, uint32_t t0, uint32_t n_sweeps,
                             uint32_t k0, uint32_t k1, int block, hipStream_t stream) {
    if (precision == 1)
        k_persistent<1><<<n_replicas, block, lds_bytes, stream>>>(ws.sys, ws.species, pos, orient,
                                                                  ws.stats, t0, n_sweeps, k0, k1);
    else
        k_persistent<0><<<n_replicas, block, lds_bytes, stream>>>(ws.sys, ws.species, pos, orient,
                                                                  ws.stats, t0, n_sweeps, k0, k1);
    return hipGetLastError();
}

hipError_t validate_state(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                          const double* orient, hipStream_t stream) {
    const int N = rh.N;
    if (rh.kind == kDisk)
        k_validate<0><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, orient, ws.overlap_out);
    else if (rh.kind == kPolygon)
        k_validate<2><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, orient, ws.overlap_out);
    else
        k_validate<4><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, orient, ws.overlap_out);
    return hipGetLastError();
}

hipError_t count_pairs(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                       const double* orient, hipStream_t stream) {
    const int N = rh.N;
    if (rh.kind == kDisk)
        k_count<kDisk><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, ws.species, r, pos, orient,
                                                                ws.start, ws.members, ws.cell_of,
                                                                ws.overlap_out);
    else if (rh.kind == kPolygon)
        k_count<kPolygon><<<blocks_for(N, 256), 256, 0, stream>>>(
            ws.sys, ws.species, r, pos, orient, ws.start, ws.members, ws.cell_of, ws.overlap_out);
    else
        k_count<kPolyhedron><<<blocks_for(N, 256), 256, 0, stream>>>(
            ws.sys, ws.species, r, pos, orient, ws.start, ws.members, ws.cell_of, ws.overlap_out);
    return hipGetLastError();
}

}  // namespace hpmc
