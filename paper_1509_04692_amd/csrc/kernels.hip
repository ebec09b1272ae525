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
#include <algorithm>

#include "device_common.hpp"
#include "engine.hpp"
#include "launch.hpp"

namespace hpmc {

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

// Phase totals of a trace build: per traced kernel kNumPhases cycle sums and
// a wave count (zero until read with reset).
#ifdef HPMC_TRACE
__device__ unsigned long long g_phase_trace[kTraceWords];
#endif

__device__ __forceinline__ void trace_flush(const PhaseClock& pc, int kernel) {
#ifdef HPMC_TRACE
    pc.flush(g_phase_trace + kernel * (kNumPhases + 1));
#endif
}

hipError_t read_phase_trace(unsigned long long* out, bool reset) {
#ifdef HPMC_TRACE
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess) e = hipMemcpyFromSymbol(out, HIP_SYMBOL(g_phase_trace), sizeof(g_phase_trace));
    if (e == hipSuccess && reset) {
        const unsigned long long zero[kTraceWords] = {};
        e = hipMemcpyToSymbol(HIP_SYMBOL(g_phase_trace), zero, sizeof(zero));
        if (e == hipSuccess) e = hipDeviceSynchronize();
    }
    return e;
#else
    (void)out;
    (void)reset;
    return hipErrorNotSupported;
#endif
}

// ---------------------------------------------------------------------------
// Grid path: global cell list.
// ---------------------------------------------------------------------------
__global__ void k_fill_u64(unsigned long long* __restrict__ p, unsigned long long v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_set_clock(Clock* __restrict__ clock, uint32_t t, uint32_t k0, uint32_t k1,
                            uint32_t n) {
    if (threadIdx.x == 0) *clock = Clock{t, k0, k1, n};
}

__global__ void k_set_chunk(Clock* __restrict__ clock, uint32_t n) {
    if (threadIdx.x == 0) clock->n = n;
}

__global__ void k_advance_clock(Clock* __restrict__ clock) {
    if (threadIdx.x == 0) clock->t += clock->n;
}

// Global cell lists of the grid path.  Every kernel below serves the
// replicas list[0 .. gridDim.y): blockIdx.y picks the replica, whose slice
// of the arrays starts at the offsets in its SysDev; blocks beyond the
// replica's size return at once (whole blocks, before any barrier).
template <int D>
__global__ void __launch_bounds__(256) k_assign(const SysDev* __restrict__ sys,
                                                const int32_t* __restrict__ list,
                                                const double* __restrict__ pos_base,
                                                const Clock* __restrict__ clock, int shifted,
                                                uint32_t* __restrict__ count,
                                                uint32_t* __restrict__ cell_of,
                                                uint32_t* __restrict__ slot_of) {
    const SysDev S = sys[list[blockIdx.y]];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= S.N) return;
    const Clock ck = *clock;
    double sh[3];
    grid_shift(S, ck.t, ck.k0, ck.k1, shifted, sh);
    const uint32_t c = particle_cell<D>(S, PosView{const_cast<double*>(pos_base) + S.pos_off, S.N}, (uint32_t)i, sh);
    cell_of[S.slot_off + i] = c;
    slot_of[S.slot_off + i] = atomicAdd(count + S.cell_off + c, 1u);
}

// The whole cell list of a small replica in one work-group of 1024 lanes
// (blockIdx.x picks the replica): the same arrays as the multi-kernel build
// (cell_of, slot_of, start, members in ascending tag order, and the sorted
// binary32 copy when shifted) with the histogram and its scan in LDS, in one
// launch instead of six.  Used when every replica of the launch has at most
// kSmallBuildN particles and kSmallBuildCells cells.
template <int D>
__global__ void __launch_bounds__(1024) k_build_small(const SysDev* __restrict__ sys,
                                                      const int32_t* __restrict__ list,
                                                      const double* __restrict__ pos_base,
                                                      const Clock* __restrict__ clock, int shifted,
                                                      uint32_t* __restrict__ cell_of,
                                                      uint32_t* __restrict__ slot_of,
                                                      uint32_t* __restrict__ start,
                                                      uint32_t* __restrict__ members,
                                                      float* __restrict__ xs) {
    __shared__ uint32_t cnt[kSmallBuildCells + 1];
    __shared__ uint32_t sm[16];
    const SysDev S = sys[list[blockIdx.x]];
    const int N = S.N, nc = S.ncells, tid = threadIdx.x;
    const Clock ck = *clock;
    double sh[3];
    grid_shift(S, ck.t, ck.k0, ck.k1, shifted, sh);
    const PosView pos{const_cast<double*>(pos_base) + S.pos_off, N};
    uint32_t* cof = cell_of + S.slot_off;
    uint32_t* sof = slot_of + S.slot_off;
    uint32_t* st = start + S.cell_off;
    uint32_t* mem = members + S.slot_off;
    for (int c = tid; c < nc; c += 1024) cnt[c] = 0u;
    __syncthreads();
    for (int i = tid; i < N; i += 1024) {
        const uint32_t c = particle_cell<D>(S, pos, (uint32_t)i, sh);
        cof[i] = c;
        sof[i] = atomicAdd(&cnt[c], 1u);
    }
    __syncthreads();
    // exclusive scan of the histogram: lane t owns cells [t chunk, (t + 1) chunk)
    const int chunk = (nc + 1023) / 1024, c0 = tid * chunk;
    uint32_t sum = 0;
    for (int j = 0; j < chunk; ++j) sum += c0 + j < nc ? cnt[c0 + j] : 0u;
    uint32_t total;
    uint32_t run = block_exclusive_scan(sum, sm, total);
    for (int j = 0; j < chunk; ++j) {
        if (c0 + j < nc) {
            const uint32_t v = cnt[c0 + j];
            cnt[c0 + j] = run;
            st[c0 + j] = run;
            run += v;
        }
    }
    if (tid == 0) {
        cnt[nc] = (uint32_t)N;
        st[nc] = (uint32_t)N;
    }
    __syncthreads();
    for (int i = tid; i < N; i += 1024) mem[cnt[cof[i]] + sof[i]] = (uint32_t)i;
    __syncthreads();
    // occupants of each cell in ascending tag order (a handful per cell)
    for (int c = tid; c < nc; c += 1024) {
        const uint32_t b = cnt[c], e = cnt[c + 1];
        for (uint32_t p = b + 1; p < e; ++p) {
            const uint32_t v = mem[p];
            uint32_t q = p;
            while (q > b && mem[q - 1] > v) {
                mem[q] = mem[q - 1];
                --q;
            }
            mem[q] = v;
        }
    }
    if (!shifted) return;
    __syncthreads();
    const XsView<D> xv{xs + kXsStride * S.slot_off};
    for (int p = tid; p < N; p += 1024) {
        double y[3];
        particle_grid<D>(S, pos, mem[p], sh, y);
        xv.store((uint32_t)p, y);
    }
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
__global__ void __launch_bounds__(256) k_scan_tiles(const SysDev* __restrict__ sys,
                                                    const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ count,
                                                    uint32_t* __restrict__ partial) {
    __shared__ uint32_t sm[16];
    const SysDev S = sys[list[blockIdx.y]];
    const int nc = S.ncells;
    if ((int)blockIdx.x * kScanTile >= nc) return;
    const uint32_t* cnt = count + S.cell_off;
    const int base = blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += base + j < nc ? cnt[base + j] : 0u;
    uint32_t total;
    block_exclusive_scan(s, sm, total);
    if (threadIdx.x == 0) partial[S.part_off + blockIdx.x] = total;
}

// Start offsets of a tile's cells: the tile's exclusive scan plus the sum of
// the earlier tiles' totals (read straight from the tile sums, so no separate
// scan of them is launched).  The histogram is cleared behind the read, so
// the next build starts from zero counts.
__global__ void __launch_bounds__(256) k_scan_apply(const SysDev* __restrict__ sys,
                                                    const int32_t* __restrict__ list,
                                                    uint32_t* __restrict__ count,
                                                    const uint32_t* __restrict__ partial,
                                                    uint32_t* __restrict__ start) {
    __shared__ uint32_t sm[16];
    const SysDev S = sys[list[blockIdx.y]];
    const int nc = S.ncells;
    if ((int)blockIdx.x * kScanTile >= nc) return;
    uint32_t* cnt = count + S.cell_off;
    uint32_t* st = start + S.cell_off;
    uint32_t before = 0;
    for (int j = threadIdx.x; j < (int)blockIdx.x; j += blockDim.x) before += partial[S.part_off + j];
    uint32_t prefix;
    (void)block_exclusive_scan(before, sm, prefix);
    const int base = blockIdx.x * kScanTile + threadIdx.x * 8;
    uint32_t v[8], s = 0;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        v[j] = base + j < nc ? cnt[base + j] : 0u;
        if (base + j < nc) cnt[base + j] = 0u;
        s += v[j];
    }
    uint32_t total;
    uint32_t run = block_exclusive_scan(s, sm, total) + prefix;
#pragma unroll
    for (int j = 0; j < 8; ++j) {
        if (base + j < nc) st[base + j] = run;
        run += v[j];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) st[nc] = (uint32_t)S.N;
}

__global__ void __launch_bounds__(256) k_scatter(const SysDev* __restrict__ sys,
                                                 const int32_t* __restrict__ list,
                                                 const uint32_t* __restrict__ cell_of,
                                                 const uint32_t* __restrict__ slot_of,
                                                 const uint32_t* __restrict__ start,
                                                 uint32_t* __restrict__ members) {
    const SysDev S = sys[list[blockIdx.y]];
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < S.N)
        members[S.slot_off + start[S.cell_off + cell_of[S.slot_off + i]] + slot_of[S.slot_off + i]] =
            (uint32_t)i;
}

// Occupants of each cell in ascending tag order (atomics scatter them in
// arbitrary order; cells hold a handful, so insertion sort).
__global__ void __launch_bounds__(256) k_sort_cells(const SysDev* __restrict__ sys,
                                                    const int32_t* __restrict__ list,
                                                    const uint32_t* __restrict__ start,
                                                    uint32_t* __restrict__ members) {
    const SysDev S = sys[list[blockIdx.y]];
    const int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= S.ncells) return;
    uint32_t* mem = members + S.slot_off;
    const uint32_t b = start[S.cell_off + c], e = start[S.cell_off + c + 1];
    for (uint32_t p = b + 1; p < e; ++p) {
        const uint32_t v = mem[p];
        uint32_t q = p;
        while (q > b && mem[q - 1] > v) {
            mem[q] = mem[q - 1];
            --q;
        }
        mem[q] = v;
    }
}

// Cell-sorted binary32 copy of the shifted-frame coordinates (slot order).
template <int D>
__global__ void __launch_bounds__(256) k_gather_xs(const SysDev* __restrict__ sys,
                                                   const int32_t* __restrict__ list,
                                                   const double* __restrict__ pos_base,
                                                   const Clock* __restrict__ clock,
                                                   const uint32_t* __restrict__ members,
                                                   float* __restrict__ xs) {
    const SysDev S = sys[list[blockIdx.y]];
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= S.N) return;
    const Clock ck = *clock;
    double sh[3], y[3];
    grid_shift(S, ck.t, ck.k0, ck.k1, 1, sh);
    particle_grid<D>(S, PosView{const_cast<double*>(pos_base) + S.pos_off, S.N}, members[S.slot_off + p],
                     sh, y);
    XsView<D>{xs + kXsStride * S.slot_off}.store((uint32_t)p, y);
}

// One colour pass of the grid path: one wave per tile of 64/G active cells,
// four waves per work-group.
template <int KIND, int PREC, int G, int NV, int Q>
__global__ void __launch_bounds__(256) k_update(const SysDev* __restrict__ sys,
                                                const SpeciesDev* __restrict__ spc,
                                                const int32_t* __restrict__ list,
                                                double* __restrict__ pos_base,
                                                double* __restrict__ ori_base,
                                                const uint32_t* __restrict__ start,
                                                const uint32_t* __restrict__ members,
                                                float* __restrict__ xs, int rnd,
                                                uint32_t colour, const Clock* __restrict__ clock,
                                                unsigned long long* __restrict__ stats) {
    constexpr int D = Traits<KIND>::dim;
    __shared__ uint32_t scratch_words[4][kWaveScratchWords];
    const int r = list[blockIdx.y];
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    Counters ct = {};
    PhaseClock pc;
    pc.start();
    const int half = S.n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    const int wave = threadIdx.x >> 6;
    const int a0 = (blockIdx.x * 4 + wave) * (64 / G);
    if (rnd < S.rounds && a0 < n_act) {  // replicas with fewer rounds sit this one out
        const Clock ck = *clock;
        const uint32_t t = ck.t, k0 = ck.k0, k1 = ck.k1;
        double sh[3];
        grid_shift(S, t, k0, k1, 1, sh);
        const PosView pos{pos_base + S.pos_off, S.N};
        const GlobalCells cl{start + S.cell_off, members + S.slot_off};
        const uint32_t select = (uint32_t)rnd * (1u << D) + colour;
        pass_tile<KIND, PREC, G, NV, false, Q>(S, P, pos, ori_base + S.orient_off, cl,
                                            XsView<D>{xs + kXsStride * S.slot_off}, colour, select,
                                            t, k0, k1, sh, a0, n_act,
                                            wave_scratch(scratch_words[wave]), ct, pc);
    }
    flush_block(ct, &scratch_words[0][0], stat_stripe(stats, r));
    pc.mark<kPhOther>();
    trace_flush(pc, kTraceUpdate);
}

// ---------------------------------------------------------------------------
// Global-queue variant of a colour pass (the paper's second variant), three
// kernels: (1) one lane per active cell proposes its move, keeps the trial
// state in global memory and appends every pre-filter hit to its replica's
// queue; (2) one lane per queued pair runs the binary64 circumsphere test and
// the full test and marks the owner cell on an overlap; (3) one lane per
// active cell applies the moves of unmarked cells.  There is no early exit:
// every queued pair is tested.
//
// Queue bound: active cells of one colour are two cells apart on every axis,
// so a slot lies in the 3^dim neighbourhood of at most 2^dim of them, and a
// replica queues at most 2^dim N pairs per pass.
// ---------------------------------------------------------------------------
template <int KIND>
__global__ void __launch_bounds__(256) k_gq_scan(const SysDev* __restrict__ sys,
                                                 const SpeciesDev* __restrict__ spc,
                                                 const int32_t* __restrict__ list,
                                                 const double* __restrict__ pos_base,
                                                 const double* __restrict__ ori_base,
                                                 const uint32_t* __restrict__ start,
                                                 const uint32_t* __restrict__ members,
                                                 const float* __restrict__ xs, int rnd,
                                                 uint32_t colour, const Clock* __restrict__ clock,
                                                 GlobalQueue gq, unsigned long long* __restrict__ stats) {
    constexpr int D = Traits<KIND>::dim;
    __shared__ uint32_t red[4 * kNumStats];
    __shared__ uint2 stage[4][128];
    const int r = list[blockIdx.y];
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    Counters ct = {};
    const int half = S.n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    const int a = (int)(blockIdx.x * 256 + threadIdx.x);
    if (rnd < S.rounds && (int)(blockIdx.x * 256) < n_act) {  // uniform over the work-group
        const Clock ck = *clock;
        double sh[3];
        grid_shift(S, ck.t, ck.k0, ck.k1, 1, sh);
        const PosView pos{const_cast<double*>(pos_base) + S.pos_off, S.N};
        const double* ori = ori_base + S.orient_off;
        const GlobalCells cl{start + S.cell_off, members + S.slot_off};
        const XsView<D> xv{const_cast<float*>(xs) + kXsStride * S.slot_off};
        const uint32_t select = (uint32_t)rnd * (1u << D) + colour;
        int cc[3] = {0, 0, 0};
        uint32_t c = 0, i = 0, pi = 0;
        bool live = false, c_rot = false, c_moved = false;
        double xn[3] = {0.0, 0.0, 0.0};
        double qn[4] = {1.0, 0.0, 0.0, 0.0};
        if (a < n_act) {
            propose<KIND>(S, P, pos, ori, cl, colour, select, ck.t, ck.k0, ck.k1, sh, a, cc, c, i, pi,
                          live, xn, qn, c_rot, c_moved, ct);
            ct.attempted_rot += c_rot ? 1u : 0u;
            ct.cell_reject += (c_moved && !live) ? 1u : 0u;
            const size_t o = (size_t)S.cell_off + a, T = (size_t)gq.cell_total;
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) gq.trial[ax * T + o] = xn[ax];
#pragma unroll
            for (int q = 0; q < 4; ++q) gq.trial[(3 + q) * T + o] = qn[q];
            gq.meta[o] = i;
            gq.meta[T + o] = pi;
            gq.meta[2 * T + o] = (live ? 1u : 0u) | (c_rot ? 2u : 0u) | (c_moved ? 4u : 0u);
            gq.flag[o] = 0u;
        }
        double yn[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int ax = 0; ax < D; ++ax) yn[ax] = grid_coord(xn[ax], sh[ax], S.L);
        uint2* ent = gq.entries + ((size_t)S.slot_off * kGqPerSlot);
        const uint32_t cap = (uint32_t)S.N << D;
        const float t2 = S.scan_t2;
        // hits are staged per wave in LDS and appended 64 at a time, one
        // atomic per 64 entries
        uint2* st = stage[threadIdx.x >> 6];
        const uint32_t lane = __lane_id();
        uint32_t staged = 0;  // wave-uniform, < 64 between iterations
        auto append = [&](uint32_t m) {
            wave_sync();
            uint32_t base = 0;
            if (lane == 0) base = atomicAdd(gq.count + r, m);
            base = (uint32_t)__shfl((int)base, 0, 64);
            if (lane < m && base + lane < cap) ent[base + lane] = st[lane];
            const uint32_t left = staged - m;
            const uint2 v = lane < left ? st[m + lane] : make_uint2(0u, 0u);
            wave_sync();
            if (lane < left) st[lane] = v;
            staged = left;
            wave_sync();
        };
        for (int ri = 0; ri < Neighbourhood<D>::ranges; ++ri) {
            uint32_t p = 0, e = 0;
            float ref[3] = {0.0f, 0.0f, 0.0f};
            if (live) neighbour_range<D>(cl, cc, S.n, ri, S.L, yn, p, e, ref);
            for (;;) {
                const bool work = p < e;
                if (wave_ballot(work) == 0ull) break;
                const uint32_t slot = work ? p : 0u;
                float v[3];
                xv.load(slot, v);
                const float rx = v[0] - ref[0], ry = v[1] - ref[1];
                float r2 = fmaf(ry, ry, rx * rx);
                if constexpr (D == 3) {
                    const float rz = v[2] - ref[2];
                    r2 = fmaf(rz, rz, r2);
                }
                r2 = (work && slot != pi) ? r2 : INFINITY;
                const bool hit = r2 < t2;
                p += work ? 1u : 0u;
                const uint64_t hm = wave_ballot(hit);
                if (hit) st[staged + lanes_below(hm)] = make_uint2((uint32_t)a, slot);
                staged += (uint32_t)__builtin_popcountll(hm);
                if (staged >= 64u) append(64u);
            }
        }
        if (staged) append(staged);
    }
    flush_block(ct, red, stat_stripe(stats, r));
}

template <int KIND, int PREC, int NV>
__global__ void __launch_bounds__(256) k_gq_test(const SysDev* __restrict__ sys,
                                                 const SpeciesDev* __restrict__ spc,
                                                 const int32_t* __restrict__ list,
                                                 const double* __restrict__ pos_base,
                                                 const double* __restrict__ ori_base,
                                                 const uint32_t* __restrict__ members, int rnd,
                                                 GlobalQueue gq, unsigned long long* __restrict__ stats) {
    constexpr int D = Traits<KIND>::dim;
    __shared__ uint32_t red[4 * kNumStats];
    const int r = list[blockIdx.y];
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    Counters ct = {};
    if (rnd < S.rounds) {
        const uint32_t cap = (uint32_t)S.N << D;
        const uint32_t nq = min(gq.count[r], cap);
        const uint2* ent = gq.entries + ((size_t)S.slot_off * kGqPerSlot);
        const double* pos = pos_base + S.pos_off;
        const double* ori = ori_base + S.orient_off;
        const size_t T = (size_t)gq.cell_total;
        for (uint32_t q = blockIdx.x * 256 + threadIdx.x; q < nq; q += gridDim.x * 256) {
            const uint2 e = ent[q];
            const size_t o = (size_t)S.cell_off + e.x;
            const uint32_t k = members[S.slot_off + e.y];
            double r3[3] = {0.0, 0.0, 0.0};
#pragma unroll
            for (int ax = 0; ax < D; ++ax)
                r3[ax] = min_image(pos[(size_t)ax * S.N + k] - gq.trial[ax * T + o], S.L, S.inv_L);
            double r2 = r3[0] * r3[0] + r3[1] * r3[1];
            if constexpr (D == 3) r2 = r2 + r3[2] * r3[2];
            if (r2 < P.circ2) {
                double qi[4], qk[4];
#pragma unroll
                for (int c = 0; c < 4; ++c) qi[c] = gq.trial[(3 + c) * T + o];
                load_orient<KIND>(ori, S.N, k, qk);
                if (full_test<KIND, PREC, NV>(P, r3, qi, qk, ct)) gq.flag[o] = 1u;
            }
        }
    }
    flush_block(ct, red, stat_stripe(stats, r));
}

template <int KIND>
__global__ void __launch_bounds__(256) k_gq_apply(const SysDev* __restrict__ sys,
                                                  const int32_t* __restrict__ list,
                                                  double* __restrict__ pos_base,
                                                  double* __restrict__ ori_base,
                                                  float* __restrict__ xs, int rnd,
                                                  const Clock* __restrict__ clock, GlobalQueue gq,
                                                  unsigned long long* __restrict__ stats) {
    constexpr int D = Traits<KIND>::dim;
    __shared__ uint32_t red[4 * kNumStats];
    const int r = list[blockIdx.y];
    const SysDev S = sys[r];
    Counters ct = {};
    const int half = S.n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    const int a = (int)(blockIdx.x * 256 + threadIdx.x);
    if (rnd < S.rounds && a < n_act) {
        const size_t o = (size_t)S.cell_off + a, T = (size_t)gq.cell_total;
        const uint32_t bits = gq.meta[2 * T + o];
        if (bits & 1u) {
            const bool rejected = gq.flag[o] != 0u;
            ct.overlap_reject += rejected ? 1u : 0u;
            ct.accept += rejected ? 0u : 1u;
            if (!rejected) {
                const uint32_t i = gq.meta[o], pi = gq.meta[T + o];
                const int N = S.N;
                if (bits & 4u) {
                    const Clock ck = *clock;
                    double sh[3], xn[3] = {0.0, 0.0, 0.0}, yn[3] = {0.0, 0.0, 0.0};
                    grid_shift(S, ck.t, ck.k0, ck.k1, 1, sh);
                    double* pos = pos_base + S.pos_off;
#pragma unroll
                    for (int ax = 0; ax < D; ++ax) {
                        xn[ax] = gq.trial[ax * T + o];
                        pos[(size_t)ax * N + i] = xn[ax];
                        yn[ax] = grid_coord(xn[ax], sh[ax], S.L);
                    }
                    XsView<D>{xs + kXsStride * S.slot_off}.store(pi, yn);
                }
                if (bits & 2u) {
                    double* ori = ori_base + S.orient_off;
                    constexpr int NC = Traits<KIND>::ncomp;
#pragma unroll
                    for (int c = 0; c < NC; ++c) ori[(size_t)c * N + i] = gq.trial[(3 + c) * T + o];
                }
            }
        }
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) gq.count[r] = 0u;  // the test kernel has read it
    flush_block(ct, red, stat_stripe(stats, r));
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
    start += S.cell_off;
    members += S.slot_off;
    cell_of += S.slot_off;
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
                        found += full_test<KIND, 0, 0>(P, rr, qi, qk, dummy) ? 1u : 0u;
                    }
                }
    }
    const uint32_t s = wave_sum(found);
    if (__lane_id() == 0 && s) atomicAdd(out + r, (unsigned long long)s);
}

// Volume-perturbation counts: out[b] += number of pairs i < k that overlap
// (binary64 circumsphere test, then the full test) once their minimum-image
// separation r is scaled by 1 - scales[b], orientations unchanged.  The
// unshifted cell list is searched `reach` cells around each particle (the
// host checks that 2R / (1 - scales[n - 1]) stays within that reach).  A pair
// whose separation fails the circumsphere test at the largest scale factor
// fails it at every smaller one, so it is skipped whole.
template <int KIND>
__global__ void __launch_bounds__(256) k_scale_count(const SysDev* __restrict__ sys,
                                                     const SpeciesDev* __restrict__ spc, int r,
                                                     const double* __restrict__ pos_base,
                                                     const double* __restrict__ ori_base,
                                                     const uint32_t* __restrict__ start,
                                                     const uint32_t* __restrict__ members,
                                                     const uint32_t* __restrict__ cell_of,
                                                     const double* __restrict__ scales, int n_s,
                                                     int reach, unsigned long long* __restrict__ out) {
    constexpr int D = Traits<KIND>::dim;
    __shared__ uint32_t hist[kMaxHistBins];
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    const double* pos = pos_base + S.pos_off;
    const double* ori = ori_base + S.orient_off;
    start += S.cell_off;
    members += S.slot_off;
    cell_of += S.slot_off;
    const int N = S.N, n = S.n;
    for (int b = threadIdx.x; b < n_s; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    Counters dummy = {};
    if (i < N) {
        const uint32_t c = cell_of[i];
        const int cc[3] = {(int)(c % (uint32_t)n), (int)((c / (uint32_t)n) % (uint32_t)n),
                           (int)(c / ((uint32_t)n * (uint32_t)n))};
        double xi[3] = {0.0, 0.0, 0.0}, qi[4];
#pragma unroll
        for (int a = 0; a < D; ++a) xi[a] = pos[a * N + i];
        load_orient<KIND>(ori, N, (uint32_t)i, qi);
        const double f_min = 1.0 - scales[n_s - 1];
        const int zlo = D == 3 ? -reach : 0, zhi = D == 3 ? reach : 0;
        for (int oz = zlo; oz <= zhi; ++oz)
            for (int oy = -reach; oy <= reach; ++oy)
                for (int ox = -reach; ox <= reach; ++ox) {
                    const int x = (cc[0] + ox + n) % n, y = (cc[1] + oy + n) % n,
                              z = D == 3 ? (cc[2] + oz + n) % n : 0;
                    const uint32_t cn = (uint32_t)(x + n * (y + n * z));
                    for (uint32_t p = start[cn]; p < start[cn + 1]; ++p) {
                        const uint32_t k = members[p];
                        if (k <= (uint32_t)i) continue;
                        double rr[3] = {0.0, 0.0, 0.0};
#pragma unroll
                        for (int a = 0; a < D; ++a) rr[a] = min_image(pos[a * N + k] - xi[a], S.L, S.inv_L);
                        double m2 = (rr[0] * f_min) * (rr[0] * f_min) + (rr[1] * f_min) * (rr[1] * f_min);
                        if constexpr (D == 3) m2 = m2 + (rr[2] * f_min) * (rr[2] * f_min);
                        if (!(m2 < P.circ2)) continue;
                        double qk[4];
                        load_orient<KIND>(ori, N, k, qk);
                        for (int b = 0; b < n_s; ++b) {
                            const double f = 1.0 - scales[b];
                            double rs[3] = {0.0, 0.0, 0.0};
#pragma unroll
                            for (int a = 0; a < D; ++a) rs[a] = rr[a] * f;
                            double s2 = rs[0] * rs[0] + rs[1] * rs[1];
                            if constexpr (D == 3) s2 = s2 + rs[2] * rs[2];
                            if (s2 < P.circ2 && full_test<KIND, 0, 0>(P, rs, qi, qk, dummy))
                                atomicAdd(hist + b, 1u);
                        }
                    }
                }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_s; b += blockDim.x)
        if (hist[b]) atomicAdd(out + b, (unsigned long long)hist[b]);
}

// Histogram of pair separations (pairs i < k with edges2[b] <= r^2 <
// edges2[b + 1]) over the unshifted cell list; cells within `reach` of the
// particle's cell are searched (edges2[n_bins] < (reach * w)^2 keeps the
// search complete).  One LDS histogram per work-group, one atomic per bin.
template <int D>
__global__ void __launch_bounds__(256) k_pair_hist(const SysDev* __restrict__ sys, int r,
                                                   const double* __restrict__ pos_base,
                                                   const uint32_t* __restrict__ start,
                                                   const uint32_t* __restrict__ members,
                                                   const uint32_t* __restrict__ cell_of,
                                                   const double* __restrict__ edges2, int n_bins,
                                                   int reach, unsigned long long* __restrict__ out) {
    __shared__ uint32_t hist[kMaxHistBins];
    const SysDev S = sys[r];
    const double* pos = pos_base + S.pos_off;
    start += S.cell_off;
    members += S.slot_off;
    cell_of += S.slot_off;
    const int N = S.N, n = S.n;
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x) hist[b] = 0u;
    __syncthreads();
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < N) {
        const uint32_t c = cell_of[i];
        const int cc[3] = {(int)(c % (uint32_t)n), (int)((c / (uint32_t)n) % (uint32_t)n),
                           (int)(c / ((uint32_t)n * (uint32_t)n))};
        double xi[3] = {0.0, 0.0, 0.0};
#pragma unroll
        for (int a = 0; a < D; ++a) xi[a] = pos[a * N + i];
        const double lo = edges2[0], hi = edges2[n_bins];
        const int zlo = D == 3 ? -reach : 0, zhi = D == 3 ? reach : 0;
        for (int oz = zlo; oz <= zhi; ++oz)
            for (int oy = -reach; oy <= reach; ++oy)
                for (int ox = -reach; ox <= reach; ++ox) {
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
                        if (!(lo <= r2 && r2 < hi)) continue;
                        int b = 0;
                        while (b + 1 < n_bins && edges2[b + 1] <= r2) ++b;
                        atomicAdd(hist + b, 1u);
                    }
                }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < n_bins; b += blockDim.x)
        if (hist[b]) atomicAdd(out + b, (unsigned long long)hist[b]);
}

// ---------------------------------------------------------------------------
// Persistent path: one work-group owns one replica and runs whole sweeps.
// LDS (dynamic), in this order: positions D*N f64 (residency >= 1),
// orientations ncomp*N f64 (residency >= 2), the cell-sorted binary32
// coordinates (N float2 / float4; not at residency 3, where the pre-filter
// computes them from the positions), members N u16, inclusive ends ncells
// u16, a union (counts ncells u32 while building the cell list / wave queues
// and flags during the passes) and 16 scan words.  At residency 3 the
// replica's whole state stays in LDS between the launch's first load and its
// last store, both coalesced.
// ---------------------------------------------------------------------------
__host__ __device__ inline size_t align16(size_t x) { return (x + 15) & ~(size_t)15; }

struct BatchLayout {
    size_t pos, ori, xs, mem, ends, uni, scan, total;
};

// Residency level: 0 = particle data in global memory, 1 = positions in LDS,
// 2 = positions and orientations in LDS, 3 = the same without the binary32
// copy.  wave_words: per-wave scratch (wave_scratch_words).  ghost_cap > 0
// (2D, res <= 2): the cell list has ghost edge columns, 2 n more cells and up
// to ghost_cap more slots.
__host__ __device__ inline BatchLayout batch_layout(int dim, int ncomp, int N, int ncells,
                                                    int nwaves, int res, int wave_words, int n = 0,
                                                    int ghost_cap = 0) {
    BatchLayout b;
    const size_t slots = (size_t)N + (size_t)ghost_cap;
    if (ghost_cap > 0) ncells += 2 * n;
    size_t o = 0;
    b.pos = o;
    o += res >= 1 ? align16((size_t)dim * N * 8) : 0;
    b.ori = o;
    o += res >= 2 ? align16((size_t)ncomp * N * 8) : 0;
    b.xs = o;
    o += res <= 2 ? align16(slots * (size_t)xs_bytes(dim)) : 0;
    b.mem = o;
    o += align16(slots * 2);
    b.ends = o;
    o += align16((size_t)ncells * 2);
    b.uni = o;
    const size_t uni_words = (size_t)ncells > (size_t)nwaves * wave_words
                                 ? (size_t)ncells
                                 : (size_t)nwaves * wave_words;
    o += align16(uni_words * 4);
    b.scan = o;
    o += 16 * 4;
    b.total = o;
    return b;
}

template <int KIND, int PREC, int RES, int NV, bool GH>
__global__ void __launch_bounds__(kBatchBlock) k_batch(const SysDev* __restrict__ sys,
                                                       const SpeciesDev* __restrict__ spc,
                                                       const int32_t* __restrict__ list,
                                                       double* __restrict__ pos_base,
                                                       double* __restrict__ ori_base,
                                                       unsigned long long* __restrict__ stats,
                                                       const Clock* __restrict__ clock) {
    constexpr int D = Traits<KIND>::dim;
    static_assert(!GH || (D == 2 && RES <= 2), "ghost edge columns: 2D, binary32 copy in LDS");
    extern __shared__ __align__(16) unsigned char lds[];
    const int r = list[blockIdx.x];
    const SysDev S = sys[r];
    const SpeciesDev& P = spc[S.species];
    const int tid = threadIdx.x, B = blockDim.x, nwaves = B >> 6, wave = tid >> 6;
    const int N = S.N, nc = S.ncells, n = S.n;
    constexpr int NC = Traits<KIND>::ncomp;
    constexpr int WW = wave_scratch_words(KIND, PREC);
    constexpr bool XS = RES <= 2;  // binary32 cell-sorted copy kept in LDS
    const int gcap = GH ? S.ghost_cap : 0;
    const int nst = GH ? nc + 2 * n : nc;  // stored cells (with the ghost columns)
    const BatchLayout lay = batch_layout(D, NC, N, nc, nwaves, RES, WW, n, gcap);
    double* gpos = pos_base + S.pos_off;
    double* gori = ori_base + S.orient_off;
    const PosView pos{RES >= 1 ? reinterpret_cast<double*>(lds + lay.pos) : gpos, N};
    double* ori = RES >= 2 ? reinterpret_cast<double*>(lds + lay.ori) : gori;
    const XsView<D> xs{reinterpret_cast<float*>(lds + lay.xs)};
    uint16_t* mem = reinterpret_cast<uint16_t*>(lds + lay.mem);
    uint16_t* ends = reinterpret_cast<uint16_t*>(lds + lay.ends);
    uint32_t* uni = reinterpret_cast<uint32_t*>(lds + lay.uni);
    uint32_t* sm = reinterpret_cast<uint32_t*>(lds + lay.scan);
    if constexpr (RES >= 1) {
        for (int k = tid; k < D * N; k += B) pos.p[k] = gpos[k];
    }
    if constexpr (RES >= 2) {
        for (int k = tid; k < NC * N; k += B) ori[k] = gori[k];
    }
    __syncthreads();
    Counters ct = {};
    PhaseClock pc;
    pc.start();
    const Clock ck = *clock;
    const uint32_t t0 = ck.t, k0 = ck.k0, k1 = ck.k1, n_sweeps = ck.n;
    const int half = n / 2;
    const int n_act = D == 3 ? half * half * half : half * half;
    // active cells per wave and pass: at most 64 (one per lane), spread
    // evenly over the waves a pass needs, so that no wave holds a short
    // remainder tile; polyhedra of four or more vertices (long XenoCollide
    // walks) spread down to 32 cells per wave, which puts more waves on a pass
    const int min_tile = KIND == kPolyhedron && P.nv >= 4 ? 32 : 64;
    const int wv = min(nwaves, (n_act + min_tile - 1) / min_tile);
    const int tile = min(64, (n_act + wv - 1) / wv);
    const int chunk = (nst + B - 1) / B;
    const WaveScratch wscr = wave_scratch(uni + wave * WW);
    // storage cell of grid coordinates y, and the side of its ghost copy:
    // +1 (column 0, copied after the row's last cell, x + L), -1 (column
    // n - 1, copied before the first, x - L), 0 (none)
    auto stored_cell = [&](const double (&y)[3], int& gh) -> uint32_t {
        if constexpr (GH) {
            const int cx = cell_of_coord(y[0], S.inv_w, n), cy = cell_of_coord(y[1], S.inv_w, n);
            gh = cx == 0 ? 1 : (cx == n - 1 ? -1 : 0);
            return (uint32_t)(cx + 1 + (n + 2) * cy);
        } else {
            gh = 0;
            return cell_of_grid<D>(S, y);
        }
    };
    for (uint32_t sw = 0; sw < n_sweeps; ++sw) {
        const uint32_t t = t0 + sw;
        double sh[3];
        grid_shift(S, t, k0, k1, 1, sh);
        // counting sort of the shifted grid (ascending tags within a cell); the
        // first kOwn particles of each thread keep their cell and binary32
        // shifted-frame coordinates in registers between the passes
        constexpr int kOwn = kBatchOwn;
        uint32_t own_cell[kOwn];
        int own_gh[kOwn];
        float own_y[kOwn][3];
        double own_x[kOwn];
        uint32_t* count = uni;
        for (int c = tid; c < nst; c += B) count[c] = 0u;
        __syncthreads();
        pc.mark<kPhBuild>();
#pragma unroll
        for (int j = 0; j < kOwn; ++j) {
            const int i = tid + j * B;
            own_cell[j] = 0u;
            own_gh[j] = 0;
            own_x[j] = 0.0;
            own_y[j][0] = own_y[j][1] = own_y[j][2] = 0.0f;
            if (i < N) {
                double y[3];
                particle_grid<D>(S, pos, (uint32_t)i, sh, y);
                own_cell[j] = stored_cell(y, own_gh[j]);
                own_x[j] = y[0];
#pragma unroll
                for (int a = 0; a < 3; ++a) own_y[j][a] = (float)y[a];
                atomicAdd(count + own_cell[j], 1u);
                if (GH && own_gh[j]) atomicAdd(count + own_cell[j] + own_gh[j] * n, 1u);
            }
        }
        for (int i = tid + kOwn * B; i < N; i += B) {
            double y[3];
            particle_grid<D>(S, pos, (uint32_t)i, sh, y);
            int gh;
            const uint32_t c = stored_cell(y, gh);
            atomicAdd(count + c, 1u);
            if (GH && gh) atomicAdd(count + c + gh * n, 1u);
        }
        __syncthreads();
        pc.mark<kPhCount>();
        uint32_t total;
        {
            const int c0 = tid * chunk, c1 = min(nst, c0 + chunk);
            uint32_t s = 0;
            for (int c = c0; c < c1; ++c) s += count[c];
            uint32_t run = block_exclusive_scan(s, sm, total);
            for (int c = c0; c < c1; ++c) {
                const uint32_t v = count[c];
                count[c] = run;
                run += v;
            }
        }
        if (GH && total > (uint32_t)(N + gcap)) {
            // more edge-column particles than the bound for a state without
            // overlaps allows: stop before any write, report it
            if (tid == 0) atomicAdd(stat_stripe(stats, r) + kCellOverflow, 1ull);
            break;
        }
        __syncthreads();
        pc.mark<kPhPrefix>();
        // scatter the tags and their binary32 coordinates (ghost copies too)
#pragma unroll
        for (int j = 0; j < kOwn; ++j) {
            const int i = tid + j * B;
            if (i < N) {
                const uint32_t slot = atomicAdd(count + own_cell[j], 1u);
                mem[slot] = (uint16_t)i;
                if constexpr (XS) xs.store(slot, own_y[j]);
                if constexpr (GH) {
                    if (own_gh[j]) {
                        const uint32_t g = atomicAdd(count + own_cell[j] + own_gh[j] * n, 1u);
                        mem[g] = (uint16_t)i;
                        const float gy[3] = {(float)(own_x[j] + (double)own_gh[j] * S.L), own_y[j][1], own_y[j][2]};
                        xs.store(g, gy);
                    }
                }
            }
        }
        for (int i = tid + kOwn * B; i < N; i += B) {
            double y[3];
            particle_grid<D>(S, pos, (uint32_t)i, sh, y);
            int gh;
            const uint32_t c = stored_cell(y, gh);
            const uint32_t slot = atomicAdd(count + c, 1u);
            mem[slot] = (uint16_t)i;
            if constexpr (XS) xs.store(slot, y);
            if constexpr (GH) {
                if (gh) {
                    const uint32_t g = atomicAdd(count + c + gh * n, 1u);
                    mem[g] = (uint16_t)i;
                    const double gy[3] = {y[0] + (double)gh * S.L, y[1], y[2]};
                    xs.store(g, gy);
                }
            }
        }
        __syncthreads();
        pc.mark<kPhScatter>();
        // ascending tags within each cell; the coordinates move with their tags
        for (int c = tid; c < nst; c += B) {
            const uint32_t b = c ? count[c - 1] : 0u, e = count[c];
            ends[c] = (uint16_t)e;
            for (uint32_t p = b + 1; p < e; ++p) {
                const uint16_t v = mem[p];
                float vy[3];
                if constexpr (XS) xs.load(p, vy);
                uint32_t q = p;
                while (q > b && mem[q - 1] > v) {
                    mem[q] = mem[q - 1];
                    if constexpr (XS) {
                        float m[3];
                        xs.load(q - 1, m);
                        xs.store(q, m);
                    }
                    --q;
                }
                mem[q] = v;
                if constexpr (XS) xs.store(q, vy);
            }
        }
        __syncthreads();
        pc.mark<kPhSort>();
        using CellList = std::conditional_t<GH, LdsGhostCells, LdsCells>;
        const CellList cl{ends, mem};
        const uint32_t ncol = 1u << D;
        for (int rnd = 0; rnd < S.rounds; ++rnd) {
            for (uint32_t colour = 0; colour < ncol; ++colour) {
                const uint32_t select = (uint32_t)rnd * ncol + colour;
                for (int a0 = wave * tile; a0 < n_act; a0 += nwaves * tile) {
                    const int a1 = min(a0 + tile, n_act);
                    if constexpr (XS) {
                        // ghost columns make x-first order free of wrapped
                        // ranges; plain lists index y first
                        pass_tile<KIND, PREC, 1, NV, true, kWaveQueue, !GH>(S, P, pos, ori, cl, xs, colour,
                                                                            select, t, k0, k1, sh, a0,
                                                                            a1, wscr, ct, pc);
                    } else {
                        const PosXsView<D> pxs{mem, pos.p, N, sh[0], sh[1], sh[2], S.L};
                        pass_tile<KIND, PREC, 1, NV, false, kWaveQueue, true>(
                            S, P, pos, ori, cl, pxs, colour, select, t, k0, k1, sh, a0, a1, wscr, ct, pc);
                    }
                }
                pc.mark<kPhOther>();
                __syncthreads();
                pc.mark<kPhBarrier>();
            }
        }
    }
    __syncthreads();
    if constexpr (RES >= 1) {
        for (int k = tid; k < D * N; k += B) gpos[k] = pos.p[k];
    }
    if constexpr (RES >= 2) {
        for (int k = tid; k < NC * N; k += B) gori[k] = ori[k];
    }
    flush(ct, stat_stripe(stats, r));
    pc.mark<kPhOther>();
    trace_flush(pc, kTraceBatch);
}

// ---------------------------------------------------------------------------
// Host launchers.
// ---------------------------------------------------------------------------
static inline int blocks_for(long n, int b) { return (int)((n + b - 1) / b); }

size_t persistent_lds_bytes(int kind, int precision, int ncells, int n, int N, int res, int block,
                            int ghost_cap) {
    const int dim = kind == kPolyhedron ? 3 : 2;
    const int ncomp = orient_comps(kind);
    return batch_layout(dim, ncomp, N, ncells, block / 64, res, wave_scratch_words(kind, precision), n,
                        ghost_cap)
        .total;
}

hipError_t fill_u64(unsigned long long* p, unsigned long long v, size_t n, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    k_fill_u64<<<blocks_for((long)n, 256), 256, 0, stream>>>(p, v, n);
    return hipGetLastError();
}

hipError_t set_clock(const Workspace& ws, uint32_t t, uint32_t k0, uint32_t k1, uint32_t n,
                     hipStream_t stream) {
    k_set_clock<<<1, 64, 0, stream>>>(ws.clock, t, k0, k1, n);
    return hipGetLastError();
}

hipError_t set_chunk(const Workspace& ws, uint32_t n, hipStream_t stream) {
    k_set_chunk<<<1, 64, 0, stream>>>(ws.clock, n);
    return hipGetLastError();
}

hipError_t advance_clock(const Workspace& ws, hipStream_t stream) {
    k_advance_clock<<<1, 64, 0, stream>>>(ws.clock);
    return hipGetLastError();
}

hipError_t build_cells(const Workspace& ws, const int32_t* list, int count, int dim, int64_t n_max,
                       int64_t nc_max, const double* pos, int shifted, hipStream_t stream) {
    if (n_max <= kSmallBuildN && nc_max <= kSmallBuildCells) {
        if (dim == 3)
            k_build_small<3><<<count, 1024, 0, stream>>>(ws.sys, list, pos, ws.clock, shifted, ws.cell_of,
                                                        ws.slot_of, ws.start, ws.members, ws.xs);
        else
            k_build_small<2><<<count, 1024, 0, stream>>>(ws.sys, list, pos, ws.clock, shifted, ws.cell_of,
                                                        ws.slot_of, ws.start, ws.members, ws.xs);
        return hipGetLastError();
    }
    const dim3 by_cell(blocks_for(nc_max, 256), count), by_particle(blocks_for(n_max, 256), count);
    const dim3 by_tile(blocks_for(nc_max, kScanTile), count);
    // the histogram is all zero here: cleared at init and by every k_scan_apply
    if (dim == 3)
        k_assign<3><<<by_particle, 256, 0, stream>>>(ws.sys, list, pos, ws.clock, shifted, ws.count,
                                                     ws.cell_of, ws.slot_of);
    else
        k_assign<2><<<by_particle, 256, 0, stream>>>(ws.sys, list, pos, ws.clock, shifted, ws.count,
                                                     ws.cell_of, ws.slot_of);
    k_scan_tiles<<<by_tile, 256, 0, stream>>>(ws.sys, list, ws.count, ws.partial);
    k_scan_apply<<<by_tile, 256, 0, stream>>>(ws.sys, list, ws.count, ws.partial, ws.start);
    k_scatter<<<by_particle, 256, 0, stream>>>(ws.sys, list, ws.cell_of, ws.slot_of, ws.start,
                                               ws.members);
    k_sort_cells<<<by_cell, 256, 0, stream>>>(ws.sys, list, ws.start, ws.members);
    if (shifted) {
        if (dim == 3)
            k_gather_xs<3><<<by_particle, 256, 0, stream>>>(ws.sys, list, pos, ws.clock, ws.members,
                                                            ws.xs);
        else
            k_gather_xs<2><<<by_particle, 256, 0, stream>>>(ws.sys, list, pos, ws.clock, ws.members,
                                                            ws.xs);
    }
    return hipGetLastError();
}

hipError_t build_cells_one(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                           int shifted, hipStream_t stream) {
    return build_cells(ws, ws.ident + r, 1, rh.dim, rh.N, rh.ncells, pos, shifted, stream);
}

template <int KIND, int PREC, int G, int NV, int Q>
static void launch_passes_g(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                            hipStream_t stream) {
    const int cells_per_block = 4 * (64 / G);
    const uint32_t ncol = 1u << g.dim;
    const dim3 grid(blocks_for(g.n_act_max, cells_per_block), g.count);
    for (int rnd = 0; rnd < g.rounds_max; ++rnd)
        for (uint32_t colour = 0; colour < ncol; ++colour)
            k_update<KIND, PREC, G, NV, Q><<<grid, 256, 0, stream>>>(
                ws.sys, ws.species, ws.batch_list + g.first, pos, orient, ws.start, ws.members, ws.xs,
                rnd, colour, ws.clock, ws.stats);
}

template <int KIND, int PREC, int NV, int Q>
static void launch_passes_nv(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                             hipStream_t stream) {
    // 16 to 64 lanes per cell: the wave queue only (few cells per wave, so a
    // pass of a small system runs more, shorter waves)
    if constexpr (Q == kWaveQueue) {
        switch (g.lanes) {
            case 64: launch_passes_g<KIND, PREC, 64, NV, Q>(ws, g, pos, orient, stream); return;
            case 32: launch_passes_g<KIND, PREC, 32, NV, Q>(ws, g, pos, orient, stream); return;
            case 16: launch_passes_g<KIND, PREC, 16, NV, Q>(ws, g, pos, orient, stream); return;
            default: break;
        }
    }
    switch (g.lanes) {
        case 64:
        case 32:
        case 16:
        case 8: launch_passes_g<KIND, PREC, 8, NV, Q>(ws, g, pos, orient, stream); break;
        case 4: launch_passes_g<KIND, PREC, 4, NV, Q>(ws, g, pos, orient, stream); break;
        case 2: launch_passes_g<KIND, PREC, 2, NV, Q>(ws, g, pos, orient, stream); break;
        default: launch_passes_g<KIND, PREC, 1, NV, Q>(ws, g, pos, orient, stream); break;
    }
}

template <int KIND, int PREC, int NV>
static void launch_global_queue(const Workspace& ws, const BatchGroup& g, double* pos,
                                double* orient, hipStream_t stream) {
    const uint32_t ncol = 1u << g.dim;
    const dim3 by_cell(blocks_for(g.n_act_max, 256), g.count);
    const int64_t cap = g.n_max << g.dim;
    const dim3 by_entry((unsigned)std::min<int64_t>(blocks_for(cap, 256), 4096), g.count);
    const int32_t* list = ws.batch_list + g.first;
    for (int rnd = 0; rnd < g.rounds_max; ++rnd)
        for (uint32_t colour = 0; colour < ncol; ++colour) {
            k_gq_scan<KIND><<<by_cell, 256, 0, stream>>>(ws.sys, ws.species, list, pos, orient,
                                                         ws.start, ws.members, ws.xs, rnd, colour,
                                                         ws.clock, ws.gq, ws.stats);
            k_gq_test<KIND, PREC, NV><<<by_entry, 256, 0, stream>>>(ws.sys, ws.species, list, pos,
                                                                    orient, ws.members, rnd, ws.gq,
                                                                    ws.stats);
            k_gq_apply<KIND><<<by_cell, 256, 0, stream>>>(ws.sys, list, pos, orient, ws.xs, rnd,
                                                          ws.clock, ws.gq, ws.stats);
        }
}

template <int KIND, int PREC, int NV>
static void launch_passes_q(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                            int queue, hipStream_t stream) {
    if constexpr (KIND == kSpheropolygon) {  // the wave queue only (checked at init)
        launch_passes_nv<KIND, PREC, NV, kWaveQueue>(ws, g, pos, orient, stream);
        return;
    }
    if (queue == kQueueGlobal)
        launch_global_queue<KIND, PREC, NV>(ws, g, pos, orient, stream);
    else if (queue == kQueueRegister)
        launch_passes_nv<KIND, PREC, NV, kRegisterQueue>(ws, g, pos, orient, stream);
    else
        launch_passes_nv<KIND, PREC, NV, kWaveQueue>(ws, g, pos, orient, stream);
}

template <int KIND, int PREC>
static void launch_passes(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                          int queue, hipStream_t stream) {
    if (KIND == kPolygon && g.nv == 5)
        launch_passes_q<KIND, PREC, 5>(ws, g, pos, orient, queue, stream);
    else
        launch_passes_q<KIND, PREC, 0>(ws, g, pos, orient, queue, stream);
}

hipError_t grid_passes(const Workspace& ws, const BatchGroup& g, double* pos, double* orient,
                       int precision, int queue, hipStream_t stream) {
    if (g.kind == kDisk)
        launch_passes<kDisk, 0>(ws, g, pos, orient, queue, stream);
    else if (g.kind == kPolygon && precision == 1)
        launch_passes<kPolygon, 1>(ws, g, pos, orient, queue, stream);
    else if (g.kind == kPolygon)
        launch_passes<kPolygon, 0>(ws, g, pos, orient, queue, stream);
    else if (g.kind == kSpheropolygon)
        launch_passes<kSpheropolygon, 0>(ws, g, pos, orient, queue, stream);
    else if (precision == 1)
        launch_passes<kPolyhedron, 1>(ws, g, pos, orient, queue, stream);
    else
        launch_passes<kPolyhedron, 0>(ws, g, pos, orient, queue, stream);
    return hipGetLastError();
}

template <int KIND, int PREC, int RES, int NV, bool GH = false>
static hipError_t launch_batch(const Workspace& ws, const int32_t* list, int n, int block, size_t lds,
                               double* pos, double* orient, bool prepare, hipStream_t stream) {
    auto kern = k_batch<KIND, PREC, RES, NV, GH>;
    if (prepare)  // raise the dynamic-LDS limit (not a stream operation; done before capture)
        return hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)lds);
    if (block < 64 || block > kBatchBlock || block % 64 != 0) return hipErrorInvalidValue;
    kern<<<n, block, lds, stream>>>(ws.sys, ws.species, list, pos, orient, ws.stats, ws.clock);
    return hipGetLastError();
}

template <int KIND, int PREC, int NV>
static hipError_t launch_batch_res(const Workspace& ws, const BatchGroup& g, double* pos,
                                   double* orient, bool prepare, hipStream_t stream) {
    const int32_t* list = ws.batch_list + g.first;
    if constexpr (KIND != kPolyhedron) {
        // 2D kinds keep ghost edge columns at the levels where they fit
        if ((g.ghost >> g.resident) & 1) {
            if (g.resident == 2 && KIND != kDisk)
                return launch_batch<KIND, PREC, 2, NV, true>(ws, list, g.count, g.block, g.lds_bytes, pos,
                                                             orient, prepare, stream);
            if (g.resident >= 1)
                return launch_batch<KIND, PREC, 1, NV, true>(ws, list, g.count, g.block, g.lds_bytes, pos,
                                                             orient, prepare, stream);
            return launch_batch<KIND, PREC, 0, NV, true>(ws, list, g.count, g.block, g.lds_bytes, pos,
                                                         orient, prepare, stream);
        }
    }
    if (g.resident >= 3)
        return launch_batch<KIND, PREC, 3, NV>(ws, list, g.count, g.block, g.lds_bytes, pos, orient,
                                               prepare, stream);
    if (g.resident >= 2 && KIND != kDisk)
        return launch_batch<KIND, PREC, 2, NV>(ws, list, g.count, g.block, g.lds_bytes, pos, orient,
                                               prepare, stream);
    if (g.resident >= 1)
        return launch_batch<KIND, PREC, 1, NV>(ws, list, g.count, g.block, g.lds_bytes, pos, orient,
                                               prepare, stream);
    return launch_batch<KIND, PREC, 0, NV>(ws, list, g.count, g.block, g.lds_bytes, pos, orient,
                                           prepare, stream);
}

hipError_t persistent_sweeps(const Workspace& ws, const BatchGroup& g, double* pos,
                             double* orient, int precision, bool prepare, hipStream_t stream) {
    if (g.kind == kDisk)
        return launch_batch_res<kDisk, 0, 0>(ws, g, pos, orient, prepare, stream);
    if (g.kind == kPolygon) {
        if (precision == 1)
            return g.nv == 5 ? launch_batch_res<kPolygon, 1, 5>(ws, g, pos, orient, prepare, stream)
                             : launch_batch_res<kPolygon, 1, 0>(ws, g, pos, orient, prepare, stream);
        return g.nv == 5 ? launch_batch_res<kPolygon, 0, 5>(ws, g, pos, orient, prepare, stream)
                         : launch_batch_res<kPolygon, 0, 0>(ws, g, pos, orient, prepare, stream);
    }
    if (g.kind == kSpheropolygon)
        return launch_batch_res<kSpheropolygon, 0, 0>(ws, g, pos, orient, prepare, stream);
    if (precision == 1)
        return launch_batch_res<kPolyhedron, 1, 0>(ws, g, pos, orient, prepare, stream);
    return launch_batch_res<kPolyhedron, 0, 0>(ws, g, pos, orient, prepare, stream);
}

hipError_t pair_histogram(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                          int n_bins, int reach, hipStream_t stream) {
    const int N = rh.N;
    hipError_t e = fill_u64(ws.hist_out, 0ull, (size_t)n_bins, stream);
    if (e != hipSuccess) return e;
    if (rh.dim == 3)
        k_pair_hist<3><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, ws.start, ws.members,
                                                               ws.cell_of, ws.hist_edges, n_bins,
                                                               reach, ws.hist_out);
    else
        k_pair_hist<2><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, ws.start, ws.members,
                                                               ws.cell_of, ws.hist_edges, n_bins,
                                                               reach, ws.hist_out);
    return hipGetLastError();
}

hipError_t scale_counts(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                        const double* orient, int n_s, int reach, hipStream_t stream) {
    const int N = rh.N;
    hipError_t e = fill_u64(ws.hist_out, 0ull, (size_t)n_s, stream);
    if (e != hipSuccess) return e;
    const dim3 grid(blocks_for(N, 256));
    if (rh.kind == kDisk)
        k_scale_count<kDisk><<<grid, 256, 0, stream>>>(ws.sys, ws.species, r, pos, orient, ws.start,
                                                       ws.members, ws.cell_of, ws.hist_edges, n_s,
                                                       reach, ws.hist_out);
    else if (rh.kind == kPolygon)
        k_scale_count<kPolygon><<<grid, 256, 0, stream>>>(ws.sys, ws.species, r, pos, orient,
                                                          ws.start, ws.members, ws.cell_of,
                                                          ws.hist_edges, n_s, reach, ws.hist_out);
    else if (rh.kind == kSpheropolygon)
        k_scale_count<kSpheropolygon><<<grid, 256, 0, stream>>>(ws.sys, ws.species, r, pos, orient,
                                                                ws.start, ws.members, ws.cell_of,
                                                                ws.hist_edges, n_s, reach, ws.hist_out);
    else
        k_scale_count<kPolyhedron><<<grid, 256, 0, stream>>>(ws.sys, ws.species, r, pos, orient,
                                                             ws.start, ws.members, ws.cell_of,
                                                             ws.hist_edges, n_s, reach, ws.hist_out);
    return hipGetLastError();
}

// Isotropic box change: x -> x k, wrapped into [0, L_new).
__global__ void __launch_bounds__(256) k_scale_box(double* __restrict__ p, int64_t n, double k,
                                                   double L_new) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = p[i] * k;
    double y = x;
    if (x >= L_new)
        y = x - L_new;
    else if (x < 0.0)
        y = x + L_new;
    if (y >= L_new) y = 0.0;
    p[i] = y;
}

hipError_t scale_box(double* pos, int64_t n, double k, double L_new, hipStream_t stream) {
    if (n == 0) return hipSuccess;
    k_scale_box<<<blocks_for(n, 256), 256, 0, stream>>>(pos, n, k, L_new);
    return hipGetLastError();
}

hipError_t validate_state(const Workspace& ws, const ReplicaHost& rh, int r, const double* pos,
                          const double* orient, hipStream_t stream) {
    const int N = rh.N;
    if (rh.kind == kDisk)
        k_validate<0><<<blocks_for(N, 256), 256, 0, stream>>>(ws.sys, r, pos, orient, ws.overlap_out);
    else if (rh.kind == kPolygon || rh.kind == kSpheropolygon)
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
    else if (rh.kind == kSpheropolygon)
        k_count<kSpheropolygon><<<blocks_for(N, 256), 256, 0, stream>>>(
            ws.sys, ws.species, r, pos, orient, ws.start, ws.members, ws.cell_of, ws.overlap_out);
    else
        k_count<kPolyhedron><<<blocks_for(N, 256), 256, 0, stream>>>(
            ws.sys, ws.species, r, pos, orient, ws.start, ws.members, ws.cell_of, ws.overlap_out);
    return hipGetLastError();
}

}  // namespace hpmc
