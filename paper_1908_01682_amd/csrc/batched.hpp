// Batched form: many independent problems (different N, t_stop, dust-to-gas
// ratio, cell count) advanced n_steps in ONE persistent launch.
//
// Each workgroup owns one problem instance for the whole launch and runs the
// full IDIC step (bin -> density -> predictor -> cell solve -> update) with
// block barriers between the phases.  No workgroup ever waits on another, so
// the launch cannot deadlock whatever the residency.  Instances are dispatched
// largest first (longest-processing-time order) so that the big ones start
// early.  Every per-particle and per-cell computation calls the same device
// functions as the single-problem kernels, so an instance evolves bitwise as
// it would alone through tfsph_step.
#pragma once

#include "binning.hpp"
#include "sph.hpp"

namespace tfsph {

constexpr int kBatchMaxBlock = 1024;

template <typename R>
struct Inst {
    Geom<R> G;
    Phys<R> Ph;
    Phase<R> Pg, Pd;     // caller arrays of this instance (slices of the packed state)
    Sorted<R> Sg, Sd;    // workspace slices
    CellSolve<R> *cs;    // [ncell] per-cell solve
};

// exclusive scan of one int per thread for any blockDim.x <= 1024 (wave64)
__device__ __forceinline__ int block_scan_any(int v, int *lds_waves, int &total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int nwaves = (blockDim.x + 63) >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    int pre = 0;
    total = 0;
    for (int w = 0; w < nwaves; ++w) {
        const int t = lds_waves[w];
        if (w < wave) pre += t;
        total += t;
    }
    __syncthreads();
    return pre + x - v;
}

// start[c] = sum of count[0..c), start[ncell] = total, for one instance: each
// thread sums a contiguous run of cells, one block scan combines the runs.
// The run's counts are loaded kRunLoad at a time with every load issued before
// the sum uses it, so a run costs a few memory latencies, not one per cell; a
// run of at most kRunLoad cells keeps its counts in registers for the second
// pass.
constexpr int kRunLoad = 16;
__device__ __forceinline__ void block_scan_cells(const int *count, int *start, int ncell, int *lds)
{
    const int per = (ncell + blockDim.x - 1) / blockDim.x;
    const int c0 = min(int(threadIdx.x) * per, ncell), c1 = min(c0 + per, ncell);
    int v[kRunLoad];
    int s = 0;
    for (int c = c0; c < c1; c += kRunLoad) {
#pragma unroll
        for (int u = 0; u < kRunLoad; ++u) v[u] = c + u < c1 ? count[c + u] : 0;
#pragma unroll
        for (int u = 0; u < kRunLoad; ++u) s += v[u];
    }
    int total;
    int ex = block_scan_any(s, lds, total);
    const bool held = per <= kRunLoad;     // v[] still holds the run's counts
    for (int c = c0; c < c1; c += kRunLoad) {
        if (!held) {
#pragma unroll
            for (int u = 0; u < kRunLoad; ++u) v[u] = c + u < c1 ? count[c + u] : 0;
        }
#pragma unroll
        for (int u = 0; u < kRunLoad; ++u) {
            if (c + u < c1) start[c + u] = ex;
            ex += v[u];
        }
    }
    if (threadIdx.x == 0) start[ncell] = total;
}

// One IDIC step of instance I by the whole block.  Slots for the next step's
// counting sort are claimed while the particles are finished (the new cell is
// known there); `first` does the counting from scratch for the first step of
// a launch, since the state may have been written outside this kernel.
template <typename R, int DIM>
__device__ __forceinline__ void batched_step(const Inst<R> &I, int *lds, unsigned int *flags, int &bad, int &one,
                                             R &s2, bool first)
{
    const int tid = threadIdx.x, nt = blockDim.x;
    const Geom<R> &G = I.G;
    const int ncell = G.ncell;
    const int ng = I.Sg.n, nd = I.Sd.n;

    if (first) {
        for (int c = tid; c < ncell; c += nt) {
            I.Sg.count[c] = 0;
            I.Sd.count[c] = 0;
        }
        __syncthreads();
        // loop bounds are uniform across each wave (claim_slot shuffles)
        for (int base = 0; base < ng; base += nt) {
            const int i = base + tid;
            const int key = i < ng ? safe_cell(I.Pg.cell[i], ncell) : -1;
            const int sl = claim_slot(I.Sg.count, key);
            if (i < ng) I.Sg.slot[i] = sl;
        }
        for (int base = 0; base < nd; base += nt) {
            const int i = base + tid;
            const int key = i < nd ? safe_cell(I.Pd.cell[i], ncell) : -1;
            const int sl = claim_slot(I.Sd.count, key);
            if (i < nd) I.Sd.slot[i] = sl;
        }
        __syncthreads();
    }
    block_scan_cells(I.Sg.count, I.Sg.start, ncell, lds);
    block_scan_cells(I.Sd.count, I.Sd.start, ncell, lds);
    __syncthreads();
    for (int i = tid; i < ng; i += nt) {
        const int pos = I.Sg.start[safe_cell(I.Pg.cell[i], ncell)] + I.Sg.slot[i];
        I.Sg.tmp_idx[pos] = i;
        I.Sg.tmp_id[pos] = I.Pg.id[i];
    }
    for (int i = tid; i < nd; i += nt) {
        const int pos = I.Sd.start[safe_cell(I.Pd.cell[i], ncell)] + I.Sd.slot[i];
        I.Sd.tmp_idx[pos] = i;
        I.Sd.tmp_id[pos] = I.Pd.id[i];
    }
    for (int c = tid; c < ncell; c += nt) {       // counts are consumed: clear for the claims below
        I.Sg.count[c] = 0;
        I.Sd.count[c] = 0;
    }
    __syncthreads();
    for (int j = tid; j < ng; j += nt) rank_gather_one(G, I.Pg, I.Sg, j, flags);
    for (int j = tid; j < nd; j += nt) rank_gather_one(G, I.Pd, I.Sd, j, flags);
    __syncthreads();
    for (int a = tid; a < ng; a += nt) density_store<R, DIM>(G, I.Ph, I.Sg, a, 1);
    __syncthreads();
    for (int a = tid; a < ng; a += nt) gas_predict<R, DIM>(G, I.Ph, I.Sg, I.Pg, a);
    __syncthreads();
    for (int c = tid; c < ncell; c += nt) one += solve_cell<R, DIM>(I.Ph, I.Sg, I.Sd, c, I.cs[c]) ? 1 : 0;
    __syncthreads();
    for (int base = 0; base < ng; base += nt) {
        const int a = base + tid;
        int key = -1;
        if (a < ng) {
            bad |= !gas_finish<R, DIM>(G, I.Ph, I.Sg, I.Pg, a, I.cs[I.Sg.cell[a]], s2, nullptr, &key);
        }
        const int sl = claim_slot(I.Sg.count, key);
        if (a < ng) I.Sg.slot[a] = sl;
    }
    for (int base = 0; base < nd; base += nt) {
        const int j = base + tid;
        int key = -1;
        if (j < nd) {
            bad |= !dust_finish<R, DIM>(G, I.Ph, I.Sd, I.Pd, j, I.cs[I.Sd.cell[j]], s2, nullptr, &key);
        }
        const int sl = claim_slot(I.Sd.count, key);
        if (j < nd) I.Sd.slot[j] = sl;
    }
    __syncthreads();
}

// grid = number of instances; block b advances instance order[b] by n_steps
template <typename R, int DIM>
__global__ void __launch_bounds__(kBatchMaxBlock)
k_batched(const Inst<R> *__restrict__ insts, const int *__restrict__ order, int n_steps, Flags F)
{
    __shared__ int lds[kBatchMaxBlock / 64];
    __shared__ int s_bad, s_one;
    if (threadIdx.x == 0) { s_bad = 0; s_one = 0; }
    const Inst<R> &I = insts[order[blockIdx.x]];
    int bad = 0, one = 0;
    R s2 = signal_floor(I.Ph);
    for (int s = 0; s < n_steps; ++s) batched_step<R, DIM>(I, lds, F.word, bad, one, s2, s == 0);
    if (I.Ph.vlim2 > R(0) && s2 > I.Ph.vlim2) atomicOr(F.word, kFlagCfl);
    if (bad) atomicOr(&s_bad, 1);
    if (one) atomicAdd(&s_one, one);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_bad) atomicOr(F.word, 1u);
        if (s_one) {
            atomicOr(F.word, 2u);
            atomicAdd(F.one_phase, (unsigned long long)s_one);
        }
    }
}

// ---------------------------------------------------------------------------
// Flattened form: one launch per phase of the step covers every instance.  The
// blocks of a launch are dealt out per instance, so a block never straddles two
// instances: a table gives each block of a launch its instance and its block
// index inside that instance's items (gas particles, dust particles or cells,
// kBlock items per block), one 8-byte scalar load per block (a search over the
// instances' first blocks would be a chain of dependent loads at the start of
// every block).  Each item calls the same device functions as the
// single-problem kernels and the persistent kernel, so every instance evolves
// bitwise as it does through tfsph_step.  The launch time is that of the whole
// batch's work spread over the chip, not that of its largest instance.
// ---------------------------------------------------------------------------
struct FlatTable {
    int n_inst;
    int blocks_g;            // blocks over gas particles: the first blocks of a launch over both phases
    const int2 *part;        // [blocks_g + blocks_d] (instance, block in the instance): gas, then dust
    const int2 *cells;       // [blocks_c] the same over cells, cells_per_block cells per block
    int cells_per_block;
};

// Item index of this thread inside its instance, for a launch over gas blocks
// then dust blocks (gas = true for the first blocks_g blocks).
__device__ __forceinline__ int flat_item(const FlatTable &T, bool &gas, int &inst)
{
    const int2 e = T.part[blockIdx.x];
    gas = int(blockIdx.x) < T.blocks_g;
    inst = e.x;
    return e.y * kBlock + int(threadIdx.x);
}

__device__ __forceinline__ int flat_cell_item(const FlatTable &T, int &inst)
{
    const int2 e = T.cells[blockIdx.x];
    inst = e.x;
    const int c = int(threadIdx.x) < T.cells_per_block ? int(threadIdx.x) : 1 << 30;
    return e.y * T.cells_per_block + c;
}

// clear both histograms (the first step of a call counts from the caller's arrays)
template <typename R>
__global__ void __launch_bounds__(kBlock) k_flat_zero(const Inst<R> *__restrict__ insts, FlatTable T)
{
    int i;
    const int c = flat_cell_item(T, i);
    const Inst<R> &I = insts[i];
    if (c < I.G.ncell) {
        I.Sg.count[c] = 0;
        I.Sd.count[c] = 0;
    }
}

// histogram + slot claims from the caller's arrays
template <typename R>
__global__ void __launch_bounds__(kBlock) k_flat_count(const Inst<R> *__restrict__ insts, FlatTable T)
{
    bool gas;
    int inst;
    const int i = flat_item(T, gas, inst);
    const Inst<R> &I = insts[inst];
    const Phase<R> &P = gas ? I.Pg : I.Pd;
    const Sorted<R> &S = gas ? I.Sg : I.Sd;
    const int key = i < S.n ? safe_cell(P.cell[i], I.G.ncell) : -1;     // every lane claims (wave shuffles)
    const int sl = claim_slot(S.count, key);
    if (i < S.n) S.slot[i] = sl;
}

// exclusive scan of each instance's histograms, one block per instance and phase,
// in tiles of kFlatScanPer cells per thread staged in LDS: the counts are read (and
// cleared) and the offsets written with coalesced accesses, each thread sums a run
// of kFlatScanPer cells of the tile, and a running prefix carries over the tiles
constexpr int kFlatScanPer = 8;
template <typename R>
__global__ void __launch_bounds__(kBatchMaxBlock) k_flat_scan(const Inst<R> *__restrict__ insts)
{
    __shared__ int lds[kBatchMaxBlock / 64];
    __shared__ int tile[kBatchMaxBlock * kFlatScanPer];
    const Inst<R> &I = insts[blockIdx.x >> 1];
    const Sorted<R> &S = (blockIdx.x & 1) ? I.Sd : I.Sg;
    const int ncell = I.G.ncell;
    const int t = int(threadIdx.x);
    constexpr int kTile = kBatchMaxBlock * kFlatScanPer;
    int prefix = 0;
    for (int base = 0; base < ncell; base += kTile) {
#pragma unroll
        for (int k = 0; k < kFlatScanPer; ++k) {
            const int c = base + k * kBatchMaxBlock + t;
            int v = 0;
            if (c < ncell) {
                v = S.count[c];
                S.count[c] = 0;     // consumed: zero for the next step's claims
            }
            tile[k * kBatchMaxBlock + t] = v;
        }
        __syncthreads();
        int loc[kFlatScanPer];
        int run = 0;
#pragma unroll
        for (int k = 0; k < kFlatScanPer; ++k) {
            loc[k] = run;
            run += tile[t * kFlatScanPer + k];
        }
        int total;
        const int ex = block_scan_any(run, lds, total) + prefix;
#pragma unroll
        for (int k = 0; k < kFlatScanPer; ++k) tile[t * kFlatScanPer + k] = ex + loc[k];
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kFlatScanPer; ++k) {
            const int c = base + k * kBatchMaxBlock + t;
            if (c < ncell) S.start[c] = tile[k * kBatchMaxBlock + t];
        }
        prefix += total;
        __syncthreads();        // the next tile overwrites tile[]
    }
    if (t == 0) S.start[ncell] = prefix;
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_flat_scatter(const Inst<R> *__restrict__ insts, FlatTable T)
{
    bool gas;
    int inst;
    const int i = flat_item(T, gas, inst);
    const Inst<R> &I = insts[inst];
    const Phase<R> &P = gas ? I.Pg : I.Pd;
    const Sorted<R> &S = gas ? I.Sg : I.Sd;
    if (i >= S.n) return;
    const int pos = S.start[safe_cell(P.cell[i], I.G.ncell)] + S.slot[i];
    S.tmp_idx[pos] = i;
    S.tmp_id[pos] = P.id[i];
}

template <typename R>
__global__ void __launch_bounds__(kBlock) k_flat_rank_gather(const Inst<R> *__restrict__ insts, FlatTable T,
                                                             unsigned int *flags)
{
    bool gas;
    int inst;
    const int j = flat_item(T, gas, inst);
    const Inst<R> &I = insts[inst];
    const Sorted<R> &S = gas ? I.Sg : I.Sd;
    if (j < S.n) rank_gather_one(I.G, gas ? I.Pg : I.Pd, S, j, flags);
}

template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock) k_flat_density(const Inst<R> *__restrict__ insts, FlatTable T)
{
    const int2 e = T.part[blockIdx.x];
    const Inst<R> &I = insts[e.x];
    const int a = e.y * kBlock + int(threadIdx.x);
    if (a < I.Sg.n) density_store<R, DIM>(I.G, I.Ph, I.Sg, a, 1);
}

// KIND: the force-loop kind (kForce*) when every instance has the same one, so
// the kernel holds the registers of that loop only (in 1D the isothermal loops
// need 64 VGPRs against about 100 for the general one); -1 picks each
// instance's kind at run time.  Either way an instance runs the loop that
// tfsph_step runs for it.
template <typename R, int DIM, int KIND>
__global__ void __launch_bounds__(kBlock) k_flat_predict(const Inst<R> *__restrict__ insts, FlatTable T)
{
    const int2 e = T.part[blockIdx.x];
    const Inst<R> &I = insts[e.x];
    const int a = e.y * kBlock + int(threadIdx.x);
    if (a < I.Sg.n) gas_predict<R, DIM, KIND>(I.G, I.Ph, I.Sg, I.Pg, a);
}

// cell sums, implicit solve, particle update, move and carry of a run of
// kFlatCells cells of one instance (the single-problem update kernel's block),
// with the slot claims of the next step's counting sort
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1)))
k_flat_update(const Inst<R> *__restrict__ insts, FlatTable T, Flags F)
{
    extern __shared__ unsigned char smem_raw[];
    const int2 e = T.cells[blockIdx.x];
    const Inst<R> &I = insts[e.x];
    const int c0 = e.y * T.cells_per_block;
    const int c1 = min(c0 + T.cells_per_block, I.G.ncell);
    update_block<R, DIM, true>(I.G, I.Ph, I.Sg, I.Sd, I.Pg, I.Pd, F, c0, c1, smem_raw);
}

}  // namespace tfsph
