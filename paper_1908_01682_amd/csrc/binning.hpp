// Binning of particles into the drag volumes (Section 2.3: the region is split
// into disjoint volumes at each time instant) as a deterministic counting sort.
//
//   count    : slot_i = atomicAdd(count[cell_i], 1)       (integer, any order)
//   scan     : start = exclusive prefix sum of count        (2 or 3 launches, integer)
//   scatter  : tmp[start[c] + slot_i] = (i, id_i)          (unordered inside a cell)
//   rank     : final position = start[c] + #{k in cell c : id_k < id_i}
//              and every field of particle i is gathered to it
//
// The final order is lexicographic (cell, id), independent of the order in
// which the atomics were served, so the whole sort is bitwise reproducible.
#pragma once

#include "common.hpp"

namespace tfsph {

constexpr int kScanItems = 8;                      // items per thread in a scan tile
constexpr int kScanTile = kBlock * kScanItems;     // 2048 cells per tile

// --- carry every offset of a phase into its cell (initial canonical form) ----
template <typename R>
__global__ void __launch_bounds__(kBlock) k_canonicalize(Geom<R> G, Phase<R> P, Flags F)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= P.n) return;
    int c[3];
    int lin = P.cell[i];
    bool ok = lin >= 0 && lin < G.ncell;
    if (!ok) lin = 0;
    split_cell(G, lin, c[0], c[1], c[2]);
    for (int d = 0; d < G.dim; ++d) {
        R o = P.off[d][i];
        ok &= carry(o, c[d], G.delta[d], G.nc[d]);
        P.off[d][i] = o;
    }
    P.cell[i] = join_cell(G, c[0], c[1], c[2]);
    if (!ok) atomicOr(F.word, 1u);
}

// --- zero the histograms of both phases ---------------------------------------
static __global__ void __launch_bounds__(kBlock) k_fill_zero(int *a, int na, int *b, int nb)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < na) a[i] = 0;
    if (i < nb) b[i] = 0;
}

// --- histogram + slot claim (both phases in one grid) ---------------------------
// Lanes of a wave usually hold a few runs of equal cell keys (the arrays are in
// the previous step's cell order), so each run claims its slots with one atomic
// issued by its first lane; slot = base + position inside the run.
__device__ __forceinline__ int claim_slot(int *count, int key)
{
    const int lane = threadIdx.x & 63;
    const int prev = __shfl_up(key, 1, 64);
    const bool head = lane == 0 || key != prev;
    int s = head ? lane : 0;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int t = __shfl_up(s, off, 64);
        if (lane >= off) s = max(s, t);
    }
    const unsigned long long heads = __ballot(head);
    const unsigned long long above = s == 63 ? 0ull : (heads & ~((2ull << s) - 1ull));
    const int next = above ? __ffsll((long long)above) - 1 : 64;
    int base = 0;
    if (head && key >= 0) base = atomicAdd(count + key, next - s);
    base = __shfl(base, s, 64);
    return base + (lane - s);
}

static __global__ void __launch_bounds__(kBlock)
k_count(const int *cell_g, int n_g, int *count_g, int *slot_g,
        const int *cell_d, int n_d, int *count_d, int *slot_d, int blocks_g, int ncell, unsigned int *flags)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int i = (gas ? blockIdx.x : blockIdx.x - blocks_g) * kBlock + threadIdx.x;
    const int n = gas ? n_g : n_d;
    int key = -1;
    if (i < n) {
        const int raw = gas ? cell_g[i] : cell_d[i];
        key = safe_cell(raw, ncell);
        if (key != raw) atomicOr(flags, 4u);
    }
    const int s = claim_slot(gas ? count_g : count_d, key);
    if (i < n) (gas ? slot_g : slot_d)[i] = s;
}

// --- block-wide exclusive scan of one int per thread (256 threads, wave64) ----
__device__ __forceinline__ int block_exclusive_scan(int v, int *lds_waves, int &total)
{
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    int x = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int y = __shfl_up(x, off, 64);
        if (lane >= off) x += y;
    }
    if (lane == 63) lds_waves[wave] = x;
    __syncthreads();
    int wave_prefix = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < kBlock / 64; ++w) {
        const int t = lds_waves[w];
        if (w < wave) wave_prefix += t;
        total += t;
    }
    __syncthreads();
    return wave_prefix + x - v;
}

// tile sums: grid (tiles, 2 phases)
static __global__ void __launch_bounds__(kBlock)
k_scan_reduce(const int *count_g, const int *count_d, int ncell, int *partial, int ntiles)
{
    const int *count = blockIdx.y == 0 ? count_g : count_d;
    const int base = blockIdx.x * kScanTile;
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        if (i < ncell) s += count[i];
    }
    __shared__ int lds[kBlock / 64];
    int total;
    block_exclusive_scan(s, lds, total);
    if (threadIdx.x == 0) partial[blockIdx.y * ntiles + blockIdx.x] = total;
}

// exclusive scan of the tile sums, one block per phase; writes start[ncell] = n
static __global__ void __launch_bounds__(kBlock)
k_scan_top(int *partial, int ntiles, int *start_g, int *start_d, int ncell)
{
    int *p = partial + blockIdx.y * ntiles;
    __shared__ int lds[kBlock / 64];
    int carry_in = 0;
    for (int base = 0; base < ntiles; base += kBlock) {
        const int i = base + threadIdx.x;
        const int v = i < ntiles ? p[i] : 0;
        int total;
        const int ex = block_exclusive_scan(v, lds, total);
        if (i < ntiles) p[i] = carry_in + ex;
        carry_in += total;
    }
    if (threadIdx.x == 0) (blockIdx.y == 0 ? start_g : start_d)[ncell] = carry_in;
}

// at most this many tiles: k_scan_down sums the preceding tile totals itself
// and k_scan_top is not launched
constexpr int kScanInlineTiles = 4 * kBlock;

// per-tile exclusive scan plus tile prefix -> start[], and the counts reset to
// zero (every count array is zero between binnings: cleared once when its
// workspace is set up, then here).  With `inline_prefix`
// the prefix is the sum of the raw tile totals of the tiles before this one
// (and the last tile writes start[ncell]); otherwise k_scan_top has turned
// partial[] into exclusive prefixes.
static __global__ void __launch_bounds__(kBlock)
k_scan_down(const int *count_g, const int *count_d, int ncell, const int *partial, int ntiles, int *start_g,
            int *start_d, int inline_prefix)
{
    const int *count = blockIdx.y == 0 ? count_g : count_d;
    int *start = blockIdx.y == 0 ? start_g : start_d;
    const int base = blockIdx.x * kScanTile;
    __shared__ int tile[kScanTile];
    __shared__ int lds[kBlock / 64];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        tile[k * kBlock + threadIdx.x] = i < ncell ? count[i] : 0;
        // the counts are consumed here: leave them zero for the next binning's claims
        if (i < ncell) const_cast<int *>(count)[i] = 0;
    }
    int prefix = 0;
    if (inline_prefix) {
        int s = 0;
        for (int t = threadIdx.x; t < (int)blockIdx.x; t += kBlock) s += partial[blockIdx.y * ntiles + t];
        int total;
        block_exclusive_scan(s, lds, total);
        prefix = total;
    } else {
        prefix = partial[blockIdx.y * ntiles + blockIdx.x];
    }
    __syncthreads();
    int loc[kScanItems];
    int s = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        loc[k] = s;
        s += tile[threadIdx.x * kScanItems + k];
    }
    int total;
    const int ex = block_exclusive_scan(s, lds, total) + prefix;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) tile[threadIdx.x * kScanItems + k] = ex + loc[k];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int i = base + k * kBlock + threadIdx.x;
        if (i < ncell) start[i] = tile[k * kBlock + threadIdx.x];
    }
    if (inline_prefix && blockIdx.x == (unsigned)ntiles - 1 && threadIdx.x == 0) start[ncell] = prefix + total;
}

// --- scatter (index, id) into cell ranges ----------------------------------------
static __global__ void __launch_bounds__(kBlock)
k_scatter(const int *cell_g, const int *id_g, const int *slot_g, const int *start_g, int n_g, int *idx_g, int *tid_g,
          const int *cell_d, const int *id_d, const int *slot_d, const int *start_d, int n_d, int *idx_d, int *tid_d,
          int blocks_g, int ncell)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int i = (gas ? blockIdx.x : blockIdx.x - blocks_g) * kBlock + threadIdx.x;
    if (i >= (gas ? n_g : n_d)) return;
    const int c = safe_cell(gas ? cell_g[i] : cell_d[i], ncell);
    const int pos = (gas ? start_g : start_d)[c] + (gas ? slot_g : slot_d)[i];
    (gas ? idx_g : idx_d)[pos] = i;
    (gas ? tid_g : tid_d)[pos] = gas ? id_g[i] : id_d[i];
}

// --- rank by id inside the cell and gather every field ---------------------------
template <typename R>
__device__ __forceinline__ void rank_gather_one(const Geom<R> &G, const Phase<R> &P, const Sorted<R> &S, int j,
                                                unsigned int *flags)
{
    const int i = S.tmp_idx[j];
    const int myid = S.tmp_id[j];
    const int c = safe_cell(P.cell[i], G.ncell);
    // the fields to gather depend on i alone: their loads go out before the rank loop
    R o[3] = {R(0), R(0), R(0)}, v[3] = {R(0), R(0), R(0)};
    for (int d = 0; d < G.dim; ++d) {
        o[d] = P.off[d][i];
        v[d] = P.vel[d][i];
    }
    const R m = P.mass ? P.mass[i] : P.m_uniform;
    const R en = S.energy ? P.energy[i] : R(0);
    const int b = S.start[c];
    const int e = S.start[c + 1];
    int rank = 0;
    if (e - b <= kMaxRankCell) {
        for (int k = b; k < e; k += kChunk) {
            int t[kChunk];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) t[u] = S.tmp_id[min(k + u, e - 1)];
#pragma unroll
            for (int u = 0; u < kChunk; ++u) rank += (k + u < e && t[u] < myid) ? 1 : 0;
        }
    } else {
        rank = j - b;
        atomicOr(flags, 8u);
    }
    const int dst = b + rank;
    if (S.src) S.src[dst] = i;
    S.cell[dst] = c;
    S.id[dst] = myid;
    for (int d = 0; d < G.dim; ++d) S.vel[d][dst] = v[d];
    S.pos[dst] = mk4<R>(o[0], o[1], o[2], m);
    if (S.energy) S.energy[dst] = en;
    if (j == 0) {
        // the pair loops read up to kPad records past the end: keep them finite
        for (int k = 0; k < kPad; ++k) {
            S.pos[S.n + k] = mk4<R>(R(0), R(0), R(0), R(0));
            if (S.frc) S.frc[S.n + k] = mk4<R>(R(0), R(0), R(0), R(0));
        }
    }
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_rank_gather(Geom<R> G, Phase<R> Pg, Sorted<R> Sg, Phase<R> Pd, Sorted<R> Sd, int blocks_g, unsigned int *flags)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int j = (gas ? blockIdx.x : blockIdx.x - blocks_g) * kBlock + threadIdx.x;
    if (gas) {
        if (j < Sg.n) rank_gather_one(G, Pg, Sg, j, flags);
    } else {
        if (j < Sd.n) rank_gather_one(G, Pd, Sd, j, flags);
    }
}

// --- copy the sorted workspace back to the caller's arrays -------------------------
template <typename R>
__global__ void __launch_bounds__(kBlock) k_copy_back(Geom<R> G, Sorted<R> S, Phase<R> P, int with_rho)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= S.n) return;
    P.cell[j] = S.cell[j];
    P.id[j] = S.id[j];
    const R4<R> q = S.pos[j];
    const R o[3] = {q.x, q.y, q.z};
    for (int d = 0; d < G.dim; ++d) {
        P.off[d][j] = o[d];
        P.vel[d][j] = S.vel[d][j];
    }
    if (S.has_mass && P.mass) const_cast<R *>(P.mass)[j] = q.w;
    if (S.energy) P.energy[j] = S.energy[j];
    if (with_rho && P.rho) P.rho[j] = S.rho[j];
}

// --- absolute FP64 positions <-> (cell, offset) --------------------------------------
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_from_positions(Geom<R> G, double lo0, double lo1, double lo2, double D0, double D1, double D2, int n,
                 const double *x, int *cell, R *off0, R *off1, R *off2, unsigned int *bad)
{
#pragma clang fp contract(off)
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lo0, lo1, lo2};
    const double D[3] = {D0, D1, D2};
    R *off[3] = {off0, off1, off2};
    int c[3] = {0, 0, 0};
    bool ok = true;
    for (int d = 0; d < G.dim; ++d) {
        const double rel = x[(size_t)d * n + i] - lo[d];
        double k = floor(rel / D[d]);
        if (!(k > -2.0e9 && k < 2.0e9)) { k = 0.0; ok = false; }
        int ck = wrap_index((int)((long long)k % G.nc[d]), G.nc[d]);
        R o = ok ? R(rel - k * D[d]) : R(0);
        ok &= carry(o, ck, G.delta[d], G.nc[d]);
        c[d] = ck;
        off[d][i] = o;
    }
    cell[i] = join_cell(G, c[0], c[1], c[2]);
    if (!ok && bad) atomicOr(bad, 1u);
}

template <typename R>
__global__ void __launch_bounds__(kBlock)
k_to_positions(Geom<R> G, double lo0, double lo1, double lo2, double D0, double D1, double D2, int n,
               const int *cell, const R *off0, const R *off1, const R *off2, double *x)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const double lo[3] = {lo0, lo1, lo2};
    const double D[3] = {D0, D1, D2};
    const R *off[3] = {off0, off1, off2};
    int c[3];
    split_cell(G, cell[i], c[0], c[1], c[2]);
    for (int d = 0; d < G.dim; ++d) x[(size_t)d * n + i] = lo[d] + double(c[d]) * D[d] + double(off[d][i]);
}

}  // namespace tfsph
