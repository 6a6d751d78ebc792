// Launch sequences of one IDIC step shared by the library's entry points:
// binning (counting sort into canonical (cell, id) order), gas density, and
// the fused force + predictor + cell solve + update kernel.
#pragma once

#include "binning.hpp"
#include "host.hpp"
#include "sph.hpp"

namespace tfsph_host {

inline int ntiles_of(int ncell) { return (ncell + kScanTile - 1) / kScanTile; }

inline int default_cells_per_block(int dim) { return dim == 1 ? 128 : (dim == 2 ? 64 : 32); }
// upper bound of tfsph_set_cells_per_block: the block's cell solves sit in LDS
// next to the staged particle records (under 64 KiB in FP64)
constexpr int kMaxCellsPerBlock = 256;

// zero the cell counts of a phase pair: once per workspace, before its first binning
template <typename R>
inline tfsph_status enqueue_zero_counts(int ncell, Sorted<R> &Sg, Sorted<R> &Sd, hipStream_t st)
{
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks_for(ncell)), dim3(kBlock), 0, st, Sg.count, ncell, Sd.count, ncell);
    LAUNCH_CHECK("fill_zero");
    return TFSPH_OK;
}

// count + scan + scatter + rank/gather of both phases into the workspace:
// counting sort of both phases into (cell, id) order.  The counts must be zero
// on entry (enqueue_zero_counts() once, then every binning leaves them zero).
template <typename R>
inline tfsph_status enqueue_bin(int ng, int nd, const Geom<R> &G, const Phase<R> &Pg, const Phase<R> &Pd,
                                Sorted<R> &Sg, Sorted<R> &Sd, int *partial, const Flags &F, hipStream_t st)
{
    const int ncell = G.ncell;
    const int ntiles = ntiles_of(ncell);
    const int bg = blocks_for(ng), bd = blocks_for(nd);
    if (bg + bd > 0) {
        hipLaunchKernelGGL(k_count, dim3(bg + bd), dim3(kBlock), 0, st, Pg.cell, ng, Sg.count, Sg.slot, Pd.cell,
                           nd, Sd.count, Sd.slot, bg, ncell, F.word);
        LAUNCH_CHECK("count");
    }
    hipLaunchKernelGGL(k_scan_reduce, dim3(ntiles, 2), dim3(kBlock), 0, st, Sg.count, Sd.count, ncell, partial, ntiles);
    LAUNCH_CHECK("scan_reduce");
    const int inline_prefix = ntiles <= kScanInlineTiles ? 1 : 0;
    if (!inline_prefix) {
        hipLaunchKernelGGL(k_scan_top, dim3(1, 2), dim3(kBlock), 0, st, partial, ntiles, Sg.start, Sd.start, ncell);
        LAUNCH_CHECK("scan_top");
    }
    hipLaunchKernelGGL(k_scan_down, dim3(ntiles, 2), dim3(kBlock), 0, st, Sg.count, Sd.count, ncell, partial, ntiles,
                       Sg.start, Sd.start, inline_prefix);
    LAUNCH_CHECK("scan_down");
    if (bg + bd > 0) {
        hipLaunchKernelGGL(k_scatter, dim3(bg + bd), dim3(kBlock), 0, st, Pg.cell, Pg.id, Sg.slot, Sg.start, ng,
                           Sg.tmp_idx, Sg.tmp_id, Pd.cell, Pd.id, Sd.slot, Sd.start, nd, Sd.tmp_idx, Sd.tmp_id, bg, ncell);
        LAUNCH_CHECK("scatter");
        hipLaunchKernelGGL(k_rank_gather<R>, dim3(bg + bd), dim3(kBlock), 0, st, G, Pg, Sg, Pd, Sd, bg, F.word);
        LAUNCH_CHECK("rank_gather");
    }
    return TFSPH_OK;
}


// kernel variant: 0 (auto) and 1 = global-memory pair loops (neighbour masks
// when S.nmask is set)
template <typename R, int DIM>
inline tfsph_status enqueue_density(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &S, int want_frc,
                                    hipStream_t st, int variant = 0)
{
    (void)variant;
    if (S.n == 0) return TFSPH_OK;
    hipLaunchKernelGGL((k_density<R, DIM>), dim3(blocks_for(S.n)), dim3(kBlock), 0, st, G, Ph, S, want_frc);
    LAUNCH_CHECK("density");
    return TFSPH_OK;
}

// Explicit gas terms and predictor v~, one thread per gas particle.  The
// pair loop has a launch of its own: a block that owns whole cells holds a
// varying number of particles, and the few past a multiple of the block size
// would take a whole extra round of the pair loop.
template <typename R, int DIM>
inline tfsph_status enqueue_force(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sg, const Phase<R> &Pg,
                                  hipStream_t st)
{
    if (Sg.n == 0) return TFSPH_OK;
    const dim3 grid(blocks_for(Sg.n)), block(kBlock);
    if (Ph.av || Ph.eos != 0)
        hipLaunchKernelGGL((k_gas_predict<R, DIM, kForceGeneral>), grid, block, 0, st, G, Ph, Sg, Pg);
    else if (Sg.has_mass)
        hipLaunchKernelGGL((k_gas_predict<R, DIM, kForceIsoMass>), grid, block, 0, st, G, Ph, Sg, Pg);
    else
        hipLaunchKernelGGL((k_gas_predict<R, DIM, kForceIsoUniform>), grid, block, 0, st, G, Ph, Sg, Pg);
    LAUNCH_CHECK("gas_predict");
    return TFSPH_OK;
}

// Cell sums, implicit solve, particle update, move and carry.
template <typename R, int DIM>
inline tfsph_status enqueue_update(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sg, const Sorted<R> &Sd,
                                   const Phase<R> &Pg, const Phase<R> &Pd, const Flags &F, int cpb, hipStream_t st)
{
    const int nblocks = (G.ncell + cpb - 1) / cpb;
    const size_t lds = update_lds_bytes<R>(cpb);
    hipLaunchKernelGGL((k_update<R, DIM>), dim3(nblocks), dim3(kBlock), lds, st, G, Ph, Sg, Sd, Pg, Pd, F, cpb, nblocks);
    LAUNCH_CHECK("update");
    return TFSPH_OK;
}

}  // namespace tfsph_host
