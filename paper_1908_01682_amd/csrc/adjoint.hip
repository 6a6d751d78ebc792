// Host side of the checkpointed adjoint (declarations and contract:
// include/tfsph.h).
#include "../../include/tfsph.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <vector>

#include "adjoint.hpp"
#include "enqueue.hpp"
#include "host.hpp"

using namespace tfsph;
using namespace tfsph_host;

namespace {

// blocks of k_adj_cell: runs of default_cells_per_block cells
inline int adj_cell_blocks(int ncell, int dim)
{
    const int cpb = default_cells_per_block(dim);
    return (ncell + cpb - 1) / cpb;
}

// caller-like state arrays carved from the workspace
template <typename R>
struct StateBuf {
    Phase<R> g, d;
};

template <typename R>
Phase<R> carve_state_phase(Carver &cv, int n, int dim, bool mass, bool rho, R mu)
{
    Phase<R> P{};
    P.n = n;
    P.cell = cv.take<int>(n);
    P.id = cv.take<int>(n);
    for (int k = 0; k < 3; ++k) {
        P.off[k] = k < dim ? cv.take<R>(n) : nullptr;
        P.vel[k] = k < dim ? cv.take<R>(n) : nullptr;
    }
    P.mass = mass ? cv.take<R>(n) : nullptr;
    P.m_uniform = mu;
    P.rho = rho ? cv.take<R>(n) : nullptr;
    P.energy = nullptr;
    return P;
}

template <typename R>
AdjPhase<R> carve_adj(Carver &cv, int n, int dim, bool with_x, bool with_v)
{
    AdjPhase<R> A{};
    for (int k = 0; k < 3; ++k) {
        A.x[k] = (with_x && k < dim) ? cv.take<R>(n) : nullptr;
        A.v[k] = (with_v && k < dim) ? cv.take<R>(n) : nullptr;
    }
    return A;
}

template <typename R>
struct AdjLayout {
    StateBuf<R> W;
    std::vector<StateBuf<R>> ckpt;
    std::vector<Sorted<R>> tg, td;      // tapes per step of a segment
    int *partial;
    Flags F;
    AdjPhase<R> cur_g, cur_d, nxt_g, nxt_d;
    AdjPhase<R> vtb_g, ubi_d;           // sorted scratch (v component used)
    R *abar[3];
    R *rhobar_g, *rhobar_d;
    R *xacc_g[3], *xacc_d[3];
    double *sbar_part, *loss_part, *acc;  // acc[0] = loss, acc[1] = dL/dlog t_stop
    double *sbar_step;                    // per-step sums of sbar_part
    size_t bytes;
};

template <typename R>
void adj_layout(AdjLayout<R> &L, char *base, const tfsph_params *p, int ng, int nd, int K, int nseg, bool mg,
                bool md, double mug, double mud)
{
    Carver cv;
    cv.base = base;
    const int dim = p->dim, ncell = ncell_of(p);
    L.W.g = carve_state_phase<R>(cv, ng, dim, mg, true, R(mug));
    L.W.d = carve_state_phase<R>(cv, nd, dim, md, false, R(mud));
    L.ckpt.assign(nseg, StateBuf<R>{});
    for (int s = 0; s < nseg; ++s) {
        L.ckpt[s].g = carve_state_phase<R>(cv, ng, dim, mg, false, R(mug));
        L.ckpt[s].d = carve_state_phase<R>(cv, nd, dim, md, false, R(mud));
    }
    // tapes of one segment's steps, plus one for the binning of the final state
    L.tg.assign(K + 1, Sorted<R>{});
    L.td.assign(K + 1, Sorted<R>{});
    for (int t = 0; t <= K; ++t) {
        L.tg[t] = carve_phase<R>(cv, ng, dim, ncell, PhaseFlags{mg, false, true, mask_rows_of(p)});
        L.tg[t].src = cv.take<int>(ng);
        L.td[t] = carve_phase<R>(cv, nd, dim, ncell, PhaseFlags{md, false, false});
        L.td[t].src = cv.take<int>(nd);
    }
    L.partial = cv.take<int>(size_t(2) * ntiles_of(ncell));
    L.F.word = cv.take<unsigned int>(64);
    L.F.one_phase = cv.take<unsigned long long>(8);
    L.cur_g = carve_adj<R>(cv, ng, dim, true, true);
    L.cur_d = carve_adj<R>(cv, nd, dim, true, true);
    L.nxt_g = carve_adj<R>(cv, ng, dim, true, true);
    L.nxt_d = carve_adj<R>(cv, nd, dim, true, true);
    L.vtb_g = carve_adj<R>(cv, ng, dim, false, true);
    L.ubi_d = carve_adj<R>(cv, nd, dim, false, true);
    for (int k = 0; k < 3; ++k) {
        L.abar[k] = k < dim ? cv.take<R>(ng) : nullptr;
        L.xacc_g[k] = k < dim ? cv.take<R>(ng) : nullptr;
        L.xacc_d[k] = k < dim ? cv.take<R>(nd) : nullptr;
    }
    L.rhobar_g = cv.take<R>(ng);
    L.rhobar_d = cv.take<R>(nd);
    // d/dlog t_stop partials: one per block of k_adj_cell and reverse step, summed once at the end
    L.sbar_part = cv.take<double>(size_t(nseg) * K * adj_cell_blocks(ncell, dim));
    L.sbar_step = cv.take<double>(size_t(nseg) * K);
    L.loss_part = cv.take<double>(blocks_for(nd));
    L.acc = cv.take<double>(4);
    L.bytes = cv.off + 256;
}

template <typename T>
tfsph_status copy_dev(const T *in, T *out, int n, hipStream_t st)
{
    if (n <= 0 || !in || !out) return TFSPH_OK;
    hipLaunchKernelGGL(k_copy<T>, dim3(blocks_for(n)), dim3(kBlock), 0, st, in, out, n);
    LAUNCH_CHECK("copy");
    return TFSPH_OK;
}

template <typename T>
tfsph_status fill_dev(T *out, T v, int n, hipStream_t st)
{
    if (n <= 0 || !out) return TFSPH_OK;
    hipLaunchKernelGGL(k_fill<T>, dim3(blocks_for(n)), dim3(kBlock), 0, st, out, v, n);
    LAUNCH_CHECK("fill");
    return TFSPH_OK;
}

#define TRY(expr)                           \
    do {                                    \
        tfsph_status r_ = (expr);           \
        if (r_ != TFSPH_OK) return r_;      \
    } while (0)

template <typename R>
tfsph_status copy_state(const Phase<R> &in, const Phase<R> &out, int dim, hipStream_t st)
{
    TRY(copy_dev<int>(in.cell, out.cell, in.n, st));
    TRY(copy_dev<int>(in.id, out.id, in.n, st));
    for (int k = 0; k < dim; ++k) {
        TRY(copy_dev<R>(in.off[k], out.off[k], in.n, st));
        TRY(copy_dev<R>(in.vel[k], out.vel[k], in.n, st));
    }
    if (in.mass && out.mass) TRY(copy_dev<R>(in.mass, const_cast<R *>(out.mass), in.n, st));
    return TFSPH_OK;
}

template <typename R, int DIM>
tfsph_status fwd_step(const Geom<R> &G, const Phys<R> &Ph, AdjLayout<R> &L, int slot, hipStream_t st)
{
    Sorted<R> &Sg = L.tg[slot], &Sd = L.td[slot];
    TRY(enqueue_bin<R>(L.W.g.n, L.W.d.n, G, L.W.g, L.W.d, Sg, Sd, L.partial, L.F, st));
    TRY((enqueue_density<R, DIM>(G, Ph, Sg, 1, st)));
    TRY((enqueue_force<R, DIM>(G, Ph, Sg, L.W.g, st)));
    TRY((enqueue_update<R, DIM>(G, Ph, Sg, Sd, L.W.g, L.W.d, L.F, default_cells_per_block(DIM), st)));
    return TFSPH_OK;
}

template <typename R>
tfsph_status unsort(int n, int dim, const int *src, R *const in[3], R *const out[3], hipStream_t st)
{
    if (n == 0) return TFSPH_OK;
    hipLaunchKernelGGL(k_adj_unsort<R>, dim3(blocks_for(n)), dim3(kBlock), 0, st, n, dim, src, in[0], in[1], in[2],
                       out[0], out[1], out[2]);
    LAUNCH_CHECK("unsort");
    return TFSPH_OK;
}

// reverse of global step `step`, whose tapes are in slot `slot`
template <typename R, int DIM>
tfsph_status rev_step(const Geom<R> &G, const Phys<R> &Ph, AdjLayout<R> &L, int slot, int step, hipStream_t st)
{
    Sorted<R> &Sg = L.tg[slot], &Sd = L.td[slot];
    const int ng = Sg.n, nd = Sd.n;
    const int cpb = default_cells_per_block(DIM);
    const int nb = adj_cell_blocks(G.ncell, DIM);
    hipLaunchKernelGGL((k_adj_cell<R, DIM>), dim3(nb), dim3(kBlock), adj_cell_lds_bytes<R>(cpb), st, G, Ph, Sg, Sd,
                       L.cur_g, L.cur_d, L.vtb_g, L.abar[0], L.abar[1], L.abar[2], L.ubi_d,
                       L.sbar_part + size_t(step) * nb, cpb);
    LAUNCH_CHECK("adj_cell");
    if (ng > 0) {
        hipLaunchKernelGGL((k_adj_force<R, DIM>), dim3(blocks_for(ng)), dim3(kBlock), 0, st, G, Ph, Sg, L.abar[0],
                           L.abar[1], L.abar[2], L.cur_g, L.xacc_g[0], L.xacc_g[1], L.xacc_g[2], L.rhobar_g);
        LAUNCH_CHECK("adj_force");
        hipLaunchKernelGGL((k_adj_density<R, DIM>), dim3(blocks_for(ng)), dim3(kBlock), 0, st, G, Sg, L.rhobar_g,
                           L.xacc_g[0], L.xacc_g[1], L.xacc_g[2]);
        LAUNCH_CHECK("adj_density");
    }
    // undo the step's sorts: gas (x from xacc, v from vtb), dust (x from cur, v from ubi)
    const int bg = blocks_for(ng), bd = blocks_for(nd);
    if (bg + bd > 0) {
        AdjPhase<R> in_g{}, in_d{};
        for (int k = 0; k < 3; ++k) {
            in_g.x[k] = L.xacc_g[k];
            in_g.v[k] = L.vtb_g.v[k];
            in_d.x[k] = L.cur_d.x[k];
            in_d.v[k] = L.ubi_d.v[k];
        }
        hipLaunchKernelGGL(k_adj_unsort_step<R>, dim3(bg + bd), dim3(kBlock), 0, st, ng, nd, DIM, bg, Sg.src, Sd.src,
                           in_g, L.nxt_g, in_d, L.nxt_d);
        LAUNCH_CHECK("adj_unsort_step");
    }
    std::swap(L.cur_g, L.nxt_g);
    std::swap(L.cur_d, L.nxt_d);
    return TFSPH_OK;
}

template <typename R, int DIM>
tfsph_status run_adjoint(const tfsph_params *p, const tfsph_state *s, int n_steps, int K, const R *target,
                         void *dv0[3], void *du0[3], double *dlogt, double *loss, char *ws, hipStream_t st)
{
    const int ng = (int)s->gas.n, nd = (int)s->dust.n;
    const int nseg = (n_steps + K - 1) / K;
    AdjLayout<R> L;
    adj_layout<R>(L, ws, p, ng, nd, K, nseg, s->gas.mass != nullptr, s->dust.mass != nullptr, s->gas.mass_uniform,
                  s->dust.mass_uniform);
    const Geom<R> G = make_geom<R>(p);
    const Phys<R> Ph = make_phys<R>(p);
    const Phase<R> Ig = make_phase<R>(s->gas, DIM), Id = make_phase<R>(s->dust, DIM);

    HIP_TRY(hipMemsetAsync(L.F.word, 0, 256, st));
    HIP_TRY(hipMemsetAsync(L.F.one_phase, 0, 64, st));
    TRY(fill_dev<double>(L.acc, 0.0, 4, st));
    for (int t = 0; t <= K; ++t) TRY(enqueue_zero_counts<R>(G.ncell, L.tg[t], L.td[t], st));
    // forward sweep with checkpoints
    TRY(copy_state<R>(Ig, L.W.g, DIM, st));
    TRY(copy_state<R>(Id, L.W.d, DIM, st));
    // (the last segment's steps keep their tapes, so that segment is not replayed)
    const int last_first = (nseg - 1) * K;
    for (int i = 0; i < n_steps; ++i) {
        if (i % K == 0) {
            TRY(copy_state<R>(L.W.g, L.ckpt[i / K].g, DIM, st));
            TRY(copy_state<R>(L.W.d, L.ckpt[i / K].d, DIM, st));
        }
        TRY((fwd_step<R, DIM>(G, Ph, L, i >= last_first ? i - last_first : 0, st)));
    }
    // loss on the final dust positions and its position adjoint
    Sorted<R> &Fg = L.tg[K], &Fd = L.td[K];
    TRY(enqueue_bin<R>(ng, nd, G, L.W.g, L.W.d, Fg, Fd, L.partial, L.F, st));
    for (int k = 0; k < DIM; ++k) {
        TRY(fill_dev<R>(L.cur_g.x[k], R(0), ng, st));
        TRY(fill_dev<R>(L.cur_g.v[k], R(0), ng, st));
        TRY(fill_dev<R>(L.cur_d.v[k], R(0), nd, st));
        TRY(fill_dev<R>(L.cur_d.x[k], R(0), nd, st));
        TRY(fill_dev<R>(L.xacc_d[k], R(0), nd, st));
    }
    if (nd > 0) {
        const int nbd = blocks_for(nd);
        hipLaunchKernelGGL((k_adj_loss<R, DIM>), dim3(nbd), dim3(kBlock), 0, st, G, Fd, target, nd, L.rhobar_d,
                           L.loss_part);
        LAUNCH_CHECK("adj_loss");
        hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kBlock), 0, st, L.loss_part, nbd, 1.0 / nd, L.acc + 0, 0);
        LAUNCH_CHECK("adj_reduce");
        hipLaunchKernelGGL((k_adj_density<R, DIM>), dim3(nbd), dim3(kBlock), 0, st, G, Fd, L.rhobar_d,
                           L.xacc_d[0], L.xacc_d[1], L.xacc_d[2]);
        LAUNCH_CHECK("adj_density");
        TRY(unsort<R>(nd, DIM, Fd.src, L.xacc_d, L.cur_d.x, st));
    }
    // backward sweep, segment by segment
    for (int seg = nseg - 1; seg >= 0; --seg) {
        const int first = seg * K, len = std::min(K, n_steps - first);
        if (seg < nseg - 1) {
            TRY(copy_state<R>(L.ckpt[seg].g, L.W.g, DIM, st));
            TRY(copy_state<R>(L.ckpt[seg].d, L.W.d, DIM, st));
            for (int t = 0; t < len; ++t) TRY((fwd_step<R, DIM>(G, Ph, L, t, st)));
        }
        for (int t = len - 1; t >= 0; --t) TRY((rev_step<R, DIM>(G, Ph, L, t, first + t, st)));
    }
    // d/dlog t_stop: every step's block partials, in a fixed order that does not depend on K
    hipLaunchKernelGGL(k_adj_reduce_rows, dim3(n_steps), dim3(kBlock), 0, st, L.sbar_part,
                       adj_cell_blocks(G.ncell, DIM), L.sbar_step);
    LAUNCH_CHECK("adj_reduce_rows");
    hipLaunchKernelGGL(k_adj_reduce, dim3(1), dim3(kBlock), 0, st, L.sbar_step, n_steps, 1.0, L.acc + 1, 1);
    LAUNCH_CHECK("adj_reduce");
    // gradients by id
    if (ng > 0) {
        hipLaunchKernelGGL(k_adj_by_id<R>, dim3(blocks_for(ng)), dim3(kBlock), 0, st, ng, DIM, Ig.id, L.cur_g.v[0],
                           L.cur_g.v[1], L.cur_g.v[2], static_cast<R *>(dv0[0]), static_cast<R *>(DIM > 1 ? dv0[1] : nullptr),
                           static_cast<R *>(DIM > 2 ? dv0[2] : nullptr));
        LAUNCH_CHECK("adj_by_id");
    }
    if (nd > 0) {
        hipLaunchKernelGGL(k_adj_by_id<R>, dim3(blocks_for(nd)), dim3(kBlock), 0, st, nd, DIM, Id.id, L.cur_d.v[0],
                           L.cur_d.v[1], L.cur_d.v[2], static_cast<R *>(du0[0]), static_cast<R *>(DIM > 1 ? du0[1] : nullptr),
                           static_cast<R *>(DIM > 2 ? du0[2] : nullptr));
        LAUNCH_CHECK("adj_by_id");
    }
    TRY(copy_dev<double>(L.acc + 0, loss, 1, st));
    TRY(copy_dev<double>(L.acc + 1, dlogt, 1, st));
    return TFSPH_OK;
}

tfsph_status check_adjoint_args(const tfsph_params *p, int64_t ng, int64_t nd, int32_t n_steps, int32_t K)
{
    tfsph_status r = tfsph_validate(p);
    if (r != TFSPH_OK) return r;
    if (p->scheme != TFSPH_SCHEME_IDIC)
        return fail(TFSPH_E_UNSUPPORTED, "the adjoint differentiates the first-order step only");
    if (p->eos != TFSPH_ISOTHERMAL || p->av_alpha != 0.0 || p->av_beta != 0.0)
        return fail(TFSPH_E_UNSUPPORTED, "the adjoint covers the isothermal EOS without artificial viscosity");
    if (n_steps < 1) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 1");
    if (K < 1) return fail(TFSPH_E_INVALID_ARG, "ckpt_every must be >= 1");
    if (ng < 0 || nd < 0 || ng > 0x7fffffffLL || nd > 0x7fffffffLL)
        return fail(TFSPH_E_INVALID_ARG, "particle counts must be in [0, 2^31)");
    return TFSPH_OK;
}

template <typename R>
size_t adjoint_bytes(const tfsph_params *p, int ng, int nd, int n_steps, int K)
{
    const int nseg = (n_steps + K - 1) / K;
    AdjLayout<R> L;
    adj_layout<R>(L, nullptr, p, ng, nd, std::min(K, n_steps), nseg, true, true, 1.0, 1.0);
    return L.bytes;
}

}  // namespace

extern "C" tfsph_status tfsph_adjoint_workspace_size(const tfsph_params *p, int64_t n_gas, int64_t n_dust,
                                                     int32_t n_steps, int32_t ckpt_every, size_t *bytes)
{
    tfsph_status r = check_adjoint_args(p, n_gas, n_dust, n_steps, ckpt_every);
    if (r != TFSPH_OK) return r;
    if (!bytes) return fail(TFSPH_E_INVALID_ARG, "bytes is NULL");
    *bytes = p->precision == TFSPH_F64 ? adjoint_bytes<double>(p, (int)n_gas, (int)n_dust, n_steps, ckpt_every)
                                       : adjoint_bytes<float>(p, (int)n_gas, (int)n_dust, n_steps, ckpt_every);
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_step_adjoint(const tfsph_params *p, const tfsph_state *initial, int32_t n_steps,
                                           int32_t ckpt_every, const void *target, void *dL_dv0_gas[3],
                                           void *dL_du0_dust[3], double *dL_dlog_tstop, double *loss,
                                           void *workspace, size_t ws_bytes, void *hip_stream)
{
    if (!initial) return fail(TFSPH_E_INVALID_ARG, "initial state is NULL");
    tfsph_status r = check_adjoint_args(p, initial->gas.n, initial->dust.n, n_steps, ckpt_every);
    if (r != TFSPH_OK) return r;
    r = check_phase(initial->gas, p->dim, false, false, "gas");
    if (r != TFSPH_OK) return r;
    r = check_phase(initial->dust, p->dim, false, false, "dust");
    if (r != TFSPH_OK) return r;
    if (!dL_dlog_tstop || !loss) return fail(TFSPH_E_INVALID_ARG, "output scalars are NULL");
    if (initial->dust.n > 0 && !target) return fail(TFSPH_E_INVALID_ARG, "target is NULL");
    for (int k = 0; k < p->dim; ++k) {
        if (initial->gas.n > 0 && (!dL_dv0_gas || !dL_dv0_gas[k])) return fail(TFSPH_E_INVALID_ARG, "dL_dv0_gas[%d] is NULL", k);
        if (initial->dust.n > 0 && (!dL_du0_dust || !dL_du0_dust[k]))
            return fail(TFSPH_E_INVALID_ARG, "dL_du0_dust[%d] is NULL", k);
    }
    size_t need = 0;
    r = tfsph_adjoint_workspace_size(p, initial->gas.n, initial->dust.n, n_steps, ckpt_every, &need);
    if (r != TFSPH_OK) return r;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(TFSPH_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return fail(TFSPH_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    const int K = std::min(ckpt_every, n_steps);
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    char *ws = static_cast<char *>(workspace);
    if (p->precision == TFSPH_F64) {
        const double *t = static_cast<const double *>(target);
        switch (p->dim) {
        case 1: return run_adjoint<double, 1>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
        case 2: return run_adjoint<double, 2>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
        default: return run_adjoint<double, 3>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
        }
    }
    const float *t = static_cast<const float *>(target);
    switch (p->dim) {
    case 1: return run_adjoint<float, 1>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
    case 2: return run_adjoint<float, 2>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
    default: return run_adjoint<float, 3>(p, initial, n_steps, K, t, dL_dv0_gas, dL_du0_dust, dL_dlog_tstop, loss, ws, st);
    }
}
