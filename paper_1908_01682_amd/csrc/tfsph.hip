// Host runtime of the TFSPH library: parameter validation, workspace
// planning, and the launch sequence of one IDIC step (Section 2.3).
// Declarations and the contract of every entry point: include/tfsph.h.
#include "../../include/tfsph.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <new>
#include <vector>

#include "binning.hpp"
#include "common.hpp"
#include "host.hpp"
#include "sph.hpp"
#include "enqueue.hpp"
#include "imex.hpp"
#include "pairdrag.hpp"

using namespace tfsph;
using namespace tfsph_host;

namespace tfsph_host {
thread_local char g_last_error[512] = "";
}

extern "C" const char *tfsph_status_string(tfsph_status s)
{
    switch (s) {
    case TFSPH_OK: return "TFSPH_OK";
    case TFSPH_E_INVALID_ARG: return "TFSPH_E_INVALID_ARG";
    case TFSPH_E_WORKSPACE: return "TFSPH_E_WORKSPACE";
    case TFSPH_E_HIP: return "TFSPH_E_HIP";
    case TFSPH_E_UNSUPPORTED: return "TFSPH_E_UNSUPPORTED";
    case TFSPH_E_STATE: return "TFSPH_E_STATE";
    }
    return "TFSPH_E_UNKNOWN";
}

extern "C" const char *tfsph_last_error(void) { return g_last_error; }

// ----------------------------------------------------------------------------
// validation (host only)
// ----------------------------------------------------------------------------
static bool finite_pos(double x) { return std::isfinite(x) && x > 0.0; }

extern "C" tfsph_status tfsph_validate(const tfsph_params *p)
{
    g_last_error[0] = 0;
    if (!p) return fail(TFSPH_E_INVALID_ARG, "params is NULL");
    if (p->dim < 1 || p->dim > 3) return fail(TFSPH_E_INVALID_ARG, "dim must be 1, 2 or 3 (got %d)", p->dim);
    if (p->precision != TFSPH_F32 && p->precision != TFSPH_F64)
        return fail(TFSPH_E_INVALID_ARG, "unknown precision %d", p->precision);
    if (p->eos != TFSPH_ISOTHERMAL && p->eos != TFSPH_ADIABATIC) return fail(TFSPH_E_INVALID_ARG, "unknown eos %d", p->eos);
    if (!finite_pos(p->h)) return fail(TFSPH_E_INVALID_ARG, "h must be positive and finite");
    long long ncell = 1;
    for (int d = 0; d < 3; ++d) {
        if (d >= p->dim) {
            if (p->n_cells[d] != 1) return fail(TFSPH_E_INVALID_ARG, "n_cells[%d] must be 1 for dim %d", d, p->dim);
            continue;
        }
        if (p->n_cells[d] < 1) return fail(TFSPH_E_INVALID_ARG, "n_cells[%d] must be >= 1", d);
        if (!(std::isfinite(p->box_lo[d]) && std::isfinite(p->box_hi[d]) && p->box_hi[d] > p->box_lo[d]))
            return fail(TFSPH_E_INVALID_ARG, "box axis %d must satisfy box_lo < box_hi (finite)", d);
        const int W = window_of(p, d);
        if (W > kMaxWindow) return fail(TFSPH_E_INVALID_ARG, "neighbour window %d cells on axis %d exceeds %d", W, d, kMaxWindow);
        if (p->n_cells[d] < 2 * W + 1)
            return fail(TFSPH_E_INVALID_ARG, "axis %d has %d cells; the 2h window needs at least %d", d, p->n_cells[d], 2 * W + 1);
        ncell *= p->n_cells[d];
        if (ncell > 0x7fffffffLL - 1) return fail(TFSPH_E_INVALID_ARG, "too many cells");
    }
    if (!(std::isfinite(p->K) && p->K >= 0.0)) return fail(TFSPH_E_INVALID_ARG, "K must be >= 0 and finite");
    if (!(std::isfinite(p->t_stop_epstein) && p->t_stop_epstein >= 0.0))
        return fail(TFSPH_E_INVALID_ARG, "t_stop_epstein must be >= 0 and finite");
    if (p->K > 0.0 && p->t_stop_epstein > 0.0)
        return fail(TFSPH_E_INVALID_ARG, "K and t_stop_epstein select different drag laws: set at most one");
    if (p->K == 0.0 && p->t_stop_epstein == 0.0 && !finite_pos(p->t_stop))
        return fail(TFSPH_E_INVALID_ARG, "t_stop must be positive (or K or t_stop_epstein > 0)");
    if (!finite_pos(p->dt)) return fail(TFSPH_E_INVALID_ARG, "dt must be positive");
    if (p->scheme < TFSPH_SCHEME_IDIC || p->scheme > TFSPH_SCHEME_ISPH)
        return fail(TFSPH_E_INVALID_ARG, "scheme must be TFSPH_SCHEME_IDIC, _IMEX2, _MK or _ISPH (got %d)", p->scheme);
    if (p->eos == TFSPH_ISOTHERMAL && !finite_pos(p->c_s)) return fail(TFSPH_E_INVALID_ARG, "c_s must be positive");
    if (p->eos == TFSPH_ADIABATIC && !(std::isfinite(p->gamma) && p->gamma > 1.0))
        return fail(TFSPH_E_INVALID_ARG, "gamma must be > 1");
    if (!(p->av_alpha >= 0.0 && p->av_beta >= 0.0 && std::isfinite(p->av_alpha) && std::isfinite(p->av_beta)))
        return fail(TFSPH_E_INVALID_ARG, "viscosity coefficients must be >= 0");
    for (int d = 0; d < 3; ++d)
        if (!std::isfinite(p->g[d])) return fail(TFSPH_E_INVALID_ARG, "g must be finite");
    if (!(std::isfinite(p->cfl) && p->cfl >= 0.0)) return fail(TFSPH_E_INVALID_ARG, "cfl must be >= 0 and finite");
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_cfl_dt(const tfsph_params *p, double signal_speed, double *dt)
{
    g_last_error[0] = 0;
    if (!p || !dt) return fail(TFSPH_E_INVALID_ARG, "params / dt is NULL");
    if (!(std::isfinite(p->cfl) && p->cfl > 0.0)) return fail(TFSPH_E_INVALID_ARG, "cfl must be positive and finite");
    if (!finite_pos(p->h)) return fail(TFSPH_E_INVALID_ARG, "h must be positive and finite");
    if (!(std::isfinite(signal_speed) && signal_speed >= 0.0))
        return fail(TFSPH_E_INVALID_ARG, "signal speed must be >= 0 and finite");
    // eq. (4): tau = CFL h / max(v, c); the isothermal sound speed is a floor of the signal speed
    const double s = p->eos == TFSPH_ISOTHERMAL ? std::max(signal_speed, p->c_s) : signal_speed;
    if (!(s > 0.0)) return fail(TFSPH_E_INVALID_ARG, "signal speed is zero: no Courant bound");
    *dt = p->cfl * p->h / s;
    return TFSPH_OK;
}

// ----------------------------------------------------------------------------
// workspace layout
// ----------------------------------------------------------------------------
namespace {


// Workspace of the second-order IMEX step beyond the first-order one: the
// binning of the stage-2 and stage-3 positions (with the level-n index of each
// sorted slot), the stage predictors as a phase to bin, and the stage data.
template <typename R>
struct ImexViews {
    Sorted<R> Sg, Sd;
    Phase<R> Qg, Qd;
    Stage<R> Xg, Xd;
};

template <typename R>
Phase<R> carve_stage_phase(Carver &cv, int n, int dim, bool mass, bool energy, double m_uniform)
{
    Phase<R> Q{};
    Q.n = n;
    Q.cell = cv.take<int>(n);
    Q.id = cv.take<int>(n);
    for (int d = 0; d < dim; ++d) {
        Q.off[d] = cv.take<R>(n);
        Q.vel[d] = cv.take<R>(n);
    }
    Q.mass = mass ? cv.take<R>(n) : nullptr;
    Q.m_uniform = R(m_uniform);
    Q.energy = energy ? cv.take<R>(n) : nullptr;
    return Q;
}

template <typename R>
Stage<R> carve_stage(Carver &cv, int n, int dim, bool gas, bool energy)
{
    Stage<R> X{};
    for (int d = 0; d < dim; ++d) {
        X.v2[d] = cv.take<R>(n);
        X.dv2[d] = cv.take<R>(n);
        if (gas) {
            X.acc1[d] = cv.take<R>(n);
            X.acc2[d] = cv.take<R>(n);
        }
    }
    if (gas && energy) {
        X.de1 = cv.take<R>(n);
        X.de2 = cv.take<R>(n);
    }
    return X;
}

template <typename R>
void carve_imex(Carver &cv, const tfsph_params *p, int ng, int nd, PhaseFlags fg, PhaseFlags fd, double mg_uniform,
                double md_uniform, ImexViews<R> &V)
{
    const int ncell = ncell_of(p);
    V.Sg = carve_phase<R>(cv, ng, p->dim, ncell, fg);
    V.Sg.src = cv.take<int>(ng);
    V.Sd = carve_phase<R>(cv, nd, p->dim, ncell, fd);
    V.Sd.src = cv.take<int>(nd);
    V.Qg = carve_stage_phase<R>(cv, ng, p->dim, fg.mass, fg.energy, mg_uniform);
    V.Qd = carve_stage_phase<R>(cv, nd, p->dim, fd.mass, false, md_uniform);
    V.Xg = carve_stage<R>(cv, ng, p->dim, true, fg.energy);
    V.Xd = carve_stage<R>(cv, nd, p->dim, false, false);
}

template <typename R>
size_t plan_bytes(const tfsph_params *p, int ng, int nd, PhaseFlags fg, PhaseFlags fd)
{
    Carver cv;
    const int ncell = ncell_of(p);
    carve_phase<R>(cv, ng, p->dim, ncell, fg);
    carve_phase<R>(cv, nd, p->dim, ncell, fd);
    cv.take<int>(size_t(2) * ntiles_of(ncell));
    cv.take<unsigned int>(64);
    cv.take<unsigned long long>(8);
    if (p->scheme == TFSPH_SCHEME_IMEX2) {
        ImexViews<R> V;
        carve_imex<R>(cv, p, ng, nd, fg, fd, 0.0, 0.0, V);
    }
    if (p->scheme == TFSPH_SCHEME_MK || p->scheme == TFSPH_SCHEME_ISPH) {
        cv.take<R4<R>>(size_t(ng) + kPad);
        cv.take<R4<R>>(size_t(nd) + kPad);
    }
    return cv.off + 256;
}

}  // namespace

// event pairs bracketing launches of one kernel kind
struct KernelTimer {
    std::vector<hipEvent_t> ev;   // pairs: start, stop
    size_t used = 0;              // events recorded so far
};

// one captured chunk of steps, tied to the state's array addresses
struct StepGraph {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    unsigned long long key = 0;
};

struct tfsph_ctx {
    tfsph_params p;
    bool profiling = false;
    bool prof_rotate = false;   // time one kernel kind per sampled step, in turn
    int prof_every = 1;         // rotating mode: every prof_every-th step is sampled
    int prof_kind = 0;          // the kind timed in the current step (-1: none)
    long long prof_steps = 0;   // steps dispatched since profiling was enabled
    KernelTimer timers[4];
    StepGraph sg;
    hipStream_t capture_stream = nullptr;
    int variant = 0;            // TFSPH_VARIANT_*
    int ng, nd;
    PhaseFlags fg, fd;
    double mg_uniform, md_uniform;
    char *ws;
    size_t ws_bytes;
    hipStream_t last_stream;
    int cells_per_block;
};

// record one event of a (start, stop) pair for kernel kind k when profiling
static tfsph_status timer_mark(tfsph_ctx *c, int k, hipStream_t st)
{
    if (!c->profiling || (c->prof_rotate && k != c->prof_kind)) return TFSPH_OK;
    KernelTimer &T = c->timers[k];
    if (T.used == T.ev.size()) {
        hipEvent_t e;
        HIP_TRY(hipEventCreate(&e));
        T.ev.push_back(e);
    }
    HIP_TRY(hipEventRecord(T.ev[T.used++], st));
    return TFSPH_OK;
}

#define MARK(k)                                         \
    do {                                                \
        tfsph_status m_ = timer_mark(c, (k), st);       \
        if (m_ != TFSPH_OK) return m_;                  \
    } while (0)

static PhaseFlags gas_flags(const tfsph_params *p, bool mass_array)
{
    return PhaseFlags{mass_array, p->eos == TFSPH_ADIABATIC, true, mask_rows_of(p)};
}

static PhaseFlags dust_flags(bool mass_array) { return PhaseFlags{mass_array, false, false}; }

extern "C" tfsph_status tfsph_workspace_size(const tfsph_params *p, int64_t n_gas, int64_t n_dust, size_t *bytes)
{
    tfsph_status s = tfsph_validate(p);
    if (s != TFSPH_OK) return s;
    if (!bytes) return fail(TFSPH_E_INVALID_ARG, "bytes is NULL");
    if (n_gas < 0 || n_dust < 0 || n_gas > 0x7fffffffLL || n_dust > 0x7fffffffLL)
        return fail(TFSPH_E_INVALID_ARG, "particle counts must be in [0, 2^31)");
    // sized for per-particle masses on both phases (the largest layout)
    PhaseFlags fg = gas_flags(p, true), fd = dust_flags(true);
    *bytes = p->precision == TFSPH_F64 ? plan_bytes<double>(p, (int)n_gas, (int)n_dust, fg, fd)
                                       : plan_bytes<float>(p, (int)n_gas, (int)n_dust, fg, fd);
    return TFSPH_OK;
}

// ----------------------------------------------------------------------------
// typed views
// ----------------------------------------------------------------------------
namespace {

template <typename R>
void carve_all(const tfsph_ctx *c, Sorted<R> &Sg, Sorted<R> &Sd, int *&partial, Flags &F,
               ImexViews<R> *imex = nullptr, VelRho<R> *vr = nullptr)
{
    Carver cv;
    cv.base = c->ws;
    const int ncell = ncell_of(&c->p);
    Sg = carve_phase<R>(cv, c->ng, c->p.dim, ncell, c->fg);
    Sd = carve_phase<R>(cv, c->nd, c->p.dim, ncell, c->fd);
    partial = cv.take<int>(size_t(2) * ntiles_of(ncell));
    F.word = cv.take<unsigned int>(64);
    F.one_phase = cv.take<unsigned long long>(8);
    if (imex) carve_imex<R>(cv, &c->p, c->ng, c->nd, c->fg, c->fd, c->mg_uniform, c->md_uniform, *imex);
    if (vr) {
        vr->gas = cv.take<R4<R>>(size_t(c->ng) + kPad);
        vr->dust = cv.take<R4<R>>(size_t(c->nd) + kPad);
    }
}

}  // namespace

tfsph_status tfsph_host::check_phase(const tfsph_phase &ph, int dim, bool need_rho, bool need_energy, const char *name)
{
    if (ph.n < 0 || ph.n > 0x7fffffffLL) return fail(TFSPH_E_INVALID_ARG, "%s.n out of range", name);
    if (ph.n == 0) return TFSPH_OK;
    if (!ph.cell || !ph.id) return fail(TFSPH_E_INVALID_ARG, "%s.cell / %s.id is NULL", name, name);
    for (int d = 0; d < dim; ++d)
        if (!ph.off[d] || !ph.vel[d]) return fail(TFSPH_E_INVALID_ARG, "%s.off[%d] / vel[%d] is NULL", name, d, d);
    if (!ph.mass && !(std::isfinite(ph.mass_uniform) && ph.mass_uniform > 0.0))
        return fail(TFSPH_E_INVALID_ARG, "%s: mass is NULL and mass_uniform is not positive", name);
    if (need_rho && !ph.rho) return fail(TFSPH_E_INVALID_ARG, "%s.rho is NULL", name);
    if (need_energy && !ph.energy) return fail(TFSPH_E_INVALID_ARG, "%s.energy is NULL (adiabatic EOS)", name);
    return TFSPH_OK;
}

namespace {

tfsph_status check_state_matches(const tfsph_ctx *c, const tfsph_state *s)
{
    if (!s) return fail(TFSPH_E_INVALID_ARG, "state is NULL");
    if (s->gas.n != c->ng || s->dust.n != c->nd)
        return fail(TFSPH_E_STATE, "state sizes (%lld, %lld) differ from init (%d, %d)", (long long)s->gas.n,
                    (long long)s->dust.n, c->ng, c->nd);
    if ((s->gas.mass != nullptr) != c->fg.mass || (s->dust.mass != nullptr) != c->fd.mass)
        return fail(TFSPH_E_STATE, "per-particle mass arrays present/absent differently from init");
    tfsph_status st = check_phase(s->gas, c->p.dim, true, c->p.eos == TFSPH_ADIABATIC, "gas");
    if (st != TFSPH_OK) return st;
    return check_phase(s->dust, c->p.dim, false, false, "dust");
}

template <typename R, int DIM>
tfsph_status enqueue_step(tfsph_ctx *c, tfsph_state *s, hipStream_t st)
{
    const Geom<R> G = make_geom<R>(&c->p);
    const Phys<R> Ph = make_phys<R>(&c->p);
    Phase<R> Pg = make_phase<R>(s->gas, DIM), Pd = make_phase<R>(s->dust, DIM);
    Sorted<R> Sg, Sd;
    int *partial;
    Flags F;
    carve_all<R>(c, Sg, Sd, partial, F);
    if (c->variant != TFSPH_VARIANT_AUTO) Sg.nmask = nullptr;    // scan the whole window in both passes
    MARK(TFSPH_KERNEL_BIN);
    tfsph_status r = enqueue_bin<R>(c->ng, c->nd, G, Pg, Pd, Sg, Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_BIN);
    if (c->ng > 0) {
        MARK(TFSPH_KERNEL_DENSITY);
        r = enqueue_density<R, DIM>(G, Ph, Sg, 1, st, c->variant);
        if (r != TFSPH_OK) return r;
        MARK(TFSPH_KERNEL_DENSITY);
    }
    if (c->ng > 0) {
        MARK(TFSPH_KERNEL_FORCE);
        r = enqueue_force<R, DIM>(G, Ph, Sg, Pg, st);
        if (r != TFSPH_OK) return r;
        MARK(TFSPH_KERNEL_FORCE);
    }
    MARK(TFSPH_KERNEL_UPDATE);
    r = enqueue_update<R, DIM>(G, Ph, Sg, Sd, Pg, Pd, F, c->cells_per_block, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_UPDATE);
    return TFSPH_OK;
}

template <typename R>
ImexCoef<R> imex_coef(double tau)
{
    const double gam = 1.0 - 1.0 / std::sqrt(2.0);
    const double del = 1.0 - 1.0 / (2.0 * gam);
    ImexCoef<R> C;
    C.tau = R(tau);
    C.gtau = R(gam * tau);
    C.del = R(del);
    C.omd = R(1.0 - del);
    C.rg = R((1.0 - gam) / gam);
    return C;
}

// one drag solve over gamma tau on the binning (Sg, Sd) of a stage
template <typename R, int DIM, bool FINAL>
tfsph_status enqueue_relax(const tfsph_ctx *c, const Geom<R> &G, const Phys<R> &PhE, const ImexViews<R> &V,
                           const Phase<R> &Pg, const Phase<R> &Pd, const R *rho1, const Flags &F, hipStream_t st)
{
    const int cpb = c->cells_per_block;
    const int nblocks = (G.ncell + cpb - 1) / cpb;
    hipLaunchKernelGGL((k_imex_relax<R, DIM, FINAL>), dim3(nblocks), dim3(kBlock), update_lds_bytes<R>(cpb), st, G,
                       PhE, V.Sg, V.Sd, V.Xg, V.Xd, Pg, Pd, rho1, F, cpb, nblocks);
    LAUNCH_CHECK("imex_relax");
    return TFSPH_OK;
}

// explicit gas terms at a stage, with the pair-loop kind of the run
template <typename R, int DIM, typename L>
void launch_by_kind(const Phys<R> &Ph, const Sorted<R> &S, L &&launch)
{
    if (Ph.av || Ph.eos != 0)
        launch(IntC<kForceGeneral>{});
    else if (S.has_mass)
        launch(IntC<kForceIsoMass>{});
    else
        launch(IntC<kForceIsoUniform>{});
}

// One second-order IMEX step: see imex.hpp for the stages.
// reuse: this step follows an IMEX step of the same call on the same stream, so
// its stage-1 binning is that step's last one (k_imex_rebin)
template <typename R, int DIM>
tfsph_status enqueue_step_imex(tfsph_ctx *c, tfsph_state *s, hipStream_t st, bool reuse)
{
    const Geom<R> G = make_geom<R>(&c->p);
    const Phys<R> Ph = make_phys<R>(&c->p);
    tfsph_params pe = c->p;
    pe.dt = c->p.dt * (1.0 - 1.0 / std::sqrt(2.0));
    for (int d = 0; d < 3; ++d) pe.g[d] = 0.0;      // predictors already hold the explicit terms
    Phys<R> PhE = make_phys<R>(&pe);
    PhE.vlim2 = Ph.vlim2;                            // the Courant bound is on the whole step tau
    const ImexCoef<R> C = imex_coef<R>(c->p.dt);
    Phase<R> Pg = make_phase<R>(s->gas, DIM), Pd = make_phase<R>(s->dust, DIM);
    Sorted<R> Sg, Sd;
    int *partial;
    Flags F;
    ImexViews<R> V;
    carve_all<R>(c, Sg, Sd, partial, F, &V);
    if (c->variant != TFSPH_VARIANT_AUTO) Sg.nmask = V.Sg.nmask = nullptr;
    const int ng = c->ng, nd = c->nd;
    const int bg = blocks_for(ng), bd = blocks_for(nd);
    tfsph_status r;

    // stage 1: volumes and explicit terms at level n, stage-2 predictors
    MARK(TFSPH_KERNEL_BIN);
    if (reuse) {
        const int nb = std::max(std::max(bg, bd), blocks_for(G.ncell + 1));
        hipLaunchKernelGGL((k_imex_rebin<R>), dim3(2 * nb), dim3(kBlock), 0, st, G, Pg, Sg, V.Sg.start, Pd, Sd,
                           V.Sd.start, nb);
        LAUNCH_CHECK("imex_rebin");
    } else {
        r = enqueue_bin<R>(ng, nd, G, Pg, Pd, Sg, Sd, partial, F, st);
        if (r != TFSPH_OK) return r;
    }
    MARK(TFSPH_KERNEL_BIN);
    if (ng > 0) {
        MARK(TFSPH_KERNEL_DENSITY);
        r = enqueue_density<R, DIM>(G, Ph, Sg, 1, st, c->variant);
        if (r != TFSPH_OK) return r;
        MARK(TFSPH_KERNEL_DENSITY);
    }
    MARK(TFSPH_KERNEL_FORCE);
    if (ng > 0) {
        launch_by_kind<R, DIM>(Ph, Sg, [&](auto K) {
            hipLaunchKernelGGL((k_imex_gas1<R, DIM, decltype(K)::value>), dim3(bg), dim3(kBlock), 0, st, G, Ph, Sg,
                               V.Xg, V.Qg, C, F);
        });
        LAUNCH_CHECK("imex_gas1");
    }
    if (nd > 0) {
        hipLaunchKernelGGL((k_imex_dust1<R, DIM>), dim3(bd), dim3(kBlock), 0, st, G, Ph, Sd, V.Qd, C, F);
        LAUNCH_CHECK("imex_dust1");
    }
    MARK(TFSPH_KERNEL_FORCE);

    // stage 2: volumes at the stage-2 positions, drag over gamma tau, explicit terms at Y2
    MARK(TFSPH_KERNEL_BIN);
    r = enqueue_bin<R>(ng, nd, G, V.Qg, V.Qd, V.Sg, V.Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_BIN);
    MARK(TFSPH_KERNEL_UPDATE);
    r = enqueue_relax<R, DIM, false>(c, G, PhE, V, Pg, Pd, nullptr, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_UPDATE);
    if (ng > 0) {
        MARK(TFSPH_KERNEL_DENSITY);
        r = enqueue_density<R, DIM>(G, Ph, V.Sg, 1, st, c->variant);
        if (r != TFSPH_OK) return r;
        MARK(TFSPH_KERNEL_DENSITY);
        MARK(TFSPH_KERNEL_FORCE);
        launch_by_kind<R, DIM>(Ph, V.Sg, [&](auto K) {
            hipLaunchKernelGGL((k_imex_gas2<R, DIM, decltype(K)::value>), dim3(bg), dim3(kBlock), 0, st, G, Ph,
                               V.Sg, V.Xg, F);
        });
        LAUNCH_CHECK("imex_gas2");
        MARK(TFSPH_KERNEL_FORCE);
    }

    // stage 3: predictors in level-n order, volumes at the stage-3 positions, last drag solve
    MARK(TFSPH_KERNEL_UPDATE);
    if (bg + bd > 0) {
        hipLaunchKernelGGL((k_imex_stage3<R, DIM>), dim3(bg + bd), dim3(kBlock), 0, st, G, Ph, Sg, Sd, V.Xg, V.Xd,
                           V.Qg, V.Qd, C, bg, F);
        LAUNCH_CHECK("imex_stage3");
    }
    MARK(TFSPH_KERNEL_UPDATE);
    MARK(TFSPH_KERNEL_BIN);
    r = enqueue_bin<R>(ng, nd, G, V.Qg, V.Qd, V.Sg, V.Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_BIN);
    MARK(TFSPH_KERNEL_UPDATE);
    r = enqueue_relax<R, DIM, true>(c, G, PhE, V, Pg, Pd, Sg.rho, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_UPDATE);
    return TFSPH_OK;
}

// sticky flags (64 words) and the one-phase count / signal-speed words (8) to zero
__global__ void k_clear_flags(unsigned int *word, unsigned long long *one_phase)
{
    word[threadIdx.x] = 0u;
    if (threadIdx.x < 8) one_phase[threadIdx.x] = 0ull;
}

// copy the flags and the one-phase count into caller arrays (either may be null)
__global__ void k_export_flags(const unsigned int *word, const unsigned long long *one_phase, uint32_t *flags_out,
                               int64_t *one_phase_out)
{
    if (threadIdx.x != 0) return;
    if (flags_out) *flags_out = word[0];
    if (one_phase_out) *one_phase_out = (int64_t)one_phase[0];
}

// One step of the comparison schemes (MK or ISPH): binning, both summation
// densities, the explicit gas pass of the IDIC step, then one thread per gas
// particle and one per dust particle for the drag and the update.
template <typename R, int DIM, int SCHEME>
tfsph_status enqueue_step_pair(tfsph_ctx *c, tfsph_state *s, hipStream_t st)
{
    const Geom<R> G = make_geom<R>(&c->p);
    const Phys<R> Ph = make_phys<R>(&c->p);
    Phase<R> Pg = make_phase<R>(s->gas, DIM), Pd = make_phase<R>(s->dust, DIM);
    Sorted<R> Sg, Sd;
    int *partial;
    Flags F;
    VelRho<R> VR;
    carve_all<R>(c, Sg, Sd, partial, F, nullptr, &VR);
    if (c->variant != TFSPH_VARIANT_AUTO) Sg.nmask = nullptr;
    MARK(TFSPH_KERNEL_BIN);
    tfsph_status r = enqueue_bin<R>(c->ng, c->nd, G, Pg, Pd, Sg, Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_BIN);
    MARK(TFSPH_KERNEL_DENSITY);
    if (c->ng > 0) {
        r = enqueue_density<R, DIM>(G, Ph, Sg, 1, st, c->variant);
        if (r != TFSPH_OK) return r;
        hipLaunchKernelGGL((k_pack_vel_rho<R, DIM>), dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, Sg, VR.gas);
        LAUNCH_CHECK("pack_vel_rho");
    }
    if (c->nd > 0) {
        r = enqueue_density<R, DIM>(G, Ph, Sd, 0, st, 0);
        if (r != TFSPH_OK) return r;
        hipLaunchKernelGGL((k_pack_vel_rho<R, DIM>), dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, Sd, VR.dust);
        LAUNCH_CHECK("pack_vel_rho");
    }
    MARK(TFSPH_KERNEL_DENSITY);
    MARK(TFSPH_KERNEL_FORCE);
    r = enqueue_force<R, DIM>(G, Ph, Sg, Pg, st);
    if (r != TFSPH_OK) return r;
    MARK(TFSPH_KERNEL_FORCE);
    MARK(TFSPH_KERNEL_UPDATE);
    if (c->ng > 0) {
        hipLaunchKernelGGL((k_pair_gas<R, DIM, SCHEME>), dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, G, Ph, Sg, Sd,
                           VR.dust, Pg, F);
        LAUNCH_CHECK("pair_gas");
    }
    if (c->nd > 0) {
        hipLaunchKernelGGL((k_pair_dust<R, DIM, SCHEME>), dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, G, Ph, Sg, Sd,
                           VR.gas, Pd, F);
        LAUNCH_CHECK("pair_dust");
    }
    MARK(TFSPH_KERNEL_UPDATE);
    return TFSPH_OK;
}

template <typename R>
tfsph_status enqueue_init(tfsph_ctx *c, tfsph_state *s, hipStream_t st)
{
    const Geom<R> G = make_geom<R>(&c->p);
    Phase<R> Pg = make_phase<R>(s->gas, c->p.dim), Pd = make_phase<R>(s->dust, c->p.dim);
    Sorted<R> Sg, Sd;
    int *partial;
    Flags F;
    ImexViews<R> V;
    const bool imex = c->p.scheme == TFSPH_SCHEME_IMEX2;
    carve_all<R>(c, Sg, Sd, partial, F, imex ? &V : nullptr);
    // a fill kernel rather than a memset node: the no-allocation entry point
    // enqueues this sequence on streams a caller may be capturing
    hipLaunchKernelGGL(k_clear_flags, dim3(1), dim3(64), 0, st, F.word, F.one_phase);
    LAUNCH_CHECK("clear_flags");
    tfsph_status z = enqueue_zero_counts<R>(G.ncell, Sg, Sd, st);
    if (z != TFSPH_OK) return z;
    if (imex) {
        z = enqueue_zero_counts<R>(G.ncell, V.Sg, V.Sd, st);
        if (z != TFSPH_OK) return z;
    }
    if (c->ng > 0) {
        hipLaunchKernelGGL(k_canonicalize<R>, dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, G, Pg, F);
        LAUNCH_CHECK("canonicalize");
    }
    if (c->nd > 0) {
        hipLaunchKernelGGL(k_canonicalize<R>, dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, G, Pd, F);
        LAUNCH_CHECK("canonicalize");
    }
    const Phys<R> Ph = make_phys<R>(&c->p);
    if (c->ng > 0) {
        hipLaunchKernelGGL(k_signal_speed<R>, dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, G, Ph, Pg, 1, F);
        LAUNCH_CHECK("signal_speed");
    }
    if (c->nd > 0) {
        hipLaunchKernelGGL(k_signal_speed<R>, dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, G, Ph, Pd, 0, F);
        LAUNCH_CHECK("signal_speed");
    }
    tfsph_status r = enqueue_bin<R>(c->ng, c->nd, G, Pg, Pd, Sg, Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    if (c->ng > 0) {
        hipLaunchKernelGGL(k_copy_back<R>, dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, G, Sg, Pg, 0);
        LAUNCH_CHECK("copy_back");
    }
    if (c->nd > 0) {
        hipLaunchKernelGGL(k_copy_back<R>, dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, G, Sd, Pd, 0);
        LAUNCH_CHECK("copy_back");
    }
    return TFSPH_OK;
}

template <typename R, int DIM>
tfsph_status enqueue_density(tfsph_ctx *c, tfsph_state *s, int phase, hipStream_t st)
{
    const Geom<R> G = make_geom<R>(&c->p);
    const Phys<R> Ph = make_phys<R>(&c->p);
    Phase<R> Pg = make_phase<R>(s->gas, DIM), Pd = make_phase<R>(s->dust, DIM);
    Sorted<R> Sg, Sd;
    int *partial;
    Flags F;
    carve_all<R>(c, Sg, Sd, partial, F);
    tfsph_status r = enqueue_bin<R>(c->ng, c->nd, G, Pg, Pd, Sg, Sd, partial, F, st);
    if (r != TFSPH_OK) return r;
    Sorted<R> &S = phase == 0 ? Sg : Sd;
    if (S.n > 0) {
        hipLaunchKernelGGL((k_density<R, DIM>), dim3(blocks_for(S.n)), dim3(kBlock), 0, st, G, Ph, S, 0);
        LAUNCH_CHECK("density");
    }
    if (c->ng > 0) {
        hipLaunchKernelGGL(k_copy_back<R>, dim3(blocks_for(c->ng)), dim3(kBlock), 0, st, G, Sg, Pg, phase == 0);
        LAUNCH_CHECK("copy_back");
    }
    if (c->nd > 0) {
        hipLaunchKernelGGL(k_copy_back<R>, dim3(blocks_for(c->nd)), dim3(kBlock), 0, st, G, Sd, Pd, phase == 1);
        LAUNCH_CHECK("copy_back");
    }
    return TFSPH_OK;
}

// follows: the previous step of the same call was enqueued just before on st
template <typename R>
tfsph_status dispatch_step(tfsph_ctx *c, tfsph_state *s, hipStream_t st, bool follows = false)
{
    const bool imex = c->p.scheme == TFSPH_SCHEME_IMEX2;
    if (c->profiling) {
        const long long i = c->prof_steps++;
        c->prof_kind = i % c->prof_every == 0 ? int((i / c->prof_every) % 4) : -1;
    }
    if (c->p.scheme == TFSPH_SCHEME_MK || c->p.scheme == TFSPH_SCHEME_ISPH) {
        const bool mk = c->p.scheme == TFSPH_SCHEME_MK;
        switch (c->p.dim) {
        case 1: return mk ? enqueue_step_pair<R, 1, kPairMK>(c, s, st) : enqueue_step_pair<R, 1, kPairISPH>(c, s, st);
        case 2: return mk ? enqueue_step_pair<R, 2, kPairMK>(c, s, st) : enqueue_step_pair<R, 2, kPairISPH>(c, s, st);
        default: return mk ? enqueue_step_pair<R, 3, kPairMK>(c, s, st) : enqueue_step_pair<R, 3, kPairISPH>(c, s, st);
        }
    }
    switch (c->p.dim) {
    case 1: return imex ? enqueue_step_imex<R, 1>(c, s, st, follows) : enqueue_step<R, 1>(c, s, st);
    case 2: return imex ? enqueue_step_imex<R, 2>(c, s, st, follows) : enqueue_step<R, 2>(c, s, st);
    default: return imex ? enqueue_step_imex<R, 3>(c, s, st, follows) : enqueue_step<R, 3>(c, s, st);
    }
}

template <typename R>
tfsph_status dispatch_density(tfsph_ctx *c, tfsph_state *s, int phase, hipStream_t st)
{
    switch (c->p.dim) {
    case 1: return enqueue_density<R, 1>(c, s, phase, st);
    case 2: return enqueue_density<R, 2>(c, s, phase, st);
    default: return enqueue_density<R, 3>(c, s, phase, st);
    }
}


}  // namespace

// ----------------------------------------------------------------------------
// public entry points
// ----------------------------------------------------------------------------
extern "C" tfsph_status tfsph_init(tfsph_ctx **out, const tfsph_params *p, tfsph_state *s, void *workspace,
                                   size_t ws_bytes, void *hip_stream)
{
    if (!out) return fail(TFSPH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    tfsph_status r = tfsph_validate(p);
    if (r != TFSPH_OK) return r;
    if (!s) return fail(TFSPH_E_INVALID_ARG, "state is NULL");
    r = check_phase(s->gas, p->dim, true, p->eos == TFSPH_ADIABATIC, "gas");
    if (r != TFSPH_OK) return r;
    r = check_phase(s->dust, p->dim, false, false, "dust");
    if (r != TFSPH_OK) return r;
    size_t need = 0;
    r = tfsph_workspace_size(p, s->gas.n, s->dust.n, &need);
    if (r != TFSPH_OK) return r;
    if (!workspace) return fail(TFSPH_E_WORKSPACE, "workspace is NULL");
    if (reinterpret_cast<uintptr_t>(workspace) % 256) return fail(TFSPH_E_WORKSPACE, "workspace must be 256-byte aligned");
    if (ws_bytes < need) return fail(TFSPH_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    tfsph_ctx *c = new (std::nothrow) tfsph_ctx();
    if (!c) return fail(TFSPH_E_INVALID_ARG, "out of host memory");
    c->p = *p;
    c->ng = (int)s->gas.n;
    c->nd = (int)s->dust.n;
    c->fg = gas_flags(p, s->gas.mass != nullptr);
    c->fd = dust_flags(s->dust.mass != nullptr);
    c->mg_uniform = s->gas.mass_uniform;
    c->md_uniform = s->dust.mass_uniform;
    c->ws = static_cast<char *>(workspace);
    c->ws_bytes = ws_bytes;
    c->last_stream = static_cast<hipStream_t>(hip_stream);
    c->cells_per_block = default_cells_per_block(p->dim);
    r = p->precision == TFSPH_F64 ? enqueue_init<double>(c, s, c->last_stream) : enqueue_init<float>(c, s, c->last_stream);
    if (r != TFSPH_OK) {
        delete c;
        return r;
    }
    *out = c;
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_step(tfsph_ctx *c, tfsph_state *s, int32_t n_steps, void *hip_stream)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (n_steps < 0) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 0");
    tfsph_status r = check_state_matches(c, s);
    if (r != TFSPH_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    c->last_stream = st;
    for (int i = 0; i < n_steps; ++i) {
        r = c->p.precision == TFSPH_F64 ? dispatch_step<double>(c, s, st, i > 0) : dispatch_step<float>(c, s, st, i > 0);
        if (r != TFSPH_OK) return r;
    }
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_density(tfsph_ctx *c, tfsph_state *s, int32_t phase, void *hip_stream)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (phase != 0 && phase != 1) return fail(TFSPH_E_INVALID_ARG, "phase must be 0 (gas) or 1 (dust)");
    tfsph_status r = check_state_matches(c, s);
    if (r != TFSPH_OK) return r;
    if (phase == 1 && c->nd > 0 && !s->dust.rho) return fail(TFSPH_E_INVALID_ARG, "dust.rho is NULL");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    c->last_stream = st;
    return c->p.precision == TFSPH_F64 ? dispatch_density<double>(c, s, phase, st)
                                       : dispatch_density<float>(c, s, phase, st);
}

extern "C" tfsph_status tfsph_get_flags(tfsph_ctx *c, uint32_t *flags, int64_t *one_phase_cells)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    Sorted<float> Sg, Sd;
    int *partial;
    Flags F;
    if (c->p.precision == TFSPH_F64) {
        Sorted<double> a, b;
        carve_all<double>(c, a, b, partial, F);
    } else {
        carve_all<float>(c, Sg, Sd, partial, F);
    }
    unsigned int w = 0;
    unsigned long long n = 0;
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(&w, F.word, sizeof(w), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&n, F.one_phase, sizeof(n), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(F.word, 0, sizeof(w)));
    HIP_TRY(hipMemset(F.one_phase, 0, sizeof(n)));
    if (flags) *flags = w;
    if (one_phase_cells) *one_phase_cells = (int64_t)n;
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_signal_speed(tfsph_ctx *c, double *signal_speed)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (!signal_speed) return fail(TFSPH_E_INVALID_ARG, "signal_speed is NULL");
    Sorted<float> Sg, Sd;
    int *partial;
    Flags F;
    if (c->p.precision == TFSPH_F64) {
        Sorted<double> a, b;
        carve_all<double>(c, a, b, partial, F);
    } else {
        carve_all<float>(c, Sg, Sd, partial, F);
    }
    unsigned long long bits = 0;
    HIP_TRY(hipStreamSynchronize(c->last_stream));
    HIP_TRY(hipMemcpy(&bits, F.one_phase + 1, sizeof(bits), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(F.one_phase + 1, 0, sizeof(bits)));
    double s2;
    std::memcpy(&s2, &bits, sizeof(s2));
    *signal_speed = std::sqrt(s2);
    return TFSPH_OK;
}

static void drop_graph(StepGraph &g)
{
    if (g.exec) (void)hipGraphExecDestroy(g.exec);
    if (g.graph) (void)hipGraphDestroy(g.graph);
    g = StepGraph{};
}

extern "C" tfsph_status tfsph_set_cells_per_block(tfsph_ctx *c, int32_t cells)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (cells < 1 || cells > kMaxCellsPerBlock)
        return fail(TFSPH_E_INVALID_ARG, "cells per block %d outside [1, %d]", cells, kMaxCellsPerBlock);
    c->cells_per_block = cells;
    drop_graph(c->sg);
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_set_kernel_variant(tfsph_ctx *c, int32_t variant)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (variant < 0 || variant > 2)
        return fail(TFSPH_E_INVALID_ARG, "unknown kernel variant %d", variant);
    if (variant == TFSPH_VARIANT_LDS_BRICKS)
        return fail(TFSPH_E_UNSUPPORTED, "the LDS-brick pair loops are not built (they were slower than the global "
                                         "loops, and the force pass sums its pair terms in FP64)");
    c->variant = variant;
    drop_graph(c->sg);
    return TFSPH_OK;
}

static tfsph_status start_profile(tfsph_ctx *c, bool on, bool rotate, int every)
{
    if (on) {
        for (auto &T : c->timers) T.used = 0;
        c->prof_steps = 0;
    }
    c->profiling = on;
    c->prof_rotate = rotate;
    c->prof_every = every;
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_profile(tfsph_ctx *c, int32_t enable)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (enable < 0 || enable > 2) return fail(TFSPH_E_INVALID_ARG, "profile mode %d outside 0..2", enable);
    return start_profile(c, enable != 0, enable == 2, 1);
}

extern "C" tfsph_status tfsph_profile_sampled(tfsph_ctx *c, int32_t every)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (every < 1) return fail(TFSPH_E_INVALID_ARG, "sampling interval %d below 1", every);
    return start_profile(c, true, true, every);
}

extern "C" tfsph_status tfsph_profile_read(tfsph_ctx *c, int32_t kernel, double *total_ms, int64_t *launches)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (kernel < 0 || kernel > 3) return fail(TFSPH_E_INVALID_ARG, "unknown kernel id %d", kernel);
    KernelTimer &T = c->timers[kernel];
    double sum = 0.0;
    for (size_t i = 0; i + 1 < T.used; i += 2) {
        HIP_TRY(hipEventSynchronize(T.ev[i + 1]));
        float ms = 0.f;
        HIP_TRY(hipEventElapsedTime(&ms, T.ev[i], T.ev[i + 1]));
        sum += ms;
    }
    if (total_ms) *total_ms = sum;
    if (launches) *launches = (int64_t)(T.used / 2);
    return TFSPH_OK;
}

static unsigned long long state_key(const tfsph_state *s, int chunk)
{
    // FNV-1a over every array address and the chunk length
    unsigned long long h = 1469598103934665603ull;
    auto mix = [&h](const void *p) {
        unsigned long long v = (unsigned long long)(uintptr_t)p;
        for (int i = 0; i < 8; ++i) {
            h ^= (v >> (8 * i)) & 0xff;
            h *= 1099511628211ull;
        }
    };
    for (const tfsph_phase *ph : {&s->gas, &s->dust}) {
        mix(ph->cell), mix(ph->mass), mix(ph->rho), mix(ph->energy), mix(ph->id);
        for (int d = 0; d < 3; ++d) mix(ph->off[d]), mix(ph->vel[d]);
    }
    mix((const void *)(uintptr_t)chunk);
    return h;
}


extern "C" tfsph_status tfsph_step_graph(tfsph_ctx *c, tfsph_state *s, int32_t n_steps, int32_t chunk, void *hip_stream)
{
    if (!c) return fail(TFSPH_E_INVALID_ARG, "ctx is NULL");
    if (n_steps < 0) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 0");
    if (chunk < 1 || chunk > 256) return fail(TFSPH_E_INVALID_ARG, "chunk must be in 1..256");
    tfsph_status r = check_state_matches(c, s);
    if (r != TFSPH_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    c->last_stream = st;
    const int n_full = n_steps / chunk, rem = n_steps % chunk;
    if (n_full > 0) {
        const unsigned long long key = state_key(s, chunk);
        if (!c->sg.exec || c->sg.key != key) {
            drop_graph(c->sg);
            if (!c->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking));
            const bool prof = c->profiling;
            c->profiling = false;
            HIP_TRY(hipStreamBeginCapture(c->capture_stream, hipStreamCaptureModeThreadLocal));
            for (int i = 0; i < chunk && r == TFSPH_OK; ++i)
                r = c->p.precision == TFSPH_F64 ? dispatch_step<double>(c, s, c->capture_stream, i > 0)
                                                : dispatch_step<float>(c, s, c->capture_stream, i > 0);
            hipGraph_t g = nullptr;
            hipError_t e = hipStreamEndCapture(c->capture_stream, &g);
            c->profiling = prof;
            if (r != TFSPH_OK) {
                if (g) (void)hipGraphDestroy(g);
                return r;
            }
            if (e != hipSuccess) return fail(TFSPH_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
            c->sg.graph = g;
            HIP_TRY(hipGraphInstantiate(&c->sg.exec, g, nullptr, nullptr, 0));
            c->sg.key = key;
        }
        for (int k = 0; k < n_full; ++k) HIP_TRY(hipGraphLaunch(c->sg.exec, st));
    }
    for (int i = 0; i < rem; ++i) {
        r = c->p.precision == TFSPH_F64 ? dispatch_step<double>(c, s, st, i > 0) : dispatch_step<float>(c, s, st, i > 0);
        if (r != TFSPH_OK) return r;
    }
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_destroy(tfsph_ctx *c)
{
    if (c) {
        for (auto &T : c->timers)
            for (hipEvent_t e : T.ev) (void)hipEventDestroy(e);
        drop_graph(c->sg);
        if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    }
    delete c;
    return TFSPH_OK;
}

// ----------------------------------------------------------------------------
// Entry point for callers that cannot allocate: the workspace is the library's
// own device array `scratch` (one copy per GPU, held until the process ends).
// Host code never passes the array's name to a kernel or a copy: on the host
// it is only a stand-in for the symbol.  Its device address is looked up once
// per device with hipGetSymbolAddress and kept in g_scratch_ptr.
// ----------------------------------------------------------------------------
namespace {
constexpr size_t kScratchBytes = size_t(64) << 20;     // 64 MiB per GPU
constexpr int kMaxDevices = 64;
void *g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mutex;
}  // namespace

__device__ __align__(256) unsigned char scratch[kScratchBytes];

static tfsph_status scratch_of_current_device(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(TFSPH_E_UNSUPPORTED, "device %d beyond %d devices", dev, kMaxDevices);
    std::lock_guard<std::mutex> lock(g_scratch_mutex);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !ptr)
            return fail(TFSPH_E_HIP, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_step_noalloc(const tfsph_params *p, tfsph_state *s, int32_t n_steps, uint32_t *flags_out,
                                           int64_t *one_phase_out, void *hip_stream)
{
    tfsph_status r = tfsph_validate(p);
    if (r != TFSPH_OK) return r;
    if (!s) return fail(TFSPH_E_INVALID_ARG, "state is NULL");
    if (n_steps < 0) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 0");
    r = check_phase(s->gas, p->dim, true, p->eos == TFSPH_ADIABATIC, "gas");
    if (r != TFSPH_OK) return r;
    r = check_phase(s->dust, p->dim, false, false, "dust");
    if (r != TFSPH_OK) return r;
    const PhaseFlags fg = gas_flags(p, s->gas.mass != nullptr), fd = dust_flags(s->dust.mass != nullptr);
    const size_t need = p->precision == TFSPH_F64 ? plan_bytes<double>(p, (int)s->gas.n, (int)s->dust.n, fg, fd)
                                                  : plan_bytes<float>(p, (int)s->gas.n, (int)s->dust.n, fg, fd);
    if (need > kScratchBytes)
        return fail(TFSPH_E_WORKSPACE, "the problem needs %zu bytes of workspace; the library's static scratch holds %zu",
                    need, kScratchBytes);
    void *ws = nullptr;
    r = scratch_of_current_device(&ws);
    if (r != TFSPH_OK) return r;
    // a context on the stack: nothing is allocated on the host or the device
    tfsph_ctx c;
    c.p = *p;
    c.ng = (int)s->gas.n;
    c.nd = (int)s->dust.n;
    c.fg = fg;
    c.fd = fd;
    c.mg_uniform = s->gas.mass_uniform;
    c.md_uniform = s->dust.mass_uniform;
    c.ws = static_cast<char *>(ws);
    c.ws_bytes = kScratchBytes;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    c.last_stream = st;
    c.cells_per_block = default_cells_per_block(p->dim);
    r = p->precision == TFSPH_F64 ? enqueue_init<double>(&c, s, st) : enqueue_init<float>(&c, s, st);
    if (r != TFSPH_OK) return r;
    for (int i = 0; i < n_steps; ++i) {
        r = p->precision == TFSPH_F64 ? dispatch_step<double>(&c, s, st, i > 0) : dispatch_step<float>(&c, s, st, i > 0);
        if (r != TFSPH_OK) return r;
    }
    if (flags_out || one_phase_out) {
        Sorted<float> Sg, Sd;
        int *partial;
        Flags F;
        if (p->precision == TFSPH_F64) {
            Sorted<double> a, b;
            carve_all<double>(&c, a, b, partial, F);
        } else {
            carve_all<float>(&c, Sg, Sd, partial, F);
        }
        hipLaunchKernelGGL(k_export_flags, dim3(1), dim3(64), 0, st, F.word, F.one_phase, flags_out, one_phase_out);
        LAUNCH_CHECK("export_flags");
    }
    return TFSPH_OK;
}

namespace {
template <typename R>
tfsph_status enqueue_positions(const tfsph_params *p, int n, const double *x, int32_t *cell, void *const off[3],
                               double *xout, bool to_cells, hipStream_t st)
{
    const Geom<R> G = make_geom<R>(p);
    double D[3];
    for (int d = 0; d < 3; ++d) D[d] = d < p->dim ? (p->box_hi[d] - p->box_lo[d]) / p->n_cells[d] : 1.0;
    R *o[3];
    for (int d = 0; d < 3; ++d) o[d] = d < p->dim ? static_cast<R *>(off[d]) : nullptr;
    if (n == 0) return TFSPH_OK;
    if (to_cells) {
        hipLaunchKernelGGL(k_from_positions<R>, dim3(blocks_for(n)), dim3(kBlock), 0, st, G, p->box_lo[0], p->box_lo[1],
                           p->box_lo[2], D[0], D[1], D[2], n, x, cell, o[0], o[1], o[2], (unsigned int *)nullptr);
    } else {
        hipLaunchKernelGGL(k_to_positions<R>, dim3(blocks_for(n)), dim3(kBlock), 0, st, G, p->box_lo[0], p->box_lo[1],
                           p->box_lo[2], D[0], D[1], D[2], n, cell, o[0], o[1], o[2], xout);
    }
    LAUNCH_CHECK("positions");
    return TFSPH_OK;
}

tfsph_status check_positions_args(const tfsph_params *p, int64_t n, const void *x, const int32_t *cell, void *const off[3])
{
    tfsph_status r = tfsph_validate(p);
    if (r != TFSPH_OK) return r;
    if (n < 0 || n > 0x7fffffffLL) return fail(TFSPH_E_INVALID_ARG, "n out of range");
    if (n == 0) return TFSPH_OK;
    if (!x || !cell || !off) return fail(TFSPH_E_INVALID_ARG, "NULL array");
    for (int d = 0; d < p->dim; ++d)
        if (!off[d]) return fail(TFSPH_E_INVALID_ARG, "off[%d] is NULL", d);
    return TFSPH_OK;
}
}  // namespace

extern "C" tfsph_status tfsph_positions_to_cells(const tfsph_params *p, int64_t n, const double *x, int32_t *cell,
                                                 void *off[3], void *hip_stream)
{
    tfsph_status r = check_positions_args(p, n, x, cell, off);
    if (r != TFSPH_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    return p->precision == TFSPH_F64 ? enqueue_positions<double>(p, (int)n, x, cell, off, nullptr, true, st)
                                     : enqueue_positions<float>(p, (int)n, x, cell, off, nullptr, true, st);
}

extern "C" tfsph_status tfsph_cells_to_positions(const tfsph_params *p, int64_t n, const int32_t *cell,
                                                 void *const off[3], double *x, void *hip_stream)
{
    tfsph_status r = check_positions_args(p, n, x, cell, off);
    if (r != TFSPH_OK) return r;
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    return p->precision == TFSPH_F64 ? enqueue_positions<double>(p, (int)n, nullptr, const_cast<int32_t *>(cell), off, x, false, st)
                                     : enqueue_positions<float>(p, (int)n, nullptr, const_cast<int32_t *>(cell), off, x, false, st);
}
