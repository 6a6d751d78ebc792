// Host-side helpers shared by the library's translation units: error
// reporting, workspace carving and the typed device views of a problem.
#pragma once

#include "../../include/tfsph.h"

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>

#include "common.hpp"

namespace tfsph_host {

using namespace tfsph;

extern thread_local char g_last_error[512];

inline tfsph_status fail(tfsph_status s, const char *fmt, ...)
{
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_last_error, sizeof(g_last_error), fmt, ap);
    va_end(ap);
    return s;
}

#define HIP_TRY(expr)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (expr);                                                                \
        if (e_ != hipSuccess) return fail(TFSPH_E_HIP, "%s: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

#define LAUNCH_CHECK(name)                                                                          \
    do {                                                                                            \
        hipError_t e_ = hipGetLastError();                                                          \
        if (e_ != hipSuccess) return fail(TFSPH_E_HIP, "launch %s: %s", name, hipGetErrorString(e_)); \
    } while (0)

inline int window_of(const tfsph_params *p, int d)
{
    const double D = (p->box_hi[d] - p->box_lo[d]) / p->n_cells[d];
    return (int)std::ceil(2.0 * p->h / D - 1e-12);
}

// 64-bit neighbour masks per gas particle: one per pair of opposite window
// rows, (nrow + 1) / 2 with nrow = (2 wy + 1)(2 wz + 1), when the window spans
// at most 5 cells along x, else 0 (no masks; the force pass scans the window).
inline int mask_rows_of(const tfsph_params *p)
{
    if (window_of(p, 0) > 2) return 0;
    int r = 1;
    for (int d = 1; d < p->dim; ++d) r *= 2 * window_of(p, d) + 1;
    return (r + 1) / 2;
}

struct Carver {
    size_t off = 0;
    char *base = nullptr;
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~size_t(255);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += sizeof(T) * (count ? count : 1);
        return p;
    }
};

struct PhaseFlags {
    bool mass;      // per-particle mass array present
    bool energy;    // energy array present
    bool prs;       // gas: force record and predictor scratch
    int mask_rows = 0;   // gas: rows of neighbour bits per particle (0: no masks)
};

template <typename R>
Sorted<R> carve_phase(Carver &cv, int n, int dim, int ncell, PhaseFlags f)
{
    Sorted<R> S{};
    S.n = n;
    S.has_mass = f.mass ? 1 : 0;
    S.cell = cv.take<int>(n);
    S.id = cv.take<int>(n);
    S.pos = cv.take<R4<R>>(size_t(n) + kPad);
    S.frc = f.prs ? cv.take<R4<R>>(size_t(n) + kPad) : nullptr;
    for (int d = 0; d < 3; ++d) {
        S.vel[d] = d < dim ? cv.take<R>(n) : nullptr;
        S.vt[d] = (f.prs && d < dim) ? cv.take<R>(n) : nullptr;
    }
    S.energy = f.energy ? cv.take<R>(n) : nullptr;
    S.rho = cv.take<R>(n);
    S.count = cv.take<int>(ncell);
    S.start = cv.take<int>(size_t(ncell) + 1);
    S.slot = cv.take<int>(n);
    S.tmp_idx = cv.take<int>(n);
    S.tmp_id = cv.take<int>(n);
    S.nmask = f.mask_rows > 0 ? cv.take<unsigned long long>(size_t(f.mask_rows) * n) : nullptr;
    return S;
}

inline int ncell_of(const tfsph_params *p)
{
    int n = 1;
    for (int d = 0; d < p->dim; ++d) n *= p->n_cells[d];
    return n;
}

inline int blocks_for(int n) { return (n + kBlock - 1) / kBlock; }

template <typename R>
Geom<R> make_geom(const tfsph_params *p)
{
    Geom<R> G{};
    static const double sig[4] = {0.0, 2.0 / 3.0, 10.0 / (7.0 * M_PI), 1.0 / M_PI};
    G.dim = p->dim;
    G.ncell = ncell_of(p);
    for (int d = 0; d < 3; ++d) {
        G.nc[d] = d < p->dim ? p->n_cells[d] : 1;
        G.win[d] = d < p->dim ? window_of(p, d) : 0;
        G.delta[d] = d < p->dim ? R((p->box_hi[d] - p->box_lo[d]) / p->n_cells[d]) : R(1);
    }
    G.h = R(p->h);
    G.inv_h = R(1.0 / p->h);
    G.support2 = R(4.0 * p->h * p->h);
    G.wnorm = R(sig[p->dim] / std::pow(p->h, p->dim));
    G.gnorm = R(sig[p->dim] / std::pow(p->h, p->dim + 1));
    return G;
}

template <typename R>
Phys<R> make_phys(const tfsph_params *p)
{
    Phys<R> P{};
    P.eos = p->eos;
    P.av = (p->av_alpha != 0.0 || p->av_beta != 0.0) ? 1 : 0;
    P.cs = R(p->c_s);
    P.cs2 = R(p->c_s * p->c_s);
    P.gm1 = R(p->gamma - 1.0);
    P.ggm1 = R(p->gamma * (p->gamma - 1.0));
    P.tau = R(p->dt);
    P.drag_law = p->K > 0.0 ? 1 : (p->t_stop_epstein > 0.0 ? 2 : 0);
    P.beta = P.drag_law == 0 ? R(p->dt / p->t_stop) : R(0);
    double vol = 1.0;
    for (int d = 0; d < p->dim; ++d) vol *= (p->box_hi[d] - p->box_lo[d]) / p->n_cells[d];
    P.tauKV = R(p->dt * p->K * vol);
    P.tau_VTE = P.drag_law == 2 ? R(p->dt / (vol * p->t_stop_epstein)) : R(0);
    for (int d = 0; d < 3; ++d) P.g[d] = d < p->dim ? R(p->g[d]) : R(0);
    P.av_alpha = R(p->av_alpha);
    P.av_beta = R(p->av_beta);
    P.eta2 = R(0.01 * p->h * p->h);
    P.h = R(p->h);
    P.vlim2 = p->cfl > 0.0 ? R((p->cfl * p->h / p->dt) * (p->cfl * p->h / p->dt)) : R(0);
    P.inv_tstop = P.drag_law == 0 ? R(1.0 / p->t_stop) : R(0);
    P.Kc = R(p->K);
    P.inv_te = P.drag_law == 2 ? R(1.0 / p->t_stop_epstein) : R(0);
    return P;
}

template <typename R>
Phase<R> make_phase(const tfsph_phase &ph, int dim)
{
    Phase<R> P{};
    P.n = (int)ph.n;
    P.cell = ph.cell;
    for (int d = 0; d < 3; ++d) {
        P.off[d] = d < dim ? static_cast<R *>(ph.off[d]) : nullptr;
        P.vel[d] = d < dim ? static_cast<R *>(ph.vel[d]) : nullptr;
    }
    P.mass = static_cast<const R *>(ph.mass);
    P.m_uniform = R(ph.mass_uniform);
    P.rho = static_cast<R *>(ph.rho);
    P.energy = static_cast<R *>(ph.energy);
    P.id = ph.id;
    return P;
}

tfsph_status check_phase(const tfsph_phase &ph, int dim, bool need_rho, bool need_energy, const char *name);

}  // namespace tfsph_host
