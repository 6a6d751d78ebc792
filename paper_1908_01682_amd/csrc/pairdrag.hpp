// The paper's two comparison schemes for the drag, both without drag volumes
// (Sections 2.1 and 2.2).  They share the SPH part of the IDIC step (binning,
// summation densities, the gas pressure / viscosity terms and energy
// equation, x^{n+1} = x^n + tau v^{n+1}) and replace its cell solve:
//
// MK, eqs. (8)-(10): explicit pairwise drag with the velocities of level n.
//   For gas a and dust j, X_aj = K_aj / (rho_a rho_j) ((v_a - u_j) . r)
//   / (r^2 + eta^2) r W(r), eta^2 = 0.001 h^2;
//   dv_a/dt gets -sigma sum_j m_j X_aj, du_j/dt gets +sigma sum_a m_a X_aj,
//   with sigma = the dimension (the paper's sigma = 1 in 1D; sigma = d makes
//   the kernel average of r r / r^2 the identity).
// ISPH, eqs. (11)-(16): every particle interpolates the other phase at its
//   own position (velocity, density; at a dust point also the gas pressure)
//   and solves its own two-velocity system with first-order differences:
//   alpha = tau K / rho_g, beta = tau K / rho_d at the point, predictors
//   v~ = v + tau A and u~ = u + tau g; the gas keeps
//   v = ((1 + beta) v~ + alpha u~) / D, the dust u = (beta v~ + (1 + alpha) u~)
//   / D, D = 1 + alpha + beta.  At a dust point A is the gas pressure gradient
//   -sum_i m_i (P_i + P_j) grad_j W_ij + g, P = p / rho^2, summed here as
//   -(sum_i m_i P_i grad W + P_j sum_i m_i grad W).
//
// All sums are gathers over the other phase's window in the sorted
// workspace (no atomics), so results are bitwise reproducible.  One thread
// per particle; each writes its particle's new state to the caller's arrays
// at its sorted index, as k_update does.  The other phase has no neighbour
// masks from a density pass, so for_support() finds each point's partners
// row pair by row pair from positions alone before the pair terms are
// evaluated for those only, each reading its partner's velocity and density
// from one packed record (k_pack_vel_rho).
#pragma once

#include "sph.hpp"

namespace tfsph {

enum { kPairMK = 0, kPairISPH = 1 };

// Each phase's velocity and summation density packed per sorted particle,
// (vx, vy, vz, rho), so that a partner costs one 16-byte load instead of four
// scattered ones; written after the density pass of the phase.
template <typename R>
struct VelRho {
    R4<R> *gas;
    R4<R> *dust;
};

template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock) k_pack_vel_rho(Sorted<R> S, R4<R> *vr)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= S.n) return;
    vr[i] = mk4<R>(S.vel[0][i], DIM > 1 ? S.vel[1][i] : R(0), DIM > 2 ? S.vel[2][i] : R(0), S.rho[i]);
}

// Visit the particles of another phase inside the support of a point, in the
// order of for_window(), with the same fn(b, q, rx, ry, rz, valid): each pair
// of rows of the window is first scanned for candidates with r^2 below
// (kMaskQ h)^2, a little beyond the support q < 2, and only those are handed
// to fn (walk_bits()); a pair of rows with more than kMaskBits candidates is
// handed over whole.  Every pair term vanishes exactly for q >= 2 (W = W' =
// 0), so the sums are those of for_window().  Windows wider than 2 cells
// along x use for_window().
template <typename R, int DIM, typename Fn>
__device__ __forceinline__ void for_support(const Geom<R> &G, int cx, int cy, int cz, const R oa[3],
                                            const int *__restrict__ start, const R4<R> *__restrict__ data, Fn &&fn)
{
    const R cut = R(kMaskQ) * G.h;
    const R cut2 = cut * cut;
    auto inside = [&](int, const R4<R> &, R rx, R ry, R rz, bool ok) {
        return ok && rx * rx + ry * ry + rz * rz < cut2;
    };
    const bool rows = with_row_width(G.win[0], [&](auto W) {
        constexpr int WX = decltype(W)::value;
        constexpr int NC = 2 * WX + 1;
        R rx0[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) rx0[k] = oa[0] - R(k - WX) * G.delta[0];
        const bool wave_rows_contiguous = __ballot(cx < WX || cx + WX >= G.nc[0]) == 0ull;
        for_window_pairs<R, DIM, WX>(G, cx, cy, cz, oa, start, [&](int, auto &bs, auto &be, const R *ry0,
                                                                   const R *rz0) {
            int P[2 * NC], shift[2 * NC];
            if (pair_segments<NC>(bs, be, P, shift) > kMaskBits) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int k = 0; k < NC; ++k)
                        visit_range<R, DIM>(bs[t][k], be[t][k], data, rx0[k], ry0[t], rz0[t], fn);
                return;
            }
            unsigned long long m = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t)
#pragma unroll
                for (int k = 0; k < NC; ++k)
                    m |= visit_range_bits<R, DIM>(bs[t][k], be[t][k], data, rx0[k], ry0[t], rz0[t],
                                                  t ? P[NC + k] : P[k], inside);
            if (wave_rows_contiguous)
                walk_bits<R, DIM, NC, true, R>(m, P, shift, rx0, ry0, rz0, data, fn);
            else
                walk_bits<R, DIM, NC, false, R>(m, P, shift, rx0, ry0, rz0, data, fn);
        });
    });
    if (!rows) for_window<R, DIM>(G, cx, cy, cz, oa, start, data, fn);
}

// K of eq. (7) at a point or a pair, by drag law
template <typename R>
__device__ __forceinline__ R drag_coef(const Phys<R> &Ph, R rho_g, R rho_d)
{
    if (Ph.drag_law == 1) return Ph.Kc;
    if (Ph.drag_law == 2) return rho_g * rho_d * Ph.inv_te;
    return rho_d * Ph.inv_tstop;
}

// K / (rho_g rho_d) of the MK pair term from the inverse densities: the
// t_stop law needs 1/rho_g only, the Epstein law neither
template <typename R>
__device__ __forceinline__ R drag_over_rhos(const Phys<R> &Ph, R inv_rho_g, R inv_rho_d)
{
    if (Ph.drag_law == 1) return Ph.Kc * inv_rho_g * inv_rho_d;
    if (Ph.drag_law == 2) return Ph.inv_te;
    return Ph.inv_tstop * inv_rho_g;
}

// x^{n+1} = x^n + tau v^{n+1}, carry, and the caller's arrays at sorted index i,
// from the particle's own cell, id, record and density that the kernel loaded
// before its walk (a load here would hold the wave for a memory latency)
template <typename R, int DIM>
__device__ __forceinline__ bool store_moved(const Geom<R> &G, const Phys<R> &Ph, const Phase<R> &P, int i,
                                            int cell, int id, const R4<R> &me, R rho, const R v[3], R &s2,
                                            bool has_mass)
{
    int cc[3];
    split_cell(G, cell, cc[0], cc[1], cc[2]);
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
    R v2 = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        R o = oo[d] + Ph.tau * v[d];
        ok &= finite_r(v[d]);
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        P.vel[d][i] = v[d];
        P.off[d][i] = o;
        v2 += v[d] * v[d];
    }
    s2 = fmax(s2, v2);
    P.cell[i] = join_cell(G, cc[0], cc[1], cc[2]);
    P.id[i] = id;
    if (has_mass && P.mass) const_cast<R *>(P.mass)[i] = me.w;
    if (P.rho) P.rho[i] = rho;
    return ok;
}

// One gas particle of MK or ISPH after the explicit gas pass of the IDIC
// step (k_gas_predict: the predictor v~ = v + tau (A + g) in Sg.vt, the new
// energy in the caller's array): the drag from the dust window, update, move.
template <typename R, int DIM, int SCHEME>
__global__ void __launch_bounds__(kBlock)
k_pair_gas(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, const R4<R> *__restrict__ vrd, Phase<R> Pg,
           Flags F)
{
    const int a = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    R s2 = signal_floor(Ph);
    int bad = 0, lonely = 0;
    if (a < Sg.n) {
        const R vt[3] = {Sg.vt[0][a], DIM > 1 ? Sg.vt[1][a] : R(0), DIM > 2 ? Sg.vt[2][a] : R(0)};
        const int cell = Sg.cell[a], id = Sg.id[a];
        int cx, cy, cz;
        split_cell(G, cell, cx, cy, cz);
        const R4<R> me = Sg.pos[a];
        const R oa[3] = {me.x, me.y, me.z};
        const R rho_a = Sg.rho[a];
        R vn[3];
        if constexpr (SCHEME == kPairMK) {
            // the drag of eq. (8) takes the velocities of level n
            const R va[3] = {Sg.vel[0][a], DIM > 1 ? Sg.vel[1][a] : R(0), DIM > 2 ? Sg.vel[2][a] : R(0)};
            const R eta2 = R(0.001) * G.h * G.h;
            const R inv_rho_a = R(1) / rho_a;
            R dx = R(0), dy = R(0), dz = R(0);
            for_support<R, DIM>(G, cx, cy, cz, oa, Sd.start, Sd.pos, [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
                if (!ok) return;
                const R r2 = rx * rx + ry * ry + rz * rz;
                const R w = spline_f(fsqrt(r2) * G.inv_h);
                const R4<R> ub = vrd[b];
                const R inv_rho_b = Ph.drag_law == 1 ? frcp(ub.w) : R(0);   // the K law only
                const R vr = (va[0] - ub.x) * rx + (DIM > 1 ? (va[1] - ub.y) * ry : R(0)) +
                             (DIM > 2 ? (va[2] - ub.z) * rz : R(0));
                const R X = q.w * drag_over_rhos(Ph, inv_rho_a, inv_rho_b) * vr * frcp(r2 + eta2) * w;
                dx -= X * rx;
                dy -= X * ry;
                dz -= X * rz;
            });
            const R sw = R(DIM) * G.wnorm;
            const R dr[3] = {dx * sw, dy * sw, dz * sw};
#pragma unroll
            for (int d = 0; d < DIM; ++d) vn[d] = vt[d] + Ph.tau * dr[d];
        } else {
            R rd = R(0), ux = R(0), uy = R(0), uz = R(0);
            for_support<R, DIM>(G, cx, cy, cz, oa, Sd.start, Sd.pos, [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
                if (!ok) return;
                const R r2 = rx * rx + ry * ry + rz * rz;
                const R mw = q.w * spline_f(fsqrt(r2) * G.inv_h);
                const R4<R> ub = vrd[b];
                const R f = mw * frcp(ub.w);
                rd += mw;
                ux += f * ub.x;
                if (DIM > 1) uy += f * ub.y;
                if (DIM > 2) uz += f * ub.z;
            });
            rd *= G.wnorm;
            const R ua[3] = {ux * G.wnorm, uy * G.wnorm, uz * G.wnorm};
            R alpha = R(0), beta = R(0);
            if (rd > R(0)) {
                const R K = drag_coef(Ph, rho_a, rd);
                alpha = Ph.tau * K / rho_a;
                beta = Ph.tau * K / rd;
            } else {
                lonely = 1;
            }
            const R D = R(1) + alpha + beta;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const R ut = (rd > R(0) ? ua[d] : R(0)) + Ph.tau * Ph.g[d];
                vn[d] = ((R(1) + beta) * vt[d] + alpha * ut) / D;
            }
        }
        if (Sg.energy && Ph.eos != 0) s2 = fmax(s2, Ph.ggm1 * Pg.energy[a]);
        bad = !store_moved<R, DIM>(G, Ph, Pg, a, cell, id, me, rho_a, vn, s2, Sg.has_mass);
    }
    publish_speed(Ph, F, s2);
    if (bad) atomicOr(F.word, 1u);
    if (lonely) {
        atomicOr(F.word, 2u);
        atomicAdd(F.one_phase, 1ull);
    }
}

// One dust particle of MK or ISPH: the drag (MK) or the interpolated gas state
// and pressure gradient (ISPH) from the gas window, update, move.  ISPH walks
// the gas records frc = (ox, oy, oz, P = p / rho^2) of the density pass.
template <typename R, int DIM, int SCHEME>
__global__ void __launch_bounds__(kBlock)
k_pair_dust(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, const R4<R> *__restrict__ vrg, Phase<R> Pd,
            Flags F)
{
    const int j = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    R s2 = signal_floor(Ph);
    int bad = 0, lonely = 0;
    if (j < Sd.n) {
        const int cell = Sd.cell[j], id = Sd.id[j];
        int cx, cy, cz;
        split_cell(G, cell, cx, cy, cz);
        const R4<R> me = Sd.pos[j];
        const R oj[3] = {me.x, me.y, me.z};
        const R uj[3] = {Sd.vel[0][j], DIM > 1 ? Sd.vel[1][j] : R(0), DIM > 2 ? Sd.vel[2][j] : R(0)};
        const R rho_j = Sd.rho[j];
        R un[3];
        if constexpr (SCHEME == kPairMK) {
            const R eta2 = R(0.001) * G.h * G.h;
            const R inv_rho_j = R(1) / rho_j;
            R dx = R(0), dy = R(0), dz = R(0);
            for_support<R, DIM>(G, cx, cy, cz, oj, Sg.start, Sg.pos, [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
                if (!ok) return;
                const R r2 = rx * rx + ry * ry + rz * rz;
                const R w = spline_f(fsqrt(r2) * G.inv_h);
                const R4<R> vb = vrg[b];
                const R inv_rho_b = Ph.drag_law == 2 ? R(0) : frcp(vb.w);   // not needed by the Epstein law
                const R vr = (vb.x - uj[0]) * rx + (DIM > 1 ? (vb.y - uj[1]) * ry : R(0)) +
                             (DIM > 2 ? (vb.z - uj[2]) * rz : R(0));
                const R X = q.w * drag_over_rhos(Ph, inv_rho_b, inv_rho_j) * vr * frcp(r2 + eta2) * w;
                dx += X * rx;
                dy += X * ry;
                dz += X * rz;
            });
            const R sw = R(DIM) * G.wnorm;
            const R dr[3] = {dx * sw, dy * sw, dz * sw};
#pragma unroll
            for (int d = 0; d < DIM; ++d) un[d] = uj[d] + Ph.tau * (Ph.g[d] + dr[d]);
        } else {
            R rg = R(0), pj = R(0), vx = R(0), vy = R(0), vz = R(0);
            R gp[3] = {R(0), R(0), R(0)}, g1[3] = {R(0), R(0), R(0)};
            for_support<R, DIM>(G, cx, cy, cz, oj, Sg.start, Sg.frc, [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
                if (!ok) return;
                const R r2 = rx * rx + ry * ry + rz * rz;
                const R r = fsqrt(r2);
                const R qq = r * G.inv_h;
                const R m = Sg.pos[b].w;
                const R4<R> vb = vrg[b];
                const R rho_b = vb.w;
                const R mw = m * spline_f(qq);
                const R f = mw * frcp(rho_b);
                rg += mw;
                pj += mw * (q.w * rho_b);                   // m_b W p_b / rho_b (P_b = p_b / rho_b^2)
                vx += f * vb.x;
                if (DIM > 1) vy += f * vb.y;
                if (DIM > 2) vz += f * vb.z;
                const R ir = r2 > R(0) ? frcp(r) : R(0);
                const R md = m * spline_df(qq) * ir;           // m_b grad_j W / (gnorm r_vec)
                const R rr[3] = {rx, ry, rz};
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    gp[d] += md * q.w * rr[d];
                    g1[d] += md * rr[d];
                }
            });
            rg *= G.wnorm;
            R alpha = R(0), beta = R(0), A[3] = {R(0), R(0), R(0)};
            const R vj[3] = {vx * G.wnorm, vy * G.wnorm, vz * G.wnorm};
            if (rg > R(0)) {
                const R Pj = pj * G.wnorm / (rg * rg);
#pragma unroll
                for (int d = 0; d < DIM; ++d) A[d] = -(gp[d] + Pj * g1[d]) * G.gnorm;
                const R K = drag_coef(Ph, rg, rho_j);
                alpha = Ph.tau * K / rg;
                beta = Ph.tau * K / rho_j;
            } else {
                lonely = 1;
            }
            const R D = R(1) + alpha + beta;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                const R vt = vj[d] + Ph.tau * (A[d] + Ph.g[d]);
                const R ut = uj[d] + Ph.tau * Ph.g[d];
                un[d] = (beta * vt + (R(1) + alpha) * ut) / D;
            }
        }
        bad = !store_moved<R, DIM>(G, Ph, Pd, j, cell, id, me, rho_j, un, s2, Sd.has_mass);
    }
    publish_speed(Ph, F, s2);
    if (bad) atomicOr(F.word, 1u);
    if (lonely) {
        atomicOr(F.word, 2u);
        atomicAdd(F.one_phase, 1ull);
    }
}

}  // namespace tfsph
