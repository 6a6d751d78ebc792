// Second-order IMEX step: the ARS(2,2,2) pair of Ascher, Ruuth & Spiteri
// (1997) with the drag in cell (Section 2.3, eqs. 19-21) as its implicit part
// and the drift, the SPH pressure and viscosity terms, gravity and the gas
// energy equation as its explicit part.  With gamma = 1 - 1/sqrt(2) and
// delta = 1 - 1/(2 gamma), from y^n = Y1:
//   Y2 = y^n + gamma tau f(Y1) + gamma tau g(Y2)
//   Y3 = y^n + tau (delta f(Y1) + (1 - delta) f(Y2)) + tau (1 - gamma) g(Y2)
//            + gamma tau g(Y3),   y^{n+1} = Y3.
// Each implicit stage is the first-order drag solve over gamma tau on the
// volumes of that stage's positions.  The stage-2 rate comes from its own
// equation, tau (1 - gamma) g(Y2) = ((1 - gamma) / gamma) (Y2 - Y2~), which
// keeps its digits when the drag is stiff.
//
// Per-particle stage data live in the order of the step's first binning
// ("level-n order"); the later binnings record, for each sorted slot, the
// level-n index it came from (Sorted::src).
#pragma once

#include "sph.hpp"

namespace tfsph {

template <typename R>
struct ImexCoef {
    R tau;    // tau
    R gtau;   // gamma tau
    R del;    // delta
    R omd;    // 1 - delta
    R rg;     // (1 - gamma) / gamma
};

// Stage data of one phase, level-n order (gas fields null for dust).
template <typename R>
struct Stage {
    R *acc1[3], *acc2[3];   // gas: explicit accelerations with g at Y1, Y2
    R *de1, *de2;           // gas, adiabatic: de/dt at Y1, Y2
    R *v2[3];               // velocity after the stage-2 drag solve
    R *dv2[3];              // its drag increment v2 - v2~
};

template <typename R>
__device__ __forceinline__ void set_flag(const Flags &F, bool bad)
{
    if (bad) atomicOr(F.word, 1u);
}

// Stage 1 of the gas, one thread per particle a of the level-n order S:
// explicit terms f(Y1) (stored) and the stage-2 predictor into Q at a:
//   x2 = x^n + gamma tau v^n,  v2~ = v^n + gamma tau (A + g),  e2 = e^n + gamma tau de/dt.
template <typename R, int DIM, int KIND>
__global__ void TFSPH_STAGE_OCCUPANCY(R, KIND) __launch_bounds__(kBlock)
k_imex_gas1(Geom<R> G, Phys<R> Ph, Sorted<R> S, Stage<R> X, Phase<R> Q, ImexCoef<R> C, Flags F)
{
    const int a = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (a >= S.n) return;
    // the particle's own fields are loaded before the neighbour walk, which hides their latency
    const int c0 = S.cell[a], id = S.id[a];
    const R4<R> me = S.pos[a];
    R v0[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) v0[d] = S.vel[d][a];
    R acc[3], dedt;
    gas_force_at<R, DIM, KIND>(G, Ph, S, a, acc, dedt);
    int cc[3];
    split_cell(G, c0, cc[0], cc[1], cc[2]);
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R A = acc[d] + Ph.g[d];
        const R v = v0[d];
        R o = oo[d] + C.gtau * v;
        ok &= finite_r(A);
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        X.acc1[d][a] = A;
        Q.off[d][a] = o;
        Q.vel[d][a] = v + C.gtau * A;
    }
    Q.cell[a] = join_cell(G, cc[0], cc[1], cc[2]);
    Q.id[a] = id;
    if (Q.mass) const_cast<R *>(Q.mass)[a] = me.w;
    if (S.energy) {
        X.de1[a] = dedt;
        Q.energy[a] = S.energy[a] + C.gtau * dedt;
    }
    set_flag<R>(F, !ok);
}

// Stage 1 of the dust: x2 = x^n + gamma tau u^n, u2~ = u^n + gamma tau g.
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock) k_imex_dust1(Geom<R> G, Phys<R> Ph, Sorted<R> S, Phase<R> Q, ImexCoef<R> C,
                                                        Flags F)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    if (j >= S.n) return;
    int cc[3];
    split_cell(G, S.cell[j], cc[0], cc[1], cc[2]);
    const R4<R> me = S.pos[j];
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R u = S.vel[d][j];
        R o = oo[d] + C.gtau * u;
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        Q.off[d][j] = o;
        Q.vel[d][j] = u + C.gtau * Ph.g[d];
    }
    Q.cell[j] = join_cell(G, cc[0], cc[1], cc[2]);
    Q.id[j] = S.id[j];
    if (Q.mass) const_cast<R *>(Q.mass)[j] = me.w;
    set_flag<R>(F, !ok);
}

// Explicit terms f(Y2) of the gas at the stage-2 binning S2 (velocities v2,
// energies e2), stored at the level-n index src[a].
template <typename R, int DIM, int KIND>
__global__ void TFSPH_STAGE_OCCUPANCY(R, KIND) __launch_bounds__(kBlock)
k_imex_gas2(Geom<R> G, Phys<R> Ph, Sorted<R> S, Stage<R> X, Flags F)
{
    const int a = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (a >= S.n) return;
    const int i = S.src[a];       // loaded before the neighbour walk, which hides its latency
    R acc[3], dedt;
    gas_force_at<R, DIM, KIND>(G, Ph, S, a, acc, dedt);
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R A = acc[d] + Ph.g[d];
        ok &= finite_r(A);
        X.acc2[d][i] = A;
    }
    if (S.energy) X.de2[i] = dedt;
    set_flag<R>(F, !ok);
}

// Stage-3 predictor in level-n order, both phases in one grid (blocks below
// blocks_g are gas):
//   x3 = x^n + tau (delta v^n + (1 - delta) v2)
//   v3~ = v^n + tau (delta A1 + (1 - delta) A2) + rg (v2 - v2~)
//   e3 = e^n + tau (delta de1 + (1 - delta) de2)
//   dust: u3~ = u^n + tau g + rg (u2 - u2~).
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_imex_stage3(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, Stage<R> Xg, Stage<R> Xd, Phase<R> Qg,
              Phase<R> Qd, ImexCoef<R> C, int blocks_g, Flags F)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int i = (gas ? blockIdx.x : blockIdx.x - blocks_g) * kBlock + threadIdx.x;
    const Sorted<R> &S = gas ? Sg : Sd;
    const Stage<R> &X = gas ? Xg : Xd;
    const Phase<R> &Q = gas ? Qg : Qd;
    if (i >= S.n) return;
    int cc[3];
    split_cell(G, S.cell[i], cc[0], cc[1], cc[2]);
    const R4<R> me = S.pos[i];
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R v0 = S.vel[d][i];
        R o = oo[d] + C.tau * (C.del * v0 + C.omd * X.v2[d][i]);
        R kick;
        if (gas)
            kick = C.tau * (C.del * X.acc1[d][i] + C.omd * X.acc2[d][i]);
        else
            kick = C.tau * Ph.g[d];          // (the dust stage data hold no accelerations)
        const R v = v0 + kick + C.rg * X.dv2[d][i];
        ok &= finite_r(v);
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        Q.off[d][i] = o;
        Q.vel[d][i] = v;
    }
    Q.cell[i] = join_cell(G, cc[0], cc[1], cc[2]);
    Q.id[i] = S.id[i];
    if (Q.mass) const_cast<R *>(Q.mass)[i] = me.w;
    if (gas && S.energy) Q.energy[i] = S.energy[i] + C.tau * (C.del * X.de1[i] + C.omd * X.de2[i]);
    set_flag<R>(F, !ok);
}

// Stage-1 binning of an IMEX step that follows another one in the same call.
// The final drag solve of that step wrote the caller's arrays at the sorted
// index of its last binning, with the positions that binning used, so they are
// already in canonical (cell, id) order with those cells: a counting sort would
// leave every particle in place.  This copies them into the sorted layout (the
// same values k_rank_gather would gather) and takes that binning's cell
// offsets.  One thread per particle of either phase (gas blocks first); the
// first ncell + 1 threads of each phase also copy its offsets.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_imex_rebin(Geom<R> G, Phase<R> Pg, Sorted<R> Sg, const int *__restrict__ start_g, Phase<R> Pd, Sorted<R> Sd,
             const int *__restrict__ start_d, int blocks_g)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int t = (gas ? int(blockIdx.x) : int(blockIdx.x) - blocks_g) * kBlock + int(threadIdx.x);
    const Phase<R> &P = gas ? Pg : Pd;
    const Sorted<R> &S = gas ? Sg : Sd;
    if (t <= G.ncell) S.start[t] = (gas ? start_g : start_d)[t];
    if (t >= S.n) return;
    S.cell[t] = P.cell[t];
    S.id[t] = P.id[t];
    R o[3] = {R(0), R(0), R(0)};
    for (int d = 0; d < G.dim; ++d) {
        o[d] = P.off[d][t];
        S.vel[d][t] = P.vel[d][t];
    }
    S.pos[t] = mk4<R>(o[0], o[1], o[2], P.mass ? P.mass[t] : P.m_uniform);
    if (S.energy) S.energy[t] = P.energy[t];
    if (S.src) S.src[t] = t;
}

// Implicit drag over gamma tau on the binning (Sg, Sd) whose velocities are the
// stage predictors (Ph carries tau = gamma tau and g = 0, so the cell sums
// take the predictors as they are).  Cell sums and solve as in k_update.
// FINAL = false (stage 2): the new velocities replace the predictors in place
// and go, with their increments, to the level-n order stage data.
// FINAL = true (stage 3): the state y^{n+1} goes to the caller's arrays at the
// sorted index, with the level-n density rho1[src] of each gas particle.
template <typename R, int DIM, bool FINAL>
__global__ void __launch_bounds__(kBlock)
k_imex_relax(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, Stage<R> Xg, Stage<R> Xd, Phase<R> Pg, Phase<R> Pd,
             const R *__restrict__ rho1, Flags F, int cells_per_block, int nblocks)
{
    extern __shared__ unsigned char smem_raw[];
    R4<R> *stg = reinterpret_cast<R4<R> *>(smem_raw);          // [kStage] gas: m, v~
    R4<R> *std_ = stg + kStage;                                  // [kStage] dust: m, u~
    CellSolve<R> *cs = reinterpret_cast<CellSolve<R> *>(std_ + kStage);
    __shared__ int s_bad, s_one;
    const int blk = xcd_block(nblocks);
    const int c0 = blk * cells_per_block;
    const int c1 = min(c0 + cells_per_block, G.ncell);
    if (threadIdx.x == 0) { s_bad = 0; s_one = 0; }

    const int ga = Sg.start[c0], gb = Sg.start[c1];
    const int da = Sd.start[c0], db = Sd.start[c1];
    const bool staged = gb - ga <= kStage && db - da <= kStage;
    if (staged) {
        for (int i = threadIdx.x; i < gb - ga; i += kBlock) {
            const int a = ga + i;
            stg[i] = mk4<R>(Sg.pos[a].w, Sg.vel[0][a], DIM > 1 ? Sg.vel[1][a] : R(0), DIM > 2 ? Sg.vel[2][a] : R(0));
        }
        for (int i = threadIdx.x; i < db - da; i += kBlock) {
            const int j = da + i;
            std_[i] = mk4<R>(Sd.pos[j].w, Sd.vel[0][j], DIM > 1 ? Sd.vel[1][j] : R(0), DIM > 2 ? Sd.vel[2][j] : R(0));
        }
    }
    __syncthreads();

    int one = 0;
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) {
        CellSums<R> S;
        const int g0 = Sg.start[c], g1 = Sg.start[c + 1], d0 = Sd.start[c], d1 = Sd.start[c + 1];
        if (staged) {
            cell_sums_with<R, DIM>(
                Ph, g0 - ga, g1 - ga, d0 - da, d1 - da,
                [&](int i, R &m, R *v) {
                    const R4<R> q = stg[i];
                    m = q.x;
                    v[0] = q.y;
                    v[1] = q.z;
                    v[2] = q.w;
                },
                [&](int i, R &m, R *u) {
                    const R4<R> q = std_[i];
                    m = q.x;
                    u[0] = q.y;
                    u[1] = q.z;
                    u[2] = q.w;
                },
                S);
        } else {
            cell_sums_with<R, DIM>(
                Ph, g0, g1, d0, d1,
                [&](int i, R &m, R *v) {
                    m = Sg.pos[i].w;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) v[d] = Sg.vel[d][i];
                },
                [&](int i, R &m, R *u) {
                    m = Sd.pos[i].w;
#pragma unroll
                    for (int d = 0; d < DIM; ++d) u[d] = Sd.vel[d][i];
                },
                S);
        }
        one += solve_from_sums<R, DIM>(Ph, S, cs[c - c0]) ? 1 : 0;
    }
    if (one) atomicAdd(&s_one, one);
    __syncthreads();

    int bad = 0;
    R s2 = signal_floor(Ph);
    for (int a = ga + threadIdx.x; a < gb; a += kBlock) {
        const CellSolve<R> &Cs = cs[Sg.cell[a] - c0];
        const R inv = R(1) / (R(1) + Cs.alpha);
        const int i = Sg.src[a];
        const R4<R> me = Sg.pos[a];
        const R oo[3] = {me.x, me.y, me.z};
        const R4<R> sv = staged ? stg[a - ga] : R4<R>{};      // (m, v~) from LDS when staged
        R v2 = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const R vt = staged ? (d == 0 ? sv.y : d == 1 ? sv.z : sv.w) : Sg.vel[d][a];
            const R v = (vt + Cs.alpha * Cs.U[d]) * inv;
            bad |= !finite_r(v);
            if constexpr (FINAL) {
                Pg.vel[d][a] = v;
                Pg.off[d][a] = oo[d];
                v2 += v * v;
            } else {
                Sg.vel[d][a] = v;
                Xg.v2[d][i] = v;
                Xg.dv2[d][i] = v - vt;
            }
        }
        if constexpr (FINAL) {
            Pg.cell[a] = Sg.cell[a];
            Pg.id[a] = Sg.id[a];
            if (Sg.has_mass && Pg.mass) const_cast<R *>(Pg.mass)[a] = me.w;
            if (Sg.energy) Pg.energy[a] = Sg.energy[a];
            Pg.rho[a] = rho1[i];
            s2 = fmax(s2, v2);
            if (Ph.eos != 0 && Sg.energy) s2 = fmax(s2, Ph.ggm1 * Sg.energy[a]);
        }
    }
    for (int j = da + threadIdx.x; j < db; j += kBlock) {
        const CellSolve<R> &Cs = cs[Sd.cell[j] - c0];
        const R inv = R(1) / (R(1) + Cs.beta);
        const int i = Sd.src[j];
        const R4<R> me = Sd.pos[j];
        const R oo[3] = {me.x, me.y, me.z};
        const R4<R> su = staged ? std_[j - da] : R4<R>{};     // (m, u~) from LDS when staged
        R u2 = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const R ut = staged ? (d == 0 ? su.y : d == 1 ? su.z : su.w) : Sd.vel[d][j];
            const R u = (ut + Cs.beta * Cs.V[d]) * inv;
            bad |= !finite_r(u);
            if constexpr (FINAL) {
                Pd.vel[d][j] = u;
                Pd.off[d][j] = oo[d];
                u2 += u * u;
            } else {
                Sd.vel[d][j] = u;
                Xd.v2[d][i] = u;
                Xd.dv2[d][i] = u - ut;
            }
        }
        if constexpr (FINAL) {
            Pd.cell[j] = Sd.cell[j];
            Pd.id[j] = Sd.id[j];
            if (Sd.has_mass && Pd.mass) const_cast<R *>(Pd.mass)[j] = me.w;
            s2 = fmax(s2, u2);
        }
    }
    if constexpr (FINAL) publish_speed(Ph, F, s2);
    if (bad) atomicOr(&s_bad, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        if (s_bad) atomicOr(F.word, 1u);
        if (s_one) {
            atomicOr(F.word, 2u);
            atomicAdd(F.one_phase, (unsigned long long)s_one);
        }
    }
}

}  // namespace tfsph
