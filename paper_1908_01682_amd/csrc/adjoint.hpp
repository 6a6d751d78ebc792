// Hand-written reverse mode of the IDIC step (Section 2.3, eqs. 17-21) for
// the isothermal EOS without artificial viscosity.
//
// The cells and the neighbour sets of every step are held at the values of
// the forward pass (they are piecewise constant in the inputs).  With
// w = dL/dv_new + tau dL/dx_new (the position update x_new = x + tau v_new),
// the reverse of one step is, per cell (alpha, beta, V*, U* as in the forward
// solve, D = 1 + alpha + beta):
//   Ubar = sum_a w_a alpha/(1+alpha),   alphabar = sum_a w_a.(U* - v_a)/(1+alpha)
//   Vbar = sum_j z_j beta/(1+beta),     betabar  = sum_j z_j.(V* - u_j)/(1+beta)
//   V~bar = (Vbar (1+beta) + Ubar beta) / D,   U~bar = (Vbar alpha + Ubar (1+alpha)) / D
//   alphabar += (Vbar.(U~ - V*) + Ubar.(U~ - U*)) / D
//   betabar  += (Vbar.(V~ - V*) + Ubar.(V~ - U*)) / D
//   d/d log t_stop += -alpha alphabar - beta betabar      (alpha, beta proportional to 1/t_stop;
//                                                          with K held constant, d/d log(1/K))
//   v~bar_a = w_a/(1+alpha) + (m_a/M_g) V~bar,   ubar_j = z_j/(1+beta) + (m_j/M_d) U~bar
// then through the explicit SPH terms (A = tau v~bar):
//   Pbar_a = -sum_b (m_b Abar_a - m_a Abar_b) . G_ab
//   xbar_a -= sum_b (P_a + P_b) H_ab (m_b Abar_a - m_a Abar_b)
//   rhobar_a = -Pbar_a P_a / rho_a                         (P = c_s^2 / rho)
//   xbar_a += sum_b (m_b rhobar_a + m_a rhobar_b) G_ab
// with G = grad W and H its Hessian.  Every sum is in gather form over the
// symmetric neighbour relation: no atomics, fixed order.
#pragma once

#include "sph.hpp"

namespace tfsph {

// f''(q) = 1.5 max(2-q, 0) - 6 max(1-q, 0) of the cubic spline
template <typename R>
__device__ __forceinline__ R spline_ddf(R q)
{
    const R t2 = fmax(R(2) - q, R(0));
    const R t1 = fmax(R(1) - q, R(0));
    return R(1.5) * t2 - R(6) * t1;
}

// Adjoint arrays of one phase (SoA, per axis).
template <typename R>
struct AdjPhase {
    R *x[3];
    R *v[3];
};

// ---------------------------------------------------------------------------
// per-cell reverse of the implicit update and cell solve.  A block owns a run
// of cells_per_block cells: its particles' records (m, v~ or u~, and the
// incoming adjoint w = vbar + tau xbar) are staged in LDS with coalesced loads
// (up to kAdjStage per phase, else read from global memory), one thread per
// cell runs the serial cell sums and the reverse of the 2x2 solve, and the
// per-particle outputs are written one thread per particle.
// ---------------------------------------------------------------------------
constexpr int kAdjStage = kBlock;

template <typename R>
struct AdjCellOut {
    R ia, ib, rg, rd;       // 1/(1+alpha), 1/(1+beta), 1/M_g, 1/M_d
    R Vtb[3], Utb[3];       // adjoints of the cell's mean predictor velocities
    int both;               // the cell holds both phases (drag acts)
};

template <typename R>
constexpr size_t adj_cell_lds_bytes(int cells_per_block)
{
    return sizeof(AdjCellOut<R>) * cells_per_block + 4 * sizeof(R4<R>) * kAdjStage;
}

template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_cell(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, AdjPhase<R> outg, AdjPhase<R> outd,
           AdjPhase<R> vtb_g /* v: v~bar (sorted) */, R *abar0, R *abar1, R *abar2, AdjPhase<R> ubi_d,
           double *sbar_part, int cells_per_block)
{
    extern __shared__ unsigned char smem_raw[];
    R4<R> *gm = reinterpret_cast<R4<R> *>(smem_raw);      // [kAdjStage] gas: m, v~
    R4<R> *gw = gm + kAdjStage;                             // [kAdjStage] gas: w
    R4<R> *dm = gw + kAdjStage;                             // [kAdjStage] dust: m, u~
    R4<R> *dw = dm + kAdjStage;                             // [kAdjStage] dust: z
    AdjCellOut<R> *co = reinterpret_cast<AdjCellOut<R> *>(dw + kAdjStage);
    __shared__ double red[kBlock];
    R *abar[3] = {abar0, abar1, abar2};
    const R tau = Ph.tau;
    const int c0 = blockIdx.x * cells_per_block;
    const int c1 = min(c0 + cells_per_block, G.ncell);
    const int ga = Sg.start[c0], gb = Sg.start[c1];
    const int da = Sd.start[c0], db = Sd.start[c1];
    const bool staged = gb - ga <= kAdjStage && db - da <= kAdjStage;

    // w of gas particle a: the adjoint reaching its new velocity (through x^{n+1} = x + tau v too)
    auto w_of = [&](int a, int d) { return outg.v[d][a] + tau * outg.x[d][a]; };
    auto z_of = [&](int j, int d) { return outd.v[d][j] + tau * outd.x[d][j]; };
    if (staged) {
        for (int i = threadIdx.x; i < gb - ga; i += kBlock) {
            const int a = ga + i;
            gm[i] = mk4<R>(Sg.pos[a].w, Sg.vt[0][a], DIM > 1 ? Sg.vt[1][a] : R(0), DIM > 2 ? Sg.vt[2][a] : R(0));
            gw[i] = mk4<R>(w_of(a, 0), DIM > 1 ? w_of(a, 1) : R(0), DIM > 2 ? w_of(a, 2) : R(0), R(0));
        }
        for (int i = threadIdx.x; i < db - da; i += kBlock) {
            const int j = da + i;
            dm[i] = mk4<R>(Sd.pos[j].w, Sd.vel[0][j], DIM > 1 ? Sd.vel[1][j] : R(0), DIM > 2 ? Sd.vel[2][j] : R(0));
            dw[i] = mk4<R>(z_of(j, 0), DIM > 1 ? z_of(j, 1) : R(0), DIM > 2 ? z_of(j, 2) : R(0), R(0));
        }
    }
    __syncthreads();
    // per-particle reads, from LDS when staged
    auto gas_m = [&](int a, R &m, R *v) {
        if (staged) {
            const R4<R> q = gm[a - ga];
            m = q.x; v[0] = q.y; v[1] = q.z; v[2] = q.w;
        } else {
            m = Sg.pos[a].w;
#pragma unroll
            for (int d = 0; d < DIM; ++d) v[d] = Sg.vt[d][a];
        }
    };
    auto dust_m = [&](int j, R &m, R *u) {
        if (staged) {
            const R4<R> q = dm[j - da];
            m = q.x; u[0] = q.y; u[1] = q.z; u[2] = q.w;
        } else {
            m = Sd.pos[j].w;
#pragma unroll
            for (int d = 0; d < DIM; ++d) u[d] = Sd.vel[d][j];
        }
    };
    auto gas_w = [&](int a, R *w) {
        if (staged) {
            const R4<R> q = gw[a - ga];
            w[0] = q.x; w[1] = q.y; w[2] = q.z;
        } else {
#pragma unroll
            for (int d = 0; d < DIM; ++d) w[d] = w_of(a, d);
        }
    };
    auto dust_w = [&](int j, R *z) {
        if (staged) {
            const R4<R> q = dw[j - da];
            z[0] = q.x; z[1] = q.y; z[2] = q.z;
        } else {
#pragma unroll
            for (int d = 0; d < DIM; ++d) z[d] = z_of(j, d);
        }
    };

    // (1) one thread per cell: sums, solve and its reverse
    double sbar = 0.0;
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) {
        CellSums<R> S;
        const int g0 = Sg.start[c], g1 = Sg.start[c + 1];
        const int d0 = Sd.start[c], d1 = Sd.start[c + 1];
        cell_sums_with<R, DIM>(Ph, g0, g1, d0, d1, gas_m, dust_m, S);
        CellSolve<R> C;
        solve_from_sums<R, DIM>(Ph, S, C);
        AdjCellOut<R> &o = co[c - c0];
        o.both = S.ng > 0 && S.nd > 0;
        if (o.both) {
            const R ia = R(1) / (R(1) + C.alpha), ib = R(1) / (R(1) + C.beta);
            R Ubar[3] = {R(0), R(0), R(0)}, Vbar[3] = {R(0), R(0), R(0)};
            R abar_c = R(0), bbar_c = R(0);
            for (int a = g0; a < g1; ++a) {
                R m, vt[3], w[3];
                gas_m(a, m, vt);
                gas_w(a, w);
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    const R vnew = (vt[d] + C.alpha * C.U[d]) * ia;
                    Ubar[d] += w[d] * C.alpha * ia;
                    abar_c += w[d] * (C.U[d] - vnew) * ia;
                }
            }
            for (int j = d0; j < d1; ++j) {
                R m, u[3], z[3];
                dust_m(j, m, u);
                dust_w(j, z);
#pragma unroll
                for (int d = 0; d < DIM; ++d) {
                    const R ut = u[d] + tau * Ph.g[d];
                    const R unew = (ut + C.beta * C.V[d]) * ib;
                    Vbar[d] += z[d] * C.beta * ib;
                    bbar_c += z[d] * (C.V[d] - unew) * ib;
                }
            }
            const R D = R(1) + C.alpha + C.beta;
#pragma unroll
            for (int d = 0; d < DIM; ++d) {
                o.Vtb[d] = (Vbar[d] * (R(1) + C.beta) + Ubar[d] * C.beta) / D;
                o.Utb[d] = (Vbar[d] * C.alpha + Ubar[d] * (R(1) + C.alpha)) / D;
                abar_c += (Vbar[d] * (S.Ut[d] - C.V[d]) + Ubar[d] * (S.Ut[d] - C.U[d])) / D;
                bbar_c += (Vbar[d] * (S.Vt[d] - C.V[d]) + Ubar[d] * (S.Vt[d] - C.U[d])) / D;
            }
            sbar += -double(C.alpha) * double(abar_c) - double(C.beta) * double(bbar_c);
            o.ia = ia;
            o.ib = ib;
            o.rg = R(1) / S.Mg;
            o.rd = R(1) / S.Md;
        }
    }
    __syncthreads();

    // (2) one thread per particle: the adjoints of v~ and u~
    for (int a = ga + threadIdx.x; a < gb; a += kBlock) {
        const AdjCellOut<R> &o = co[Sg.cell[a] - c0];
        R m, vt[3], w[3];
        gas_m(a, m, vt);
        gas_w(a, w);
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            const R vb = o.both ? w[d] * o.ia + m * o.rg * o.Vtb[d] : w[d];
            vtb_g.v[d][a] = vb;
            abar[d][a] = tau * vb;
        }
    }
    for (int j = da + threadIdx.x; j < db; j += kBlock) {
        const AdjCellOut<R> &o = co[Sd.cell[j] - c0];
        R m, u[3], z[3];
        dust_m(j, m, u);
        dust_w(j, z);
#pragma unroll
        for (int d = 0; d < DIM; ++d) ubi_d.v[d][j] = o.both ? z[d] * o.ib + m * o.rd * o.Utb[d] : z[d];
    }

    // block sum of d/d log t_stop in a fixed tree order
    red[threadIdx.x] = sbar;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) sbar_part[blockIdx.x] = red[0];
}

// ---------------------------------------------------------------------------
// pair pass 1 (gas): reverse of the pressure acceleration
// ---------------------------------------------------------------------------
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_force(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, const R *abar0, const R *abar1, const R *abar2,
            AdjPhase<R> outg /* x: xbar of the step output (sorted) */, R *xacc0, R *xacc1, R *xacc2, R *rhobar)
{
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= Sg.n) return;
    const R *abar[3] = {abar0, abar1, abar2};
    R *xacc[3] = {xacc0, xacc1, xacc2};
    int cx, cy, cz;
    split_cell(G, Sg.cell[a], cx, cy, cz);
    const R4<R> me = Sg.frc[a];
    const R oa[3] = {me.x, me.y, me.z};
    const R Pa = me.w;
    const R ma = Sg.pos[a].w;
    const bool per_mass = Sg.has_mass != 0;
    const R Aa[3] = {abar[0][a], DIM > 1 ? abar[1][a] : R(0), DIM > 2 ? abar[2][a] : R(0)};
    R Pbar = R(0);
    R xb[3] = {R(0), R(0), R(0)};
    const R inv_h = G.inv_h;
    auto term = [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
        const R r2 = rx * rx + ry * ry + rz * rz;
        if (ok && r2 < G.support2 && r2 > R(0)) {
            const R ir = frsq(r2);
            const R r = r2 * ir;
            const R qq = r * inv_h;
            const R f1 = spline_df(qq) * ir;                       // f'(q) / r
            const R f2 = (spline_ddf(qq) * inv_h - f1) * ir * ir;  // (f''/h - f'/r) / r^2
            const R mb = per_mass ? Sg.pos[b].w : ma;
            const R w0 = mb * Aa[0] - ma * abar[0][b];
            const R w1 = DIM > 1 ? mb * Aa[1] - ma * abar[1][b] : R(0);
            const R w2 = DIM > 2 ? mb * Aa[2] - ma * abar[2][b] : R(0);
            const R rw = rx * w0 + ry * w1 + rz * w2;
            Pbar -= f1 * rw;                                      // (w . G) / gnorm
            const R ps = Pa + q.w;
            xb[0] -= ps * (f1 * w0 + f2 * rw * rx);
            xb[1] -= ps * (f1 * w1 + f2 * rw * ry);
            xb[2] -= ps * (f1 * w2 + f2 * rw * rz);
        }
    };
    // the neighbours recorded by the step's density pass when the tape has masks
    if (Sg.nmask)
        for_neighbours<R, DIM>(G, cx, cy, cz, oa, Sg.start, Sg.frc, Sg.nmask + a, Sg.n, term);
    else
        for_window<R, DIM>(G, cx, cy, cz, oa, Sg.start, Sg.frc, term);
    Pbar *= G.gnorm;
    rhobar[a] = -Pbar * Pa / Sg.rho[a];
#pragma unroll
    for (int d = 0; d < DIM; ++d) xacc[d][a] = outg.x[d][a] + xb[d] * G.gnorm;
}

// ---------------------------------------------------------------------------
// pair pass 2 (any phase): reverse of the summation density
//   xbar_a += sum_b (m_b rhobar_a + m_a rhobar_b) grad W_ab
// ---------------------------------------------------------------------------
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_density(Geom<R> G, Sorted<R> S, const R *rhobar, R *xacc0, R *xacc1, R *xacc2)
{
    const int a = blockIdx.x * kBlock + threadIdx.x;
    if (a >= S.n) return;
    R *xacc[3] = {xacc0, xacc1, xacc2};
    int cx, cy, cz;
    split_cell(G, S.cell[a], cx, cy, cz);
    const R4<R> me = S.pos[a];
    const R oa[3] = {me.x, me.y, me.z};
    const R ma = me.w;
    const R ra = rhobar[a];
    R xb[3] = {R(0), R(0), R(0)};
    auto term = [&](int b, const R4<R> &q, R rx, R ry, R rz, bool ok) {
        const R r2 = rx * rx + ry * ry + rz * rz;
        if (ok && r2 < G.support2 && r2 > R(0)) {
            const R ir = frsq(r2);
            const R f1 = spline_df(r2 * ir * G.inv_h) * ir;
            const R c = (q.w * ra + ma * rhobar[b]) * f1;
            xb[0] += c * rx;
            xb[1] += c * ry;
            xb[2] += c * rz;
        }
    };
    if (S.nmask)
        for_neighbours<R, DIM>(G, cx, cy, cz, oa, S.start, S.pos, S.nmask + a, S.n, term);
    else
        for_window<R, DIM>(G, cx, cy, cz, oa, S.start, S.pos, term);
#pragma unroll
    for (int d = 0; d < DIM; ++d) xacc[d][a] += xb[d] * G.gnorm;
}

// ---------------------------------------------------------------------------
// loss: L = (1/N) sum_j (rho_j - target[id_j])^2 over the (sorted) dust
// ---------------------------------------------------------------------------
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock)
k_adj_loss(Geom<R> G, Sorted<R> S, const R *target, int n_total, R *rhobar, double *loss_part)
{
    const int j = blockIdx.x * kBlock + threadIdx.x;
    double l = 0.0;
    if (j < S.n) {
        const R rho = density_at<R, DIM>(G, S, j);
        const int id = S.id[j];
        const R t = (id >= 0 && id < n_total) ? target[id] : R(0);
        const R resid = rho - t;
        rhobar[j] = R(2) * resid / R(n_total);
        l = double(resid) * double(resid);
    }
    __shared__ double red[kBlock];
    red[threadIdx.x] = l;
    __syncthreads();
    for (int s = kBlock / 2; s > 0; s >>= 1) {
        if (threadIdx.x < s) red[threadIdx.x] += red[threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss_part[blockIdx.x] = red[0];
}

// sum n partials in a fixed order into *acc (one block); scale applied to the sum
__global__ void __launch_bounds__(kBlock) k_adj_reduce(const double *part, int n, double scale, double *acc,
                                                       int accumulate)
{
    __shared__ double red[kBlock];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *acc = (accumulate ? *acc : 0.0) + scale * red[0];
}

// out[b] = sum of part[b n .. (b + 1) n) in a fixed order, one block per row b
__global__ void __launch_bounds__(kBlock) k_adj_reduce_rows(const double *part, int n, double *out)
{
    __shared__ double red[kBlock];
    const double *row = part + size_t(blockIdx.x) * n;
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += kBlock) s += row[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = kBlock / 2; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

// out[src[dst]] = in[dst] for each axis (undo one step's sort); also zero-fills nothing
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_adj_unsort(int n, int dim, const int *src, const R *in0, const R *in1, const R *in2, R *out0, R *out1, R *out2)
{
    const int dst = blockIdx.x * kBlock + threadIdx.x;
    if (dst >= n) return;
    const int i = src[dst];
    if (i < 0 || i >= n) return;
    out0[i] = in0[dst];
    if (dim > 1) out1[i] = in1[dst];
    if (dim > 2) out2[i] = in2[dst];
}

// The four unsorts of a reverse step in one launch: blocks below blocks_g undo
// the gas sort (src_g) for positions and velocities, the others the dust sort.
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_adj_unsort_step(int ng, int nd, int dim, int blocks_g, const int *src_g, const int *src_d, AdjPhase<R> in_g,
                  AdjPhase<R> out_g, AdjPhase<R> in_d, AdjPhase<R> out_d)
{
    const bool gas = int(blockIdx.x) < blocks_g;
    const int dst = (gas ? blockIdx.x : blockIdx.x - blocks_g) * kBlock + threadIdx.x;
    const int n = gas ? ng : nd;
    if (dst >= n) return;
    const int i = (gas ? src_g : src_d)[dst];
    if (i < 0 || i >= n) return;
    const AdjPhase<R> &in = gas ? in_g : in_d;
    const AdjPhase<R> &out = gas ? out_g : out_d;
    for (int d = 0; d < dim; ++d) {
        out.x[d][i] = in.x[d][dst];
        out.v[d][i] = in.v[d][dst];
    }
}

// out[d][id[i]] = in[d][i]  (final gradient in id order)
template <typename R>
__global__ void __launch_bounds__(kBlock)
k_adj_by_id(int n, int dim, const int *id, const R *in0, const R *in1, const R *in2, R *out0, R *out1, R *out2)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i >= n) return;
    const int k = id[i];
    if (k < 0 || k >= n) return;
    out0[k] = in0[i];
    if (dim > 1) out1[k] = in1[i];
    if (dim > 2) out2[k] = in2[i];
}

// plain element copy (state snapshots), n elements of T
template <typename T>
__global__ void __launch_bounds__(kBlock) k_copy(const T *in, T *out, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = in[i];
}

template <typename T>
__global__ void __launch_bounds__(kBlock) k_fill(T *out, T v, int n)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i < n) out[i] = v;
}

}  // namespace tfsph
