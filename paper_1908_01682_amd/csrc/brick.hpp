// LDS-staged pair sums for 2D / 3D.
//
// A block owns a brick of BX x BY x BZ cells.  It copies the packed records of
// every particle in the brick's halo (the brick grown by the neighbour window
// W on each side, periodic) into LDS once, then every target particle of the
// brick loops over its window from LDS: one ds_read_b128 per candidate instead
// of a scattered 16-byte global load.  The window is walked in the same order
// and with the same arithmetic as for_window(), so the sums are bitwise those
// of the global-memory kernels.  A brick whose halo exceeds the LDS capacity
// falls back to the global loop for its targets.
//
// The update kernel also owns its brick's cells for the drag: per-cell sums,
// closed-form solve and particle update run on the brick's cells.
#pragma once

#include "sph.hpp"

namespace tfsph {

template <int DIM>
struct BrickShape;
template <>
struct BrickShape<2> {
    static constexpr int BX = 8, BY = 8, BZ = 1;
};
template <>
struct BrickShape<3> {
    static constexpr int BX = 4, BY = 4, BZ = 4;
};

// halo particles held in LDS: 48 KiB of records in either precision
template <typename R>
constexpr int brick_cap() { return sizeof(R) == 4 ? 3072 : 1536; }
constexpr int kBrickMaxHalo = 512;     // halo cells

struct BrickGrid {
    int nb[3];          // bricks per axis
    int nbricks;
    int hx, hy, hz;     // halo extent in cells
    int nhalo;          // halo cells
};

template <int DIM>
__device__ __forceinline__ void brick_origin(const BrickGrid &B, int brick, int &bx0, int &by0, int &bz0)
{
    using S = BrickShape<DIM>;
    const int ix = brick % B.nb[0];
    const int r = brick / B.nb[0];
    const int iy = r % B.nb[1];
    const int iz = r / B.nb[1];
    bx0 = ix * S::BX;
    by0 = iy * S::BY;
    bz0 = iz * S::BZ;
}

// Block-wide exclusive scan of one int per thread (NT threads).
template <int NT>
__device__ __forceinline__ int brick_scan(int v, int *lds_waves, int &total)
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
    int pre = 0;
    total = 0;
#pragma unroll
    for (int w = 0; w < NT / 64; ++w) {
        const int t = lds_waves[w];
        if (w < wave) pre += t;
        total += t;
    }
    __syncthreads();
    return pre + x - v;
}

// LDS view of a loaded halo.
template <typename R>
struct Halo {
    R4<R> *data;        // [cap] records in halo-cell order
    int *hstart;        // [nhalo + 1] LDS start of each halo cell
    int *gstart;        // [nhalo] global start of each halo cell
    int total;          // particles in the halo, or -1 if it did not fit
};

// Load the halo of brick (bx0, by0, bz0) from (start, data) into LDS.
// Must be called by the whole block.
template <typename R, int DIM, int NT>
__device__ void load_halo(const Geom<R> &G, const BrickGrid &B, int bx0, int by0, int bz0, const int *start,
                          const R4<R> *data, Halo<R> &H, int *lds_waves)
{
    const int W0 = G.win[0], W1 = DIM > 1 ? G.win[1] : 0, W2 = DIM > 2 ? G.win[2] : 0;
    // per-thread run of halo cells (nhalo <= kBrickMaxHalo <= 2 * NT)
    int cnt[2] = {0, 0}, gs[2] = {0, 0};
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int hc = threadIdx.x * 2 + k;
        if (hc < B.nhalo) {
            const int lx = hc % B.hx, r = hc / B.hx;
            const int ly = r % B.hy, lz = r / B.hy;
            const int cx = wrap_index(bx0 + lx - W0, G.nc[0]);
            const int cy = DIM > 1 ? wrap_index(by0 + ly - W1, G.nc[1]) : 0;
            const int cz = DIM > 2 ? wrap_index(bz0 + lz - W2, G.nc[2]) : 0;
            const int c = join_cell(G, cx, cy, cz);
            gs[k] = start[c];
            cnt[k] = start[c + 1] - gs[k];
        }
    }
    int total;
    const int ex = brick_scan<NT>(cnt[0] + cnt[1], lds_waves, total);
#pragma unroll
    for (int k = 0; k < 2; ++k) {
        const int hc = threadIdx.x * 2 + k;
        if (hc < B.nhalo) {
            H.hstart[hc] = ex + (k ? cnt[0] : 0);
            H.gstart[hc] = gs[k];
        }
    }
    if (threadIdx.x == 0) H.hstart[B.nhalo] = total;
    H.total = total <= brick_cap<R>() ? total : -1;
    __syncthreads();
    if (H.total < 0) return;
    // copy: element e of the halo belongs to the last halo cell with hstart <= e
    for (int e = threadIdx.x; e < total; e += NT) {
        int lo = 0, hi = B.nhalo - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (H.hstart[mid] <= e) lo = mid;
            else hi = mid - 1;
        }
        H.data[e] = data[H.gstart[lo] + (e - H.hstart[lo])];
    }
    __syncthreads();
}

// Walk the window of a target in halo cell (tx, ty, tz) (local halo coords),
// exactly as for_window() walks it in global memory.
template <typename R, int DIM, typename Fn>
__device__ __forceinline__ void for_window_halo(const Geom<R> &G, const BrickGrid &B, const Halo<R> &H, int tx,
                                                int ty, int tz, const R oa[3], Fn &&fn)
{
    const int wz = DIM > 2 ? G.win[2] : 0;
    const int wy = DIM > 1 ? G.win[1] : 0;
    const int wx = G.win[0];
    const int nrow = (2 * wy + 1) * (2 * wz + 1);
    // rows in the pair order of for_window_pairs()
    for (int i = 0; 2 * i < nrow; ++i) {
        const int nt = 2 * i == nrow - 1 ? 1 : 2;
#pragma unroll 1
        for (int t = 0; t < nt; ++t) {
            const int l = t ? nrow - 1 - i : i;
            int dy, dz;
            row_offsets(l, wy, wz, dy, dz);
            const R rz0 = DIM > 2 ? oa[2] - R(dz) * G.delta[2] : R(0);
            const R ry0 = DIM > 1 ? oa[1] - R(dy) * G.delta[1] : R(0);
            const int row = B.hx * ((ty + dy) + B.hy * (tz + dz));
            for (int dx = -wx; dx <= wx; ++dx) {
                const R rx0 = oa[0] - R(dx) * G.delta[0];
                const int hc = (tx + dx) + row;
                visit_range<R, DIM, false>(H.hstart[hc], H.hstart[hc + 1], H.data, rx0, ry0, rz0, fn);
            }
        }
    }
}

// Enumerate the brick's own cells: cell k (0 <= k < BX*BY*BZ) -> halo coords and
// whether it exists (bricks at the upper edge may stick out of the grid).
template <typename R, int DIM>
__device__ __forceinline__ bool brick_cell(const Geom<R> &G, int bx0, int by0, int bz0, int k, int &lx, int &ly,
                                           int &lz, int &c)
{
    using S = BrickShape<DIM>;
    const int ix = k % S::BX, r = k / S::BX;
    const int iy = r % S::BY, iz = r / S::BY;
    const int cx = bx0 + ix, cy = by0 + iy, cz = bz0 + iz;
    lx = ix + G.win[0];
    ly = iy + (DIM > 1 ? G.win[1] : 0);
    lz = iz + (DIM > 2 ? G.win[2] : 0);
    if (cx >= G.nc[0] || (DIM > 1 && cy >= G.nc[1]) || (DIM > 2 && cz >= G.nc[2])) {
        c = -1;
        return false;
    }
    c = join_cell(G, cx, cy, cz);
    return true;
}

template <int DIM>
__device__ __forceinline__ int xcd_brick(int nbricks)
{
    const int b = blockIdx.x;
    const int per = nbricks / 8;
    if (per == 0 || b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

// Shared-memory layout of the brick kernels.
template <typename R>
struct BrickSmem {
    R4<R> data[brick_cap<R>()];
    int hstart[kBrickMaxHalo + 1];
    int gstart[kBrickMaxHalo];
    int tstart[65];             // per brick cell: first target index (flattened over the brick)
    int waves[16];
};

// Targets of the brick, flattened: target t lives in brick cell k with
// tstart[k] <= t < tstart[k+1]; returns the brick cell of t.
__device__ __forceinline__ int find_brick_cell(const int *tstart, int ncells, int t)
{
    int lo = 0, hi = ncells - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (tstart[mid] <= t) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// Fill tstart[] with the target counts of the brick's cells (from the LDS
// halo offsets); returns the number of targets.
template <typename R, int DIM>
__device__ int brick_targets(const Geom<R> &G, const BrickGrid &B, int bx0, int by0, int bz0, const Halo<R> &H,
                             int *tstart)
{
    using S = BrickShape<DIM>;
    constexpr int NC = S::BX * S::BY * S::BZ;
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < NC; ++k) {
            tstart[k] = t;
            int lx, ly, lz, c;
            if (brick_cell<R, DIM>(G, bx0, by0, bz0, k, lx, ly, lz, c)) {
                const int hc = lx + B.hx * (ly + B.hy * lz);
                t += H.hstart[hc + 1] - H.hstart[hc];
            }
        }
        tstart[NC] = t;
    }
    __syncthreads();
    return tstart[NC];
}

// ---------------------------------------------------------------------------
// density, brick form: same sums as k_density
// ---------------------------------------------------------------------------
template <typename R, int DIM, int NT>
__global__ void __launch_bounds__(NT) k_density_brick(Geom<R> G, Phys<R> Ph, Sorted<R> S, BrickGrid B,
                                                      int want_frc)
{
    using Sh = BrickShape<DIM>;
    constexpr int NC = Sh::BX * Sh::BY * Sh::BZ;
    __shared__ BrickSmem<R> sm;
    const int brick = xcd_brick<DIM>(B.nbricks);
    int bx0, by0, bz0;
    brick_origin<DIM>(B, brick, bx0, by0, bz0);
    Halo<R> H;           // members assigned one by one: a brace initialiser of LDS
    H.data = sm.data;    // addresses becomes a constant global, which the backend rejects
    H.hstart = sm.hstart;
    H.gstart = sm.gstart;
    H.total = 0;
    load_halo<R, DIM, NT>(G, B, bx0, by0, bz0, S.start, S.pos, H, sm.waves);
    const int T = brick_targets<R, DIM>(G, B, bx0, by0, bz0, H, sm.tstart);
    for (int t = threadIdx.x; t < T; t += NT) {
        const int k = find_brick_cell(sm.tstart, NC, t);
        int lx, ly, lz, c;
        brick_cell<R, DIM>(G, bx0, by0, bz0, k, lx, ly, lz, c);
        const int hc = lx + B.hx * (ly + B.hy * lz);
        const int a = H.gstart[hc] + (t - sm.tstart[k]);     // global sorted index
        if (H.total < 0) {
            Sorted<R> Sw = S;
            Sw.nmask = nullptr;       // bricks never use neighbour masks
            density_store<R, DIM>(G, Ph, Sw, a, want_frc);
            continue;
        }
        const R4<R> me = sm.data[H.hstart[hc] + (t - sm.tstart[k])];
        const R oa[3] = {me.x, me.y, me.z};
        R acc = R(0);
        for_window_halo<R, DIM>(G, B, H, lx, ly, lz, oa, [&](int, const R4<R> &q, R rx, R ry, R rz, bool ok) {
            const R r2 = rx * rx + ry * ry + rz * rz;
            const R qq = fsqrt(r2) * G.inv_h;
            const R m = ok ? q.w : R(0);
            acc += m * spline_f(qq);
        });
        const R rho = acc * G.wnorm;
        S.rho[a] = rho;
        if (want_frc) {
            const R e = S.energy ? S.energy[a] : R(0);
            S.frc[a] = mk4<R>(me.x, me.y, me.z, pressure_of(Ph, rho, e) / (rho * rho));
        }
    }
}

// ---------------------------------------------------------------------------
// update, brick form (isothermal, no viscosity, uniform gas mass): force from
// LDS, predictor, then the brick cells' drag solve and particle updates
// ---------------------------------------------------------------------------
template <typename R, int DIM, int NT>
__global__ void __launch_bounds__(NT) k_update_brick(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd,
                                                     Phase<R> Pg, Phase<R> Pd, Flags F, BrickGrid B)
{
    using Sh = BrickShape<DIM>;
    constexpr int NC = Sh::BX * Sh::BY * Sh::BZ;
    __shared__ BrickSmem<R> sm;
    __shared__ CellSolve<R> cs[NC];
    __shared__ int cell_of[NC];
    __shared__ int s_bad, s_one;
    const int brick = xcd_brick<DIM>(B.nbricks);
    int bx0, by0, bz0;
    brick_origin<DIM>(B, brick, bx0, by0, bz0);
    if (threadIdx.x == 0) { s_bad = 0; s_one = 0; }
    Halo<R> H;           // members assigned one by one: a brace initialiser of LDS
    H.data = sm.data;    // addresses becomes a constant global, which the backend rejects
    H.hstart = sm.hstart;
    H.gstart = sm.gstart;
    H.total = 0;
    load_halo<R, DIM, NT>(G, B, bx0, by0, bz0, Sg.start, Sg.frc, H, sm.waves);
    const int T = brick_targets<R, DIM>(G, B, bx0, by0, bz0, H, sm.tstart);

    // (1) explicit gas terms and predictor
    for (int t = threadIdx.x; t < T; t += NT) {
        const int k = find_brick_cell(sm.tstart, NC, t);
        int lx, ly, lz, c;
        brick_cell<R, DIM>(G, bx0, by0, bz0, k, lx, ly, lz, c);
        const int hc = lx + B.hx * (ly + B.hy * lz);
        const int a = H.gstart[hc] + (t - sm.tstart[k]);
        if (H.total < 0) {
            Sorted<R> Sw = Sg;
            Sw.nmask = nullptr;
            gas_predict<R, DIM>(G, Ph, Sw, Pg, a);
            continue;
        }
        const R4<R> me = sm.data[H.hstart[hc] + (t - sm.tstart[k])];
        const R oa[3] = {me.x, me.y, me.z};
        const R Pa = me.w;
        const R mu_m = Sg.pos[a].w;
        R ax = R(0), ay = R(0), az = R(0);
        for_window_halo<R, DIM>(G, B, H, lx, ly, lz, oa, [&](int, const R4<R> &q, R rx, R ry, R rz, bool ok) {
            const R r2 = rx * rx + ry * ry + rz * rz;
            const R r = fsqrt(r2);
            const R ir = (ok && r2 > R(0)) ? frcp(r) : R(0);
            const R fac = mu_m * (Pa + q.w) * spline_df(r * G.inv_h) * ir;
            ax -= fac * rx;
            ay -= fac * ry;
            az -= fac * rz;
        });
        const R acc[3] = {ax * G.gnorm, ay * G.gnorm, az * G.gnorm};
#pragma unroll
        for (int d = 0; d < DIM; ++d) Sg.vt[d][a] = Sg.vel[d][a] + Ph.tau * (acc[d] + Ph.g[d]);
    }
    __syncthreads();

    // (2) per-cell sums and implicit solve for the brick's cells
    int one = 0;
    for (int k = threadIdx.x; k < NC; k += NT) {
        int lx, ly, lz, c;
        const bool own = brick_cell<R, DIM>(G, bx0, by0, bz0, k, lx, ly, lz, c);
        cell_of[k] = c;
        if (own) one += solve_cell<R, DIM>(Ph, Sg, Sd, c, cs[k]) ? 1 : 0;
    }
    if (one) atomicAdd(&s_one, one);
    __syncthreads();

    // (3) implicit particle update, move, carry: gas targets, then the brick's dust
    int bad = 0;
    R s2 = signal_floor(Ph);
    for (int t = threadIdx.x; t < T; t += NT) {
        const int k = find_brick_cell(sm.tstart, NC, t);
        int lx, ly, lz, c;
        brick_cell<R, DIM>(G, bx0, by0, bz0, k, lx, ly, lz, c);
        const int hc = lx + B.hx * (ly + B.hy * lz);
        const int a = H.gstart[hc] + (t - sm.tstart[k]);
        bad |= !gas_finish<R, DIM>(G, Ph, Sg, Pg, a, cs[k], s2);
    }
    __syncthreads();
    // dust targets: reuse tstart for the brick's dust counts
    if (threadIdx.x == 0) {
        int t = 0;
        for (int k = 0; k < NC; ++k) {
            sm.tstart[k] = t;
            const int c = cell_of[k];
            if (c >= 0) t += Sd.start[c + 1] - Sd.start[c];
        }
        sm.tstart[NC] = t;
    }
    __syncthreads();
    const int TD = sm.tstart[NC];
    for (int t = threadIdx.x; t < TD; t += NT) {
        const int k = find_brick_cell(sm.tstart, NC, t);
        const int j = Sd.start[cell_of[k]] + (t - sm.tstart[k]);
        bad |= !dust_finish<R, DIM>(G, Ph, Sd, Pd, j, cs[k], s2);
    }
    publish_speed(Ph, F, s2);
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
