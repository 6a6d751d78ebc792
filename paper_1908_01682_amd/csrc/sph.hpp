// SPH sums and the fused IDIC update (Section 2.3, eqs. 17-21).
//
// k_density  : rho_a = sum_b m_b W(|r_ab|, h) over the cell window, self
//              included; also stores p_a / rho_a^2 for the force pass.
// k_gas_predict : explicit gas terms of eq. (19) and the predictor v~, one
//              thread per gas particle.
// k_update   : one block owns a contiguous run of cells (both phases).  It
//              sums mass and momentum of each cell serially in (cell, id)
//              order (no float atomics), solves the 2x2 implicit system of
//              each cell in closed form, updates every particle of its cells,
//              moves it and carries its offset back into [0, Delta).
#pragma once

#include "binning.hpp"
#include "common.hpp"

namespace tfsph {

// Load the chunk of kScanChunk records starting at b of a range ending at b1.
// Padded arrays (sorted pos / frc in global memory, kPad spare records at
// the end) are read straight past b1 from one address; otherwise (LDS) the
// indices are clamped to the range.
template <bool Padded, typename V>
__device__ __forceinline__ void load_chunk(const V *__restrict__ data, int b, int b1, V q[kScanChunk])
{
    if (Padded) {
        const V *p = data + b;
#pragma unroll
        for (int k = 0; k < kScanChunk; ++k) q[k] = p[k];
    } else {
#pragma unroll
        for (int k = 0; k < kScanChunk; ++k) q[k] = data[min(b + k, b1 - 1)];
    }
}

// Visit candidates [b0, b1) of one cell: records are loaded kScanChunk at a time
// so one memory wait serves several candidates; fn(b, q, rx, ry, rz, valid)
// gets the record, r = x_a - x_b and whether b is a real candidate (false
// past b1 in the last chunk; such records are finite but belong elsewhere).
template <typename R, int DIM, bool Padded = true, typename T = R, typename Fn>
__device__ __forceinline__ void visit_range(int b0, int b1, const R4<R> *__restrict__ data, T rx0, T ry0, T rz0,
                                            Fn &fn)
{
    for (int b = b0; b < b1; b += kScanChunk) {
        R4<R> q[kScanChunk];
        load_chunk<Padded>(data, b, b1, q);
        const int rem = b1 - b;        // >= 1: candidate k of the chunk is real when k < rem
#pragma unroll
        for (int k = 0; k < kScanChunk; ++k) {
            const T rx = rx0 - T(q[k].x);
            const T ry = DIM > 1 ? ry0 - T(q[k].y) : T(0);
            const T rz = DIM > 2 ? rz0 - T(q[k].z) : T(0);
            fn(b + k, q[k], rx, ry, rz, k == 0 || k < rem);
        }
    }
}

// Cell ranges [bs[k], be[k]) of one row of the window: cells cx - WX + k,
// k = 0..2 WX (wrapped), of the row starting at linear index `row`.
template <int WX, typename R>
__device__ __forceinline__ void row_ranges(const Geom<R> &G, int cx, int row, const int *__restrict__ start,
                                           int bs[2 * WX + 1], int be[2 * WX + 1])
{
#pragma unroll
    for (int k = 0; k <= 2 * WX; ++k) {
        const int lin = wrap_index(cx - WX + k, G.nc[0]) + row;
        bs[k] = start[lin];
        be[k] = start[lin + 1];
    }
}

// Rows of the window are the (dy, dz) offsets, numbered l = (dz + wz)(2 wy + 1)
// + (dy + wy), l = 0 .. nrow - 1.  They are visited in pairs of opposite rows,
// l = i and nrow - 1 - i for i = 0, 1, ..., the centre row alone last: opposite
// rows hold complementary parts of a particle's support, so the pair's
// neighbour count varies much less between particles than a row's does.
__device__ __forceinline__ void row_offsets(int l, int wy, int wz, int &dy, int &dz)
{
    const int ny = 2 * wy + 1;
    dz = l / ny - wz;
    dy = l % ny - wy;
}

// Walk the window of cell (cx, cy, cz) pair by pair for a window of WX =
// G.win[0] cells on each side along x: pair_fn(i, bs, be, ry0, rz0) gets the
// pair number, the cell ranges of its two rows (bs[t], be[t] as row_ranges;
// the centre row's partner is empty) and the y / z parts of x_a - x_b of each
// row before the candidate's own offset is subtracted.
template <typename R, int DIM, int WX, typename T = R, typename PairFn>
__device__ __forceinline__ void for_window_pairs(const Geom<R> &G, int cx, int cy, int cz, const R oa[3],
                                                 const int *__restrict__ start, PairFn &&pair_fn)
{
    const int wz = DIM > 2 ? G.win[2] : 0;
    const int wy = DIM > 1 ? G.win[1] : 0;
    const int nrow = (2 * wy + 1) * (2 * wz + 1);
    for (int i = 0; 2 * i < nrow; ++i) {
        int bs[2][2 * WX + 1], be[2][2 * WX + 1];
        T ry0[2], rz0[2];
#pragma unroll
        for (int t = 0; t < 2; ++t) {
            const int l = t ? nrow - 1 - i : i;
            if (t == 1 && l == i) {
#pragma unroll
                for (int k = 0; k <= 2 * WX; ++k) bs[1][k] = be[1][k] = 0;
                ry0[1] = ry0[0];
                rz0[1] = rz0[0];
                continue;
            }
            int dy, dz;
            row_offsets(l, wy, wz, dy, dz);
            const int z = DIM > 2 ? wrap_index(cz + dz, G.nc[2]) : 0;
            const int y = DIM > 1 ? wrap_index(cy + dy, G.nc[1]) : 0;
            rz0[t] = DIM > 2 ? T(oa[2]) - T(dz) * T(G.delta[2]) : T(0);
            ry0[t] = DIM > 1 ? T(oa[1]) - T(dy) * T(G.delta[1]) : T(0);
            row_ranges<WX>(G, cx, G.nc[0] * (y + G.nc[1] * z), start, bs[t], be[t]);
        }
        pair_fn(i, bs, be, ry0, rz0);
    }
}

template <int V> struct IntC { static constexpr int value = V; };

// Call f(IntC<wx>) for a window of wx = 1 or 2 cells along x; false (f not
// called) for wider windows.
template <typename F>
__device__ __forceinline__ bool with_row_width(int wx, F &&f)
{
    if (wx == 1) {
        f(IntC<1>{});
        return true;
    }
    if (wx == 2) {
        f(IntC<2>{});
        return true;
    }
    return false;
}

// Visit every particle of a phase in the neighbour window of a point with
// offsets oa[] in cell (cx, cy, cz).  Order: rows in the pair order of
// for_window_pairs(), inside a row x offsets ascending, then cell order.  The
// cell ranges of a pair of rows are loaded together before it is walked.
template <typename R, int DIM, typename T = R, typename Fn>
__device__ __forceinline__ void for_window(const Geom<R> &G, int cx, int cy, int cz, const R oa[3],
                                           const int *__restrict__ start, const R4<R> *__restrict__ data, Fn &&fn)
{
    const bool rows = with_row_width(G.win[0], [&](auto W) {
        constexpr int WX = decltype(W)::value;
        for_window_pairs<R, DIM, WX, T>(G, cx, cy, cz, oa, start, [&](int, auto &bs, auto &be, const T *ry0,
                                                                       const T *rz0) {
#pragma unroll
            for (int t = 0; t < 2; ++t) {
#pragma unroll
                for (int k = 0; k <= 2 * WX; ++k) {
                    const T rx0 = T(oa[0]) - T(k - WX) * T(G.delta[0]);
                    visit_range<R, DIM, true, T>(bs[t][k], be[t][k], data, rx0, ry0[t], rz0[t], fn);
                }
            }
        });
    });
    if (rows) return;
    const int wx = G.win[0];
    const int wz = DIM > 2 ? G.win[2] : 0;
    const int wy = DIM > 1 ? G.win[1] : 0;
    const int nrow = (2 * wy + 1) * (2 * wz + 1);
    for (int i = 0; 2 * i < nrow; ++i) {
        for (int t = 0; t < 2; ++t) {
            const int l = t ? nrow - 1 - i : i;
            if (t == 1 && l == i) break;
            int dy, dz;
            row_offsets(l, wy, wz, dy, dz);
            const int z = DIM > 2 ? wrap_index(cz + dz, G.nc[2]) : 0;
            const T rz0 = DIM > 2 ? T(oa[2]) - T(dz) * T(G.delta[2]) : T(0);
            const int y = DIM > 1 ? wrap_index(cy + dy, G.nc[1]) : 0;
            const T ry0 = DIM > 1 ? T(oa[1]) - T(dy) * T(G.delta[1]) : T(0);
            const int row = G.nc[0] * (y + G.nc[1] * z);
            for (int dx = -wx; dx <= wx; ++dx) {
                const int lin = wrap_index(cx + dx, G.nc[0]) + row;
                const T rx0 = T(oa[0]) - T(dx) * T(G.delta[0]);
                visit_range<R, DIM, true, T>(start[lin], start[lin + 1], data, rx0, ry0, rz0, fn);
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Neighbour masks.  Positions do not change between the density pass and the
// force pass, so the density pass records, for every gas particle and every
// pair of rows of its window (for_window_pairs()), which candidates lie inside
// the support: bit p of pair i is the p-th candidate of the pair in walking
// order (first row, then its opposite; in a row cells dx = -wx..wx, each in
// cell order).  A pair with more than 64 candidates is not recorded; the force
// pass scans such a pair.  The support test is q = sqrt(r^2) / h below kMaskQ
// = 2 (1 + 1e-5), and every force term vanishes exactly for q >= 2 (f'(q) = 0),
// so walking the set bits gives bitwise the sums of the scan.  Masks exist only
// for windows of at most 2 cells on each side along x.
// ---------------------------------------------------------------------------
constexpr int kMaskBits = 64;

// As visit_range(), for the density pass: fn(...) returns whether the
// candidate is a neighbour; returns those answers as bits p0 + (b - b0).
template <typename R, int DIM, typename Fn>
__device__ __forceinline__ unsigned long long visit_range_bits(int b0, int b1, const R4<R> *__restrict__ data, R rx0,
                                                               R ry0, R rz0, int p0, Fn &fn)
{
    unsigned long long m = 0;
    for (int b = b0; b < b1; b += kScanChunk) {
        R4<R> q[kScanChunk];
        load_chunk<true>(data, b, b1, q);
        unsigned nib = 0;
        const int rem = b1 - b;        // >= 1: candidate k of the chunk is real when k < rem
#pragma unroll
        for (int k = 0; k < kScanChunk; ++k) {
            const R rx = rx0 - q[k].x;
            const R ry = DIM > 1 ? ry0 - q[k].y : R(0);
            const R rz = DIM > 2 ? rz0 - q[k].z : R(0);
            nib |= fn(b + k, q[k], rx, ry, rz, k == 0 || k < rem) ? (1u << k) : 0u;
        }
        // bits past 63 only occur in rows longer than kMaskBits, which are
        // never read back
        m |= (unsigned long long)nib << ((p0 + b - b0) & (kMaskBits - 1));
    }
    return m;
}

// Walk the window of a point like for_window() and store the neighbour mask
// of each pair of rows at mask[i * stride] (window of at most 2 cells along x).
template <typename R, int DIM, typename Fn>
__device__ __forceinline__ void for_window_recording(const Geom<R> &G, int cx, int cy, int cz, const R oa[3],
                                                     const int *__restrict__ start, const R4<R> *__restrict__ data,
                                                     unsigned long long *mask, int stride, Fn &&fn)
{
    with_row_width(G.win[0], [&](auto W) {
        constexpr int WX = decltype(W)::value;
        for_window_pairs<R, DIM, WX>(G, cx, cy, cz, oa, start, [&](int i, auto &bs, auto &be, const R *ry0,
                                                                    const R *rz0) {
            unsigned long long m = 0;
            int p0 = 0;
#pragma unroll
            for (int t = 0; t < 2; ++t) {
#pragma unroll
                for (int k = 0; k <= 2 * WX; ++k) {
                    const R rx0 = oa[0] - R(k - WX) * G.delta[0];
                    m |= visit_range_bits<R, DIM>(bs[t][k], be[t][k], data, rx0, ry0[t], rz0[t], p0, fn);
                    p0 += be[t][k] - bs[t][k];
                }
            }
            mask[size_t(i) * stride] = m;
        });
    });
}

// Walking positions of the 2 NC cell ranges (segments) of a pair of rows:
// segment s = t NC + k (row t, cell k) starts at position P[s]; index b of a
// candidate at position p of segment s is p + shift[s].  Returns the pair's
// candidate count.
template <int NC>
__device__ __forceinline__ int pair_segments(const int bs[2][NC], const int be[2][NC], int P[2 * NC],
                                             int shift[2 * NC])
{
    int len = 0;
#pragma unroll
    for (int s = 0; s < 2 * NC; ++s) {
        const int t = s / NC, k = s % NC;
        P[s] = len;
        shift[s] = bs[t][k] - len;
        len += be[t][k] - bs[t][k];
    }
    return len;
}

// Next set bit of m (its position, kept when m is empty) and clear it.
__device__ __forceinline__ bool pop_bit(unsigned long long &m, int &p)
{
    const bool ok = m != 0;
    // m | bit 63 keeps the count defined when m is empty
    const int pj = __builtin_ctzll(m | (1ull << 63));
    p = ok ? pj : p;
    m &= m - 1;
    return ok;
}

// Visit the candidates of one pair of rows whose bits are set in m (bit p =
// the p-th candidate in walking order; segments P, shift as pair_segments(),
// rx0[k] the x part of x_a - x_b for cell k of a row before the candidate's
// own offset, ry0 / rz0 per row as for_window_pairs()); fn(b, q, rx, ry, rz,
// valid) as for for_window().  Candidates are taken kWalk at a time; a lane
// with fewer left repeats its last one with valid = false.  A set bit p is
// decoded by the segment (row t, cell k) it falls in: the row is the second
// one when p >= P[NC], the cell the last one of that row whose segment starts
// at or before p.  With RowRuns (no lane's window wraps around the box along
// x) the cells of every row are consecutive in the sorted order, so one index
// shift serves the whole row.
template <typename R, int DIM, int NC, bool RowRuns, typename T, typename Fn>
__device__ __forceinline__ void walk_bits(unsigned long long m, const int (&P)[2 * NC], const int (&shift)[2 * NC],
                                          const T (&rx0)[NC], const T *ry0, const T *rz0,
                                          const R4<R> *__restrict__ data, Fn &fn)
{
    int p = 0;
    while (m) {
        int b[kWalk];
        T x0[kWalk], y0[kWalk], z0[kWalk];
        bool ok[kWalk];
#pragma unroll
        for (int j = 0; j < kWalk; ++j) {
            ok[j] = pop_bit(m, p);
            const bool t1 = p >= P[NC];
            const int sh0 = shift[0], sh1 = shift[NC];
            int sh = t1 ? sh1 : sh0;
            T xx = rx0[0];
#pragma unroll
            for (int k = 1; k < NC; ++k) {
                const int p0 = P[k], p1 = P[NC + k];
                const bool ge = p >= (t1 ? p1 : p0);
                if constexpr (!RowRuns) {
                    const int s0 = shift[k], s1 = shift[NC + k];
                    sh = ge ? (t1 ? s1 : s0) : sh;
                }
                const T x = rx0[k];
                xx = ge ? x : xx;
            }
            b[j] = p + sh;
            x0[j] = xx;
            y0[j] = DIM > 1 ? (t1 ? ry0[1] : ry0[0]) : ry0[0];
            z0[j] = DIM > 2 ? (t1 ? rz0[1] : rz0[0]) : rz0[0];
        }
        R4<R> q[kWalk];
#pragma unroll
        for (int j = 0; j < kWalk; ++j) q[j] = data[b[j]];
#pragma unroll
        for (int j = 0; j < kWalk; ++j) {
            const T rx = x0[j] - T(q[j].x);
            const T ry = DIM > 1 ? y0[j] - T(q[j].y) : T(0);
            const T rz = DIM > 2 ? z0[j] - T(q[j].z) : T(0);
            fn(b[j], q[j], rx, ry, rz, ok[j]);
        }
    }
}

// Visit the neighbours of a point recorded in mask[i * stride] (pairs of at
// most kMaskBits candidates) or, for longer pairs, every candidate of the
// pair; fn(b, q, rx, ry, rz, valid) as for for_window(), neighbours walked by
// walk_bits().
template <typename R, int DIM, typename T = R, typename Fn>
__device__ __forceinline__ void for_neighbours(const Geom<R> &G, int cx, int cy, int cz, const R oa[3],
                                               const int *__restrict__ start, const R4<R> *__restrict__ data,
                                               const unsigned long long *__restrict__ mask, int stride, Fn &&fn)
{
    with_row_width(G.win[0], [&](auto W) {
        constexpr int WX = decltype(W)::value;
        constexpr int NC = 2 * WX + 1;          // cells per row
        T rx0[NC];
#pragma unroll
        for (int k = 0; k < NC; ++k) rx0[k] = T(oa[0]) - T(k - WX) * T(G.delta[0]);
        const bool wave_rows_contiguous = __ballot(cx < WX || cx + WX >= G.nc[0]) == 0ull;
        for_window_pairs<R, DIM, WX, T>(G, cx, cy, cz, oa, start, [&](int i, auto &bs, auto &be, const T *ry0,
                                                                       const T *rz0) {
            int P[2 * NC], shift[2 * NC];
            if (pair_segments<NC>(bs, be, P, shift) > kMaskBits) {
#pragma unroll
                for (int t = 0; t < 2; ++t)
#pragma unroll
                    for (int k = 0; k < NC; ++k)
                        visit_range<R, DIM, true, T>(bs[t][k], be[t][k], data, rx0[k], ry0[t], rz0[t], fn);
                return;
            }
            const unsigned long long m0 = mask[size_t(i) * stride];
            if (wave_rows_contiguous)
                walk_bits<R, DIM, NC, true, T>(m0, P, shift, rx0, ry0, rz0, data, fn);
            else
                walk_bits<R, DIM, NC, false, T>(m0, P, shift, rx0, ry0, rz0, data, fn);
        });
    });
}

template <typename R>
__device__ __forceinline__ R pressure_of(const Phys<R> &Ph, R rho, R e)
{
    return Ph.eos == 0 ? Ph.cs2 * rho : Ph.gm1 * rho * e;
}

template <typename R>
__device__ __forceinline__ R sound_of(const Phys<R> &Ph, R e)
{
    return Ph.eos == 0 ? Ph.cs : sqrt(Ph.ggm1 * e);
}

// --------------------------------------------------------------------------
// Summation density of phase S at its own sorted particle a.  With `record`
// (gas, masks allocated) the neighbour mask rows of a are stored as well; with
// `own` a's record is returned there (it stays in registers for the caller).
// --------------------------------------------------------------------------
template <typename R, int DIM>
__device__ __forceinline__ R density_at(const Geom<R> &G, const Sorted<R> &S, int a, bool record = false,
                                        R4<R> *own = nullptr)
{
    int cx, cy, cz;
    split_cell(G, S.cell[a], cx, cy, cz);
    const R4<R> me = S.pos[a];
    if (own) *own = me;
    const R oa[3] = {me.x, me.y, me.z};
    R acc = R(0);
    auto term = [&](int, const R4<R> &q, R rx, R ry, R rz, bool ok) {
        const R r2 = rx * rx + ry * ry + rz * rz;
        const R qq = fsqrt(r2) * G.inv_h;
        const R m = ok ? q.w : R(0);
        acc += m * spline_f(qq);
        return ok && qq < R(kMaskQ);
    };
    if (record && S.nmask)
        for_window_recording<R, DIM>(G, cx, cy, cz, oa, S.start, S.pos, S.nmask + a, S.n, term);
    else
        for_window<R, DIM>(G, cx, cy, cz, oa, S.start, S.pos, term);
    return acc * G.wnorm;
}

// density of particle a into S.rho[a]; with want_frc also the force-pass
// record (ox, oy, oz, p / rho^2) and, when allocated, the neighbour masks
template <typename R, int DIM>
__device__ __forceinline__ void density_store(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &S, int a,
                                              int want_frc)
{
    R4<R> me;
    const R rho = density_at<R, DIM>(G, S, a, want_frc != 0, &me);
    S.rho[a] = rho;
    if (want_frc) {
        const R e = S.energy ? S.energy[a] : R(0);
        S.frc[a] = mk4<R>(me.x, me.y, me.z, pressure_of(Ph, rho, e) / (rho * rho));
    }
}

// Block-to-work map.  Consecutive block ids land on different XCDs
// (round-robin dispatch over 8 XCDs); remap so that each XCD works on one
// contiguous slab of cells and the neighbour halos stay in its own L2.
__device__ __forceinline__ int xcd_block(int nblocks)
{
    const int b = blockIdx.x;
    const int per = nblocks / 8;
    if (per == 0 || b >= per * 8) return b;
    return (b % 8) * per + b / 8;
}

template <typename R, int DIM>
__global__ void TFSPH_DENSITY_OCCUPANCY(R) __launch_bounds__(kBlock) k_density(Geom<R> G, Phys<R> Ph, Sorted<R> S,
                                                                         int want_frc)
{
    const int a = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (a >= S.n) return;
    density_store<R, DIM>(G, Ph, S, a, want_frc);
}

// --------------------------------------------------------------------------
// Explicit gas terms at sorted gas particle a: acceleration (without g) and
// de/dt.
//   A_a   = -sum_b m_b (P_a + P_b + Pi_ab) grad_a W_ab,   P = p / rho^2
//   de_a  =  sum_b m_b (P_a + Pi_ab / 2) v_ab . grad_a W_ab
//   Pi_ab = (-alpha cbar mu + beta mu^2) / rhobar  if v_ab . r_ab < 0
//   mu    = h v_ab . r_ab / (r^2 + 0.01 h^2)
// --------------------------------------------------------------------------
// Kinds of gas force loop: isothermal without viscosity and with a uniform
// mass (the common case), the same with per-particle masses, and the general
// one (artificial viscosity and / or the adiabatic EOS with de/dt).
enum { kForceIsoUniform = 0, kForceIsoMass = 1, kForceGeneral = 2 };

template <typename R>
__device__ __forceinline__ int force_kind(const Phys<R> &Ph, const Sorted<R> &S)
{
    if (Ph.av || Ph.eos != 0) return kForceGeneral;
    return S.has_mass ? kForceIsoMass : kForceIsoUniform;
}

// s -= f x, with the product rounded to the term type first when the sum is
// wider (same-type operands keep the contraction into one fused multiply-add)
template <typename A, typename T>
__device__ __forceinline__ void sub_prod(A &s, T f, T x)
{
    if constexpr (std::is_same<A, T>::value)
        s -= f * x;
    else
        s -= A(f * x);
}

template <typename R, int DIM, int KIND>
__device__ __forceinline__ void gas_force_at(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &S, int a,
                                             R acc[3], R &dedt)
{
    using T = typename ForceArith<R>::T;
    using A = typename ForceArith<R>::A;
    int cx, cy, cz;
    split_cell(G, S.cell[a], cx, cy, cz);
    const R4<R> *pos = S.pos;
    const T mu_m = S.pos[a].w;        // uniform mass (kForceIsoUniform)
    const T inv_h = G.inv_h;
    A ax = A(0), ay = A(0), az = A(0), de = A(0);
    // Neighbours from the masks of the density pass when present, else the window, with the
    // separations (o_a - d Delta) - o_b formed in SS (FP64 for an FP32 state) and rounded once to
    // the term type: fn(b, P_b, rx, ry, rz, valid).
    using SS = typename std::conditional<sizeof(R) == 4, double, R>::type;
    const R4<R> me = S.frc[a];
    const T Pa = T(me.w);
    const R oa[3] = {me.x, me.y, me.z};
    auto visit = [&](auto &&fn0) {
        auto fn = [&](int b, const R4<R> &q, SS rx, SS ry, SS rz, bool ok) { fn0(b, T(q.w), T(rx), T(ry), T(rz), ok); };
        if (S.nmask)
            for_neighbours<R, DIM, SS>(G, cx, cy, cz, oa, S.start, S.frc, S.nmask + a, S.n, fn);
        else
            for_window<R, DIM, SS>(G, cx, cy, cz, oa, S.start, S.frc, fn);
    };
    if constexpr (KIND != kForceGeneral) {
        visit([&](int b, T Pb, T rx, T ry, T rz, bool ok) {
            const T r2 = rx * rx + ry * ry + rz * rz;
            T r, ir;
            if constexpr (std::is_same<T, double>::value && std::is_same<R, float>::value) {
                // FP64 terms of an FP32 state: 1/r from the hardware FP32 reciprocal square root
                // and one Newton step in FP64 (relative error about 1e-14)
                const double y0 = double(frsq(float(r2)));
                const double y = y0 * (1.5 - 0.5 * r2 * (y0 * y0));
                const bool live = ok && r2 > 0.0;
                ir = live ? y : 0.0;              // self pair and padding contribute 0
                r = live ? r2 * y : 0.0;
            } else {
                r = fsqrt(r2);
                ir = (ok && r2 > T(0)) ? frcp(r) : T(0);    // self pair and padding contribute 0
            }
            const T mb = KIND == kForceIsoMass ? T(pos[b].w) : mu_m;
            const T fac = mb * (Pa + Pb) * spline_df(r * inv_h) * ir;
            sub_prod(ax, fac, rx);
            sub_prod(ay, fac, ry);
            sub_prod(az, fac, rz);
        });
    } else {
        const bool per_mass = S.has_mass != 0;
        const T va[3] = {S.vel[0][a], DIM > 1 ? S.vel[1][a] : R(0), DIM > 2 ? S.vel[2][a] : R(0)};
        const T rhoa = S.rho[a];
        const T ca = sound_of(Ph, S.energy ? S.energy[a] : R(0));
        visit([&](int b, T Pb, T rx, T ry, T rz, bool ok) {
            const T r2 = rx * rx + ry * ry + rz * rz;
            const T r = fsqrt(r2);
            const T qq = r * inv_h;
            if (ok && qq < T(2) && r2 > T(0)) {
                const T gfac = spline_df(qq) * frcp(r);   // grad_a W = gfac * gnorm * r_vec
                const T vx = va[0] - T(S.vel[0][b]);
                const T vy = DIM > 1 ? va[1] - T(S.vel[1][b]) : T(0);
                const T vz = DIM > 2 ? va[2] - T(S.vel[2][b]) : T(0);
                const T vr = vx * rx + vy * ry + vz * rz;
                T Pi = T(0);
                if (Ph.av && vr < T(0)) {
                    const T mu = T(Ph.h) * vr / (r2 + T(Ph.eta2));
                    const T cb = sound_of(Ph, S.energy ? S.energy[b] : R(0));
                    const T cbar = T(0.5) * (ca + cb);
                    const T rbar = T(0.5) * (rhoa + T(S.rho[b]));
                    Pi = (-T(Ph.av_alpha) * cbar * mu + T(Ph.av_beta) * mu * mu) / rbar;
                }
                const T mb = per_mass ? T(pos[b].w) : mu_m;
                const T fac = mb * (Pa + Pb + Pi) * gfac;
                sub_prod(ax, fac, rx);
                sub_prod(ay, fac, ry);
                sub_prod(az, fac, rz);
                if constexpr (std::is_same<A, T>::value)
                    de += mb * (Pa + T(0.5) * Pi) * gfac * vr;
                else
                    de += A(mb * (Pa + T(0.5) * Pi) * gfac * vr);
            }
        });
    }
    if constexpr (std::is_same<A, R>::value) {
        acc[0] = ax * G.gnorm;
        acc[1] = ay * G.gnorm;
        acc[2] = az * G.gnorm;
        dedt = de * G.gnorm;
    } else {
        acc[0] = R(ax * A(G.gnorm));
        acc[1] = R(ay * A(G.gnorm));
        acc[2] = R(az * A(G.gnorm));
        dedt = R(de * A(G.gnorm));
    }
}

// gas force of particle a with the loop kind picked at run time
template <typename R, int DIM>
__device__ __forceinline__ void gas_force_any(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &S, int a,
                                              R acc[3], R &dedt)
{
    switch (force_kind(Ph, S)) {
    case kForceIsoUniform: gas_force_at<R, DIM, kForceIsoUniform>(G, Ph, S, a, acc, dedt); break;
    case kForceIsoMass: gas_force_at<R, DIM, kForceIsoMass>(G, Ph, S, a, acc, dedt); break;
    default: gas_force_at<R, DIM, kForceGeneral>(G, Ph, S, a, acc, dedt); break;
    }
}

// --------------------------------------------------------------------------
// Per-cell closed-form implicit solve (eqs. 17-21 with first-order time
// differences).  With eps = M_d / M_g, alpha = eps tau / t_stop and
// beta = tau / t_stop (or, K held constant, alpha = tau K V / M_g and
// beta = tau K V / M_d for the cell volume V; or, with t*_stop = T_E / rho*_g,
// alpha = tau M_d / (V T_E) and beta = tau M_g / (V T_E)) the new cell means solve
//   (1 + alpha) V - alpha U = V~,   -beta V + (1 + beta) U = U~,
// so with D = 1 + alpha + beta:
//   V = ((1 + beta) V~ + alpha U~) / D,   U = (beta V~ + (1 + alpha) U~) / D.
// A cell without gas or without dust gets alpha = beta = 0 (no drag).
// --------------------------------------------------------------------------
template <typename R>
struct CellSolve {
    R alpha, beta;
    R V[3], U[3];
};

// Particle count, mass and mean predictor velocity of each phase in one cell.
template <typename R>
struct CellSums {
    int ng, nd;
    R Mg, Md;
    R Vt[3], Ut[3];
};

// Sums over gas [g0, g1) and dust [d0, d1) of one cell; gas(i, m, v) and
// dust(i, m, u) fetch a particle's mass and velocity (v~ for gas, u before the
// gravity kick for dust).  Particles are fetched kChunk at a time (indices
// clamped to the cell) and then added one by one in cell order.
template <typename R, int DIM, typename GasAt, typename DustAt>
__device__ __forceinline__ void cell_sums_with(const Phys<R> &Ph, int g0, int g1, int d0, int d1, GasAt &&gas,
                                               DustAt &&dust, CellSums<R> &S)
{
    R Mg = R(0), Md = R(0);
    R Pg[3] = {R(0), R(0), R(0)}, Pd[3] = {R(0), R(0), R(0)};
    for (int a = g0; a < g1; a += kChunk) {
        R m[kChunk], v[kChunk][3];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) gas(min(a + k, g1 - 1), m[k], v[k]);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (a + k < g1) {
                Mg += m[k];
#pragma unroll
                for (int d = 0; d < DIM; ++d) Pg[d] += m[k] * v[k][d];
            }
        }
    }
    for (int j = d0; j < d1; j += kChunk) {
        R m[kChunk], u[kChunk][3];
#pragma unroll
        for (int k = 0; k < kChunk; ++k) dust(min(j + k, d1 - 1), m[k], u[k]);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            if (j + k < d1) {
                Md += m[k];
#pragma unroll
                for (int d = 0; d < DIM; ++d) Pd[d] += m[k] * (u[k][d] + Ph.tau * Ph.g[d]);
            }
        }
    }
    S.ng = g1 - g0;
    S.nd = d1 - d0;
    S.Mg = Mg;
    S.Md = Md;
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        S.Vt[d] = S.ng > 0 ? Pg[d] / Mg : R(0);
        S.Ut[d] = S.nd > 0 ? Pd[d] / Md : R(0);
    }
}

// Mass and mean predictor velocity of each phase in cell c, summed serially
// in canonical (cell, id) order (eqs. 17, 21 with mass weights).
template <typename R, int DIM>
__device__ __forceinline__ void cell_sums(const Phys<R> &Ph, const Sorted<R> &Sg, const Sorted<R> &Sd, int c,
                                          CellSums<R> &S)
{
    cell_sums_with<R, DIM>(
        Ph, Sg.start[c], Sg.start[c + 1], Sd.start[c], Sd.start[c + 1],
        [&](int i, R &m, R *v) {
            m = Sg.pos[i].w;
#pragma unroll
            for (int d = 0; d < DIM; ++d) v[d] = Sg.vt[d][i];
        },
        [&](int i, R &m, R *u) {
            m = Sd.pos[i].w;
#pragma unroll
            for (int d = 0; d < DIM; ++d) u[d] = Sd.vel[d][i];
        },
        S);
}

// closed-form implicit solve from the cell sums; true for a one-phase cell
template <typename R, int DIM>
__device__ __forceinline__ bool solve_from_sums(const Phys<R> &Ph, const CellSums<R> &S, CellSolve<R> &out)
{
    const bool both = S.ng > 0 && S.nd > 0;
    if (both) {
        if (Ph.drag_law == 1) {
            // K* = K, rho*_g = M_g / V, rho*_d = M_d / V
            out.alpha = Ph.tauKV / S.Mg;
            out.beta = Ph.tauKV / S.Md;
        } else if (Ph.drag_law == 2) {
            // t*_stop = T_E / rho*_g: tau K* / rho*_g = tau rho*_d / T_E, tau K* / rho*_d = tau rho*_g / T_E
            out.alpha = Ph.tau_VTE * S.Md;
            out.beta = Ph.tau_VTE * S.Mg;
        } else {
            const R eps = S.Md / S.Mg;
            out.beta = Ph.beta;
            out.alpha = eps * Ph.beta;
        }
        const R D = R(1) + out.alpha + out.beta;
#pragma unroll
        for (int d = 0; d < DIM; ++d) {
            out.V[d] = ((R(1) + out.beta) * S.Vt[d] + out.alpha * S.Ut[d]) / D;
            out.U[d] = (out.beta * S.Vt[d] + (R(1) + out.alpha) * S.Ut[d]) / D;
        }
    } else {
        out.alpha = out.beta = R(0);
#pragma unroll
        for (int d = 0; d < DIM; ++d) out.V[d] = out.U[d] = R(0);
    }
    return !both && (S.ng > 0 || S.nd > 0);
}

template <typename R, int DIM>
__device__ __forceinline__ bool solve_cell(const Phys<R> &Ph, const Sorted<R> &Sg, const Sorted<R> &Sd, int c,
                                           CellSolve<R> &out)
{
    CellSums<R> S;
    cell_sums<R, DIM>(Ph, Sg, Sd, c, S);
    return solve_from_sums<R, DIM>(Ph, S, out);
}

// Explicit part of eq. (19) for sorted gas particle a: v~ = v + tau (A + g)
// into the predictor scratch, e += tau de/dt into the caller's energy array.
template <typename R, int DIM, int KIND = -1>
__device__ __forceinline__ void gas_predict(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sg,
                                            const Phase<R> &Pg, int a)
{
    // the particle's own velocity is loaded before the neighbour walk, which hides its latency
    R v0[3];
#pragma unroll
    for (int d = 0; d < DIM; ++d) v0[d] = Sg.vel[d][a];
    R acc[3], dedt;
    if constexpr (KIND < 0)
        gas_force_any<R, DIM>(G, Ph, Sg, a, acc, dedt);
    else
        gas_force_at<R, DIM, KIND>(G, Ph, Sg, a, acc, dedt);
#pragma unroll
    for (int d = 0; d < DIM; ++d) Sg.vt[d][a] = v0[d] + Ph.tau * (acc[d] + Ph.g[d]);
    if (Sg.energy) Pg.energy[a] = Sg.energy[a] + Ph.tau * dedt;
}

// A sorted particle's own fields that the finish functions read, loaded ahead
// of the cell sums by the update kernels so that their latency hides there.
template <typename R>
struct Own {
    int cell, id;
    R4<R> pos;
    R rho;
};

template <typename R>
__device__ __forceinline__ Own<R> own_of(const Sorted<R> &S, int a, bool with_rho)
{
    return Own<R>{S.cell[a], S.id[a], S.pos[a], with_rho ? S.rho[a] : R(0)};
}

// Implicit update of eq. (19) for gas particle a of cell C, then
// x^{n+1} = x^n + tau v^{n+1} and the carry; writes the caller's arrays at a
// (and the new cell to *new_cell when given).  With use_own, `own` holds a's
// fields already loaded.
template <typename R, int DIM>
__device__ __forceinline__ bool gas_finish(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sg,
                                           const Phase<R> &Pg, int a, const CellSolve<R> &C, R &s2,
                                           const R4<R> *staged = nullptr, int *new_cell = nullptr,
                                           bool use_own = false, const Own<R> &own = Own<R>{})
{
    const int c = use_own ? own.cell : Sg.cell[a];
    const R inv = R(1) / (R(1) + C.alpha);
    int cc[3];
    split_cell(G, c, cc[0], cc[1], cc[2]);
    const R4<R> me = use_own ? own.pos : Sg.pos[a];
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
    // v~ from the block's LDS copy when it has one: (m, v~x, v~y, v~z)
    R vt[3];
    if (staged) {
        vt[0] = staged->y;
        vt[1] = staged->z;
        vt[2] = staged->w;
    } else {
#pragma unroll
        for (int d = 0; d < DIM; ++d) vt[d] = Sg.vt[d][a];
    }
    R v2 = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R v = (vt[d] + C.alpha * C.U[d]) * inv;
        R o = oo[d] + Ph.tau * v;
        ok &= finite_r(v);
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        Pg.vel[d][a] = v;
        Pg.off[d][a] = o;
        v2 += v * v;
    }
    // signal speed of eq. (4): max(|v|, c), with the sound speed of the new energy
    s2 = fmax(s2, v2);
    if (Ph.eos != 0 && Sg.energy) s2 = fmax(s2, Ph.ggm1 * Pg.energy[a]);
    const int cn = join_cell(G, cc[0], cc[1], cc[2]);
    Pg.cell[a] = cn;
    if (new_cell) *new_cell = cn;
    Pg.id[a] = use_own ? own.id : Sg.id[a];
    if (Sg.has_mass && Pg.mass) const_cast<R *>(Pg.mass)[a] = me.w;
    Pg.rho[a] = use_own ? own.rho : Sg.rho[a];
    return ok;
}

// Implicit update of eq. (20) for dust particle j of cell C, then move + carry
// (the new cell also to *new_cell when given; use_own and `own` as for gas_finish()).
template <typename R, int DIM>
__device__ __forceinline__ bool dust_finish(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sd,
                                            const Phase<R> &Pd, int j, const CellSolve<R> &C, R &s2,
                                            const R4<R> *staged = nullptr, int *new_cell = nullptr,
                                            bool use_own = false, const Own<R> &own = Own<R>{})
{
    const int c = use_own ? own.cell : Sd.cell[j];
    const R inv = R(1) / (R(1) + C.beta);
    int cc[3];
    split_cell(G, c, cc[0], cc[1], cc[2]);
    const R4<R> me = use_own ? own.pos : Sd.pos[j];
    const R oo[3] = {me.x, me.y, me.z};
    bool ok = true;
    // u from the block's LDS copy when it has one: (m, ux, uy, uz)
    R uu[3];
    if (staged) {
        uu[0] = staged->y;
        uu[1] = staged->z;
        uu[2] = staged->w;
    } else {
#pragma unroll
        for (int d = 0; d < DIM; ++d) uu[d] = Sd.vel[d][j];
    }
    R u2 = R(0);
#pragma unroll
    for (int d = 0; d < DIM; ++d) {
        const R ut = uu[d] + Ph.tau * Ph.g[d];
        const R u = (ut + C.beta * C.V[d]) * inv;
        R o = oo[d] + Ph.tau * u;
        ok &= finite_r(u);
        ok &= carry(o, cc[d], G.delta[d], G.nc[d]);
        Pd.vel[d][j] = u;
        Pd.off[d][j] = o;
        u2 += u * u;
    }
    s2 = fmax(s2, u2);
    const int cn = join_cell(G, cc[0], cc[1], cc[2]);
    Pd.cell[j] = cn;
    if (new_cell) *new_cell = cn;
    Pd.id[j] = use_own ? own.id : Sd.id[j];
    if (Sd.has_mass && Pd.mass) const_cast<R *>(Pd.mass)[j] = me.w;
    return ok;
}

// Courant bound of eq. (4), tau < CFL h / max(|v|, c).  A thread's largest
// squared signal speed s2 (isothermal: starts at c_s^2) sets TFSPH_FLAG_CFL when
// it exceeds (CFL h / tau)^2, and raises the device maximum in F.one_phase[1]:
// the bit pattern of a non-negative double orders like its value, so the
// maximum is an integer maximum and does not depend on the order of arrival.
// Every lane of the wave must call it (wave-wide maximum first).
template <typename R>
__device__ __forceinline__ R signal_floor(const Phys<R> &Ph)
{
    return Ph.eos == 0 ? Ph.cs2 : R(0);
}

template <typename R>
__device__ __forceinline__ void publish_speed(const Phys<R> &Ph, const Flags &F, R s2)
{
    if (Ph.vlim2 > R(0) && s2 > Ph.vlim2) atomicOr(F.word, kFlagCfl);
    double m = double(s2);
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = fmax(m, __shfl_xor(m, off, 64));
    if ((threadIdx.x & 63) == 0 && m > 0.0) {
        unsigned long long *dst = F.one_phase + 1;
        const unsigned long long bits = (unsigned long long)__double_as_longlong(m);
        if (bits > __atomic_load_n(dst, __ATOMIC_RELAXED)) atomicMax(dst, bits);
    }
}

// Signal speed of a phase held in the caller's arrays (any order): the device
// maximum of publish_speed() for the state tfsph_init() starts from.
template <typename R>
__global__ void __launch_bounds__(kBlock) k_signal_speed(Geom<R> G, Phys<R> Ph, Phase<R> P, int gas, Flags F)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    R s2 = signal_floor(Ph);
    if (i < P.n) {
        R v2 = R(0);
        for (int d = 0; d < G.dim; ++d) v2 += P.vel[d][i] * P.vel[d][i];
        s2 = fmax(s2, v2);
        if (gas && Ph.eos != 0 && P.energy) s2 = fmax(s2, Ph.ggm1 * P.energy[i]);
    }
    publish_speed(Ph, F, s2);
}

// Explicit gas terms and predictor, one thread per gas particle, specialised
// on the kind of force loop.
template <typename R, int DIM, int KIND>
__global__ void TFSPH_FORCE_OCCUPANCY(R, KIND) __launch_bounds__(kBlock) k_gas_predict(Geom<R> G, Phys<R> Ph, Sorted<R> Sg,
                                                                             Phase<R> Pg)
{
    const int a = xcd_block(gridDim.x) * kBlock + threadIdx.x;
    if (a >= Sg.n) return;
    gas_predict<R, DIM, KIND>(G, Ph, Sg, Pg, a);
}

// Records of a block's particles staged in LDS for the cell sums: up to
// kStage per phase (mass and velocity), else the sums read global memory.
constexpr int kStage = 2 * kBlock;

template <typename R>
constexpr size_t update_lds_bytes(int cells_per_block)
{
    return sizeof(CellSolve<R>) * cells_per_block + 2 * sizeof(R4<R>) * kStage;
}

// Cell sums, implicit solve and particle updates of the cells [c0, c1) of one
// block; the predictor v~ (and e) of the gas comes from k_gas_predict.  The
// block first copies mass and velocity of its particles into LDS with
// coalesced loads, so the serial per-cell sums read LDS.  With CLAIM the
// finished particles also claim their slots in the next step's counting sort
// (the new cell is known here; the histograms must be zero on entry).
template <typename R, int DIM, bool CLAIM>
__device__ __forceinline__ void update_block(const Geom<R> &G, const Phys<R> &Ph, const Sorted<R> &Sg,
                                             const Sorted<R> &Sd, const Phase<R> &Pg, const Phase<R> &Pd,
                                             const Flags &F, int c0, int c1, unsigned char *smem_raw)
{
    R4<R> *stg = reinterpret_cast<R4<R> *>(smem_raw);          // [kStage] gas: m, v~
    R4<R> *std_ = stg + kStage;                                  // [kStage] dust: m, u
    CellSolve<R> *cs = reinterpret_cast<CellSolve<R> *>(std_ + kStage);
    __shared__ int s_bad, s_one;
    if (threadIdx.x == 0) { s_bad = 0; s_one = 0; }

    const int ga = Sg.start[c0], gb = Sg.start[c1];
    const int da = Sd.start[c0], db = Sd.start[c1];
    const bool staged = gb - ga <= kStage && db - da <= kStage;
    if (staged) {
        for (int i = threadIdx.x; i < gb - ga; i += kBlock) {
            const int a = ga + i;
            stg[i] = mk4<R>(Sg.pos[a].w, Sg.vt[0][a], DIM > 1 ? Sg.vt[1][a] : R(0), DIM > 2 ? Sg.vt[2][a] : R(0));
        }
        for (int i = threadIdx.x; i < db - da; i += kBlock) {
            const int j = da + i;
            std_[i] = mk4<R>(Sd.pos[j].w, Sd.vel[0][j], DIM > 1 ? Sd.vel[1][j] : R(0), DIM > 2 ? Sd.vel[2][j] : R(0));
        }
    }
    // the first gas and dust particle of each thread in (2): their fields are loaded now, so
    // that the cell sums hide the latency
    const int a0 = ga + int(threadIdx.x), j0 = da + int(threadIdx.x);
    Own<R> og{}, od{};
    if (a0 < gb) og = own_of(Sg, a0, true);
    if (j0 < db) od = own_of(Sd, j0, false);
    __syncthreads();

    // (1) per-cell sums in canonical order and the implicit solve
    int one = 0;
    for (int c = c0 + threadIdx.x; c < c1; c += kBlock) {
        CellSums<R> S;
        if (staged) {
            cell_sums_with<R, DIM>(
                Ph, Sg.start[c] - ga, Sg.start[c + 1] - ga, Sd.start[c] - da, Sd.start[c + 1] - da,
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
            cell_sums<R, DIM>(Ph, Sg, Sd, c, S);
        }
        one += solve_from_sums<R, DIM>(Ph, S, cs[c - c0]) ? 1 : 0;
    }
    if (one) atomicAdd(&s_one, one);
    __syncthreads();

    // (2) implicit particle update (eqs. 19-20), position update, carry
    int bad = 0;
    R s2 = signal_floor(Ph);
    if constexpr (CLAIM) {
        // every lane of a wave takes part in each claim (wave shuffles); the gas and the dust
        // particle of a thread claim together, so the two atomics are in flight at once
        const int ng = gb - ga, nd = db - da;
        for (int base = 0; base < max(ng, nd); base += kBlock) {
            const int i = base + threadIdx.x;
            int kg = -1, kd = -1;
            const bool first = base == 0;
            if (i < ng) {
                const int cg = first ? og.cell : Sg.cell[ga + i];
                bad |= !gas_finish<R, DIM>(G, Ph, Sg, Pg, ga + i, cs[cg - c0], s2, staged ? &stg[i] : nullptr,
                                           &kg, first, og);
            }
            if (i < nd) {
                const int cd = first ? od.cell : Sd.cell[da + i];
                bad |= !dust_finish<R, DIM>(G, Ph, Sd, Pd, da + i, cs[cd - c0], s2, staged ? &std_[i] : nullptr,
                                            &kd, first, od);
            }
            const int sg = claim_slot(Sg.count, kg);
            const int sd = claim_slot(Sd.count, kd);
            if (i < ng) Sg.slot[ga + i] = sg;
            if (i < nd) Sd.slot[da + i] = sd;
        }
    } else {
        for (int a = a0; a < gb; a += kBlock) {
            const bool first = a == a0;
            const int cg = first ? og.cell : Sg.cell[a];
            bad |= !gas_finish<R, DIM>(G, Ph, Sg, Pg, a, cs[cg - c0], s2, staged ? &stg[a - ga] : nullptr, nullptr,
                                       first, og);
        }
        for (int j = j0; j < db; j += kBlock) {
            const bool first = j == j0;
            const int cd = first ? od.cell : Sd.cell[j];
            bad |= !dust_finish<R, DIM>(G, Ph, Sd, Pd, j, cs[cd - c0], s2, staged ? &std_[j - da] : nullptr, nullptr,
                                        first, od);
        }
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

// One block per contiguous run of cells_per_block cells.
template <typename R, int DIM>
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 8 : 1)))
k_update(Geom<R> G, Phys<R> Ph, Sorted<R> Sg, Sorted<R> Sd, Phase<R> Pg, Phase<R> Pd, Flags F, int cells_per_block,
         int nblocks)
{
    extern __shared__ unsigned char smem_raw[];
    const int blk = xcd_block(nblocks);
    const int c0 = blk * cells_per_block;
    const int c1 = min(c0 + cells_per_block, G.ncell);
    update_block<R, DIM, false>(G, Ph, Sg, Sd, Pg, Pd, F, c0, c1, smem_raw);
}

}  // namespace tfsph
