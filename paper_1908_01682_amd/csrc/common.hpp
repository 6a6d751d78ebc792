// Device-side building blocks shared by every TFSPH kernel (gfx950, wave64).
//
// Position representation: linear cell index + per-axis offset inside the
// cell, 0 <= off < Delta.  Pair separations are formed as
// (off_a - d Delta) - off_b where d is the window offset of b's cell, so no
// absolute coordinate (and no periodic wrap of a coordinate) is ever formed;
// FP32 keeps ~1e-7 of a cell width of resolution anywhere in the box.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace tfsph {

constexpr int kBlock = 256;          // threads per block of the streaming kernels
constexpr int kMaxWindow = 128;      // largest neighbour window half-width (cells)

// --------------------------------------------------------------------------
// Smoothing kernel W(h, r) of Section 2.1: M4 cubic spline, support 2h,
// W = sigma_d h^-d f(r/h) with f = 1 - 1.5 q^2 + 0.75 q^3 on [0,1),
// 0.25 (2-q)^3 on [1,2), 0 beyond.  The same function is written here without
// branches as f = 0.25 max(2-q, 0)^3 - max(1-q, 0)^3 (for q < 1 the two cubes
// expand to the first polynomial), so f, f' and f'' vanish beyond the support
// and a pair loop needs no range test.
// --------------------------------------------------------------------------
// saturate to [0, 1]
__device__ __forceinline__ float sat(float x) { return __builtin_amdgcn_fmed3f(x, 0.0f, 1.0f); }
__device__ __forceinline__ double sat(double x) { return fmin(fmax(x, 0.0), 1.0); }

// For q >= 0: t1 = max(1-q, 0) = sat(1 - q) and s = max(2-q, 0) / 2 =
// sat(1 - q/2), so f = 0.25 (2s)^3 - t1^3 = 2 s^3 - t1^3.
template <typename R>
__device__ __forceinline__ R spline_f(R q)
{
    const R s = sat(R(1) - R(0.5) * q);
    const R t1 = sat(R(1) - q);
    return R(2) * (s * s * s) - t1 * t1 * t1;
}

// f'(q) = 3 max(1-q, 0)^2 - 0.75 max(2-q, 0)^2 = 3 (t1^2 - s^2)
template <typename R>
__device__ __forceinline__ R spline_df(R q)
{
    const R s = sat(R(1) - R(0.5) * q);
    const R t1 = sat(R(1) - q);
    return R(3) * (t1 * t1 - s * s);
}

// Tuning knobs, fixed at compile time: records loaded together before any is
// used (cell sums, id ranking), candidates loaded together by the window
// scans of the pair kernels, neighbours taken together by the mask walk, and
// an optional waves-per-SIMD floor for the pair kernels.
#ifndef TFSPH_CHUNK
#define TFSPH_CHUNK 4
#endif
// Two candidates per load in the window scans: the 3D density pass takes
// 0.347 ms against 0.370 with four (fewer registers held by loads in flight).
#ifndef TFSPH_SCAN_CHUNK
#define TFSPH_SCAN_CHUNK 2
#endif
#ifndef TFSPH_WALK
#define TFSPH_WALK 2
#endif
#ifdef TFSPH_PAIR_WAVES_PER_EU
#define TFSPH_DENSITY_OCCUPANCY(R) __attribute__((amdgpu_waves_per_eu(TFSPH_PAIR_WAVES_PER_EU)))
#define TFSPH_FORCE_OCCUPANCY(R, KIND) TFSPH_DENSITY_OCCUPANCY(R)
#define TFSPH_STAGE_OCCUPANCY(R, KIND) TFSPH_DENSITY_OCCUPANCY(R)
#else
// Waves per SIMD of the FP32 density pass on the 3D box, against the
// compiler's choice: at 7 (72 VGPRs, 12 bytes spilled per lane) it takes 0.336 ms
// against 0.345 at 6 (79 VGPRs).  FP64 would spill heavily, so it keeps the
// compiler's choice.
#define TFSPH_DENSITY_OCCUPANCY(R) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 7 : 1)))
// The force passes sum FP64 terms (120 VGPRs, 4 waves per SIMD): the compiler's
// choice.  On the 3D box the isothermal pass takes 0.276 ms; held to 5 waves, or
// walking 1 or 3 neighbours per step, it is slower.
#ifndef TFSPH_FORCE_WAVES
#define TFSPH_FORCE_WAVES 1
#endif
#define TFSPH_FORCE_OCCUPANCY(R, KIND) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? TFSPH_FORCE_WAVES : 1)))
#define TFSPH_STAGE_OCCUPANCY(R, KIND) TFSPH_FORCE_OCCUPANCY(R, KIND)
#endif
// Arithmetic of the pressure-force pair sums of an FP32 state.  The pressure
// force of a smooth flow is a small difference of large pair terms (in the
// 2D wave of amplitude 1e-2 about 1e-3 of a term), so the rounding of each
// FP32 term, not of the state, decides the long-run error.  Separations are
// always formed in FP64 from the FP32 offsets; 2 (the default): FP64 terms
// and sums; 4: terms rounded once to FP32, FP64 sums.
// Over 1000 steps of that wave (64^2 + 64^2, FP32 state, against the FP64
// oracle) the dust velocity's relative L2 is 2.36e-3 with FP32 separations,
// terms and sums, 2.04e-3 with FP32 terms summed in FP64, 0.89e-3 with the
// default and 1.40e-3 with 4.
#ifndef TFSPH_FORCE_ARITH
#define TFSPH_FORCE_ARITH 2
#endif

template <typename R>
struct ForceArith {
    using T = R;     // pair terms
    using A = R;     // sums
};
template <>
struct ForceArith<float> {
    using T = typename std::conditional<(TFSPH_FORCE_ARITH == 2), double, float>::type;
    using A = double;
};
// Candidates recorded as neighbours in the masks: q < kMaskQ = 2 (1 + 1e-5).
// The force pass forms q again from FP64 separations, which can differ from
// the FP32 q by about 1e-6 relative; the margin keeps every pair with a
// non-zero force term in the masks, and the pairs it adds have q >= 2, whose
// terms are exactly zero.  So walking the masks and scanning the window give
// the same sums bit for bit.
constexpr float kMaskQ = 2.0f * (1.0f + 1e-5f);
constexpr int kChunk = TFSPH_CHUNK;
constexpr int kScanChunk = TFSPH_SCAN_CHUNK;
constexpr int kWalk = TFSPH_WALK;
// records past the end of a sorted pos / frc array that may be read
constexpr int kPad = kChunk > kScanChunk ? kChunk : kScanChunk;

// Grid + kernel geometry of one problem (uniform periodic cells, Section 2.3).
template <typename R>
struct Geom {
    int dim;
    int nc[3];
    int ncell;
    int win[3];          // neighbour window half width per axis
    R delta[3];          // cell width per axis
    R h, inv_h;
    R support2;          // (2h)^2
    R wnorm;             // sigma_d / h^d
    R gnorm;             // sigma_d / h^(d+1)
};

// Physics of the step: EOS, drag, time step, viscosity.
template <typename R>
struct Phys {
    int eos;             // 0 isothermal, 1 adiabatic
    int av;              // artificial viscosity on
    R cs;                // isothermal sound speed
    R cs2;
    R gm1;               // gamma - 1
    R ggm1;              // gamma (gamma - 1): c^2 = ggm1 * e
    R tau;               // time step
    R beta;              // tau / t_stop (t_stop held constant)
    int drag_law;        // 0: t_stop held constant; 1: K held constant; 2: t*_stop = T_E / rho*_g
    R tauKV;             // law 1: tau K V for a drag volume V
    R tau_VTE;           // law 2: tau / (V T_E)
    R g[3];
    R av_alpha, av_beta;
    R eta2;              // 0.01 h^2 in the viscosity denominator
    R h;
    R vlim2;             // Courant bound of eq. (4): (CFL h / tau)^2; 0 = no check
    // the drag coefficient K of eq. (7) at a point of the pairwise schemes, by drag law:
    // law 0: rho_d / t_stop; law 1: K; law 2: rho_g rho_d / T_E
    R inv_tstop, Kc, inv_te;
};

// Caller-owned arrays of one phase.
template <typename R>
struct Phase {
    int n;
    int *cell;
    R *off[3];
    R *vel[3];
    const R *mass;       // nullable: uniform mass m_uniform
    R m_uniform;
    R *rho;              // nullable for dust
    R *energy;           // nullable
    int *id;
};

// Packed 4-vectors: float4 / double4.
template <typename R> struct V4;
template <> struct V4<float> { using T = float4; };
template <> struct V4<double> { using T = double4; };
template <typename R> using R4 = typename V4<R>::T;

template <typename R>
__device__ __forceinline__ R4<R> mk4(R a, R b, R c, R d)
{
    R4<R> v;
    v.x = a;
    v.y = b;
    v.z = c;
    v.w = d;
    return v;
}

// Hardware square root / reciprocal square root / reciprocal in FP32 (about
// 1 ulp); exact IEEE operations in FP64.
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float frsq(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsq(double x) { return 1.0 / sqrt(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }

// Workspace arrays of one phase: the step's canonical (cell, id) ordered copy
// plus binning scratch.  Offsets and mass travel packed as pos = (ox, oy, oz, m)
// so one 16-byte load serves a neighbour candidate; the gas force pass reads
// frc = (ox, oy, oz, p / rho^2) written by the density pass.
template <typename R>
struct Sorted {
    int n;
    int has_mass;        // per-particle masses (copied back to the caller)
    int *cell;
    R4<R> *pos;          // (ox, oy, oz, m)
    R4<R> *frc;          // gas: (ox, oy, oz, p / rho^2)
    R *vel[3];
    R *energy;           // nullable
    int *id;
    R *rho;              // summation density
    R *vt[3];            // predictor velocity v~ (gas)
    int *count;          // [ncell] histogram
    int *start;          // [ncell + 1] exclusive offsets
    int *slot;           // [n] slot claimed inside the cell during counting
    int *tmp_idx;        // [n] unsorted-within-cell scatter of source indices
    int *tmp_id;         // [n] ids in the same layout
    int *src;            // nullable [n]: index in the unsorted arrays of sorted particle dst
    unsigned long long *nmask;   // nullable [rows][n]: neighbour bits per window row (gas)
};

struct Flags {
    unsigned int *word;                 // sticky TFSPH_FLAG_* bits
    unsigned long long *one_phase;      // [0]: count of one-phase cells; [1]: bits of the largest
                                        // squared signal speed max(|v|, c)^2 (a double) seen
};

constexpr unsigned int kFlagCfl = 16u;  // TFSPH_FLAG_CFL

// A cell index read from caller memory; anything out of range is treated as
// cell 0 (and reported by the kernels that read it) so no access leaves the
// cell arrays.
__device__ __forceinline__ int safe_cell(int c, int ncell)
{
    return (c >= 0 && c < ncell) ? c : 0;
}

// Cells up to this size are ranked by id (each particle counts the smaller ids
// of its cell, so a crowded cell costs the square of its population); above
// it a cell keeps the order of its slot claims and is flagged.
constexpr int kMaxRankCell = 1 << 16;

__device__ __forceinline__ int wrap_index(int c, int n)
{
    c %= n;
    return c < 0 ? c + n : c;
}

template <typename R>
__device__ __forceinline__ bool finite_r(R x)
{
    return x == x && x - x == R(0);
}

// Carry rule of the binning: bring off into [0, D) moving the cell index by
// whole cells (a point exactly on a face belongs to the upper cell).  Offsets
// more than a few cells away are first reduced with floor; non-finite or
// absurdly large offsets are reset to 0 in the same cell and reported, so the
// cell index always stays a valid array index.
template <typename R>
__device__ __forceinline__ bool carry(R &o, int &c, R D, int n)
{
#pragma clang fp contract(off)
    bool ok = true;
    if (!(o >= R(-4) * D && o < R(5) * D)) {
        const R lim = D * R(n) * R(4);
        if (!(o > -lim && o < lim)) {
            o = R(0);
            ok = false;
        } else {
            const R k = floor(o / D);
            o = o - k * D;
            c += int(k);
            c = wrap_index(c, n);
        }
    }
    for (int it = 0; it < 8 && o < R(0); ++it) { o += D; c -= 1; }
    for (int it = 0; it < 8 && o >= D; ++it) { o -= D; c += 1; }
    if (o < R(0) || o >= D) { o = R(0); ok = false; }
    c = wrap_index(c, n);
    return ok;
}

template <typename R>
__device__ __forceinline__ void split_cell(const Geom<R> &G, int lin, int &cx, int &cy, int &cz)
{
    cx = lin % G.nc[0];
    const int r = lin / G.nc[0];
    cy = r % G.nc[1];
    cz = r / G.nc[1];
}

template <typename R>
__device__ __forceinline__ int join_cell(const Geom<R> &G, int cx, int cy, int cz)
{
    return cx + G.nc[0] * (cy + G.nc[1] * cz);
}

template <typename R>
__device__ __forceinline__ R mass_of(const R *m, R mu, int i)
{
    return m ? m[i] : mu;
}

}  // namespace tfsph
