/*
 * tfsph.h -- C ABI of the MI355X (gfx950) two-fluid SPH library with
 * implicit drag-in-cell (IDIC) coupling.
 *
 * Method: Stoyanovskaya, Glushko, Snytnikov & Snytnikov, "Monodisperse
 * gas-solid mixtures with intense interphase interaction in Two-Fluid
 * Smoothed Particle Hydrodynamics" (arXiv:1908.01682).  Gas particles carry
 * the continuity/momentum equations (1) and dust particles (2), coupled by
 * the drag (3) in the K-form (7).  The drag is evaluated per volume ("cell"):
 * Section 2.3, eqs. (17)-(21).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Every pointer inside tfsph_state / tfsph_phase and every workspace
 *    pointer is DEVICE memory owned by the caller.  The library never
 *    allocates device memory on the step paths; it writes only into the
 *    arrays and the workspace it is given.
 *  - Real arrays are float (TFSPH_F32) or double (TFSPH_F64), as chosen by
 *    tfsph_params.precision; void* is used so one ABI serves both.
 *  - Positions are stored in cell-relative form: a linear cell index
 *    cell = cx + nx (cy + ny cz) and per-axis offsets 0 <= off < Delta_d
 *    with Delta_d = (box_hi[d] - box_lo[d]) / n_cells[d].  The absolute
 *    position is box_lo + (cx, cy, cz) Delta + off.  The box is periodic.
 *  - Calls are asynchronous on the given HIP stream (hipStream_t passed as
 *    void*, NULL = default stream).  Host-detectable argument errors are
 *    returned synchronously before anything is enqueued; numerical trouble
 *    is recorded in sticky device flags read with tfsph_get_flags().
 *  - Nothing throws across the ABI.  A failing call returns a negative
 *    tfsph_status and leaves a message for tfsph_last_error() (thread local).
 *  - Calls that share a context, a state or a workspace must not overlap in
 *    time on different streams.
 */
#ifndef TFSPH_H
#define TFSPH_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    TFSPH_OK = 0,
    TFSPH_E_INVALID_ARG = -1,   /* bad parameter or pointer; nothing enqueued */
    TFSPH_E_WORKSPACE = -2,     /* workspace missing, too small or misaligned */
    TFSPH_E_HIP = -3,           /* a HIP runtime call failed (message has the HIP error) */
    TFSPH_E_UNSUPPORTED = -4,   /* valid request outside what this build implements */
    TFSPH_E_STATE = -5          /* context/state mismatch (sizes differ from init) */
} tfsph_status;

/* sticky device flags (bit mask) */
enum {
    TFSPH_FLAG_NONFINITE = 1u,         /* a velocity, offset or density became NaN/Inf */
    TFSPH_FLAG_EMPTY_PHASE_CELL = 2u,  /* some cell held particles of one phase only */
    TFSPH_FLAG_BAD_CELL = 4u,          /* a state cell index was out of range (treated as cell 0) */
    TFSPH_FLAG_CELL_OVERFLOW = 8u,     /* a cell held more than 65536 particles of one phase: its
                                          in-cell order fell back to arrival order (not reproducible) */
    TFSPH_FLAG_CFL = 16u               /* with tfsph_params.cfl > 0: after some step the Courant
                                          bound of eq. (4), tau < CFL h / max(|v|, c), no longer
                                          held for the next step (see tfsph_signal_speed) */
};

enum { TFSPH_F32 = 0, TFSPH_F64 = 1 };
enum { TFSPH_ISOTHERMAL = 0, TFSPH_ADIABATIC = 1 };
enum { TFSPH_SCHEME_IDIC = 0, TFSPH_SCHEME_IMEX2 = 1, TFSPH_SCHEME_MK = 2, TFSPH_SCHEME_ISPH = 3 };

/* Run parameters; symbols follow the paper. */
typedef struct {
    int32_t dim;            /* 1, 2 or 3 */
    int32_t n_cells[3];     /* drag volumes per axis (Section 2.3); axes >= dim must be 1 */
    double box_lo[3];       /* periodic box [box_lo, box_hi) */
    double box_hi[3];
    double h;               /* smoothing length of W(h, r) (Section 2.1); kernel support 2h */
    int32_t eos;            /* TFSPH_ISOTHERMAL: p = c_s^2 rho; TFSPH_ADIABATIC: p = (gamma-1) rho e */
    double c_s;             /* isothermal sound speed */
    double gamma;           /* adiabatic index (adiabatic EOS only) */
    double t_stop;          /* velocity relaxation time of eq. (3); K = rho_d / t_stop (eq. 7) */
    double g[3];            /* gravity acceleration of eqs. (1)-(2) */
    double dt;              /* time step tau (eq. 4 bounds it; tau > t_stop is allowed) */
    double av_alpha;        /* artificial viscosity alpha, beta (0, 0 = off) */
    double av_beta;
    int32_t precision;      /* TFSPH_F32 or TFSPH_F64 for every real array */
    double K;               /* 0: t_stop is held constant.  > 0: the drag coefficient K of eq. (7)
                               is held constant and t_stop is unused: per drag volume of size V
                               (length in 1D, area in 2D) with masses M_g, M_d the volume averages
                               are rho*_g = M_g / V, rho*_d = M_d / V, so t*_stop = rho*_d / K
                               (Section 2.3) */
    double t_stop_epstein;  /* 0: unused.  > 0 (with K == 0): t*_stop = t_stop_epstein / rho*_g per
                               drag volume, the Epstein regime at fixed grain size and sound speed
                               (t_stop_epstein is the stopping time at unit gas density); t_stop
                               is unused */
    int32_t scheme;         /* time discretisation of tfsph_step:
                               TFSPH_SCHEME_IDIC: the paper's step, eqs. (19)-(21) with first-order
                               time differences (Section 2.3);
                               TFSPH_SCHEME_IMEX2: second order, the ARS(2,2,2) IMEX pair of Ascher,
                               Ruuth & Spiteri (1997) with the drag in cell as its implicit part and
                               the drift, pressure, viscosity, gravity and energy terms as its
                               explicit part; each implicit stage is the first-order drag solve over
                               gamma tau (gamma = 1 - 1/sqrt(2)) on that stage's volumes.  Per step:
                               three binnings, two density and force passes, two drag solves; rho
                               on exit is the density at the start of the step and the one-phase
                               count covers both solves.
                               The paper's two comparison schemes, with no drag volumes (the cells
                               only serve the neighbour search):
                               TFSPH_SCHEME_MK: the explicit pairwise drag of Monaghan & Kocharyan,
                               Section 2.1, eqs. (8)-(10): for gas a and dust j,
                               X = K_aj/(rho_a rho_j) ((v_a - u_j).r) r W(r)/(r^2 + eta^2),
                               eta^2 = 0.001 h^2, enters dv_a/dt as -sigma sum_j m_j X and du_j/dt
                               as +sigma sum_a m_a X with the velocities of level n, sigma = dim;
                               v += tau (A + g + drag), u += tau (g + drag); stable for tau below
                               about t_stop (eq. 5).
                               TFSPH_SCHEME_ISPH: the semi-implicit drag with SPH interpolation,
                               Section 2.2, eqs. (11)-(16): each particle interpolates the other
                               phase's velocity and density (dust points also the gas pressure)
                               and solves its own 2x2 system with alpha = tau K/rho_g,
                               beta = tau K/rho_d at the point; gas keeps v, dust keeps u.  A
                               particle with no particle of the other phase within 2h gets no drag
                               and is counted as a one-phase cell.
                               In all schemes K follows the drag law: K (K > 0), rho_d/t_stop, or
                               rho_g rho_d/t_stop_epstein; on exit both rho arrays (dust rho when
                               given) hold the summation densities of the last step.
                               The batched and adjoint entry points accept TFSPH_SCHEME_IDIC only
                               (TFSPH_E_UNSUPPORTED otherwise). */
    double cfl;             /* Courant number CFL of eq. (4) (the paper takes CFL < 1).  0: no check.
                               > 0: at the end of every step each particle's signal speed
                               s = max(|v|, c) is compared with CFL h / tau, where c is the gas sound
                               speed (c_s, or sqrt(gamma (gamma-1) e) per gas particle for the
                               adiabatic EOS), and TFSPH_FLAG_CFL is set where it is exceeded.  The
                               largest s is kept either way (tfsph_signal_speed). */
} tfsph_params;

/* One particle phase (gas: indices a, b; dust: j, k in the paper's notation).
 * Every array has n entries; off[d], vel[d] for d < dim. */
typedef struct {
    int64_t n;
    int32_t *cell;          /* linear cell index (in/out) */
    void *off[3];           /* offsets inside the cell, 0 <= off < Delta (in/out) */
    void *vel[3];           /* velocity: v for gas, u for dust (in/out) */
    void *mass;             /* per-particle mass, or NULL to use mass_uniform (in/out: reordered) */
    double mass_uniform;
    void *rho;              /* summation density at the start of the last step (out);
                               required for gas, may be NULL for dust */
    void *energy;           /* specific internal energy, gas with adiabatic EOS only (in/out) */
    int32_t *id;            /* particle ids, unique within the phase (in, travel with the particle) */
} tfsph_phase;

typedef struct {
    tfsph_phase gas;
    tfsph_phase dust;
} tfsph_state;

typedef struct tfsph_ctx tfsph_ctx;   /* opaque; host memory only */

/* Human-readable name of a status code (static string). */
const char *tfsph_status_string(tfsph_status s);

/* Detail of the last failure on the calling thread ("" if none). */
const char *tfsph_last_error(void);

/* Host-only check of a parameter set (no device call).  Fails with
 * TFSPH_E_INVALID_ARG when: dim not in 1..3; a cell count < 1 or, on an
 * axis >= dim, != 1; box_hi <= box_lo; h <= 0; an axis with fewer than
 * 2W+1 cells where W = ceil(2h / Delta) is the neighbour window; W > 128;
 * K or t_stop_epstein < 0 or non-finite, or both > 0; both 0 with t_stop <= 0
 * or non-finite; dt <= 0 or non-finite; isothermal with c_s <= 0; adiabatic
 * with gamma <= 1; negative viscosity coefficients; unknown eos/precision;
 * more than 2^31-1 cells. */
tfsph_status tfsph_validate(const tfsph_params *p);

/* Host-only: bytes of device workspace tfsph_init() needs for n_gas, n_dust
 * particles (each 0 .. 2^31-1).  The workspace must be 256-byte aligned. */
tfsph_status tfsph_workspace_size(const tfsph_params *p, int64_t n_gas, int64_t n_dust, size_t *bytes);

/* Create a context for one simulation and bring the state into canonical
 * form on the device: every offset is carried into [0, Delta) (the cell
 * index moves accordingly, periodic wrap), and both phases are reordered in
 * place into (cell, id) lexicographic order.  The workspace (device,
 * caller-owned, at least tfsph_workspace_size() bytes) is used by every later
 * call on this context and must stay allocated until tfsph_destroy().
 * Errors: TFSPH_E_INVALID_ARG (params, NULL arrays, n mismatch with mass/
 * energy requirements), TFSPH_E_WORKSPACE, TFSPH_E_HIP. */
tfsph_status tfsph_init(tfsph_ctx **out, const tfsph_params *p, tfsph_state *s, void *workspace,
                        size_t ws_bytes, void *hip_stream);

/* Advance the state n_steps IDIC time steps (Section 2.3), in place.  One
 * step n -> n+1:
 *   (a) bin both phases into the volumes at level n (counting sort, order
 *       (cell, id), deterministic);
 *   (b) gas summation density rho_a = sum_b m_b W(|r_ab|, h) and pressure;
 *   (c) explicit terms of eq. (19): v~_a = v_a + tau (-sum_b m_b (p_a/rho_a^2
 *       + p_b/rho_b^2 + Pi_ab) grad_a W_ab + g), e_a += tau de_a/dt for the
 *       adiabatic EOS; u~_j = u_j + tau g (eq. 20);
 *   (d) per cell: M_g, M_d and the momenta of v~, u~ (eqs. 17, 21), the
 *       implicit solve of eqs. (19)-(21) for the new cell means
 *       (eps = M_d/M_g, alpha = eps tau/t_stop, beta = tau/t_stop; with
 *       K > 0: alpha = tau K V/M_g, beta = tau K V/M_d for the volume V;
 *       with t_stop_epstein = T_E > 0: alpha = tau M_d/(V T_E),
 *       beta = tau M_g/(V T_E)),
 *       then v_a = (v~_a + alpha U*)/(1+alpha), u_j = (u~_j + beta V*)/(1+beta);
 *       cells with one phase only get no drag;
 *   (e) x += tau v_new, offsets carried back into [0, Delta).
 * On return the arrays hold level n+N, ordered by the cells of the last
 * step's start; rho holds the gas density used by that step.  Sums are
 * evaluated in a fixed order: results are bitwise reproducible.
 * Errors: TFSPH_E_INVALID_ARG (n_steps < 0), TFSPH_E_STATE (n differ from
 * init), TFSPH_E_HIP. */
tfsph_status tfsph_step(tfsph_ctx *ctx, tfsph_state *s, int32_t n_steps, void *hip_stream);

/* Summation density of one phase over itself at the current positions,
 * written to that phase's rho array (phase 0 = gas, 1 = dust; dust density
 * is a diagnostic, the gas density of a step is computed by tfsph_step).
 * Reorders the phase into canonical (cell, id) order first. */
tfsph_status tfsph_density(tfsph_ctx *ctx, tfsph_state *s, int32_t phase, void *hip_stream);

/* Read and clear the sticky flags and the count of one-phase cells seen
 * since the last call.  Synchronises the context's last stream. */
tfsph_status tfsph_get_flags(tfsph_ctx *ctx, uint32_t *flags, int64_t *one_phase_cells);

/* Largest signal speed max over particles of max(|v|, c) (eq. 4; c as for
 * tfsph_params.cfl; with the isothermal EOS c_s is included) seen since the
 * last call: the state tfsph_init() started from and the end of every step
 * since (tfsph_step, tfsph_step_graph).  Reads and clears it; synchronises the
 * context's last stream.  The maximum does not depend on the order in which
 * particles are visited. */
tfsph_status tfsph_signal_speed(tfsph_ctx *ctx, double *signal_speed);

/* Host only: the time step of the Courant bound, eq. (4):
 *   *dt = p->cfl * p->h / max(signal_speed, c)
 * with c = p->c_s for the isothermal EOS and no floor for the adiabatic one
 * (the signal speed from tfsph_signal_speed() already holds each gas
 * particle's sound speed).  Only cfl, h, eos and c_s of p are read.
 * TFSPH_E_INVALID_ARG when cfl or h are not positive and finite, the signal
 * speed is negative or non-finite, or the bound is infinite (zero speed). */
tfsph_status tfsph_cfl_dt(const tfsph_params *p, double signal_speed, double *dt);

/* Replay form of tfsph_step: the launches of `chunk` consecutive steps are
 * captured once into a hipGraph (on a private stream of default priority,
 * no memset nodes) and the graph is replayed on hip_stream; n_steps need not
 * be a multiple of chunk (the remainder runs eagerly).  Results are bitwise
 * those of tfsph_step.  The graph is tied to the state's array addresses:
 * a state with other addresses is captured anew.  chunk in 1..256. */
tfsph_status tfsph_step_graph(tfsph_ctx *ctx, tfsph_state *s, int32_t n_steps, int32_t chunk, void *hip_stream);

/* ---------------------------------------------------------------------------
 * Batched form: many independent problems (instances) with their own
 * parameters, advanced together, either by one persistent kernel launch per
 * call or by six launches per step over every instance (the form is chosen
 * with tfsph_batch_tuning, below).  The packed state holds every instance's particles back to back: instance i
 * owns gas particles [gas_offset[i], gas_offset[i+1]) and dust particles
 * [dust_offset[i], dust_offset[i+1]) of the packed arrays; its cell indices
 * are local to its own grid.  Each instance's offsets must already be in
 * [0, Delta_i) (tfsph_positions_to_cells with that instance's params).
 * In the persistent form one workgroup advances one instance for all n_steps
 * (block barriers only, no inter-workgroup waiting); instances start largest
 * first.  In either form every instance evolves bitwise as it would alone
 * through tfsph_step.
 * ------------------------------------------------------------------------- */
typedef struct tfsph_batch tfsph_batch;

typedef struct {
    int32_t n_inst;
    const tfsph_params *params;     /* host [n_inst]; all with the same dim (1 or 2) and precision */
    const int64_t *gas_offset;      /* host [n_inst + 1], non-decreasing, [0] = 0, [n_inst] = packed gas.n */
    const int64_t *dust_offset;     /* host [n_inst + 1] */
    const double *mass_gas;         /* host [n_inst]: uniform gas mass of each instance (packed gas.mass NULL) */
    const double *mass_dust;        /* host [n_inst]: uniform dust mass (packed dust.mass NULL) */
} tfsph_batch_desc;

/* Forms of the batched step (results are bitwise the same):
 *  - TFSPH_BATCH_PERSISTENT: one persistent launch per call, one workgroup per
 *    instance for all its steps (no workgroup waits on another); the launch
 *    lasts as long as the largest instance takes on one compute unit.
 *  - TFSPH_BATCH_FLAT: each phase of a step (scan, scatter, rank + gather,
 *    density, force + predictor, cell sums + solve + update) is one launch over
 *    every instance, with blocks dealt out per instance (a block never
 *    straddles two); six launches per step, best replayed as a hipGraph. */
enum { TFSPH_BATCH_PERSISTENT = 0, TFSPH_BATCH_FLAT = 1 };

typedef struct {
    int32_t block;                  /* persistent form: threads per workgroup, multiple of 64 in
                                       64..1024 (0 = 512); the flattened form uses 256 */
    int32_t form;                   /* TFSPH_BATCH_PERSISTENT (0) or TFSPH_BATCH_FLAT */
    int32_t cells_per_block;        /* flattened form: cells per workgroup of its update launch,
                                       1..256 (0 = the single-problem default for the dimension) */
} tfsph_batch_tuning;

/* Host-only: workspace bytes for a batch (256-byte aligned buffer). */
tfsph_status tfsph_batch_workspace_size(const tfsph_batch_desc *desc, size_t *bytes);

/* Validate every instance (tfsph_validate), bind the packed state and the
 * workspace, upload the instance table and the launch order.  The host
 * arrays of desc may be freed after return.  tuning may be NULL. */
tfsph_status tfsph_batch_init(tfsph_batch **out, const tfsph_batch_desc *desc, tfsph_state *packed,
                              const tfsph_batch_tuning *tuning, void *workspace, size_t ws_bytes, void *hip_stream);

/* Change the launch shape (results do not depend on it).  A new cells_per_block
 * rewrites the flattened form's block table on the stream of the batch's last
 * call (or of init), waits for that stream, and drops the flattened form's
 * captured graphs. */
tfsph_status tfsph_batch_set_tuning(tfsph_batch *b, const tfsph_batch_tuning *tuning);

/* Advance every instance n_steps IDIC steps: one kernel launch (persistent
 * form) or six launches per step (flattened form).  The packed state must be
 * the one bound at init (TFSPH_E_STATE otherwise). */
tfsph_status tfsph_step_batched(tfsph_batch *b, tfsph_state *packed, int32_t n_steps, void *hip_stream);

/* Same, through a hipGraph captured once per (n_steps, form, block) and replayed. */
tfsph_status tfsph_step_batched_graph(tfsph_batch *b, tfsph_state *packed, int32_t n_steps, void *hip_stream);

/* Flags and one-phase-cell count over all instances since the last call (syncs). */
tfsph_status tfsph_batch_get_flags(tfsph_batch *b, uint32_t *flags, int64_t *one_phase_cells);

tfsph_status tfsph_batch_destroy(tfsph_batch *b);

/* ---------------------------------------------------------------------------
 * Hand-written adjoint (reverse mode) of n_steps IDIC steps for the
 * dust-density misfit
 *     L = (1/N_d) sum_j (rho_d,j(T) - target[id_j])^2,
 *     rho_d,j = sum_k m_k W(|x_j - x_k|, h)   (dust only, at the final state),
 * with respect to log t_stop and the initial velocities v0 (gas) and u0
 * (dust).  With the drag coefficient K held constant (p->K > 0) the scalar is
 * the derivative with respect to log(1/K) (= -dL/dlog K), with the Epstein
 * law (p->t_stop_epstein > 0) with respect to log t_stop_epstein: alpha and
 * beta scale like 1/t_stop, K and 1/t_stop_epstein in the three forms.  Cells and
 * neighbour sets are held at their forward values (they
 * are piecewise constant in the inputs).  Memory is bounded by checkpointing:
 * the state is saved every ckpt_every steps in a forward sweep; then for each
 * segment, last first, the segment is replayed from its checkpoint with every
 * step's sorted state taped, and reversed step by step.  All sums are in
 * gather form (no atomics) and reduced in a fixed order: bitwise
 * reproducible.  Isothermal EOS without artificial viscosity only
 * (TFSPH_E_UNSUPPORTED otherwise).
 *
 *   initial      device state at t = 0; read only.  Offsets must lie in
 *                [0, Delta); ids must be a permutation of 0..n-1 per phase.
 *   target       device [n_dust] real, indexed by dust id
 *   dL_dv0_gas   device [dim] arrays of [n_gas] real, indexed by gas id (out)
 *   dL_du0_dust  device [dim] arrays of [n_dust] real, indexed by dust id (out)
 *   dL_dlog_tstop, loss   device double (out)
 * ------------------------------------------------------------------------- */
tfsph_status tfsph_adjoint_workspace_size(const tfsph_params *p, int64_t n_gas, int64_t n_dust, int32_t n_steps,
                                          int32_t ckpt_every, size_t *bytes);

tfsph_status tfsph_step_adjoint(const tfsph_params *p, const tfsph_state *initial, int32_t n_steps,
                                int32_t ckpt_every, const void *target, void *dL_dv0_gas[3], void *dL_du0_dust[3],
                                double *dL_dlog_tstop, double *loss, void *workspace, size_t ws_bytes,
                                void *hip_stream);

/* Pair-loop implementation of a context's steps.
 *  - TFSPH_VARIANT_AUTO (the default): the density pass scans the neighbour
 *    window in global memory and records, per gas particle and window row, a
 *    64-bit mask of the candidates inside the support (rows of at most 64
 *    candidates, windows of at most 5 cells along x); the force pass visits
 *    only those and scans the rest.  The masks take 8 bytes per gas particle
 *    and row of the window in the workspace (tfsph_workspace_size).
 *  - TFSPH_VARIANT_GLOBAL: both passes scan the whole window in global memory.
 *  - TFSPH_VARIANT_LDS_BRICKS: not built (TFSPH_E_UNSUPPORTED): blocks of
 *    cells staged in LDS were slower than the global loops.
 * Both variants visit neighbours in the same order with the same arithmetic,
 * and terms outside the support are exactly zero, so results are bitwise
 * equal.  Selecting a variant drops the context's cached step graph.  Returns
 * TFSPH_E_INVALID_ARG for an unknown variant or a null context. */
enum { TFSPH_VARIANT_AUTO = 0, TFSPH_VARIANT_GLOBAL = 1, TFSPH_VARIANT_LDS_BRICKS = 2 };
tfsph_status tfsph_set_kernel_variant(tfsph_ctx *ctx, int32_t variant);

/* Cells owned by one 256-thread block of the update kernel (cell sums,
 * implicit solve, particle update), in [1, 256]; the default depends on the
 * dimension.  Results do not depend on it (each cell is summed serially by
 * one thread).  Drops the context's cached step graph.  Returns
 * TFSPH_E_INVALID_ARG outside that range or for a null context. */
tfsph_status tfsph_set_cells_per_block(tfsph_ctx *ctx, int32_t cells);

/* Kernel timing for measurement.  tfsph_profile(ctx, 1) starts recording a
 * HIP event pair around every launch of the timed kernels on the stream the
 * launch uses (it creates the events on the host; nothing is allocated on the
 * device); tfsph_profile(ctx, 2) does the same for one kernel kind per step,
 * the kinds taken in turn (step i times kind i mod 4, counted from the call),
 * so that the events perturb the steps they bracket less;
 * tfsph_profile_sampled(ctx, every) does the same in every `every`-th step
 * only (step i is timed when i mod every = 0, kind (i / every) mod 4; every
 * >= 1, else TFSPH_E_INVALID_ARG);
 * tfsph_profile(ctx, 0) stops and keeps what was recorded.  Steps replayed
 * from a graph are not timed.  Another mode returns TFSPH_E_INVALID_ARG.
 * tfsph_profile_read() synchronises, then returns the summed duration in ms
 * and the number of launches of one kernel:
 *   TFSPH_KERNEL_UPDATE  (cell sums + implicit solve + particle update; with
 *                         TFSPH_VARIANT_LDS_BRICKS also the gas force),
 *   TFSPH_KERNEL_DENSITY (gas summation density and neighbour masks),
 *   TFSPH_KERNEL_BIN     (count + scan + scatter + rank/gather, as one span),
 *   TFSPH_KERNEL_FORCE   (gas pressure force + predictor).
 * Returns TFSPH_E_INVALID_ARG for another kernel id. */
enum { TFSPH_KERNEL_UPDATE = 0, TFSPH_KERNEL_DENSITY = 1, TFSPH_KERNEL_BIN = 2, TFSPH_KERNEL_FORCE = 3 };
tfsph_status tfsph_profile(tfsph_ctx *ctx, int32_t enable);
tfsph_status tfsph_profile_sampled(tfsph_ctx *ctx, int32_t every);
tfsph_status tfsph_profile_read(tfsph_ctx *ctx, int32_t kernel, double *total_ms, int64_t *launches);

/* Convert n absolute FP64 positions x (device, layout [dim][n], inside or
 * outside the box) to the cell-relative form: cell = floor((x - box_lo)/Delta)
 * evaluated in FP64 (periodic wrap), off = (x - box_lo) - cell Delta rounded
 * to the state precision and carried into [0, Delta).  cell, off[d] are
 * device arrays of n entries.  Host-checked arguments; async on the stream. */
tfsph_status tfsph_positions_to_cells(const tfsph_params *p, int64_t n, const double *x, int32_t *cell, void *off[3],
                                      void *hip_stream);

/* Inverse conversion: x[d*n + i] = box_lo[d] + c_d Delta_d + off[d][i] in FP64
 * (device arrays). */
tfsph_status tfsph_cells_to_positions(const tfsph_params *p, int64_t n, const int32_t *cell, void *const off[3],
                                      double *x, void *hip_stream);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): tfsph_init
 * followed by tfsph_step(n_steps) in one call, with no context and no
 * caller workspace.  The workspace is the library's static device array of
 * 64 MiB per GPU (held from the library's first use on that GPU until the
 * process ends); the call makes no hipMalloc/hipFree or other allocating
 * call, and enqueues its kernels asynchronously on hip_stream.
 *   p, s           as for tfsph_init / tfsph_step: on return the state holds
 *                  level n_steps in canonical order (bitwise what tfsph_init +
 *                  tfsph_step give)
 *   flags_out      device uint32 (nullable): the sticky TFSPH_FLAG_* bits of
 *                  this call (the canonical ordering and every step)
 *   one_phase_out  device int64 (nullable): one-phase cells counted by this
 *                  call
 * Errors (host-side, nothing enqueued): those of tfsph_init, n_steps < 0, and
 * TFSPH_E_WORKSPACE when the problem needs more workspace than the static
 * array holds (tfsph_workspace_size() for the same sizes is an upper bound of
 * the need).  Every call on one GPU shares that GPU's array and starts by
 * clearing what must start at zero; calls that overlap in time on one GPU
 * (other streams, other threads) race and must not be issued. */
tfsph_status tfsph_step_noalloc(const tfsph_params *p, tfsph_state *s, int32_t n_steps, uint32_t *flags_out,
                                int64_t *one_phase_out, void *hip_stream);

/* Release the context (host memory only; the workspace stays the caller's). *//* Release the context (host memory only; the workspace stays the caller's). */
tfsph_status tfsph_destroy(tfsph_ctx *ctx);

#ifdef __cplusplus
}
#endif

#endif /* TFSPH_H */
