/*
 * FP64 CPU oracle for one IDIC ("implicit drag in cell") time step of
 * two-fluid SPH (Stoyanovskaya, Glushko, Snytnikov & Snytnikov,
 * arXiv:1908.01682).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the plain, slow reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header
 * or constant with the HIP library.
 *
 * State of one phase (gas: indices a,b; dust: indices j,k -- Section 2):
 *   cell[i]            linear drag-cell index  cx + nx (cy + ny cz)
 *   off[d*n + i]       offset of the particle inside its cell along axis d,
 *                      0 <= off < Delta_d  (absolute x = lo + cx Delta + off)
 *   vel[d*n + i]       velocity
 *   mass[i], id[i], rho[i] (output), energy[i] (gas, adiabatic EOS only)
 *
 * Every sum over particles is evaluated serially per particle in a fixed
 * canonical order: neighbour cells in lexicographic window order (z, then y,
 * then x offsets), and inside a cell by (cell, id) order.  OpenMP only splits
 * the outer loop, so results do not depend on the thread count.
 *
 * Readings of points the paper leaves open (all restated in the design notes):
 *  - smoothing kernel: M4 cubic spline with support 2h (the paper's W(h, r),
 *    Section 2.1, type not named);
 *  - gas density: summation density over gas particles, self included;
 *  - the explicit SPH terms of eq. (19) are applied before the cell solve
 *    (unsplit first-order step, Section 2.3);
 *  - cell means of eq. (21) are mass weighted, eps* = M_d / M_g (eq. 17 with
 *    equal masses);
 *  - a cell holding only one phase gets no drag this step (eq. 17 needs
 *    N > 0 and L > 0);
 *  - positions move with the new velocity, x^{n+1} = x^n + tau v^{n+1}.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    int32_t dim;
    int32_t nc[3];
    double lo[3];
    double hi[3];
    double h;
    int32_t eos;        /* 0: isothermal p = c_s^2 rho; 1: adiabatic p = (gamma-1) rho e */
    double cs;
    double gamma;
    double tstop;
    double g[3];
    double dt;
    double av_alpha;
    double av_beta;
    double K;           /* > 0: drag coefficient K of eq. (7) held constant, t*_stop = rho*_d / K per volume */
    double tse;         /* > 0: Epstein-like law t*_stop = tse / rho*_g per volume (tse: t_stop at unit
                           gas density) */
} orc_params;

typedef struct {
    int64_t n;
    int32_t *cell;
    double *off;        /* [dim][n] */
    double *vel;        /* [dim][n] */
    double *mass;       /* [n] */
    double *rho;        /* [n], written by the density sums (may be NULL for dust) */
    double *energy;     /* [n] or NULL */
    int32_t *id;        /* [n] */
} orc_phase;

#define ORC_PI 3.14159265358979323846

/* ------------------------------------------------------------------------ */
/* Smoothing kernel W(h, r): M4 cubic spline, support 2h.                    */
/* W = sigma_d h^-d f(q), q = r/h,                                           */
/*   f = 1 - 3/2 q^2 + 3/4 q^3 (q < 1),  1/4 (2 - q)^3 (1 <= q < 2),  0.      */
/* sigma_1 = 2/3, sigma_2 = 10/(7 pi), sigma_3 = 1/pi.                       */
/* ------------------------------------------------------------------------ */
static double orc_sigma(int dim)
{
    if (dim == 1) return 2.0 / 3.0;
    if (dim == 2) return 10.0 / (7.0 * ORC_PI);
    return 1.0 / ORC_PI;
}

double orc_kernel_w(int dim, double h, double r)
{
    double q = r / h;
    double f;
    if (q < 1.0) f = 1.0 - 1.5 * q * q + 0.75 * q * q * q;
    else if (q < 2.0) { double t = 2.0 - q; f = 0.25 * t * t * t; }
    else f = 0.0;
    return orc_sigma(dim) * f / pow(h, dim);
}

/* dW/dr */
double orc_kernel_dw(int dim, double h, double r)
{
    double q = r / h;
    double fp;
    if (q < 1.0) fp = -3.0 * q + 2.25 * q * q;
    else if (q < 2.0) { double t = 2.0 - q; fp = -0.75 * t * t; }
    else fp = 0.0;
    return orc_sigma(dim) * fp / pow(h, dim + 1);
}

/* ------------------------------------------------------------------------ */
/* Geometry helpers                                                          */
/* ------------------------------------------------------------------------ */
static double orc_delta(const orc_params *p, int d) { return (p->hi[d] - p->lo[d]) / p->nc[d]; }

static int64_t orc_ncells(const orc_params *p)
{
    int64_t n = 1;
    for (int d = 0; d < p->dim; ++d) n *= p->nc[d];
    return n;
}

static void orc_split(const orc_params *p, int32_t lin, int c[3])
{
    c[0] = c[1] = c[2] = 0;
    c[0] = lin % p->nc[0];
    if (p->dim > 1) c[1] = (lin / p->nc[0]) % p->nc[1];
    if (p->dim > 2) c[2] = lin / (p->nc[0] * p->nc[1]);
}

static int32_t orc_join(const orc_params *p, const int c[3])
{
    int32_t lin = c[0];
    if (p->dim > 1) lin += p->nc[0] * c[1];
    if (p->dim > 2) lin += p->nc[0] * p->nc[1] * c[2];
    return lin;
}

static int orc_wrapi(int c, int n) { c %= n; return c < 0 ? c + n : c; }

/* neighbour-window half width in cells along axis d: every particle within 2h
 * of a particle lies in a cell at most W cells away. */
static int orc_window(const orc_params *p, int d)
{
    if (d >= p->dim) return 0;
    return (int)ceil(2.0 * p->h / orc_delta(p, d) - 1e-12);
}

/* ------------------------------------------------------------------------ */
/* Binning (Section 2.3: "at each time instant" the region is split into    */
/* disjoint volumes).  Volumes = uniform periodic Cartesian cells.  A       */
/* position exactly on a face belongs to the upper cell.  The carry rule     */
/* below is floor((x - lo) / Delta) written for the (cell, offset) form.     */
/* ------------------------------------------------------------------------ */
void orc_canonicalize(const orc_params *p, orc_phase *ph)
{
    const int64_t n = ph->n;
    for (int64_t i = 0; i < n; ++i) {
        int c[3];
        orc_split(p, ph->cell[i], c);
        for (int d = 0; d < p->dim; ++d) {
            double D = orc_delta(p, d);
            double o = ph->off[d * n + i];
            while (o < 0.0) { o += D; c[d] -= 1; }
            while (o >= D) { o -= D; c[d] += 1; }
            c[d] = orc_wrapi(c[d], p->nc[d]);
            ph->off[d * n + i] = o;
        }
        ph->cell[i] = orc_join(p, c);
    }
}

/* (cell, id) lexicographic order */
static const orc_phase *orc_sort_ph;
static int orc_cmp(const void *A, const void *B)
{
    int64_t a = *(const int64_t *)A, b = *(const int64_t *)B;
    int32_t ca = orc_sort_ph->cell[a], cb = orc_sort_ph->cell[b];
    if (ca != cb) return ca < cb ? -1 : 1;
    int32_t ia = orc_sort_ph->id[a], ib = orc_sort_ph->id[b];
    return (ia > ib) - (ia < ib);
}

static void orc_permute_d(double *x, const int64_t *perm, int64_t n, double *tmp)
{
    for (int64_t i = 0; i < n; ++i) tmp[i] = x[perm[i]];
    memcpy(x, tmp, sizeof(double) * n);
}

static void orc_permute_i(int32_t *x, const int64_t *perm, int64_t n, int32_t *tmp)
{
    for (int64_t i = 0; i < n; ++i) tmp[i] = x[perm[i]];
    memcpy(x, tmp, sizeof(int32_t) * n);
}

/* Reorder all arrays of a phase into (cell, id) order; with perm_out, the
 * particle now at k was at perm_out[k] before.  Not thread safe (qsort
 * comparator uses a file-scope pointer); called from serial code. */
static void orc_sort_perm(const orc_params *p, orc_phase *ph, int64_t *perm_out)
{
    const int64_t n = ph->n;
    if (n == 0) return;
    int64_t *perm = (int64_t *)malloc(sizeof(int64_t) * n);
    double *tmp = (double *)malloc(sizeof(double) * n);
    int32_t *tmpi = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int64_t i = 0; i < n; ++i) perm[i] = i;
    orc_sort_ph = ph;
    qsort(perm, (size_t)n, sizeof(int64_t), orc_cmp);
    orc_sort_ph = NULL;
    for (int d = 0; d < p->dim; ++d) {
        orc_permute_d(ph->off + d * n, perm, n, tmp);
        orc_permute_d(ph->vel + d * n, perm, n, tmp);
    }
    orc_permute_d(ph->mass, perm, n, tmp);
    if (ph->rho) orc_permute_d(ph->rho, perm, n, tmp);
    if (ph->energy) orc_permute_d(ph->energy, perm, n, tmp);
    orc_permute_i(ph->cell, perm, n, tmpi);
    orc_permute_i(ph->id, perm, n, tmpi);
    if (perm_out) memcpy(perm_out, perm, sizeof(int64_t) * n);
    free(perm); free(tmp); free(tmpi);
}

void orc_sort(const orc_params *p, orc_phase *ph) { orc_sort_perm(p, ph, NULL); }

/* start[c] = first sorted index of cell c, start[ncells] = n */
void orc_cell_start(const orc_params *p, const orc_phase *ph, int64_t *start)
{
    int64_t nc = orc_ncells(p);
    for (int64_t c = 0; c <= nc; ++c) start[c] = 0;
    for (int64_t i = 0; i < ph->n; ++i) start[ph->cell[i] + 1] += 1;
    for (int64_t c = 0; c < nc; ++c) start[c + 1] += start[c];
}

/* ------------------------------------------------------------------------ */
/* Neighbour iteration.  For particle a in cell ca, visit every cell in the  */
/* window and every particle b in it; r_ab = x_a - x_b with the periodic     */
/* image of b that lies in the window.                                       */
/* ------------------------------------------------------------------------ */
typedef void (*orc_pair_fn)(void *ctx, int64_t a, int64_t b, const double r[3]);

static void orc_for_neighbours(const orc_params *p, const orc_phase *A, int64_t a,
                               const orc_phase *B, const int64_t *startB,
                               orc_pair_fn fn, void *ctx)
{
    int ca[3];
    orc_split(p, A->cell[a], ca);
    int W[3] = {orc_window(p, 0), orc_window(p, 1), orc_window(p, 2)};
    double D[3] = {orc_delta(p, 0), p->dim > 1 ? orc_delta(p, 1) : 0.0, p->dim > 2 ? orc_delta(p, 2) : 0.0};
    const int64_t na = A->n, nb = B->n;
    for (int dz = -W[2]; dz <= W[2]; ++dz)
        for (int dy = -W[1]; dy <= W[1]; ++dy)
            for (int dx = -W[0]; dx <= W[0]; ++dx) {
                int cb[3] = {orc_wrapi(ca[0] + dx, p->nc[0]), orc_wrapi(ca[1] + dy, p->nc[1]),
                             orc_wrapi(ca[2] + dz, p->nc[2])};
                int32_t lin = orc_join(p, cb);
                int dd[3] = {dx, dy, dz};
                for (int64_t b = startB[lin]; b < startB[lin + 1]; ++b) {
                    double r[3] = {0.0, 0.0, 0.0};
                    for (int d = 0; d < p->dim; ++d)
                        r[d] = A->off[d * na + a] - (B->off[d * nb + b] + dd[d] * D[d]);
                    fn(ctx, a, b, r);
                }
            }
}

/* ------------------------------------------------------------------------ */
/* SPH summation density  rho_a = sum_b m_b W(|r_ab|, h)   (self included).  */
/* The paper uses rho^n_{a,g} in eqs. (8), (12), (19) without writing it.   */
/* ------------------------------------------------------------------------ */
typedef struct { const orc_params *p; const orc_phase *B; double acc; } orc_dens_ctx;

static void orc_dens_pair(void *vctx, int64_t a, int64_t b, const double r[3])
{
    (void)a;
    orc_dens_ctx *c = (orc_dens_ctx *)vctx;
    double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (rr < 2.0 * c->p->h) c->acc += c->B->mass[b] * orc_kernel_w(c->p->dim, c->p->h, rr);
}

/* ph must be in (cell, id) order with matching start[] */
void orc_density(const orc_params *p, const orc_phase *ph, const int64_t *start, double *rho_out)
{
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < ph->n; ++a) {
        orc_dens_ctx c = {p, ph, 0.0};
        orc_for_neighbours(p, ph, a, ph, start, orc_dens_pair, &c);
        rho_out[a] = c.acc;
    }
}

/* ------------------------------------------------------------------------ */
/* Equation of state.  Isothermal gas (Section 3: "isothermal gas-dust       */
/* mixture") p = c_s^2 rho; the shock tube uses an ideal gas p=(g-1) rho e.  */
/* ------------------------------------------------------------------------ */
static double orc_pressure(const orc_params *p, double rho, double e)
{
    return p->eos == 0 ? p->cs * p->cs * rho : (p->gamma - 1.0) * rho * e;
}

static double orc_sound(const orc_params *p, double rho, double e)
{
    if (p->eos == 0) return p->cs;
    (void)rho;
    return sqrt(p->gamma * (p->gamma - 1.0) * e);
}

/* ------------------------------------------------------------------------ */
/* Explicit gas terms of eq. (19):                                           */
/*   A_a = - sum_b m_b (p_a/rho_a^2 + p_b/rho_b^2 + Pi_ab) grad_a W_ab + g    */
/* and, for the adiabatic EOS, the SPH internal-energy equation              */
/*   de_a/dt = sum_b m_b (p_a/rho_a^2 + Pi_ab/2) v_ab . grad_a W_ab.          */
/* Pi_ab is the Monaghan-Gingold artificial viscosity (zero when alpha =     */
/* beta = 0, which is every isothermal case).                                */
/* ------------------------------------------------------------------------ */
typedef struct {
    const orc_params *p; const orc_phase *G; const double *pres; const double *snd;
    double acc[3]; double dedt;
} orc_force_ctx;

static void orc_force_pair(void *vctx, int64_t a, int64_t b, const double r[3])
{
    orc_force_ctx *c = (orc_force_ctx *)vctx;
    const orc_params *p = c->p;
    const orc_phase *G = c->G;
    if (a == b) return;
    double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    double rr = sqrt(rr2);
    if (!(rr < 2.0 * p->h) || rr == 0.0) return;
    const int64_t n = G->n;
    double dw = orc_kernel_dw(p->dim, p->h, rr);
    double grad[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < p->dim; ++d) grad[d] = dw * r[d] / rr;
    double rhoa = G->rho[a], rhob = G->rho[b];
    double Pa = c->pres[a] / (rhoa * rhoa), Pb = c->pres[b] / (rhob * rhob);
    double vr = 0.0, vg = 0.0;
    for (int d = 0; d < p->dim; ++d) {
        double vab = G->vel[d * n + a] - G->vel[d * n + b];
        vr += vab * r[d];
        vg += vab * grad[d];
    }
    double Pi = 0.0;
    if ((p->av_alpha != 0.0 || p->av_beta != 0.0) && vr < 0.0) {
        double mu = p->h * vr / (rr2 + 0.01 * p->h * p->h);
        double cbar = 0.5 * (c->snd[a] + c->snd[b]);
        double rbar = 0.5 * (rhoa + rhob);
        Pi = (-p->av_alpha * cbar * mu + p->av_beta * mu * mu) / rbar;
    }
    double mb = G->mass[b];
    for (int d = 0; d < p->dim; ++d) c->acc[d] -= mb * (Pa + Pb + Pi) * grad[d];
    c->dedt += mb * (Pa + 0.5 * Pi) * vg;
}

void orc_gas_forces(const orc_params *p, const orc_phase *G, const int64_t *start,
                    double *acc_out /* [dim][n] */, double *dedt_out /* [n] or NULL */)
{
    const int64_t n = G->n;
    double *pres = (double *)malloc(sizeof(double) * (n ? n : 1));
    double *snd = (double *)malloc(sizeof(double) * (n ? n : 1));
    for (int64_t a = 0; a < n; ++a) {
        double e = G->energy ? G->energy[a] : 0.0;
        pres[a] = orc_pressure(p, G->rho[a], e);
        snd[a] = orc_sound(p, G->rho[a], e);
    }
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        orc_force_ctx c = {p, G, pres, snd, {0.0, 0.0, 0.0}, 0.0};
        orc_for_neighbours(p, G, a, G, start, orc_force_pair, &c);
        for (int d = 0; d < p->dim; ++d) acc_out[d * n + a] = c.acc[d] + p->g[d];
        if (dedt_out) dedt_out[a] = c.dedt;
    }
    free(pres); free(snd);
}

/* ------------------------------------------------------------------------ */
/* One IDIC step n -> n+1 (Section 2.3, eqs. 17-21), both phases sorted on   */
/* entry and exit.  Returns the number of cells that held one phase only.    */
/* ------------------------------------------------------------------------ */
typedef struct {
    double Mg, Md, Pg[3], Pd[3];
    double alpha, beta, V[3], U[3];
    int64_t N, L;
} orc_cell;

/* ------------------------------------------------------------------------ */
/* Drag in cell (Section 2.3, eqs. 17-21) with first-order time differences  */
/* over a step tau_eff: the current velocities of both phases are the        */
/* predictors v~, u~; per volume the mass-weighted means solve the 2x2       */
/* system, then every particle relaxes toward the other phase's new mean.    */
/* Both phases sorted with matching starts.  Returns the number of volumes   */
/* that hold one phase only (no drag there).                                 */
/* ------------------------------------------------------------------------ */
static int64_t orc_drag_cells(const orc_params *p, orc_phase *G, orc_phase *Dd, const int64_t *sg,
                              const int64_t *sd, double tau, double vol, orc_cell *cells)
{
    const int dim = p->dim;
    const int64_t nc = orc_ncells(p);
    const int64_t ng = G->n, nd = Dd->n;
    /* eq. (17), (21): per-volume masses and momenta, canonical order */
    int64_t empty = 0;
#pragma omp parallel for schedule(static) reduction(+ : empty)
    for (int64_t c = 0; c < nc; ++c) {
        orc_cell *C = &cells[c];
        memset(C, 0, sizeof(*C));
        C->N = sg[c + 1] - sg[c];
        C->L = sd[c + 1] - sd[c];
        for (int64_t a = sg[c]; a < sg[c + 1]; ++a) {
            C->Mg += G->mass[a];
            for (int d = 0; d < dim; ++d) C->Pg[d] += G->mass[a] * G->vel[d * ng + a];
        }
        for (int64_t j = sd[c]; j < sd[c + 1]; ++j) {
            C->Md += Dd->mass[j];
            for (int d = 0; d < dim; ++d) C->Pd[d] += Dd->mass[j] * Dd->vel[d * nd + j];
        }
        if (C->N > 0 && C->L > 0) {
            if (p->K > 0.0) {
                /* K* = K with the volume averages rho*_g = M_g / V, rho*_d = M_d / V:
                 * tau K* / rho*_g and tau K* / rho*_d */
                C->alpha = tau * p->K * vol / C->Mg;
                C->beta = tau * p->K * vol / C->Md;
            } else if (p->tse > 0.0) {
                /* t*_stop = tse / rho*_g, K* = rho*_d / t*_stop = rho*_d rho*_g / tse:
                 * tau K* / rho*_g = tau rho*_d / tse, tau K* / rho*_d = tau rho*_g / tse */
                C->alpha = tau * (C->Md / vol) / p->tse;
                C->beta = tau * (C->Mg / vol) / p->tse;
            } else {
                /* eq. (17)-(18): eps = M_d / M_g; K over the cell gas density is eps / t_stop,
                 * K over the cell dust density is 1 / t_stop */
                double eps = C->Md / C->Mg;
                C->beta = tau / p->tstop;
                C->alpha = eps * C->beta;
            }
            double Dt = 1.0 + C->alpha + C->beta;
            for (int d = 0; d < dim; ++d) {
                double Vt = C->Pg[d] / C->Mg, Ut = C->Pd[d] / C->Md;
                /* cell means at n+1 solve (1+alpha)V - alpha U = V~, -beta V + (1+beta) U = U~ */
                C->V[d] = ((1.0 + C->beta) * Vt + C->alpha * Ut) / Dt;
                C->U[d] = (C->beta * Vt + (1.0 + C->alpha) * Ut) / Dt;
            }
        } else {
            C->alpha = C->beta = 0.0;
            if (C->N > 0 || C->L > 0) empty += 1;
        }
    }

    /* eq. (19)-(20) with the other phase's velocity uniform over the volume */
    for (int64_t c = 0; c < nc; ++c) {
        const orc_cell *C = &cells[c];
        for (int64_t a = sg[c]; a < sg[c + 1]; ++a)
            for (int d = 0; d < dim; ++d)
                G->vel[d * ng + a] = (G->vel[d * ng + a] + C->alpha * C->U[d]) / (1.0 + C->alpha);
        for (int64_t j = sd[c]; j < sd[c + 1]; ++j)
            for (int d = 0; d < dim; ++d)
                Dd->vel[d * nd + j] = (Dd->vel[d * nd + j] + C->beta * C->V[d]) / (1.0 + C->beta);
    }
    return empty;
}

int64_t orc_step(const orc_params *p, orc_phase *G, orc_phase *Dd, int32_t nsteps,
                 double *cell_diag /* optional [ncells][2+2*dim]: alpha, beta, V*, U* of the last step */)
{
    const int dim = p->dim;
    const int64_t nc = orc_ncells(p);
    const int64_t ng = G->n, nd = Dd->n;
    const double tau = p->dt;
    double vol = 1.0;   /* volume of one drag cell (length in 1D, area in 2D) */
    for (int d = 0; d < dim; ++d) vol *= (p->hi[d] - p->lo[d]) / p->nc[d];
    int64_t *sg = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    double *acc = (double *)malloc(sizeof(double) * (dim * ng + 1));
    double *dedt = (double *)malloc(sizeof(double) * (ng + 1));
    orc_cell *cells = (orc_cell *)malloc(sizeof(orc_cell) * nc);
    int64_t empty_total = 0;

    for (int32_t s = 0; s < nsteps; ++s) {
        /* volumes at level n */
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
        orc_sort(p, G);
        orc_sort(p, Dd);
        orc_cell_start(p, G, sg);
        orc_cell_start(p, Dd, sd);

        /* explicit SPH terms at level n */
        orc_density(p, G, sg, G->rho);
        orc_gas_forces(p, G, sg, acc, G->energy ? dedt : NULL);

        /* predictor: v~ = v + tau A, u~ = u + tau g, e += tau de/dt */
        for (int d = 0; d < dim; ++d) {
            for (int64_t a = 0; a < ng; ++a) G->vel[d * ng + a] += tau * acc[d * ng + a];
            for (int64_t j = 0; j < nd; ++j) Dd->vel[d * nd + j] += tau * p->g[d];
        }
        if (G->energy)
            for (int64_t a = 0; a < ng; ++a) G->energy[a] += tau * dedt[a];

        empty_total += orc_drag_cells(p, G, Dd, sg, sd, tau, vol, cells);
        if (cell_diag && s == nsteps - 1) {
            int w = 2 + 2 * dim;
            for (int64_t c = 0; c < nc; ++c) {
                cell_diag[c * w + 0] = cells[c].alpha;
                cell_diag[c * w + 1] = cells[c].beta;
                for (int d = 0; d < dim; ++d) {
                    cell_diag[c * w + 2 + d] = cells[c].V[d];
                    cell_diag[c * w + 2 + dim + d] = cells[c].U[d];
                }
            }
        }

        /* positions: x^{n+1} = x^n + tau v^{n+1}, then back into [0, Delta) */
        for (int d = 0; d < dim; ++d) {
            for (int64_t a = 0; a < ng; ++a) G->off[d * ng + a] += tau * G->vel[d * ng + a];
            for (int64_t j = 0; j < nd; ++j) Dd->off[d * nd + j] += tau * Dd->vel[d * nd + j];
        }
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
    }
    free(sg); free(sd); free(acc); free(dedt); free(cells);
    return empty_total;
}

/* ------------------------------------------------------------------------ */
/* Second-order IMEX step: the ARS(2,2,2) pair of Ascher, Ruuth & Spiteri   */
/* (Appl. Numer. Math. 25, 1997), with gamma = 1 - 1/sqrt(2) and             */
/* delta = 1 - 1/(2 gamma).  Split of the two-fluid system (eqs. 1-2):       */
/*   explicit part f: dx/dt = v (u), the SPH pressure and viscosity terms    */
/*                    and g of eq. (19), de/dt of the gas;                   */
/*   implicit part g: the drag in cell of eqs. (19)-(21), i.e. each gas       */
/*                    particle relaxes toward the dust mean of its volume at  */
/*                    rate K* / rho*_g and each dust particle toward the gas */
/*                    mean at rate K* / rho*_d, volumes and rates frozen at   */
/*                    the stage's positions.                                  */
/* Stages (Y1 = y^n):                                                        */
/*   Y2 = y^n + gamma tau f(Y1) + gamma tau g(Y2)                             */
/*   Y3 = y^n + tau (delta f(Y1) + (1 - delta) f(Y2))                         */
/*            + tau (1 - gamma) g(Y2) + gamma tau g(Y3),    y^{n+1} = Y3.     */
/* Each implicit stage is the paper's first-order drag solve with time step   */
/* gamma tau on the predictor formed from the explicit terms.  The stage-2    */
/* drag rate comes from its own equation, g(Y2) = (Y2 - Y2~) / (gamma tau),   */
/* so tau (1 - gamma) g(Y2) = ((1 - gamma) / gamma) (Y2 - Y2~).  rho on exit  */
/* is the summation density at level n, as for the first-order step.         */
/* ------------------------------------------------------------------------ */
typedef struct {
    orc_phase ph;
    int32_t *cell, *id;
    double *off, *vel, *mass, *rho, *energy;
} orc_stage_copy;

static void orc_stage_alloc(orc_stage_copy *q, const orc_phase *src, int dim)
{
    const int64_t n = src->n, m = n ? n : 1;
    q->cell = (int32_t *)malloc(sizeof(int32_t) * m);
    q->id = (int32_t *)malloc(sizeof(int32_t) * m);
    q->off = (double *)malloc(sizeof(double) * dim * m);
    q->vel = (double *)malloc(sizeof(double) * dim * m);
    q->mass = (double *)malloc(sizeof(double) * m);
    q->rho = (double *)malloc(sizeof(double) * m);
    q->energy = src->energy ? (double *)malloc(sizeof(double) * m) : NULL;
    q->ph.n = n;
    q->ph.cell = q->cell; q->ph.id = q->id; q->ph.off = q->off; q->ph.vel = q->vel;
    q->ph.mass = q->mass; q->ph.rho = q->rho; q->ph.energy = q->energy;
}

static void orc_stage_free(orc_stage_copy *q)
{
    free(q->cell); free(q->id); free(q->off); free(q->vel); free(q->mass); free(q->rho); free(q->energy);
}

int64_t orc_step_imex(const orc_params *p, orc_phase *G, orc_phase *Dd, int32_t nsteps)
{
    const int dim = p->dim;
    const int64_t nc = orc_ncells(p);
    const int64_t ng = G->n, nd = Dd->n;
    const double tau = p->dt;
    const double gam = 1.0 - 1.0 / sqrt(2.0);
    const double del = 1.0 - 1.0 / (2.0 * gam);
    const double gtau = gam * tau;
    const double rg = (1.0 - gam) / gam;
    double vol = 1.0;
    for (int d = 0; d < dim; ++d) vol *= (p->hi[d] - p->lo[d]) / p->nc[d];
    const int64_t mg = ng ? ng : 1, md = nd ? nd : 1;
    int64_t *sg = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sq = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sr = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *pg = (int64_t *)malloc(sizeof(int64_t) * mg);
    int64_t *pd = (int64_t *)malloc(sizeof(int64_t) * md);
    /* per particle, in the order of level n (gas: A1, A2 include g) */
    double *A1 = (double *)malloc(sizeof(double) * dim * mg), *A2 = (double *)malloc(sizeof(double) * dim * mg);
    double *E1 = (double *)malloc(sizeof(double) * mg), *E2 = (double *)malloc(sizeof(double) * mg);
    double *V2 = (double *)malloc(sizeof(double) * dim * mg), *D2 = (double *)malloc(sizeof(double) * dim * mg);
    double *U2 = (double *)malloc(sizeof(double) * dim * md), *F2 = (double *)malloc(sizeof(double) * dim * md);
    double *At = (double *)malloc(sizeof(double) * dim * mg), *Et = (double *)malloc(sizeof(double) * mg);
    double *Pq = (double *)malloc(sizeof(double) * dim * mg), *Pr = (double *)malloc(sizeof(double) * dim * md);
    orc_cell *cells = (orc_cell *)malloc(sizeof(orc_cell) * nc);
    orc_stage_copy Q, Rr;
    orc_stage_alloc(&Q, G, dim);
    orc_stage_alloc(&Rr, Dd, dim);
    int64_t empty_total = 0;

    for (int32_t s = 0; s < nsteps; ++s) {
        /* stage 1: volumes and explicit terms at level n */
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
        orc_sort(p, G);
        orc_sort(p, Dd);
        orc_cell_start(p, G, sg);
        orc_cell_start(p, Dd, sd);
        orc_density(p, G, sg, G->rho);
        orc_gas_forces(p, G, sg, A1, G->energy ? E1 : NULL);

        /* stage 2 predictor: Y2~ = y^n + gamma tau f(Y1) */
        for (int64_t a = 0; a < ng; ++a) {
            Q.cell[a] = G->cell[a];
            Q.id[a] = G->id[a];
            Q.mass[a] = G->mass[a];
            for (int d = 0; d < dim; ++d) {
                Q.off[d * ng + a] = G->off[d * ng + a] + gtau * G->vel[d * ng + a];
                Q.vel[d * ng + a] = G->vel[d * ng + a] + gtau * A1[d * ng + a];
            }
            if (G->energy) Q.energy[a] = G->energy[a] + gtau * E1[a];
        }
        for (int64_t j = 0; j < nd; ++j) {
            Rr.cell[j] = Dd->cell[j];
            Rr.id[j] = Dd->id[j];
            Rr.mass[j] = Dd->mass[j];
            for (int d = 0; d < dim; ++d) {
                Rr.off[d * nd + j] = Dd->off[d * nd + j] + gtau * Dd->vel[d * nd + j];
                Rr.vel[d * nd + j] = Dd->vel[d * nd + j] + gtau * p->g[d];
            }
        }
        /* volumes at the stage-2 positions, implicit drag over gamma tau */
        orc_canonicalize(p, &Q.ph);
        orc_canonicalize(p, &Rr.ph);
        orc_sort_perm(p, &Q.ph, pg);
        orc_sort_perm(p, &Rr.ph, pd);
        orc_cell_start(p, &Q.ph, sq);
        orc_cell_start(p, &Rr.ph, sr);
        memcpy(Pq, Q.vel, sizeof(double) * dim * ng);
        memcpy(Pr, Rr.vel, sizeof(double) * dim * nd);
        empty_total += orc_drag_cells(p, &Q.ph, &Rr.ph, sq, sr, gtau, vol, cells);
        for (int64_t k = 0; k < ng; ++k)
            for (int d = 0; d < dim; ++d) {
                V2[d * ng + pg[k]] = Q.vel[d * ng + k];
                D2[d * ng + pg[k]] = Q.vel[d * ng + k] - Pq[d * ng + k];
            }
        for (int64_t k = 0; k < nd; ++k)
            for (int d = 0; d < dim; ++d) {
                U2[d * nd + pd[k]] = Rr.vel[d * nd + k];
                F2[d * nd + pd[k]] = Rr.vel[d * nd + k] - Pr[d * nd + k];
            }
        /* explicit terms at Y2 */
        orc_density(p, &Q.ph, sq, Q.rho);
        orc_gas_forces(p, &Q.ph, sq, At, Q.energy ? Et : NULL);
        for (int64_t k = 0; k < ng; ++k) {
            for (int d = 0; d < dim; ++d) A2[d * ng + pg[k]] = At[d * ng + k];
            if (Q.energy) E2[pg[k]] = Et[k];
        }

        /* stage 3 predictor, in the order of level n:
         * Y3~ = y^n + tau (delta f(Y1) + (1 - delta) f(Y2)) + tau (1 - gamma) g(Y2) */
        for (int64_t a = 0; a < ng; ++a) {
            for (int d = 0; d < dim; ++d) {
                const double v0 = G->vel[d * ng + a];
                G->off[d * ng + a] += tau * (del * v0 + (1.0 - del) * V2[d * ng + a]);
                G->vel[d * ng + a] = v0 + tau * (del * A1[d * ng + a] + (1.0 - del) * A2[d * ng + a])
                                     + rg * D2[d * ng + a];
            }
            if (G->energy) G->energy[a] += tau * (del * E1[a] + (1.0 - del) * E2[a]);
        }
        for (int64_t j = 0; j < nd; ++j)
            for (int d = 0; d < dim; ++d) {
                const double u0 = Dd->vel[d * nd + j];
                Dd->off[d * nd + j] += tau * (del * u0 + (1.0 - del) * U2[d * nd + j]);
                Dd->vel[d * nd + j] = u0 + tau * p->g[d] + rg * F2[d * nd + j];
            }
        /* volumes at the stage-3 positions, implicit drag over gamma tau: y^{n+1} = Y3 */
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
        orc_sort(p, G);
        orc_sort(p, Dd);
        orc_cell_start(p, G, sg);
        orc_cell_start(p, Dd, sd);
        empty_total += orc_drag_cells(p, G, Dd, sg, sd, gtau, vol, cells);
    }
    orc_stage_free(&Q);
    orc_stage_free(&Rr);
    free(sg); free(sd); free(sq); free(sr); free(pg); free(pd);
    free(A1); free(A2); free(E1); free(E2); free(V2); free(D2); free(U2); free(F2);
    free(At); free(Et); free(Pq); free(Pr); free(cells);
    return empty_total;
}

/* ------------------------------------------------------------------------ */
/* The paper's two comparison schemes for the drag (Section 2.1 and 2.2).    */
/* Both share the SPH part of the IDIC step above: summation densities, the  */
/* gas pressure (and viscosity) terms of eq. (8) / (12), the gas energy      */
/* equation, and the symplectic position update x^{n+1} = x^n + tau v^{n+1}. */
/* They differ from it only in how the drag is computed.                     */
/*                                                                           */
/* The drag coefficient of a pair or a point follows the run's drag law:     */
/*   K held constant (p->K > 0):       K;                                    */
/*   t_stop held constant:             K = rho_d / t_stop (eq. 7), rho_d the */
/*                                     dust density at the point;            */
/*   Epstein, t_stop = tse / rho_g:    K = rho_g rho_d / tse (eq. 10 and 16  */
/*                                     with c_s / (s rho_s) = 1 / tse).      */
/* ------------------------------------------------------------------------ */
static double orc_drag_K(const orc_params *p, double rho_g, double rho_d)
{
    if (p->K > 0.0) return p->K;
    if (p->tse > 0.0) return rho_g * rho_d / p->tse;
    return rho_d / p->tstop;
}

/* --- Monaghan-Kocharyan explicit pairwise drag, eqs. (8)-(10) ----------- */
/* For gas a and dust j with r_ja = x_j - x_a, the pair term                 */
/*   X_aj = K_aj / (rho_a rho_j) ((v_a - u_j) . r_ja) / (r_ja^2 + eta^2)     */
/*          r_ja W(r_ja, h),          eta^2 = 0.001 h^2,                     */
/* enters dv_a/dt as -sigma sum_j m_j X_aj and du_j/dt as +sigma sum_a m_a   */
/* X_aj, with the velocities of level n.  sigma = 1 in 1D (stated); for d    */
/* dimensions sigma = d, which makes the kernel average of r r / r^2 equal   */
/* the identity, so a uniform relative velocity feels the continuum drag.    */
typedef struct {
    const orc_params *p; const orc_phase *A; const orc_phase *B;
    const double *rhoA; const double *rhoB; int a_is_gas;
    double acc[3];
} orc_mk_ctx;

static void orc_mk_pair(void *vctx, int64_t a, int64_t b, const double r[3])
{
    orc_mk_ctx *c = (orc_mk_ctx *)vctx;
    const orc_params *p = c->p;
    const int dim = p->dim;
    const double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double rr = sqrt(rr2);
    if (!(rr < 2.0 * p->h)) return;
    const int64_t na = c->A->n, nb = c->B->n;
    /* gas velocity minus dust velocity, whichever phase is the target */
    double dv[3] = {0.0, 0.0, 0.0};
    for (int d = 0; d < dim; ++d) {
        const double va = c->A->vel[d * na + a], vb = c->B->vel[d * nb + b];
        dv[d] = c->a_is_gas ? va - vb : vb - va;
    }
    const double rho_g = c->a_is_gas ? c->rhoA[a] : c->rhoB[b];
    const double rho_d = c->a_is_gas ? c->rhoB[b] : c->rhoA[a];
    double vr = 0.0;
    for (int d = 0; d < dim; ++d) vr += dv[d] * r[d];
    const double eta2 = 0.001 * p->h * p->h;
    const double X = orc_drag_K(p, rho_g, rho_d) / (rho_g * rho_d) * vr / (rr2 + eta2) *
                     orc_kernel_w(dim, p->h, rr);
    const double sgn = c->a_is_gas ? -1.0 : 1.0;
    for (int d = 0; d < dim; ++d) c->acc[d] += sgn * (double)dim * c->B->mass[b] * X * r[d];
}

/* drag accelerations of every particle of A from the particles of B */
static void orc_mk_drag(const orc_params *p, const orc_phase *A, const orc_phase *B, const int64_t *startB,
                        const double *rhoA, const double *rhoB, int a_is_gas, double *out /* [dim][nA] */)
{
    const int64_t n = A->n;
#pragma omp parallel for schedule(static)
    for (int64_t a = 0; a < n; ++a) {
        orc_mk_ctx c = {p, A, B, rhoA, rhoB, a_is_gas, {0.0, 0.0, 0.0}};
        orc_for_neighbours(p, A, a, B, startB, orc_mk_pair, &c);
        for (int d = 0; d < p->dim; ++d) out[d * n + a] = c.acc[d];
    }
}

/* One explicit MK step n -> n+1 (first order in time): v^{n+1} = v^n + tau   */
/* (pressure + g + drag), u^{n+1} = u^n + tau (g + drag), e^{n+1} = e^n + tau */
/* de/dt, then x^{n+1} = x^n + tau v^{n+1}.  rho of both phases on exit is    */
/* the summation density of level n.  Stable only for tau below about t_stop */
/* (eq. 5).                                                                   */
void orc_step_mk(const orc_params *p, orc_phase *G, orc_phase *Dd, int32_t nsteps)
{
    const int dim = p->dim;
    const int64_t nc = orc_ncells(p);
    const int64_t ng = G->n, nd = Dd->n, mg = ng ? ng : 1, md = nd ? nd : 1;
    const double tau = p->dt;
    int64_t *sg = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    double *acc = (double *)malloc(sizeof(double) * dim * mg);
    double *dedt = (double *)malloc(sizeof(double) * mg);
    double *dg = (double *)malloc(sizeof(double) * dim * mg);
    double *dd = (double *)malloc(sizeof(double) * dim * md);
    for (int32_t s = 0; s < nsteps; ++s) {
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
        orc_sort(p, G);
        orc_sort(p, Dd);
        orc_cell_start(p, G, sg);
        orc_cell_start(p, Dd, sd);
        orc_density(p, G, sg, G->rho);
        orc_density(p, Dd, sd, Dd->rho);
        orc_gas_forces(p, G, sg, acc, G->energy ? dedt : NULL);
        orc_mk_drag(p, G, Dd, sd, G->rho, Dd->rho, 1, dg);
        orc_mk_drag(p, Dd, G, sg, Dd->rho, G->rho, 0, dd);
        for (int d = 0; d < dim; ++d) {
            for (int64_t a = 0; a < ng; ++a) G->vel[d * ng + a] += tau * (acc[d * ng + a] + dg[d * ng + a]);
            for (int64_t j = 0; j < nd; ++j) Dd->vel[d * nd + j] += tau * (p->g[d] + dd[d * nd + j]);
        }
        if (G->energy)
            for (int64_t a = 0; a < ng; ++a) G->energy[a] += tau * dedt[a];
        for (int d = 0; d < dim; ++d) {
            for (int64_t a = 0; a < ng; ++a) G->off[d * ng + a] += tau * G->vel[d * ng + a];
            for (int64_t j = 0; j < nd; ++j) Dd->off[d * nd + j] += tau * Dd->vel[d * nd + j];
        }
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
    }
    free(sg); free(sd); free(acc); free(dedt); free(dg); free(dd);
}

/* --- ISPH: semi-implicit drag with SPH interpolation, eqs. (11)-(16) ----- */
/* At every particle the other phase's velocity is interpolated (eq. 11):    */
/*   at dust j:  v_j = sum_a m_a (v_a / rho_a) W_aj;                         */
/*   at gas a:   u_a = sum_j m_j (u_j / rho_j) W_ja;                         */
/* with the other quantities the scheme marks as interpolated: the dust      */
/* density at a gas point, rho_a,d = sum_j m_j W_ja; at a dust point the gas  */
/* density rho_j,g = sum_a m_a W_aj and pressure p_j = sum_a m_a (p_a/rho_a)  */
/* W_aj.  Every particle then solves its own two-velocity system with first- */
/* order time differences (eqs. 12-15): with alpha = tau K / rho_g and       */
/* beta = tau K / rho_d at the point, and the predictors v~ = v + tau A,     */
/* u~ = u + tau g,                                                           */
/*   (1 + alpha) v - alpha u = v~,   -beta v + (1 + beta) u = u~,            */
/* the gas particle keeps v (eq. 12) and the dust particle keeps u (eq. 15). */
/* At a gas particle A is its SPH acceleration of eq. (12); at a dust point  */
/* it is the gas pressure gradient of eq. (14),                              */
/*   A_j = -sum_i m_i (p_i / rho_i^2 + p_j / rho_j,g^2) grad_j W_ij + g.      */
/* eq. (15) writes rho^n_{a,d} for the dust density, read as rho^n_{j,d}, the */
/* dust particle's own.  A particle with no particle of the other phase      */
/* within 2h gets no drag (counted in the return value).                     */
typedef struct {
    const orc_params *p; const orc_phase *B; const double *rhoB; const double *presB;
    double rho, vel[3], pres;
} orc_interp_ctx;

static void orc_interp_pair(void *vctx, int64_t a, int64_t b, const double r[3])
{
    (void)a;
    orc_interp_ctx *c = (orc_interp_ctx *)vctx;
    const orc_params *p = c->p;
    const double rr = sqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
    if (!(rr < 2.0 * p->h)) return;
    const double mW = c->B->mass[b] * orc_kernel_w(p->dim, p->h, rr);
    const int64_t nb = c->B->n;
    c->rho += mW;
    for (int d = 0; d < p->dim; ++d) c->vel[d] += mW * c->B->vel[d * nb + b] / c->rhoB[b];
    if (c->presB) c->pres += mW * c->presB[b] / c->rhoB[b];
}

typedef struct {
    const orc_params *p; const orc_phase *G; const double *rhoG; const double *presG;
    double Pj;      /* p_j / rho_j,g^2 at the dust point */
    double acc[3];
} orc_dpg_ctx;

static void orc_dust_pgrad_pair(void *vctx, int64_t j, int64_t i, const double r[3])
{
    (void)j;
    orc_dpg_ctx *c = (orc_dpg_ctx *)vctx;
    const orc_params *p = c->p;
    const double rr2 = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
    const double rr = sqrt(rr2);
    if (!(rr < 2.0 * p->h) || rr == 0.0) return;
    const double dw = orc_kernel_dw(p->dim, p->h, rr);
    const double Pi = c->presG[i] / (c->rhoG[i] * c->rhoG[i]);
    for (int d = 0; d < p->dim; ++d) c->acc[d] -= c->G->mass[i] * (Pi + c->Pj) * dw * r[d] / rr;
}

int64_t orc_step_isph(const orc_params *p, orc_phase *G, orc_phase *Dd, int32_t nsteps)
{
    const int dim = p->dim;
    const int64_t nc = orc_ncells(p);
    const int64_t ng = G->n, nd = Dd->n, mg = ng ? ng : 1, md = nd ? nd : 1;
    const double tau = p->dt;
    int64_t *sg = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    int64_t *sd = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    double *acc = (double *)malloc(sizeof(double) * dim * mg);
    double *dedt = (double *)malloc(sizeof(double) * mg);
    double *pres = (double *)malloc(sizeof(double) * mg);
    double *vnew = (double *)malloc(sizeof(double) * dim * mg);
    double *unew = (double *)malloc(sizeof(double) * dim * md);
    int64_t lonely_total = 0;
    for (int32_t s = 0; s < nsteps; ++s) {
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
        orc_sort(p, G);
        orc_sort(p, Dd);
        orc_cell_start(p, G, sg);
        orc_cell_start(p, Dd, sd);
        orc_density(p, G, sg, G->rho);
        orc_density(p, Dd, sd, Dd->rho);
        orc_gas_forces(p, G, sg, acc, G->energy ? dedt : NULL);
        for (int64_t a = 0; a < ng; ++a) pres[a] = orc_pressure(p, G->rho[a], G->energy ? G->energy[a] : 0.0);
        int64_t lonely = 0;
        /* gas particles: eqs. (12)-(13) */
#pragma omp parallel for schedule(static) reduction(+ : lonely)
        for (int64_t a = 0; a < ng; ++a) {
            orc_interp_ctx c = {p, Dd, Dd->rho, NULL, 0.0, {0.0, 0.0, 0.0}, 0.0};
            orc_for_neighbours(p, G, a, Dd, sd, orc_interp_pair, &c);
            const double rho_g = G->rho[a];
            double alpha = 0.0, beta = 0.0;
            if (c.rho > 0.0) {
                const double K = orc_drag_K(p, rho_g, c.rho);
                alpha = tau * K / rho_g;
                beta = tau * K / c.rho;
            } else {
                lonely += 1;
            }
            const double D = 1.0 + alpha + beta;
            for (int d = 0; d < dim; ++d) {
                const double vt = G->vel[d * ng + a] + tau * acc[d * ng + a];
                const double ut = (c.rho > 0.0 ? c.vel[d] : 0.0) + tau * p->g[d];
                vnew[d * ng + a] = ((1.0 + beta) * vt + alpha * ut) / D;
            }
        }
        /* dust particles: eqs. (14)-(15) */
#pragma omp parallel for schedule(static) reduction(+ : lonely)
        for (int64_t j = 0; j < nd; ++j) {
            orc_interp_ctx c = {p, G, G->rho, pres, 0.0, {0.0, 0.0, 0.0}, 0.0};
            orc_for_neighbours(p, Dd, j, G, sg, orc_interp_pair, &c);
            const double rho_d = Dd->rho[j];
            double alpha = 0.0, beta = 0.0, Aj[3] = {0.0, 0.0, 0.0};
            if (c.rho > 0.0) {
                orc_dpg_ctx q = {p, G, G->rho, pres, c.pres / (c.rho * c.rho), {0.0, 0.0, 0.0}};
                orc_for_neighbours(p, Dd, j, G, sg, orc_dust_pgrad_pair, &q);
                for (int d = 0; d < dim; ++d) Aj[d] = q.acc[d];
                const double K = orc_drag_K(p, c.rho, rho_d);
                alpha = tau * K / c.rho;
                beta = tau * K / rho_d;
            } else {
                lonely += 1;
            }
            const double D = 1.0 + alpha + beta;
            for (int d = 0; d < dim; ++d) {
                const double vt = c.vel[d] + tau * (Aj[d] + p->g[d]);
                const double ut = Dd->vel[d * nd + j] + tau * p->g[d];
                unew[d * nd + j] = (beta * vt + (1.0 + alpha) * ut) / D;
            }
        }
        lonely_total += lonely;
        memcpy(G->vel, vnew, sizeof(double) * dim * ng);
        memcpy(Dd->vel, unew, sizeof(double) * dim * nd);
        if (G->energy)
            for (int64_t a = 0; a < ng; ++a) G->energy[a] += tau * dedt[a];
        for (int d = 0; d < dim; ++d) {
            for (int64_t a = 0; a < ng; ++a) G->off[d * ng + a] += tau * G->vel[d * ng + a];
            for (int64_t j = 0; j < nd; ++j) Dd->off[d * nd + j] += tau * Dd->vel[d * nd + j];
        }
        orc_canonicalize(p, G);
        orc_canonicalize(p, Dd);
    }
    free(sg); free(sd); free(acc); free(dedt); free(pres); free(vnew); free(unew);
    return lonely_total;
}

/* Density sums on the phase's current positions (sorts the phase first). */
void orc_phase_density(const orc_params *p, orc_phase *ph, double *rho_out)
{
    int64_t nc = orc_ncells(p);
    int64_t *st = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    orc_canonicalize(p, ph);
    orc_sort(p, ph);
    orc_cell_start(p, ph, st);
    orc_density(p, ph, st, rho_out);
    free(st);
}

/* Gas forces on the current positions (sorts the phase, fills rho). */
void orc_phase_forces(const orc_params *p, orc_phase *G, double *acc_out, double *dedt_out)
{
    int64_t nc = orc_ncells(p);
    int64_t *st = (int64_t *)malloc(sizeof(int64_t) * (nc + 1));
    orc_canonicalize(p, G);
    orc_sort(p, G);
    orc_cell_start(p, G, st);
    orc_density(p, G, st, G->rho);
    orc_gas_forces(p, G, st, acc_out, dedt_out);
    free(st);
}

int orc_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* Threads for the following calls (results do not depend on it: every
 * per-particle and per-cell sum is serial in canonical order). */
void orc_set_num_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}
