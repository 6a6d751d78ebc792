// Host side of the batched form (declarations and contract: include/tfsph.h):
// instance table, largest-first launch order, either one persistent kernel per
// call or the flattened launches of every step (block tables per instance),
// optional hipGraph replay.
#include "../../include/tfsph.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <map>
#include <new>
#include <numeric>
#include <tuple>
#include <vector>

#include "batched.hpp"
#include "enqueue.hpp"
#include "host.hpp"

using namespace tfsph;
using namespace tfsph_host;

namespace {

constexpr int kDefaultBatchBlock = 512;
// cells per block of the flattened form's update launch (the single-problem default)
inline int kFlatCells(int dim) { return default_cells_per_block(dim); }

struct InstLayout {
    int ng, nd, ncell;
    bool mass_g, mass_d;
};

template <typename R>
size_t batch_bytes(const std::vector<InstLayout> &L, int dim, Carver &cv, std::vector<Inst<R>> *table,
                   const tfsph_batch_desc *desc, const tfsph_state *packed)
{
    const int n = (int)L.size();
    Inst<R> *dev_table = cv.take<Inst<R>>(n);
    int *order = cv.take<int>(n);
    unsigned int *word = cv.take<unsigned int>(64);
    unsigned long long *one = cv.take<unsigned long long>(8);
    // block tables of the flattened form: over the particles of both phases, and over the
    // cells at one cell per block (the most blocks any cells_per_block gives)
    size_t part = 0, cells = 0;
    for (const InstLayout &l : L) {
        part += size_t(blocks_for(l.ng)) + size_t(blocks_for(l.nd));
        cells += size_t(l.ncell);
    }
    int2 *tab_part = cv.take<int2>(part);
    int2 *tab_cells = cv.take<int2>(cells);
    (void)dev_table, (void)order, (void)word, (void)one, (void)tab_part, (void)tab_cells;
    for (int i = 0; i < n; ++i) {
        PhaseFlags fg{L[i].mass_g, false, true}, fd{L[i].mass_d, false, false};
        Sorted<R> Sg = carve_phase<R>(cv, L[i].ng, dim, L[i].ncell, fg);
        Sorted<R> Sd = carve_phase<R>(cv, L[i].nd, dim, L[i].ncell, fd);
        CellSolve<R> *cs = cv.take<CellSolve<R>>(L[i].ncell);
        if (table) {
            Inst<R> I{};
            const tfsph_params *p = &desc->params[i];
            I.G = make_geom<R>(p);
            I.Ph = make_phys<R>(p);
            tfsph_phase g = packed->gas, d = packed->dust;
            const int64_t go = desc->gas_offset[i], dof = desc->dust_offset[i];
            auto shift = [](void *base, int64_t k, size_t sz) -> void * {
                return base ? static_cast<char *>(base) + k * sz : nullptr;
            };
            const size_t rs = sizeof(R);
            g.n = L[i].ng;
            d.n = L[i].nd;
            g.cell = g.cell ? g.cell + go : nullptr;
            d.cell = d.cell ? d.cell + dof : nullptr;
            g.id = g.id ? g.id + go : nullptr;
            d.id = d.id ? d.id + dof : nullptr;
            for (int k = 0; k < 3; ++k) {
                g.off[k] = shift(g.off[k], go, rs), g.vel[k] = shift(g.vel[k], go, rs);
                d.off[k] = shift(d.off[k], dof, rs), d.vel[k] = shift(d.vel[k], dof, rs);
            }
            g.mass = shift(g.mass, go, rs);
            d.mass = shift(d.mass, dof, rs);
            g.rho = shift(g.rho, go, rs);
            d.rho = shift(d.rho, dof, rs);
            g.energy = nullptr;
            d.energy = nullptr;
            g.mass_uniform = desc->mass_gas ? desc->mass_gas[i] : packed->gas.mass_uniform;
            d.mass_uniform = desc->mass_dust ? desc->mass_dust[i] : packed->dust.mass_uniform;
            I.Pg = make_phase<R>(g, dim);
            I.Pd = make_phase<R>(d, dim);
            I.Sg = Sg;
            I.Sd = Sd;
            I.cs = cs;
            table->push_back(I);
        }
    }
    return cv.off + 256;
}

// Deal the entries e[s, s + m) of a block table out so that the blocks a launch
// sends to one XCD (block b goes to XCD b % 8, round robin) take one contiguous
// run of entries: neighbouring blocks of an instance, which read each other's
// halos, then share that XCD's L2.
void xcd_deal(int2 *e, int s, int m)
{
    const std::vector<int2> run(e + s, e + s + m);
    int k = 0;
    for (int x = 0; x < 8; ++x)
        for (int b = s; b < s + m; ++b)
            if (b % 8 == x) e[b] = run[k++];
}

tfsph_status check_desc(const tfsph_batch_desc *desc, std::vector<InstLayout> &L, int &dim, int &prec)
{
    if (!desc || desc->n_inst < 1) return fail(TFSPH_E_INVALID_ARG, "batch needs at least one instance");
    if (!desc->params || !desc->gas_offset || !desc->dust_offset)
        return fail(TFSPH_E_INVALID_ARG, "batch desc has NULL arrays");
    dim = desc->params[0].dim;
    prec = desc->params[0].precision;
    if (dim != 1 && dim != 2) return fail(TFSPH_E_UNSUPPORTED, "batched instances must be 1D or 2D (dim %d)", dim);
    if (desc->gas_offset[0] != 0 || desc->dust_offset[0] != 0)
        return fail(TFSPH_E_INVALID_ARG, "offsets must start at 0");
    L.clear();
    for (int i = 0; i < desc->n_inst; ++i) {
        const tfsph_params *p = &desc->params[i];
        tfsph_status r = tfsph_validate(p);
        if (r != TFSPH_OK) return fail(r, "instance %d: %s", i, tfsph_last_error());
        if (p->scheme != TFSPH_SCHEME_IDIC)
            return fail(TFSPH_E_UNSUPPORTED, "instance %d: the batched form runs the first-order step only", i);
        if (p->dim != dim || p->precision != prec)
            return fail(TFSPH_E_INVALID_ARG, "instance %d: dim/precision differ from instance 0", i);
        if (p->eos != TFSPH_ISOTHERMAL) return fail(TFSPH_E_UNSUPPORTED, "instance %d: batched form is isothermal", i);
        const int64_t ng = desc->gas_offset[i + 1] - desc->gas_offset[i];
        const int64_t nd = desc->dust_offset[i + 1] - desc->dust_offset[i];
        if (ng < 0 || nd < 0 || ng > 0x7fffffffLL || nd > 0x7fffffffLL)
            return fail(TFSPH_E_INVALID_ARG, "instance %d: offsets not non-decreasing", i);
        L.push_back(InstLayout{(int)ng, (int)nd, ncell_of(p), false, false});
    }
    return TFSPH_OK;
}

}  // namespace

struct tfsph_batch {
    int n_inst = 0, dim = 1, prec = 0, block = kDefaultBatchBlock, form = TFSPH_BATCH_PERSISTENT;
    int flat_cpb = 0;              // cells per block of the flattened form's update launch
    int flat_kind = -1;            // force-loop kind of every instance (kForce*), -1 if they differ
    FlatTable flat{};
    int flat_blocks_g = 0, flat_blocks_d = 0, flat_blocks_c = 0;
    std::vector<int> host_ncell;   // cells of each instance
    std::vector<int2> host_part;   // block table over particles (kept alive for the async upload)
    std::vector<int2> host_cells;  // block table over cells, sized for one cell per block
    int2 *dev_cells = nullptr;     // its device copy (in the workspace)
    tfsph_state bound{};
    char *ws = nullptr;
    size_t ws_bytes = 0;
    void *table = nullptr;        // device
    int *order = nullptr;         // device
    Flags F{};
    std::vector<char> host_table; // kept alive for the async upload
    std::vector<int> host_order;
    hipStream_t last_stream = nullptr, capture_stream = nullptr;
    struct G {
        hipGraph_t graph = nullptr;
        hipGraphExec_t exec = nullptr;
    };
    std::map<std::tuple<int, int, int>, G> graphs;   // (n_steps, form, block) -> graph
};

// Block table of the flattened form over cells ((instance, block in the instance)
// at b->flat_cpb cells per block), uploaded on st, which is then synchronized (the
// host table is rewritten by the next call); flattened-form graphs captured with
// another table are dropped.
static tfsph_status upload_flat_cells(tfsph_batch *b, hipStream_t st)
{
    const int n = b->n_inst;
    int k = 0;
    for (int i = 0; i < n; ++i) {
        const int nb = (b->host_ncell[i] + b->flat_cpb - 1) / b->flat_cpb;
        for (int j = 0; j < nb; ++j) b->host_cells[k++] = make_int2(i, j);
    }
    xcd_deal(b->host_cells.data(), 0, k);
    b->flat_blocks_c = k;
    b->flat.cells_per_block = b->flat_cpb;
    for (auto it = b->graphs.begin(); it != b->graphs.end();) {
        if (std::get<1>(it->first) == TFSPH_BATCH_FLAT) {
            if (it->second.exec) (void)hipGraphExecDestroy(it->second.exec);
            if (it->second.graph) (void)hipGraphDestroy(it->second.graph);
            it = b->graphs.erase(it);
        } else {
            ++it;
        }
    }
    if (k) HIP_TRY(hipMemcpyAsync(b->dev_cells, b->host_cells.data(), sizeof(int2) * k, hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_batch_workspace_size(const tfsph_batch_desc *desc, size_t *bytes)
{
    std::vector<InstLayout> L;
    int dim, prec;
    tfsph_status r = check_desc(desc, L, dim, prec);
    if (r != TFSPH_OK) return r;
    if (!bytes) return fail(TFSPH_E_INVALID_ARG, "bytes is NULL");
    for (auto &l : L) l.mass_g = l.mass_d = true;   // largest layout
    Carver cv;
    *bytes = prec == TFSPH_F64 ? batch_bytes<double>(L, dim, cv, nullptr, desc, nullptr)
                               : batch_bytes<float>(L, dim, cv, nullptr, desc, nullptr);
    return TFSPH_OK;
}

static tfsph_status set_tuning(tfsph_batch *b, const tfsph_batch_tuning *t)
{
    int blk = (t && t->block) ? t->block : kDefaultBatchBlock;
    if (blk < 64 || blk > kBatchMaxBlock || blk % 64) return fail(TFSPH_E_INVALID_ARG, "block must be a multiple of 64 in 64..1024");
    const int form = t ? t->form : TFSPH_BATCH_PERSISTENT;
    if (form != TFSPH_BATCH_PERSISTENT && form != TFSPH_BATCH_FLAT)
        return fail(TFSPH_E_INVALID_ARG, "form must be TFSPH_BATCH_PERSISTENT or TFSPH_BATCH_FLAT (%d)", form);
    const int cpb = (t && t->cells_per_block) ? t->cells_per_block : kFlatCells(b->dim);
    if (cpb < 1 || cpb > kMaxCellsPerBlock)
        return fail(TFSPH_E_INVALID_ARG, "cells_per_block must be in 1..%d (0 = default), got %d", kMaxCellsPerBlock, cpb);
    b->block = blk;
    b->form = form;
    if (cpb != b->flat_cpb) {
        b->flat_cpb = cpb;
        if (b->dev_cells) return upload_flat_cells(b, b->last_stream);
    }
    return TFSPH_OK;
}

template <typename R>
static tfsph_status batch_setup(tfsph_batch *b, const tfsph_batch_desc *desc, std::vector<InstLayout> &L,
                                tfsph_state *packed, hipStream_t st)
{
    std::vector<Inst<R>> table;
    table.reserve(L.size());
    Carver cv;
    cv.base = b->ws;
    batch_bytes<R>(L, b->dim, cv, &table, desc, packed);
    Carver head;
    head.base = b->ws;
    b->table = head.take<Inst<R>>(L.size());
    b->order = head.take<int>(L.size());
    b->F.word = head.take<unsigned int>(64);
    b->F.one_phase = head.take<unsigned long long>(8);
    // block tables of the flattened form: (instance, block in the instance) of every block of
    // the launches over both phases' particles (gas blocks, then dust blocks) and over the cells
    const int n = (int)L.size();
    size_t ncell_total = 0;
    b->host_part.clear();
    b->host_ncell.resize(n);
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < blocks_for(L[i].ng); ++j) b->host_part.push_back(make_int2(i, j));
    b->flat_blocks_g = (int)b->host_part.size();
    for (int i = 0; i < n; ++i)
        for (int j = 0; j < blocks_for(L[i].nd); ++j) b->host_part.push_back(make_int2(i, j));
    b->flat_blocks_d = (int)b->host_part.size() - b->flat_blocks_g;
    xcd_deal(b->host_part.data(), 0, b->flat_blocks_g);
    xcd_deal(b->host_part.data(), b->flat_blocks_g, b->flat_blocks_d);
    for (int i = 0; i < n; ++i) {
        b->host_ncell[i] = L[i].ncell;
        ncell_total += size_t(L[i].ncell);
    }
    b->host_cells.assign(ncell_total, make_int2(0, 0));
    int2 *part = head.take<int2>(b->host_part.size());
    b->dev_cells = head.take<int2>(ncell_total);
    b->flat.n_inst = n;
    b->flat.blocks_g = b->flat_blocks_g;
    b->flat.part = part;
    b->flat.cells = b->dev_cells;
    if (!b->host_part.empty())
        HIP_TRY(hipMemcpyAsync(part, b->host_part.data(), sizeof(int2) * b->host_part.size(), hipMemcpyHostToDevice, st));
    tfsph_status rc = upload_flat_cells(b, st);
    if (rc != TFSPH_OK) return rc;
    // largest-first order (work ~ particles); ties by index
    b->host_order.resize(L.size());
    std::iota(b->host_order.begin(), b->host_order.end(), 0);
    std::stable_sort(b->host_order.begin(), b->host_order.end(), [&L](int x, int y) {
        return (long long)L[x].ng + L[x].nd > (long long)L[y].ng + L[y].nd;
    });
    // the force-loop kind each instance runs (the rule of force_kind()): one shared kind lets
    // the flattened force launch be specialised on it
    int kind = -2;
    for (const Inst<R> &I : table) {
        const int k = (I.Ph.av || I.Ph.eos != 0) ? kForceGeneral : (I.Sg.has_mass ? kForceIsoMass : kForceIsoUniform);
        kind = (kind == -2 || kind == k) ? k : -1;
    }
    b->flat_kind = kind < 0 ? -1 : kind;
    b->host_table.resize(sizeof(Inst<R>) * table.size());
    std::copy(reinterpret_cast<const char *>(table.data()), reinterpret_cast<const char *>(table.data()) + b->host_table.size(),
              b->host_table.begin());
    HIP_TRY(hipMemcpyAsync(b->table, b->host_table.data(), b->host_table.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(b->order, b->host_order.data(), sizeof(int) * L.size(), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemsetAsync(b->F.word, 0, 256, st));
    HIP_TRY(hipMemsetAsync(b->F.one_phase, 0, 64, st));
    HIP_TRY(hipStreamSynchronize(st));
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_batch_init(tfsph_batch **out, const tfsph_batch_desc *desc, tfsph_state *packed,
                                         const tfsph_batch_tuning *tuning, void *workspace, size_t ws_bytes,
                                         void *hip_stream)
{
    if (!out) return fail(TFSPH_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    std::vector<InstLayout> L;
    int dim, prec;
    tfsph_status r = check_desc(desc, L, dim, prec);
    if (r != TFSPH_OK) return r;
    if (!packed) return fail(TFSPH_E_INVALID_ARG, "packed state is NULL");
    if (packed->gas.n != desc->gas_offset[desc->n_inst] || packed->dust.n != desc->dust_offset[desc->n_inst])
        return fail(TFSPH_E_STATE, "packed state sizes differ from the offsets");
    // per-instance uniform masses come from the descriptor (checked below)
    tfsph_phase gchk = packed->gas, dchk = packed->dust;
    gchk.mass_uniform = dchk.mass_uniform = 1.0;
    r = check_phase(gchk, dim, true, false, "gas");
    if (r != TFSPH_OK) return r;
    r = check_phase(dchk, dim, false, false, "dust");
    if (r != TFSPH_OK) return r;
    for (int i = 0; i < desc->n_inst; ++i) {
        if (!packed->gas.mass && !(desc->mass_gas && desc->mass_gas[i] > 0.0))
            return fail(TFSPH_E_INVALID_ARG, "instance %d: no gas mass", i);
        if (!packed->dust.mass && !(desc->mass_dust && desc->mass_dust[i] > 0.0))
            return fail(TFSPH_E_INVALID_ARG, "instance %d: no dust mass", i);
        L[i].mass_g = packed->gas.mass != nullptr;
        L[i].mass_d = packed->dust.mass != nullptr;
    }
    size_t need = 0;
    r = tfsph_batch_workspace_size(desc, &need);
    if (r != TFSPH_OK) return r;
    if (!workspace || reinterpret_cast<uintptr_t>(workspace) % 256)
        return fail(TFSPH_E_WORKSPACE, "workspace must be non-NULL and 256-byte aligned");
    if (ws_bytes < need) return fail(TFSPH_E_WORKSPACE, "workspace has %zu bytes, needs %zu", ws_bytes, need);
    tfsph_batch *b = new (std::nothrow) tfsph_batch();
    if (!b) return fail(TFSPH_E_INVALID_ARG, "out of host memory");
    b->n_inst = desc->n_inst;
    b->dim = dim;
    b->prec = prec;
    b->bound = *packed;
    b->ws = static_cast<char *>(workspace);
    b->ws_bytes = ws_bytes;
    b->last_stream = static_cast<hipStream_t>(hip_stream);
    r = set_tuning(b, tuning);
    if (r == TFSPH_OK)
        r = prec == TFSPH_F64 ? batch_setup<double>(b, desc, L, packed, b->last_stream)
                              : batch_setup<float>(b, desc, L, packed, b->last_stream);
    if (r != TFSPH_OK) {
        delete b;
        return r;
    }
    *out = b;
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_batch_set_tuning(tfsph_batch *b, const tfsph_batch_tuning *tuning)
{
    if (!b) return fail(TFSPH_E_INVALID_ARG, "batch is NULL");
    return set_tuning(b, tuning);
}

static bool same_state(const tfsph_state &a, const tfsph_state &b)
{
    for (auto pr : {std::make_pair(&a.gas, &b.gas), std::make_pair(&a.dust, &b.dust)}) {
        const tfsph_phase &x = *pr.first, &y = *pr.second;
        if (x.n != y.n || x.cell != y.cell || x.id != y.id || x.mass != y.mass || x.rho != y.rho) return false;
        for (int d = 0; d < 3; ++d)
            if (x.off[d] != y.off[d] || x.vel[d] != y.vel[d]) return false;
    }
    return true;
}

// The flattened form: every phase of a step is one launch over all instances.  The
// first step counts from the caller's arrays; later steps use the slots claimed by
// the previous step's finish kernel.
template <typename R, int DIM>
static tfsph_status launch_flat_t(tfsph_batch *b, int n_steps, hipStream_t st)
{
    auto *t = static_cast<const Inst<R> *>(b->table);
    const FlatTable T = b->flat;
    const dim3 blk(kBlock);
    const dim3 gd(b->flat_blocks_g + b->flat_blocks_d), gg(b->flat_blocks_g), gc(b->flat_blocks_c);
    if (gc.x) hipLaunchKernelGGL((k_flat_zero<R>), gc, blk, 0, st, t, T);
    if (gd.x) hipLaunchKernelGGL((k_flat_count<R>), gd, blk, 0, st, t, T);
    LAUNCH_CHECK("flat_count");
    const size_t lds = update_lds_bytes<R>(T.cells_per_block);
    for (int s = 0; s < n_steps; ++s) {
        hipLaunchKernelGGL((k_flat_scan<R>), dim3(2 * b->n_inst), dim3(kBatchMaxBlock), 0, st, t);
        if (gd.x) {
            hipLaunchKernelGGL((k_flat_scatter<R>), gd, blk, 0, st, t, T);
            hipLaunchKernelGGL((k_flat_rank_gather<R>), gd, blk, 0, st, t, T, b->F.word);
        }
        if (gg.x) {
            hipLaunchKernelGGL((k_flat_density<R, DIM>), gg, blk, 0, st, t, T);
            switch (b->flat_kind) {
            case kForceIsoUniform:
                hipLaunchKernelGGL((k_flat_predict<R, DIM, kForceIsoUniform>), gg, blk, 0, st, t, T);
                break;
            case kForceIsoMass: hipLaunchKernelGGL((k_flat_predict<R, DIM, kForceIsoMass>), gg, blk, 0, st, t, T); break;
            case kForceGeneral: hipLaunchKernelGGL((k_flat_predict<R, DIM, kForceGeneral>), gg, blk, 0, st, t, T); break;
            default: hipLaunchKernelGGL((k_flat_predict<R, DIM, -1>), gg, blk, 0, st, t, T); break;
            }
        }
        if (gc.x) hipLaunchKernelGGL((k_flat_update<R, DIM>), gc, blk, lds, st, t, T, b->F);
        LAUNCH_CHECK("flat_step");
    }
    return TFSPH_OK;
}

static tfsph_status launch_flat(tfsph_batch *b, int n_steps, hipStream_t st)
{
    if (n_steps == 0) return TFSPH_OK;
    if (b->prec == TFSPH_F64)
        return b->dim == 1 ? launch_flat_t<double, 1>(b, n_steps, st) : launch_flat_t<double, 2>(b, n_steps, st);
    return b->dim == 1 ? launch_flat_t<float, 1>(b, n_steps, st) : launch_flat_t<float, 2>(b, n_steps, st);
}

static tfsph_status launch_batched(tfsph_batch *b, int n_steps, hipStream_t st)
{
    if (n_steps == 0) return TFSPH_OK;
    if (b->form == TFSPH_BATCH_FLAT) return launch_flat(b, n_steps, st);
    const dim3 grid(b->n_inst), block(b->block);
    if (b->prec == TFSPH_F64) {
        auto *t = static_cast<const Inst<double> *>(b->table);
        if (b->dim == 1) hipLaunchKernelGGL((k_batched<double, 1>), grid, block, 0, st, t, b->order, n_steps, b->F);
        else hipLaunchKernelGGL((k_batched<double, 2>), grid, block, 0, st, t, b->order, n_steps, b->F);
    } else {
        auto *t = static_cast<const Inst<float> *>(b->table);
        if (b->dim == 1) hipLaunchKernelGGL((k_batched<float, 1>), grid, block, 0, st, t, b->order, n_steps, b->F);
        else hipLaunchKernelGGL((k_batched<float, 2>), grid, block, 0, st, t, b->order, n_steps, b->F);
    }
    LAUNCH_CHECK("batched");
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_step_batched(tfsph_batch *b, tfsph_state *packed, int32_t n_steps, void *hip_stream)
{
    if (!b) return fail(TFSPH_E_INVALID_ARG, "batch is NULL");
    if (n_steps < 0) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 0");
    if (!packed || !same_state(*packed, b->bound)) return fail(TFSPH_E_STATE, "packed state differs from the one bound at init");
    b->last_stream = static_cast<hipStream_t>(hip_stream);
    return launch_batched(b, n_steps, b->last_stream);
}

extern "C" tfsph_status tfsph_step_batched_graph(tfsph_batch *b, tfsph_state *packed, int32_t n_steps, void *hip_stream)
{
    if (!b) return fail(TFSPH_E_INVALID_ARG, "batch is NULL");
    if (n_steps < 0) return fail(TFSPH_E_INVALID_ARG, "n_steps must be >= 0");
    if (!packed || !same_state(*packed, b->bound)) return fail(TFSPH_E_STATE, "packed state differs from the one bound at init");
    hipStream_t st = static_cast<hipStream_t>(hip_stream);
    b->last_stream = st;
    if (n_steps == 0) return TFSPH_OK;
    auto key = std::make_tuple((int)n_steps, b->form, b->form == TFSPH_BATCH_FLAT ? 0 : b->block);
    auto it = b->graphs.find(key);
    if (it == b->graphs.end()) {
        if (!b->capture_stream) HIP_TRY(hipStreamCreateWithFlags(&b->capture_stream, hipStreamNonBlocking));
        HIP_TRY(hipStreamBeginCapture(b->capture_stream, hipStreamCaptureModeThreadLocal));
        tfsph_status r = launch_batched(b, n_steps, b->capture_stream);
        hipGraph_t g = nullptr;
        hipError_t e = hipStreamEndCapture(b->capture_stream, &g);
        if (r != TFSPH_OK) {
            if (g) (void)hipGraphDestroy(g);
            return r;
        }
        if (e != hipSuccess) return fail(TFSPH_E_HIP, "hipStreamEndCapture: %s", hipGetErrorString(e));
        tfsph_batch::G gg;
        gg.graph = g;
        HIP_TRY(hipGraphInstantiate(&gg.exec, g, nullptr, nullptr, 0));
        it = b->graphs.emplace(key, gg).first;
    }
    HIP_TRY(hipGraphLaunch(it->second.exec, st));
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_batch_get_flags(tfsph_batch *b, uint32_t *flags, int64_t *one_phase_cells)
{
    if (!b) return fail(TFSPH_E_INVALID_ARG, "batch is NULL");
    unsigned int w = 0;
    unsigned long long n = 0;
    HIP_TRY(hipStreamSynchronize(b->last_stream));
    HIP_TRY(hipMemcpy(&w, b->F.word, sizeof(w), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(&n, b->F.one_phase, sizeof(n), hipMemcpyDeviceToHost));
    HIP_TRY(hipMemset(b->F.word, 0, sizeof(w)));
    HIP_TRY(hipMemset(b->F.one_phase, 0, sizeof(n)));
    if (flags) *flags = w;
    if (one_phase_cells) *one_phase_cells = (int64_t)n;
    return TFSPH_OK;
}

extern "C" tfsph_status tfsph_batch_destroy(tfsph_batch *b)
{
    if (b) {
        for (auto &kv : b->graphs) {
            if (kv.second.exec) (void)hipGraphExecDestroy(kv.second.exec);
            if (kv.second.graph) (void)hipGraphDestroy(kv.second.graph);
        }
        if (b->capture_stream) (void)hipStreamDestroy(b->capture_stream);
    }
    delete b;
    return TFSPH_OK;
}
