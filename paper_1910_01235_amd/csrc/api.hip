// C ABI implementation: plans, workspace layout, launch sequences, graphs.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "mxe_internal.h"
#include "node_poly.h"

using namespace mxe;

namespace {

thread_local std::string g_err;

mxe_status fail(mxe_status s, const std::string& msg) {
    g_err = msg;
    return s;
}

#define HIP_OK(call)                                                                   \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return fail(MXE_EDEVICE, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

}  // namespace

struct mxe_plan {
    mxe_params p;
    mxe_eam e;
    Model model;
    int n_sys = 0;
    std::vector<mxe_system> systems;        // current system of each slot
    std::vector<int64_t> cap_sites, cap_cells;  // slot capacities
    double r_cap = 0.0, r_cell = 0.0;
    std::vector<char> dirty;     // slot rebound since the last call
    std::vector<int> steps_new;  // mxe_advance budgets to apply at the next call (-1: keep)
    bool resume = false;         // calls rebuild only dirty slots
    bool tables_dirty = true;    // chunk tables changed since the last upload
    void* tables_ws = nullptr;   // workspace that holds the uploaded tables
    void* lists_ws = nullptr;    // workspace whose neighbour lists this plan built
    std::vector<SysDesc> sys;
    std::vector<Chunk> chunks, pchunks;
    // cells in use: entry 0 holds their count, entries 1.. (system, global cell);
    // the count lives in device memory so that a captured graph stays valid
    // when slots are rebound
    std::vector<int2> acells;
    int64_t n_sites = 0, n_cells = 0, pair_cap_total = 0;
    // workspace layout (byte offsets)
    size_t o_sys, o_ctl, o_chunks, o_pchunks, o_site_sys, o_cell_count, o_cell_start, o_cell_sites, o_cell_rec;
    size_t o_cell_of, o_slot_of, o_chunk_up, o_acell;
    size_t o_nbr, o_cnt, o_lo, o_pid, o_hoff, o_pi, o_pj, o_pnew, o_fblk, o_dblk, o_G, o_A, o_B;
    size_t o_v, o_qr, o_sref, o_emit, o_srec, o_bond, o_nbond, o_part, o_part_sub;
    size_t ws_bytes = 0;
    // chunk tables hold the occupied slots' chunks first; launches cover that
    // prefix (rounded up to a power of two)
    int64_t live_chunks = 0, live_pchunks = 0;
    int live_sys = 0;  // occupied slots
    // graph cache for mxe_run, per buffers and launch extents: one diffusion
    // step, or (relax_chunk > 0) a chunk of lean relaxation iterations, one
    // iteration with the build chain and the Euler step; mxe_advance's chunk
    // of lean free-running iterations and its iteration with the chain
    struct Graphs {
        hipGraphExec_t step = nullptr, chunk = nullptr, full = nullptr, master = nullptr, advance = nullptr,
                       advance_full = nullptr;
        bool chunk_lean = false, advance_lean = false;  // recorded lean (see lean_chunks)
        std::vector<hipGraphExec_t> all() const { return {step, chunk, full, master, advance, advance_full}; }
    };
    hipStream_t cap_stream = nullptr;
    std::map<std::vector<const void*>, Graphs> graphs;
    // chunked relaxations: systems still relaxing and systems stalled for a
    // build after a chunk, two slots of two ints of pinned host memory written
    // by the device, and their events
    int* act_host = nullptr;
    int* act_dev = nullptr;
    hipEvent_t act_ev[2] = {nullptr, nullptr};
    // profiling: event pairs bracketing launches, per kernel family
    bool prof_on = false;
    bool prof_pair_only = false;  // MXE_PROFILE_PAIR: only the pair kernel is bracketed
    struct ProfMark {
        int family;
        size_t start, end;  // indices into prof_events
    };
    std::vector<hipEvent_t> prof_events;  // pool, reused after each read
    size_t prof_next = 0;                 // next unused event of the pool
    long prof_last = -1;                  // end event a chained family may start from, or -1
    std::vector<ProfMark> prof_marks;
    hipError_t prof_err = hipSuccess;
};

namespace {

// Cell grid of a system (validates box and temperature); cells must be at
// least as wide as the largest list radius the plan allows.
mxe_status slot_cells(const mxe_plan* P, const mxe_system& ms, int s, int64_t* ncell) {
    if (!(ms.T > 0)) return fail(MXE_EINVAL, "system " + std::to_string(s) + ": T must be positive");
    int64_t n = 1;
    for (int a = 0; a < 3; ++a) {
        if (!(ms.box[a] > 0))
            return fail(MXE_EINVAL, "system " + std::to_string(s) + ": box lengths must be positive");
        if (ms.periodic[a] && !(ms.box[a] > 2.0 * P->r_cap))
            return fail(MXE_EINVAL, "system " + std::to_string(s) +
                                        ": periodic box length must exceed twice the list radius " +
                                        std::to_string(P->r_cap));
        n *= std::max(1, std::min((int)std::floor(ms.box[a] / P->r_cell), 1024));
    }
    *ncell = n;
    return MXE_OK;
}

// Chunk tables: the chunks of occupied slots first (in slot order), then those
// of empty slots, so that launches can cover the occupied prefix alone. A
// system's chunks stay contiguous and in site order from its chunk_first; no
// result depends on which block or table position takes a chunk.
void order_tables(mxe_plan* P) {
    P->chunks.clear();
    P->pchunks.clear();
    P->live_chunks = P->live_pchunks = 0;
    P->live_sys = 0;
    for (int pass = 0; pass < 2; ++pass)
        for (int s = 0; s < P->n_sys; ++s) {
            SysDesc& d = P->sys[s];
            if ((d.n_sites > 0) != (pass == 0)) continue;
            d.chunk_first = (int)P->chunks.size();
            for (int c = 0; c < d.n_chunks; ++c) {
                const int64_t a = (int64_t)c * kChunk;
                P->chunks.push_back(Chunk{s, (int)(d.site_off + std::min<int64_t>(a, d.n_sites)),
                                          (int)(d.site_off + std::min<int64_t>(a + kChunk, d.n_sites)), 0});
            }
            for (int64_t a = 0; a < d.pair_cap; a += kPairChunk)
                P->pchunks.push_back(Chunk{s, (int)(d.pair_base + a),
                                           (int)(d.pair_base + std::min<int64_t>(d.pair_cap, a + kPairChunk)), 0});
            if (pass == 0) {
                P->live_sys += 1;
                P->live_chunks = (int64_t)P->chunks.size();
                P->live_pchunks = (int64_t)P->pchunks.size();
            }
        }
}

// Launch extent over a table whose first `live` entries are in use: the whole
// table when all are, else `live` rounded up to a power of two (at least 64),
// so that few distinct extents, and recorded graphs, occur.
int launch_extent(int64_t live, int64_t total) {
    if (live >= total) return (int)total;
    int64_t e = 64;
    while (e < live) e <<= 1;
    return (int)std::min(e, total);
}

// Points slot s at system ms (n_sites <= capacity; 0 leaves the slot empty).
// Offsets and capacities stay fixed; the chunk tables are reordered (order:
// false defers that to the caller).
void bind_slot(mxe_plan* P, int s, const mxe_system& ms, bool order = true) {
    SysDesc& d = P->sys[s];
    d.n_sites = ms.n_sites;
    int64_t ncell = 1;
    for (int a = 0; a < 3; ++a) {
        d.box[a] = ms.box[a];
        d.periodic[a] = ms.periodic[a] ? 1 : 0;
        const int nc = std::max(1, std::min((int)std::floor(ms.box[a] / P->r_cell), 1024));
        d.nc[a] = nc;
        d.cell_w[a] = ms.box[a] / nc;
        ncell *= nc;
    }
    d.n_cells = ms.n_sites > 0 ? ncell : 0;
    d.T = ms.T;
    d.kT = kBoltzmannEv * ms.T;
    d.beta = 1.0 / d.kT;
    d.D = P->p.nu0 * std::exp(-d.beta * P->p.Qm);
    P->systems[s] = ms;
    P->dirty[s] = 1;
    P->tables_dirty = true;
    // cells in use, slot by slot (the neighbour search runs one block per entry)
    P->acells.assign(1, make_int2(0, 0));
    for (int t = 0; t < (int)P->sys.size(); ++t)
        for (int64_t c = 0; c < P->sys[t].n_cells; ++c)
            P->acells.push_back(make_int2(t, (int)(P->sys[t].cell_off + c)));
    P->acells[0].x = (int)P->acells.size() - 1;
    if (order) order_tables(P);
}

}  // namespace

extern "C" mxe_status mxe_plan_check_system(const mxe_plan* P, int slot, const mxe_system* sys);

extern "C" mxe_status mxe_plan_set_system(mxe_plan* P, int slot, const mxe_system* sys) {
    if (!P || !sys) return fail(MXE_EINVAL, "null argument");
    if (slot < 0 || slot >= P->n_sys) return fail(MXE_EINVAL, "slot out of range");
    const mxe_status r = mxe_plan_check_system(P, slot, sys);
    if (r != MXE_OK) return r;
    bind_slot(P, slot, *sys);
    return MXE_OK;
}

extern "C" mxe_status mxe_plan_check_system(const mxe_plan* P, int slot, const mxe_system* sys) {
    if (!P || !sys) return fail(MXE_EINVAL, "null argument");
    if (slot < 0 || slot >= P->n_sys) return fail(MXE_EINVAL, "slot out of range");
    if (sys->n_sites < 0 || sys->n_sites > P->cap_sites[slot])
        return fail(MXE_ERANGE, "slot " + std::to_string(slot) + " holds at most " +
                                    std::to_string(P->cap_sites[slot]) + " sites");
    if (sys->n_sites == 0) return MXE_OK;
    int64_t ncell = 0;
    mxe_status r = slot_cells(P, *sys, slot, &ncell);
    if (r != MXE_OK) return r;
    if (ncell > P->cap_cells[slot])
        return fail(MXE_ERANGE, "slot " + std::to_string(slot) + ": box needs " + std::to_string(ncell) +
                                    " cells, capacity " + std::to_string(P->cap_cells[slot]));
    return MXE_OK;
}

extern "C" mxe_status mxe_plan_layout(const mxe_plan* P, int item, size_t* offset, size_t* bytes) {
    if (!P || !offset || !bytes) return fail(MXE_EINVAL, "null argument");
    const size_t N = (size_t)P->n_sites;
    switch (item) {
        case MXE_L_NBR: *offset = P->o_nbr; *bytes = sizeof(int) * N * P->p.k_max; break;
        case MXE_L_NBR_COUNT: *offset = P->o_cnt; *bytes = sizeof(int) * N; break;
        case MXE_L_BOND: *offset = P->o_bond; *bytes = sizeof(int) * N * P->p.bond_max; break;
        case MXE_L_BOND_COUNT: *offset = P->o_nbond; *bytes = sizeof(int) * N; break;
        default: return fail(MXE_EINVAL, "unknown layout item");
    }
    return MXE_OK;
}

extern "C" mxe_status mxe_plan_set_resume(mxe_plan* P, int on) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    P->resume = on != 0;
    return MXE_OK;
}

extern "C" int64_t mxe_plan_slot_offset(const mxe_plan* P, int slot) {
    if (!P || slot < 0 || slot > P->n_sys) return -1;
    return slot == P->n_sys ? P->n_sites : P->sys[slot].site_off;
}

extern "C" void mxe_default_params(mxe_params* p) {
    std::memset(p, 0, sizeof(*p));
    p->nu0 = 1.0e13;
    p->Qm = 0.69;
    p->kin_c = 1.0;
    p->dt_safety = 0.5;
    p->max_relax = 50;
    p->ftol = 1.0e-3;
    p->fire_dt0 = 0.05;
    p->fire_dtmax = 0.15;
    p->fire_alpha0 = 0.1;
    p->fire_finc = 1.1;
    p->fire_fdec = 0.5;
    p->fire_falpha = 0.99;
    p->fire_nmin = 5;
    p->sigma_min = 0.01;
    p->sigma_cap = 0.3;
    p->skin = 0.15;
    p->r_bond = 3.09;
    p->k_max = 96;
    p->bond_max = 16;
    p->precision = MXE_FP64;
}

extern "C" mxe_status mxe_plan_create(const mxe_params* params, const mxe_eam* eam, int n_systems,
                                      const mxe_system* systems, mxe_plan** out) {
    if (!out) return fail(MXE_EINVAL, "out is NULL");
    *out = nullptr;
    if (!params || !eam || !systems || n_systems < 1) return fail(MXE_EINVAL, "null argument or n_systems < 1");
    const mxe_params& p = *params;
    if (p.precision != MXE_FP64 && p.precision != MXE_FP32_MIXED) return fail(MXE_EINVAL, "bad precision");
    if (p.k_max < 1 || p.k_max > 256 || p.bond_max < 1 || p.bond_max > 64 || p.max_relax < 0)
        return fail(MXE_EINVAL, "k_max must lie in [1, 256], bond_max in [1, 64], max_relax >= 0");
    if (p.gather_lanes != 0 && p.gather_lanes != 8 && p.gather_lanes != 16 && p.gather_lanes != 32 &&
        p.gather_lanes != 64)
        return fail(MXE_EINVAL, "gather_lanes must be 0, 8, 16, 32 or 64");
    if (p.force_lanes != 0 && p.force_lanes != 8 && p.force_lanes != 16 && p.force_lanes != 32 &&
        p.force_lanes != 64)
        return fail(MXE_EINVAL, "force_lanes must be 0, 8, 16, 32 or 64");
    if (p.gather_stride < 0 || p.gather_stride > 4096)
        return fail(MXE_EINVAL, "gather_stride must lie in [0, 4096]");
    if (p.relax_chunk < 0 || p.relax_chunk > 1024) return fail(MXE_EINVAL, "relax_chunk must lie in [0, 1024]");
    if (p.pair_split != 0 && p.pair_split != 1 && p.pair_split != 2 && p.pair_split != 4 && p.pair_split != 8 &&
        p.pair_split != 16)
        return fail(MXE_EINVAL, "pair_split must be 0, 1, 2, 4, 8 or 16");
    if (p.pair_block != 0 && p.pair_block != 64 && p.pair_block != 128 && p.pair_block != 256)
        return fail(MXE_EINVAL, "pair_block must be 0, 64, 128 or 256");
    if (p.quad_rule != MXE_QUAD_GH27 && p.quad_rule != MXE_QUAD_DEGREE3)
        return fail(MXE_EINVAL, "quad_rule must be MXE_QUAD_GH27 (0) or MXE_QUAD_DEGREE3 (1)");
    if (!(p.sigma_min > 0) || !(p.sigma_cap > p.sigma_min) || !(p.skin > 0) || !(p.dt_safety > 0) ||
        !(p.r_bond > 0) || !(p.ftol >= 0) || !(p.fire_dt0 > 0) || !(p.fire_dtmax > 0))
        return fail(MXE_EINVAL, "bad sigma_min / sigma_cap / skin / dt_safety / r_bond / ftol / FIRE steps");
    if (!(eam->r_c > eam->r_s) || !(eam->r_s > 0)) return fail(MXE_EINVAL, "need 0 < r_s < r_c");
    for (int c = 0; c < 2; ++c)
        if (!(eam->r_e[c] > 0)) return fail(MXE_EINVAL, "r_e must be positive");
    for (int k = 0; k < 3; ++k)
        for (int l = 0; l < 3; ++l)
            if (eam->pair_a[k][l] != eam->pair_a[l][k]) return fail(MXE_EINVAL, "pair_a must be symmetric");

    mxe_plan* P = new mxe_plan();
    P->p = p;
    P->e = *eam;
    P->n_sys = n_systems;
    P->systems.assign(systems, systems + n_systems);

    Model& m = P->model;
    std::memset(&m, 0, sizeof(m));
    for (int k = 0; k < 3; ++k) {
        m.c4[k] = eam->embed_c[k];
        m.b4[k] = eam->emit_b[k];
        for (int l = 0; l < 3; ++l) m.a4[k][l] = eam->pair_a[k][l];
    }
    for (int c = 0; c < 2; ++c) {
        m.r_e[c] = eam->r_e[c];
        m.inv_re[c] = 1.0 / eam->r_e[c];
        m.alpha[c] = eam->alpha[c];
        m.gamma[c] = eam->gamma[c];
    }
    m.r_s = eam->r_s;
    m.r_c = eam->r_c;
    m.taper_inv_w = 1.0 / (eam->r_c - eam->r_s);
    m.ftol = p.ftol;
    m.dt0 = p.fire_dt0;
    m.dtmax = p.fire_dtmax;
    m.alpha0 = p.fire_alpha0;
    m.finc = p.fire_finc;
    m.fdec = p.fire_fdec;
    m.falpha = p.fire_falpha;
    m.nmin = p.fire_nmin;
    m.max_relax = p.max_relax;
    m.sigma_min = p.sigma_min;
    m.sigma_cap = p.sigma_cap;
    m.skin = p.skin;
    m.r_bond = p.r_bond;
    m.kin_c = p.kin_c;
    m.dt_safety = p.dt_safety;
    m.nu0 = p.nu0;
    m.Qm = p.Qm;
    m.gather_lanes = p.gather_lanes ? p.gather_lanes : 8;
    m.force_lanes = p.force_lanes ? p.force_lanes : 16;
    m.gather_stride = p.gather_stride ? p.gather_stride : 1;
    m.pair_block = p.pair_block ? p.pair_block : 256;
    m.pair_shift = 0;
    while ((1 << m.pair_shift) < (p.pair_split ? p.pair_split : 2)) ++m.pair_shift;
    // exponent ratios alpha : gamma = P : Q per pair class, in lowest terms
    for (int c = 0; c < 2; ++c) {
        m.ratio_pq[c] = 0;
        const double al = eam->alpha[c], ga = eam->gamma[c];
        for (int q = 1; q <= 15 && !m.ratio_pq[c]; ++q)
            for (int pp = 1; pp <= 15 && !m.ratio_pq[c]; ++pp)
                if (std::fabs(al * q - ga * pp) <= 1e-12 * std::fmax(std::fabs(al), std::fabs(ga)) && al > 0 &&
                    ga > 0)
                    m.ratio_pq[c] = pp * 16 + q;
        m.u_rate[c] = m.ratio_pq[c] ? m.alpha[c] / (double)(m.ratio_pq[c] >> 4) : 0.0;
    }
    m.quad_rule = p.quad_rule;
    // near-minimax remainder polynomials of node_poly.h
    static_assert(sizeof(kExpE) == sizeof(m.poly.ex) && sizeof(kTaperS) == sizeof(m.poly.sn) &&
                      sizeof(kTaperC) == sizeof(m.poly.cs),
                  "node polynomial degrees");
    {  // the exponential's remainder in base 2 (argument f = r / ln2)
        constexpr long double kLn2 = 0.693147180559945309417232121458176568L;
        for (int k = 0; k < PolyCoef::kExp; ++k) {
            const int deg = PolyCoef::kExp - 1 - k;  // highest degree first
            long double sc = kLn2 * kLn2 * kLn2;
            for (int e = 0; e < deg; ++e) sc *= kLn2;
            m.poly.ex[k] = (double)((long double)kExpE[k] * sc);
        }
        m.poly.ln2 = (double)kLn2;
        m.poly.ln2sq_half = (double)(kLn2 * kLn2 / 2);
    }
    std::memcpy(m.poly.sn, kTaperS, sizeof(kTaperS));
    std::memcpy(m.poly.cs, kTaperC, sizeof(kTaperC));

    // largest list radius the cells must cover
    P->r_cap = eam->r_c + 3.0 * std::sqrt(2.0) * p.sigma_cap + p.skin;
    P->r_cell = std::max(P->r_cap, p.r_bond);
    int64_t site_off = 0, cell_off = 0, pair_base = 0;
    P->sys.resize(n_systems);
    P->dirty.assign(n_systems, 1);
    P->steps_new.assign(n_systems, 0);
    P->cap_sites.resize(n_systems);
    P->cap_cells.resize(n_systems);
    for (int s = 0; s < n_systems; ++s) {
        const mxe_system& ms = systems[s];
        if (ms.n_sites < 1) {
            delete P;
            return fail(MXE_EINVAL, "system " + std::to_string(s) + ": n_sites < 1");
        }
        int64_t ncell = 0;
        mxe_status r = slot_cells(P, ms, s, &ncell);
        if (r != MXE_OK) {
            delete P;
            return r;
        }
        // capacities: the given system, and room for the cells of any dense
        // system of up to n_sites sites (a slot can be rebound later)
        P->cap_sites[s] = ms.n_sites;
        P->cap_cells[s] = std::max<int64_t>(ncell, ms.n_sites / 8 + 64);
        SysDesc& d = P->sys[s];
        std::memset(&d, 0, sizeof(d));
        d.site_off = site_off;
        d.cell_off = cell_off;
        d.pair_base = pair_base;
        d.pair_cap = (ms.n_sites * (int64_t)p.k_max + 1) / 2;
        d.chunk_first = (int)P->chunks.size();
        for (int64_t a = 0; a < ms.n_sites; a += kChunk) P->chunks.push_back(Chunk{s, 0, 0, 0});
        d.n_chunks = (int)P->chunks.size() - d.chunk_first;
        for (int64_t a = 0; a < d.pair_cap; a += kPairChunk) {
            Chunk c{s, (int)(pair_base + a), (int)(pair_base + std::min<int64_t>(d.pair_cap, a + kPairChunk)), 0};
            P->pchunks.push_back(c);
        }
        site_off += ms.n_sites;
        cell_off += P->cap_cells[s];
        pair_base += d.pair_cap;
    }
    P->n_sites = site_off;
    P->n_cells = cell_off;
    P->pair_cap_total = pair_base;
    if (site_off * (int64_t)p.k_max >= (int64_t)INT32_MAX || pair_base >= (int64_t)INT32_MAX ||
        site_off * 4 >= (int64_t)INT32_MAX || cell_off >= (int64_t)INT32_MAX) {
        delete P;
        return fail(MXE_ERANGE, "plan too large for 32-bit indices");
    }
    for (int s = 0; s < n_systems; ++s) bind_slot(P, s, systems[s], false);
    order_tables(P);
    for (int s = 0; s < n_systems; ++s) m.fold_rows |= P->sys[s].n_chunks > kChunk;

    // workspace layout
    const size_t A = 256;
    const int64_t N = P->n_sites;
    const size_t mom_elt = p.precision == MXE_FP32_MIXED ? sizeof(float) : sizeof(double);
    size_t o = 0;
    auto take = [&](size_t bytes) {
        const size_t r = o;
        o = align_up(o + bytes, A);
        return r;
    };
    P->o_sys = take(sizeof(SysDesc) * n_systems);
    P->o_ctl = take(sizeof(SysCtl) * n_systems);
    P->o_chunks = take(sizeof(Chunk) * P->chunks.size());
    P->o_pchunks = take(sizeof(Chunk) * P->pchunks.size());
    P->o_site_sys = take(sizeof(int) * N);
    P->o_cell_count = take(sizeof(int) * P->n_cells);
    P->o_cell_start = take(sizeof(int) * P->n_cells);
    P->o_cell_sites = take(sizeof(int) * N);
    P->o_cell_rec = take(sizeof(double) * 4 * N);
    P->o_cell_of = take(sizeof(int) * N);
    P->o_slot_of = take(sizeof(int) * N);
    P->o_chunk_up = take(sizeof(int) * P->chunks.size());
    P->o_acell = take(sizeof(int2) * (P->n_cells + 1));
    P->o_nbr = take(sizeof(int) * N * p.k_max);
    P->o_cnt = take(sizeof(int) * N);
    P->o_lo = take(sizeof(int) * N);
    P->o_pid = take(sizeof(int) * N * p.k_max);
    P->o_hoff = take(sizeof(int) * N);
    P->o_pi = take(sizeof(int) * P->pair_cap_total);
    P->o_pnew = take(sizeof(int) * P->pair_cap_total);
    P->o_pj = take(sizeof(int) * P->pair_cap_total);
    P->o_fblk = take(mom_elt * kFBlk * P->pair_cap_total);
    P->o_dblk = take(mom_elt * 2 * P->pair_cap_total);
    P->o_G = take(sizeof(double) * N);
    P->o_A = take(sizeof(double) * N);
    P->o_B = take(sizeof(double) * N);
    P->o_v = take(sizeof(double) * 4 * N);
    P->o_qr = take(sizeof(double) * 3 * N);
    P->o_sref = take(sizeof(double) * N);
    P->o_emit = take(sizeof(double) * N);
    P->o_srec = take(mom_elt * kSRec * N);  // stored in the moments' precision
    P->o_bond = take(sizeof(int) * N * p.bond_max);
    P->o_nbond = take(sizeof(int) * N);
    P->o_part = take(sizeof(double) * kNPart * P->chunks.size());
    P->o_part_sub = take(sizeof(double) * kNPart * kForceSplit * P->chunks.size());
    P->ws_bytes = o;
    *out = P;
    return MXE_OK;
}

extern "C" void mxe_plan_destroy(mxe_plan* plan) {
    if (!plan) return;
    for (hipEvent_t e : plan->prof_events) (void)hipEventDestroy(e);
    for (hipEvent_t e : plan->act_ev)
        if (e) (void)hipEventDestroy(e);
    if (plan->act_host) (void)hipHostFree(plan->act_host);
    for (auto& kv : plan->graphs)
        for (hipGraphExec_t g : kv.second.all())
            if (g) (void)hipGraphExecDestroy(g);
    if (plan->cap_stream) (void)hipStreamDestroy(plan->cap_stream);
    delete plan;
}

extern "C" mxe_status mxe_workspace_bytes(const mxe_plan* plan, size_t* bytes) {
    if (!plan || !bytes) return fail(MXE_EINVAL, "null argument");
    *bytes = plan->ws_bytes;
    return MXE_OK;
}

extern "C" int64_t mxe_plan_sites(const mxe_plan* plan) { return plan ? plan->n_sites : 0; }

namespace {

mxe_status make_dev(const mxe_plan* P, const mxe_state* st, const mxe_out* out, void* ws,
                    size_t ws_bytes, Dev* d) {
    if (!st || !out || !ws) return fail(MXE_EINVAL, "null state, out or workspace");
    if (ws_bytes < P->ws_bytes)
        return fail(MXE_ENOMEM, "workspace has " + std::to_string(ws_bytes) + " bytes, plan needs " +
                                    std::to_string(P->ws_bytes));
    if (((uintptr_t)ws) % 256 != 0) return fail(MXE_EINVAL, "workspace must be 256-byte aligned");
    const void* need[] = {st->qx, st->qy, st->qz, st->sigma, st->x, st->type, out->fx, out->fy,
                          out->fz, out->fsigma, out->mu, out->dxdt, out->rho_bar, out->rho0,
                          out->e_site, out->scalars};
    for (const void* q : need)
        if (!q) return fail(MXE_EINVAL, "a state or output pointer is NULL");
    if ((st->reservoir == nullptr) != (st->res_value == nullptr))
        return fail(MXE_EINVAL, "reservoir and res_value must both be given or both be NULL");
    char* w = (char*)ws;
    Dev& D = *d;
    std::memset(&D, 0, sizeof(D));
    D.qx = st->qx;
    D.qy = st->qy;
    D.qz = st->qz;
    D.sigma = st->sigma;
    D.x = st->x;
    D.type = st->type;
    D.res = st->reservoir;
    D.res_val = st->res_value;
    D.T_site = st->T_site;
    D.fx = out->fx;
    D.fy = out->fy;
    D.fz = out->fz;
    D.fs = out->fsigma;
    D.mu = out->mu;
    D.dxdt = out->dxdt;
    D.rho_bar = out->rho_bar;
    D.rho0 = out->rho0;
    D.e_site = out->e_site;
    D.scalars = out->scalars;
    const int64_t N = P->n_sites;
    D.sys = (SysDesc*)(w + P->o_sys);
    D.ctl = (SysCtl*)(w + P->o_ctl);
    D.chunks = (Chunk*)(w + P->o_chunks);
    D.pchunks = (Chunk*)(w + P->o_pchunks);
    D.site_sys = (int*)(w + P->o_site_sys);
    D.cell_count = (int*)(w + P->o_cell_count);
    D.cell_start = (int*)(w + P->o_cell_start);
    D.cell_sites = (int*)(w + P->o_cell_sites);
    D.cell_rec = (double4*)(w + P->o_cell_rec);
    D.cell_of = (int*)(w + P->o_cell_of);
    D.slot_of = (int*)(w + P->o_slot_of);
    D.chunk_up = (int*)(w + P->o_chunk_up);
    D.acell = (int2*)(w + P->o_acell);
    D.nbr = (int*)(w + P->o_nbr);
    D.nbr_cnt = (int*)(w + P->o_cnt);
    D.nbr_lo = (int*)(w + P->o_lo);
    D.pid = (int*)(w + P->o_pid);
    D.half_off = (int*)(w + P->o_hoff);
    D.pair_i = (int*)(w + P->o_pi);
    D.pnew = (int*)(w + P->o_pnew);
    D.pair_j = (int*)(w + P->o_pj);
    D.fblk = (void*)(w + P->o_fblk);
    D.dblk = (void*)(w + P->o_dblk);
    D.G = (double*)(w + P->o_G);
    D.Ahat = (double*)(w + P->o_A);
    D.Bhat = (double*)(w + P->o_B);
    double* v = (double*)(w + P->o_v);
    D.vx = v;
    D.vy = v + N;
    D.vz = v + 2 * N;
    D.vs = v + 3 * N;
    double* qr = (double*)(w + P->o_qr);
    D.qrx = qr;
    D.qry = qr + N;
    D.qrz = qr + 2 * N;
    D.sref = (double*)(w + P->o_sref);
    D.emit = (double*)(w + P->o_emit);
    D.srec = (void*)(w + P->o_srec);
    D.bond = (int*)(w + P->o_bond);
    D.nbond = (int*)(w + P->o_nbond);
    D.part = (double*)(w + P->o_part);
    D.part_sub = (double*)(w + P->o_part_sub);
    D.n_sites = (int)N;
    D.n_sys = P->n_sys;
    D.n_chunks = launch_extent(P->live_chunks, (int64_t)P->chunks.size());
    D.n_pchunks = launch_extent(P->live_pchunks, (int64_t)P->pchunks.size());
    D.K = P->p.k_max;
    D.bond_max = P->p.bond_max;
    D.n_cells = P->n_cells;
    D.pair_cap_total = P->pair_cap_total;
    return MXE_OK;
}

// What a call builds first: the neighbour lists (evaluate, relax), the lists
// and the bonds (run), or the bonds alone (step).
enum CallBuild { BUILD_LISTS, BUILD_LISTS_BONDS, BUILD_BONDS };

// Tables are re-uploaded at every call so a workspace needs no separate setup.
// Uploads the system descriptors (with this call's rebuild requests) and, when
// they changed or the workspace differs, the chunk tables; then initialises
// the call and builds the lists of every system that must be rebuilt (and the
// bonds), or only the bonds.
mxe_status begin_call(mxe_plan* P, const Dev& d, hipStream_t s, CallBuild what, bool advance = false) {
    P->prof_last = -1;  // the untimed launches below break the profiling chain
    const bool lists = what != BUILD_BONDS;
    // a workspace the plan has not built lists in holds none: build everything
    const bool new_ws = P->tables_ws != (void*)d.sys;
    const bool new_lists = P->lists_ws != (void*)d.sys;
    for (int k = 0; k < P->n_sys; ++k) {
        P->sys[k].force_build = (lists && (!P->resume || new_lists || P->dirty[k])) ? 1 : 0;
        // free-running budgets: a workspace new to the plan holds none
        int sn = advance ? P->steps_new[k] : -1;
        if (advance && new_lists && sn < 0) sn = 0;
        P->sys[k].steps_new = sn;
    }
    HIP_OK(hipMemcpyAsync(d.sys, P->sys.data(), sizeof(SysDesc) * P->sys.size(), hipMemcpyHostToDevice, s));
    if (advance) std::fill(P->steps_new.begin(), P->steps_new.end(), -1);
    if (P->tables_dirty || new_ws) {
        HIP_OK(hipMemcpyAsync(d.chunks, P->chunks.data(), sizeof(Chunk) * P->chunks.size(),
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d.pchunks, P->pchunks.data(), sizeof(Chunk) * P->pchunks.size(),
                              hipMemcpyHostToDevice, s));
        HIP_OK(hipMemcpyAsync(d.acell, P->acells.data(), sizeof(int2) * P->acells.size(),
                              hipMemcpyHostToDevice, s));
        P->tables_dirty = false;
        P->tables_ws = (void*)d.sys;
    }
    launch_ws_init(d, s);
    launch_sys_init(d, P->model, s, advance ? 1 : 0);
    if (lists) {
        std::fill(P->dirty.begin(), P->dirty.end(), 0);
        P->lists_ws = (void*)d.sys;
        launch_build(d, P->model, what == BUILD_LISTS_BONDS, true, s);
    } else {
        launch_bonds(d, P->model, s);
    }
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

// Records the next event of the pool on stream s; returns its index or -1.
long prof_record(mxe_plan* P, hipStream_t s) {
    if (P->prof_next == P->prof_events.size()) {
        hipEvent_t e;
        const hipError_t r = hipEventCreate(&e);
        if (r != hipSuccess) {
            P->prof_err = r;
            return -1;
        }
        P->prof_events.push_back(e);
    }
    const hipError_t r = hipEventRecord(P->prof_events[P->prof_next], s);
    if (r != hipSuccess) {
        P->prof_err = r;
        return -1;
    }
    return (long)P->prof_next++;
}

// Runs `launch` on stream s; with profiling on, brackets it with events. A
// chained family starts from the previous family's end event (they directly
// follow each other on the stream), so consecutive families share one event:
// every event on the stream is a point where the queue drains, and one per
// family boundary costs half as many as a pair per family.
template <typename F>
void timed(mxe_plan* P, int family, hipStream_t s, F&& launch, bool chain = false) {
    if (!P->prof_on) {
        launch();
        return;
    }
    if (P->prof_pair_only && family != MXE_K_PAIR) {
        launch();
        P->prof_last = -1;  // an unbracketed launch breaks the chain
        return;
    }
    const long start = (chain && P->prof_last >= 0) ? P->prof_last : prof_record(P, s);
    launch();
    const long end = start >= 0 ? prof_record(P, s) : -1;
    P->prof_last = end;
    if (end >= 0) P->prof_marks.push_back({family, (size_t)start, (size_t)end});
}

// The pair kernel always gets a start event of its own, so that its time (the
// roofline's) holds no launch gap before it.
void enqueue_eval(mxe_plan* P, const Dev& d, hipStream_t s) {
    const int prec = P->p.precision;
    timed(P, MXE_K_PAIR, s, [&] { launch_pair(d, P->model, prec, s); });
    timed(P, MXE_K_DENSITY, s, [&] { launch_density(d, P->model, prec, s); }, true);
    timed(P, MXE_K_FORCE, s, [&] { launch_force(d, P->model, prec, s); }, true);
}

// One relaxation iteration; free_run (mxe_advance) also takes the Euler step
// of every system whose relaxation ended in it. A lean iteration (chunked
// relaxations of small plans) launches no build chain (8 launches): a system
// whose lists expired takes no iteration until one with the chain.
void enqueue_iteration(mxe_plan* P, const Dev& d, hipStream_t s, bool free_run = false, bool lean = false) {
    if (!lean) timed(P, MXE_K_BUILD, s, [&] { launch_build(d, P->model, false, false, s); }, true);
    enqueue_eval(P, d, s);
    timed(P, MXE_K_FIRE, s, [&] {
        launch_control(d, P->model, free_run ? 2 : 1, s);
        launch_update(d, P->model, s);
    }, true);
    if (free_run) timed(P, MXE_K_MASTER, s, [&] { launch_master(d, P->model, 0.0, s, 1); }, true);
}

void enqueue_relax(mxe_plan* P, const Dev& d, hipStream_t s) {
    launch_relax_init(d, P->model, s);
    P->prof_last = -1;  // an untimed launch breaks the chain
    for (int k = 0; k <= P->p.max_relax; ++k) enqueue_iteration(P, d, s);
}

void enqueue_diffusion_step(mxe_plan* P, const Dev& d, hipStream_t s) {
    enqueue_relax(P, d, s);
    timed(P, MXE_K_MASTER, s, [&] { launch_master(d, P->model, 0.0, s); }, true);
}

// Pinned host slots and events of the early exit, made on first use.
mxe_status ensure_active_slots(mxe_plan* P) {
    if (P->act_host) return MXE_OK;
    int* h = nullptr;
    HIP_OK(hipHostMalloc((void**)&h, 4 * sizeof(int), hipHostMallocMapped));
    void* dp = nullptr;
    hipError_t e = hipHostGetDevicePointer(&dp, h, 0);
    for (int k = 0; k < 2 && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&P->act_ev[k], hipEventDisableTiming);
    if (e != hipSuccess) {
        for (hipEvent_t& ev : P->act_ev)
            if (ev) {
                (void)hipEventDestroy(ev);
                ev = nullptr;
            }
        (void)hipHostFree(h);
        return fail(MXE_EDEVICE, std::string("early-exit slots: ") + hipGetErrorString(e));
    }
    h[0] = h[2] = 1;
    h[1] = h[3] = 0;
    P->act_host = h;
    P->act_dev = (int*)dp;
    return MXE_OK;
}

// Waits (polling) for the event of a slot, then reads its counts.
mxe_status read_active(mxe_plan* P, int slot, int* active, int* stalled) {
    for (;;) {
        const hipError_t e = hipEventQuery(P->act_ev[slot]);
        if (e == hipSuccess) break;
        if (e != hipErrorNotReady) return fail(MXE_EDEVICE, std::string("early-exit event: ") + hipGetErrorString(e));
        std::this_thread::yield();
    }
    std::atomic_thread_fence(std::memory_order_acquire);
    *active = ((volatile int*)P->act_host)[2 * slot];
    *stalled = ((volatile int*)P->act_host)[2 * slot + 1];
    return MXE_OK;
}

// Lean chunks for plans of one occupied system or of at most this many
// occupied sites. A stalled system waits up to two chunks for its build (the
// host reads one chunk behind): in a plan of many systems some system stalls in
// nearly every chunk, and the build chain's early-exit launches, which lean
// iterations save, are a small share of a large plan's iteration. Measured on
// the 256 serving-mix requests (500 to 48,668 sites): one at a time 10.3 ->
// 9.1 s with lean chunks, all in one plan 4.35 -> 4.7 s; the 256k-site vacancy
// lattice alone, eager, chunks of 2: 33.3 -> 33.1 ms per step.
constexpr int64_t kLeanMaxSites = 65536;

bool lean_chunks(const mxe_plan* P) {
    return P->live_sys <= 1 || P->live_chunks * (int64_t)kChunk <= kLeanMaxSites;
}

// A relaxation in chunks of relax_chunk iterations, lean ones for small plans
// (one graph replay each, or eager launches). After every chunk, k_active writes how many systems are
// still relaxing and how many are stalled for a build into a host slot; the
// host reads chunk c's counts after it has enqueued chunk c + 1, so the device
// never waits for the host. It stops once none is relaxing, and enqueues one
// iteration with the build chain (graph full, or eager) whenever some are
// stalled: they take it as the iteration they waited for. A stalled system
// takes no iteration, so the relaxation of each system runs the same FIRE
// iterations with the same lists as the fixed sequence; chunks enqueued past
// the end run as no-ops. A system waits at most two chunks per build, which
// bounds the chunks.
mxe_status enqueue_relax_chunked(mxe_plan* P, const Dev& d, hipStream_t s, hipGraphExec_t graph,
                                 hipGraphExec_t full, bool lean) {
    launch_relax_init(d, P->model, s);
    P->prof_last = -1;
    const int K = P->p.relax_chunk;
    const int n_cap = 3 * (P->p.max_relax + 1) + 4;
    bool full_prev = false;  // an iteration with the chain followed chunk c - 1
    for (int c = 0; c < n_cap; ++c) {
        if (graph) {
            HIP_OK(hipGraphLaunch(graph, s));
        } else {
            for (int k = 0; k < K; ++k) enqueue_iteration(P, d, s, false, lean);
        }
        launch_active(d, P->act_dev + 2 * (c & 1), 0, s);
        P->prof_last = -1;  // an untimed launch breaks the chain
        HIP_OK(hipEventRecord(P->act_ev[c & 1], s));
        bool full_now = false;
        if (c >= 1) {
            int active = 1, stalled = 0;
            const mxe_status r = read_active(P, (c - 1) & 1, &active, &stalled);
            if (r != MXE_OK) return r;
            if (active == 0) break;
            // stalls counted after chunk c - 1 are over once an iteration with
            // the chain followed it
            if (stalled > 0 && !full_prev) {
                if (full) HIP_OK(hipGraphLaunch(full, s));
                else enqueue_iteration(P, d, s);
                full_now = true;
            }
        }
        full_prev = full_now;
    }
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

// Records what `enqueue` launches on the plan's capture stream into *exec.
template <typename F>
mxe_status capture(mxe_plan* P, F&& enqueue, hipGraphExec_t* exec) {
    if (!P->cap_stream) HIP_OK(hipStreamCreateWithFlags(&P->cap_stream, hipStreamNonBlocking));
    HIP_OK(hipStreamBeginCapture(P->cap_stream, hipStreamCaptureModeRelaxed));
    enqueue(P->cap_stream);
    hipGraph_t g = nullptr;
    const hipError_t e1 = hipStreamEndCapture(P->cap_stream, &g);
    if (e1 != hipSuccess) return fail(MXE_EDEVICE, std::string("graph capture: ") + hipGetErrorString(e1));
    const hipError_t e2 = hipGraphInstantiate(exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e2 != hipSuccess) {
        *exec = nullptr;
        return fail(MXE_EDEVICE, std::string("graph instantiate: ") + hipGetErrorString(e2));
    }
    return MXE_OK;
}

}  // namespace

extern "C" mxe_status mxe_evaluate(mxe_plan* P, const mxe_state* st, const mxe_out* out, void* ws,
                                   size_t ws_bytes, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    Dev d;
    mxe_status r = make_dev(P, st, out, ws, ws_bytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = begin_call(P, d, s, BUILD_LISTS);
    if (r != MXE_OK) return r;
    launch_relax_init(d, P->model, s);
    enqueue_eval(P, d, s);
    launch_control(d, P->model, 0, s);
    P->prof_last = -1;
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

extern "C" mxe_status mxe_relax(mxe_plan* P, const mxe_state* st, const mxe_out* out, void* ws,
                                size_t ws_bytes, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    Dev d;
    mxe_status r = make_dev(P, st, out, ws, ws_bytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = begin_call(P, d, s, BUILD_LISTS);
    if (r != MXE_OK) return r;
    if (P->p.relax_chunk > 0) {
        r = ensure_active_slots(P);
        if (r != MXE_OK) return r;
        return enqueue_relax_chunked(P, d, s, nullptr, nullptr, lean_chunks(P));
    }
    enqueue_relax(P, d, s);
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

extern "C" mxe_status mxe_step(mxe_plan* P, const mxe_state* st, const mxe_out* out, double dt_in,
                               void* ws, size_t ws_bytes, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (!std::isfinite(dt_in)) return fail(MXE_EINVAL, "dt_in must be finite");
    Dev d;
    mxe_status r = make_dev(P, st, out, ws, ws_bytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = begin_call(P, d, s, BUILD_BONDS);
    if (r != MXE_OK) return r;
    timed(P, MXE_K_MASTER, s, [&] { launch_master(d, P->model, dt_in, s); });
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

extern "C" mxe_status mxe_run(mxe_plan* P, const mxe_state* st, const mxe_out* out, int n_steps,
                              int use_graph, void* ws, size_t ws_bytes, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (n_steps < 0) return fail(MXE_EINVAL, "n_steps < 0");
    Dev d;
    mxe_status r = make_dev(P, st, out, ws, ws_bytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = begin_call(P, d, s, BUILD_LISTS_BONDS);
    if (r != MXE_OK) return r;
    const bool chunked = P->p.relax_chunk > 0;
    if (chunked) {
        r = ensure_active_slots(P);
        if (r != MXE_OK) return r;
    }
    if (!use_graph || P->prof_on) {
        for (int k = 0; k < n_steps; ++k) {
            if (!chunked) {
                enqueue_diffusion_step(P, d, s);
                continue;
            }
            r = enqueue_relax_chunked(P, d, s, nullptr, nullptr, lean_chunks(P));
            if (r != MXE_OK) return r;
            timed(P, MXE_K_MASTER, s, [&] { launch_master(d, P->model, 0.0, s); });
        }
        HIP_OK(hipGetLastError());
        return MXE_OK;
    }
    const std::vector<const void*> key = {st->qx, st->qy, st->qz, st->sigma, st->x, st->type,
                                          st->reservoir, st->res_value, st->T_site, out->fx, out->fy,
                                          out->fz, out->fsigma, out->mu, out->dxdt, out->rho_bar,
                                          out->rho0, out->e_site, out->scalars, ws,
                                          (const void*)(intptr_t)d.n_chunks, (const void*)(intptr_t)d.n_pchunks};
    if (!P->graphs.count(key) && P->graphs.size() >= 16) {  // bounded cache: start afresh
        for (auto& kv : P->graphs)
            for (hipGraphExec_t g : kv.second.all())
                if (g) HIP_OK(hipGraphExecDestroy(g));
        P->graphs.clear();
    }
    mxe_plan::Graphs& G = P->graphs[key];
    if (!chunked && !G.step) {
        r = capture(P, [&](hipStream_t c) { enqueue_diffusion_step(P, d, c); }, &G.step);
        if (r != MXE_OK) return r;
    }
    const bool lean = lean_chunks(P);
    if (chunked && G.master && G.chunk_lean != lean) {  // recorded for the other kind of chunk
        for (hipGraphExec_t* g : {&G.chunk, &G.full, &G.master})
            if (*g) {
                HIP_OK(hipGraphExecDestroy(*g));
                *g = nullptr;
            }
    }
    if (chunked && !G.master) {
        G.chunk_lean = lean;
        r = capture(P, [&](hipStream_t c) {
            for (int k = 0; k < P->p.relax_chunk; ++k) enqueue_iteration(P, d, c, false, lean);
        }, &G.chunk);
        if (r != MXE_OK) return r;
        r = capture(P, [&](hipStream_t c) { enqueue_iteration(P, d, c); }, &G.full);
        if (r != MXE_OK) return r;
        r = capture(P, [&](hipStream_t c) { launch_master(d, P->model, 0.0, c); }, &G.master);
        if (r != MXE_OK) return r;
    }
    for (int k = 0; k < n_steps; ++k) {
        if (!chunked) {
            HIP_OK(hipGraphLaunch(G.step, s));
            continue;
        }
        r = enqueue_relax_chunked(P, d, s, G.chunk, G.full, lean);
        if (r != MXE_OK) return r;
        HIP_OK(hipGraphLaunch(G.master, s));
    }
    return MXE_OK;
}

extern "C" mxe_status mxe_plan_set_steps(mxe_plan* P, int slot, int n_steps) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (slot < 0 || slot >= P->n_sys) return fail(MXE_EINVAL, "slot out of range");
    if (n_steps < 0) return fail(MXE_EINVAL, "n_steps < 0");
    P->steps_new[slot] = n_steps;
    return MXE_OK;
}

extern "C" mxe_status mxe_advance(mxe_plan* P, const mxe_state* st, const mxe_out* out, int max_iters,
                                  int use_graph, void* ws, size_t ws_bytes, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (max_iters < 0) return fail(MXE_EINVAL, "max_iters < 0");
    if (P->p.relax_chunk <= 0) return fail(MXE_EINVAL, "mxe_advance needs params.relax_chunk > 0");
    if (!P->resume) return fail(MXE_EINVAL, "mxe_advance needs resume mode (mxe_plan_set_resume)");
    Dev d;
    mxe_status r = make_dev(P, st, out, ws, ws_bytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    r = ensure_active_slots(P);
    if (r != MXE_OK) return r;
    r = begin_call(P, d, s, BUILD_LISTS_BONDS, true);
    if (r != MXE_OK) return r;
    const int K = P->p.relax_chunk;
    const bool lean = lean_chunks(P);
    hipGraphExec_t g = nullptr, gf = nullptr;
    if (use_graph && !P->prof_on) {
        const std::vector<const void*> key = {st->qx, st->qy, st->qz, st->sigma, st->x, st->type,
                                              st->reservoir, st->res_value, st->T_site, out->fx, out->fy,
                                              out->fz, out->fsigma, out->mu, out->dxdt, out->rho_bar,
                                              out->rho0, out->e_site, out->scalars, ws,
                                              (const void*)(intptr_t)d.n_chunks,
                                              (const void*)(intptr_t)d.n_pchunks};
        if (!P->graphs.count(key) && P->graphs.size() >= 16) {  // bounded cache: start afresh
            for (auto& kv : P->graphs)
                for (hipGraphExec_t e : kv.second.all())
                    if (e) HIP_OK(hipGraphExecDestroy(e));
            P->graphs.clear();
        }
        mxe_plan::Graphs& G = P->graphs[key];
        if (G.advance && G.advance_lean != lean) {  // recorded for the other kind of chunk
            for (hipGraphExec_t* e : {&G.advance, &G.advance_full})
                if (*e) {
                    HIP_OK(hipGraphExecDestroy(*e));
                    *e = nullptr;
                }
        }
        if (!G.advance) {
            G.advance_lean = lean;
            r = capture(P, [&](hipStream_t c) {
                for (int k = 0; k < K; ++k) enqueue_iteration(P, d, c, true, lean);
            }, &G.advance);
            if (r != MXE_OK) return r;
            r = capture(P, [&](hipStream_t c) { enqueue_iteration(P, d, c, true); }, &G.advance_full);
            if (r != MXE_OK) return r;
        }
        g = G.advance;
        gf = G.advance_full;
    }
    // chunks of K free-running iterations (lean for small plans) until no system has steps left
    // or max_iters are enqueued, with an iteration with the build chain after a
    // chunk that left systems stalled (both read one chunk behind, as in
    // enqueue_relax_chunked; stalls seen after the last chunk wait for the next
    // call)
    const int n_chunks = (max_iters + K - 1) / K;
    bool full_prev = false;
    for (int c = 0; c < n_chunks; ++c) {
        if (g) {
            HIP_OK(hipGraphLaunch(g, s));
        } else {
            for (int k = 0; k < K; ++k) enqueue_iteration(P, d, s, true, lean);
        }
        launch_active(d, P->act_dev + 2 * (c & 1), 1, s);
        P->prof_last = -1;
        HIP_OK(hipEventRecord(P->act_ev[c & 1], s));
        bool full_now = false;
        if (c >= 1) {
            int active = 1, stalled = 0;
            r = read_active(P, (c - 1) & 1, &active, &stalled);
            if (r != MXE_OK) return r;
            if (active == 0) break;
            if (stalled > 0 && !full_prev) {
                if (gf) HIP_OK(hipGraphLaunch(gf, s));
                else enqueue_iteration(P, d, s, true);
                full_now = true;
            }
        }
        full_prev = full_now;
    }
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

// ---------------------------------------------------------------------------
// Allocation-free entry point: the workspace is a library-held device array.
// ---------------------------------------------------------------------------
// One copy per device, allocated when the code object loads and held until the
// process ends. Host code never passes the array's name to a kernel or a copy
// (on the host it is only a stand-in): it uses the device address that
// hipGetSymbolAddress returns for the current device.
static constexpr size_t kScratchBytes = (size_t)MXE_NOALLOC_SCRATCH_BYTES;
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's scratch (looked up once per device).
mxe_status scratch_for_current_device(void** out) {
    int dev = -1;
    HIP_OK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MXE_EDEVICE, "device index out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* ptr = nullptr;
        size_t bytes = 0;
        HIP_OK(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
        HIP_OK(hipGetSymbolSize(&bytes, HIP_SYMBOL(scratch)));
        if (!ptr || ((uintptr_t)ptr) % 256 != 0 || bytes < kScratchBytes)
            return fail(MXE_EDEVICE, "scratch symbol: unexpected address or size");
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return MXE_OK;
}

}  // namespace

extern "C" mxe_status mxe_run_noalloc(mxe_plan* P, const mxe_state* st, const mxe_out* out,
                                      int n_steps, void* stream) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (n_steps < 0) return fail(MXE_EINVAL, "n_steps < 0");
    if (P->ws_bytes > kScratchBytes)
        return fail(MXE_ENOMEM, "plan needs " + std::to_string(P->ws_bytes) +
                                    " workspace bytes; the allocation-free entry point holds " +
                                    std::to_string(kScratchBytes) + " per device");
    if (P->prof_on) return fail(MXE_EINVAL, "profiling creates events: switch it off for mxe_run_noalloc");
    void* ws = nullptr;
    mxe_status r = scratch_for_current_device(&ws);
    if (r != MXE_OK) return r;
    Dev d;
    r = make_dev(P, st, out, ws, kScratchBytes, &d);
    if (r != MXE_OK) return r;
    hipStream_t s = (hipStream_t)stream;
    // Any call on this device may have overwritten the scratch since this plan
    // last used it: upload every table and rebuild every list and bond.
    P->tables_ws = P->lists_ws = nullptr;
    r = begin_call(P, d, s, BUILD_LISTS_BONDS);
    P->tables_ws = P->lists_ws = nullptr;
    if (r != MXE_OK) return r;
    for (int k = 0; k < n_steps; ++k) enqueue_diffusion_step(P, d, s);
    HIP_OK(hipGetLastError());
    return MXE_OK;
}

extern "C" mxe_status mxe_profile(mxe_plan* P, int on) {
    if (!P) return fail(MXE_EINVAL, "null plan");
    if (on != MXE_PROFILE_OFF && on != MXE_PROFILE_ALL && on != MXE_PROFILE_PAIR)
        return fail(MXE_EINVAL, "profile mode must be MXE_PROFILE_OFF, _ALL or _PAIR");
    P->prof_on = on != MXE_PROFILE_OFF;
    P->prof_pair_only = on == MXE_PROFILE_PAIR;
    P->prof_last = -1;
    return MXE_OK;
}

extern "C" mxe_status mxe_profile_read(mxe_plan* P, double* ms, int64_t* launches) {
    if (!P || !ms || !launches) return fail(MXE_EINVAL, "null argument");
    for (int k = 0; k < MXE_NPROF; ++k) {
        ms[k] = 0.0;
        launches[k] = 0;
    }
    if (P->prof_err != hipSuccess) {
        const hipError_t e = P->prof_err;
        P->prof_err = hipSuccess;
        P->prof_marks.clear();
        P->prof_next = 0;
        P->prof_last = -1;
        return fail(MXE_EDEVICE, std::string("profiling event: ") + hipGetErrorString(e));
    }
    for (const auto& mk : P->prof_marks) {
        HIP_OK(hipEventSynchronize(P->prof_events[mk.end]));
        float t = 0.0f;
        HIP_OK(hipEventElapsedTime(&t, P->prof_events[mk.start], P->prof_events[mk.end]));
        ms[mk.family] += (double)t;
        launches[mk.family] += 1;
    }
    P->prof_marks.clear();
    P->prof_next = 0;
    P->prof_last = -1;
    return MXE_OK;
}

extern "C" const char* mxe_status_string(mxe_status s) {
    switch (s) {
        case MXE_OK: return "ok";
        case MXE_EINVAL: return "invalid argument";
        case MXE_ENOMEM: return "workspace too small";
        case MXE_EDEVICE: return "HIP runtime error";
        case MXE_ERANGE: return "size limit exceeded";
    }
    return "unknown status";
}

extern "C" const char* mxe_last_error(void) { return g_err.c_str(); }
