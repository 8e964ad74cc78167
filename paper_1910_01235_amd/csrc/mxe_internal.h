// Internal definitions shared by the HIP translation units of the library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "mxe.h"

namespace mxe {

constexpr int kFBlk = 16;           // force block per pair: 16 moments = one 128-byte line (FP64)
constexpr int kSRec = 8;            // per-site record: A~, B~, b, pair amplitude against A, B, S, 2 pad
constexpr int kChunk = 256;         // sites per site-chunk; block size of per-site kernels
constexpr int kPairChunk = 4096;    // pair slots per pair-chunk
constexpr int kNPart = 8;           // partial sums per site-chunk
constexpr int kForceSplit = 8;      // force-gather blocks (and partial rows) per site chunk
constexpr int kGatherSplit = 8;     // density-gather blocks per site chunk
constexpr int kWave = 64;
constexpr double kBoltzmannEv = 8.617333262e-5;  // eV/K

// moment slots of a pair (lo, hi) = (i, j), computed at rbar = q_hi - q_lo;
// this is also the layout of the pair's force block. Width derivatives are
// stored divided by the width of their end: (d<g>/dsigma_lo)/sigma_lo and
// (d<g>/dsigma_hi)/sigma_hi; under the product rule both equal (d<g>/ds)/s.
enum {
    M_PHI = 0, M_GPHI = 1, M_SPHI = 4,   // <phi>, grad <phi> (3), lo-end width term
    M_F = 5, M_GF = 6, M_SF = 9,         // <f>, grad <f> (3), lo-end width term
    M_F0 = 10, M_GF0 = 11,               // f(|rbar|), grad f(|rbar|) (3)
    M_SPHI_HI = 14, M_SF_HI = 15         // hi-end width terms of <phi>, <f>
};

// partial-sum slots of a site-chunk
enum { P_E = 0, P_FMAX = 1, P_FV = 2, P_FF = 3, P_VV = 4, P_SUMX = 5, P_RATE = 6, P_RES = 7 };

struct SysDesc {
    int64_t site_off, n_sites;
    int64_t cell_off, n_cells;
    int64_t pair_base, pair_cap;
    double box[3];
    double cell_w[3];
    int nc[3];
    int periodic[3];
    double T, kT, beta, D;  // reference temperature and its derived constants
    int chunk_first, n_chunks;
    int force_build;  // rebuild lists and bonds at the start of the call
    int steps_new;    // mxe_advance: a new step budget from this call on, or -1
};

struct SysCtl {
    double fire_dt, fire_alpha;
    double c_keep, mix_v, mix_f;
    // largest squared displacement and largest widening (sigma - sigma_build, at
    // least 0) of any site since the last build, as bits of non-negative doubles
    unsigned long long drift_bits, widen_bits;
    double dt_master;
    int npos, k, done, converged, updates, evals;
    int rebuild, n_rebuilds, total_evals;
    double pair_evals;
    int n_pairs;
    int status;
    // free-running steps (mxe_advance): diffusion steps still to run, and the
    // flag that the relaxation ended in this iteration (its Euler step follows)
    int steps_left, stepping;
    // lean iterations (chunked relaxations, no build chain): the lists had
    // expired, so this iteration was not taken (set by k_control each
    // iteration, read by k_update and by the host's count)
    int stall;
};

struct Chunk {
    int sys;
    int start;  // first global index
    int end;    // one past the last global index
    int pad;
};

// Polynomial coefficients of the FP64 node arithmetic, highest degree first:
// near-minimax remainders of e^r on |r| <= ln2/2 and of the taper's sine and
// cosine on |z| <= pi/2 (in w = z^2), from node_poly.h. They travel in the
// kernel arguments so that the kernels read them into scalar registers.
struct PolyCoef {
    static constexpr int kExp = 9, kSin = 8, kCos = 7;
    // 2^f = 1 + f (ln2 + f (ln2^2/2 + f E2(f))) with E2(f) = ln2^3 E(f ln2), where
    // e^r = 1 + r (1 + r (1/2 + r E(r))); ex holds E2 and ln2, ln2sq_half the
    // two leading coefficients (all rounded from extended precision)
    double ex[kExp];
    double ln2, ln2sq_half;
    double sn[kSin];  // S(w): sin z = z (1 - w S(w)), S(0) = 1/3!
    double cs[kCos];  // C(w): cos z = 1 + w (-1/2 + w C(w)), C(0) = 1/4!
};

// Analytic EAM and run parameters, passed by value to the kernels.
struct Model {
    double c4[4], b4[4];    // per species (A, B, S, none): embedding strength, emission
    double a4[4][4];        // pair amplitude, zero row/column for "none"
    double r_e[2], inv_re[2], alpha[2], gamma[2];
    double r_s, r_c, taper_inv_w;
    double ftol, dt0, dtmax, alpha0, finc, fdec, falpha;
    int nmin, max_relax;
    double sigma_min, sigma_cap, skin, r_bond, kin_c, dt_safety, nu0, Qm;
    int gather_lanes, pair_block;  // launch shapes (tuned per workload): density gather, pair kernel
    int force_lanes;               // lanes per site of the force gather
    int quad_rule;                 // MXE_QUAD_GH27 or MXE_QUAD_DEGREE3
    PolyCoef poly;
    int gather_stride;             // chunk visit stride of the gathers (xcd_unit_strided)
    int pair_shift;                // log2 of the pair-kernel blocks per pair chunk
    int ratio_pq[2];               // per class: 16 P + Q when alpha : gamma = P : Q (P, Q <= 15), else 0
    double u_rate[2];              // per class with a ratio: alpha / P (divided on the host, not per pair)
    int fold_rows;                 // a system has more site chunks than the FIRE control has threads:
                                   // the force gather's partial rows are folded per chunk by a launch of their own
};

// Every device pointer the kernels use.
struct Dev {
    // state
    double *qx, *qy, *qz, *sigma, *x;
    const int8_t* type;
    const int8_t* res;     // reservoir kind per site, or null
    const double* res_val; // held x or mu per site, or null
    const double* T_site;  // per-site temperature, or null (uniform)
    // outputs
    double *fx, *fy, *fz, *fs, *mu, *dxdt, *rho_bar, *rho0, *e_site, *scalars;
    // workspace
    SysDesc* sys;
    SysCtl* ctl;
    Chunk* chunks;
    Chunk* pchunks;
    int* site_sys;
    int* cell_count;   // sites per cell (zero between builds)
    int* cell_start;   // first entry of each cell in cell_sites
    int* cell_sites;   // 4 * site index + site type, grouped by cell, N entries
    double4* cell_rec; // (qx, qy, qz, sigma) of the same entries
    int *cell_of, *slot_of;
    int* chunk_up;     // per site chunk: owned (upper) pairs found by the build
    int2* acell;       // [0].x: number of cells in use; [0].y: 1 while any system's lists
                       // are being rebuilt; [1 + b]: (system, global cell)
    int *nbr, *nbr_cnt, *nbr_lo, *pid, *half_off;
    int *pair_i, *pair_j;
    int* pnew;         // per pair: its number after the renumbering by geometric class
    void* fblk;   // [pair][kFBlk] force blocks (T)
    void* dblk;   // [pair][2] density pair (<f>, f0) (T)
    double *G, *Ahat, *Bhat;
    double* emit;  // density emitted by each site, b_i (refreshed when x changes)
    void* srec;    // per-site record read by the force gather, kSRec values of the moment type
    double *vx, *vy, *vz, *vs;
    double *qrx, *qry, *qrz, *sref;
    int *bond, *nbond;
    double* part;
    double* part_sub;  // [chunk][kForceSplit][kNPart]: the force gather's block rows
    int n_sites, n_sys, n_chunks, n_pchunks;
    int K, bond_max;
    int64_t n_cells, pair_cap_total;
};

// ---------------------------------------------------------------------------
// Site occupancy model: a site holds species sp1 with probability p1 = x (1 for a
// fixed host atom) and species sp0 with 1 - p1. Species 3 is "nothing".
// ---------------------------------------------------------------------------
__host__ __device__ inline int occ_sp1(int t) { return t == MXE_SITE_ALLOY ? 1 : (t == MXE_SITE_INTERSTITIAL ? 2 : 0); }
__host__ __device__ inline int occ_sp0(int t) { return t == MXE_SITE_ALLOY ? 0 : 3; }
__host__ __device__ inline double occ_p1(int t, double x) { return t == MXE_SITE_HOST_FIXED ? 1.0 : x; }
__host__ __device__ inline bool occ_mobile(int t) { return t != MXE_SITE_HOST_FIXED; }
// weight of site i's energy share, T / T_i (1 at uniform temperature)
// (T_sys: the system's reference temperature, read once before a site loop)
__device__ inline double theta_at(const Dev& d, double T_sys, int i) {
    return d.T_site != nullptr ? T_sys / d.T_site[i] : 1.0;
}

// Running maximum of non-negative doubles kept as their bit patterns (ordered
// like the values). The maxima only grow, so a value that does not exceed a
// (possibly stale) read of the current one needs no atomic: one block in many
// contends for the line instead of all of them.
__device__ inline void raise_max(unsigned long long* bits, double v) {
    const unsigned long long b = (unsigned long long)__double_as_longlong(v);
    if (b > *(volatile unsigned long long*)bits) atomicMax(bits, b);
}

// The lists of a system stay valid while 2 max|dq| + 3 sqrt(2) max(sigma -
// sigma_build, 0) <= skin (maxima since the last build, recorded by the FIRE
// update); true when they must be rebuilt.
__device__ inline bool lists_expired(const SysCtl& c, const Model& m) {
    const double drift = __longlong_as_double((long long)c.drift_bits);
    const double widen = __longlong_as_double((long long)c.widen_bits);
    return 2.0 * sqrt(drift) + 3.0 * sqrt(2.0) * widen > m.skin;
}

// After a build of system s: count it, clear the request and the maxima,
// publish the pair count (one thread per system).
__device__ inline void finish_build(const Dev& d, int s) {
    SysCtl& c = d.ctl[s];
    if (!c.rebuild) return;
    c.n_rebuilds += 1;
    c.rebuild = 0;
    d.acell[0].y = 0;  // set again by the next system that needs a rebuild
    c.drift_bits = 0ull;
    c.widen_bits = 0ull;
    d.scalars[(int64_t)s * MXE_NSCALARS + MXE_S_PAIRS] = (double)c.n_pairs;
    d.scalars[(int64_t)s * MXE_NSCALARS + MXE_S_REBUILDS] = (double)c.n_rebuilds;
}

// is mobile site i (of type t) a reservoir site of the given kind?
__device__ inline bool held(const Dev& d, int i, int t, int kind) {
    return d.res != nullptr && d.res[i] == kind && occ_mobile(t);
}
__host__ __device__ inline bool occ_partial(int t) {  // vibrating fraction w = x
    return t == MXE_SITE_HOST_VAC || t == MXE_SITE_INTERSTITIAL;
}
__host__ __device__ inline bool is_inter(int t) { return t == MXE_SITE_INTERSTITIAL; }
// interaction class of a pair: 0 host-host, 1 host-interstitial, -1 none
__host__ __device__ inline int pair_cls(int ti, int tj) {
    const bool a = is_inter(ti), b = is_inter(tj);
    return (a && b) ? -1 : ((a || b) ? 1 : 0);
}

// A value that is the same on every lane (a kernel argument), passed through
// readfirstlane: it stays in scalar registers, and a select between such
// values stays a select instead of becoming one load from a selected address.
__device__ inline double uniform_value(double v) {
    const int lo = __builtin_amdgcn_readfirstlane(__double2loint(v));
    const int hi = __builtin_amdgcn_readfirstlane(__double2hiint(v));
    return __hiloint2double(hi, lo);
}
// v4[k] of a per-species table in the kernel arguments (the same on every
// lane), for a per-lane k, selected from the four values: indexed by a lane's
// value, the table would be read with a vector load, and waiting for that
// load waits for every load and store the thread has in flight.
__device__ inline double sp4(const double* v4, int k) {
    const double v0 = uniform_value(v4[0]), v1 = uniform_value(v4[1]);
    const double v2 = uniform_value(v4[2]), v3 = uniform_value(v4[3]);
    const double a = k == 1 ? v1 : v0;
    const double b = k == 3 ? v3 : v2;
    return k < 2 ? a : b;
}
// per-species value mixed by the site's occupancy
__device__ inline double mixval(const double* v4, int t, double x) {
    const double p = occ_p1(t, x);
    return p * sp4(v4, occ_sp1(t)) + (1.0 - p) * sp4(v4, occ_sp0(t));
}
// the same divided by the vibrating fraction w (closed form)
__device__ inline double mixhat(const double* v4, int t, double x) {
    return occ_partial(t) ? sp4(v4, occ_sp1(t)) : mixval(v4, t, x);
}
__device__ inline double mixdx(const double* v4, int t) {
    return occ_mobile(t) ? sp4(v4, occ_sp1(t)) - sp4(v4, occ_sp0(t)) : 0.0;
}
// mixhat with the table indexed by the lane's species (the same value)
__device__ inline double mixhat_indexed(const double* v4, int t, double x) {
    const double p = occ_p1(t, x);
    return occ_partial(t) ? v4[occ_sp1(t)] : p * v4[occ_sp1(t)] + (1.0 - p) * v4[occ_sp0(t)];
}

// index ranges for grid-stride loops
__device__ inline int gtid() { return blockIdx.x * blockDim.x + threadIdx.x; }

// XCD-aware chunk order. The hardware deals workgroups to the 8 XCDs in turn,
// so consecutive chunks (neighbouring sites) would land in 8 different L2
// caches. Workgroup b takes chunk (b % 8) * per + b / 8 instead: each XCD
// sweeps one contiguous range of chunks and the neighbours' data a gather
// reads (pair blocks from both ends, site records) stay in its own L2.
// Launch xcd_grid(n) workgroups; a workgroup whose chunk is >= n exits.
constexpr int kXcd = 8;
__device__ inline int xcd_chunk(int n) {
    const int per = (n + kXcd - 1) / kXcd;
    return (int)(blockIdx.x % kXcd) * per + (int)(blockIdx.x / kXcd);
}
__host__ __device__ inline int xcd_grid(int n) { return (n + kXcd - 1) / kXcd * kXcd; }

// The gathers' chunk order. Each XCD takes a contiguous range of whole chunks
// (split blocks per chunk) and visits it as a table of rows of S chunks, column
// by column: chunks S apart are visited one after the other. When S is the
// number of chunks in one layer of the lattice order (the sites one step
// along the slowest axis away), a pair block read from one end is read from
// the other end a few chunks later, while it is still in the XCD's L2 (on the
// 256k-site vacancy lattice, 25 chunks per layer: force gather 418 -> 386 us).
// S = 1 is plain order. Launch xcd_grid_chunks(n, split) workgroups; a
// workgroup given a unit >= n_chunks * split exits.
__host__ __device__ inline int xcd_grid_chunks(int n_chunks, int split) {
    return (n_chunks + kXcd - 1) / kXcd * kXcd * split;
}
__device__ inline int xcd_unit_strided(int n_chunks, int split, int S) {
    const int per = (n_chunks + kXcd - 1) / kXcd;
    const int x = (int)(blockIdx.x % kXcd), k = (int)(blockIdx.x / kXcd);
    const int nC = min(per, n_chunks - x * per);  // chunks of this XCD's range
    const int v = k / split, part = k % split;     // the v-th chunk this XCD visits
    if (nC <= 0 || v >= nC) return n_chunks * split;
    const int Sx = min(max(S, 1), nC);
    const int R = (nC + Sx - 1) / Sx;              // rows; the last holds q chunks
    const int q = nC - (R - 1) * Sx;               // columns 0..q-1 have R chunks
    int p, r;
    if (v < q * R) {
        p = v / R;
        r = v % R;
    } else {
        const int w = v - q * R;
        p = q + w / (R - 1);
        r = w % (R - 1);
    }
    return (x * per + r * Sx + p) * split + part;
}
__device__ inline int gstride() { return gridDim.x * blockDim.x; }

__device__ inline double wave_sum(double v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Host-side launchers (each defined next to its kernels).
// ---------------------------------------------------------------------------
void launch_ws_init(const Dev& d, hipStream_t s);
void launch_sys_init(const Dev& d, const Model& m, hipStream_t s, int advance = 0);
// bonds: also rebuild the bond lists; finish: count the build and clear the
// request at the end of the chain (otherwise the next k_control does it)
void launch_build(const Dev& d, const Model& m, bool bonds, bool finish, hipStream_t s);
// bonds of every system from the current positions; lists untouched
void launch_bonds(const Dev& d, const Model& m, hipStream_t s);
void launch_relax_init(const Dev& d, const Model& m, hipStream_t s);
void launch_pair(const Dev& d, const Model& m, int precision, hipStream_t s);
void launch_density(const Dev& d, const Model& m, int precision, hipStream_t s);
void launch_force(const Dev& d, const Model& m, int precision, hipStream_t s);
void launch_control(const Dev& d, const Model& m, int mode, hipStream_t s);
void launch_update(const Dev& d, const Model& m, hipStream_t s);
// systems not done (steps = 0) or with diffusion steps left (steps = 1) ->
// out[0], and systems stalled for a build -> out[1]
void launch_active(const Dev& d, int* out, int steps, hipStream_t s);
// free_run: only systems whose relaxation ended in this iteration step
void launch_master(const Dev& d, const Model& m, double dt_in, hipStream_t s, int free_run = 0);
// relaxation state at the start of a relaxation (FIRE scalars and counters)
// A system whose iteration is not taken: its relaxation finished, or its
// lists expired and no build runs in this iteration (a lean iteration; in an
// iteration with the build chain k_bin has set rebuild). The maxima behind
// lists_expired change only in k_update, the iteration's last kernel, so
// every kernel before it reaches the same decision.
__device__ inline bool idle(const SysCtl& c, const Model& m) {
    return c.done || (!c.rebuild && lists_expired(c, m));
}

__device__ inline void relax_start(SysCtl& c, const Model& m) {
    c.fire_dt = m.dt0;
    c.fire_alpha = m.alpha0;
    c.npos = 0;
    c.k = 0;
    c.done = 0;
    c.converged = 0;
    c.updates = 0;
    c.evals = 0;
    c.stall = 0;
}

}  // namespace mxe
