// Neighbour lists, pair lists and nearest-neighbour bonds (cell binning).
//
// A pair interacts only if some quadrature node lies inside r_c, which needs
// |rbar| < r_c + reach: the farthest node of the 27-node product rule sits
// 3 s from the mean, that of the degree-3 rule sqrt(6) max(sigma_i, sigma_j).
// The list holds every pair with |rbar| < r_c + reach_build + skin, where
// reach_build uses both widths at the time of the build. The pair stays listed while
// 2 max|dq| + 3 sqrt(2) max(sigma - sigma_build, 0) <= skin over the system's
// sites, since |rbar| loses at most |dq_i| + |dq_j| and
// s <= s_build + sqrt(2) max(sigma - sigma_build, 0) (the degree-3 reach grows by
// less: sqrt(6) < 3 sqrt(2)). The FIRE update records both maxima; the build
// runs when their sum leaves the skin. Cells are as wide as the
// largest radius allowed by sigma_cap.
//
// Build chain per system (each kernel skips systems whose rebuild flag is 0):
//   k_bin        raises the system's flag when the lists may miss a pair; cell
//                of each site and its slot in the cell (atomic count)
//   k_cell_scan  per system: cell offsets (exclusive scan of the counts)
//   k_fill       place each site in its cell (order within a cell is not
//                deterministic; rows are sorted afterwards, so nothing depends on it)
//   k_nbr        one block per cell in use: the stencil's candidates staged in
//                LDS, one wave per site tests them; survivors are compacted by
//                ballot and sorted (bitonic, in registers); at the start of a
//                call also the bonds (same-type sites closer than r_bond, sorted);
//                per-chunk count of "upper" neighbours (larger index)
//   k_half       per chunk: offset of each site's first owned pair (each
//                unordered pair is owned by its lower site), from the upper
//                counts of the system's earlier chunks; the system's pair count;
//                clears the cell counts for the next build
//   k_pid        per site: pair id of every row entry (binary search in the
//                sorted row of the other end); pair endpoint arrays; clears the
//                chunk's upper count for the next build
//   k_build_done per system: clear the flag, count the build (within a
//                relaxation the following k_control does this instead)
#include "mxe_internal.h"

namespace mxe {

namespace {

__device__ inline int cell_coord(double u, double box, double w, int nc, bool periodic) {
    if (periodic) u -= box * floor(u / box);
    double v = u / w;
    if (!(v >= 0.0)) return 0;            // also catches NaN
    if (v >= (double)nc) return nc - 1;
    return (int)v;
}

__device__ inline void min_image(const SysDesc& S, double& dx, double& dy, double& dz) {
    if (S.periodic[0]) dx -= S.box[0] * rint(dx / S.box[0]);
    if (S.periodic[1]) dy -= S.box[1] * rint(dy / S.box[1]);
    if (S.periodic[2]) dz -= S.box[2] * rint(dz / S.box[2]);
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace and per-call initialisation
// ---------------------------------------------------------------------------
__global__ void k_fill_site_sys(Dev d) {
    for (int i = gtid(); i < d.n_sites; i += gstride()) {
        int lo = 0, hi = d.n_sys - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (d.sys[mid].site_off <= i) lo = mid; else hi = mid - 1;
        }
        d.site_sys[i] = lo;
    }
}

__global__ void k_zero_int(int* p, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) p[i] = 0;
}

void launch_ws_init(const Dev& d, hipStream_t s) {
    const int g = (int)std::min<int64_t>(4096, (d.n_sites + 255) / 256);
    k_fill_site_sys<<<g, 256, 0, s>>>(d);
    const int gc = (int)std::min<int64_t>(4096, (d.n_cells + 255) / 256);
    k_zero_int<<<gc, 256, 0, s>>>(d.cell_count, d.n_cells);
    k_zero_int<<<(d.n_chunks + 255) / 256, 256, 0, s>>>(d.chunk_up, d.n_chunks);
}

// advance (mxe_advance): systems keep their relaxation state, counters and
// step budget across calls; a system given a new budget (steps_new >= 0)
// starts afresh: counters cleared, a new relaxation, the budget set.
__global__ void k_sys_init(Dev d, Model m, int advance) {
    const int s = gtid();
    if (s >= d.n_sys) return;
    SysCtl& c = d.ctl[s];
    const SysDesc& S = d.sys[s];
    // A forced system rebuilds everything; otherwise its lists, pair count and
    // any pending rebuild request carry over from the previous call.
    if (S.force_build) {
        c.rebuild = 2;
        c.n_pairs = 0;
        c.drift_bits = 0ull;
        c.widen_bits = 0ull;
    }
    if (c.rebuild) d.acell[0].y = 1;  // the neighbour search runs
    if (advance && S.steps_new < 0) return;
    c.status = 0;
    c.n_rebuilds = 0;
    c.total_evals = 0;
    c.pair_evals = 0.0;
    c.done = 0;
    c.k = 0;
    c.stepping = 0;
    if (!advance) c.steps_left = 0;  // a call of the lockstep scheme ends any step budget
    if (advance) {
        relax_start(c, m);
        c.steps_left = S.n_sites > 0 ? S.steps_new : 0;
        c.done = c.steps_left > 0 ? 0 : 1;
        d.scalars[(int64_t)s * MXE_NSCALARS + MXE_S_STEPS_LEFT] = (double)c.steps_left;
    }
}

// widths, occupancies, positions and site temperatures are checked
__global__ __launch_bounds__(kChunk) void k_site_init(Dev d, Model m) {
    const Chunk ch = d.chunks[blockIdx.x];
    const int i = ch.start + threadIdx.x;
    int st = 0;
    if (i < ch.end) {
        const double sg = d.sigma[i];
        double xi = d.x[i];
        if (held(d, i, d.type[i], MXE_RES_FIX_X)) {  // held fraction (set at the call start)
            xi = d.res_val[i];
            d.x[i] = xi;
        }
        if (!(sg > 0.0) || !isfinite(sg)) st |= MXE_STAT_NONFINITE;
        if (sg > m.sigma_cap) st |= MXE_STAT_SIGMA_CAP;
        if (!isfinite(xi) || xi < -1e-12 || xi > 1.0 + 1e-12) st |= MXE_STAT_X_RANGE;
        if (!isfinite(d.qx[i]) || !isfinite(d.qy[i]) || !isfinite(d.qz[i])) st |= MXE_STAT_NONFINITE;
        if (d.T_site != nullptr && !(d.T_site[i] > 0.0 && isfinite(d.T_site[i]))) st |= MXE_STAT_TEMP;
        d.emit[i] = mixval(m.b4, d.type[i], xi);
    }
    if (st) atomicOr(&d.ctl[ch.sys].status, st);
}

void launch_sys_init(const Dev& d, const Model& m, hipStream_t s, int advance) {
    k_sys_init<<<(d.n_sys + 63) / 64, 64, 0, s>>>(d, m, advance);
    k_site_init<<<d.n_chunks, kChunk, 0, s>>>(d, m);
}

// ---------------------------------------------------------------------------
// Build chain
// ---------------------------------------------------------------------------
namespace {

__device__ inline int64_t site_cell(const SysDesc& S, double q0, double q1, double q2) {
    const int cx = cell_coord(q0, S.box[0], S.cell_w[0], S.nc[0], S.periodic[0]);
    const int cy = cell_coord(q1, S.box[1], S.cell_w[1], S.nc[1], S.periodic[1]);
    const int cz = cell_coord(q2, S.box[2], S.cell_w[2], S.nc[2], S.periodic[2]);
    return S.cell_off + ((int64_t)cx * S.nc[1] + cy) * S.nc[2] + cz;
}

// fixed-order exclusive scan over a 1024-thread block, one value per thread
__device__ inline int block_excl_scan_1024(int v, int* lds, int& total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        const int u = (t >= o) ? lds[t - o] : 0;
        __syncthreads();
        lds[t] += u;
        __syncthreads();
    }
    total = lds[1023];
    const int incl = lds[t];
    __syncthreads();
    return incl - v;
}

}  // namespace

// Decides whether the system's lists must be rebuilt (every block reads the
// same maxima and reaches the same decision), then bins the sites.
__global__ __launch_bounds__(kChunk) void k_bin(Dev d, Model m) {
    const Chunk ch = d.chunks[blockIdx.x];
    SysCtl& c = d.ctl[ch.sys];
    if (!c.rebuild) {
        if (!lists_expired(c, m)) return;
        if (threadIdx.x == 0) {  // the same values from every block
            c.rebuild = 1;
            d.acell[0].y = 1;
        }
    }
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    const SysDesc& S = d.sys[ch.sys];
    const double q0 = d.qx[i], q1 = d.qy[i], q2 = d.qz[i];
    d.qrx[i] = q0;
    d.qry[i] = q1;
    d.qrz[i] = q2;
    d.sref[i] = d.sigma[i];
    const int64_t cell = site_cell(S, q0, q1, q2);
    d.cell_of[i] = (int)cell;
    d.slot_of[i] = atomicAdd(&d.cell_count[cell], 1);
}

// Bins every site for a bonds-only build: the cells as k_bin forms them, but
// no rebuild decision and no change to the lists' reference positions.
__global__ __launch_bounds__(kChunk) void k_bond_bin(Dev d) {
    const Chunk ch = d.chunks[blockIdx.x];
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    const SysDesc& S = d.sys[ch.sys];
    const int64_t cell = site_cell(S, d.qx[i], d.qy[i], d.qz[i]);
    d.cell_of[i] = (int)cell;
    d.slot_of[i] = atomicAdd(&d.cell_count[cell], 1);
}

// One block per system: cell offsets into the per-system range of cell_sites.
// all: every system (the bonds-only build), else the systems being rebuilt.
__global__ __launch_bounds__(1024) void k_cell_scan(Dev d, int all) {
    __shared__ int lds[1024];
    const int s = blockIdx.x;
    if (!all && !d.ctl[s].rebuild) return;
    const SysDesc& S = d.sys[s];
    const int64_t nc = S.n_cells;
    const int per = (int)((nc + 1023) / 1024);
    const int64_t a = min(nc, (int64_t)threadIdx.x * per), b = min(nc, a + per);
    int sum = 0;
    for (int64_t c = a; c < b; ++c) sum += d.cell_count[S.cell_off + c];
    int total;
    int run = (int)S.site_off + block_excl_scan_1024(sum, lds, total);
    for (int64_t c = a; c < b; ++c) {
        d.cell_start[S.cell_off + c] = run;
        run += d.cell_count[S.cell_off + c];
    }
}

// Places each site in its cell and copies its position, width and type into
// the cell-ordered records, so candidates of one cell are contiguous in memory.
__global__ __launch_bounds__(kChunk) void k_fill(Dev d, int all) {
    const Chunk ch = d.chunks[blockIdx.x];
    if (!all && !d.ctl[ch.sys].rebuild) return;
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    const int pos = d.cell_start[d.cell_of[i]] + d.slot_of[i];
    d.cell_sites[pos] = i * 4 + d.type[i];
    d.cell_rec[pos] = make_double4(d.qx[i], d.qy[i], d.qz[i], d.sigma[i]);
}

// Cell of stencil offset (lane / 9 - 1, lane / 3 % 3 - 1, lane % 3 - 1) around the
// cell (c0, c1, c2), or -1 if it falls outside an open axis or repeats a cell an
// earlier offset already covers (periodic axes with fewer than three cells).
__device__ inline int64_t stencil_lane_cell(const SysDesc& S, const int c[3], int lane) {
    const int o[3] = {lane / 9 - 1, (lane / 3) % 3 - 1, lane % 3 - 1};
    int v[3];
    for (int a = 0; a < 3; ++a) {
        const int nc = S.nc[a];
        int w = c[a] + o[a];
        if (S.periodic[a]) {
            w = (w + nc) % nc;
            // keep the first offset (in the order -1, 0, +1) that reaches w
            for (int p = -1; p < o[a]; ++p)
                if ((c[a] + p + nc) % nc == w) return -1;
        } else if (w < 0 || w >= nc) {
            return -1;
        }
        v[a] = w;
    }
    return S.cell_off + ((int64_t)v[0] * S.nc[1] + v[1]) * S.nc[2] + v[2];
}

// Bitonic sort of 64 E ints held E per lane (element r * 64 + lane), ascending.
// Partners closer than 64 sit in other lanes (exchanged by shuffles), partners
// 64 or more apart in the same lane.
template <int E>
__device__ inline void wave_sort(int (&v)[E], int lane) {
    constexpr int N = kWave * E;
#pragma unroll
    for (int k = 2; k <= N; k <<= 1) {
#pragma unroll
        for (int j = k >> 1; j > 0; j >>= 1) {
            if (j >= kWave) {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int r2 = r ^ (j / kWave);
                    if (r2 > r) {
                        const bool asc = ((r * kWave + lane) & k) == 0;
                        const int a = v[r], b = v[r2];
                        const bool swap = (a > b) == asc;
                        v[r] = swap ? b : a;
                        v[r2] = swap ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int r = 0; r < E; ++r) {
                    const int o = __shfl_xor(v[r], j);
                    const bool lower = (lane & j) == 0;
                    const bool asc = ((r * kWave + lane) & k) == 0;
                    v[r] = (lower == asc) ? min(v[r], o) : max(v[r], o);
                }
            }
        }
    }
}

constexpr int kCellTile = 704;  // stencil candidates staged in LDS at a time (5 blocks per CU)
constexpr int kNbrGrid = 16384;  // blocks of the neighbour search at most

// One block per cell in use at a time. Every site of a cell has the same 27-cell stencil,
// so the block stages the stencil's candidates (site index and type, position
// and width) in LDS, kCellTile at a time, and its waves test the cell's sites
// against them, one site per wave and round. Per candidate and site the test
// is the list-radius test below; hits are compacted by ballot into an LDS row,
// which is sorted in registers (E entries per lane) and written out.
// The radius test is a superset test: the minimum image uses the reciprocal
// box length and s_ij an FP32 square root, and the radius is padded by 1e-6 A,
// so every pair the exact test admits is admitted (an extra pair whose nodes
// all lie beyond r_c contributes exact zeros). Rows are sorted, so they do not
// depend on the order of the sites within a cell.
template <int E>
__global__ __launch_bounds__(kChunk) void k_nbr(Dev d, Model m, int bonds, int bonds_only) {
    constexpr int K2 = kWave * E;
    constexpr int kWaves = kChunk / kWave;
    __shared__ int rows[kWaves][K2];
    __shared__ int brows[kWaves][kWave];  // bond partners of each wave's site
    __shared__ int tj[kCellTile];        // 4 * site index + type
    __shared__ double4 trec[kCellTile];  // position and width
    __shared__ int st_start[27], st_pre[28];  // stencil cells: first record, prefix of counts
    __shared__ int sh_center;                 // prefix of the cell itself in the stencil
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    // The cells in use (count read from the table) are dealt to the XCDs in
    // contiguous ranges; the blocks of an XCD stride through their range.
    // With no system rebuilding, every block leaves after one load.
    const int2 a0 = d.acell[0];
    if (a0.y == 0 && !bonds_only) return;
    const int na = a0.x;
    const int per = (na + kXcd - 1) / kXcd;
    const int x0 = (int)(blockIdx.x % kXcd) * per, x1 = min(na, x0 + per);
    const int nq = (int)gridDim.x / kXcd;
    for (int b = x0 + (int)(blockIdx.x / kXcd); b < x1; b += nq) {
        const int2 ac = d.acell[1 + b];
        const int s = ac.x, g = ac.y;
        if (!bonds_only && !d.ctl[s].rebuild) continue;
        const int nsite = d.cell_count[g];
        if (nsite == 0) continue;  // both skips are uniform over the block
        const SysDesc& S = d.sys[s];
        // bonds of other systems are kept, except in a bonds-only build (all systems)
        const bool sys_bonds = bonds_only != 0 || (bonds != 0 && S.force_build != 0);
        __syncthreads();  // the previous cell's tile and stencil are no longer read
        if (wave == 0) {
            const int lc = g - (int)S.cell_off;
            const int c[3] = {lc / (S.nc[1] * S.nc[2]), (lc / S.nc[2]) % S.nc[1], lc % S.nc[2]};
            int cnt = 0, start = 0;
            bool center = false;
            if (lane < 27) {
                const int64_t cell = stencil_lane_cell(S, c, lane);
                if (cell >= 0) {
                    cnt = d.cell_count[cell];
                    start = d.cell_start[cell];
                    center = cell == g;
                }
            }
            int incl = cnt;  // inclusive wave scan of the counts (lanes >= 27 hold zero)
#pragma unroll
            for (int o = 1; o < 32; o <<= 1) {
                const int u = __shfl_up(incl, o);
                if (lane >= o) incl += u;
            }
            if (lane < 27) {
                st_start[lane] = start;
                st_pre[lane] = incl - cnt;
            }
            if (lane == 26) st_pre[27] = incl;
            // the cell itself is one of the stencil cells (the first offset reaching it)
            const int cl = __ffsll((long long)__ballot(center)) - 1;
            const int cpre = __shfl(incl - cnt, cl);
            if (lane == 0) sh_center = cpre;
        }
        __syncthreads();
        const int T = st_pre[27];
        const int ntiles = (T + kCellTile - 1) / kCellTile;
        const double reach = m.r_c + m.skin + 1e-6;
        const bool d3 = m.quad_rule == MXE_QUAD_DEGREE3;
        const double ib0 = 1.0 / S.box[0], ib1 = 1.0 / S.box[1], ib2 = 1.0 / S.box[2];
        // minimum image: periodic axes subtract box * rint(d / box), open axes nothing
        const double pb0 = S.periodic[0] ? S.box[0] : 0.0, pb1 = S.periodic[1] ? S.box[1] : 0.0,
                     pb2 = S.periodic[2] ? S.box[2] : 0.0;
        const int K = d.K;
        int* row = rows[wave];
        bool over = false, bond_over = false;

        // stage candidates [t0, t1) of the stencil into the tile (whole block); a
        // thread past t1 loads candidate t0 (always valid) and stores nothing
        auto stage = [&](int t0, int t1) {
            constexpr int kPer = (kCellTile + kChunk - 1) / kChunk;  // entries per thread
            int pos[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = t0 + u * kChunk + (int)threadIdx.x;
                const int ec = e < t1 ? e : t0;
                int L = 0;  // stencil cell holding candidate ec: last L with st_pre[L] <= ec
#pragma unroll
                for (int step = 16; step > 0; step >>= 1)
                    if (L + step < 27 && st_pre[L + step] <= ec) L += step;
                pos[u] = st_start[L] + (ec - st_pre[L]);
            }
            int jt[kPer];
            double4 rj[kPer];
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                jt[u] = d.cell_sites[pos[u]];
                rj[u] = d.cell_rec[pos[u]];
            }
#pragma unroll
            for (int u = 0; u < kPer; ++u) {
                const int e = u * kChunk + (int)threadIdx.x;
                if (t0 + e < t1) {
                    tj[e] = jt[u];
                    trec[e] = rj[u];
                }
            }
        };

        if (ntiles == 1) {
            stage(0, T);
            __syncthreads();
        }
        for (int r0 = 0; r0 < nsite; r0 += kWaves) {
            const int k = r0 + wave;  // this wave's site of the cell in this round
            const bool has = k < nsite;
            int i = 0, ti = 0;
            double qi0 = 0.0, qi1 = 0.0, qi2 = 0.0, si2 = 0.0;
            float sig_i = 0.0f;
            if (has) {
                int jt;
                double4 ri;
                if (ntiles == 1) {  // the cell's own records lie in the staged stencil
                    jt = tj[sh_center + k];
                    ri = trec[sh_center + k];
                } else {
                    const int pos = d.cell_start[g] + k;
                    jt = d.cell_sites[pos];
                    ri = d.cell_rec[pos];
                }
                i = jt >> 2;
                ti = jt & 3;
                qi0 = ri.x;
                qi1 = ri.y;
                qi2 = ri.z;
                si2 = ri.w * ri.w;
                sig_i = (float)ri.w;
            }
            // bonds of a mobile site: same-type sites closer than r_bond, by the
            // exact FP64 distance (minimum image by division)
            const bool site_bonds = sys_bonds && has && occ_mobile(ti);
            int* brow = brows[wave];
            int n = 0, nb = 0;
            for (int t = 0; t < ntiles; ++t) {
                const int t0 = t * kCellTile, t1 = min(T, t0 + kCellTile);
                if (ntiles > 1) {
                    __syncthreads();  // every wave is done with the previous tile
                    stage(t0, t1);
                    __syncthreads();
                }
                if (!has) continue;
                for (int base = 0; base < t1 - t0; base += kWave) {
                    const int e = base + lane;
                    const bool in = e < t1 - t0;
                    const int jt = tj[in ? e : 0];
                    const double4 rj = trec[in ? e : 0];
                    const int j = jt >> 2;
                    double dx = rj.x - qi0, dy = rj.y - qi1, dz = rj.z - qi2;
                    dx -= pb0 * rint(dx * ib0);
                    dy -= pb1 * rint(dy * ib1);
                    dz -= pb2 * rint(dz * ib2);
                    // the rule's farthest node from the mean: 3 s under the product
                    // rule, sqrt(6) max(sigma_i, sigma_j) under the degree-3 rule
                    const double rl =
                        reach + (d3 ? 2.449489742783178 * (double)fmaxf(sig_i, (float)rj.w)
                                    : 3.0 * (double)__builtin_sqrtf((float)(si2 + rj.w * rj.w)));
                    const bool ok = !bonds_only & in & (j != i) & (pair_cls(ti, jt & 3) >= 0) &
                                    (dx * dx + dy * dy + dz * dz < rl * rl);
                    const unsigned long long mask = __ballot(ok);
                    const int pos = n + __popcll(mask & __lanemask_lt());
                    if (ok && pos < K2) row[pos] = j;
                    n += __popcll(mask);
                    if (site_bonds) {  // uniform over the wave
                        double bx = rj.x - qi0, by = rj.y - qi1, bz = rj.z - qi2;
                        min_image(S, bx, by, bz);
                        const bool okb = in & (j != i) & ((jt & 3) == ti) &
                                         (bx * bx + by * by + bz * bz < m.r_bond * m.r_bond);
                        const unsigned long long bmask = __ballot(okb);
                        const int bpos = nb + __popcll(bmask & __lanemask_lt());
                        if (okb && bpos < kWave) brow[bpos] = j;
                        nb += __popcll(bmask);
                    }
                }
            }
            if (has) {
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
                if (!bonds_only) {  // the row (not in a bonds-only build)
                    if (n > K) over = true;
                    const int nk = min(n, K);
                    int lo = 0;
                    int* out = d.nbr + (int64_t)i * K;
                    if (E > 1 && n <= kWave) {  // a short row: one entry per lane suffices
                        int v[1] = {lane < n ? row[lane] : 0x7fffffff};
                        wave_sort<1>(v, lane);
                        if (lane < nk) {
                            out[lane] = v[0];
                            lo += (v[0] < i);
                        }
                    } else {
                        int v[E];
    #pragma unroll
                        for (int r = 0; r < E; ++r) {
                            const int t = r * kWave + lane;
                            v[r] = t < min(n, K2) ? row[t] : 0x7fffffff;
                        }
                        wave_sort<E>(v, lane);
    #pragma unroll
                        for (int r = 0; r < E; ++r) {
                            const int t = r * kWave + lane;
                            if (t < nk) {
                                out[t] = v[r];
                                lo += (v[r] < i);
                            }
                        }
                    }
    #pragma unroll
                    for (int o = 32; o > 0; o >>= 1) lo += __shfl_xor(lo, o);
                    if (lane == 0) {
                        d.nbr_cnt[i] = nk;
                        d.nbr_lo[i] = lo;
                        // owned pairs per site chunk (an integer sum: order-independent)
                        atomicAdd(&d.chunk_up[S.chunk_first + (i - (int)S.site_off) / kChunk], nk - lo);
                    }
                }
                if (sys_bonds) {  // uniform over the wave
                    const int B = d.bond_max, nbk = min(nb, B);
                    if (nb > B) bond_over = true;
                    int v[1] = {lane < min(nb, kWave) ? brow[lane] : 0x7fffffff};
                    wave_sort<1>(v, lane);
                    if (lane < nbk) d.bond[(int64_t)i * B + lane] = v[0];
                    if (lane == 0) d.nbond[i] = nbk;
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
        }
        if (lane == 0 && over) atomicOr(&d.ctl[s].status, MXE_STAT_KMAX);
        if (lane == 0 && bond_over) atomicOr(&d.ctl[s].status, MXE_STAT_BONDS);
    }
}

// Per chunk: each site's first owned pair = chunk offset + in-chunk prefix.
__global__ __launch_bounds__(kChunk) void k_half(Dev d) {
    __shared__ int lds[kChunk];
    __shared__ int wsum[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    SysCtl& c = d.ctl[ch.sys];
    if (!c.rebuild) return;
    const SysDesc& S = d.sys[ch.sys];
    const int t = threadIdx.x, lane = t & (kWave - 1), wave = t / kWave;
    // the chunk's first owned pair: the upper counts of the system's earlier
    // chunks (an integer sum, so its order does not matter)
    const int b = (int)blockIdx.x - S.chunk_first;
    int pre = 0;
    for (int k = t; k < b; k += kChunk) pre += d.chunk_up[S.chunk_first + k];
#pragma unroll
    for (int o = kWave / 2; o > 0; o >>= 1) pre += __shfl_xor(pre, o);
    if (lane == 0) wsum[wave] = pre;
    // the cell counts are not read again in this build: clear them for the next
    for (int64_t cc = (int64_t)b * kChunk + t; cc < S.n_cells; cc += (int64_t)S.n_chunks * kChunk)
        d.cell_count[S.cell_off + cc] = 0;
    __syncthreads();
    int chunk_off = 0;
    for (int w = 0; w < kChunk / kWave; ++w) chunk_off += wsum[w];
    if (t == 0 && b == S.n_chunks - 1) {  // the system's last chunk: its pair count
        const int total = chunk_off + d.chunk_up[blockIdx.x];
        c.n_pairs = total;
        if (total > S.pair_cap) atomicOr(&c.status, MXE_STAT_PAIRS);
    }
    const int i = ch.start + t;
    const int u = i < ch.end ? d.nbr_cnt[i] - d.nbr_lo[i] : 0;
    lds[t] = u;
    __syncthreads();
    for (int o = 1; o < kChunk; o <<= 1) {
        const int v = (t >= o) ? lds[t - o] : 0;
        __syncthreads();
        lds[t] += v;
        __syncthreads();
    }
    if (i < ch.end) d.half_off[i] = chunk_off + lds[t] - u;
}

// One wavefront per site, lanes over its row: the pair id of an entry (i, j)
// is owned by the lower site; for j < i it is found by binary search of i in
// j's sorted row (i lies in j's upper part). The searches are chains of
// scattered loads and the kernel needs few registers, so a chunk's block has
// kPidThreads threads to keep more rows in flight (a scan of j's upper part
// with 16-B loads, one round trip, measured slower: 190 -> 250-307 us).
constexpr int kPidThreads = 2 * kChunk;

__global__ __launch_bounds__(kPidThreads) void k_pid(Dev d) {
    const int cb = xcd_chunk(d.n_chunks);
    if (cb >= d.n_chunks) return;
    const Chunk ch = d.chunks[cb];
    const int s = ch.sys;
    if (!d.ctl[s].rebuild) return;
    const SysDesc& S = d.sys[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int K = d.K;
    bool bad = false;
    if (threadIdx.x == 0) d.chunk_up[cb] = 0;  // read for the last time by k_half: the next build counts afresh
    for (int i = ch.start + wave; i < ch.end; i += kPidThreads / kWave) {
        const int cnt = d.nbr_cnt[i], lo = d.nbr_lo[i], hoff = d.half_off[i];
        const int* row = d.nbr + (int64_t)i * K;
        int* prow = d.pid + (int64_t)i * K;
        for (int k = lane; k < cnt; k += kWave) {
            const int j = row[k];
            int local;
            if (j > i) {
                local = hoff + (k - lo);
                if (local < S.pair_cap) {
                    const int64_t p = S.pair_base + local;
                    d.pair_i[p] = i;
                    d.pair_j[p] = j;
                }
            } else {
                // i > j lies in j's upper part [lo_j, cnt_j): search only there
                const int* rj = d.nbr + (int64_t)j * K;
                const int cj = d.nbr_cnt[j], lj = d.nbr_lo[j];
                int l = lj, h = cj;
                while (l < h) {
                    const int mid = (l + h) >> 1;
                    if (rj[mid] < i) l = mid + 1; else h = mid;
                }
                if (l >= cj || rj[l] != i) {
                    bad = true;
                    prow[k] = -1;
                    continue;
                }
                local = d.half_off[j] + (l - lj);
            }
            prow[k] = (local < S.pair_cap) ? (int)(S.pair_base + local) : -1;
        }
    }
    if (bad) atomicOr(&d.ctl[s].status, MXE_STAT_KMAX);
}

// Pair numbering by geometric class. Within each pair chunk the pairs are
// renumbered so that pairs of one class are consecutive: the distance |rbar|
// in 0.25-A bins, the octant of rbar and its dominant axis. A wavefront of the
// pair kernel then holds pairs of similar geometry, whose quadrature nodes
// take the same branches (inside or beyond r_c, inside or within the taper),
// so whole wavefronts skip nodes beyond r_c and the taper polynomial where no
// pair needs them. The pair endpoints are permuted in place (each block reads
// its whole chunk before writing it) and the new number of each old pair goes
// to pnew, from which k_pid_remap rewrites the rows' pair ids. Numbers within
// a bucket come from LDS atomics: the assignment of numbers may vary from run
// to run, but each pair's moments do not depend on its number, and every
// gather sums over its row in row order, so results are unchanged.
constexpr int kPairBins = 32 * 24;
// One kChunk-thread block per pair chunk: a thread takes pairs kOrderThreads
// apart, so a bucket keeps the pairs of neighbouring sites close together. A
// 512-thread block renumbers faster (89 -> 79 us on a 256k-site system) but the
// density gather then reads its pairs with less reuse (170 -> 176 us per
// evaluation), which costs more than a build saves.
constexpr int kOrderThreads = kChunk;

__global__ __launch_bounds__(kOrderThreads) void k_pair_order(Dev d) {
    __shared__ int cnt[kPairBins], start[kPairBins], wsum[kOrderThreads / kWave];
    const Chunk ch = d.pchunks[blockIdx.x];
    const SysCtl& c = d.ctl[ch.sys];
    if (!c.rebuild) return;
    const SysDesc& S = d.sys[ch.sys];
    const int64_t pend = min((int64_t)ch.end, S.pair_base + min((int64_t)c.n_pairs, S.pair_cap));
    if (pend <= ch.start) return;
    for (int b = threadIdx.x; b < kPairBins; b += blockDim.x) cnt[b] = 0;
    __syncthreads();
    constexpr int kPer = kPairChunk / kOrderThreads;
    int key[kPer], pi[kPer], pj[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        const int64_t p = ch.start + (int64_t)u * kOrderThreads + threadIdx.x;
        key[u] = -1;
        pi[u] = pj[u] = 0;
        if (p < pend) {
            const int i = d.pair_i[p], j = d.pair_j[p];
            pi[u] = i;
            pj[u] = j;
            double rx = d.qx[j] - d.qx[i], ry = d.qy[j] - d.qy[i], rz = d.qz[j] - d.qz[i];
            min_image(S, rx, ry, rz);
            const double ax = fabs(rx), ay = fabs(ry), az = fabs(rz);
            const double db = sqrt(rx * rx + ry * ry + rz * rz) * 4.0;
            const int rb = (db >= 0.0 && db < 31.0) ? (int)db : 31;  // a NaN position lands in bin 31
            const int oct = (rx < 0.0 ? 4 : 0) + (ry < 0.0 ? 2 : 0) + (rz < 0.0 ? 1 : 0);
            const int dom = (ax >= ay && ax >= az) ? 0 : (ay >= az ? 1 : 2);
            key[u] = rb * 24 + oct * 3 + dom;
            atomicAdd(&cnt[key[u]], 1);
        }
    }
    __syncthreads();
    {  // exclusive prefix of the bin counts: kBinsPerT consecutive bins per
       // thread, a wave scan of the thread totals, then the waves' totals
        constexpr int kBinsPerT = (kPairBins + kOrderThreads - 1) / kOrderThreads;
        const int lane = threadIdx.x & (kWave - 1), wave = threadIdx.x / kWave;
        int c[kBinsPerT], tot = 0;
#pragma unroll
        for (int u = 0; u < kBinsPerT; ++u) {
            const int b = threadIdx.x * kBinsPerT + u;
            c[u] = b < kPairBins ? cnt[b] : 0;
            tot += c[u];
        }
        int incl = tot;
#pragma unroll
        for (int o = 1; o < kWave; o <<= 1) {
            const int v = __shfl_up(incl, o);
            if (lane >= o) incl += v;
        }
        if (lane == kWave - 1) wsum[wave] = incl;
        __syncthreads();
        int run = incl - tot;
        for (int w = 0; w < wave; ++w) run += wsum[w];
#pragma unroll
        for (int u = 0; u < kBinsPerT; ++u) {
            const int b = threadIdx.x * kBinsPerT + u;
            if (b < kPairBins) start[b] = run;
            run += c[u];
        }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
        if (key[u] < 0) continue;
        const int64_t p = ch.start + (int64_t)u * kOrderThreads + threadIdx.x;
        const int64_t t = ch.start + atomicAdd(&start[key[u]], 1);
        d.pair_i[t] = pi[u];
        d.pair_j[t] = pj[u];
        d.pnew[p] = (int)t;
    }
}

// Rows' pair ids follow the renumbering of k_pair_order.
__global__ __launch_bounds__(kPidThreads) void k_pid_remap(Dev d) {
    const int cb = xcd_chunk(d.n_chunks);
    if (cb >= d.n_chunks) return;
    const Chunk ch = d.chunks[cb];
    if (!d.ctl[ch.sys].rebuild) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int K = d.K;
    for (int i = ch.start + wave; i < ch.end; i += kPidThreads / kWave) {
        const int cnt = d.nbr_cnt[i];
        int* prow = d.pid + (int64_t)i * K;
        for (int k = lane; k < cnt; k += kWave) {
            const int p = prow[k];
            if (p >= 0) prow[k] = d.pnew[p];
        }
    }
}

__global__ void k_build_done(Dev d) {
    const int s = gtid();
    if (s < d.n_sys) finish_build(d, s);
}

int row_pow2(int K) {
    int k2 = 64;
    while (k2 < K) k2 <<= 1;
    return k2;
}

void launch_nbr(const Dev& d, const Model& m, int bonds, int bonds_only, hipStream_t s) {
    const int gc = std::min(xcd_grid((int)d.n_cells), kNbrGrid);
    switch (row_pow2(d.K)) {
        case 64: k_nbr<1><<<gc, kChunk, 0, s>>>(d, m, bonds, bonds_only); break;
        case 128: k_nbr<2><<<gc, kChunk, 0, s>>>(d, m, bonds, bonds_only); break;
        default: k_nbr<4><<<gc, kChunk, 0, s>>>(d, m, bonds, bonds_only); break;
    }
}

// The bonds of every system from the current positions, lists untouched: the
// cells are binned and filled afresh (the cell counts start at zero, as at
// every call) and the neighbour search only collects the bonds.
void launch_bonds(const Dev& d, const Model& m, hipStream_t s) {
    k_bond_bin<<<d.n_chunks, kChunk, 0, s>>>(d);
    k_cell_scan<<<d.n_sys, 1024, 0, s>>>(d, 1);
    k_fill<<<d.n_chunks, kChunk, 0, s>>>(d, 1);
    launch_nbr(d, m, 1, 1, s);
}

void launch_build(const Dev& d, const Model& m, bool bonds, bool finish, hipStream_t s) {
    k_bin<<<d.n_chunks, kChunk, 0, s>>>(d, m);
    k_cell_scan<<<d.n_sys, 1024, 0, s>>>(d, 0);
    k_fill<<<d.n_chunks, kChunk, 0, s>>>(d, 0);
    launch_nbr(d, m, bonds ? 1 : 0, 0, s);
    k_half<<<d.n_chunks, kChunk, 0, s>>>(d);
    k_pid<<<xcd_grid(d.n_chunks), kPidThreads, 0, s>>>(d);
    k_pair_order<<<d.n_pchunks, kOrderThreads, 0, s>>>(d);
    k_pid_remap<<<xcd_grid(d.n_chunks), kPidThreads, 0, s>>>(d);
    if (finish) k_build_done<<<(d.n_sys + 63) / 64, 64, 0, s>>>(d);
}

}  // namespace mxe
