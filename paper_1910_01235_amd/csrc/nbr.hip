// Neighbour lists, pair lists and nearest-neighbour bonds (cell binning).
//
// A pair interacts only if some quadrature node lies inside r_c, which needs
// |rbar| < r_c + 3 s (the farthest node of the rule sits 3 s from the mean).
// The list holds every pair with |rbar| < r_c + 3 s_build + skin, where s_build
// uses both widths at the time of the build. The pair stays listed while
// 2 max|dq| + 3 sqrt(2) max(sigma - sigma_build) <= skin, since
// s <= s_build + sqrt(2) max(sigma - sigma_build); each site checks its own share
// (|dq| <= skin/4, 3 sqrt(2) (sigma - sigma_build) <= skin/2) and requests a
// rebuild of its system otherwise. Cells are as wide as the largest radius
// allowed by sigma_cap.
//
// Build chain per system (each kernel skips systems whose rebuild flag is 0):
//   k_bin        cell of each site and its slot in the cell (atomic count)
//   k_cell_scan  per system: cell offsets (exclusive scan of the counts)
//   k_fill       place each site in its cell
//   k_sort_cells sort each cell by site index (deterministic order)
//   k_nbr        one wavefront per site: lanes test the stencil's candidates,
//                survivors are compacted by ballot and sorted (bitonic, in LDS);
//                per-chunk count of "upper" neighbours (larger index)
//   k_bonds      per mobile site: same-type sites closer than r_bond (sorted)
//   k_scan       per system: offsets of the chunks' upper counts; pair count;
//                clears the cell counts for the next build
//   k_half       per chunk: offset of each site's first owned pair (each
//                unordered pair is owned by its lower site)
//   k_pid        per site: pair id of every row entry (binary search in the
//                sorted row of the other end); pair endpoint arrays
//   k_build_done per system: clear the flag, count the build
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

// distinct cell indices of the 3-wide stencil along one axis
__device__ inline int stencil_axis(int c, int nc, bool periodic, int out[3]) {
    int n = 0;
    for (int o = -1; o <= 1; ++o) {
        int v = c + o;
        if (periodic) {
            v = (v + nc) % nc;
        } else if (v < 0 || v >= nc) {
            continue;
        }
        bool dup = false;
        for (int k = 0; k < n; ++k) dup |= (out[k] == v);
        if (!dup) out[n++] = v;
    }
    return n;
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
}

__global__ void k_sys_init(Dev d) {
    const int s = gtid();
    if (s >= d.n_sys) return;
    SysCtl& c = d.ctl[s];
    c.sigmax_bits = 0ull;
    c.rebuild = 1;
    c.status = 0;
    c.n_rebuilds = 0;
    c.total_evals = 0;
    c.pair_evals = 0.0;
    c.done = 0;
    c.k = 0;
    c.n_pairs = 0;
}

// widths and occupancies are checked, and the largest width recorded
__global__ __launch_bounds__(kChunk) void k_site_init(Dev d, Model m) {
    __shared__ double red[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    const int i = ch.start + threadIdx.x;
    double sg = 0.0;
    int st = 0;
    if (i < ch.end) {
        sg = d.sigma[i];
        const double xi = d.x[i];
        if (!(sg > 0.0) || !isfinite(sg)) st |= MXE_STAT_NONFINITE;
        if (sg > m.sigma_cap) st |= MXE_STAT_SIGMA_CAP;
        if (!isfinite(xi) || xi < -1e-12 || xi > 1.0 + 1e-12) st |= MXE_STAT_X_RANGE;
        if (!isfinite(d.qx[i]) || !isfinite(d.qy[i]) || !isfinite(d.qz[i])) st |= MXE_STAT_NONFINITE;
        if (!(sg > 0.0)) sg = 0.0;
    }
    if (st) atomicOr(&d.ctl[ch.sys].status, st);
    double v = sg;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double mx = red[0];
        for (int w = 1; w < kChunk / kWave; ++w) mx = fmax(mx, red[w]);
        atomicMax(&d.ctl[ch.sys].sigmax_bits, (unsigned long long)__double_as_longlong(mx));
    }
}

void launch_sys_init(const Dev& d, const Model& m, hipStream_t s) {
    k_sys_init<<<(d.n_sys + 63) / 64, 64, 0, s>>>(d);
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

// the up-to-27 distinct cells around site position q (stencil order)
__device__ inline int stencil_cells(const SysDesc& S, double q0, double q1, double q2, int64_t cells[27]) {
    int cx[3], cy[3], cz[3];
    const int nx = stencil_axis(cell_coord(q0, S.box[0], S.cell_w[0], S.nc[0], S.periodic[0]), S.nc[0], S.periodic[0], cx);
    const int ny = stencil_axis(cell_coord(q1, S.box[1], S.cell_w[1], S.nc[1], S.periodic[1]), S.nc[1], S.periodic[1], cy);
    const int nz = stencil_axis(cell_coord(q2, S.box[2], S.cell_w[2], S.nc[2], S.periodic[2]), S.nc[2], S.periodic[2], cz);
    int n = 0;
    for (int a = 0; a < nx; ++a)
        for (int b = 0; b < ny; ++b)
            for (int c = 0; c < nz; ++c)
                cells[n++] = S.cell_off + ((int64_t)cx[a] * S.nc[1] + cy[b]) * S.nc[2] + cz[c];
    return n;
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

__global__ __launch_bounds__(kChunk) void k_bin(Dev d) {
    const Chunk ch = d.chunks[blockIdx.x];
    if (!d.ctl[ch.sys].rebuild) return;
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

// One block per system: cell offsets into the per-system range of cell_sites.
__global__ __launch_bounds__(1024) void k_cell_scan(Dev d) {
    __shared__ int lds[1024];
    const int s = blockIdx.x;
    if (!d.ctl[s].rebuild) return;
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

__global__ __launch_bounds__(kChunk) void k_fill(Dev d) {
    const Chunk ch = d.chunks[blockIdx.x];
    if (!d.ctl[ch.sys].rebuild) return;
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    d.cell_sites[d.cell_start[d.cell_of[i]] + d.slot_of[i]] = i;
}

__global__ void k_sort_cells(Dev d) {
    for (int64_t cell = gtid(); cell < d.n_cells; cell += gstride()) {
        const int s = find_sys_cell(d.sys, d.n_sys, cell);
        if (!d.ctl[s].rebuild) continue;
        const int n = d.cell_count[cell];
        int* c = d.cell_sites + d.cell_start[cell];
        for (int a = 1; a < n; ++a) {
            const int v = c[a];
            int b = a - 1;
            while (b >= 0 && c[b] > v) {
                c[b + 1] = c[b];
                --b;
            }
            c[b + 1] = v;
        }
    }
}

// One wavefront per site. The wave walks the stencil's candidates as one flat
// list (lane-strided), keeps those within the pair's list radius, compacts
// them into an LDS row by ballot, then sorts the row by site index.
__global__ __launch_bounds__(kChunk) void k_nbr(Dev d, Model m, int K2) {
    extern __shared__ int lds_rows[];  // kChunk / kWave rows of K2 entries
    __shared__ int cstart[kChunk / kWave][28], cpre[kChunk / kWave][28];
    __shared__ int wave_up[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    const int s = ch.sys;
    if (!d.ctl[s].rebuild) return;
    const SysDesc& S = d.sys[s];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    int* row = lds_rows + wave * K2;
    const int K = d.K;
    const double reach = m.r_c + m.skin;
    int up_sum = 0;
    bool over = false;
    for (int i = ch.start + wave; i < ch.end; i += kChunk / kWave) {
        const double qi0 = d.qx[i], qi1 = d.qy[i], qi2 = d.qz[i];
        const double si2 = d.sigma[i] * d.sigma[i];
        const int ti = d.type[i];
        int64_t cells[27];
        const int nc = stencil_cells(S, qi0, qi1, qi2, cells);
        if (lane == 0) {
            int acc = 0;
            for (int c = 0; c < nc; ++c) {
                cstart[wave][c] = d.cell_start[cells[c]];
                cpre[wave][c] = acc;
                acc += d.cell_count[cells[c]];
            }
            cpre[wave][nc] = acc;
        }
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        const int total = cpre[wave][nc];
        int n = 0;
        for (int base = 0; base < total; base += kWave) {
            const int e = base + lane;
            bool ok = false;
            int j = 0;
            if (e < total) {
                int c = 0;
                while (cpre[wave][c + 1] <= e) ++c;
                j = d.cell_sites[cstart[wave][c] + (e - cpre[wave][c])];
                if (j != i && pair_cls(ti, d.type[j]) >= 0) {
                    double dx = d.qx[j] - qi0, dy = d.qy[j] - qi1, dz = d.qz[j] - qi2;
                    min_image(S, dx, dy, dz);
                    const double sj = d.sigma[j];
                    const double rl = reach + 3.0 * sqrt(si2 + sj * sj);
                    ok = dx * dx + dy * dy + dz * dz < rl * rl;
                }
            }
            const unsigned long long mask = __ballot(ok);
            const int pos = n + __popcll(mask & __lanemask_lt());
            if (ok && pos < K2) row[pos] = j;
            n += __popcll(mask);
        }
        if (n > K) over = true;
        const int nk = min(n, K);
        for (int k = nk + lane; k < K2; k += kWave) row[k] = 0x7fffffff;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
        // bitonic sort of the K2-entry row (ascending)
        for (int kk = 2; kk <= K2; kk <<= 1) {
            for (int jj = kk >> 1; jj > 0; jj >>= 1) {
                for (int t = lane; t < K2; t += kWave) {
                    const int u = t ^ jj;
                    if (u > t) {
                        const int a = row[t], b = row[u];
                        const bool asc = (t & kk) == 0;
                        if ((a > b) == asc) {
                            row[t] = b;
                            row[u] = a;
                        }
                    }
                }
                __builtin_amdgcn_wave_barrier();
                __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
            }
        }
        int lo = 0;
        int* out = d.nbr + (int64_t)i * K;
        for (int k = lane; k < nk; k += kWave) {
            const int j = row[k];
            out[k] = j;
            lo += (j < i);
        }
        lo = (int)wave_sum((double)lo);
        if (lane == 0) {
            d.nbr_cnt[i] = nk;
            d.nbr_lo[i] = lo;
        }
        up_sum += nk - lo;
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "wavefront");
    }
    if (lane == 0) {
        wave_up[wave] = up_sum;
        if (over) atomicOr(&d.ctl[s].status, MXE_STAT_KMAX);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0;
        for (int w = 0; w < kChunk / kWave; ++w) t += wave_up[w];
        d.chunk_up[blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(kChunk) void k_bonds(Dev d, Model m) {
    const Chunk ch = d.chunks[blockIdx.x];
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    const int s = ch.sys;
    const SysDesc& S = d.sys[s];
    const int B = d.bond_max;
    const int ti = d.type[i];
    int n = 0;
    bool over = false;
    int* out = d.bond + (int64_t)i * B;
    if (occ_mobile(ti)) {
        const double rb2 = m.r_bond * m.r_bond;
        const double qi0 = d.qx[i], qi1 = d.qy[i], qi2 = d.qz[i];
        int64_t cells[27];
        const int nc = stencil_cells(S, qi0, qi1, qi2, cells);
        for (int c = 0; c < nc; ++c) {
            const int cn = d.cell_count[cells[c]];
            const int* cs = d.cell_sites + d.cell_start[cells[c]];
            for (int e = 0; e < cn; ++e) {
                const int j = cs[e];
                if (j == i || d.type[j] != ti) continue;
                double dx = d.qx[j] - qi0, dy = d.qy[j] - qi1, dz = d.qz[j] - qi2;
                min_image(S, dx, dy, dz);
                if (dx * dx + dy * dy + dz * dz >= rb2) continue;
                if (n >= B) {
                    over = true;
                    continue;
                }
                int p = n;
                while (p > 0 && out[p - 1] > j) {
                    out[p] = out[p - 1];
                    --p;
                }
                out[p] = j;
                ++n;
            }
        }
    }
    d.nbond[i] = n;
    if (over) atomicOr(&d.ctl[s].status, MXE_STAT_BONDS);
}

// One block per system: offsets of the chunks' owned-pair counts, the pair
// count, and cleared cell counts for the next build.
__global__ __launch_bounds__(1024) void k_scan(Dev d) {
    __shared__ int lds[1024];
    const int s = blockIdx.x;
    if (!d.ctl[s].rebuild) return;
    const SysDesc& S = d.sys[s];
    const int nch = S.n_chunks;
    const int per = (nch + 1023) / 1024;
    const int a = min(nch, (int)threadIdx.x * per), b = min(nch, a + per);
    int sum = 0;
    for (int c = a; c < b; ++c) sum += d.chunk_up[S.chunk_first + c];
    int total;
    int run = block_excl_scan_1024(sum, lds, total);
    for (int c = a; c < b; ++c) {
        d.chunk_off[S.chunk_first + c] = run;
        run += d.chunk_up[S.chunk_first + c];
    }
    if (threadIdx.x == 0) {
        d.ctl[s].n_pairs = total;
        if (total > S.pair_cap) atomicOr(&d.ctl[s].status, MXE_STAT_PAIRS);
    }
    for (int64_t c = S.cell_off + threadIdx.x; c < S.cell_off + S.n_cells; c += 1024) d.cell_count[c] = 0;
}

// Per chunk: each site's first owned pair = chunk offset + in-chunk prefix.
__global__ __launch_bounds__(kChunk) void k_half(Dev d) {
    __shared__ int lds[kChunk];
    const Chunk ch = d.chunks[blockIdx.x];
    if (!d.ctl[ch.sys].rebuild) return;
    const int i = ch.start + threadIdx.x;
    const int u = i < ch.end ? d.nbr_cnt[i] - d.nbr_lo[i] : 0;
    const int t = threadIdx.x;
    lds[t] = u;
    __syncthreads();
    for (int o = 1; o < kChunk; o <<= 1) {
        const int v = (t >= o) ? lds[t - o] : 0;
        __syncthreads();
        lds[t] += v;
        __syncthreads();
    }
    if (i < ch.end) d.half_off[i] = d.chunk_off[blockIdx.x] + lds[t] - u;
}

__global__ __launch_bounds__(kChunk) void k_pid(Dev d) {
    const Chunk ch = d.chunks[blockIdx.x];
    const int s = ch.sys;
    if (!d.ctl[s].rebuild) return;
    const int i = ch.start + threadIdx.x;
    if (i >= ch.end) return;
    const SysDesc& S = d.sys[s];
    const int K = d.K;
    const int cnt = d.nbr_cnt[i], lo = d.nbr_lo[i], hoff = d.half_off[i];
    const int* row = d.nbr + (int64_t)i * K;
    int* prow = d.pid + (int64_t)i * K;
    bool bad = false;
    for (int k = 0; k < cnt; ++k) {
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
            // position of i in j's sorted row; i > j lies in j's upper part
            const int* rj = d.nbr + (int64_t)j * K;
            int l = 0, h = d.nbr_cnt[j];
            while (l < h) {
                const int mid = (l + h) >> 1;
                if (rj[mid] < i) l = mid + 1; else h = mid;
            }
            if (l >= d.nbr_cnt[j] || rj[l] != i) {
                bad = true;
                prow[k] = -1;
                continue;
            }
            local = d.half_off[j] + (l - d.nbr_lo[j]);
        }
        prow[k] = (local < S.pair_cap) ? (int)(S.pair_base + local) : -1;
    }
    if (bad) atomicOr(&d.ctl[s].status, MXE_STAT_KMAX);
}

__global__ void k_build_done(Dev d) {
    const int s = gtid();
    if (s >= d.n_sys) return;
    SysCtl& c = d.ctl[s];
    if (!c.rebuild) return;
    c.n_rebuilds += 1;
    c.rebuild = 0;
    d.scalars[(int64_t)s * MXE_NSCALARS + MXE_S_PAIRS] = (double)c.n_pairs;
    d.scalars[(int64_t)s * MXE_NSCALARS + MXE_S_REBUILDS] = (double)c.n_rebuilds;
}

int row_pow2(int K) {
    int k2 = 64;
    while (k2 < K) k2 <<= 1;
    return k2;
}

void launch_build(const Dev& d, const Model& m, bool bonds, hipStream_t s) {
    k_bin<<<d.n_chunks, kChunk, 0, s>>>(d);
    k_cell_scan<<<d.n_sys, 1024, 0, s>>>(d);
    k_fill<<<d.n_chunks, kChunk, 0, s>>>(d);
    const int gc = (int)std::min<int64_t>(2048, (d.n_cells + 255) / 256);
    k_sort_cells<<<gc, 256, 0, s>>>(d);
    const int K2 = row_pow2(d.K);
    k_nbr<<<d.n_chunks, kChunk, (size_t)(kChunk / kWave) * K2 * sizeof(int), s>>>(d, m, K2);
    if (bonds) k_bonds<<<d.n_chunks, kChunk, 0, s>>>(d, m);
    k_scan<<<d.n_sys, 1024, 0, s>>>(d);
    k_half<<<d.n_chunks, kChunk, 0, s>>>(d);
    k_pid<<<d.n_chunks, kChunk, 0, s>>>(d);
    k_build_done<<<(d.n_sys + 63) / 64, 64, 0, s>>>(d);
}

}  // namespace mxe
