// Relaxation control (FIRE) and the master-equation step.
//
// Relaxation (Sec. 4): positions and widths move at fixed x to lower the
// mean-field free energy. The relaxer is FIRE (Bitzek et al., PRL 97, 170201,
// 2006) with unit mass and semi-implicit Euler steps on the normalised forces.
// Each system keeps its own FIRE scalars; a system that has converged (or hit
// the iteration cap) is marked done and every later kernel skips it, so a
// fixed launch sequence of max_relax + 1 iterations serves every system.
//
// Kinetic law (Sec. 3.1, Eq. MassTransport with Eq. attempt_freq_mass): the
// flux over a bond is evaluated once per direction from the pair's canonical
// (lower index, higher index) order, so the two ends receive exactly opposite
// contributions and sum(x) is conserved up to the rounding of the Euler sums.
// Time step: dt_safety over the largest per-site outflow or inflow rate,
// weighted by the occupancy that can move, which keeps x inside [0, 1].
#include "mxe_internal.h"

namespace mxe {

namespace {

// Fixed-order block reductions over kChunk threads (deterministic).
__device__ inline double block_sum(double v, double* lds) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = lds[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t += lds[w];
    return t;
}
__device__ inline double block_max(double v, double* lds) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
    __syncthreads();
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = lds[0];
    for (int w = 1; w < (int)(blockDim.x >> 6); ++w) t = fmax(t, lds[w]);
    return t;
}

__device__ inline double* sc(const Dev& d, int s) { return d.scalars + (int64_t)s * MXE_NSCALARS; }

}  // namespace

__global__ void k_relax_init(Dev d, Model m) {
    const int s = gtid();
    if (s >= d.n_sys) return;
    relax_start(d.ctl[s], m);
}

void launch_relax_init(const Dev& d, const Model& m, hipStream_t s) {
    k_relax_init<<<(d.n_sys + 63) / 64, 64, 0, s>>>(d, m);
}

// The force gather's partial sums of site chunk cb (energy, largest force
// component, F.v, F.F, v.v, sum of x): folded already (fold_rows), or its
// kForceSplit rows combined here, pairwise with the lower half first.
__device__ inline void chunk_row(const Dev& d, const Model& m, int cb, double v[6]) {
    static_assert(kForceSplit >= 2 && (kForceSplit & (kForceSplit - 1)) == 0, "fold width");
    if (m.fold_rows) {
        const double* P = d.part + (int64_t)cb * kNPart;
#pragma unroll
        for (int j = 0; j < 6; ++j) v[j] = P[j];
        return;
    }
    const double2* R = (const double2*)(d.part_sub + (int64_t)cb * kForceSplit * kNPart);
    double r[kForceSplit][6];
#pragma unroll
    for (int k = 0; k < kForceSplit; ++k) {
        const double2 a = R[k * (kNPart / 2)], b = R[k * (kNPart / 2) + 1], c = R[k * (kNPart / 2) + 2];
        r[k][0] = a.x, r[k][1] = a.y, r[k][2] = b.x, r[k][3] = b.y, r[k][4] = c.x, r[k][5] = c.y;
    }
#pragma unroll
    for (int w = 1; w < kForceSplit; w <<= 1) {
#pragma unroll
        for (int k = 0; k < kForceSplit; k += 2 * w) {
#pragma unroll
            for (int j = 0; j < 6; ++j)
                r[k][j] = j == P_FMAX ? fmax(r[k][j], r[k + w][j]) : r[k][j] + r[k + w][j];
        }
    }
#pragma unroll
    for (int j = 0; j < 6; ++j) v[j] = r[0][j];
}

// One block per system: reduce the chunk partials in chunk order, then run
// the FIRE decision (mode 1) or only record the evaluation (mode 0). Mode 2
// (free-running steps) is mode 1 where a system whose relaxation ends with
// steps left is marked to take its Euler step in this iteration.
__global__ __launch_bounds__(kChunk) void k_control(Dev d, Model m, int mode) {
    __shared__ double lds[kChunk / kWave];
    const int s = blockIdx.x;
    SysCtl& c = d.ctl[s];
    if (c.done) return;
    // a lean iteration whose lists had expired: not taken (k_update reads the
    // flag, as its own blocks move the maxima the decision rests on)
    if (idle(c, m)) {
        if (threadIdx.x == 0) c.stall = 1;
        return;
    }
    // a build earlier in this iteration is counted here (the chain's own
    // finishing kernel is not launched within relaxations)
    if (threadIdx.x == 0) {
        c.stall = 0;
        finish_build(d, s);
    }
    const SysDesc& S = d.sys[s];
    if (S.n_sites == 0) {  // an empty slot evaluates nothing and counts nothing
        if (threadIdx.x == 0) {
            c.done = 1;
            c.converged = 1;
        }
        return;
    }
    // each chunk's row of partial sums (its kForceSplit force-gather rows
    // combined pairwise in a fixed order), then the chunks in thread order. A
    // plan with a system of more chunks than this block has threads has the
    // rows folded by k_force_fold (many blocks, the same order): one block
    // reading eight rows per chunk of a large system waits on too many misses.
    double e = 0.0, fm = 0.0, fv = 0.0, ff = 0.0, vv = 0.0, sx = 0.0;
    for (int k = threadIdx.x; k < S.n_chunks; k += blockDim.x) {
        double v[6];
        chunk_row(d, m, S.chunk_first + k, v);
        e += v[P_E];
        fm = fmax(fm, v[P_FMAX]);
        fv += v[P_FV];
        ff += v[P_FF];
        vv += v[P_VV];
        sx += v[P_SUMX];
    }
    e = block_sum(e, lds);
    fm = block_max(fm, lds);
    fv = block_sum(fv, lds);
    ff = block_sum(ff, lds);
    vv = block_sum(vv, lds);
    sx = block_sum(sx, lds);
    if (threadIdx.x != 0) return;
    double* out = sc(d, s);
    c.evals += 1;
    c.total_evals += 1;
    c.pair_evals += (double)c.n_pairs;
    out[MXE_S_PAIR_EVALS] = c.pair_evals;
    out[MXE_S_F] = e;
    out[MXE_S_FMAX] = fm;
    out[MXE_S_SUMX] = sx;
    out[MXE_S_TOTAL_EVALS] = (double)c.total_evals;
    if (!isfinite(e) || !isfinite(ff)) c.status |= MXE_STAT_NONFINITE;
    if (mode >= 1) {
        if (fm <= m.ftol) {
            c.done = 1;
            c.converged = 1;
        } else if (c.k >= m.max_relax || (c.status & MXE_STAT_NONFINITE)) {
            c.done = 1;
        } else {
            double dt = c.fire_dt, alpha = c.fire_alpha;
            bool reset = (c.k == 0);
            if (c.k > 0) {
                if (fv > 0.0) {
                    c.npos += 1;
                    if (c.npos > m.nmin) {
                        dt = fmin(dt * m.finc, m.dtmax);
                        alpha *= m.falpha;
                    }
                } else {
                    c.npos = 0;
                    dt *= m.fdec;
                    alpha = m.alpha0;
                    reset = true;
                }
            }
            if (reset) {
                fv = 0.0;
                vv = 0.0;
            }
            // |v + dt f| from the old velocity's reductions (no second pass)
            const double vnorm = sqrt(vv + 2.0 * dt * fv + dt * dt * ff);
            const double fnorm = sqrt(ff);
            c.fire_dt = dt;
            c.fire_alpha = alpha;
            c.c_keep = reset ? 0.0 : 1.0;
            c.mix_v = fnorm > 0.0 ? 1.0 - alpha : 1.0;
            c.mix_f = fnorm > 0.0 ? alpha * (vnorm / fnorm) : 0.0;
            c.updates += 1;
        }
        c.k += 1;
        if (mode == 2 && c.done && c.steps_left > 0) c.stepping = 1;
        out[MXE_S_UPDATES] = (double)c.updates;
        out[MXE_S_CONVERGED] = (double)c.converged;
        out[MXE_S_EVALS] = (double)c.evals;
    }
    out[MXE_S_STATUS] = (double)c.status;
}

void launch_control(const Dev& d, const Model& m, int mode, hipStream_t s) {
    k_control<<<d.n_sys, kChunk, 0, s>>>(d, m, mode);
}

// Number of systems still relaxing (not done; steps = 0) or with diffusion
// steps left (steps = 1), and the number stalled for a build, written by one
// block to out[0] and out[1] (host-mapped ints): the host reads them between
// chunks of iterations, to stop once the first is zero and to enqueue an
// iteration with the build chain while the second is not.
__global__ __launch_bounds__(kChunk) void k_active(const SysCtl* ctl, int n_sys, int steps, int* out) {
    __shared__ int lds[2][kChunk / kWave];
    int n = 0, st = 0;
    for (int s = threadIdx.x; s < n_sys; s += blockDim.x) {
        n += (steps ? ctl[s].steps_left > 0 : !ctl[s].done) ? 1 : 0;
        st += (ctl[s].stall && !ctl[s].done) ? 1 : 0;
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        n += __shfl_xor(n, o);
        st += __shfl_xor(st, o);
    }
    if ((threadIdx.x & 63) == 0) {
        lds[0][threadIdx.x >> 6] = n;
        lds[1][threadIdx.x >> 6] = st;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int t = 0, u = 0;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) {
            t += lds[0][w];
            u += lds[1][w];
        }
        ((volatile int*)out)[0] = t;
        ((volatile int*)out)[1] = u;
    }
}

void launch_active(const Dev& d, int* out, int steps, hipStream_t s) {
    k_active<<<1, kChunk, 0, s>>>(d.ctl, d.n_sys, steps, out);
}

// FIRE velocity mixing and position/width update; records the largest
// displacement and widening since the last build, from which the next build
// decides whether the lists still hold.
__global__ __launch_bounds__(kChunk) void k_update(Dev d, Model m) {
    __shared__ double lds[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    SysCtl& c = d.ctl[ch.sys];
    if (c.done || c.stall) return;  // as k_control decided for this iteration
    const int i = ch.start + threadIdx.x;
    const double dt = c.fire_dt, mv = c.mix_v, mf = c.mix_f;
    const bool keep = c.c_keep != 0.0;
    double sg_new = 0.0, drift = 0.0, widen = 0.0;
    if (i < ch.end) {
        const double f[4] = {d.fx[i], d.fy[i], d.fz[i], d.fs[i]};
        double* v[4] = {d.vx + i, d.vy + i, d.vz + i, d.vs + i};
        double* y[4] = {d.qx + i, d.qy + i, d.qz + i, d.sigma + i};
        double yn[4];  // new positions and width, kept in registers (no reloads)
#pragma unroll
        for (int a = 0; a < 4; ++a) {
            const double vt = (keep ? *v[a] : 0.0) + dt * f[a];
            const double vn = mv * vt + mf * f[a];
            *v[a] = vn;
            yn[a] = *y[a] + dt * vn;
        }
        if (yn[3] < m.sigma_min) {
            yn[3] = m.sigma_min;
            atomicOr(&c.status, MXE_STAT_SIGMA_MIN);
        }
#pragma unroll
        for (int a = 0; a < 4; ++a) *y[a] = yn[a];
        sg_new = yn[3];
        if (sg_new > m.sigma_cap) atomicOr(&c.status, MXE_STAT_SIGMA_CAP);
        const double dx = yn[0] - d.qrx[i], dy = yn[1] - d.qry[i], dz = yn[2] - d.qrz[i];
        drift = dx * dx + dy * dy + dz * dz;
        widen = fmax(sg_new - d.sref[i], 0.0);
    }
    const double md = block_max(drift, lds);
    const double mw = block_max(widen, lds);
    if (threadIdx.x == 0) {
        raise_max(&c.drift_bits, md);
        raise_max(&c.widen_bits, mw);
    }
}

void launch_update(const Dev& d, const Model& m, hipStream_t s) {
    k_update<<<d.n_chunks, kChunk, 0, s>>>(d, m);
}

// ---------------------------------------------------------------------------
// Master equation
// ---------------------------------------------------------------------------
// free_run (mxe_advance): only systems whose relaxation ended in this
// iteration take the step; the others' blocks leave at once (uniformly).
__global__ __launch_bounds__(kChunk) void k_flux(Dev d, Model m, int free_run) {
    __shared__ double lds[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    if (free_run && !d.ctl[ch.sys].stepping) return;
    const SysDesc& S = d.sys[ch.sys];
    const int i = ch.start + threadIdx.x;
    double rate = 0.0;
    if (i < ch.end) {
        double acc = 0.0, rout = 0.0, rin = 0.0;
        const int ti = d.type[i];
        if (occ_mobile(ti) && d.T_site != nullptr) {
            // site temperatures: a hop a -> b has attempt rate nu0 e^{-beta_a Qm} and
            // driving factor e^{c beta_a (mu_a - mu_b)}, both at its source site, so
            // the pair's net flux is the same seen from either end
            const int nb = d.nbond[i];
            const int* row = d.bond + (int64_t)i * d.bond_max;
            for (int b = 0; b < nb; ++b) {
                const int j = row[b];
                const bool i_lo = i < j;
                const int lo = i_lo ? i : j, hi = i_lo ? j : i;
                const double xl = d.x[lo], xh = d.x[hi];
                const double bl = 1.0 / (kBoltzmannEv * d.T_site[lo]);
                const double bh = 1.0 / (kBoltzmannEv * d.T_site[hi]);
                const double r_hl = m.nu0 * exp(-bh * m.Qm) * exp(m.kin_c * bh * (d.mu[hi] - d.mu[lo]));
                const double r_lh = m.nu0 * exp(-bl * m.Qm) * exp(m.kin_c * bl * (d.mu[lo] - d.mu[hi]));
                const double J = xh * (1.0 - xl) * r_hl - xl * (1.0 - xh) * r_lh;  // net hi -> lo
                acc += i_lo ? J : -J;
                const double xj = i_lo ? xh : xl;
                rout += (1.0 - xj) * (i_lo ? r_lh : r_hl);
                rin += xj * (i_lo ? r_hl : r_lh);
            }
        } else if (occ_mobile(ti)) {
            const double D = S.D, cb = m.kin_c * S.beta;
            const int nb = d.nbond[i];
            const int* row = d.bond + (int64_t)i * d.bond_max;
            for (int b = 0; b < nb; ++b) {
                const int j = row[b];
                const bool i_lo = i < j;
                const int lo = i_lo ? i : j, hi = i_lo ? j : i;
                const double xl = d.x[lo], xh = d.x[hi];
                const double arg = cb * (d.mu[hi] - d.mu[lo]);
                const double e_hl = exp(arg);   // rate factor of a hop hi -> lo
                const double e_lh = exp(-arg);  // rate factor of a hop lo -> hi
                // net flux from hi into lo
                const double J = D * (xh * (1.0 - xl) * e_hl - xl * (1.0 - xh) * e_lh);
                acc += i_lo ? J : -J;
                const double xj = i_lo ? xh : xl;
                rout += D * (1.0 - xj) * (i_lo ? e_lh : e_hl);
                rin += D * xj * (i_lo ? e_hl : e_lh);
            }
        }
        d.dxdt[i] = acc;
        rate = fmax(rout, rin);
    }
    const double mx = block_max(rate, lds);
    if (threadIdx.x == 0) d.part[(int64_t)blockIdx.x * kNPart + P_RATE] = mx;
}

__global__ __launch_bounds__(kChunk) void k_mstep_ctl(Dev d, Model m, double dt_in, int free_run) {
    __shared__ double lds[kChunk / kWave];
    const int s = blockIdx.x;
    if (free_run && !d.ctl[s].stepping) return;
    const SysDesc& S = d.sys[s];
    // an empty slot's chunks lie beyond the launched prefix: no rows, rate 0
    const int nck = S.n_sites > 0 ? S.n_chunks : 0;
    double r = 0.0;
    for (int k = threadIdx.x; k < nck; k += blockDim.x)
        r = fmax(r, d.part[(int64_t)(S.chunk_first + k) * kNPart + P_RATE]);
    r = block_max(r, lds);
    if (threadIdx.x != 0) return;
    const double dt = dt_in > 0.0 ? dt_in : (r > 0.0 ? m.dt_safety / r : 0.0);
    d.ctl[s].dt_master = dt;
    double* out = sc(d, s);
    out[MXE_S_DT] = dt;
    out[MXE_S_TIME] += dt;
}

// Forward-Euler update of x (Sec. 4), then held-x sites are reset to their
// value; the matter they took up in the step goes to the reservoir account.
__global__ __launch_bounds__(kChunk) void k_euler(Dev d, Model m, int free_run) {
    __shared__ double lds[kChunk / kWave];
    const Chunk ch = d.chunks[blockIdx.x];
    if (free_run && !d.ctl[ch.sys].stepping) return;
    const int i = ch.start + threadIdx.x;
    double xi = 0.0, taken = 0.0;
    if (i < ch.end) {
        xi = d.x[i];
        const int ti = d.type[i];
        if (occ_mobile(ti)) {
            xi += d.ctl[ch.sys].dt_master * d.dxdt[i];
            if (held(d, i, ti, MXE_RES_FIX_X)) {
                taken = xi - d.res_val[i];
                xi = d.res_val[i];
            }
            d.x[i] = xi;
            d.emit[i] = mixval(m.b4, ti, xi);
            if (!(xi >= -1e-12 && xi <= 1.0 + 1e-12)) atomicOr(&d.ctl[ch.sys].status, MXE_STAT_X_RANGE);
        }
    }
    const double t = block_sum(xi, lds);
    const double r = d.res != nullptr ? block_sum(taken, lds) : 0.0;
    if (threadIdx.x == 0) {
        d.part[(int64_t)blockIdx.x * kNPart + P_SUMX] = t;
        d.part[(int64_t)blockIdx.x * kNPart + P_RES] = r;
    }
}

// free_run: the step is counted off the system's budget and, if steps are
// left, its next relaxation starts with the next iteration.
__global__ __launch_bounds__(kChunk) void k_estep_ctl(Dev d, Model m, int free_run) {
    __shared__ double lds[kChunk / kWave];
    const int s = blockIdx.x;
    if (free_run && !d.ctl[s].stepping) return;
    const SysDesc& S = d.sys[s];
    const int nck = S.n_sites > 0 ? S.n_chunks : 0;  // as in k_mstep_ctl
    double t = 0.0, r = 0.0;
    for (int k = threadIdx.x; k < nck; k += blockDim.x) {
        t += d.part[(int64_t)(S.chunk_first + k) * kNPart + P_SUMX];
        r += d.part[(int64_t)(S.chunk_first + k) * kNPart + P_RES];
    }
    t = block_sum(t, lds);
    r = d.res != nullptr ? block_sum(r, lds) : 0.0;
    if (threadIdx.x != 0) return;
    double* out = sc(d, s);
    out[MXE_S_SUMX] = t;
    out[MXE_S_RESERVOIR] += r;
    SysCtl& c = d.ctl[s];
    out[MXE_S_STATUS] = (double)c.status;
    if (free_run) {
        c.stepping = 0;
        c.steps_left -= 1;
        out[MXE_S_STEPS_LEFT] = (double)c.steps_left;
        if (c.steps_left > 0) relax_start(c, m);
    }
}

void launch_master(const Dev& d, const Model& m, double dt_in, hipStream_t s, int free_run) {
    k_flux<<<d.n_chunks, kChunk, 0, s>>>(d, m, free_run);
    k_mstep_ctl<<<d.n_sys, kChunk, 0, s>>>(d, m, dt_in, free_run);
    k_euler<<<d.n_chunks, kChunk, 0, s>>>(d, m, free_run);
    k_estep_ctl<<<d.n_sys, kChunk, 0, s>>>(d, m, free_run);
}

}  // namespace mxe
