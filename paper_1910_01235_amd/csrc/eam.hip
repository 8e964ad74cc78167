// Mean-field EAM evaluation: pair moments, density pass, force / mu pass.
//
// Phase averages (App. A): a pair term depends on q_j - q_i only; for two
// independent Gaussian packets of per-axis widths sigma_i, sigma_j this is a
// Gaussian of mean rbar = qbar_j - qbar_i and width s = sqrt(sigma_i^2 + sigma_j^2),
// averaged here by the 27-node product Gauss-Hermite rule (per axis: nodes
// 0, +-sqrt(3), weights 2/3, 1/6, 1/6). The Taylor form of the embedding
// (App. B.2, Eq. F_taylor_mxe) needs the density at the mean positions as well.
//
// The work is split so that each unordered pair's quadrature runs once:
//   k_pair     one thread per pair (i < j): 27 nodes -> 14 moments; both radial
//              shapes share each node's distance. Stored per pair as one force
//              block (16 slots: a 128-byte line in FP64) and one density pair
//              (<f>, f0), so a gather from either end reads whole lines.
//   k_density  one wavefront per site, lanes over its neighbour row: gathers
//              rho_bar = sum_j b_j <f>, rho0 = sum_j b_j f0 (Eq. EAM-density-
//              substitutional-ave), then the Taylor embedding terms.
//   k_force    one wavefront per site: gathers the moments with the sign of the
//              pair's direction and the neighbours' embedding terms, giving the
//              exact gradient of the free energy, mu and the site's energy share,
//              plus the chunk partial sums that drive FIRE.
// Accumulation over neighbours is FP64 in both precisions; the FP32-mixed
// variant runs the node arithmetic and stores the moments in FP32.
#include "mxe_internal.h"

namespace mxe {

namespace {

template <typename T> struct Math;

template <> struct Math<double> {
    static __device__ inline double ex(double v) { return exp(v); }
    static __device__ inline double sq(double v) { return sqrt(v); }
    static __device__ inline void scpi(double t, double* s, double* c) { sincospi(t, s, c); }
};
template <> struct Math<float> {
    static __device__ inline float ex(float v) { return __expf(v); }
    static __device__ inline float sq(float v) { return __fsqrt_rn(v); }
    static __device__ inline void scpi(float t, float* s, float* c) { sincospif(t, s, c); }
};

// Radial shapes of both pair functions at distance r (r < r_c):
// g = exp(-a (r/r_e - 1)) S(r), and their derivatives.
template <typename T>
__device__ inline void shapes(T r, T inv_re, T al, T ga, T r_s, T tw, T& gp, T& dgp, T& gf, T& dgf) {
    const T u = r * inv_re - T(1);
    const T ep = Math<T>::ex(-al * u);
    const T ef = Math<T>::ex(-ga * u);
    T S = T(1), dS = T(0);
    if (r > r_s) {
        T sn, cs;
        Math<T>::scpi((r - r_s) * tw, &sn, &cs);
        S = T(0.5) * (T(1) + cs);
        dS = T(-0.5) * T(3.14159265358979323846) * tw * sn;
    }
    gp = ep * S;
    dgp = ep * (dS - al * inv_re * S);
    gf = ef * S;
    dgf = ef * (dS - ga * inv_re * S);
}

template <typename T>
__device__ inline void pair_moments(const Model& m, int cls, double rx, double ry, double rz,
                                    double s, T out[kMom]) {
    constexpr T kSqrt3 = T(1.7320508075688772935);
    const T inv_re = (T)m.inv_re[cls], al = (T)m.alpha[cls], ga = (T)m.gamma[cls];
    const T r_s = (T)m.r_s, tw = (T)m.taper_inv_w;
    const T rc2 = (T)(m.r_c * m.r_c);
    const T h = (T)s * kSqrt3;
    const T X[3] = {(T)rx - h, (T)rx, (T)rx + h};
    const T Y[3] = {(T)ry - h, (T)ry, (T)ry + h};
    const T Z[3] = {(T)rz - h, (T)rz, (T)rz + h};
    const T X2[3] = {X[0] * X[0], X[1] * X[1], X[2] * X[2]};
    const T Y2[3] = {Y[0] * Y[0], Y[1] * Y[1], Y[2] * Y[2]};
    const T Z2[3] = {Z[0] * Z[0], Z[1] * Z[1], Z[2] * Z[2]};
    constexpr T w1[3] = {T(1.0 / 6.0), T(2.0 / 3.0), T(1.0 / 6.0)};
#pragma unroll
    for (int k = 0; k < kMom; ++k) out[k] = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T r2 = X2[a] + Y2[b] + Z2[c];
                if (r2 < rc2 && r2 > T(0)) {
                    const T W = w1[a] * w1[b] * w1[c];
                    const T r = Math<T>::sq(r2);
                    const T rinv = T(1) / r;
                    T gp, dgp, gf, dgf;
                    shapes<T>(r, inv_re, al, ga, r_s, tw, gp, dgp, gf, dgf);
                    // node offset zeta = sqrt(3) (a-1, b-1, c-1); d . zeta
                    T dz = T(0);
                    if (a != 1) dz += (a == 2 ? X[a] : -X[a]);
                    if (b != 1) dz += (b == 2 ? Y[b] : -Y[b]);
                    if (c != 1) dz += (c == 2 ? Z[c] : -Z[c]);
                    dz *= kSqrt3;
                    const T cp = W * dgp * rinv, cf = W * dgf * rinv;
                    out[M_PHI] += W * gp;
                    out[M_GPHI + 0] += cp * X[a];
                    out[M_GPHI + 1] += cp * Y[b];
                    out[M_GPHI + 2] += cp * Z[c];
                    out[M_SPHI] += cp * dz;
                    out[M_F] += W * gf;
                    out[M_GF + 0] += cf * X[a];
                    out[M_GF + 1] += cf * Y[b];
                    out[M_GF + 2] += cf * Z[c];
                    out[M_SF] += cf * dz;
                    if (a == 1 && b == 1 && c == 1) {  // node at the mean: rho|_0 terms
                        const T g0 = dgf * rinv;
                        out[M_F0] = gf;
                        out[M_GF0 + 0] = g0 * X[1];
                        out[M_GF0 + 1] = g0 * Y[1];
                        out[M_GF0 + 2] = g0 * Z[1];
                    }
                }
            }
        }
    }
    const T sinv = T(1) / (T)s;
    out[M_SPHI] *= sinv;
    out[M_SF] *= sinv;
}

__device__ inline void min_image(const SysDesc& S, double& dx, double& dy, double& dz) {
    if (S.periodic[0]) dx -= S.box[0] * rint(dx / S.box[0]);
    if (S.periodic[1]) dy -= S.box[1] * rint(dy / S.box[1]);
    if (S.periodic[2]) dz -= S.box[2] * rint(dz / S.box[2]);
}

}  // namespace

// 16-byte vector of T, for whole-line loads and stores of the pair blocks
template <typename T>
struct alignas(16) Vec16 {
    static constexpr int n = 16 / sizeof(T);
    T v[n];
};

template <typename T>
__global__ __launch_bounds__(256) void k_pair(Dev d, Model m) {
    const Chunk ch = d.pchunks[blockIdx.x];
    const SysCtl& c = d.ctl[ch.sys];
    if (c.done) return;
    const SysDesc& S = d.sys[ch.sys];
    const int64_t pend = min((int64_t)ch.end, S.pair_base + min((int64_t)c.n_pairs, S.pair_cap));
    Vec16<T>* fblk = (Vec16<T>*)d.fblk;
    constexpr int per = kFBlk / Vec16<T>::n;  // vectors per force block
    T* dblk = (T*)d.dblk;
    for (int64_t p = ch.start + threadIdx.x; p < pend; p += blockDim.x) {
        const int i = d.pair_i[p], j = d.pair_j[p];
        double rx = d.qx[j] - d.qx[i], ry = d.qy[j] - d.qy[i], rz = d.qz[j] - d.qz[i];
        min_image(S, rx, ry, rz);
        const double si = d.sigma[i], sj = d.sigma[j];
        const double s = sqrt(si * si + sj * sj);
        const int cls = pair_cls(d.type[i], d.type[j]);
        T out[kFBlk];
#pragma unroll
        for (int k = 0; k < kFBlk; ++k) out[k] = T(0);
        if (cls >= 0 && rx * rx + ry * ry + rz * rz < (m.r_c + 3.0 * s) * (m.r_c + 3.0 * s))
            pair_moments<T>(m, cls, rx, ry, rz, s, out);
#pragma unroll
        for (int v = 0; v < per; ++v) {
            Vec16<T> b;
#pragma unroll
            for (int e = 0; e < Vec16<T>::n; ++e) b.v[e] = out[v * Vec16<T>::n + e];
            fblk[p * per + v] = b;
        }
        dblk[2 * p] = out[M_F];
        dblk[2 * p + 1] = out[M_F0];
    }
}

template <typename T>
__global__ __launch_bounds__(kChunk) void k_density(Dev d, Model m) {
    const Chunk ch = d.chunks[blockIdx.x];
    if (d.ctl[ch.sys].done) return;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const T* dblk = (const T*)d.dblk;
    const int K = d.K;
    for (int i = ch.start + wave; i < ch.end; i += kChunk / kWave) {
        const int cnt = d.nbr_cnt[i];
        double rb = 0.0, r0 = 0.0;
        for (int k = lane; k < cnt; k += kWave) {
            const int j = d.nbr[(int64_t)i * K + k];
            const int p = d.pid[(int64_t)i * K + k];
            if (p < 0) continue;
            const double bj = mixval(m.b4, d.type[j], d.x[j]);
            rb += bj * (double)dblk[2 * (int64_t)p];
            r0 += bj * (double)dblk[2 * (int64_t)p + 1];
        }
        rb = wave_sum(rb);
        r0 = wave_sum(r0);
        if (lane == 0) {
            const int ti = d.type[i];
            const double xi = d.x[i];
            d.rho_bar[i] = rb;
            d.rho0[i] = r0;
            double G = 0.0, A = 0.0, B = 0.0;
            const bool embeds = m.c4[occ_sp1(ti)] != 0.0 || m.c4[occ_sp0(ti)] != 0.0;
            if (embeds) {
                if (r0 > 1e-12) {
                    // F~(rho) = -sqrt(rho): F~' = -1/(2 sqrt rho), F~'' = 1/(4 rho^1.5)
                    const double sq = sqrt(r0);
                    const double F1 = -0.5 / sq, F2 = 0.25 / (sq * r0);
                    const double ch_i = mixhat(m.c4, ti, xi);
                    G = -sq + F1 * (rb - r0);
                    A = ch_i * F1;
                    B = ch_i * F2 * (rb - r0);
                } else {
                    atomicOr(&d.ctl[ch.sys].status, MXE_STAT_RHO);
                }
            }
            d.G[i] = G;
            d.Ahat[i] = A;
            d.Bhat[i] = B;
        }
    }
}

// Gradient of F (App. B.2.1) for site i, normalised by its vibrating
// fraction w_i, with the pair amplitude a_ij = sum_kl p_ik p_jl a_kl, the
// emissions b, the embedding strengths c, A_j = c_j F~'(rho0_j) and
// B_j = c_j F~''(rho0_j)(rho_bar_j - rho0_j):
//   -dF/dq_i / w_i = sum_j sign [ahat grad<phi> + (Ahat_i b_j + A_j bhat_i) grad<f>
//                                + (Bhat_i b_j + B_j bhat_i) grad f0]
//   -dF/dsigma_i / w_i = -sigma_i sum_j [ahat <phi>_s + (Ahat_i b_j + A_j bhat_i) <f>_s] / s
//                       + 3 kT / sigma_i
//   mu_i = sum_j da_ij/dx_i <phi> + db_i/dx_i sum_j (A_j <f> + B_j f0)
//          + dc_i/dx_i G_i - 3 kT dw_i/dx_i ln sigma_i
template <typename T>
__global__ __launch_bounds__(kChunk) void k_force(Dev d, Model m) {
    __shared__ double red[kChunk / kWave][6];
    const Chunk ch = d.chunks[blockIdx.x];
    const int sys = ch.sys;
    if (d.ctl[sys].done) return;
    const SysDesc& S = d.sys[sys];
    const double kT = S.kT;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const Vec16<T>* fblk = (const Vec16<T>*)d.fblk;
    constexpr int per = kFBlk / Vec16<T>::n;
    const int K = d.K;
    // running chunk partials, held by lane 0 of each wave
    double pe = 0.0, pfmax = 0.0, pfv = 0.0, pff = 0.0, pvv = 0.0, psx = 0.0;
    int bad = 0;
    for (int i = ch.start + wave; i < ch.end; i += kChunk / kWave) {
        const int ti = d.type[i];
        const double xi = d.x[i], si = d.sigma[i];
        const double Ahi = d.Ahat[i], Bhi = d.Bhat[i];
        const double pi1 = occ_p1(ti, xi);
        const int i1 = occ_sp1(ti), i0 = occ_sp0(ti);
        const double bhat_i = mixhat(m.b4, ti, xi), db_i = mixdx(m.b4, ti);
        const bool part_i = occ_partial(ti), mob_i = occ_mobile(ti);
        const int cnt = d.nbr_cnt[i];
        double fx = 0.0, fy = 0.0, fz = 0.0, fsg = 0.0, mu = 0.0, ep = 0.0;
        for (int k = lane; k < cnt; k += kWave) {
            const int j = d.nbr[(int64_t)i * K + k];
            const int p = d.pid[(int64_t)i * K + k];
            if (p < 0) continue;
            const int tj = d.type[j];
            const double xj = d.x[j];
            const double pj1 = occ_p1(tj, xj);
            const int j1 = occ_sp1(tj), j0 = occ_sp0(tj);
            const double a1 = pj1 * m.a4[i1][j1] + (1.0 - pj1) * m.a4[i1][j0];
            const double a0 = pj1 * m.a4[i0][j1] + (1.0 - pj1) * m.a4[i0][j0];
            const double aij = pi1 * a1 + (1.0 - pi1) * a0;
            const double ahat = part_i ? a1 : aij;
            const double dadx = mob_i ? a1 - a0 : 0.0;
            const double wj = occ_partial(tj) ? xj : 1.0;
            const double Aj = wj * d.Ahat[j], Bj = wj * d.Bhat[j];
            const double bj = mixval(m.b4, tj, xj);
            const double hA = Ahi * bj + Aj * bhat_i;
            const double hB = Bhi * bj + Bj * bhat_i;
            const double sg = j > i ? 1.0 : -1.0;
            T mb[kFBlk];
#pragma unroll
            for (int v = 0; v < per; ++v) {
                const Vec16<T> b = fblk[(int64_t)p * per + v];
#pragma unroll
                for (int e = 0; e < Vec16<T>::n; ++e) mb[v * Vec16<T>::n + e] = b.v[e];
            }
            const double mphi = (double)mb[M_PHI];
            const double mf = (double)mb[M_F];
            const double mf0 = (double)mb[M_F0];
            fx += sg * (ahat * (double)mb[M_GPHI + 0] + hA * (double)mb[M_GF + 0] + hB * (double)mb[M_GF0 + 0]);
            fy += sg * (ahat * (double)mb[M_GPHI + 1] + hA * (double)mb[M_GF + 1] + hB * (double)mb[M_GF0 + 1]);
            fz += sg * (ahat * (double)mb[M_GPHI + 2] + hA * (double)mb[M_GF + 2] + hB * (double)mb[M_GF0 + 2]);
            fsg += ahat * (double)mb[M_SPHI] + hA * (double)mb[M_SF];
            mu += dadx * mphi + db_i * (Aj * mf + Bj * mf0);
            ep += aij * mphi;
        }
        fx = wave_sum(fx);
        fy = wave_sum(fy);
        fz = wave_sum(fz);
        fsg = wave_sum(fsg);
        mu = wave_sum(mu);
        ep = wave_sum(ep);
        if (lane == 0) {
            const double Gi = d.G[i];
            const double lns = log(si);
            const double fs = -si * fsg + 3.0 * kT / si;
            const double wi = part_i ? xi : 1.0;
            double mui = 0.0, mix = 0.0;
            if (mob_i) {
                mui = mu + mixdx(m.c4, ti) * Gi - 3.0 * kT * (part_i ? 1.0 : 0.0) * lns;
                if (xi > 0.0) mix += xi * log(xi);
                if (xi < 1.0) mix += (1.0 - xi) * log(1.0 - xi);
                mix *= kT;
            }
            const double ei = 0.5 * ep + mixval(m.c4, ti, xi) * Gi - 3.0 * kT * wi * lns + mix;
            d.fx[i] = fx;
            d.fy[i] = fy;
            d.fz[i] = fz;
            d.fs[i] = fs;
            d.mu[i] = mui;
            d.e_site[i] = ei;
            const double vx = d.vx[i], vy = d.vy[i], vz = d.vz[i], vs = d.vs[i];
            pe += ei;
            psx += xi;
            pfmax = fmax(pfmax, fmax(fmax(fabs(fx), fabs(fy)), fmax(fabs(fz), fabs(fs))));
            pfv += fx * vx + fy * vy + fz * vz + fs * vs;
            pff += fx * fx + fy * fy + fz * fz + fs * fs;
            pvv += vx * vx + vy * vy + vz * vz + vs * vs;
            if (!isfinite(fx + fy + fz + fs + ei + mui)) bad = 1;
        }
    }
    if (lane == 0) {
        red[wave][0] = pe;
        red[wave][1] = pfmax;
        red[wave][2] = pfv;
        red[wave][3] = pff;
        red[wave][4] = pvv;
        red[wave][5] = psx;
        if (bad) atomicOr(&d.ctl[sys].status, MXE_STAT_NONFINITE);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double* P = d.part + (int64_t)blockIdx.x * kNPart;
        double e = red[0][0], fm = red[0][1], fv = red[0][2], ff = red[0][3], vv = red[0][4], sx = red[0][5];
        for (int w = 1; w < kChunk / kWave; ++w) {
            e += red[w][0];
            fm = fmax(fm, red[w][1]);
            fv += red[w][2];
            ff += red[w][3];
            vv += red[w][4];
            sx += red[w][5];
        }
        P[P_E] = e;
        P[P_FMAX] = fm;
        P[P_FV] = fv;
        P[P_FF] = ff;
        P[P_VV] = vv;
        P[P_SUMX] = sx;
    }
}

void launch_pair(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) k_pair<float><<<d.n_pchunks, 256, 0, s>>>(d, m);
    else k_pair<double><<<d.n_pchunks, 256, 0, s>>>(d, m);
}

void launch_density(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) k_density<float><<<d.n_chunks, kChunk, 0, s>>>(d, m);
    else k_density<double><<<d.n_chunks, kChunk, 0, s>>>(d, m);
}

void launch_force(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) k_force<float><<<d.n_chunks, kChunk, 0, s>>>(d, m);
    else k_force<double><<<d.n_chunks, kChunk, 0, s>>>(d, m);
}

}  // namespace mxe
