// Mean-field EAM evaluation: pair moments, density pass, force / mu pass.
//
// Phase averages (App. A): a pair term depends on q_j - q_i only; for two
// independent Gaussian packets of per-axis widths sigma_i, sigma_j this is a
// Gaussian of mean rbar = qbar_j - qbar_i and width s = sqrt(sigma_i^2 + sigma_j^2),
// averaged by the 27-node product Gauss-Hermite rule (per axis: nodes
// 0, +-sqrt(3), weights 2/3, 1/6, 1/6). Alternatively the degree-3 rule of
// App. A, Eq. (QuadRule), integrates the pair's six coordinates directly:
// 12 nodes, each displacing one end by +-sqrt(6) sigma along one axis, all
// weighted 1/12. The Taylor form of the embedding (App. B.2, Eq. F_taylor_mxe)
// needs the density at the mean positions as well.
//
// The work is split so that each unordered pair's quadrature runs once:
//   k_pair     one thread per pair (i < j): 27 (or 12 + centre) nodes -> 16
//              moments; both radial shapes share each node's distance. Stored per pair as one force
//              block (16 slots: a 128-byte line in FP64) and one density pair
//              (<f>, f0), so a gather from either end reads whole lines.
//   k_density  kLPS lanes per site, lanes over its neighbour row: gathers
//              rho_bar = sum_j b_j <f>, rho0 = sum_j b_j f0 (Eq. EAM-density-
//              substitutional-ave), then the Taylor embedding terms.
//   k_force    kLPS lanes per site: gathers the moments with the sign of the
//              pair's direction and the neighbours' embedding terms, giving the
//              exact gradient of the free energy, mu and the site's energy share,
//              plus the chunk partial sums that drive FIRE.
// Accumulation over neighbours is FP64 in both precisions; the FP32-mixed
// variant runs the node arithmetic and stores the moments in FP32.
#include "mxe_internal.h"

namespace mxe {

namespace {

// ---------------------------------------------------------------------------
// Node arithmetic. The arguments are bounded by the pair geometry: distances
// lie in (0, r_c), so exp sees arguments of modest size and the taper argument
// lies in [0, 1]. The FP64 routines below exploit that (no special cases):
//  * exp: the exponent arrives in base 2, y = x log2(e), formed by one
//    multiply-add from the distance (the shape constants fold log2(e) in).
//    y = n + f with n = rint(y) and |f| <= 1/2 exact, and 2^f = e^r with
//    r = f ln2: 1 + r (1 + r (1/2 + r E(r))) with near-minimax E of degree 8
//    (relative error below 4e-17), written as a polynomial in f, then
//    scaling by 2^n. Forming y costs |y| ulp-sized error, as forming the
//    natural exponent from the distance did before.
//  * 1/sqrt: the hardware reciprocal square root refined by one second-order
//    step (the series of (1 - e)^(-1/2) to e^2).
//  * taper: with v = t - 1/2 and z = pi v (|z| <= pi/2), cos(pi t) = -sin z and
//    sin(pi t) = cos z: sin z = z (1 - w S(w)), cos z = 1 + w (-1/2 + w C(w))
//    with w = z^2 and near-minimax S (degree 7, error ~1e-18) and C (degree 6,
//    ~6e-17), against degrees 10 and 9 for Taylor series of the same accuracy.
// The FP32 variant uses the hardware exp2, rsq and sin/cos instructions.
// ---------------------------------------------------------------------------
// The polynomial coefficients arrive in the kernel arguments (Model::poly):
// the kernels read them with scalar loads and each FMA takes its coefficient
// as a scalar operand. An FP64 FMA cannot encode a 64-bit literal, so
// compile-time constants would cost a move into vector registers at every use.
__device__ inline double exp2_bounded(double y, const PolyCoef& c) {
    const double n = rint(y);
    const double f = y - n;  // exact
    double p = c.ex[0];
#pragma unroll
    for (int k = 1; k < PolyCoef::kExp; ++k) p = fma(p, f, c.ex[k]);
    p = fma(p, f, c.ln2sq_half);
    p = fma(p, f, c.ln2);
    p = fma(p, f, 1.0);
    return ldexp(p, (int)n);
}

// The hardware estimate y0 is good to 24 bits (measured: relative error below
// 5.3e-8). With e = 1 - a y0^2, (1 - e)^(-1/2) = 1 + e/2 + 3e^2/8 + O(e^3), so one
// second-order step y0 + y0 e (1/2 + 3e/8) leaves a truncation near 5e^3/16
// (below 1e-22) and about one ulp of rounding: five operations where two Newton
// steps take seven.
__device__ inline double rsqrt_refined(double a) {
    const double y = __builtin_amdgcn_rsq(a);
    const double e = fma(-a * y, y, 1.0);
    return fma(y * e, fma(e, 0.375, 0.5), y);
}

// S(t) = (1 + cos(pi t)) / 2 and sin(pi t) for t in [0, 1], from
// z = pi (t - 1/2) in [-pi/2, pi/2]
__device__ inline void taper_terms(double z, double& S, double& sn, const PolyCoef& c) {
    const double z2 = z * z;
    double ps = c.sn[0];  // sin z = z (1 - w S(w))
#pragma unroll
    for (int k = 1; k < PolyCoef::kSin; ++k) ps = fma(ps, z2, c.sn[k]);
    ps = fma(-ps, z2, 1.0);
    const double sinz = ps * z;
    double pc = c.cs[0];
#pragma unroll
    for (int k = 1; k < PolyCoef::kCos; ++k) pc = fma(pc, z2, c.cs[k]);
    pc = fma(pc, z2, -0.5);
    pc = fma(pc, z2, 1.0);
    S = 0.5 * (1.0 - sinz);
    sn = pc;
}

// Per-pair constants of the two radial shapes g = exp(-a (r/r_e - 1)) S(r)
// (a = alpha for phi, gamma for f) and of the taper S.
template <typename T>
struct ShapeK {
    T p1, p0, f1, f0;  // base-2 exponents: -a (r/r_e - 1) log2(e) = r x1 + x0
    T u1, u0;          // the same for u = exp(-(alpha / P) t) (ratio kernels only)
    bool second;       // the pair is of the second ratio of a two-ratio kernel
    T kp, kf;          // a / r_e: minus the slope of each natural exponent
    T r_s, tw;         // taper start and 1 / taper width
    T kz, kd;          // pi / width (the taper's z per unit distance), -pi / (2 width)
};

// Exponent ratios. When alpha : gamma = P : Q in small integers, both radial
// exponentials are powers of one: exp(-alpha t) = u^P and exp(-gamma t) = u^Q
// with u = exp(-(alpha / P) t), t = r / r_e - 1. A ratio code kPQ = 16 P + Q
// (0: two exponentials) is a compile-time property of the pair kernel; the
// host picks the kernel whose codes match the potential's classes.
template <int kPQ> constexpr int kRatioP = kPQ >> 4;
template <int kPQ> constexpr int kRatioQ = kPQ & 15;

// u^n by squaring, with the squares shared between the two powers
template <int n, typename T>
__device__ inline T ipow(T u) {
    static_assert(n >= 1 && n <= 15, "power");
    if constexpr (n == 1) return u;
    else if constexpr (n % 2 == 0) {
        const T h = ipow<n / 2>(u);
        return h * h;
    } else {
        return ipow<n - 1>(u) * u;
    }
}

template <typename T, int kPQ = 0, int kPQ1 = kPQ>
__device__ inline ShapeK<T> shape_consts(const Model& m, int cls) {
    constexpr double kLog2e = 1.4426950408889634;
    constexpr double kPi = 3.141592653589793;
    // selected from both classes' values rather than indexed by the per-lane
    // class: an indexed kernel argument is a vector load whose wait would also
    // wait for the pair data the loop prefetches
    const bool c1 = cls != 0;
    const double ir = c1 ? m.inv_re[1] : m.inv_re[0], al = c1 ? m.alpha[1] : m.alpha[0];
    const double ga = c1 ? m.gamma[1] : m.gamma[0], tw = m.taper_inv_w;
    ShapeK<T> k;
    k.p1 = (T)(-al * ir * kLog2e);
    k.p0 = (T)(al * kLog2e);
    k.f1 = (T)(-ga * ir * kLog2e);
    k.f0 = (T)(ga * kLog2e);
    k.u1 = k.u0 = T(0);
    k.second = kPQ1 != kPQ && cls != 0;
    if constexpr (kPQ != 0) {
        // alpha / P of the pair's class (the kernels are compiled for the
        // plan's ratio codes), selected like the other class values
        const double g = c1 ? m.u_rate[1] : m.u_rate[0];
        k.u1 = (T)(-g * ir * kLog2e);
        k.u0 = (T)(g * kLog2e);
    }
    k.kp = (T)(al * ir);
    k.kf = (T)(ga * ir);
    k.r_s = (T)m.r_s;
    k.tw = (T)tw;
    k.kz = (T)(kPi * tw);
    k.kd = (T)(-0.5 * kPi * tw);
    return k;
}

template <typename T> struct Math;

template <> struct Math<double> {
    static __device__ inline double ex2(double y, const PolyCoef& c) { return exp2_bounded(y, c); }
    static __device__ inline double rsq(double v) { return rsqrt_refined(v); }
    // d = r - r_s in [0, width]
    static __device__ inline void taper(double d, const ShapeK<double>& k, double& S, double& sn,
                                        const PolyCoef& c) {
        taper_terms(fma(d, k.kz, -1.5707963267948966), S, sn, c);
    }
};
template <> struct Math<float> {
    static __device__ inline float ex2(float y, const PolyCoef&) { return __builtin_amdgcn_exp2f(y); }
    static __device__ inline float rsq(float v) { return __frsqrt_rn(v); }
    static __device__ inline void taper(float d, const ShapeK<float>& k, float& S, float& sn,
                                        const PolyCoef&) {
        // sin(pi x), cos(pi x) for x = d / width in [0, 1]; the hardware sine
        // and cosine take turns (sin(2 pi y)), so y = x / 2 in [0, 1/2]
        const float y = 0.5f * d * k.tw;
        sn = __builtin_amdgcn_sinf(y);
        S = 0.5f * (1.0f + __builtin_amdgcn_cosf(y));
    }
};

// Both radial shapes and their derivatives at distance r (r < r_c). A
// two-ratio kernel (kPQ1 != kPQ) serves pairs of ratio P+1 : Q+1 with the same
// body: one more factor u on both powers, chosen per lane and folded into the
// taper value, so that it costs no multiply below the taper's start.
template <typename T, int kPQ = 0, int kPQ1 = kPQ>
__device__ inline void shapes(T r, const ShapeK<T>& k, T& gp, T& dgp, T& gf, T& dgf, const PolyCoef& pc) {
    T ep, ef, t = T(1);
    if constexpr (kPQ != 0) {
        const T u = Math<T>::ex2(fma(r, k.u1, k.u0), pc);
        ep = ipow<kRatioP<kPQ>>(u);
        ef = ipow<kRatioQ<kPQ>>(u);
        if constexpr (kPQ1 != kPQ) {
            static_assert(kRatioP<kPQ1> == kRatioP<kPQ> + 1 && kRatioQ<kPQ1> == kRatioQ<kPQ> + 1,
                          "two-ratio kernels differ by one in both powers");
            t = k.second ? u : T(1);
        }
    } else {
        ep = Math<T>::ex2(fma(r, k.p1, k.p0), pc);
        ef = Math<T>::ex2(fma(r, k.f1, k.f0), pc);
    }
    // the factor t common to both shapes rides on the taper: S t and S' t
    T S = t, dS = T(0);
    if (r > k.r_s) {
        T sn;
        Math<T>::taper(r - k.r_s, k, S, sn, pc);
        dS = k.kd * sn;
        if constexpr (kPQ1 != kPQ) {
            S *= t;
            dS *= t;
        }
    }
    gp = ep * S;
    dgp = ep * (dS - k.kp * S);
    gf = ef * S;
    dgf = ef * (dS - k.kf * S);
}

// 27-node product rule on the relative coordinate (width s). Node n sits at
// rbar + h zeta_n with zeta_n in {-1, 0, 1}^3 and h = sqrt(3) s. With
// c_n = W_n g'(r_n) / r_n for a shape g, the gradient sum_n c_n (rbar + h zeta_n)
// equals rbar A + h (P - M) and the width sum sqrt(3) sum_n c_n zeta_n . (rbar + h zeta_n)
// equals sqrt(3) (rbar . (P - M) + h sum_k (P_k + M_k)), where A = sum_n c_n and
// P_k, M_k sum c_n over the nodes with zeta_k = +1 and -1. So a node only adds
// c_n to a few sums: to its x plane a (whose three sums give A, P_x and M_x)
// and to the y and z sums its offset selects.
template <typename T, int kPQ = 0, int kPQ1 = kPQ>
__device__ inline void pair_moments_gh27(const Model& m, int cls, double rx, double ry, double rz,
                                         double s, T out[kFBlk]) {
    constexpr T kSqrt3 = T(1.7320508075688772935);
    const ShapeK<T> K = shape_consts<T, kPQ, kPQ1>(m, cls);
    const T rc2 = (T)(m.r_c * m.r_c);
    const T h = (T)s * kSqrt3;
    const T R[3] = {(T)rx, (T)ry, (T)rz};
    const T X2[3] = {(R[0] - h) * (R[0] - h), R[0] * R[0], (R[0] + h) * (R[0] + h)};
    const T Y2[3] = {(R[1] - h) * (R[1] - h), R[1] * R[1], (R[1] + h) * (R[1] + h)};
    const T Z2[3] = {(R[2] - h) * (R[2] - h), R[2] * R[2], (R[2] + h) * (R[2] + h)};
    constexpr T w1[3] = {T(1.0 / 6.0), T(2.0 / 3.0), T(1.0 / 6.0)};
#pragma unroll
    for (int k = 0; k < kFBlk; ++k) out[k] = T(0);
    // [shape][offset index]: shape 0 = phi, 1 = f; the middle y, z entries stay unused
    T sx[2][3] = {}, sy[2][3] = {}, sz[2][3] = {};
    // f and f'/r at the mean separation: the FP64 kernel keeps these two and
    // forms the gradient after the loop (four live values fewer, no spill);
    // the FP32 kernel measured faster writing the four terms at the node
    T f_mid = T(0), g_mid = T(0);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
#pragma unroll
        for (int b = 0; b < 3; ++b) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const T r2 = X2[a] + Y2[b] + Z2[c];
                if (r2 < rc2 && r2 > T(0)) {
                    const T W = w1[a] * w1[b] * w1[c];
                    const T rinv = Math<T>::rsq(r2);
                    const T r = r2 * rinv;
                    T gp, dgp, gf, dgf;
                    shapes<T, kPQ, kPQ1>(r, K, gp, dgp, gf, dgf, m.poly);
                    const T wr = W * rinv;
                    const T cp = wr * dgp, cf = wr * dgf;
                    out[M_PHI] += W * gp;
                    out[M_F] += W * gf;
                    sx[0][a] += cp;
                    sx[1][a] += cf;
                    if (b != 1) {
                        sy[0][b] += cp;
                        sy[1][b] += cf;
                    }
                    if (c != 1) {
                        sz[0][c] += cp;
                        sz[1][c] += cf;
                    }
                    if (a == 1 && b == 1 && c == 1) {  // node at the mean: rho|_0 terms
                        f_mid = gf;
                        g_mid = dgf * rinv;
                        if constexpr (sizeof(T) != sizeof(double)) {
                            out[M_F0] = f_mid;
#pragma unroll
                            for (int k = 0; k < 3; ++k) out[M_GF0 + k] = g_mid * R[k];
                        }
                    }
                }
            }
        }
    }
    if constexpr (sizeof(T) == sizeof(double)) {
        out[M_F0] = f_mid;
#pragma unroll
        for (int k = 0; k < 3; ++k) out[M_GF0 + k] = g_mid * R[k];
    }
    const T sinv = T(1) / (T)s;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int g = q == 0 ? M_GPHI : M_GF, w = q == 0 ? M_SPHI : M_SF;
        const T A = sx[q][0] + sx[q][1] + sx[q][2];
        const T B[3] = {sx[q][2] - sx[q][0], sy[q][2] - sy[q][0], sz[q][2] - sz[q][0]};
        const T C = (sx[q][0] + sx[q][2]) + (sy[q][0] + sy[q][2]) + (sz[q][0] + sz[q][2]);
#pragma unroll
        for (int k = 0; k < 3; ++k) out[g + k] = R[k] * A + h * B[k];
        out[w] = kSqrt3 * (R[0] * B[0] + R[1] * B[1] + R[2] * B[2] + h * C) * sinv;
    }
    // d/dsigma_e = (sigma_e / s) d/ds: divided by sigma_e both ends get (d/ds)/s
    out[M_SPHI_HI] = out[M_SPHI];
    out[M_SF_HI] = out[M_SF];
}

// The density shape f and its derivative at r < r_c.
template <typename T>
__device__ inline void density_shape(T r, const ShapeK<T>& k, T& g, T& dg, const PolyCoef& pc) {
    const T e = Math<T>::ex2(fma(r, k.f1, k.f0), pc);
    T S = T(1), dS = T(0);
    if (r > k.r_s) {
        T sn;
        Math<T>::taper(r - k.r_s, k, S, sn, pc);
        dS = k.kd * sn;
    }
    g = e * S;
    dg = e * (dS - k.kf * S);
}

// Degree-3 rule of App. A in the pair's six coordinates. A node that moves the
// lo end by -c h e_a or the hi end by +c h e_a (h = sqrt(6) sigma_end, c = +-1)
// sits at d = rbar + c h e_a, and d.(dd/dsigma_end) = c sqrt(6) d_a.
template <typename T, int kPQ = 0, int kPQ1 = kPQ>
__device__ inline void pair_moments_d3(const Model& m, int cls, double rx, double ry, double rz,
                                       double si, double sj, T out[kFBlk]) {
    constexpr T kSqrt6 = T(2.4494897427831780982);
    constexpr T W = T(1.0 / 12.0);
    const ShapeK<T> K = shape_consts<T, kPQ, kPQ1>(m, cls);
    const T rc2 = (T)(m.r_c * m.r_c);
    const T R[3] = {(T)rx, (T)ry, (T)rz};
    const T R2[3] = {R[0] * R[0], R[1] * R[1], R[2] * R[2]};
    const T other[3] = {R2[1] + R2[2], R2[0] + R2[2], R2[0] + R2[1]};
#pragma unroll
    for (int k = 0; k < kFBlk; ++k) out[k] = T(0);
    // Node sums by offset. A node's gradient term is g'/r d_b, where d_b = R_b
    // off the node's axis and R_a + c h_e on it, and its width term is
    // c d_a g'/r; with U[q][e] = sum of g'/r over end e's six nodes and
    // P[q][e][a] = sum over c of c g'/r on axis a, the gradient is
    // R_b (U_lo + U_hi) + h_lo P_lo,b + h_hi P_hi,b and end e's width sum is
    // R.P_e + h_e U_e (q: 0 = phi, 1 = f). Two sums per node and shape
    // instead of four.
    const T hh[2] = {kSqrt6 * (T)si, kSqrt6 * (T)sj};
    T P[2][2][3] = {}, U[2][2] = {};
#pragma unroll
    for (int e = 0; e < 2; ++e) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
#pragma unroll
            for (int c = -1; c <= 1; c += 2) {
                const T da = R[a] + T(c) * hh[e];
                const T r2 = other[a] + da * da;
                if (r2 < rc2 && r2 > T(0)) {
                    const T rinv = Math<T>::rsq(r2);
                    const T r = r2 * rinv;
                    T gp, dgp, gf, dgf;
                    shapes<T, kPQ, kPQ1>(r, K, gp, dgp, gf, dgf, m.poly);
                    const T cp = W * dgp * rinv, cf = W * dgf * rinv;
                    out[M_PHI] += W * gp;
                    out[M_F] += W * gf;
                    U[0][e] += cp;
                    U[1][e] += cf;
                    if (c > 0) {
                        P[0][e][a] += cp;
                        P[1][e][a] += cf;
                    } else {
                        P[0][e][a] -= cp;
                        P[1][e][a] -= cf;
                    }
                }
            }
        }
    }
    // (d<g>/dsigma_e) / sigma_e = sqrt(6) (width sum of end e) / sigma_e
    const T fi = kSqrt6 / (T)si, fj = kSqrt6 / (T)sj;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int g = q == 0 ? M_GPHI : M_GF;
        const T tot = U[q][0] + U[q][1];
#pragma unroll
        for (int b = 0; b < 3; ++b) out[g + b] = R[b] * tot + hh[0] * P[q][0][b] + hh[1] * P[q][1][b];
        const T w0 = R[0] * P[q][0][0] + R[1] * P[q][0][1] + R[2] * P[q][0][2] + hh[0] * U[q][0];
        const T w1 = R[0] * P[q][1][0] + R[1] * P[q][1][1] + R[2] * P[q][1][2] + hh[1] * U[q][1];
        out[q == 0 ? M_SPHI : M_SF] = w0 * fi;
        out[q == 0 ? M_SPHI_HI : M_SF_HI] = w1 * fj;
    }
    const T r2c = other[0] + R2[0];
    if (r2c < rc2 && r2c > T(0)) {  // the density at the mean positions
        const T rinv = Math<T>::rsq(r2c);
        T gf, dgf;
        density_shape<T>(r2c * rinv, K, gf, dgf, m.poly);
        const T g0 = dgf * rinv;
        out[M_F0] = gf;
        out[M_GF0 + 0] = g0 * R[0];
        out[M_GF0 + 1] = g0 * R[1];
        out[M_GF0 + 2] = g0 * R[2];
    }
}

// A system's periodic box, copied into registers before a pair loop: read
// through the system record inside the loop, the compiler reloads it after
// every store (it may alias) and waits for every load in flight.
struct Box {
    double len[3], inv[3];  // lengths and their reciprocals
    bool periodic[3];
};

__device__ inline Box box_of(const SysDesc& S) {
    Box b;
    for (int k = 0; k < 3; ++k) {
        b.len[k] = S.box[k];
        b.inv[k] = 1.0 / S.box[k];
        b.periodic[k] = S.periodic[k] != 0;
    }
    return b;
}

// kRcp: the image multiple by the reciprocal length. It differs from the
// quotient's rounding only within an ulp of a half-integer, i.e. for a
// separation of half a box, which no listed pair has (lists reach less than
// half a box), so the results are the same. The FP32-mixed kernels take it
// (three divisions fewer per pair); the FP64 kernels, at their register limit,
// would spill the three reciprocals and keep the division.
template <bool kRcp>
__device__ inline void min_image(const Box& B, double& dx, double& dy, double& dz) {
    if (kRcp) {
        if (B.periodic[0]) dx -= B.len[0] * rint(dx * B.inv[0]);
        if (B.periodic[1]) dy -= B.len[1] * rint(dy * B.inv[1]);
        if (B.periodic[2]) dz -= B.len[2] * rint(dz * B.inv[2]);
    } else {
        if (B.periodic[0]) dx -= B.len[0] * rint(dx / B.len[0]);
        if (B.periodic[1]) dy -= B.len[1] * rint(dy / B.len[1]);
        if (B.periodic[2]) dz -= B.len[2] * rint(dz / B.len[2]);
    }
}

}  // namespace

// 16-byte vector of T, for whole-line loads and stores of the pair blocks
template <typename T>
struct alignas(16) Vec16 {
    static constexpr int n = 16 / sizeof(T);
    T v[n];
};

// The 16 moments of one pair from its mean separation (before the minimum
// image), its two widths and its class.
// kPQ0, kPQ1: the ratio codes the kernel is compiled for, per pair class
// (host-host, host-interstitial), served by one body (two bodies in one
// loop spill at the FP64 kernels' 128 VGPRs).
template <typename T, int kRule, int kPQ0 = 0, int kPQ1 = 0>
__device__ inline void pair_all_moments(const Model& m, const Box& B, double rx, double ry,
                                        double rz, double si, double sj, int cls, T out[kFBlk]) {
#pragma unroll
    for (int k = 0; k < kFBlk; ++k) out[k] = T(0);
    min_image<sizeof(T) == sizeof(float)>(B, rx, ry, rz);
    const double s = sqrt(si * si + sj * sj);
    // a pair contributes iff some node lies inside r_c: the farthest node is
    // 3 s from rbar under the product rule, sqrt(6) max(sigma) under degree 3
    const double reach = kRule == MXE_QUAD_DEGREE3 ? 2.449489742783178 * fmax(si, sj) : 3.0 * s;
    if (cls >= 0 && rx * rx + ry * ry + rz * rz < (m.r_c + reach) * (m.r_c + reach)) {
        if (kRule == MXE_QUAD_DEGREE3) pair_moments_d3<T, kPQ0, kPQ1>(m, cls, rx, ry, rz, si, sj, out);
        else pair_moments_gh27<T, kPQ0, kPQ1>(m, cls, rx, ry, rz, s, out);
    }
}

// The FP64 kernels are held at 128 VGPRs (4 waves per SIMD): the 27-node
// kernel's node sums would otherwise take 131 and drop to 3 waves. The FP32
// ones at 5 waves (the two-exponential 27-node kernel would take 110 VGPRs,
// 4 waves: 0.249 -> 0.241 ms at 5 on the 256k-site vacancy crystal).
template <typename T, int kBS, int kRule, int kPQ0 = 0, int kPQ1 = 0>
__global__ __launch_bounds__(kBS) __attribute__((amdgpu_waves_per_eu(sizeof(T) == 8 ? 4 : 5)))
void k_pair(Dev d, Model m) {
    // Two latency measures:
    //  * a software pipeline of the pair data: the endpoint indices are loaded
    //    two pairs ahead and the endpoints' positions, widths and types one
    //    pair ahead, so the quadrature of a pair never waits for the dependent
    //    loads of its own data;
    //  * a thread's 16 moments are staged in LDS and written back as
    //    contiguous ranges of force blocks (a wavefront's 64, or the block's
    //    kBS), 16 B per lane and store, so a store covers whole cache lines
    //    instead of 16 B of 64 lines.
    constexpr int per = kFBlk / Vec16<T>::n;  // vectors per force block
    constexpr int kRow = per + 1;             // LDS row (odd stride against bank conflicts)
    // pair chunks are sized to capacity and only the leading ones are active,
    // so they keep the plain order (contiguous ranges per XCD would idle XCDs);
    // 2^pair_shift blocks share a chunk, each taking a contiguous sub-range
    const Chunk ch = d.pchunks[blockIdx.x >> m.pair_shift];
    const SysCtl& c = d.ctl[ch.sys];
    if (idle(c, m)) return;  // uniform over the block
    const SysDesc& S = d.sys[ch.sys];
    const Box B = box_of(S);
    const int64_t sub = kPairChunk >> m.pair_shift;
    const int64_t cstart = ch.start + (int64_t)(blockIdx.x & ((1u << m.pair_shift) - 1)) * sub;
    const int64_t pend =
        min(min((int64_t)ch.end, cstart + sub), S.pair_base + min((int64_t)c.n_pairs, S.pair_cap));
    Vec16<T>* fblk = (Vec16<T>*)d.fblk;
    T* dblk = (T*)d.dblk;

    // a pair past the chunk end reads site 0 (always present) and computes nothing
    __shared__ Vec16<T> stage[kBS * kRow];
    auto ends = [&](int64_t q, int& a, int& b) {
        a = 0;
        b = 0;
        if (q < pend) {
            a = d.pair_i[q];
            b = d.pair_j[q];
        }
    };
    struct Ends {
        double xi, yi, zi, si, xj, yj, zj, sj;
        int ti, tj;
    };
    auto site_data = [&](int a, int b) {
        return Ends{d.qx[a], d.qy[a], d.qz[a], d.sigma[a], d.qx[b], d.qy[b], d.qz[b], d.sigma[b],
                    (int)d.type[a], (int)d.type[b]};
    };
    const int64_t p0 = cstart + threadIdx.x;
    int ia, ja;
    ends(p0, ia, ja);
    Ends cur = site_data(ia, ja);
    ends(p0 + kBS, ia, ja);  // indices of the next pair
    // the loop head uses the next pair's indices, arrived either here or
    // before the previous batch's stores: with this wait both ways in
    // agree, and the head waits for nothing (it would else wait for the
    // stores in flight, see below)
    __builtin_amdgcn_s_waitcnt(0x0F70);
    for (int64_t base = cstart; base < pend; base += kBS) {  // uniform over the block
        const int64_t p = base + threadIdx.x;
        const Ends nxt = site_data(ia, ja);  // next pair's data (its indices arrived earlier)
        ends(p + 2 * kBS, ia, ja);           // indices two pairs ahead
        T out[kFBlk];
        pair_all_moments<T, kRule, kPQ0, kPQ1>(m, B, cur.xj - cur.xi, cur.yj - cur.yi, cur.zj - cur.zi, cur.si,
                                               cur.sj, p < pend ? pair_cls(cur.ti, cur.tj) : -1, out);
        // Loads and stores share one counter: a wait for a load also waits
        // for everything issued before it, and where the compiler cannot
        // count what was issued after it (the store loop below has a
        // variable trip count) it waits for everything, this batch's stores
        // included. The prefetched loads have long arrived by now and the
        // previous batch's stores are a whole quadrature old: wait here,
        // before this batch's stores, and nothing the next batch needs is
        // in flight behind them (vmcnt 0; expcnt and lgkmcnt not waited on).
        __builtin_amdgcn_s_waitcnt(0x0F70);
        if (p < pend) {
            dblk[2 * p] = out[M_F];
            dblk[2 * p + 1] = out[M_F0];
        }
#pragma unroll
        for (int v = 0; v < per; ++v) {
            Vec16<T> b;
#pragma unroll
            for (int e = 0; e < Vec16<T>::n; ++e) b.v[e] = out[v * Vec16<T>::n + e];
            stage[threadIdx.x * kRow + v] = b;
        }
        // (not the FP64 two-exponential 27-node kernel: there it spills at 128 VGPRs)
        if constexpr (kRule == MXE_QUAD_GH27 && (kPQ0 != 0 || sizeof(T) == sizeof(float))) {
            // each wavefront writes its own 64 blocks (one contiguous range):
            // no block barrier, as a wavefront's LDS operations execute in
            // order (the wave barriers only keep the compiler from moving LDS
            // accesses across); the loop stays rolled, as unrolled the
            // compiler waits for each store before reusing its data register
            __builtin_amdgcn_wave_barrier();
            const int w0 = (int)(threadIdx.x & ~(kWave - 1)), ln = (int)(threadIdx.x & (kWave - 1));
            const int64_t wb = base + w0;
            const int nw = (int)max((int64_t)0, min((int64_t)kWave, pend - wb));
#pragma unroll 1
            for (int q = ln; q < nw * per; q += kWave) fblk[wb * per + q] = stage[(w0 + q / per) * kRow + q % per];
            __builtin_amdgcn_wave_barrier();
        } else {
            // the degree-3 kernels measured faster writing block-wide
            // (FP64 0.293 against 0.304 ms, FP32 0.178 against 0.192 ms on the
            // 256k-site vacancy crystal)
            __syncthreads();
            const int nb = (int)min((int64_t)kBS, pend - base);  // pairs of this batch
            for (int q = threadIdx.x; q < nb * per; q += kBS) fblk[base * per + q] = stage[(q / per) * kRow + q % per];
            __syncthreads();  // the stage is rewritten by the next batch
        }
        cur = nxt;
    }
}

// Gathers run LPS lanes per site, so one wavefront serves 64 / LPS sites at a
// time and keeps that many sites' loads in flight.
// Density gather: row entries per lane in flight, so that a site's lanes hold
// 64 entries at once (one iteration for most rows). Measured with 8 lanes
// (the tuned width): 8 entries per lane beat 2, 4 and 6 (82 VGPRs in FP64,
// 5 waves per SIMD instead of 8).
template <int kLPS>
constexpr int kDensDepth = kLPS >= 64 ? 1 : 64 / kLPS;
// kLPS (8, 16, 32 or 64) is chosen per plan (tuned); kGroups sites run per block.

template <int LPS>
__device__ inline double group_sum(double v) {
#pragma unroll
    for (int o = LPS / 2; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

template <typename T, int kLPS>
__global__ __launch_bounds__(kChunk) void k_density(Dev d, Model m) {
    constexpr int kGroups = kChunk / kLPS;
    // kGatherSplit blocks per site chunk, each taking a contiguous part of it
    const int ub = xcd_unit_strided(d.n_chunks, kGatherSplit, m.gather_stride);
    if (ub >= d.n_chunks * kGatherSplit) return;
    const Chunk ch = d.chunks[ub / kGatherSplit];
    constexpr int kPart = kChunk / kGatherSplit;
    const int i_lo = ch.start + (ub % kGatherSplit) * kPart, i_hi = min(ch.end, i_lo + kPart);
    if (idle(d.ctl[ch.sys], m)) return;
    const int grp = threadIdx.x / kLPS, sub = threadIdx.x % kLPS;
    const T* dblk = (const T*)d.dblk;
    const int K = d.K;
    for (int i = i_lo + grp; i < i_hi; i += kGroups) {
        const int cnt = d.nbr_cnt[i];
        const int* row = d.nbr + (int64_t)i * K;
        const int* prow = d.pid + (int64_t)i * K;
        double rb = 0.0, r0 = 0.0;
        // a lane takes kDensDepth entries per iteration (k, k + kLPS, ...): their
        // loads are in flight together and they are added in entry order
        // (loading the next entries' (j, pair id) ahead measured slower in FP64)
        for (int k = sub; k < cnt; k += kDensDepth<kLPS> * kLPS) {
            int jc[kDensDepth<kLPS>], pc[kDensDepth<kLPS>];
#pragma unroll
            for (int u = 0; u < kDensDepth<kLPS>; ++u) {
                const int kk = k + u * kLPS;
                jc[u] = 0;
                pc[u] = -1;
                if (kk < cnt) {
                    jc[u] = row[kk];
                    pc[u] = prow[kk];
                }
            }
            double bj[kDensDepth<kLPS>], fa[kDensDepth<kLPS>], fb[kDensDepth<kLPS>];
#pragma unroll
            for (int u = 0; u < kDensDepth<kLPS>; ++u) {  // an absent entry reads pair 0 and site 0, adds nothing
                const int64_t pp = pc[u] < 0 ? 0 : pc[u];
                bj[u] = d.emit[pc[u] < 0 ? 0 : jc[u]];
                fa[u] = (double)dblk[2 * pp];
                fb[u] = (double)dblk[2 * pp + 1];
            }
#pragma unroll
            for (int u = 0; u < kDensDepth<kLPS>; ++u) {
                if (pc[u] < 0) continue;
                rb += bj[u] * fa[u];
                r0 += bj[u] * fb[u];
            }
        }
        rb = group_sum<kLPS>(rb);
        r0 = group_sum<kLPS>(r0);
        if (sub == 0) {
            // (the per-species tables are indexed by the site's species and
            // loads follow stores here: each such load's wait also waits for
            // the stores in flight, yet the forms without those waits, as in
            // the force gather, measured slower in this kernel: 150 -> 156-159
            // us on the 256k-site vacancy crystal)
            const int ti = d.type[i];
            const double xi = d.x[i];
            d.rho_bar[i] = rb;
            d.rho0[i] = r0;
            // the embedding share c_i G_i carries the site's weight theta_i = T / T_i
            const double th = theta_at(d, d.sys[ch.sys].T, i);
            const double emit_i = d.emit[i];
            double G = 0.0, A = 0.0, B = 0.0;
            const bool embeds = m.c4[occ_sp1(ti)] != 0.0 || m.c4[occ_sp0(ti)] != 0.0;
            if (embeds) {
                if (r0 > 1e-12) {
                    // F~(rho) = -sqrt(rho): F~' = -1/(2 sqrt rho), F~'' = 1/(4 rho^1.5)
                    const double sq = sqrt(r0);
                    const double F1 = -0.5 / sq, F2 = 0.25 / (sq * r0);
                    const double ch_i = mixhat_indexed(m.c4, ti, xi);
                    G = -sq + F1 * (rb - r0);
                    A = th * ch_i * F1;
                    B = th * ch_i * F2 * (rb - r0);
                } else {
                    atomicOr(&d.ctl[ch.sys].status, MXE_STAT_RHO);
                }
            }
            d.G[i] = G;
            d.Ahat[i] = A;
            d.Bhat[i] = B;
            // record read by the force gather of the neighbours: A~ = w A^, B~ = w B^,
            // the emission, the pair amplitude against a partner of species A, B, S
            // and the site's weight theta
            const double w = occ_partial(ti) ? xi : 1.0;
            const double p1 = occ_p1(ti, xi);
            const int s1 = occ_sp1(ti), s0 = occ_sp0(ti);
            // (kept in the moments' precision: FP32 in the mixed variant)
            T* R = (T*)d.srec + (int64_t)i * kSRec;
            R[0] = (T)(w * A);
            R[1] = (T)(w * B);
            R[2] = (T)emit_i;
            for (int k = 0; k < 3; ++k) R[3 + k] = (T)(p1 * m.a4[k][s1] + (1.0 - p1) * m.a4[k][s0]);
            R[6] = (T)th;
            R[7] = T(0);
        }
    }
}

// Gradient of F (App. B.2.1) for site i, normalised by its vibrating
// fraction w_i, with the pair amplitude a_ij = sum_kl p_ik p_jl a_kl, the
// emissions b, the embedding strengths c, A_j = c_j F~'(rho0_j) and
// B_j = c_j F~''(rho0_j)(rho_bar_j - rho0_j):
//   -dF/dq_i / w_i = sum_j sign [ahat grad<phi> + (Ahat_i b_j + A_j bhat_i) grad<f>
//                                + (Bhat_i b_j + B_j bhat_i) grad f0]
//   -dF/dsigma_i / w_i = -sigma_i sum_j [ahat <phi>_si + (Ahat_i b_j + A_j bhat_i) <f>_si]
//                       + 3 kT / sigma_i,   <g>_si = (d<g>/dsigma_i) / sigma_i
//   mu_i = sum_j da_ij/dx_i <phi> + db_i/dx_i sum_j (A_j <f> + B_j f0)
//          + dc_i/dx_i G_i - 3 kT dw_i/dx_i ln sigma_i
// Force gather layout: kLPS lanes per site; inside them, groups of kQ lanes
// share one row entry, each lane loading its part of the pair's force block
// (4 / kQ quarters of four slots: 4q' .. 4q'+3) and the neighbour's record.
// A wave-wide block load then touches one cache line per entry instead of one
// per lane. FP64 blocks (128 B) take four lanes per entry; the 64-B FP32
// blocks take two, so twice the entries are in flight for the same registers.
template <typename T>
constexpr int kQ = sizeof(T) == sizeof(double) ? 4 : 2;

// At most 128 VGPRs (4 waves per SIMD): the FP32 variant would otherwise take
// 129 and drop to 3 waves; fewer waves measured slower in every variant tried.
template <typename T, int kLPS>
__global__ __launch_bounds__(kChunk) __attribute__((amdgpu_waves_per_eu(4))) void k_force(Dev d, Model m) {
    constexpr int kGroups = kChunk / kLPS;
    __shared__ double red[kGroups][6];
    // kForceSplit blocks per site chunk, each taking a contiguous part of it
    // and writing its own partial row (combined per chunk by k_force_fold or the FIRE control)
    const int ub = xcd_unit_strided(d.n_chunks, kForceSplit, m.gather_stride);
    if (ub >= d.n_chunks * kForceSplit) return;
    const int cb = ub / kForceSplit;
    constexpr int kPart = kChunk / kForceSplit;
    const Chunk ch = d.chunks[cb];
    const int i_lo = ch.start + (ub % kForceSplit) * kPart, i_hi = min(ch.end, i_lo + kPart);
    const int sys = ch.sys;
    if (idle(d.ctl[sys], m)) return;
    const SysDesc& S = d.sys[sys];
    const double kT = S.kT, T_sys = S.T;
    const bool site_T = d.T_site != nullptr;
    const int grp = threadIdx.x / kLPS, sub = threadIdx.x % kLPS;
    constexpr int kQL = kQ<T>;                // lanes per entry
    constexpr int kQuarters = 4 / kQL;        // quarters of the block per lane
    const int q = sub % kQL, es = sub / kQL;  // the lane's part of the block; entry slot
    const Vec16<T>* fblk = (const Vec16<T>*)d.fblk;
    constexpr int per = kFBlk / Vec16<T>::n;  // vectors per block
    constexpr int perq = per / kQL;           // vectors per lane
    const int K = d.K;
    double pe = 0.0, pfmax = 0.0, pfv = 0.0, pff = 0.0, pvv = 0.0, psx = 0.0;
    int bad = 0;
    for (int i = i_lo + grp; i < i_hi; i += kGroups) {
        // the site's loads, and its first row entry's, in one round trip (the
        // entry loaded unconditionally, its index clamped into the row)
        const int cnt = d.nbr_cnt[i];
        const int* row = d.nbr + (int64_t)i * K;
        const int* prow = d.pid + (int64_t)i * K;
        const int e0 = min(es, K - 1);
        const int j0 = row[e0], p0 = prow[e0];
        const int ti = d.type[i];
        const double xi = d.x[i], si = d.sigma[i];
        const double Ahi = d.Ahat[i], Bhi = d.Bhat[i];
        const double pi1 = occ_p1(ti, xi);
        const int i1 = occ_sp1(ti), i0 = occ_sp0(ti);
        const double bhat_i = mixhat(m.b4, ti, xi), db_i = mixdx(m.b4, ti);
        const bool part_i = occ_partial(ti), mob_i = occ_mobile(ti);
        const double th_i = theta_at(d, T_sys, i);
        double fx = 0.0, fy = 0.0, fz = 0.0, fsg = 0.0, mu = 0.0, ep = 0.0;
        // the next entry's (j, pair id) load while this entry's block and record
        // are fetched, so an iteration waits for one round trip instead of three
        int jn = es < cnt ? j0 : 0, pn = es < cnt ? p0 : -1;
        for (int k = es; k < cnt; k += kLPS / kQL) {
            const int j = jn, p = pn;
            if (k + kLPS / kQL < cnt) {
                jn = row[k + kLPS / kQL];
                pn = prow[k + kLPS / kQL];
            }
            if (p < 0) continue;
            T mq[4 * kQuarters];
#pragma unroll
            for (int v = 0; v < perq; ++v) {
                const Vec16<T> b = fblk[(int64_t)p * per + q * perq + v];
#pragma unroll
                for (int e = 0; e < Vec16<T>::n; ++e) mq[v * Vec16<T>::n + e] = b.v[e];
            }
            double Aj, Bj, bj, ampA[3], th_j;
            if constexpr (sizeof(T) == sizeof(double)) {
                const double2* R = (const double2*)((const double*)d.srec + (int64_t)j * kSRec);
                const double2 r01 = R[0], r23 = R[1], r45 = R[2];
                Aj = r01.x;
                Bj = r01.y;
                bj = r23.x;
                ampA[0] = r23.y;
                ampA[1] = r45.x;
                ampA[2] = r45.y;
                th_j = site_T ? R[3].x : 1.0;
            } else {
                const float4* R = (const float4*)((const float*)d.srec + (int64_t)j * kSRec);
                const float4 r0 = R[0], r1 = R[1];
                Aj = r0.x;
                Bj = r0.y;
                bj = r0.z;
                ampA[0] = r0.w;
                ampA[1] = r1.x;
                ampA[2] = r1.y;
                th_j = r1.z;
            }
            const double a1 = ampA[i1];
            const double a0 = i0 < 3 ? ampA[i0] : 0.0;
            const double aij = pi1 * a1 + (1.0 - pi1) * a0;
            // the pair term sits half in each end's share: weight (theta_i + theta_j) / 2
            const double tij = site_T ? 0.5 * (th_i + th_j) : 1.0;
            const double ahat = tij * (part_i ? a1 : aij);
            const double dadx = mob_i ? tij * (a1 - a0) : 0.0;
            const double hA = Ahi * bj + Aj * bhat_i;
            const double hB = Bhi * bj + Bj * bhat_i;
            const double sg = j > i ? 1.0 : -1.0;
#pragma unroll
            for (int u = 0; u < kQuarters; ++u) {
                const int qd = q * kQuarters + u;  // the quarter of the block
                const double m0 = (double)mq[4 * u], m1 = (double)mq[4 * u + 1];
                const double m2 = (double)mq[4 * u + 2], m3 = (double)mq[4 * u + 3];
                if (qd == 0) {         // <phi>, grad <phi>
                    ep += aij * m0;
                    mu += dadx * m0;
                    const double c = sg * ahat;
                    fx += c * m1;
                    fy += c * m2;
                    fz += c * m3;
                } else if (qd == 1) {  // lo-end width term of <phi>, <f>, grad <f> (x, y)
                    if (sg > 0.0) fsg += ahat * m0;
                    mu += db_i * Aj * m1;
                    const double c = sg * hA;
                    fx += c * m2;
                    fy += c * m3;
                } else if (qd == 2) {  // grad <f> (z), lo-end width term of <f>, f0, grad f0 (x)
                    fz += sg * hA * m0;
                    if (sg > 0.0) fsg += hA * m1;
                    mu += db_i * Bj * m2;
                    fx += sg * hB * m3;
                } else {              // grad f0 (y, z), hi-end width terms of <phi>, <f>
                    const double c = sg * hB;
                    fy += c * m0;
                    fz += c * m1;
                    if (sg < 0.0) fsg += ahat * m2 + hA * m3;
                }
            }
        }
        fx = group_sum<kLPS>(fx);
        fy = group_sum<kLPS>(fy);
        fz = group_sum<kLPS>(fz);
        fsg = group_sum<kLPS>(fsg);
        mu = group_sum<kLPS>(mu);
        ep = group_sum<kLPS>(ep);
        if (sub == 0) {
            // every load before the first store (a load issued behind stores
            // waits for them)
            const double Gi = d.G[i];
            const double vx = d.vx[i], vy = d.vy[i], vz = d.vz[i], vs = d.vs[i];
            const double lns = log(si);
            const double fs = -si * fsg + 3.0 * kT / si;
            const double wi = part_i ? xi : 1.0;
            double mui = 0.0, mix = 0.0;
            if (mob_i) {
                // mu_i = gamma_i / beta_i: the x_i-derivative divided by theta_i
                mui = (mu + th_i * mixdx(m.c4, ti) * Gi - 3.0 * kT * (part_i ? 1.0 : 0.0) * lns) / th_i;
                if (held(d, i, ti, MXE_RES_FIX_MU)) mui = d.res_val[i];  // held after the forces
                if (xi > 0.0) mix += xi * log(xi);
                if (xi < 1.0) mix += (1.0 - xi) * log(1.0 - xi);
                mix *= kT;
            }
            const double ei = th_i * (0.5 * ep + mixval(m.c4, ti, xi) * Gi) - 3.0 * kT * wi * lns + mix;
            d.fx[i] = fx;
            d.fy[i] = fy;
            d.fz[i] = fz;
            d.fs[i] = fs;
            d.mu[i] = mui;
            d.e_site[i] = ei;
            pe += ei;
            psx += xi;
            pfmax = fmax(pfmax, fmax(fmax(fabs(fx), fabs(fy)), fmax(fabs(fz), fabs(fs))));
            pfv += fx * vx + fy * vy + fz * vz + fs * vs;
            pff += fx * fx + fy * fy + fz * fz + fs * fs;
            pvv += vx * vx + vy * vy + vz * vz + vs * vs;
            if (!isfinite(fx + fy + fz + fs + ei + mui)) bad = 1;
        }
    }
    if (sub == 0) {
        red[grp][0] = pe;
        red[grp][1] = pfmax;
        red[grp][2] = pfv;
        red[grp][3] = pff;
        red[grp][4] = pvv;
        red[grp][5] = psx;
        if (bad) atomicOr(&d.ctl[sys].status, MXE_STAT_NONFINITE);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double e = red[0][0], fm = red[0][1], fv = red[0][2], ff = red[0][3], vv = red[0][4], sx = red[0][5];
        for (int g = 1; g < kGroups; ++g) {
            e += red[g][0];
            fm = fmax(fm, red[g][1]);
            fv += red[g][2];
            ff += red[g][3];
            vv += red[g][4];
            sx += red[g][5];
        }
        double* Q = d.part_sub + (int64_t)ub * kNPart;
        Q[P_E] = e;
        Q[P_FMAX] = fm;
        Q[P_FV] = fv;
        Q[P_FF] = ff;
        Q[P_VV] = vv;
        Q[P_SUMX] = sx;
    }
}

// A site chunk's kForceSplit partial rows summed into the chunk's row, by
// kForceSplit lanes per chunk with a fixed butterfly order (the order the FIRE
// control uses when it folds the rows itself). Launched for plans with a
// system of more chunks than the control block has threads; a fence in every
// force block instead would write back the L2.
__global__ __launch_bounds__(kChunk) void k_force_fold(Dev d, Model m) {
    static_assert(kForceSplit <= kWave && (kForceSplit & (kForceSplit - 1)) == 0, "fold width");
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    const int cb = t / kForceSplit, k = t % kForceSplit;
    const bool live = cb < d.n_chunks && !idle(d.ctl[d.chunks[cb < d.n_chunks ? cb : 0].sys], m);
    double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (live) {
        const double2* R = (const double2*)(d.part_sub + ((int64_t)cb * kForceSplit + k) * kNPart);
        const double2 a = R[0], b = R[1], c = R[2];
        v[0] = a.x, v[1] = a.y, v[2] = b.x, v[3] = b.y, v[4] = c.x, v[5] = c.y;
    }
#pragma unroll
    for (int o = 1; o < kForceSplit; o <<= 1) {
#pragma unroll
        for (int j = 0; j < 6; ++j) {
            const double w = __shfl_xor(v[j], o);
            v[j] = j == P_FMAX ? fmax(v[j], w) : v[j] + w;
        }
    }
    if (live && k == 0) {
        double* P = d.part + (int64_t)cb * kNPart;
        for (int j = 0; j < 6; ++j) P[j] = v[j];
    }
}

template <typename T, int kRule, int kPQ0, int kPQ1>
void launch_pair_q(const Dev& d, const Model& m, int bs, hipStream_t s) {
    switch (bs) {
        case 64: k_pair<T, 64, kRule, kPQ0, kPQ1><<<d.n_pchunks << m.pair_shift, 64, 0, s>>>(d, m); break;
        case 128: k_pair<T, 128, kRule, kPQ0, kPQ1><<<d.n_pchunks << m.pair_shift, 128, 0, s>>>(d, m); break;
        default: k_pair<T, 256, kRule, kPQ0, kPQ1><<<d.n_pchunks << m.pair_shift, 256, 0, s>>>(d, m); break;
    }
}

// Kernels compiled for the exponent ratios of the analytic EAM of the
// synthetic workloads (host-host 8 : 6 = 4 : 3, host-interstitial 5 : 4);
// any other potential takes the two-exponential kernel.
template <typename T, int kRule>
void launch_pair_r(const Dev& d, const Model& m, int bs, hipStream_t s) {
    if (m.ratio_pq[0] == 0x43 && m.ratio_pq[1] == 0x54)
        launch_pair_q<T, kRule, 0x43, 0x54>(d, m, bs, s);
    else
        launch_pair_q<T, kRule, 0, 0>(d, m, bs, s);
}

template <typename T>
void launch_pair_t(const Dev& d, const Model& m, int bs, hipStream_t s) {
    if (m.quad_rule == MXE_QUAD_DEGREE3) launch_pair_r<T, MXE_QUAD_DEGREE3>(d, m, bs, s);
    else launch_pair_r<T, MXE_QUAD_GH27>(d, m, bs, s);
}

template <typename T>
void launch_density_t(const Dev& d, const Model& m, int lps, hipStream_t s) {
    switch (lps) {
        case 8: k_density<T, 8><<<xcd_grid_chunks(d.n_chunks, kGatherSplit), kChunk, 0, s>>>(d, m); break;
        case 32: k_density<T, 32><<<xcd_grid_chunks(d.n_chunks, kGatherSplit), kChunk, 0, s>>>(d, m); break;
        case 64: k_density<T, 64><<<xcd_grid_chunks(d.n_chunks, kGatherSplit), kChunk, 0, s>>>(d, m); break;
        default: k_density<T, 16><<<xcd_grid_chunks(d.n_chunks, kGatherSplit), kChunk, 0, s>>>(d, m); break;
    }
}

template <typename T>
void launch_force_t(const Dev& d, const Model& m, int lps, hipStream_t s) {
    switch (lps) {
        case 8: k_force<T, 8><<<xcd_grid_chunks(d.n_chunks, kForceSplit), kChunk, 0, s>>>(d, m); break;
        case 32: k_force<T, 32><<<xcd_grid_chunks(d.n_chunks, kForceSplit), kChunk, 0, s>>>(d, m); break;
        case 64: k_force<T, 64><<<xcd_grid_chunks(d.n_chunks, kForceSplit), kChunk, 0, s>>>(d, m); break;
        default: k_force<T, 16><<<xcd_grid_chunks(d.n_chunks, kForceSplit), kChunk, 0, s>>>(d, m); break;
    }
}

void launch_pair(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) launch_pair_t<float>(d, m, m.pair_block, s);
    else launch_pair_t<double>(d, m, m.pair_block, s);
}

void launch_density(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) launch_density_t<float>(d, m, m.gather_lanes, s);
    else launch_density_t<double>(d, m, m.gather_lanes, s);
}

void launch_force(const Dev& d, const Model& m, int precision, hipStream_t s) {
    if (precision == MXE_FP32_MIXED) launch_force_t<float>(d, m, m.force_lanes, s);
    else launch_force_t<double>(d, m, m.force_lanes, s);
    if (m.fold_rows) k_force_fold<<<(d.n_chunks * kForceSplit + kChunk - 1) / kChunk, kChunk, 0, s>>>(d, m);
}

}  // namespace mxe
