/*
 * mxe_oracle.c -- plain FP64 CPU oracle of the MXE mean-field EAM evaluation,
 * FIRE relaxation and master-equation update (arXiv:1910.01235).
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the tests, the smoke check and the CPU
 * baseline leg of the benchmark. Nothing in the GPU product path uses it.
 *
 * The code follows the paper's formulas directly, with no blocking or fusion:
 *   - mean-field free energy: Sec. 2.1, Eq. (Grand-Canonical-Free-Energy), with
 *     the trial Hamiltonian of Eq. (localHamiltonian) giving a Gaussian of
 *     per-axis variance sigma^2 = 1/(beta m omega^2) (App. A, exponent of p0);
 *   - EAM thermalisation: App. B.2, Eqs. (EAM_mxe), (F_taylor_mxe); alloys with
 *     occupancies: App. B.2.1, Eqs. (EAM-Substitutional-ave),
 *     (EAM-density-substitutional-ave);
 *   - phase averages by Gauss-Hermite quadrature: App. A, Eq. (QuadRule), here
 *     the 3-point-per-axis product rule on the pair's relative coordinate;
 *   - kinetic law: Sec. 3.1, Eqs. (MassTransport), (attempt_freq_mass);
 *   - staggered relax / forward-Euler diffusion step: Sec. 4.
 * Readings of silent or inconsistent points of the paper are listed in the
 * design notes; each is marked "reading" where it is used below.
 */
#include "mxe_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define KB_EV 8.617333262e-5 /* Boltzmann constant, eV/K (CODATA 2018) */

enum { T_HOST_VAC = 0, T_ALLOY = 1, T_INTERSTITIAL = 2, T_HOST_FIXED = 3 };
enum { SP_A = 0, SP_B = 1, SP_S = 2, SP_NONE = 3 };

int oref_num_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* threads of later parallel loops (timing of the CPU baseline only) */
void oref_set_num_threads(int n) {
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* ------------------------------------------------------------------------ */
/* Occupancy model (Sec. 2, Eq. occupancy; App. B.2.1).                      */
/* Each site holds species sp1 with probability p1 and species sp0 with      */
/* p0 = 1 - p1. p1 = x for mobile sites and 1 for a fixed host atom.         */
/* ------------------------------------------------------------------------ */
static int sp1_of(int t) {
    switch (t) {
        case T_HOST_VAC: return SP_A;
        case T_ALLOY: return SP_B;
        case T_INTERSTITIAL: return SP_S;
        default: return SP_A;
    }
}
static int sp0_of(int t) { return t == T_ALLOY ? SP_A : SP_NONE; }
static double p1_of(int t, double x) { return t == T_HOST_FIXED ? 1.0 : x; }
static int is_mobile(int t) { return t != T_HOST_FIXED; }
/* vibrating fraction w (reading: empty sites carry no vibrational entropy) */
static double w_of(int t, double x) {
    return (t == T_HOST_VAC || t == T_INTERSTITIAL) ? x : 1.0;
}
static double dw_of(int t) { return (t == T_HOST_VAC || t == T_INTERSTITIAL) ? 1.0 : 0.0; }
static int is_interstitial(int t) { return t == T_INTERSTITIAL; }

static double sp_val(const double* v, int sp) { return sp == SP_NONE ? 0.0 : v[sp]; }

/* site value of a per-species quantity, linear in the occupancy */
static double site_val(const double* v, int t, double x) {
    double p1 = p1_of(t, x);
    return p1 * sp_val(v, sp1_of(t)) + (1.0 - p1) * sp_val(v, sp0_of(t));
}
/* derivative of site_val with respect to x (zero for an immobile site) */
static double site_dval(const double* v, int t) {
    if (!is_mobile(t)) return 0.0;
    return sp_val(v, sp1_of(t)) - sp_val(v, sp0_of(t));
}
/* site value divided by w, in closed form (own occupancy factor set to 1) */
static double site_hat(const double* v, int t, double x) {
    if (t == T_HOST_VAC || t == T_INTERSTITIAL) return sp_val(v, sp1_of(t));
    return site_val(v, t, x);
}

static double a_sp(const oref_eam* e, int k, int l) {
    if (k == SP_NONE || l == SP_NONE) return 0.0;
    return e->pair_a[k][l];
}
/* a_ij = sum_{k,l} p_ik p_jl a_kl  (Eq. EAM-Substitutional-ave) */
static double pair_amp(const oref_eam* e, int ti, double xi, int tj, double xj) {
    double pi1 = p1_of(ti, xi), pj1 = p1_of(tj, xj);
    int i1 = sp1_of(ti), i0 = sp0_of(ti), j1 = sp1_of(tj), j0 = sp0_of(tj);
    return pi1 * pj1 * a_sp(e, i1, j1) + pi1 * (1 - pj1) * a_sp(e, i1, j0) +
           (1 - pi1) * pj1 * a_sp(e, i0, j1) + (1 - pi1) * (1 - pj1) * a_sp(e, i0, j0);
}
static double pair_amp_dxi(const oref_eam* e, int ti, int tj, double xj) {
    if (!is_mobile(ti)) return 0.0;
    double pj1 = p1_of(tj, xj);
    int i1 = sp1_of(ti), i0 = sp0_of(ti), j1 = sp1_of(tj), j0 = sp0_of(tj);
    return pj1 * (a_sp(e, i1, j1) - a_sp(e, i0, j1)) +
           (1 - pj1) * (a_sp(e, i1, j0) - a_sp(e, i0, j0));
}
static double pair_amp_hat(const oref_eam* e, int ti, double xi, int tj, double xj) {
    if (ti == T_HOST_VAC || ti == T_INTERSTITIAL) {
        double pj1 = p1_of(tj, xj);
        int i1 = sp1_of(ti), j1 = sp1_of(tj), j0 = sp0_of(tj);
        return pj1 * a_sp(e, i1, j1) + (1 - pj1) * a_sp(e, i1, j0);
    }
    return pair_amp(e, ti, xi, tj, xj);
}

/* pair class: 0 host-host, 1 host-interstitial, -1 no interaction */
static int pair_class(int ti, int tj) {
    int a = is_interstitial(ti), b = is_interstitial(tj);
    if (a && b) return -1;
    return (a || b) ? 1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Quadrature (App. A). The pair function depends on q_j - q_i only; with    */
/* independent Gaussians of per-axis std sigma_i, sigma_j the difference is  */
/* Gaussian with mean rbar and std s = sqrt(sigma_i^2 + sigma_j^2), so the   */
/* 6-D average is a 3-D one. Per axis: 3-point Gauss-Hermite for N(0,1):     */
/* nodes 0, +-sqrt(3), weights 2/3, 1/6, 1/6 (the exp(-t^2) rule with nodes  */
/* 0, +-sqrt(3/2) after t = z/sqrt(2)).                                      */
/* ------------------------------------------------------------------------ */
void oref_quadrature(double zeta[27][3], double w[27]) {
    const double node1[3] = {-sqrt(3.0), 0.0, sqrt(3.0)};
    const double wt1[3] = {1.0 / 6.0, 2.0 / 3.0, 1.0 / 6.0};
    int k = 0;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            for (int c = 0; c < 3; ++c) {
                zeta[k][0] = node1[a];
                zeta[k][1] = node1[b];
                zeta[k][2] = node1[c];
                w[k] = wt1[a] * wt1[b] * wt1[c];
                ++k;
            }
}

/* g(r) = exp(-a (r/r_e - 1)) S(r); S = 1 below r_s, cosine taper to 0 at r_c */
void oref_shape(const oref_eam* e, double r, double r_e, double a, double* g, double* dg) {
    if (r >= e->r_c) {
        *g = 0.0;
        *dg = 0.0;
        return;
    }
    double ex = exp(-a * (r / r_e - 1.0));
    double S = 1.0, dS = 0.0;
    if (r > e->r_s) {
        double width = e->r_c - e->r_s;
        double t = (r - e->r_s) / width;
        S = 0.5 * (1.0 + cos(M_PI * t));
        dS = -0.5 * M_PI * sin(M_PI * t) / width;
    }
    *g = ex * S;
    *dg = -(a / r_e) * ex * S + ex * dS;
}

void oref_pair_average(const oref_eam* e, int cls, const double rbar[3], double s,
                       double out[14]) {
    double zeta[27][3], w[27];
    oref_quadrature(zeta, w);
    for (int m = 0; m < 14; ++m) out[m] = 0.0;
    double re = e->r_e[cls], al = e->alpha[cls], ga = e->gamma[cls];
    for (int k = 0; k < 27; ++k) {
        double d[3], r2 = 0.0, dz = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = rbar[a] + s * zeta[k][a];
            r2 += d[a] * d[a];
            dz += d[a] * zeta[k][a];
        }
        double r = sqrt(r2);
        if (r >= e->r_c || r == 0.0) continue;
        double gp, dgp, gf, dgf;
        oref_shape(e, r, re, al, &gp, &dgp);
        oref_shape(e, r, re, ga, &gf, &dgf);
        out[0] += w[k] * gp;
        for (int a = 0; a < 3; ++a) out[1 + a] += w[k] * dgp * d[a] / r;
        out[4] += w[k] * dgp * dz / r;
        out[5] += w[k] * gf;
        for (int a = 0; a < 3; ++a) out[6 + a] += w[k] * dgf * d[a] / r;
        out[9] += w[k] * dgf * dz / r;
    }
    /* density at the mean positions (Eq. F_taylor: rho|_0) and its gradient */
    double r0 = sqrt(rbar[0] * rbar[0] + rbar[1] * rbar[1] + rbar[2] * rbar[2]);
    if (r0 > 0.0) {
        double g0, dg0;
        oref_shape(e, r0, re, ga, &g0, &dg0);
        out[10] = g0;
        for (int a = 0; a < 3; ++a) out[11 + a] = dg0 * rbar[a] / r0;
    }
}

/* Degree-3 rule of App. A, Eq. (QuadRule), for the N_q = 6 coordinates of a
 * pair. In the scaled variables chi = (q - qbar)/(sqrt(2) sigma) the weight
 * is exp(-|chi|^2); the M = 2 N_q nodes sit at +-r on each coordinate axis
 * with r^2 = N_q/2, and each weight pi^(N_q/2)/(2 N_q) times the
 * normalisation pi^(-N_q/2) is 1/(2 N_q). */
void oref_stroud_nodes(double sigma_i, double sigma_j, double off[12][6], double w[12]) {
    const int nq = 6;
    const double r = sqrt(nq / 2.0);
    int k = 0;
    for (int axis = 0; axis < nq; ++axis)
        for (int sgn = -1; sgn <= 1; sgn += 2) {
            for (int a = 0; a < nq; ++a) off[k][a] = 0.0;
            double sig = axis < 3 ? sigma_i : sigma_j;
            off[k][axis] = sqrt(2.0) * sig * (sgn * r);
            w[k] = 1.0 / (2.0 * nq);
            ++k;
        }
}

static void pair_moments_stroud(const oref_eam* e, int cls, const double rbar[3], double si,
                                double sj, double out[16]) {
    double off[12][6], w[12];
    oref_stroud_nodes(si, sj, off, w);
    for (int m = 0; m < 16; ++m) out[m] = 0.0;
    double re = e->r_e[cls], al = e->alpha[cls], ga = e->gamma[cls];
    for (int k = 0; k < 12; ++k) {
        /* d = (q_j + dq_j) - (q_i + dq_i); d d/dsigma_i = -dq_i/sigma_i, d d/dsigma_j = dq_j/sigma_j */
        double d[3], r2 = 0.0, ddi = 0.0, ddj = 0.0;
        for (int a = 0; a < 3; ++a) {
            d[a] = rbar[a] + off[k][3 + a] - off[k][a];
            r2 += d[a] * d[a];
        }
        for (int a = 0; a < 3; ++a) {
            ddi += d[a] * (-off[k][a] / si);
            ddj += d[a] * (off[k][3 + a] / sj);
        }
        double r = sqrt(r2);
        if (r >= e->r_c || r == 0.0) continue;
        double gp, dgp, gf, dgf;
        oref_shape(e, r, re, al, &gp, &dgp);
        oref_shape(e, r, re, ga, &gf, &dgf);
        out[0] += w[k] * gp;
        for (int a = 0; a < 3; ++a) out[1 + a] += w[k] * dgp * d[a] / r;
        out[4] += w[k] * dgp * ddi / r;
        out[14] += w[k] * dgp * ddj / r;
        out[5] += w[k] * gf;
        for (int a = 0; a < 3; ++a) out[6 + a] += w[k] * dgf * d[a] / r;
        out[9] += w[k] * dgf * ddi / r;
        out[15] += w[k] * dgf * ddj / r;
    }
    double r0 = sqrt(rbar[0] * rbar[0] + rbar[1] * rbar[1] + rbar[2] * rbar[2]);
    if (r0 > 0.0) {
        double g0, dg0;
        oref_shape(e, r0, re, ga, &g0, &dg0);
        out[10] = g0;
        for (int a = 0; a < 3; ++a) out[11 + a] = dg0 * rbar[a] / r0;
    }
}

void oref_pair_moments(const oref_eam* e, int cls, const double rbar[3], double si, double sj,
                       double out[16]) {
    if (e->quad_rule == 1) {
        pair_moments_stroud(e, cls, rbar, si, sj, out);
        return;
    }
    /* product rule: the average depends on s = sqrt(si^2 + sj^2) only, so
     * d/dsigma_i = (sigma_i / s) d/ds */
    double m[14];
    double s = sqrt(si * si + sj * sj);
    oref_pair_average(e, cls, rbar, s, m);
    for (int k = 0; k < 14; ++k) out[k] = m[k];
    out[4] = (si / s) * m[4];
    out[9] = (si / s) * m[9];
    out[14] = (sj / s) * m[4];
    out[15] = (sj / s) * m[9];
}

/* ------------------------------------------------------------------------ */
/* Geometry: minimum image and neighbour search.                            */
/* ------------------------------------------------------------------------ */
static void min_image(const oref_box* b, const double* qi, const double* qj, double d[3]) {
    for (int a = 0; a < 3; ++a) {
        d[a] = qj[a] - qi[a];
        if (b->periodic[a]) d[a] -= b->box[a] * round(d[a] / b->box[a]);
    }
}

typedef struct {
    int n;
    int* start; /* n+1 */
    int* j;     /* start[n] */
} csr;

static void csr_free(csr* c) {
    free(c->start);
    free(c->j);
    c->start = c->j = NULL;
}

static int cmp_int(const void* a, const void* b) {
    int x = *(const int*)a, y = *(const int*)b;
    return (x > y) - (x < y);
}

/* All pairs with |r| < radius. method 0: all pairs; 1: cell list. */
static int build_csr(const oref_box* b, const double* q, double radius, int method, csr* out) {
    int n = b->n;
    for (int a = 0; a < 3; ++a)
        if (b->periodic[a] && !(b->box[a] > 2.0 * radius)) return OREF_EINVAL;
    int* cnt = (int*)calloc((size_t)n + 1, sizeof(int));
    int cap = 64 * n + 64;
    int* list = (int*)malloc(sizeof(int) * (size_t)cap);
    int total = 0;
    double r2max = radius * radius;
    if (method == 0) {
        for (int i = 0; i < n; ++i) {
            for (int j = 0; j < n; ++j) {
                if (j == i) continue;
                double d[3];
                min_image(b, q + 3 * i, q + 3 * j, d);
                if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < r2max) {
                    if (total == cap) {
                        cap *= 2;
                        list = (int*)realloc(list, sizeof(int) * (size_t)cap);
                    }
                    list[total++] = j;
                    cnt[i + 1]++;
                }
            }
        }
    } else {
        /* plain cell list: cells at least `radius` wide; bounds of the
         * non-periodic axes taken from the positions */
        double lo[3], ext[3];
        int nc[3];
        for (int a = 0; a < 3; ++a) {
            if (b->periodic[a]) {
                lo[a] = 0.0;
                ext[a] = b->box[a];
            } else {
                double mn = q[a], mx = q[a];
                for (int i = 1; i < n; ++i) {
                    if (q[3 * i + a] < mn) mn = q[3 * i + a];
                    if (q[3 * i + a] > mx) mx = q[3 * i + a];
                }
                lo[a] = mn;
                ext[a] = mx - mn + 1e-9;
            }
            nc[a] = (int)floor(ext[a] / radius);
            if (nc[a] < 1) nc[a] = 1;
        }
        int ncell = nc[0] * nc[1] * nc[2];
        int* head = (int*)malloc(sizeof(int) * (size_t)ncell);
        int* next = (int*)malloc(sizeof(int) * (size_t)n);
        int* cell_of = (int*)malloc(sizeof(int) * (size_t)n);
        for (int c = 0; c < ncell; ++c) head[c] = -1;
        for (int i = n - 1; i >= 0; --i) {
            int ci[3];
            for (int a = 0; a < 3; ++a) {
                double u = q[3 * i + a] - lo[a];
                if (b->periodic[a]) u -= ext[a] * floor(u / ext[a]);
                int c = (int)floor(u / ext[a] * nc[a]);
                if (c < 0) c = 0;
                if (c >= nc[a]) c = nc[a] - 1;
                ci[a] = c;
            }
            int c = (ci[0] * nc[1] + ci[1]) * nc[2] + ci[2];
            cell_of[i] = c;
            next[i] = head[c];
            head[c] = i;
        }
        int* row = (int*)malloc(sizeof(int) * (size_t)n);
        for (int i = 0; i < n; ++i) {
            int c = cell_of[i];
            int ci[3] = {c / (nc[1] * nc[2]), (c / nc[2]) % nc[1], c % nc[2]};
            /* distinct neighbouring cell indices per axis */
            int cand[3][3], ncand[3];
            for (int a = 0; a < 3; ++a) {
                ncand[a] = 0;
                for (int o = -1; o <= 1; ++o) {
                    int v = ci[a] + o;
                    if (b->periodic[a]) v = ((v % nc[a]) + nc[a]) % nc[a];
                    else if (v < 0 || v >= nc[a]) continue;
                    int dup = 0;
                    for (int k = 0; k < ncand[a]; ++k) dup |= (cand[a][k] == v);
                    if (!dup) cand[a][ncand[a]++] = v;
                }
            }
            int nr = 0;
            for (int x0 = 0; x0 < ncand[0]; ++x0)
                for (int y0 = 0; y0 < ncand[1]; ++y0)
                    for (int z0 = 0; z0 < ncand[2]; ++z0) {
                        int cc = (cand[0][x0] * nc[1] + cand[1][y0]) * nc[2] + cand[2][z0];
                        for (int j = head[cc]; j >= 0; j = next[j]) {
                            if (j == i) continue;
                            double d[3];
                            min_image(b, q + 3 * i, q + 3 * j, d);
                            if (d[0] * d[0] + d[1] * d[1] + d[2] * d[2] < r2max) row[nr++] = j;
                        }
                    }
            qsort(row, (size_t)nr, sizeof(int), cmp_int);
            for (int k = 0; k < nr; ++k) {
                if (total == cap) {
                    cap *= 2;
                    list = (int*)realloc(list, sizeof(int) * (size_t)cap);
                }
                list[total++] = row[k];
            }
            cnt[i + 1] = nr;
        }
        free(row);
        free(head);
        free(next);
        free(cell_of);
    }
    for (int i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    out->n = n;
    out->start = cnt;
    out->j = list;
    return OREF_OK;
}

int oref_neighbors(const oref_box* b, const double* q, double radius, int method, int kmax,
                   int* counts, int* list) {
    csr c;
    int st = build_csr(b, q, radius, method, &c);
    if (st != OREF_OK) return st;
    int total = c.start[b->n];
    int worst = 0;
    for (int i = 0; i < b->n; ++i) {
        int k = c.start[i + 1] - c.start[i];
        if (k > worst) worst = k;
        counts[i] = k;
        for (int m = 0; m < k && m < kmax; ++m) list[(size_t)i * kmax + m] = c.j[c.start[i] + m];
    }
    csr_free(&c);
    if (worst > kmax) return -worst;
    return total;
}

/* ------------------------------------------------------------------------ */
/* Mean-field free energy and its exact gradients.                          */
/* ------------------------------------------------------------------------ */
typedef struct {
    const oref_eam* e;
    const oref_box* b;
    const double *q, *sigma, *x;
    const int8_t* type;
    csr nb;
    double kT;            /* k_B T of the reference temperature */
    const double* T_site; /* per-site temperatures or NULL */
    /* pass-1 results */
    double *rho_bar, *rho0, *G, *Atil, *Btil, *Ahat, *Bhat;
    char* need1; /* pass 1 required for this site */
} evalctx;

/* Does some quadrature node of the pair reach inside r_c?  The farthest node
 * of the product rule is 3 s from rbar, and that of the degree-3 rule
 * sqrt(6) max(sigma_i, sigma_j) <= 3 s, so pairs with |rbar| >= r_c + 3 s
 * give zero under either rule. */
static int pair_active(const evalctx* c, int i, int j, double d[3], double* s, int* cls) {
    *cls = pair_class(c->type[i], c->type[j]);
    if (*cls < 0) return 0;
    min_image(c->b, c->q + 3 * i, c->q + 3 * j, d);
    *s = sqrt(c->sigma[i] * c->sigma[i] + c->sigma[j] * c->sigma[j]);
    double r = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
    return r < c->e->r_c + 3.0 * (*s);
}

static int has_embedding(const oref_eam* e, int t) {
    return sp_val(e->embed_c, sp1_of(t)) != 0.0 || sp_val(e->embed_c, sp0_of(t)) != 0.0;
}

/* Weight of site i's energy share in k_B T times the free entropy of
 * Eq. (Grand-Canonical-Free-Energy): beta_i / beta = T / T_i (1 at uniform T). */
static double theta_of(const evalctx* c, int i) {
    return c->T_site ? c->b->T / c->T_site[i] : 1.0;
}

/* pass 1: rho_bar_i = sum_j b_j <f_ij>, rho0_i = sum_j b_j f(|rbar_ij|);
 * Taylor embedding (Eq. F_taylor_mxe) with F~(rho) = -sqrt(rho):
 *   G = F~(rho0) + F~'(rho0) (rho_bar - rho0),
 *   A = c F~'(rho0), B = c F~''(rho0) (rho_bar - rho0). */
static int pass1_site(evalctx* c, int i) {
    double rb = 0.0, r0 = 0.0;
    for (int k = c->nb.start[i]; k < c->nb.start[i + 1]; ++k) {
        int j = c->nb.j[k];
        double d[3], s, m[16];
        int cls;
        if (!pair_active(c, i, j, d, &s, &cls)) continue;
        oref_pair_moments(c->e, cls, d, c->sigma[i], c->sigma[j], m);
        double bj = site_val(c->e->emit_b, c->type[j], c->x[j]);
        rb += bj * m[5];
        r0 += bj * m[10];
    }
    c->rho_bar[i] = rb;
    c->rho0[i] = r0;
    int t = c->type[i];
    if (!has_embedding(c->e, t)) {
        c->G[i] = c->Atil[i] = c->Btil[i] = c->Ahat[i] = c->Bhat[i] = 0.0;
        return OREF_OK;
    }
    if (!(r0 > 1e-12)) return OREF_ERANGE;
    double sq = sqrt(r0);
    double F0 = -sq, F1 = -0.5 / sq, F2 = 0.25 / (sq * r0);
    c->G[i] = F0 + F1 * (rb - r0);
    double ci = site_val(c->e->embed_c, t, c->x[i]);
    double ch = site_hat(c->e->embed_c, t, c->x[i]);
    /* the embedding share c_i G_i enters with weight theta_i */
    double th = theta_of(c, i);
    c->Atil[i] = th * ci * F1;
    c->Btil[i] = th * ci * F2 * (rb - r0);
    c->Ahat[i] = th * ch * F1;
    c->Bhat[i] = th * ch * F2 * (rb - r0);
    return OREF_OK;
}

/* pass 2 for site i: raw gradient, normalised force, mu, energy share. */
static void pass2_site(const evalctx* c, int i, double grad[4], double force[4], double* mu,
                       double* esite) {
    const oref_eam* e = c->e;
    int ti = c->type[i];
    double xi = c->x[i], si = c->sigma[i];
    double g[4] = {0, 0, 0, 0}, gh[4] = {0, 0, 0, 0};
    double mui = 0.0, epair = 0.0;
    for (int k = c->nb.start[i]; k < c->nb.start[i + 1]; ++k) {
        int j = c->nb.j[k];
        double d[3], s, m[16];
        int cls;
        if (!pair_active(c, i, j, d, &s, &cls)) continue;
        oref_pair_moments(e, cls, d, si, c->sigma[j], m);
        int tj = c->type[j];
        double xj = c->x[j];
        double aij = pair_amp(e, ti, xi, tj, xj);
        double ahat = pair_amp_hat(e, ti, xi, tj, xj);
        double dadx = pair_amp_dxi(e, ti, tj, xj);
        double bi = site_val(e->emit_b, ti, xi), bj = site_val(e->emit_b, tj, xj);
        double bhat = site_hat(e->emit_b, ti, xi), dbdx = site_dval(e->emit_b, ti);
        double cA = c->Atil[i] * bj + c->Atil[j] * bi;
        double cB = c->Btil[i] * bj + c->Btil[j] * bi;
        double hA = c->Ahat[i] * bj + c->Atil[j] * bhat;
        double hB = c->Bhat[i] * bj + c->Btil[j] * bhat;
        /* the pair term sits half in each end's share: weight (theta_i + theta_j)/2 */
        double tij = 0.5 * (theta_of(c, i) + theta_of(c, j));
        for (int a = 0; a < 3; ++a) {
            g[a] -= tij * aij * m[1 + a] + cA * m[6 + a] + cB * m[11 + a];
            gh[a] -= tij * ahat * m[1 + a] + hA * m[6 + a] + hB * m[11 + a];
        }
        g[3] += tij * aij * m[4] + cA * m[9];
        gh[3] += tij * ahat * m[4] + hA * m[9];
        mui += tij * dadx * m[0] + dbdx * (c->Atil[j] * m[5] + c->Btil[j] * m[10]);
        epair += 0.5 * aij * m[0];
    }
    /* vibrational part: -3 kT w ln sigma (Eq. Grand-Canonical-Free-Energy with
     * omega = 1/(sigma sqrt(beta m)); weighting by w is a reading) */
    double wi = w_of(ti, xi);
    g[3] -= 3.0 * c->kT * wi / si;
    gh[3] -= 3.0 * c->kT / si;
    /* mu_i = d(F - E_mix)/dx_i (reading: the mixing entropy enters through the
     * x(1-x) prefactors of the kinetic law) */
    /* mu_i = gamma_i / beta_i: the x_i-derivative of the functional divided by theta_i */
    double thi = theta_of(c, i);
    if (is_mobile(ti)) {
        mui += thi * site_dval(e->embed_c, ti) * c->G[i] - 3.0 * c->kT * dw_of(ti) * log(si);
        mui /= thi;
    } else {
        mui = 0.0;
    }
    double mix = 0.0;
    if (is_mobile(ti)) {
        if (xi > 0.0) mix += xi * log(xi);
        if (xi < 1.0) mix += (1.0 - xi) * log(1.0 - xi);
        mix *= c->kT;
    }
    double ci = site_val(e->embed_c, ti, xi);
    if (grad)
        for (int a = 0; a < 4; ++a) grad[a] = g[a];
    if (force)
        for (int a = 0; a < 4; ++a) force[a] = -gh[a];
    if (mu) *mu = mui;
    if (esite) *esite = thi * (epair + ci * c->G[i]) - 3.0 * c->kT * wi * log(si) + mix;
}

static double max_sigma(const double* sigma, int n) {
    double m = 0.0;
    for (int i = 0; i < n; ++i)
        if (sigma[i] > m) m = sigma[i];
    return m;
}

static int ctx_init(evalctx* c, const oref_eam* e, const oref_box* b, const double* q,
                    const double* sigma, const double* x, const int8_t* type) {
    memset(c, 0, sizeof(*c));
    c->e = e;
    c->b = b;
    c->q = q;
    c->sigma = sigma;
    c->x = x;
    c->type = type;
    c->kT = KB_EV * b->T;
    c->T_site = b->T_site;
    if (b->T_site)
        for (int i = 0; i < b->n; ++i)
            if (!(b->T_site[i] > 0.0)) return OREF_EINVAL;
    for (int i = 0; i < b->n; ++i)
        if (!(sigma[i] > 0.0)) return OREF_EINVAL;
    double radius = e->r_c + 3.0 * sqrt(2.0) * max_sigma(sigma, b->n) + 1e-6;
    int method = b->n <= 2048 ? 0 : 1;
    int st = build_csr(b, q, radius, method, &c->nb);
    if (st != OREF_OK) return st;
    size_t n = (size_t)b->n;
    c->rho_bar = (double*)calloc(n, sizeof(double));
    c->rho0 = (double*)calloc(n, sizeof(double));
    c->G = (double*)calloc(n, sizeof(double));
    c->Atil = (double*)calloc(n, sizeof(double));
    c->Btil = (double*)calloc(n, sizeof(double));
    c->Ahat = (double*)calloc(n, sizeof(double));
    c->Bhat = (double*)calloc(n, sizeof(double));
    c->need1 = (char*)calloc(n, 1);
    return OREF_OK;
}

static void ctx_free(evalctx* c) {
    csr_free(&c->nb);
    free(c->rho_bar);
    free(c->rho0);
    free(c->G);
    free(c->Atil);
    free(c->Btil);
    free(c->Ahat);
    free(c->Bhat);
    free(c->need1);
}

/* setchemicalpotential (Sec. 4): after the forces, mu of a held mobile site
 * is replaced by the held value */
static double held_mu(const oref_box* b, const int8_t* type, int i, double mu) {
    if (b->res && b->res[i] == OREF_RES_FIX_MU && is_mobile(type[i])) return b->res_val[i];
    return mu;
}

int oref_evaluate(const oref_eam* e, const oref_box* b, const double* q, const double* sigma,
                  const double* x, const int8_t* type, double* rho_bar, double* rho0,
                  double* grad, double* force, double* mu, double* e_site, double* F_out) {
    evalctx c;
    int st = ctx_init(&c, e, b, q, sigma, x, type);
    if (st != OREF_OK) {
        ctx_free(&c);
        return st;
    }
    int n = b->n, bad = 0;
#pragma omp parallel for schedule(dynamic, 64) reduction(| : bad)
    for (int i = 0; i < n; ++i) bad |= (pass1_site(&c, i) != OREF_OK);
    if (bad) {
        ctx_free(&c);
        return OREF_ERANGE;
    }
    double* es = (double*)malloc(sizeof(double) * (size_t)n);
#pragma omp parallel for schedule(dynamic, 64)
    for (int i = 0; i < n; ++i) {
        double g4[4], f4[4], m;
        pass2_site(&c, i, g4, f4, &m, &es[i]);
        if (grad)
            for (int a = 0; a < 4; ++a) grad[4 * i + a] = g4[a];
        if (force)
            for (int a = 0; a < 4; ++a) force[4 * i + a] = f4[a];
        if (mu) mu[i] = held_mu(b, type, i, m);
    }
    double F = 0.0;
    for (int i = 0; i < n; ++i) F += es[i];
    if (e_site) memcpy(e_site, es, sizeof(double) * (size_t)n);
    if (rho_bar) memcpy(rho_bar, c.rho_bar, sizeof(double) * (size_t)n);
    if (rho0) memcpy(rho0, c.rho0, sizeof(double) * (size_t)n);
    if (F_out) *F_out = F;
    free(es);
    ctx_free(&c);
    return OREF_OK;
}

int oref_evaluate_sites(const oref_eam* e, const oref_box* b, const double* q,
                        const double* sigma, const double* x, const int8_t* type, int n_sel,
                        const int* sel, double* rho_bar, double* rho0, double* force,
                        double* mu, double* e_site) {
    evalctx c;
    int st = ctx_init(&c, e, b, q, sigma, x, type);
    if (st != OREF_OK) {
        ctx_free(&c);
        return st;
    }
    /* pass 1 is needed at the selected sites and at their neighbours */
    for (int s = 0; s < n_sel; ++s) {
        int i = sel[s];
        if (i < 0 || i >= b->n) {
            ctx_free(&c);
            return OREF_EINVAL;
        }
        c.need1[i] = 1;
        for (int k = c.nb.start[i]; k < c.nb.start[i + 1]; ++k) c.need1[c.nb.j[k]] = 1;
    }
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int i = 0; i < b->n; ++i)
        if (c.need1[i]) bad |= (pass1_site(&c, i) != OREF_OK);
    if (bad) {
        ctx_free(&c);
        return OREF_ERANGE;
    }
#pragma omp parallel for schedule(dynamic, 4)
    for (int s = 0; s < n_sel; ++s) {
        int i = sel[s];
        double f4[4], m, es;
        pass2_site(&c, i, NULL, f4, &m, &es);
        if (force)
            for (int a = 0; a < 4; ++a) force[4 * s + a] = f4[a];
        if (mu) mu[s] = held_mu(b, type, i, m);
        if (e_site) e_site[s] = es;
        if (rho_bar) rho_bar[s] = c.rho_bar[i];
        if (rho0) rho0[s] = c.rho0[i];
    }
    ctx_free(&c);
    return OREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Kinetic law (Sec. 3.1, Eq. MassTransport), nearest-neighbour bonds.      */
/* ------------------------------------------------------------------------ */
int oref_bonds(const oref_box* b, const double* q, const int8_t* type, double r_bond, int bmax,
               int* nbond, int* bonds) {
    csr c;
    int st = build_csr(b, q, r_bond, b->n <= 2048 ? 0 : 1, &c);
    if (st != OREF_OK) return st;
    int worst = 0;
    for (int i = 0; i < b->n; ++i) {
        int nb = 0;
        if (is_mobile(type[i])) {
            for (int k = c.start[i]; k < c.start[i + 1]; ++k) {
                int j = c.j[k];
                if (type[j] != type[i]) continue;
                if (nb < bmax) bonds[(size_t)i * bmax + nb] = j;
                ++nb;
            }
        }
        if (nb > worst) worst = nb;
        nbond[i] = nb < bmax ? nb : bmax;
    }
    csr_free(&c);
    return worst > bmax ? -worst : OREF_OK;
}

/* dx_i/dt = sum_j D [x_j (1 - x_i) e^{c beta (mu_j - mu_i)} - x_i (1 - x_j) e^{c beta (mu_i - mu_j)}]
 * with D = nu0 exp(-beta Qm) (Eq. attempt_freq_mass). Reading of the sign:
 * the driving force of the hop a -> b is mu_a - mu_b, so matter flows from
 * high to low mu. Time step (reading of the stability remark of Sec. 4):
 * C_dt over the largest per-site rate of outflow, sum_j D (1 - x_j) e^{c beta (mu_i - mu_j)},
 * or inflow, sum_j D x_j e^{c beta (mu_j - mu_i)}. Then
 * x_i' >= x_i (1 - dt Rout_i) and 1 - x_i' >= (1 - x_i)(1 - dt Rin_i), so every
 * x stays inside [0, 1] for C_dt <= 1. */
int oref_master_rates(const oref_box* b, const oref_params* p, const double* x,
                      const int8_t* type, const double* mu, int bmax, const int* nbond,
                      const int* bonds, double* dxdt, double* dt) {
    double beta = 1.0 / (KB_EV * b->T);
    double D = p->nu0 * exp(-beta * p->Qm);
    double cb = p->kin_c * beta;
    double rmax = 0.0;
    for (int i = 0; i < b->n; ++i) {
        double acc = 0.0, rout = 0.0, rin = 0.0;
        if (is_mobile(type[i]) && b->T_site) {
            /* site temperatures (reading): a hop a -> b has attempt rate
             * D_a = nu0 e^{-beta_a Qm} and driving factor e^{c beta_a (mu_a - mu_b)},
             * both at the source site, so each hop has one rate in both
             * equations and matter is conserved */
            double bi = 1.0 / (KB_EV * b->T_site[i]);
            double Di = p->nu0 * exp(-bi * p->Qm);
            for (int k = 0; k < nbond[i]; ++k) {
                int j = bonds[(size_t)i * bmax + k];
                double bj = 1.0 / (KB_EV * b->T_site[j]);
                double Dj = p->nu0 * exp(-bj * p->Qm);
                double in = Dj * exp(p->kin_c * bj * (mu[j] - mu[i]));
                double out = Di * exp(p->kin_c * bi * (mu[i] - mu[j]));
                acc += x[j] * (1.0 - x[i]) * in - x[i] * (1.0 - x[j]) * out;
                rout += (1.0 - x[j]) * out;
                rin += x[j] * in;
            }
        } else if (is_mobile(type[i])) {
            for (int k = 0; k < nbond[i]; ++k) {
                int j = bonds[(size_t)i * bmax + k];
                double in = exp(cb * (mu[j] - mu[i]));
                double out = exp(cb * (mu[i] - mu[j]));
                acc += D * (x[j] * (1.0 - x[i]) * in - x[i] * (1.0 - x[j]) * out);
                rout += D * (1.0 - x[j]) * out;
                rin += D * x[j] * in;
            }
        }
        dxdt[i] = acc;
        if (rout > rmax) rmax = rout;
        if (rin > rmax) rmax = rin;
    }
    *dt = rmax > 0.0 ? p->dt_safety / rmax : 0.0;
    return OREF_OK;
}

/* Forward-Euler step (Sec. 4) followed by setatomicfraction: the mass
 * transport update comes first, then held sites are reset (Algorithm 1 calls
 * the transport fix at the start of the step and the fraction fix after it). */
int oref_master_step(const oref_box* b, const oref_params* p, double* x, const int8_t* type,
                     const double* mu, int bmax, const int* nbond, const int* bonds,
                     double dt_in, double* dxdt, double* dt, double* uptake) {
    double h;
    int st = oref_master_rates(b, p, x, type, mu, bmax, nbond, bonds, dxdt, &h);
    if (st != OREF_OK) return st;
    if (dt_in > 0.0) h = dt_in;
    double taken = 0.0;
    for (int i = 0; i < b->n; ++i) {
        if (!is_mobile(type[i])) continue;
        x[i] += h * dxdt[i];
        if (b->res && b->res[i] == OREF_RES_FIX_X) {
            taken += x[i] - b->res_val[i];
            x[i] = b->res_val[i];
        }
    }
    if (uptake) *uptake += taken;
    *dt = h;
    return OREF_OK;
}

/* ------------------------------------------------------------------------ */
/* Relaxation at fixed x (Sec. 4: positions and frequencies maximise the    */
/* free entropy). The relaxer is FIRE (Bitzek et al. 2006) with unit mass,  */
/* semi-implicit Euler, on the occupancy-normalised forces.                 */
/* ------------------------------------------------------------------------ */
int oref_relax(const oref_eam* e, const oref_box* b, const oref_params* p, double* q,
               double* sigma, const double* x, const int8_t* type, double* force,
               double* mu, double* e_site, double* F_out, double* fmax_out, int* converged,
               int* n_evals) {
    int n = b->n;
    size_t ndof = 4 * (size_t)n;
    double* f = (double*)malloc(sizeof(double) * ndof);
    double* v = (double*)calloc(ndof, sizeof(double));
    double dt = p->dt0, alpha = p->alpha0;
    int npos = 0, updates = 0, conv = 0, evals = 0, st = OREF_OK;
    double fmax = 0.0;
    for (int k = 0; k <= p->max_relax; ++k) {
        st = oref_evaluate(e, b, q, sigma, x, type, NULL, NULL, NULL, f, mu, e_site, F_out);
        ++evals;
        if (st != OREF_OK) break;
        fmax = 0.0;
        for (size_t d = 0; d < ndof; ++d)
            if (fabs(f[d]) > fmax) fmax = fabs(f[d]);
        if (fmax <= p->ftol) {
            conv = 1;
            break;
        }
        if (k == p->max_relax) break;
        double P = 0.0, ff = 0.0, vv = 0.0;
        for (size_t d = 0; d < ndof; ++d) {
            P += f[d] * v[d];
            ff += f[d] * f[d];
            vv += v[d] * v[d];
        }
        int reset = 0;
        if (k > 0) {
            if (P > 0.0) {
                ++npos;
                if (npos > p->nmin) {
                    dt = fmin(dt * p->finc, p->dtmax);
                    alpha *= p->falpha;
                }
            } else {
                npos = 0;
                dt *= p->fdec;
                alpha = p->alpha0;
                reset = 1;
            }
        } else {
            reset = 1; /* v is zero at the first update */
        }
        if (reset) {
            for (size_t d = 0; d < ndof; ++d) v[d] = 0.0;
            P = 0.0;
            vv = 0.0;
        }
        /* |v + dt f|^2 written out so the GPU needs one fused reduction */
        double vnorm = sqrt(vv + 2.0 * dt * P + dt * dt * ff);
        double fnorm = sqrt(ff);
        for (size_t d = 0; d < ndof; ++d) {
            v[d] += dt * f[d];
            if (fnorm > 0.0) v[d] = (1.0 - alpha) * v[d] + alpha * (vnorm / fnorm) * f[d];
        }
        for (int i = 0; i < n; ++i) {
            for (int a = 0; a < 3; ++a) q[3 * i + a] += dt * v[4 * i + a];
            sigma[i] += dt * v[4 * i + 3];
            if (sigma[i] < p->sigma_min) sigma[i] = p->sigma_min;
        }
        ++updates;
    }
    if (force) memcpy(force, f, sizeof(double) * ndof);
    if (fmax_out) *fmax_out = fmax;
    if (converged) *converged = conv;
    if (n_evals) *n_evals = evals;
    free(f);
    free(v);
    return st == OREF_OK ? updates : st;
}

/* Staggered scheme (Sec. 4, Alg. 1): per step relax at fixed x, then one
 * forward-Euler step of x using mu from the last evaluation. */
int oref_run(const oref_eam* e, const oref_box* b, const oref_params* p, int n_steps,
             double* q, double* sigma, double* x, const int8_t* type, double* mu,
             double* dxdt, double* t_out, double* rec) {
    int n = b->n;
    int bmax = 16;
    int* nbond = (int*)malloc(sizeof(int) * (size_t)n);
    int* bonds = (int*)malloc(sizeof(int) * (size_t)n * bmax);
    int st = oref_bonds(b, q, type, p->r_bond, bmax, nbond, bonds);
    if (st != OREF_OK) {
        free(nbond);
        free(bonds);
        return st;
    }
    double t = t_out ? *t_out : 0.0;
    double uptake = 0.0;
    if (b->res)
        for (int i = 0; i < n; ++i)
            if (b->res[i] == OREF_RES_FIX_X && is_mobile(type[i])) x[i] = b->res_val[i];
    for (int s = 0; s < n_steps; ++s) {
        double F, fmax, dt;
        int conv, nev;
        int upd = oref_relax(e, b, p, q, sigma, x, type, NULL, mu, NULL, &F, &fmax, &conv, &nev);
        if (upd < 0) {
            st = upd;
            break;
        }
        oref_master_step(b, p, x, type, mu, bmax, nbond, bonds, 0.0, dxdt, &dt, &uptake);
        double sx = 0.0;
        for (int i = 0; i < n; ++i) sx += x[i];
        t += dt;
        if (rec) {
            rec[7 * s + 0] = upd;
            rec[7 * s + 1] = conv;
            rec[7 * s + 2] = F;
            rec[7 * s + 3] = fmax;
            rec[7 * s + 4] = dt;
            rec[7 * s + 5] = sx;
            rec[7 * s + 6] = uptake;
        }
    }
    if (t_out) *t_out = t;
    free(nbond);
    free(bonds);
    return st;
}
