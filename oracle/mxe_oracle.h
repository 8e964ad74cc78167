/*
 * mxe_oracle.h -- plain FP64 CPU oracle for the mean-field EAM + master-equation
 * method of Ponga et al., "MXE" (arXiv:1910.01235).
 *
 * TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark may load this library. The GPU product path
 * never links, imports or calls it, and shares no code with it.
 *
 * Conventions: units eV, Angstrom, K, s. Positions are row-major [n][3].
 * Site types: 0 host site holding an atom or a vacancy, 1 substitutional
 * alloy site (B vs A), 2 interstitial site (solute vs empty), 3 fixed host
 * atom (x == 1, immobile). Species: 0 = A, 1 = B, 2 = S.
 */
#ifndef MXE_ORACLE_H
#define MXE_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct {
    double embed_c[3];    /* F_k(rho) = -embed_c[k] * sqrt(rho)                */
    double emit_b[3];     /* density emitted by species k (prefactor of f)      */
    double pair_a[3][3];  /* pair amplitude a_kl (symmetric)                    */
    double r_e[2];        /* per pair class: 0 host-host, 1 host-interstitial  */
    double alpha[2];      /* phi shape exp(-alpha (r/r_e - 1)) * taper          */
    double gamma[2];      /* f shape exp(-gamma (r/r_e - 1)) * taper            */
    double r_s, r_c;      /* cosine taper from r_s to r_c                       */
    int quad_rule;        /* phase-average rule: 0 = 27-node Gauss-Hermite product
                           * rule on the pair's relative coordinate; 1 = the
                           * degree-3 rule of App. A in the 6-D pair space     */
} oref_eam;

/* reservoir kinds of a site (Sec. 4: the setatomicfraction and
 * setchemicalpotential commands hold x, or mu, of a group at a given value) */
#define OREF_RES_NONE 0
#define OREF_RES_FIX_X 1
#define OREF_RES_FIX_MU 2

typedef struct {
    int n;
    double box[3];
    int periodic[3];
    double T;             /* temperature, K (the reference when T_site is set) */
    const int8_t* res;    /* per-site reservoir kind (OREF_RES_*), or NULL    */
    const double* res_val;/* the held x or mu of reservoir sites, or NULL     */
    const double* T_site; /* per-site temperature T_i (K), or NULL = uniform T.
                           * The relaxed functional is k_B T times the mean-field
                           * free entropy of Eq. (Grand-Canonical-Free-Energy),
                           * whose energy shares carry beta_i: each site's share
                           * is weighted by theta_i = T / T_i; mu_i = gamma_i /
                           * beta_i; each hop of the kinetic law runs at its
                           * source site's temperature.                      */
} oref_box;

typedef struct {
    double nu0, Qm;       /* hop attempt frequency (1/s), migration energy (eV) */
    double kin_c;         /* exponent factor of the kinetic law (1 = paper)      */
    double dt_safety;     /* C_dt of the adaptive time-step rule                 */
    int max_relax;        /* FIRE iteration cap                                  */
    double ftol;          /* force tolerance, eV/A                               */
    double dt0, dtmax, alpha0, finc, fdec, falpha;
    int nmin;
    double sigma_min;
    double r_bond;        /* nearest-neighbour bond radius of the kinetic law    */
} oref_params;

/* status codes */
#define OREF_OK 0
#define OREF_EINVAL (-1)
#define OREF_ERANGE (-5)

int oref_num_threads(void);
void oref_set_num_threads(int n);

/* 27-node product Gauss-Hermite rule for a standard 3-D normal variable. */
void oref_quadrature(double zeta[27][3], double w[27]);

/* Phase-averaged moments of one pair with mean separation rbar and relative
 * width s (class cls). out[14] = <phi>, grad<phi>(3), d<phi>/ds,
 * <f>, grad<f>(3), d<f>/ds, f0, grad f0 (3). */
void oref_pair_average(const oref_eam* e, int cls, const double rbar[3], double s,
                       double out[14]);

/* Degree-3 rule of App. A (Eq. QuadRule) for the 6-D coordinates of a pair
 * (q_i, q_j): 12 nodes, off[k] = (dq_i, dq_j) displacements from the means,
 * all weights 1/12. */
void oref_stroud_nodes(double sigma_i, double sigma_j, double off[12][6], double w[12]);

/* Pair moments under the rule selected by e->quad_rule, for rbar = qbar_j - qbar_i
 * and widths sigma_i, sigma_j. out[16] = <phi>, grad<phi>(3), d<phi>/dsigma_i,
 * <f>, grad<f>(3), d<f>/dsigma_i, f0, grad f0 (3), d<phi>/dsigma_j, d<f>/dsigma_j.
 * Gradients are with respect to rbar. */
void oref_pair_moments(const oref_eam* e, int cls, const double rbar[3], double sigma_i,
                       double sigma_j, double out[16]);

/* Radial shape and its derivative (taper included). */
void oref_shape(const oref_eam* e, double r, double r_e, double a, double* g, double* dg);

/* Full evaluation. Any output pointer may be NULL. On mobile sites marked
 * OREF_RES_FIX_MU the returned mu is the held value (applied after the forces).
 * grad:  raw gradient dF/d(qx,qy,qz,sigma), [n][4]
 * force: occupancy-normalised force -dF/dy / w, [n][4]
 * Returns OREF_OK or an error code; *F_out = total free energy. */
int oref_evaluate(const oref_eam* e, const oref_box* b, const double* q,
                  const double* sigma, const double* x, const int8_t* type,
                  double* rho_bar, double* rho0, double* grad, double* force,
                  double* mu, double* e_site, double* F_out);

/* Same outputs for a subset of sites sel[0..n_sel-1] (outputs indexed 0..n_sel-1). */
int oref_evaluate_sites(const oref_eam* e, const oref_box* b, const double* q,
                        const double* sigma, const double* x, const int8_t* type,
                        int n_sel, const int* sel, double* rho_bar, double* rho0,
                        double* force, double* mu, double* e_site);

/* Neighbour search: all j != i with minimum-image |r_ij| < radius.
 * method 0 = all pairs, 1 = cell list. Rows sorted by j.
 * Returns total count, or a negative error / -(needed) if kmax is exceeded. */
int oref_neighbors(const oref_box* b, const double* q, double radius, int method,
                   int kmax, int* counts, int* list);

/* Static nearest-neighbour bonds between mobile sites of the same type. */
int oref_bonds(const oref_box* b, const double* q, const int8_t* type, double r_bond,
               int bmax, int* nbond, int* bonds);

/* Master-equation rates: dxdt[n]; returns the stable time step in *dt. */
int oref_master_rates(const oref_box* b, const oref_params* p, const double* x,
                      const int8_t* type, const double* mu, int bmax, const int* nbond,
                      const int* bonds, double* dxdt, double* dt);

/* One forward-Euler step of x: rates as above, x += dt dxdt on mobile sites,
 * then mobile sites marked OREF_RES_FIX_X are reset to their held value; the
 * matter they took up in the step (x after the update minus the held value)
 * is added to *uptake. dt_in > 0 replaces the stable step. Returns the step
 * used in *dt. */
int oref_master_step(const oref_box* b, const oref_params* p, double* x, const int8_t* type,
                     const double* mu, int bmax, const int* nbond, const int* bonds,
                     double dt_in, double* dxdt, double* dt, double* uptake);

/* FIRE relaxation of (q, sigma) at fixed x. q and sigma are updated in place.
 * Outputs of the last evaluation go to the given arrays. Returns the number
 * of FIRE updates made; *converged = 1 if max|f| <= ftol was reached. */
int oref_relax(const oref_eam* e, const oref_box* b, const oref_params* p, double* q,
               double* sigma, const double* x, const int8_t* type, double* force,
               double* mu, double* e_site, double* F_out, double* fmax_out,
               int* converged, int* n_evals);

/* Staggered run: n_steps x (relax, master-equation Euler step). Mobile
 * OREF_RES_FIX_X sites are set to their held value before the first step.
 * rec[n_steps][7] = relax updates, converged, F, max|f|, dt, sum x (after
 * step), reservoir uptake accumulated since the start of the run. */
int oref_run(const oref_eam* e, const oref_box* b, const oref_params* p, int n_steps,
             double* q, double* sigma, double* x, const int8_t* type, double* mu,
             double* dxdt, double* t_out, double* rec);

#ifdef __cplusplus
}
#endif
#endif
