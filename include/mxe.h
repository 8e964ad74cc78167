/*
 * mxe.h -- C ABI of the MI355X mean-field EAM + master-equation library.
 *
 * Method: Ponga et al., "MXE" (arXiv:1910.01235). The library evaluates the
 * mean-field free energy of Sec. 2.1, Eq. (Grand-Canonical-Free-Energy), for
 * the thermalised EAM of App. B.2 (Eqs. EAM_mxe, F_taylor_mxe) with site
 * occupancies (App. B.2.1, Eqs. EAM-Substitutional-ave,
 * EAM-density-substitutional-ave), phase averages by Gauss-Hermite quadrature
 * (App. A, Eq. QuadRule; here the 27-node product rule on each pair's relative
 * coordinate), relaxes positions and widths at fixed occupancy, and advances
 * the occupancy field with the kinetic law of Sec. 3.1 (Eqs. MassTransport,
 * attempt_freq_mass) by forward Euler in the staggered scheme of Sec. 4
 * (Alg. 1). Inputs follow the paper's statement of the problem (Sec. 4 and
 * the program summary): sites with mean positions, widths, species
 * occupancies and a temperature; outputs are relaxed positions and widths,
 * chemical potentials, dx/dt, the time step and the free energy.
 *
 * Conventions shared by every entry point
 *   Units: eV, Angstrom, K, s.
 *   Batches: a plan covers n_systems >= 1 independent systems whose sites are
 *     concatenated in system order; every per-site array holds sum(n_sites)
 *     entries. Systems never interact.
 *   Ownership: the caller allocates and owns every device buffer (state,
 *     outputs, workspace). The library never allocates device memory; a plan
 *     owns host memory, one HIP stream used only to record graphs, the graphs
 *     it records and, with params.relax_chunk > 0, 16 bytes of pinned host
 *     memory and two events. The one exception is mxe_run_noalloc's fixed scratch
 *     array, held per device from the library's first use there until the
 *     process ends. All device pointers must be valid for the current HIP
 *     device.
 *   Asynchrony: every call only enqueues work on `stream` (a hipStream_t
 *     passed as void*, 0 = the null stream) and returns at once; with
 *     params.relax_chunk > 0, mxe_relax and mxe_run wait on the host between
 *     chunks of relaxation iterations while they enqueue. Return codes
 *     report argument and plan errors; errors the device detects are written
 *     to the per-system status scalar, to be read after the stream syncs.
 *   Determinism: no floating-point atomics; results are bitwise reproducible
 *     run to run, and a system's results do not depend on the other systems
 *     of its batch.
 *   Errors: no exception or abort crosses the ABI. mxe_last_error() returns a
 *     thread-local message for the last failing call of the calling thread.
 *   Threads: calls on one plan must not overlap (a plan holds the workspace
 *     binding and graph cache). Different plans are independent.
 */
#ifndef MXE_H
#define MXE_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MXE_OK = 0,
    MXE_EINVAL = -1,   /* invalid argument or inconsistent plan            */
    MXE_ENOMEM = -2,   /* workspace smaller than mxe_workspace_bytes()      */
    MXE_EDEVICE = -3,  /* a HIP runtime call failed                         */
    MXE_ERANGE = -5    /* a size limit of the plan would be exceeded        */
} mxe_status;

typedef enum { MXE_FP64 = 0, MXE_FP32_MIXED = 1 } mxe_precision;

/* phase-average quadrature rule */
typedef enum { MXE_QUAD_GH27 = 0, MXE_QUAD_DEGREE3 = 1 } mxe_quad_rule;

/* Site types. Each site holds its mobile species with probability x and the
 * complement with 1 - x (Sec. 2, Eq. occupancy; App. B.2.1):
 *   HOST_VAC      atom A or vacancy        (x = fraction of A)
 *   ALLOY         species B or species A   (x = fraction of B)
 *   INTERSTITIAL  solute S or empty        (x = fraction of S)
 *   HOST_FIXED    atom A, x == 1, immobile                                   */
typedef enum {
    MXE_SITE_HOST_VAC = 0,
    MXE_SITE_ALLOY = 1,
    MXE_SITE_INTERSTITIAL = 2,
    MXE_SITE_HOST_FIXED = 3
} mxe_site_type;

/* Analytic EAM (App. B.2): species A = 0, B = 1, S = 2; vacancy/empty carry
 * nothing. Embedding F_k(rho) = -embed_c[k] sqrt(rho); species k emits density
 * emit_b[k] g_f(r); pair energy a_kl g_phi(r). Radial shapes per pair class
 * (0 host-host, 1 host-interstitial; interstitial pairs do not interact):
 * g_phi = exp(-alpha (r/r_e - 1)) S(r), g_f = exp(-gamma (r/r_e - 1)) S(r),
 * S = 1 below r_s, (1 + cos(pi (r - r_s)/(r_c - r_s)))/2 up to r_c, 0 beyond.
 * Performance only: when alpha : gamma is 4 : 3 in class 0 and 5 : 4 in class
 * 1 (within 1e-12 relative), both shapes of a node are powers of one
 * exponential and the pair kernel computes one exponential per node instead
 * of two; any other exponents take the two-exponential kernel (the results
 * agree to rounding). */
typedef struct {
    double embed_c[3];
    double emit_b[3];
    double pair_a[3][3]; /* symmetric */
    double r_e[2];
    double alpha[2];
    double gamma[2];
    double r_s, r_c;
} mxe_eam;

typedef struct {
    /* kinetic law: D = nu0 exp(-Qm / kT); rate factor exp(kin_c beta dmu)    */
    double nu0, Qm, kin_c;
    /* Euler step dt = dt_safety / (largest per-site outflow or inflow rate)   */
    double dt_safety;
    /* FIRE relaxation of (q, sigma) at fixed x                                */
    int max_relax;       /* updates per relaxation; max_relax + 1 evaluations */
    double ftol;         /* convergence: max |f| <= ftol (eV/A)               */
    double fire_dt0, fire_dtmax, fire_alpha0, fire_finc, fire_fdec, fire_falpha;
    int fire_nmin;
    double sigma_min;    /* widths are clamped from below                     */
    double sigma_cap;    /* widths above this flag MXE_STAT_SIGMA_CAP; sizes the cells */
    double skin;         /* neighbour-list skin (A)                           */
    double r_bond;       /* kinetic-law bond radius: same-type sites closer   */
    int k_max;           /* neighbour-list row length (max neighbours/site), <= 256 */
    int bond_max;        /* max bonds per site, <= 64                         */
    mxe_precision precision;
    /* launch shapes (performance only; results do not depend on them beyond
     * the order of floating-point sums): lanes per site in the density gather
     * (0 = 8; 8, 16, 32, 64; force_lanes below sets the force gather's) and
     * threads per block of the pair kernel (0 = 256; 64, 128, 256) */
    int gather_lanes;
    int pair_block;
    /* phase-average rule (App. A): MXE_QUAD_GH27 (default) integrates the
     * pair's relative coordinate with the 27-node Gauss-Hermite product rule;
     * MXE_QUAD_DEGREE3 uses the 12-node degree-3 rule of Eq. (QuadRule) in
     * the pair's 6-D coordinate space (each end displaced by +-sqrt(6) sigma
     * along one axis, weights 1/12) */
    int quad_rule;
    /* launch shape: lanes per site in the force/mu gather (0 = 16; 8, 16, 32,
     * 64), performance only as gather_lanes */
    int force_lanes;
    /* launch shape: the gathers visit each XCD's chunks of 256 sites S apart
     * (0 = 1: in order). Best when S is the number of chunks between a site and
     * its neighbours one lattice layer away (25 for 40^3 FCC cells in lattice
     * order); performance only, results are bitwise the same for every S */
    int gather_stride;
    /* relaxation schedule (performance only): 0 (default) enqueues every
     * relaxation as its fixed max_relax + 1 FIRE iterations and returns at once
     * (systems that have finished skip the rest). K > 0 (at most 1024) enqueues
     * the iterations in chunks of K and, after each chunk, reads on the host how
     * many systems are still relaxing; once none is, the relaxation ends after
     * at most one more chunk (read one chunk behind, so the device never waits
     * for the host). In plans of one occupied system, or of at most 65,536
     * occupied sites, the chunks' iterations are lean: no neighbour-build chain (5 launches per iteration
     * instead of 13); a system whose lists expired stalls, taking no
     * iteration, and the host enqueues one iteration with the chain once it
     * reads a stall, after which the system takes the iteration it waited for.
     * Larger plans keep the chain in every iteration. mxe_relax and mxe_run then
     * block the calling thread while they enqueue (the work stays ordered on
     * the caller's stream), and the first such call allocates 16 bytes of
     * pinned host memory and two events that the plan keeps. Results are
     * bitwise those of K = 0: an iteration after a system has finished changes
     * nothing of it, and a stalled system's iterations use the same lists as
     * the fixed sequence's. */
    int relax_chunk;
    /* launch shape: pair-kernel blocks per chunk of 4096 pair slots (0 = 2; 1, 2,
     * 4, 8 or 16). More blocks give small systems more parallel work at the
     * cost of a pipeline prologue per block; performance only, results are
     * bitwise the same for every value */
    int pair_split;
} mxe_params;

typedef struct {
    int64_t n_sites;
    double box[3];       /* periodic axis: period; open axis: extent [0, box) */
    int periodic[3];
    double T;            /* temperature (K), uniform over the system           */
} mxe_system;

/* Reservoir kinds of a mobile site (Sec. 4: the setatomicfraction and
 * setchemicalpotential commands hold the molar fraction, or the chemical
 * potential, of a group of sites at a given value). */
typedef enum {
    MXE_RES_NONE = 0,
    MXE_RES_FIX_X = 1,   /* x is reset to the held value after every Euler step
                          * and at the start of every call; the matter the site
                          * took up in a step is added to MXE_S_RESERVOIR      */
    MXE_RES_FIX_MU = 2   /* mu is replaced by the held value after the forces  */
} mxe_reservoir;

/* Device buffers, SoA FP64, concatenated over systems. reservoir and
 * res_value are optional (both NULL: no reservoir sites); when given, one
 * int8 kind (mxe_reservoir) and one held value per site. Reservoir kinds
 * on HOST_FIXED sites are ignored. */
typedef struct {
    double* qx;
    double* qy;
    double* qz;
    double* sigma;
    double* x;
    const int8_t* type;
    const int8_t* reservoir;
    const double* res_value;
    /* optional per-site temperatures T_i (K), NULL = the system's T. Sec. 2
     * gives every site its own beta_i: the relaxation then minimises k_B T
     * (T = the system's reference temperature) times the mean-field free
     * entropy of Eq. (Grand-Canonical-Free-Energy), whose energy shares carry
     * beta_i (weight T / T_i); mu_i = gamma_i / beta_i; each hop of the
     * kinetic law (Eqs. MassTransport, attempt_freq_mass) runs at its source
     * site's temperature, so matter stays conserved. */
    const double* T_site;
} mxe_state;

/* Outputs. fx..fsigma are the occupancy-normalised forces -dF/dy / w_i that
 * drive the relaxation (w = x on HOST_VAC and INTERSTITIAL sites, else 1).
 * mu_i = d(F - E_mix)/dx_i (0 on HOST_FIXED sites). e_site sums to F.
 * scalars: MXE_NSCALARS doubles per system, indexed by mxe_scalar. */
typedef struct {
    double* fx;
    double* fy;
    double* fz;
    double* fsigma;
    double* mu;
    double* dxdt;
    double* rho_bar;
    double* rho0;
    double* e_site;
    double* scalars;
} mxe_out;

typedef enum {
    MXE_S_F = 0,          /* free energy of the last evaluation (eV)           */
    MXE_S_FMAX = 1,       /* max |f| over all DOF of the last evaluation        */
    MXE_S_DT = 2,         /* last Euler time step (s)                           */
    MXE_S_TIME = 3,       /* accumulated time; in/out, the caller sets it       */
    MXE_S_SUMX = 4,       /* sum of x after the last step / at the last eval    */
    MXE_S_UPDATES = 5,    /* FIRE updates of the last relaxation                */
    MXE_S_CONVERGED = 6,  /* 1 if the last relaxation reached ftol              */
    MXE_S_EVALS = 7,      /* evaluations of the last relaxation                 */
    MXE_S_STATUS = 8,     /* OR of mxe_stat_bits since the call started         */
    MXE_S_REBUILDS = 9,   /* neighbour-list builds during the call              */
    MXE_S_TOTAL_EVALS = 10, /* evaluations during the call                       */
    MXE_S_PAIRS = 11,     /* pairs in the current neighbour list                */
    MXE_S_PAIR_EVALS = 12, /* pair quadratures during the call                  */
    MXE_S_RESERVOIR = 13, /* matter taken up by held-x sites; in/out, accumulated
                           * like MXE_S_TIME: sum x + this stays constant      */
    MXE_S_STEPS_LEFT = 14, /* mxe_advance: diffusion steps the system still has
                            * to run (0: its budget is spent)                   */
    MXE_NSCALARS = 16
} mxe_scalar;

typedef enum {
    MXE_STAT_NONFINITE = 1,   /* non-finite force, energy or x               */
    MXE_STAT_X_RANGE = 2,     /* x left [-1e-12, 1 + 1e-12]                   */
    MXE_STAT_RHO = 4,         /* rho0 <= 0 on a site with an embedding        */
    MXE_STAT_SIGMA_MIN = 8,   /* a width was clamped at sigma_min (warning)   */
    MXE_STAT_KMAX = 16,       /* neighbour row overflow: results invalid      */
    MXE_STAT_TEMP = 32,       /* a site temperature is not positive and finite */
    MXE_STAT_PAIRS = 64,      /* pair buffer overflow: results invalid        */
    MXE_STAT_BONDS = 128,     /* bond row overflow: results invalid           */
    MXE_STAT_SIGMA_CAP = 256  /* a width exceeded sigma_cap: results invalid  */
} mxe_stat_bits;

typedef struct mxe_plan mxe_plan;

/* Fill *p with the library defaults (FP64, FIRE constants of Bitzek et al.,
 * kin_c = 1, dt_safety = 0.5, sigma_cap = 0.3, skin = 0.15, k_max = 96,
 * bond_max = 16). */
void mxe_default_params(mxe_params* p);

/* Create a plan for n_systems systems. Validates sizes: every periodic box
 * length must exceed twice the largest neighbour radius
 * r_c + 3 sqrt(2) sigma_cap + skin. Returns MXE_EINVAL on bad input, with
 * *out = NULL. The plan copies everything it needs from its arguments. */
mxe_status mxe_plan_create(const mxe_params* params, const mxe_eam* eam, int n_systems,
                           const mxe_system* systems, mxe_plan** out);

void mxe_plan_destroy(mxe_plan* plan);

/* Size in bytes of the device workspace the plan needs (a single buffer,
 * 256-byte aligned by the caller's allocator). The workspace persists state
 * between calls (neighbour lists, FIRE velocities): pass the same buffer to
 * every call of a run. */
mxe_status mxe_workspace_bytes(const mxe_plan* plan, size_t* bytes);

/* Total number of sites of the plan (length of every per-site array): the sum
 * of the slot capacities. */
int64_t mxe_plan_sites(const mxe_plan* plan);

/* Batching with slots. Each system given to mxe_plan_create is a slot whose
 * n_sites is the slot's capacity; the slot's sites occupy the range
 * [mxe_plan_slot_offset(slot), mxe_plan_slot_offset(slot + 1)) of every
 * per-site array. mxe_plan_set_system rebinds a slot to another system of at
 * most that many sites (its first n_sites entries of the range; n_sites = 0
 * leaves the slot empty), with its own box, periodicity and temperature. The
 * change applies from the next call. Launches cover the occupied slots only
 * (their chunks come first in the plan's tables; the extent is rounded up to a
 * power of two), so many empty slots cost little. Returns MXE_ERANGE if the system does not fit the slot
 * (sites, or cells of its box), MXE_EINVAL for a bad box or temperature. A
 * system's results do not depend on its slot, its capacity or the other slots. */
mxe_status mxe_plan_set_system(mxe_plan* plan, int slot, const mxe_system* sys);
/* Would mxe_plan_set_system accept sys for this slot? Host-only check with the
 * same results (MXE_OK, MXE_ERANGE: too many sites or cells for the slot,
 * MXE_EINVAL: bad box, temperature or slot); the plan is not changed. */
mxe_status mxe_plan_check_system(const mxe_plan* plan, int slot, const mxe_system* sys);
/* First site of a slot; slot == n_systems gives the total. -1 if out of range. */
int64_t mxe_plan_slot_offset(const mxe_plan* plan, int slot);
/* Resume mode. Off (default): every call rebuilds all neighbour lists and
 * bonds, since the caller may have changed any state between calls. On: calls
 * rebuild only slots rebound since the previous call (and everything on a
 * workspace the plan has not used before); the caller must not modify the
 * positions or widths of other slots between calls. */
mxe_status mxe_plan_set_resume(mxe_plan* plan, int on);

/* One evaluation at the current state: pass 1 (rho_bar, rho0, the Taylor
 * embedding G, A, B of Eq. F_taylor_mxe) and pass 2 (forces, mu, e_site);
 * writes F, FMAX, SUMX, PAIRS, STATUS scalars. Rebuilds the neighbour lists. */
mxe_status mxe_evaluate(mxe_plan* plan, const mxe_state* state, const mxe_out* out, void* ws,
                        size_t ws_bytes, void* stream);

/* FIRE relaxation of (q, sigma) at fixed x (Sec. 4: the relaxation step of
 * the staggered scheme), at most params.max_relax updates per system; the
 * outputs hold the last evaluation. Systems relax independently. */
mxe_status mxe_relax(mxe_plan* plan, const mxe_state* state, const mxe_out* out, void* ws,
                     size_t ws_bytes, void* stream);

/* One forward-Euler step of the kinetic law (Sec. 3.1, Sec. 4) using out->mu
 * from the previous evaluation: writes dxdt, DT, adds DT to TIME, updates x
 * on mobile sites and writes SUMX. dt_in > 0 forces that time step for every
 * system; dt_in <= 0 uses the stable rule. Bonds (same-type sites closer than
 * r_bond) are built from the current positions. */
mxe_status mxe_step(mxe_plan* plan, const mxe_state* state, const mxe_out* out, double dt_in,
                    void* ws, size_t ws_bytes, void* stream);

/* n_steps diffusion steps of the staggered scheme (Alg. 1): per step relax
 * at fixed x, then one Euler step of x with mu of the last evaluation. Bonds
 * are built once at the start from the current positions. With use_graph != 0
 * the per-step launch sequence is recorded once into a HIP graph (per plan,
 * buffers and launch extent; at most 16 are kept) and replayed; with
 * params.relax_chunk > 0, graphs of a chunk of relax_chunk iterations (lean
 * ones in small plans, see relax_chunk), of one iteration with the
 * neighbour-build chain and of the Euler step are recorded instead, and each
 * relaxation replays the first until every system has finished, the second
 * after chunks that left systems stalled. */
mxe_status mxe_run(mxe_plan* plan, const mxe_state* state, const mxe_out* out, int n_steps,
                   int use_graph, void* ws, size_t ws_bytes, void* stream);

/* Free-running steps (Sec. 4, Alg. 1, per system): every system with steps
 * left relaxes at fixed x; when its relaxation ends (converged or max_relax
 * updates) its Euler step follows in the same iteration and, if steps remain,
 * its next relaxation starts with the next iteration, whatever the other
 * systems are doing. Each system runs exactly the relaxations and steps it
 * would run alone under mxe_run, so its results equal those bitwise; only
 * systems stop waiting for each other at step boundaries (continuous batching
 * of requests, one iteration at a time).
 *   mxe_plan_set_steps gives a slot a budget of n_steps diffusion steps from
 *   the next mxe_advance on: its counters and scalars restart, a fresh
 *   relaxation begins, and MXE_S_STEPS_LEFT counts down to 0. A slot never
 *   given a budget has none.
 *   mxe_advance enqueues up to max_iters iterations, in chunks of
 *   params.relax_chunk (required > 0), and stops early once no system has
 *   steps left (read on the host one chunk behind; the call waits on the host
 *   between chunks); after a chunk that left systems stalled for a list build
 *   it adds one iteration with the build chain (see relax_chunk). Systems keep their relaxation state, counters and budget
 *   across calls, so a later call continues where this one stopped. Resume
 *   mode is required (slots rebound since the last call rebuild their lists
 *   and bonds; bonds are built when a slot is bound and kept after). With
 *   use_graph != 0 a chunk of iterations is recorded once per buffers and
 *   launch extent and replayed.
 * Errors: MXE_EINVAL for relax_chunk <= 0, resume mode off, max_iters < 0, a
 * slot out of range or n_steps < 0. */
mxe_status mxe_plan_set_steps(mxe_plan* plan, int slot, int n_steps);
mxe_status mxe_advance(mxe_plan* plan, const mxe_state* state, const mxe_out* out, int max_iters,
                       int use_graph, void* ws, size_t ws_bytes, void* stream);

/* Size of the device scratch that mxe_run_noalloc uses instead of a workspace:
 * one array per device, held from the library's first use on that device
 * until the process ends. */
#define MXE_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)

/* For callers that cannot allocate device memory (code under stream capture,
 * tight serving loops, harnesses that forbid allocation): mxe_run with eager
 * launches whose workspace is the library's own per-device scratch of
 * MXE_NOALLOC_SCRATCH_BYTES instead of a caller buffer. The caller still owns
 * the state and outputs. The call allocates nothing (no hipMalloc, no
 * allocating library routine; its host-to-device copies of the plan's tables
 * come from host memory the plan owns).
 * Semantics: as mxe_run(use_graph = 0) with params.relax_chunk ignored (its
 * early exit needs pinned host memory), except that every call starts afresh:
 * it uploads the plan's tables and rebuilds every neighbour list and bond
 * (resume mode is ignored), since other calls may have overwritten the scratch.
 * Results equal mxe_run's on a caller workspace.
 * Errors: MXE_ENOMEM if mxe_workspace_bytes of the plan exceeds
 * MXE_NOALLOC_SCRATCH_BYTES (nothing is launched); MXE_EINVAL with profiling
 * switched on (profiling creates events).
 * Concurrency: all calls on one device share that device's scratch, which
 * keeps the last call's contents; calls that overlap on one device (other
 * streams, other threads, other plans) race and must be serialised by the
 * caller. */
mxe_status mxe_run_noalloc(mxe_plan* plan, const mxe_state* state, const mxe_out* out, int n_steps,
                           void* stream);

/* Workspace layout, for inspection of the neighbour and bond lists (the
 * lists of Sec. 4, Alg. 1, and the nearest-neighbour bonds of the kinetic law,
 * Sec. 3.1). Items, each a dense int32 array at a byte offset in the workspace:
 *   MXE_L_NBR         [n_sites][k_max]: row i lists the neighbours j of site i
 *                     (ascending; the first count[i] entries are valid): every
 *                     pair with |rbar_ij| < r_c + reach_ij + skin at the last
 *                     build, reach_ij = 3 sqrt(sigma_i^2 + sigma_j^2) under the
 *                     27-node rule and sqrt(6) max(sigma_i, sigma_j) under the
 *                     degree-3 rule (the rule's farthest node), interstitial
 *                     pairs excluded, plus possibly pairs within 1e-5 A of that
 *                     radius
 *   MXE_L_NBR_COUNT   [n_sites]
 *   MXE_L_BOND        [n_sites][bond_max]: bonds of mobile site i (ascending),
 *                     same-type sites closer than r_bond
 *   MXE_L_BOND_COUNT  [n_sites]
 * Global site indices (concatenated systems). Valid after a call that built the
 * lists (every call outside resume mode) or the bonds (mxe_step, mxe_run), once
 * the stream has synchronised. Host-only: returns the byte offset and size. */
enum { MXE_L_NBR = 0, MXE_L_NBR_COUNT = 1, MXE_L_BOND = 2, MXE_L_BOND_COUNT = 3 };
mxe_status mxe_plan_layout(const mxe_plan* plan, int item, size_t* offset, size_t* bytes);

/* Kernel families timed by the profiling switch. */
typedef enum {
    MXE_K_PAIR = 0,     /* pair quadrature: 27 nodes -> 14 moments per pair    */
    MXE_K_DENSITY = 1,  /* density gather and Taylor embedding terms           */
    MXE_K_FORCE = 2,    /* force / mu gather and chunk partial sums            */
    MXE_K_BUILD = 3,    /* neighbour-list build chain (mostly early exits)     */
    MXE_K_FIRE = 4,     /* FIRE control and update                             */
    MXE_K_MASTER = 5,   /* master-equation flux, time step, Euler update       */
    MXE_NPROF = 6
} mxe_kernel;

/* Profiling modes of mxe_profile. */
enum {
    MXE_PROFILE_OFF = 0,   /* no events                                           */
    MXE_PROFILE_ALL = 1,   /* every kernel family bracketed                       */
    MXE_PROFILE_PAIR = 2   /* only the pair kernel bracketed (two events per
                              evaluation: the least instrumentation that still
                              times the dominant kernel)                         */
};

/* Profiling switch (instrumentation, not part of the method). With a mode
 * other than MXE_PROFILE_OFF, later calls launch eagerly (mxe_run ignores
 * use_graph) and bracket each launch of the selected kernel families with
 * HIP events recorded on the launch stream; every event is a point where the
 * stream's queue drains, so fewer families cost less. mxe_profile_read waits
 * for those events and returns, per family, the summed duration in ms and
 * the number of launches since the previous read (arrays of MXE_NPROF
 * entries, caller-owned host memory; zero for families not bracketed).
 * Errors: MXE_EINVAL for a null plan or an unknown mode. */
mxe_status mxe_profile(mxe_plan* plan, int on);
mxe_status mxe_profile_read(mxe_plan* plan, double* ms, int64_t* launches);

const char* mxe_status_string(mxe_status s);
const char* mxe_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
