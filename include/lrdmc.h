/*
 * lrdmc.h -- C ABI of the MI355X (gfx950) lattice-regularized diffusion Monte
 * Carlo hot path: the per-walker projection step between branchings, run for
 * the whole walker population on one GPU, and the weight-based
 * reconfiguration that follows it.
 *
 * Method: K. Nakano, S. Sorella, M. Casula, "Load-Balanced Diffusion Monte
 * Carlo Method with Lattice Regularization", arXiv:2508.12033.
 *   - conventional continuous-time scheme: Sec. II.B, Algorithm 1;
 *   - load-balanced fixed-N_proj scheme: Sec. II.C, Algorithm 2;
 *   - reconfiguration and estimators: Sec. II.A;
 *   - fixed-node lattice Hamiltonian, regularized potential: App. D.
 *
 * Conventions for every call:
 *   - Return value: 0 = success, < 0 = error (LRDMC_ERR_*).  No C++
 *     exception crosses this boundary.  lrdmc_last_error() returns a
 *     thread-local message describing the last error of the calling thread.
 *   - Host arrays are owned by the caller and are copied during the call.
 *   - The device workspace is owned by the caller (any device allocation,
 *     e.g. a torch tensor), must stay valid until lrdmc_destroy and is never
 *     freed by the library.  The handle owns only host-side metadata.
 *   - All device work is enqueued on the caller's HIP stream (passed as
 *     void* = hipStream_t); calls that return host results synchronise that
 *     stream.  A handle is not thread-safe.
 *   - Units: bohr and hartree.
 *   - Electrons 0..n_up-1 are spin up.  Lattice move p = (3 i + d) * 2 + s
 *     moves electron i by +a (s = 0) or -a (s = 1) along versor d (the axis
 *     x, y, z, or its randomly rotated image when lrdmc_params.rotate = 1).
 */
#ifndef LRDMC_H
#define LRDMC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- status codes ------------------------------------------------------ */
#define LRDMC_OK                   0
#define LRDMC_ERR_INVALID_ARG     -1  /* bad size, pointer or parameter */
#define LRDMC_ERR_HIP             -2  /* a HIP runtime call failed */
#define LRDMC_ERR_WORKSPACE       -3  /* workspace smaller than lrdmc_workspace_bytes */
#define LRDMC_ERR_SINGULAR        -4  /* a Slater matrix is exactly singular */
#define LRDMC_ERR_ALL_DEAD        -5  /* every walker weight is zero at branching */
#define LRDMC_ERR_UNSUPPORTED     -6  /* sizes beyond what the kernels support */
#define LRDMC_ERR_NONFINITE       -7  /* a walker ended a phase with a NaN or infinite
                                         e_L or W, or a NaN or +inf log-weight (-inf is a
                                         dead walker), or a reconfiguration produced a
                                         non-finite weight sum or walker average */
#define LRDMC_ERR_NEG_WEIGHT      -8  /* strict mode only: W - E_0 <= 0 at some
                                         load-balanced step, so b_x = bbar / (W - E_0) is
                                         not a weight (Sec. II.C requires W - E_0 > 0) */
#define LRDMC_ERR_NO_MOVE         -9  /* strict mode only: a configuration with no
                                         allowed lattice move (bbar = 0) */
/* A positive return value of lrdmc_step and lrdmc_run (when they fill their
 * statistics) is a warning count: the number of walker-steps at which
 * W - E_0 <= 0 or bbar = 0 (n_neg_weight + n_no_move).  In the load-balanced
 * scheme such a walker's weight is set to zero and it dies at the next
 * reconfiguration; in the conventional scheme a walker with bbar = 0 stays in
 * place until its projection time is used up.  With lrdmc_params.strict = 1
 * the same events return LRDMC_ERR_NEG_WEIGHT / LRDMC_ERR_NO_MOVE instead
 * (the walker state is updated either way). */

/* ---- enumerations ------------------------------------------------------ */
#define LRDMC_SCHEME_LB    0   /* load-balanced, fixed N_proj (Algorithm 2) */
#define LRDMC_SCHEME_CONV  1   /* conventional continuous time (Algorithm 1) */

#define LRDMC_FP64         0   /* every step in FP64, one wavefront per
                                  walker; per system the layout that puts
                                  more walkers on a CU: all walker state in
                                  LDS, or the coefficient block, Slater rows
                                  and (if that fits more walkers) the inverse
                                  of the spin not moving in global memory
                                  (the only choice from 64 electrons on); at
                                  most 64
                                  electrons per spin, beyond that
                                  lrdmc_workspace_bytes returns 0 */
#define LRDMC_MIXED_FP32   1   /* mixed precision (an extension: the paper
                                  computes in FP64): orbital rows,
                                  Sherman-Morrison updates, ratios and Jastrow
                                  in FP32; positions, weights, local-energy
                                  accumulation, the periodic refresh of the
                                  inverse and the estimator values handed to
                                  the reconfiguration in FP64; orbital
                                  product on FP32 MFMA */
#define LRDMC_MIXED_BF16   2   /* as LRDMC_MIXED_FP32, with the orbital
                                  product on BF16 MFMA (FP32 accumulation) */

#define LRDMC_BASIS_S      0   /* exp(-alpha r^2) */
#define LRDMC_BASIS_PX     1   /* (x-X) exp(-alpha r^2), likewise PY, PZ */
#define LRDMC_BASIS_PY     2
#define LRDMC_BASIS_PZ     3
#define LRDMC_BASIS_STO1S  4   /* exp(-zeta r) */

#define LRDMC_CORE_BARE    0   /* -Z/r; lattice bound -Z/max(r,a) (App. D) */
#define LRDMC_CORE_SOFT    1   /* -Z/sqrt(r^2 + rc^2), a softened local core */

#define LRDMC_NU_OPT_OWN   0   /* nu_max for electron i iff one of its own 6
                                  moves crosses the node (App. D nu_opt) */
#define LRDMC_NU_OPT_ANY   1   /* iff any of the 6N moves crosses the node */
#define LRDMC_NU_MAX       2   /* nu_max = max(nu_zv, nu^a_ei) for every electron */

/* ---- system description (App. D Hamiltonian, Jastrow-Slater guide) ---- */
typedef struct lrdmc_system {
    int32_t n_atoms;
    const double *atom_pos;      /* [n_atoms][3] */
    const double *atom_charge;   /* [n_atoms] Z (bare) or valence Z_v (soft core) */
    const int32_t *atom_core;    /* [n_atoms] LRDMC_CORE_* */
    const double *core_rc;       /* [n_atoms] soft-core radius (ignored if bare) */
    const int32_t *atom_species; /* [n_atoms] in [0, n_species): e-n Jastrow row */
    int32_t n_basis;
    const int32_t *basis_atom;   /* [n_basis] centre */
    const int32_t *basis_type;   /* [n_basis] LRDMC_BASIS_* */
    const double *basis_exp;     /* [n_basis] alpha (Gaussian) or zeta (Slater) */
    int32_t n_orb;               /* >= max(n_up, n_dn); spin s uses columns 0..n_s-1 */
    const double *mo_coeff;      /* [n_basis][n_orb] row-major */
    int32_t n_up, n_dn;
    int32_t n_species;
    const double *jastrow;       /* [2 + n_species][3]: (A, B, b) of
                                    u(r) = (A r + B r^2)/(1 + b r); row 0 parallel
                                    e-e, row 1 antiparallel e-e, row 2+s e-n */
    int32_t n_walkers;           /* walkers of this system */
    uint64_t system_id;          /* second Philox key word */
    /* Non-local (semi-local) pseudopotential, App. D: the non-local elements
     * V^nl_{x',x} of the fixed-node Hamiltonian under the determinant
     * locality approximation (the guiding-function ratio of a non-local
     * element replaced by the determinant ratio D(x')/D(x)).  Term t adds
     * ecp_coef[t] r^ecp_pow[t] exp(-ecp_exp[t] r^2) to channel ecp_l[t]
     * (0, 1 or 2) of atom ecp_atom[t]; the channels of atom I act on an
     * electron at distance r < ecp_rcut[I] from it.  Reading: the projector
     * onto channel l is integrated by the 6-point octahedral quadrature of
     * the sphere of radius r around the atom along the walker's lattice
     * versors (weights 1/6); quadrature point q of electron i is proposal
     * 6N + 6i + q (after the 6N lattice moves) with element
     * V_q = sum_l (2l+1)/6 v_l(r) P_l(cos theta_q).  Positive
     * V_q D(x')/D(x) enter the spin-flip term, negative ones are moves of
     * rate -V_q D(x')/D(x).  The cutoff spheres of different atoms must not
     * overlap (LRDMC_ERR_INVALID_ARG otherwise).  n_ecp = 0: no non-local
     * part (the pointers are ignored).  FP64 precision only; the mixed
     * kinds and lrdmc_walker_derivs return LRDMC_ERR_UNSUPPORTED. */
    int32_t n_ecp;
    const int32_t *ecp_atom;     /* [n_ecp] */
    const int32_t *ecp_l;        /* [n_ecp] 0, 1, 2 */
    const int32_t *ecp_pow;      /* [n_ecp] 0, 1, 2 */
    const double *ecp_coef;      /* [n_ecp] */
    const double *ecp_exp;       /* [n_ecp] >= 0 */
    const double *ecp_rcut;      /* [n_atoms] cutoff radius, 0: no channels */
} lrdmc_system;

/* ---- run parameters ---------------------------------------------------- */
typedef struct lrdmc_params {
    int32_t scheme;          /* LRDMC_SCHEME_* */
    int32_t precision;       /* LRDMC_FP64 or LRDMC_MIXED_*; the mixed kinds keep
                                per-walker orbital data in HBM and support
                                larger systems than the FP64 layout */
    double a;                /* lattice space (bohr) */
    double tau;              /* conventional: projection time per branching */
    int32_t n_proj;          /* load-balanced: steps per branching */
    uint64_t seed;           /* first Philox key word */
    int32_t refresh_every;   /* moves between FP64 refreshes of the inverses and Jastrow caches,
                                >= 1 (the Python binding defaults to 128 in FP64, 16 mixed).
                                FP64: Gauss-Jordan rebuild.  Mixed: one or two Newton-Schulz
                                corrections of the carried FP32 inverse on FP64 MFMA (also at
                                the start of every phase), a Gauss-Jordan rebuild when its
                                residual is 3e-3 or more, after a tiny determinant ratio, and
                                for rows rebuilt from positions; the FP32 Jastrow caches are
                                rebuilt at every fourth scheduled refresh (and at the start of
                                a phase and after a tiny ratio) */
    int32_t nu_opt_mode;     /* LRDMC_NU_* */
    int32_t p_corr;          /* correcting factors: product of the p previous
                                average weights (Sec. II.A) */
    int32_t e0_window;       /* E_0 = mean of the last e0_window walker-averaged
                                local energies (load-balanced, Algorithm 2) */
    int32_t trace_cap;       /* > 0: record every walker's moves, up to this many
                                per branching, for the parity harness */
    int32_t strict;          /* 1: weight events are errors (LRDMC_ERR_NEG_WEIGHT,
                                LRDMC_ERR_NO_MOVE) instead of a warning count */
    int32_t rotate;          /* 1: randomized lattice (App. D: the versors of the
                                discretized Laplacian rotate with random angles).
                                Reading: each walker draws one uniformly random
                                rotation R at the start of every projection phase
                                from its own Philox stream (counter (slot, branching,
                                attempt, 4)), and its 6N moves that phase are
                                r_i +- a R e_d (every precision).  The adjoint pass
                                (lrdmc_walker_derivs) evaluates the fixed axes only
                                and returns LRDMC_ERR_UNSUPPORTED then.  0: fixed
                                x, y, z axes */
    int32_t n_therm;         /* branchings left out of the energy estimate (equilibration);
                                0: the first 10 % */
} lrdmc_params;

/* ---- statistics returned to the caller --------------------------------- */
typedef struct lrdmc_step_stats {
    int64_t walker_iters;    /* sum over walkers of the iterations that
                                evaluated all 6N ratios */
    int32_t max_iters;       /* slowest walker (conventional) or N_proj */
    int32_t min_iters;
    int64_t n_neg_weight;    /* evaluations with W - E_0 <= 0 (walker weight set to 0) */
    int64_t n_no_move;       /* evaluations with no allowed move (bbar = 0) */
    int64_t n_refresh;       /* FP64 refreshes performed (scheduled + forced) */
    int64_t n_small_ratio;   /* forced refreshes after |R_det| < 1e-6 */
    int64_t n_capped;        /* conventional walkers stopped by the termination
                                bound of 1000 * tau * 3N / a^2 + 10000 iterations */
    int64_t n_nonfinite;     /* walkers that ended the phase with a non-finite value
                                (the call then returns LRDMC_ERR_NONFINITE) */
    double elapsed_ms;       /* device time of the phase (HIP events) */
} lrdmc_step_stats;

typedef struct lrdmc_branch_stats {
    double log_wbar;         /* log of the average weight before reconfiguration */
    double e_bar;            /* walker-averaged local energy (Sec. II.A / II.C) */
    double e0;               /* E_0 after the update */
    double max_lw;           /* largest log-weight */
    int32_t n_distinct;      /* distinct parents kept by the comb */
    double elapsed_ms;       /* device time of the reconfiguration */
} lrdmc_branch_stats;

typedef struct lrdmc_energy {
    double energy;           /* correcting-factor estimate of E_0 (Sec. II.A) */
    double sigma;            /* blocking error bar */
    int32_t n_used;          /* branchings used */
} lrdmc_energy;

typedef struct lrdmc_tune_entry {
    int32_t threads;          /* workgroup size of the mixed-precision phase kernel */
    int32_t order_big_first;  /* 1: systems with more electrons first in the launch */
    float ms;                 /* projected time of a full phase */
    int32_t system;           /* -1: every mixed system in one launch; k >= 0: system k
                                 launched alone; -2: one launch per system, each with
                                 its fastest workgroup size (ms: their sum) */
} lrdmc_tune_entry;

/* ---- calls ------------------------------------------------------------- */

/* Bytes of device workspace needed for these systems and parameters.  Pure
 * function; 0 on invalid input (see lrdmc_last_error). */
size_t lrdmc_workspace_bytes(const lrdmc_system *sys, int n_sys, const lrdmc_params *prm);

/* Validate the inputs, upload the systems into the workspace, place every
 * walker at init_pos ([sum of n_walkers][n_up+n_dn][3] host FP64, walkers of
 * system 0 first), evaluate the local energies and set E_0 to their
 * unweighted mean.  The paper updates E_0 after every branching (Sec. II.C,
 * Algorithm 2) but states no starting value and no update formula; the
 * reading taken here is E_0^(0) = unweighted mean of the initial walkers'
 * e_L, and after branching n the mean of the walker-averaged e_L of the last
 * e0_window branchings.  A non-finite initial e_L returns
 * LRDMC_ERR_SINGULAR.  Synchronises `stream`.  *out receives the handle. */
int lrdmc_init_system(const lrdmc_system *sys, int n_sys, const lrdmc_params *prm,
                      const double *init_pos, void *dev_workspace, size_t ws_bytes,
                      void *stream, struct lrdmc_handle **out);

/* One projection phase for every walker (Algorithm 1 inner loop until every
 * tau_left = 0, or Algorithm 2 inner loop of N_proj steps): ratios of all 6N
 * lattice moves, lattice-regularized local energy with the fixed-node terms
 * on the diagonal, weight update, heat-bath move, Sherman-Morrison update.
 * Load-balanced: after the last move the walker's e_L and W are evaluated at
 * its final configuration for the estimator weight w / (W - E_0) of
 * Sec. II.C; W - E_0 <= 0 there also sets the weight to zero (counted in
 * n_neg_weight).  Asynchronous on the handle's stream when st == NULL (errors
 * found on the device then surface at the next call that synchronises);
 * otherwise synchronises, fills *st and returns LRDMC_ERR_SINGULAR,
 * LRDMC_ERR_NONFINITE, the warning count or (strict) LRDMC_ERR_NEG_WEIGHT /
 * LRDMC_ERR_NO_MOVE. */
int lrdmc_step(struct lrdmc_handle *h, lrdmc_step_stats *st);

/* Reconfiguration (Sec. II.A): walker-averaged local energy, FP64 prefix sum
 * of the weights, comb with N_w correlated numbers, gather of the selected
 * walkers, weights reset to 1; then appends (log wbar, e_bar) to the history
 * and updates E_0 (Algorithm 2), both on the device.  Synchronises and copies
 * the new history records to the host.  Returns LRDMC_ERR_ALL_DEAD when every
 * weight was zero and LRDMC_ERR_NONFINITE when the weight sums or the walker
 * average were not finite (nothing is appended to the history then). */
int lrdmc_branch(struct lrdmc_handle *h, lrdmc_branch_stats *st);

/* n_branchings cycles of (projection phase, reconfiguration) as by
 * lrdmc_step + lrdmc_branch, with E_0, the branching index and the history
 * kept on the device: each cycle is one replay of a HIP graph captured at the
 * first call (one graph per walker buffer slot), so the host issues one
 * launch per cycle and synchronises only at the end.  st: counters summed
 * over all cycles (max/min over all phases), elapsed time of the whole run;
 * bst: the last reconfiguration.  Either may be NULL. */
int lrdmc_run(struct lrdmc_handle *h, int n_branchings, lrdmc_step_stats *st,
              lrdmc_branch_stats *bst);

/* Autotuner of the mixed-precision launch.  Candidates: every mixed-precision
 * system of the handle in one launch, for each workgroup size (256, 128 or 64
 * threads per walker) and order of the systems; and, with several systems,
 * one launch per system with its own LDS block and its own fastest workgroup
 * size.  Each is timed on a copy of the current walkers for n_steps and
 * 2 n_steps load-balanced steps, and the one with the shortest projected full
 * phase (fixed cost plus N_proj times the per-step cost) is kept for later
 * phases.  The walkers, weights, E_0 and random streams of the run are not
 * changed.  log (may be NULL) receives up to log_cap timings, *n_log their
 * number.  Synchronises.  No effect for FP64 handles. */
int lrdmc_autotune(struct lrdmc_handle *h, int n_steps, lrdmc_tune_entry *log, int log_cap,
                   int *n_log);

/* Fix the mixed-precision launch instead of tuning it: every mixed system in
 * one launch with threads per walker workgroup (64, 128 or 256), or threads =
 * 0: one launch per system, each with its own LDS block and the workgroup size
 * of the last tuning (256 before any); order_big_first: the order of the
 * systems (1: more electrons first).  No effect on results beyond FP32
 * summation order. */
int lrdmc_set_launch(struct lrdmc_handle *h, int threads, int order_big_first);

/* Energy estimate from the branching history (Sec. II.A correcting factors,
 * the first n_therm branchings, or the first 10 % if n_therm = 0, dropped).  When forces ([n_atoms][3], host) or
 * jgrad ([3 (2 + n_species)], host) is non-NULL, the adjoint pass
 * (lrdmc_walker_derivs) runs over the current walkers of system 0 and the
 * weighted population (omega = w/(W - E_0) load-balanced, w conventional)
 * gives, for every parameter theta,
 *   dE/dtheta = <de_L/dtheta> + 2 <(e_L - E) d log|Psi|/dtheta>
 * (the mixed-estimator form; an approximation in DMC, the paper defines no
 * force estimator).  forces = -dE/dR_I; jgrad = dE/d(Jastrow table).
 * Synchronises. */
int lrdmc_energy_forces(struct lrdmc_handle *h, lrdmc_energy *e, double *forces, double *jgrad);

/* Number of parameters theta of system isys: 3 n_atoms nuclear coordinates,
 * then the Jastrow table [2 + n_species][3] row-major. */
int lrdmc_n_theta(struct lrdmc_handle *h, int isys);

/* Adjoint pass: per walker of system isys, at its current configuration, the
 * lattice-regularized local energy e_L (App. D, W - bbar) and log|Psi_G|, and
 * their derivatives with respect to theta (basis functions move with their
 * nucleus; the nu_opt and node choices are held at the evaluated branch).
 * FP64, inverses recomputed by Gauss-Jordan.  theta: host [n_theta]
 * replacing the system's parameters for this call only, or NULL.  Outputs are
 * device pointers: eL, logpsi [n_walkers]; deL, dlogpsi [n_walkers][n_theta]
 * (NULL: kept in the library's workspace).  Synchronises.  Systems whose
 * per-walker adjoint data exceed one workgroup's LDS return
 * LRDMC_ERR_UNSUPPORTED. */
int lrdmc_walker_derivs(struct lrdmc_handle *h, int isys, const double *theta, double *eL,
                        double *logpsi, double *deL, double *dlogpsi);

/* Host copies of the walker state of system `isys` for the parity harness.
 * Any pointer may be NULL.  pos [nw][N][3], lw/eL/W [nw], iters [nw],
 * sel [nw] (parents chosen by the last lrdmc_branch), trace [nw][trace_cap]
 * (moves of the last phase; -1 marks the conventional stopping iteration,
 * -2 unused).  Synchronises. */
int lrdmc_get_walkers(struct lrdmc_handle *h, int isys, double *pos, double *lw, double *eL,
                      double *W, int32_t *iters, int32_t *sel, int32_t *trace);

/* Mixed precisions only: per walker of system isys, [nw][4] host doubles
 * describing the last phase at its final configuration: e_L, W and bbar as
 * the mixed-precision step computed them, and the largest ratio error
 * max_p |R_p - R_p(FP64)| / max(1, |R_p(FP64)|).  The e_L and W that the
 * library reports (lrdmc_get_walkers) and uses for the reconfiguration are
 * the FP64 evaluation of the same configuration.  Valid until the next
 * reconfiguration, which reorders the walkers.  Synchronises. */
int lrdmc_get_precision_report(struct lrdmc_handle *h, int isys, double *out);

/* Overwrite positions (and log-weights if lw != NULL) of system `isys`. */
int lrdmc_set_walkers(struct lrdmc_handle *h, int isys, const double *pos, const double *lw);

/* Current E_0 of system isys; set_e0 overrides it (for the parity harness). */
double lrdmc_get_e0(struct lrdmc_handle *h, int isys);
int lrdmc_set_e0(struct lrdmc_handle *h, int isys, double e0);

/* ---- reconfiguration of a population held by the caller --------------- */

/* Device workspace bytes of lrdmc_reconfigure for nw walkers (0 and an error
 * message for nw < 1): (nw rounded up to 32 + 16) doubles. */
size_t lrdmc_reconfigure_workspace_bytes(int nw);

/* The reconfiguration of Sec. II.A on device arrays owned by the caller,
 * without a handle (for callers that keep their walkers themselves, e.g. one
 * shard of a population): the inclusive FP64 prefix C of exp(lw - max lw) in
 * walker order, the comb sel[alpha] = min{beta : C_beta > (xi + alpha) C_N / nw}
 * with one Philox uniform xi = U(seed, sysid; slot 0, branching j, 0, comb),
 * and the walker average of e_L with weights w (scheme LRDMC_SCHEME_CONV) or
 * w / (W - E_0) (LRDMC_SCHEME_LB, Sec. II.C); walkers with lw = -inf are dead
 * and never selected.  Arguments (all pointers device memory, caller-owned):
 *   lw, eL [nw] (and W [nw] for LB; may be NULL for CONV) -- read only;
 *   sel [nw] int32 -- written: parent index of each new walker;
 *   out [8] doubles -- written: [0] log of the average weight
 *     log(C_N / nw) + max lw, [1] walker-averaged e_L, [2] max lw, [3] number
 *     of distinct parents, [4] status 0 ok, 1 every weight zero (sel then
 *     all 0), 2 non-finite sums;
 *   ws -- scratch of lrdmc_reconfigure_workspace_bytes(nw), 256-byte
 *     aligned, overwritten.
 * Enqueued on `stream` (hipStream_t) without synchronising and without
 * allocating; captures into a HIP graph (no memset or copy nodes).  Returns
 * LRDMC_ERR_INVALID_ARG / LRDMC_ERR_WORKSPACE for bad arguments before any
 * device work, LRDMC_ERR_HIP if a launch fails. */
int lrdmc_reconfigure(int scheme, int nw, const double *lw, const double *eL, const double *W,
                      double e0, uint64_t seed, uint64_t sysid, int j, int32_t *sel,
                      double *out, void *ws, size_t ws_bytes, void *stream);

/* Largest population of lrdmc_reconfigure_noalloc. */
#define LRDMC_NOALLOC_MAX_WALKERS 1048576

/* lrdmc_reconfigure without a workspace argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid allocation): its prefix sums and sums live in a fixed
 * device array of the library (8 MiB, one copy per GPU, held until the
 * process ends), so the call allocates nothing.  Same arguments, results and
 * errors as lrdmc_reconfigure; nw > LRDMC_NOALLOC_MAX_WALKERS returns
 * LRDMC_ERR_INVALID_ARG before any device work.  The arrays and the stream
 * must belong to the device current on the calling thread.  The first call on
 * a device looks up the array's device address (hipGetSymbolAddress); make it
 * outside a graph capture.  Every call on one GPU shares that GPU's array:
 * calls that overlap on one GPU (different streams or threads without
 * ordering between them) race and give wrong results; calls ordered on one
 * stream are safe (each call rewrites what it reads). */
int lrdmc_reconfigure_noalloc(int scheme, int nw, const double *lw, const double *eL,
                              const double *W, double e0, uint64_t seed, uint64_t sysid, int j,
                              int32_t *sel, double *out, void *stream);

/* Branching index j used in the Philox counters of the next phase. */
int lrdmc_get_branch_index(struct lrdmc_handle *h);

void lrdmc_destroy(struct lrdmc_handle *h);
const char *lrdmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* LRDMC_H */
