/*
 * hmc.h -- C ABI of the MI355X (gfx950) HIP library for the Hybrid Monte Carlo hot path
 * of the O(3) spin-fermion model (Lunts, Albergo, Lindsey, arXiv:2204.14241).
 *
 * The library applies the space-time fermion matrix M[phi] of Eq. (17) and its adjoint,
 * solves the normal equations (M^dagger M) x = chi by conjugate gradient (Methods C,
 * Eq. 22), evaluates the pseudofermion action of Eq. (21) and its gradient, the boson
 * action of Eq. (2), and runs leapfrog HMC trajectories with a Metropolis decision
 * (Methods D, Eq. 27-29).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - Return value: HMC_OK (0) on success, a negative HMC_ERR_* code otherwise; no
 *    exception crosses the ABI.  hmc_last_error() gives a message for the calling thread.
 *  - Pointers named phi, in, out, b, x, chi, eta, pi, force are DEVICE pointers owned
 *    by the caller; they must be 16-byte aligned.  Host pointers are marked "host".
 *  - stream is a hipStream_t passed as void* (NULL = the null stream).  Work is
 *    enqueued on it; entry points that must read a device scalar back (CG convergence,
 *    actions, trajectories) synchronise with it before returning.
 *  - Layouts (row-major, index order of Eq. 17):
 *      boson field phi     : double[3][L_tau][L][L]   (float for the *_f32 entry points)
 *      spinor (one vector) : complex[4][L_tau][L][L] with component c = 2*band + spin,
 *                            band 0 = the paper's band x, spin 0 = up; complex numbers
 *                            are interleaved (re, im) pairs: complex128 for FP64 entry
 *                            points, complex64 for *_f32 ones.
 *      n vectors           : n consecutive spinors, stride 4*L_tau*L*L complex.
 *  - A context is bound to the device current at hmc_create and is not thread-safe; use
 *    one context per stream.
 *  - The library allocates no device memory.  Scratch space is a caller-owned device
 *    buffer of hmc_workspace_bytes() bytes handed over with hmc_set_workspace(); entry
 *    points that need it fail with HMC_ERR_WORKSPACE until it is set.  The library
 *    allocates a small pinned host buffer and events for its own status reads.
 */
#ifndef HMC_H
#define HMC_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HMC_OK                 0
#define HMC_ERR_INVALID_ARG   -1   /* bad size, parameter or pointer                     */
#define HMC_ERR_NOT_CONVERGED -2   /* CG hit cg_maxit; x and stats are still written     */
#define HMC_ERR_NONFINITE     -3   /* NaN/Inf met in a reduction; trajectory rejected    */
#define HMC_ERR_HIP           -4   /* a HIP runtime call failed (see hmc_last_error)     */
#define HMC_ERR_WORKSPACE     -5   /* workspace missing or too small                     */

#define HMC_FP64  0                /* all arithmetic in double                           */
#define HMC_MIXED 1                /* FP32 Krylov iterations, FP64 reliable updates      */

#define HMC_MAX_RHS 16             /* most right-hand sides one solve accepts            */

#define HMC_PRECOND_NONE    0      /* plain CG on M^dagger M                             */
#define HMC_PRECOND_FOURIER 1      /* CG preconditioned with P = (K K^dagger)^{-1}, K the
                                      phi-independent part of M (Methods C, Eq. 23-26):
                                      (x, y) FFTs, and along tau the exact inverse of K
                                      per frequency (what the twisted tau FFT diagonalises) */

/* Model and run parameters.  Eq. (17) for the fermion terms, Eq. (2) for the boson. */
typedef struct hmc_params {
    double t[2][2];      /* nearest-neighbour hopping t[band][direction]; direction 0 is
                            the slower spatial index x, 1 the faster index y             */
    double mu[2];        /* chemical potential per band                                  */
    double lambda;       /* Yukawa coefficient (the paper's g in Eq. 17)                 */
    double r, c, u;      /* boson mass squared, velocity, quartic coupling (Eq. 2)       */
    double eps;          /* leapfrog step                                                */
    int    n_leap;       /* leapfrog steps per trajectory                                */
    int    n_pf;         /* pseudofermions per trajectory (each carries full weight)     */
    double cg_tol;       /* relative true-residual target ||b - A x|| / ||b||            */
    int    cg_maxit;     /* iteration cap per solve                                      */
    int    precision;    /* HMC_FP64 or HMC_MIXED                                        */
    int    reliable_every; /* mixed precision: FP64 reliable update every k iterations    */
    int    max_rhs;      /* right-hand sides the workspace is sized for (0: n_pf)        */
    int    precond;      /* HMC_PRECOND_NONE or HMC_PRECOND_FOURIER.  The Fourier form
                            needs L and L_tau whose prime factors are <= 7, an L x L
                            slice (FP64 in FP64 solves) that fits the GPU's LDS
                            (L <= 100 on gfx950) and L_tau <= 320 (mixed) or 256 (FP64);
                            otherwise HMC_ERR_INVALID_ARG                                */
    double tn[2][2];     /* hopping by two sites along direction d, tn[band][d]: the
                            next-nearest-neighbour terms of the production model (the
                            paper's t_tilde_{h,alpha} along x, t_tilde_{v,alpha} along y);
                            zero for the nearest-neighbour model                         */
} hmc_params;

/* Per-solve statistics (host struct filled by the solver entry points). */
typedef struct hmc_cg_stats {
    int    n;                          /* right-hand sides solved                          */
    int    status;                     /* HMC_OK, HMC_ERR_NOT_CONVERGED or NONFINITE       */
    int    iterations[HMC_MAX_RHS];    /* Krylov iterations per right-hand side            */
    int    reliable_updates[HMC_MAX_RHS]; /* FP64 true-residual recomputations             */
    double true_resid[HMC_MAX_RHS];    /* final ||b - A x|| / ||b|| evaluated in FP64       */
} hmc_cg_stats;

/* Per-trajectory statistics (host struct). */
typedef struct hmc_traj_stats {
    double dH;            /* H(end) - H(start)                                           */
    double H0, H1;        /* Hamiltonians of Eq. (28) at the two ends                    */
    double S_pf0, S_pf1;  /* pseudofermion action at the start (|eta|^2) and end         */
    double S_b0, S_b1;    /* boson action                                                */
    double K0, K1;        /* kinetic energy 1/2 |pi|^2                                   */
    int    accepted;      /* 1 if u < exp(-dH)                                           */
    int    cg_solves;     /* solves run (n_leap + 1, each over n_pf right-hand sides)    */
    long   cg_iterations; /* Krylov iterations summed over solves and right-hand sides   */
    double max_true_resid;/* largest final relative residual over all solves             */
    int    status;        /* worst status met                                            */
} hmc_traj_stats;

typedef struct hmc_ctx hmc_ctx;

/* Create a context for an L x L x L_tau lattice with Trotter step dtau (Methods A).
 * L must be even (the ordering-vector phase (-1)^(x+y) needs it), 4 <= L <= 256;
 * L_tau >= 2; L_tau*L*L < 2^26; dtau > 0.  params is copied.  *out receives the handle.
 * Errors: HMC_ERR_INVALID_ARG, HMC_ERR_HIP. */
int hmc_create(int L, int L_tau, double dtau, const hmc_params* params, hmc_ctx** out);

/* Release the context (not the caller's buffers). */
int hmc_destroy(hmc_ctx* ctx);

/* Update run parameters (eps, n_leap, n_pf, cg_tol, cg_maxit, precision, reliable_every
 * and the model couplings).  n_pf and max_rhs may not exceed the capacity the workspace
 * was sized for.  Errors: HMC_ERR_INVALID_ARG. */
int hmc_set_params(hmc_ctx* ctx, const hmc_params* params);

/* Bytes of device workspace the context needs (sized for max_rhs right-hand sides in
 * the precision set at creation, plus trajectory state). */
size_t hmc_workspace_bytes(const hmc_ctx* ctx);

/* Hand over a device buffer of at least hmc_workspace_bytes() bytes, 256-byte aligned.
 * The caller keeps ownership and must keep it alive while the context uses it.
 * Errors: HMC_ERR_INVALID_ARG, HMC_ERR_WORKSPACE. */
int hmc_set_workspace(hmc_ctx* ctx, void* dev_ptr, size_t bytes);

/* out_k = M[phi] in_k for k < n (Eq. 17): diagonal -(1 + dtau mu_band), forward time
 * link +1 (-1 from the last slice to the first: antiperiodic), hopping -dtau t, on-site
 * dtau lambda (-1)^(x+y) (phi . Pauli) across the two bands.  in and out must not
 * overlap.  No workspace needed.  Errors: HMC_ERR_INVALID_ARG, HMC_ERR_HIP. */
int hmc_apply_M(hmc_ctx* ctx, const double* phi, const void* in, void* out, int n, void* stream);

/* out_k = M[phi]^dagger in_k: the same time-local part (it is Hermitian) and the
 * backward time link from tau - 1 with the sign of that link. */
int hmc_apply_Mdag(hmc_ctx* ctx, const double* phi, const void* in, void* out, int n, void* stream);

/* out_k = M^dagger M in_k, the normal operator of Eq. (22) (n <= max_rhs).  The
 * nearest-neighbour operator is applied in one pass over memory: M in_k is formed band by
 * band in LDS and never stored (read in and phi, write out; see hmc_set_mdm_shape).  With
 * the two-site hops (params.tn nonzero) two passes, the intermediate M in_k in the
 * workspace.  The workspace must be set either way.  in and out must not overlap.  Errors as
 * above plus HMC_ERR_WORKSPACE. */
int hmc_apply_MdagM(hmc_ctx* ctx, const double* phi, const void* in, void* out, int n, void* stream);

/* FP32 forms of the three applies: phi is float[3][L_tau][L][L], spinors complex64.
 * Arithmetic and accumulation are FP32. */
int hmc_apply_M_f32(hmc_ctx* ctx, const float* phi, const void* in, void* out, int n, void* stream);
int hmc_apply_Mdag_f32(hmc_ctx* ctx, const float* phi, const void* in, void* out, int n, void* stream);
int hmc_apply_MdagM_f32(hmc_ctx* ctx, const float* phi, const void* in, void* out, int n, void* stream);

/* hmc_apply_MdagM (FP64, two passes) for callers that cannot allocate device memory or use a
 * workspace: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  The intermediate M in lives in a static device buffer of the library
 * (HMC_NOALLOC_SCRATCH_BYTES per GPU, held until the process ends) instead of the workspace;
 * the context's workspace need not be set.  Nothing is allocated, freed or synchronised.
 * n * 4 * L_tau * L^2 * 16 bytes must fit the buffer (n = 1 up to 1,048,576 sites, e.g.
 * 40 x 40 x 100 with n <= 6), else HMC_ERR_INVALID_ARG.  Every call on one GPU shares that
 * GPU's buffer and leaves its intermediate there: calls that overlap on one GPU (two streams,
 * two threads) race and must be serialised by the caller.  One-lattice contexts only.
 * Results are bitwise those of hmc_apply_M followed by hmc_apply_Mdag.  Errors:
 * HMC_ERR_INVALID_ARG, HMC_ERR_HIP. */
#define HMC_NOALLOC_SCRATCH_BYTES (64u << 20)
int hmc_apply_MdagM_noalloc(hmc_ctx* ctx, const double* phi, const void* in, void* out, int n, void* stream);

/* Solve (M^dagger M) x_k = b_k, k < n <= max_rhs, by conjugate gradient from x = 0
 * (Methods C).  b, x: complex128 spinors.  Convergence: the FP64 true residual
 * ||b - A x|| / ||b|| <= cg_tol, evaluated once the iterated residual passes that bound
 * (CG restarts from the true residual if it does not).  With precision HMC_MIXED the
 * Krylov iterations run in FP32 (complex64 vectors, FP32 phi, FP64 dot products) and x,
 * r are refreshed in FP64 every reliable_every iterations.  stats (host, may be NULL)
 * receives per-right-hand-side counts and residuals.  Synchronises the stream.
 * Errors: HMC_ERR_NOT_CONVERGED (x still written), HMC_ERR_NONFINITE, INVALID_ARG,
 * WORKSPACE, HIP. */
int hmc_cg_solve(hmc_ctx* ctx, const double* phi, const void* b, void* x, int n,
                 hmc_cg_stats* stats, void* stream);

/* Pseudofermion heat-bath (Methods D): chi_k = M[phi]^dagger eta_k for standard complex
 * Gaussian eta_k (drawn by the caller), so that chi ~ CN(0, M^dagger M). */
int hmc_heatbath(hmc_ctx* ctx, const double* phi, const void* eta, void* chi, int n_pf, void* stream);

#define HMC_FORCE_PF    1          /* include dS_PF/dphi                                  */
#define HMC_FORCE_BOSON 2          /* include dS_B/dphi                                   */

/* Gradient dS/dphi of S = S_PF + S_B (selected by flags) at phi, with
 * S_PF = sum_k chi_k^dagger (M^dagger M)^{-1} chi_k (Eq. 21).  Solves by CG (settings of
 * the context), then per site: Y = M x, dS_PF/dphi_l = -2 dtau lambda (-1)^(x+y)
 * Re sum_k [Y_{band x}^dagger Pauli_l x_{band y} + Y_{band y}^dagger Pauli_l x_{band x}].
 * force: double[3][L_tau][L][L] (overwritten).  S_pf (DEVICE scalar, may be NULL) receives
 * sum_k Re <chi_k, x_k> (0 without HMC_FORCE_PF), written on the stream after the gradient;
 * stats (host, may be NULL) the solver statistics.  Synchronises the stream (the solver reads
 * its convergence status).  Errors as hmc_cg_solve. */
int hmc_force(hmc_ctx* ctx, const double* phi, const void* chi, int n_pf, double* force,
              double* S_pf, int flags, hmc_cg_stats* stats, void* stream);

/* The same gradient from given solutions x_k of (M^dagger M) x_k = chi_k (no solve):
 * for callers that keep the solutions.  Does not synchronise. */
int hmc_force_from_solution(hmc_ctx* ctx, const double* phi, const void* x, int n_pf,
                            double* force, int flags, void* stream);

/* Pseudofermion action sum_k chi_k^dagger (M^dagger M)^{-1} chi_k (Eq. 21) by CG; the
 * solutions are written to x (device, n_pf complex128 spinors) when x is not NULL.
 * S (host) receives the value.  Synchronises the stream. */
int hmc_pf_action(hmc_ctx* ctx, const double* phi, const void* chi, int n_pf, void* x,
                  double* S, hmc_cg_stats* stats, void* stream);

/* Boson action S_B (Eq. 2; time-derivative coefficient 1/(2 c^2), forward differences,
 * periodic in time and space).  S (host) receives it.  Synchronises the stream. */
int hmc_boson_action(hmc_ctx* ctx, const double* phi, double* S, void* stream);

/* One HMC trajectory (Methods D).  chi_k = M[phi0]^dagger eta_k; H0 = |pi0|^2/2 + S_B +
 * sum_k |eta_k|^2; n_leap kick-drift-kick steps of size eps (half kicks kept separate),
 * each drift followed by a CG solve per pseudofermion and the gradient; H1 uses the
 * last solve.  Accept iff u_uniform < exp(-dH).  phi_inout holds phi0 on entry and the
 * chain's next field on return (the proposal if accepted, phi0 otherwise).  pi0 is not
 * modified.  stats (host) receives energies, the decision and solver counts.
 * Synchronises the stream.  Errors: as hmc_cg_solve; on any error phi_inout is
 * restored to phi0 and the trajectory counts as rejected. */
int hmc_trajectory(hmc_ctx* ctx, double* phi_inout, const double* pi0, const void* eta,
                   int n_pf, double u_uniform, hmc_traj_stats* stats, void* stream);

/* The molecular-dynamics part of a trajectory alone (Eq. 29): n_leap kick-drift-kick steps
 * of size eps on (phi_inout, pi_inout) in place, with the pseudofermions chi (n_pf
 * complex128 spinors, e.g. from hmc_heatbath) held fixed.  No heat-bath and no Metropolis
 * decision; stats receives the energies at both ends (S_pf0 from the solve at the start,
 * S_pf1 from the last one), dH and solver counts.  Leapfrog is reversible: running it again
 * from (phi_out, -pi_out) returns (phi_in, -pi_in) up to rounding and solver tolerance.
 * Synchronises the stream.  Errors: as hmc_cg_solve (phi and pi are then undefined). */
int hmc_leapfrog(hmc_ctx* ctx, double* phi_inout, double* pi_inout, const void* chi, int n_pf,
                 hmc_traj_stats* stats, void* stream);

/* Fourier-diagonal HMC metric ("Scale-invariant sampling": Eq. 30 and the momentum draw
 * and kinetic energy stated with it).  The metric of Eq. (28) is G = Sigma^{-1} with
 * Sigma = F diag(sigma) F^*, F the unitary DFT over (tau, x, y) of each component of a
 * boson-shaped field; sigma is a device array double[3][L_tau][L][L] indexed by frequency
 * (component l, n_tau, k_x, k_y in natural order), positive and finite.  A real field's
 * estimate (Eq. 30) is even in k; the operators use the even part of any table.
 *
 * hmc_set_metric keeps the pointer (NULL: the identity metric, the default): the caller keeps
 * the array alive and unchanged while trajectories or the calls below run.  With a metric set,
 * hmc_trajectory and hmc_leapfrog drift by dphi/dt = Sigma pi and report the kinetic energy
 * 1/2 pi^T Sigma pi; their pi0 should then come from hmc_metric_momenta.  One-lattice contexts
 * only; L and L_tau need prime factors <= 7 and an L x L FP64 slice must fit the LDS (L <= 100
 * on gfx950).  Errors: HMC_ERR_INVALID_ARG. */
int hmc_set_metric(hmc_ctx* ctx, const double* sigma);

/* The metric operations on boson-shaped fields (device double[3][L_tau][L][L], 16-byte
 * aligned), with the metric set on the context (sigma = 1 if none).  They use the FP64 CG
 * scratch vector of the workspace, so they may not overlap a solve on another stream.
 *   momenta:    pi = F(sigma^{-1/2} . F^* xi), for a real standard normal field xi: then
 *               pi ~ N(0, G) (xi and pi may alias);
 *   kinetic:    *K = 1/2 pi^T Sigma pi = 1/2 sum_k sigma(k) |(F pi)(k)|^2 (host double);
 *   norm2:      *out = v^T G v = sum_k |(F v)(k)|^2 / sigma(k), the squared jump distance of
 *               Eq. (32) for v = phi' - phi (host double);
 *   accumulate: acc(k) += |(F phi)(k)|^2, one sample's term of the estimate of Eq. (30);
 *               acc has sigma's layout (divide by the number of samples afterwards).
 * kinetic and norm2 synchronise the stream.  Errors: HMC_ERR_INVALID_ARG, HMC_ERR_WORKSPACE,
 * HMC_ERR_HIP. */
int hmc_metric_momenta(hmc_ctx* ctx, const double* xi, double* pi, void* stream);
int hmc_metric_kinetic(hmc_ctx* ctx, const double* pi, double* K, void* stream);
int hmc_metric_norm2(hmc_ctx* ctx, const double* v, double* out, void* stream);
int hmc_metric_accumulate(hmc_ctx* ctx, const double* phi, double* acc, void* stream);

/* Bosonic observables ("Estimation of observables", Eq. 33-34; Supplementary Note 1).
 *   hmc_sdw_accumulate: chi_acc(n, kx, ky) += dtau sum_l |(F phi_l)(n, kx, ky)|^2, F the unitary
 *     space-time DFT: one sample's term of the SDW susceptibility of Eq. (34) (divide by the
 *     number of samples afterwards).  chi_acc: device double[L_tau][L][L] indexed by frequency.
 *     Needs the lattices the metric supports (factors <= 7, L <= 100); uses the FP64 CG
 *     residual of the workspace as scratch.
 *   hmc_order_parameter: Phi[l] = sum over all sites of phi_l (host double[3]); synchronises.
 *   hmc_binder: B = 1 - 3 <|Phi|^4> / (5 <|Phi|^2>^2) over S samples Phi[S][3] (host arrays;
 *     NaN for S < 1 or a NULL array).  0 for an isotropic Gaussian Phi, 2/5 at fixed |Phi|.
 * Errors: HMC_ERR_INVALID_ARG, HMC_ERR_WORKSPACE, HMC_ERR_HIP. */
int hmc_sdw_accumulate(hmc_ctx* ctx, const double* phi, double* chi_acc, void* stream);
int hmc_order_parameter(hmc_ctx* ctx, const double* phi, double* Phi, void* stream);
double hmc_binder(const double* Phi, int S);

/* Warm-up tuning of the step size and trajectory length ("Online HMC hyperparameter
 * tuning": Eq. 31 and Eq. 32).  Host state, owned by the caller; plain arithmetic, no GPU.
 *
 * Step size (Eq. 31, read from the explanation beside it: one step of eps is worth two of
 * eps/2 per solve while alpha(eps/2)^2 <= 2 alpha(eps); violated when alpha(eps) = 0):
 * hmc_tuner_add_step takes the energy errors dH of two single-step proposals (n_leap = 1) at
 * eps and eps/2, adds alpha = min(1, exp(-dH)) of each to the window sums, and once `window`
 * pairs are in, multiplies eps by `factor` if the rule holds for the window means and divides
 * it otherwise, then restarts the window.
 * Length (Eq. 32): hmc_tuner_add_jump adds ||phi' - phi||_G^2 alpha of a proposal of length
 * n to that length's sums; hmc_tuner_best_length returns the n <= n_cap with the largest mean
 * (the smallest on ties; 0 before any sample).  hmc_jitter(u, n_max) = 1 + min(floor(u n_max),
 * n_max - 1), a length uniform on {1, ..., n_max} for u uniform on [0, 1) (0 if n_max < 1 or
 * u is outside [0, 1)).
 * Errors: HMC_ERR_INVALID_ARG (eps <= 0, window < 1, factor <= 1, n_cap outside
 * [1, HMC_TUNER_MAX_LEN], n outside [1, n_cap], non-finite inputs). */
#define HMC_TUNER_MAX_LEN 256
typedef struct hmc_tuner {
    double eps;             /* step size of the next warm-up iteration                     */
    double factor;          /* multiplicative change of eps (> 1)                          */
    int    window;          /* single-step pairs per decision (>= 1)                       */
    int    n_cap;           /* warm-up trajectory lengths are drawn from {1, ..., n_cap}   */
    int    count;           /* pairs in the current window                                 */
    int    pad;
    double sum_alpha_eps;   /* window sums of alpha(eps) and alpha(eps/2)                  */
    double sum_alpha_half;
    double esjd_sum[HMC_TUNER_MAX_LEN + 1];   /* per length: sum of ||dphi||_G^2 alpha     */
    long   esjd_count[HMC_TUNER_MAX_LEN + 1]; /* per length: proposals                     */
} hmc_tuner;

int hmc_tuner_init(hmc_tuner* t, double eps, int window, double factor, int n_cap);
int hmc_tuner_add_step(hmc_tuner* t, double dH_eps, double dH_half);
int hmc_tuner_add_jump(hmc_tuner* t, int n, double sqdist, double dH);
int hmc_tuner_best_length(const hmc_tuner* t);
int hmc_jitter(double u, int n_max);

/* Result of one warm-up iteration (host struct). */
typedef struct hmc_warmup_stats {
    double eps;             /* step size used by the three proposals                       */
    double eps_next;        /* step size after the rule (t->eps on return)                  */
    double dH_eps;          /* energy error of the single step of eps                      */
    double dH_half;         /* ... and of eps/2                                             */
    double dH;              /* energy error of the jittered proposal                       */
    double sqdist;          /* ||phi' - phi||_G^2 of that proposal (G: the context's metric) */
    int    n_leap;          /* its length, hmc_jitter(u_length, t->n_cap)                   */
    int    accepted;        /* u_accept < exp(-dH)                                          */
    long   cg_iterations;   /* Krylov iterations of the three proposals                     */
    double max_true_resid;  /* largest final relative residual of their solves              */
} hmc_warmup_stats;

/* One warm-up iteration on a one-lattice context, in this order: momenta pi = F(sigma^{-1/2}
 * . F^* xi) under the context's metric (pi = xi without one); two single-step proposals from
 * (phi, pi) at t->eps and t->eps / 2, neither accepted, whose dH go to hmc_tuner_add_step
 * after the third; a proposal of n_leap = hmc_jitter(u_length, t->n_cap) steps of t->eps,
 * whose ||phi' - phi||_G^2 and dH go to hmc_tuner_add_jump; its Metropolis decision by
 * u_accept (phi_inout becomes phi' or stays).  Each proposal is a full trajectory as in
 * hmc_trajectory (heat-bath of the same eta, CG solves, energies); eps and n_leap of the
 * context's parameters are untouched.  xi: a real standard normal field, phi's layout.
 * Synchronises the stream.  Errors: as hmc_trajectory (phi_inout is then restored and the
 * tuner unchanged); HMC_ERR_INVALID_ARG for an invalid tuner. */
int hmc_warmup_iteration(hmc_ctx* ctx, hmc_tuner* t, double* phi_inout, const double* xi, const void* eta,
                         int n_pf, double u_accept, double u_length, hmc_warmup_stats* stats,
                         void* stream);

/* Sampled kernel timing, for measuring the solver kernels inside real work.  When
 * enabled, the CG driver times the middle iteration of every status chunk in which all
 * right-hand sides are iterating (start and stop timestamps taken by the two kernels'
 * own dispatches, hipExtLaunchKernel events, so nothing is inserted between kernels) and
 * adds the two kernel durations to the accumulators below.  Eager launches only (no
 * samples while CG chunks replay from graphs).  Enabling resets them.
 * Index: [0] CG step A (t = M p with the fused p update), FP32 Krylov precision;
 * [1] CG step B (r -= alpha M^dagger t), FP32; [2] step A, FP64; [3] step B, FP64.
 * With the Fourier preconditioner the three passes of z = P r in the same sampled
 * iteration: [4] forward slice FFT, [5] time-direction pass, [6] inverse slice FFT, FP32;
 * [7], [8], [9] the same in FP64.  [10], [11]: step A of the iteration after the sampled one,
 * FP32 and FP64 (step A updates the solution every second iteration, so [0] and [10] time
 * one launch of each kind). */
#define HMC_KT_SLOTS 12
typedef struct hmc_kernel_times {
    double ms[HMC_KT_SLOTS];     /* summed durations in milliseconds                      */
    long   count[HMC_KT_SLOTS];  /* number of sampled launches                            */
} hmc_kernel_times;

int hmc_set_kernel_timing(hmc_ctx* ctx, int enable);

/* Launch shape of the CG kernels for solves in `precision` (HMC_FP64, HMC_MIXED, or -1
 * for both): at most max_per_rhs workgroups per right-hand side (1..4096; defaults 1024
 * FP64, 512 mixed); workgroup b sweeps tiles b, b + count, ...  Results depend on it only
 * through the order of the FP64 partial sums.  hmc_get_cg_workgroups returns the count in
 * use for `precision` (the request capped at the number of tiles). */
int hmc_set_cg_workgroups(hmc_ctx* ctx, int precision, int max_per_rhs);
int hmc_get_cg_workgroups(const hmc_ctx* ctx, int precision);

/* Launch shape of the one-pass M^dagger M (hmc_apply_MdagM and hmc_apply_MdagM_f32 on the
 * nearest-neighbour operator): each workgroup owns a band of `rows` lattice rows of one vector
 * and marches through `slices` consecutive time slices, holding M in for its rows and the rows
 * beside them in LDS; with slices = 1 each workgroup takes one slice of its band and forms
 * M in at the previous slice itself.  0 selects the default (12 rows FP32, 6 rows FP64, one
 * slice; rows are capped so that the band's M in fits 64 KB of LDS).  precision: HMC_FP64,
 * HMC_MIXED or -1 for both.  Results do not depend on the shape.  hmc_get_mdm_shape reports the
 * shape an apply of n vectors uses: rows, slices and the workgroup count (host ints). */
int hmc_set_mdm_shape(hmc_ctx* ctx, int precision, int rows, int slices);
int hmc_get_mdm_shape(const hmc_ctx* ctx, int precision, int n, int* rows, int* slices, int* workgroups);

/* CG step A (the direction update, t = M p and the fused x update) as a march (one lattice;
 * with the production model's two-site hops the band carries two rows beside it on either side
 * instead of one): each workgroup owns a band of `rows` lattice rows of one
 * right-hand side and walks `slices` consecutive time slices, holding the new direction of two
 * consecutive slices in LDS and loading the next slice while it computes the current one, so
 * that every value of r (z), p, x and phi leaves HBM once.  rows = 0 switches back to the tile
 * kernels; slices = 0 picks about one workgroup per compute unit.  Default for one-lattice
 * contexts: 8 rows (FP32) / 4 rows (FP64), 8 slices, or the autotuner's choice.  precision:
 * HMC_FP64, HMC_MIXED or -1 for both.  The algebra is that of the tile kernels; only the order
 * of the FP64 partial sums differs.  One-lattice contexts only (HMC_ERR_INVALID_ARG on a
 * batch: hmc_batch_set_cg_march); lattices whose band does not fit (rows + 2 rows, or rows + 4
 * with the two-site hops, of one thread per element in FP64 or per pair in FP32, at most 512
 * threads) keep the tile kernels.  The FP64 setting also cuts the reliable update's FP64
 * stencils into marches (nearest-neighbour operator). */
int hmc_set_cg_march(hmc_ctx* ctx, int precision, int rows, int slices);
/* The setting in use for `precision` (host ints; rows 0: the tile kernels). */
int hmc_get_cg_march(const hmc_ctx* ctx, int precision, int* rows, int* slices);

/* Whether CG step B (r -= alpha M^dagger t, Methods C) also marches when step A does, with
 * step A's cut (enable != 0), or runs its tile kernel (0).  The march reads t once through LDS
 * (helps where the tile kernel re-reads t from HBM or L2: FP64, several right-hand sides, the
 * two-site hops); with one FP32 right-hand side of the nearest-neighbour model the two are
 * within a few percent (the tile kernel reads t while the MALL still holds it).  Default: on in
 * both precisions; hmc_autotune times both.  precision: HMC_FP64, HMC_MIXED or -1.  Results
 * depend on it only through the order of the FP64 partial sums.  hmc_get_cg_march_step_b
 * returns the setting (-1 on a bad argument). */
int hmc_set_cg_march_step_b(hmc_ctx* ctx, int precision, int enable);
int hmc_get_cg_march_step_b(const hmc_ctx* ctx, int precision);

/* Result of hmc_autotune (host struct).  Index [0] FP64, [1] mixed precision. */
#define HMC_TUNE_MAX 12
#define HMC_TUNE_MARCH_MAX 16
typedef struct hmc_tune_result {
    int    cg_workgroups[2];   /* chosen workgroups per right-hand side                       */
    double us_per_iter[2];     /* measured time per CG iteration at the choice (microseconds) */
    int    candidates;         /* launch shapes timed, both precisions                         */
    int    tried[2];           /* workgroup counts timed per precision (<= HMC_TUNE_MAX)       */
    int    tried_workgroups[2][HMC_TUNE_MAX];  /* each count timed ...                         */
    double tried_us[2][HMC_TUNE_MAX];          /* ... and its time per CG iteration (us)       */
    int    march_rows[2];      /* chosen step-A march (hmc_set_cg_march): rows, 0 = tile kernels */
    int    march_slices[2];    /* ... and slices per segment                                   */
    int    mtried[2];          /* march shapes timed per precision (<= HMC_TUNE_MARCH_MAX)     */
    int    mtried_rows[2][HMC_TUNE_MARCH_MAX];
    int    mtried_slices[2][HMC_TUNE_MARCH_MAX];
    double mtried_us[2][HMC_TUNE_MARCH_MAX];
    int    from_cache;         /* 1: the shapes came from the on-disk cache, nothing was timed */
    int    march_step_b[2];    /* 1: step B marches with step A's cut; 0: its tile kernel      */
    double step_b_us[2][2];    /* us per iteration with step B's tile kernel [0] and march [1] at
                                  the chosen cut (0: not timed)                                */
} hmc_tune_result;

/* Autotuner of the CG launch shape.  For each precision, times 100 CG iterations on the
 * caller's phi and right-hand sides b (n complex128 spinors, n <= max_rhs) with HIP events on
 * the stream: first at each candidate workgroup count of the tile kernels (12 multiples of 8
 * from 128 to 4096, capped at the tile count), then, for a one-lattice nearest-neighbour
 * context, at each step-A march shape (rows per band x slices per segment, up to 16 that fit)
 * with the chosen count; keeps the fastest.  The choice is remembered process-wide for later
 * contexts of the same lattice, right-hand-side count and device, and written to an on-disk
 * cache keyed by (L, L_tau, right-hand sides, device, kernel-source hash): the file named by
 * the environment variable HMC_TUNE_CACHE, else $XDG_CACHE_HOME/hmc/tune.txt, else
 * $HOME/.cache/hmc/tune.txt (HMC_TUNE_CACHE=off disables it).  hmc_create applies a cached
 * choice; hmc_autotune with the variable HMC_TUNE_REUSE=1 returns a cached choice without
 * timing.  Uses the context's workspace (no other allocation); the run parameters are restored
 * afterwards.  Synchronises the stream.  Errors: as hmc_cg_solve. */
int hmc_autotune(hmc_ctx* ctx, const double* phi, const void* b, int n, hmc_tune_result* out,
                 void* stream);
int hmc_get_kernel_times(const hmc_ctx* ctx, hmc_kernel_times* out);

/* Replay the CG status chunks from HIP graphs (enable != 0) instead of launching each
 * kernel.  A chunk (reliable_every FP32 iterations plus the FP64 reliable update in mixed
 * precision, 32 iterations plus the residual check in FP64) is captured once per solve shape
 * (precision, pointers, right-hand sides, launch shape, coefficients) and relaunched on the
 * caller's stream; results are bitwise those of eager launches.  Capture uses a private
 * stream of the context.  Default: off for a single lattice, on for a batch. */
int hmc_set_graphs(hmc_ctx* ctx, int enable);

/* Replay each leapfrog step's drift and CG solve (Methods D, the update of phi by Eq. (29)
 * and the solve of Eq. (22) at the new phi), and a trajectory's first solve, from one
 * HIP graph (enable != 0): the drift, the solve's start and K status chunks, with K the most
 * iterations of any right-hand side in the previous solve plus a tenth and one chunk, rounded
 * up to an even count.  The host reads the CG records once after the graph and finishes a
 * solve that needs more chunks with ordinary launches; chunks past convergence do nothing.
 * Graphs are cached per shape (K, pointers, step size, launch shape, coefficients), at most 8.
 * The force and the kicks stay ordinary launches.  Results are bitwise those of eager
 * launches.  Applies with the identity metric (hmc_set_metric not in use); otherwise it is
 * ignored.  Default: off. */
int hmc_set_step_graphs(hmc_ctx* ctx, int enable);

/* -----------------------------------------------------------------------------------------
 * Batch of independent lattices.
 *
 * The study of the phase diagram (Results, "Numerical results"; Supplementary Note 1) and
 * the scaling studies (Supplementary Note 6) run many independent Markov chains at
 * different L, L_tau and boson mass r.  A batch advances nchains such lattices together:
 * every CG launch and every site kernel covers all of them, so small lattices still fill
 * the GPU, and each chain keeps its own convergence test, energies and Metropolis
 * decision.  All chains share dtau and every hmc_params field except r (per chain); each
 * chain carries params.n_pf right-hand sides.
 *
 * Layouts (device, caller-owned, 16-byte aligned): the per-chain arrays of the single-
 * lattice layout concatenated in chain order.
 *   phi, pi   : double, chain i at elements [phi_offsets[i], phi_offsets[i+1]),
 *               3 * L_tau_i * L_i^2 of them.
 *   spinors   : complex128 (FP64) or complex64 (HMC_MIXED in hmc_batch_apply), chain i at
 *               complex elements [spinor_offsets[i], spinor_offsets[i+1]) holding its n_pf
 *               right-hand sides one after another.
 * hmc_batch_layout() returns both offset tables.  A batch is not thread-safe; the library
 * allocates no device memory (workspace as for one lattice). */
typedef struct hmc_batch hmc_batch;

/* L, L_tau, r: host arrays of nchains entries.  Each lattice obeys the rules of hmc_create;
 * params->n_pf >= 1.  Errors: HMC_ERR_INVALID_ARG (geometry, parameters, or more than
 * 16384 chain-right-hand-side pairs, or 2^31 complex elements), HMC_ERR_HIP. */
int hmc_batch_create(int nchains, const int* L, const int* L_tau, const double* r, double dtau,
                     const hmc_params* params, hmc_batch** out);
int hmc_batch_destroy(hmc_batch* batch);
size_t hmc_batch_workspace_bytes(const hmc_batch* batch);
int hmc_batch_set_workspace(hmc_batch* batch, void* ptr, size_t bytes);

/* phi_offsets, spinor_offsets: host arrays of nchains + 1 entries (element and complex
 * offsets, see above; the last entry is the total). */
int hmc_batch_layout(const hmc_batch* batch, long long* phi_offsets, long long* spinor_offsets);

/* As hmc_set_cg_workgroups, per (chain, right-hand side); each is capped at the tile count
 * of its lattice.  hmc_batch_get_cg_workgroups returns the requested maximum. */
int hmc_batch_set_cg_workgroups(hmc_batch* batch, int precision, int max_per_unit);
int hmc_batch_get_cg_workgroups(const hmc_batch* batch, int precision);
int hmc_batch_set_graphs(hmc_batch* batch, int enable);
/* As hmc_set_step_graphs, for the batch's trajectories. */
int hmc_batch_set_step_graphs(hmc_batch* batch, int enable);

/* Step A of CG, and the FP64 stencils of its reliable update, as marches of row bands through
 * time slices (as hmc_set_cg_march), each lattice of the batch with its own cut: at most `rows`
 * rows per band (and at most what a 512-thread workgroup holds for the lattice's L: one element
 * per thread in FP64, two in FP32), `slices` slices per segment (0: 8; more when a lattice's
 * partial-sum slots require it).  The reliable update uses the FP64 setting.  rows = 0 selects
 * the tile kernels; so does a lattice that fits no cut (then for the whole batch) and the
 * production model's two-site hops.  Defaults: 4 rows FP64, 8 FP32, 8 slices; hmc_batch_autotune
 * searches them.  precision: HMC_FP64, HMC_MIXED or -1 for both.  Results depend on the cut only
 * through the order of the FP64 partial sums; a chain reproduces, bit for bit, a one-lattice
 * context given the same cut.  hmc_batch_get_cg_march reports the cut chain `chain` uses in
 * `precision` (0 rows: the tile kernels) and whether step B marches with it. */
int hmc_batch_set_cg_march(hmc_batch* batch, int precision, int rows, int slices);
int hmc_batch_get_cg_march(const hmc_batch* batch, int chain, int precision, int* rows, int* slices,
                           int* ru_rows, int* ru_slices, int* step_b);
/* As hmc_set_cg_march_step_b, for the batch. */
int hmc_batch_set_cg_march_step_b(hmc_batch* batch, int precision, int enable);

/* Replace the run parameters; n_pf must equal the value given at creation. */
int hmc_batch_set_params(hmc_batch* batch, const hmc_params* params);

/* out = M in (dagger = 0) or M^dagger in (dagger != 0), Eq. (17), for every right-hand side
 * of every chain.  precision HMC_FP64: phi double, in/out complex128; HMC_MIXED: phi float,
 * in/out complex64.  Asynchronous on the stream. */
int hmc_batch_apply(hmc_batch* batch, int dagger, int precision, const void* phi, const void* in,
                    void* out, void* stream);

/* Solve (M^dagger M) x = b for every right-hand side of every chain (Methods, "Solving the
 * linear system"; Eq. 22), each to params.cg_tol relative residual with its own stopping
 * test, in params.precision.  iterations (int) and true_resid (double, the FP64 relative
 * residual at exit) are optional host arrays of nchains * n_pf entries in chain-major order.
 * Synchronises the stream.  Errors: as hmc_cg_solve. */
int hmc_batch_cg_solve(hmc_batch* batch, const double* phi, const void* b, void* x,
                       int* iterations, double* true_resid, void* stream);

/* As hmc_autotune for the whole batch (the launch shape is shared by all chains); the
 * choice is kept by the batch only. */
int hmc_batch_autotune(hmc_batch* batch, const double* phi, const void* b, hmc_tune_result* out,
                       void* stream);

/* One HMC trajectory of every chain (Methods, "HMC"; Eq. 27-29): heat-bath chi = M^dagger eta
 * per chain, n_leap leapfrog steps of size eps on all chains at once, then a Metropolis
 * decision per chain with its own uniform u[i] (host array): chain i is accepted iff
 * u[i] < exp(-dH_i).  Rejected chains get phi back from the start of the trajectory.
 * dH (double) and accepted (int): host arrays of nchains entries.  totals: solver counts over
 * all chains and accepted = the number of accepted chains.  pi0 is not modified.
 * Synchronises the stream.  Errors: as hmc_trajectory; on an error every chain is rejected
 * and phi restored. */
int hmc_batch_trajectory(hmc_batch* batch, double* phi, const double* pi0, const void* eta,
                         const double* u, double* dH, int* accepted, hmc_traj_stats* totals,
                         void* stream);

/* -----------------------------------------------------------------------------------------
 * Streaming reference (a measurement aid; no step of the method).
 *
 * The stencil kernels are bound by HBM bandwidth, and the rate an MI355X sustains depends
 * on the mix of reads and writes.  hmc_stream_probe runs a plain grid-stride streaming
 * kernel (16-byte vectors, 256-thread workgroups, `grid` workgroups; 0 = 2048) over
 * `bytes` per stream (a positive multiple of 16), so that each kernel of the path can be
 * compared with the streaming rate of its own mix:
 *   HMC_PROBE_READ   reads src (bytes); writes one double per workgroup to dst (grid doubles);
 *   HMC_PROBE_WRITE  writes dst (bytes); src unused (may be NULL);
 *   HMC_PROBE_COPY   reads src, writes dst (bytes each);
 *   HMC_PROBE_3R3W   reads three streams (src: 3 * bytes) and writes three (dst: 3 * bytes),
 *                    the mix of one fused CG step;
 *   HMC_PROBE_READ_NT as HMC_PROBE_READ with nontemporal loads, eight in flight per thread.
 * Device pointers, 16-byte aligned, caller-owned; asynchronous on the stream.  Errors:
 * HMC_ERR_INVALID_ARG (kind, size, alignment, NULL, grid outside [1, 65536]), HMC_ERR_HIP. */
#define HMC_PROBE_READ  0
#define HMC_PROBE_WRITE 1
#define HMC_PROBE_COPY  2
#define HMC_PROBE_3R3W  3
#define HMC_PROBE_READ_NT 4
int hmc_stream_probe(int kind, const void* src, void* dst, size_t bytes, int grid, void* stream);

/* Text for an HMC_* code. */
const char* hmc_strerror(int code);

/* Message describing the last error raised on the calling thread ("" if none). */
const char* hmc_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* HMC_H */
