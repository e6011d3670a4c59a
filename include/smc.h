/*
 * smc.h — C ABI of the MI355X move stage of Gaussian-mixture sequential Monte Carlo
 * (arXiv 2503.16028, "Sequential Monte Carlo with Gaussian Mixture Approximation for
 * Infinite-Dimensional Statistical Inverse Problems").
 *
 * Conventions shared by every call
 *  - Array arguments are DEVICE pointers owned by the caller, unless marked "host".
 *    Arrays are row-major and particle-major: row n of an [N][K] array is particle n.
 *  - A particle is the vector xi of K whitened Karhunen-Loeve coefficients of the
 *    log-permeability u = sum_i sqrt(lambda_i) xi_i phi_i (prior mu_0 = N(0, C), Sec. 2.1;
 *    C_0 = (I - Delta)^{-2}, Sec. 3.2).  2D: K = kl*kl, index k*kl + l for
 *    phi_kl = c_k c_l cos(k pi x) cos(l pi y); 1D: K = kl, index k-1 for sqrt(2) sin(k pi x).
 *  - Every call is asynchronous on `stream` (a hipStream_t; NULL = the default stream),
 *    validates all arguments on the host before launching anything, and returns an
 *    smc_status.  On SMC_E_INVAL nothing was launched and no output was touched.
 *    Errors reported by the HIP runtime surface as SMC_E_HIP at that call or a later one.
 *    smc_last_error() gives a text for the last non-OK status of the calling thread.
 *  - No call allocates device memory except smc_problem_create, which allocates all the
 *    workspace the other calls need for up to n_max particles.  Calls on one problem
 *    share that workspace: they must not run concurrently on different streams.
 *  - Failures found on the device (a solve that does not converge, a stalled temperature
 *    step, a non-finite potential) set bits in the problem's device status word, read by
 *    smc_status_flags(), and are also visible per particle in the outputs.
 */
#ifndef SMC_H
#define SMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SMC_OK = 0,
    SMC_E_INVAL = -1,     /* invalid argument: nothing launched */
    SMC_E_HIP = -2,       /* HIP runtime error */
    SMC_E_NOCONV = -3,    /* (flag) a forward solve did not converge */
    SMC_E_STALL = -4,     /* (flag) temperature bisection found no positive step */
    SMC_E_NONFINITE = -5, /* (flag) no particle had a finite potential */
    SMC_E_NOMEM = -6      /* workspace allocation failed */
} smc_status;

/* Bits of the device status word. */
#define SMC_FLAG_NOCONV 1
#define SMC_FLAG_STALL 2
#define SMC_FLAG_NONFINITE 4
#define SMC_FLAG_BADWEIGHTS 8
#define SMC_FLAG_BADLEVEL 16   /* a level map named a grid the problem does not have */
#define SMC_FLAG_BADPARAM 32   /* a device-side beta or tau was out of range (moves rejected) */

/* Level-map value that parks a particle: it is not solved and not moved (see smc_forward_batch
 * and smc_gmpcn_stage), and it sets no flag.  A sampler whose temperature has reached 1 parks
 * its particles while the samplers sharing its launch go on. */
#define SMC_LEVEL_PARKED (-1)

typedef enum {
    SMC_FP64 = 0,        /* conjugate gradients in FP64 */
    SMC_FP32_REFINE = 1  /* FP32 conjugate gradients inside FP64 residual refinement */
} smc_precision;

typedef void* smc_stream; /* hipStream_t */
typedef struct smc_problem_s* smc_problem;
typedef struct smc_graph_s* smc_graph;   /* an instantiated, replayable stage */

/* Problem definition (host memory; copied by smc_problem_create).
 * Forward map (Sec. 3.2, eq. (example2:PDE), gradient on the state):
 *   -div(e^u grad w) = f on (0,1)^dim, w = 0 on the boundary, discretised in flux form on a
 *   grid of n intervals per axis (h = 1/n, nodes i/n), face coefficient exp((u_P + u_Q)/2).
 * Observation F(u) = (w(x_1), ..., w(x_Nd)) at grid nodes; potential (Sec. 2.1)
 *   Phi = |F(u) - y|^2 / (2 sigma^2). */
typedef struct {
    int32_t dim;            /* 1 or 2 */
    int32_t n_levels;       /* number of grids, 1..3 (several grids: mixed-resolution runs) */
    int32_t grid_n[3];      /* intervals per axis of each grid: powers of two, 2D 16..256, 1D 8..1024 */
    int32_t kl;             /* KL modes per axis: 2D kl*kl cosine modes, kl <= 32; 1D kl <= 64 */
    int32_t kr;             /* modes the mixture moves (the kr largest eigenvalues), 1..64, <= K */
    int32_t n_obs;          /* 1..64 observations */
    int32_t obs_den;        /* observation coordinates are obs_num / obs_den */
    const int32_t* obs_num; /* host [n_obs][dim]; each point must be a node of every grid */
    const double* y;        /* host [n_obs] data */
    double sigma;           /* noise standard deviation, > 0 */
    double f;               /* constant source term */
    int64_t n_max;          /* largest particle count any call will pass */
    double tol64;           /* stop when ||f - A w||_2 <= tol64 ||f||_2 with the FP64 operator */
    double tol_inner;       /* FP32 inner solves reduce their residual by this factor */
    int32_t max_iter;       /* cap on conjugate-gradient iterations per solve (all sweeps) */
    int32_t max_sweeps;     /* cap on FP64 refinement sweeps per solve */
    int32_t precond;        /* SMC_PRECOND_AUTO or SMC_PRECOND_JACOBI */
} smc_problem_desc;

/* Problem without a PDE: the paper's Example 1 (Sec. 3.1), a mixture likelihood in L^2(0, 1).
 * Prior N(0, (I - alpha Delta)^{-2}) with the Neumann cosine eigenpairs phi_0 = 1,
 * phi_k = sqrt(2) cos(k pi x), lambda_k = (1 + alpha k^2 pi^2)^{-2}, k = 0 .. K-1, so
 * u = sum_k sqrt(lambda_k) xi_k phi_k; likelihood (eq. (example1phi))
 *   exp(-Phi(u)) = sum_i exp(-|u - f_i|^2 / (2 sigma^2)),
 * each f_i given by its coefficients c[i][k] = <f_i, phi_k> (f_i in the span of the K modes),
 * so Phi(xi) = -log sum_i exp(-sum_k (sqrt(lambda_k) xi_k - c_ik)^2 / (2 sigma^2)).
 * The active modes are 0 .. kr-1 (lambda decreases with k).  Such a problem supports the
 * prior draw, smc_phi_batch, the pCN-GM moves and stages, smc_gm_fit, smc_gm_draw, tempering
 * and resampling; calls that need a grid (synthesis, forward maps, gradients, tiles, level
 * maps) return SMC_E_INVAL. */
typedef struct {
    int32_t K;          /* modes, 1..1024 */
    int32_t kr;         /* modes the mixture moves, 1..min(64, K) */
    double alpha;       /* prior operator I - alpha Delta, alpha > 0 (0.01 in the paper) */
    int32_t n_terms;    /* likelihood terms, 1..16 */
    const double* c;    /* host [n_terms][K] coefficients of the centres, finite */
    double sigma;       /* > 0 */
    int64_t n_max;      /* largest particle count any call will pass, 1..2^24 */
} smc_l2mix_desc;

/* Preconditioner of the conjugate gradients.  AUTO: the fast-Poisson (sine-transform)
 * preconditioner on the matrix cores for FP32 solves on 32^2, 64^2 and 128^2 grids, Jacobi
 * scaling elsewhere; JACOBI: Jacobi scaling everywhere. */
#define SMC_PRECOND_AUTO 0
#define SMC_PRECOND_JACOBI 1

/* Mixture {w_j, m_j, C_j} of Sec. 2.3 (C_j shares the prior's eigenfunctions), in whitened
 * coordinates over the kr active modes; all device pointers.
 *   logw[M]        log mixture weights (normalised)
 *   mean[M][kr]    whitened means  m~_ji = <m_j, phi_i> / sqrt(lambda_i)
 *   scale[M][kr]   variance ratios s_ji = lambda_ji / lambda_i  (> 0)
 * Outside the active modes every component has mean 0 and scale 1. */
typedef struct {
    int32_t M;            /* 1..16 */
    int32_t kr;           /* must equal the problem's kr */
    const double* logw;
    const double* mean;
    const double* scale;
} smc_gm;

/* Create a problem: copies the definition, tabulates the prior and the grids on the device,
 * allocates all workspace for n_max particles.  *out is set only on SMC_OK. */
int smc_problem_create(const smc_problem_desc* desc, smc_problem* out);
/* Create a problem of the L^2 mixture kind (smc_l2mix_desc); *out is set only on SMC_OK. */
int smc_problem_create_l2mix(const smc_l2mix_desc* desc, smc_problem* out);
/* Free a problem and its workspace (waits for the device).  NULL is ignored. */
void smc_problem_destroy(smc_problem p);
/* Text of the last non-OK status returned on the calling thread. */
const char* smc_last_error(void);
/* The 53-bit integer (w0 >> 5) 2^26 + (w1 >> 6) of the Philox4x32-10 words w of counter
 * (block, word, ctr lo, ctr hi) under key (seed lo, seed hi): the kernels' generator, computed on
 * the host for draws a caller passes in (the resampling uniform u53 of smc_resample; the drivers
 * use block 0x80000001, word 0, counter stage * 2^20).  Pure host arithmetic. */
uint64_t smc_philox_u53(uint64_t seed, uint64_t ctr, uint32_t block, uint32_t word);
/* K, the active mode list (host out [kr]) and the observation count; any pointer may be NULL. */
int smc_problem_info(smc_problem p, int32_t* K, int32_t* active, int32_t* n_obs);
/* Synchronise `stream`, return the device status word in *flags (host) and clear it if
 * `clear` is nonzero. */
int smc_status_flags(smc_problem p, smc_stream stream, int32_t* flags, int32_t clear);

/* Initial draw of Alg. 1: xi[N][K] ~ N(0, I) from Philox4x32-10 (Salmon et al., SC'11) with
 * key = (seed lo, seed hi), counter = (i/2, particle, ctr lo, ctr hi) and Box-Muller. */
int smc_prior_sample(smc_problem p, int64_t N, uint64_t seed, uint64_t ctr, double* xi,
                     smc_stream stream);

/* Nodal field u = sum_i sqrt(lambda_i) xi_i phi_i on grid `level`: u[N][n+1][n+1]
 * (2D, index [j][i] for the node (i/n, j/n)) or u[N][n+1] (1D). */
int smc_synthesize(smc_problem p, int64_t N, const double* xi, int32_t level, double* u,
                   smc_stream stream);

/* Forward map G = F(u(xi)) for N particles (one PDE solve each, Sec. 3.2).
 *   level  [N] device, grid index per particle, or NULL for grid 0.  With a level map the
 *          particles are grouped by grid on the device and each grid is solved by a launch in
 *          the shape of its single-grid launch, with the same results (2D, grids of 64, 128 and
 *          256 intervals; with the Jacobi-only preconditioner one persistent launch serves all);
 *          a particle whose level is out of range gets G = NaN, iters = -1 and sets
 *          SMC_FLAG_BADLEVEL; level SMC_LEVEL_PARKED gives the same outputs without a solve
 *          and without the flag
 *   prec   smc_precision (1D problems always solve directly in FP64)
 *   G      [N][n_obs] out; NaN rows for solves that did not converge
 *   iters  [N] out, conjugate-gradient iterations, -1 when not converged; may be NULL */
int smc_forward_batch(smc_problem p, int64_t N, const double* xi, const int32_t* level,
                      int32_t prec, double* G, int32_t* iters, smc_stream stream);

/* Potential of each particle for either problem kind: the forward map and Phi = |G - y|^2 /
 * (2 sigma^2) (one solve each; level and prec as in smc_forward_batch), or the closed form of
 * an L^2 mixture problem (level must be NULL there; prec is ignored).
 *   xi [N][K] in, phi [N] out (+inf where a solve does not converge), iters [N] out or NULL. */
int smc_phi_batch(smc_problem p, int64_t N, const double* xi, const int32_t* level, int32_t prec,
                  double* phi, int32_t* iters, smc_stream stream);

/* Potential Phi = |G - y|^2 / (2 sigma^2) (Sec. 2.1): phi[N] out, +inf for non-finite rows. */
int smc_potential(smc_problem p, int64_t N, const double* G, double* phi, smc_stream stream);

/* n_moves steps of the pCN-GM kernel (Sec. 2.3, Alg. 2) targeting exp(-tau Phi) mu_0:
 *   proposal  v = gamma xi + (1 - gamma) m_j + beta sqrt(s_j) z on the active modes and
 *             v = gamma xi + beta z elsewhere, gamma = sqrt(1 - beta^2), component
 *             j = min{j : w_1 + ... + w_j > U_comp}, z ~ N(0, I);
 *   acceptance a = min{1, rho(dv) Q(v, dxi) / (rho(dxi) Q(xi, dv))} (eqs. (auv of pCN-GMM)),
 *             accept iff log U_acc < log a.
 * Move m draws from counter ctr + m: normals as in smc_prior_sample, (U_comp, U_acc) from
 * block 0x80000000.  M = 1 with zero mean and unit scale is plain pCN.
 *   xi [N][K], phi [N] in/out (phi must be the potential of xi); n_acc [N] out (accept count).
 * A proposal whose solve does not converge gets Phi = +inf and is rejected. */
int smc_gmpcn_move(smc_problem p, int64_t N, const smc_gm* gm, double beta, double tau,
                   int32_t n_moves, uint64_t seed, uint64_t ctr, const int32_t* level,
                   int32_t prec, double* xi, double* phi, int32_t* n_acc, smc_stream stream);

/* The proposal of smc_gmpcn_move's move 0 by itself (a parity hook): v[N][K] out, drawn as there
 * from counter ctr, and logr[N] out, the log of rho_0(v) Q(v, xi) / (rho_0(xi) Q(xi, v)) with
 * rho_0 the prior density and Q the pCN-GM proposal (eqs. (auv of pCN-GMM)-(auv of pCN-GMM4)
 * without the potential), which the move adds to tau (Phi(xi) - Phi(v)).  v must not alias xi. */
int smc_gmpcn_propose(smc_problem p, int64_t N, const smc_gm* gm, double beta, uint64_t seed, uint64_t ctr,
                      const double* xi, double* v, double* logr, smc_stream stream);

/* Parameters of a move stage for several independent samplers at once, all in device memory
 * so that a captured stage can be replayed after they change.  Group g (the particles with
 * level[n] == g, or every particle without a level map) has its own mixture, beta and tau:
 *   logw [G][M], mean [G][M][kr], scale [G][M][kr] (pad unused components with logw = -inf),
 *   beta [G], tau [G], ctr [1] (move m draws from counter *ctr + m), all device pointers. */
typedef struct {
    int32_t n_groups; /* the problem's n_levels with a level map, else 1 */
    int32_t M, kr;
    const double* logw;
    const double* mean;
    const double* scale;
    const double* beta;
    const double* tau;
    const uint64_t* ctr;
    uint64_t seed;
} smc_stage;

/* n_moves pCN-GM steps as smc_gmpcn_move, with each particle's beta, tau and mixture taken
 * from its group in `st`, read on the device when the kernels run.  Particles of a group with
 * beta outside (0, 1] or tau outside [0, 1] keep their state and set SMC_FLAG_BADPARAM.
 * Particles whose level is SMC_LEVEL_PARKED (read when the kernels run, so a captured stage
 * follows changes to the map) keep xi and phi, get n_acc = 0 and cost no solve. */
int smc_gmpcn_stage(smc_problem p, int64_t N, const int32_t* level, const smc_stage* st, int32_t n_moves,
                    int32_t prec, double* xi, double* phi, int32_t* n_acc, smc_stream stream);

/* Capture smc_gmpcn_stage with these exact arguments (pointers and sizes) on `stream` (a created
 * stream, not the null stream) into an instantiated HIP graph; nothing runs until it is launched.
 * Each smc_stage_graph_launch replays the whole stage on `stream`: every kernel of every move
 * in one submission, with the device-side parameters as they are at that time.  The graph
 * uses the problem's workspace: replays and other calls on the same problem must not overlap. */
int smc_stage_graph_create(smc_problem p, int64_t N, const int32_t* level, const smc_stage* st,
                           int32_t n_moves, int32_t prec, double* xi, double* phi, int32_t* n_acc,
                           smc_stream stream, smc_graph* out);
int smc_stage_graph_launch(smc_graph g, smc_stream stream);
void smc_stage_graph_destroy(smc_graph g);

/* A whole tempering stage of G independent samplers captured into one graph (Alg. 1 with the
 * pCN-GM mutation of Alg. 2): for every group g, the tempering step (App. C), systematic
 * resampling, the gather of the selected rows, and (M > 1) the mixture fit; then n_moves
 * pCN-GM moves of all groups (as smc_gmpcn_stage); then a rule on the device that records the
 * stage, adapts each group's step size and parks a group that has reached temperature 1.
 * Every per-stage value lives in device memory, so each smc_stage_graph_launch runs the next
 * stage with no host work between launches; the caller reads tau after a launch to decide whether
 * to launch again (with a level map, a stage launched after every group has reached 1 changes no
 * row; without one, its moves still run, at temperature 1).
 * Group g owns the rows [off_g, off_g + counts[g]), off_g = counts[0] + ... + counts[g-1]; with
 * a level map (G = the problem's n_levels, level[row] = g at the start) group g solves on grid g,
 * without one (G = 1) every row is group 0.  Random numbers: stage s (s = *ctr / stride) moves
 * with counter s stride + m, and group g resamples and seeds its fit with counter s stride + g,
 * as smc_philox_u53 and smc_gm_fit would with those counters: the graph gives the bits of the
 * same calls made one by one.
 * A group at temperature 1 still passes through tempering (uniform weights), resampling (then the
 * identity) and its fit, which leave its rows as they are; its moves are skipped once it is
 * parked, and it is recorded no more.  The rule, per running group: rate = accepted moves /
 * (rows * max(1, n_moves)); record[s-1][g][0..4] = tau, h, beta of the stage, rate, log-evidence
 * increment (rows past max_stages are not written); beta doubles (at most 1) above a rate of 0.3
 * and halves below 0.15; with a level map, a group with tau >= 1 sets its rows to
 * SMC_LEVEL_PARKED.  Then *ctr += stride.
 * All arrays are device arrays that stay valid while the graph exists; the graph reads and
 * writes them in place and uses the problem's workspace (launches must not overlap other calls
 * on the problem).  Errors: SMC_E_INVAL (nothing captured) for a NULL array other than level,
 * flags and (max_stages = 0) record, G out of range, a group outside 1..2^20 rows (the tempering
 * step's limit), more rows than n_max, M outside
 * 1..16, kr unlike the problem's, stride 0, xi2 or phi2 aliasing xi or phi, or a level map the
 * problem cannot mix; SMC_E_HIP if capture or instantiation fails. */
typedef struct {
    int32_t n_groups;                /* G: 1, or the problem's n_levels with a level map */
    int64_t counts[4];               /* host: rows of each group (the first G entries) */
    int32_t M, kr, fit_iters;        /* mixture components (M = 1: the given single component,
                                        no fit), active modes, EM steps of the fit */
    int32_t n_moves, max_stages;     /* moves per stage; rows of `record` */
    double ess_frac, var_floor;      /* ESS target fraction; variance floor of the fit */
    uint64_t seed, stride;           /* random stream; counter spacing of the stages */
    double* xi; double* phi;         /* [N][K], [N]: the particles and their potentials */
    double* xi2; double* phi2;       /* [N][K], [N]: gather scratch */
    double* W; int32_t* idx;         /* [N]: weights and resampling indices */
    double* tau; double* tau_new;    /* [G]: temperatures */
    double* h; double* log_z;        /* [G]: last step and log-evidence increment */
    double* beta;                    /* [G]: step sizes, adapted by the rule */
    double* logw; double* mean; double* scale;   /* [G][M], [G][M][kr], [G][M][kr] */
    uint64_t* ctr;                   /* [1]: s * stride during stage s (start it at stride) */
    int32_t* level;                  /* [N] level map, or NULL for G = 1 */
    int32_t* n_acc;                  /* [N]: accepted moves of the stage */
    double* record;                  /* [max_stages][G][5] */
    int32_t* flags;                  /* status word of tempering and resampling (may be NULL) */
} smc_sampler_graph_desc;

int smc_sampler_graph_create(smc_problem p, const smc_sampler_graph_desc* d, int32_t prec, smc_stream stream,
                             smc_graph* out);

/* Forward solve that keeps its FP64 solution (the forward state of the adjoint gradient), on
 * grid 0 of a 2D problem: as smc_forward_batch, and w[N][n][n] out with element [g][c] the
 * solution at the node ((c+1)/n, (g+1)/n); index n-1 is boundary padding and holds 0.  The
 * caller owns w; passing it to smc_value_and_grad later skips the forward solve there.
 * G may be NULL. */
int smc_forward_state(smc_problem p, int64_t N, const double* xi, int32_t prec, double* G, double* w,
                      int32_t* iters, smc_stream stream);

/* Potential and its gradient in whitened coordinates, g = dPhi/dxi, by one adjoint solve per
 * particle (the extra PDE solve that Sec. 2.4 counts for gradient-informed moves), 2D only:
 *   A(u) w = f,  A(u) lam = P^T (P w - y) / sigma^2  (A is symmetric),
 *   dPhi/du_P = -(1/2) sum over the faces (P,Q) at node P of a_PQ (lam_P - lam_Q)(w_P - w_Q) / h^2,
 *   g = sqrt(lambda) (B^T dPhi/du B)  (the transpose of the synthesis).
 *   w     [N][n][n] forward states from smc_forward_state for the same xi and grid, or NULL to
 *         solve the forward problems here (recomputation from the checkpoint xi)
 *   phi   [N] out (may be NULL); grad [N][K] out, NaN rows where a solve did not converge
 *   iters [N] out (may be NULL): total conjugate-gradient iterations, -1 if a solve failed.
 * Both solves run at precision prec to the problem's FP64 tolerance. */
int smc_value_and_grad(smc_problem p, int64_t N, const double* xi, int32_t prec, const double* w,
                       double* phi, double* grad, int32_t* iters, smc_stream stream);

/* n_moves pCN-Langevin steps (named in Sec. 2.4; the Crank-Nicolson step of App. B with the
 * tempered potential's drift explicit) targeting exp(-tau Phi) mu_0 on grid 0 of a 2D problem:
 *   v = gamma xi - (1 - gamma) tau g(xi) + beta z,  gamma = sqrt(1 - beta^2),  g = dPhi/dxi,
 *   accept iff log U_acc < min{0, log of the ratio of target times proposal densities}.
 * Each proposal costs a forward and an adjoint solve.  Random numbers as in smc_gmpcn_move.
 *   xi [N][K], phi [N], grad [N][K] in/out (phi and grad must belong to xi, e.g. from
 *   smc_value_and_grad); n_acc [N] out.  A proposal with a failed solve is rejected. */
int smc_pcnl_move(smc_problem p, int64_t N, double beta, double tau, int32_t n_moves, uint64_t seed,
                  uint64_t ctr, int32_t prec, double* xi, double* phi, double* grad, int32_t* n_acc,
                  smc_stream stream);

/* SMC-GM mutation (Alg. 3, Sec. 2.4): N independent draws from the mixture, each accepted, and
 * their potentials.  The draw is the pCN-GM proposal with beta = 1 (eq. (GMM beta=1)):
 *   v = m_j + sqrt(s_j) z on the active modes, v = z elsewhere, z ~ N(0, I),
 *   component j = min{j : w_1 + ... + w_j > U_comp},
 * with the normals and U_comp that a pCN-GM move of the same particle draws at counter ctr.
 *   xi  [N][K] out (the draws; no input state), phi [N] out (+inf where the solve does not
 *       converge), iters [N] out or NULL; level: grid of each particle or NULL (grid 0).
 * The caller owns every array; gm's arrays are read on the device during the call's kernels. */
int smc_gm_draw(smc_problem p, int64_t N, const smc_gm* gm, uint64_t seed, uint64_t ctr,
                const int32_t* level, int32_t prec, double* xi, double* phi, int32_t* iters,
                smc_stream stream);

/* Gaussian-mixture fit of a particle cloud on the device: the stage input of the pCN-GM move
 * (Sec. 2.3) and of SMC-GM (Sec. 2.4, Alg. 3).  The paper's estimator (its reference [Feng2018])
 * is not described there; this is EM with diagonal covariances on the problem's K_r active
 * whitened coordinates of xi[0..N):
 *   seeding  k-means++: centre 0 is row floor(u_0 N / 2^53); centre m >= 1 is row
 *            min{n : C_n > floor(u_m Q / 2^53)}, where C_n = sum_{i<=n} q_i, Q = C_{N-1},
 *            q_i = floor(d2_i 2^(40-e)), d2_i the squared distance of row i to its nearest
 *            centre (coordinates summed in pairwise order over 64 zero-padded slots),
 *            max_i d2_i = f 2^e with f in [1/2, 1); row floor(u_m N / 2^53) if Q = 0.  u_m is
 *            the 53-bit integer (w0 >> 5) 2^26 + (w1 >> 6) of Philox block 0x80000002,
 *            particle word m, counter ctr.  The choice is exact integer arithmetic.
 *   start    w_j = 1/M, m_j = the seeded rows, s_j = max(variance of the cloud, var_floor);
 *   EM       `iters` steps: responsibilities in log space, then w_j = N_j / N,
 *            m_j = sum R x / N_j, s_j = max(sum R x^2 / N_j - m_j^2, var_floor),
 *            N_j = sum_n R_nj + 1e-300; partial sums are added in a fixed order.
 *   out: logw [M] (normalised), mean [M][kr], scale [M][kr] (the variances s_j, the smc_gm
 *   scale), centers [M] (the seeded rows; may be NULL).  1 <= N <= min(n_max, 2^24),
 *   1 <= M <= 16, 0 <= iters <= 100000, var_floor > 0.  Calls on one problem share its
 *   workspace: do not run two on different streams at once. */
int smc_gm_fit(smc_problem p, int64_t N, const double* xi, int32_t M, int32_t iters, double var_floor,
               uint64_t seed, uint64_t ctr, double* logw, double* mean, double* scale, int32_t* centers,
               smc_stream stream);

/* The fit of smc_gm_fit without a problem handle and without allocating device memory, for
 * callers that cannot allocate (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Its workspace is a fixed array in the library's device image (about 8.8 MB,
 * held by each device the library runs on until the process ends), so
 *   1 <= N <= smc_gm_fit_noalloc_max() (32768); larger N returns SMC_E_INVAL.
 *   active [kr] device int32: the coordinates of xi[N][K] to fit (the problem's active modes in
 *          smc_gm_fit), each in 0..K-1; 1 <= kr <= min(64, K), K <= 1024.
 * Other arguments, outputs and results as smc_gm_fit (the same kernels: bit-identical results for
 * the same inputs).  Every call on a device shares that device's array, which keeps the last
 * call's contents (nothing in it must start at zero): calls that overlap on one device, on any
 * streams, race and give wrong results. */
int smc_gm_fit_noalloc(int64_t N, int32_t K, int32_t kr, const int32_t* active, const double* xi, int32_t M,
                       int32_t iters, double var_floor, uint64_t seed, uint64_t ctr, double* logw, double* mean,
                       double* scale, int32_t* centers, smc_stream stream);
int64_t smc_gm_fit_noalloc_max(void);

/* Re-weighting and next temperature (Alg. 1; App. C): with tau = *tau_in (device scalar),
 * choose h in (0, 1 - tau] with ESS(h) = ess_frac * N, where ESS = 1 / sum W^2 and
 * W_n ∝ exp(-h Phi_n): the largest h (to a relative 2^-52, or (1 - tau) 2^-64) whose ESS still
 * passes, found by safeguarded Newton steps on log ESS; take h = 1 - tau when that already passes.
 * Outputs (device): *h, *tau_new (= 1 exactly on the last stage), W[N] normalised weights,
 * *log_z_inc = log((1/N) sum exp(-h Phi)).  Non-finite Phi get weight 0.  A zero step while
 * tau < 1 sets SMC_FLAG_STALL (at tau = 1 the step is 0 and *tau_new = 1 without a flag), and
 * no finite potential sets SMC_FLAG_NONFINITE in *flags (device, may be NULL), which is or-ed,
 * never cleared.  N <= 1048576. */
int smc_temper(int64_t N, const double* phi, const double* tau_in, double ess_frac, double* h,
               double* tau_new, double* W, double* log_z_inc, int32_t* flags, smc_stream stream);

/* Systematic resampling (Alg. 1, resampling step) on an exact integer CDF:
 *   q_n = floor(W_n 2^53), C_n = q_0 + ... + q_n, Q = C_{N-1},
 *   idx_i = min{n : C_n > floor((i 2^53 + u53) Q / (N 2^53))},  i = 0..N-1.
 * u53 in [0, 2^53) is the uniform times 2^53.  idx[N] out (nondecreasing).
 * W must be normalised, as smc_temper writes it: every W_n finite and in [0, 1], and
 * sum W <= 1 + 2N 2^-53 (rounding of an FP64 normalisation), so that Q <= 2^53 + 2N.  Weights
 * that break this (a W_n > 1, negative or NaN, or a total above that bound), and all-zero
 * weights, set SMC_FLAG_BADWEIGHTS in *flags (device, may be NULL) and give idx = 0..N-1.
 * 1 <= N <= 2^24. */
int smc_resample(int64_t N, const double* W, uint64_t u53, int32_t* idx, int32_t* flags,
                 smc_stream stream);

/* Row gather after resampling: xi_out[i] = xi_in[idx[i]], phi_out[i] = phi_in[idx[i]]
 * (phi pointers may be NULL).  Outputs must not alias inputs. */
int smc_gather(int64_t N, int32_t K, const int32_t* idx, const double* xi_in,
               const double* phi_in, double* xi_out, double* phi_out, smc_stream stream);

/* The fast-Poisson preconditioner of the forward solves by itself (for tests): for each of N
 * grids, z = L^{-1} r with L the constant-coefficient Dirichlet Laplacian of grid `level`, up
 * to a positive constant factor, computed with sine transforms on the matrix cores in FP16 (the
 * input scaled by a power of two from its norm, the result scaled back).
 * r, z: [N][n][n] FP32, element [g][c] for the node ((c+1)/n, (g+1)/n); index n-1 is boundary
 * padding and must hold 0 in r.  Grids of 32, 64, 128 and 256 intervals. */
int smc_precond_apply(smc_problem p, int32_t level, int64_t N, const float* r, float* z, smc_stream stream);

/* Tile shape of the fast-Poisson solver of a grid (FP32+refinement, single-grid calls): grid rows
 * per thread, so that one particle's workgroup has n*n/rows threads.  Different shapes give the
 * same solution up to rounding (the reduction order changes).
 *   smc_tile_candidates  the shapes the library has for grid n (rows[8] out, *count out);
 *                        the first is the default; grid 256 has the single entry 0
 *   smc_set_tile         choose one for grid `level` (0 = default); smc_get_tile reads it back.
 *                        The forward-and-adjoint solve (smc_value_and_grad, smc_pcnl_move) at
 *                        128^2 runs as two launches of the 32-row shape by default, and as one
 *                        launch of both passes with 16 rows set here
 *   smc_autotune         time every candidate on N synthetic prior particles (drawn by the
 *                        library into its own workspace), reps timed launches each after one
 *                        warm-up, keep the fastest; *rows out, ms[count] out (may be NULL): mean
 *                        milliseconds per forward launch (synthesis and solve) of each candidate.
 *                        Synchronises `stream`; overwrites the problem's workspace, so no other
 *                        call on p may be in flight. */
int smc_tile_candidates(int32_t n, int32_t* rows, int32_t* count);
/* Launch structure of a move stage (smc_gmpcn_move, smc_gmpcn_stage and their graphs) without a
 * level map, at SMC_FP32_REFINE on a 2D grid solved on chip with the fast-Poisson preconditioner
 * (128^2 at 32 or 16 rows per thread, 64^2 at 8): enabled, the whole stage is one persistent
 * launch in which each workgroup runs every move of a particle (proposal, synthesis, solve,
 * decision) before taking the next; disabled (the default: measured faster, since the solve fills a
 * compute unit and the fused launch then runs the synthesis one particle per compute unit too),
 * each move is one launch per step.  Both give the same bits. */
int smc_set_stage_fusion(smc_problem p, int32_t enable);
int smc_set_tile(smc_problem p, int32_t level, int32_t rows);
int smc_get_tile(smc_problem p, int32_t level, int32_t* rows);
int smc_autotune(smc_problem p, int32_t level, int64_t N, int32_t reps, smc_stream stream, int32_t* rows,
                 double* ms);

/* Solver timing.  smc_profile(p, 1) clears and starts: every forward-solve launch made by
 * smc_forward_batch, smc_forward_state, smc_value_and_grad, smc_gmpcn_move and smc_pcnl_move on p
 * is then bracketed by two HIP events recorded on
 * the call's stream, and the solve kernels add their conjugate-gradient iterations, FP64
 * residual sweeps, solve count and fast-Poisson preconditioner applications to device
 * counters.  smc_profile(p, 0) stops.  smc_profile_read synchronises `stream` and returns the
 * summed kernel time (ms), the number of timed launches and those totals (host outputs, any
 * may be NULL). */
int smc_profile(smc_problem p, int32_t enable);
int smc_profile_read(smc_problem p, smc_stream stream, double* ms, int64_t* launches, int64_t* iters,
                     int64_t* sweeps, int64_t* solves, int64_t* precond_apps);

#ifdef __cplusplus
}
#endif
#endif /* SMC_H */
