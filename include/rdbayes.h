/*
 * rdbayes — batched Bayesian parameter identification for the Schnakenberg
 * (activator-depleted) reaction-diffusion system on MI355X (gfx950).
 *
 * Method: Campillo-Funollet, Venkataraman, Madzvamuse, "A Bayesian approach
 * to parameter identification with an application to Turing systems"
 * (arXiv:1605.04718).
 *
 * The library evaluates, for thousands of parameter vectors at once, the
 * observation operator G (Sec. 2: parameters -> model solution at the
 * measured time), the log-likelihood Phi = -log rho(y - G(p)) of eq. (logl)
 * for Gaussian noise, and Metropolis-Hastings steps (Sec. 2, Algorithm 1)
 * of independent chains, all in HIP kernels on one GPU.
 *
 * The forward model is eq. (schnakenberg) with the kinetics of
 * eq. (reactions), on the unit square mapped from a uniformly growing domain
 * rho(t) = exp(r t) (r = 0: stationary), discretised as in Sec. 3.1.1: a
 * cell-centred n x n grid (h = 1/n) with the 5-point Laplacian and mirror
 * (zero-flux) ghosts, and the IMEX backward-Euler step with one Picard
 * linearisation
 *   [1/dt + 2 r + g (1 - u^n v^n)] u^{n+1} - rho_n^-2 Lap_h u^{n+1} = u^n/dt + g a
 *   [1/dt + 2 r + g (u^n)^2]       v^{n+1} - d rho_n^-2 Lap_h v^{n+1} = v^n/dt + g b
 * (g = gamma; both systems solved by unpreconditioned conjugate gradients,
 * stopping when ||r||_2 <= cg_rtol ||rhs||_2 on the recursive residual).
 *
 * Conventions for every entry point:
 *  - Return value: RD_OK (0) or a negative call error (RD_E*).  A call
 *    error is reported synchronously before any work is enqueued; the text
 *    is available from rd_last_error() (thread-local).
 *  - Numerical failures are not call errors: they are reported per item in
 *    `status` as RD_ST_* bit flags, and a failed solve has Phi = +inf, so a
 *    proposal that needs it is rejected (the "robust" likelihood of Sec. 2).
 *  - "dev" arrays are device pointers on the current HIP device, owned by
 *    the caller, and must stay valid until the stream has finished the call.
 *    "host" arrays are read during the call only.
 *  - Batch calls only enqueue work on `stream` (a hipStream_t, NULL = the
 *    null stream) and never synchronise; results are valid once the caller
 *    has synchronised that stream.  A problem handle may be used from one
 *    stream at a time (its workspace is shared by its calls).
 *  - Parameter vectors are float64 [n][4]: natural theta = (a, b, gamma, d),
 *    sampling coordinates phi = (a, b, ln gamma, ln d).
 *  - Fields are row-major [n_cells_y][n_cells_x] with x fastest.
 */
#ifndef RDBAYES_H
#define RDBAYES_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum {
    RD_OK = 0,
    RD_EINVAL = -1,       /* bad argument, shape or size */
    RD_EHIP = -2,         /* a HIP runtime call failed */
    RD_ENOMEM = -3,       /* device allocation failed */
    RD_EUNSUPPORTED = -4, /* valid request this build does not implement */
    RD_ETIMEOUT = -5,     /* rd_check_solves: a cooperative group wait gave up */
    RD_EIO = -6           /* rd_chains_save / rd_chains_load: file error */
};

/* Per-item status bits. */
enum {
    RD_ST_NOT_CONVERGED = 1, /* CG reached cg_maxit */
    RD_ST_BREAKDOWN = 2,     /* p.Ap <= 0: the implicit operator lost definiteness */
    RD_ST_NONFINITE = 4,     /* NaN/Inf in a field or reduction */
    RD_ST_OUT_OF_PRIOR = 8,  /* proposal outside the prior box: not solved */
    RD_ST_BAD_GRID = 16,     /* grid_id outside [0, n_grids): not solved */
    RD_ST_NOT_STEADY = 32,   /* steady-state stopping: n_steps reached first */
    RD_ST_GROUP_TIMEOUT = 64 /* 256 x 256 cooperative solve: a workgroup of the
                                item's group gave up waiting for the others (a
                                scheduling failure, not a numerical one); the
                                item is not solved and rd_check_solves reports
                                RD_ETIMEOUT */
};

enum { RD_PRECISION_FP32 = 0, RD_PRECISION_FP64 = 1 };
enum { RD_MODE_PLAIN = 0, RD_MODE_DA = 1 };
enum { RD_MAX_GRIDS = 8 };

typedef struct rd_problem rd_problem; /* opaque; owned by the library */

/* One grid class: a grid size, a growth law and its data set. */
typedef struct {
    int32_t n;            /* cells per side; 32, 64, 128 or 256 */
    int32_t growth;       /* 0: rho = 1; 1: rho(t) = exp(growth_rate t) */
    double growth_rate;   /* r of rho = exp(r t); dilution term 2 r (m = 2) */
    const double *u0;     /* host [n*n] initial u (fixed for every proposal) */
    const double *v0;     /* host [n*n] initial v */
    const double *y;      /* host [n*n] observed u at T = dt * n_steps, or NULL
                             (then likelihood calls on this class fail RD_EINVAL) */
    double sigma;         /* standard deviation of the Gaussian noise of y */
} rd_grid_desc;

/* Problem description (copied by init_problem). */
typedef struct {
    int32_t n_grids;               /* 1 .. RD_MAX_GRIDS */
    const rd_grid_desc *grids;     /* host [n_grids] */
    double dt;                     /* time step tau */
    int32_t n_steps;               /* T = dt * n_steps */
    double cg_rtol;                /* CG stop: ||r|| <= cg_rtol ||rhs|| */
    int32_t cg_maxit;              /* CG iteration cap per solve (<= 0: 10 n^2) */
    int32_t precision;             /* RD_PRECISION_FP32: fields (as hi + lo) and CG
                                      vectors in FP32, the CG step lengths in
                                      FP32 from FP64 dot products, Phi in FP64.
                                      RD_PRECISION_FP64: everything FP64 */
    uint32_t free_mask;            /* bit i set: sampling coordinate i moves */
    double lo[4], hi[4];           /* uniform prior box in sampling coordinates */
    double step[4];                /* random-walk proposal s.d. per coordinate */
    int32_t max_batch;             /* largest n / n_chains any call will pass */
    double prop_chol[16];          /* optional lower-triangular proposal factor L
                                      (row-major [4][4]): when any entry is
                                      nonzero the random walk is
                                      phi'_i = phi_i + sum_{j<=i} L[i][j] z_j on
                                      the free coordinates (a correlated Gaussian
                                      step, still symmetric) and step[] is not
                                      used; all zero: phi'_i = phi_i + step_i z_i */
    /* Prior (Sec. 3.1.2, Cases 1-4).  prior_kind[i] = RD_PRIOR_UNIFORM:
     * uniform on [lo[i], hi[i]] (Case 1; zero-initialised descriptors get
     * this); RD_PRIOR_NORMAL: N(prior_mean[i], prior_sd[i]^2) in sampling
     * coordinate i without a bound, i.e. log-normal in gamma or d (Case 3).
     * turing_support = 1: the support is also restricted to the Turing
     * space of eq. (turing) at (a, b, d = exp(phi_3)) (Case 2).  The
     * acceptance ratio gains pi(proposal) / pi(state) (plain steps and the
     * first delayed-acceptance stage; it cancels from the second); a
     * proposal outside the support is rejected without a solve. */
    int32_t prior_kind[4];
    double prior_mean[4];
    double prior_sd[4];            /* > 0 where prior_kind is RD_PRIOR_NORMAL */
    int32_t turing_support;
    /* Steady-state stopping (Sec. 3.1.2): steady_tol > 0 ends each solve
     * after the first step whose discrete time derivative of (u, v) has an
     * L2 norm over the unit square below steady_tol,
     * sqrt(h^2 sum (du^2 + dv^2)) / dt with h = 1/n; n_steps is then a cap
     * (reaching it sets RD_ST_NOT_STEADY, Phi = +inf).  0: fixed horizon. */
    double steady_tol;
} rd_problem_desc;

enum { RD_PRIOR_UNIFORM = 0, RD_PRIOR_NORMAL = 1 };

/* Creates a problem: validates the description, uploads the initial fields
 * and data, sizes the workspace for max_batch items and picks the solver
 * tile shape for each grid class (autotuned once per device and grid class,
 * see rd_autotune).  Synchronous.  Errors: RD_EINVAL, RD_EHIP, RD_ENOMEM,
 * RD_EUNSUPPORTED (grid size without a kernel, FP64 at n = 256 resident). */
int32_t init_problem(const rd_problem_desc *desc, rd_problem **out);

/* Releases the workspace (synchronises the device first).  NULL is a no-op. */
int32_t destroy_problem(rd_problem *p);

/* forward_solve_batch plus steps_out (dev int32 [n]): the IMEX steps each
 * item took (its stopping step with steady-state stopping, else n_steps). */
int32_t forward_solve_steady_batch(rd_problem *p, int32_t n, const double *theta,
                                   const int32_t *grid_id, void *u_out, void *v_out,
                                   int32_t *status, int32_t *cg_iters, int32_t *steps_out,
                                   void *stream);

/* G(theta) for n parameter vectors (Sec. 2 observation operator): integrate
 * each from the initial fields of its grid class to T.
 *   theta    dev float64 [n][4] natural parameters (a, b, gamma, d)
 *   grid_id  dev int32 [n] grid class of each item, or NULL (class 0).
 *            With several classes the batch runs as one persistent launch
 *            over all classes, largest grids first; an id outside
 *            [0, n_grids) marks the item RD_ST_BAD_GRID (not solved).
 *   u_out    dev [n][M*M] final u (float32 for FP32 problems, float64 for
 *            FP64 problems), M = the largest grid size of the problem; item
 *            c of size N occupies the first N*N values of row c (row-major,
 *            x fastest).  NULL: not written.
 *   v_out    same layout for v, or NULL
 *   status   dev int32 [n] RD_ST_* bits (0 = success), required
 *   cg_iters dev int32 [n][2] total CG iterations of the u and v systems,
 *            or NULL
 * n = 0 is a no-op (array arguments may then be NULL).
 * Errors: RD_EINVAL (n < 0 or n > max_batch, NULL status). */
int32_t forward_solve_batch(rd_problem *p, int32_t n, const double *theta,
                            const int32_t *grid_id, void *u_out, void *v_out,
                            int32_t *status, int32_t *cg_iters, void *stream);

/* Phi(theta; y) = |y - G(theta)|^2 / (2 sigma^2) for each item, eq. (logl)
 * with Gaussian noise (the additive constant is dropped; only differences
 * enter Algorithm 1).  The solve and the misfit run fused in one kernel; the
 * misfit is accumulated in float64.  A failed solve gives phi = +inf.
 *   phi dev float64 [n]; status dev int32 [n]; cg_iters dev int32 [n][2] or NULL */
int32_t log_likelihood_batch(rd_problem *p, int32_t n, const double *theta,
                             const int32_t *grid_id, double *phi, int32_t *status,
                             int32_t *cg_iters, void *stream);

/* log_likelihood_batch without allocation, for callers that cannot
 * allocate device memory at call time (code under HIP graph capture, tight
 * serving loops, harnesses that forbid it).  Same results as
 * log_likelihood_batch with grid_id = NULL (the same kernels; items are
 * independent, so the launch shape does not change any result), but the
 * solve's scratch (queue head and one workspace slot per workgroup) lives
 * in a file-scope device array of the library, 256 B + 96 MiB, one copy per
 * device, held until the process ends, instead of the problem's workspace.
 * The call allocates nothing (no hipMalloc, events or library routines that
 * allocate) and enqueues a fill kernel and the solve kernel on `stream`.
 * The launch uses at most as many workgroups as slots fit in the 96 MiB
 * (256 at 128 x 128 FP32, 64 at 128 x 128 FP64), so it is never wider than
 * the scratch; larger batches are served by the persistent queue.
 * Every call on a device shares that device's array: calls that overlap on
 * one device (other streams, other problems, other threads) race and must
 * be serialised by the caller.  One grid class only; the cooperative
 * 256 x 256 FP32 tile is not served (select a streamed tile).
 * Errors: RD_EINVAL (n outside [0, max_batch], NULL theta/phi/status, no
 * data y), RD_EUNSUPPORTED (several grid classes, cooperative tile, a slot
 * larger than the scratch), RD_EHIP. */
int32_t log_likelihood_batch_noalloc(rd_problem *p, int32_t n, const double *theta, double *phi,
                                     int32_t *status, int32_t *cg_iters, void *stream);

/* Misfit of caller-supplied u fields against the data of their grid class
 * (the misfit kernel alone).  u dev [n][N*N] in the problem's precision. */
int32_t field_misfit_batch(rd_problem *p, int32_t n, const void *u, const int32_t *grid_id,
                           double *phi, void *stream);

/* State of a batch of independent Metropolis chains; all arrays are
 * caller-owned device arrays with n_chains rows. */
typedef struct {
    int32_t n_chains;
    double *phi;           /* dev [n][4] current state, sampling coordinates */
    double *loglik;        /* dev [n] Phi at the current state (+inf allowed) */
    double *loglik_sur;    /* dev [n] surrogate Phi~ at the current state
                              (RD_MODE_DA only, else may be NULL) */
    const int32_t *grid_id;/* dev [n] grid class per chain, or NULL (class 0) */
    uint64_t *n_accept;    /* dev [n] accepted proposals */
    uint64_t *n_accept1;   /* dev [n] first-stage accepts (DA), or NULL */
    uint64_t *n_solves;    /* dev [n] forward solves performed */
    uint64_t *cg_iters;    /* dev [n][2] CG iterations (u, v) summed over those
                              solves, or NULL */
    double *trace;         /* dev [trace_rows][n][4] states after each step, or NULL:
                              the step with index s writes row s - trace_step0
                              (rows outside [0, trace_rows) are not written) */
    uint32_t seed;         /* Philox key word 1 (key word 0 = chain index) */
    uint64_t step;         /* index of the next step; advanced by the calls */
    uint64_t trace_step0;  /* step index of trace row 0 */
    int32_t trace_rows;    /* rows the trace holds */
    uint64_t *imex_steps;  /* dev [n] IMEX steps completed, summed over the chain's
                              solves (a solve that fails at step s counts s), or NULL */
    uint64_t *fail_bits;   /* dev [n][8] solves whose status has bit k set
                              (RD_ST_* = 1 << k), or NULL */
} rd_chains;

/* n_steps Metropolis-Hastings steps (Sec. 2, Algorithm 1) of every chain.
 * Proposal: phi' = phi + step .* z on the free coordinates, z ~ N(0, I) by
 * Box-Muller from Philox4x32-10 (key = (chain, seed), counter = (step lo,
 * step hi, purpose 0, block)).  A proposal outside the prior box is rejected
 * without a solve (status RD_ST_OUT_OF_PRIOR is not reported: it is a
 * rejection).  Otherwise Phi(phi') is computed by the fused solve + misfit
 * and the proposal is accepted iff log U < Phi(phi) - Phi(phi'), U in (0,1)
 * from purpose 1.
 * mode RD_MODE_DA: delayed acceptance (Christen and Fox 2005): first stage
 * on the surrogate (requires surrogate_create + surrogate data), uniform from
 * purpose 2; only first-stage accepts are solved; the second stage accepts
 * iff log U < [Phi(phi) - Phi(phi')] - [Phi~(phi) - Phi~(phi')].
 * On a created stream the steps are replayed from one captured HIP graph per
 * chains layout, mode and stream: the layout's first step runs as direct
 * launches, the next one (in the same call or a later one) is captured and
 * every later step replays it; on the null stream, and while
 * rd_solver_timing is on, steps are launched directly.
 * chains->step is advanced by n_steps on return (host field).  The trace
 * keeps one row per step across calls (row = step - trace_step0).
 * Errors: RD_EINVAL (shapes, NULL required arrays), RD_EUNSUPPORTED (DA
 * without a surrogate). */
int32_t mcmc_step_batch(rd_problem *p, rd_chains *chains, int32_t n_steps, int32_t mode,
                        void *stream);

/* Checkpoint and resume of chains (Sec. 2: chains are long, and a run that
 * stops can continue).  The state of a chain is its present point, Phi (and
 * Phi~ under delayed acceptance) there, its counters, and the host fields
 * seed and step; the random numbers of step s depend only on (chain, seed,
 * s), so a chain loaded from a file continues exactly as the saved one
 * would have.  The trace is output, not state, and is neither saved nor
 * restored (trace_step0 and trace_rows are left as they are).
 * rd_chains_save copies every non-NULL array of *chains to the host on
 * `stream`, waits for it and writes `path`: a 48-byte header (magic
 * "RDCHAINS", version 1, n_chains, seed, a mask of the arrays present,
 * step) followed by those arrays in the order phi, loglik, loglik_sur,
 * grid_id, n_accept, n_accept1, n_solves, cg_iters, imex_steps, fail_bits,
 * n_chains rows each, host byte order.
 * rd_chains_load reads such a file into *chains (same n_chains): every
 * non-NULL array of *chains except grid_id must be in the file and is
 * overwritten; arrays the file has and *chains does not are skipped;
 * grid_id, an input, is compared with the file's and never written; seed
 * and step are set from the file.  Synchronous on `stream`; the surrogate
 * and the problem are not part of the file (resume DA chains with the same
 * surrogate).  Errors: RD_EINVAL (NULL or inconsistent arguments, not a
 * chain file, other n_chains, a missing array, another grid_id), RD_EIO
 * (open, short read or write), RD_EHIP. */
int32_t rd_chains_save(const rd_chains *chains, const char *path, void *stream);
int32_t rd_chains_load(rd_chains *chains, const char *path, void *stream);

/* The two halves of one plain step, for samplers on an external Phi (the
 * non-intrusive use of Sec. 2, and toy targets in tests):
 * propose_batch writes phi_prop dev float64 [n][4] and inside dev int32 [n]
 * (1 = in the prior box) for step chains->step; accept_batch then takes
 * Phi(phi_prop) from the caller (dev float64 [n], ignored where inside = 0),
 * applies the accept test of that same step, updates the chains and
 * advances chains->step by one. */
int32_t propose_batch(rd_problem *p, rd_chains *chains, double *phi_prop, int32_t *inside,
                      void *stream);
int32_t accept_batch(rd_problem *p, rd_chains *chains, const double *phi_prop,
                     const int32_t *inside, const double *loglik_prop, void *stream);

/* ---- parallel Metropolis-Hastings (Sec. 2, Algorithm 2) -----------------
 * One step of a chain evaluates Phi at N proposals at once and produces N
 * states: the stationary distribution of the (N+1)-state transition matrix
 * A(i, j) = min(1, r(x_i, x_j)) / N over the proposals and the present
 * state, r(x, y) = exp(Phi(x) - Phi(y)) pi0(y) / pi0(x), gives the
 * probabilities of N draws.  As printed the proposals are drawn around the
 * present state; here they are drawn around an auxiliary point z ~ k(x, .)
 * (Calderhead's construction, which the algorithm cites), for which A leaves
 * the posterior invariant with this symmetric random-walk kernel.  Random
 * numbers: purpose 6 (z), 7 (proposal j: blocks 2j, 2j+1), 8 (draw n:
 * block n).  The N draws fill trace rows chains->step .. chains->step + N - 1,
 * the last draw is the next present state, chains->step advances by N,
 * n_accept counts draws other than the present state and n_solves the
 * proposals solved.  1 <= n_prop <= 256 and n_chains * n_prop <= max_batch.
 *
 * pmh_step_batch: n_iter steps with Phi from this library's fused solve
 * (n_chains * n_prop items per launch).  pmh_propose_batch and
 * pmh_resample_batch: the two halves around an external Phi; proposals are
 * dev float64 [n_chains * n_prop][4] (item c * n_prop + j), inside and
 * loglik_prop dev [n_chains * n_prop]; pmh_resample_batch advances
 * chains->step by n_prop.  Errors: RD_EINVAL. */
int32_t pmh_step_batch(rd_problem *p, rd_chains *chains, int32_t n_prop, int32_t n_iter,
                       void *stream);
int32_t pmh_propose_batch(rd_problem *p, rd_chains *chains, int32_t n_prop, double *phi_prop,
                          int32_t *inside, void *stream);
int32_t pmh_resample_batch(rd_problem *p, rd_chains *chains, int32_t n_prop,
                           const double *phi_prop, const int32_t *inside,
                           const double *loglik_prop, void *stream);

/* ---- surrogate (first stage of delayed acceptance) ----------------------
 * An MLP 4 -> width x depth (GELU) -> (n/ds)^2 maps the sampling coordinates
 * (scaled to [-1, 1] on the prior box) to the block-mean-downsampled u field
 * (per-pixel standardised).  Trained and evaluated by BF16 MFMA kernels with
 * FP32 accumulation and FP32 master weights. */

/* Creates (or re-creates) the surrogate of grid class 0 with PyTorch-default
 * uniform(+-1/sqrt(fan_in)) initialisation from `seed`; out_side = the side of
 * the downsampled field (32); width 512, depth 4 in the reference setup.
 * Errors: RD_EINVAL (sizes), RD_ENOMEM. */
int32_t surrogate_create(rd_problem *p, int32_t width, int32_t depth, int32_t out_side,
                         uint32_t seed);

/* Block means of u fields: dev [n][N*N] (problem precision) -> dev float32
 * [n][out_side^2] (non-overlapping (N/out_side)^2 blocks). */
int32_t downsample_batch(rd_problem *p, int32_t n, const void *u, float *out, void *stream);

/* Sets the per-pixel standardisation (dev float32 [out^2] mean and sd) and the
 * first-stage data: ybar = block means of y (computed by the library), and the
 * first-stage noise s.d. sigma1 (per pixel). */
int32_t surrogate_set_scaling(rd_problem *p, const float *mean, const float *sd,
                              double sigma1, void *stream);

/* Box (host double [4] lo < hi, sampling coordinates) over which the
 * network's inputs are mapped to [-1, 1]; the prior box by default.  A
 * surrogate trained near the posterior uses a box around it, so that the
 * small differences between nearby parameters survive the FP32/BF16 input
 * path.  Set it before training.  Errors: RD_EINVAL. */
int32_t surrogate_set_input_box(rd_problem *p, const double *lo, const double *hi);

/* One Adam step (lr, beta1 0.9, beta2 0.999, eps 1e-8) on a batch:
 *   phi dev float64 [batch][4] sampling coordinates
 *   target dev float32 [batch][out^2] standardised downsampled fields
 *   loss_out dev float64 [1] mean squared error of the batch (before the
 *   step), or NULL.  batch <= 4096. */
int32_t surrogate_train_step(rd_problem *p, int32_t batch, const double *phi, const float *target,
                             double lr, double *loss_out, void *stream);

/* Surrogate prediction: dev float64 [n][4] -> dev float32 [n][out^2]
 * (standardised space if raw = 1, else de-standardised u block means). */
int32_t surrogate_forward(rd_problem *p, int32_t n, const double *phi, float *out, int32_t raw,
                          void *stream);

/* Surrogate misfit Phi~ = |ybar - u~|^2 / (2 sigma1^2) per item: dev [n]. */
int32_t surrogate_loglik_batch(rd_problem *p, int32_t n, const double *phi, double *phi_sur,
                               void *stream);

/* Layer `layer` (0 = input layer) of the surrogate: dir = 0 copies the FP32
 * master weights [out][in] (row-major) and biases [out] to caller memory
 * (dev float32), dir = 1 copies them in (and refreshes the BF16 copy),
 * dir = 2 copies out the weight and bias gradients of the last
 * surrogate_train_step. */
int32_t surrogate_params(rd_problem *p, int32_t layer, float *w, float *b, int32_t dir,
                         void *stream);

/* ---- utilities ----------------------------------------------------------- */

/* Re-runs the tile-shape autotuner for every grid class of p (a few timed
 * trial solves) and keeps the fastest; returns the chosen cells-per-thread
 * of each class in cpt_out (host int32 [n_grids], may be NULL).  With
 * several grid classes it also times the mixed-class launch at 512 and 1024
 * threads per workgroup and keeps the faster (see rd_mixed_threads).  The
 * choice is cached per device, grid size and precision for later problems. */
int32_t rd_autotune(rd_problem *p, int32_t *cpt_out);

/* Selects the tile of grid class `grid` by its cells per thread (the value
 * rd_autotune reports), overriding the default and any cached choice for
 * this problem only.  Supported values depend on the grid size and
 * precision; at 256 x 256 in FP32, cpt = 16 selects the cooperative tile
 * (four workgroups share an item, each holding a 64-row strip resident).
 * Errors: RD_EINVAL (NULL problem, grid out of range), RD_EUNSUPPORTED (no
 * kernel for that cpt at this size and precision). */
int32_t rd_set_tile(rd_problem *p, int32_t grid, int32_t cpt);

/* Sets the workgroup size (512 or 1024) of the launch that serves batches
 * mixing grid classes, overriding the default and any cached choice for
 * this problem only.  With 1024 and 256 x 256 FP32 classes, one launch
 * serves all classes (the 256 x 256 items by groups of four workgroups);
 * with 512 a cooperative launch for those items precedes the mixed launch.
 * Errors: RD_EINVAL (NULL problem, other sizes). */
int32_t rd_set_mixed_threads(rd_problem *p, int32_t threads);

/* First stage of delayed acceptance (mcmc_step_batch with RD_MODE_DA):
 * `substeps` Metropolis steps on the surrogate posterior prior x exp(-Phi~)
 * from the present state x instead of one screened proposal.  Substep j
 * proposes z' = z + step .* dz (or z + L dz) from the substep state z and
 * accepts iff log U_j < [Phi~(z) - Phi~(z')] + [log pi(z') - log pi(z)];
 * the end point y goes to the full solve and the second stage (accept iff
 * log U < [Phi(x) - Phi(y)] - [Phi~(x) - Phi~(y)]) when some substep moved,
 * else the step stays at x without a solve.  The surrogate's kernel is
 * reversible for the surrogate posterior, so the step leaves the posterior
 * invariant (delayed acceptance of Christen and Fox 2005 with the surrogate
 * transition as the proposal).  Random numbers: substep 0 uses purposes 0
 * and 2 (so substeps = 1 is the one-proposal step), substep j >= 1
 * purpose 9 (blocks 2j, 2j + 1) and 10 (block j).  n_accept1 counts the
 * steps whose proposal reached the second stage.  1 <= substeps <= 256
 * (default 1).  Errors: RD_EINVAL. */
int32_t rd_set_da_substeps(rd_problem *p, int32_t substeps);

/* Number of Metropolis steps held as captured HIP graphs (one per chains
 * layout, mode and stream; host int32 out).  Every setting that changes
 * what a step launches (tile, mixed workgroup size, surrogate, substeps,
 * group-wait hook) drops them, so the next step is captured anew.
 * Errors: RD_EINVAL. */
int32_t rd_captured_graphs(const rd_problem *p, int32_t *count);

/* Workgroup size of the launch that serves batches mixing grid classes
 * (host int32 out).  Errors: RD_EINVAL (NULL argument). */
int32_t rd_mixed_threads(const rd_problem *p, int32_t *threads);

/* Accumulated device time (ms, measured with HIP events on the launch
 * stream) and launch count of the fused solve kernel since the last reset;
 * reset = 1 clears after reading.  Timing is recorded only while enabled. */
int32_t rd_solver_timing(rd_problem *p, int32_t enable, double *ms_total, int64_t *launches,
                         int32_t reset);

/* Synchronises the device and reports whether any cooperative workgroup
 * (the 256 x 256 FP32 tile, alone or inside a mixed batch) gave up a bounded
 * group wait since the problem was created or last reset.  Such a wait ends
 * after 10 s only when a member of the group can never arrive (not while
 * every member is resident, which the launch guarantees); its items carry
 * RD_ST_GROUP_TIMEOUT.  Batch calls never synchronise, so this is where the
 * condition becomes a call error.
 *   group_timeouts host int64 out (may be NULL): members that gave up
 *   reset = 1 clears the count after reading.
 * Returns RD_OK, RD_ETIMEOUT (count > 0; rd_last_error has the count),
 * RD_EINVAL or RD_EHIP. */
int32_t rd_check_solves(rd_problem *p, int64_t *group_timeouts, int32_t reset);

/* Test hook for the failure path above: the bound of a cooperative group
 * wait in 100 MHz real-time-counter ticks (<= 0: the 10 s default), and a
 * delay (ticks, <= 1e8) that member 1 of every group sleeps before the
 * group's first exchange (0: none).  A delay well above the bound makes the
 * other members give up, so a test can drive the whole failure path from the
 * host while every kernel still runs to its end.  Applies to later batch
 * calls of this problem only.  Errors: RD_EINVAL. */
int32_t rd_set_coop_wait(rd_problem *p, int64_t wait_ticks, int64_t stall_ticks);

const char *rd_status_string(int32_t status_or_error);
const char *rd_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* RDBAYES_H */
