/*
 * xrdvi — C ABI of the MI355X (gfx950) hot path of variational Bayesian
 * crystalline-phase identification from X-ray diffraction.
 *
 * The model (paper, Appendix A): observed counts y_i at diffraction angles
 * x_i (2-theta, degrees) follow a Poisson law around the profile
 *     f(x_i) = B_i + sum_k h_k sum_m I_m^(k) V(x_i; p_m^(k) + mu_k, w_k, r_k)
 * with V the pseudo-Voigt (1-r) G + r L of a unit-area Gaussian G and a
 * unit-area Lorentzian L sharing full width at half maximum w.  Each
 * candidate phase k carries four latents phi_k = (h_k, mu_k, w_k, r_k):
 * weight, shift, width and Lorentz fraction.  Priors (Sec. 2.2 and
 * Appendix B.2): h ~ Exp(rate lambda), mu ~ N(0, mu_sd), w ~ Gamma(shape,
 * rate), r ~ U(0,1).  The posterior is approximated by a mean-field
 * Gaussian q (Sec. 3.2) over unconstrained z with h = exp(z_h), mu = z_mu,
 * w = exp(z_w), r = logistic(z_r); its parameters are loc (means) and
 * logscale (log standard deviations), each laid out [D][K] with rows
 * (h, mu, w, r), D = 4.
 *
 * Asymmetric peaks (Appendix A.2, asymmetry factor A(x; alpha), which is
 * alpha at and above the peak centre rho and 1 below it; prior
 * alpha ~ N(1, 0.2), Appendix B.2): a problem created with `asymmetric`
 * set gives each phase a fifth latent alpha = exp(z_alpha) (D = 5, row 4)
 * and evaluates
 *     V_alpha(x) = 2/(1 + alpha) * [(1-r) G + r L](x; rho, A w) * A
 * i.e. the pseudo-Voigt with full width w below rho and alpha w above,
 * scaled to unit area (continuous at rho; alpha = 1 gives V).  Every array
 * documented below as [..][D][K] then has five rows.
 *
 * Conventions for every call:
 *  - Return value: XRDVI_OK (0) or a negative error code; a message for the
 *    last error of the calling thread is available from xrdvi_last_error().
 *    No exception or abort crosses this interface.
 *  - "device" pointers are HIP device memory on the context's GPU; "host"
 *    pointers are ordinary memory.  The caller owns every pointer it passes
 *    and keeps device inputs valid until the work enqueued on `stream` has
 *    completed.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Calls only enqueue
 *    work on it and never synchronise unless stated.
 *  - Arguments checked on the host before any work is enqueued fail with
 *    XRDVI_EINVAL and leave outputs untouched.
 *  - A context, problem or tape may be used from one thread at a time.
 *  - A problem is used only while its context lives and a tape only while
 *    its problem lives; the *_destroy calls themselves may run in any order.
 */
#ifndef XRDVI_H
#define XRDVI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define XRDVI_API __attribute__((visibility("default")))

enum {
    XRDVI_OK = 0,
    XRDVI_PENDING = 1,
    XRDVI_EINVAL = -1,     /* invalid argument, detected on the host        */
    XRDVI_ENOMEM = -2,     /* device or host allocation failed / never fits */
    XRDVI_EDEVICE = -3,    /* a HIP runtime call failed                     */
    XRDVI_EBUSY = -4,      /* serving queue full                            */
    XRDVI_ENOENT = -5,     /* unknown ticket                                */
    XRDVI_ECANCELED = -6,  /* request cancelled                             */
    XRDVI_ENONFINITE = -7  /* an analysis produced a non-finite ELBO        */
};

typedef struct xrdvi_ctx xrdvi_ctx;
typedef struct xrdvi_problem xrdvi_problem;
typedef struct xrdvi_tape xrdvi_tape;
typedef struct xrdvi_server xrdvi_server;

/* Prior hyper-parameters (Sec. 2.2; Appendix B.2). */
typedef struct {
    double lambda_h;  /* rate of the exponential prior on h; 0 selects
                         1 / max_i(y_i - B_i), the paper's choice        */
    double mu_sd;     /* sd of the normal prior on the shift, 0.03 deg    */
    double w_shape;   /* gamma prior on the width: shape 3 ...            */
    double w_rate;    /* ... and rate 100 (mean 0.03 deg)                  */
    double alpha_mean;  /* normal prior on the asymmetry alpha: mean 1 ...  */
    double alpha_sd;    /* ... and sd 0.2 (used only with `asymmetric`)     */
} xrdvi_prior;

/*
 * One diffractogram and its candidate set (Appendix A.1).  HOST pointers;
 * the library copies and validates them at xrdvi_problem_create.
 *   x[N]        2-theta grid, finite, strictly ascending, inside (0, 180)
 *   y[N]        observed counts, finite, >= 0 (non-integers are accepted;
 *               ln y! is taken as lgamma(y + 1))
 *   bg[N]       background B_i, finite, > 0 (estimated beforehand)
 *   peak_off[K+1] CSR offsets of the ragged peak lists: peak_off[0] = 0,
 *               non-decreasing; phase k owns peaks peak_off[k]..peak_off[k+1]-1
 *   peak_pos[T] peak positions p_m (deg), finite; T = peak_off[K]
 *   peak_int[T] relative intensities I_m in [0, 1]
 *   cutoff      c >= 0: peak m of phase k contributes only at points with
 *               rho - c w <= x_i <= rho + c w (rho = p_m + mu_k, w = FWHM;
 *               the upper bound is rho + (c w) alpha for asymmetric peaks);
 *               c = 0 keeps every point (the paper's dense sum)
 *   asymmetric  0: symmetric peaks (D = 4); 1: asymmetric peaks (D = 5)
 *   width_law   0: every peak of phase k has full width w_k (the paper's
 *               pseudo-Voigt); 1: the width grows with the Bragg angle,
 *               W = w_k sec(rho / 2) = w_k / |cos(rho pi / 360)| (Appendix
 *               A.2 defines sec(x) = 1/cos(x) for the lost width formula),
 *               w_k being the width at 2-theta -> 0; W replaces w in the
 *               shape and in the window, rho - c W .. rho + (c W) alpha.
 *               Requires every peak_pos inside (0, 180).
 */
typedef struct {
    int32_t N, K;
    const double *x, *y, *bg;
    const int32_t *peak_off;
    const double *peak_pos, *peak_int;
    double cutoff;
    xrdvi_prior prior;
    int32_t asymmetric;
    int32_t width_law;
} xrdvi_problem_desc;

XRDVI_API const char *xrdvi_last_error(void);
XRDVI_API int xrdvi_version(void);

/* Host-only validation of a problem description (no GPU needed).  Returns
 * XRDVI_OK or XRDVI_EINVAL with a message. */
XRDVI_API int xrdvi_validate(const xrdvi_problem_desc *desc);

/* Context bound to one GPU (`device` index).  Owns a growable workspace for
 * xrdvi_profile and xrdvi_window_plan. */
XRDVI_API int xrdvi_ctx_create(int device, xrdvi_ctx **out);
XRDVI_API int xrdvi_ctx_destroy(xrdvi_ctx *ctx);

/* Validates `desc`, copies it to the device and lays it out for the kernels
 * (peaks ordered by position inside each phase, tile-relative coordinates,
 * ln y!).  Synchronous.  The problem must not outlive its context. */
XRDVI_API int xrdvi_problem_create(xrdvi_ctx *ctx,
                                   const xrdvi_problem_desc *desc,
                                   xrdvi_problem **out);
XRDVI_API int xrdvi_problem_destroy(xrdvi_problem *prob);
/* Sizes and the resolved prior rate lambda_h. Any output may be NULL. */
XRDVI_API int xrdvi_problem_info(const xrdvi_problem *prob, int32_t *N,
                                 int32_t *K, int32_t *total_peaks,
                                 double *lambda_h);

/* Latent types per phase of a problem: 4, or 5 for asymmetric peaks (D in
 * the array shapes below); negative (XRDVI_EINVAL) for NULL. */
XRDVI_API int xrdvi_problem_latents(const xrdvi_problem *prob);

/* Per-step device state for S samples of one problem: noise, samples,
 * window plan and the adjoint's per-tile partial sums (never the S x K x N
 * peak basis).  Holds the saved state between xrdvi_elbo_fwd and
 * xrdvi_elbo_bwd. */
XRDVI_API int xrdvi_tape_create(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                                int32_t S, xrdvi_tape **out);
XRDVI_API int xrdvi_tape_destroy(xrdvi_tape *tape);

/*
 * Profile f[s][i] = B_i + sum_k h_k C_k(x_i) (Appendix A.2, signal and
 * profile equations) at given constrained latents.
 *   phi    device double [S][D][K], rows (h, mu, w, r[, alpha]); requires
 *          h >= 0, w > 0, 0 <= r <= 1, alpha > 0 (other values give
 *          unspecified output)
 *   f_out  device float [S][N]
 * Peak values are evaluated in FP32 on tile-relative coordinates and summed
 * onto the FP64 background.  The first call at a larger S grows the
 * context workspace (allocation, synchronous).
 */
XRDVI_API int xrdvi_profile(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                            int32_t S, const double *phi, float *f_out,
                            void *stream);

/*
 * Allocation-free variant of xrdvi_profile, for callers that cannot allocate
 * device memory: code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc.  Same arguments, kernels and results (bit for bit)
 * as xrdvi_profile; the per-call state lives in a static 64 MiB device array
 * of the library (one per GPU, held until the process ends; its address is
 * looked up once per device by xrdvi_ctx_create), and the call allocates
 * nothing.  A problem and S whose per-call state needs more than 64 MiB are
 * rejected with XRDVI_EINVAL (xrdvi_profile serves them).  Every call on one
 * GPU shares that GPU's array: calls that overlap on one GPU (different
 * streams, or threads) race and give unspecified output; serialise them.
 */
XRDVI_API int xrdvi_profile_static(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                                   int32_t S, const double *phi, float *f_out,
                                   void *stream);

/*
 * Window plan: the points whose peak sum (Appendix A.2, profile function)
 * includes peak m at sample s.  The paper sums every peak over every point
 * (Sec. 2.3, the dense peak function); here a peak's terms are kept within
 * c full widths of its centre, and c = 0 is the paper's dense sum.  For
 * each sample s and peak m (caller's peak order),
 * lo[s][m] = first grid index inside [rho - c w, rho + c w] (upper bound
 * rho + (c w) alpha for asymmetric peaks) and hi[s][m] = one past the last
 * (lo = hi when empty), with rho = p_m + mu and the bounds formed in FP64 by
 * single rounded operations.  With c = 0 every window is [0, N).
 *   phi     device double [S][D][K]
 *   lo, hi  device int32 [S][T]
 */
XRDVI_API int xrdvi_window_plan(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                                int32_t S, const double *phi, int32_t *lo,
                                int32_t *hi, void *stream);

/*
 * ELBO forward (Sec. 3.2): draws z_s = loc + exp(logscale) * eps_s for
 * s < S, evaluates the profile, the Poisson log-likelihood (Appendix A.2)
 * and the estimate
 *   L = (1/S) sum_s [ln p(Y|phi_s) + ln p(phi_s) + ln|J(z_s)|]
 *       + sum_j logscale_j + (D K / 2) (1 + ln 2 pi).
 *   loc, logscale  device double [D][K]
 *   eps            device double [S][D][K] standard-normal noise, or NULL to
 *                  draw it on the device from Philox4x32-10 keyed by
 *                  (seed, step) with Box-Muller (counter (j/4, s, step))
 *   need_grad      non-zero: also run the recomputing adjoint so that
 *                  xrdvi_elbo_bwd can follow (fused forward + adjoint)
 *   elbo_out       device double [1]
 *   loglik_out     device double [S] (ln p(Y|phi_s)), or NULL
 *   tape           created for this problem with the same S
 * The tape keeps copies of eps, the samples and exp(logscale), so loc and
 * logscale may change after the call.
 */
XRDVI_API int xrdvi_elbo_fwd(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                             int32_t S, const double *loc,
                             const double *logscale, const double *eps,
                             uint64_t seed, uint64_t step, int32_t need_grad,
                             double *elbo_out, double *loglik_out,
                             xrdvi_tape *tape, void *stream);

/*
 * ELBO gradient.  The method turns inference into an optimisation solved by
 * the gradient method with stochastic VI (Sec. 2.1), maximising the ELBO
 * over the mean-field Gaussian's parameters (Sec. 3.2); this call gives
 * g times dL/dloc and dL/dlogscale of the reparameterised estimate computed
 * by the last xrdvi_elbo_fwd on this tape (which must have had need_grad
 * set; else XRDVI_EINVAL), with g = grad_scale, further multiplied by
 * *grad_scale_dev when that device pointer is non-NULL (an upstream
 * gradient that stays on the device).  Window edges are held fixed (the
 * estimate is piecewise smooth in the parameters when c > 0).
 *   grad_loc, grad_logscale  device double [D][K]
 */
XRDVI_API int xrdvi_elbo_bwd(xrdvi_ctx *ctx, const xrdvi_tape *tape,
                             double grad_scale, const double *grad_scale_dev,
                             double *grad_loc, double *grad_logscale,
                             void *stream);

/*
 * Adam ascent step (Kingma & Ba 2015) on n coordinates, the optimiser of
 * the stochastic VI loop (the paper runs 1000 optimisation steps, Sec. 4):
 *   m1 = b1 m1 + (1-b1) g,  m2 = b2 m2 + (1-b2) g^2,
 *   theta += lr (m1 / (1 - b1^t)) / (sqrt(m2 / (1 - b2^t)) + eps)
 * theta, m1, m2 (updated in place), grad: device double [n]; t >= 1.
 */
XRDVI_API int xrdvi_adam_step(xrdvi_ctx *ctx, int32_t n, double *theta,
                              double *m1, double *m2, const double *grad,
                              int32_t t, double lr, double beta1, double beta2,
                              double eps, void *stream);

/* ---- serving: continuous batching of whole analyses ------------------------
 *
 * An analysis is `steps` stochastic-VI optimisation steps (ELBO forward,
 * adjoint gradient, Adam with beta = (0.9, 0.999), eps = 1e-8) of one
 * problem with S samples per step; the noise of step n is Philox4x32-10
 * keyed by (seed, n) as in xrdvi_elbo_fwd, so the result depends only on
 * the request.  The server keeps each admitted analysis's problem and
 * variational state resident in a device arena, admits queued requests in
 * arrival order as soon as a slot and arena memory are free, and advances
 * all resident analyses together with batched kernels (optionally replayed
 * from one captured hipGraph).
 */
typedef struct {
    xrdvi_problem_desc problem;     /* host pointers, copied at submit       */
    int32_t S;                      /* samples per step, 1..1024             */
    int32_t steps;                  /* optimisation steps, >= 1              */
    uint64_t seed;                  /* noise key                             */
    double lr;                      /* Adam step size; 0 selects 1e-2        */
    const double *init_loc;         /* host [D][K] or NULL: m_h = ln(0.01 /
                                       lambda), m_mu = 0, m_w = ln 0.1,
                                       m_r = 0, m_alpha = 0                 */
    const double *init_logscale;    /* host [D][K] or NULL: ln 0.1           */
    double *out_loc;                /* host [D][K] or NULL; written before
                                       poll reports completion              */
    double *out_logscale;           /* host [D][K] or NULL                   */
    double *out_elbo_trace;         /* host [steps] or NULL: ELBO per step   */
} xrdvi_request;

typedef struct {
    int32_t state;        /* XRDVI_PENDING, XRDVI_OK or a negative error     */
    int32_t steps_done;
    double t_arrive;      /* seconds on the server clock: submit, ...        */
    double t_admit;       /* ... admission (-1 before), ...                  */
    double t_done;        /* ... completion (-1 before)                      */
    double final_elbo;    /* ELBO estimate of the last step                  */
} xrdvi_status;

typedef struct {
    int32_t device;
    int32_t max_slots;         /* analyses resident at once, 1..512          */
    int32_t max_queue;         /* queued requests before XRDVI_EBUSY         */
    int32_t steps_per_launch;  /* optimisation steps per batched launch      */
    int32_t use_graph;         /* non-zero: replay the steps from a hipGraph */
    void *arena;               /* device memory for resident analyses, or
                                  NULL to let the server allocate it         */
    size_t arena_bytes;
    size_t resident_bytes;     /* > 0: cap on the summed footprint of the
                                  resident analyses (one is always admitted
                                  when none is resident); 0: no cap beyond
                                  max_slots and the arena                    */
} xrdvi_server_config;

/* Creates a server with its own stream (default priority) and scheduler
 * thread.  A caller-supplied arena must stay valid until destroy. */
XRDVI_API int xrdvi_server_create(const xrdvi_server_config *cfg,
                                  xrdvi_server **out);
/* Cancels everything not finished, joins the scheduler, frees resources. */
XRDVI_API int xrdvi_server_destroy(xrdvi_server *srv);
/* Queues a request (host inputs copied; the caller may free them on
 * return).  XRDVI_EINVAL for an invalid problem or parameters,
 * XRDVI_ENOMEM if it can never fit the arena, XRDVI_EBUSY if the queue is
 * full.  Thread-safe. */
XRDVI_API int xrdvi_submit(xrdvi_server *srv, const xrdvi_request *req,
                           uint64_t *ticket);
/* Arena bytes a request occupies while resident (its problem, per-step
 * state, variational and Adam state and ELBO trace, in 256-byte aligned
 * pieces), for sizing a server's arena or resident cap.  Host only:
 * validates the request like xrdvi_submit (XRDVI_EINVAL) and copies
 * nothing. */
XRDVI_API int xrdvi_request_footprint(const xrdvi_request *req, size_t *bytes);
/* XRDVI_PENDING while queued or running; XRDVI_OK once the outputs have
 * been written (reported once: the ticket is then forgotten and later
 * polls return XRDVI_ENOENT); XRDVI_ECANCELED, XRDVI_ENONFINITE or
 * XRDVI_EDEVICE when it failed.  `st` (may be NULL) receives the state and
 * the time stamps.  Thread-safe. */
XRDVI_API int xrdvi_poll(xrdvi_server *srv, uint64_t ticket,
                         xrdvi_status *st);
/* Cancels a queued or running request (its outputs are not written).
 * Thread-safe. */
XRDVI_API int xrdvi_cancel(xrdvi_server *srv, uint64_t ticket);
/* Current time (seconds) on the clock of the status time stamps. */
XRDVI_API double xrdvi_server_clock(xrdvi_server *srv);

/* One analysis at a time on `stream`, with the per-step launches of
 * xrdvi_elbo_fwd / xrdvi_elbo_bwd / xrdvi_adam_step: the sequential
 * reference of the serving loop (same kernels and noise keys).
 * Synchronous; fills the request's outputs and *st. */
XRDVI_API int xrdvi_plain_run(xrdvi_ctx *ctx, const xrdvi_request *req,
                              xrdvi_status *st, void *stream);

/*
 * Copies the constrained samples phi_s = T(z_s) drawn by the last
 * xrdvi_elbo_fwd on `tape` into phi_out (device double [S][D][K]), e.g. to
 * inspect the approximate posterior or to count the peak-points of the
 * step with xrdvi_window_plan.
 */
XRDVI_API int xrdvi_tape_samples(xrdvi_ctx *ctx, const xrdvi_tape *tape,
                                 double *phi_out, void *stream);

/*
 * Unnormalised log posterior density in the unconstrained coordinates and
 * its gradient, at S positions (Sec. 3.2 transforms; App. A.2 likelihood;
 * Sec. 2.2 and App. B.2 priors):
 *   logp_s = ln p(Y | phi(z_s)) + ln p(phi(z_s)) + ln|d phi / d z|(z_s)
 *   grad_s = d logp_s / d z_s
 * computed by the same fused forward and adjoint kernels as the ELBO (the
 * ELBO estimate is the mean of logp over its samples plus the entropy).
 *   z         device double [S][D][K] positions (rows as loc)
 *   logp_out  device double [S]
 *   grad_out  device double [S][D][K], or NULL for the density only
 *   tape      created for this problem with the same S (its ELBO state is
 *             overwritten: a later xrdvi_elbo_bwd needs a new forward)
 */
XRDVI_API int xrdvi_logpost(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                            int32_t S, const double *z, double *logp_out,
                            double *grad_out, xrdvi_tape *tape, void *stream);

/*
 * Hamiltonian Monte Carlo over the same posterior (the sampling method the
 * paper compares stochastic VI with: 1000 samples after 1000 burn-in
 * iterations, Sec. 4 and Table 1).  Every gradient is one xrdvi_logpost
 * evaluation of all chains together.  Iteration i of chain c draws its
 * momentum p ~ N(0, I) from Philox4x32-10 keyed by (seed, i) (counter
 * (j/4, c, i), Box-Muller as for the ELBO noise), takes n_leapfrog leapfrog
 * steps, and accepts with probability min(1, exp(H0 - H1)),
 * H = -logp + |p|^2 / 2, using u = (v0 + 0.5) / 2^32 of the Philox block
 * with counter (0, c, i) and key seed ^ 0x9E3779B97F4A7C15.  During the
 * n_warmup iterations each chain adapts its step size by dual averaging
 * (Hoffman and Gelman 2014: mu = ln(10 step_size), gamma = 0.05, t0 = 10,
 * kappa = 0.75, target acceptance target_accept), then keeps the averaged
 * step for the n_draws kept iterations.  A non-finite Hamiltonian is a
 * rejection.  Synchronous.
 *   z           device double [chains][D][K]: initial positions in, final
 *               positions out
 *   draws       device double [n_draws][chains][D][K] or NULL
 *   logp_draws  device double [n_draws][chains] or NULL
 *   accept_out  host double [chains]: acceptance rate of the kept
 *               iterations, or NULL
 *   step_out    host double [chains]: final step sizes, or NULL
 */
typedef struct {
    int32_t chains;        /* 1..1024 */
    int32_t n_warmup;      /* >= 0 */
    int32_t n_draws;       /* >= 0 */
    int32_t n_leapfrog;    /* >= 1 */
    double step_size;      /* initial step size, > 0 */
    double target_accept;  /* in (0, 1); 0 selects 0.8 */
    uint64_t seed;
} xrdvi_hmc_config;

XRDVI_API int xrdvi_hmc(xrdvi_ctx *ctx, const xrdvi_problem *prob,
                        const xrdvi_hmc_config *cfg, double *z, double *draws,
                        double *logp_draws, double *accept_out,
                        double *step_out, void *stream);

/*
 * Background estimate before an analysis (App. A.2: the background is
 * estimated beforehand by an iterative least-squares method), by asymmetric
 * least squares (Eilers and Boelens 2005): starting from w = 1, n_iter
 * times solve (W + lambda D^T D) z = W y (D the second-difference
 * operator, W = diag(w)) and set w_i = p where y_i > z_i and 1 - p elsewhere;
 * the last z is the background.  FP64; one wave per spectrum solves the
 * pentadiagonal system in parallel (blocks separated by 2-row separators,
 * each factored as L D L^T, then the Schur complement on the separators).
 *   B, N      spectra and points per spectrum (>= 1)
 *   y         device double [B][N] counts
 *   lambda    smoothness (>= 0; e.g. 1e5 - 1e8 for 2-theta steps of 0.01 -
 *             0.02 deg); p in (0, 0.5) (e.g. 0.001 - 0.05)
 *   bg_out    device double [B][N] (may not alias y)
 *   scratch   device memory of 4 B N doubles, owned by the caller
 * The result can be <= 0 where counts are low; a problem description needs
 * bg > 0, so clamp it before xrdvi_problem_create.
 */
XRDVI_API int xrdvi_background(xrdvi_ctx *ctx, int32_t B, int32_t N,
                               const double *y, double lambda, double p,
                               int32_t n_iter, double *bg_out, void *scratch,
                               void *stream);

/*
 * Posterior readout of a converged analysis (Sec. 4: phases are identified
 * by their area ratio, with a threshold of 1 %).  Under q the weight h_k is
 * log-normal, so with m = loc[0][k] and s = exp(logscale[0][k]):
 *   E_q[h_k] = exp(m + s^2/2),  sd_q[h_k] = E_q[h_k] sqrt(exp(s^2) - 1).
 * Peaks have unit area, so phase k's area is E_q[h_k] sum_m I_m; its ratio
 * is that area over the sum of all phases' areas, and selected[k] = 1 when
 * the ratio exceeds `threshold`.  Host arrays only; no GPU work.
 *   K, peak_off[K+1], peak_int[T]  the candidate set, as in the problem
 *                                  description
 *   loc_h, logscale_h              host double [K]: row 0 (h) of loc and
 *                                  logscale, e.g. a served request's output
 *   threshold                      in [0, 1) (0.01 in the paper)
 *   mean_h, sd_h, area_ratio       host double [K], each may be NULL
 *   selected                       host int32 [K] or NULL
 * XRDVI_EINVAL for malformed arguments or a total area that is not
 * positive and finite.
 */
XRDVI_API int xrdvi_readout(int32_t K, const int32_t *peak_off,
                            const double *peak_int, const double *loc_h,
                            const double *logscale_h, double threshold,
                            double *mean_h, double *sd_h, double *area_ratio,
                            int32_t *selected);

/*
 * Kernel timing for measurement: while enabled, every fused profile /
 * likelihood / adjoint launch issued through `ctx` is bracketed by HIP
 * events recorded on the launch's own stream.  xrdvi_timing_read waits for
 * the recorded events and returns the summed kernel time (ms) and launch
 * count; reset != 0 clears them.  Disabled by default; enabling costs two
 * event records per launch.
 */
XRDVI_API int xrdvi_timing_enable(xrdvi_ctx *ctx, int32_t enable);
XRDVI_API int xrdvi_timing_read(xrdvi_ctx *ctx, double *ms_total,
                                int64_t *launches, int32_t reset);

#ifdef __cplusplus
}
#endif
#endif /* XRDVI_H */
