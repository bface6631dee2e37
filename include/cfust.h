/*
 * cfust.h -- C ABI of the MI355X (gfx950) CFUST mixture E-step / M-step library.
 *
 * The model is the finite mixture of canonical fundamental skew t (CFUST)
 * distributions of Lee, Leemaqz & McLachlan, "A simple multithreaded
 * implementation of the EM algorithm for mixture models":
 *   component density  Sec. 2 eq. (4):
 *     f_h(y) = 2^q t_p(y; mu, Omega, nu) T_q(c(y) sqrt((nu+p)/(nu+d(y))); 0, Lambda, nu+p),
 *     Omega = Sigma + Delta Delta^T, c(y) = Delta^T Omega^{-1}(y-mu),
 *     Lambda = I_q - Delta^T Omega^{-1} Delta, d(y) = (y-mu)^T Omega^{-1}(y-mu);
 *   E-step  Sec. 3.1 eqs. (7)-(17); M-step  Sec. 3.2 eqs. (18)-(22);
 *   log-likelihood  Sec. 4.3 eq. (27).
 * The normal limit nu -> infinity of the family (CFUSN in Table 1) is
 * selected per component by nu_h = +INFINITY: t_p becomes the normal density
 * phi_p(y; mu, Omega), every T becomes the normal CDF with limit c(y)
 * (the dof ratios tend to 1), W = 1 so w = 1 and e1 = 0, the truncated
 * moments are the normal ones, and the M-step keeps nu_h infinite.  A mixture
 * may hold normal and t components together.
 * The q-variate t CDFs (T_q, and the T_{q-1}, T_{q-2} that the truncated-t
 * moments of eqs. (16)-(17) need) are estimated by separation of variables on
 * a randomly shifted rank-1 lattice whose generating vector and shifts the
 * caller supplies (cfust_qmc).
 *
 * Conventions for every call:
 *   - All array arguments are DEVICE pointers owned by the caller unless marked
 *     "host".  Matrices are row-major FP64.  Per-(component, observation)
 *     outputs use the structure-of-arrays layout [g][k][n].
 *   - Calls are asynchronous on `stream` (a hipStream_t passed as void*; NULL
 *     is the default stream).  They return synchronously only the result of
 *     host-side argument checks; numeric failures found on the device are
 *     reported through the optional int32 status words (see cfust_status).
 *   - No call throws.  The handle owns a workspace that grows on demand;
 *     cfust_reserve() sizes it up front so that later calls do not allocate.
 *   - Results depend only on the inputs, (N, S, z, shifts) and the precision.
 */
#ifndef CFUST_H
#define CFUST_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define CFUST_MAX_P 16      /* data dimension p */
#define CFUST_MAX_Q 8       /* skewing dimension q; also the largest T_m dimension */
#define CFUST_MAX_G 64      /* mixture components */
#define CFUST_LATTICE_DIM 8 /* lattice coordinates: an m-variate T_m uses the first m-1, the moment
                              integrals of the direct estimator the first m */
#define CFUST_MAX_SHIFTS 64

typedef enum {
    CFUST_OK = 0,
    CFUST_EINVAL = -1,       /* bad dimensions, null pointer, unsupported size */
    CFUST_ENOTSPD = -2,      /* Omega_h, Lambda_h, Sigma_h or sum tau e3 not positive definite */
    CFUST_ENUMERIC = -3,     /* non-finite result */
    CFUST_EDEVICE = -4,      /* HIP runtime error */
    CFUST_ENOMEM = -5,       /* workspace allocation failed */
    CFUST_EUNSUPPORTED = -6  /* device is not gfx950 */
} cfust_status;

/* Device status word bits (int32, written by the kernels; 0 = all good). */
#define CFUST_DEV_NOTSPD_OMEGA   (1 << 0)
#define CFUST_DEV_NOTSPD_LAMBDA  (1 << 1)
#define CFUST_DEV_BADPARAM       (1 << 2)   /* nu <= 0, pi < 0, non-finite parameter */
#define CFUST_DEV_NOTSPD_E3      (1 << 3)   /* M-step: sum tau e3 not SPD -> Delta_h kept */
#define CFUST_DEV_NOTSPD_SIGMA   (1 << 4)   /* M-step: new Sigma_h not SPD -> theta_h kept */
#define CFUST_DEV_FROZEN         (1 << 5)   /* M-step: n_h < p+1 -> theta_h kept */
#define CFUST_DEV_NU_CLAMPED     (1 << 6)   /* M-step: nu root outside [1, 200] -> clamped */

typedef struct cfust_ctx *cfust_handle;

/* Create a handle bound to HIP device `device` (must be gfx950). */
cfust_status cfust_create(cfust_handle *handle, int device);
cfust_status cfust_destroy(cfust_handle handle);
/* Text of the last host-side error on this handle (never NULL). */
const char *cfust_last_error(cfust_handle handle);

typedef struct {
    int32_t n;   /* observations, n >= 0 */
    int32_t p;   /* 1 <= p <= CFUST_MAX_P */
    int32_t q;   /* 1 <= q <= CFUST_MAX_Q */
    int32_t g;   /* 1 <= g <= CFUST_MAX_G */
} cfust_dims;

/* Psi = (pi, theta_1..theta_g), Sec. 2: device FP64, row-major.
 * pi[g], mu[g][p], Sigma[g][p][p], Delta[g][p][q], nu[g] (nu > 0, or
 * +INFINITY for the normal limit of that component). */
typedef struct {
    const double *pi, *mu, *Sigma, *Delta, *nu;
} cfust_params;

typedef struct {
    double *pi, *mu, *Sigma, *Delta, *nu;
} cfust_params_out;

enum { CFUST_FP64 = 0, CFUST_MIXED = 1 };

/* Lattice rule.  Point k (0 <= k < N) of shift s in coordinate j is
 *   t = frac(k z[j] / N + shifts[s][j]),  x = 1 - |2t - 1|  (clamped to [2^-24, 1-2^-24]).
 * precision: CFUST_FP64 evaluates everything in FP64 (the univariate t
 * probabilities and quantiles of the integrand come from FP64 Chebyshev
 * tables of each dof, within about 1e-14 of the exact values, the quantile
 * polished by a Newton step; an integral with a dof above 1000, past the
 * tables, takes the exact continued-fraction transforms); CFUST_MIXED
 * evaluates the lattice integrand in FP32 on FP32 tables of each dof
 * (per-shift FP32 sums, combined in FP64; an integral whose FP32 product
 * underflows is redone in FP64) and keeps the Cholesky factors,
 * log-densities, log-sum-exp and M-step in FP64. */
typedef struct {
    int32_t N;               /* 2 <= N <= 65536 points per shift */
    int32_t S;               /* 1 <= S <= CFUST_MAX_SHIFTS shifts */
    const int32_t *z;        /* device [CFUST_LATTICE_DIM], 0 < z[j] < N */
    const double *shifts;    /* device [S][CFUST_LATTICE_DIM], each in [0,1) */
    int32_t precision;       /* CFUST_FP64 or CFUST_MIXED */
} cfust_qmc;

/* E-step outputs.  w, e1, e2, e3 are double* when precision == CFUST_FP64
 * and float* when CFUST_MIXED.  e3 holds the packed upper triangle (i <= k,
 * row-major order) of the symmetric q x q matrix. */
typedef struct {
    double *tau;         /* [g][n]  posterior membership, eq. (12) */
    double *logf_obs;    /* [n]     log f(y_j; Psi), the summands of eq. (27) */
    double *loglik;      /* [1]     log-likelihood, eq. (27) */
    void *w;             /* [g][n]      eq. (13) */
    void *e1;            /* [g][n]      eq. (15) */
    void *e2;            /* [g][q][n]   eq. (16) */
    void *e3;            /* [g][q(q+1)/2][n] eq. (17) */
    double *logf_comp;   /* optional [g][n]: log f_h(y_j), eq. (4) */
    double *cdf_stderr;  /* optional [g][n]: lattice standard error of the T_q of eq. (4) */
    int32_t *status;     /* optional [1]: device status bits, OR-ed in */
} cfust_estep_out;

/* E-step, Sec. 3.1: for every (component h, observation j) the CFUST
 * log-density (eq. 4), tau (eq. 12), w (eq. 13, with "nu d" read as nu + d),
 * e1 (eq. 15, one-step-late form as printed), e2, e3 (eqs. 16-17, moments of
 * the truncated t of Sec. 3.1), and the log-likelihood (eq. 27).
 * y: device FP64 [p][n] (feature-major).  Components whose log-density is
 * -inf get tau = 0 and zero e-terms. */
cfust_status cfust_estep(cfust_handle handle, const double *y, cfust_dims dims,
                         const cfust_params *params, const cfust_qmc *qmc,
                         const cfust_estep_out *out, void *stream);

/* Allocation-free E-step, for callers that cannot allocate device memory
 * (work under HIP stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): the same arguments, kernels and results as cfust_estep, bit for
 * bit, but its workspace is a fixed device array of CFUST_NOALLOC_WS_BYTES
 * that the library holds on every device it is loaded on until the process
 * ends (its address is looked up once per device by cfust_create).  The call
 * makes no hipMalloc, hipFree or other allocating call and records no
 * profiling events.  Workspace needed: about g n (12 J + 16) bytes plus 85 KB
 * per component, J = lattice integrals per pair (2 at q = 2, 12 at q = 4,
 * 38 at q = 8), plus (8 (q - 1) + 4) N S bytes of lattice coordinates in mixed
 * precision when that table is at most 16 MB (e.g. n up to ~26000 at
 * p = q = 8, g = 5, N = 8192, S = 8); a larger call returns
 * CFUST_EINVAL before any launch.  All calls on one device share that
 * device's array, which keeps the last call's contents: calls that overlap on
 * one device (other streams, other threads, other handles) race and must be
 * serialised by the caller.  CFUST_EDEVICE if the array's address could not
 * be obtained at cfust_create. */
#define CFUST_NOALLOC_WS_BYTES (64u << 20)
cfust_status cfust_estep_noalloc(cfust_handle handle, const double *y, cfust_dims dims,
                                 const cfust_params *params, const cfust_qmc *qmc,
                                 const cfust_estep_out *out, void *stream);

/* M-step, Sec. 3.2 eqs. (18)-(22), in the order pi, mu (with Delta^(k)),
 * Delta (with mu^(k+1)), Sigma (with both), nu.  Eq. (22) is solved with the
 * last sum added ("+"), by 8 rounds of 256-point multisection of [1, 200]
 * (clamped outside); an infinite nu (normal limit) is kept.
 * `es` is the output of cfust_estep at the same dims/precision; `in` is
 * Psi^(k) (only mu, Delta, Sigma, nu are read), `out` receives Psi^(k+1)
 * (`out` may alias `in`).  A component with n_h < p+1, or whose update is not
 * SPD, keeps theta_h and sets a status bit.  status: optional device int32[1]. */
cfust_status cfust_mstep(cfust_handle handle, const double *y, cfust_dims dims,
                         const cfust_estep_out *es, int32_t precision,
                         const cfust_params *in, const cfust_params_out *out,
                         int32_t *status, void *stream);

/* Log-likelihood only (eq. 27): evaluates the density (4) of every pair and
 * the log-sum-exp over components, without the moments.  logf_obs: optional
 * device [n]; loglik: device [1]; status: optional device int32[1]. */
cfust_status cfust_loglik(cfust_handle handle, const double *y, cfust_dims dims,
                          const cfust_params *params, const cfust_qmc *qmc,
                          double *loglik, double *logf_obs, int32_t *status, void *stream);

/* Batch of multivariate t probabilities T_m(b; 0, L L^T, nu) (the T_q of
 * Sec. 2 eq. 4), one per item.  1 <= m <= CFUST_MAX_Q.
 * b: device [batch][m] upper limits; L: device [nmat][m][m] lower Cholesky
 * factors; mat_idx: device int32 [batch] in [0, nmat); nu: device [batch] > 0 (+INFINITY: the normal CDF).
 * p: device [batch] estimates; logp (optional): log of the estimate computed
 * without underflow of the first factor; stderr_ (optional): standard error
 * over shifts (0 for m = 1). */
cfust_status mvt_cdf_batch(cfust_handle handle, int32_t m, int32_t batch, const double *b,
                           const double *L, const int32_t *mat_idx, int32_t nmat,
                           const double *nu, const cfust_qmc *qmc,
                           double *p, double *logp, double *stderr_, void *stream);

/* ------------------------------------------------------------------------
 * Surrogate network (learned replacement of the lattice estimate of T_m,
 * m = 2..4, with the lattice as fallback).  A 16 -> 256 -> 256 -> 256 -> 256
 * -> 16 perceptron, tanh-form GELU, BF16 weights/activations, FP32
 * accumulation on the matrix cores, FP32 master weights and Adam.  Input
 * features (FP32 before rounding to BF16): the m standardised limits
 * z_i = b_i/sqrt(R_ii) as z_i/6, the m(m-1)/2 correlations,
 * (ln nu - ln 2)/(ln 30 - ln 2), the marginal log-CDFs ln T_nu(z_i)/10, zero
 * padding.  Output 0 is (ln T_m - sum_i ln T_nu(z_i)) / 5 (the correction to
 * the independence value), output 1 the predicted log10 of its absolute
 * error.  All buffers are device memory owned by the caller; B (rows) must
 * be a positive multiple of 64; rows are independent.
 * ---------------------------------------------------------------------- */
#define CFUST_MLP_IN 16
#define CFUST_MLP_HIDDEN 256
#define CFUST_MLP_OUT 16
#define CFUST_MLP_LAYERS 5

/* Layer l maps K_l -> N_l (K = 16, 256, 256, 256, 256; N = 256, 256, 256, 256, 16).
 * W[l]: BF16 [N_l][K_l]; Wt[l]: the same matrix transposed, BF16 [K_l][N_l];
 * b[l]: FP32 [N_l]. */
typedef struct {
    void *W[CFUST_MLP_LAYERS];
    void *Wt[CFUST_MLP_LAYERS];
    float *b[CFUST_MLP_LAYERS];
} cfust_mlp_weights;

/* Saved activations for the backward pass: X[l] = input of layer l, BF16
 * [B][K_l] (X[0] is written as a copy of the input); XT[l] its transpose
 * [K_l][B]; Z[l] = pre-activation of hidden layer l, FP32 [B][N_l], l < 4. */
typedef struct {
    uint16_t *X[CFUST_MLP_LAYERS];
    uint16_t *XT[CFUST_MLP_LAYERS];
    float *Z[CFUST_MLP_LAYERS - 1];
} cfust_mlp_acts;

/* Gradients: dW[l] FP32 [N_l][K_l], db[l] FP32 [N_l] (overwritten). */
typedef struct {
    float *dW[CFUST_MLP_LAYERS];
    float *db[CFUST_MLP_LAYERS];
} cfust_mlp_grads;

/* FP32 master weights and Adam moments, same shapes as the gradients. */
typedef struct {
    float *W[CFUST_MLP_LAYERS], *mW[CFUST_MLP_LAYERS], *vW[CFUST_MLP_LAYERS];
    float *b[CFUST_MLP_LAYERS], *mb[CFUST_MLP_LAYERS], *vb[CFUST_MLP_LAYERS];
} cfust_mlp_master;

/* Forward pass: out FP32 [B][CFUST_MLP_OUT].  X0: BF16 [B][CFUST_MLP_IN].
 * acts (optional) receives what cfust_mlp_backward needs. */
cfust_status cfust_mlp_forward(cfust_handle handle, const cfust_mlp_weights *w, const uint16_t *X0,
                               int32_t B, float *out, const cfust_mlp_acts *acts, void *stream);
/* Backward pass from dout = dLoss/dout (FP32 [B][CFUST_MLP_OUT]) through the
 * activations saved by the forward pass; writes grads. */
cfust_status cfust_mlp_backward(cfust_handle handle, const cfust_mlp_weights *w, const cfust_mlp_acts *acts,
                                const float *dout, int32_t B, const cfust_mlp_grads *grads, void *stream);
/* Adam step `step` (1-based) on the master weights; refreshes the BF16 W, Wt. */
cfust_status cfust_mlp_adam(cfust_handle handle, const cfust_mlp_master *master, const cfust_mlp_grads *grads,
                            const cfust_mlp_weights *w, float lr, float beta1, float beta2, float eps,
                            int32_t step, void *stream);
/* Training loss: sum over the first nvalid rows of (out0 - label)^2 +
 * lam (out1 - log10(|out0 - label| + 1e-6))^2 into loss_sum[1], and its
 * gradient divided by nvalid into dout (padding rows get 0). */
cfust_status cfust_mlp_loss(cfust_handle handle, const float *out, const float *label, int32_t B,
                            int32_t nvalid, float lam, float *dout, float *loss_sum, void *stream);

/* Surrogate configuration for cfust_estep_surrogate.  model[m] (m = 2..4)
 * holds the trained weights of the network for T_m, or NULL to use the
 * lattice for that dimension.  A lattice integral is answered by the network
 * when its inputs lie in the training domain and the predicted absolute
 * error of ln T_m is at most tol; otherwise the lattice estimate is used.
 * tol = 0 therefore reproduces cfust_estep exactly. */
typedef struct {
    const cfust_mlp_weights *model[CFUST_MAX_Q + 1];
    float tol;
    int32_t *n_fallback;   /* optional device int32[1]: integrals sent to the lattice */
} cfust_surrogate;

/* E-step with the surrogate for the T_m of dimension 2..4 (same outputs as
 * cfust_estep; cdf_stderr is left unwritten for network-answered items). */
cfust_status cfust_estep_surrogate(cfust_handle handle, const double *y, cfust_dims dims,
                                   const cfust_params *params, const cfust_qmc *qmc,
                                   const cfust_surrogate *sur, const cfust_estep_out *out, void *stream);

/* Network features of a batch of T_m problems (same arguments as
 * mvt_cdf_batch): X0 BF16 [rows_pad][CFUST_MLP_IN] (rows >= batch zeroed),
 * inrange (optional) int32 [batch]: 1 inside the training domain
 * (|b_i / sqrt(R_ii)| <= 6, 2 <= nu <= 30); base (optional) FP64 [batch]:
 * sum_i ln T_nu(z_i), the value output 0 corrects. */
cfust_status cfust_mlp_features(cfust_handle handle, int32_t m, int32_t batch, int32_t rows_pad,
                                const double *b, const double *L, const int32_t *mat_idx, int32_t nmat,
                                const double *nu, uint16_t *X0, int32_t *inrange, double *base, void *stream);

/* Autotuner: times the variants of the lattice kernel (lattice points per
 * lane per loop trip) for every integral dimension these dims use, at this
 * lattice size and precision, on `stream`, and caches the fastest in the
 * handle (key: device architecture, m, N, S, precision).  Later calls with
 * the same key use the cached choice.  Synchronises the stream; call it
 * outside stream capture.  chosen (optional, host int32[CFUST_MAX_Q+1])
 * receives the choice per m (0 = not applicable). */
cfust_status cfust_autotune(cfust_handle handle, const double *y, cfust_dims dims,
                            const cfust_params *params, const cfust_qmc *qmc, int32_t *chosen,
                            void *stream);

/* Timing of the lattice-integrand kernels.  While enabled, HIP events
 * bracket the main lattice kernel of each integral dimension launched by
 * cfust_estep / cfust_loglik and the persistent queue kernels of the batch
 * calls (not inside a captured graph), on the call's stream (creating
 * events: do not enable during stream capture). */
cfust_status cfust_profile_enable(cfust_handle handle, int enable);
/* Waits for the recorded events, adds up their durations per integral
 * dimension m (0..CFUST_MAX_Q) into host arrays ms[CFUST_MAX_Q+1] and
 * launches[CFUST_MAX_Q+1], and clears the record. */
cfust_status cfust_profile_read(cfust_handle handle, double *ms, int32_t *launches);

/* Size the workspace for calls up to these dims and lattice sizes, so that
 * later calls allocate nothing (e.g. under stream capture). */
cfust_status cfust_reserve(cfust_handle handle, cfust_dims dims, const cfust_qmc *qmc);

/* ------------------------------------------------------------------------
 * Batches of independent fits (e.g. the starts of the initialisation of
 * Sec. 3.3, Algorithm 1, or fits of several data sets, each with its own n,
 * p, q, g).  A batch runs
 * the E-step (Sec. 3.1) and M-step (Sec. 3.2) of all its fits with one launch
 * per kernel kind: the lattice integrals of every fit form one work queue per
 * integral dimension m, drained by a persistent kernel in
 * longest-processing-time order (tiles of observations x component x
 * integral).  Each fit's results equal those of cfust_estep / cfust_mstep on
 * that fit alone, bit for bit.
 * ---------------------------------------------------------------------- */
#define CFUST_MAX_FITS 1024

/* One fit.  All pointers are device memory owned by the caller and must stay
 * valid for the life of the batch.  params is read by the E-step and
 * overwritten in place by the M-step (Psi^(k) -> Psi^(k+1)).  out: tau,
 * logf_obs, loglik, w, e1, e2, e3 are required (FP32 e-terms in mixed
 * precision, as for cfust_estep); logf_comp and cdf_stderr are optional;
 * out.status is ignored (use status).  A fit with n > 0 whose tau, w, e1,
 * e2, e3 are all NULL is log-likelihood only: its E-step computes log f and the
 * log-likelihood (eq. 27) as cfust_loglik does, and a batch holding one
 * cannot run cfust_batch_mstep or cfust_fit_batch. */
typedef struct {
    cfust_dims dims;
    const double *y;             /* [p][n] */
    cfust_params_out params;
    cfust_estep_out out;
    int32_t *status;             /* optional [1]: device status bits of this fit, OR-ed in */
} cfust_fit;

typedef struct cfust_batch_ctx *cfust_batch;

/* Plan a batch of 1 <= nfits <= CFUST_MAX_FITS fits (host array `fits`,
 * copied) with one lattice rule for all of them.  Allocates the batch's own
 * device workspace; later batch calls allocate nothing. */
cfust_status cfust_batch_create(cfust_handle handle, int32_t nfits, const cfust_fit *fits, const cfust_qmc *qmc,
                                cfust_batch *batch);
cfust_status cfust_batch_destroy(cfust_batch batch);

/* E-step of every fit (cfust_estep semantics per fit). */
cfust_status cfust_batch_estep(cfust_batch batch, void *stream);
/* M-step of every fit (cfust_mstep semantics per fit, in place). */
cfust_status cfust_batch_mstep(cfust_batch batch, void *stream);

/* `iters` EM iterations of every fit: E-step, convergence check, M-step.
 * The log-likelihood (eq. 27) of iteration k of fit f goes to trace[k][f]
 * (optional device FP64 [iters][nfits]).  Convergence is Aitken's criterion
 * of Sec. 3.4 (eqs. 24-26): from the third iteration on, a fit stops when
 * |l_inf^(k+1) - l^(k+1)| < tol, with a^(k) = (l^(k+1) - l^(k)) / (l^(k) -
 * l^(k-1)) and l_inf^(k+1) = l^(k) + (l^(k+1) - l^(k)) / (1 - a^(k)); an
 * unchanged log-likelihood also stops it, and so does a non-finite one.
 * tol <= 0 runs all iterations.  A stopped fit is retired on the device: its
 * M-step and all later work are skipped, so its parameters and E-step
 * outputs stay those of its last E-step.  A fit that is never retired ends
 * after its last M-step (parameters one step ahead of the outputs, as in a
 * plain loop of cfust_estep, cfust_mstep).  iters_done (optional device int32
 * [nfits]) receives the E-steps run per fit.  use_graph != 0 captures one
 * iteration in a HIP graph (on first use, and again after cfust_batch_tune)
 * and replays it; 0 launches the kernels directly.  Do not call while
 * `stream` is being captured. */
cfust_status cfust_fit_batch(cfust_batch batch, int32_t iters, double tol, int32_t use_graph, double *trace,
                             int32_t *iters_done, void *stream);

/* Autotuner of the batch's lattice queues: times, for each integral
 * dimension, the persistent kernel with tiles of 4, 8 or 16 observations and
 * one or two blocks per resident slot, and the one-block-per-tile form of
 * the same queue (tiles of 4), each with (mixed, N a multiple of 128) 1 or 2
 * lattice points per lane per trip, on a prefix of the queue, and keeps the
 * fastest.  Synchronises the stream.  chosen (optional, host int32
 * [(CFUST_MAX_Q+1) * 3]) receives (rows per tile, blocks per slot -- 0 for
 * one block per tile --, points per lane) per m (zeros where no queue). */
cfust_status cfust_batch_tune(cfust_batch batch, int32_t *chosen, void *stream);

/* ------------------------------------------------------------------------
 * Starting values, Sec. 3.3 (eq. 23, Algorithm 1).  For every starting
 * partition s (labels[s][j] in [0, g): the component of observation j) and
 * every alpha[a] in (0, 1), each cluster h gives, from its sample mean ybar,
 * sample covariance S (divisor n_h - 1), s* = diag(S) and third central
 * moments m3:
 *     delta_i = sign(m3_i) sqrt(pi (1 - alpha) s*_i / (pi - 2))   (sign 0: +),
 *     Sigma_h = S - (1 - alpha) diag(s*)   on the skewed coordinates,
 *     mu_h = ybar - sqrt(2/pi) delta,   Delta_h[:, l] = delta_l e_l (l < q),
 *     nu_h = nu0,   pi_h = n_h / n
 * (nu0 > 0, or +INFINITY for starting values of the normal limit; the
 * square root covers s*_i; with q < p the first q coordinates are
 * skewed).  A candidate (s, a) is invalid when a cluster has n_h < p + 1 or a
 * Sigma_h that is not positive definite.  The log-likelihood (eq. 27) of
 * every valid candidate is evaluated in one density-only batch with the
 * lattice rule qmc; the first candidate with the largest value is written to
 * `best` (device arrays of the sizes of cfust_params).  loglik (optional,
 * device FP64 [nstarts][nalpha]) receives every candidate's value (-inf when
 * invalid); best_index (optional, device int32 [1]) the flat index
 * s * nalpha + a, or -1 when no candidate is valid (best is then unwritten).
 * 1 <= nstarts * nalpha <= CFUST_MAX_FITS; q <= p.  y: device [p][n];
 * labels: device int32 [nstarts][n]; alpha: host [nalpha].  Allocates its
 * own scratch and synchronises the device before returning. */
cfust_status cfust_init(cfust_handle handle, const double *y, cfust_dims dims, int32_t nstarts,
                        const int32_t *labels, int32_t nalpha, const double *alpha, double nu0,
                        const cfust_qmc *qmc, const cfust_params_out *best, double *loglik,
                        int32_t *best_index, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* CFUST_H */
