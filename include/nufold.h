/*
 * nufold: forward-folding binned-likelihood engine for reactor-neutrino
 * oscillation fits on AMD Instinct MI355X (gfx950).
 *
 * One model evaluation follows the paper's likelihood (Eq. 3-6, 9) and its
 * three-step signal calculation ("Structure of the framework"):
 *   1. every MC event is weighted by the survival probability (Eq. 1, or the
 *      exact three-flavour form that Eq. 10 rewrites) and summed into fine
 *      reconstructed-energy bins per dataset and source;
 *   2. the fine spectrum is rescaled by rate normalisations and flux-shape
 *      parameters;
 *   3. an area-conserving quadratic spline of the fine spectrum is integrated
 *      over the pre-images of the analysis bins under the second-order
 *      energy-scale polynomial; data-driven background templates are added;
 * then the binned Poisson negative log-likelihood (deviance form) plus
 * Gaussian and correlated-Gaussian priors is reduced in FP64, and its
 * gradient is obtained by one adjoint (reverse) pass.
 *
 * Conventions
 *   - Return codes: 0 OK; >0 warnings; <0 errors (see NF_* below).
 *     nf_last_error() returns a message owned by the context.
 *   - A context owns all device memory it allocates and is used by one host
 *     thread at a time.
 *   - Host-pointer calls are synchronous. Calls taking device pointers are
 *     enqueued on the context's stream and return without synchronising.
 *   - Units: energies in MeV, baselines in m, dm2_ee and dm2_31 in 1e-3 eV^2,
 *     dm2_21 in 1e-5 eV^2 ("fit units").
 *   - Parameter vectors theta have nf_num_params() entries, in the order of
 *     the model description's "params" list.
 */
#ifndef NUFOLD_H
#define NUFOLD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define NF_OK 0
#define NF_WDOMAIN 1   /* some expectation <= 0, energy map not monotone, or oscillation
                          parameter outside its domain: NLL = +inf, gradient = 0        */
#define NF_WNOCONV 2   /* fit stopped at its iteration limit before reaching the EDM goal */
#define NF_EINVAL -1   /* invalid argument: NaN/inf, bad size or index, null pointer      */
#define NF_ESTATE -2   /* call out of order (evaluation before events and data are set)  */
#define NF_ENOMEM -3   /* device or host allocation failed                                 */
#define NF_EDEVICE -4  /* no usable HIP device, or a HIP call failed                       */
#define NF_EPARSE -5   /* model description is not valid JSON or violates the schema      */

/* precision modes */
#define NF_M64 0       /* everything FP64; event stream u = L/E as f64, weights f32         */
#define NF_M32 1       /* per-event oscillation weight and per-lane sums in FP32 (u, w f32);
                          per-wave and later sums, bin stages, NLL and gradient in FP64     */

typedef struct nf_ctx nf_ctx;
typedef struct nf_mlp nf_mlp;  /* surrogate network (see nf_mlp_create) */

/*
 * Create a context from a JSON model description (paper: "Structure of the
 * framework", the configuration component). Schema:
 *   {"params": [{"name", "start", "prior": [mean, sigma] | null, "fixed"}],
 *    "cov_priors": [{"params": [names], "mean": [..], "cov": [[..]]}],
 *    "osc": {"formula": "eq1" | "3nu" | "4nu", <slot>: {"param": name} | {"value": v}},
 *    "datasets": [{"fine": {"y0", "width", "n"}, "edges": [Nb+1],
 *                  "sources": [{"baseline_m", "norm": [names]}], "norm": [names],
 *                  "flux": {"params": [M names], "basis": [M][n]},
 *                  "escale": {"c0", "c1", "c2": name | null},
 *                  "backgrounds": [{"rate": name | null, "scale",
 *                                   "template": [Nb], "shape": [Nb names|null] | null}]}]}
 * eq1 slots: sin2_2t13, dm2_ee, sin2_t12, dm2_21 (Eq. 1).
 * 3nu slots: sin2_t12, sin2_t13, dm2_21, dm2_31 (exact vacuum form; sign of dm2_31 = ordering).
 * 4nu slots: sin2_t13, dm2_31, sin2_2t14, dm2_41 (vacuum 3+1 form of the paper's sterile-neutrino
 *   searches, "Extensions of the framework": P = 1 - sum_{i<j} 4|U_ei|^2|U_ej|^2 sin^2(dm2_ji L/4E)
 *   over four mass states, |U_e1..4|^2 = c12 c13 c14, s12 c13 c14, s13 c14, s14 in squared sines
 *   and cosines; dm2_41 in 1e-3 eV^2), plus "sin2_t12" and "dm2_21" as {"value": v} constants.
 * model_json: NUL-terminated, caller-owned, copied. mode: NF_M64 or NF_M32.
 * hip_stream: hipStream_t to order device work on, or NULL for a stream the
 * context creates and owns. On error *out is NULL and the return code says why
 * (NF_EPARSE for schema errors, NF_EDEVICE without a GPU).
 */
int nf_create(nf_ctx** out, const char* model_json, int mode, void* hip_stream);

/* Free the context and every device buffer it owns. NULL is allowed. */
void nf_destroy(nf_ctx* ctx);

/* Message for the last non-OK return on this context (or of the last failed
 * nf_create when ctx is NULL). Valid until the next call on the context. */
const char* nf_last_error(const nf_ctx* ctx);

int nf_num_params(const nf_ctx* ctx);
int nf_num_datasets(const nf_ctx* ctx);
/* Number of analysis bins of dataset d, or NF_EINVAL. */
int nf_num_bins(const nf_ctx* ctx, int dataset);
/* Index of a named parameter, or NF_EINVAL if unknown. */
int nf_param_index(const nf_ctx* ctx, const char* name);

/*
 * Load the MC events of one dataset (paper: events are copied to the device
 * once and sorted by energy for locality; "GPU accelerated computation").
 * n events, SoA: e_true (MeV, > 0), e_reco (MeV), source index (< number of
 * sources; NULL means all 0), weight (NULL means all 1). Events with e_reco
 * outside the dataset's fine range [y0, y0 + n*width) are dropped and counted.
 * on_device != 0: the four pointers are device pointers; otherwise host.
 * The context copies the data; the caller keeps ownership. Replaces any
 * previous events of the dataset. n == 0 is allowed (empty signal).
 */
int nf_set_events(nf_ctx* ctx, int dataset, int64_t n, const double* e_true,
                  const double* e_reco, const uint8_t* source, const float* weight,
                  int on_device);

/* Number of events of a dataset dropped as out of range by nf_set_events. */
int64_t nf_dropped_events(const nf_ctx* ctx, int dataset);

/*
 * Observed counts n_{d,i} of one dataset (Eq. 3-5, 9): nbins must equal
 * nf_num_bins(dataset); counts >= 0 and finite (non-integer values allowed,
 * e.g. Asimov data). Copied; on_device as above.
 */
int nf_set_data(nf_ctx* ctx, int dataset, int nbins, const double* counts, int on_device);

/*
 * Evaluate NLL(theta) = sum_{d,i} [mu - n + n ln(n/mu)] + priors
 * (Eq. 3-6, 9 in deviance form: constants dropped, 2*NLL at a best fit is the
 * saturated-model statistic of Eq. 8). theta: host, nf_num_params() values.
 * Returns NF_OK, NF_WDOMAIN (nll = +inf), NF_EINVAL (NaN/inf in theta) or
 * NF_ESTATE (events or data missing for some dataset).
 */
int nf_eval_nll(nf_ctx* ctx, const double* theta, double* nll);

/* As nf_eval_nll, plus dNLL/dtheta in grad (host, nf_num_params() values),
 * from one forward fold with forward-mode oscillation derivatives and one
 * adjoint pass over the bin stages. */
int nf_eval_nll_grad(nf_ctx* ctx, const double* theta, double* nll, double* grad);

/*
 * Device-pointer evaluation, enqueued on the context stream, no host sync.
 * theta_dev: P doubles. out_dev: 1 + P doubles (NLL, then gradient; the
 * gradient part is left untouched when want_grad == 0). status_dev: NULL or
 * one int32 receiving the status bits (1 = domain warning). Inputs are not
 * validated on the host (NaN parameters produce a domain warning).
 */
int nf_eval_device(nf_ctx* ctx, const double* theta_dev, double* out_dev,
                   int32_t* status_dev, int want_grad);

/*
 * Allocation-free device evaluation, for callers that cannot allocate device
 * memory: code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc. Arguments, outputs and result are those of
 * nf_eval_device (same kernels); the evaluation's scratch (fold partials,
 * per-segment moments and spectra, fine-bin rows, arrival counters) lives in
 * one static device array per GPU of NF_NOALLOC_SCRATCH_BYTES bytes, part of
 * the library's code object and held until the process ends, instead of the
 * context's own buffers. The call enqueues a fill kernel that clears the
 * part of the array that must start at zero, then the fold and the bin
 * stages, on the context's stream; it calls no hipMalloc, hipFree or other
 * allocating routine (the context itself was set up by nf_create and
 * nf_set_events beforehand). The array keeps the last call's contents, and
 * every call on one GPU uses the same array: calls that can overlap on one
 * GPU (other streams or contexts, without ordering between them) race and
 * give wrong results. Needs 8 (6 KT + G) + 4 (G + KT) + 8 NM nitems +
 * 8 13 G + 8 R bytes (each part rounded up to 256; KT fine bins, G segments,
 * nitems work items, NM fold moments, R the parameter-pass values: about
 * KT + 5 analysis bins + 2 background terms + prior rows); a context that
 * needs more gets NF_EINVAL and an error message with its need.
 */
#define NF_NOALLOC_SCRATCH_BYTES (16u << 20)
int nf_eval_device_noalloc(nf_ctx* ctx, const double* theta_dev, double* out_dev,
                           int32_t* status_dev, int want_grad);

/*
 * n device evaluations in order, launched as one HIP graph on the context's
 * stream: evaluation i reads theta_dev + i*P and writes NLL and gradient to
 * out_dev + i*(1+P) (and its status to status_dev[i] when status_dev is not
 * NULL), exactly as nf_eval_device would. The graph is captured on the first
 * call and replayed by later calls with the same n, pointers and want_grad
 * (it reads the current contents of theta_dev); other arguments, new events
 * or changed launch options capture a new one. 1 <= n <= NF_MAX_GRAPH_EVALS.
 * Asynchronous like nf_eval_device; per-kernel timing (option "timing") does
 * not cover these launches. Each evaluation is that of nf_eval_device
 * (Eq. 3-6 and 9 with the adjoint gradient).
 */
#define NF_MAX_GRAPH_EVALS 4096
int nf_eval_device_many(nf_ctx* ctx, int n, const double* theta_dev, double* out_dev,
                        int32_t* status_dev, int want_grad);

/* Expected counts mu_{d,i}(theta) for every dataset, concatenated in dataset
 * order (host buffer of sum_d nf_num_bins(d) doubles). Needs events only. */
int nf_expected(nf_ctx* ctx, const double* theta, double* mu);

/*
 * Tuning knobs. key: "chunk" (events per fold work item, multiple of 256,
 * default 4096), "fold_block" (threads per fold workgroup: 64, 128 or 256),
 * "tail_threads" (bin-stage threads of the single evaluation: 256, 512 or
 * 1024), "batch_threads" (bin-stage threads per fit in batched launches: 256,
 * 512, 1024, or 0 = chosen from the model size), "batch_fit_tile" (fits per
 * wavefront tile of the batched fold, which reads each event once per tile:
 * 1, 2, 4 or 8, default 4). Changing "chunk" rebuilds
 * the work-item list. "deterministic" (0/1, default 0): with 1 the fold
 * kernel hands each fine bin's source rows to the last source to finish,
 * which sums them in source order, so repeated evaluations agree bit for bit;
 * with 0 each source adds its rows with device-scope atomic adds (no waiting
 * at the end of the fold; the order of those additions, and so the last bits
 * of the result, may vary between runs). "timing" (0/1) turns per-kernel event
 * timing on or off (see nf_timing). "stage_cache" (0/1, default 0): with 1,
 * the host-pointer evaluations (nf_eval_nll, nf_eval_nll_grad, nf_expected)
 * skip the event fold when the oscillation parameters and every source-norm
 * parameter equal those of the previous such evaluation (exact equality) and
 * reuse its fine-bin spectra; only the bin stages run (paper: stages are
 * recomputed only when the parameters they depend on change, "Structure of
 * the framework"). Results are those of a full evaluation. Other entry points
 * clear the kept spectra before they run. Returns NF_EINVAL for unknown
 * keys/values.
 */
int nf_set_option(nf_ctx* ctx, const char* key, int64_t value);

/* Current value of an option of nf_set_option (same keys) into *value.
 * NF_EINVAL for unknown keys or null pointers. */
int nf_get_option(nf_ctx* ctx, const char* key, int64_t* value);

/*
 * Autotuner: times the launch choices above on this context's model, events
 * and data (evaluations at theta, P host values, `evals` timed evaluations
 * per candidate, device time from HIP events) and keeps the fastest:
 * tail_threads first, then chunk x fold_block (both skipped when evals = 0);
 * then, if batch > 0 and batch data are set (nf_set_data_batch),
 * batch_fit_tile x batch_threads for batched launches of `batch` fits. In
 * each sweep the current choice is timed first, and a candidate replaces the
 * best so far only when it is more than 1% faster, so timing noise does not
 * move the configuration between equivalent choices. best (nullable): 5
 * values chunk, fold_block, tail_threads, batch_threads, batch_fit_tile.
 * best_us (nullable): 2 values, the mean device time of one evaluation and
 * of one batched evaluation (0 if not tuned), microseconds.
 * Needs events and data. Replaces the options in place.
 */
int nf_autotune(nf_ctx* ctx, const double* theta, int evals, int batch, int64_t* best, double* best_us);

/*
 * Fit options and result (paper: "Structure of the framework" -- minimise
 * -ln L until the estimated distance to the minimum is below a threshold).
 */
#define NF_SURROGATE 1  /* nf_fit_opts.warm_start: starts proposed by the attached surrogate */
typedef struct {
  double edm_tol;   /* stop when EDM = 1/2 g^T H g < edm_tol; <= 0 selects 1e-7     */
  int max_iter;     /* accepted iterations; <= 0 selects 1000                        */
  int want_cov;     /* 1: covariance = inverse of the central-difference Hessian of
                       the adjoint gradient at the minimum (2 evaluations per free
                       parameter), written to result->cov                           */
  int warm_start;   /* 0: every fit starts at its start vector; NF_SURROGATE: the
                       surrogate's input parameters of each start vector are first
                       replaced by the best of its start grid fitted to that fit's
                       observed counts on the surrogate (nf_set_surrogate), and the
                       exact NLL judges: the proposal replaces the start only where
                       it is lower there; the exact fit then runs from the chosen
                       start. NF_ESTATE if no surrogate is attached.                 */
  int pad_;
} nf_fit_opts;

typedef struct {
  double nll;       /* NLL at the returned point (deviance form, see nf_eval_nll)    */
  double edm;       /* estimated distance to the minimum at the returned point       */
  int status;       /* 0 converged, 2 iteration limit, 3 line search failed,
                       4 start point out of domain                                   */
  int iters;        /* accepted iterations                                           */
  int evals;        /* model evaluations (fold + bin stages + gradient)              */
  int pad_;
  double* theta;    /* caller-owned, nf_num_params() values, or NULL                 */
  double* cov;      /* caller-owned P x P row-major, or NULL; zero rows/columns for
                       fixed parameters; NaN when the Hessian is not positive
                       definite                                                      */
} nf_fit_result;

/*
 * Minimise NLL(theta) over the free parameters from `start` (host, P values).
 * fixed: NULL (use the model's "fixed" flags) or P bytes, nonzero = fixed.
 * The minimiser is limited-memory BFGS with a strong-Wolfe line search and
 * runs on the device: each iteration is one evaluation (fold, bin stages,
 * adjoint gradient) followed by the step, captured in a HIP graph and
 * replayed until the device reports convergence. Returns NF_OK (converged),
 * NF_WNOCONV (iteration limit or line-search failure; result filled),
 * NF_WDOMAIN (start point out of domain), or an error. Needs events and data.
 */
int nf_fit(nf_ctx* ctx, const double* start, const uint8_t* fixed, const nf_fit_opts* opts,
           nf_fit_result* result);

/*
 * Attach a surrogate network to a context for warm starts (not in the paper:
 * the learned part proposes start points only; every reported NLL comes from
 * the exact fold). net (caller-owned, must stay alive while attached; NULL
 * detaches) maps x (n_in values) to the standardised log expectations of all
 * analysis bins, concatenated in dataset order (its n_out must equal their
 * total): log mu_j = y_j out_std_j + out_mean_j. Input i is parameter
 * param_index[i] through x_i = (theta_i - center_i) / half_i. A warm start
 * of one fit runs nf_mlp_fit_inputs (surrogate Poisson deviance plus the
 * input prior x_prior, x_weight; `iters` Adam steps of size lr) from each of
 * the n_starts rows of `starts` (n_starts x n_in, in x units) on that fit's
 * observed counts, keeps the row of lowest surrogate deviance, clips it to
 * [-1, 1] and writes center + half x into the fit's start vector. All arrays
 * are copied. NF_EINVAL for bad sizes or indices.
 */
int nf_set_surrogate(nf_ctx* ctx, nf_mlp* net, int n_in, const int* param_index, const double* center,
                     const double* half, const float* out_mean, const float* out_std, const float* x_prior,
                     const float* x_weight, int n_starts, const float* starts, int iters, float lr);

/*
 * Batched pseudo-experiments and scans (paper: parallel fits with individual
 * settings and start values for ensembles and profile-likelihood scans).
 *
 * nf_set_data_batch: nsets observed-count vectors, each the concatenation of
 * all datasets' analysis bins (sum_d nf_num_bins(d) values), row-major.
 * Replaces any previous batch data. Copied; on_device as in nf_set_events.
 */
int nf_set_data_batch(nf_ctx* ctx, int nsets, const double* counts, int on_device);

/*
 * B evaluations in one batched fold (events read once per tile of fits) and
 * one workgroup per fit for the bin stages. theta: B x P (host). data_idx:
 * B rows of the batch data (NULL: row f for fit f). nll: B values (host);
 * grad: B x P (host) or NULL. NF_WDOMAIN when some evaluation is out of domain
 * (its NLL is +inf).
 */
int nf_eval_batch(nf_ctx* ctx, int B, const double* theta, const int* data_idx, double* nll, double* grad);

/*
 * B independent fits (pseudo-experiments or scan points) advanced together:
 * every iteration is one batched fold (fits whose oscillation parameters did
 * not change since their last fold reuse it, so scan points with fixed
 * oscillation parameters fold once), one workgroup per fit for the bin
 * stages, adjoint gradient and L-BFGS step, captured in a HIP graph and
 * replayed until every fit has stopped. start: B x P. fixed: NULL (model's
 * flags) or P bytes shared by all fits. data_idx: as in nf_eval_batch.
 * Outputs (host, each nullable): theta_out B x P, nll_out, edm_out B,
 * status_out, iters_out, evals_out B (status codes as in nf_fit_result).
 * opts->want_cov is ignored. NF_OK when every fit converged, else NF_WNOCONV.
 */
int nf_fit_batch(nf_ctx* ctx, int B, const double* start, const uint8_t* fixed, const int* data_idx,
                 const nf_fit_opts* opts, double* theta_out, double* nll_out, double* edm_out,
                 int* status_out, int* iters_out, int* evals_out);

/*
 * Mixed ensembles (paper: parallel fits of pseudo-experiment ensembles; here
 * ensembles drawn from several models at once, e.g. a single-detector and a
 * three-detector model of uneven bin and parameter counts): the batched fits
 * of n contexts advanced together. Each member is one context with its own
 * batch data (nf_set_data_batch) and the arguments of nf_fit_batch; contexts
 * must be distinct and on one device. Every iteration is one HIP graph that
 * holds every member's batched fold and bin-stage + L-BFGS launches on
 * branches of their own (forked from and joined to the first member's
 * stream, so the members' kernels run side by side), replayed until every fit
 * of every member has stopped; opts (nullable) applies to all members.
 * Results per member as in nf_fit_batch. Returns NF_OK when every fit
 * converged, NF_WNOCONV when some did not (first member's nf_last_error), or
 * the error of the first member whose arguments are invalid (on that
 * member's context).
 */
typedef struct {
  nf_ctx* ctx;
  int B;                    /* fits of this member                                      */
  int pad_;
  const double* start;      /* B x P (P of this member's model), host                   */
  const uint8_t* fixed;     /* NULL or P bytes                                          */
  const int* data_idx;      /* NULL (fit f uses batch row f) or B rows                  */
  double* theta_out;        /* outputs, host, each nullable: B x P, then B values each  */
  double* nll_out;
  double* edm_out;
  int* status_out;
  int* iters_out;
  int* evals_out;
} nf_batch_member;
int nf_fit_batch_group(int n, const nf_batch_member* members, const nf_fit_opts* opts);

/*
 * Expected counts mu (Eq. 3-5: signal from the fold and bin stages plus
 * backgrounds) for B parameter vectors in one batched launch. Rows whose
 * oscillation parameters are equal share one event fold, so a set of
 * nuisance-parameter draws at one oscillation point reads the events once.
 * theta: B x P (host); mu: B x (sum_d nf_num_bins(d)) (host), datasets
 * concatenated. Needs events (not data). NF_WDOMAIN when some row is out of
 * domain (its mu is not meaningful).
 */
int nf_expected_batch(nf_ctx* ctx, int B, const double* theta, double* mu);

/*
 * Per-kernel device time, measured with HIP start and stop events carried by
 * the fold and the bin-stage kernel dispatches themselves (hipExtLaunchKernel:
 * the events take each kernel's own start and end times) for every
 * evaluation enqueued by nf_eval_* while option "timing" is 1. nf_timing synchronises the stream and returns, for the
 * evaluations enqueued since the last reset: their count, the summed fold
 * time and the summed bin-stage time (ms). reset != 0 starts a new window.
 */
int nf_timing(nf_ctx* ctx, int reset, int64_t* count, double* fold_ms, double* tail_ms);

/*
 * Mean time (microseconds, over n samples) between two timing events recorded
 * back to back on the context stream with no work between them: the fixed
 * cost (event packets, dispatch and completion of the timed launch) that is
 * included in every per-kernel duration nf_timing reports. Synchronises.
 */
int nf_timing_overhead(nf_ctx* ctx, int n, double* us);

/*
 * ---------------------------------------------------------------------------
 * Surrogate: a dense network  x (n_in) -> [Linear -> GELU] x depth -> Linear
 * -> y (n_out)  that maps a subset of the parameters to the (standardised)
 * log expectations of the analysis bins. It only proposes start points for
 * fits; every NLL the library reports comes from the exact fold above.
 * Layer l has weights W_l (d_in x d_out, row-major) and bias b_l (d_out);
 * the flat parameter vector is W_0, b_0, W_1, b_1, ... in that order.
 * GELU(z) = z Phi(z) with the exact normal CDF. Matrix products run on the
 * matrix cores with BF16 operands (weights, activations and back-propagated
 * gradients rounded to BF16, round-to-nearest-even) and FP32 accumulation;
 * biases, pre-activations, master weights and optimiser state are FP32.
 * Each handle owns its device memory and is used by one host thread at a time.
 * Host-pointer calls are synchronous. Return codes as above.
 */

/* Create a network; parameters start at zero (set them with nf_mlp_set_params).
 * max_batch bounds B in every call. hip_stream as in nf_create. */
int nf_mlp_create(nf_mlp** out, int n_in, int width, int depth, int n_out, int max_batch, void* hip_stream);
void nf_mlp_destroy(nf_mlp* net);
const char* nf_mlp_last_error(const nf_mlp* net);  /* NULL net: error of the last failed create */
int64_t nf_mlp_num_params(const nf_mlp* net);

/* Copy the flat FP32 parameter vector in (also resets the optimiser state) or out. */
int nf_mlp_set_params(nf_mlp* net, const float* params);
int nf_mlp_get_params(nf_mlp* net, float* params);

/* y = f(x) for B rows: x B x n_in, y B x n_out, FP32, host (on_device = 0)
 * or device pointers (on_device = 1). */
int nf_mlp_forward(nf_mlp* net, int B, const float* x, float* y, int on_device);

/* Back-propagation of dy = dL/dy (B x n_out) at x: grad (nullable) receives
 * dL/d(parameters) in the flat layout, dx (nullable) dL/dx (B x n_in). */
int nf_mlp_grad(nf_mlp* net, int B, const float* x, const float* dy, float* grad, float* dx, int on_device);

/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8, bias-corrected) on the
 * mean squared error  L = sum (y - t)^2 / (B n_out)  of the batch x -> t.
 * loss (nullable, host) receives L before the step. With device pointers and
 * loss NULL the step is only enqueued on the network's stream. */
int nf_mlp_train_step(nf_mlp* net, int B, const float* x, const float* t, float lr, float* loss, int on_device);

/* Training steps as replays of one captured HIP graph per batch size (on,
 * the default) or as separate launches (on = 0). Both run the same kernels on
 * the same buffers and give bit-identical results; the graph saves the
 * launch overhead of the step's ~40 kernels. Changing B re-captures.
 * Returns NF_OK or NF_EINVAL (null net). */
int nf_mlp_use_graphs(nf_mlp* net, int on);

/* Warm start: for each of B rows, minimise over the inputs x the surrogate
 * Poisson deviance  sum_j [mu_j - n_j + n_j ln(n_j / mu_j)],
 * mu_j = exp(y_j out_std_j + out_mean_j), plus the Gaussian input prior
 * 1/2 sum_i x_weight_i (x_i - x_prior_i)^2, by `iters` Adam steps of size lr
 * on all rows at once. x: B x n_in (host, in: start, out: result); nobs: B x
 * n_out observed counts; out_mean, out_std: n_out; x_prior, x_weight: n_in;
 * nll (nullable): B values of the objective at the returned x. */
int nf_mlp_fit_inputs(nf_mlp* net, int B, float* x, const float* nobs, const float* out_mean,
                      const float* out_std, const float* x_prior, const float* x_weight, int iters, float lr,
                      float* nll);

#ifdef __cplusplus
}
#endif
#endif /* NUFOLD_H */
