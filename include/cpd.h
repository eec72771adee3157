/*
 * cpd.h - C ABI of libcpdmi, block-randomized SGD with importance sampling
 * for CP tensor decomposition on AMD Instinct MI355X (gfx950).
 *
 * The method (Yu & Li, "A block-randomized stochastic method with importance
 * sampling for CP tensor decomposition"): every step draws a mode n uniformly,
 * samples B rows of the Khatri-Rao product Z^(n) by drawing one row of every
 * other factor independently from that factor's leverage-score or
 * squared-row-norm distribution (Section 3.1, Lemmas 2 and 4, Algorithm 3),
 * gathers the matching mode-n fibres of the tensor (Algorithm 1), forms the
 * sampled KRP rows H as Hadamard products of the gathered factor rows, and
 * applies the reweighted stochastic gradient
 *     G = A^(n) (H^T W H) - X_s^T W H,   W = diag(1 / (B p_f))
 * (Section 3.2) with a fixed, decreasing (Theorem 9) or AdaGrad step
 * (Algorithms 4 and 5).  Convergence is measured by fit = 1 - Tol with Tol the
 * squared relative error of Section 5.2.
 *
 * Conventions
 *   - Every call returns a cpd_status: 0 = OK, > 0 informational, < 0 error.
 *     Nothing aborts or throws across this interface.  cpd_last_error()
 *     returns a thread-local message for the last failing call of the thread.
 *   - Indices are 0-based.  Mode k has size dims[k].
 *   - The dense input tensor is stored with mode 1 varying fastest: entry
 *     (i_0, ..., i_{N-1}) sits at offset i_0 + dims[0]*(i_1 + dims[1]*(...)),
 *     the order in which the paper's mode-n unfolding map enumerates entries.
 *   - Factor matrices are dims[k] x R, row-major (the R values of one row are
 *     contiguous), FP32.
 *   - Device pointers belong to the HIP device that is current when the call
 *     is made; a handle remembers its device and stream.
 *   - A handle is not thread-safe.  Distinct handles on distinct streams may
 *     be driven concurrently from distinct threads.
 */
#ifndef CPD_H
#define CPD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#if defined(__GNUC__)
#define CPD_API __attribute__((visibility("default")))
#else
#define CPD_API
#endif

#define CPD_MAX_MODES 8
#define CPD_MAX_RANK 128             /* up to 64 on every path; 65..128 on the grid path
                                        (CPD_PATH_AUTO picks it) with the Euclidean or
                                        uniform sampler; batches, the server and
                                        cpd_variance take R <= 64 */
#define CPD_MAX_BATCH 1048576
#define CPD_MAX_PERSISTENT_BATCH 4096  /* largest B of the one-workgroup step */
#define CPD_MAX_DIM 4096

typedef int32_t cpd_status;

enum {
  CPD_OK = 0,
  CPD_PENDING = 1,              /* cpd_poll: request not finished yet */
  CPD_E_INVALID = -1,           /* bad argument or unsupported size */
  CPD_E_OOM = -2,               /* workspace too small / can never fit */
  CPD_E_HIP = -3,               /* a HIP runtime call failed */
  CPD_E_RANK_DEFICIENT = -4,    /* leverage scores of a rank-deficient factor */
  CPD_E_DEGENERATE = -5,        /* all sampling weights of a factor are zero */
  CPD_E_DIVERGED = -6,          /* a factor became non-finite */
  CPD_E_QUEUE_FULL = -7,        /* serving: admission queue is full */
  CPD_E_NOT_FOUND = -8,         /* serving: unknown ticket */
  CPD_E_CANCELLED = -9          /* serving: request cancelled */
};

/* Row distributions of Section 3.1 (uniform is the BrasCPD / AdasCPD arm). */
enum { CPD_SAMPLER_UNIFORM = 0, CPD_SAMPLER_LEVERAGE = 1, CPD_SAMPLER_EUCLIDEAN = 2 };

/* Step rules: fixed alpha (Algorithm 4), AdaGrad (Algorithm 5), and the
 * decreasing alpha_t = beta / (t + gamma) of Theorem 9. */
enum { CPD_RULE_FIXED = 0, CPD_RULE_ADAGRAD = 1, CPD_RULE_DECREASING = 2 };

enum { CPD_F32 = 0, CPD_BF16 = 1, CPD_F64 = 2 };

/* Execution of one step.  PERSISTENT: one workgroup runs many steps in one
 * launch, every phase in its LDS (B <= CPD_MAX_PERSISTENT_BATCH and the
 * step's LDS within 160 KiB).  GRID: every step is three launches over the
 * whole GPU (the fibre gather and contraction split over blocks of up to
 * 512 fibres, a fixed-order sum of the block parts with the update, the
 * CDF refresh), for mini-batches too large for one workgroup.  AUTO picks
 * PERSISTENT when it fits.  Both draw the same indices from the same
 * Philox stream and CDFs; their iterates differ only in FP32 summation
 * order.  Batched and served decompositions use PERSISTENT. */
enum { CPD_PATH_AUTO = 0, CPD_PATH_PERSISTENT = 1, CPD_PATH_GRID = 2 };
enum { CPD_HOST = 0, CPD_DEVICE = 1 };

typedef struct cpd_problem {
  int32_t N;                       /* number of modes, 2..CPD_MAX_MODES */
  int32_t dims[CPD_MAX_MODES];     /* mode sizes, 1..CPD_MAX_DIM */
  int32_t R;                       /* rank, 1..CPD_MAX_RANK */
  int32_t B;                       /* mini-batch size |F_n|, 1..CPD_MAX_BATCH */
  uint64_t seed;                   /* Philox key word 0 */
  uint64_t stream_id;              /* Philox key word 1 */
} cpd_problem;

typedef struct cpd_options {
  int32_t sampler;                 /* CPD_SAMPLER_* */
  int32_t rule;                    /* CPD_RULE_* */
  double alpha;                    /* fixed step */
  double eta;                      /* AdaGrad base step */
  double b;                        /* AdaGrad offset (0 allowed) */
  double beta, gamma;              /* decreasing step alpha_t = beta/(t+gamma) */
  int32_t storage;                 /* tensor storage: CPD_F32 or CPD_BF16 */
  int32_t nonneg;                  /* 1: project the updated factor onto A >= 0 */
  int32_t fit_every;               /* steps between fit checks (serving/batch) */
  double fit_target;               /* stop when fit >= target (serving/batch) */
  int64_t max_steps;               /* stop after this many steps (serving/batch) */
  int32_t ksplit[CPD_MAX_MODES];   /* tile choice of the mode-k contraction: the number
                                      of parts its fibre range is split into across
                                      waves (0 = library default; see
                                      cpd_batch_member_info).  Results depend on it
                                      only through the FP32 summation order. */
  int32_t path;                    /* how a step is executed: CPD_PATH_* */
  int32_t rescale_every;           /* k > 0: after every step that brings the step
                                      counter t to a multiple of k, rescale the factor
                                      columns as cpd_rescale does (single handles
                                      only); 0 = never */
} cpd_options;

typedef struct cpd_handle cpd_handle;

/* Thread-local message describing the last error of the calling thread. */
CPD_API const char* cpd_last_error(void);

/* Library version string. */
CPD_API const char* cpd_version(void);

/*
 * cpd_workspace_size: device bytes that cpd_init needs for this problem
 * (N mode-major copies of the tensor, factors, AdaGrad accumulators, CDFs,
 * host-input staging and scratch).  Pure; no device call.
 * Errors: CPD_E_INVALID for sizes outside the limits above.
 */
CPD_API cpd_status cpd_workspace_size(const cpd_problem* p, const cpd_options* o, size_t* bytes);

/*
 * cpd_init: bind a decomposition to a caller-owned device workspace.
 *   X        dense tensor (layout above), element type x_dtype (CPD_F32 or
 *            CPD_F64), in host memory (x_space = CPD_HOST) or on the device.
 *            It is rounded to the storage type (FP32 round-to-nearest, then
 *            BF16 round-to-nearest-even) and written as N copies, copy n
 *            holding the mode-n fibres as contiguous rows (row j = the
 *            unfolding column j of the Section 1 index map).
 *   A0       N host pointers, A0[k] is dims[k] x R row-major FP32.
 *   ws       device memory of at least cpd_workspace_size bytes, 256-byte
 *            aligned; owned by the caller and must outlive the handle.
 *   stream   hipStream_t (NULL = the default stream) on which all work of
 *            the handle is enqueued.
 * Returns after the tensor and factors are in ws, so X and A0 may be freed.
 * Errors: CPD_E_INVALID, CPD_E_OOM (ws too small), CPD_E_HIP,
 *         CPD_E_RANK_DEFICIENT / CPD_E_DEGENERATE (initial distributions).
 */
CPD_API cpd_status cpd_init(const cpd_problem* p, const cpd_options* o, const void* X, int32_t x_dtype,
                    int32_t x_space, const float* const* A0, void* ws, size_t ws_bytes,
                    void* stream, cpd_handle** out);

/*
 * cpd_sample: the mini-batch that step t would draw with the current factors
 * (Algorithm 3): mode n, idx (device, B x (N-1) int32, row f = the sampled
 * row indices of the modes k != n in ascending k) and p (device, B doubles,
 * p_f = prod_k q_k(i_k)/Q_k).  No state changes.  Synchronous.
 * Errors: CPD_E_INVALID, CPD_E_HIP, or a sticky error of the handle.
 */
CPD_API cpd_status cpd_sample(cpd_handle* h, uint64_t t, int32_t* mode, int32_t* idx_dev, double* p_dev);

/*
 * cpd_step: enqueue nsteps steps (t .. t+nsteps-1) on the handle's stream
 * (one persistent launch, or three launches per step on the GRID path).
 * With rescale_every = k > 0 the steps run in stretches that end where t
 * reaches a multiple of k, each followed by the two launches of
 * cpd_rescale.  Asynchronous: a non-finite factor or a sampling failure is
 * recorded on the device and reported by the next synchronising call
 * (cpd_sync, cpd_fit, cpd_read_*).
 */
CPD_API cpd_status cpd_step(cpd_handle* h, int64_t nsteps);

/*
 * cpd_step_replay: one step with caller-supplied mode and indices (device
 * idx_dev as returned by cpd_sample); the probabilities come from the
 * handle's current distributions.  Asynchronous like cpd_step.
 */
CPD_API cpd_status cpd_step_replay(cpd_handle* h, int32_t mode, const int32_t* idx_dev);

/*
 * cpd_rescale: rescale the factor columns in place (the remark after the
 * fixed-step error bound, Section 4.2, suggests scaling the factors after
 * each iteration to keep them bounded; it gives no formula).  For every
 * rank component r whose N column norms nu_k = ||A^(k)(:, r)|| are positive
 * and finite, column r of factor k is multiplied by g / nu_k with g the
 * geometric mean of the nu_k, so the CP model [[A]] is unchanged.  Other
 * components are left as they are; the AdaGrad accumulators are not
 * touched.  The sampling distributions of every mode are then rebuilt from
 * the rescaled factors.  Norms and scales in FP64, factors in FP32.
 * Asynchronous on the handle's stream; does nothing once the handle holds
 * an error status.  Errors: CPD_E_INVALID (null handle), CPD_E_HIP.
 */
CPD_API cpd_status cpd_rescale(cpd_handle* h);

/* Wait for the handle's stream; returns the handle's sticky device status. */
CPD_API cpd_status cpd_sync(cpd_handle* h);

/*
 * cpd_fit: fit = 1 - ||X - [[A]]||^2 / ||X||^2 of the stored tensor, in FP64
 * (Gram-Hadamard form for ||[[A]]||^2, one streaming pass for <X, [[A]]>).
 * Synchronous.
 */
CPD_API cpd_status cpd_fit(cpd_handle* h, double* fit);

/* Current step counter t. */
CPD_API cpd_status cpd_get_step(cpd_handle* h, int64_t* t);

/* Copy factor n (dims[n] x R FP32) to dst in host or device memory. Synchronous. */
CPD_API cpd_status cpd_read_factors(cpd_handle* h, int32_t n, float* dst, int32_t dst_space);

/* Copy the integer-valued FP64 CDF of mode n (dims[n] doubles) to host dst. */
CPD_API cpd_status cpd_read_cdf(cpd_handle* h, int32_t n, double* dst);

/*
 * cpd_read_state / cpd_write_state: serialise {t, factors, AdaGrad
 * accumulators} to a host buffer.  With buf == NULL, *bytes receives the
 * size.  Writing a state recomputes the distributions, so a run resumed from
 * a state continues bit for bit.
 */
CPD_API cpd_status cpd_read_state(cpd_handle* h, void* buf, size_t* bytes);
CPD_API cpd_status cpd_write_state(cpd_handle* h, const void* buf, size_t bytes);

/*
 * cpd_variance: the exact variance of the sampled gradient of mode n at the
 * current factors, for mini-batches of the handle's B drawn by `sampler`
 * (any of the three, independent of the handle's own), from the variance
 * theorem of Section 4 (Table 1 lists its per-sampler forms):
 *   out[0] = E ||G - grad f||_F^2
 *          = (1/B) (sum_j ||r_j||^2 ||z_j||^2 / p_j - ||grad f||_F^2),
 *   out[1] = (1/B) sum_j ||r_j||^2 ||z_j||^2 / p_j,
 *   out[2] = (1/B) ||grad f||_F^2,
 * with z_j row j of the Khatri-Rao product Z^(n), r_j = A^(n) z_j - x_j the
 * residual of fibre j, p_j = prod_{k != n} q_k(i_k) / Q_k the probability of
 * the integer-valued distributions the sampler builds from the current
 * factors, and grad f = A^(n) (hadamard_{k != n} A^(k)T A^(k)) - X_(n) Z^(n).
 * One pass over copy n; FP32 products, FP64 sums.
 *   ws        caller-owned device scratch of at least
 *             cpd_variance_workspace_size(h, n) bytes, 256-byte aligned,
 *             used only during the call (no allocation inside the call).
 * Synchronous on the handle's stream.  The handle's state is not changed.
 * Errors: CPD_E_INVALID, CPD_E_OOM (ws too small), CPD_E_RANK_DEFICIENT
 * (leverage), CPD_E_HIP.
 */
CPD_API cpd_status cpd_variance_workspace_size(cpd_handle* h, int32_t n, size_t* bytes);
CPD_API cpd_status cpd_variance(cpd_handle* h, int32_t n, int32_t sampler, void* ws, size_t ws_bytes,
                                double* out);

/*
 * cpd_variance_noalloc: cpd_variance without a scratch argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, serving
 * loops, harnesses that forbid allocation).  It allocates nothing: its
 * scratch is one static array of the library per device (20 MiB, held from
 * the first call on that device until the process ends), which covers every
 * problem within this header's limits (the request is refused with
 * CPD_E_INVALID if a mode's scratch ever exceeded it).  Results are those of
 * cpd_variance bit for bit.  All calls on one device share that array, which
 * keeps the last call's contents: calls that overlap on one device (from
 * different threads or streams) race and must be serialised by the caller.
 * Synchronous on the handle's stream.  Errors as cpd_variance.
 */
CPD_API cpd_status cpd_variance_noalloc(cpd_handle* h, int32_t n, int32_t sampler, double* out);

/* Release the handle (the workspace stays the caller's). */
CPD_API cpd_status cpd_destroy(cpd_handle* h);

/* ------------------------------------------------------------------------
 * Batched decompositions: many independent problems (different sizes,
 * ranks, samplers) advanced together, one persistent workgroup per problem,
 * every member in the same launch (one launch per 16-column rank-tile class,
 * run concurrently).  Each member runs exactly the computation of a single
 * handle created with the same problem and options (including the ksplit
 * the batch reports), so its results are those of that handle, bit for bit.
 * Members stop on their own: after a fit check with fit >= fit_target, or
 * once t reaches max_steps (options of that member).
 * ------------------------------------------------------------------------ */
typedef struct cpd_batch cpd_batch;

typedef struct cpd_member_info {
  int64_t t;                      /* steps taken */
  double fit;                     /* last fit check */
  int32_t done;                   /* stopped (target fit, step limit or error) */
  cpd_status status;              /* sticky device status of the member */
  int64_t t_done;                 /* t at the check that stopped it */
  double seconds_done;            /* device time from its first distributions to that check */
  int32_t ksplit[CPD_MAX_MODES];  /* tile choice used for each mode */
} cpd_member_info;

/* Device bytes cpd_batch_create needs for these members. */
CPD_API cpd_status cpd_batch_workspace_size(const cpd_problem* ps, const cpd_options* os,
                                            int32_t count, size_t* bytes);

/*
 * cpd_batch_create: count members, problem ps[i] with options os[i].
 *   X[i]        member i's dense tensor (layout as cpd_init), all of element
 *               type x_dtype in space x_space.
 *   A0          count * CPD_MAX_MODES host pointers: A0[i*CPD_MAX_MODES + k]
 *               is member i's initial factor k (dims[k] x R FP32).
 *   ws          caller-owned device workspace of cpd_batch_workspace_size
 *               bytes, 256-byte aligned; must outlive the batch.
 *   tune        1: time the candidate tile choices (ksplit) of every mode on
 *               the members themselves, keep the fastest, then restart each
 *               member from A0.  Choices are cached per (mode size, rank, B,
 *               storage) for the life of the process.  0: library defaults
 *               (or os[i].ksplit where given).
 * All members must share os[i].fit_every (the round length).
 * Errors: as cpd_init, per member (the message names it).
 */
CPD_API cpd_status cpd_batch_create(const cpd_problem* ps, const cpd_options* os, int32_t count,
                                    const void* const* X, int32_t x_dtype, int32_t x_space,
                                    const float* const* A0, void* ws, size_t ws_bytes,
                                    void* stream, int32_t tune, cpd_batch** out);

/* Every member not yet done advances nsteps (capped at its max_steps).  Async. */
CPD_API cpd_status cpd_batch_step(cpd_batch* b, int64_t nsteps);

/*
 * cpd_batch_fits: fit check of every member not yet done (one launch for all),
 * marking members that reach their target as done; fits[i] receives member
 * i's last fit.  Synchronous.
 */
CPD_API cpd_status cpd_batch_fits(cpd_batch* b, double* fits);

/*
 * cpd_batch_run: replay rounds of {fit_every steps of every member, fit
 * check of every member} from a captured HIP graph until every member is
 * done or max_rounds rounds ran.  *remaining receives the number of members
 * not done.  Synchronous.
 */
CPD_API cpd_status cpd_batch_run(cpd_batch* b, int64_t max_rounds, int32_t* remaining);

/* Wait for the batch's work; returns the first member error, else CPD_OK. */
CPD_API cpd_status cpd_batch_sync(cpd_batch* b);

/* Member i's counters and tile choices.  Synchronous. */
CPD_API cpd_status cpd_batch_member_info(cpd_batch* b, int32_t i, cpd_member_info* out);

/* Copy member i's factor n to dst (host or device).  Synchronous. */
CPD_API cpd_status cpd_batch_read_factors(cpd_batch* b, int32_t i, int32_t n, float* dst,
                                          int32_t dst_space);

/* Release the batch (the workspace stays the caller's). */
CPD_API cpd_status cpd_batch_destroy(cpd_batch* b);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.  Requests wait in a
 * queue; a request is admitted as soon as a slot is free and its workspace
 * (cpd_workspace_size bytes) fits in the free part of the server's arena.
 * Admission (tensor layout, distributions) runs on its own stream while the
 * admitted requests step, so newcomers join the running set at the next
 * round; a round is round_steps steps of every admitted request followed by
 * one fit check of all of them.  A request leaves when its fit reaches
 * options.fit_target or its t reaches options.max_steps; its factors are
 * copied out and its slot and arena space are reused.  Each request runs
 * exactly the computation of a single handle stepped in rounds of
 * round_steps with a fit check after each round, so its result does not
 * depend on the other requests in the mix.
 * ------------------------------------------------------------------------ */
typedef struct cpd_server cpd_server;

typedef struct cpd_server_config {
  int32_t max_slots;        /* requests on the device at once, 1..4096 */
  int32_t queue_capacity;   /* waiting requests beyond which cpd_submit refuses */
  int32_t round_steps;      /* steps per round = steps between fit checks, >= 1 */
  int32_t pad;
} cpd_server_config;

typedef struct cpd_request {
  cpd_problem problem;
  cpd_options options;            /* fit_every is ignored (round_steps applies) */
  const void* X;                  /* dense tensor (layout as cpd_init).  A device X is
                                     read at admission on the server's own stream, which
                                     is not ordered after any stream of the caller: the
                                     caller completes every write to X (e.g. synchronises
                                     the stream that produced it) before cpd_submit */
  int32_t x_dtype;                /* CPD_F32 or CPD_F64 */
  int32_t x_space;                /* CPD_HOST or CPD_DEVICE (current device) */
  const float* A0[CPD_MAX_MODES]; /* initial factors, host */
  float* out[CPD_MAX_MODES];      /* host buffers for the final factors (NULL: not copied) */
} cpd_request;

typedef struct cpd_result {
  cpd_status status;          /* CPD_OK, or the request's error */
  int32_t reached;            /* 1 if fit >= fit_target */
  double fit;                 /* fit at the last check */
  int64_t steps;              /* steps taken */
  double seconds_queued;      /* submit -> admission started (host clock) */
  double seconds_admit;       /* admission (layout, distributions) */
  double seconds_to_fit;      /* first distributions -> stopping check (device clock) */
  double seconds_total;       /* submit -> result available (host clock) */
} cpd_result;

/*
 * cpd_server_create: start the request loop on the current device.  arena is
 * caller-owned device memory (256-byte aligned) from which admitted requests
 * get their workspaces; it must outlive the server.  stream is ignored (the
 * server owns its streams).
 */
CPD_API cpd_status cpd_server_create(const cpd_server_config* cfg, void* arena, size_t arena_bytes,
                                     cpd_server** out);

/*
 * cpd_submit: queue a request.  X, A0 and the out buffers must stay valid
 * until cpd_poll reports a final status for the ticket.
 * Errors: CPD_E_INVALID (bad problem), CPD_E_OOM (its workspace can never fit
 * in the arena), CPD_E_QUEUE_FULL.
 */
CPD_API cpd_status cpd_submit(cpd_server* s, const cpd_request* r, uint64_t* ticket);

/*
 * cpd_poll: non-blocking.  CPD_PENDING while the request waits or runs;
 * otherwise fills *out, forgets the ticket and returns CPD_OK.
 * CPD_E_NOT_FOUND for an unknown (or already collected) ticket.
 */
CPD_API cpd_status cpd_poll(cpd_server* s, uint64_t ticket, cpd_result* out);

/* Counters: requests waiting, running, finished and not yet collected. */
CPD_API cpd_status cpd_server_stats(cpd_server* s, int32_t* waiting, int32_t* running,
                                    int32_t* finished);

/*
 * cpd_server_destroy: stop the loop.  Running requests are abandoned;
 * uncollected results are dropped.
 */
CPD_API cpd_status cpd_server_destroy(cpd_server* s);

#ifdef __cplusplus
}
#endif

#endif /* CPD_H */
