/*
 * hawkes.h -- C ABI of the MI355X (gfx950) library for the exact
 * log-likelihood of the multivariate linear exponential Hawkes process and
 * its gradient, evaluated as a parallel scan of affine transition maps.
 *
 * Paper: "Massively Parallel Exact Inference for Hawkes Processes"
 * (arXiv 2604.01342).
 *
 *   Intensity (Background, eq. 1), K decay kernels:
 *     lambda_p(t) = mu_p + sum_k sum_{j : t_j < t} alpha[k][p][m_j] * beta_k * exp(-beta_k (t - t_j))
 *   with one decay per kernel shared by every node (HAWKES_BETA_SHARED,
 *   beta[k] is the paper's gamma_k), or, with K = 1, one decay per target
 *   node, beta_p in place of beta_k (HAWKES_BETA_PER_TARGET).
 *   Log-likelihood (eq. 2):
 *     L = sum_i log lambda_{m_i}(t_i) - sum_p int_0^T lambda_p(t) dt
 *   Gradients: eqs. 8, 9, 10 (Appendix "Parameter Gradient Formulas").
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  - All array arguments are DEVICE pointers owned by the caller (for example
 *    PyTorch tensors).  The library allocates nothing: scratch space is the
 *    caller's `workspace` (size from the matching *_workspace_bytes query,
 *    256-byte aligned, contents need not be initialised).
 *  - Calls are asynchronous and ordered on `stream`; they neither synchronise
 *    with the host nor read device memory from the host, so they can be
 *    captured into a HIP graph.  Two calls that share a workspace must be
 *    ordered on one stream.
 *  - Layouts: t[n] float64, nondecreasing, 0 <= t[i] <= T; marks[n] int32 in
 *    [0, m); mu[m] float32; alpha[k*m*m] float32, kernel-major then
 *    row-major, alpha[(k*m + p)*m + q] is the excitation of target p by a
 *    source event of node q through kernel k (eq. 1 uses alpha_{p, m_j});
 *    beta[k] (shared decay) or beta[m] (per target, k = 1) float32 (> 0).
 *  - Ties: events with equal time stamps excite later events in index order,
 *    which is what the recurrence of eq. 4 computes.
 *  - Outputs are float64: loglik[1], g_mu[m], g_alpha[k*m*m] (same layout as
 *    alpha), g_beta[k] (shared) or g_beta[m] (per target).  Any gradient
 *    pointer may be NULL to skip that output.
 *  - Precision: time differences are formed in float64.  The forward pass
 *    (state, decays, intensities, log-likelihood and the dL/dmu, dL/dbeta
 *    terms) is float64 in every mode.  The dense dL/dalpha kernels keep a
 *    float64 state and float64 accumulators with float32 decay factors
 *    (each exponent is formed and range-reduced in float64).
 *    Every sum over events (log-likelihood, gradients) is accumulated in
 *    float64 in a fixed order, so repeated calls return bitwise-identical
 *    results, with one exception: in the large-M engine, dL/dalpha sums its
 *    terms through LDS atomics of several waves, whose order (hence
 *    last-bit rounding) can vary between calls.
 *  - Size limits (LDS per workgroup, read from the device; 160 KiB on
 *    MI355X, of which the shared-decay forward kernel keeps 2 KiB for
 *    itself): shared decay m <= 6741, decay per target m <= 4352; larger m
 *    returns HAWKES_EUNSUPPORTED.  The workspace of every large-M call is
 *    independent of n (the events are taken in chunks).
 *  - Errors: every function returns a hawkes_status.  Host-detectable
 *    argument errors return HAWKES_EINVAL (or HAWKES_EWORKSPACE for a short
 *    workspace) before anything is launched, and the outputs are untouched.
 *    Data-dependent preconditions (sorted times, marks in range, positive
 *    parameters) are not checked by the compute calls: violating them gives
 *    meaningless numbers but never an out-of-bounds access (marks are clamped
 *    for addressing).  hawkes_check_inputs() checks them on the device.
 *    A failed kernel launch returns HAWKES_EDEVICE.
 */
#ifndef HAWKES_H
#define HAWKES_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

#define HAWKES_ABI_VERSION 5

/* Decay kernels per problem (hawkes_problem.k), shared-decay mode. */
#define HAWKES_MAX_KERNELS 8

typedef enum hawkes_status {
    HAWKES_OK = 0,
    HAWKES_EINVAL = 1,        /* bad argument (NULL pointer, size, mode) */
    HAWKES_EWORKSPACE = 2,    /* workspace NULL or smaller than required */
    HAWKES_EDEVICE = 3,       /* a HIP call or kernel launch failed */
    HAWKES_EUNSUPPORTED = 4   /* valid request this build does not implement (m above the limits) */
} hawkes_status;

typedef enum hawkes_beta_mode {
    HAWKES_BETA_SHARED = 0,     /* beta[k]: one decay per kernel for every target (eq. 1) */
    HAWKES_BETA_PER_TARGET = 1  /* beta[m]: decay beta_p of the target's kernel (k = 1) */
} hawkes_beta_mode;

/* One event sequence.  `chunk_log2` selects constant-memory processing: the
 * sequence is evaluated in consecutive chunks of 2^chunk_log2 events, each
 * carrying only an M-vector state into the next (the batching of the
 * "Time Complexity Analysis and Batching" section and Algorithm 2), so the
 * workspace does not grow with n (except the per-target gradient's 4 bytes
 * per event, see above).  0 selects the default (2^20).  Valid range 12..26. */
typedef struct hawkes_problem {
    int64_t n;           /* number of events, >= 0 */
    int32_t m;           /* number of nodes M, >= 1 */
    int32_t k;           /* number of decay kernels, 1..HAWKES_MAX_KERNELS (1 with
                            HAWKES_BETA_PER_TARGET; otherwise HAWKES_EINVAL) */
    int32_t beta_mode;   /* hawkes_beta_mode */
    int32_t chunk_log2;  /* 0 = default */
    double  T;           /* window end, >= 0 and >= t[n-1] */
} hawkes_problem;

/* Launch parameters that an autotuner may choose; 0 keeps the library's own
 * rule.  They change how the work is laid out, never what is computed:
 * results agree to rounding whatever the values.  Process-wide:
 * hawkes_set_tuning() applies to every later call, the workspace queries
 * included, whose sizes depend on it (query again after changing it; a call
 * whose workspace was sized under other values returns HAWKES_EWORKSPACE if
 * it is too small).  Set it between calls, not while calls run on other
 * threads.  Intended for callers that time candidate values on their own
 * inputs, as the Python package's autotuner does.
 *   dense_cols    shared-decay large-M engine: width in nodes of the tiles of
 *                 the dense dL/dalpha kernel: 64, 128 or 256 (128 needs
 *                 chunk_log2 <= 25 and 256 <= 24; otherwise the library's
 *                 rule applies)
 *   dense_ranges  the same kernel: event ranges per chunk, each with its own
 *                 partial sums: a power of two, 1..4096 (fewer if a chunk
 *                 has fewer segments)
 *   item_log2     small-M engine: log2 of the events per lane item, 4..16; a
 *                 value too small for the engine's bound on the item count
 *                 (and so on its workspace) is raised to the smallest that
 *                 fits
 *   dense_rows    the dense dL/dalpha kernel's tile height: 16 (float64
 *                 register accumulators) or 32 (float32 register
 *                 accumulators added to a float64 tile every few windows);
 *                 32 applies only with 256-column tiles and 128-record
 *                 windows (M > 128, chunk_log2 <= 24) */
typedef struct hawkes_tuning {
    int32_t dense_cols;
    int32_t dense_ranges;
    int32_t item_log2;
    int32_t dense_rows;
} hawkes_tuning;

/* Replace the process-wide tuning (NULL: all zero, the library's rules).
 * HAWKES_EINVAL for a value outside the ranges above; the tuning is then
 * unchanged. */
hawkes_status hawkes_set_tuning(const hawkes_tuning* t);

/* Copy the current tuning to *t.  HAWKES_EINVAL if t is NULL. */
hawkes_status hawkes_get_tuning(hawkes_tuning* t);

/* Human-readable name of a status code (static storage). */
const char* hawkes_status_string(hawkes_status s);

/* HAWKES_ABI_VERSION of the loaded library. */
int hawkes_version(void);

/* Workspace bytes needed by hawkes_loglik (with_grad = 0) or
 * hawkes_loglik_grad (with_grad = 1) for problem p; 0 if p is invalid. */
size_t hawkes_workspace_bytes(const hawkes_problem* p, int with_grad);

/* Log-likelihood only (eq. 2).  loglik: device float64[1]. */
hawkes_status hawkes_loglik(const hawkes_problem* p,
                            const double* t, const int32_t* marks,
                            const float* mu, const float* alpha, const float* beta,
                            double* loglik,
                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Log-likelihood and its gradient (eqs. 2, 8, 9, 10).  Outputs overwrite the
 * destination arrays; NULL gradient pointers are skipped. */
hawkes_status hawkes_loglik_grad(const hawkes_problem* p,
                                 const double* t, const int32_t* marks,
                                 const float* mu, const float* alpha, const float* beta,
                                 double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                 void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * computation as hawkes_loglik_grad, with the workspace taken from a fixed
 * device array inside the library (HAWKES_NOALLOC_SCRATCH_BYTES per device,
 * reserved when the library's code is loaded on a device and held until the
 * process ends) instead of a caller argument.  The call allocates nothing:
 * its first call on a device only resolves that array's address there (no
 * allocation); every later call reuses it.  The caller still owns and passes
 * the inputs and outputs, with the layouts and NULL rules of
 * hawkes_loglik_grad (loglik is required).
 * Limit: problems whose hawkes_workspace_bytes(p, 1) exceeds
 * HAWKES_NOALLOC_SCRATCH_BYTES return HAWKES_EWORKSPACE before anything is
 * launched; a smaller chunk_log2 shrinks the workspace of long sequences.
 * Argument errors return what hawkes_loglik_grad returns.
 * Every call on a device shares that device's array, which keeps the last
 * call's contents (each call re-initialises what it needs): calls that may
 * overlap on one device, on different streams or from different threads,
 * race and must be ordered by the caller.
 * ------------------------------------------------------------------------- */
#define HAWKES_NOALLOC_SCRATCH_BYTES (64u << 20)

hawkes_status hawkes_loglik_grad_noalloc(const hawkes_problem* p,
                                         const double* t, const int32_t* marks,
                                         const float* mu, const float* alpha, const float* beta,
                                         double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                         hipStream_t stream);

/* The same, with dL/dalpha restricted to alpha's support, for models with a
 * sparse interaction matrix (the sparse cross-node influence that the
 * penalty of section "Background" aims at; sections "Introduction" and
 * "Conclusion" state the method's compatibility with such optimizations):
 * g_alpha[p][q] is eq. 9 where alpha[p][q] != 0 and 0 elsewhere, so a zero
 * entry of alpha stays a fixed zero under gradient steps.  loglik, g_mu and g_beta equal
 * hawkes_loglik_grad's.  With one shared decay and M > 8 the first term of
 * eq. 9 is summed only over the nonzeros, inside the forward pass (float64
 * atomics: the summation order, and so the last bits, vary between calls),
 * and the dense dL/dalpha kernels do not run; the other configurations
 * compute the dense gradient and zero it off the support.  Same workspace
 * as hawkes_loglik_grad. */
hawkes_status hawkes_loglik_grad_support(const hawkes_problem* p,
                                         const double* t, const int32_t* marks,
                                         const float* mu, const float* alpha, const float* beta,
                                         double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/* Intensities at the events, lambda_out[i] = lambda_{m_i}(t_i) (eq. 1) as
 * float32 (the value the log-likelihood uses).  Same workspace as
 * hawkes_loglik. */
hawkes_status hawkes_intensity(const hawkes_problem* p,
                               const double* t, const int32_t* marks,
                               const float* mu, const float* alpha, const float* beta,
                               float* lambda_out,
                               void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * Maximum-likelihood step (the training loop of Algorithm 1: forward pass,
 * backward pass, optimizer step).  hawkes_adam_step evaluates the
 * log-likelihood and gradient like hawkes_loglik_grad (same workspace size),
 * then applies one projected Adam step to the training objective of
 * section "Background", the per-event negative log-likelihood plus the
 * hinge-l1 sparsity penalty
 *     -L/n + lambda1 * sum_{p != q} alpha_pq 1{alpha_pq < h}
 * (off-diagonal entries only: self-excitation is not penalised), in place
 * on mu, alpha and beta (float32).  The penalty's gradient is lambda1 on the
 * off-diagonal entries below h (compared as float32) and 0 elsewhere;
 * lambda1 = 0 gives the plain per-event NLL.  First and second moments are
 * float32, bias corrections come from a step counter kept in the device
 * state, then mu >= floor_mu, alpha >= 0, beta >= floor_beta.  Flag bits
 * HAWKES_ADAM_LOG_MU, HAWKES_ADAM_LOG_BETA and HAWKES_ADAM_LOG_ALPHA make
 * the step act on log mu, log beta, log alpha instead (gradient of the loss,
 * penalty included, times x; update x <- x e^{-lr step}, then the floor):
 * relative steps, for parameters far smaller than lr.  A zero alpha entry
 * then stays zero (its gradient in log space is 0): the support is fixed.  All gradient
 * outputs are required (they hold the gradient of L, without the penalty,
 * at the parameters before the step; so is loglik).  The call is
 * stream-ordered and host-sync-free, so a whole step can be captured in a
 * HIP graph and replayed; each replay advances the counter.
 * The state (size from hawkes_adam_state_bytes, caller-owned device memory)
 * must be zeroed once with hawkes_adam_init before the first step.
 * ------------------------------------------------------------------------- */
#define HAWKES_ADAM_LOG_MU 1u
#define HAWKES_ADAM_LOG_BETA 2u
#define HAWKES_ADAM_LOG_ALPHA 4u

typedef struct hawkes_adam {
    float lr, beta1, beta2, eps;   /* step size, moment decays, denominator floor */
    float floor_mu, floor_beta;    /* projection bounds (floor_beta > 0) */
    float lambda1, h;              /* penalty weight (>= 0) and hinge point (> 0 when lambda1 > 0) */
    uint32_t flags;                /* HAWKES_ADAM_LOG_* bits; other bits must be 0 */
} hawkes_adam;

size_t hawkes_adam_state_bytes(const hawkes_problem* p);
hawkes_status hawkes_adam_init(const hawkes_problem* p, void* state, size_t state_bytes, hipStream_t stream);
hawkes_status hawkes_adam_step(const hawkes_problem* p, const double* t, const int32_t* marks,
                               float* mu, float* alpha, float* beta, const hawkes_adam* cfg,
                               void* state, size_t state_bytes,
                               double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                               void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * Batched: S independent sequences in one launch sequence (no host sync).
 * Sequence s owns events [ev_off[s], ev_off[s+1]) of t/marks, has m_s[s]
 * nodes, window end T_s[s] and one shared decay beta[s].  Its parameters are
 * packed back to back: mu at sum_{r<s} m_s[r], alpha at sum_{r<s} m_s[r]^2
 * (row-major m_s[s] x m_s[s]); the library computes these offsets on the
 * device.  Outputs use the same packing: loglik[S], g_mu (like mu),
 * g_alpha (like alpha), g_beta[S].
 * Host arguments: S >= 1, n_total = ev_off[S] (the length of t), and
 * max_m >= every m_s[s].
 * With max_m <= 8 every sequence is evaluated by the small-M engine in one
 * stream-ordered launch sequence that neither synchronises nor reads device
 * memory from the host (graph-capturable).  With max_m > 8 the call reads
 * ev_off, m_s and T_s to the host (it SYNCHRONISES the stream and cannot be
 * captured in a graph), evaluates the sequences of at most 8 nodes with the
 * small-M engine and each larger one with the large-M engine (node limit as
 * for hawkes_loglik), one after another on the stream; m_s[s] outside
 * [1, max_m] or offsets outside [0, n_total] then return HAWKES_EINVAL.
 * ------------------------------------------------------------------------- */
size_t hawkes_batched_workspace_bytes(int32_t S, int64_t n_total, int32_t max_m, int with_grad);

hawkes_status hawkes_loglik_batched(int32_t S, int64_t n_total, int32_t max_m,
                                    const int64_t* ev_off, const int32_t* m_s, const double* T_s,
                                    const double* t, const int32_t* marks,
                                    const float* mu, const float* alpha, const float* beta,
                                    double* loglik,
                                    void* workspace, size_t workspace_bytes, hipStream_t stream);

hawkes_status hawkes_loglik_grad_batched(int32_t S, int64_t n_total, int32_t max_m,
                                         const int64_t* ev_off, const int32_t* m_s, const double* T_s,
                                         const double* t, const int32_t* marks,
                                         const float* mu, const float* alpha, const float* beta,
                                         double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                         void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * Simulation (input side, not part of the likelihood path): events of the
 * process on [0, T0] from its branching (cluster) representation, the
 * construction of the paper's synthetic studies (section "Results").  Node
 * p's baseline events form a Poisson process of rate mu_p; every event of
 * node q has Poisson(sum_{k,p} alpha[k][p][q]) children, each of (kernel k,
 * node p) with probability proportional to alpha[k][p][q], delayed by an
 * exponential time of rate beta[k] (HAWKES_BETA_SHARED, k kernels) or
 * beta[p] (HAWKES_BETA_PER_TARGET, k = 1); children after T0 are dropped and
 * generations repeat until none is left.  Parameters use the layouts of
 * hawkes_loglik (device pointers).
 * Output: every event on [0, T0], sorted by time (ties, which have
 * probability zero, keep generation order), in t_out / marks_out (device,
 * capacity entries each); *n_out (host) receives the count.  The result
 * depends only on seed and the parameters (every random number is
 * Philox4x64-10, Salmon et al. 2011, at a counter naming its use).
 * The call SYNCHRONISES with the host (generation sizes are read back), so
 * it cannot be captured in a graph.  If the events exceed capacity it
 * returns HAWKES_EWORKSPACE with *n_out set to a count that already exceeds
 * it: call again with a larger capacity (same seed, same result).
 * Workspace: hawkes_simulate_workspace_bytes(m, k, capacity), about 40 bytes
 * per event of capacity plus 12 bytes per entry of alpha.
 * ------------------------------------------------------------------------- */
size_t hawkes_simulate_workspace_bytes(int32_t m, int32_t k, int64_t capacity);

hawkes_status hawkes_simulate(int32_t m, int32_t k, int32_t beta_mode,
                              const float* mu, const float* alpha, const float* beta,
                              double T0, uint64_t seed, int64_t capacity,
                              double* t_out, int32_t* marks_out, int64_t* n_out,
                              void* workspace, size_t workspace_bytes, hipStream_t stream);

/* The simulator's generator evaluated on the host: out = Philox4x64-10 of
 * counter ctr under key (key[0], key[1]), for checking it against other
 * implementations of the published definition. */
void hawkes_philox4x64_10(const uint64_t ctr[4], const uint64_t key[2], uint64_t out[4]);

/* ----------------------------------------------------------------------------
 * Baseline: the sequential recurrence of the "Sequential Recurrence" section
 * (eqs. 4, 11, 12) evaluated event by event in index order by one
 * workgroup whose lanes own slices of the M-vector state.  Same inputs,
 * outputs, precision and workspace as hawkes_loglik_grad; shared beta only.
 * It exists to measure the parallel scan against; it is not fast.
 * ------------------------------------------------------------------------- */
hawkes_status hawkes_sequential_loglik_grad(const hawkes_problem* p,
                                            const double* t, const int32_t* marks,
                                            const float* mu, const float* alpha, const float* beta,
                                            double* loglik, double* g_mu, double* g_alpha, double* g_beta,
                                            void* workspace, size_t workspace_bytes, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * Device-side input validation.  Writes to *status_out (device int32) the OR
 * of: 1 times not nondecreasing, 2 a mark outside [0,m), 4 a time outside
 * [0,T], 8 mu <= 0 or not finite, 16 alpha < 0 or not finite, 32 beta <= 0
 * or not finite; 0 when all preconditions hold.  Stream-ordered.
 * ------------------------------------------------------------------------- */
hawkes_status hawkes_check_inputs(const hawkes_problem* p,
                                  const double* t, const int32_t* marks,
                                  const float* mu, const float* alpha, const float* beta,
                                  int32_t* status_out, hipStream_t stream);

/* ----------------------------------------------------------------------------
 * Diagnostics: per-kernel device timing.  While enabled, every call records a
 * pair of hipEvents on its stream around each launch of the selected kernels;
 * hawkes_timing_read waits for those events and returns the summed
 * milliseconds and the number of launches of one kernel.
 * hawkes_timing_enable(on): 0 stops recording, a negative value selects every
 * kernel, a positive value is a bit mask of kernel ids (bit k: kernel k), so
 * that a caller can time one kernel without the others' bookkeeping.  Kernel
 * ids:
 *   0 dense dL/dalpha (large-M engine)   1 forward scan (large-M engine)
 *   2 segment aggregates (large-M)       3 segment carry scan (large-M)
 *   4 per-item evaluation (small-M)      5 small-M aggregates and scans
 *   6 partition of a chunk's events by node block (large-M, gradient only)
 *   7 state checkpoints of the dense dL/dalpha (large-M, shared decay)
 * Recording is host-side bookkeeping only (no device allocation); the events
 * are destroyed by hawkes_timing_read / hawkes_timing_reset.  Not for use
 * during graph capture.
 * ------------------------------------------------------------------------- */
#define HAWKES_TIMING_KERNELS 8
hawkes_status hawkes_timing_enable(int on);
hawkes_status hawkes_timing_reset(void);
hawkes_status hawkes_timing_read(int kernel_id, double* total_ms, int64_t* launches);

#ifdef __cplusplus
}
#endif

#endif /* HAWKES_H */
