/*
 * qm.h -- C ABI of libqm, the MI355X (gfx950) quantile-mechanics library.
 *
 * Elementwise maps over device-resident arrays, after Shaw, Luu & Brickman,
 * "Quantile Mechanics II: Changes of Variables in Monte Carlo Methods and
 * GPU-Optimized Normal Quantiles":
 *
 *   qm_normal_quantile        w = Phi^{-1}(u)            (Section 1, eq. 1)
 *   qm_recycle_exp_to_normal  z = Q(x) = sign(x) Phi^{-1}(1 - e^{-|x|}/2)
 *                                                         (Section 6)
 *   qm_recycle_student_t      t = F_nu^{-1}(Phi(z))       (Section 1 recycling
 *                                composite, Section 3 recycling ODE)
 *   qm_recycle_exp_to_hyperbolic
 *                             x = F^{-1}(F0(v)), two-sided exponential base
 *                             -> hyperbolic target        (Section 8.1)
 *   qm_recycle_exp_to_vg      the same base -> variance-gamma target,
 *                             lambda in [1, 8]             (Section 8.2)
 *   qm_generate               the uniforms of a counter-based stream, or w
 *                             of them, drawn and mapped in one pass
 *   qm_generate_student_t, qm_generate_hyperbolic, qm_generate_vg
 *                             Student t / hyperbolic / variance-gamma
 *                             samples drawn the same way, through the maps
 *   qm_run_batch              many such requests in one persistent launch
 *   qm_submit / qm_poll       continuous-batching serving loop
 *
 * Conventions (all entry points):
 *   - Every function is plain C, never throws, and returns a qm_status.
 *   - Array arguments are device pointers owned by the caller; the library
 *     never frees them.  Input and output have the same dtype and n
 *     elements, are contiguous, and may be identical (in place); a partial
 *     overlap is QM_E_INVAL.  Any alignment of the element type is accepted.
 *   - hip_stream is a hipStream_t (NULL = the null stream).  The synchronous
 *     calls only enqueue work on that stream and return; buffers must stay
 *     alive until the stream has completed it.
 *   - n = 0 succeeds without a launch.
 *   - Non-finite and out-of-range elements are never errors: they map to
 *     NaN / +-inf per element as documented per call.
 *   - Arguments are validated before any device work: a NULL context or
 *     pointer (with n > 0), an unknown dtype/mode/kind, or an invalid nu is
 *     reported and nothing is launched.
 */
#ifndef QM_H
#define QM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t qm_status;

#define QM_OK 0         /* success / request complete */
#define QM_PENDING 1    /* qm_poll: request not complete yet */
#define QM_E_INVAL (-1) /* bad argument: NULL, overlap, unknown enum, bad nu, request over budget */
#define QM_E_DTYPE (-2) /* mode not available for this dtype/kind */
#define QM_E_NOMEM (-3) /* device or host allocation failed */
#define QM_E_HIP (-4)   /* HIP runtime error; text via qm_last_error() */
#define QM_E_CLOSED (-5)/* context is shutting down */
#define QM_E_TICKET (-6)/* unknown ticket */

/* element type of both input and output */
enum qm_dtype { QM_F32 = 0, QM_F64 = 1 };

/*
 * Precision form.
 *   QM_PLAIN       full precision of the dtype.  F64: relative error within
 *                  2e-15 of Phi^{-1} (absolute 2e-18 where |w| < 1e-3) on the
 *                  whole double range.  F32: the FP64 evaluation rounded to
 *                  float.
 *   QM_F32_REFINE  dtype QM_F32 only: FP32 rational seed plus one FP64
 *                  correction step against an FP64 erf (|u - 1/2| <= 0.45)
 *                  or erfc (beyond); relative error within 2e-7 (absolute
 *                  2e-10 near 0).
 *   QM_PAPER       the paper's constants verbatim, valid only on the paper's
 *                  domain: F64 the (13,13) rational of Section 7.2 / Appendix
 *                  B (v <= 42, u >= 2.875e-19), F32 the (5,6) rational of
 *                  Section 6.1 / Appendix A (v <= 25).  Outside that domain the
 *                  result degrades as the rational does.
 *   QM_PAPER_T2    qm_normal_quantile with dtype QM_F64 only: the paper's
 *                  own hybrid of Section 7.3 / Appendix C, constants
 *                  verbatim -- the T2 intermediate v = |u - 1/2| /
 *                  sqrt(u(1-u)) and its (14,15) rational when v < 15.5 on
 *                  every lane of a 64-lane wave, else the whole wave takes
 *                  QM_PAPER's (13,13) path.  Same domain and accuracy as
 *                  QM_PAPER.  Which path an element takes depends on the
 *                  other elements of its wave, so batches, serving and
 *                  qm_generate (whose outputs are bitwise those of single
 *                  calls) reject it with QM_E_INVAL.
 */
enum qm_mode { QM_PLAIN = 0, QM_F32_REFINE = 1, QM_PAPER = 2, QM_PAPER_T2 = 3 };

/* QM_UNIFORM (the uniforms themselves) is accepted by qm_generate only. */
enum qm_kind { QM_NORMAL_QUANTILE = 0, QM_STUDENT_T = 1, QM_EXP_TO_NORMAL = 2, QM_UNIFORM = 3, QM_EXP_TO_HYPERBOLIC = 4,
               QM_EXP_TO_VG = 5 };

typedef struct qm_ctx qm_ctx;

/*
 * Create a context on HIP device `hip_device`.  hbm_budget_bytes bounds the
 * bytes (input + output of admitted requests) that the serving loop keeps in
 * flight; 0 means no serving budget (qm_submit then rejects every request).
 * The context owns the per-nu Student t tables and the serving state.
 * Each kernel family has its own launch shape (workgroups of 256 per compute
 * unit x 16-byte vectors in flight per lane, from measured sweeps: light
 * FP64 maps 2 x 4, the other FP32 maps 32 x 2, FP64 quantile 64 x 4,
 * FP32+refine quantile 16 x 4, fused generation 64 x 4 (FP64) and 32 x 2
 * (FP32), Student t 2 x 4 (FP64) and 3 x 4 (FP32), exp -> hyperbolic or
 * variance-gamma 16 x 4 (FP64) and 16 x 2 (FP32)); the environment
 * variables QM_BLOCKS_PER_CU (1..64) and QM_UNROLL (1, 2 or 4), read here,
 * override every family, and QM_SHAPE_STREAM, QM_SHAPE_STREAM32,
 * QM_SHAPE_NQ64, QM_SHAPE_NQ32, QM_SHAPE_GEN64, QM_SHAPE_GEN32,
 * QM_SHAPE_T64, QM_SHAPE_T32, QM_SHAPE_H64, QM_SHAPE_H32 ("blocks,unroll")
 * one family each.  QM_COMPACT=0 turns off the quantiles' gathering of
 * non-central lanes across the wave (the results are bitwise the same
 * either way).
 * Errors: QM_E_INVAL (out == NULL or no such device), QM_E_HIP, QM_E_NOMEM.
 */
qm_status qm_init(int hip_device, uint64_t hbm_budget_bytes, qm_ctx** out);

/*
 * Stop the serving loop, wait for requests already on the device, fail the
 * ones still queued (their qm_poll then returns QM_E_CLOSED), and free the
 * context.  NULL is a no-op.
 */
void qm_shutdown(qm_ctx* ctx);

/*
 * w[i] = Phi^{-1}(u[i]) (Section 1, eq. 1).  QM_PAPER: the paper's
 * exponential change of variable v = -log(2 min(u, 1-u)) and its rational
 * in v (Section 7.2) for every u.  QM_PLAIN and QM_F32_REFINE: the hybrid of
 * Section 7.3 / Appendix C -- a central piece for |u - 1/2| <= 0.45 (a
 * fitted rational in 0.2025 - (u - 1/2)^2, no logarithm; in place of the
 * paper's T2 intermediate variable), and the exponential-coordinate path
 * elsewhere, with a fitted rational in sqrt(v) for 42 < v (beyond the
 * paper's domain, Section 4.3).  u = 0 -> -inf, u = 1 -> +inf, u outside
 * [0,1] or NaN -> NaN, u = 1/2 -> +0.  QM_PAPER_T2: the paper's hybrid
 * as printed, for comparison (see enum qm_mode).
 * dtype/mode: F64 {PLAIN, PAPER, PAPER_T2}; F32 {PLAIN, F32_REFINE, PAPER}.
 */
qm_status qm_normal_quantile(qm_ctx* ctx, const void* d_u, void* d_w, uint64_t n,
                             int dtype, int mode, void* hip_stream);

/*
 * t[i] = F_nu^{-1}(Phi(z[i])), the normal -> Student t recycling map
 * (Section 1 recycling composite, Section 3).  nu is the real number of
 * degrees of freedom: finite and >= 0.3, or +inf (identity).  The map is
 * the solution of the Gaussian-background recycling ODE (Section 3.1) with
 * centre conditions Q(0) = 0, Q'(0) = gamma (Section 3.1); the library
 * integrates it on the host once per nu (cached in the context) and
 * evaluates piecewise polynomials on the device (degree 15 for F64,
 * degree 7 for F32 outputs).  Accuracy: relative 2e-15 (F64) / 2e-7 (F32)
 * for |z| <= 40, which holds the normal quantile of every positive double;
 * the two-term tail of Sections 3.3/3.5 takes over only where it is as
 * accurate, and beyond |z| = 40 for every nu, with error O(w^{4/nu}),
 * w = K q(|z|).  z = +-inf -> +-inf, NaN -> NaN, and t may overflow to
 * +-inf for small nu.
 * dtype/mode: F64 PLAIN; F32 F32_REFINE.
 * Errors: QM_E_INVAL for nu < 0.3, NaN or -inf (below 0.3 the per-nu
 * cells that meet 2e-15 no longer fit the 64 KB of LDS a launch may use).
 */
qm_status qm_recycle_student_t(qm_ctx* ctx, const void* d_z, void* d_t, uint64_t n,
                               int dtype, int mode, double nu, void* hip_stream);

/*
 * z[i] = sign(x[i]) Phi^{-1}(1 - e^{-|x[i]|}/2): the exponential -> normal
 * recycling map, formal solution of the exponential-background recycling
 * ODE with Q(0) = 0, Q'(0) = sqrt(pi/2), extended by odd symmetry
 * (Section 6).  Exp(1) inputs give half-normal magnitudes; signed (Laplace)
 * inputs give N(0,1).  No logarithm is taken: v = |x| is the rational's
 * variable directly.  +-0 -> +-0, +-inf -> +-inf, NaN -> NaN.
 * dtype/mode: F64 {PLAIN, PAPER}; F32 {F32_REFINE, PLAIN} (PLAIN: the FP64
 * map of the widened input, rounded once to FP32).
 */
qm_status qm_recycle_exp_to_normal(qm_ctx* ctx, const void* d_x, void* d_z, uint64_t n,
                                   int dtype, int mode, void* hip_stream);

/*
 * x[i] = mu + Q(v[i]), the exponential -> hyperbolic recycling map
 * (Section 8.1).  Target: the hyperbolic density
 *   f(x) = gamma / (2 alpha delta K_1(delta gamma)) exp(-alpha sqrt(delta^2 + (x-mu)^2) + beta (x-mu)),
 * gamma = sqrt(alpha^2 - beta^2).  Base: the two-sided exponential with the
 * target's masses p+ (x > mu) and p- (x < mu), density
 * p+ (alpha-beta) e^{-(alpha-beta) v} on v > 0 and p- (alpha+beta) e^{(alpha+beta) v}
 * on v < 0 (qm_hyperbolic_masses gives log p+ and log p-; a base sample is
 * -log(U)/(alpha-beta) with probability p+, log(U)/(alpha+beta) otherwise).
 * Q = F^{-1}(F0(v)) is the solution of the left and right recycling ODEs
 * with Q(0) = 0 and Q'(0) = f0(0+-)/f(0) (Section 8.1); the library
 * integrates them on the host once per (alpha, beta, delta) (cached in the
 * context, about a second) and evaluates piecewise polynomials of degree 11
 * on the device.  Accuracy: relative 2e-15 in x - mu (F64), 2e-7 (F32, the
 * F64 evaluation rounded once) for every v.  v = +-inf -> +-inf, NaN -> NaN.
 * dtype/mode: F64 PLAIN; F32 F32_REFINE.
 * Errors: QM_E_INVAL for alpha <= |beta|, delta <= 0, a non-finite
 * parameter or mu, NULL, unaligned or partially overlapping buffers.
 */
qm_status qm_recycle_exp_to_hyperbolic(qm_ctx* ctx, const void* d_v, void* d_x, uint64_t n, int dtype, int mode,
                                       double alpha, double beta, double delta, double mu, void* hip_stream);

/*
 * log p+ and log p- (host doubles; either pointer may be NULL): the
 * hyperbolic target's masses on each side of mu (Section 8.1), which the
 * base of qm_recycle_exp_to_hyperbolic carries.  Builds and caches the
 * table like that call.  Errors as for it.
 */
qm_status qm_hyperbolic_masses(qm_ctx* ctx, double alpha, double beta, double delta, double* log_p_plus,
                               double* log_p_minus);

/*
 * x[i] = mu + Q(v[i]), the exponential -> variance-gamma recycling map
 * (Section 8.2) for real lambda in [1, 8].  Target: the variance-gamma
 * density
 *   f(x) = (alpha^2 - beta^2)^lambda e^{beta (x-mu)} |x-mu|^{lambda-1/2} K_{lambda-1/2}(alpha |x-mu|)
 *          / ((2 alpha)^{lambda-1/2} sqrt(pi) Gamma(lambda)),  |beta| < alpha,
 * from the same two-sided exponential base as qm_recycle_exp_to_hyperbolic
 * with this target's masses (qm_vg_masses).  The library builds, on the
 * host once per (lambda, alpha, beta), the same piecewise polynomials as
 * for the hyperbolic map and evaluates them with the same kernel.  For
 * integer lambda the Bessel function is elementary and each side's map is
 * solved directly from its closed-form masses; lambda = 1 is the base
 * itself (Q(v) = v).  For other lambda the recycling ODE of Section 8.2 is
 * integrated, with H = alpha K_{lambda-3/2}/K_{lambda-1/2} - beta from the
 * Riccati equation of that Bessel ratio and the origin's non-analytic
 * neighbourhood from its expansion (a build takes a few seconds).  Where
 * 2 lambda is not an integer the density carries |x|^(2 lambda - 1) at 0,
 * which no polynomial cell matches near v = 0: the table's first octave
 * (v < v0) is then one series in v and v^(2 lambda - 1), evaluated on the
 * kernel's far path (one pow per element there).  Accuracy as for the
 * hyperbolic map.
 * dtype/mode: F64 PLAIN; F32 F32_REFINE.
 * Errors: QM_E_INVAL for lambda outside [1, 8] or a table the builder
 * cannot meet the accuracy for, alpha <= |beta|, a non-finite parameter or
 * mu, NULL, unaligned or overlapping buffers.
 */
qm_status qm_recycle_exp_to_vg(qm_ctx* ctx, const void* d_v, void* d_x, uint64_t n, int dtype, int mode, double lambda,
                               double alpha, double beta, double mu, void* hip_stream);

/* log p+ and log p- of the variance-gamma target (as qm_hyperbolic_masses). */
qm_status qm_vg_masses(qm_ctx* ctx, double lambda, double alpha, double beta, double* log_p_plus,
                       double* log_p_minus);

/*
 * Fused generation and transform.  Draws the open uniforms of elements
 * first .. first+n-1 of the counter-based stream Philox4x32-10 (Salmon et
 * al., SC'11) with key (seed, stream), maps them, and writes only the
 * results to d_out (n elements of dtype).  Element e of the stream:
 *   F64: block e/2 (counter (e/2 mod 2^32, e/2 div 2^32, 0, 0)); the 64-bit
 *        value of words (0,1) for even e, (2,3) for odd e (low word
 *        first); its top 53 bits k give u = (k + 1/2) 2^-53.
 *   F32: word e mod 4 of block e/4; its top 23 bits k give
 *        u = (k + 1/2) 2^-23, exact, in [2^-24, 1 - 2^-24].
 *   (F64: the sum k + 1/2 rounds to nearest, a tie to even for k >= 2^52,
 *   so u lies in [2^-54, 1] and is 1 with probability 2^-53; Phi^{-1}
 *   maps it to +inf.)
 * kind QM_UNIFORM writes u (mode QM_PLAIN); kind QM_NORMAL_QUANTILE writes
 * Phi^{-1}(u), bitwise equal to qm_normal_quantile of the same u, with the
 * dtype/mode pairs of qm_normal_quantile.  Any sub-range of a stream can be
 * generated independently; the results do not depend on the launch.
 * Errors: QM_E_INVAL for seed or stream >= 2^32, first + n beyond 2^63, a
 * NULL d_out (n > 0), an unaligned d_out or another kind; QM_E_DTYPE for a
 * mode the dtype does not offer.
 */
qm_status qm_generate(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                      int kind, int dtype, int mode, void* hip_stream);

/*
 * Fused generation of Student t samples: element e of the stream is
 * t = F_nu^{-1}(Phi(z)) of the normal z that qm_generate (kind
 * QM_NORMAL_QUANTILE, same dtype and mode) writes for element e, computed
 * in registers by the same device code as qm_generate followed by
 * qm_recycle_student_t, and bitwise equal to that two-call chain.  Only t
 * is written.  nu as for qm_recycle_student_t (+inf gives the normals).
 * dtype/mode: F64 PLAIN; F32 F32_REFINE.  Other arguments and errors as for
 * qm_generate, and QM_E_INVAL for an invalid nu.
 */
qm_status qm_generate_student_t(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                                int dtype, int mode, double nu, void* hip_stream);

/*
 * Fused generation of hyperbolic samples (Section 8.1): element e's open
 * uniform u (as qm_generate kind QM_UNIFORM writes it, widened to FP64 for
 * F32) becomes a sample of the two-sided exponential base,
 *   v = log(u * (1 / p-)) * (1 / (alpha + beta))        for u < p-,
 *   v = -log((1 - u) * (1 / p+)) * (1 / (alpha - beta))  otherwise,
 * with p- = exp(log p-), p+ = exp(log p+) of qm_hyperbolic_masses and the
 * reciprocals each rounded once (all in FP64; the products are correctly
 * rounded, the logarithm is within about an ulp), and then
 * x = mu + Q(v) as qm_recycle_exp_to_hyperbolic maps it.  Only x is written.
 * dtype/mode: F64 PLAIN; F32 F32_REFINE.  Other arguments and errors as for
 * qm_generate and qm_recycle_exp_to_hyperbolic.
 */
qm_status qm_generate_hyperbolic(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                                 int dtype, int mode, double alpha, double beta, double delta, double mu,
                                 void* hip_stream);

/*
 * Fused generation of variance-gamma samples (Section 8.2, lambda in
 * [1, 8]): as qm_generate_hyperbolic, with the variance-gamma target's
 * masses (qm_vg_masses) and the map of qm_recycle_exp_to_vg.
 */
qm_status qm_generate_vg(qm_ctx* ctx, uint64_t seed, uint64_t stream, uint64_t first, void* d_out, uint64_t n,
                         int dtype, int mode, double lambda, double alpha, double beta, double mu, void* hip_stream);

/* One request of a batch or of the serving loop. */
typedef struct {
    uint32_t kind;      /* enum qm_kind */
    uint32_t dtype;     /* enum qm_dtype */
    uint32_t mode;      /* enum qm_mode */
    uint32_t reserved;  /* must be 0 */
    double nu;          /* QM_STUDENT_T: nu; QM_EXP_TO_VG: lambda */
    const void* d_in;   /* device input, n elements of dtype */
    void* d_out;        /* device output, n elements of dtype */
    uint64_t n;
    uint64_t user_tag;  /* opaque to the library */
    double alpha, beta, delta, mu;  /* QM_EXP_TO_HYPERBOLIC: the target's parameters;
                                       QM_EXP_TO_VG: alpha, beta and mu (delta unused) */
} qm_request;

/*
 * Run `count` requests (host array) of mixed kinds (every kind but
 * QM_UNIFORM), dtypes, modes, nu and hyperbolic parameters as one
 * persistent launch on hip_stream: workgroups claim fixed-size chunks
 * from a device counter; each chunk belongs to one request and is evaluated
 * by the same device code as the single-request call with that kind, dtype
 * and mode, so each output is bitwise identical to the single call's.
 * Validation covers every request before anything is launched; the first
 * invalid one decides the status.  Student t and hyperbolic tables not yet
 * in the context are built by this call, on the host, before the launch.
 * The call returns after enqueueing; the descriptor upload is ordered on
 * hip_stream.
 */
qm_status qm_run_batch(qm_ctx* ctx, const qm_request* reqs, uint64_t count, void* hip_stream);

/* Most requests with n > 0 that one qm_run_batch_noalloc call takes. */
#define QM_BATCH_NOALLOC_MAX_REQUESTS 4096

/*
 * qm_run_batch for callers that cannot allocate memory (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc).
 * Same requests, same kernel, bitwise the same outputs as qm_run_batch;
 * the call itself allocates nothing, on the device or the host.
 *
 * Memory: the batch header and descriptors go to a fixed device array
 * (QM_BATCH_NOALLOC_MAX_REQUESTS records, about 768 KiB) that the library
 * holds once per GPU until the process ends, its address looked up by
 * qm_init; they are staged through the context's pinned host buffer, also
 * set up by qm_init.  The claim counter is rewritten to 0 by every call.
 *
 * Ordering: the upload and the launch are ordered on hip_stream.  All calls
 * on one GPU share that device array, so two calls whose work overlaps on
 * the GPU (different streams, or several contexts on one GPU) race and give
 * undefined results: order them on one stream, or synchronize between.
 * Calls on one context from several host threads are serialized.  A call
 * waits until the previous call's descriptor upload has left the host
 * buffer.
 *
 * Errors: as qm_run_batch, plus QM_E_INVAL when more than
 * QM_BATCH_NOALLOC_MAX_REQUESTS requests have n > 0, and QM_E_INVAL when a
 * request needs a Student t, hyperbolic or variance-gamma table that the
 * context does not hold yet (this call does not build tables: make one
 * call with those parameters first, n = 0 is enough).  Nothing is launched
 * on error.
 */
qm_status qm_run_batch_noalloc(qm_ctx* ctx, const qm_request* reqs, uint64_t count, void* hip_stream);


/*
 * Serving loop.  qm_submit validates and enqueues one request and returns a
 * ticket; it returns at once unless the request needs a Student t or
 * hyperbolic table the context does not hold yet, which it first builds in
 * the calling thread (so the scheduler never waits for a build).  A scheduler thread admits queued requests in
 * arrival order while the bytes (in + out) of requests in flight stay within
 * the context's HBM budget, and launches everything admitted since its
 * previous launch as one batch; batches run on several streams, so requests
 * admitted while others are on the GPU overlap with them.  Per-request state
 * (descriptors, chunk counters) lives on the device for the batch's life.
 * Completion is per request: the workgroup that writes a request's last
 * chunk raises a flag in host-coherent memory once all of the request's
 * stores have reached device memory, and the scheduler reports the request
 * complete as soon as it sees the flag, while the rest of its batch may
 * still run (in a batch of more than 4096 requests with n > 0, at the
 * batch's end).
 * Ordering: the serving streams are the library's own and are not ordered
 * after any stream of the caller.  The request's input must therefore be
 * complete in device memory, and its output no longer read or written by
 * other work, when qm_submit is called (synchronize the stream that
 * produced the input first).  Buffers must stay alive until qm_poll returns
 * QM_OK or an error.
 * qm_submit errors: QM_E_INVAL (as qm_run_batch, or request larger than the
 * whole budget), QM_E_DTYPE, QM_E_CLOSED.
 * qm_poll returns QM_OK once the request's output is complete in device
 * memory, QM_PENDING before that, QM_E_TICKET for an unknown ticket, and
 * QM_E_CLOSED for a request failed by qm_shutdown.  A finished ticket keeps
 * reporting its final status until 65536 later requests have finished;
 * then it is forgotten and reports QM_E_TICKET (the server's memory stays
 * bounded however long it runs).
 */
qm_status qm_submit(qm_ctx* ctx, const qm_request* req, uint64_t* ticket);
qm_status qm_poll(qm_ctx* ctx, uint64_t ticket);

/*
 * qm_poll, also giving the request's submit time and (with QM_OK) the time
 * the scheduler observed its completion, in nanoseconds of the monotonic
 * clock (CLOCK_MONOTONIC, the clock of C++ steady_clock), so that a caller
 * can measure latency from its own scheduled arrival times.  Either pointer
 * may be NULL.
 */
qm_status qm_poll_times(qm_ctx* ctx, uint64_t ticket, uint64_t* submit_ns, uint64_t* done_ns);

/*
 * Serving statistics since qm_init.  Returns the number of completed
 * requests and writes the submit -> completion latencies, in nanoseconds, of
 * the most recent min(cap, completed, 2^20) of them into lat_ns, oldest
 * first (lat_ns may be NULL).
 */
uint64_t qm_serving_latencies(qm_ctx* ctx, uint64_t* lat_ns, uint64_t cap);

/* Counters of the serving loop (all zero before the first qm_submit). */
typedef struct {
    uint64_t submitted;                  /* requests accepted by qm_submit */
    uint64_t completed;                  /* requests finished with QM_OK */
    uint64_t failed;                     /* requests whose launch failed */
    uint64_t queued;                     /* waiting for admission now */
    uint64_t in_flight_requests;         /* admitted, not yet observed complete */
    uint64_t in_flight_bytes;            /* their input + output bytes */
    uint64_t in_flight_bytes_high_water; /* the largest in_flight_bytes so far (never above budget_bytes) */
    uint64_t budget_bytes;               /* the context's HBM budget */
    uint64_t tickets_kept;               /* tickets the server holds state for */
} qm_serving_counters;

/* Errors: QM_E_INVAL for a NULL argument. */
qm_status qm_serving_stats(qm_ctx* ctx, qm_serving_counters* out);

/* Static text for a status code. */
const char* qm_status_string(qm_status s);

/* Text of the last error reported on the calling thread ("" if none). */
const char* qm_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* QM_H */
