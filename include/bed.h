/*
 * bed.h -- C ABI of the MI355X batched symmetric eigensolver.
 *
 * Method: Householder tridiagonalization followed by the batch-efficient
 * divide-and-conquer of Y. Song, "A Short Note on Batch-efficient Divide-and-
 * Conquer Algorithm for EigenDecomposition" (arXiv 2604.27325): rank-one
 * tearing (Sec. 2.1, Eq. (1)-(3)), leaves of at most 2, 4 or 8 elements solved
 * by cyclic Jacobi (Sec. 2.2; the cutoff is a schedule choice), secular
 * equation under bounded interlacing (Sec. 2.3.1, Eq. (8)-(12)), hybrid-section
 * (Sec. 2.3.2, Eq. (13)-(17)), Halley (Sec. 2.3.3, Eq. (20)-(21)), progressive
 * removal of converged work (Sec. 2.3.4, Eq. (22)) and Loewner/Gu-Eisenstat
 * eigenvectors (Sec. 2.3.5, Eq. (23)-(25)).  The problem statement is the
 * note's: a mini-batch of symmetric matrices (Sec. 1, Sec. 2.1 "B x C x C")
 * mapped to the eigenvalue tensor lambda in R^{B x C} (Sec. 2.3.1, Eq. (12))
 * and, when required, the eigenvector matrices (Sec. 2.3.5).
 *
 * Conventions shared by every entry point
 *   Layout     packed batch-major.  Matrix b is row-major n_b x n_b starting at
 *              element sum_{c<b} n_c^2 of A (and of Q, dA); its eigenvalues
 *              start at element sum_{c<b} n_c of lambda.  A uniform batch is
 *              exactly a contiguous (batch, n, n) / (batch, n) array.
 *   Input      only the lower triangle of each A_b is read (uplo = 'L').
 *   Output     lambda ascending; Q[b][i][j] = component i of eigenvector j;
 *              each column sign-canonical (largest-magnitude entry positive,
 *              lowest index on exact ties).
 *   Sizes      1 <= n_b <= 64 everywhere.  bed_syevd and bed_syevals also
 *              take uniform binary32 batches of 64 < n <= 128 (one more
 *              tearing step above the n <= 64 kernels, Sec. 2.1); other uses
 *              of n > 64 return BED_ERR_UNSUPPORTED.
 *   Memory     A, lambda, Q, info, dlambda, dQ, dA are DEVICE pointers owned
 *              by the caller.  n arrays are HOST pointers, read during the
 *              call only.  FP32 data needs 4-byte, FP64 8-byte alignment.
 *   Aliasing   A is read-only, except that Q == A (in place) is allowed; any
 *              other overlap between inputs and outputs is undefined.
 *   Streams    `stream` is a hipStream_t (NULL = the null stream).  Calls
 *              enqueue work and return without synchronizing.
 *   Errors     synchronous: a bed_status; the message of the last failure of
 *              the calling thread is in bed_last_error().  Asynchronous, per
 *              matrix, in info[b] (info may be NULL):
 *                0   success;
 *               -1   non-finite entry in the lower triangle (lambda, Q = NaN);
 *                k>0 k secular roots stopped at the iteration cap (results
 *                    returned, accuracy not guaranteed).
 *   Threads    calls on distinct plans/streams are thread-safe; a server is
 *              internally synchronized.  One plan runs on one stream at a
 *              time: a persistent plan's work counter belongs to the plan,
 *              so runs of one plan must not overlap (create a plan per
 *              stream; the convenience entry points do so internally).
 */
#ifndef BED_H
#define BED_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum { BED_F32 = 0, BED_F64 = 1 } bed_dtype;

typedef enum {
    BED_OK = 0,
    BED_ERR_INVALID_ARG = 1, /* bad size, null or misaligned pointer, bad dtype   */
    BED_ERR_UNSUPPORTED = 2, /* n > 64 where not supported (see Sizes), n > 128   */
    BED_ERR_HIP = 3,         /* a HIP runtime call failed (see bed_last_error)    */
    BED_ERR_NOMEM = 4,       /* device or host allocation failed / over budget    */
    BED_ERR_CAPTURE = 5,     /* call would allocate or copy during stream capture */
    BED_ERR_BUSY = 6         /* server: admission refused (slots or memory full)  */
} bed_status;

/* Launch schedule of a plan.  Zero fields mean "autotuned / default".
 *   threads_big   threads per matrix for the n > 32 size class (64, 128,
 *                 256 or 512; default 512: four waves reduce to tridiagonal
 *                 form while four form the Householder product, which 256 and
 *                 fewer apply in compact-WY form instead)
 *   threads_mid   threads per matrix for 16 < n <= 32 (64, 128 or 256; default
 *                 256: one wave reduces, two form Q_H, all four merge)
 *   waves_per_cu  resident teams per compute unit for the persistent launch
 *   order         0: largest n first (LPT), 1: input order
 *   persistent    1: one persistent launch pulls matrices from a device work
 *                 counter (progressive removal at batch level); 0: one
 *                 workgroup per matrix
 *   leaf          cutoff of the divide step (Sec. 2.2): nodes of at most leaf
 *                 elements (2, 4 or 8) are solved by cyclic Jacobi instead of
 *                 being split further; 0: per size class (8 for n > 32, else 4) */
typedef struct bed_tune {
    int32_t threads_big;
    int32_t threads_mid;
    int32_t waves_per_cu;
    int32_t order;
    int32_t persistent;
    int32_t leaf;
} bed_tune;

typedef struct bed_plan bed_plan;

/* One-shot solve: lambda, Q (and info) for a packed batch.  batch == 0 is a
 * no-op.  A uniform batch is one launch with no descriptor.  Mixed sizes (or
 * a stored persistent schedule) use a plan from an internal cache keyed by
 * (dtype, n[], stream); the first call for a new key allocates its descriptor
 * (refused under capture, BED_ERR_CAPTURE).  A uniform binary32 batch of
 * 64 < n <= 128 runs in steps (reduction and tearing, the Householder
 * product when eigenvectors are wanted, the two halves on the n <= 64
 * kernels, the top merge) with a workspace kept per stream (about
 * 8 (n/2)^2 + 12n + 24 bytes per matrix, plus 4n(n - 1) with eigenvectors,
 * grown on demand; growing it synchronizes the stream and is refused under
 * capture).  A workspace that a HIP graph captured is kept until the process
 * ends (a larger one replaces it for later calls); the graph's replays share
 * it with later calls on the capture stream that fit in it, so replay the
 * graph on that stream or keep the two from overlapping. */
bed_status bed_syevd(bed_dtype dt, int64_t batch, const int32_t *n, const void *A, void *lambda,
                     void *Q, int32_t *info, void *stream);

/* Largest batch bed_syevd_noalloc accepts. */
#define BED_NOALLOC_MAX_BATCH 65536

/* bed_syevd for callers that cannot allocate memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * solve and outputs, with no allocation, copy or memset of any kind.  A
 * mixed-size batch's device work list is kept in a fixed array of the library
 * (24 bytes per matrix, BED_NOALLOC_MAX_BATCH matrices, about 1.5 MiB per GPU,
 * held until the process ends) and built by small kernels whose arguments
 * carry the sizes; matrices of one size class run in input order, each with
 * the kernel configuration bed_syevd uses for its size, so results equal
 * bed_syevd's.  The array is shared by every call on a GPU and keeps the last
 * call's list: calls that overlap in time on one GPU (different streams or
 * threads) race and give wrong results -- serialize them.  batch >
 * BED_NOALLOC_MAX_BATCH returns BED_ERR_INVALID_ARG; orders above 64 return
 * BED_ERR_UNSUPPORTED (their solve needs a workspace); other errors as for
 * bed_syevd.  A uniform batch needs no list and does not touch the array. */
bed_status bed_syevd_noalloc(bed_dtype dt, int64_t batch, const int32_t *n, const void *A,
                             void *lambda, void *Q, int32_t *info, void *stream);

/* Eigenvalues only (the note forms eigenvectors only when they are required,
 * Sec. 2.3.5): Q is not produced.  The merges carry only the first and last
 * row of each node's eigenvector block -- all that the next z (Eq. (5))
 * reads -- instead of the block product, and there is no back-transform.
 * The Householder reduction runs in the data's own precision (bed_syevd uses
 * binary64 arithmetic for binary32 data): an eigenvalue moves by at most the
 * reduction's backward error, with no eigenvalue-gap factor, so the results
 * keep bed_syevd's eigenvalue bound but are not bitwise equal to its lambda. */
bed_status bed_syevals(bed_dtype dt, int64_t batch, const int32_t *n, const void *A,
                       void *lambda, int32_t *info, void *stream);

/* Plans: descriptors (offsets, size classes, work order) and the schedule
 * are built once; bed_plan_run enqueues one launch per size class (or one
 * persistent launch per class) and allocates nothing, so it may be captured
 * into a HIP graph.  tune == NULL takes the autotuner's choice for this size
 * mix (else the default schedule).  bed_plan_create allocates and copies the
 * descriptors synchronously; `stream` is the stream the plan will run on and
 * is only inspected: while it is being captured, BED_ERR_CAPTURE is returned
 * and nothing is allocated. */
bed_status bed_plan_create(bed_plan **plan, bed_dtype dt, int64_t batch, const int32_t *n,
                           const bed_tune *tune, void *stream);
bed_status bed_plan_run(const bed_plan *plan, const void *A, void *lambda, void *Q,
                        int32_t *info, void *stream);
bed_status bed_plan_get_tune(const bed_plan *plan, bed_tune *out);
void bed_plan_destroy(bed_plan *plan);

/* Autotuner: times the candidate schedules for this size mix on `stream`
 * (synchronizing it) and stores the winner in the process cache (and in the
 * JSON file named by BED_TUNE_CACHE when set).  A, lambda, Q are scratch
 * buffers of the packed sizes.  The chosen schedule is written to *out. */
bed_status bed_autotune(bed_dtype dt, int64_t batch, const int32_t *n, const void *A, void *lambda,
                        void *Q, void *stream, bed_tune *out);

/* Stores `tune` as the schedule of this (dtype, size mix) in the process
 * cache, where bed_syevd, bed_syevals and bed_plan_create (tune == NULL) find
 * it, exactly as bed_autotune stores its winner.  Launches nothing.
 * BED_ERR_INVALID_ARG for unsupported thread counts. */
bed_status bed_tune_set(bed_dtype dt, int64_t batch, const int32_t *n, const bed_tune *tune);

/* Plans held by the convenience entry points' cache (bed_syevd and
 * bed_syevals with mixed sizes or a persistent schedule).  The cache keeps one
 * plan per (dtype, size mix, stream), at most 32 (least recently used evicted
 * once its last launch has completed), except that plans used under stream
 * capture are kept for the life of the process (a graph holds their device
 * pointers).  Such a graph's replays share the plan, and a persistent plan's
 * work counter, with later calls of the same size mix on the capture stream:
 * replay the graph on that stream or keep the two from overlapping. */
int32_t bed_cache_entries(void);

/* Backward of A = Q diag(lambda) Q^T (for differentiable use, Sec. 1):
 *   dA = Q ( diag(dlambda) + sym(F o (Q^T dQ)) ) Q^T,  sym(X) = (X + X^T)/2,
 *   F_ij = 1/(lambda_j - lambda_i) for i != j, F_ij = 0 when
 *   |lambda_i - lambda_j| <= degeneracy_eps * max(1, max_i |lambda_i|).
 * dlambda or dQ may be NULL (treated as zero).  dA has A's layout and is
 * symmetric.  degeneracy_eps <= 0 selects 1e3 * unit roundoff of dt. */
bed_status bed_syevd_backward(bed_dtype dt, int64_t batch, const int32_t *n, const void *lambda,
                              const void *Q, const void *dlambda, const void *dQ, void *dA,
                              double degeneracy_eps, void *stream);

/* Spectral matrix functions on a decomposition (lambda, Q) as produced by
 * bed_syevd, for the differentiable meta-layer use of Sec. 1 (matrix square
 * root, whitening, ...):
 *   F = Q f(Lambda) Q^T                                  (bed_spectral_apply)
 *   dA = Q ( K o (Q^T sym(dF) Q) ) Q^T,  K_ij = (f(l_i) - f(l_j))/(l_i - l_j),
 *        K_ii = f'(l_i)                                  (bed_spectral_backward)
 * the first-order perturbation of f(A) (Daleckii-Krein), with every divided
 * difference written without cancellation (e.g. 1/(sqrt l_i + sqrt l_j) for
 * the square root, e^{l_j} expm1(l_i - l_j)/(l_i - l_j) for exp).  f is one of
 * bed_fn; `param` is the exponent p of BED_FN_POW (ignored otherwise).  SQRT
 * needs lambda >= 0, INVSQRT, LOG and POW need lambda > 0 (otherwise the
 * IEEE result of the function, NaN or infinity, propagates).  F, dF, dA have
 * A's packed layout; dA is symmetric.  Errors as for bed_syevd_backward. */
typedef enum { BED_FN_SQRT = 0, BED_FN_INVSQRT = 1, BED_FN_EXP = 2, BED_FN_LOG = 3,
               BED_FN_POW = 4 } bed_fn;
bed_status bed_spectral_apply(bed_dtype dt, int64_t batch, const int32_t *n, const void *lambda,
                              const void *Q, int32_t fn, double param, void *F, void *stream);
bed_status bed_spectral_backward(bed_dtype dt, int64_t batch, const int32_t *n,
                                 const void *lambda, const void *Q, int32_t fn, double param,
                                 const void *dF, void *dA, void *stream);

/* Serving: continuous batching of eigendecomposition requests.
 *   streams      device streams the server launches on (1..16)
 *   max_inflight matrices admitted but not yet completed (0 = unlimited)
 *   mem_budget   bytes of request buffers admitted at once (0 = unlimited)
 *   max_step     most matrices packed into one launch (0 = 4096)
 * A request's A/lambda/Q are caller-owned device buffers that must stay alive
 * until bed_server_poll reports it done.  Each request is solved by the same
 * per-matrix kernel configuration (a function of n and dtype only), so its
 * result is bitwise identical alone and in any mix. */
typedef struct bed_server_opts {
    int32_t streams;
    int32_t max_inflight;
    int64_t mem_budget;
    int32_t max_step;
    int32_t device;
} bed_server_opts;

typedef struct bed_server bed_server;

bed_status bed_server_create(bed_server **s, const bed_server_opts *o);
/* Admits one request of `count` matrices of size n (packed as above).  Returns
 * BED_ERR_BUSY when admission is refused by the in-flight or memory limit
 * (nothing is queued; retry later).  `stream` is the caller's stream that
 * produces A: the server records an event on it at admission and the step
 * that reads A waits for that event, so A may still be being written by work
 * enqueued on `stream` before this call.  *ticket identifies the request. */
bed_status bed_server_submit(bed_server *s, bed_dtype dt, int32_t count, int32_t n, const void *A,
                             void *lambda, void *Q, int32_t *info, void *stream,
                             uint64_t *ticket);
/* *done = 1 once the request's results are complete in device memory;
 * *latency_us (may be NULL) = submit-to-completion-observed time. */
bed_status bed_server_poll(bed_server *s, uint64_t ticket, int32_t *done, double *latency_us);
/* Blocks until every admitted request has completed. */
bed_status bed_server_drain(bed_server *s);
void bed_server_destroy(bed_server *s);

const char *bed_status_string(bed_status st);
const char *bed_last_error(void);
/* Library version, as major*10000 + minor*100 + patch. */
int32_t bed_version(void);

#ifdef __cplusplus
}
#endif
#endif
