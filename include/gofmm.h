/*
 * gofmm.h -- C ABI of an MI355X (gfx950) evaluator for GOFMM compressions.
 *
 * GOFMM (Yu, Levitt, Reiz, Biros, "Geometry-Oblivious FMM for Compressing
 * Dense SPD Matrices", SC'17) approximates a dense SPD matrix K by a
 * hierarchical matrix K~ = D + S + UV (Sec. 1, eq. hmatrix) built only from a
 * routine that returns blocks K(I, J) (Sec. 1, problem statement), and then
 * multiplies K~ by a block W of r right-hand sides (Sec. 2.2, Alg. Evaluate).
 *
 * This library builds the compression on the host (ball tree, neighbours,
 * interaction lists, interpolative decompositions, cached blocks) and
 * evaluates U = K~ W on the GPU with hand-written HIP kernels.
 *
 * Conventions for every call:
 *   - return 0 on success, a negative GOFMM_E* code on failure; the failing
 *     call's message is available from gofmm_last_error() on the same thread;
 *   - on failure no handle is produced and nothing leaks;
 *   - all index arrays use the caller's original (unpermuted) numbering;
 *   - device pointers are HIP device addresses on the current device; the
 *     caller owns W, U and the stream; the library owns every byte of a
 *     compression, host and device, until gofmm_free.
 */
#ifndef GOFMM_H
#define GOFMM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---------------------------------------------------------------- errors */
enum {
  GOFMM_OK = 0,
  GOFMM_EINVAL = -1,     /* bad argument (n <= 0, m < 1, s < 1, tau < 0,
                            budget outside [0,1], null pointer, bad ld) */
  GOFMM_ECALLBACK = -2,  /* the sampler returned non-zero */
  GOFMM_ENOTSPD = -3,    /* K_ii <= 0 or a non-finite entry */
  GOFMM_ENOMEM = -4,     /* host or device allocation failed */
  GOFMM_EHIP = -5,       /* a HIP runtime error (message in last_error) */
  GOFMM_EIO = -6,        /* file could not be read or written / bad format */
  GOFMM_ELIMIT = -7,     /* a documented size limit was exceeded */
  GOFMM_ETIMEDOUT = -8   /* a wait ended before the awaited work finished */
};

/* distance used for the tree and the neighbours (Sec. 2.1) */
enum { GOFMM_GRAM_L2 = 0,   /* d_ij^2 = K_ii + K_jj - 2 K_ij  (eq. 3) */
       GOFMM_ANGLE = 1 };   /* d_ij = 1 - K_ij^2 / (K_ii K_jj) (eq. 4) */

/* storage precision of the device operator; accumulation is always FP32 */
enum { GOFMM_FP32 = 0,      /* FP32 storage, FP32 matrix-core products */
       GOFMM_BF16 = 1,      /* BF16 storage; right-hand operands rounded to BF16 */
       GOFMM_BF16X3 = 2 };  /* split BF16 (hi + lo) for both operands, three
                               BF16 products per step; near-FP32 accuracy */

typedef struct gofmm_compression gofmm_compression;   /* opaque */

/*
 * Entry sampler: the method's only input (Sec. 1, problem statement: a
 * routine returning the block K(I, J) for any index sets I and J).
 * Fill out[i + j * ld] = K(I[i], J[j]) in FP64 for original indices
 * I[0..nI), J[0..nJ): an nI x nJ column-major block with leading dimension
 * ld >= nI (cells outside the block must not be written).  K must be
 * symmetric (K(i,j) == K(j,i) bitwise) and positive definite.  Called only
 * inside gofmm_compress, gofmm_import and gofmm_use_device_kernel, possibly
 * from several threads at once (params.threads).  Return 0; any other value
 * aborts the call with GOFMM_ECALLBACK.
 */
typedef int (*gofmm_sampler)(void* user, int64_t nI, const int64_t* I,
                             int64_t nJ, const int64_t* J, double* out, int64_t ld);

/*
 * Method parameters (Sec. 3, parameter selection): m, s, tau, kappa, budget,
 * distance.  Fill with gofmm_default_params and override.
 */
typedef struct {
  int64_t leaf_size;        /* m: leaves hold at most m indices */
  int64_t max_rank;         /* s: cap on every skeleton rank */
  double tol;               /* tau: adaptive-rank tolerance, relative to |R_00|
                               of the pivoted QR of the sampled block */
  int32_t kappa;            /* neighbours per index (an index is its own first) */
  double budget;            /* near-field budget: each leaf keeps at most
                               floor(budget * N / m) other leaves (eq. budget);
                               0 gives the HSS form */
  int32_t distance;         /* GOFMM_GRAM_L2 | GOFMM_ANGLE */
  int32_t storage;          /* precision of P and coupling blocks K(b~, a~) */
  int32_t near_storage;     /* precision of the near blocks K(b, a) */
  uint64_t seed;            /* all random choices derive from it */
  int32_t threads;          /* host threads for compression (0 = all) */
  int32_t ann_max_iters;    /* randomized trees for the neighbour search (10) */
  double ann_target_recall; /* stop the neighbour search at this recall (0.8) */
  int32_t exact_knn;        /* 1: brute-force neighbours instead (small N) */
  int32_t device_knn;       /* 1: merge the neighbour candidates on the current
                               HIP device (the ANN task of Table 2: each leaf's
                               sampled block K(leaf, leaf), or a block of rows
                               against every index for exact_knn, becomes FP64
                               Gram distances, and every row keeps its kappa
                               nearest by (distance, index)); same lists as the
                               host, bit for bit.  Needs kappa <= 64 and
                               n < 2^31; the host still samples every block.
                               0 (default): everything on the host */
  int32_t device_id;        /* 1: the interpolative decompositions of each tree
                               level run on the current HIP device, all nodes of
                               the level together (Alg. Skeletonize: pivoted QR
                               in FP64 stopped at the adaptive rank, then
                               R11^{-1} R12), with the host's steps and
                               rounding: the same skeletons and P bit for bit.
                               The host still samples every block.  Needs at
                               most 8192 sampled rows per node (twice its
                               columns: the leaf size at a leaf, at most 2 s_max
                               above it), else GOFMM_ELIMIT.  0 (default): host */
} gofmm_params;

/* Summary of a built compression (for flop/byte accounting and reports). */
typedef struct {
  int64_t n, depth, n_leaves, n_nodes;
  int64_t rank_sum, rank_max;           /* over non-root nodes */
  int64_t near_pairs, far_pairs;        /* ordered (leaf, leaf) / (node, node) */
  double flops_per_rhs;                 /* Table 2 flops of one K~w, all phases */
  double flops_phase[4];                /* per rhs: N2S, S2S, S2N, L2L */
  int64_t operator_bytes;               /* device operator (all precisions held) */
  int64_t operator_bytes_phase[4];      /* bytes read per evaluate, by phase */
  int64_t workspace_rows;               /* rows of the r-wide skeleton workspace */
} gofmm_stats_t;

/* Defaults: m 256, s 256, tau 1e-5, kappa 32, budget 0.03, Gram-l2, FP32. */
void gofmm_default_params(gofmm_params* p);

/*
 * Build a compression of the n x n matrix behind `sampler` (Alg. Compress):
 * diagonal, randomized-tree neighbour search, metricSplit ball tree (Alg. 1),
 * LeafNear with the budget ballot (Alg. 2), FindFar / MergeFar (Alg. 3, 4)
 * with a symmetric refinement, nested IDs in FP64 (eqs. 7-8, Alg. 5), and the
 * cached blocks Kba / SKba packed for the device in the requested precision.
 * Host only: no GPU is touched until gofmm_prepare or the first evaluate.
 * params may be NULL (defaults).  On success *out is a new compression the
 * caller releases with gofmm_free.  Errors: GOFMM_EINVAL (n < 1, NULL
 * sampler or out, parameters out of range), GOFMM_ECALLBACK (the sampler
 * failed), GOFMM_ENOTSPD (K_ii <= 0 or a non-finite entry), GOFMM_ENOMEM,
 * GOFMM_ELIMIT (n or the operator beyond 32-bit row codes); *out is NULL.
 */
int gofmm_compress(int64_t n, gofmm_sampler sampler, void* user,
                   const gofmm_params* params, gofmm_compression** out);

/*
 * Load the structure that Alg. Compress produces (Sec. 2.2: tree and
 * permutation, Near and Far lists, skeletons and the interpolation matrices
 * P of eqs. 7-8) as written by gofmm_export or by an external tool in the
 * same format, check it (a partition, coverage of every leaf pair, nested
 * skeletons), and sample the cached blocks with `sampler`.  params supplies
 * storage precisions and threads only; the method parameters come from the
 * file.  Ownership and errors as for gofmm_compress, plus GOFMM_EIO for a
 * file that cannot be read or does not hold a valid structure.
 */
int gofmm_import(const char* path, gofmm_sampler sampler, void* user,
                 const gofmm_params* params, gofmm_compression** out);

/*
 * Compute the near-field blocks K(b, a) on the device instead of storing them
 * (Sec. 2.2: caching the near blocks after compression is optional; Sec. 4,
 * the memory-limited runs: evaluate them on the fly from the points).
 * kernel_state must come from gofmm_kernel_create (below) and describe the
 * matrix c was built from (same n, points in the original order, at most 8
 * coordinates); the library copies what it needs, so the state may be freed
 * afterwards.  The plan is rebuilt: P and the coupling blocks are sampled
 * again through the state (threads <= 0: all host threads), the near blocks
 * are dropped from the operator, and every evaluate computes them in FP32,
 * entry by entry from the points (kernel of the squared distance, summed
 * coordinate by coordinate, plus the shift where the two indices are equal),
 * inside the L2L launch, whatever near_storage says.  On success the device
 * copy of the previous plan is released (the next prepare or evaluate uploads
 * the new one).  Compressions in this mode cannot be
 * batched or served (GOFMM_EINVAL there).  Errors: GOFMM_EINVAL for NULL
 * arguments, a pointer that is not such a state, more than 8 coordinates or a
 * different n; sampling errors as for gofmm_compress, after which c is
 * unchanged (its previous plan and device copy stay in use).
 */
int gofmm_use_device_kernel(gofmm_compression* c, void* kernel_state, int32_t threads);

/* Write the structure of a compression (tree, permutation, lists, skeletons,
 * P; no kernel blocks) to `path`, the format gofmm_import and the test
 * oracle read.  GOFMM_EINVAL for NULL arguments, GOFMM_EIO if the file
 * cannot be written. */
int gofmm_export(const gofmm_compression* c, const char* path);

/*
 * Upload the operator to the current HIP device and size the workspace for
 * up to r_max right-hand sides.  Synchronous.  Called implicitly by the
 * first evaluate with the r of that call if not called before.
 */
int gofmm_prepare(gofmm_compression* c, int64_t r_max);

/*
 * U = K~ W (Alg. Evaluate: N2S, S2S, S2N, L2L).  W and U are device arrays
 * of n rows in the original order, row-major with leading dimensions ldw,
 * ldu >= r (FP32), and must not overlap.  Every row of U is overwritten.
 * Work is enqueued on `hip_stream` (NULL = default stream) and the call
 * returns without synchronizing.  Evaluates of one compression must run on
 * the device in the order they are made (one stream, or streams the caller
 * orders): they share its workspace, and, when the environment sets
 * GOFMM_PASSES=1, the counters of its persistent tree passes (the upward and
 * the downward pass then each run as one launch whose tiles wait for the
 * tiles they read, through counters that only grow).  r == 0 is a no-op;
 * r > r_max of a previous prepare grows the workspace synchronously.
 * Errors: GOFMM_EINVAL (NULL c, W or U, r < 0, ldw or ldu < r, W and U
 * overlapping, a compression prepared on another device), GOFMM_ELIMIT (ldw
 * above 2^32 - 1), GOFMM_ENOMEM (the workspace), GOFMM_EHIP (a launch or copy
 * failed).
 */
int gofmm_evaluate(gofmm_compression* c, int64_t r,
                   const float* W, int64_t ldw, float* U, int64_t ldu,
                   void* hip_stream);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the same
 * product as gofmm_evaluate, with the same kernels and the same bits, whose
 * skeleton workspace (w~ and u~ rows) and work-item lists live in a fixed
 * device array of the library, GOFMM_SCRATCH_BYTES bytes per device, held
 * from the first such call on a device until the process ends.  The call
 * allocates and frees no device memory: c must already be on the current
 * device (gofmm_prepare, or any earlier evaluate there); it copies the work
 * items into the array (one asynchronous host-to-device copy on hip_stream)
 * and enqueues the launches.  Every call on a device shares the one array:
 * calls that overlap on a device (different streams not ordered by the
 * caller, or several threads) race and give wrong results; calls on one
 * stream are ordered.  The opt-in persistent tree passes (GOFMM_PASSES) are
 * not used here.  Argument rules as for gofmm_evaluate.  Errors: GOFMM_EINVAL
 * also when c is not on the device yet; GOFMM_ELIMIT when the workspace for
 * r (2 sum_a s_a rows of r FP32 values, r rounded up to a multiple of 4) and
 * the work items exceed GOFMM_SCRATCH_BYTES (use a smaller r or
 * gofmm_evaluate); GOFMM_EHIP for a failed copy or launch.
 */
#define GOFMM_SCRATCH_BYTES (256ll << 20)
int gofmm_evaluate_noalloc(gofmm_compression* c, int64_t r,
                           const float* W, int64_t ldw, float* U, int64_t ldu,
                           void* hip_stream);

/*
 * Same product as gofmm_evaluate, after timing every tile configuration of
 * every launch for this r and keeping the fastest (later evaluates with the
 * same r reuse the choice).  Each configuration is timed inside whole
 * evaluates (events around the tuned launch only) when all of them fit a few
 * seconds, else by repeating the launch on its own.  Synchronizes the
 * stream.  Errors as for gofmm_evaluate.
 */
int gofmm_autotune(gofmm_compression* c, int64_t r,
                   const float* W, int64_t ldw, float* U, int64_t ldu,
                   void* hip_stream);

/*
 * k independent products U_i = K~_i W_i (Alg. Evaluate for each, Sec. 2.2)
 * in one persistent launch: a single grid walks the union of all instances'
 * tiles in step order, and a tile waits only for the tasks whose rows it
 * reads (a node's N2S for its children's, S2S for the upward pass, a node's
 * S2N for its parent's and its own S2S, the leaf output for its S2N), through
 * counters of finished tiles.  Same argument rules as gofmm_evaluate, per
 * instance; arrays c, r, W, ldw, U, ldu hold k entries each (k == 0 is a
 * no-op).  The k compressions must be distinct and share one storage
 * precision.  Errors: GOFMM_EINVAL (k < 0, NULL arrays or entries, a repeated
 * compression, outputs of two instances that overlap, mixed precisions, r < 1,
 * a compression in device-kernel mode),
 * GOFMM_EHIP.
 */
int gofmm_evaluate_batched(int32_t k, gofmm_compression* const* c, const int64_t* r,
                           const float* const* W, const int64_t* ldw,
                           float* const* U, const int64_t* ldu, void* hip_stream);

/*
 * Time the batched launch of these k products with every tile configuration
 * and keep the fastest for this set of compressions and r values (later
 * batched calls with the same set reuse it).  Leaves U_i = K~_i W_i.
 * Synchronizes the stream.
 */
int gofmm_autotune_batched(int32_t k, gofmm_compression* const* c, const int64_t* r,
                           const float* const* W, const int64_t* ldw,
                           float* const* U, const int64_t* ldu, void* hip_stream);

/*
 * Wait for the device and report the last batched launch on this process:
 * *error = 1 if a block gave up a dependency wait (see
 * gofmm_batched_spin_limit), else 0.  The flag is cleared on the next launch.
 */
int gofmm_batched_status(int32_t* error);

/*
 * Bound on the polls of one dependency wait in batched launches (default
 * 2^21, a few seconds).  A wait that reaches it sets the error flag and its
 * tile is skipped, so a launch always ends.  <= 0 restores the default.
 */
int gofmm_batched_spin_limit(int64_t polls);

/*
 * Wait for the device and report the persistent tree passes of c: *error = 1
 * if a block of one of its passes gave up a dependency wait since the last
 * call (the same bound as gofmm_batched_spin_limit), else 0.  Clears the flag.
 * An evaluate returns before its launches run, so its return code cannot
 * carry this: a wait that gives up skips its tile and the evaluate's output
 * is wrong while the call itself returned GOFMM_OK.  Callers that enable the
 * persistent passes (GOFMM_PASSES=1) must call this after their evaluates
 * and discard the outputs of any evaluate it flags.  The default separate
 * launches never wait and never set the flag.
 */
int gofmm_evaluate_status(gofmm_compression* c, int32_t* error);

/*
 * Launches of one evaluate, in order.  For launch i: its name (e.g. "n2s_leaf",
 * "n2s_l3", "s2s", "s2n_l4", "leaf"), the Table 2 flops it performs per
 * right-hand side (2 m k summed over its tasks, internal N2S/S2N counted as
 * 2 s_a (s_l + s_r)), and the operator bytes it reads.  name receives at
 * most name_len bytes including the terminator.  GOFMM_EINVAL for NULL
 * arguments or i outside [0, count).
 */
int gofmm_launch_count(const gofmm_compression* c, int32_t* count);
int gofmm_launch_info(const gofmm_compression* c, int32_t i, char* name, int32_t name_len,
                      double* flops_per_rhs, int64_t* operator_bytes);

/*
 * Per-launch timing.  While enabled, every evaluate of c records a HIP event
 * before and after each of its launches on the evaluation stream (no extra
 * synchronization).  enable: 0 off, 1 every launch, 2 + i launch i only (two
 * events per evaluate, for timing one launch inside a timed loop).
 * gofmm_profile_read waits for the recorded events, writes for each launch
 * i < n the summed milliseconds and the number of recorded launches, and
 * clears the records.
 */
int gofmm_profile(gofmm_compression* c, int32_t enable);
int gofmm_profile_read(gofmm_compression* c, int32_t n, float* total_ms, int32_t* calls);

/* Device bytes a compression holds once prepared for r_max right-hand sides
 * (operator, tables, work-item lists, workspace); host-side, no GPU call.
 * GOFMM_EINVAL for NULL arguments or r_max < 1. */
int gofmm_footprint(const gofmm_compression* c, int64_t r_max, int64_t* bytes);

/* Fill `out` with the summary of c (flops per phase as Table 2 counts them,
 * see gofmm_launch_info).  GOFMM_EINVAL for NULL arguments. */
int gofmm_stats(const gofmm_compression* c, gofmm_stats_t* out);

/* Release a compression (host and device).  NULL is ignored. */
void gofmm_free(gofmm_compression* c);

/* Message of the last failed call on this thread ("" if none). */
const char* gofmm_last_error(void);

/* ------------------------------------------------------------- serving
 * A request loop on its own host thread.  Compressions ("models") stay
 * resident on the current device; a model is admitted, in the order added,
 * once its footprint (gofmm_footprint for r_max plus two n x r_max FP32
 * staging blocks) fits the HBM budget next to the models already resident,
 * and its requests wait until then.  Requests U = K~ W for a model may be
 * submitted at any time from any thread.  Whenever one of the server's
 * streams is free, every resident model with pending requests and no work in
 * flight joins one batched persistent launch (at most max_batch models, one
 * storage precision); a model's pending requests are packed side by side as
 * columns (at most r_max in total), so requests that arrive while others run
 * are admitted as streams and models free up.  A request's result is the same
 * as its standalone evaluate, whatever it was batched with.
 */
typedef struct gofmm_server gofmm_server;

typedef struct {
  int64_t completed, failed, pending, inflight, models, admit_queue;
  int64_t batches;            /* batched launches made */
  int64_t columns;            /* right-hand sides evaluated */
  int64_t packed;             /* model launches that packed several requests */
  int64_t hbm_used, hbm_budget;
  double p50_ms, p99_ms, mean_ms, max_ms;   /* latency, submit to completion */
  double elapsed_ms;          /* since creation or the last reset */
  int64_t max_inflight;       /* most batches on the device at once */
  int64_t admissions;         /* models made resident */
  double host_ms_mean;        /* host time to form and enqueue one batch */
  double admit_ms_mean;       /* host time of one admission (upload, staging) */
  double p99_ms_admitting;    /* p99 latency of requests finished while an admission ran */
} gofmm_server_stats_t;

/* Start a server with `streams` concurrent batches (1..16) on the current
 * device.  The server owns its streams and staging; not its compressions. */
int gofmm_server_create(int64_t hbm_budget_bytes, int32_t streams, int32_t max_batch,
                        gofmm_server** out);

/* Serve compression c for requests of up to r_max right-hand sides.  c must
 * stay alive until removed; while served, its device memory belongs to the
 * server.  GOFMM_ENOMEM if its footprint alone exceeds the budget. */
int gofmm_server_add(gofmm_server* s, gofmm_compression* c, int64_t r_max, int32_t* model);

/* Wait for the model's work in flight, fail its pending requests, release its
 * device memory (the compression itself stays valid). */
int gofmm_server_remove(gofmm_server* s, int32_t model);

/* Enqueue U = K~ W (device arrays as for gofmm_evaluate, 1 <= r <= r_max).
 * W must already hold its values (the server's streams do not wait on the
 * caller's streams); W and U must stay valid and untouched until the request
 * completes. */
int gofmm_server_submit(gofmm_server* s, int32_t model, int64_t r, const float* W, int64_t ldw,
                        float* U, int64_t ldu, int64_t* request);

/* Block until the request completes (at most timeout_ms; <= 0 waits without
 * bound); its latency in ms.  The request id is then retired.  A failed
 * request returns GOFMM_EHIP with the reason; GOFMM_ETIMEDOUT leaves it
 * pending (wait again or test later). */
int gofmm_server_wait(gofmm_server* s, int64_t request, int64_t timeout_ms, double* latency_ms);

/* Non-blocking: *done = 1 (and the id is retired) if the request completed. */
int gofmm_server_test(gofmm_server* s, int64_t request, int32_t* done, double* latency_ms);

int gofmm_server_stats(gofmm_server* s, gofmm_server_stats_t* out);
int gofmm_server_reset_stats(gofmm_server* s);

/* Finish all submitted work, release every model's device memory, stop. */
void gofmm_server_destroy(gofmm_server* s);

/* ------------------------------------------------ synthetic kernel sampler
 * A ready-made thread-safe sampler for radial kernels over a point cloud the
 * library copies and keeps hidden from the method:
 *   kind 0  exp(-|x - y|^2 / (2 h^2))       (Gaussian)
 *   kind 1  1 / sqrt(1 + |x - y|^2 / h^2)   (inverse multiquadric)
 *   kind 2  1 / (|x - y| + 0.05)            (Laplacian-like)
 * plus shift on the diagonal.  points: n x dim row-major FP64 (host).
 * Pass gofmm_kernel_sample as the sampler and *state as its user pointer.
 */
int gofmm_kernel_create(int32_t kind, int64_t n, int32_t dim, const double* points,
                        double h, double shift, void** state);
/* Sampler layout as above (out[i + j * ld], ld >= nI); returns 1 for a NULL
 * state or arrays or ld < nI, 2 for an index outside [0, n). */
int gofmm_kernel_sample(void* state, int64_t nI, const int64_t* I,
                        int64_t nJ, const int64_t* J, double* out, int64_t ld);
void gofmm_kernel_free(void* state);

#ifdef __cplusplus
}
#endif
#endif /* GOFMM_H */
