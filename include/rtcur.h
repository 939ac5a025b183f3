/*
 * rtcur.h - C ABI of librtcur, Robust Tensor CUR (RTCUR) on one gfx950 GPU.
 *
 * RTCUR (Cai, Chao, Huang, Needell, "Fast Robust Tensor Principal Component
 * Analysis via Fiber CUR Decomposition", Algorithm 1) splits an observed
 * n-mode tensor X = L + S into a low-multilinear-rank part L and a sparse
 * outlier part S by alternating projections that only ever touch sampled
 * entries of X:
 *
 *   - Omega: index sets I_i (rows of mode i, |I_i| = s_i) and J_i (columns of
 *     the mode-i unfolding, |J_i| = m_i).  The sampled blocks are the core
 *     subtensor R = X(I_1, ..., I_n) and the fiber blocks C_i = X_(i)(:, J_i).
 *   - Step (I), equations 11-13: S = HT_zeta(X - L) on the blocks, with
 *     zeta_{k+1} = gamma * zeta_k (equation 12) and HT keeping |x| > zeta.
 *   - Step (II), equations 8-9: L = R x_i (C_i U_i^+) with U_i = C_i(I_i, :)
 *     truncated to rank r_i; only the factors are kept (Section 3.3).
 *   - Stop when e^(k) <= tol, e^(k) the sampled relative error of
 *     equation 14.
 *   - RTCUR-F keeps one sample; RTCUR-R draws a new one before every iteration
 *     after the first (Section 3.4).
 *
 * Conventions
 *   - Tensors are dense, C-contiguous (last mode fastest), on the device.
 *     The mode-i unfolding numbers its columns in C order over the remaining
 *     modes.
 *   - All entry points return an int status (RTCUR_OK or one of the codes
 *     below); no exception or abort crosses the ABI.  rtcur_last_error gives
 *     a per-handle message for the last failure.
 *   - A handle is not thread-safe.  All device work runs on the stream given
 *     to rtcur_create, in stream order; rtcur_solve returns after its device
 *     work has finished.
 *   - Limits: 2 <= n <= 4; 1 <= r_i <= 16 for every n; prod(r_i) <= 4096;
 *     s_i <= 256; with n = 4, r_3 * s_1 * s_2 <= 2048 (one slice of the
 *     sampled core; with n = 3 every slice, r_2 * s_1 <= 4096, fits);
 *     prod(d_i) <= 2^40.  Shapes beyond them return RTCUR_E_INVAL before
 *     any device work.
 */
#ifndef RTCUR_H
#define RTCUR_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct rtcur_s* rtcur_t;

enum rtcur_status {
    RTCUR_OK = 0,
    RTCUR_NOT_CONVERGED = 1,  /* max_iter reached with e > tol; results valid */
    RTCUR_E_INVAL = -1,       /* invalid argument                              */
    RTCUR_E_NOMEM = -2,       /* device or host allocation failed              */
    RTCUR_E_HIP = -3,         /* HIP runtime error (includes: no device)       */
    RTCUR_E_RANK = -4,        /* some U_i has numerical rank below r_i         */
    RTCUR_E_NONFINITE = -5,   /* NaN/Inf in sampled X, max|X| or e^(k)         */
    RTCUR_E_STATE = -6        /* call out of order (e.g. reconstruct first)    */
};

enum rtcur_dtype { RTCUR_F64 = 0, RTCUR_F32 = 1, RTCUR_BF16 = 2 /* compute only */ };
enum rtcur_variant { RTCUR_FIXED = 0 /* RTCUR-F */, RTCUR_RESAMPLE = 1 /* RTCUR-R */ };
enum rtcur_block_what { RTCUR_BLOCK_X = 0, RTCUR_BLOCK_C = 1, RTCUR_BLOCK_L = 2,
                        RTCUR_BLOCK_SUPPORT = 3 };

typedef struct {
    int32_t iters;       /* number of L-updates done (k)                      */
    int32_t converged;   /* 1 if e^(k) <= tol                                 */
    double err;          /* e^(k), equation 14, of the returned iterate       */
    double zeta;         /* zeta_k, the last threshold used                   */
    double zeta0;        /* zeta_0 used (given, or max|X|)                    */
    int32_t eig_steps;   /* total subspace-iteration steps of the eigensolver */
    int32_t status;      /* status of the last rtcur_solve                    */
    int32_t eig_unconverged; /* eigensolver calls that stopped at their step
                                limit before the residual test passed (a
                                near-degenerate gap sigma_r ~ sigma_{r+1})   */
    double solve_ms;     /* host wall-clock time of the solve, from the call's
                            entry to its return (device work included)        */
    int32_t batch_slot;  /* rtcur_solve_batch: index in hs of the handle that
                            solved the instance; -1 for rtcur_solve           */
    int32_t batch_seq;   /* rtcur_solve_batch: the instance's position in that
                            handle's sequence of solves (0 first); else -1    */
} rtcur_info;

/* Create a solver bound to HIP device `device` and stream `hip_stream`
 * (a hipStream_t; NULL = the null stream).  variant: RTCUR_FIXED or
 * RTCUR_RESAMPLE.  compute_dtype: RTCUR_F64 or RTCUR_F32, the precision of
 * the sampled blocks, factors and the rebuilt L; the truncated SVD and the
 * stopping-rule norms always run in float64.  RTCUR_BF16 (RTCUR_FIXED only)
 * stores the sampled blocks in bfloat16 (factors, L and arithmetic in
 * float) while e^(k) > max(tol, 1e-2), then finishes with float blocks (the
 * FP32 refinement sweep) from that iterate; results and getters are then
 * those of a float32 handle.  Fails with RTCUR_E_HIP when no usable device
 * exists.  *out is set to NULL on failure. */
int rtcur_create(rtcur_t* out, int device, void* hip_stream, int variant,
                 int compute_dtype);

/* Run Algorithm 1 on the device tensor X (x_dtype RTCUR_F64 or RTCUR_F32,
 * dims[0..n) C-contiguous, read-only, borrowed for this call only).
 *   ranks[i]   target multilinear rank r_i (Algorithm 1 input)
 *   I_sizes[i] s_i = |I_i|, with r_i <= s_i <= dims[i]
 *   J_sizes    NULL: chidori sampling, J_i = product of I_j (j != i);
 *              else m_i = |J_i| fiber columns, r_i <= m_i <= prod_{j!=i} d_j
 *   zeta0      initial threshold; <= 0 means max|X| over the whole tensor
 *   gamma      threshold decay, 0 < gamma < 1 (equation 12)
 *   tol        target e^(k) (equation 14), >= 0; stop when e^(k) <= tol
 *   max_iter   >= 1 L-updates at most; RTCUR_NOT_CONVERGED if reached
 *   seed       sampler seed; samples are a pure function of (seed, t, dims,
 *              sizes), identical to the oracle's
 *   info       optional summary (may be NULL)
 * The handle keeps the samples, blocks and factors until the next solve or
 * destroy.  Returns RTCUR_OK, RTCUR_NOT_CONVERGED or an error; after
 * RTCUR_E_RANK / RTCUR_E_NONFINITE the handle stays usable. */
int rtcur_solve(rtcur_t h, const void* X, int x_dtype, int32_t n,
                const int64_t* dims, const int32_t* ranks,
                const int64_t* I_sizes, const int64_t* J_sizes, double zeta0,
                double gamma, double tol, int32_t max_iter, uint64_t seed,
                rtcur_info* info);

/* Write the full L = R x_i (C_i U_i^+) of the last solve (Algorithm 1
 * output, expanded over every entry) into the caller's device buffer L_out
 * of prod(dims) elements, C-contiguous, dtype out_dtype (RTCUR_F64/F32).
 * RTCUR_E_STATE if no successful solve precedes it. */
int rtcur_reconstruct(rtcur_t h, void* L_out, int out_dtype);

/* Allocation-free variant of rtcur_reconstruct, for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc.  It writes the same L into L_out (same
 * kernels, same values bit for bit) but keeps its temporaries (the Tucker
 * expansion over the full mode-0 unfolding, RP x prod_{j>0} dims[j] entries
 * of the compute type, RP = max r_i padded to 4, 8 or 16, plus its work list)
 * in a static device array of 64 MiB that each GPU holds once for the
 * process, and calls no hipMalloc, hipFree, memset or host-to-device copy:
 * every step is a kernel launch on the handle's stream.  It does not wait for
 * the device: L_out is ready once the handle's stream has reached this point
 * (synchronize that stream, or order later work after it).
 *   L_out      caller's device buffer, prod(dims) elements of out_dtype
 *              (RTCUR_F64/F32), C-contiguous; written by the queued kernels
 * RTCUR_E_INVAL (nothing queued) when the temporaries exceed 64 MiB;
 * RTCUR_E_STATE if no successful solve precedes it.  All calls on one GPU
 * share that GPU's array, which keeps the last call's contents: calls that
 * overlap on one GPU (on different streams or from different threads) race
 * and must be ordered by the caller. */
int rtcur_reconstruct_noalloc(rtcur_t h, void* L_out, int out_dtype);

/* Full-grid outliers (the S-update of equation 11, S = HT_zeta(X - L) with
 * the strict threshold of equation 10, applied to every entry of X rather
 * than only to the sampled blocks), fused with the reconstruction of L:
 *   X       device, C-contiguous, prod(dims) elements of x_dtype
 *           (RTCUR_F64/F32), the dims of the last solve; read-only.
 *   zeta    threshold; <= 0 means the threshold of the returned iterate,
 *           zeta_K (zeta_0 when the solve did no iteration).
 *   S_out   caller's device buffer, prod(dims) elements of out_dtype:
 *           X - L where |X - L| > zeta, else 0 (X - L formed in the solve's
 *           compute type).
 *   L_out   NULL, or a caller's device buffer receiving L as
 *           rtcur_reconstruct would (out_dtype).
 * One read of X and one write per output; blocks until done.
 * RTCUR_E_STATE if no successful solve precedes it. */
int rtcur_outliers(rtcur_t h, const void* X, int x_dtype, double zeta, void* S_out,
                   void* L_out, int out_dtype);

/* Many independent instances (a batch of tensors of uneven shapes and
 * ranks), solved concurrently: each of the nh handles is driven by its own
 * host thread, so handles bound to distinct streams overlap their kernels on
 * the device (the HIP runtime maps a process's streams onto
 * GPU_MAX_HW_QUEUES hardware queues, 4 unless set; streams that share a
 * queue run their kernels one after another, so nh concurrent handles want
 * at least nh queues, set before the runtime starts).  Schedule: one work queue holds the instances in decreasing
 * expected cost (ties: lower j first) -- the solve times this process last
 * measured in a batch for the same problem (sizes, ranks, sample sizes, the
 * first handle's compute dtype and variant, gamma, tol, max_iter) when every
 * instance has one, else the number of entries; each handle's thread takes
 * the next instance whenever its previous solve has returned, so that slow
 * instances (many iterations or eigensolver steps) start first and do not
 * hold back the others.  Which handle solves which instance depends on timing; infos[j]
 * records it (batch_slot, batch_seq).  Each instance is Algorithm 1 exactly
 * as rtcur_solve runs it (same results bit for bit, whichever handle runs
 * it).
 *   hs, nh     nh >= 1 distinct handles (their variant and compute dtype
 *              apply); after the call each holds the state of the last
 *              instance it solved (the largest batch_seq among its own)
 *   count      number of instances (>= 0)
 *   X[j]       device tensor of instance j, x_dtype, C-contiguous, read-only
 *   n[j]       its number of modes; dims, ranks, I_sizes (and J_sizes when
 *              not NULL; NULL = chidori for all) hold 4 entries per instance
 *              (entries beyond n[j] ignored): dims[4j .. 4j+n[j])
 *   zeta0      NULL (max|X| for all) or count values (<= 0: max|X|)
 *   gamma, tol, max_iter   shared, as in rtcur_solve
 *   seeds[j]   sampler seed of instance j
 *   L_out      NULL, or count device pointers (NULL entries skipped) that
 *              receive instance j's full L (prod dims elements, out_dtype)
 *   infos      NULL or count summaries (with solve_ms, batch_slot and
 *              batch_seq); status[j] = rtcur_solve's result for instance j
 *              (or rtcur_reconstruct's error)
 * Returns the first error status by j, else RTCUR_NOT_CONVERGED if any
 * instance did not converge, else RTCUR_OK; RTCUR_E_INVAL for bad arguments
 * (NULL arrays, repeated handles) before any work. */
int rtcur_solve_batch(rtcur_t* hs, int32_t nh, int32_t count, const void* const* X,
                      int x_dtype, const int32_t* n, const int64_t* dims,
                      const int32_t* ranks, const int64_t* I_sizes, const int64_t* J_sizes,
                      const double* zeta0, double gamma, double tol, int32_t max_iter,
                      const uint64_t* seeds, void* const* L_out, int out_dtype,
                      rtcur_info* infos, int32_t* status);

/* Tile autotuner for the per-iteration kernels (the threshold pass of
 * equations 10-11 over the sampled blocks, the Gram of the truncated SVD of
 * equation 9 and the B-factor mode products of equation 8 in core form):
 * times candidate tile shapes on this problem and records the fastest in a
 * process-wide table keyed by the problem sizes (dims, ranks, I_sizes,
 * J_sizes, sampling kind, block element size), which every later layout of
 * those sizes -- on any handle, in rtcur_solve and rtcur_solve_batch --
 * uses.  Candidates, by coordinate descent from the built-in rule: rows per
 * threshold tile (8, 16, 32; 32 not for float64 blocks), columns per Gram
 * work item (512 .. 8192), Z sub-chunks per B-factor work item (1 .. 8);
 * each timed as the best of `reps` solves of `iters` iterations (tol 0,
 * gamma 0.7, zeta_0 = max|X|, seed) after one warm-up, host wall clock.
 * Tile shapes change only the order of floating-point sums (the Gram over
 * column chunks, B over sub-chunks), so results agree to rounding with the
 * built-in rule; a solve is bit-for-bit reproducible for a fixed table.
 *   X, x_dtype, n, dims, ranks, I_sizes, J_sizes   as in rtcur_solve
 *   iters (1..1000), reps (1..100), seed
 *   tile       out, 3 values: rows per tile, Gram chunk columns (0: built-in
 *              rule), B sub-chunks (0: built-in rule)
 *   tuned_ms, default_ms   out (nullable): best candidate's time and the
 *              built-in rule's
 * The handle is left holding the last candidate's solve.  Errors as
 * rtcur_solve; the table is unchanged on error. */
int rtcur_autotune(rtcur_t h, const void* X, int x_dtype, int32_t n, const int64_t* dims,
                   const int32_t* ranks, const int64_t* I_sizes, const int64_t* J_sizes,
                   int32_t iters, int32_t reps, uint64_t seed, int32_t* tile,
                   double* tuned_ms, double* default_ms);
/* Tile shapes of this handle's following solves, overriding the tuned table:
 * tile[0] rows per threshold tile (8, 16 or 32; float64 blocks use 16 for
 * 32), tile[1] columns per Gram work item (0: built-in rule, else a multiple
 * of 256), tile[2] Z sub-chunks per B-factor work item (0: built-in, at most
 * 64; raised to the minimum the partial-row limit needs).  NULL: back to the
 * table.  RTCUR_E_INVAL for other values. */
int rtcur_set_tiles(rtcur_t h, const int32_t* tile);
/* Replayed iteration graphs for this handle's RTCUR-F solves (enable != 0):
 * from the third iteration on, each pair of iterations (the threshold pass
 * and the L-update of equations 8-14, twice) is one executable HIP graph,
 * captured once per layout on a private stream and replayed with
 * hipGraphLaunch; the iteration index lives on the device.  Results are
 * bit for bit those of kernel-by-kernel launches.  Off by default: on the
 * measured stack a replayed pair takes a few microseconds longer than its
 * launches one by one, and a capture costs about half a millisecond per new
 * layout; it pays only where the host cannot keep the launch queue full.
 * Ignored while profiling is on. */
int rtcur_set_graphs(rtcur_t h, int32_t enable);
/* Empties the autotuner's table: every solve afterwards uses the built-in
 * rule.  Thread-safe; not to be called while solves run. */
int rtcur_autotune_clear(void);

/* Threshold schedule of the following solves on this handle (a learned
 * alternative to equation 12's decay, Section 3.2): iteration k <= n
 * thresholds with zeta_k = multipliers[k-1] * zeta_0, later iterations
 * continue the decay from the last one, zeta_k = gamma zeta_(k-1) (repeated
 * float64 multiplication).  n = 0 restores the geometric schedule
 * zeta_k = gamma^k zeta_0 throughout.  The multipliers (host, n positive
 * finite values) are copied; entries beyond a solve's max_iter are unused.
 * RTCUR_E_INVAL for a negative n or a non-positive multiplier. */
int rtcur_set_schedule(rtcur_t h, const double* multipliers, int32_t n);

/* Release the handle and its device workspace.  NULL-safe. */
int rtcur_destroy(rtcur_t h);

/* ---- introspection (host copies; for tests and diagnostics, not hot) ---- */

/* Indices of the sample the returned iterate lives on: which = 0 gives I_i
 * (sorted), which = 1 gives J_i as mode-i unfolding column numbers (C order,
 * sorted).  Copies min(cap, length) values; *len = length. */
int rtcur_get_indices(rtcur_t h, int32_t mode, int32_t which, int64_t* out,
                      int64_t cap, int64_t* len);

/* e^(1..k) and zeta_1..zeta_k of the last solve.  *len = k. */
int rtcur_get_history(rtcur_t h, double* err, double* zeta, int32_t cap,
                      int32_t* len);

/* One sampled block of the returned iterate as float64 on the host:
 * block 0 = R (s_1 x ... x s_n, C order), block 1+i = C_i (d_i x m_i,
 * row-major).  what: RTCUR_BLOCK_X (gathered X), RTCUR_BLOCK_C (X - S),
 * RTCUR_BLOCK_L (L on the block), RTCUR_BLOCK_SUPPORT (1.0 where S != 0).
 * *len = number of entries of the block. */
int rtcur_get_block(rtcur_t h, int32_t block, int32_t what, double* out,
                    int64_t cap, int64_t* len);

/* Tucker form of the returned L = G x_1 B_1 ... x_n B_n: core G (prod r_i,
 * C order) and B_i (d_i x r_i, row-major), float64 host buffers.  Either
 * pointer may be NULL.  B is an array of n host pointers. */
int rtcur_get_tucker(rtcur_t h, double* core, double* const* B);

/* Host-only sampler (no device needed): the index set of Algorithm 1's
 * sampling step for resample counter t, mode `mode`; which = 0 gives I_mode,
 * which = 1 gives J_mode column numbers (chidori when J_sizes is NULL).
 * Same definition as the solver uses. */
int rtcur_sample(uint64_t seed, int64_t t, int32_t n, const int64_t* dims,
                 const int64_t* I_sizes, const int64_t* J_sizes, int32_t mode,
                 int32_t which, int64_t* out, int64_t cap, int64_t* len);

/* Kernel timing for diagnostics and roofline figures.  With mask != 0 the
 * following solves record a pair of HIP events on the handle's stream around
 * every launch of the selected kernel kinds (bit k selects kind k, as
 * numbered by rtcur_get_profile; a negative mask selects all of them); only
 * launches that did work (not those skipped after the stop flag was raised)
 * are accumulated.  Each event pair makes its launch wait for the one
 * before, which costs a few microseconds, so time throughput with few kinds
 * (or none) selected.  mask = 0 stops recording; the totals persist until
 * recording is next switched on from off. */
int rtcur_set_profiling(rtcur_t h, int32_t mask);

/* Totals for kernel kind `kind` (0 .. count-1): its name (NUL-terminated,
 * truncated to name_cap), summed event time in ms and launch count.
 * RTCUR_E_INVAL when kind is out of range. */
int rtcur_get_profile(rtcur_t h, int32_t kind, char* name, int32_t name_cap,
                      double* total_ms, int64_t* launches);

const char* rtcur_strerror(int status);
const char* rtcur_last_error(rtcur_t h);

/* ---- differentiable unrolled RTCUR-F (float64, three modes) ----
 *
 * K iterations of Algorithm 1 on one fixed chidori sample (resample counter
 * 0) with the thresholds zeta_1..zeta_K as inputs instead of the decay of
 * equation 12, and the adjoint of those K iterations with respect to the
 * thresholds and to X, for learning the threshold schedule (Section 3.2's
 * zeta_k).  The threshold of equation 10 is the strict hard threshold when
 * tau = 0 and the gate S = D sigmoid((|D| / zeta - 1) / tau) when tau > 0
 * (the hard threshold has zero derivative in zeta almost everywhere; with
 * tau > 0 the forward pass is the function whose derivative the backward
 * pass returns).  The L-update is equation 8's literal form: A_i = C_i U_i^+
 * with U_i^+ the pseudo-inverse of the rank-r_i truncation (from the
 * eigendecomposition of U_i U_i^T), L = R x_i A_i on the sampled blocks.
 * All arithmetic is float64.  Block buffers hold R (s_0 x s_1 x s_2, C
 * order) then C_0, C_1, C_2 (d_i x m_i row-major), m_i = prod_{j!=i} s_j. */
typedef struct rtcur_unroll_s* rtcur_unroll_t;

/* Plan an unrolled pass: n = 3, r_i <= s_i <= min(d_i, 96), 1 <= K <= 1000;
 * draws the sample from seed.  Allocates the device workspace, including K
 * checkpoints of the factor form of L^k (R^k, A_i^k and the Grams'
 * eigenpairs: O(K (s^3 + sum_i d_i s_i)) doubles, never K block buffers). */
int rtcur_unroll_create(rtcur_unroll_t* out, int device, void* hip_stream, int32_t n,
                        const int64_t* dims, const int32_t* ranks, const int64_t* I_sizes,
                        int32_t K, uint64_t seed);
/* Number of block entries (*n_blk) and, when idx_out is not NULL (cap >=
 * n_blk), the offset in X of every block entry, in block-buffer order. */
int rtcur_unroll_blocks(rtcur_unroll_t u, int64_t* n_blk, int64_t* idx_out, int64_t cap);
/* Forward pass on the device tensor X (x_dtype RTCUR_F64 or RTCUR_F32, the
 * planned dims): zetas (host, K positive values), tau >= 0; writes L^K on
 * the blocks into L_out (device, n_blk doubles).  Blocks until done.
 * RTCUR_E_RANK when some U_i met has sigma_r <= max(s_i, m_i) 2^-52 sigma_1. */
int rtcur_unroll_forward(rtcur_unroll_t u, const void* X, int x_dtype, const double* zetas,
                         double tau, double* L_out);
/* Backward pass of the last forward: given L_bar = dloss / dL^K on the
 * blocks (device, n_blk doubles), writes dloss / dzeta_k into zeta_bar (host,
 * K) and dloss / dX into X_bar (device, prod(dims) doubles; zero off the
 * sampled blocks).  RTCUR_E_STATE without a successful forward pass. */
int rtcur_unroll_backward(rtcur_unroll_t u, const double* L_bar, double* zeta_bar,
                          double* X_bar);
int rtcur_unroll_destroy(rtcur_unroll_t u);  /* NULL-safe */
const char* rtcur_unroll_last_error(rtcur_unroll_t u);

#ifdef __cplusplus
}
#endif

#endif /* RTCUR_H */
