/* mimo_sd.h -- C ABI of the MI355X (gfx950) sphere-decoder library.
 *
 * Hot path of Dabah et al., "Performance / Complexity Trade-offs of the
 * Sphere Decoder Algorithm for Massive MIMO Systems" (arXiv 2002.09561):
 * detection of s in argmin ||y - H s||^2 over a square-QAM lattice after the
 * QR transform z = Q^T y.
 *
 * General conventions (apply to every entry point below)
 * -------------------------------------------------------
 * Memory   All array arguments are DEVICE pointers owned by the caller; the
 *          library never allocates, frees or retains them, and allocates no
 *          device memory of its own except a workspace the caller passes in.
 * Streams  `stream` is a hipStream_t passed as void* (NULL = the default
 *          stream).  Every call only enqueues work on it and returns; no call
 *          synchronises the host, so calls may be captured into a hipGraph.
 *          Results are valid once the stream has reached the call.
 * Errors   0 = MIMO_OK.  Negative codes are returned *before* any work is
 *          enqueued when an argument is invalid (checked on the host, so the
 *          checks run without a GPU); MIMO_ERR_HIP reports a failed launch.
 *          mimo_last_error() returns a thread-local text for the last error.
 *          B == 0 is a no-op that returns MIMO_OK.
 * Frames   B frames of an N x M system (N = n_rx receive antennas, M = n_tx
 *          transmit streams, M <= N).  The paper's system model is Sec. III-A
 *          Eq. (1): y = H s + n.  H is [B][N][M] complex64 row-major, y is
 *          [B][N] complex64 (complex64 = two floats, real first).
 * Lattice  Square QAM with P = sqrt(|Omega|) points per real dimension,
 *          pam = P in {2, 4, 8} (4-, 16-, 64-QAM); real amplitudes
 *          (2i - (P-1)) c with c = sqrt(3 / (2 (|Omega| - 1))), i = 0..P-1
 *          (unit average symbol energy).  The QAM index of a symbol is
 *          i_re * P + i_im.  Symbol outputs `sym` are [B][M] int32 QAM indices.
 * Real model  n = 2M real levels: x = [Re s0, Im s0, Re s1, Im s1, ...] and
 *          each complex h becomes [[Re h, -Im h], [Im h, Re h]] (rows
 *          [Re y0, Im y0, ...]).  Level k fixes x_k; searches start at level
 *          n-1 and end at level 0 (Sec. III-B: one symbol per tree level).
 * R layout "packed level order": row k of the upper-triangular n x n matrix R
 *          (entries R_kk, R_k,k+1, ..., R_k,n-1) is stored contiguously at
 *          offset (n-1-k)(n-k)/2, so the rows appear in the order the search
 *          visits them; n(n+1)/2 floats per frame.  z is [B][n].
 * Radius   Squared radius r2 (Sec. III-B "Sphere radius and pruning"): a node
 *          is kept iff its partial distance is < r2.  A NULL radius pointer
 *          means r2 = +infinity.
 * Flags    per frame, OR of MIMO_FLAG_* below.
 * Counters optional [B][4] int64, *overwritten*: nodes expanded (branched
 *          on), partial distances evaluated (children), rounds (hybrid only,
 *          else 0), pool nodes discarded as outside the sphere.
 */
#ifndef MIMO_SD_H
#define MIMO_SD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* return codes */
#define MIMO_OK 0
#define MIMO_ERR_INVALID_ARG (-1)
#define MIMO_ERR_UNSUPPORTED (-2)
#define MIMO_ERR_WORKSPACE (-3)
#define MIMO_ERR_HIP (-4)

/* per-frame flags */
#define MIMO_FLAG_FOUND 1u            /* a leaf inside the radius was found          */
#define MIMO_FLAG_EMPTY_SPHERE 2u     /* the radius left no leaf; the frame was      */
                                      /* detected again with r2 = +infinity          */
#define MIMO_FLAG_BUDGET_EXHAUSTED 4u /* node budget reached; best leaf so far       */
#define MIMO_FLAG_CERTIFIED 8u        /* hybrid pool drained within the budget        */
#define MIMO_FLAG_LEARNED_FALLBACK 16u /* a learned survivor count was invalid        */
#define MIMO_FLAG_NONFINITE_INPUT 32u /* R, z (or H, y) held a NaN or infinity: the  */
                                      /* search stopped; sym = 0, pd = +infinity     */
#define MIMO_FLAG_INVALID_FRAME 64u   /* uneven batch: the frame's descriptor is out */
                                      /* of the kernel's range; outputs untouched    */

/* limits */
#define MIMO_MAX_TX 128   /* n_tx <= 128, i.e. n <= 256 real levels */
#define MIMO_MAX_RX 128
#define MIMO_MAX_K 256    /* K-best survivors: K * pam <= 1024 */
#define MIMO_MAX_WORKERS 15
#define MIMO_HYB_MAX_CAND 64 /* hybrid worker: k_worker * pam <= 64 */
#define MIMO_HYB_MAX_CAND_CPLX 512 /* complex-level hybrid worker: k_worker * pam^2 <= 512 */

#define MIMO_MLP_IN 4
#define MIMO_MLP_HIDDEN 128
/* flat parameter vector: W1[128][4], b1[128], W2[128][128], b2[128], w3[128], b3 */
#define MIMO_MLP_NPARAM (128 * 4 + 128 + 128 * 128 + 128 + 128 + 1)

const char* mimo_last_error(void);
int32_t mimo_version(void);

/* ---------------------------------------------------------------------
 * QR preprocessing (Sec. III-B): H = Q R with R_kk > 0 and z = Q^H y,
 * emitted for the real model in packed level order.  resid[b] receives
 * ||y||^2 - ||z||^2 (the constant the search drops; 0 when N = M), or pass
 * NULL.  Limits: 1 <= n_tx <= n_rx <= 128.  Computed as a Cholesky QR in
 * FP64 (Gram matrix of [H | y], then its Cholesky factor [[R, z], [0, rho]]);
 * a frame whose H is rank-deficient in FP64 gets zero rows in R from the
 * first vanishing pivot on.
 * H [B][n_rx][n_tx] c64, y [B][n_rx] c64 -> R [B][n(n+1)/2], z [B][n] f32.
 * ------------------------------------------------------------------- */
int32_t mimo_qr_preprocess(const float* H, const float* y, int32_t B, int32_t n_rx, int32_t n_tx,
                           float* R, float* z, float* resid, void* stream);

/* ---------------------------------------------------------------------
 * MMSE preprocessing for the linear and successive-cancellation baselines
 * the paper compares against (Sec. III-A): the QR of the augmented system
 * [H; sigma_b I], [y; 0], i.e. R^H R = H^H H + sigma2[b] I and
 * R^H z = H^H y, emitted like mimo_qr_preprocess (same layout, limits and
 * method: sigma2[b] is added to the first n_tx diagonal entries of the
 * Gram matrix before the Cholesky factorisation).  Back-substitution on
 * (R, z) (linear_detect) is the linear MMSE estimate; K-best with K = 1 on
 * it is MMSE-SIC.  sigma2 [B] f32 complex noise variances (device).
 * ------------------------------------------------------------------- */
int32_t mimo_qr_preprocess_mmse(const float* H, const float* y, const float* sigma2, int32_t B, int32_t n_rx,
                                int32_t n_tx, float* R, float* z, void* stream);

/* ---------------------------------------------------------------------
 * Batched K-best (Sec. VI, the K-best algorithm): level by level from the
 * root, all P children of every survivor are evaluated with the
 * incremental partial distance of Eq. (inc), children outside the radius
 * are dropped, and the K_t best by (pd, parent rank, child index) survive;
 * the best leaf is returned.  K_t = k_sched[b * k_sched_stride + k] at level
 * k (clamped to [1, K]) when k_sched is not NULL, else K.  k_sched_stride is
 * 0 (one schedule for all frames) or n (one per frame).
 * R, z as produced by mimo_qr_preprocess; radius2 [B] or NULL.
 * Outputs: sym [B][n_tx], pd [B] (float search metric), flags [B],
 * counters [B][4] or NULL.  1 <= K <= MIMO_MAX_K, K * pam <= 1024, and
 * for more than 64 survivors the survivor lists must fit the 160 KB of LDS
 * of a compute unit (about 8 K (n/2 + 3) bytes: K = 256 of 4- or 16-QAM
 * stops at n_tx = 78), else MIMO_ERR_UNSUPPORTED.  With radius2, a frame
 * whose sphere holds no leaf (Sec. III-B leaves that case open) is detected
 * again with r2 = +infinity in a second launch on the same stream: it then
 * carries MIMO_FLAG_EMPTY_SPHERE | MIMO_FLAG_FOUND and its counters add up
 * both searches.  A frame with a NaN or infinity in R or z stops at that
 * level with MIMO_FLAG_NONFINITE_INPUT (sym 0, pd +infinity).  For K <= 64
 * without a schedule the launch is the grouped kernel of
 * kbest_detect_grouped (J = 1), except at most 8 survivors of 64-QAM at
 * 64 < n <= 208 (two frames per wavefront) and K * pam > 64 at n <= 8; the
 * detection is the same, only the order of the FP32 sums in a centre
 * differs.
 * ------------------------------------------------------------------- */
int32_t kbest_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                     int32_t K, const int32_t* k_sched, int32_t k_sched_stride,
                     const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                     int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Batched K-best over complex levels, the tree of the paper's own figures
 * (Sec. III-B branches on complex symbols: |Omega| = pam^2 children per
 * level, n_tx levels; Sec. VI for K-best).  Complex level m fixes the
 * imaginary part (real level 2m+1) and the real part (real level 2m) of
 * symbol m together: child (i_im, i_re) of a survivor has
 * pd' = pd + (b_2m+1 - R a_im)^2 + (b_2m - R a_re)^2, and the K_t best by
 * (pd, parent rank, i_im pam + i_re) survive.  K_t = k_sched[... + 2m]
 * (the level of the real part), clamped to [1, K].  Arguments, outputs and
 * flags as kbest_detect; counters[b][0] = survivors expanded,
 * counters[b][1] = real-level evaluations (2 per child).  From 512
 * candidates per level (K pam^2) or 128 real levels on, the launch is the
 * grouped kernel of kbest_detect_grouped (J = 2).
 * Limits: 1 <= K <= 64, K * pam^2 <= 2048 (K <= 32 at 64-QAM).
 * ------------------------------------------------------------------- */
int32_t kbest_detect_complex(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                             int32_t K, const int32_t* k_sched, int32_t k_sched_stride,
                             const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                             int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Grouped K-best: the detection of kbest_detect (J = 1) or of
 * kbest_detect_complex (J = 2: J real levels, one complex symbol, per step;
 * Sec. IV-B grouping), with the successors' centres taken from one matrix
 * product per group of 16 real levels (Sec. V-A evaluates all successors as
 * B = Y* - R'V; here C = (c R)[group rows, levels above] X[levels above,
 * survivors] on the matrix cores, c R split exactly into three bf16 parts,
 * FP32 sums) and the levels inside the group added one by one (Eq. (inc)).
 * The tree, the keys (pd, parent rank, child index), K_t = k_sched[level of
 * the step's lowest real level], the radius, the empty-sphere re-run, the
 * flags and the counters (counters[b][1] = J real-level evaluations per
 * child) are those of kbest_detect / kbest_detect_complex; only the order of
 * the FP32 sums in a centre differs.  Arguments and outputs as kbest_detect.
 * Limits: J in {1, 2}, 1 <= K <= 64, K * pam^J <= 2048, n_tx <= 128.
 * ------------------------------------------------------------------- */
int32_t kbest_detect_grouped(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                             int32_t K, int32_t J, const int32_t* k_sched, int32_t k_sched_stride,
                             const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                             int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Plain fallback of a learned detection (the plain K-best stays the
 * reference method): frame b is detected again by plain K-best with K
 * survivors, overwriting sym[b], pd[b], flags[b] (which then carry
 * MIMO_FLAG_LEARNED_FALLBACK) and counters[b], iff its current flags hold
 * MIMO_FLAG_LEARNED_FALLBACK or lack MIMO_FLAG_FOUND, or its search metric
 * pd[b] exceeds (sigma2[b] / 2) (n + beta sqrt(2 n)) -- beta standard
 * deviations above the mean of the noise energy a correct detection leaves
 * (chi-square with n real degrees of freedom, sigma2 the complex noise
 * variance).  Frames that keep their detection are not touched.  sym, pd,
 * flags are the outputs of the first detection (in place); sigma2 [B].
 * ------------------------------------------------------------------- */
int32_t kbest_fallback(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam, int32_t K,
                       const float* sigma2, float beta, int32_t* sym, float* pd, uint32_t* flags,
                       int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * The fallback's decision alone: sets MIMO_FLAG_LEARNED_FALLBACK in
 * flags[b] for every frame that kbest_fallback (same sigma2, beta, n_tx)
 * would detect again, and touches nothing else.  It lets the metric of the
 * frames that keep their first detection run while the fallback runs
 * (mimo_metric_select).  pd, flags, sigma2 [B] as for kbest_fallback.
 * ------------------------------------------------------------------- */
int32_t kbest_fallback_mark(const float* pd, uint32_t* flags, const float* sigma2, int32_t B, int32_t n_tx,
                            float beta, void* stream);

/* ---------------------------------------------------------------------
 * Learned-pruning labels: K-best with K survivors in which the given path
 * (normally the ML path) is forced to survive; rank[b][k] receives the
 * 1-based rank of that path's prefix among the sorted candidates of level k.
 * force_sym [B][n_tx] QAM indices; rank [B][n] int32.
 * ------------------------------------------------------------------- */
int32_t kbest_rank_labels(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                          int32_t K, const int32_t* force_sym, int32_t* rank, void* stream);

/* ---------------------------------------------------------------------
 * Hybrid SD / K-best (Sec. VI, SD-K-best): a Best-FS sphere-decoder master
 * (Alg. 1 with the Best-FS list of Sec. IV-A) feeds the right-most pool
 * nodes to n_workers K-best workers that keep k_worker survivors (or
 * k_sched[k] when k_sched is not NULL) inside the shared radius.  Run in
 * deterministic rounds: (1) the master takes the left-most node inside the
 * radius and expands it (leaf children become candidates, the others go to
 * the left of the pool, best left-most); (2) idle workers, in order, take
 * the right-most node while the pool holds >= 2 nodes; (3) busy workers
 * advance one level; (4) the best candidate by (pd, source, rank) shrinks
 * the radius.  The run ends when the pool is empty and all workers are idle
 * (flag CERTIFIED) or after node_budget expansions (> 0; flag
 * BUDGET_EXHAUSTED, best leaf so far).  n_workers = 0 is the exact Best-FS
 * SD (maximum likelihood within the radius); master_off != 0 hands the root
 * to worker 0 instead (K-best within the radius).  With radius2, a frame
 * whose pool drains without a leaf inside the sphere is run again with
 * r2 = +infinity in a second launch (flags EMPTY_SPHERE | FOUND, counters
 * summed); a NaN or infinity met in R or z ends the frame's search with
 * MIMO_FLAG_NONFINITE_INPUT (sym 0, pd +infinity).  A frame that reaches the
 * budget without any leaf has BUDGET_EXHAUSTED and no FOUND (sym 0).
 * Limits: 0 <= n_workers <= MIMO_MAX_WORKERS, k_worker * pam <= 64.
 * ------------------------------------------------------------------- */
int32_t sd_hybrid_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                         const float* radius2, int32_t n_workers, int32_t k_worker,
                         const int32_t* k_sched, int32_t k_sched_stride, int32_t master_off,
                         int64_t node_budget, int32_t* sym, float* pd, uint32_t* flags,
                         int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Hybrid SD / K-best on the complex-symbol tree (Sec. VI with the tree of
 * Sec. III-B: one complex symbol, |Omega| = pam^2 children, per node).  The
 * rounds, arguments, outputs and error behaviour are those of
 * sd_hybrid_detect, with one step fixing the real and imaginary levels
 * 2m + 1, 2m of complex symbol m together: the master expands a node into
 * pam^2 children (pd plus the two squared distances, upper level first),
 * pool depths and worker steps are complex levels, a worker keeps
 * k_sched[2m] (the step's lower real level) or k_worker survivors of its
 * k_worker * pam^2 candidates, ordered by (pd, parent rank, child index
 * c = ih * pam + il: ih the PAM index at level 2m + 1, the
 * imaginary part, il the real part's).  counters[1] counts
 * real-level evaluations: 2 pam^2 per expansion.
 * Limits: 0 <= n_workers <= MIMO_MAX_WORKERS, 1 <= k_worker <= 64,
 * k_worker * pam^2 <= MIMO_HYB_MAX_CAND_CPLX (512: 8 survivors at 64-QAM).
 * ------------------------------------------------------------------- */
int32_t sd_hybrid_detect_complex(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                 const float* radius2, int32_t n_workers, int32_t k_worker,
                                 const int32_t* k_sched, int32_t k_sched_stride, int32_t master_off,
                                 int64_t node_budget, int32_t* sym, float* pd, uint32_t* flags,
                                 int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Exact sphere decoding with the frame's tree spread over the wavefronts
 * of one workgroup (Alg. 1 with the Schnorr-Euchner child order of
 * Sec. IV-A; sub-problems go to whichever wavefront is free, under one
 * shared radius, the GPU counterpart of the dynamically balanced parallel
 * SD of Sec. V-C).  The prefixes of the top real levels (at most 512) that
 * lie inside the radius are the sub-problems, taken in order of prefix pd;
 * each is searched depth first, nearest child first, every leaf inside the
 * radius shrinking it for all wavefronts of the frame.  The result is the
 * maximum-likelihood point within the radius.
 * radius2 [B] or NULL (no radius; with redo = 1 and radius2 NULL, each
 * frame's current pd[b] x (1 + 1e-4), i.e. the earlier search's best leaf
 * stays inside).  budget: node expansions per frame (0 = none); when it is
 * spent the frame keeps its best leaf so far with BUDGET_EXHAUSTED and no
 * CERTIFIED.  redo = 1: only frames whose flags hold BUDGET_EXHAUSTED and
 * lack CERTIFIED (left unfinished by an earlier search such as
 * sd_hybrid_detect with a budget) are searched, in place: sym, pd, flags
 * overwritten, counters added to; other frames are untouched.
 * Outputs: sym [B][n_tx], pd [B] (search metric), flags (FOUND; CERTIFIED
 * when every sub-problem was searched), counters [B][4] or NULL: [0] node
 * expansions, [1] child evaluations.  The counters depend on the order in
 * which the wavefronts take the sub-problems and vary between runs; the
 * result does not, apart from leaves whose FP32 pd ties.  A frame whose
 * finite radius holds no leaf is searched again with r2 = +infinity
 * (EMPTY_SPHERE | FOUND); a NaN or infinity in R or z stops it with
 * NONFINITE_INPUT (sym 0, pd +infinity).  Limits: n_tx <= 128 (16
 * wavefronts per frame up to 232 real levels, 8 beyond), budget >= 0.
 * ------------------------------------------------------------------- */
int32_t sd_parallel_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                           const float* radius2, int64_t budget, int32_t redo, int32_t* sym, float* pd,
                           uint32_t* flags, int64_t* counters, void* stream);

/* ---------------------------------------------------------------------
 * Linear detection (the zero-forcing / MMSE baselines of Sec. III-A):
 * u = R^{-1} z by back-substitution in FP32 without decision feedback, then
 * every real level sliced to the nearest PAM amplitude on its own.  With R, z
 * from mimo_qr_preprocess this is zero forcing (u = H^+ y), from
 * mimo_qr_preprocess_mmse linear MMSE.  sym [B][n_tx] QAM indices; xhat
 * [B][n] f32 (interleaved real and imaginary estimates) or NULL.
 * ------------------------------------------------------------------- */
int32_t linear_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam, int32_t* sym,
                      float* xhat, void* stream);

/* ---------------------------------------------------------------------
 * The paper's sphere radius rule (Sec. III-B, "Sphere radius and pruning"),
 * squared: radius2[b] = n_rx * n_tx * sigma2[b], M times the expected noise
 * energy N sigma2 of a received vector, computed in FP32 (one rounding).
 * sigma2 [B] complex noise variances, radius2 [B] f32, both device; the
 * result is a radius2 argument for kbest_detect and sd_hybrid_detect.
 * Limits: 1 <= n_tx <= n_rx <= 128.
 * ------------------------------------------------------------------- */
int32_t mimo_paper_radius2(const float* sigma2, int32_t B, int32_t n_rx, int32_t n_tx, float* radius2,
                           void* stream);

/* ---------------------------------------------------------------------
 * Maximum-ratio combining (Sec. III-A): u_j = h_j^H y / ||h_j||^2 per
 * transmit stream, accumulated in FP64 from the complex64 H, y, the real and
 * imaginary parts sliced on their own.  sym [B][n_tx]; xhat [B][2 n_tx] f32
 * or NULL.  Limits as mimo_metric.
 * ------------------------------------------------------------------- */
int32_t mrc_detect(const float* H, const float* y, int32_t B, int32_t n_rx, int32_t n_tx, int32_t pam,
                   int32_t* sym, float* xhat, void* stream);

/* ---------------------------------------------------------------------
 * Metric epilogue: metric[b] = ||y_b - H_b s_b||^2 in FP64 from the
 * complex64 H, y and QAM indices sym [B][n_tx] (Eq. (2) objective).
 * ------------------------------------------------------------------- */
int32_t mimo_metric(const float* H, const float* y, const int32_t* sym, int32_t B, int32_t n_rx,
                    int32_t n_tx, int32_t pam, double* metric, void* stream);

/* ---------------------------------------------------------------------
 * Metric epilogue for a subset of frames: as mimo_metric, for the frames
 * with (flags[b] & mask) == value only; metric[b] of the others is not
 * written.  flags [B] (device).
 * ------------------------------------------------------------------- */
int32_t mimo_metric_select(const float* H, const float* y, const int32_t* sym, const uint32_t* flags,
                           uint32_t mask, uint32_t value, int32_t B, int32_t n_rx, int32_t n_tx, int32_t pam,
                           double* metric, void* stream);

/* ---------------------------------------------------------------------
 * Error counts: counts[0] += Gray-coded bit errors, counts[1] += symbol
 * errors between sym and ref ([B][n_tx] QAM indices), counts[2] += frames
 * with any error.  Bits of a symbol: Gray(i_re) || Gray(i_im), with
 * Gray(i) = i ^ (i >> 1).  counts [3] uint64 (caller zeroes it).
 * ------------------------------------------------------------------- */
int32_t mimo_error_count(const int32_t* sym, const int32_t* ref, int32_t B, int32_t n_tx,
                         int32_t pam, uint64_t* counts, void* stream);

/* ---------------------------------------------------------------------
 * Learned pruning, per-level state of each frame (the paper leaves the
 * "very close" extra-survivor rule of Sec. VI unspecified; this library
 * replaces it with a learned survivor count).  From the successive-
 * cancellation path (K-best with K = 1), for every level k:
 *   f0 = k / n,
 *   f1 = distance of the cancellation centre b_k / R_kk to the nearest
 *        decision boundary, in units of the point spacing 2c,
 *   f2 = log2(R_kk * 2c / sigma_r), sigma_r = sqrt(sigma2[b] / 2),
 *   f3 = pd of the path after level k / ((n - k) sigma_r^2).
 * sigma2 [B] is the complex noise variance.  feat [B][n][4] f32.
 * ------------------------------------------------------------------- */
int32_t prune_features(const float* R, const float* z, const float* sigma2, int32_t B,
                       int32_t n_tx, int32_t pam, float* feat, void* stream);

/* MLP 4 -> 128 -> 128 -> 1 (ReLU) forward over S states: out[s] = f(X[s]).
 * w [MIMO_MLP_NPARAM] f32, X [S][4], out [S]. */
int32_t prune_mlp_forward(const float* w, const float* X, int64_t S, float* out, void* stream);

/* Forward plus survivor schedule: k_sched[s] = clamp(ceil(2^(f(X[s]) + margin)),
 * k_min, k_max); a non-finite prediction gives k_max and sets
 * MIMO_FLAG_LEARNED_FALLBACK in flags[s / n] when flags is not NULL
 * (n = levels per frame, used only for that index). */
int32_t prune_mlp_schedule(const float* w, const float* X, int64_t S, float margin,
                           int32_t k_min, int32_t k_max, int32_t n, int32_t* k_sched,
                           uint32_t* flags, void* stream);

/* Mean pinball loss at quantile tau over S states and its gradient.
 * grad [MIMO_MLP_NPARAM] and loss [1] are overwritten.  ws is a device
 * workspace of at least prune_mlp_workspace_bytes(S) bytes. */
size_t prune_mlp_workspace_bytes(int64_t S);
int32_t prune_mlp_loss_grad(const float* w, const float* X, const float* y, int64_t S, float tau,
                            float* grad, float* loss, void* ws, size_t ws_bytes, void* stream);

/* Allocation-free variant of prune_mlp_loss_grad, for callers that cannot
 * allocate device memory (code under hipGraph capture, serving or training
 * loops, harnesses that forbid allocation).  Same arguments and results
 * (bit for bit) without the workspace: the per-state activations, deltas,
 * loss partials and partial gradient tiles live in a static device array
 * sized for MIMO_MLP_NOALLOC_MAX_S states (about 19.7 MB), which each GPU the library
 * runs on holds until the process ends.  S > MIMO_MLP_NOALLOC_MAX_S returns
 * MIMO_ERR_UNSUPPORTED.  Every call on a GPU uses that GPU's one array, so
 * calls that overlap on one GPU (other streams, other host threads) race;
 * each call overwrites everything it reads, nothing needs clearing. */
#define MIMO_MLP_NOALLOC_MAX_S 8192
int32_t prune_mlp_loss_grad_noalloc(const float* w, const float* X, const float* y, int64_t S, float tau,
                                    float* grad, float* loss, void* stream);

/* One Adam step on w with moments m, v (all [np] f32), step t >= 1. */
int32_t prune_mlp_adam_step(float* w, float* m, float* v, const float* grad, int32_t np, int32_t t,
                            float lr, float beta1, float beta2, float eps, void* stream);

/* ---------------------------------------------------------------------
 * Uneven batches: frames of different antenna counts and constellations in
 * one batch.  Frame f is described by desc[f] (device memory):
 * ------------------------------------------------------------------- */
typedef struct {
    int32_t n_rx, n_tx, pam, K; /* shape, PAM points, survivors (K-best) */
    int64_t h_off;              /* complex offset of H (n_rx x n_tx complex64) in H_flat */
    int64_t y_off;              /* complex offset of y (n_rx complex64) in y_flat */
    int64_t r_off;              /* float offset of the packed R (n(n+1)/2) in R_flat */
    int64_t z_off;              /* float offset of z (n floats) in z_flat */
    int64_t s_off;              /* int offset of the symbols (n_tx) in sym_flat */
} mimo_frame_desc;

/* QR preprocessing (Sec. III-B) of an uneven batch in one persistent launch:
 * `grid` workgroups (0 = two per compute unit) pull frames from the device
 * work counter `counter` (one int32, reset by the call on the stream).
 * Every frame needs 1 <= n_tx <= n_rx <= max_rx <= 128; a frame that does
 * not is skipped (its outputs are left untouched).  Output layout as for
 * mimo_qr_preprocess, at the frames' offsets. */
int32_t mimo_qr_preprocess_uneven(const mimo_frame_desc* desc, int32_t B, int32_t max_rx,
                                  const float* H_flat, const float* y_flat, float* R_flat, float* z_flat,
                                  int32_t* counter, int32_t grid, void* stream);

/* Batched K-best (Sec. VI) of an uneven batch in one persistent launch: one
 * wavefront per workgroup pulls frames from `counter` (reset by the call)
 * and runs K-best with the frame's own pam and K -- per frame the detection
 * kbest_detect_grouped (J = 1) returns.  Per-frame limits: pam in
 * {2, 4, 8}, 1 <= K <= 64, K * pam <= 256, 1 <= n_tx <= 64; a frame outside
 * them is skipped with flags[f] = MIMO_FLAG_INVALID_FRAME (its sym and pd
 * untouched).  sym_flat at the frames' s_off; pd [B], flags [B] indexed by
 * descriptor position.  grid = 0 picks eight workgroups per compute unit. */
int32_t kbest_detect_uneven(const mimo_frame_desc* desc, int32_t B, const float* R_flat, const float* z_flat,
                            int32_t* sym_flat, float* pd, uint32_t* flags, int32_t* counter, int32_t grid,
                            void* stream);

#ifdef __cplusplus
}
#endif
#endif
