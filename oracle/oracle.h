/* FP64 CPU oracle for the sphere-decoder / K-best / hybrid SD-K-best hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this code; only the test-suite, the smoke check and the benchmark's
 * CPU-baseline leg use it.  It shares no code, header or table with the HIP
 * path.
 *
 * Paper: Dabah et al., "Performance / Complexity Trade-offs of the Sphere
 * Decoder Algorithm for Massive MIMO Systems" (arXiv 2002.09561).
 *
 * Conventions (readings of the paper, all in plain FP64):
 *   real-valued model:  x = [Re s0, Im s0, Re s1, ...], each complex h becomes
 *     [[Re h, -Im h], [Im h, Re h]], rows [Re y0, Im y0, ...]; n = 2M levels;
 *   QR: H_r = Q R with R_kk > 0, z = Q^T y_r, resid = ||y_r||^2 - ||z||^2;
 *   level k (0..n-1) fixes x_k; the search starts at level n-1 (Sec. III-B);
 *   PAM amplitudes (2i - (P-1)) c, c = sqrt(3 / (2 (P^2 - 1)));
 *   partial distance of a node = sum over its fixed levels of
 *     (z_k - sum_{j>=k} R_kj x_j)^2  (Eq. (4));
 *   radius tests use the squared radius, keep iff pd < r2 (Alg. 1).
 * All matrices are row-major; R is the full n x n upper-triangular matrix.
 * Symbol outputs are PAM indices per real level (x_idx[k] in 0..P-1).
 *
 * "parity unpinned": none of the functions below; see the test-suite for the
 * pin of each one.
 */
#ifndef MIMO_SD_ORACLE_H
#define MIMO_SD_ORACLE_H
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* flags (oracle-side names; bit meanings mirror the problem statement) */
#define ORC_FOUND            1u   /* a leaf inside the radius was found        */
#define ORC_EMPTY_SPHERE     2u   /* finite radius left no leaf; searched again  */
                                  /* with r2 = +inf (reading of Sec. III-B)      */
#define ORC_BUDGET_EXHAUSTED 4u   /* node budget reached before the list emptied */
#define ORC_CERTIFIED        8u   /* list emptied: exact ML within the radius   */

#define ORC_LEARNED_FALLBACK 16u  /* detected again by plain K-best            */

/* counters: [0] nodes expanded (branched on), [1] PD evaluations (children),
 *           [2] rounds (hybrid only), [3] nodes discarded as stale */
#define ORC_NCOUNTERS 4

double orc_pam_scale(int P);

/* Sec. III-B: real model of one frame.  H [N][M] and y [N] are complex64
 * (interleaved float pairs).  Hr [2N][2M], yr [2N]. */
void orc_real_model(int N, int M, const float* H, const float* y, double* Hr, double* yr);

/* Sec. III-B: Householder QR of the real model; R [n][n], z [n], resid. */
int orc_qr(int N, int M, const float* H, const float* y, double* R, double* z, double* resid);

/* Eq. (2): exhaustive ML over all |Omega|^M symbol vectors, from H and y
 * directly (complex arithmetic).  s_idx [M] QAM indices, metric out. */
int orc_brute_force(int N, int M, int P, const float* H, const float* y, int* s_idx, double* metric);

/* ||y - H s||^2 in FP64 for QAM indices s_idx [M]. */
double orc_metric(int N, int M, int P, const float* H, const float* y, const int* s_idx);

/* Successive interference cancellation with a rounding slicer (the K = 1
 * special case of K-best): x_idx [n], returns the path's pd. */
double orc_zf_sic(int n, int P, const double* R, const double* z, int* x_idx);
int orc_qr_mmse(int N, int M, const float* H, const float* y, double sigma2, double* R, double* z);
void orc_linear(int n, int P, const double* R, const double* z, int* x_idx, double* u);
void orc_mrc(int N, int M, int P, const float* H, const float* y, int* s_idx, double* u);

/* Per-level partial distances of a complete path: g[k] = (z_k - sum_{j>=k} R_kj x_j)^2 */
void orc_path_terms(int n, int P, const double* R, const double* z, const int* x_idx, double* g);

/* Alg. 1 with the Best-FS list policy (Sec. IV-A).  r2 = +inf for none.
 * x_init (or NULL) is the warm-start solution that goes with r2.
 * budget = 0 for unbounded.  Returns flags. */
uint32_t orc_sesd(int n, int P, const double* R, const double* z, double r2, int64_t budget,
                  const int* x_init, int* x_out, double* pd_out, int64_t* counters);

/* K-best (Sec. VI): level-synchronous, keeps the first K_t candidates by
 * (pd, parent rank, child index).  J = symbols fixed per step (1, or 2 for
 * complex-symbol branching), K_t = k_sched[k_lo] clamped to [1, K] if k_sched else K.
 * force_path (or NULL): a complete path whose prefix is kept at every step
 * (label generation); its 1-based rank among the sorted candidates of each
 * step goes to rank_out[k_lo] (if rank_out), and fgap_out (if not NULL)
 * receives the largest relative gap between the forced prefix and the key
 * that beat it, over the decisions that would have dropped it (the K_t-th
 * survivor) or preferred another leaf (the best leaf): 0 when the forced
 * path is the search's own result, +inf when it leaves the sphere.
 * rgap_out[k_lo] (if not NULL) receives how close that step's rank is to
 * changing: the smallest relative gap between the forced candidate and any
 * other, or between the last survivor and the first dropped candidate.
 * margin_out (or NULL) receives [0] the smallest relative gap of any
 * decision taken, [1],[2] the pair. */
uint32_t orc_kbest(int n, int P, const double* R, const double* z, int K, const int* k_sched,
                   double r2, int J, const int* force_path, int* x_out, double* pd_out,
                   double* margin_out, int* rank_out, double* fgap_out, double* rgap_out,
                   int64_t* counters);

/* Hybrid SD-K-best (Sec. VI) in deterministic rounds; W workers each keep
 * Kw survivors (or k_sched[k] clamped to [1, Kw] when k_sched is not NULL,
 * k the lowest level a step fixes).  Each step fixes J real levels (1 or 2:
 * P^J children, the digit of the top level most significant; Sec. IV-B
 * grouping).  master_off hands the root to worker 0 and never expands (the
 * K-best special case). */
uint32_t orc_hybrid(int n, int P, int J, const double* R, const double* z, double r2, int W, int Kw,
                    const int* k_sched, int master_off, int64_t budget, int* x_out, double* pd_out,
                    double* margin_out, int64_t* counters);
/* The same search for one frame with a text trace of its rounds in buf. */
uint32_t orc_hybrid_trace(int n, int P, int J, const double* R, const double* z, double r2, int W, int Kw,
                          int master_off, int64_t budget, int* x_out, double* pd_out, int64_t* counters,
                          char* buf, int cap);

/* Learned-pruning state of a frame: per level k, 4 features from the SIC
 * (K = 1) path: [k/n, distance of the SIC centre to the nearest decision
 * boundary in spacing units, log2(R_kk * 2c / sigma_r), SIC pd up to level
 * k over its expectation (n-k) sigma_r^2].  feat [n][4], row k. */
void orc_prune_features(int n, int P, const double* R, const double* z, double sigma2, double* feat);

/* MLP 4 -> 128 -> 128 -> 1 with ReLU; flat weights (see ORC_MLP_* offsets). */
#define ORC_MLP_IN 4
#define ORC_MLP_H 128
#define ORC_MLP_W1 0
#define ORC_MLP_B1 (ORC_MLP_W1 + ORC_MLP_H * ORC_MLP_IN)
#define ORC_MLP_W2 (ORC_MLP_B1 + ORC_MLP_H)
#define ORC_MLP_B2 (ORC_MLP_W2 + ORC_MLP_H * ORC_MLP_H)
#define ORC_MLP_W3 (ORC_MLP_B2 + ORC_MLP_H)
#define ORC_MLP_B3 (ORC_MLP_W3 + ORC_MLP_H)
#define ORC_MLP_NPARAM (ORC_MLP_B3 + 1)

void orc_mlp_forward(const double* w, const double* X, int B, double* out);
/* mean pinball loss at quantile tau; grad (NPARAM) of the mean loss. */
double orc_mlp_loss_grad(const double* w, const double* X, const double* y, int B, double tau,
                         double* grad);
/* One Adam step (t = 1-based step count). */
void orc_adam_step(double* w, double* m, double* v, const double* g, int np, int t, double lr,
                   double beta1, double beta2, double eps);

/* The learned-pruning detector of one frame (the paper's unspecified "very
 * close" survivor rule of Sec. VI replaced by a learned per-level count):
 * features of the SIC path -> MLP -> K_t = clamp(ceil(2^(f + margin)), kmin,
 * kmax) -> K-best with that schedule; the frame is detected again by plain
 * K-best with K_fallback survivors (flag ORC_LEARNED_FALLBACK) when no leaf
 * was found or its pd exceeds (sigma2 / 2)(n + beta sqrt(2 n)).
 * k_sched_out [n] (or NULL) receives the schedule. */
uint32_t orc_learned_detect(int n, int P, const double* R, const double* z, double sigma2, const double* w,
                            double margin, int kmin, int kmax, double beta, int K_fallback, int* x_out,
                            double* pd_out, int* k_sched_out, int64_t* counters);

/* ---- batched drivers (OpenMP over frames) ---- */
void orc_batch_learned_detect(int B, int n, int P, const double* R, const double* z, const double* sigma2,
                              const double* w, double margin, int kmin, int kmax, double beta, int K_fallback,
                              int* x_out, double* pd_out, int* k_sched_out, uint32_t* flags);
void orc_batch_qr(int B, int N, int M, const float* H, const float* y, double* R, double* z,
                  double* resid);
void orc_batch_brute_force(int B, int N, int M, int P, const float* H, const float* y, int* s_idx,
                           double* metric);
void orc_batch_metric(int B, int N, int M, int P, const float* H, const float* y,
                      const int* s_idx, double* metric);
void orc_batch_qr_mmse(int B, int N, int M, const float* H, const float* y, const double* sigma2, double* R,
                       double* z);
void orc_batch_linear(int B, int n, int P, const double* R, const double* z, int* x_idx, double* u);
void orc_batch_mrc(int B, int N, int M, int P, const float* H, const float* y, int* s_idx, double* u);
void orc_batch_zf_sic(int B, int n, int P, const double* R, const double* z, int* x_idx, double* pd);
void orc_batch_sesd(int B, int n, int P, const double* R, const double* z, const double* r2,
                    int64_t budget, const int* x_init, int* x_out, double* pd_out,
                    uint32_t* flags, int64_t* counters);
void orc_batch_kbest(int B, int n, int P, const double* R, const double* z, int K,
                     const int* k_sched, int k_sched_stride, double r2, int J,
                     const int* force_path, int* x_out, double* pd_out, double* margin_out,
                     int* rank_out, double* fgap_out, double* rgap_out, uint32_t* flags,
                     int64_t* counters);
void orc_batch_hybrid(int B, int n, int P, int J, const double* R, const double* z, const double* r2, int W,
                      int Kw, const int* k_sched, int k_sched_stride, int master_off,
                      int64_t budget, int* x_out, double* pd_out, double* margin_out,
                      uint32_t* flags, int64_t* counters);
void orc_batch_prune_features(int B, int n, int P, const double* R, const double* z,
                              const double* sigma2, double* feat);

#ifdef __cplusplus
}
#endif
#endif
