/* FP64 CPU oracle for the sphere-decoder hot path.
 *
 * TEST INFRASTRUCTURE ONLY: used by the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg; never by the product library.  Plain, slow,
 * obviously-correct code that follows the paper's definitions step by step;
 * no blocking, no fusion.  Conventions are listed in oracle.h.
 */
#include "oracle.h"

#include <float.h>
#include <math.h>
#include <stdarg.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* optional text trace of a search (one event per line) */
typedef struct {
    char* buf;
    size_t cap, len;
} trace_t;

static void tr(trace_t* t, const char* fmt, ...)
{
    if (!t || !t->buf || t->len + 1 >= t->cap) return;
    va_list ap;
    va_start(ap, fmt);
    int w = vsnprintf(t->buf + t->len, t->cap - t->len, fmt, ap);
    va_end(ap);
    if (w > 0) t->len += (size_t)w;
    if (t->len >= t->cap) t->len = t->cap - 1;
}

/* ------------------------------------------------------------------ */
/* constellation (reading: unit-energy square QAM, Gray-free PAM index)  */
/* ------------------------------------------------------------------ */
double orc_pam_scale(int P) { return sqrt(3.0 / (2.0 * (double)(P * P - 1))); }

static double amp(int P, int i) { return (double)(2 * i - (P - 1)) * orc_pam_scale(P); }

static double rel_gap(double a, double b)
{
    double m = fmax(fabs(a), fabs(b));
    if (m == 0.0) return 0.0;
    return fabs(a - b) / m;
}

static void note_gap(double* margin, double a, double b)
{
    if (!margin) return;
    double g = rel_gap(a, b);
    if (g < margin[0]) {
        margin[0] = g;
        margin[1] = a;
        margin[2] = b;
    }
}

/* ------------------------------------------------------------------ */
/* Sec. III-B: real-valued model and QR preprocessing                  */
/* ------------------------------------------------------------------ */
void orc_real_model(int N, int M, const float* H, const float* y, double* Hr, double* yr)
{
    const int cols = 2 * M;
    for (int i = 0; i < N; ++i) {
        for (int j = 0; j < M; ++j) {
            double re = H[2 * (i * M + j)], im = H[2 * (i * M + j) + 1];
            Hr[(2 * i) * cols + 2 * j] = re;
            Hr[(2 * i) * cols + 2 * j + 1] = -im;
            Hr[(2 * i + 1) * cols + 2 * j] = im;
            Hr[(2 * i + 1) * cols + 2 * j + 1] = re;
        }
        yr[2 * i] = y[2 * i];
        yr[2 * i + 1] = y[2 * i + 1];
    }
}

/* Householder triangularisation of a real system [A | b] (rows x n, rows >= n):
 * the reflections that make A upper triangular are applied to b as well,
 * giving z = Q^T b; the part of the rotated b below row n is the residual
 * ||Q_2^T b||^2.  A and b are overwritten. */
static void householder(int rows, int n, double* A, double* b, double* R, double* z, double* resid)
{
    double* v = (double*)malloc(sizeof(double) * rows);
    for (int k = 0; k < n; ++k) {
        double norm2 = 0.0;
        for (int i = k; i < rows; ++i) norm2 += A[i * n + k] * A[i * n + k];
        double norm = sqrt(norm2);
        if (norm == 0.0) continue;
        double alpha = (A[k * n + k] >= 0.0) ? -norm : norm;
        for (int i = k; i < rows; ++i) v[i] = A[i * n + k];
        v[k] -= alpha;
        double vv = 0.0;
        for (int i = k; i < rows; ++i) vv += v[i] * v[i];
        if (vv == 0.0) continue;
        for (int j = k; j < n; ++j) {
            double s = 0.0;
            for (int i = k; i < rows; ++i) s += v[i] * A[i * n + j];
            double f = 2.0 * s / vv;
            for (int i = k; i < rows; ++i) A[i * n + j] -= f * v[i];
        }
        double s = 0.0;
        for (int i = k; i < rows; ++i) s += v[i] * b[i];
        double f = 2.0 * s / vv;
        for (int i = k; i < rows; ++i) b[i] -= f * v[i];
    }
    for (int k = 0; k < n; ++k) {
        double sg = (A[k * n + k] < 0.0) ? -1.0 : 1.0; /* force R_kk > 0 */
        for (int j = 0; j < n; ++j) R[k * n + j] = (j >= k) ? sg * A[k * n + j] : 0.0;
        z[k] = sg * b[k];
    }
    double r = 0.0;
    for (int i = n; i < rows; ++i) r += b[i] * b[i];
    if (resid) *resid = r;
    free(v);
}

/* Sec. III-B: QR of the real model of H, z = Q^T y_r. */
int orc_qr(int N, int M, const float* H, const float* y, double* R, double* z, double* resid)
{
    const int rows = 2 * N, n = 2 * M;
    if (M > N) return -1;
    double* A = (double*)malloc(sizeof(double) * (size_t)rows * n);
    double* b = (double*)malloc(sizeof(double) * rows);
    orc_real_model(N, M, H, y, A, b);
    householder(rows, n, A, b, R, z, resid);
    free(A);
    free(b);
    return 0;
}

/* MMSE preprocessing (the linear baselines the paper compares against,
 * Sec. III-A): the QR of the augmented system [H; sigma I_M], [y; 0], whose
 * factor satisfies R^T R = H_r^T H_r + sigma^2 I and R^T z = H_r^T y_r, so
 * back-substitution on (R, z) is the linear MMSE estimate and K = 1 on it is
 * MMSE-SIC.  sigma2 is the complex noise variance (unit-energy symbols). */
int orc_qr_mmse(int N, int M, const float* H, const float* y, double sigma2, double* R, double* z)
{
    const int n = 2 * M, rows = 2 * N + n;
    if (M > N) return -1;
    double* A = (double*)calloc((size_t)rows * n, sizeof(double));
    double* b = (double*)calloc((size_t)rows, sizeof(double));
    orc_real_model(N, M, H, y, A, b);
    const double s = sqrt(sigma2);
    for (int k = 0; k < n; ++k) A[(2 * N + k) * n + k] = s;
    householder(rows, n, A, b, R, z, NULL);
    free(A);
    free(b);
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. (2): exhaustive ML and the metric ||y - H s||^2                  */
/* ------------------------------------------------------------------ */
double orc_metric(int N, int M, int P, const float* H, const float* y, const int* s_idx)
{
    double acc = 0.0;
    for (int i = 0; i < N; ++i) {
        double er = y[2 * i], ei = y[2 * i + 1];
        for (int j = 0; j < M; ++j) {
            double sr = amp(P, s_idx[j] / P), si = amp(P, s_idx[j] % P);
            double hr = H[2 * (i * M + j)], hi = H[2 * (i * M + j) + 1];
            er -= hr * sr - hi * si;
            ei -= hr * si + hi * sr;
        }
        acc += er * er + ei * ei;
    }
    return acc;
}

int orc_brute_force(int N, int M, int P, const float* H, const float* y, int* s_idx, double* metric)
{
    const int Q = P * P;
    double total = pow((double)Q, (double)M);
    if (total > 65536.0 * 16.0) return -1;
    long count = (long)total;
    int* s = (int*)calloc((size_t)M, sizeof(int));
    double best = INFINITY;
    for (long idx = 0; idx < count; ++idx) {
        long r = idx;
        for (int m = 0; m < M; ++m) {
            s[m] = (int)(r % Q);
            r /= Q;
        }
        double d = orc_metric(N, M, P, H, y, s);
        if (d < best) {
            best = d;
            memcpy(s_idx, s, sizeof(int) * (size_t)M);
        }
    }
    free(s);
    if (metric) *metric = best;
    return 0;
}

/* ------------------------------------------------------------------ */
/* Eq. (4): partial-distance terms of a complete path                  */
/* ------------------------------------------------------------------ */
void orc_path_terms(int n, int P, const double* R, const double* z, const int* x_idx, double* g)
{
    for (int k = 0; k < n; ++k) {
        double e = z[k];
        for (int j = k; j < n; ++j) e -= R[k * n + j] * amp(P, x_idx[j]);
        g[k] = e * e;
    }
}

/* centre b_k = z_k - sum_{j>k} R_kj x_j of level k for a path fixed above k */
static double centre(int n, int P, const double* R, const double* z, int k, const int* x_idx)
{
    double b = z[k];
    for (int j = k + 1; j < n; ++j) b -= R[k * n + j] * amp(P, x_idx[j]);
    return b;
}

/* textbook PAM slicer: nearest amplitude by rounding, clamped to the alphabet */
static int slice(int P, double u)
{
    double c = orc_pam_scale(P);
    int i = (int)floor((u / c + (double)(P - 1)) / 2.0 + 0.5);
    if (i < 0) i = 0;
    if (i > P - 1) i = P - 1;
    return i;
}

double orc_zf_sic(int n, int P, const double* R, const double* z, int* x_idx)
{
    double pd = 0.0;
    for (int k = n - 1; k >= 0; --k) {
        double b = centre(n, P, R, z, k, x_idx);
        x_idx[k] = slice(P, b / R[k * n + k]);
        double e = b - R[k * n + k] * amp(P, x_idx[k]);
        pd += e * e;
    }
    return pd;
}

/* Linear detection by back-substitution without decision feedback:
 * u = R^{-1} z in FP64, then each level sliced on its own.  With the plain
 * QR this is zero forcing (u = H^+ y), with the MMSE QR linear MMSE. */
void orc_linear(int n, int P, const double* R, const double* z, int* x_idx, double* u)
{
    for (int k = n - 1; k >= 0; --k) {
        double b = z[k];
        for (int j = k + 1; j < n; ++j) b -= R[k * n + j] * u[j];
        u[k] = b / R[k * n + k];
    }
    for (int k = 0; k < n; ++k) x_idx[k] = slice(P, u[k]);
}

/* Maximum-ratio combining: u_j = h_j^H y / ||h_j||^2 per transmit stream,
 * real and imaginary parts sliced on their own (QAM index i_re P + i_im). */
void orc_mrc(int N, int M, int P, const float* H, const float* y, int* s_idx, double* u)
{
    for (int j = 0; j < M; ++j) {
        double nr = 0.0, cr = 0.0, ci = 0.0;
        for (int i = 0; i < N; ++i) {
            double hr = H[2 * (i * M + j)], hi = H[2 * (i * M + j) + 1];
            double yr = y[2 * i], yi = y[2 * i + 1];
            nr += hr * hr + hi * hi;
            cr += hr * yr + hi * yi; /* conj(h) y */
            ci += hr * yi - hi * yr;
        }
        u[2 * j] = nr > 0.0 ? cr / nr : 0.0;
        u[2 * j + 1] = nr > 0.0 ? ci / nr : 0.0;
        s_idx[j] = slice(P, u[2 * j]) * P + slice(P, u[2 * j + 1]);
    }
}

/* ------------------------------------------------------------------ */
/* Alg. 1 with the Best-FS list policy (Sec. III-B, IV-A)              */
/* ------------------------------------------------------------------ */
typedef struct {
    double pd;
    int c;
} child_t;

static int cmp_child(const void* a, const void* b)
{
    const child_t* x = (const child_t*)a;
    const child_t* y = (const child_t*)b;
    if (x->pd < y->pd) return -1;
    if (x->pd > y->pd) return 1;
    return (x->c > y->c) - (x->c < y->c);
}

static uint32_t sesd_search(int n, int P, const double* R, const double* z, double r2, int64_t budget,
                            const int* x_init, int* x_out, double* pd_out, int64_t* counters)
{
    /* The list is a stack (leftmost = most recently inserted).  Its size is
     * bounded by 1 + n (P - 1): every expansion removes one node and adds at
     * most P. */
    const int cap = n * P + 2;
    int* lt = (int*)malloc(sizeof(int) * cap);
    double* lpd = (double*)malloc(sizeof(double) * cap);
    int* lpath = (int*)malloc(sizeof(int) * (size_t)cap * n);
    int* cur = (int*)malloc(sizeof(int) * n);
    child_t* ch = (child_t*)malloc(sizeof(child_t) * P);
    int64_t expanded = 0, evaluated = 0, stale = 0;
    uint32_t flags = 0;
    double best = INFINITY;

    if (x_init) {
        memcpy(x_out, x_init, sizeof(int) * n);
        flags |= ORC_FOUND;
    }
    int top = 0;
    lt[0] = 0;
    lpd[0] = 0.0;
    for (int j = 0; j < n; ++j) lpath[j] = 0;
    top = 1;

    while (top > 0) {
        /* select_node: the leftmost node (LIFO) */
        --top;
        int t = lt[top];
        double pd = lpd[top];
        memcpy(cur, lpath + (size_t)top * n, sizeof(int) * n);
        if (pd >= r2) { /* its subtree cannot hold a leaf inside the sphere */
            ++stale;
            continue;
        }
        if (budget > 0 && expanded >= budget) {
            flags |= ORC_BUDGET_EXHAUSTED;
            break;
        }
        ++expanded;
        int k = n - 1 - t;
        double b = centre(n, P, R, z, k, cur);
        for (int c = 0; c < P; ++c) {
            double e = b - R[k * n + k] * amp(P, c);
            ch[c].pd = pd + e * e;
            ch[c].c = c;
            ++evaluated;
        }
        /* Best-FS: successors sorted by their evaluation before insertion */
        qsort(ch, (size_t)P, sizeof(child_t), cmp_child);
        int keep[8], nk = 0;
        for (int i = 0; i < P; ++i) {
            if (ch[i].pd < r2) {
                if (t + 1 == n) { /* leaf: shrink the radius, record the solution */
                    r2 = ch[i].pd;
                    best = ch[i].pd;
                    memcpy(x_out, cur, sizeof(int) * n);
                    x_out[k] = ch[i].c;
                    flags |= ORC_FOUND;
                } else {
                    keep[nk++] = i;
                }
            }
        }
        /* insert so that the best successor becomes the leftmost node */
        for (int q = nk - 1; q >= 0; --q) {
            int i = keep[q];
            lt[top] = t + 1;
            lpd[top] = ch[i].pd;
            memcpy(lpath + (size_t)top * n, cur, sizeof(int) * n);
            lpath[(size_t)top * n + k] = ch[i].c;
            ++top;
        }
    }
    if (!(flags & ORC_BUDGET_EXHAUSTED)) flags |= ORC_CERTIFIED;
    /* empty: the whole tree was searched and no leaf lies inside the sphere */
    if (!(flags & ORC_FOUND) && (flags & ORC_CERTIFIED)) flags |= ORC_EMPTY_SPHERE;
    if (pd_out) {
        if (best < INFINITY) *pd_out = best;
        else if (x_init) { /* the warm start was never beaten: report its pd */
            double* g = (double*)malloc(sizeof(double) * n);
            orc_path_terms(n, P, R, z, x_out, g);
            double s = 0.0;
            for (int k = 0; k < n; ++k) s += g[k];
            *pd_out = s;
            free(g);
        } else *pd_out = INFINITY;
    }
    if (counters) {
        counters[0] += expanded;
        counters[1] += evaluated;
        counters[3] += stale;
    }
    free(lt);
    free(lpd);
    free(lpath);
    free(cur);
    free(ch);
    return flags;
}

/* Reading of Sec. III-B, which leaves an empty sphere open: the frame is
 * searched again with r2 = +inf; its flags keep EMPTY_SPHERE and the
 * counters add up both searches. */
uint32_t orc_sesd(int n, int P, const double* R, const double* z, double r2, int64_t budget,
                  const int* x_init, int* x_out, double* pd_out, int64_t* counters)
{
    uint32_t f = sesd_search(n, P, R, z, r2, budget, x_init, x_out, pd_out, counters);
    if ((f & ORC_EMPTY_SPHERE) && isfinite(r2))
        f = sesd_search(n, P, R, z, INFINITY, budget, x_init, x_out, pd_out, counters) | ORC_EMPTY_SPHERE;
    return f;
}

/* ------------------------------------------------------------------ */
/* K-best (Sec. VI)                                                    */
/* ------------------------------------------------------------------ */
typedef struct {
    double pd;
    int parent; /* rank of the parent in the previous survivor list */
    int c;      /* child index: PAM digits of the J fixed levels, top level most significant */
} cand_t;

static int cmp_cand(const void* a, const void* b)
{
    const cand_t* x = (const cand_t*)a;
    const cand_t* y = (const cand_t*)b;
    if (x->pd < y->pd) return -1;
    if (x->pd > y->pd) return 1;
    if (x->parent != y->parent) return (x->parent > y->parent) - (x->parent < y->parent);
    return (x->c > y->c) - (x->c < y->c);
}

static int ipow(int b, int e)
{
    int r = 1;
    while (e-- > 0) r *= b;
    return r;
}

/* pd of the child that fixes levels k_hi .. k_hi-J+1 with digits of c below
 * a parent path par (levels above k_hi fixed) */
static double child_pd(int n, int P, const double* R, const double* z, int k_hi, int J, int c,
                       const int* par, double pd, int* tmp)
{
    memcpy(tmp, par, sizeof(int) * n);
    int nc = ipow(P, J);
    for (int q = 0; q < J; ++q) {
        nc /= P;
        int k = k_hi - q;
        tmp[k] = (c / nc) % P;
        double b = centre(n, P, R, z, k, tmp);
        double e = b - R[k * n + k] * amp(P, tmp[k]);
        pd += e * e;
    }
    return pd;
}

static uint32_t kbest_search(int n, int P, const double* R, const double* z, int K, const int* k_sched,
                             double r2, int J, const int* force_path, int* x_out, double* pd_out,
                             double* margin_out, int* rank_out, double* fgap_out, double* rgap_out,
                             int64_t* counters)
{
    if (J < 1 || n % J != 0) return 0;
    const int kmax = K < 1 ? 1 : K; /* K is the capacity; schedule values are clamped to it */
    const int nc = ipow(P, J);
    int* path = (int*)calloc((size_t)kmax * n, sizeof(int));
    int* npath = (int*)calloc((size_t)kmax * n, sizeof(int));
    double* spd = (double*)calloc((size_t)kmax, sizeof(double));
    double* nspd = (double*)calloc((size_t)kmax, sizeof(double));
    cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)kmax * nc);
    int* tmp = (int*)malloc(sizeof(int) * n);
    int cnt = 1; /* the root */
    int forced_rank = 0; /* rank of the forced prefix in the survivor list, -1 if absent */
    int64_t expanded = 0, evaluated = 0;
    uint32_t flags = 0;
    if (margin_out) {
        margin_out[0] = INFINITY;
        margin_out[1] = margin_out[2] = 0.0;
    }

    for (int t = 0; t < n; t += J) {
        int k_hi = n - 1 - t, k_lo = k_hi - J + 1;
        int Kt = k_sched ? k_sched[k_lo] : K;
        if (Kt > kmax) Kt = kmax;
        if (Kt < 1) Kt = 1;
        int m = 0;
        for (int r = 0; r < cnt; ++r) {
            ++expanded;
            for (int c = 0; c < nc; ++c) {
                double pd = child_pd(n, P, R, z, k_hi, J, c, path + (size_t)r * n, spd[r], tmp);
                evaluated += J;
                if (isfinite(r2)) note_gap(margin_out, pd, r2);
                if (pd < r2) {
                    cand[m].pd = pd;
                    cand[m].parent = r;
                    cand[m].c = c;
                    ++m;
                }
            }
        }
        if (m == 0) {
            flags |= ORC_EMPTY_SPHERE;
            cnt = 0;
            break;
        }
        qsort(cand, (size_t)m, sizeof(cand_t), cmp_cand);
        int keep = Kt < m ? Kt : m;
        if (t + J < n) {
            if (m > keep) note_gap(margin_out, cand[keep - 1].pd, cand[keep].pd);
        } else if (m > 1) {
            note_gap(margin_out, cand[0].pd, cand[1].pd);
        }
        if (force_path) {
            /* locate the forced prefix among the sorted candidates */
            int fc = 0;
            for (int q = 0; q < J; ++q) fc = fc * P + force_path[k_hi - q];
            int pos = -1;
            for (int i = 0; i < m; ++i)
                if (cand[i].parent == forced_rank && cand[i].c == fc) {
                    pos = i;
                    break;
                }
            if (rank_out) rank_out[k_lo] = pos >= 0 ? pos + 1 : 0;
            if (rgap_out) {
                /* how close the rank is to changing: the smallest relative gap
                 * between the forced candidate and any other, or between the
                 * last survivor and the first dropped candidate */
                double g = INFINITY;
                for (int i = 0; pos >= 0 && i < m; ++i)
                    if (i != pos) {
                        double gi = rel_gap(cand[i].pd, cand[pos].pd);
                        if (gi < g) g = gi;
                    }
                if (m > keep) {
                    double gb = rel_gap(cand[keep - 1].pd, cand[keep].pd);
                    if (gb < g) g = gb;
                }
                rgap_out[k_lo] = g;
            }
            if (fgap_out) {
                /* the decision that drops the forced prefix (or, at the leaves,
                 * prefers another leaf): relative gap of the two keys */
                double g = 0.0;
                if (pos < 0) g = INFINITY;
                else if (t + J < n && pos >= keep) g = rel_gap(cand[pos].pd, cand[keep - 1].pd);
                else if (t + J >= n && pos > 0) g = rel_gap(cand[pos].pd, cand[0].pd);
                if (g > *fgap_out) *fgap_out = g;
            }
            if (pos < 0) { /* outside the sphere: the forced path ends here */
                force_path = NULL;
            } else if (pos >= keep) { /* keep it anyway: it replaces the last survivor */
                cand_t f = cand[pos];
                for (int i = pos; i > keep - 1; --i) cand[i] = cand[i - 1];
                cand[keep - 1] = f;
                pos = keep - 1;
            }
            forced_rank = pos;
        }
        for (int i = 0; i < keep; ++i) {
            const int* par = path + (size_t)cand[i].parent * n;
            int* dst = npath + (size_t)i * n;
            memcpy(dst, par, sizeof(int) * n);
            int d = nc;
            for (int q = 0; q < J; ++q) {
                d /= P;
                dst[k_hi - q] = (cand[i].c / d) % P;
            }
            nspd[i] = cand[i].pd;
        }
        int* tp = path;
        path = npath;
        npath = tp;
        double* tq = spd;
        spd = nspd;
        nspd = tq;
        cnt = keep;
    }
    if (cnt > 0) {
        memcpy(x_out, path, sizeof(int) * n); /* survivor 0 is the best leaf */
        if (pd_out) *pd_out = spd[0];
        flags |= ORC_FOUND;
    } else if (pd_out) {
        *pd_out = INFINITY;
    }
    if (counters) {
        counters[0] += expanded;
        counters[1] += evaluated;
    }
    free(path);
    free(npath);
    free(spd);
    free(nspd);
    free(cand);
    free(tmp);
    return flags;
}

/* smaller of two near-tie margins (relative gap, the two values) */
static void merge_margin(double* margin, const double* other)
{
    if (margin && other[0] < margin[0]) memcpy(margin, other, sizeof(double) * 3);
}

/* An empty sphere is searched again with r2 = +inf (reading of Sec. III-B,
 * as for the SD). */
uint32_t orc_kbest(int n, int P, const double* R, const double* z, int K, const int* k_sched,
                   double r2, int J, const int* force_path, int* x_out, double* pd_out,
                   double* margin_out, int* rank_out, double* fgap_out, double* rgap_out,
                   int64_t* counters)
{
    if (fgap_out) *fgap_out = 0.0;
    uint32_t f = kbest_search(n, P, R, z, K, k_sched, r2, J, force_path, x_out, pd_out, margin_out,
                              rank_out, fgap_out, rgap_out, counters);
    if ((f & ORC_EMPTY_SPHERE) && isfinite(r2)) {
        double m2[3];
        if (fgap_out) *fgap_out = 0.0;
        f = kbest_search(n, P, R, z, K, k_sched, INFINITY, J, force_path, x_out, pd_out,
                         margin_out ? m2 : NULL, rank_out, fgap_out, rgap_out, counters) | ORC_EMPTY_SPHERE;
        if (margin_out) merge_margin(margin_out, m2);
    }
    return f;
}

/* ------------------------------------------------------------------ */
/* Hybrid SD-K-best (Sec. VI) in deterministic rounds                  */
/*                                                                     */
/* The paper's master/worker threads run asynchronously; this oracle    */
/* fixes one deterministic schedule.  Each round:                       */
/*  1. the master takes the leftmost pool node (discarding nodes whose  */
/*     pd is no longer inside the sphere), expands it, drops children   */
/*     outside the sphere, offers leaf children as candidates and       */
/*     inserts the others at the left, best leftmost (Best-FS);         */
/*  2. each idle worker, in worker order, takes the rightmost node while */
/*     the pool holds at least two nodes (stale nodes are discarded);   */
/*  3. each busy worker advances its K-best by one level inside the     */
/*     sphere; it goes idle when nothing is left or at the leaves,      */
/*     whose survivors become candidates;                               */
/*  4. the best candidate by (pd, source, rank) with source master <    */
/*     worker 0 < worker 1 ... shrinks the radius if it is inside it.   */
/* Steps 1-3 use the radius of the start of the round.  The run ends    */
/* when the pool is empty and every worker is idle.                     */
/* ------------------------------------------------------------------ */
typedef struct {
    double pd;
    int src;
    int rank;
    const int* path;
    int k;
    int c;
} hcand_t;

/* digits of child c (top level most significant) into levels k_hi .. k_hi-J+1 */
static void set_digits(int* path, int P, int k_hi, int J, int c)
{
    for (int q = J - 1; q >= 0; --q) {
        path[k_hi - q] = c % P;
        c /= P;
    }
}

static uint32_t hybrid_search(int n, int P, int J, const double* R, const double* z, double r2, int W, int Kw,
                              const int* k_sched, int master_off, int64_t budget, int* x_out,
                              double* pd_out, double* margin_out, int64_t* counters, trace_t* T)
{
    const int kmax = Kw < 1 ? 1 : Kw; /* Kw is the capacity; schedule values are clamped to it */
    const int PC = ipow(P, J);        /* children per step: J real levels */
    const int cap = (n / J + 1) * PC + 8;
    int* qt = (int*)malloc(sizeof(int) * cap);
    double* qpd = (double*)malloc(sizeof(double) * cap);
    int* qpath = (int*)malloc(sizeof(int) * (size_t)cap * n);
    int head = 0, size = 0;

    int nw = W > 0 ? W : 1;
    int* wbusy = (int*)calloc((size_t)nw, sizeof(int));
    int* wt = (int*)calloc((size_t)nw, sizeof(int));
    int* wcnt = (int*)calloc((size_t)nw, sizeof(int));
    double* wpd = (double*)calloc((size_t)nw * kmax, sizeof(double));
    int* wpath = (int*)calloc((size_t)nw * kmax * n, sizeof(int));
    double* npd = (double*)calloc((size_t)kmax, sizeof(double));
    int* npath = (int*)calloc((size_t)kmax * n, sizeof(int));
    cand_t* cand = (cand_t*)malloc(sizeof(cand_t) * (size_t)kmax * PC);
    /* round candidates: at most PC from the master and kmax per worker */
    hcand_t* hc = (hcand_t*)malloc(sizeof(hcand_t) * (size_t)(PC + nw * kmax));
    int* leafbuf = (int*)malloc(sizeof(int) * (size_t)(PC + nw * kmax) * n);
    int* cur = (int*)malloc(sizeof(int) * n);
    int* tmp = (int*)malloc(sizeof(int) * n);
    child_t* ch = (child_t*)malloc(sizeof(child_t) * (size_t)PC);
    int64_t expanded = 0, evaluated = 0, rounds = 0, stale = 0;
    uint32_t flags = 0;
    double best = INFINITY;
    if (margin_out) {
        margin_out[0] = INFINITY;
        margin_out[1] = margin_out[2] = 0.0;
    }

    if (master_off) {
        if (W >= 1) {
            wbusy[0] = 1;
            wt[0] = 0;
            wcnt[0] = 1;
            wpd[0] = 0.0;
            for (int j = 0; j < n; ++j) wpath[j] = 0;
        }
    } else {
        qt[0] = 0;
        qpd[0] = 0.0;
        for (int j = 0; j < n; ++j) qpath[j] = 0;
        size = 1;
    }

    for (;;) {
        int any_busy = 0;
        for (int w = 0; w < W; ++w) any_busy |= wbusy[w];
        if (size == 0 && !any_busy) {
            flags |= ORC_CERTIFIED;
            break;
        }
        if (budget > 0 && expanded >= budget) {
            flags |= ORC_BUDGET_EXHAUSTED;
            break;
        }
        ++rounds;
        const double r2r = r2;
        int nh = 0;
        tr(T, "round %lld r2 %.6g pool %d\n", (long long)rounds, r2r, size);

        /* 1. master */
        if (!master_off) {
            while (size > 0) {
                int slot = head;
                head = (head + 1) % cap;
                --size;
                int t = qt[slot];
                double pd = qpd[slot];
                if (isfinite(r2r)) note_gap(margin_out, pd, r2r);
                if (pd >= r2r) {
                    ++stale;
                    tr(T, "master stale depth %d pd %.6g\n", t, pd);
                    continue;
                }
                memcpy(cur, qpath + (size_t)slot * n, sizeof(int) * n);
                ++expanded;
                tr(T, "master expand depth %d pd %.6g\n", t, pd);
                int k = n - 1 - t; /* the step fixes levels k .. k-J+1 */
                for (int c = 0; c < PC; ++c) {
                    ch[c].pd = child_pd(n, P, R, z, k, J, c, cur, pd, tmp);
                    ch[c].c = c;
                    evaluated += J;
                }
                qsort(ch, (size_t)PC, sizeof(child_t), cmp_child);
                int nk = 0;
                for (int i = 0; i < PC; ++i) {
                    if (isfinite(r2r)) note_gap(margin_out, ch[i].pd, r2r);
                    if (ch[i].pd < r2r) nk = i + 1;
                }
                for (int i = 0; i + 1 < nk; ++i) note_gap(margin_out, ch[i].pd, ch[i + 1].pd);
                for (int i = 0; i < nk; ++i) tr(T, "  child %d pd %.6g%s\n", ch[i].c, ch[i].pd, t + J == n ? " leaf" : "");
                if (t + J == n) {
                    for (int i = 0; i < nk; ++i) {
                        int* lp = leafbuf + (size_t)nh * n;
                        memcpy(lp, cur, sizeof(int) * n);
                        set_digits(lp, P, k, J, ch[i].c);
                        hc[nh].pd = ch[i].pd;
                        hc[nh].src = 0;
                        hc[nh].rank = i;
                        hc[nh].path = lp;
                        ++nh;
                    }
                } else {
                    for (int i = nk - 1; i >= 0; --i) {
                        head = (head - 1 + cap) % cap;
                        ++size;
                        qt[head] = t + J;
                        qpd[head] = ch[i].pd;
                        memcpy(qpath + (size_t)head * n, cur, sizeof(int) * n);
                        set_digits(qpath + (size_t)head * n, P, k, J, ch[i].c);
                    }
                }
                break;
            }
        }

        /* 2. idle workers take the rightmost node */
        for (int w = 0; w < W; ++w) {
            if (wbusy[w]) continue;
            while (size >= 2) {
                int slot = (head + size - 1) % cap;
                --size;
                if (isfinite(r2r)) note_gap(margin_out, qpd[slot], r2r);
                if (qpd[slot] >= r2r) {
                    ++stale;
                    tr(T, "worker %d stale depth %d pd %.6g\n", w, qt[slot], qpd[slot]);
                    continue;
                }
                tr(T, "worker %d takes depth %d pd %.6g\n", w, qt[slot], qpd[slot]);
                wbusy[w] = 1;
                wt[w] = qt[slot];
                wcnt[w] = 1;
                wpd[(size_t)w * kmax] = qpd[slot];
                memcpy(wpath + (size_t)w * kmax * n, qpath + (size_t)slot * n, sizeof(int) * n);
                break;
            }
        }

        /* 3. busy workers advance one K-best level */
        for (int w = 0; w < W; ++w) {
            if (!wbusy[w]) continue;
            int t = wt[w], k = n - 1 - t; /* the step fixes levels k .. k-J+1; K_t read at the lowest */
            int Kt = k_sched ? k_sched[k - J + 1] : Kw;
            if (Kt > kmax) Kt = kmax;
            if (Kt < 1) Kt = 1;
            double* spd = wpd + (size_t)w * kmax;
            int* sp = wpath + (size_t)w * kmax * n;
            int m = 0;
            for (int r = 0; r < wcnt[w]; ++r) {
                ++expanded;
                for (int c = 0; c < PC; ++c) {
                    double pd = child_pd(n, P, R, z, k, J, c, sp + (size_t)r * n, spd[r], tmp);
                    evaluated += J;
                    if (isfinite(r2r)) note_gap(margin_out, pd, r2r);
                    if (pd < r2r) {
                        cand[m].pd = pd;
                        cand[m].parent = r;
                        cand[m].c = c;
                        ++m;
                    }
                }
            }
            if (m == 0) {
                wbusy[w] = 0;
                tr(T, "worker %d depth %d nothing inside: idle\n", w, t);
                continue;
            }
            qsort(cand, (size_t)m, sizeof(cand_t), cmp_cand);
            int keep = Kt < m ? Kt : m;
            if (m > keep && t + J < n) note_gap(margin_out, cand[keep - 1].pd, cand[keep].pd);
            for (int i = 0; i < keep; ++i)
                tr(T, "worker %d depth %d keeps parent %d child %d pd %.6g%s\n", w, t, cand[i].parent, cand[i].c,
                   cand[i].pd, t + J == n ? " leaf" : "");
            for (int i = 0; i < keep; ++i) {
                memcpy(npath + (size_t)i * n, sp + (size_t)cand[i].parent * n, sizeof(int) * n);
                set_digits(npath + (size_t)i * n, P, k, J, cand[i].c);
                npd[i] = cand[i].pd;
            }
            memcpy(sp, npath, sizeof(int) * (size_t)keep * n);
            memcpy(spd, npd, sizeof(double) * keep);
            wcnt[w] = keep;
            wt[w] = t + J;
            if (t + J == n) {
                for (int i = 0; i < keep; ++i) {
                    int* lp = leafbuf + (size_t)nh * n;
                    memcpy(lp, sp + (size_t)i * n, sizeof(int) * n);
                    hc[nh].pd = spd[i];
                    hc[nh].src = 1 + w;
                    hc[nh].rank = i;
                    hc[nh].path = lp;
                    ++nh;
                }
                wbusy[w] = 0;
            }
        }

        /* 4. merge the round's candidates and update the radius once */
        int bi = -1;
        for (int i = 0; i < nh; ++i) {
            if (bi < 0) {
                bi = i;
                continue;
            }
            const hcand_t* a = &hc[i];
            const hcand_t* b = &hc[bi];
            int better = (a->pd < b->pd) || (a->pd == b->pd && (a->src < b->src ||
                          (a->src == b->src && a->rank < b->rank)));
            if (better) bi = i;
        }
        if (bi >= 0) {
            for (int i = 0; i < nh; ++i)
                if (i != bi) note_gap(margin_out, hc[i].pd, hc[bi].pd);
            if (isfinite(r2)) note_gap(margin_out, hc[bi].pd, r2);
            if (hc[bi].pd < r2) {
                r2 = hc[bi].pd;
                best = hc[bi].pd;
                memcpy(x_out, hc[bi].path, sizeof(int) * n);
                flags |= ORC_FOUND;
                tr(T, "radius %.6g from source %d\n", r2, hc[bi].src);
            }
        }
    }
    tr(T, "end expanded %lld evaluated %lld rounds %lld stale %lld\n", (long long)expanded,
       (long long)evaluated, (long long)rounds, (long long)stale);
    /* empty: the pool drained and no leaf lies inside the sphere */
    if (!(flags & ORC_FOUND) && (flags & ORC_CERTIFIED)) flags |= ORC_EMPTY_SPHERE;
    if (pd_out) *pd_out = best;
    if (counters) {
        counters[0] += expanded;
        counters[1] += evaluated;
        counters[2] += rounds;
        counters[3] += stale;
    }
    free(qt);
    free(qpd);
    free(qpath);
    free(wbusy);
    free(wt);
    free(wcnt);
    free(wpd);
    free(wpath);
    free(npd);
    free(npath);
    free(cand);
    free(hc);
    free(leafbuf);
    free(cur);
    free(tmp);
    free(ch);
    return flags;
}

/* An empty sphere is searched again with r2 = +inf (reading of Sec. III-B).
 * J real levels per step (1 or 2; n a multiple of J). */
uint32_t orc_hybrid(int n, int P, int J, const double* R, const double* z, double r2, int W, int Kw,
                    const int* k_sched, int master_off, int64_t budget, int* x_out, double* pd_out,
                    double* margin_out, int64_t* counters)
{
    if (J < 1 || n % J != 0) return 0;
    uint32_t f = hybrid_search(n, P, J, R, z, r2, W, Kw, k_sched, master_off, budget, x_out, pd_out,
                               margin_out, counters, NULL);
    if ((f & ORC_EMPTY_SPHERE) && isfinite(r2)) {
        double m2[3];
        f = hybrid_search(n, P, J, R, z, INFINITY, W, Kw, k_sched, master_off, budget, x_out, pd_out,
                          margin_out ? m2 : NULL, counters, NULL) | ORC_EMPTY_SPHERE;
        if (margin_out) merge_margin(margin_out, m2);
    }
    return f;
}

/* One frame of the hybrid with a text trace of its rounds written to buf
 * (at most cap bytes, NUL-terminated): the round-start radius and pool
 * size, every pop (expanded or stale) with its depth and pd, the children
 * kept, the workers' hand-offs and levels, and each radius update. */
uint32_t orc_hybrid_trace(int n, int P, int J, const double* R, const double* z, double r2, int W, int Kw,
                          int master_off, int64_t budget, int* x_out, double* pd_out, int64_t* counters,
                          char* buf, int cap)
{
    trace_t T = {buf, (size_t)(cap > 0 ? cap : 0), 0};
    if (cap > 0) buf[0] = 0;
    if (J < 1 || n % J != 0) return 0;
    return hybrid_search(n, P, J, R, z, r2, W, Kw, NULL, master_off, budget, x_out, pd_out, NULL, counters, &T);
}

/* ------------------------------------------------------------------ */
/* Learned-pruning state from the SIC path                             */
/* ------------------------------------------------------------------ */
void orc_prune_features(int n, int P, const double* R, const double* z, double sigma2, double* feat)
{
    const double c = orc_pam_scale(P);
    const double sr = sqrt(sigma2 / 2.0); /* real noise standard deviation */
    int* x = (int*)calloc((size_t)n, sizeof(int));
    double pd = 0.0;
    for (int k = n - 1; k >= 0; --k) {
        double b = centre(n, P, R, z, k, x);
        double u = b / R[k * n + k];
        x[k] = slice(P, u);
        double e = b - R[k * n + k] * amp(P, x[k]);
        pd += e * e;
        /* decision boundaries sit at the even multiples of c between the
         * outermost points; distance to the nearest one in units of 2c */
        double v = u / c;
        double nb = 2.0 * floor(v / 2.0 + 0.5);
        if (nb > (double)(P - 2)) nb = (double)(P - 2);
        if (nb < -(double)(P - 2)) nb = -(double)(P - 2);
        double d = fabs(v - nb) / 2.0;
        double* f = feat + (size_t)k * 4;
        f[0] = (double)k / (double)n;
        f[1] = d;
        f[2] = log2(R[k * n + k] * 2.0 * c / sr);
        f[3] = pd / ((double)(n - k) * sr * sr);
    }
    free(x);
}

/* ------------------------------------------------------------------ */
/* MLP 4 -> 128 -> 128 -> 1 (ReLU), pinball loss, Adam                 */
/* ------------------------------------------------------------------ */
/* One state through the MLP, FP64 throughout. */
static void mlp_one(const double* w, const double* x, double* a1, double* h1, double* a2,
                    double* h2, double* out)
{
    const int H = ORC_MLP_H;
    for (int i = 0; i < H; ++i) {
        double s = w[ORC_MLP_B1 + i];
        for (int j = 0; j < ORC_MLP_IN; ++j) s += w[ORC_MLP_W1 + i * ORC_MLP_IN + j] * x[j];
        a1[i] = s;
        h1[i] = s > 0.0 ? s : 0.0;
    }
    for (int i = 0; i < H; ++i) {
        double s = w[ORC_MLP_B2 + i];
        for (int j = 0; j < H; ++j) s += w[ORC_MLP_W2 + i * H + j] * h1[j];
        a2[i] = s;
        h2[i] = s > 0.0 ? s : 0.0;
    }
    double s = w[ORC_MLP_B3];
    for (int j = 0; j < H; ++j) s += w[ORC_MLP_W3 + j] * h2[j];
    *out = s;
}

void orc_mlp_forward(const double* w, const double* X, int B, double* out)
{
    double a1[ORC_MLP_H], h1[ORC_MLP_H], a2[ORC_MLP_H], h2[ORC_MLP_H];
    for (int b = 0; b < B; ++b) mlp_one(w, X + (size_t)b * ORC_MLP_IN, a1, h1, a2, h2, out + b);
}

double orc_mlp_loss_grad(const double* w, const double* X, const double* y, int B, double tau,
                         double* grad)
{
    const int H = ORC_MLP_H;
    double a1[ORC_MLP_H], h1[ORC_MLP_H], a2[ORC_MLP_H], h2[ORC_MLP_H], d2[ORC_MLP_H], d1[ORC_MLP_H];
    memset(grad, 0, sizeof(double) * ORC_MLP_NPARAM);
    double loss = 0.0;
    for (int b = 0; b < B; ++b) {
        const double* x = X + (size_t)b * ORC_MLP_IN;
        double o;
        mlp_one(w, x, a1, h1, a2, h2, &o);
        double r = y[b] - o;
        loss += r > 0.0 ? tau * r : (tau - 1.0) * r;
        double dout = (r > 0.0 ? -tau : 1.0 - tau) / (double)B;
        grad[ORC_MLP_B3] += dout;
        for (int j = 0; j < H; ++j) {
            grad[ORC_MLP_W3 + j] += dout * h2[j];
            d2[j] = a2[j] > 0.0 ? dout * w[ORC_MLP_W3 + j] : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            grad[ORC_MLP_B2 + i] += d2[i];
            for (int j = 0; j < H; ++j) grad[ORC_MLP_W2 + i * H + j] += d2[i] * h1[j];
        }
        for (int j = 0; j < H; ++j) {
            double s = 0.0;
            for (int i = 0; i < H; ++i) s += w[ORC_MLP_W2 + i * H + j] * d2[i];
            d1[j] = a1[j] > 0.0 ? s : 0.0;
        }
        for (int i = 0; i < H; ++i) {
            grad[ORC_MLP_B1 + i] += d1[i];
            for (int j = 0; j < ORC_MLP_IN; ++j) grad[ORC_MLP_W1 + i * ORC_MLP_IN + j] += d1[i] * x[j];
        }
    }
    return loss / (double)B;
}

void orc_adam_step(double* w, double* m, double* v, const double* g, int np, int t, double lr,
                   double beta1, double beta2, double eps)
{
    double c1 = 1.0 - pow(beta1, (double)t), c2 = 1.0 - pow(beta2, (double)t);
    for (int i = 0; i < np; ++i) {
        m[i] = beta1 * m[i] + (1.0 - beta1) * g[i];
        v[i] = beta2 * v[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = m[i] / c1, vh = v[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}

/* ------------------------------------------------------------------ */
/* Learned-pruning detector: per-level state -> MLP -> survivor counts  */
/* -> K-best with that schedule -> plain K-best where the first result  */
/* is flagged or fails the noise test                                   */
/* ------------------------------------------------------------------ */
/* survivor count of one state: clamp(ceil(2^(f + margin)), kmin, kmax) */
static int learned_count(double f, double margin, int kmin, int kmax)
{
    if (!isfinite(f)) return kmax;
    double e = f + margin;
    if (e > 30.0) e = 30.0;
    double k = ceil(exp2(e));
    if (k < (double)kmin) return kmin;
    if (k > (double)kmax) return kmax;
    return (int)k;
}

uint32_t orc_learned_detect(int n, int P, const double* R, const double* z, double sigma2, const double* w,
                            double margin, int kmin, int kmax, double beta, int K_fallback, int* x_out,
                            double* pd_out, int* k_sched_out, int64_t* counters)
{
    double* feat = (double*)malloc(sizeof(double) * (size_t)n * 4);
    double* pred = (double*)malloc(sizeof(double) * (size_t)n);
    int* ks = k_sched_out ? k_sched_out : (int*)malloc(sizeof(int) * (size_t)n);
    orc_prune_features(n, P, R, z, sigma2, feat);
    orc_mlp_forward(w, feat, n, pred);
    for (int k = 0; k < n; ++k) ks[k] = learned_count(pred[k], margin, kmin, kmax);
    double pd = INFINITY;
    uint32_t f = orc_kbest(n, P, R, z, kmax, ks, INFINITY, 1, NULL, x_out, &pd, NULL, NULL, NULL, NULL, counters);
    /* the noise test: a correct detection leaves a chi-square noise energy
     * with n real degrees of freedom, of mean n sigma2 / 2 */
    const double bound = 0.5 * sigma2 * ((double)n + beta * sqrt(2.0 * (double)n));
    if (!(f & ORC_FOUND) || !(pd <= bound)) {
        f = orc_kbest(n, P, R, z, K_fallback, NULL, INFINITY, 1, NULL, x_out, &pd, NULL, NULL, NULL, NULL,
                      counters) | ORC_LEARNED_FALLBACK;
    }
    if (pd_out) *pd_out = pd;
    free(feat);
    free(pred);
    if (!k_sched_out) free(ks);
    return f;
}

/* ------------------------------------------------------------------ */
/* batched drivers                                                     */
/* ------------------------------------------------------------------ */
void orc_batch_learned_detect(int B, int n, int P, const double* R, const double* z, const double* sigma2,
                              const double* w, double margin, int kmin, int kmax, double beta, int K_fallback,
                              int* x_out, double* pd_out, int* k_sched_out, uint32_t* flags)
{
#pragma omp parallel for schedule(dynamic, 2)
    for (int b = 0; b < B; ++b) {
        uint32_t f = orc_learned_detect(n, P, R + (size_t)b * n * n, z + (size_t)b * n, sigma2[b], w, margin, kmin,
                                        kmax, beta, K_fallback, x_out + (size_t)b * n, pd_out ? pd_out + b : NULL,
                                        k_sched_out ? k_sched_out + (size_t)b * n : NULL, NULL);
        if (flags) flags[b] = f;
    }
}

void orc_batch_qr(int B, int N, int M, const float* H, const float* y, double* R, double* z,
                  double* resid)
{
    const int n = 2 * M;
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b)
        orc_qr(N, M, H + (size_t)b * N * M * 2, y + (size_t)b * N * 2, R + (size_t)b * n * n,
               z + (size_t)b * n, resid ? resid + b : NULL);
}

void orc_batch_qr_mmse(int B, int N, int M, const float* H, const float* y, const double* sigma2, double* R,
                       double* z)
{
    const int n = 2 * M;
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b)
        orc_qr_mmse(N, M, H + (size_t)b * N * M * 2, y + (size_t)b * N * 2, sigma2[b], R + (size_t)b * n * n,
                    z + (size_t)b * n);
}

void orc_batch_linear(int B, int n, int P, const double* R, const double* z, int* x_idx, double* u)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b)
        orc_linear(n, P, R + (size_t)b * n * n, z + (size_t)b * n, x_idx + (size_t)b * n, u + (size_t)b * n);
}

void orc_batch_mrc(int B, int N, int M, int P, const float* H, const float* y, int* s_idx, double* u)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b)
        orc_mrc(N, M, P, H + (size_t)b * N * M * 2, y + (size_t)b * N * 2, s_idx + (size_t)b * M,
                u + (size_t)b * 2 * M);
}

void orc_batch_brute_force(int B, int N, int M, int P, const float* H, const float* y, int* s_idx,
                           double* metric)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b)
        orc_brute_force(N, M, P, H + (size_t)b * N * M * 2, y + (size_t)b * N * 2,
                        s_idx + (size_t)b * M, metric ? metric + b : NULL);
}

void orc_batch_metric(int B, int N, int M, int P, const float* H, const float* y,
                      const int* s_idx, double* metric)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b)
        metric[b] = orc_metric(N, M, P, H + (size_t)b * N * M * 2, y + (size_t)b * N * 2,
                               s_idx + (size_t)b * M);
}

void orc_batch_zf_sic(int B, int n, int P, const double* R, const double* z, int* x_idx, double* pd)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b) {
        double v = orc_zf_sic(n, P, R + (size_t)b * n * n, z + (size_t)b * n, x_idx + (size_t)b * n);
        if (pd) pd[b] = v;
    }
}

void orc_batch_sesd(int B, int n, int P, const double* R, const double* z, const double* r2,
                    int64_t budget, const int* x_init, int* x_out, double* pd_out,
                    uint32_t* flags, int64_t* counters)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
        int64_t ctr[ORC_NCOUNTERS] = {0, 0, 0, 0};
        uint32_t f = orc_sesd(n, P, R + (size_t)b * n * n, z + (size_t)b * n,
                              r2 ? r2[b] : INFINITY, budget,
                              x_init ? x_init + (size_t)b * n : NULL, x_out + (size_t)b * n,
                              pd_out ? pd_out + b : NULL, ctr);
        if (flags) flags[b] = f;
        if (counters)
            for (int i = 0; i < ORC_NCOUNTERS; ++i) counters[(size_t)b * ORC_NCOUNTERS + i] = ctr[i];
    }
}

void orc_batch_kbest(int B, int n, int P, const double* R, const double* z, int K,
                     const int* k_sched, int k_sched_stride, double r2, int J,
                     const int* force_path, int* x_out, double* pd_out, double* margin_out,
                     int* rank_out, double* fgap_out, double* rgap_out, uint32_t* flags, int64_t* counters)
{
#pragma omp parallel for schedule(dynamic, 4)
    for (int b = 0; b < B; ++b) {
        int64_t ctr[ORC_NCOUNTERS] = {0, 0, 0, 0};
        uint32_t f = orc_kbest(n, P, R + (size_t)b * n * n, z + (size_t)b * n, K,
                               k_sched ? k_sched + (size_t)b * k_sched_stride : NULL, r2, J,
                               force_path ? force_path + (size_t)b * n : NULL,
                               x_out + (size_t)b * n, pd_out ? pd_out + b : NULL,
                               margin_out ? margin_out + (size_t)b * 3 : NULL,
                               rank_out ? rank_out + (size_t)b * n : NULL,
                               fgap_out ? fgap_out + b : NULL, rgap_out ? rgap_out + (size_t)b * n : NULL,
                               ctr);
        if (flags) flags[b] = f;
        if (counters)
            for (int i = 0; i < ORC_NCOUNTERS; ++i) counters[(size_t)b * ORC_NCOUNTERS + i] = ctr[i];
    }
}

void orc_batch_hybrid(int B, int n, int P, int J, const double* R, const double* z, const double* r2, int W,
                      int Kw, const int* k_sched, int k_sched_stride, int master_off,
                      int64_t budget, int* x_out, double* pd_out, double* margin_out,
                      uint32_t* flags, int64_t* counters)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int b = 0; b < B; ++b) {
        int64_t ctr[ORC_NCOUNTERS] = {0, 0, 0, 0};
        uint32_t f = orc_hybrid(n, P, J, R + (size_t)b * n * n, z + (size_t)b * n, r2 ? r2[b] : INFINITY, W, Kw,
                                k_sched ? k_sched + (size_t)b * k_sched_stride : NULL, master_off,
                                budget, x_out + (size_t)b * n, pd_out ? pd_out + b : NULL,
                                margin_out ? margin_out + (size_t)b * 3 : NULL, ctr);
        if (flags) flags[b] = f;
        if (counters)
            for (int i = 0; i < ORC_NCOUNTERS; ++i) counters[(size_t)b * ORC_NCOUNTERS + i] = ctr[i];
    }
}

void orc_batch_prune_features(int B, int n, int P, const double* R, const double* z,
                              const double* sigma2, double* feat)
{
#pragma omp parallel for schedule(static)
    for (int b = 0; b < B; ++b)
        orc_prune_features(n, P, R + (size_t)b * n * n, z + (size_t)b * n, sigma2[b],
                           feat + (size_t)b * n * 4);
}
