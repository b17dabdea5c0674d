// QR preprocessing (Sec. III-B): H = Q R with R_kk real positive and
// z = Q^H y, emitted for the real model in packed level order.
//
// Method: Cholesky QR in FP64.  With A = [H | y] (N x (M+1)), the Gram matrix
// G = A^H A equals Rt^H Rt for Rt = [[R, z], [0, rho]], where R is the unique
// upper-triangular factor of H with a positive real diagonal (the factor a
// Householder QR yields once its rows are normalised to R_kk > 0), z is the
// first M entries of Q^H y and rho^2 = ||y||^2 - ||z||^2.  Products of the
// complex64 inputs are exact in FP64 and every sum rounds at 2^-53, so the
// error of R, which the Gram form amplifies by cond(H)^2, stays far below
// the FP32 rounding of the output for any channel with cond(H) < 10^5.
//
// A frame takes one thread per 4 x 4 complex tile of G's upper triangle
// (the tile stays in registers for the whole frame); frames of 4 to 6 waves
// run two per workgroup.
//   1. Gram: [H | y] streams through LDS in chunks of up to 16 rows (as many
//      as let each thread stage at most 4 elements), staged twice: an FP64
//      copy for the tile-row operand and an FP32 copy for the tile-column
//      operand, converted when read.  With two FP64 operands the loop is
//      bound by LDS reads, with two FP32 ones by the conversions' VALU
//      issue; one of each balances the two.  The next chunk is prefetched
//      into registers while the current one is consumed; each thread
//      accumulates conj(a_i)^T a_j over the rows for its tile.  The products
//      of FP32 inputs are exact in FP64, so the arithmetic is that of FP64
//      copies.
//   2. Right-looking Cholesky: at step k the owners of row k of the current
//      Schur complement publish it in LDS (double-buffered, so one barrier per
//      step) and every thread applies G_ij -= conj(g_ki) g_kj / g_kk to its
//      rows i > k.  Row k keeps its unscaled values; R_kj = g_kj / sqrt(g_kk).
//   3. Output: each thread scales its tile rows and writes the real blocks
//      [[a, -b], [b, a]] of R, and z from the column M.
// The complex factor maps onto the real model blockwise: R_2k,2k+1 = 0 and
// R_2k,2k = R_2k+1,2k+1 = R_kk.
#include "common.hpp"

namespace mimo {

constexpr int CQ_T = 4;       // tile edge in complex entries
constexpr int CQ_RCH_MAX = 16;  // rows of [H | y] per LDS chunk, at most
constexpr int CQ_PF = 4;        // chunk elements a thread stages, at most
constexpr int CQ_MAX_THREADS = 576;  // 33 x 34 / 2 = 561 tiles at n_tx = 128
constexpr int CQ_MAX_WG = 768;       // two frames of up to 6 waves per workgroup
// pivots below the smallest normal double count as zero: their row of R is 0
// and the Cholesky update skips them, so R stays finite for singular H
constexpr double CQ_PIVOT_MIN = 2.2250738585072014e-308;

struct CqShape {
    int C;       // M + 1 columns of [H | y]
    int nb;      // tile rows/columns: ceil(C / 4)
    int CP;      // padded columns 4 nb
    int ntiles;  // nb (nb + 1) / 2 upper-triangular tiles
};

__host__ __device__ inline CqShape cq_shape(int M)
{
    CqShape s;
    s.C = M + 1;
    s.nb = (s.C + CQ_T - 1) / CQ_T;
    s.CP = s.nb * CQ_T;
    s.ntiles = s.nb * (s.nb + 1) / 2;
    return s;
}

// one thread per tile (rounded up to whole waves)
__host__ __device__ inline int cq_threads(int M)
{
    const CqShape s = cq_shape(M);
    return (s.ntiles + WAVE - 1) / WAVE * WAVE;
}

// rows of [H | y] per LDS chunk for nthr threads: as many as let every
// thread stage at most CQ_PF elements, at most CQ_RCH_MAX
__host__ __device__ inline int cq_rows(int M, int nthr)
{
    const int r = CQ_PF * nthr / cq_shape(M).CP;
    return r < CQ_RCH_MAX ? (r < 1 ? 1 : r) : CQ_RCH_MAX;
}

// LDS bytes: row buffers [2][CP] complex double, pivots [CP] and a 4-entry
// spare [4] double, chunk buffers [2][rch][CP] complex double, then the same
// as complex float (at most 154 KB for two frames of up to 6 waves)
__host__ __device__ inline size_t cq_lds_bytes(int M, int rch)
{
    const int CP = cq_shape(M).CP;
    return (size_t)CP * (2 * 16 + 8) + CQ_T * 8 + (size_t)2 * rch * CP * (16 + 8);
}

struct cd {
    double x, y;
};

// element e of chunk c of [H | y] (rows rch c .. rch c + rch - 1, zero-padded
// to CP columns; e = row * CP + col).  Branch-free: an element outside the frame
// loads H[0] and is replaced by zero, so a thread's loads issue back to back.
// row = e / CP by a float reciprocal: e < 2^12 keeps it exact.
__device__ __forceinline__ float2 cq_elem(const float2* __restrict__ Hf, const float2* __restrict__ yf, int N, int M,
                                          int CP, float rcp_cp, int tot, int rch, int c, int e)
{
    const int row = (int)(((float)e + 0.5f) * rcp_cp);
    const int col = e - row * CP;
    const int i = c * rch + row;
    const bool valid = e < tot && i < N && col <= M;
    const float2* p = col < M ? Hf + ((size_t)i * M + col) : yf + i;
    p = valid ? p : Hf;
    const float2 v = *p;
    return valid ? v : make_float2(0.f, 0.f);
}

// LDS slot of chunk element e (row, col = 4J + q) in the chunk layout
// [row][q][J], so that the lanes of a wave (consecutive J) read neighbours.
__device__ __forceinline__ int cq_lds_slot(int e, int CP, int nb, float rcp_cp)
{
    const int row = (int)(((float)e + 0.5f) * rcp_cp);
    const int col = e - row * CP;
    const int J = col >> 2, q = col & 3;
    return row * CP + q * nb + J;
}

// 1 / d for d >= CQ_PIVOT_MIN (else 0, so the result
// is always finite): hardware reciprocal refined by two Newton steps
__device__ __forceinline__ double cq_inv(double d)
{
    double inv = __builtin_amdgcn_rcp(d);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    inv = fma(inv, fma(-d, inv, 1.0), inv);
    return d >= CQ_PIVOT_MIN ? inv : 0.0;
}

// publish register row LR of the tile (a compile-time index keeps the tile
// in registers).  A published row is stored in planes: column j = 4J + q at
// [q][J], so the lanes of a wave, which hold consecutive J, read 16-byte
// neighbours (no LDS bank conflicts).  In the diagonal tile the entries up to
// and including the pivot are published as zeros: a reader scales the entry
// in its own row's column, so the rows that are already final (up to the
// pivot row) get a zero update without a per-row mask, and the entries left
// of the diagonal, which no output reads, are not updated.  The owner of the
// diagonal entry also publishes its reciprocal, which every thread of the next
// step needs, and records the pivot for the output.
template <int LR>
__device__ __forceinline__ void cq_store_row(cd* row, double* rinv, double* pivot, int nb, int I, int J,
                                             const double (&gr)[CQ_T][CQ_T], const double (&gi)[CQ_T][CQ_T])
{
#pragma unroll
    for (int c = 0; c < CQ_T; ++c) {
        const bool z = J == I && c <= LR;
        row[c * nb + J] = {z ? 0.0 : gr[LR][c], z ? 0.0 : gi[LR][c]};
    }
    if (J == I) {
        *rinv = cq_inv(gr[LR][LR]);
        *pivot = gr[LR][LR];
    }
}

// orders one wave's LDS writes before its later LDS reads (a wave's LDS
// operations complete in order; this keeps the compiler from reordering them
// and waits for the writes)
__device__ __forceinline__ void cq_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_s_waitcnt(0xC07F);  // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// one step k of the right-looking Cholesky; S = k mod 4 (row k+1 sits in
// register row (S + 1) mod 4 of the tiles that publish it).  NBC > 0 fixes
// the tile-row count at compile time (else nb_ is used): the plane offsets
// q nb of the LDS rows then fold into the instructions' offset fields.  wg:
// the step's tiles span several waves (workgroup barrier), else one wave
// runs the step alone.
template <int S, int NBC>
__device__ __forceinline__ void cq_step(int k, int M, int nb_, bool wg, bool has_tile, int I, int J, int i0,
                                        cd* rowbuf, double* rinv, double* diag, double (&gr)[CQ_T][CQ_T],
                                        double (&gi)[CQ_T][CQ_T])
{
    const int nb = NBC > 0 ? NBC : nb_;
    const int CP = CQ_T * nb;
    if (wg)
        __syncthreads();  // row k published; the other buffer is free
    else
        cq_wave_sync();
    const cd* rk = rowbuf + (k & 1) * CP;
    if (has_tile && i0 + CQ_T - 1 > k) {
        const double inv = rinv[k & 1];  // 1 / g_kk
        double ur[CQ_T], ui[CQ_T], vr[CQ_T], vi[CQ_T];
#pragma unroll
        for (int r = 0; r < CQ_T; ++r) {
            const cd a = rk[r * nb + I];  // 0 for the final rows <= k
            ur[r] = a.x * inv;
            ui[r] = -a.y * inv;
            const cd b = rk[r * nb + J];
            vr[r] = b.x;
            vi[r] = b.y;
        }
        // G_ij -= conj(g_ki) g_kj / g_kk
#pragma unroll
        for (int r = 0; r < CQ_T; ++r)
#pragma unroll
            for (int q = 0; q < CQ_T; ++q) {
                gr[r][q] = fma(-ur[r], vr[q], gr[r][q]);
                gr[r][q] = fma(ui[r], vi[q], gr[r][q]);
                gi[r][q] = fma(-ur[r], vi[q], gi[r][q]);
                gi[r][q] = fma(-ui[r], vr[q], gi[r][q]);
            }
        if (k + 1 < M && (k + 1) / CQ_T == I)
            cq_store_row<(S + 1) & (CQ_T - 1)>(rowbuf + ((k + 1) & 1) * CP, rinv + ((k + 1) & 1), diag + k + 1, nb,
                                               I, J, gr, gi);
    }
}

template <int NBC>
__device__ __forceinline__ void cholqr_frame(const float2* __restrict__ Hf, const float2* __restrict__ yf, int N,
                                             int M, float* __restrict__ Rf, float* __restrict__ zf,
                                             float* __restrict__ resid_out, const float* __restrict__ load,
                                             unsigned char* smem, int tid, int nthr, bool live)
{
    const CqShape sh = cq_shape(M);
    const int nb = NBC > 0 ? NBC : sh.nb;
    const int CP = CQ_T * nb;
    const int n = 2 * M;
    cd* rowbuf = reinterpret_cast<cd*>(smem);                   // [2][4][nb]
    double* diag = reinterpret_cast<double*>(rowbuf + 2 * CP);  // [CP] pivots, then [4] spare
    const int rch = cq_rows(M, nthr);
    cd* ach64 = reinterpret_cast<cd*>(diag + CP + CQ_T);          // [2][rch][4][nb] complex double
    float2* ach32 = reinterpret_cast<float2*>(ach64 + 2 * rch * CP);  // [2][rch][4][nb] complex float

    // tile (I, J), I <= J, enumerated row by row from thread `toff` on: the
    // idle lanes of the frame's last wave move to its first, so that the
    // last wave holds as many of the trailing tile rows as fit (see step 2)
    const int tpf = cq_threads(M);       // the frame's threads, whole waves
    const int toff = tpf - sh.ntiles;    // threads before the first tile
    const bool has_tile = tid >= toff && tid < tpf;
    int I = 0, J = 0;
    if (has_tile) {
        int rem = tid - toff;
        while (rem >= sh.nb - I) {
            rem -= sh.nb - I;
            ++I;
        }
        J = I + rem;
    }
    const int i0 = CQ_T * I, j0 = CQ_T * J;

    double gr[CQ_T][CQ_T], gi[CQ_T][CQ_T];
#pragma unroll
    for (int r = 0; r < CQ_T; ++r)
#pragma unroll
        for (int c = 0; c < CQ_T; ++c) gr[r][c] = gi[r][c] = 0.0;

    // ---- 1. Gram matrix over chunks of 16 rows
    const int nchunk = (N + rch - 1) / rch;
    const int tot = rch * CP;
    const float rcp_cp = 1.0f / (float)CP;
    float2 pf[CQ_PF];
#pragma unroll
    for (int q = 0; q < CQ_PF; ++q) pf[q] = cq_elem(Hf, yf, N, M, CP, rcp_cp, tot, rch, 0, tid + q * nthr);
    for (int c = 0; c < nchunk; ++c) {
        cd* buf64 = ach64 + (c & 1) * tot;
        float2* buf32 = ach32 + (c & 1) * tot;
#pragma unroll
        for (int q = 0; q < CQ_PF; ++q) {
            const int e = tid + q * nthr;
            if (e < tot) {
                const int slot = cq_lds_slot(e, CP, nb, rcp_cp);
                buf64[slot] = {(double)pf[q].x, (double)pf[q].y};
                buf32[slot] = pf[q];
            }
        }
        __syncthreads();  // chunk c visible; chunk c-1's buffer no longer read
        if (c + 1 < nchunk) {
#pragma unroll
            for (int q = 0; q < CQ_PF; ++q)
                pf[q] = cq_elem(Hf, yf, N, M, CP, rcp_cp, tot, rch, c + 1, tid + q * nthr);
        }
        if (has_tile) {
            const int nr = min(rch, N - c * rch);
            for (int rr = 0; rr < nr; ++rr) {
                const cd* row64 = buf64 + rr * CP;
                const float2* row32 = buf32 + rr * CP;
                double ar[CQ_T], ai[CQ_T], br[CQ_T], bi[CQ_T];
#pragma unroll
                for (int q = 0; q < CQ_T; ++q) {
                    const cd a = row64[q * nb + I];
                    const float2 b = row32[q * nb + J];
                    ar[q] = a.x;
                    ai[q] = a.y;
                    br[q] = (double)b.x;
                    bi[q] = (double)b.y;
                }
                // G_ij += conj(a_i) a_j
#pragma unroll
                for (int r = 0; r < CQ_T; ++r)
#pragma unroll
                    for (int q = 0; q < CQ_T; ++q) {
                        gr[r][q] = fma(ar[r], br[q], gr[r][q]);
                        gr[r][q] = fma(ai[r], bi[q], gr[r][q]);
                        gi[r][q] = fma(ar[r], bi[q], gi[r][q]);
                        gi[r][q] = fma(-ai[r], br[q], gi[r][q]);
                    }
            }
        }
    }

    // MMSE preprocessing: G + sigma^2 I on the first M diagonal entries (the
    // Gram matrix of [H; sigma I], whose factor is the QR of that system)
    if (load && has_tile && I == J) {
        const double l = (double)*load;
#pragma unroll
        for (int r = 0; r < CQ_T; ++r)
            if (i0 + r < M) gr[r][r] += l;
    }

    // ---- 2. right-looking Cholesky, one barrier per step (unrolled by the
    //         tile edge so the published register row is a constant).  Step
    //         k updates the tiles of tile rows >= k / 4 only; from the first
    //         tile row whose tiles all sit in the frame's last wave (tiles
    //         are numbered row by row), that wave runs the remaining steps
    //         alone, without workgroup barriers, and the other waves go on
    //         to the output: their rows and pivots are final by then.
    const int last0 = tpf - WAVE - toff > 0 ? tpf - WAVE - toff : 0;  // first tile of the last wave
    int Iw = 0;  // first tile row starting at or after last0 (tile (I, I) is number I nb - I (I - 1) / 2)
    while (Iw * nb - Iw * (Iw - 1) / 2 < last0) ++Iw;
    const int k1 = min(M, CQ_T * Iw);
    const bool tail = tid >= tpf - WAVE;  // this thread's wave runs the steps k >= k1
    double* rinv = diag + CP;        // [2] reciprocal pivots of the published rows
    if (has_tile && I == 0) cq_store_row<0>(rowbuf, rinv, diag, nb, I, J, gr, gi);
    for (int kb = 0; kb < M; kb += CQ_T) {
        if (kb >= k1 && !tail) break;
        // the tail wave is the workgroup's critical path: its instructions go
        // ahead of the other waves' output on the same SIMD
        if (kb == k1) __builtin_amdgcn_s_setprio(2);
        cq_step<0, NBC>(kb, M, nb, kb < k1, has_tile, I, J, i0, rowbuf, rinv, diag, gr, gi);
        if (kb + 1 < M) cq_step<1, NBC>(kb + 1, M, nb, kb + 1 < k1, has_tile, I, J, i0, rowbuf, rinv, diag, gr, gi);
        if (kb + 2 < M) cq_step<2, NBC>(kb + 2, M, nb, kb + 2 < k1, has_tile, I, J, i0, rowbuf, rinv, diag, gr, gi);
        if (kb + 3 < M) cq_step<3, NBC>(kb + 3, M, nb, kb + 3 < k1, has_tile, I, J, i0, rowbuf, rinv, diag, gr, gi);
    }
    if (tail) cq_wave_sync();  // the tail's own last pivot writes
    __builtin_amdgcn_s_setprio(0);

    // ---- 3. output: R_ij = g_ij / sqrt(g_ii), real blocks in packed level order
    if (has_tile && live) {
#pragma unroll
        for (int r = 0; r < CQ_T; ++r) {
            const int i = i0 + r;
            if (i >= M) continue;
            const double d = diag[i];
            const bool pos = d >= CQ_PIVOT_MIN;
            const double s = pos ? sqrt(d) : 0.0;
            const double is = pos ? 1.0 / s : 0.0;
            float* row_re = Rf + r_row_off(n, 2 * i);
            float* row_im = Rf + r_row_off(n, 2 * i + 1);
#pragma unroll
            for (int q = 0; q < CQ_T; ++q) {
                const int j = j0 + q;
                if (j < i || j > M) continue;
                const float vx = (float)(gr[r][q] * is), vy = (float)(gi[r][q] * is);
                if (j == M) {
                    zf[2 * i] = vx;
                    zf[2 * i + 1] = vy;
                } else if (j == i) {
                    row_re[0] = (float)s;
                    row_re[1] = 0.f;
                    row_im[0] = (float)s;
                } else {
                    row_re[2 * (j - i)] = vx;
                    row_re[2 * (j - i) + 1] = -vy;
                    row_im[2 * (j - i) - 1] = vy;
                    row_im[2 * (j - i)] = vx;
                }
            }
        }
        // rho^2 = ||y||^2 - ||z||^2 is the Schur complement left at (M, M)
        if (resid_out && I == J && I == M / CQ_T) {
            const int r = M & (CQ_T - 1);
            const double v = r == 0 ? gr[0][0] : r == 1 ? gr[1][1] : r == 2 ? gr[2][2] : gr[3][3];
            *resid_out = (float)(v > 0.0 ? v : 0.0);
        }
    }
    __syncthreads();  // the LDS may be reused by the next frame
}

// Frames of up to 6 waves are processed two per workgroup (12 waves, 3 per
// SIMD): a workgroup of 6 waves at 3 waves per SIMD leaves the second
// workgroup of a CU no room on the SIMDs that hold two of its waves.  tpf
// threads per frame; a second half beyond the batch computes the last frame
// again and stores nothing.  NBC: compile-time tile-row count, or 0.
template <int NBC>
__global__ void __launch_bounds__(CQ_MAX_WG) qr_kernel(const float2* __restrict__ H, const float2* __restrict__ y,
                                                       int N, int M, float* __restrict__ R, float* __restrict__ z,
                                                       float* __restrict__ resid, const float* __restrict__ load,
                                                       int B, int fpw, int tpf)
{
    extern __shared__ __align__(16) unsigned char smem_qr[];
    const int half = (int)threadIdx.x / tpf;
    const int f = (int)blockIdx.x * fpw + half;
    const bool live = f < B;
    const int frame = live ? f : B - 1;
    const int n = 2 * M;
    const size_t lds = (cq_lds_bytes(M, cq_rows(M, tpf)) + 15) & ~(size_t)15;
    cholqr_frame<NBC>(H + (size_t)frame * N * M, y + (size_t)frame * N, N, M, R + (size_t)frame * r_packed_size(n),
                     z + (size_t)frame * n, resid ? resid + frame : nullptr, load ? load + frame : nullptr,
                     smem_qr + half * lds,
                     (int)threadIdx.x - half * tpf, tpf, live);
}

// Uneven batch: frames of different sizes pulled from a device work counter
// by a persistent grid sized for the largest frame.
__global__ void __launch_bounds__(CQ_MAX_THREADS) qr_uneven_kernel(const mimo_frame_desc* __restrict__ desc, int B,
                                                                   const float2* __restrict__ H,
                                                                   const float2* __restrict__ y,
                                                                   float* __restrict__ R, float* __restrict__ z,
                                                                   int* __restrict__ counter, int max_rx)
{
    extern __shared__ __align__(16) unsigned char smem_qr[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int f = next;
        __syncthreads();
        if (f >= B) break;
        const mimo_frame_desc d = desc[f];
        // the workgroup and its LDS are sized for n_tx <= n_rx <= max_rx
        if (d.n_tx < 1 || d.n_tx > d.n_rx || d.n_rx > max_rx) continue;
        cholqr_frame<0>(H + d.h_off, y + d.y_off, d.n_rx, d.n_tx, R + d.r_off, z + d.z_off, nullptr, nullptr, smem_qr,
                         (int)threadIdx.x, (int)blockDim.x, true);
    }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

// dynamic LDS beyond 64 KB (n_tx > 100) must be allowed per kernel
static int32_t cq_allow_lds(const void* kernel, size_t lds)
{
    if (lds <= 64 * 1024) return MIMO_OK;
    hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return fail(MIMO_ERR_HIP, "mimo_qr_preprocess: LDS attribute: %s", hipGetErrorString(e));
    return MIMO_OK;
}


}  // namespace mimo

namespace mimo {

static int32_t launch_qr(const char* who, const float* H, const float* y, const float* load, int32_t B, int32_t n_rx,
                         int32_t n_tx, float* R, float* z, float* resid, void* stream)
{
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", who);
    if (n_tx < 1 || n_rx < n_tx)
        return fail(MIMO_ERR_INVALID_ARG, "%s: need 1 <= n_tx <= n_rx (got %d, %d)", who, n_tx, n_rx);
    if (n_tx > MIMO_MAX_TX || n_rx > MIMO_MAX_RX)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: n_rx, n_tx <= %d", who, MIMO_MAX_RX);
    if (B == 0) return MIMO_OK;
    if (!H || !y || !R || !z) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", who);
    const int threads = cq_threads(n_tx);
    if (threads > CQ_MAX_THREADS) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx = %d", who, n_tx);
    const float2* H2 = reinterpret_cast<const float2*>(H);
    const float2* y2 = reinterpret_cast<const float2*>(y);
    const int waves = threads / WAVE;
    const int fpw = (waves >= 4 && waves <= 6) ? 2 : 1;
    const size_t lds = fpw * ((cq_lds_bytes(n_tx, cq_rows(n_tx, threads)) + 15) & ~(size_t)15);
    const int grid = (B + fpw - 1) / fpw;
    hipStream_t st = (hipStream_t)stream;
    // compile-time tile rows for 32, 64, 100 and 128 transmit antennas
    const int nb = cq_shape(n_tx).nb;
    auto kern = nb == 9    ? qr_kernel<9>
                : nb == 17 ? qr_kernel<17>
                : nb == 26 ? qr_kernel<26>
                : nb == 33 ? qr_kernel<33>
                           : qr_kernel<0>;
    if (int32_t rc = cq_allow_lds((const void*)kern, lds)) return rc;
    hipLaunchKernelGGL(kern, dim3(grid), dim3(fpw * threads), lds, st, H2, y2, n_rx, n_tx, R, z, resid, load, B,
                       fpw, threads);
    return check_launch(who);
}

}  // namespace mimo

extern "C" int32_t mimo_qr_preprocess(const float* H, const float* y, int32_t B, int32_t n_rx, int32_t n_tx,
                                      float* R, float* z, float* resid, void* stream)
{
    return mimo::launch_qr("mimo_qr_preprocess", H, y, nullptr, B, n_rx, n_tx, R, z, resid, stream);
}

extern "C" int32_t mimo_qr_preprocess_mmse(const float* H, const float* y, const float* sigma2, int32_t B,
                                           int32_t n_rx, int32_t n_tx, float* R, float* z, void* stream)
{
    if (B > 0 && !sigma2) return mimo::fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess_mmse: null sigma2");
    return mimo::launch_qr("mimo_qr_preprocess_mmse", H, y, sigma2, B, n_rx, n_tx, R, z, nullptr, stream);
}

extern "C" int32_t mimo_qr_preprocess_uneven(const mimo_frame_desc* desc, int32_t B, int32_t max_rx,
                                             const float* H_flat, const float* y_flat, float* R_flat, float* z_flat,
                                             int32_t* counter, int32_t grid, void* stream)
{
    using namespace mimo;
    if (B < 0 || grid < 0) return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess_uneven: B < 0 or grid < 0");
    if (max_rx < 1 || max_rx > MIMO_MAX_RX)
        return fail(MIMO_ERR_UNSUPPORTED, "mimo_qr_preprocess_uneven: 1 <= max_rx <= %d", MIMO_MAX_RX);
    if (B == 0) return MIMO_OK;
    if (!desc || !H_flat || !y_flat || !R_flat || !z_flat || !counter)
        return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess_uneven: null pointer");
    // n_tx <= n_rx <= max_rx: size the workgroup and LDS for n_tx = max_rx;
    // smaller frames use a prefix of the threads and stage fewer elements
    const int mt = max_rx < MIMO_MAX_TX ? max_rx : MIMO_MAX_TX;
    const int threads = cq_threads(mt);
    if (threads > CQ_MAX_THREADS) return fail(MIMO_ERR_UNSUPPORTED, "mimo_qr_preprocess_uneven: max_rx = %d", max_rx);
    size_t lds = 0;  // the largest need over the frame sizes the workgroup can meet
    for (int m = 1; m <= mt; ++m) {
        const size_t b = cq_lds_bytes(m, cq_rows(m, threads));
        lds = b > lds ? b : lds;
    }
    hipStream_t st = (hipStream_t)stream;
    if (grid == 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = 2 * (cus > 0 ? cus : 256);
    }
    if (grid > B) grid = B;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    const float2* H2 = reinterpret_cast<const float2*>(H_flat);
    const float2* y2 = reinterpret_cast<const float2*>(y_flat);
    if (int32_t rc = cq_allow_lds((const void*)qr_uneven_kernel, lds)) return rc;
    hipLaunchKernelGGL(qr_uneven_kernel, dim3(grid), dim3(threads), lds, st, desc, B, H2, y2, R_flat, z_flat, counter,
                       mt);
    return check_launch("mimo_qr_preprocess_uneven");
}
