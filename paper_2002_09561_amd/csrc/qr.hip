// QR preprocessing (Sec. III-B): H = Q R, z = Q^H y, emitted for the real
// model in packed level order.
//
// One workgroup per frame, one wave per chunk of QR_RB = 16 rows.  The
// N x (M+1) matrix [H | y] lives in registers: lane l of every wave owns the
// columns l, l + 64, ... (CB = ceil((M+1)/64) of them) for the rows of its
// wave's chunk.  Householder step k:
//   1. every wave broadcasts its rows of column k from the owner lane
//      (readlane: wave-uniform values) and publishes the chunk's partial
//      squared norm in LDS;
//   2. every thread forms the reflector v = x - alpha e1 with
//      alpha = -phase(x0) ||x|| (wave-uniform scalars);
//   3. phase 1: partial w_j = sum_i conj(v_i) A_ij over the chunk's rows;
//   4. phase 2: w_j = sum of the chunk partials, A_ij -= tau v_i w_j.
// Rows outside [k, N) carry v_i = 0, so the updates need no row guards.
// The complex QR maps onto the real model blockwise: with R_kk
// made real positive, the real R has R_2k,2k+1 = 0 and R_2k,2k = R_2k+1,2k+1.
#include "common.hpp"

namespace mimo {

constexpr int QR_RB = 16;  // rows per wave held in registers

struct c32 {
    float x, y;
};

__device__ inline c32 cmul(c32 a, c32 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }

// QR of one frame by the whole workgroup (rc = blockDim.x / 64 waves of
// QR_RB rows; waves beyond the frame's rows only take part in the barriers).
template <int CB>
__device__ __forceinline__ void qr_frame(const float2* __restrict__ Hf, const float2* __restrict__ yf, int N, int M,
                                         float* __restrict__ Rf, float* __restrict__ zf, float* __restrict__ resid_out,
                                         float* smem_qr)
{
    const int lane = threadIdx.x & 63;
    const int r = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);  // wave index = row chunk (uniform)
    const int rc = blockDim.x >> 6;
    const int rc_used = (N + QR_RB - 1) / QR_RB;
    const int row0 = r * QR_RB;
    const int ncol = CB * WAVE;
    const int n = 2 * M;

    // LDS: x0s[2] c32, wpart[rc][ncol] c32, alpha[M] c32, pnorm[2][rc] f32
    c32* x0s = reinterpret_cast<c32*>(smem_qr);
    c32* wpart = x0s + 2;
    c32* alpha_s = wpart + rc * ncol;
    float* pnorm = reinterpret_cast<float*>(alpha_s + M);

    c32 A[QR_RB][CB];
#pragma unroll
    for (int q = 0; q < QR_RB; ++q) {
        const int i = row0 + q;
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            const int j = lane + cb * WAVE;
            float2 v = make_float2(0.f, 0.f);
            if (i < N) {
                if (j < M) v = Hf[(size_t)i * M + j];
                else if (j == M) v = yf[i];
            }
            A[q][cb] = {v.x, v.y};
        }
    }

    for (int k = 0; k < M; ++k) {
        const int buf = k & 1;
        float* pn = pnorm + buf * rc;
        const int kcb = k / WAVE, klane = k % WAVE;
        // 1. column k of this wave's rows, broadcast from its owner lane
        //    (wave-uniform values), and the chunk's partial squared norm over
        //    rows >= k; the wave holding row k publishes x0 = A_kk
        c32 colk[QR_RB];
        float s = 0.f;
#pragma unroll
        for (int q = 0; q < QR_RB; ++q) {
            c32 x = A[q][0];
#pragma unroll
            for (int cb = 1; cb < CB; ++cb)
                if (cb == kcb) x = A[q][cb];
            colk[q].x = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x.x), klane));
            colk[q].y = __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, x.y), klane));
            const int i = row0 + q;
            if (i >= k && i < N) s = fmaf(colk[q].x, colk[q].x, fmaf(colk[q].y, colk[q].y, s));
        }
        if (lane == 0) {
            pn[r] = s;
#pragma unroll
            for (int q = 0; q < QR_RB; ++q)
                if (row0 + q == k) x0s[buf] = colk[q];
        }
        __syncthreads();
        if (row0 + QR_RB <= k || row0 >= N) {  // finished or empty chunk: only the barrier remains
            __syncthreads();
            continue;
        }
        // 2. reflector scalars (uniform)
        float norm2 = 0.f;
        for (int rr = 0; rr < rc; ++rr) norm2 += pn[rr];
        const c32 x0 = x0s[buf];
        const float ax0 = sqrtf(x0.x * x0.x + x0.y * x0.y);
        const float norm = sqrtf(norm2);
        const c32 ph = ax0 > 0.f ? c32{x0.x / ax0, x0.y / ax0} : c32{1.f, 0.f};
        const c32 alpha = {-ph.x * norm, -ph.y * norm};
        const c32 v0 = {x0.x - alpha.x, x0.y - alpha.y};
        const float vn2 = norm2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
        const float tau = (norm > 0.f && vn2 > 0.f) ? 2.f / vn2 : 0.f;
        // v_i of this chunk's rows: zero above row k and below row N-1, so the
        // updates below are exact no-ops there
        c32 vr[QR_RB];
#pragma unroll
        for (int q = 0; q < QR_RB; ++q) {
            const int i = row0 + q;
            vr[q] = (i > k && i < N) ? colk[q] : (i == k ? v0 : c32{0.f, 0.f});
        }
        // 3. phase 1: partial w_j = sum_i conj(v_i) A_ij over this chunk
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if ((cb + 1) * WAVE <= k || cb * WAVE > M) continue;  // block finished or beyond [H | y] (uniform)
            c32 sw = {0.f, 0.f};
#pragma unroll
            for (int q = 0; q < QR_RB; ++q) {
                sw.x = fmaf(vr[q].x, A[q][cb].x, sw.x);
                sw.x = fmaf(vr[q].y, A[q][cb].y, sw.x);
                sw.y = fmaf(vr[q].x, A[q][cb].y, sw.y);
                sw.y = fmaf(-vr[q].y, A[q][cb].x, sw.y);
            }
            wpart[r * ncol + lane + cb * WAVE] = sw;
        }
        __syncthreads();
        // 4. phase 2: apply the reflector.  Finished columns (j < k) have w_j = 0
        //    up to rounding of their (never used) sub-diagonal residue; the pivot
        //    column's new values below the diagonal are never read either: its
        //    diagonal is alpha, kept in alpha_s.
#pragma unroll
        for (int cb = 0; cb < CB; ++cb) {
            if ((cb + 1) * WAVE <= k || cb * WAVE > M) continue;
            const int j = lane + cb * WAVE;
            c32 wj = {0.f, 0.f};
            for (int rr = k / QR_RB; rr < rc_used; ++rr) {  // chunks with rows >= k wrote this step's partials
                const c32 t = wpart[rr * ncol + j];
                wj.x += t.x;
                wj.y += t.y;
            }
            wj.x *= tau;
            wj.y *= tau;
#pragma unroll
            for (int q = 0; q < QR_RB; ++q) {
                A[q][cb].x = fmaf(-vr[q].x, wj.x, A[q][cb].x);
                A[q][cb].x = fmaf(vr[q].y, wj.y, A[q][cb].x);
                A[q][cb].y = fmaf(-vr[q].x, wj.y, A[q][cb].y);
                A[q][cb].y = fmaf(-vr[q].y, wj.x, A[q][cb].y);
            }
        }
        if (lane == 0 && k >= row0 && k < row0 + QR_RB) alpha_s[k] = (tau > 0.f) ? alpha : x0;
    }
    __syncthreads();

    // make R_kk real positive: scale row i by d_i = conj(a_i) / |a_i|, then
    // write the real blocks [[a, -b], [b, a]] in packed level order
    float rs = 0.f;
#pragma unroll
    for (int q = 0; q < QR_RB; ++q) {
        const int i = row0 + q;
        if (i < M) {
            const c32 a = alpha_s[i];
            const float aa = sqrtf(a.x * a.x + a.y * a.y);
            const float inv = aa > 0.f ? 1.f / aa : 0.f;
            const c32 d = aa > 0.f ? c32{a.x * inv, -a.y * inv} : c32{1.f, 0.f};
            float* row_re = Rf + r_row_off(n, 2 * i);
            float* row_im = Rf + r_row_off(n, 2 * i + 1);
#pragma unroll
            for (int cb = 0; cb < CB; ++cb) {
                const int j = lane + cb * WAVE;
                if (j < i || j > M) continue;
                c32 v = cmul(d, A[q][cb]);
                if (j == i) v = {aa > 0.f ? aa : A[q][cb].x, 0.f};
                if (j == M) {
                    zf[2 * i] = v.x;
                    zf[2 * i + 1] = v.y;
                } else {
                    row_re[2 * (j - i)] = v.x;
                    row_re[2 * (j - i) + 1] = -v.y;
                    if (j > i) row_im[2 * (j - i) - 1] = v.y;
                    row_im[2 * (j - i)] = v.x;
                }
            }
        }
#pragma unroll
        for (int cb = 0; cb < CB; ++cb)
            if (i >= M && i < N && lane + cb * WAVE == M) rs += A[q][cb].x * A[q][cb].x + A[q][cb].y * A[q][cb].y;
    }
    if (resid_out) {
        // rows >= M of the rotated y: only the lanes owning column M contribute
        __syncthreads();
        float part = wave_sum(rs);
        if (lane == 0) pnorm[r] = part;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int rr = 0; rr < rc; ++rr) s += pnorm[rr];
            *resid_out = s;
        }
    }
    __syncthreads();  // the LDS may be reused by the next frame
}

template <int CB>
__global__ void __launch_bounds__(512, CB <= 2 ? 4 : 2) qr_kernel(const float2* __restrict__ H, const float2* __restrict__ y, int N,
                                                 int M, float* __restrict__ R, float* __restrict__ z,
                                                 float* __restrict__ resid)
{
    extern __shared__ float smem_qr[];
    const int frame = blockIdx.x;
    const int n = 2 * M;
    qr_frame<CB>(H + (size_t)frame * N * M, y + (size_t)frame * N, N, M, R + (size_t)frame * r_packed_size(n),
                 z + (size_t)frame * n, resid ? resid + frame : nullptr, smem_qr);
}

// Uneven batch: frames of different sizes pulled from a device work counter
// by a persistent grid; every workgroup has enough waves for the largest frame.
__global__ void __launch_bounds__(512, 2) qr_uneven_kernel(const mimo_frame_desc* __restrict__ desc, int B,
                                                           const float2* __restrict__ H, const float2* __restrict__ y,
                                                           float* __restrict__ R, float* __restrict__ z,
                                                           int* __restrict__ counter)
{
    extern __shared__ float smem_qr[];
    __shared__ int next;
    for (;;) {
        if (threadIdx.x == 0) next = atomicAdd(counter, 1);
        __syncthreads();
        const int f = next;
        __syncthreads();
        if (f >= B) break;
        const mimo_frame_desc d = desc[f];
        qr_frame<2>(H + d.h_off, y + d.y_off, d.n_rx, d.n_tx, R + d.r_off, z + d.z_off, nullptr, smem_qr);
    }
}

__global__ void reset_counter_kernel(int* counter) { *counter = 0; }

template <int CB>
static int32_t launch_qr(const float* H, const float* y, int B, int N, int M, float* R, float* z, float* resid,
                         hipStream_t st)
{
    const int rc = (N + QR_RB - 1) / QR_RB;
    const size_t lds = sizeof(c32) * (2 + rc * CB * WAVE + M) + sizeof(float) * (2 * rc);
    hipLaunchKernelGGL(qr_kernel<CB>, dim3(B), dim3(rc * WAVE), lds, st, reinterpret_cast<const float2*>(H),
                       reinterpret_cast<const float2*>(y), N, M, R, z, resid);
    return check_launch("mimo_qr_preprocess");
}

}  // namespace mimo

extern "C" int32_t mimo_qr_preprocess(const float* H, const float* y, int32_t B, int32_t n_rx, int32_t n_tx,
                                      float* R, float* z, float* resid, void* stream)
{
    using namespace mimo;
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: B < 0");
    if (n_tx < 1 || n_rx < n_tx)
        return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: need 1 <= n_tx <= n_rx (got %d, %d)", n_tx, n_rx);
    if (n_tx > MIMO_MAX_TX || n_rx > MIMO_MAX_RX)
        return fail(MIMO_ERR_UNSUPPORTED, "mimo_qr_preprocess: n_rx, n_tx <= %d", MIMO_MAX_RX);
    if (B == 0) return MIMO_OK;
    if (!H || !y || !R || !z) return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: null pointer");
    hipStream_t st = (hipStream_t)stream;
    const int cols = n_tx + 1;
    if (cols <= WAVE) return launch_qr<1>(H, y, B, n_rx, n_tx, R, z, resid, st);
    if (cols <= 2 * WAVE) return launch_qr<2>(H, y, B, n_rx, n_tx, R, z, resid, st);
    return launch_qr<3>(H, y, B, n_rx, n_tx, R, z, resid, st);
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
    hipStream_t st = (hipStream_t)stream;
    const int rc = (max_rx + QR_RB - 1) / QR_RB;
    const size_t lds = sizeof(c32) * (2 + rc * 2 * WAVE + MIMO_MAX_TX) + sizeof(float) * (2 * rc);
    if (grid == 0) {
        int dev = 0, cus = 0;
        hipGetDevice(&dev);
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = 2 * (cus > 0 ? cus : 256);
    }
    if (grid > B) grid = B;
    hipLaunchKernelGGL(reset_counter_kernel, dim3(1), dim3(1), 0, st, counter);
    hipLaunchKernelGGL(qr_uneven_kernel, dim3(grid), dim3(rc * WAVE), lds, st, desc, B,
                       reinterpret_cast<const float2*>(H_flat), reinterpret_cast<const float2*>(y_flat), R_flat,
                       z_flat, counter);
    return check_launch("mimo_qr_preprocess_uneven");
}
