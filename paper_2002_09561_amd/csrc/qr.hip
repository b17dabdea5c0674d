// QR preprocessing (Sec. III-B): H = Q R, z = Q^H y, emitted for the real
// model in packed level order.
//
// One workgroup per frame.  The N x (M+1) matrix [H | y] lives in registers:
// lane l of wave w owns column j = (w % ncg) * 64 + l and the rows of chunk
// r = w / ncg (32 rows per chunk).  Each Householder step k
//   1. the owners of column k publish it (and partial norms) in LDS,
//   2. every thread forms the reflector v = x - alpha e1 (alpha = -phase(x0) ||x||),
//   3. phase 1: partial w_j = sum_i conj(v_i) A_ij over the thread's rows,
//   4. phase 2: w_j = sum of the chunk partials, A_ij -= tau v_i w_j.
// The complex QR maps onto the real model blockwise: with R_kk made real
// and positive, the real R has R_2k,2k+1 = 0 and R_2k,2k = R_2k+1,2k+1.
#include "common.hpp"

namespace mimo {

constexpr int QR_CH = 32;  // rows per chunk held in registers

struct c32 {
    float x, y;
};

__device__ inline c32 cmul(c32 a, c32 b) { return {a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x}; }
__device__ inline c32 cmulc(c32 a, c32 b)  // conj(a) * b
{
    return {a.x * b.x + a.y * b.y, a.x * b.y - a.y * b.x};
}

__global__ void __launch_bounds__(768) qr_kernel(const float2* __restrict__ H, const float2* __restrict__ y,
                                                 int N, int M, int ncg, int rc, float* __restrict__ R,
                                                 float* __restrict__ z, float* __restrict__ resid)
{
    extern __shared__ float smem_qr[];
    const int frame = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int cg = w % ncg, r = w / ncg;
    const int j = cg * WAVE + lane;     // owned column (j == M is y)
    const int row0 = r * QR_CH;
    const int ncol = ncg * WAVE;
    const int n = 2 * M;

    // LDS: colv[2][N] c32, wpart[rc][ncol] c32, pnorm[2][rc] f32, alpha[M] c32
    c32* colv = reinterpret_cast<c32*>(smem_qr);
    c32* wpart = colv + 2 * N;
    float* pnorm = reinterpret_cast<float*>(wpart + rc * ncol);
    c32* alpha_s = reinterpret_cast<c32*>(pnorm + 2 * rc + (2 * rc) % 2);

    const float2* Hf = H + (size_t)frame * N * M;
    const float2* yf = y + (size_t)frame * N;

    c32 A[QR_CH];
#pragma unroll
    for (int q = 0; q < QR_CH; ++q) {
        const int i = row0 + q;
        float2 v = make_float2(0.f, 0.f);
        if (i < N) {
            if (j < M) v = Hf[(size_t)i * M + j];
            else if (j == M) v = yf[i];
        }
        A[q] = {v.x, v.y};
    }

    for (int k = 0; k < M; ++k) {
        const int buf = k & 1;
        c32* cv = colv + buf * N;
        float* pn = pnorm + buf * rc;
        // 1. publish column k and the chunk's partial norm
        if (j == k) {
            float s = 0.f;
#pragma unroll
            for (int q = 0; q < QR_CH; ++q) {
                const int i = row0 + q;
                if (i >= k && i < N) {
                    cv[i] = A[q];
                    s += A[q].x * A[q].x + A[q].y * A[q].y;
                }
            }
            pn[r] = s;
        }
        __syncthreads();
        // 2. reflector scalars (uniform)
        float norm2 = 0.f;
        for (int rr = 0; rr < rc; ++rr) norm2 += pn[rr];
        const c32 x0 = cv[k];
        const float ax0 = sqrtf(x0.x * x0.x + x0.y * x0.y);
        const float norm = sqrtf(norm2);
        c32 ph = ax0 > 0.f ? c32{x0.x / ax0, x0.y / ax0} : c32{1.f, 0.f};
        const c32 alpha = {-ph.x * norm, -ph.y * norm};
        const c32 v0 = {x0.x - alpha.x, x0.y - alpha.y};
        const float vn2 = norm2 - ax0 * ax0 + (v0.x * v0.x + v0.y * v0.y);
        const float tau = (norm > 0.f && vn2 > 0.f) ? 2.f / vn2 : 0.f;
        // 3. phase 1: partial w_j over this chunk
        const bool active = (j > k) && (j <= M);
        if (active) {
            c32 s = {0.f, 0.f};
#pragma unroll
            for (int q = 0; q < QR_CH; ++q) {
                const int i = row0 + q;
                if (i >= k && i < N) {
                    const c32 vi = (i == k) ? v0 : cv[i];
                    const c32 t = cmulc(vi, A[q]);
                    s.x += t.x;
                    s.y += t.y;
                }
            }
            wpart[r * ncol + j] = s;
        }
        __syncthreads();
        // 4. phase 2: apply the reflector
        if (active) {
            c32 wj = {0.f, 0.f};
            for (int rr = 0; rr < rc; ++rr) {
                wj.x += wpart[rr * ncol + j].x;
                wj.y += wpart[rr * ncol + j].y;
            }
            wj.x *= tau;
            wj.y *= tau;
#pragma unroll
            for (int q = 0; q < QR_CH; ++q) {
                const int i = row0 + q;
                if (i >= k && i < N) {
                    const c32 vi = (i == k) ? v0 : cv[i];
                    const c32 t = cmul(vi, wj);
                    A[q].x -= t.x;
                    A[q].y -= t.y;
                }
            }
        } else if (j == k) {
#pragma unroll
            for (int q = 0; q < QR_CH; ++q) {
                const int i = row0 + q;
                if (i == k) {
                    A[q] = (tau > 0.f) ? alpha : x0;
                    alpha_s[k] = A[q];
                } else if (i > k && i < N && tau > 0.f) {
                    A[q] = {0.f, 0.f};
                }
            }
        }
    }
    __syncthreads();

    // make R_kk real positive: scale row k by d_k = conj(a_k) / |a_k|, then
    // write the real blocks [[a, -b], [b, a]] in packed level order
    float* Rf = R + (size_t)frame * r_packed_size(n);
    float* zf = z + (size_t)frame * n;
    float rs = 0.f;
#pragma unroll
    for (int q = 0; q < QR_CH; ++q) {
        const int i = row0 + q;
        if (i < M && j >= i && j <= M) {
            const c32 a = alpha_s[i];
            const float aa = sqrtf(a.x * a.x + a.y * a.y);
            const c32 d = aa > 0.f ? c32{a.x / aa, -a.y / aa} : c32{1.f, 0.f};
            c32 v = cmul(d, A[q]);
            if (j == i) v = {aa > 0.f ? aa : A[q].x, 0.f};
            if (j == M) {
                zf[2 * i] = v.x;
                zf[2 * i + 1] = v.y;
            } else {
                const int re = 2 * i, im = 2 * i + 1;
                float* row_re = Rf + r_row_off(n, re);
                float* row_im = Rf + r_row_off(n, im);
                row_re[2 * j - re] = v.x;
                row_re[2 * j + 1 - re] = -v.y;
                if (j > i) row_im[2 * j - im] = v.y;
                row_im[2 * j + 1 - im] = v.x;
            }
        }
        if (i >= M && i < N && j == M) rs += A[q].x * A[q].x + A[q].y * A[q].y;
    }
    if (resid) {
        // rows >= M of the rotated y: only the threads owning column M contribute
        float* red = pnorm;  // reuse: rc floats
        __syncthreads();
        if (j == M) red[r] = rs;
        __syncthreads();
        if (threadIdx.x == 0) {
            float s = 0.f;
            for (int rr = 0; rr < rc; ++rr) s += red[rr];
            resid[frame] = s;
        }
    }
}

}  // namespace mimo

extern "C" int32_t mimo_qr_preprocess(const float* H, const float* y, int32_t B, int32_t n_rx,
                                      int32_t n_tx, float* R, float* z, float* resid, void* stream)
{
    using namespace mimo;
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: B < 0");
    if (n_tx < 1 || n_rx < n_tx)
        return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: need 1 <= n_tx <= n_rx (got %d, %d)", n_tx, n_rx);
    if (n_tx > MIMO_MAX_TX || n_rx > MIMO_MAX_RX)
        return fail(MIMO_ERR_UNSUPPORTED, "mimo_qr_preprocess: n_rx, n_tx <= %d", MIMO_MAX_RX);
    if (B == 0) return MIMO_OK;
    if (!H || !y || !R || !z) return fail(MIMO_ERR_INVALID_ARG, "mimo_qr_preprocess: null pointer");
    const int ncg = (n_tx + 1 + WAVE - 1) / WAVE;
    const int rc = (n_rx + QR_CH - 1) / QR_CH;
    const int threads = ncg * rc * WAVE;
    const size_t lds = sizeof(c32) * (2 * n_rx + rc * ncg * WAVE + n_tx) + sizeof(float) * (2 * rc + 2);
    hipLaunchKernelGGL(qr_kernel, dim3(B), dim3(threads), lds, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(H), reinterpret_cast<const float2*>(y), n_rx, n_tx, ncg,
                       rc, R, z, resid);
    return check_launch("mimo_qr_preprocess");
}
