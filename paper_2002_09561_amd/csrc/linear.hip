// Linear baselines the paper compares the sphere decoder against (Sec. III-A):
// zero forcing and linear MMSE by back-substitution on (R, z) without
// decision feedback (R, z from the plain or the MMSE QR), and maximum-ratio
// combining on (H, y).
#include "common.hpp"

namespace mimo {

constexpr int LIN_RPL = 4;  // row entries per lane: n <= 256

__device__ __forceinline__ void lin_load(const float* __restrict__ Rf, const float* __restrict__ zf, int n, int k,
                                         int lane, float (&r)[LIN_RPL], float& zk)
{
    if (k < 0) return;
    const float* rk = Rf + r_row_off(n, k);
#pragma unroll
    for (int i = 0; i < LIN_RPL; ++i) {
        const int t = lane + WAVE * i;
        r[i] = t < n - k ? rk[t] : 0.f;
    }
    zk = zf[k];
}

// u_k = (z_k - sum_{t>0} R_k,k+t u_{k+t}) / R_kk for one level; the sum is
// split over the lanes and reduced in a fixed order
__device__ __forceinline__ void lin_level(int k, int n, int lane, const float (&r)[LIN_RPL], float zk, float* ua)
{
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < LIN_RPL; ++i) {
        const int t = lane + WAVE * i;
        if (t >= 1 && t < n - k) acc = fmaf(r[i], ua[k + t], acc);
    }
    acc = wave_sum(acc);
    const float rkk = __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, r[0])));
    if (lane == 0) ua[k] = (zk - acc) / rkk;
    __syncthreads();  // ua[k] visible to the wave
}

__device__ __forceinline__ int lin_slice_f(float u, float c, int P)
{
    int i = (int)floorf((u / c + (float)(P - 1)) * 0.5f + 0.5f);
    return i < 0 ? 0 : (i > P - 1 ? P - 1 : i);
}

// One wave per frame, FP32 with FP32 accumulation; the R rows of the next
// two levels are loaded while the current one is used.
__global__ void __launch_bounds__(64) linear_kernel(const float* __restrict__ R, const float* __restrict__ z, int n,
                                                    int P, int32_t* __restrict__ sym, float* __restrict__ xhat)
{
    __shared__ float ua[256];
    const int f = blockIdx.x, lane = threadIdx.x;
    const float* Rf = R + (size_t)f * r_packed_size(n);
    const float* zf = z + (size_t)f * n;
    float ra[LIN_RPL], rb[LIN_RPL], za = 0.f, zb = 0.f;
    lin_load(Rf, zf, n, n - 1, lane, ra, za);
    lin_load(Rf, zf, n, n - 2, lane, rb, zb);
    // n = 2 n_tx is even: levels go in pairs (k, k-1) from buffers a and b
    for (int k = n - 1; k >= 1; k -= 2) {
        float rc[LIN_RPL], zc = za;
#pragma unroll
        for (int i = 0; i < LIN_RPL; ++i) rc[i] = ra[i];
        lin_load(Rf, zf, n, k - 2, lane, ra, za);
        lin_level(k, n, lane, rc, zc, ua);
#pragma unroll
        for (int i = 0; i < LIN_RPL; ++i) rc[i] = rb[i];
        zc = zb;
        lin_load(Rf, zf, n, k - 3, lane, rb, zb);
        lin_level(k - 1, n, lane, rc, zc, ua);
    }
    const float c = pam_scale(P);
    const int M = n / 2;
    for (int m = lane; m < M; m += WAVE) {
        const float ur = ua[2 * m], ui = ua[2 * m + 1];  // levels 2m (real part) and 2m + 1 (imaginary part)
        sym[(size_t)f * M + m] = lin_slice_f(ur, c, P) * P + lin_slice_f(ui, c, P);
        if (xhat) {
            xhat[(size_t)f * n + 2 * m] = ur;
            xhat[(size_t)f * n + 2 * m + 1] = ui;
        }
    }
}

// One wave per frame: lanes along the columns of H (coalesced row reads),
// ||h_j||^2 and conj(h_j) y accumulated over the rows in FP64, then
// u_j = conj(h_j) y / ||h_j||^2 sliced per real and imaginary part in FP64.
__global__ void __launch_bounds__(256) mrc_kernel(const float2* __restrict__ H, const float2* __restrict__ y, int B,
                                                  int N, int M, int P, int32_t* __restrict__ sym,
                                                  float* __restrict__ xhat)
{
    const int lane = threadIdx.x & 63;
    const int f = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
    if (f >= B) return;
    constexpr int CPL = (MIMO_MAX_TX + WAVE - 1) / WAVE;  // columns per lane
    double nr[CPL], cr[CPL], ci[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) nr[c] = cr[c] = ci[c] = 0.0;
    const float2* Hf = H + (size_t)f * N * M;
    const float2* yf = y + (size_t)f * N;
    for (int i = 0; i < N; ++i) {
        const float2 yi = yf[i];
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            const int j = lane + WAVE * c;
            if (j < M) {
                const float2 h = Hf[(size_t)i * M + j];
                const double hr = h.x, hi = h.y;
                nr[c] += hr * hr + hi * hi;
                cr[c] += hr * (double)yi.x + hi * (double)yi.y;
                ci[c] += hr * (double)yi.y - hi * (double)yi.x;
            }
        }
    }
    const double cs = sqrt(3.0 / (2.0 * (double)(P * P - 1)));
#pragma unroll
    for (int c = 0; c < CPL; ++c) {
        const int j = lane + WAVE * c;
        if (j >= M) continue;
        const double ur = nr[c] > 0.0 ? cr[c] / nr[c] : 0.0;
        const double ui = nr[c] > 0.0 ? ci[c] / nr[c] : 0.0;
        int ir = (int)floor((ur / cs + (double)(P - 1)) / 2.0 + 0.5);
        int ii = (int)floor((ui / cs + (double)(P - 1)) / 2.0 + 0.5);
        ir = ir < 0 ? 0 : (ir > P - 1 ? P - 1 : ir);
        ii = ii < 0 ? 0 : (ii > P - 1 ? P - 1 : ii);
        sym[(size_t)f * M + j] = ir * P + ii;
        if (xhat) {
            xhat[(size_t)f * 2 * M + 2 * j] = (float)ur;
            xhat[(size_t)f * 2 * M + 2 * j + 1] = (float)ui;
        }
    }
}

// The paper's radius rule (Sec. III-B, squared): r2 = N M sigma2 per frame,
// M times the expected noise energy N sigma2 of a receive vector.
__global__ void __launch_bounds__(256) paper_radius_kernel(const float* __restrict__ sigma2, int B, float nm,
                                                           float* __restrict__ radius2)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f < B) radius2[f] = nm * sigma2[f];
}

}  // namespace mimo

extern "C" int32_t mimo_paper_radius2(const float* sigma2, int32_t B, int32_t n_rx, int32_t n_tx, float* radius2,
                                      void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1 || n_rx < n_tx) return fail(MIMO_ERR_INVALID_ARG, "mimo_paper_radius2: bad sizes");
    if (n_tx > MIMO_MAX_TX || n_rx > MIMO_MAX_RX) return fail(MIMO_ERR_UNSUPPORTED, "mimo_paper_radius2: size limit");
    if (B == 0) return MIMO_OK;
    if (!sigma2 || !radius2) return fail(MIMO_ERR_INVALID_ARG, "mimo_paper_radius2: null pointer");
    hipLaunchKernelGGL(paper_radius_kernel, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream, sigma2, B,
                       (float)(n_rx * n_tx), radius2);
    return check_launch("mimo_paper_radius2");
}

extern "C" int32_t linear_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam, int32_t* sym,
                                 float* xhat, void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "linear_detect: bad sizes");
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "linear_detect: pam must be 2, 4 or 8");
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "linear_detect: n_tx > %d", MIMO_MAX_TX);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym) return fail(MIMO_ERR_INVALID_ARG, "linear_detect: null pointer");
    hipLaunchKernelGGL(linear_kernel, dim3(B), dim3(WAVE), 0, (hipStream_t)stream, R, z, 2 * n_tx, pam, sym, xhat);
    return check_launch("linear_detect");
}

extern "C" int32_t mrc_detect(const float* H, const float* y, int32_t B, int32_t n_rx, int32_t n_tx, int32_t pam,
                              int32_t* sym, float* xhat, void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1 || n_rx < 1) return fail(MIMO_ERR_INVALID_ARG, "mrc_detect: bad sizes");
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "mrc_detect: pam must be 2, 4 or 8");
    if (n_tx > MIMO_MAX_TX || n_rx > MIMO_MAX_RX) return fail(MIMO_ERR_UNSUPPORTED, "mrc_detect: size limit");
    if (B == 0) return MIMO_OK;
    if (!H || !y || !sym) return fail(MIMO_ERR_INVALID_ARG, "mrc_detect: null pointer");
    hipLaunchKernelGGL(mrc_kernel, dim3((B + 3) / 4), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(H), reinterpret_cast<const float2*>(y), B, n_rx, n_tx, pam,
                       sym, xhat);
    return check_launch("mrc_detect");
}
