// Epilogues of the detection path: FP64 metric ||y - H s||^2 (the Eq. (2)
// objective), Gray bit / symbol error counts, and the per-level state of the
// successive-cancellation path used by the learned survivor count.
#include "common.hpp"

namespace mimo {

__device__ inline double amp_d(int P, int i)
{
    return (double)(2 * i - (P - 1)) * sqrt(3.0 / (2.0 * (double)(P * P - 1)));
}

__device__ __forceinline__ double xor_lanes_f64(double v, int m, int lane)
{
    return __builtin_bit_cast(double, xor_lanes_u64(__builtin_bit_cast(uint64_t, v), m, lane));
}

// One wave per frame, four rows of H at a time: the 16 lanes of a row group
// run along the row, two adjacent columns per 16-byte load (coalesced
// 256-byte segments; with an odd n_tx the rows are not 16-byte aligned and
// the columns are loaded one by one), up to 8 columns per lane,
// the row's residual y_i - sum_j h_ij s_j is reduced over those 16 lanes in
// FP64 in a fixed order (DPP exchanges only), and each group accumulates
// |residual|^2 over its rows; the four group sums are added at the end.
// row groups (of four rows) per loop step: one keeps the kernel at 56
// registers, so that six of its waves still fit on a SIMD beside one wave of
// the K = 64 fallback (176 registers) that runs at the same time
constexpr int MU = 1;
__global__ void __launch_bounds__(256) metric_kernel(const float2* __restrict__ H, const float2* __restrict__ y,
                                                     const int32_t* __restrict__ sym, int B, int N, int M, int P,
                                                     const uint32_t* __restrict__ flags, uint32_t mask,
                                                     uint32_t value, double* __restrict__ out)
{
    const int lane = threadIdx.x & 63;
    const int g = lane >> 4, l = lane & 15;
    const int f = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
    if (f >= B) return;
    if (flags && (flags[f] & mask) != value) return;  // frame not selected (uniform per wave)
    // lane l holds columns 2l + 32c and 2l + 1 + 32c; a row of an even-M frame is 16-byte aligned
    constexpr int CPL = (MIMO_MAX_TX + 31) / 32;
    const bool v4 = (M & 1) == 0;
    double sr[2 * CPL], si[2 * CPL];
#pragma unroll
    for (int c = 0; c < 2 * CPL; ++c) {
        const int j = 2 * l + 32 * (c >> 1) + (c & 1);
        sr[c] = si[c] = 0.0;
        if (j < M) {
            const int q = sym[(size_t)f * M + j];
            sr[c] = amp_d(P, q / P);
            si[c] = amp_d(P, q % P);
        }
    }
    const float2* Hf = H + (size_t)f * N * M;
    const float2* yf = y + (size_t)f * N;
    double acc = 0.0;
    for (int i0 = 0; i0 < N; i0 += 4 * MU) {
        double pr[MU], pi[MU];
#pragma unroll
        for (int u = 0; u < MU; ++u) pr[u] = pi[u] = 0.0;
#pragma unroll
        for (int u = 0; u < MU; ++u) {
            const int i = i0 + 4 * u + g;
#pragma unroll
            for (int c = 0; c < CPL; ++c) {
                const int j = 2 * l + 32 * c;
                if (i < N && j < M) {
                    float2 h0, h1;
                    if (v4) {
                        const float4 hh = *reinterpret_cast<const float4*>(Hf + (size_t)i * M + j);
                        h0 = make_float2(hh.x, hh.y);
                        h1 = make_float2(hh.z, hh.w);
                    } else {
                        h0 = Hf[(size_t)i * M + j];
                        h1 = j + 1 < M ? Hf[(size_t)i * M + j + 1] : make_float2(0.f, 0.f);
                    }
                    pr[u] += (double)h0.x * sr[2 * c] - (double)h0.y * si[2 * c];
                    pi[u] += (double)h0.x * si[2 * c] + (double)h0.y * sr[2 * c];
                    pr[u] += (double)h1.x * sr[2 * c + 1] - (double)h1.y * si[2 * c + 1];
                    pi[u] += (double)h1.x * si[2 * c + 1] + (double)h1.y * sr[2 * c + 1];
                }
            }
        }
#pragma unroll
        for (int m = 8; m >= 1; m >>= 1) {
#pragma unroll
            for (int u = 0; u < MU; ++u) {
                pr[u] += xor_lanes_f64(pr[u], m, lane);
                pi[u] += xor_lanes_f64(pi[u], m, lane);
            }
        }
#pragma unroll
        for (int u = 0; u < MU; ++u) {
            const int i = i0 + 4 * u + g;
            if (i < N) {
                const float2 yy = yf[i];
                const double er = (double)yy.x - pr[u], ei = (double)yy.y - pi[u];
                acc += er * er + ei * ei;
            }
        }
    }
    acc += xor_lanes_f64(acc, 16, lane);
    acc += xor_lanes_f64(acc, 32, lane);
    if (lane == 0) out[f] = acc;
}

// one wave per frame
__global__ void __launch_bounds__(256) errors_kernel(const int32_t* __restrict__ sym, const int32_t* __restrict__ ref,
                                                     int B, int M, int P, unsigned long long* __restrict__ counts)
{
    const int lane = threadIdx.x & 63;
    const int f = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
    if (f >= B) return;
    unsigned bits = 0, syms = 0;
    for (int m = lane; m < M; m += WAVE) {
        const int a = sym[(size_t)f * M + m], b = ref[(size_t)f * M + m];
        const int ar = a / P, ai = a % P, br = b / P, bi = b % P;
        const unsigned ga = (unsigned)(((ar ^ (ar >> 1)) * P) | (ai ^ (ai >> 1)));
        const unsigned gb = (unsigned)(((br ^ (br >> 1)) * P) | (bi ^ (bi >> 1)));
        bits += __popc(ga ^ gb);
        syms += (a != b);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        bits += __shfl_xor(bits, m, WAVE);
        syms += __shfl_xor(syms, m, WAVE);
    }
    if (lane == 0 && syms) {
        atomicAdd(&counts[0], (unsigned long long)bits);
        atomicAdd(&counts[1], (unsigned long long)syms);
        atomicAdd(&counts[2], 1ull);
    }
}

// Per-level state of the K = 1 (successive-cancellation) path.  Level k:
// centre b = z_k - sum_{j>k} R_kj x_j, nearest PAM point a, path metric
// pd += (b - R_kk a)^2; the features are k/n, the centre's distance to the
// nearest decision boundary in units of the spacing, log2(R_kk 2c / sigma_r)
// and pd / ((n - k) sigma_r^2).
//
// Four frames per wave, 16 lanes per frame: lane l of a frame holds the
// decided amplitudes x_j of the levels j = l + 16 i in registers and loads
// the matching entries R_kj of each row (coalesced 64-byte segments), so the
// centre is SL register FMAs and a 16-lane reduction (DPP).  Six row
// buffers keep the loads of the next five or six levels in flight while the
// current one is used (the kernel waits on memory latency, not on issue).
// SL levels per lane (16 SL >= n): 13 for up to 208 levels, else 16.
//
// Row k of the frame through a buffer resource that spans the wave's four
// frames: lane l's slot i holds R_k,l+16i, read at byte offset
// 4 (fbase + row_off(k) - k + l) + 64 i (the slot's part is the load's
// immediate offset).  Slots whose levels all lie at or left of the diagonal
// are not loaded (a uniform branch).  A loaded lane whose level is not in
// row k (j <= k or j >= n) reads another row or frame of the same buffer, or
// nothing (an offset outside the buffer reads 0), and a slot not loaded keeps
// an earlier row's values: either way its level has amplitude 0 (not yet
// decided, or beyond n), and the centre drops such entries outright (a
// select, not a product with 0), so a non-finite R in a neighbouring frame
// cannot reach this frame.
template <int SL>
__device__ __forceinline__ void feat_load(__amdgpu_buffer_rsrc_t rs, int fbase, const float* __restrict__ zf, int n,
                                          int k, int l, float (&r)[SL], float& rkk, float& zk)
{
    if (k < 0) return;
    const int row = fbase + (int)r_row_off(n, k);  // float index of R_kk in the buffer
    const int v = 4 * (row - k + l);               // may be negative: then out of range
#pragma unroll
    for (int i = 0; i < SL; ++i)
        if (16 * i + 15 > k && 16 * i < n)
            r[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, v + 64 * i, 0, 0));
    rkk = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, 4 * row, 0, 0));
    zk = zf[k];
}

template <int SL>
__device__ __forceinline__ void feat_level(int k, int n, int P, float c, float rc, float lc, float rs2, int lane,
                                           const float (&r)[SL], float rkk, float zk,
                                           float (&xr)[SL], float& pd, float* __restrict__ featf, bool live)
{
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < SL; ++i) acc = fmaf(xr[i] != 0.f ? r[i] : 0.f, xr[i], acc);
#pragma unroll
    for (int m = 8; m >= 1; m >>= 1) acc += shfl_xor_f(acc, m);
    const float b = zk - acc;
    const float u = b / rkk;
    const float v = u * rc;  // u / c
    int i = (int)floorf((v + (float)(P - 1)) * 0.5f + 0.5f);
    i = i < 0 ? 0 : (i > P - 1 ? P - 1 : i);
    const float a = (float)(2 * i - (P - 1)) * c;
    const float e = fmaf(-rkk, a, b);
    pd = fmaf(e, e, pd);
    float nb = 2.f * floorf(v * 0.5f + 0.5f);
    nb = fminf(fmaxf(nb, -(float)(P - 2)), (float)(P - 2));
    const int l = lane & 15;
    if (l == 0 && live)
        *reinterpret_cast<float4*>(featf + (size_t)k * 4) =
            make_float4((float)k / (float)n, fabsf(v - nb) * 0.5f, log2f(rkk) + lc, pd * rs2 / (float)(n - k));
    // level k's decision goes to lane k mod 16, slot k / 16 (uniform index)
    const int slot = k >> 4;
    const float cur = xr[slot];
    xr[slot] = l == (k & 15) ? a : cur;
}

template <int SL>
__global__ void __launch_bounds__(256) features_kernel(const float* __restrict__ R, const float* __restrict__ z,
                                                       const float* __restrict__ sigma2, int B, int n, int P,
                                                       float* __restrict__ feat)
{
    const int lane = threadIdx.x & 63, l = lane & 15;
    const int f0 = __builtin_amdgcn_readfirstlane((blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6)) * 4);
    const int fr = f0 + (lane >> 4);
    if (f0 >= B) return;  // whole wave beyond the batch
    const bool live = fr < B;
    const int f = live ? fr : B - 1;  // a slot beyond the batch repeats the last frame, storing nothing
    // the wave's frames f0 .. f0 + 3 (fewer at the end of the batch) as one buffer
    const int size = (int)r_packed_size(n);
    const int nf = B - f0 < 4 ? B - f0 : 4;
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(R + (size_t)f0 * size), 0, nf * size * (int)sizeof(float), 0x00020000);
    const int fbase = (f - f0) * size;
    const float* zf = z + (size_t)f * n;
    float* featf = feat + (size_t)f * n * 4;
    const float c = pam_scale(P);
    const float s2r = sigma2[f] * 0.5f;  // sigma_r^2
    const float lc = log2f(2.f * c / sqrtf(s2r));
    const float rs2 = 1.f / s2r;
    const float rc = 1.f / c;
    float xr[SL];
#pragma unroll
    for (int i = 0; i < SL; ++i) xr[i] = 0.f;
    float pd = 0.f;
    float ra[SL], rb[SL], rc4[SL], rd[SL], re[SL], rf[SL];
    float rka = 0.f, rkb = 0.f, rkc = 0.f, rkd = 0.f, rke = 0.f, rkf = 0.f;
    float za = 0.f, zb = 0.f, zc = 0.f, zd = 0.f, ze = 0.f, zf6 = 0.f;
#pragma unroll
    for (int i = 0; i < SL; ++i) ra[i] = rb[i] = rc4[i] = rd[i] = re[i] = rf[i] = 0.f;
    feat_load<SL>(rs, fbase, zf, n, n - 1, l, ra, rka, za);
    feat_load<SL>(rs, fbase, zf, n, n - 2, l, rb, rkb, zb);
    feat_load<SL>(rs, fbase, zf, n, n - 3, l, rc4, rkc, zc);
    feat_load<SL>(rs, fbase, zf, n, n - 4, l, rd, rkd, zd);
    feat_load<SL>(rs, fbase, zf, n, n - 5, l, re, rke, ze);
    feat_load<SL>(rs, fbase, zf, n, n - 6, l, rf, rkf, zf6);
    int k = n - 1;
    for (; k >= 5; k -= 6) {
        feat_level<SL>(k, n, P, c, rc, lc, rs2, lane, ra, rka, za, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 6, l, ra, rka, za);
        feat_level<SL>(k - 1, n, P, c, rc, lc, rs2, lane, rb, rkb, zb, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 7, l, rb, rkb, zb);
        feat_level<SL>(k - 2, n, P, c, rc, lc, rs2, lane, rc4, rkc, zc, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 8, l, rc4, rkc, zc);
        feat_level<SL>(k - 3, n, P, c, rc, lc, rs2, lane, rd, rkd, zd, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 9, l, rd, rkd, zd);
        feat_level<SL>(k - 4, n, P, c, rc, lc, rs2, lane, re, rke, ze, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 10, l, re, rke, ze);
        feat_level<SL>(k - 5, n, P, c, rc, lc, rs2, lane, rf, rkf, zf6, xr, pd, featf, live);
        feat_load<SL>(rs, fbase, zf, n, k - 11, l, rf, rkf, zf6);
    }
    // n is even: 0, 2 or 4 levels remain, in buffers a, b, c, d
    if (k >= 0) feat_level<SL>(k, n, P, c, rc, lc, rs2, lane, ra, rka, za, xr, pd, featf, live);
    if (k >= 1) feat_level<SL>(k - 1, n, P, c, rc, lc, rs2, lane, rb, rkb, zb, xr, pd, featf, live);
    if (k >= 2) feat_level<SL>(k - 2, n, P, c, rc, lc, rs2, lane, rc4, rkc, zc, xr, pd, featf, live);
    if (k >= 3) feat_level<SL>(k - 3, n, P, c, rc, lc, rs2, lane, rd, rkd, zd, xr, pd, featf, live);
}

}  // namespace mimo

namespace mimo {

static int32_t launch_metric(const char* who, const float* H, const float* y, const int32_t* sym, int32_t B,
                             int32_t n_rx, int32_t n_tx, int32_t pam, const uint32_t* flags, uint32_t mask,
                             uint32_t value, double* metric, void* stream)
{
    if (B < 0 || n_tx < 1 || n_rx < n_tx) return fail(MIMO_ERR_INVALID_ARG, "%s: bad sizes", who);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", who);
    if (n_rx > MIMO_MAX_RX || n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: size limit", who);
    if (B == 0) return MIMO_OK;
    if (!H || !y || !sym || !metric) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", who);
    hipLaunchKernelGGL(metric_kernel, dim3((B + 3) / 4), dim3(256), 0, (hipStream_t)stream,
                       reinterpret_cast<const float2*>(H), reinterpret_cast<const float2*>(y), sym, B, n_rx, n_tx,
                       pam, flags, mask, value, metric);
    return check_launch(who);
}

}  // namespace mimo

extern "C" int32_t mimo_metric(const float* H, const float* y, const int32_t* sym, int32_t B, int32_t n_rx,
                               int32_t n_tx, int32_t pam, double* metric, void* stream)
{
    return mimo::launch_metric("mimo_metric", H, y, sym, B, n_rx, n_tx, pam, nullptr, 0u, 0u, metric, stream);
}

extern "C" int32_t mimo_metric_select(const float* H, const float* y, const int32_t* sym, const uint32_t* flags,
                                      uint32_t mask, uint32_t value, int32_t B, int32_t n_rx, int32_t n_tx,
                                      int32_t pam, double* metric, void* stream)
{
    if (B > 0 && !flags) return mimo::fail(MIMO_ERR_INVALID_ARG, "mimo_metric_select: null flags");
    return mimo::launch_metric("mimo_metric_select", H, y, sym, B, n_rx, n_tx, pam, flags, mask, value, metric,
                               stream);
}

extern "C" int32_t mimo_error_count(const int32_t* sym, const int32_t* ref, int32_t B, int32_t n_tx, int32_t pam,
                                    uint64_t* counts, void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "mimo_error_count: bad sizes");
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "mimo_error_count: bad pam");
    if (B == 0) return MIMO_OK;
    if (!sym || !ref || !counts) return fail(MIMO_ERR_INVALID_ARG, "mimo_error_count: null pointer");
    hipLaunchKernelGGL(errors_kernel, dim3((B + 3) / 4), dim3(256), 0, (hipStream_t)stream, sym, ref, B, n_tx, pam,
                       reinterpret_cast<unsigned long long*>(counts));
    return check_launch("mimo_error_count");
}

extern "C" int32_t prune_features(const float* R, const float* z, const float* sigma2, int32_t B, int32_t n_tx,
                                  int32_t pam, float* feat, void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "prune_features: bad sizes");
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "prune_features: bad pam");
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "prune_features: n_tx > %d", MIMO_MAX_TX);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sigma2 || !feat) return fail(MIMO_ERR_INVALID_ARG, "prune_features: null pointer");
    if (2 * n_tx <= 208)
        hipLaunchKernelGGL(features_kernel<13>, dim3((B + 15) / 16), dim3(256), 0, (hipStream_t)stream, R, z, sigma2,
                           B, 2 * n_tx, pam, feat);
    else
        hipLaunchKernelGGL(features_kernel<16>, dim3((B + 15) / 16), dim3(256), 0, (hipStream_t)stream, R, z, sigma2,
                           B, 2 * n_tx, pam, feat);
    return check_launch("prune_features");
}
