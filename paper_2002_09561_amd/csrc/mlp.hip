// Learned survivor count: MLP 4 -> 128 -> 128 -> 1 (ReLU), its pinball-loss
// backward pass and an Adam step.
//
// Inference (forward and schedule) runs on the matrix cores, 16 states per
// wavefront and step, in the transposed form H1^T = W1 X^T, H2^T = W2 H1^T:
//   * layer 1: FP32 MFMA 16x16x4 (K = the 4 features), bias as the
//     accumulator's initial value;
//   * layer 2: FP16 MFMA 16x16x32 with FP32 accumulation on split operands:
//     ReLU(h1) = a_hi + a_lo and W2 = w_hi + w_lo, each part a binary16
//     value (a_hi the rounding of the FP32 value, a_lo the rounding of the
//     exact remainder), and W2 h1 is accumulated as w_hi a_hi + w_hi a_lo +
//     w_lo a_hi (three MFMAs; every product of two halves is exact in FP32).
//     The dropped w_lo a_lo and the split's rounding are below 2^-21 of
//     |W2| h1, so layer 2 keeps FP32 accuracy at a fraction of the cost of
//     FP32 matrix instructions.  The W2 fragments (hi and lo, 64 KB) are
//     staged once per workgroup of eight waves in LDS (each lane's fragment
//     a 16-byte neighbour of the next lane's);
//   * layer 3, biases and ReLU in FP32 on the vector ALUs.
// The hidden units of layer 1 are computed in a permuted order so that its
// result registers are already laid out as layer 2's B operand.
// Training (loss and gradient) runs in FP32 on the matrix cores (FP32 MFMA
// 16x16x4), 16 states per wavefront: the forward pass, the loss and the
// deltas back through W2, with the per-state activations and deltas written
// feature-major ([128][S]).  The weight gradients are then products over the
// states, G_[W2|b2] = D2 [H1^T | 1], G_[W1|b1] = D1 [X | 1] and
// G_[W3|b3] = dout [H2^T | 1], taken in 16 x 16 tiles on the matrix cores
// (FP32 MFMA 16x16x4) over fixed chunks of states, and the chunks' partial
// tiles are summed in chunk order: the result does not depend on scheduling.
#include <mutex>

#include "common.hpp"

namespace mimo {

constexpr int HID = MIMO_MLP_HIDDEN;
constexpr int NIN = MIMO_MLP_IN;
constexpr int OW1 = 0, OB1 = OW1 + HID * NIN, OW2 = OB1 + HID, OB2 = OW2 + HID * HID, OW3 = OB2 + HID,
              OB3 = OW3 + HID;

// h1 = relu(W1 x + b1)
__device__ inline void mlp_layer1(const float* __restrict__ w, const float x[NIN], float h1[HID])
{
#pragma unroll
    for (int i = 0; i < HID; ++i) {
        float s = w[OB1 + i];
#pragma unroll
        for (int j = 0; j < NIN; ++j) s = fmaf(w[OW1 + i * NIN + j], x[j], s);
        h1[i] = fmaxf(s, 0.f);
    }
}

typedef _Float16 half8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// hidden unit computed by row i (0..15) of layer-1 block hb (0..7): rows
// 4g..4g+3 of blocks 2t and 2t+1 hold units 32t + 8g + (0..3) and
// 32t + 8g + (4..7), i.e. the eight units that lane group g feeds to the
// K = 32 step t of layer 2
__host__ __device__ inline int mlp_perm(int hb, int i)
{
    return 32 * (hb >> 1) + 8 * (i >> 2) + 4 * (hb & 1) + (i & 3);
}

// S states, 16 SG per wavefront and step (SG groups of 16 share each W2
// fragment read from LDS); SCHED: K_t = clamp(ceil(2^(yhat + margin)), kmin,
// kmax) into ks (non-finite yhat: kmax and the frame flagged for fallback),
// else yhat into out
constexpr int MLP_SG = 2;                                    // state groups per wave step
constexpr int MLP_WG = 768;                                  // twelve waves (3 per SIMD) share the staged W2
constexpr size_t MLP_W2_LDS = 2 * 8 * 4 * WAVE * sizeof(half8);  // hi and lo fragments: 64 KB

template <bool SCHED>
__global__ void __launch_bounds__(MLP_WG) mlp_infer_kernel(const float* __restrict__ w, const float* __restrict__ X,
                                                           int64_t S, float* __restrict__ out, float margin, int kmin,
                                                           int kmax, int n, int32_t* __restrict__ ks,
                                                           uint32_t* __restrict__ flags)
{
    constexpr int SG = MLP_SG;
    __shared__ f32x4 cb1[8 * 4];  // b1 in the permuted order, [hb][g] -> rows 4g..4g+3
    __shared__ f32x4 cb2[32];     // b2, [nb][g] -> units 16nb + 4g .. +3
    __shared__ f32x4 cw3[32];     // w3, same layout
    const int tid = threadIdx.x, lane = tid & 63;
    const int g = lane >> 4, s16 = lane & 15;
    if (tid < HID) {
        reinterpret_cast<float*>(cb1)[tid] = w[OB1 + mlp_perm(tid >> 4, tid & 15)];
        reinterpret_cast<float*>(cb2)[tid] = w[OB2 + tid];
        reinterpret_cast<float*>(cw3)[tid] = w[OW3 + tid];
    }
    // layer-1 A operand of block hb: row s16 (unit mlp_perm(hb, s16)), feature g
    float a1[8];
#pragma unroll
    for (int hb = 0; hb < 8; ++hb) a1[hb] = w[OW1 + mlp_perm(hb, s16) * NIN + g];
    // layer-2 A operand of output block nb, step t, for lane (g, s16):
    // W2[16nb + s16][32t + 8g + e], e = 0..7, split into w2h + w2l at
    // [(4nb + t) 64 + lane]
    extern __shared__ half8 w2dyn[];
    half8* w2h = w2dyn;
    half8* w2l = w2dyn + 8 * 4 * WAVE;
    for (int idx = tid; idx < 8 * 4 * WAVE; idx += blockDim.x) {
        const int f = idx / WAVE, ln = idx % WAVE;
        const int nb = f >> 2, t = f & 3;
        const float* row = w + OW2 + (16 * nb + (ln & 15)) * HID + 32 * t + 8 * (ln >> 4);
        half8 h, l;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float v = row[e];
            h[e] = (_Float16)v;
            l[e] = (_Float16)(v - (float)h[e]);  // the remainder is exact in FP32
        }
        w2h[idx] = h;
        w2l[idx] = l;
    }
    const float b3 = w[OB3];
    __syncthreads();

    const int64_t ngrp = (S + 16 * SG - 1) / (16 * SG);
    const int64_t nwaves = (int64_t)gridDim.x * (blockDim.x / WAVE);
    for (int64_t grp = (int64_t)blockIdx.x * (blockDim.x / WAVE) + (tid >> 6); grp < ngrp; grp += nwaves) {
        float xb[SG];  // layer-1 B operand of group q: feature g of state s16
#pragma unroll
        for (int q = 0; q < SG; ++q) {
            const int64_t s = (grp * SG + q) * 16 + s16;
            xb[q] = s < S ? X[s * NIN + g] : 0.f;
        }
        asm volatile("" ::: "memory");  // W2 fragments are read from LDS each step, not hoisted into registers
        f32x4 d2[SG][8];
#pragma unroll
        for (int q = 0; q < SG; ++q)
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) d2[q][nb] = f32x4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int t = 0; t < 4; ++t) {
            half8 bh[SG], bl[SG];
#pragma unroll
            for (int q = 0; q < SG; ++q) {
                const f32x4 h0 = __builtin_amdgcn_mfma_f32_16x16x4f32(a1[2 * t], xb[q], cb1[(2 * t) * 4 + g], 0, 0, 0);
                const f32x4 h1 =
                    __builtin_amdgcn_mfma_f32_16x16x4f32(a1[2 * t + 1], xb[q], cb1[(2 * t + 1) * 4 + g], 0, 0, 0);
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float r = fmaxf(e < 4 ? h0[e] : h1[e - 4], 0.f);
                    bh[q][e] = (_Float16)r;
                    bl[q][e] = (_Float16)(r - (float)bh[q][e]);
                }
            }
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                const half8 ah = w2h[(4 * nb + t) * WAVE + lane], al = w2l[(4 * nb + t) * WAVE + lane];
#pragma unroll
                for (int q = 0; q < SG; ++q) {
                    d2[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(al, bh[q], d2[q][nb], 0, 0, 0);
                    d2[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bl[q], d2[q][nb], 0, 0, 0);
                    d2[q][nb] = __builtin_amdgcn_mfma_f32_16x16x32_f16(ah, bh[q], d2[q][nb], 0, 0, 0);
                }
            }
        }
#pragma unroll
        for (int q = 0; q < SG; ++q) {
            const int64_t s = (grp * SG + q) * 16 + s16;
            // lane (g, s16) holds units 16nb + 4g + r of state s16
            float part = 0.f;
#pragma unroll
            for (int nb = 0; nb < 8; ++nb) {
                const f32x4 bb = cb2[nb * 4 + g], ww = cw3[nb * 4 + g];
#pragma unroll
                for (int r = 0; r < 4; ++r) part = fmaf(ww[r], fmaxf(d2[q][nb][r] + bb[r], 0.f), part);
            }
            part += __builtin_bit_cast(float, xor_lanes(__builtin_bit_cast(uint32_t, part), 16, lane));
            part += __builtin_bit_cast(float, xor_lanes(__builtin_bit_cast(uint32_t, part), 32, lane));
            const float yhat = part + b3;
            if (g == 0 && s < S) {
                if (!SCHED) {
                    out[s] = yhat;
                } else {
                    int k;
                    if (!isfinite(yhat)) {
                        k = kmax;
                        if (flags) atomicOr(&flags[s / n], MIMO_FLAG_LEARNED_FALLBACK);
                    } else {
                        const float e = fminf(yhat + margin, 30.f);
                        const float kk = ceilf(exp2f(e));
                        k = kk < (float)kmin ? kmin : (kk > (float)kmax ? kmax : (int)kk);
                    }
                    ks[s] = k;
                }
            }
        }
    }
}

static int mlp_infer_grid(int64_t S)
{
    int dev = 0, cus = 0;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    const int64_t waves = MLP_WG / WAVE;
    const int64_t want = ((S + 16 * MLP_SG - 1) / (16 * MLP_SG) + waves - 1) / waves;
    const int64_t cap = (int64_t)(cus > 0 ? cus : 256);  // one workgroup per compute unit (144 VGPRs per lane)
    return (int)(want < cap ? want : cap);
}

template <bool SCHED>
static int32_t launch_mlp_infer(int64_t S, hipStream_t st, const float* w, const float* X, float* out, float margin,
                                int kmin, int kmax, int n, int32_t* ks, uint32_t* flags)
{
    static bool lds_set = false;  // the attribute is set once per process (idempotent if two threads race)
    if (!lds_set) {
        hipError_t e = hipFuncSetAttribute((const void*)mlp_infer_kernel<SCHED>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)MLP_W2_LDS);
        if (e != hipSuccess) return fail(MIMO_ERR_HIP, "MLP inference: LDS attribute: %s", hipGetErrorString(e));
        lds_set = true;
    }
    hipLaunchKernelGGL(mlp_infer_kernel<SCHED>, dim3(mlp_infer_grid(S)), dim3(MLP_WG), MLP_W2_LDS, st, w, X, S, out,
                       margin, kmin, kmax, n, ks, flags);
    return check_launch(SCHED ? "prune_mlp_schedule" : "prune_mlp_forward");
}

// per state: activations and deltas, feature-major in the workspace, on the
// matrix cores (FP32 MFMA 16x16x4).  A wavefront takes 16 states, lane l
// feeding state l % 16: layer 1 is W1 [X^T] (K = 4), layer 2 W2 H1^T and the
// delta through it W2^T D2^T (K = 128, 32 k-steps per 16 rows); a
// wavefront's H1^T, then its D2^T, pass through LDS (128 x 16 floats) to
// become the B operand.  Lane l holds rows 16 rb + 4 (l / 16) + i of each
// 16-row block rb, column l % 16.  The loss of a workgroup's 64 states is
// summed in a fixed order into lpart[blockIdx.x].
constexpr int BK_WAVES = 4, BK_STATES = 16 * BK_WAVES;

__host__ __device__ constexpr int64_t loss_parts(int64_t S) { return (S + BK_STATES - 1) / BK_STATES; }

typedef float f32x4b __attribute__((ext_vector_type(4)));

__global__ void __launch_bounds__(64 * BK_WAVES) mlp_backward_mfma(const float* __restrict__ w,
                                                                  const float* __restrict__ X,
                                                                  const float* __restrict__ y, int64_t S, float tau,
                                                                  float* __restrict__ H1, float* __restrict__ H2,
                                                                  float* __restrict__ D2, float* __restrict__ D1,
                                                                  float* __restrict__ dout,
                                                                  float* __restrict__ lpart)
{
    __shared__ float tb[BK_WAVES][HID][16];
    __shared__ float red[BK_WAVES];
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int col = lane & 15, kq = lane >> 4;
    const int64_t s = (int64_t)blockIdx.x * BK_STATES + 16 * wave + col;
    const bool live = s < S;
    float (*T)[16] = tb[wave];

    // layer 1: a1 = W1 x + b1 (one k-step, K = the 4 features)
    f32x4b a1[8];
    {
        const float xb = live ? X[s * NIN + kq] : 0.f;
#pragma unroll
        for (int rb = 0; rb < 8; ++rb) {
            f32x4b c;
#pragma unroll
            for (int i = 0; i < 4; ++i) c[i] = w[OB1 + 16 * rb + 4 * kq + i];
            a1[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[OW1 + (16 * rb + col) * NIN + kq], xb, c, 0, 0, 0);
        }
    }
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * rb + 4 * kq + i;
            const float h = fmaxf(a1[rb][i], 0.f);
            T[r][col] = h;
            if (live) H1[(int64_t)r * S + s] = h;
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");

    // layer 2: a2 = W2 h1 + b2
    f32x4b a2[8];
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) a2[rb][i] = w[OB2 + 16 * rb + 4 * kq + i];
    for (int q = 0; q < HID / 4; ++q) {
        const float b = T[4 * q + kq][col];
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
            a2[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[OW2 + (16 * rb + col) * HID + 4 * q + kq], b, a2[rb], 0,
                                                          0, 0);
    }
    // ReLU, layer 3 (this lane's 32 rows, then the four row groups of the column)
    float out = 0.f;
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int r = 16 * rb + 4 * kq + i;
            const float h = fmaxf(a2[rb][i], 0.f);
            if (live) H2[(int64_t)r * S + s] = h;
            out = fmaf(w[OW3 + r], h, out);
        }
    out += __shfl_xor(out, 16, WAVE);
    out += __shfl_xor(out, 32, WAVE);
    out += w[OB3];
    const float r = live ? y[s] - out : 0.f;
    const float loss = live ? (r > 0.f ? tau * r : (tau - 1.f) * r) : 0.f;
    const float dz = live ? (r > 0.f ? -tau : 1.f - tau) / (float)S : 0.f;
    if (live && kq == 0) dout[s] = dz;

    // delta of layer 2 (zero where the ReLU was off), into LDS for the delta through W2
    __builtin_amdgcn_wave_barrier();  // every lane has read T for layer 2
#pragma unroll
    for (int rb = 0; rb < 8; ++rb)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int rr = 16 * rb + 4 * kq + i;
            const float d2 = a2[rb][i] > 0.f ? dz * w[OW3 + rr] : 0.f;
            T[rr][col] = d2;
            if (live) D2[(int64_t)rr * S + s] = d2;
        }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    // delta of layer 1: W2^T d2, masked by layer 1's ReLU
    f32x4b d1[8];
#pragma unroll
    for (int rb = 0; rb < 8; ++rb) d1[rb] = f32x4b{0.f, 0.f, 0.f, 0.f};
    for (int q = 0; q < HID / 4; ++q) {
        const float b = T[4 * q + kq][col];
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
            d1[rb] = __builtin_amdgcn_mfma_f32_16x16x4f32(w[OW2 + (4 * q + kq) * HID + 16 * rb + col], b, d1[rb], 0,
                                                          0, 0);
    }
    if (live) {
#pragma unroll
        for (int rb = 0; rb < 8; ++rb)
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int rr = 16 * rb + 4 * kq + i;
                D1[(int64_t)rr * S + s] = a1[rb][i] > 0.f ? d1[rb][i] : 0.f;
            }
    }
    // the workgroup's loss: columns 0..15 of each wavefront in order, then the wavefronts
    float l = kq == 0 ? loss : 0.f;
#pragma unroll
    for (int m = 1; m < 16; m <<= 1) l += __shfl_xor(l, m, WAVE);
    if (lane == 0) red[wave] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int v = 0; v < BK_WAVES; ++v) t += red[v];
        lpart[blockIdx.x] = t;
    }
}

// Weight-gradient tiles.  Tile t < 72: rows 16 (t / 9) .. of D2, columns
// 16 (t % 9) .. of [H1^T | 1] (column 128 the ones); t < 80: rows 16 (t - 72)
// .. of D1, columns [X | 1] (column 4 the ones); t < 89: row 0 is dout,
// columns 16 (t - 80) .. of [H2^T | 1].  Entries past the sources are zero.
constexpr int GT_W2 = 0, GT_W1 = 72, GT_W3 = 80, GT_N = 89;
constexpr int G_CHUNK_MIN = 256;  // states per chunk, at least
constexpr int G_CHUNKS_MAX = 64;

__host__ __device__ constexpr int grad_chunks(int64_t S)
{
    const int64_t c = (S + G_CHUNK_MIN - 1) / G_CHUNK_MIN;
    return (int)(c < 1 ? 1 : (c > G_CHUNKS_MAX ? G_CHUNKS_MAX : c));
}

// states per chunk: a multiple of 16 (four MFMA k-steps per load round)
__host__ __device__ inline int64_t grad_chunk_len(int64_t S)
{
    const int C = grad_chunks(S);
    const int64_t L = (S + C - 1) / C;
    return (L + 15) & ~(int64_t)15;
}

// row r of the A operand of tile t at state s
__device__ __forceinline__ float grad_a(int t, int r, int64_t s, int64_t S, const float* __restrict__ D2,
                                        const float* __restrict__ D1, const float* __restrict__ dout)
{
    if (s >= S) return 0.f;
    if (t < GT_W1) return D2[(int64_t)(16 * (t / 9) + r) * S + s];
    if (t < GT_W3) return D1[(int64_t)(16 * (t - GT_W1) + r) * S + s];
    return r == 0 ? dout[s] : 0.f;
}

// column c of the B operand of tile t at state s
__device__ __forceinline__ float grad_b(int t, int c, int64_t s, int64_t S, const float* __restrict__ H1,
                                        const float* __restrict__ X, const float* __restrict__ H2)
{
    if (s >= S) return 0.f;
    if (t < GT_W1) {
        const int j = 16 * (t % 9) + c;
        return j < HID ? H1[(int64_t)j * S + s] : (j == HID ? 1.f : 0.f);
    }
    if (t < GT_W3) return c < NIN ? X[s * NIN + c] : (c == NIN ? 1.f : 0.f);
    const int j = 16 * (t - GT_W3) + c;
    return j < HID ? H2[(int64_t)j * S + s] : (j == HID ? 1.f : 0.f);
}

typedef float f32x4g __attribute__((ext_vector_type(4)));

// one wavefront per (tile, chunk): the chunk's partial 16 x 16 tile.  Lane l
// feeds row / column l % 16 at states s0 + 4 (l / 16) + e of the e-th of four
// MFMA k-steps (the same states for A and B, so each step sums over them)
__global__ void __launch_bounds__(256) mlp_grad_tiles(int64_t S, const float* __restrict__ X,
                                                      const float* __restrict__ H1, const float* __restrict__ H2,
                                                      const float* __restrict__ D2, const float* __restrict__ D1,
                                                      const float* __restrict__ dout, float* __restrict__ part)
{
    const int job = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
    const int C = grad_chunks(S);
    if (job >= GT_N * C) return;  // uniform per wavefront
    const int lane = threadIdx.x & 63;
    const int t = job % GT_N, c = job / GT_N;
    const int64_t L = grad_chunk_len(S), s_beg = (int64_t)c * L, s_end = s_beg + L;
    const int rc = lane & 15, kq = lane >> 4;
    f32x4g acc = {0.f, 0.f, 0.f, 0.f};
    for (int64_t s0 = s_beg; s0 < s_end; s0 += 16) {
        float a[4], b[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t s = s0 + 4 * kq + e;
            a[e] = grad_a(t, rc, s, S, D2, D1, dout);
            b[e] = grad_b(t, rc, s, S, H1, X, H2);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[e], b[e], acc, 0, 0, 0);
    }
    // lane l holds rows 4 (l / 16) + i of column l % 16
    float* out = part + ((size_t)c * GT_N + t) * 256;
#pragma unroll
    for (int i = 0; i < 4; ++i) out[(4 * kq + i) * 16 + rc] = acc[i];
}

// Tiles in groups of up to three that share an operand: a W2 tile row block
// (the same 16 rows of D2) over three column blocks, three W1 tiles (the same
// [X | 1] columns), three W3 tiles (the same dout row).  The shared operand
// is loaded once per k-step for the group, instead of once per tile.
constexpr int GT_G = 30;              // 24 W2 groups, 3 W1, 3 W3
constexpr int64_t G_GROUP_MIN_LEN = 512;  // states per chunk from which the groups are launched

__device__ __forceinline__ void grad_group(int g, int& t0, int& nt, bool& share_a)
{
    if (g < 24) {  // W2: row block g / 3, column blocks 3 (g % 3) .. + 2
        t0 = GT_W2 + 9 * (g / 3) + 3 * (g % 3);
        nt = 3;
        share_a = true;
    } else if (g < 27) {  // W1: tiles 72-74, 75-77, 78-79
        t0 = GT_W1 + 3 * (g - 24);
        nt = GT_W3 - t0 < 3 ? GT_W3 - t0 : 3;
        share_a = false;
    } else {  // W3: tiles 80-82, 83-85, 86-88
        t0 = GT_W3 + 3 * (g - 27);
        nt = 3;
        share_a = true;
    }
}

// one wavefront per (tile group, chunk): the chunk's partial 16 x 16 tiles.
// Lane l feeds row / column l % 16 at states s0 + 4 (l / 16) + e of the e-th
// of four MFMA k-steps (the same states for A and B, so each step sums over
// them); every tile takes the same products in the same order as alone.
__global__ void __launch_bounds__(256) mlp_grad_tile_groups(int64_t S, const float* __restrict__ X,
                                                            const float* __restrict__ H1, const float* __restrict__ H2,
                                                            const float* __restrict__ D2, const float* __restrict__ D1,
                                                            const float* __restrict__ dout, float* __restrict__ part)
{
    const int job = blockIdx.x * (blockDim.x / WAVE) + (threadIdx.x >> 6);
    const int C = grad_chunks(S);
    if (job >= GT_G * C) return;  // uniform per wavefront
    const int lane = threadIdx.x & 63;
    const int g = job % GT_G, c = job / GT_G;
    int t0, nt;
    bool share_a;
    grad_group(g, t0, nt, share_a);
    const int64_t L = grad_chunk_len(S), s_beg = (int64_t)c * L, s_end = s_beg + L;
    const int rc = lane & 15, kq = lane >> 4;
    f32x4g acc[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) acc[k] = f32x4g{0.f, 0.f, 0.f, 0.f};
    for (int64_t s0 = s_beg; s0 < s_end; s0 += 16) {
        float sh[4], own[3][4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int64_t s = s0 + 4 * kq + e;
            sh[e] = share_a ? grad_a(t0, rc, s, S, D2, D1, dout) : grad_b(t0, rc, s, S, H1, X, H2);
#pragma unroll
            for (int k = 0; k < 3; ++k)
                if (k < nt) own[k][e] = share_a ? grad_b(t0 + k, rc, s, S, H1, X, H2) : grad_a(t0 + k, rc, s, S, D2, D1, dout);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            if (k < nt) {
#pragma unroll
                for (int e = 0; e < 4; ++e)
                    acc[k] = share_a ? __builtin_amdgcn_mfma_f32_16x16x4f32(sh[e], own[k][e], acc[k], 0, 0, 0)
                                     : __builtin_amdgcn_mfma_f32_16x16x4f32(own[k][e], sh[e], acc[k], 0, 0, 0);
            }
        }
    }
    // lane l holds rows 4 (l / 16) + i of column l % 16
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        if (k < nt) {
            float* out = part + ((size_t)c * GT_N + t0 + k) * 256;
#pragma unroll
            for (int i = 0; i < 4; ++i) out[(4 * kq + i) * 16 + rc] = acc[k][i];
        }
    }
}

// one thread per parameter (and one for the loss): its tile entry summed
// over the chunks in order
__global__ void __launch_bounds__(256) mlp_grad_sum(int64_t S, const float* __restrict__ part,
                                                    const float* __restrict__ lpart, int nlpart,
                                                    float* __restrict__ grad, float* __restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > MIMO_MLP_NPARAM) return;
    if (p == MIMO_MLP_NPARAM) {
        float acc = 0.f;
        for (int b = 0; b < nlpart; ++b) acc += lpart[b];
        *loss = acc / (float)S;
        return;
    }
    int t, r, col;
    if (p < OB1) {  // W1[i][j]
        const int i = p / NIN;
        t = GT_W1 + i / 16, r = i % 16, col = p % NIN;
    } else if (p < OW2) {  // b1[i]
        const int i = p - OB1;
        t = GT_W1 + i / 16, r = i % 16, col = NIN;
    } else if (p < OB2) {  // W2[i][j]
        const int i = (p - OW2) / HID, j = (p - OW2) % HID;
        t = GT_W2 + 9 * (i / 16) + j / 16, r = i % 16, col = j % 16;
    } else if (p < OW3) {  // b2[i]
        const int i = p - OB2;
        t = GT_W2 + 9 * (i / 16) + 8, r = i % 16, col = 0;
    } else if (p < OB3) {  // W3[j]
        const int j = p - OW3;
        t = GT_W3 + j / 16, r = 0, col = j % 16;
    } else {  // b3
        t = GT_W3 + 8, r = 0, col = 0;
    }
    const int C = grad_chunks(S);
    float acc = 0.f;
    for (int c = 0; c < C; ++c) acc += part[((size_t)c * GT_N + t) * 256 + r * 16 + col];
    grad[p] = acc;
}

__global__ void __launch_bounds__(256) adam_kernel(float* __restrict__ w, float* __restrict__ m, float* __restrict__ v,
                                                   const float* __restrict__ g, int np, float lr, float b1, float b2,
                                                   float c1, float c2, float eps)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= np) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

}  // namespace mimo

using namespace mimo;

extern "C" int32_t prune_mlp_forward(const float* w, const float* X, int64_t S, float* out, void* stream)
{
    if (S < 0) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_forward: S < 0");
    if (S == 0) return MIMO_OK;
    if (!w || !X || !out) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_forward: null pointer");
    return launch_mlp_infer<false>(S, (hipStream_t)stream, w, X, out, 0.f, 1, 1, 1, nullptr, nullptr);
}

extern "C" int32_t prune_mlp_schedule(const float* w, const float* X, int64_t S, float margin, int32_t k_min,
                                      int32_t k_max, int32_t n, int32_t* k_sched, uint32_t* flags, void* stream)
{
    if (S < 0 || n < 1) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_schedule: S < 0 or n < 1");
    if (k_min < 1 || k_max < k_min || k_max > MIMO_MAX_K)
        return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_schedule: need 1 <= k_min <= k_max <= %d", MIMO_MAX_K);
    if (S == 0) return MIMO_OK;
    if (!w || !X || !k_sched) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_schedule: null pointer");
    return launch_mlp_infer<true>(S, (hipStream_t)stream, w, X, nullptr, margin, k_min, k_max, n, k_sched, flags);
}

extern "C" size_t prune_mlp_workspace_bytes(int64_t S)
{
    using namespace mimo;
    if (S < 0) S = 0;
    const int64_t nblk = loss_parts(S);
    // activations and deltas, dout, loss partials (padded to 64 floats), then the partial tiles
    const int64_t head = (4 * HID * S + S + nblk + 64 + 63) & ~(int64_t)63;
    return sizeof(float) * (size_t)(head + (int64_t)grad_chunks(S) * GT_N * 256);
}

namespace mimo {

// The loss and gradient of S states with the per-state activations, deltas
// and loss partials in the workspace ws (prune_mlp_workspace_bytes(S)).
static int32_t mlp_loss_grad_ws(const char* who, const float* w, const float* X, const float* y, int64_t S,
                                float tau, float* grad, float* loss, float* ws, hipStream_t st)
{
    float* f = ws;
    float* H1 = f;
    float* H2 = H1 + HID * S;
    float* D2 = H2 + HID * S;
    float* D1 = D2 + HID * S;
    float* dout = D1 + HID * S;
    float* lpart = dout + S;
    const int nblk = (int)loss_parts(S);
    hipLaunchKernelGGL(mlp_backward_mfma, dim3(nblk), dim3(64 * BK_WAVES), 0, st, w, X, y, S, tau, H1, H2, D2, D1,
                       dout, lpart);
    int32_t rc = check_launch(who);
    if (rc) return rc;
    float* part = f + ((4 * HID * S + S + nblk + 64 + 63) & ~(int64_t)63);
    // long chunks: tile groups (fewer loads); short ones: one tile per
    // wavefront (three times the wavefronts to hide the loads' latency).
    // Both give the same partial tiles.
    if (grad_chunk_len(S) >= G_GROUP_MIN_LEN) {
        const int jobs = GT_G * grad_chunks(S);
        hipLaunchKernelGGL(mlp_grad_tile_groups, dim3((jobs + 3) / 4), dim3(256), 0, st, S, X, H1, H2, D2, D1, dout,
                           part);
    } else {
        const int jobs = GT_N * grad_chunks(S);
        hipLaunchKernelGGL(mlp_grad_tiles, dim3((jobs + 3) / 4), dim3(256), 0, st, S, X, H1, H2, D2, D1, dout, part);
    }
    rc = check_launch(who);
    if (rc) return rc;
    hipLaunchKernelGGL(mlp_grad_sum, dim3((MIMO_MLP_NPARAM + 1 + 255) / 256), dim3(256), 0, st, S, part, lpart, nblk,
                       grad, loss);
    return check_launch(who);
}

static int32_t mlp_loss_grad_check(const char* who, const float* w, const float* X, const float* y, int64_t S,
                                   float tau, const float* grad, const float* loss)
{
    if (S < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: S < 1", who);
    if (!(tau > 0.f && tau < 1.f)) return fail(MIMO_ERR_INVALID_ARG, "%s: tau in (0, 1)", who);
    if (!w || !X || !y || !grad || !loss) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", who);
    return MIMO_OK;
}

// Scratch of the allocation-free entry point: the workspace of up to
// MIMO_MLP_NOALLOC_MAX_S states in a static device array, one copy per GPU
// for the life of the process.  Host code never passes the array's name to
// a kernel (on the host it is only a stand-in for the symbol): the device
// address is looked up once per device with that device current and kept.
constexpr size_t NOALLOC_FLOATS =
    (((size_t)4 * HID * MIMO_MLP_NOALLOC_MAX_S + MIMO_MLP_NOALLOC_MAX_S + loss_parts(MIMO_MLP_NOALLOC_MAX_S) + 64 +
      63) & ~(size_t)63) +
    (size_t)grad_chunks(MIMO_MLP_NOALLOC_MAX_S) * GT_N * 256;
static __device__ __align__(256) float scratch[NOALLOC_FLOATS];

constexpr int MAX_DEVICES = 64;
static std::mutex g_scratch_mu;
static float* g_scratch_ptr[MAX_DEVICES];

static int32_t scratch_for_current_device(const char* who, float** out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(MIMO_ERR_HIP, "%s: hipGetDevice: %s", who, hipGetErrorString(e));
    if (dev < 0 || dev >= MAX_DEVICES) return fail(MIMO_ERR_UNSUPPORTED, "%s: device %d beyond %d", who, dev, MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(MIMO_ERR_HIP, "%s: scratch address on device %d: %s", who, dev, hipGetErrorString(e));
        g_scratch_ptr[dev] = static_cast<float*>(p);
    }
    *out = g_scratch_ptr[dev];
    return MIMO_OK;
}

}  // namespace mimo

extern "C" int32_t prune_mlp_loss_grad(const float* w, const float* X, const float* y, int64_t S, float tau,
                                       float* grad, float* loss, void* ws, size_t ws_bytes, void* stream)
{
    const char* who = "prune_mlp_loss_grad";
    int32_t rc = mlp_loss_grad_check(who, w, X, y, S, tau, grad, loss);
    if (rc) return rc;
    if (!ws) return fail(MIMO_ERR_INVALID_ARG, "%s: null workspace", who);
    if (ws_bytes < prune_mlp_workspace_bytes(S))
        return fail(MIMO_ERR_WORKSPACE, "%s: workspace %zu < %zu", who, ws_bytes, prune_mlp_workspace_bytes(S));
    return mlp_loss_grad_ws(who, w, X, y, S, tau, grad, loss, static_cast<float*>(ws), (hipStream_t)stream);
}

extern "C" int32_t prune_mlp_loss_grad_noalloc(const float* w, const float* X, const float* y, int64_t S, float tau,
                                               float* grad, float* loss, void* stream)
{
    const char* who = "prune_mlp_loss_grad_noalloc";
    int32_t rc = mlp_loss_grad_check(who, w, X, y, S, tau, grad, loss);
    if (rc) return rc;
    if (S > MIMO_MLP_NOALLOC_MAX_S)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: S = %lld states exceed the static scratch of %d", who, (long long)S,
                    MIMO_MLP_NOALLOC_MAX_S);
    float* ws = nullptr;
    rc = scratch_for_current_device(who, &ws);
    if (rc) return rc;
    return mlp_loss_grad_ws(who, w, X, y, S, tau, grad, loss, ws, (hipStream_t)stream);
}

extern "C" int32_t prune_mlp_adam_step(float* w, float* m, float* v, const float* grad, int32_t np, int32_t t,
                                       float lr, float beta1, float beta2, float eps, void* stream)
{
    if (np < 1 || t < 1) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_adam_step: np < 1 or t < 1");
    if (!w || !m || !v || !grad) return fail(MIMO_ERR_INVALID_ARG, "prune_mlp_adam_step: null pointer");
    const float c1 = 1.f - powf(beta1, (float)t), c2 = 1.f - powf(beta2, (float)t);
    hipLaunchKernelGGL(adam_kernel, dim3((np + 255) / 256), dim3(256), 0, (hipStream_t)stream, w, m, v, grad, np, lr,
                       beta1, beta2, c1, c2, eps);
    return check_launch("prune_mlp_adam_step");
}
