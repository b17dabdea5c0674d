// Batched K-best detection (Sec. VI) on the real-valued tree, one wavefront
// per frame.
//
// Per level k (n-1 down to 0):
//   * row k of R (scaled by the PAM spacing c) is staged in LDS;
//   * every survivor's cancellation centre b = z_k - sum_{j>k} R_kj x_j is a
//     dot product of that row with the survivor's path (PAM indices, one
//     byte per level, in LDS), split over 64/KCAP lanes per survivor; the
//     amplitude 2i-(P-1) is folded as 2 * sum(R i) - (P-1) * sum(R);
//   * each child c of survivor s gets pd' = pd_s + (b - R_kk a_c)^2 (FP32
//     FMA) -- the incremental evaluation of Eq. (inc);
//   * children outside the radius are dropped and the rest are sorted in the
//     wave by the 64-bit key (pd bits, s * P + c), which orders them by
//     (pd, parent rank, child index) because survivors stay sorted;
//   * the first K_t keys become the next survivors; their paths are copied
//     from the parents with the new symbol written at level k.
#include "common.hpp"

namespace mimo {

struct KbestArgs {
    const float* R;
    const float* z;
    int n;                 // real levels
    int K;                 // survivors (cap of the schedule)
    const int32_t* k_sched;
    int k_sched_stride;
    const float* radius2;
    const int32_t* force_sym;  // label mode: forced path (QAM indices) or NULL
    int32_t* rank;             // label mode output [B][n]
    int32_t* sym;
    float* pd;
    uint32_t* flags;
    int64_t* counters;
};

template <int P, int E>
struct KbestShape {
    static constexpr int NC = WAVE * E;                  // candidates per level
    static constexpr int KCAP = NC / P;                  // survivor capacity
    static constexpr int L = KCAP >= WAVE ? 1 : WAVE / KCAP;  // lanes per survivor
    static constexpr int SPL = KCAP >= WAVE ? KCAP / WAVE : 1; // survivors per lane
};

inline int kb_row_words(int n) { return (n + 3) / 4 + 1; }  // odd-ish stride against bank conflicts

template <int P, int E>
__host__ __device__ inline size_t kbest_lds_bytes(int n)
{
    using S = KbestShape<P, E>;
    const int nw = (n + 3) / 4, stride = nw + 1;
    return sizeof(uint32_t) * 2 * S::KCAP * stride  // paths
           + sizeof(float) * 2 * S::KCAP           // survivor pd
           + sizeof(float) * nw * 4                // staged R row
           + sizeof(int32_t) * S::KCAP;            // selected candidate ids
}

// K-best of one frame by one wavefront; lds as sized by kbest_lds_bytes.
template <int P, int E>
__device__ void kbest_frame(const KbestArgs& a, int frame, unsigned char* lds)
{
    using S = KbestShape<P, E>;
    constexpr int KCAP = S::KCAP, L = S::L, SPL = S::SPL;
    const int lane = threadIdx.x & 63;
    const int n = a.n;
    const int nw = (n + 3) / 4, stride = nw + 1;
    uint32_t* path = reinterpret_cast<uint32_t*>(lds);
    float* spd = reinterpret_cast<float*>(path + 2 * KCAP * stride);
    float* rrow = spd + 2 * KCAP;
    int32_t* sel = reinterpret_cast<int32_t*>(rrow + nw * 4);

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;
    const int32_t* fsym = a.force_sym ? a.force_sym + (size_t)frame * (n / 2) : nullptr;

    if (lane == 0) spd[0] = 0.f;
    int cnt = 1, fs = 0;
    int64_t expanded = 0;
    uint32_t flags = 0;
    __syncthreads();

    for (int k = n - 1; k >= 0; --k) {
        const int cur = (n - 1 - k) & 1, nxt = cur ^ 1;
        uint32_t* pc = path + cur * KCAP * stride;
        uint32_t* pn = path + nxt * KCAP * stride;
        float* sc = spd + cur * KCAP;
        float* sn = spd + nxt * KCAP;
        // stage row k: rrow[j] = c R_kj, j in [k, n)
        const float* rk = Rf + r_row_off(n, k);
        float rsum = 0.f;
        for (int t = lane; t < n - k; t += WAVE) {
            const float v = cs * rk[t];
            rrow[k + t] = v;
            if (t > 0) rsum += v;
        }
        rsum = wave_sum(rsum);
        __syncthreads();
        const float rkk = rrow[k];
        const float zk = zf[k];
        // cancellation centres
        float bu[SPL];
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const int s = (KCAP >= WAVE) ? lane + WAVE * u : lane / L;
            const int q = (L > 1) ? (lane % L) : 0;
            float acc = 0.f;
            if (s < cnt) {
                const uint32_t* prow = pc + s * stride;
                for (int wd = (k + 1) / 4 + q; wd < nw; wd += L) {
                    const uint32_t d = prow[wd];
#pragma unroll
                    for (int bb = 0; bb < 4; ++bb) {
                        const int j = 4 * wd + bb;
                        if (j > k && j < n) acc = fmaf(rrow[j], (float)((d >> (8 * bb)) & 0xffu), acc);
                    }
                }
            }
#pragma unroll
            for (int m = 1; m < L; m <<= 1) acc += shfl_xor_f(acc, m);
            bu[u] = zk - (2.f * acc - (float)(P - 1) * rsum);
        }
        // children and keys
        uint64_t key[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int m = e * WAVE + lane;
            const int s = m / P, c = m % P;
            const int u = (KCAP >= WAVE) ? (e / P) : 0;
            const int src = (KCAP >= WAVE) ? (s % WAVE) : (s * L);
            const float b = shfl_f(bu[u], src);
            key[e] = ~0ull;
            if (s < cnt) {
                const float ee = fmaf(-rkk, (float)(2 * c - (P - 1)), b);
                const float pdc = fmaf(ee, ee, sc[s]);
                if (pdc < r2) key[e] = ((uint64_t)__float_as_uint(pdc) << 32) | (uint32_t)m;
            }
        }
        expanded += cnt;
        bitonic_sort<E>(key, lane);
        int nvalid = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) nvalid += __popcll(__ballot(key[e] != ~0ull));
        if (nvalid == 0) {
            flags |= MIMO_FLAG_EMPTY_SPHERE;
            cnt = 0;
            break;
        }
        int Kt = ks ? ks[k] : a.K;
        if (Kt > a.K) Kt = a.K;
        if (Kt < 1) Kt = 1;
        const int keep = Kt < nvalid ? Kt : nvalid;
        if (fsym) {
            // label mode: rank of the forced prefix; keep it in the last slot if needed
            const int sy = fsym[k >> 1];
            const int fc = (k & 1) ? (sy % P) : (sy / P);
            const uint32_t fm = (uint32_t)(fs * P + fc);
            int pos = -1;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const uint64_t bal = __ballot(key[e] != ~0ull && (uint32_t)key[e] == fm);
                if (bal && pos < 0) pos = e * WAVE + (__ffsll((unsigned long long)bal) - 1);
            }
            if (lane == 0) a.rank[(size_t)frame * n + k] = pos + 1;
            if (pos >= keep) {
                const int pe = pos / WAVE, pl = pos % WAVE;
                uint64_t fk = 0;
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (e == pe) fk = shfl_u64(key[e], pl);
                const int te = (keep - 1) / WAVE, tl = (keep - 1) % WAVE;
#pragma unroll
                for (int e = 0; e < E; ++e)
                    if (e == te && lane == tl) key[e] = fk;
                pos = keep - 1;
            }
            fs = pos;
        }
        // new survivors: sorted positions 0 .. keep-1
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int i = e * WAVE + lane;
            if (i < keep) {
                sn[i] = __uint_as_float((uint32_t)(key[e] >> 32));
                sel[i] = (int32_t)(uint32_t)key[e];
            }
        }
        __syncthreads();
        // copy parent paths (levels >= k) and write symbol k
        const int w0 = k / 4;
        for (int i = 0; i < keep; ++i) {
            const int m = sel[i];
            const int s = m / P, c = m % P;
            const uint32_t* src = pc + s * stride;
            uint32_t* dst = pn + i * stride;
            for (int wd = w0 + lane; wd < nw; wd += WAVE) {
                uint32_t d = src[wd];
                if (wd == w0) {
                    const int sh = 8 * (k & 3);
                    d = (d & ~(0xffu << sh)) | ((uint32_t)c << sh);
                }
                dst[wd] = d;
            }
        }
        __syncthreads();
        cnt = keep;
    }

    if (lane == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? spd[(n & 1) * KCAP] : INFINITY;
        if (a.counters) {
            int64_t* c = a.counters + (size_t)frame * 4;
            c[0] = expanded;
            c[1] = expanded * P;
            c[2] = 0;
            c[3] = 0;
        }
    }
    // outputs: survivor 0 of the last buffer is the best leaf
    const uint32_t* best = path + (n & 1) * KCAP * stride;
    if (!a.sym) return;
    for (int m = lane; m < n / 2; m += WAVE) {
        int v = 0;
        if (cnt > 0) {
            const int ire = (best[(2 * m) >> 2] >> (8 * ((2 * m) & 3))) & 0xff;
            const int iim = (best[(2 * m + 1) >> 2] >> (8 * ((2 * m + 1) & 3))) & 0xff;
            v = ire * P + iim;
        }
        a.sym[(size_t)frame * (n / 2) + m] = v;
    }
}

template <int P, int E>
__global__ void __launch_bounds__(64) kbest_kernel(KbestArgs a)
{
    extern __shared__ unsigned char smem_kb[];
    kbest_frame<P, E>(a, blockIdx.x, smem_kb);
}

template <int P, int E>
static int32_t launch_kbest(const KbestArgs& a, int B, hipStream_t st)
{
    const size_t lds = kbest_lds_bytes<P, E>(a.n);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)kbest_kernel<P, E>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return fail(MIMO_ERR_HIP, "kbest: LDS attribute: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL((kbest_kernel<P, E>), dim3(B), dim3(WAVE), lds, st, a);
    return check_launch("kbest_detect");
}

template <int P>
static int32_t dispatch_kbest_p(const KbestArgs& a, int B, hipStream_t st)
{
    const int need = a.K * P;  // candidates per level
    if (need <= 64) return launch_kbest<P, 1>(a, B, st);
    if (need <= 128) return launch_kbest<P, 2>(a, B, st);
    if (need <= 256) return launch_kbest<P, 4>(a, B, st);
    if (need <= 512) return launch_kbest<P, 8>(a, B, st);
    return launch_kbest<P, 16>(a, B, st);
}

static int32_t dispatch_kbest(const KbestArgs& a, int pam, int B, hipStream_t st)
{
    switch (pam) {
    case 2: return dispatch_kbest_p<2>(a, B, st);
    case 4: return dispatch_kbest_p<4>(a, B, st);
    default: return dispatch_kbest_p<8>(a, B, st);
    }
}

static int32_t validate_common(const char* who, int B, int n_tx, int pam, int K)
{
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", who);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", who);
    if (n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: n_tx < 1", who);
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx > %d", who, MIMO_MAX_TX);
    if (K < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: K < 1", who);
    if (K > MIMO_MAX_K || K * pam > 1024)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: K <= %d and K * pam <= 1024", who, MIMO_MAX_K);
    return MIMO_OK;
}

}  // namespace mimo

extern "C" int32_t kbest_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                int32_t K, const int32_t* k_sched, int32_t k_sched_stride,
                                const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                                int64_t* counters, void* stream)
{
    using namespace mimo;
    int32_t rc = validate_common("kbest_detect", B, n_tx, pam, K);
    if (rc) return rc;
    const int n = 2 * n_tx;
    if (k_sched && k_sched_stride != 0 && k_sched_stride != n)
        return fail(MIMO_ERR_INVALID_ARG, "kbest_detect: k_sched_stride must be 0 or n = %d", n);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "kbest_detect: null pointer");
    KbestArgs a{R, z, n, K, k_sched, k_sched_stride, radius2, nullptr, nullptr, sym, pd, flags, counters};
    return dispatch_kbest(a, pam, B, (hipStream_t)stream);
}

extern "C" int32_t kbest_rank_labels(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                     int32_t K, const int32_t* force_sym, int32_t* rank, void* stream)
{
    using namespace mimo;
    int32_t rc = validate_common("kbest_rank_labels", B, n_tx, pam, K);
    if (rc) return rc;
    if (B == 0) return MIMO_OK;
    if (!R || !z || !force_sym || !rank) return fail(MIMO_ERR_INVALID_ARG, "kbest_rank_labels: null pointer");
    KbestArgs a{R, z, 2 * n_tx, K, nullptr, 0, nullptr, force_sym, rank, nullptr, nullptr, nullptr, nullptr};
    return dispatch_kbest(a, pam, B, (hipStream_t)stream);
}
