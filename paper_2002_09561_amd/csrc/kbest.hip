// Batched K-best detection (Sec. VI) on the real-valued tree, one wavefront
// per frame.
//
// Per level k (n-1 down to 0):
//   * row k of R (scaled by the PAM spacing c, zero at and below the
//     diagonal) is staged in LDS;
//   * every survivor's cancellation centre b = z_k - sum_{j>k} R_kj x_j is a
//     dot product of that row with the survivor's path, held in LDS as packed
//     fp16 amplitudes (exact small integers: one mixed-precision FMA per term,
//     FP32 accumulation), split over 64/KCAP lanes per survivor;
//   * each child c of survivor s gets pd' = pd_s + (b - R_kk a_c)^2 (FP32
//     FMA) -- the incremental evaluation of Eq. (inc);
//   * children outside the radius are dropped; the K_t smallest keys
//     (pd bits, s * P + c) -- i.e. (pd, parent rank, child index), since the
//     survivors are kept sorted -- are found by a bitwise binary search on
//     the pd bits with ballot counts, compacted, and put in order by rank
//     counting among the K_t kept keys only;
//   * the survivors' paths are copied from their parents with the new
//     amplitude written at level k.
#include "common.hpp"
#include "kbest_common.hpp"

namespace mimo {

// marks (MIMO_FLAG_LEARNED_FALLBACK) the frames the fallback will detect again
__global__ void fallback_mark_kernel(const float* __restrict__ pd, uint32_t* __restrict__ flags,
                                     const float* __restrict__ sigma2, float beta, int n, int B)
{
    const int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= B) return;
    const uint32_t fl = flags[f];
    if (!kb_first_stands(fl, pd[f], sigma2[f], beta, n)) flags[f] = fl | MIMO_FLAG_LEARNED_FALLBACK;
}


// K-best of one frame by one wavefront; lds as sized by kbest_lds_bytes.
template <int P, int E>
__device__ __forceinline__ void kbest_frame(const KbestArgs& a, int frame, unsigned char* lds)
{
    using S = KbestShape<P, E>;
    constexpr int KCAP = S::KCAP, L = S::L, SPL = S::SPL;
    const int lane = threadIdx.x & 63;
    const int n = a.n;
    const int nw = kb_words(n), stride = kb_stride(n);
    uint32_t* path = reinterpret_cast<uint32_t*>(lds);
    float* spd = reinterpret_cast<float*>(path + 2 * KCAP * stride);
    float* rrow = spd + 2 * KCAP;
    int32_t* sel = reinterpret_cast<int32_t*>(rrow + 2 * nw + 4);
    uint64_t* skey = reinterpret_cast<uint64_t*>(sel + KCAP + (KCAP & 1));

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;
    const int32_t* fsym = a.force_sym ? a.force_sym + (size_t)frame * (n / 2) : nullptr;

    // zero paths: a half-word not yet written is multiplied by a zero of the
    // staged row and must be a finite number
    for (int i = lane; i < 2 * KCAP * stride; i += WAVE) path[i] = 0u;
    if (lane == 0) spd[0] = 0.f;
    int cnt = 1, fs = 0;
    int64_t expanded = 0;
    uint32_t flags = 0;
    __syncthreads();

    // software pipeline: row k-1 of R is loaded while level k is processed
    constexpr int RPL = 4;  // row entries per lane (n <= 256)
    float rnext[RPL];
    float rkk_next, zk_next;
    {
        const float* rk = Rf + r_row_off(n, n - 1);
#pragma unroll
        for (int i = 0; i < RPL; ++i) rnext[i] = (lane + WAVE * i < 1) ? rk[lane + WAVE * i] : 0.f;
        rkk_next = rk[0];
        zk_next = zf[n - 1];
    }

    for (int k = n - 1; k >= 0; --k) {
        const int cur = (n - 1 - k) & 1, nxt = cur ^ 1;
        uint32_t* pc = path + cur * KCAP * stride;
        uint32_t* pn = path + nxt * KCAP * stride;
        float* sc = spd + cur * KCAP;
        float* sn = spd + nxt * KCAP;
        // stage row k: rrow[j] = c R_kj for j > k, rrow[k] = 0
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int t = lane + WAVE * i;
            if (t < n - k) rrow[k + t] = t == 0 ? 0.f : cs * rnext[i];
        }
        const float rkk = cs * rkk_next;
        const float zk = zk_next;
        if (k > 0) {  // issue the loads of row k-1
            const float* rk = Rf + r_row_off(n, k - 1);
#pragma unroll
            for (int i = 0; i < RPL; ++i) {
                const int t = lane + WAVE * i;
                rnext[i] = t < n - k + 1 ? rk[t] : 0.f;
            }
            rkk_next = rk[0];
            zk_next = zf[k - 1];
        }
        kb_wave_sync();
        // cancellation centres: words from the one holding level k+1
        const int w0 = (k + 1) >> 1;
        float bu[SPL];
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const int s = (KCAP >= WAVE) ? lane + WAVE * u : lane / L;
            const int q = (L > 1) ? (lane % L) : 0;
            float acc = 0.f;
            if (s < cnt) {
                const uint32_t* prow = pc + s * stride;
                for (int wd = w0 + q; wd < nw; wd += L) {
                    const uint32_t d = prow[wd];
                    const float2 rr = *reinterpret_cast<const float2*>(rrow + 2 * wd);
                    acc = fmaf(rr.x, half_lo(d), acc);
                    acc = fmaf(rr.y, half_hi(d), acc);
                }
            }
#pragma unroll
            for (int m = 1; m < L; m <<= 1) acc += shfl_xor_f(acc, m);
            bu[u] = zk - acc;
        }
        // a NaN or infinity in R or z reaches every centre of the level
        bool bad = !kb_finite(rkk);
#pragma unroll
        for (int u = 0; u < SPL; ++u) {
            const int s = (KCAP >= WAVE) ? lane + WAVE * u : lane / L;
            bad = bad || (s < cnt && !kb_finite(bu[u]));
        }
        if (__ballot(bad)) {
            flags |= MIMO_FLAG_NONFINITE_INPUT;
            cnt = 0;
            break;
        }
        // children: key = (pd bits, candidate index s * P + c)
        uint32_t kh[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int m = e * WAVE + lane;
            const int s = m / P, c = m % P;
            const int u = (KCAP >= WAVE) ? (e / P) : 0;
            const int src = (KCAP >= WAVE) ? (s % WAVE) : (s * L);
            const float b = shfl_f(bu[u], src);
            kh[e] = ~0u;
            if (s < cnt) {
                const float ee = fmaf(-rkk, (float)(2 * c - (P - 1)), b);
                const float pdc = fmaf(ee, ee, sc[s]);
                if (pdc < r2) kh[e] = __float_as_uint(pdc);
            }
        }
        expanded += cnt;
        int nvalid = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e * WAVE < cnt * P) nvalid += __popcll(__ballot(kh[e] != ~0u));
        if (nvalid == 0) {
            flags |= MIMO_FLAG_EMPTY_SPHERE;
            cnt = 0;
            break;
        }
        int Kt = ks ? ks[k] : a.K;
        Kt = Kt > a.K ? a.K : (Kt < 1 ? 1 : Kt);

        int fm = -1;
        if (fsym) {
            const int sy = fsym[k >> 1];
            fm = fs * P + ((k & 1) ? (sy % P) : (sy / P));
            if (fs < 0) fm = -1;
        }
        int fpos = -1;
        int keep;
        if constexpr (E <= 2) {
            if (cnt * P <= WAVE)
                keep = kb_select_sort<E, 1>(kh, nvalid, Kt, fm, lane, sn, sel, &fpos);
            else
                keep = kb_select_sort<E, E>(kh, nvalid, Kt, fm, lane, sn, sel, &fpos);
        } else {
            keep = kb_select<E, (KCAP + WAVE - 1) / WAVE>(kh, cnt * P, nvalid, Kt, fm, lane, sn, sel, skey, &fpos);
        }
        if (fsym) {
            if (lane == 0) a.rank[(size_t)frame * n + k] = fpos + 1;
            fs = fpos >= 0 ? (fpos < keep ? fpos : keep - 1) : -1;
        }
        kb_wave_sync();
        // copy parent paths (words from the one holding level k) and write level k
        const int wk = k >> 1;
        const int nwk = nw - wk;
        int g = 1;  // survivors copied per pass: 64 / (words rounded up to a power of two)
        while (g * 2 * nwk <= WAVE && g < KCAP) g *= 2;
        const int span = WAVE / g;
        for (int i0 = 0; i0 < keep; i0 += g) {
            const int i = i0 + lane / span;
            if (i >= keep) continue;
            const int m = sel[i];
            const int s = m / P, c = m % P;
            for (int wd = wk + lane % span; wd < nw; wd += span) {
                uint32_t d = pc[s * stride + wd];
                if (wd == wk) {
                    const uint32_t hb = half_bits((float)(2 * c - (P - 1)));
                    d = (k & 1) ? ((d & 0x0000ffffu) | (hb << 16)) : ((d & 0xffff0000u) | hb);
                }
                pn[i * stride + wd] = d;
            }
        }
        kb_wave_sync();
        cnt = keep;
    }

    if (lane == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.fb_sigma2) flags |= MIMO_FLAG_LEARNED_FALLBACK;
        if (a.rerun) flags |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? spd[(n & 1) * KCAP] : INFINITY;
        if (a.counters) kb_write_counters(a, frame, expanded, P);
    }
    // outputs: survivor 0 of the last buffer is the best leaf
    const uint32_t* best = path + (n & 1) * KCAP * stride;
    if (!a.sym) return;
    for (int m = lane; m < n / 2; m += WAVE) {
        int v = 0;
        if (cnt > 0) {
            const uint32_t d = best[m];  // levels 2m (real part) and 2m+1 (imaginary part)
            const int ire = ((int)half_lo(d) + (P - 1)) / 2;
            const int iim = ((int)half_hi(d) + (P - 1)) / 2;
            v = ire * P + iim;
        }
        a.sym[(size_t)frame * (n / 2) + m] = v;
    }
}

// Register-path variant for KCAP <= 64 (L >= 1 lanes per survivor): lane
// (s, q) holds the path words w = q + L i (two fp16 amplitudes each) of
// survivor s in registers; after the selection each new survivor's lanes
// fetch the live words of their parent with cross-lane shuffles.  LDS holds
// only the staged row and the selection arrays.
template <int NWMAX>
__host__ __device__ inline size_t kbest_reg_lds_bytes(int kcap)
{
    return sizeof(float) * 2 * kcap + sizeof(float) * (2 * NWMAX + 16) + sizeof(int32_t) * kcap +
           sizeof(uint64_t) * 2 * WAVE;  // compaction buffer of the bounded selection
}

template <int P, int E, int NWMAX>
__device__ __forceinline__ void kbest_frame_reg(const KbestArgs& a, int frame, unsigned char* lds)
{
    using S = KbestShape<P, E>;
    constexpr int KCAP = S::KCAP, L = S::L;
    static_assert(KCAP <= 64, "register variant holds at most one survivor per lane");
    static_assert(NWMAX % L == 0, "a survivor's lanes share its path capacity evenly");
    constexpr int NWL = NWMAX / L;  // path words per lane
    constexpr int CHW = NWL < 8 ? NWL : 8;  // words per guarded chunk
    const int lane = threadIdx.x & 63;
    const int s_own = lane / L, q = lane % L;
    const int n = a.n;
    const int nw = n / 2;
    float* spd = reinterpret_cast<float*>(lds);
    float* rrow = spd + 2 * KCAP;
    int32_t* sel = reinterpret_cast<int32_t*>(rrow + 2 * NWMAX + 16);
    uint64_t* skey = reinterpret_cast<uint64_t*>(sel + KCAP);

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;
    const int32_t* fsym = a.force_sym ? a.force_sym + (size_t)frame * (n / 2) : nullptr;
    // the frame's R as one buffer: a row is loaded with one address and the
    // entry in the immediate offset; a lane past the end of the row reads the
    // next rows (or, past the frame, 0), which the staging never stores
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(Rf), 0, (int)r_packed_size(n) * (int)sizeof(float), 0x00020000);

    uint32_t pw[NWL];
#pragma unroll
    for (int i = 0; i < NWL; ++i) pw[i] = 0u;  // unassigned levels are amplitude 0
    for (int t = lane; t < 2 * NWMAX + 16; t += WAVE) rrow[t] = 0.f;
    if (lane == 0) spd[0] = 0.f;
    int cnt = 1, fs = 0;
    int64_t expanded = 0;
    uint32_t flags = 0;
    const int i_hi = (nw + L - 1) / L;  // words beyond nw read zero row entries

    constexpr int RPL = 4;
    float rnext[RPL];
    float rkk_next, zk_next;
    {
        const float* rk = Rf + r_row_off(n, n - 1);
#pragma unroll
        for (int i = 0; i < RPL; ++i) rnext[i] = (lane + WAVE * i < 1) ? rk[lane + WAVE * i] : 0.f;
        rkk_next = rk[0];
        zk_next = zf[n - 1];
    }
    __syncthreads();

    for (int k = n - 1; k >= 0; --k) {
        const int cur = (n - 1 - k) & 1, nxt = cur ^ 1;
        float* sc = spd + cur * KCAP;
        float* sn = spd + nxt * KCAP;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int t = lane + WAVE * i;
            if (t < n - k) rrow[k + t] = t == 0 ? 0.f : cs * rnext[i];
        }
        const float rkk = cs * rkk_next;
        const float zk = zk_next;
        if (k > 0) {
            const float* rk = Rf + r_row_off(n, k - 1);
            const int v = 4 * ((int)r_row_off(n, k - 1) + lane);
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                rnext[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, v + 4 * WAVE * i, 0, 0));
            rkk_next = rk[0];
            zk_next = zf[k - 1];
        }
        kb_wave_sync();
        // centre of this lane's survivor: levels <= k hold amplitude 0 and
        // rrow[k] = 0, so whole words can be summed from the one of level k+1
        // words are taken in chunks of CHW: a word below the live range holds
        // amplitude 0 (a level not yet fixed) and a word beyond nw meets zero
        // row entries, so whole chunks can be summed
        const int i_lo = ((k + 1) >> 1) / L;
        // four partial sums (by word parity and half) keep the FMA chains short
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > i_lo && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW && i < NWL; ++i) {
                    const float2 rr = *reinterpret_cast<const float2*>(rrow + 2 * (q + L * i));
                    if (i & 1) {
                        a2 = fmaf(rr.x, half_lo(pw[i]), a2);
                        a3 = fmaf(rr.y, half_hi(pw[i]), a3);
                    } else {
                        a0 = fmaf(rr.x, half_lo(pw[i]), a0);
                        a1 = fmaf(rr.y, half_hi(pw[i]), a1);
                    }
                }
            }
        }
        float acc = (a0 + a1) + (a2 + a3);
#pragma unroll
        for (int m = 1; m < L; m <<= 1) acc += shfl_xor_f(acc, m);
        const float bown = zk - acc;
        // a NaN or infinity in R or z reaches every centre of the level
        if (__ballot(!kb_finite(rkk) || (s_own < cnt && !kb_finite(bown)))) {
            flags |= MIMO_FLAG_NONFINITE_INPUT;
            cnt = 0;
            break;
        }
        uint32_t kh[E];
        const int ncand = cnt * P;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            kh[e] = ~0u;
            if (e * WAVE >= ncand) continue;  // block without candidates (uniform)
            const int m = e * WAVE + lane;
            const int s = m / P, c = m % P;
            const float b = shfl_f(bown, s * L);
            if (s < cnt) {
                const float ee = fmaf(-rkk, (float)(2 * c - (P - 1)), b);
                const float pdc = fmaf(ee, ee, sc[s]);
                if (pdc < r2) kh[e] = __float_as_uint(pdc);
            }
        }
        expanded += cnt;
        int nvalid = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e * WAVE < cnt * P) nvalid += __popcll(__ballot(kh[e] != ~0u));
        if (nvalid == 0) {
            flags |= MIMO_FLAG_EMPTY_SPHERE;
            cnt = 0;
            break;
        }
        int Kt = ks ? ks[k] : a.K;
        Kt = Kt > a.K ? a.K : (Kt < 1 ? 1 : Kt);
        Kt = Kt > KCAP ? KCAP : Kt;  // the instantiation's survivor capacity
        int fm = -1;
        if (fsym && fs >= 0) {
            const int sy = fsym[k >> 1];
            fm = fs * P + ((k & 1) ? (sy % P) : (sy / P));
        }
        int fpos = -1;
        int keep;
        if constexpr (E <= 2) {
            // the candidates sit in lanes 0 .. cnt P - 1: sort only as many lanes
            if (cnt * P <= 32)
                keep = kb_select_sort<E, 1, 32>(kh, nvalid, Kt, fm, lane, sn, sel, &fpos);
            else if (cnt * P <= WAVE)
                keep = kb_select_sort<E, 1>(kh, nvalid, Kt, fm, lane, sn, sel, &fpos);
            else
                keep = kb_select_sort<E, E>(kh, nvalid, Kt, fm, lane, sn, sel, &fpos);
        } else {
            keep = kb_select_merge<E, P>(kh, cnt * P, nvalid, Kt, fm, lane, sn, sel, skey, &fpos);
        }
        if (fsym) {
            if (lane == 0) a.rank[(size_t)frame * n + k] = fpos + 1;
            fs = fpos >= 0 ? (fpos < keep ? fpos : keep - 1) : -1;
        }
        kb_wave_sync();
        // new survivor s_own takes its parent's words (those holding levels >= k)
        int src = lane, cnew = 0;
        if (s_own < keep) {
            const int m = sel[s_own];
            src = (m / P) * L + q;
            cnew = m % P;
        }
        const int wk = k >> 1, ik = wk / L;
        // (words below level k hold zeros for every survivor: moving them is harmless)
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > ik && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW && i < NWL; ++i) pw[i] = (uint32_t)__shfl((int)pw[i], src, WAVE);
            }
        }
        if (s_own < keep && q == wk % L) {
            const uint32_t hb = half_bits((float)(2 * cnew - (P - 1)));
            // only the chunk holding word ik is visited (uniform guard)
#pragma unroll
            for (int c0 = 0; c0 < NWL; c0 += CHW) {
                if (ik >= c0 && ik < c0 + CHW) {
#pragma unroll
                    for (int i = c0; i < c0 + CHW && i < NWL; ++i)
                        if (i == ik)
                            pw[i] = (k & 1) ? ((pw[i] & 0x0000ffffu) | (hb << 16)) : ((pw[i] & 0xffff0000u) | hb);
                }
            }
        }
        cnt = keep;
    }

    if (lane == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.fb_sigma2) flags |= MIMO_FLAG_LEARNED_FALLBACK;
        if (a.rerun) flags |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? spd[(n & 1) * KCAP] : INFINITY;
        if (a.counters) kb_write_counters(a, frame, expanded, P);
    }
    // survivor 0 (lanes 0 .. L-1) is the best leaf; word w holds symbol w
    if (!a.sym || s_own != 0) return;
#pragma unroll
    for (int i = 0; i < NWL; ++i) {
        const int w = q + L * i;
        if (w < nw) {
            int v = 0;
            if (cnt > 0) {
                const int ire = ((int)half_lo(pw[i]) + (P - 1)) / 2;
                const int iim = ((int)half_hi(pw[i]) + (P - 1)) / 2;
                v = ire * P + iim;
            }
            a.sym[(size_t)frame * nw + w] = v;
        }
    }
}

// K-best over complex levels (the paper's own tree, Sec. III-B: one complex
// symbol, i.e. P^2 children, per level).  Complex level m fixes the real
// levels k_hi = 2m + 1 (imaginary part) and k_lo = 2m (real part); the
// interleaved real model has R[k_lo][k_hi] = 0, so both centres depend on the
// levels above k_hi only and are computed together.  Child c = i_im P + i_re
// of survivor s has pd' = pd_s + (b_hi - R_hi a_im)^2 + (b_lo - R_lo a_re)^2
// (added in that order); the key is (pd', s P^2 + c).  One wavefront per
// frame, survivor paths in registers as in the real-level variant (lane
// (s, q) holds words q + L i), candidate blocks of 64 selected by sorting and
// merging.  K_t = k_sched[k_lo].
template <int P, int E>
struct KbestCplxShape {
    static constexpr int PC = P * P;                       // children per survivor
    static constexpr int KCAP = WAVE * E / PC;             // survivor capacity
    static constexpr int L = WAVE / KCAP;                  // lanes per survivor
};

template <int NWMAX>
__host__ __device__ inline size_t kbest_cplx_lds_bytes(int kcap)
{
    const int L = WAVE / kcap;
    const int nwx = NWMAX > L ? NWMAX : L;
    return sizeof(uint64_t) * 2 * WAVE + sizeof(float) * 2 * kcap + sizeof(float) * 2 * (2 * nwx + 16) +
           sizeof(int32_t) * kcap;
}

template <int P, int E, int NWMAX>
__device__ __forceinline__ void kbest_frame_cplx(const KbestArgs& a, int frame, unsigned char* lds)
{
    using S = KbestCplxShape<P, E>;
    constexpr int PC = S::PC, KCAP = S::KCAP, L = S::L;
    static_assert(KCAP >= 1 && KCAP <= 64, "one survivor per lane at most, one at least");
    constexpr int NWX = NWMAX > L ? NWMAX : L;  // words covered by the lanes of a survivor
    constexpr int NWL = NWX / L;                // path words per lane
    constexpr int CHW = NWL < 8 ? NWL : 8;      // words per guarded chunk
    constexpr int RW = 2 * NWX + 16;            // staged row length
    const int lane = threadIdx.x & 63;
    const int s_own = lane / L, q = lane % L;
    const int n = a.n;
    const int nw = n / 2;
    uint64_t* skey = reinterpret_cast<uint64_t*>(lds);  // compaction buffer of the bounded selection
    float* spd = reinterpret_cast<float*>(skey + 2 * WAVE);
    float* rhi = spd + 2 * KCAP;  // c R[k_hi][j], zero at j <= k_hi
    float* rlo = rhi + RW;        // c R[k_lo][j], zero at j <= k_hi
    int32_t* sel = reinterpret_cast<int32_t*>(rlo + RW);

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;

    uint32_t pw[NWL];
#pragma unroll
    for (int i = 0; i < NWL; ++i) pw[i] = 0u;  // unassigned levels are amplitude 0
    for (int t = lane; t < 2 * RW; t += WAVE) rhi[t] = 0.f;
    if (lane == 0) spd[0] = 0.f;
    int cnt = 1;
    int64_t expanded = 0;
    uint32_t flags = 0;
    const int i_hi = (nw + L - 1) / L;  // words beyond nw read zero row entries

    // rows k_hi, k_lo of the next complex level are loaded while the current one is used
    constexpr int RPL = 4;
    float nh[RPL], nl[RPL];
    float rkh_next, rkl_next, zh_next, zl_next;
    auto load_rows = [&](int m) {
        const float* rh = Rf + r_row_off(n, 2 * m + 1);
        const float* rl = Rf + r_row_off(n, 2 * m);
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int t = lane + WAVE * i;
            nh[i] = t < n - 2 * m - 1 ? rh[t] : 0.f;
            nl[i] = t < n - 2 * m ? rl[t] : 0.f;
        }
        rkh_next = rh[0];
        rkl_next = rl[0];
        zh_next = zf[2 * m + 1];
        zl_next = zf[2 * m];
    };
    load_rows(nw - 1);
    __syncthreads();

    for (int m = nw - 1; m >= 0; --m) {
        const int k_hi = 2 * m + 1, k_lo = 2 * m;
        const int cur = (nw - 1 - m) & 1, nxt = cur ^ 1;
        float* sc = spd + cur * KCAP;
        float* sn = spd + nxt * KCAP;
        // stage: row k_hi from column k_hi, row k_lo from column k_lo (its
        // entry at k_hi is the structural zero); entries at and below the
        // complex level meet amplitude 0 in every path
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int t = lane + WAVE * i;
            if (t < n - k_hi) rhi[k_hi + t] = t == 0 ? 0.f : cs * nh[i];
            if (t < n - k_lo) rlo[k_lo + t] = t <= 1 ? 0.f : cs * nl[i];
        }
        const float rkh = cs * rkh_next, rkl = cs * rkl_next;
        const float zh = zh_next, zl = zl_next;
        if (m > 0) load_rows(m - 1);
        kb_wave_sync();
        // centres of this lane's survivor from the words above word m
        const int i_lo = (m + 1) / L;
        float ah = 0.f, al = 0.f, ah2 = 0.f, al2 = 0.f;  // partial sums by half: shorter FMA chains
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > i_lo && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW; ++i) {
                    const int w = q + L * i;
                    const float2 rh = *reinterpret_cast<const float2*>(rhi + 2 * w);
                    const float2 rl = *reinterpret_cast<const float2*>(rlo + 2 * w);
                    const float xl = half_lo(pw[i]), xh = half_hi(pw[i]);
                    ah = fmaf(rh.x, xl, ah);
                    ah2 = fmaf(rh.y, xh, ah2);
                    al = fmaf(rl.x, xl, al);
                    al2 = fmaf(rl.y, xh, al2);
                }
            }
        }
        ah += ah2;
        al += al2;
#pragma unroll
        for (int j = 1; j < L; j <<= 1) {
            ah += shfl_xor_f(ah, j);
            al += shfl_xor_f(al, j);
        }
        const float bh_own = zh - ah, bl_own = zl - al;
        // a NaN or infinity in R or z reaches every centre of the level
        if (__ballot(!kb_finite(rkh) || !kb_finite(rkl) ||
                     (s_own < cnt && !(kb_finite(bh_own) && kb_finite(bl_own))))) {
            flags |= MIMO_FLAG_NONFINITE_INPUT;
            cnt = 0;
            break;
        }
        uint32_t kh[E];
        const int ncand = cnt * PC;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            kh[e] = ~0u;
            if (e * WAVE >= ncand) continue;  // block without candidates (uniform)
            const int mm = e * WAVE + lane;
            const int s = mm / PC, c = mm % PC;
            const float bh = shfl_f(bh_own, s * L), bl = shfl_f(bl_own, s * L);
            if (s < cnt) {
                const float eh = fmaf(-rkh, (float)(2 * (c / P) - (P - 1)), bh);
                const float el = fmaf(-rkl, (float)(2 * (c % P) - (P - 1)), bl);
                const float pdc = fmaf(el, el, fmaf(eh, eh, sc[s]));
                if (pdc < r2) kh[e] = __float_as_uint(pdc);
            }
        }
        expanded += cnt;
        int nvalid = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e * WAVE < ncand) nvalid += __popcll(__ballot(kh[e] != ~0u));
        if (nvalid == 0) {
            flags |= MIMO_FLAG_EMPTY_SPHERE;
            cnt = 0;
            break;
        }
        int Kt = ks ? ks[k_lo] : a.K;
        Kt = Kt > a.K ? a.K : (Kt < 1 ? 1 : Kt);
        int fpos = -1;
        int keep;
        if constexpr (E <= 2) {
            if (ncand <= WAVE)
                keep = kb_select_sort<E, 1>(kh, nvalid, Kt, -1, lane, sn, sel, &fpos);
            else
                keep = kb_select_sort<E, E>(kh, nvalid, Kt, -1, lane, sn, sel, &fpos);
        } else {
            keep = kb_select_merge<E, PC>(kh, ncand, nvalid, Kt, -1, lane, sn, sel, skey, &fpos);
        }
        kb_wave_sync();
        // new survivor s_own takes its parent's words above word m and writes word m
        int src = lane, cnew = 0;
        if (s_own < keep) {
            const int mm = sel[s_own];
            src = (mm / PC) * L + q;
            cnew = mm % PC;
        }
        const int im = m / L;
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > im && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW; ++i) pw[i] = (uint32_t)__shfl((int)pw[i], src, WAVE);
            }
        }
        if (s_own < keep && q == m % L) {
            const uint32_t wd = half_bits((float)(2 * (cnew % P) - (P - 1))) |
                                (half_bits((float)(2 * (cnew / P) - (P - 1))) << 16);
#pragma unroll
            for (int c0 = 0; c0 < NWL; c0 += CHW) {
                if (im >= c0 && im < c0 + CHW) {
#pragma unroll
                    for (int i = c0; i < c0 + CHW; ++i)
                        if (i == im) pw[i] = wd;
                }
            }
        }
        cnt = keep;
    }

    if (lane == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.rerun) flags |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? spd[(nw & 1) * KCAP] : INFINITY;
        if (a.counters) kb_write_counters(a, frame, expanded, PC * 2);  // real-level evaluations
    }
    // survivor 0 (lanes 0 .. L-1) is the best leaf; word w holds symbol w
    if (!a.sym || s_own != 0) return;
#pragma unroll
    for (int i = 0; i < NWL; ++i) {
        const int w = q + L * i;
        if (w < nw) {
            int v = 0;
            if (cnt > 0) {
                const int ire = ((int)half_lo(pw[i]) + (P - 1)) / 2;
                const int iim = ((int)half_hi(pw[i]) + (P - 1)) / 2;
                v = ire * P + iim;
            }
            a.sym[(size_t)frame * nw + w] = v;
        }
    }
}

template <int P, int E, int NWMAX>
__global__ void __launch_bounds__(64) kbest_cplx_kernel(KbestArgs a)
{
    extern __shared__ unsigned char smem_kbc[];
    if (kb_keep_first(a, blockIdx.x)) return;
    kbest_frame_cplx<P, E, NWMAX>(a, blockIdx.x, smem_kbc);
}

template <int P, int E>
static int32_t launch_kbest_cplx(const KbestArgs& a, int B, hipStream_t st)
{
    constexpr int KCAP = KbestCplxShape<P, E>::KCAP;
    if (a.n <= 64)
        hipLaunchKernelGGL((kbest_cplx_kernel<P, E, 32>), dim3(B), dim3(WAVE), kbest_cplx_lds_bytes<32>(KCAP), st, a);
    else
        hipLaunchKernelGGL((kbest_cplx_kernel<P, E, 128>), dim3(B), dim3(WAVE), kbest_cplx_lds_bytes<128>(KCAP), st,
                           a);
    return check_launch("kbest_detect_complex");
}

// smallest block count E (a power of two) with 64 E >= K P^2 candidates
template <int P>
static int32_t dispatch_kbest_cplx_p(const KbestArgs& a, int B, hipStream_t st)
{
    const int need = a.K * P * P;
    if constexpr (P == 2) {
        if (need <= 64) return launch_kbest_cplx<2, 1>(a, B, st);
        if (need <= 128) return launch_kbest_cplx<2, 2>(a, B, st);
        return launch_kbest_cplx<2, 4>(a, B, st);
    } else {
        if (need <= 64) return launch_kbest_cplx<P, 1>(a, B, st);
        if (need <= 128) return launch_kbest_cplx<P, 2>(a, B, st);
        if (need <= 256) return launch_kbest_cplx<P, 4>(a, B, st);
        if (need <= 512) return launch_kbest_cplx<P, 8>(a, B, st);
        return launch_kbest_cplx<P, 16>(a, B, st);
    }
}

template <int P, int E, int NWMAX>
__global__ void __launch_bounds__(64) kbest_reg_kernel(KbestArgs a)
{
    extern __shared__ unsigned char smem_kbr[];
    if (kb_keep_first(a, blockIdx.x)) return;
    kbest_frame_reg<P, E, NWMAX>(a, blockIdx.x, smem_kbr);
}

// K-best with at most 8 survivors and P = 8 (at most 64 candidates per
// level), two frames per wavefront: the learned detector's case, where most
// levels have at most four survivors, so that one frame's candidates fill
// half a wave and a 32-lane sort.  Lanes 32h .. 32h+31 hold frame 2b+h:
// four lanes per survivor (path words q + 4i in registers), one or two
// candidates per lane (two while some frame of the pair has more than four
// survivors), sorted within the half.  Keys and the tie rule are those of
// the one-frame kernels; a centre is summed over four lanes instead of
// eight, which can move a pd by an FP32 rounding.
constexpr int PR_P = 8;
constexpr int PR_KCAP = 8;                 // survivors per frame
constexpr int PR_HALF = WAVE / 2;          // lanes per frame
constexpr int PR_L = PR_HALF / PR_KCAP;    // lanes per survivor

// bitonic sort within each half of the wave, ascending in lane & 31
__device__ __forceinline__ void pr_sort32(uint64_t& key, int lane)
{
    const int h = lane & (PR_HALF - 1);
#pragma unroll
    for (int size = 2; size <= PR_HALF; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            const uint64_t o = xor_lanes_u64(key, j, lane);
            const bool take_max = ((h & size) != 0) != ((h & j) != 0);
            key = ((o < key) != take_max) ? o : key;
        }
    }
}

// bitonic sort of 64 keys per half, element 32 r + (lane & 31) in key[r]:
// ascending, so key[0] ends with the 32 smallest
__device__ __forceinline__ void pr_sort64(uint64_t (&key)[2], int lane)
{
    const int h = lane & (PR_HALF - 1);
#pragma unroll
    for (int size = 2; size <= 2 * PR_HALF; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            if (j == PR_HALF) {  // elements h and 32 + h sit in one lane (size = 64: ascending)
                const uint64_t lo = key[1] < key[0] ? key[1] : key[0];
                const uint64_t hi = key[1] < key[0] ? key[0] : key[1];
                key[0] = lo;
                key[1] = hi;
            } else {
#pragma unroll
                for (int r = 0; r < 2; ++r) {
                    const int x = PR_HALF * r + h;
                    const uint64_t o = xor_lanes_u64(key[r], j, lane);
                    const bool take_max = ((x & size) != 0) != ((x & j) != 0);
                    key[r] = ((o < key[r]) != take_max) ? o : key[r];
                }
            }
        }
    }
}

template <int NWMAX>
__host__ __device__ inline size_t kbest_pair_lds_bytes()
{
    return 2 * sizeof(float) * (3 * PR_KCAP + 2 * NWMAX + 16);  // per frame: pd [2][8], sel [8], R row
}

template <int NWMAX>
__global__ void __launch_bounds__(WAVE) kbest_pair_kernel(KbestArgs a, int B)
{
    constexpr int P = PR_P, KCAP = PR_KCAP, L = PR_L;
    constexpr int NWL = NWMAX / L;                     // path words per lane
    constexpr int CHW = NWL < 8 ? NWL : 8;             // words per guarded chunk
    constexpr int RPL = (2 * NWMAX + PR_HALF - 1) / PR_HALF;  // row entries per lane (n <= 2 NWMAX)
    constexpr int HW = 3 * KCAP + 2 * NWMAX + 16;      // LDS words per frame
    static_assert(NWMAX % L == 0, "a survivor's lanes share its path capacity evenly");
    extern __shared__ __align__(16) unsigned char smem_kp[];
    const int lane = threadIdx.x & 63, half = lane / PR_HALF, hl = lane % PR_HALF;
    const int fr = 2 * (int)blockIdx.x + half;
    const bool live = fr < B;
    const int frame = live ? fr : B - 1;  // a half beyond the batch repeats the last frame, storing nothing
    const int s_own = hl / L, q = hl % L;
    const int n = a.n, nw = n / 2;
    float* spd = reinterpret_cast<float*>(smem_kp) + half * HW;  // [2][KCAP] survivor pd by level parity
    int32_t* sel = reinterpret_cast<int32_t*>(spd + 2 * KCAP);   // [KCAP]
    float* rrow = spd + 3 * KCAP;                                // [2 NWMAX + 16] staged R row

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;
    const uint64_t hmask = half ? 0xffffffff00000000ull : 0x00000000ffffffffull;
    // the R rows of the wave's two frames as one buffer: a row is loaded with
    // one address and the entry in the immediate offset; a lane past the end
    // of the row reads the next rows (or, past the buffer, 0), which the
    // staging below never stores
    const int f0 = 2 * (int)blockIdx.x;
    const int rsz = (int)r_packed_size(n);
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(a.R + (size_t)f0 * rsz), 0, (B - f0 < 2 ? B - f0 : 2) * rsz * (int)sizeof(float),
        0x00020000);
    const int fb = (frame - f0) * rsz;

    uint32_t pw[NWL];
#pragma unroll
    for (int i = 0; i < NWL; ++i) pw[i] = 0u;  // unassigned levels are amplitude 0
    for (int t = hl; t < 2 * NWMAX + 16; t += PR_HALF) rrow[t] = 0.f;
    if (hl == 0) spd[0] = 0.f;
    int cnt = 1;
    int64_t expanded = 0;
    uint32_t flags = 0;
    const int i_hi = (nw + L - 1) / L;  // words beyond nw read zero row entries

    float rnext[RPL];
    float rkk_next, zk_next;
    {
        const float* rk = Rf + r_row_off(n, n - 1);
#pragma unroll
        for (int i = 0; i < RPL; ++i) rnext[i] = (hl + PR_HALF * i < 1) ? rk[hl + PR_HALF * i] : 0.f;
        rkk_next = rk[0];
        zk_next = zf[n - 1];
    }
    kb_wave_sync();

    for (int k = n - 1; k >= 0; --k) {
        const int cur = (n - 1 - k) & 1;
        const float* sc = spd + cur * KCAP;
        float* sn = spd + (cur ^ 1) * KCAP;
#pragma unroll
        for (int i = 0; i < RPL; ++i) {
            const int t = hl + PR_HALF * i;
            if (t < n - k) rrow[k + t] = t == 0 ? 0.f : cs * rnext[i];
        }
        const float rkk = cs * rkk_next;
        const float zk = zk_next;
        if (k > 0) {
            const float* rk = Rf + r_row_off(n, k - 1);
            const int v = 4 * (fb + (int)r_row_off(n, k - 1) + hl);
#pragma unroll
            for (int i = 0; i < RPL; ++i)
                rnext[i] = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(rs, v + 4 * PR_HALF * i, 0, 0));
            rkk_next = rk[0];
            zk_next = zf[k - 1];
        }
        kb_wave_sync();
        // centre of this lane's survivor (levels <= k hold amplitude 0 and rrow[k] = 0)
        const int i_lo = ((k + 1) >> 1) / L;
        float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > i_lo && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW && i < NWL; ++i) {
                    const float2 rr = *reinterpret_cast<const float2*>(rrow + 2 * (q + L * i));
                    if (i & 1) {
                        a2 = fmaf(rr.x, half_lo(pw[i]), a2);
                        a3 = fmaf(rr.y, half_hi(pw[i]), a3);
                    } else {
                        a0 = fmaf(rr.x, half_lo(pw[i]), a0);
                        a1 = fmaf(rr.y, half_hi(pw[i]), a1);
                    }
                }
            }
        }
        float acc = (a0 + a1) + (a2 + a3);
        acc += shfl_xor_f(acc, 1);
        acc += shfl_xor_f(acc, 2);
        const float bown = zk - acc;
        // a NaN or infinity in this frame's R or z reaches every centre of the
        // level: the frame ends here (its partner goes on)
        const bool bad = (__ballot(!kb_finite(rkk) || (s_own < cnt && !kb_finite(bown))) & hmask) != 0;
        if (bad && cnt > 0) {
            flags |= MIMO_FLAG_NONFINITE_INPUT;
            cnt = 0;
        }
        // candidates m = hl (and 32 + hl): child m % P of survivor m / P
        const int cmax = max(cnt, (int)xor_lanes((uint32_t)cnt, PR_HALF, lane));
        const bool two = cmax * P > PR_HALF;  // the same in both halves
        uint64_t key[2] = {~0ull, ~0ull};
        int nvalid = 0;
#pragma unroll
        for (int e = 0; e < 2; ++e) {
            if (e == 1 && !two) break;
            const int m = PR_HALF * e + hl;
            const int s = m / P, c = m % P;
            const float b = shfl_f(bown, PR_HALF * half + s * L);
            uint32_t kh = ~0u;
            if (s < cnt) {
                const float ee = fmaf(-rkk, (float)(2 * c - (P - 1)), b);
                const float pdc = fmaf(ee, ee, sc[s]);
                if (pdc < r2) kh = __float_as_uint(pdc);
            }
            nvalid += __popcll(__ballot(kh != ~0u) & hmask);
            key[e] = kh == ~0u ? ~0ull : (((uint64_t)kh << 32) | (uint32_t)m);
        }
        expanded += cnt;
        if (cnt > 0 && nvalid == 0) flags |= MIMO_FLAG_EMPTY_SPHERE;  // this frame ends here
        int Kt = ks ? ks[k] : a.K;
        Kt = Kt > a.K ? a.K : (Kt < 1 ? 1 : Kt);
        const int keep = Kt < nvalid ? Kt : nvalid;
        if (two) pr_sort64(key, lane);
        else pr_sort32(key[0], lane);
        if (hl < keep) {
            sn[hl] = __uint_as_float((uint32_t)(key[0] >> 32));
            sel[hl] = (int32_t)(uint32_t)key[0];
        }
        kb_wave_sync();
        // new survivor s_own takes its parent's words (those holding levels >= k)
        int src = lane, cnew = 0;
        if (s_own < keep) {
            const int m = sel[s_own];
            src = PR_HALF * half + (m / P) * L + q;
            cnew = m % P;
        }
        const int wk = k >> 1, ik = wk / L;
#pragma unroll
        for (int c0 = 0; c0 < NWL; c0 += CHW) {
            if (c0 + CHW > ik && c0 < i_hi) {
#pragma unroll
                for (int i = c0; i < c0 + CHW && i < NWL; ++i) pw[i] = (uint32_t)__shfl((int)pw[i], src, WAVE);
            }
        }
        if (s_own < keep && q == wk % L) {
            const uint32_t hb = half_bits((float)(2 * cnew - (P - 1)));
#pragma unroll
            for (int c0 = 0; c0 < NWL; c0 += CHW) {
                if (ik >= c0 && ik < c0 + CHW) {
#pragma unroll
                    for (int i = c0; i < c0 + CHW && i < NWL; ++i)
                        if (i == ik)
                            pw[i] = (k & 1) ? ((pw[i] & 0x0000ffffu) | (hb << 16)) : ((pw[i] & 0xffff0000u) | hb);
                }
            }
        }
        cnt = keep;
    }

    if (live && hl == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? spd[(n & 1) * KCAP] : INFINITY;
        if (a.counters) kb_write_counters(a, frame, expanded, P);
    }
    // survivor 0 (lanes 32h .. 32h+3) is the best leaf; word w holds symbol w
    if (!live || !a.sym || s_own != 0) return;
#pragma unroll
    for (int i = 0; i < NWL; ++i) {
        const int w = q + L * i;
        if (w < nw) {
            int v = 0;
            if (cnt > 0) {
                const int ire = ((int)half_lo(pw[i]) + (P - 1)) / 2;
                const int iim = ((int)half_hi(pw[i]) + (P - 1)) / 2;
                v = ire * P + iim;
            }
            a.sym[(size_t)frame * nw + w] = v;
        }
    }
}

template <int P, int E>
static int32_t launch_kbest_reg(const KbestArgs& a, int B, hipStream_t st)
{
    using S = KbestShape<P, E>;
    // path capacity (words) by frame size: the lanes of a survivor sum and move
    // whole chunks of words, so a capacity close to n / 2 wastes the least
    if (a.n <= 64) {
        hipLaunchKernelGGL((kbest_reg_kernel<P, E, 32>), dim3(B), dim3(WAVE), kbest_reg_lds_bytes<32>(S::KCAP), st, a);
    } else if (a.n <= 208) {
        hipLaunchKernelGGL((kbest_reg_kernel<P, E, 104>), dim3(B), dim3(WAVE), kbest_reg_lds_bytes<104>(S::KCAP), st,
                           a);
    } else {
        hipLaunchKernelGGL((kbest_reg_kernel<P, E, 128>), dim3(B), dim3(WAVE), kbest_reg_lds_bytes<128>(S::KCAP), st,
                           a);
    }
    return check_launch("kbest_detect");
}

template <int P, int E>
__global__ void __launch_bounds__(64) kbest_kernel(KbestArgs a)
{
    extern __shared__ unsigned char smem_kb[];
    if (kb_keep_first(a, blockIdx.x)) return;
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

template <int P, int E>
static int32_t launch_kbest_any(const KbestArgs& a, int B, hipStream_t st)
{
    if constexpr (KbestShape<P, E>::KCAP <= 64) return launch_kbest_reg<P, E>(a, B, st);
    else return launch_kbest<P, E>(a, B, st);
}

template <int P>
static int32_t dispatch_kbest_p(const KbestArgs& a, int B, hipStream_t st)
{
    const int need = a.K * P;  // candidates per level
    if constexpr (P == PR_P) {
        // at most 8 survivors of 64-QAM, 64 < n <= 208, detection mode: two frames per wavefront
        if (need <= 64 && a.n > 64 && a.n <= 208 && !a.fb_sigma2 && !a.force_sym && !a.rerun) {
            hipLaunchKernelGGL(kbest_pair_kernel<104>, dim3((B + 1) / 2), dim3(WAVE), kbest_pair_lds_bytes<104>(), st,
                               a, B);
            return check_launch("kbest_detect");
        }
    }
    if (need <= 64) return launch_kbest_any<P, 1>(a, B, st);
    if (need <= 128) return launch_kbest_any<P, 2>(a, B, st);
    if (need <= 256) return launch_kbest_any<P, 4>(a, B, st);
    if (need <= 512) return launch_kbest_any<P, 8>(a, B, st);
    return launch_kbest_any<P, 16>(a, B, st);
}

// Real-level K-best: the grouped kernel (interference above each group of 16
// levels from one matrix product, paths as group segments) is faster on
// gfx950 for K <= 64 at every measured shape but two, which keep the
// row-recompute kernels: at most 8 survivors of 64-QAM at 64 < n <= 208
// (two frames per wavefront), and K pam > 64 at n <= 8.  With a per-level
// schedule it is faster too (32x32 16-QAM with the learned schedule, cap 64
// and mean K_t 14: 1.77 against 2.30 ms; 1.06-2.7x at 10x10 to 64x64 with
// caps 16 and 64), except for a cap of 9 to 16 survivors of 64-QAM: its two
// blocks of children per lane allow no bound, so both are sorted at every
// level, while the row-recompute kernels sort only the blocks the level's
// survivors fill (16x16, K_t 2-6: 0.32 against 0.27 ms).  Label mode (forced
// path and rank output) is served by the row-recompute kernels only.
static bool grouped_real_preferred(const KbestArgs& a, int pam)
{
    if (a.force_sym || a.K > 64) return false;
    if (pam == 8 && a.K <= 8 && a.n > 64 && a.n <= 208 && !a.fb_sigma2 && !a.rerun) return false;
    if (a.n <= 8 && a.K * pam > 64) return false;
    if (a.k_sched && pam == 8 && a.K > 8 && a.K <= 16) return false;
    return true;
}

static int32_t dispatch_kbest(const KbestArgs& a, int pam, int B, hipStream_t st)
{
    if (grouped_real_preferred(a, pam)) return dispatch_grouped(a, pam, 1, B, st);
    switch (pam) {
    case 2: return dispatch_kbest_p<2>(a, B, st);
    case 4: return dispatch_kbest_p<4>(a, B, st);
    default: return dispatch_kbest_p<8>(a, B, st);
    }
}

// LDS bytes of the survivor-list (LDS) variant the dispatch picks for K
// survivors of P points at n levels; 0 for the register variants, whose LDS
// need is a few KB at any n
template <int P, int E>
static size_t lds_need_pe(int n)
{
    if constexpr (KbestShape<P, E>::KCAP <= 64) return 0;
    else return kbest_lds_bytes<P, E>(n);
}

template <int P>
static size_t kbest_lds_need_p(int K, int n)
{
    const int need = K * P;
    if (need <= 64) return lds_need_pe<P, 1>(n);
    if (need <= 128) return lds_need_pe<P, 2>(n);
    if (need <= 256) return lds_need_pe<P, 4>(n);
    if (need <= 512) return lds_need_pe<P, 8>(n);
    return lds_need_pe<P, 16>(n);
}

static size_t kbest_lds_need(int pam, int K, int n)
{
    return pam == 2 ? kbest_lds_need_p<2>(K, n) : (pam == 4 ? kbest_lds_need_p<4>(K, n) : kbest_lds_need_p<8>(K, n));
}

constexpr size_t LDS_PER_CU = 160 * 1024;

static int32_t validate_common(const char* who, int B, int n_tx, int pam, int K)
{
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", who);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", who);
    if (n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: n_tx < 1", who);
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx > %d", who, MIMO_MAX_TX);
    if (K < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: K < 1", who);
    if (K > MIMO_MAX_K || K * pam > 1024)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: K <= %d and K * pam <= 1024", who, MIMO_MAX_K);
    const size_t lds = kbest_lds_need(pam, K, 2 * n_tx);
    if (lds > LDS_PER_CU)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: K = %d survivors of %d levels need %zu bytes of LDS (> %zu)", who, K,
                    2 * n_tx, lds, LDS_PER_CU);
    return MIMO_OK;
}

// frames whose finite radius left no leaf are detected again with r2 = +inf
static int32_t rerun_empty(const KbestArgs& a, int pam, int B, hipStream_t st, bool complex_levels);

// Complex-level K-best: the grouped kernel with J = 2 from 512 candidates
// per level (K pam^2) or 128 real levels on, where it measured faster; the
// row-recompute kernel below that.
static int32_t dispatch_kbest_complex(const KbestArgs& a, int pam, int B, hipStream_t st)
{
    if (a.K * pam * pam >= 512 || a.n >= 128) return dispatch_grouped(a, pam, 2, B, st);
    switch (pam) {
    case 2: return dispatch_kbest_cplx_p<2>(a, B, st);
    case 4: return dispatch_kbest_cplx_p<4>(a, B, st);
    default: return dispatch_kbest_cplx_p<8>(a, B, st);
    }
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
    KbestArgs a{R, z, n, K, k_sched, k_sched_stride, radius2, nullptr, nullptr, sym, pd, flags, counters, nullptr, 0.f};
    rc = dispatch_kbest(a, pam, B, (hipStream_t)stream);
    if (rc || !radius2) return rc;
    return rerun_empty(a, pam, B, (hipStream_t)stream, false);
}

extern "C" int32_t kbest_detect_complex(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                        int32_t K, const int32_t* k_sched, int32_t k_sched_stride,
                                        const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                                        int64_t* counters, void* stream)
{
    using namespace mimo;
    int32_t rc = validate_common("kbest_detect_complex", B, n_tx, pam, K);
    if (rc) return rc;
    if (K > 64 || K * pam * pam > 2048)
        return fail(MIMO_ERR_UNSUPPORTED, "kbest_detect_complex: K <= 64 and K * pam^2 <= 2048");
    const int n = 2 * n_tx;
    if (k_sched && k_sched_stride != 0 && k_sched_stride != n)
        return fail(MIMO_ERR_INVALID_ARG, "kbest_detect_complex: k_sched_stride must be 0 or n = %d", n);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "kbest_detect_complex: null pointer");
    KbestArgs a{R, z, n, K, k_sched, k_sched_stride, radius2, nullptr, nullptr, sym, pd, flags, counters, nullptr, 0.f};
    hipStream_t st = (hipStream_t)stream;
    rc = dispatch_kbest_complex(a, pam, B, st);
    if (rc || !radius2) return rc;
    return rerun_empty(a, pam, B, st, true);
}

namespace mimo {
static int32_t rerun_empty(const KbestArgs& a, int pam, int B, hipStream_t st, bool complex_levels)
{
    KbestArgs r = a;
    r.radius2 = nullptr;
    r.rerun = 1;
    if (!complex_levels) return dispatch_kbest(r, pam, B, st);
    return dispatch_kbest_complex(r, pam, B, st);
}
}  // namespace mimo

extern "C" int32_t kbest_rank_labels(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                     int32_t K, const int32_t* force_sym, int32_t* rank, void* stream)
{
    using namespace mimo;
    int32_t rc = validate_common("kbest_rank_labels", B, n_tx, pam, K);
    if (rc) return rc;
    if (B == 0) return MIMO_OK;
    if (!R || !z || !force_sym || !rank) return fail(MIMO_ERR_INVALID_ARG, "kbest_rank_labels: null pointer");
    KbestArgs a{R, z, 2 * n_tx, K, nullptr, 0, nullptr, force_sym, rank, nullptr, nullptr, nullptr, nullptr, nullptr, 0.f};
    return dispatch_kbest(a, pam, B, (hipStream_t)stream);
}

extern "C" int32_t kbest_fallback_mark(const float* pd, uint32_t* flags, const float* sigma2, int32_t B,
                                       int32_t n_tx, float beta, void* stream)
{
    using namespace mimo;
    if (B < 0 || n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "kbest_fallback_mark: bad sizes");
    if (!(beta >= 0.f)) return fail(MIMO_ERR_INVALID_ARG, "kbest_fallback_mark: beta must be >= 0");
    if (B == 0) return MIMO_OK;
    if (!pd || !flags || !sigma2) return fail(MIMO_ERR_INVALID_ARG, "kbest_fallback_mark: null pointer");
    hipLaunchKernelGGL(fallback_mark_kernel, dim3((B + 255) / 256), dim3(256), 0, (hipStream_t)stream, pd, flags,
                       sigma2, beta, 2 * n_tx, B);
    return check_launch("kbest_fallback_mark");
}

extern "C" int32_t kbest_fallback(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam, int32_t K,
                                  const float* sigma2, float beta, int32_t* sym, float* pd, uint32_t* flags,
                                  int64_t* counters, void* stream)
{
    using namespace mimo;
    int32_t rc = validate_common("kbest_fallback", B, n_tx, pam, K);
    if (rc) return rc;
    if (!(beta >= 0.f)) return fail(MIMO_ERR_INVALID_ARG, "kbest_fallback: beta must be >= 0");
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sigma2 || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "kbest_fallback: null pointer");
    KbestArgs a{R, z, 2 * n_tx, K, nullptr, 0, nullptr, nullptr, nullptr, sym, pd, flags, counters, sigma2, beta};
    return dispatch_kbest(a, pam, B, (hipStream_t)stream);
}
