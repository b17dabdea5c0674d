// K-best device helpers shared by the K-best translation units: the launch
// arguments, frame skipping in fallback and re-run modes, per-frame counters,
// fp16 path-word access and the in-wave selections of the K_t smallest keys.
#pragma once

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
    // fallback mode: only frames flagged LEARNED_FALLBACK, or whose search
    // metric pd exceeds (sigma2/2) (n + beta sqrt(2n)), are detected again
    const float* fb_sigma2;
    float fb_beta;
    // re-run mode: only frames whose finite radius left no leaf (EMPTY_SPHERE
    // without FOUND or NONFINITE_INPUT) are detected again, with r2 = +inf;
    // their flags keep EMPTY_SPHERE and their counters accumulate
    int rerun;
};

// does a frame stand as it is in re-run mode?
__device__ inline bool kb_rerun_skips(uint32_t fl)
{
    return !(fl & MIMO_FLAG_EMPTY_SPHERE) || (fl & (MIMO_FLAG_FOUND | MIMO_FLAG_NONFINITE_INPUT));
}

// does a first detection stand?  Not when flagged for the fallback or not
// found, nor when its search metric exceeds (sigma2 / 2) (n + beta sqrt(2 n))
__device__ inline bool kb_first_stands(uint32_t fl, float pd, float sigma2, float beta, int n)
{
    if (fl & MIMO_FLAG_LEARNED_FALLBACK) return false;
    if (!(fl & MIMO_FLAG_FOUND)) return false;
    const float nf = (float)n;
    const float bound = 0.5f * sigma2 * (nf + beta * sqrtf(2.f * nf));
    return pd <= bound;
}

// fallback mode: does frame `frame` keep its first detection?
__device__ inline bool kb_keep_first(const KbestArgs& a, int frame)
{
    if (a.rerun) return kb_rerun_skips(a.flags[frame]);
    if (!a.fb_sigma2) return false;
    return kb_first_stands(a.flags[frame], a.pd[frame], a.fb_sigma2[frame], a.fb_beta, a.n);
}

template <int P, int E>
struct KbestShape {
    static constexpr int NC = WAVE * E;                  // candidates per level
    static constexpr int KCAP = NC / P;                  // survivor capacity
    static constexpr int L = KCAP >= WAVE ? 1 : WAVE / KCAP;  // lanes per survivor
    static constexpr int SPL = KCAP >= WAVE ? KCAP / WAVE : 1; // survivors per lane
};

// words of a path: two fp16 amplitudes per 32-bit word; odd stride against bank conflicts
__host__ __device__ inline int kb_words(int n) { return (n + 1) / 2; }
__host__ __device__ inline int kb_stride(int n) { return kb_words(n) | 1; }

template <int P, int E>
__host__ __device__ inline size_t kbest_lds_bytes(int n)
{
    using S = KbestShape<P, E>;
    return sizeof(uint32_t) * 2 * S::KCAP * kb_stride(n)  // paths
           + sizeof(float) * 2 * S::KCAP                   // survivor pd
           + sizeof(float) * (2 * kb_words(n) + 4)         // staged R row
           + sizeof(int32_t) * S::KCAP                     // selected candidate ids
           + sizeof(uint64_t) * S::KCAP;                   // compacted keys
}

// per-frame counters: overwritten, or added to in re-run mode
__device__ inline void kb_write_counters(const KbestArgs& a, int frame, int64_t expanded, int evals_per_node)
{
    int64_t* c = a.counters + (size_t)frame * 4;
    if (a.rerun) {
        c[0] += expanded;
        c[1] += expanded * evals_per_node;
    } else {
        c[0] = expanded;
        c[1] = expanded * evals_per_node;
        c[2] = 0;
        c[3] = 0;
    }
}

__device__ inline bool kb_finite(float v) { return __builtin_isfinite(v); }

__device__ inline float half_lo(uint32_t d) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(d & 0xffffu)); }
__device__ inline float half_hi(uint32_t d) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(d >> 16)); }
__device__ inline uint32_t half_bits(float a) { return (uint32_t)__builtin_bit_cast(unsigned short, (_Float16)a); }

__device__ inline void kb_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Selection of the `keep` smallest keys (pd bits kh, candidate index
// e * 64 + lane) of one level, written in sorted order to sn (pd) and sel
// (candidate index).  Label mode (fm >= 0): the forced candidate's rank among
// all candidates is returned and the candidate is kept in the last slot if
// it would be dropped.  Returns the number kept; *fpos_out receives the
// forced candidate's 0-based rank (-1 when absent).
template <int E, int KS>
__device__ __forceinline__ int kb_select(const uint32_t (&kh)[E], int ncand, int nvalid, int Kt, int fm, int lane, float* sn,
                                int32_t* sel, uint64_t* skey, int* fpos_out)
{
    // blocks e with e * 64 >= ncand hold no candidate (uniform skips)
    int keep = Kt < nvalid ? Kt : nvalid;
    int fpos = -1;
    uint64_t fkey = 0;
    bool add_forced = false;
    if (fm >= 0) {
        const int fe = fm / WAVE, fl = fm % WAVE;
        uint32_t fh = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e == fe) fh = __shfl(kh[e], fl, WAVE);
        fkey = ((uint64_t)fh << 32) | (uint32_t)fm;
        int below = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e * WAVE >= ncand) continue;
            const uint64_t key = ((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane);
            below += __popcll(__ballot(kh[e] != ~0u && key < fkey));
        }
        fpos = (fh != ~0u) ? below : -1;
        if (fpos >= keep) {  // select keep-1, then add the forced one
            --keep;
            add_forced = true;
        }
    }
    bool take[E];
    if (keep == nvalid) {
#pragma unroll
        for (int e = 0; e < E; ++e) take[e] = kh[e] != ~0u;
    } else {
        // bitwise binary search for the keep-th smallest pd bits, over the
        // bits where the smallest and largest valid keys differ
        uint32_t lo = ~0u, hi = 0u;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e * WAVE >= ncand) continue;
            if (kh[e] != ~0u) {
                lo = min(lo, kh[e]);
                hi = max(hi, kh[e]);
            }
        }
#pragma unroll
        for (int m = 32; m >= 1; m >>= 1) {
            lo = min(lo, (uint32_t)__shfl_xor(lo, m, WAVE));
            hi = max(hi, (uint32_t)__shfl_xor(hi, m, WAVE));
        }
        const int top = (lo == hi) ? -1 : 31 - __clz(lo ^ hi);  // highest differing bit
        uint32_t v = top < 0 ? lo : (lo & ~((2u << top) - 1u));   // common prefix, low bits clear
        for (int bit = top; bit >= 0; --bit) {
            const uint32_t cand = v | (1u << bit);
            int c = 0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (e * WAVE < ncand) c += __popcll(__ballot(kh[e] < cand));
            if (c < keep) v = cand;
        }
        int clt = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            take[e] = kh[e] < v;
            if (e * WAVE < ncand) clt += __popcll(__ballot(take[e]));
        }
        // ties on the pd bits: lowest candidate indices first
        for (int need = keep - clt; need > 0; --need) {
            uint32_t mloc = ~0u;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (kh[e] == v && !take[e]) mloc = min(mloc, (uint32_t)(e * WAVE + lane));
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) mloc = min(mloc, (uint32_t)__shfl_xor(mloc, m, WAVE));
#pragma unroll
            for (int e = 0; e < E; ++e)
                if ((uint32_t)(e * WAVE + lane) == mloc) take[e] = true;
        }
    }
    if (add_forced) {
#pragma unroll
        for (int e = 0; e < E; ++e)
            if ((uint32_t)(e * WAVE + lane) == (uint32_t)fm) take[e] = true;
        ++keep;
    }
    // compaction in candidate order
    int base = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e * WAVE >= ncand) continue;
        const uint64_t bal = __ballot(take[e]);
        if (take[e]) {
            const int slot = base + (int)__popcll(bal & ((1ull << lane) - 1ull));
            skey[slot] = ((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane);
        }
        base += (int)__popcll(bal);
    }
    kb_wave_sync();
    // sort the kept keys in the wave; survivor slot = rank
    uint64_t sk[KS];
#pragma unroll
    for (int e = 0; e < KS; ++e) {
        const int i = e * WAVE + lane;
        sk[e] = i < keep ? skey[i] : ~0ull;
    }
    bitonic_sort<KS>(sk, lane);
#pragma unroll
    for (int e = 0; e < KS; ++e) {
        const int r = e * WAVE + lane;
        if (r < keep) {
            sn[r] = __uint_as_float((uint32_t)(sk[e] >> 32));
            sel[r] = (int32_t)(uint32_t)sk[e];
        }
    }
    *fpos_out = fpos;
    return keep;
}

// Selection by sorting, for at most 128 candidates (ES = 1 or 2 blocks of
// 64): all candidate keys (pd bits, candidate index; invalid = ~0) are put
// in order by one in-wave bitonic sort and the first `keep` survive; with one
// block whose candidates sit in lanes 0 .. LIM-1, only those lanes are sorted.
// Same contract and result as kb_select; no ballot counting.
template <int E, int ES, int LIM = WAVE>
__device__ __forceinline__ int kb_select_sort(const uint32_t (&kh)[E], int nvalid, int Kt, int fm, int lane,
                                              float* sn, int32_t* sel, int* fpos_out)
{
    static_assert(ES <= E && ES <= 2, "sort selection covers one or two blocks");
    const int keep = Kt < nvalid ? Kt : nvalid;
    uint64_t key[ES];
#pragma unroll
    for (int e = 0; e < ES; ++e)
        key[e] = kh[e] == ~0u ? ~0ull : (((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane));
    uint64_t fkey = ~0ull;
    if (fm >= 0) {
        const int fe = fm / WAVE, fl = fm % WAVE;
        uint32_t fh = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e == fe) fh = __shfl(kh[e], fl, WAVE);
        if (fh != ~0u) fkey = ((uint64_t)fh << 32) | (uint32_t)fm;
    }
    if constexpr (ES == 1) sort_lanes<LIM>(key[0], lane);
    else bitonic_sort<ES>(key, lane);
    int fpos = -1;
    if (fkey != ~0ull) {  // the forced candidate's rank = its sorted position
#pragma unroll
        for (int e = 0; e < ES; ++e) {
            const uint64_t b = __ballot(key[e] == fkey);
            if (b) fpos = e * WAVE + (int)__builtin_ctzll(b);
        }
    }
    const bool add_forced = fpos >= keep;  // it takes the last slot
#pragma unroll
    for (int e = 0; e < ES; ++e) {
        const int r = e * WAVE + lane;
        if (r < keep) {
            const uint64_t k = (add_forced && r == keep - 1) ? fkey : key[e];
            sn[r] = __uint_as_float((uint32_t)(k >> 32));
            sel[r] = (int32_t)(uint32_t)k;
        }
    }
    *fpos_out = fpos;
    return keep;
}

// The 64 smallest of the nb <= 128 keys in skey[0 .. nb-1], ascending over
// the lanes (~0 past nb): with at most 64, one register sorted in the
// smallest lane groups that hold them; else the first 64 ascending and the
// rest descending over the wave (in its top 16, 32 or 64 lanes, sorted as
// complements), merged with truncation.
__device__ __forceinline__ uint64_t kb_top64(const uint64_t* skey, int nb, int lane)
{
    uint64_t k0 = lane < nb ? skey[lane] : ~0ull;
    if (nb <= WAVE) {
        if (nb <= 16) sort_lanes<16>(k0, lane);
        else if (nb <= 32) sort_lanes<32>(k0, lane);
        else sort_lanes<WAVE>(k0, lane);
        return k0;
    }
    const int c1 = nb - WAVE;
    const int lim = c1 <= 16 ? 16 : (c1 <= 32 ? 32 : WAVE);
    const int i1 = lane - (WAVE - lim);
    uint64_t k1 = i1 >= 0 && i1 < c1 ? ~skey[WAVE + i1] : 0ull;
    sort_lanes<WAVE>(k0, lane);
    if (lim == 16) sort_lanes<16>(k1, lane);
    else if (lim == 32) sort_lanes<32>(k1, lane);
    else sort_lanes<WAVE>(k1, lane);
    k1 = ~k1;
    k0 = k1 < k0 ? k1 : k0;  // the 64 smallest, a bitonic sequence
    return merge_lanes(k0, lane);
}

// Selection with a bound, when at least `keep` parents (groups of PC
// candidates) were expanded.  Each parent's smallest child exists, so the
// largest of those minima, T, is at least the keep-th smallest pd: no
// candidate above T can survive.  The valid candidates with pd bits <= T are
// compacted through LDS (skey, 128 entries) and sorted with the smallest
// network that holds them; the result is that of sorting all candidates.
// At high SNR a parent's second child lies far above the best children of
// the others, so about `keep` candidates remain; when more than 128 do, the
// 64th smallest of the first 128 is the tighter bound of a second pass.
// Returns -1 (nothing written) when more than 128 remain after it.
template <int E, int PC>
__device__ __forceinline__ int kb_select_bounded(const uint32_t (&kh)[E], int ncand, int keep, int fm, int lane,
                                                 float* sn, int32_t* sel, uint64_t* skey, int* fpos_out)
{
    uint32_t t = 0u;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e * WAVE >= ncand) continue;  // uniform
        uint32_t mn = kh[e];
#pragma unroll
        for (int j = 1; j < PC; j <<= 1) mn = min(mn, xor_lanes(mn, j, lane));
        if (e * WAVE + lane < ncand) t = max(t, mn);  // groups of expanded parents only
    }
#pragma unroll
    for (int j = 1; j < WAVE; j <<= 1) t = max(t, xor_lanes(t, j, lane));
    uint64_t fkey = ~0ull;
    int fpos = -1;
    if (fm >= 0) {  // label mode: the forced candidate's rank among all candidates
        const int fe = fm / WAVE, fl = fm % WAVE;
        uint32_t fh = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e == fe) fh = __shfl(kh[e], fl, WAVE);
        if (fh != ~0u) {
            fkey = ((uint64_t)fh << 32) | (uint32_t)fm;
            int below = 0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (e * WAVE < ncand)
                    below += __popcll(__ballot(((((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane)) < fkey) &&
                                               kh[e] != ~0u));
            fpos = below;
        }
    }
    // a second pass when more than 128 candidates lie below T: the 64th
    // smallest of the first 128 bounds the keep-th smallest as well
    uint64_t res = ~0ull;
    for (int pass = 0; pass < 2; ++pass) {
        int base = 0;
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (e * WAVE >= ncand) continue;
            const bool take = kh[e] != ~0u && kh[e] <= t;
            const uint64_t bal = __ballot(take);
            if (take) {
                const int slot = base + (int)__popcll(bal & ((1ull << lane) - 1ull));
                if (slot < 2 * WAVE) skey[slot] = ((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane);
            }
            base += (int)__popcll(bal);
        }
        if (base > 2 * WAVE && pass == 1) return -1;  // nothing written to sn and sel
        kb_wave_sync();
        res = kb_top64(skey, base < 2 * WAVE ? base : 2 * WAVE, lane);
        if (base <= 2 * WAVE) break;
        t = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(res >> 32), WAVE - 1);
        kb_wave_sync();  // every lane has read skey before the next pass writes it
    }
    const bool add_forced = fpos >= keep;  // it takes the last slot
    if (lane < keep) {
        const uint64_t k = (add_forced && lane == keep - 1) ? fkey : res;
        sn[lane] = __uint_as_float((uint32_t)(k >> 32));
        sel[lane] = (int32_t)(uint32_t)k;
    }
    *fpos_out = fpos;
    return keep;
}

// Selection by sorting and merging, for KCAP <= 64 and E >= 2 blocks of 64
// candidates.  Each non-empty block is sorted across the lanes (even blocks
// ascending, odd ones descending); then pairs of sorted blocks are merged
// with truncation: the lane-wise minimum of an ascending and a descending
// block is a bitonic sequence holding the 64 smallest keys of the pair, which
// six half-cleaner stages put in order (ascending or descending as the next
// merge needs).  Block 0 ends with the 64 smallest keys in ascending order,
// the first `keep` of which survive.  Keys are distinct, so the result is the
// one of a full sort.  Same contract as kb_select.
template <int E, int PC>
__device__ __forceinline__ int kb_select_merge(const uint32_t (&kh)[E], int ncand, int nvalid, int Kt, int fm, int lane,
                                               float* sn, int32_t* sel, uint64_t* skey, int* fpos_out)
{
    const int keep = Kt < nvalid ? Kt : nvalid;  // <= 64
    if (ncand / PC >= keep) {  // uniform: at least `keep` parents
        const int k = kb_select_bounded<E, PC>(kh, ncand, keep, fm, lane, sn, sel, skey, fpos_out);
        if (k >= 0) return k;
    }
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; ++e)
        key[e] = kh[e] == ~0u ? ~0ull : (((uint64_t)kh[e] << 32) | (uint32_t)(e * WAVE + lane));
    uint64_t fkey = ~0ull;
    int fpos = -1;
    if (fm >= 0) {  // label mode: the forced candidate's rank among all candidates
        const int fe = fm / WAVE, fl = fm % WAVE;
        uint32_t fh = 0;
#pragma unroll
        for (int e = 0; e < E; ++e)
            if (e == fe) fh = __shfl(kh[e], fl, WAVE);
        if (fh != ~0u) {
            fkey = ((uint64_t)fh << 32) | (uint32_t)fm;
            int below = 0;
#pragma unroll
            for (int e = 0; e < E; ++e)
                if (e * WAVE < ncand) below += __popcll(__ballot(key[e] < fkey));
            fpos = below;
        }
    }
    // 1. sort every block, even ones ascending and odd ones descending
    //    (branch-free: all E blocks are full at nearly every level)
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e & 1) sort_lanes<WAVE, true>(key[e], lane);
        else sort_lanes<WAVE, false>(key[e], lane);
    }
    // 2. merge with truncation: (e, e + w) -> e, direction by the parity of e / 2w
#pragma unroll
    for (int w = 1; w < E; w <<= 1) {
#pragma unroll
        for (int e = 0; e < E; e += 2 * w) {
            const uint64_t b = key[e + w];
            const uint64_t c = b < key[e] ? b : key[e];
            key[e] = ((e / (2 * w)) & 1) ? merge_lanes<true>(c, lane) : merge_lanes<false>(c, lane);
        }
    }
    const bool add_forced = fpos >= keep;  // it takes the last slot
    if (lane < keep) {
        const uint64_t k = (add_forced && lane == keep - 1) ? fkey : key[0];
        sn[lane] = __uint_as_float((uint32_t)(k >> 32));
        sel[lane] = (int32_t)(uint32_t)k;
    }
    *fpos_out = fpos;
    return keep;
}

// the grouped K-best launch (J = 1 or 2 real levels per step) for K <= 64 and
// K pam^J <= 1024; arguments validated by the caller
int32_t dispatch_grouped(const KbestArgs& a, int pam, int J, int B, hipStream_t st);

}  // namespace mimo
