// Grouped K-best: the tree of kbest_detect (J = 1, real levels) or of
// kbest_detect_complex (J = 2, one complex symbol per step), with the
// successor evaluation of Sec. V-A done as one matrix product per group of
// levels on the matrix cores.
//
// The paper evaluates all successors of a node at once as B = Y* - R'V, the
// columns of V being the successors' fixed symbols (Sec. V-A), and branches
// on J symbols per step (Sec. IV-B).  On a wavefront that holds K_t survivors
// of one frame the heavy part of that product is the interference of the
// levels already fixed:
//
//     C[k][s] = sum_{j > k} (c R)[k][j] x_s[j]
//
// for the rows k of the next levels and every survivor s.  The levels are
// cut into groups of 16 (group h = levels 16h .. 16h + 15).  When a group
// starts, the interference of every level above it is one product
// C = (c R)[group rows, levels above] X[levels above, survivors], computed on
// v_mfma_f32_16x16x32_bf16: c R is split exactly into three bf16 parts
// (8 significant bits each, truncated: hi + mid + lo reproduces the FP32
// value), the amplitudes 2i - (P-1) are exact in bf16, every product is exact
// and the sums are FP32.  Inside the group, the centre of level k of
// survivor s is
//
//     b = z_k - C[k][origin(s)] - sum_{k < j in group, fixed} (c R)[k][j] x_s[j]
//
// where origin(s) is the survivor, at the start of the group, that s descends
// from (Eq. (inc): the part above the group is computed once per group, the
// rest level by level).  Children and radius test are those of the other
// K-best kernels.
//
// Lane (s, q) evaluates children q, q + L, ... of its own survivor s (no
// exchange; the candidate index s P^J + c is carried in the key), and the
// K_t smallest keys (pd, parent rank, child) are selected as in the other
// K-best kernels: a bound from the survivors' smallest children, compaction
// of the candidates below it, and an in-wave sort.  The survivors stay in key
// order, so the tree, the ties and the result are those of kbest_detect /
// kbest_detect_complex; only the order of the FP32 sums in a centre differs.
//
// Paths are never copied level by level.  A survivor carries its origin and
// the 16 amplitude bytes of the current group (4 registers, a + 8 per level,
// 8 = not yet fixed); when the group ends every survivor's amplitudes (as 16
// nibbles) and origin are written once to a per-group segment table in LDS.  The path of a
// survivor is the chain segment(h, s) -> segment(h + 1, parent) -> ..., which
// is what the matrix product's B operand reads.
#include "common.hpp"
#include "kbest_common.hpp"

namespace mimo {

typedef __bf16 gk_bf16x8 __attribute__((ext_vector_type(8)));
typedef float gk_f32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t gk_u32x4 __attribute__((ext_vector_type(4)));
typedef uint32_t gk_u32x2 __attribute__((ext_vector_type(2)));

constexpr int GK_LEVELS = 16;       // levels per group = rows of one matrix-core tile
constexpr int GK_CAND_MAX = 2048;   // K pam^J candidates per step (beyond 1024: pam^J = 64 only)
constexpr uint32_t GK_UNFIXED = 0x08080808u;

template <int P, int J, int E>
struct GroupedShape {
    static constexpr int PC = J == 1 ? P : P * P;                 // children per survivor
    static constexpr int KCAP = WAVE * E / PC;                     // survivor capacity
    static constexpr int L = WAVE / KCAP;                          // lanes per survivor
    static constexpr int NT = KCAP >= 16 ? KCAP / 16 : 1;          // survivor tiles of 16 columns
    static constexpr int CST = KCAP >= 16 ? KCAP : 16;             // row stride of C in LDS
};

// LDS of one frame: compaction keys, segment words [G][KCAP][2], C [16][CST]
// unless the group's interference stays in the matrix-core result registers
// (CR), in-group rows [16][16], diagonal [16], z [16], selected pds [KCAP],
// selected candidates [KCAP], segment parents [G][KCAP] (bytes)
__host__ __device__ inline size_t gk_lds_bytes(int kcap, int G, bool cr = false)
{
    const int cst = kcap >= 16 ? kcap : 16;
    const size_t segw = ((size_t)2 * G * kcap + 3) & ~(size_t)3;  // whole 16-byte units
    return sizeof(uint64_t) * 2 * WAVE + sizeof(uint32_t) * segw + (cr ? 0 : sizeof(float) * 16 * cst) +
           sizeof(float) * (256 + 32) + sizeof(float) * kcap + sizeof(int32_t) * kcap + (size_t)G * kcap;
}

// Entry (r, col) of the group's interference C held in the result registers
// of the matrix product: column tile col / 16, in lane 16 (r / 4) + col % 16,
// element r % 4 (r is uniform, col this lane's own).  One lane permute per
// column tile, then this lane's tile is kept.
template <int NT>
__device__ __forceinline__ float gk_cread(const gk_f32x4 (&c)[NT], int r, int col, int lane)
{
    const int i = r & 3;
    const int src = (((r >> 2) << 4) | (col & 15)) << 2;
    float v = 0.f;
#pragma unroll
    for (int t = 0; t < NT; ++t) {
        const float e = i == 0 ? c[t][0] : (i == 1 ? c[t][1] : (i == 2 ? c[t][2] : c[t][3]));
        const float x = __int_as_float(__builtin_amdgcn_ds_bpermute(src, __float_as_int(e)));
        v = (col >> 4) == t ? x : v;
    }
    return v;
}

// exact three-way bf16 split of an FP32 value by truncation: hi keeps the
// top 8 significant bits, mid the next 8 of the remainder, lo the rest (the
// remainders are exact FP32 differences, and what is left for lo has at most
// 8 significant bits)
__device__ __forceinline__ void gk_split3(float v, __bf16& hi, __bf16& mid, __bf16& lo)
{
    const float h = __uint_as_float(__float_as_uint(v) & 0xffff0000u);
    const float r1 = v - h;
    const float m = __uint_as_float(__float_as_uint(r1) & 0xffff0000u);
    const float r2 = r1 - m;
    hi = (__bf16)h;
    mid = (__bf16)m;
    lo = (__bf16)r2;
}

// eight amplitude nibbles (a + 8, level e at bits 4e) -> bf16 amplitudes a
__device__ __forceinline__ gk_bf16x8 gk_decode8(uint32_t w)
{
    gk_bf16x8 b;
#pragma unroll
    for (int e = 0; e < 8; ++e) b[e] = (__bf16)((float)((w >> (4 * e)) & 0xfu) - 8.f);
    return b;
}

// four amplitude bytes (values below 16) -> four nibbles in the low 16 bits
__device__ __forceinline__ uint32_t gk_nibbles4(uint32_t b)
{
    return (b & 0xfu) | ((b >> 4) & 0xf0u) | ((b >> 8) & 0xf00u) | ((b >> 12) & 0xf000u);
}

// sorts one register of keys ascending over lanes 0 .. LIM-1, LIM the
// smallest of 16, 32, 64 that holds `count` keys (the rest of the lanes hold
// ~0 and sort among themselves)
__device__ __forceinline__ void gk_sort_upto(uint64_t& k, int count, int lane)
{
    if (count <= 16) sort_lanes<16>(k, lane);
    else if (count <= 32) sort_lanes<32>(k, lane);
    else sort_lanes<WAVE>(k, lane);
}

// the 64 smallest of 64 * E keys (distinct), ascending in key[0]: every
// block sorted (even ones ascending, odd ones descending), then pairs merged
// with truncation (the lane-wise minimum of an ascending and a descending
// block is a bitonic sequence of the 64 smallest of the pair, put in order
// by six half-cleaner stages)
template <int E>
__device__ __forceinline__ void gk_merge_select(uint64_t (&key)[E], int lane)
{
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (e & 1) sort_lanes<WAVE, true>(key[e], lane);
        else sort_lanes<WAVE, false>(key[e], lane);
    }
#pragma unroll
    for (int w = 1; w < E; w <<= 1) {
#pragma unroll
        for (int e = 0; e < E; e += 2 * w) {
            const uint64_t b = key[e + w];
            const uint64_t c = b < key[e] ? b : key[e];
            key[e] = ((e / (2 * w)) & 1) ? merge_lanes<true>(c, lane) : merge_lanes<false>(c, lane);
        }
    }
}

// Selection of the keep = min(K_t, nvalid) smallest keys (pd bits, s PC + c)
// -- i.e. (pd, parent rank, child), the survivors being kept in order --
// written in order to sn (pd) and sel (candidate index).  Lane (s, q) holds
// children c = e L + q of survivor s in block e.  With at least keep
// survivors expanded (and more candidates than one sort over 32 lanes
// holds), the largest of their smallest children, T, bounds the keep-th
// smallest key: the keys with pd bits <= T
// (usually little more than keep) are compacted through LDS and sorted --
// one register when at most 64, else the first 64 ascending and the rest
// descending, merged with truncation.  Beyond 128 such keys (a few levels in
// a hundred at 64 survivors of 64-QAM) the 64th smallest of the first 128 is
// the tighter bound of a second compaction.  Otherwise all blocks are sorted
// and merged.
template <int E>
__device__ __forceinline__ int gk_select(const uint32_t (&kh)[E], int nvalid, int Kt, int cnt, uint32_t idx0, int L,
                                         int lane, float* sn, int32_t* sel, uint64_t* skey)
{
    const int keep = Kt < nvalid ? Kt : nvalid;  // <= 64
    const uint64_t below = (1ull << lane) - 1ull;
    uint64_t res;  // the keep smallest keys, ascending in lanes 0 .. keep-1
    bool done = false;
    if ((E >= 2 || cnt * L > 32) && cnt >= keep) {  // (else one sort over at most 32 lanes)
        uint32_t mn = kh[0];
#pragma unroll
        for (int e = 1; e < E; ++e) mn = min(mn, kh[e]);
        for (int j = 1; j < L; j <<= 1) mn = min(mn, xor_lanes(mn, j, lane));
        uint32_t t = lane / L < cnt ? mn : 0u;
        // the wave's largest: rows of 16 by DPP (quad exchanges, rotations
        // by 4 and 8), then the four row results (uniform)
        t = max(t, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0xB1, 0xF, 0xF, false));
        t = max(t, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0x4E, 0xF, 0xF, false));
        t = max(t, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0x124, 0xF, 0xF, false));
        t = max(t, (uint32_t)__builtin_amdgcn_update_dpp(0, (int)t, 0x128, 0xF, 0xF, false));
        t = max(max((uint32_t)__builtin_amdgcn_readlane((int)t, 0), (uint32_t)__builtin_amdgcn_readlane((int)t, 16)),
                max((uint32_t)__builtin_amdgcn_readlane((int)t, 32), (uint32_t)__builtin_amdgcn_readlane((int)t, 48)));
        // t = ~0u when an expanded survivor has no child inside the radius: no bound
        if (t != ~0u) {
            // a second pass when more than 128 keys lie below T: the 64th
            // smallest of the first 128 bounds the keep-th smallest as well
            for (int pass = 0; pass < 2; ++pass) {
                int base = 0;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const bool take = kh[e] <= t;
                    const uint64_t bal = __ballot(take);
                    if (take) {
                        const int slot = base + (int)__popcll(bal & below);
                        if (slot < 2 * WAVE) skey[slot] = ((uint64_t)kh[e] << 32) | (idx0 + (uint32_t)(e * L));
                    }
                    base += (int)__popcll(bal);
                }
                if (base > 2 * WAVE && pass == 1) break;  // (rare on random channels, common on near-singular ones) all blocks sorted below
                kb_wave_sync();
                const uint64_t k0 = kb_top64(skey, base < 2 * WAVE ? base : 2 * WAVE, lane);
                if (base <= 2 * WAVE) {
                    res = k0;
                    done = true;
                    break;
                }
                t = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(k0 >> 32), WAVE - 1);
                kb_wave_sync();  // every lane has read skey before the next pass writes it
            }
        }
    }
    if (!done) {
        uint64_t key[E];
#pragma unroll
        for (int e = 0; e < E; ++e)
            key[e] = kh[e] == ~0u ? ~0ull : (((uint64_t)kh[e] << 32) | (idx0 + (uint32_t)(e * L)));
        if constexpr (E == 1) {
            gk_sort_upto(key[0], cnt * L, lane);  // candidates sit in lanes below cnt L
        } else {
            gk_merge_select<E>(key, lane);
        }
        res = key[0];
    }
    if (lane < keep) {
        sn[lane] = __uint_as_float((uint32_t)(res >> 32));
        sel[lane] = (int32_t)(uint32_t)res;
    }
    return keep;
}

// CR: the group's interference C stays in the matrix-core result registers
// (read by lane permutes) instead of an LDS tile: fewer LDS bytes per frame,
// more registers; the host picks the variant that holds more frames per CU.
template <int P, int J, int E, bool CR>
__device__ __forceinline__ void kbest_frame_grouped(const KbestArgs& a, int frame, unsigned char* lds)
{
    using S = GroupedShape<P, J, E>;
    constexpr int PC = S::PC, KCAP = S::KCAP, L = S::L, NT = S::NT, CST = S::CST;
    static_assert(KCAP >= 1 && KCAP <= 64, "one survivor per lane at most, one at least");
    static_assert(J == 1 || J == 2, "one or two real levels per step");
    static_assert(E * L == PC, "a survivor's lanes hold its children over the E blocks");
    const int lane = threadIdx.x & 63;
    const int s_own = lane / L, q = lane % L;
    const int n = a.n;
    const int G = (n + GK_LEVELS - 1) / GK_LEVELS;
    uint64_t* skey = reinterpret_cast<uint64_t*>(lds);
    uint32_t* segb = reinterpret_cast<uint32_t*>(skey + 2 * WAVE);  // [G][KCAP][2]: 16 nibbles
    float* cg = reinterpret_cast<float*>(segb + ((2 * G * KCAP + 3) & ~3));  // 16-byte aligned
    float* rg = CR ? cg : cg + 16 * CST;
    float* rd = rg + 256;
    float* zg = rd + 16;
    float* sn = zg + 16;
    int32_t* sel = reinterpret_cast<int32_t*>(sn + KCAP);
    uint8_t* segp = reinterpret_cast<uint8_t*>(sel + KCAP);

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float r2 = a.radius2 ? a.radius2[frame] : INFINITY;
    const float cs = pam_scale(P);
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;
    // the frame's R as one buffer: loads past its end return 0
    const __amdgpu_buffer_rsrc_t rs = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<float*>(Rf), 0, (int)r_packed_size(n) * (int)sizeof(float), 0x00020000);

    uint32_t igw[4] = {GK_UNFIXED, GK_UNFIXED, GK_UNFIXED, GK_UNFIXED};
    int orig = s_own;
    float pd_own = 0.f;                          // pd of this lane's survivor
    const uint32_t idx0 = (uint32_t)(s_own * PC + q);  // candidate index of block 0: child q
    int cnt = 1;
    int64_t expanded = 0;
    uint32_t flags = 0;
    bool stopped = false;

    for (int h = G - 1; h >= 0 && !stopped; --h) {
        const int k0 = GK_LEVELS * h;
        const int ktop = min(k0 + GK_LEVELS - 1, n - 1);
        // in-group rows: (c R)[k0 + r][k0 + c] for c > r (the complex-level
        // tree drops the structural zero R[2m][2m+1]), the diagonal and z
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int idx = lane + WAVE * i;
            const int r = idx >> 4, c = idx & 15;
            const int k = k0 + r, j = k0 + c;
            float v = 0.f;
            if (c > r && j < n && !(J == 2 && !(r & 1) && c == r + 1)) v = cs * Rf[r_row_off(n, k) + (j - k)];
            rg[idx] = v;
        }
        if (lane < 16) {
            const int k = k0 + lane;
            rd[lane] = k < n ? cs * Rf[r_row_off(n, k)] : 0.f;
            zg[lane] = k < n ? zf[k] : 0.f;
        }
        // interference of the levels above the group, for every survivor, on the matrix cores
        gk_f32x4 acc[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = gk_f32x4{0.f, 0.f, 0.f, 0.f};
        if (h < G - 1) {
            const int row = k0 + (lane & 15);                  // A row of this lane (every row exists)
            const int roff = (int)r_row_off(n, row) - row;     // (c R)[row][j] at roff + j
            const int nch = (n - GK_LEVELS * (h + 1) + 31) / 32;
            const int upper = lane >> 5;                       // B rows from group h+1+2ch (+1 for upper lanes)
            const int bsub = (lane >> 4) & 1;                  // word of the segment: levels 0-7 or 8-15
            int anc[NT];
            bool live[NT];
#pragma unroll
            for (int t = 0; t < NT; ++t) {
                const int s = 16 * t + (lane & 15);
                live[t] = s < cnt;
                anc[t] = live[t] ? s : 0;
            }
            int g = h + 1;
            if (upper) {
                if (g < G) {
#pragma unroll
                    for (int t = 0; t < NT; ++t) anc[t] = segp[g * KCAP + anc[t]];
                }
                ++g;
            }
            for (int ch = 0; ch < nch; ++ch) {
                const int j0 = GK_LEVELS * (h + 1) + 32 * ch + 8 * (lane >> 4);
                const gk_u32x4 w0 = __builtin_amdgcn_raw_buffer_load_b128(rs, 4 * (roff + j0), 0, 0);
                const gk_u32x4 w1 = __builtin_amdgcn_raw_buffer_load_b128(rs, 4 * (roff + j0 + 4), 0, 0);
                gk_bf16x8 ahi, amid, alo;
#pragma unroll
                for (int e = 0; e < 8; ++e) {
                    const float rv = __uint_as_float(e < 4 ? w0[e] : w1[e - 4]);
                    const float v = j0 + e < n ? cs * rv : 0.f;
                    __bf16 hi, mid, lo;
                    gk_split3(v, hi, mid, lo);
                    ahi[e] = hi;
                    amid[e] = mid;
                    alo[e] = lo;
                }
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    gk_bf16x8 b;
                    if (g < G && live[t]) {
                        b = gk_decode8(segb[2 * (g * KCAP + anc[t]) + bsub]);
                    } else {
#pragma unroll
                        for (int e = 0; e < 8; ++e) b[e] = (__bf16)0.f;
                    }
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(alo, b, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(amid, b, acc[t], 0, 0, 0);
                    acc[t] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(ahi, b, acc[t], 0, 0, 0);
                }
                // two groups up for the next chunk of 32 levels
#pragma unroll
                for (int u = 0; u < 2; ++u) {
                    if (g < G) {
#pragma unroll
                        for (int t = 0; t < NT; ++t) anc[t] = segp[g * KCAP + anc[t]];
                    }
                    ++g;
                }
            }
            // lane l holds C rows 4 (l / 16) + i of survivor column 16 t + l % 16
            if constexpr (!CR) {
#pragma unroll
                for (int t = 0; t < NT; ++t) {
                    const int col = 16 * t + (lane & 15);
                    if (col < KCAP) {
#pragma unroll
                        for (int i = 0; i < 4; ++i) cg[(4 * (lane >> 4) + i) * CST + col] = acc[t][i];
                    }
                }
            }
        }
        kb_wave_sync();

        for (int k_hi = ktop; k_hi >= k0; k_hi -= J) {
            const int r_hi = k_hi - k0, r_lo = r_hi - (J - 1);
            // centres of this lane's survivor: the levels above the group
            // (C at the survivor's origin), then the fixed levels of the group
            float dh = 0.f, dl = 0.f;
#pragma unroll
            for (int d = 0; d < 4; ++d) {
                if (4 * d + 3 > r_hi) {  // a word with fixed levels above k_hi (uniform)
                    const float4 rh = *reinterpret_cast<const float4*>(rg + 16 * r_hi + 4 * d);
                    const float xs[4] = {(float)(igw[d] & 0xffu) - 8.f, (float)((igw[d] >> 8) & 0xffu) - 8.f,
                                         (float)((igw[d] >> 16) & 0xffu) - 8.f, (float)(igw[d] >> 24) - 8.f};
                    dh = fmaf(rh.x, xs[0], dh);
                    dh = fmaf(rh.y, xs[1], dh);
                    dh = fmaf(rh.z, xs[2], dh);
                    dh = fmaf(rh.w, xs[3], dh);
                    if constexpr (J == 2) {
                        const float4 rl = *reinterpret_cast<const float4*>(rg + 16 * r_lo + 4 * d);
                        dl = fmaf(rl.x, xs[0], dl);
                        dl = fmaf(rl.y, xs[1], dl);
                        dl = fmaf(rl.z, xs[2], dl);
                        dl = fmaf(rl.w, xs[3], dl);
                    }
                }
            }
            const bool above = h < G - 1;
            float ch = 0.f, cl = 0.f;  // C at the survivor's origin (the levels above the group)
            if (above) {
                if constexpr (CR) {
                    ch = gk_cread<NT>(acc, r_hi, orig, lane);
                    if constexpr (J == 2) cl = gk_cread<NT>(acc, r_lo, orig, lane);
                } else {
                    ch = cg[r_hi * CST + orig];
                    if constexpr (J == 2) cl = cg[r_lo * CST + orig];
                }
            }
            const float bh = zg[r_hi] - (ch + dh);
            const float bl = J == 2 ? zg[r_lo] - (cl + dl) : 0.f;
            const float rkh = rd[r_hi], rkl = rd[r_lo];
            const bool live = s_own < cnt;
            // a NaN or infinity in R or z reaches every centre of the level
            if (__ballot(!kb_finite(rkh) || !kb_finite(rkl) || (live && !(kb_finite(bh) && kb_finite(bl))))) {
                flags |= MIMO_FLAG_NONFINITE_INPUT;
                cnt = 0;
                stopped = true;
                break;
            }
            // children: block e, lane (s, q) holds child c = e L + q of survivor s
            uint32_t kh[E];
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int c = e * L + q;
                float pdc;
                if constexpr (J == 1) {
                    const float ee = fmaf(-rkh, (float)(2 * c - (P - 1)), bh);
                    pdc = fmaf(ee, ee, pd_own);
                } else {
                    const float eh = fmaf(-rkh, (float)(2 * (c / P) - (P - 1)), bh);
                    const float el = fmaf(-rkl, (float)(2 * (c % P) - (P - 1)), bl);
                    pdc = fmaf(el, el, fmaf(eh, eh, pd_own));
                }
                kh[e] = (live && pdc < r2) ? __float_as_uint(pdc) : ~0u;
            }
            expanded += cnt;
            int nvalid = 0;
#pragma unroll
            for (int e = 0; e < E; ++e) nvalid += __popcll(__ballot(kh[e] != ~0u));
            if (nvalid == 0) {
                flags |= MIMO_FLAG_EMPTY_SPHERE;
                cnt = 0;
                stopped = true;
                break;
            }
            int Kt = ks ? ks[k0 + r_lo] : a.K;
            Kt = Kt > a.K ? a.K : (Kt < 1 ? 1 : Kt);
            Kt = Kt > KCAP ? KCAP : Kt;
            const int keep = gk_select<E>(kh, nvalid, Kt, cnt, idx0, L, lane, sn, sel, skey);
            kb_wave_sync();
            // new survivor s_own: its parent's origin and group bytes, plus the new level(s)
            int src = lane, cnew = 0;
            float pdn = pd_own;
            if (s_own < keep) {
                const int mm = sel[s_own];
                src = (mm / PC) * L + q;
                cnew = mm % PC;
                pdn = sn[s_own];
            }
            orig = __shfl(orig, src, WAVE);
#pragma unroll
            for (int d = 0; d < 4; ++d)
                if (4 * d + 3 > r_hi) igw[d] = (uint32_t)__shfl((int)igw[d], src, WAVE);
            if (s_own < keep) {
                const int d = r_hi >> 2;
                uint32_t put, mask;
                if constexpr (J == 1) {
                    put = (uint32_t)(2 * cnew - (P - 1) + 8) << (8 * (r_hi & 3));
                    mask = 0xffu << (8 * (r_hi & 3));
                } else {  // levels r_lo (real part, even) and r_hi = r_lo + 1 (imaginary part)
                    put = ((uint32_t)(2 * (cnew % P) - (P - 1) + 8) | ((uint32_t)(2 * (cnew / P) - (P - 1) + 8) << 8))
                          << (8 * (r_lo & 3));
                    mask = 0xffffu << (8 * (r_lo & 3));
                }
#pragma unroll
                for (int dd = 0; dd < 4; ++dd)
                    if (dd == d) igw[dd] = (igw[dd] & ~mask) | put;
            }
            pd_own = pdn;
            cnt = keep;
            kb_wave_sync();  // sel and sn are read before the next level writes them
        }
        if (stopped) break;
        // the group's segment of every survivor: its bytes and its origin
        if (q == 0 && s_own < cnt) {
            *reinterpret_cast<gk_u32x2*>(segb + 2 * (h * KCAP + s_own)) =
                gk_u32x2{gk_nibbles4(igw[0]) | (gk_nibbles4(igw[1]) << 16), gk_nibbles4(igw[2]) | (gk_nibbles4(igw[3]) << 16)};
            segp[h * KCAP + s_own] = (uint8_t)orig;
        }
        kb_wave_sync();
        orig = s_own;
#pragma unroll
        for (int d = 0; d < 4; ++d) igw[d] = GK_UNFIXED;
    }

    if (lane == 0) {
        if (cnt > 0) flags |= MIMO_FLAG_FOUND;
        if (a.fb_sigma2) flags |= MIMO_FLAG_LEARNED_FALLBACK;
        if (a.rerun) flags |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.flags) a.flags[frame] = flags;
        if (a.pd) a.pd[frame] = cnt > 0 ? pd_own : INFINITY;  // survivor 0: the best leaf
        if (a.counters) kb_write_counters(a, frame, expanded, PC * J);
    }
    if (!a.sym) return;
    // lane h rebuilds survivor 0's segment of group h by following the
    // parents from group 0 up
    const int nw = n / 2;
    if (lane < G) {
        gk_u32x2 w = {0x88888888u, 0x88888888u};
        if (cnt > 0) {
            int anc = 0;
            for (int g = 0; g < lane; ++g) anc = segp[g * KCAP + anc];
            w = *reinterpret_cast<const gk_u32x2*>(segb + 2 * (lane * KCAP + anc));
        }
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int sw = 8 * lane + i;  // complex symbol: real part at level 2i of the group, imaginary part at 2i + 1
            if (sw < nw) {
                int v = 0;
                if (cnt > 0) {
                    const int are = (int)((w[i >> 2] >> (8 * (i & 3))) & 0xfu) - 8;
                    const int aim = (int)((w[i >> 2] >> (8 * (i & 3) + 4)) & 0xfu) - 8;
                    v = ((are + (P - 1)) / 2) * P + (aim + (P - 1)) / 2;
                }
                a.sym[(size_t)frame * nw + sw] = v;
            }
        }
    }
}

// Register caps where registers, not LDS, bound the waves per SIMD: with 32
// sort registers per lane (2048 candidates per complex level) the kernel
// would take 196 registers, two waves; capped at 168 for three (15 spill to
// scratch): K = 32 at 16x16 64-QAM 3.75 -> 2.70 ms per 6x10^4 frames.  With
// 16 (1024 candidates), 124 registers, four waves; capped for five (14
// spill): K = 10 at 16x16 64-QAM 0.98 -> 0.92 ms, at 100x100 3.97 -> 3.79 ms
// per 5x10^4 frames.  (The same cap on the two-frames-per-wave kernel, 84 ->
// 80 registers for six waves, made it slower.)
template <int P, int J, int E, bool CR>
__global__ void __launch_bounds__(64, (E >= 32 ? 3 : (E == 16 ? 5 : 1))) kbest_grouped_kernel(KbestArgs a)
{
    extern __shared__ unsigned char smem_kbg[];
    if (kb_keep_first(a, blockIdx.x)) return;
    kbest_frame_grouped<P, J, E, CR>(a, blockIdx.x, smem_kbg);
}

// C in registers where that holds more frames per CU (LDS-bound shapes:
// many groups), else C in LDS (fewer instructions per level); the register
// variant exists up to E = 8 blocks.  A fallback or re-run launch detects a
// few flagged frames of the batch, for which occupancy does not matter: LDS.
template <int P, int J, int E>
static int32_t launch_grouped(const KbestArgs& a, int B, hipStream_t st)
{
    using S = GroupedShape<P, J, E>;
    const int G = (a.n + GK_LEVELS - 1) / GK_LEVELS;
    const size_t lds_l = gk_lds_bytes(S::KCAP, G, false);
    if constexpr (E <= 8) {
        if (a.fb_sigma2 || a.rerun) {
            hipLaunchKernelGGL((kbest_grouped_kernel<P, J, E, false>), dim3(B), dim3(WAVE), lds_l, st, a);
            return check_launch("kbest_detect_grouped");
        }
        const size_t lds_r = gk_lds_bytes(S::KCAP, G, true);
        int occ_r = 0, occ_l = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_r, (const void*)kbest_grouped_kernel<P, J, E, true>,
                                                         WAVE, lds_r) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_l, (const void*)kbest_grouped_kernel<P, J, E, false>,
                                                         WAVE, lds_l) != hipSuccess)
            return fail(MIMO_ERR_HIP, "kbest_detect_grouped: occupancy query failed");
        if (occ_r > occ_l) {
            hipLaunchKernelGGL((kbest_grouped_kernel<P, J, E, true>), dim3(B), dim3(WAVE), lds_r, st, a);
            return check_launch("kbest_detect_grouped");
        }
    }
    hipLaunchKernelGGL((kbest_grouped_kernel<P, J, E, false>), dim3(B), dim3(WAVE), lds_l, st, a);
    return check_launch("kbest_detect_grouped");
}

// smallest block count E (a power of two) with 64 E >= K pam^J candidates
template <int P, int J>
static int32_t dispatch_grouped_pj(const KbestArgs& a, int B, hipStream_t st)
{
    constexpr int PC = J == 1 ? P : P * P;
    const int need = a.K * PC;
    if (need <= 64 && PC <= 64) return launch_grouped<P, J, 1>(a, B, st);
    if constexpr (2 * WAVE / PC <= 64) {
        if (need <= 128) return launch_grouped<P, J, 2>(a, B, st);
    }
    if constexpr (4 * WAVE / PC <= 64) {
        if (need <= 256) return launch_grouped<P, J, 4>(a, B, st);
    }
    if constexpr (8 * WAVE / PC <= 64) {
        if (need <= 512) return launch_grouped<P, J, 8>(a, B, st);
    }
    if constexpr (16 * WAVE / PC <= 64) {
        if (need <= 1024) return launch_grouped<P, J, 16>(a, B, st);
    }
    if constexpr (32 * WAVE / PC <= 64) {  // 64-QAM on the complex tree: K <= 32
        if (need <= 2048) return launch_grouped<P, J, 32>(a, B, st);
    }
    return fail(MIMO_ERR_UNSUPPORTED, "kbest_detect_grouped: K * pam^J beyond the instantiations");
}

int32_t dispatch_grouped(const KbestArgs& a, int pam, int J, int B, hipStream_t st)
{
    if (J == 1) {
        switch (pam) {
        case 2: return dispatch_grouped_pj<2, 1>(a, B, st);
        case 4: return dispatch_grouped_pj<4, 1>(a, B, st);
        default: return dispatch_grouped_pj<8, 1>(a, B, st);
        }
    }
    switch (pam) {
    case 2: return dispatch_grouped_pj<2, 2>(a, B, st);
    case 4: return dispatch_grouped_pj<4, 2>(a, B, st);
    default: return dispatch_grouped_pj<8, 2>(a, B, st);
    }
}

}  // namespace mimo

extern "C" int32_t kbest_detect_grouped(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                        int32_t K, int32_t J, const int32_t* k_sched, int32_t k_sched_stride,
                                        const float* radius2, int32_t* sym, float* pd, uint32_t* flags,
                                        int64_t* counters, void* stream)
{
    using namespace mimo;
    const char* who = "kbest_detect_grouped";
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", who);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", who);
    if (J != 1 && J != 2) return fail(MIMO_ERR_INVALID_ARG, "%s: J must be 1 or 2", who);
    if (n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: n_tx < 1", who);
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx > %d", who, MIMO_MAX_TX);
    if (K < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: K < 1", who);
    const int pc = J == 1 ? pam : pam * pam;
    if (K > 64 || K * pc > GK_CAND_MAX)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: K <= 64 and K * pam^J <= %d", who, GK_CAND_MAX);
    const int n = 2 * n_tx;
    if (k_sched && k_sched_stride != 0 && k_sched_stride != n)
        return fail(MIMO_ERR_INVALID_ARG, "%s: k_sched_stride must be 0 or n = %d", who, n);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", who);
    KbestArgs a{R, z, n, K, k_sched, k_sched_stride, radius2, nullptr, nullptr, sym, pd, flags, counters, nullptr, 0.f};
    hipStream_t st = (hipStream_t)stream;
    int32_t rc = dispatch_grouped(a, pam, J, B, st);
    if (rc || !radius2) return rc;
    KbestArgs r = a;  // frames whose finite radius left no leaf: again with r2 = +inf
    r.radius2 = nullptr;
    r.rerun = 1;
    return dispatch_grouped(r, pam, J, B, st);
}

namespace mimo {

__global__ void reset_counter_kernel_kb(int* counter) { *counter = 0; }

// Uneven batch: one wavefront per workgroup pulls frames from a device work
// counter and runs the grouped K-best (real levels) with each frame's own
// constellation and K -- per frame the detection of kbest_detect_grouped
// with J = 1.
constexpr int UNEVEN_NWMAX = 64;     // n <= 128 real levels (n_tx <= 64): at most 8 groups
constexpr int UNEVEN_KMAX = 64;      // one survivor per lane at most
constexpr int UNEVEN_CAND_MAX = 256; // K * pam: four blocks of 64 candidates

template <int P, int E>
__device__ __forceinline__ void kbest_uneven_one(const KbestArgs& a, unsigned char* lds)
{
    kbest_frame_grouped<P, 1, E, false>(a, 0, lds);
}

// At most 128 registers (four waves per SIMD): the eight inlined variants
// would otherwise take 148 (three waves), and with 11.4 KB of LDS per frame
// the CU holds 14 frames; 5 registers spill to scratch outside the hot loops.
__global__ void __launch_bounds__(64, 4) kbest_uneven_kernel(const mimo_frame_desc* __restrict__ desc, int B,
                                                          const float* __restrict__ R, const float* __restrict__ z,
                                                          int32_t* __restrict__ sym, float* __restrict__ pd,
                                                          uint32_t* __restrict__ flags, int* __restrict__ counter)
{
    extern __shared__ unsigned char smem_kbu[];
    const int lane = threadIdx.x & 63;
    for (;;) {
        int f = 0;
        if (lane == 0) f = atomicAdd(counter, 1);
        f = __builtin_amdgcn_readfirstlane(__shfl(f, 0, WAVE));
        if (f >= B) break;
        const mimo_frame_desc d = desc[f];
        const int P = __builtin_amdgcn_readfirstlane(d.pam);
        const int K = __builtin_amdgcn_readfirstlane(d.K);
        const int ntx = __builtin_amdgcn_readfirstlane(d.n_tx);
        // descriptors outside the instantiations' range are skipped, flagged
        if ((P != 2 && P != 4 && P != 8) || K < 1 || K > UNEVEN_KMAX || K * P > UNEVEN_CAND_MAX || ntx < 1 ||
            ntx > UNEVEN_NWMAX) {
            if (lane == 0) flags[f] = MIMO_FLAG_INVALID_FRAME;
            continue;
        }
        KbestArgs a{R + d.r_off, z + d.z_off, 2 * d.n_tx, K, nullptr, 0, nullptr, nullptr, nullptr,
                    sym + d.s_off, pd + f, flags + f, nullptr, nullptr, 0.f};
        const int need = K * P;
        if (P == 2) {
            if (need <= 64) kbest_uneven_one<2, 1>(a, smem_kbu);
            else kbest_uneven_one<2, 2>(a, smem_kbu);
        } else if (P == 4) {
            if (need <= 64) kbest_uneven_one<4, 1>(a, smem_kbu);
            else if (need <= 128) kbest_uneven_one<4, 2>(a, smem_kbu);
            else kbest_uneven_one<4, 4>(a, smem_kbu);
        } else {
            if (need <= 64) kbest_uneven_one<8, 1>(a, smem_kbu);
            else if (need <= 128) kbest_uneven_one<8, 2>(a, smem_kbu);
            else kbest_uneven_one<8, 4>(a, smem_kbu);
        }
        kb_wave_sync();  // the next frame reuses the LDS
    }
}

}  // namespace mimo

extern "C" int32_t kbest_detect_uneven(const mimo_frame_desc* desc, int32_t B, const float* R_flat,
                                       const float* z_flat, int32_t* sym_flat, float* pd, uint32_t* flags,
                                       int32_t* counter, int32_t grid, void* stream)
{
    using namespace mimo;
    if (B < 0 || grid < 0) return fail(MIMO_ERR_INVALID_ARG, "kbest_detect_uneven: B < 0 or grid < 0");
    if (B == 0) return MIMO_OK;
    if (!desc || !R_flat || !z_flat || !sym_flat || !pd || !flags || !counter)
        return fail(MIMO_ERR_INVALID_ARG, "kbest_detect_uneven: null pointer");
    hipStream_t st = (hipStream_t)stream;
    if (grid == 0) {
        int dev = 0, cus = 0;
        (void)hipGetDevice(&dev);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
        grid = 8 * (cus > 0 ? cus : 256);
    }
    if (grid > B) grid = B;
    // largest LDS need over the instantiations (KCAP <= 64, 8 groups)
    const size_t lds = gk_lds_bytes(64, (2 * UNEVEN_NWMAX + GK_LEVELS - 1) / GK_LEVELS);
    hipLaunchKernelGGL(reset_counter_kernel_kb, dim3(1), dim3(1), 0, st, counter);
    hipLaunchKernelGGL(kbest_uneven_kernel, dim3(grid), dim3(WAVE), lds, st, desc, B, R_flat, z_flat, sym_flat, pd,
                       flags, counter);
    return check_launch("kbest_detect_uneven");
}
