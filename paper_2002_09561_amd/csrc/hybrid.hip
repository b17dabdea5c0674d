// Hybrid SD / K-best detection (Sec. VI, SD-K-best) in deterministic rounds,
// one workgroup per frame: wave 0 is the Best-FS sphere-decoder master
// (Alg. 1 with the Best-FS list of Sec. IV-A), waves 1..W are K-best workers.
//
// The master's list is a depth-first stack, so every pool node at depth d is
// a child of the master's current path prefix at depth d-1.  The pool is
// therefore kept as the master path (a 4-bit digit per level) plus, per depth, a
// short sorted list of remaining siblings (pd, symbol): the left-most node is
// the best sibling of the deepest non-empty depth, the right-most node is
// the worst sibling of the shallowest one.
//
// One round:
//   A  master: pop left-most nodes until one lies inside the radius, expand
//      it (dot product of the path with row k of R, P child partial
//      distances, Eq. (inc)), sort the children, insert the ones inside the
//      radius at depth d+1 (best left-most) or offer the best leaf;
//   B  one thread hands right-most nodes to idle workers (pool >= 2 nodes);
//   C  every busy worker advances its K-best one level (K_w * P candidates
//      sorted in the wave by (pd bits, parent rank, child)); at the leaves it
//      offers its best survivor;
//   D  one thread takes the best offer by (pd, source) and shrinks the radius.
// A-C use the radius of the start of the round.
#include "common.hpp"

#include <utility>

namespace mimo {

struct HybArgs {
    const float* R;
    const float* z;
    int n;
    int W;
    int Kw;
    const int32_t* k_sched;
    int k_sched_stride;
    const float* radius2;
    int master_off;
    int64_t budget;
    int32_t* sym;
    float* pd;
    uint32_t* flags;
    int64_t* counters;
    // re-run mode: only frames whose finite radius left the drained pool
    // without a leaf (EMPTY_SPHERE, no FOUND or NONFINITE_INPUT) run again,
    // with r2 = +inf; flags keep EMPTY_SPHERE, counters accumulate
    int rerun;
};

__device__ inline void wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

constexpr int HY_DPW = 8;  // path digits (levels) per 32-bit word

struct HybLayout {
    int nw, stride, nd;  // words per path, padded stride, depths (steps of J levels: n / J + 1)
    size_t o_mpath, o_bpath, o_ppd, o_pc, o_lo, o_hi, o_mask, o_wst, o_wpath, o_wpd, o_sel, o_cand, o_sc, total;
    size_t o_r, o_z, o_rs;  // staged c R, z and row sums (when stage)
    size_t o_rowb;          // else each worker's copy of the row(s) of c R its step reads: [W][J][n]
    // P: children per step (pam^J)
    __host__ __device__ HybLayout(int n, int W, int Kw, int P, int J, int stage)
    {
        nw = (n + HY_DPW - 1) / HY_DPW;
        stride = nw + 1;
        nd = n / J + 1;
        const int Wc = W > 0 ? W : 1;
        size_t o = 0;
        o_mpath = o; o += 4 * nw;
        o_bpath = o; o += 4 * nw;
        o_ppd = o; o += 4 * (size_t)nd * P;
        o_pc = o; o += ((size_t)nd * P + 3) & ~(size_t)3;  // child index bytes
        o_lo = o; o += 4 * nd;
        o_hi = o; o += 4 * nd;
        o_mask = o; o += 4 * 9;
        o_wst = o; o += 4 * 8 * Wc;              // per worker: busy, depth, cnt, buf, isnew, newd, newc, newpd
        o_wpath = o; o += 4 * (size_t)Wc * 2 * Kw * stride;
        o_wpd = o; o += 4 * (size_t)Wc * 2 * Kw;
        o_sel = o; o += 4 * (size_t)Wc * Kw;
        o_cand = o; o += 4 * 3 * (Wc + 1);      // pd, ok, info per source
        o_sc = o; o += 64;                      // scalars
        o_r = o_z = o_rs = o_rowb = o;
        if (stage) {
            o_r = o; o += 4 * (size_t)r_packed_size(n);
            o_z = o; o += 4 * (size_t)n;
            o_rs = o; o += 4 * (size_t)n;
        } else {
            o_rowb = o; o += 4 * (size_t)Wc * J * n;
        }
        total = o;
    }
};

// scalar slots (int32 unless noted)
enum { SC_R2 = 0, SC_FOUND, SC_PSIZE, SC_DONE, SC_FLAGS, SC_EXP_LO, SC_EXP_HI, SC_ROUNDS, SC_STALE, SC_WEXP, SC_BUSY, SC_NEWW };

// a path holds one 4-bit PAM index per level (P <= 8), eight levels per word
__device__ inline int get_dig(const uint32_t* p, int j) { return (int)((p[j >> 3] >> (4 * (j & 7))) & 0xfu); }

__device__ inline uint32_t put_dig(uint32_t v, int lev, int c)
{
    const int sh = 4 * (lev & 7);
    return (v & ~(0xfu << sh)) | ((uint32_t)c << sh);
}

// the two digits of complex child c into the nibbles of the even level lev
// (real part, c % P) and lev + 1 (imaginary part, c / P) of one word
template <int P>
__device__ inline uint32_t put_pair(uint32_t v, int lev, int c)
{
    const int sh = 4 * (lev & 7);
    return (v & ~(0xffu << sh)) | ((uint32_t)(c % P) << sh) | ((uint32_t)(c / P) << (sh + 4));
}

// entry t of row k of c R: staged rows are scaled already
template <bool ST>
__device__ __forceinline__ float rget(const float* rk, int t, float cs)
{
    if constexpr (ST) return rk[t];
    else return cs * rk[t];
}

// sum of c R_kj over j > k: the staged sum, or lane-strided partial sums
// reduced over the wave (the staged sums are made the same way)
template <bool ST>
__device__ __forceinline__ float row_sum(const float* rk, int k, int n, const float* rs, float cs, int lane)
{
    if constexpr (ST) {
        return rs[k];
    } else {
        float v = 0.f;
        for (int t = 1 + lane; t < n - k; t += WAVE) v += cs * rk[t];
        return wave_sum(v);
    }
}

// Row k of R (entries t >= 1, lane-strided as copy_row_sum reads them) into
// registers: the next level's row, loaded one round ahead so that the load
// is in flight across the round's barriers.  pf_k records the row held.
constexpr int PF_MAX = 4;  // 4 x 64 entries: rows of up to 256 levels
__device__ inline void prefetch_row(const float* R, int n, int k, float (&pf)[PF_MAX], int lane)
{
    const float* rk = R + r_row_off(n, k);
#pragma unroll
    for (int i = 0; i < PF_MAX; ++i) {
        const int t = 1 + lane + WAVE * i;
        pf[i] = t < n - k ? rk[t] : 0.f;
    }
}

// copy_row_sum from prefetched entries (bit-identical: the same values, lanes and order)
__device__ inline float copy_row_sum_pf(const float* rk, int k, int n, float cs, float* dst, const float (&pf)[PF_MAX],
                                        int lane)
{
    float v = 0.f;
#pragma unroll
    for (int i = 0; i < PF_MAX; ++i) {
        const int t = 1 + lane + WAVE * i;
        if (t < n - k) {
            const float x = cs * pf[i];
            dst[t] = x;
            v += x;
        }
    }
    if (lane == 0) dst[0] = cs * rk[0];
    return wave_sum(v);
}

// Copy row k of R, scaled by c, into the worker's LDS buffer dst (entry t =
// c R[k][k + t]) with coalesced loads, and return the sum of entries t >= 1
// made as row_sum<false> makes it (the same lanes, order and reduction)
__device__ inline float copy_row_sum(const float* rk, int k, int n, float cs, float* dst, int lane)
{
    float v = 0.f;
    for (int t = 1 + lane; t < n - k; t += WAVE) {
        const float x = cs * rk[t];
        dst[t] = x;
        v += x;
    }
    if (lane == 0) dst[0] = cs * rk[0];
    return wave_sum(v);
}

// Copy the keep selected survivors' paths (sel[i] = parent rank * PC +
// child) to the next buffer from word w0 = lev / 8 on, the child's digit(s)
// put at level lev; all (survivor, word) pairs at once over the lanes
template <int P, int J>
__device__ inline void gather_paths(const uint32_t* pcur, uint32_t* pnxt, const int* sel, int keep, int lev, int nw,
                                    int stride, int lane)
{
    constexpr int PC = J == 1 ? P : P * P;
    const int w0 = lev >> 3, nwd = nw - w0, total = keep * nwd;
    const float inv = 1.0f / (float)nwd;  // (idx + 0.5) / nwd is 1/2 / nwd or more from the integers
    for (int idx = lane; idx < total; idx += WAVE) {
        const int i = (int)(((float)idx + 0.5f) * inv);
        const int wd = w0 + idx - i * nwd;
        const int m = sel[i];
        uint32_t v = pcur[(m / PC) * stride + wd];
        if (wd == w0) {
            if constexpr (J == 2) v = put_pair<P>(v, lev, m % PC);
            else v = put_dig(v, lev, m % PC);
        }
        pnxt[i * stride + wd] = v;
    }
}

// smallest 64-bit key over the wave (every lane gets it)
__device__ inline uint64_t wave_min_key(uint64_t v, int lane)
{
#pragma unroll
    for (int m = 1; m < WAVE; m <<= 1) {
        const uint64_t o = xor_lanes_u64(v, m, lane);
        v = o < v ? o : v;
    }
    return v;
}

// deepest (largest) / shallowest non-empty pool depth from the 9 mask
// words, read by the lanes of one wave (the pool holds a node)
__device__ inline int pool_deepest(const uint32_t* pmask, int lane)
{
    const uint32_t mk = lane < 9 ? pmask[lane] : 0u;
    const uint64_t nz = __ballot(mk != 0u);
    const int q = 63 - __clzll((long long)nz);
    const uint32_t mq = (uint32_t)__builtin_amdgcn_readlane((int)mk, q);
    return 32 * q + 31 - __clz(mq);
}

__device__ inline int pool_shallowest(const uint32_t* pmask, int lane)
{
    const uint32_t mk = lane < 9 ? pmask[lane] : 0u;
    const uint64_t nz = __ballot(mk != 0u);
    const int q = __ffsll((long long)nz) - 1;
    const uint32_t mq = (uint32_t)__builtin_amdgcn_readlane((int)mk, q);
    return 32 * q + __ffs(mq) - 1;
}

// Master expansion of a node at step depth d (child c of its parent step)
// on the complex-level tree: the children fix levels kh = lev - 1 and
// kl = lev - 2 at once.  Both centres come from the levels above kh
// (R[kl][kh] is the structural zero of the interleaved model); child
// (ih, il) has pd + e_h^2 + e_l^2 (Eq. (inc) twice, the upper level first).
// The children inside the radius are ranked by (pd, index) with one in-wave
// sort and stored at depth d + 1, or the best leaf is offered.
template <int P, bool ST>
__device__ void master_expand_pair(int n, const float* Rf, const float* zf, const float* rs, float cs, float r2r, int d,
                                   int c, float pd, uint32_t* mpath, float* ppd, uint8_t* pc, int* plo, int* phi,
                                   uint32_t* pmask, int* sc, float* cpd, int* cinfo, int* cok, int lane)
{
    constexpr int PC = P * P;
    const int lev = n - 2 * d;  // lowest level of the node's own step (n for the root)
    const int kh = lev - 1, kl = lev - 2;
    const float* rh = Rf + r_row_off(n, kh);
    const float* rl = Rf + r_row_off(n, kl);
    float ah = 0.f, al = 0.f, sh = 0.f, sl = 0.f;
    for (int j = lev + lane; j < n; j += WAVE) {
        const int sym = j == lev ? c % P : (j == lev + 1 ? c / P : get_dig(mpath, j));
        const float xh = rget<ST>(rh, j - kh, cs), xl = rget<ST>(rl, j - kl, cs);
        ah = fmaf(xh, (float)sym, ah);
        al = fmaf(xl, (float)sym, al);
        if constexpr (!ST) {
            sh += xh;
            sl += xl;
        }
    }
    ah = wave_sum(ah);
    al = wave_sum(al);
    if constexpr (ST) {  // R[kl][kh] is the structural zero: it adds nothing to the staged sum of row kl
        sh = rs[kh];
        sl = rs[kl];
    } else {
        sh = wave_sum(sh);
        sl = wave_sum(sl);
    }
    const float bh = zf[kh] - (2.f * ah - (float)(P - 1) * sh);
    const float bl = zf[kl] - (2.f * al - (float)(P - 1) * sl);
    const float dh = rget<ST>(rh, 0, cs), dl = rget<ST>(rl, 0, cs);
    if (!__builtin_isfinite(bh) || !__builtin_isfinite(bl) || !__builtin_isfinite(dh) || !__builtin_isfinite(dl)) {
        if (lane == 0) {  // uniform: NaN or inf in R or z
            sc[SC_DONE] = 1;
            atomicOr(reinterpret_cast<unsigned int*>(&sc[SC_FLAGS]), MIMO_FLAG_NONFINITE_INPUT);
        }
        return;
    }
    uint64_t key[1] = {~0ull};
    if (lane < PC) {
        const float eh = fmaf(-dh, (float)(2 * (lane / P) - (P - 1)), bh);
        const float el = fmaf(-dl, (float)(2 * (lane % P) - (P - 1)), bl);
        const float pdc = fmaf(el, el, fmaf(eh, eh, pd));
        if (pdc < r2r) key[0] = ((uint64_t)__float_as_uint(pdc) << 32) | (uint32_t)lane;
    }
    bitonic_sort<1>(key, lane);
    const int nk = __popcll(__ballot(key[0] != ~0ull));
    const float kpd = __uint_as_float((uint32_t)(key[0] >> 32));
    const int kc = (int)(uint32_t)key[0];
    if (kl == 0) {
        if (lane == 0 && nk > 0) {
            cpd[0] = kpd;
            cinfo[0] = kc;
            cok[0] = 1;
        }
    } else if (nk > 0) {
        const int dn = d + 1;
        if (lane < nk) {
            ppd[dn * PC + lane] = kpd;
            pc[dn * PC + lane] = (uint8_t)kc;
        }
        if (lane == 0) {
            plo[dn] = 0;
            phi[dn] = nk;
            pmask[dn >> 5] |= 1u << (dn & 31);
            sc[SC_PSIZE] += nk;
        }
    }
    if (lane == 0) {
        if (d > 0) mpath[lev >> 3] = put_pair<P>(mpath[lev >> 3], lev, c);  // the popped node joins the path
        uint32_t lo = (uint32_t)sc[SC_EXP_LO] + 1u;
        if (lo == 0u) sc[SC_EXP_HI] += 1;
        sc[SC_EXP_LO] = (int)lo;
    }
}

// One K-best step of a worker on the complex-level tree: each survivor s is
// given 64 / 2^ceil(log2 cnt) lanes for its two dot products; candidate
// m = s P^2 + c (c = ih P + il) sits at sort position m of 64 E keys
// ordered by (pd bits, m), i.e. (pd, parent rank, child) as in the oracle.
template <int P, int E, bool ST>
__device__ void worker_step_pair(int n, const float* Rf, const float* zf, const float* rs, float cs, float r2r,
                                 const int32_t* ks, int Kw, int w, int depth, int cnt, int buf, int* st, uint32_t* wp,
                                 float* wq, int* sel, int nw, int stride, int* sc, float* cpd, int* cinfo, int* cok,
                                 float* rowb, int lane)
{
    constexpr int PC = P * P;
    const int kh = n - 2 * depth - 1, kl = kh - 1;
    const uint32_t* pcur = wp + buf * Kw * stride;
    uint32_t* pnxt = wp + (buf ^ 1) * Kw * stride;
    const float* scur = wq + buf * Kw;
    float* snxt = wq + (buf ^ 1) * Kw;
    int Kt = ks ? __builtin_amdgcn_readfirstlane(ks[kl]) : Kw;  // K_t of the step's lower level
    Kt = Kt > Kw ? Kw : (Kt < 1 ? 1 : Kt);
    const float* rh = Rf + r_row_off(n, kh);
    const float* rl = Rf + r_row_off(n, kl);
    float sh, sl;
    if constexpr (ST) {  // the structural zero R[kl][kh] adds nothing to the staged sum of row kl
        sh = rs[kh];
        sl = rs[kl];
    } else {  // both rows into this worker's LDS buffers first, summed on the way (j > kh)
        float* bh = rowb + (size_t)w * 2 * n;
        float* bl = bh + n;
        sh = 0.f;
        sl = 0.f;
        for (int j = kh + 1 + lane; j < n; j += WAVE) {
            const float xh = cs * rh[j - kh], xl = cs * rl[j - kl];
            bh[j - kh] = xh;
            bl[j - kl] = xl;
            sh += xh;
            sl += xl;
        }
        if (lane == 0) {
            bh[0] = cs * rh[0];
            bl[0] = cs * rl[0];
        }
        sh = wave_sum(sh);
        sl = wave_sum(sl);
        wave_sync();
        rh = bh;
        rl = bl;
    }
    const int lg = 6 - (cnt <= 1 ? 0 : 32 - __clz(cnt - 1));  // log2 of the lanes per survivor
    const int G = 1 << lg, s = lane >> lg, g = lane & (G - 1);
    float ah = 0.f, al = 0.f;
    if (s < cnt) {
        const uint32_t* prow = pcur + s * stride;
        for (int wd = (kh + 1) / HY_DPW + g; wd < nw; wd += G) {
            const uint32_t dw = prow[wd];
            const int j0 = HY_DPW * wd;
            if (j0 > kh && j0 + HY_DPW <= n) {  // the whole word lies above the step
#pragma unroll
                for (int bb = 0; bb < HY_DPW; ++bb) {
                    const float v = (float)((dw >> (4 * bb)) & 0xfu);
                    ah = fmaf(rget<true>(rh, j0 + bb - kh, cs), v, ah);
                    al = fmaf(rget<true>(rl, j0 + bb - kl, cs), v, al);
                }
            } else {
#pragma unroll
                for (int bb = 0; bb < HY_DPW; ++bb) {
                    const int j = j0 + bb;
                    if (j > kh && j < n) {
                        const float v = (float)((dw >> (4 * bb)) & 0xfu);
                        ah = fmaf(rget<true>(rh, j - kh, cs), v, ah);
                        al = fmaf(rget<true>(rl, j - kl, cs), v, al);
                    }
                }
            }
        }
    }
    for (int m = 1; m < G; m <<= 1) {
        ah += shfl_xor_f(ah, m);
        al += shfl_xor_f(al, m);
    }
    const float bh = zf[kh] - (2.f * ah - (float)(P - 1) * sh);
    const float bl = zf[kl] - (2.f * al - (float)(P - 1) * sl);
    const float dh = rget<true>(rh, 0, cs), dl = rget<true>(rl, 0, cs);
    // a NaN or infinity in R or z: the frame's search stops after this round
    const bool bad = __ballot(!__builtin_isfinite(dh) || !__builtin_isfinite(dl) ||
                              (s < cnt && (!__builtin_isfinite(bh) || !__builtin_isfinite(bl)))) != 0;
    if (bad && lane == 0) {
        sc[SC_DONE] = 1;
        atomicOr(reinterpret_cast<unsigned int*>(&sc[SC_FLAGS]), MIMO_FLAG_NONFINITE_INPUT);
    }
    uint64_t key[E];
#pragma unroll
    for (int e = 0; e < E; ++e) {
        const int m = e * WAVE + lane, sm = m / PC, cc = m % PC;
        const int src = (sm < cnt ? sm : 0) << lg;
        const float bhs = shfl_f(bh, src), bls = shfl_f(bl, src);
        key[e] = ~0ull;
        if (sm < cnt && !bad) {
            const float eh = fmaf(-dh, (float)(2 * (cc / P) - (P - 1)), bhs);
            const float el = fmaf(-dl, (float)(2 * (cc % P) - (P - 1)), bls);
            const float pdc = fmaf(el, el, fmaf(eh, eh, scur[sm]));
            if (pdc < r2r) key[e] = ((uint64_t)__float_as_uint(pdc) << 32) | (uint32_t)m;
        }
    }
    int nvalid = 0;
#pragma unroll
    for (int e = 0; e < E; ++e) nvalid += __popcll(__ballot(key[e] != ~0ull));
    if (lane == 0) atomicAdd(&sc[SC_WEXP], cnt);
    if (nvalid == 0) {
        if (lane == 0) {
            st[0] = 0;
            atomicAnd(reinterpret_cast<unsigned int*>(&sc[SC_BUSY]), ~(1u << w));
        }
        return;
    }
    const int keep = Kt < nvalid ? Kt : nvalid;  // <= Kw <= 64
    // the keep smallest keys in order, lane i holding the i-th: by repeated
    // wave minima when keep is small against the sort network's depth
    // (about (6 + E) against E s (s + 1) / 2 exchanges per key, s = log2(64 E)),
    // else by sorting all 64 E keys
    constexpr int S = E == 1 ? 6 : (E == 2 ? 7 : (E == 4 ? 8 : 9));
    uint64_t res = ~0ull;
    if (keep * (6 + E) < E * S * (S + 1) / 2) {
        for (int i = 0; i < keep; ++i) {
            uint64_t m = key[0];
#pragma unroll
            for (int e = 1; e < E; ++e) m = key[e] < m ? key[e] : m;
            m = wave_min_key(m, lane);
#pragma unroll
            for (int e = 0; e < E; ++e) key[e] = key[e] == m ? ~0ull : key[e];  // keys are distinct
            res = lane == i ? m : res;
        }
    } else {
        bitonic_sort<E>(key, lane);
        res = key[0];
    }
    if (lane < keep) {
        snxt[lane] = __uint_as_float((uint32_t)(res >> 32));
        sel[lane] = (int)(uint32_t)res;
    }
    wave_sync();
    gather_paths<P, 2>(pcur, pnxt, sel, keep, kl, nw, stride, lane);
    if (lane == 0) {
        st[2] = keep;
        st[3] = buf ^ 1;
        st[1] = depth + 1;
        if (kl == 0) {  // leaves: offer the best survivor
            cpd[1 + w] = snxt[0];
            cinfo[1 + w] = buf ^ 1;
            cok[1 + w] = 1;
            st[0] = 0;
            atomicAnd(reinterpret_cast<unsigned int*>(&sc[SC_BUSY]), ~(1u << w));
        }
    }
}

// P: PAM points per real level; J: real levels per step (2: one complex
// symbol, P^2 children; the levels 2m+1, 2m of a step have the structural
// zero R[2m][2m+1] of the interleaved model, so both centres come from the
// levels above the step).  Pool depths count steps.  E: 64-key sort
// registers per lane of a complex-level worker.  ST: the frame's c R (c the
// PAM spacing), z and the sums of c R right of the diagonal of each row are
// copied to LDS first and every level reads them there.
// One sort register per lane (at most 64 candidates per worker step): at
// most 64 registers, eight waves per SIMD, so that eight 4-wave workgroups
// (3 workers) share a CU instead of seven at 68 registers; the compiler then
// keeps more scalars in vector-register lanes (100x100 64-QAM, 3 workers x 8:
// 48.8 -> 44.1 ms per 5x10^4 frames).
template <int P, int J, int E, bool ST>
__global__ void __launch_bounds__(1024, (E == 1 ? 8 : 1)) hybrid_kernel(HybArgs a)
{
    constexpr int PC = J == 1 ? P : P * P;  // children per step
    extern __shared__ unsigned char smem_hy[];
    const int frame = blockIdx.x;
    if (a.rerun) {  // uniform over the workgroup
        const uint32_t fl = a.flags[frame];
        if (!(fl & MIMO_FLAG_EMPTY_SPHERE) || (fl & (MIMO_FLAG_FOUND | MIMO_FLAG_NONFINITE_INPUT))) return;
    }
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int n = a.n, W = a.W, Kw = a.Kw;
    const HybLayout Lo(n, W, Kw, PC, J, ST);
    const int nw = Lo.nw, stride = Lo.stride;
    uint32_t* mpath = reinterpret_cast<uint32_t*>(smem_hy + Lo.o_mpath);
    uint32_t* bpath = reinterpret_cast<uint32_t*>(smem_hy + Lo.o_bpath);
    float* ppd = reinterpret_cast<float*>(smem_hy + Lo.o_ppd);
    uint8_t* pc = smem_hy + Lo.o_pc;  // the pool's child indices (< 64)
    int* plo = reinterpret_cast<int*>(smem_hy + Lo.o_lo);
    int* phi = reinterpret_cast<int*>(smem_hy + Lo.o_hi);
    uint32_t* pmask = reinterpret_cast<uint32_t*>(smem_hy + Lo.o_mask);
    int* wst = reinterpret_cast<int*>(smem_hy + Lo.o_wst);
    uint32_t* wpath = reinterpret_cast<uint32_t*>(smem_hy + Lo.o_wpath);
    float* wpd = reinterpret_cast<float*>(smem_hy + Lo.o_wpd);
    int* wsel = reinterpret_cast<int*>(smem_hy + Lo.o_sel);
    float* cpd = reinterpret_cast<float*>(smem_hy + Lo.o_cand);
    int* cok = reinterpret_cast<int*>(cpd + (W + 1));
    int* cinfo = cok + (W + 1);
    int* sc = reinterpret_cast<int*>(smem_hy + Lo.o_sc);
    float* sc_r2 = reinterpret_cast<float*>(sc + SC_R2);

    const float cs = pam_scale(P);
    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    const float* rs = nullptr;  // staged row sums
    float* rowb = reinterpret_cast<float*>(smem_hy + Lo.o_rowb);  // unstaged: the workers' row buffers
    if constexpr (ST) {  // every level reads c R, z and the row sums from LDS from here on
        float* Rs = reinterpret_cast<float*>(smem_hy + Lo.o_r);
        float* zs = reinterpret_cast<float*>(smem_hy + Lo.o_z);
        float* rss = reinterpret_cast<float*>(smem_hy + Lo.o_rs);
        const int rsz = (int)r_packed_size(n);
        for (int i = threadIdx.x; i < rsz; i += blockDim.x) Rs[i] = cs * Rf[i];
        for (int i = threadIdx.x; i < n; i += blockDim.x) zs[i] = zf[i];
        __syncthreads();
        const int nwave = blockDim.x / WAVE;
        for (int k = wave; k < n; k += nwave) {  // uniform per wave
            const float v = row_sum<false>(Rs + r_row_off(n, k), k, n, nullptr, 1.f, lane);
            if (lane == 0) rss[k] = v;
        }
        Rf = Rs;
        zf = zs;
        rs = rss;
    }
    const int32_t* ks = a.k_sched ? a.k_sched + (size_t)frame * a.k_sched_stride : nullptr;

    float pf[PF_MAX] = {0.f, 0.f, 0.f, 0.f};  // a worker's prefetched next row (R unstaged)
    int pf_k = -1;
    // ---- init
    for (int i = threadIdx.x; i < Lo.nd; i += blockDim.x) {
        plo[i] = 0;
        phi[i] = 0;
    }
    for (int i = threadIdx.x; i < nw; i += blockDim.x) {
        mpath[i] = 0;
        bpath[i] = 0;
    }
    for (int i = threadIdx.x; i < 9; i += blockDim.x) pmask[i] = 0;
    for (int i = threadIdx.x; i < 8 * (W > 0 ? W : 1); i += blockDim.x) wst[i] = 0;
    for (int i = threadIdx.x; i <= W; i += blockDim.x) cok[i] = 0;
    __syncthreads();
    if (threadIdx.x == 0) {
        *sc_r2 = a.radius2 ? a.radius2[frame] : INFINITY;
        sc[SC_FOUND] = 0;
        sc[SC_DONE] = 0;
        sc[SC_FLAGS] = 0;
        sc[SC_EXP_LO] = 0;
        sc[SC_EXP_HI] = 0;
        sc[SC_ROUNDS] = 0;
        sc[SC_STALE] = 0;
        sc[SC_WEXP] = 0;
        sc[SC_BUSY] = a.master_off && W >= 1 ? 1 : 0;
        sc[SC_NEWW] = 0;
        if (a.master_off) {
            sc[SC_PSIZE] = 0;
            if (W >= 1) {  // worker 0 starts at the root
                wst[0] = 1;   // busy
                wst[1] = 0;   // depth
                wst[2] = 1;   // survivors
                wst[3] = 0;   // buffer
                wst[4] = 0;   // not new
                wpd[0] = 0.f;
            }
        } else {  // the root is the only pool node (depth 0)
            ppd[0] = 0.f;
            pc[0] = 0;
            plo[0] = 0;
            phi[0] = 1;
            pmask[0] = 1u;
            sc[SC_PSIZE] = 1;
        }
    }
    __syncthreads();

    for (;;) {
        // ---- termination (uniform: every thread reads the same LDS state)
        const int busy_any = sc[SC_BUSY];
        const int64_t expanded = ((int64_t)(uint32_t)sc[SC_EXP_HI] << 32) | (uint32_t)sc[SC_EXP_LO];
        if (sc[SC_DONE]) break;  // non-finite input seen
        if (sc[SC_PSIZE] == 0 && !busy_any) {
            if (threadIdx.x == 0) sc[SC_FLAGS] |= MIMO_FLAG_CERTIFIED;
            break;
        }
        if (a.budget > 0 && expanded >= a.budget) {
            if (threadIdx.x == 0) sc[SC_FLAGS] |= MIMO_FLAG_BUDGET_EXHAUSTED;
            break;
        }
        const float r2r = *sc_r2;
        const uint32_t busy0 = (uint32_t)busy_any;  // the workers busy at the round start
        __syncthreads();  // everyone has read the round-start state

        // one K-best step of worker w (a node handed over this round is set up first)
        auto worker_advance = [&](const int w) {
            int* st = wst + 8 * w;
            uint32_t* wp = wpath + (size_t)w * 2 * Kw * stride;
            float* wq = wpd + (size_t)w * 2 * Kw;
            int* sel = wsel + (size_t)w * Kw;
            if (st[4]) {  // new node: survivor 0 = master prefix + its symbol(s)
                const int d = st[5], lev = n - d * J;
                uint32_t* dst = wp;  // buffer 0, survivor 0
                for (int i = lane; i < nw; i += WAVE) {
                    uint32_t v = mpath[i];
                    if (d > 0 && i == (lev >> 3)) {  // J = 2: lev is even, lev + 1 in the same word
                        if constexpr (J == 2) v = put_pair<P>(v, lev, st[6]);
                        else v = put_dig(v, lev, st[6]);
                    }
                    dst[i] = v;
                }
                if (lane == 0) {
                    wq[0] = reinterpret_cast<float*>(st)[7];
                    st[1] = d;
                    st[2] = 1;
                    st[3] = 0;
                    st[4] = 0;
                }
                wave_sync();
            }
            const int depth = __builtin_amdgcn_readfirstlane(st[1]), cnt = __builtin_amdgcn_readfirstlane(st[2]),
                      buf = __builtin_amdgcn_readfirstlane(st[3]);
            if constexpr (J == 2) {
                worker_step_pair<P, E, ST>(n, Rf, zf, rs, cs, r2r, ks, Kw, w, depth, cnt, buf, st, wp, wq, sel, nw,
                                           stride, sc, cpd, cinfo, cok, rowb, lane);
            } else {
            const int k = n - depth - 1;
            uint32_t* pcur = wp + buf * Kw * stride;
            uint32_t* pnxt = wp + (buf ^ 1) * Kw * stride;
            float* scur = wq + buf * Kw;
            float* snxt = wq + (buf ^ 1) * Kw;
            int Kt = ks ? __builtin_amdgcn_readfirstlane(ks[k]) : Kw;
            Kt = Kt > Kw ? Kw : (Kt < 1 ? 1 : Kt);
            const float* rk = Rf + r_row_off(n, k);
            // row sum (uniform) and per-survivor dot products: P lanes per survivor
            float rsum;
            if constexpr (ST) {
                rsum = rs[k];
            } else {  // the row into this worker's LDS buffer first (c R, summed on the way)
                float* bk = rowb + (size_t)w * n;
                rsum = pf_k == k ? copy_row_sum_pf(rk, k, n, cs, bk, pf, lane) : copy_row_sum(rk, k, n, cs, bk, lane);
                wave_sync();
                rk = bk;
                if (k > 0) {  // the row of the next level, in flight until the next step
                    prefetch_row(Rf, n, k - 1, pf, lane);
                    pf_k = k - 1;
                }
            }
            const int s = lane / P, cc = lane % P;
            float acc = 0.f;
            if (s < cnt) {
                const uint32_t* prow = pcur + s * stride;
                for (int wd = (k + 1) / HY_DPW + cc; wd < nw; wd += P) {
                    const uint32_t dw = prow[wd];
                    const int j0 = HY_DPW * wd;
                    if (j0 > k && j0 + HY_DPW <= n) {  // the whole word lies above level k
#pragma unroll
                        for (int bb = 0; bb < HY_DPW; ++bb)
                            acc = fmaf(rget<true>(rk, j0 + bb - k, cs), (float)((dw >> (4 * bb)) & 0xfu), acc);
                    } else {
#pragma unroll
                        for (int bb = 0; bb < HY_DPW; ++bb) {
                            const int j = j0 + bb;
                            if (j > k && j < n)
                                acc = fmaf(rget<true>(rk, j - k, cs), (float)((dw >> (4 * bb)) & 0xfu), acc);
                        }
                    }
                }
            }
#pragma unroll
            for (int m = 1; m < P; m <<= 1) acc += shfl_xor_f(acc, m);
            const float b = zf[k] - (2.f * acc - (float)(P - 1) * rsum);
            const float rkk = rget<true>(rk, 0, cs);
            // a NaN or infinity in R or z: the frame's search stops after this round
            const bool bad = __ballot(!__builtin_isfinite(rkk) || (s < cnt && !__builtin_isfinite(b))) != 0;
            if (bad && lane == 0) {
                sc[SC_DONE] = 1;
                atomicOr(reinterpret_cast<unsigned int*>(&sc[SC_FLAGS]), MIMO_FLAG_NONFINITE_INPUT);
            }
            uint64_t key[1] = {~0ull};
            if (s < cnt && !bad) {
                const float ee = fmaf(-rkk, (float)(2 * cc - (P - 1)), b);
                const float pdc = fmaf(ee, ee, scur[s]);
                if (pdc < r2r) key[0] = ((uint64_t)__float_as_uint(pdc) << 32) | (uint32_t)lane;
            }
            bitonic_sort<1>(key, lane);
            const int nvalid = __popcll(__ballot(key[0] != ~0ull));
            if (lane == 0) atomicAdd(&sc[SC_WEXP], cnt);
            if (nvalid == 0) {
                if (lane == 0) {
                    st[0] = 0;
                    atomicAnd(reinterpret_cast<unsigned int*>(&sc[SC_BUSY]), ~(1u << w));
                }
            } else {
                const int keep = Kt < nvalid ? Kt : nvalid;
                if (lane < keep) {
                    snxt[lane] = __uint_as_float((uint32_t)(key[0] >> 32));
                    sel[lane] = (int)(uint32_t)key[0];
                }
                wave_sync();
                gather_paths<P, 1>(pcur, pnxt, sel, keep, k, nw, stride, lane);
                if (lane == 0) {
                    st[2] = keep;
                    st[3] = buf ^ 1;
                    st[1] = depth + 1;
                    if (k == 0) {  // leaves: offer the best survivor
                        cpd[1 + w] = snxt[0];
                        cinfo[1 + w] = buf ^ 1;
                        cok[1 + w] = 1;
                        st[0] = 0;
                        atomicAnd(reinterpret_cast<unsigned int*>(&sc[SC_BUSY]), ~(1u << w));
                    }
                }
            }
            }
        };

        // ---- A: the master expands a node, while the workers busy since an
        // earlier round advance (C for them: neither reads what the other writes)
        if (wave >= 1 && wave <= W) {
            if ((busy0 >> (wave - 1)) & 1u) worker_advance(wave - 1);
        } else if (wave == 0 && !a.master_off) {
            int ok = 0, d = 0, c = 0;
            float pd = 0.f;
            // pop left-most nodes (deepest depth, best sibling) until one lies
            // inside the radius; the siblings of a depth are sorted by pd, so
            // when the best is outside, the whole depth is (each one counts
            // as a discarded pop)
            while (sc[SC_PSIZE] > 0) {  // uniform over wave 0
                const int dd = pool_deepest(pmask, lane);
                const int lo = __builtin_amdgcn_readfirstlane(plo[dd]), hi = __builtin_amdgcn_readfirstlane(phi[dd]);
                const float v = __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(ppd[dd * PC + lo])));
                const int take = v >= r2r ? hi - lo : 1;
                wave_sync();
                if (lane == 0) {
                    plo[dd] = lo + take;
                    if (lo + take == hi) pmask[dd >> 5] &= ~(1u << (dd & 31));
                    sc[SC_PSIZE] -= take;
                    if (v >= r2r) sc[SC_STALE] += take;
                }
                wave_sync();
                if (v < r2r) {
                    ok = 1;
                    d = dd;
                    c = pc[dd * PC + lo];
                    pd = v;
                    break;
                }
            }
            if constexpr (J == 2) {
                if (ok) master_expand_pair<P, ST>(n, Rf, zf, rs, cs, r2r, d, c, pd, mpath, ppd, pc, plo, phi, pmask, sc,
                                                  cpd, cinfo, cok, lane);
            } else {
            const int lev = n - d;  // level of the node's own symbol (n for the root)
            const int k = lev - 1;  // level its children fix
            float b = 0.f, rkk = 0.f;
            if (ok) {
                const float* rk = Rf + r_row_off(n, k);
                float acc = 0.f, rsum = 0.f;
                for (int t = 1 + lane; t < n - k; t += WAVE) {
                    const int j = k + t;
                    const int sym = (j == lev) ? c : get_dig(mpath, j);
                    const float r = rget<ST>(rk, t, cs);
                    acc = fmaf(r, (float)sym, acc);
                    if constexpr (!ST) rsum += r;
                }
                acc = wave_sum(acc);
                if constexpr (ST) rsum = rs[k];  // the same sums, made once
                else rsum = wave_sum(rsum);
                b = zf[k] - (2.f * acc - (float)(P - 1) * rsum);
                rkk = rget<ST>(rk, 0, cs);
                if (!__builtin_isfinite(b) || !__builtin_isfinite(rkk)) {  // uniform: NaN or inf in R or z
                    if (lane == 0) {
                        sc[SC_DONE] = 1;
                        atomicOr(reinterpret_cast<unsigned int*>(&sc[SC_FLAGS]), MIMO_FLAG_NONFINITE_INPUT);
                    }
                    ok = 0;
                }
            }
            if (ok) {
                float pdc = INFINITY;
                if (lane < P) {
                    const float ee = fmaf(-rkk, (float)(2 * lane - (P - 1)), b);
                    pdc = fmaf(ee, ee, pd);
                }
                // rank of each child by (pd, index)
                int rank = 0;
#pragma unroll
                for (int q = 0; q < P; ++q) {
                    const float o = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(pdc), q));
                    rank += (o < pdc) || (o == pdc && q < lane);
                }
                const bool keep = lane < P && pdc < r2r;
                const int nk = __popcll(__ballot(keep));
                if (k == 0) {
                    if (keep && rank == 0) {
                        cpd[0] = pdc;
                        cinfo[0] = lane;
                        cok[0] = 1;
                    }
                } else if (nk > 0) {
                    const int dn = d + 1;
                    if (keep) {
                        ppd[dn * P + rank] = pdc;
                        pc[dn * P + rank] = (uint8_t)lane;
                    }
                    if (lane == 0) {
                        plo[dn] = 0;
                        phi[dn] = nk;
                        pmask[dn >> 5] |= 1u << (dn & 31);
                        sc[SC_PSIZE] += nk;
                    }
                }
                if (lane == 0) {
                    if (d > 0) {  // the popped node's symbol joins the master path
                        mpath[lev >> 3] = put_dig(mpath[lev >> 3], lev, c);
                    }
                    uint32_t lo = (uint32_t)sc[SC_EXP_LO] + 1u;
                    if (lo == 0u) sc[SC_EXP_HI] += 1;
                    sc[SC_EXP_LO] = (int)lo;
                }
            }
            }
        }
        __syncthreads();

        // ---- B: idle workers, in order, take right-most nodes (shallowest
        // depth, worst sibling) while the pool holds two or more; the nodes
        // outside the radius at the right end of a depth are a run of the
        // sorted siblings and are discarded together, one pop each, as far
        // as the pool may shrink
        if (wave == 0) {
            uint64_t idle = ~(uint64_t)busy0 & ((1ull << W) - 1ull);  // idle at the round start
            while (idle) {  // uniform over wave 0
                const int w = __ffsll((long long)idle) - 1;
                idle &= idle - 1;
                bool given = false;
                while (sc[SC_PSIZE] >= 2) {
                    const int dd = pool_shallowest(pmask, lane);
                    const int lo = __builtin_amdgcn_readfirstlane(plo[dd]);
                    const int hi = __builtin_amdgcn_readfirstlane(phi[dd]);
                    const float vi = lane < hi - lo ? ppd[dd * PC + lo + lane] : 0.f;
                    const int nst = __popcll(__ballot(lane < hi - lo && vi >= r2r));
                    const int psz = sc[SC_PSIZE];
                    const int npop = nst > 0 ? (nst < psz - 1 ? nst : psz - 1) : 1;
                    wave_sync();
                    if (lane == 0) {
                        phi[dd] = hi - npop;
                        if (lo == hi - npop) pmask[dd >> 5] &= ~(1u << (dd & 31));
                        sc[SC_PSIZE] = psz - npop;
                        if (nst > 0) {
                            sc[SC_STALE] += npop;
                        } else {
                            int* st = wst + 8 * w;
                            st[0] = 1;
                            sc[SC_BUSY] |= 1 << w;
                            sc[SC_NEWW] |= 1 << w;
                            st[4] = 1;
                            st[5] = dd;
                            st[6] = pc[dd * PC + hi - 1];
                            reinterpret_cast<float*>(st)[7] = ppd[dd * PC + hi - 1];
                        }
                    }
                    wave_sync();
                    if (nst == 0) {
                        given = true;
                        break;
                    }
                }
                if (!given) break;  // fewer than two nodes: none for the later workers either
            }
        }
        __syncthreads();

        // ---- C for the workers given a node this round
        const uint32_t fresh = (uint32_t)sc[SC_NEWW];
        if (fresh) {  // uniform
            if (wave >= 1 && wave <= W && ((fresh >> (wave - 1)) & 1u)) worker_advance(wave - 1);
            __syncthreads();
        }

        // ---- D: merge offers (the smallest pd, the lowest source on ties),
        // shrink the radius once
        if (wave == 0) {
            const bool offer = lane <= W && cok[lane <= W ? lane : 0];
            const uint64_t okey = offer ? ((uint64_t)__float_as_uint(cpd[lane]) << 32) | (uint32_t)lane : ~0ull;
            const uint64_t bkey = wave_min_key(okey, lane);
            const float bpd = __uint_as_float((uint32_t)(bkey >> 32));
            if (bkey != ~0ull && bpd < *sc_r2) {  // uniform
                const int best = (int)(uint32_t)bkey;
                const uint32_t* src = best == 0 ? mpath
                                                : wpath + ((size_t)(best - 1) * 2 + cinfo[best]) * Kw * stride;
                for (int i = lane; i < nw; i += WAVE) {
                    uint32_t v = src[i];
                    if (best == 0 && i == 0) {  // the master's leaf: its path plus the child's digit(s) at the bottom
                        if constexpr (J == 2) v = put_pair<P>(v, 0, cinfo[0]);
                        else v = put_dig(v, 0, cinfo[0]);
                    }
                    bpath[i] = v;
                }
                wave_sync();
                if (lane == 0) {
                    *sc_r2 = bpd;
                    sc[SC_FOUND] = 1;
                }
            }
            if (lane <= W) cok[lane] = 0;
        }
        if (threadIdx.x == 0) {
            sc[SC_NEWW] = 0;
            uint32_t lo = (uint32_t)sc[SC_EXP_LO];
            const uint32_t add = (uint32_t)sc[SC_WEXP];
            const uint32_t nlo = lo + add;
            if (nlo < lo) sc[SC_EXP_HI] += 1;
            sc[SC_EXP_LO] = (int)nlo;
            sc[SC_WEXP] = 0;
            sc[SC_ROUNDS] += 1;
        }
        __syncthreads();
    }

    __syncthreads();
    const int nonfinite = (sc[SC_FLAGS] & MIMO_FLAG_NONFINITE_INPUT) != 0;
    const int found = sc[SC_FOUND] && !nonfinite;
    if (threadIdx.x == 0) {
        uint32_t fl = (uint32_t)sc[SC_FLAGS];
        if (found) fl |= MIMO_FLAG_FOUND;
        // the sphere is empty when the drained pool gave no leaf inside it
        else if ((fl & MIMO_FLAG_CERTIFIED) && !nonfinite) fl |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.rerun) fl |= MIMO_FLAG_EMPTY_SPHERE;
        if (a.flags) a.flags[frame] = fl;
        if (a.pd) a.pd[frame] = found ? *sc_r2 : INFINITY;
        if (a.counters) {
            const int64_t e = ((int64_t)(uint32_t)sc[SC_EXP_HI] << 32) | (uint32_t)sc[SC_EXP_LO];
            int64_t* c = a.counters + (size_t)frame * 4;
            if (a.rerun) {
                c[0] += e;
                c[1] += e * PC * J;
                c[2] += sc[SC_ROUNDS];
                c[3] += sc[SC_STALE];
            } else {
                c[0] = e;
                c[1] = e * PC * J;
                c[2] = sc[SC_ROUNDS];
                c[3] = sc[SC_STALE];
            }
        }
    }
    if (a.sym) {
        for (int m = threadIdx.x; m < n / 2; m += blockDim.x) {
            int v = 0;
            if (found) {
                const int ire = get_dig(bpath, 2 * m);
                const int iim = get_dig(bpath, 2 * m + 1);
                v = ire * P + iim;
            }
            a.sym[(size_t)frame * (n / 2) + m] = v;
        }
    }
}

template <int P, int J, int E>
static int32_t launch_hybrid(const HybArgs& a, int B, hipStream_t st, const char* name)
{
    constexpr int PC = J == 1 ? P : P * P;
    const int threads = WAVE * (1 + a.W);
    const HybLayout Ls(a.n, a.W, a.Kw, PC, J, 1), Lu(a.n, a.W, a.Kw, PC, J, 0);
    if (Lu.total > 160 * 1024)
        return fail(MIMO_ERR_UNSUPPORTED, "%s: %zu bytes of LDS needed (n_workers * k_worker too large)", name,
                    Lu.total);
    const void* fs = (const void*)hybrid_kernel<P, J, E, true>;
    const void* fu = (const void*)hybrid_kernel<P, J, E, false>;
    for (const auto& [f, L] : {std::pair<const void*, size_t>{fs, Ls.total}, {fu, Lu.total}}) {
        if (L > 64 * 1024 && L <= 160 * 1024) {
            hipError_t e = hipFuncSetAttribute(f, hipFuncAttributeMaxDynamicSharedMemorySize, (int)L);
            if (e != hipSuccess) return fail(MIMO_ERR_HIP, "%s: LDS attribute: %s", name, hipGetErrorString(e));
        }
    }
    // c R, z and the row sums in LDS when they fit and keep at least half of
    // the workgroups a CU holds without them (measured: staging wins at 1 of
    // 2 workgroups per CU, loses at 1 of 4)
    bool stage = false;
    if (Ls.total <= 160 * 1024) {
        int occ_s = 0, occ_u = 0;
        if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_s, fs, threads, Ls.total) != hipSuccess ||
            hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ_u, fu, threads, Lu.total) != hipSuccess)
            return fail(MIMO_ERR_HIP, "%s: occupancy query failed", name);
        stage = occ_s >= 1 && 2 * occ_s >= occ_u;
    }
    const HybLayout& Lo = stage ? Ls : Lu;
    if (stage) hipLaunchKernelGGL((hybrid_kernel<P, J, E, true>), dim3(B), dim3(threads), Lo.total, st, a);
    else hipLaunchKernelGGL((hybrid_kernel<P, J, E, false>), dim3(B), dim3(threads), Lo.total, st, a);
    return check_launch(name);
}

template <int J>
static int32_t launch_hybrid_pam(const HybArgs& a, int pam, int B, hipStream_t st, const char* name)
{
    if constexpr (J == 1) {
        switch (pam) {
        case 2: return launch_hybrid<2, 1, 1>(a, B, st, name);
        case 4: return launch_hybrid<4, 1, 1>(a, B, st, name);
        default: return launch_hybrid<8, 1, 1>(a, B, st, name);
        }
    } else {  // 64 E sort keys for the k_worker * pam^2 candidates of a worker step
        const int cand = a.Kw * pam * pam;
        const int E = cand <= 64 ? 1 : (cand <= 128 ? 2 : (cand <= 256 ? 4 : 8));
        switch (pam) {
        case 2:  // at most 64 * 4 candidates
            switch (E) {
            case 1: return launch_hybrid<2, 2, 1>(a, B, st, name);
            case 2: return launch_hybrid<2, 2, 2>(a, B, st, name);
            default: return launch_hybrid<2, 2, 4>(a, B, st, name);
            }
        case 4:
            switch (E) {
            case 1: return launch_hybrid<4, 2, 1>(a, B, st, name);
            case 2: return launch_hybrid<4, 2, 2>(a, B, st, name);
            case 4: return launch_hybrid<4, 2, 4>(a, B, st, name);
            default: return launch_hybrid<4, 2, 8>(a, B, st, name);
            }
        default:
            switch (E) {
            case 1: return launch_hybrid<8, 2, 1>(a, B, st, name);
            case 2: return launch_hybrid<8, 2, 2>(a, B, st, name);
            case 4: return launch_hybrid<8, 2, 4>(a, B, st, name);
            default: return launch_hybrid<8, 2, 8>(a, B, st, name);
            }
        }
    }
}

template <int J>
static int32_t hybrid_entry(const char* name, const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                            const float* radius2, int32_t n_workers, int32_t k_worker, const int32_t* k_sched,
                            int32_t k_sched_stride, int32_t master_off, int64_t node_budget, int32_t* sym, float* pd,
                            uint32_t* flags, int64_t* counters, void* stream)
{
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", name);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", name);
    if (n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: n_tx < 1", name);
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx > %d", name, MIMO_MAX_TX);
    if (n_workers < 0 || n_workers > MIMO_MAX_WORKERS)
        return fail(MIMO_ERR_INVALID_ARG, "%s: 0 <= n_workers <= %d", name, MIMO_MAX_WORKERS);
    if (J == 1 && (k_worker < 1 || k_worker * pam > MIMO_HYB_MAX_CAND))
        return fail(MIMO_ERR_INVALID_ARG, "%s: need k_worker >= 1 and k_worker * pam <= %d", name,
                    MIMO_HYB_MAX_CAND);
    if (J == 2 && (k_worker < 1 || k_worker > 64 || k_worker * pam * pam > MIMO_HYB_MAX_CAND_CPLX))
        return fail(MIMO_ERR_INVALID_ARG, "%s: need 1 <= k_worker <= 64 and k_worker * pam^2 <= %d", name,
                    MIMO_HYB_MAX_CAND_CPLX);
    if (master_off && n_workers < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: master_off needs a worker", name);
    if (node_budget < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: node_budget < 0", name);
    const int n = 2 * n_tx;
    if (k_sched && k_sched_stride != 0 && k_sched_stride != n)
        return fail(MIMO_ERR_INVALID_ARG, "%s: k_sched_stride must be 0 or n = %d", name, n);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", name);
    HybArgs a{R, z, n, n_workers, k_worker, k_sched, k_sched_stride, radius2, master_off, node_budget,
              sym, pd, flags, counters, 0};
    hipStream_t st = (hipStream_t)stream;
    const int32_t rc = launch_hybrid_pam<J>(a, pam, B, st, name);
    if (rc || !radius2) return rc;
    // frames whose finite radius left no leaf: again with r2 = +inf
    a.radius2 = nullptr;
    a.rerun = 1;
    return launch_hybrid_pam<J>(a, pam, B, st, name);
}

}  // namespace mimo

extern "C" int32_t sd_hybrid_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                    const float* radius2, int32_t n_workers, int32_t k_worker,
                                    const int32_t* k_sched, int32_t k_sched_stride, int32_t master_off,
                                    int64_t node_budget, int32_t* sym, float* pd, uint32_t* flags,
                                    int64_t* counters, void* stream)
{
    return mimo::hybrid_entry<1>("sd_hybrid_detect", R, z, B, n_tx, pam, radius2, n_workers, k_worker, k_sched,
                                 k_sched_stride, master_off, node_budget, sym, pd, flags, counters, stream);
}

extern "C" int32_t sd_hybrid_detect_complex(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                            const float* radius2, int32_t n_workers, int32_t k_worker,
                                            const int32_t* k_sched, int32_t k_sched_stride, int32_t master_off,
                                            int64_t node_budget, int32_t* sym, float* pd, uint32_t* flags,
                                            int64_t* counters, void* stream)
{
    return mimo::hybrid_entry<2>("sd_hybrid_detect_complex", R, z, B, n_tx, pam, radius2, n_workers, k_worker,
                                 k_sched, k_sched_stride, master_off, node_budget, sym, pd, flags, counters, stream);
}
