// Exact sphere decoding of one frame by the wavefronts of one workgroup
// (Alg. 1 with the Schnorr-Euchner child order of Sec. IV-A; the work
// distribution is the GPU counterpart of the dynamically balanced parallel SD
// of Sec. V-C: sub-problems handed to whichever worker is free, under one
// shared radius).
//
// The top d0 real levels of the frame's tree are enumerated at once (P^d0
// <= 512 prefixes): every prefix inside the initial radius is a sub-problem,
// and the list is sorted by prefix pd so that the likeliest subtrees go
// first.  Each wavefront takes the next sub-problem from an atomic counter
// and runs a depth-first search below it: per node the wave computes the
// centre b_k = z_k - sum_{j>k} (cR)_kj a_j (one term per lane, a wave sum),
// tries the nearest child first and the others in order of distance from the
// centre (the Schnorr-Euchner zig-zag, regenerated from the range of
// children tried at each level), and prunes a level at the first child whose
// pd is not below the radius.  A leaf inside the radius shrinks the radius of
// the whole workgroup (an atomic minimum on its bits in LDS) and is recorded
// with a 64-bit atomic minimum on (pd bits, wave).  A wave that finds the
// queue empty is done: no wave ever waits for another, so the workgroup ends
// when the last subtree is searched, or when the node budget is spent.
//
// R (scaled by the PAM spacing) and z are staged in LDS; each wave keeps its
// path, the per-level centres, parent pds and tried ranges, and its best leaf
// in LDS (3 KB for n <= 256).
#include "common.hpp"

namespace mimo {

constexpr int SP_MAX_ROOTS = 512;
constexpr int SP_LEVELS = 256;  // per-wave arrays: n <= 256

struct SpArgs {
    const float* R;
    const float* z;
    int n;
    int d0;        // levels fixed by a sub-problem's prefix
    int nroot_all; // P^d0
    const float* radius2;
    int64_t budget;  // node expansions per frame, 0 = none
    int redo;        // only frames left unfinished by an earlier search (see the header)
    int rerun;       // only frames whose search found no leaf inside a finite radius
    int32_t* sym;
    float* pd;
    uint32_t* flags;
    int64_t* counters;
};

struct SpLayout {
    size_t o_r, o_z, o_roots, o_wave, per_wave, o_sc, total;
    __host__ __device__ SpLayout(int n, int nwaves)
    {
        size_t o = 0;
        o_r = o;
        o += 4 * (size_t)n * (n + 1) / 2;
        o = (o + 15) & ~(size_t)15;
        o_z = o;
        o += 4 * (size_t)n;
        o = (o + 15) & ~(size_t)15;
        o_roots = o;
        o += 8 * (size_t)SP_MAX_ROOTS;
        per_wave = 4 * SP_LEVELS + 8 * SP_LEVELS;  // path, best path, lo, hi (bytes); centre, parent pd (floats)
        o_wave = o;
        o += per_wave * (size_t)nwaves;
        o_sc = o;
        o += 64;
        total = o;
    }
};

// scalar slots
enum { SPS_R2 = 0, SPS_QHEAD = 1, SPS_NROOT = 2, SPS_STOP = 3, SPS_FLAGS = 4, SPS_BEST = 6, SPS_NODES = 8 };

__device__ __forceinline__ int sp_load(const int* p)
{
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

__device__ __forceinline__ void sp_wave_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <int P>
__device__ __forceinline__ float sp_amp(int i)
{
    return (float)(2 * i - (P - 1));
}

template <int P>
__global__ void __launch_bounds__(1024) sd_parallel_kernel(SpArgs a)
{
    extern __shared__ __align__(16) unsigned char smem_sp[];
    const int frame = blockIdx.x;
    if (a.redo) {  // uniform over the workgroup
        const uint32_t fl = a.flags[frame];
        if ((fl & (MIMO_FLAG_CERTIFIED | MIMO_FLAG_NONFINITE_INPUT)) || !(fl & MIMO_FLAG_BUDGET_EXHAUSTED)) return;
    }
    if (a.rerun) {
        const uint32_t fl = a.flags[frame];
        if (!(fl & MIMO_FLAG_EMPTY_SPHERE) || (fl & (MIMO_FLAG_FOUND | MIMO_FLAG_NONFINITE_INPUT))) return;
    }
    const int n = a.n, d0 = a.d0;
    const int nwaves = (int)blockDim.x / WAVE;
    const SpLayout Lo(n, nwaves);
    float* Rs = reinterpret_cast<float*>(smem_sp + Lo.o_r);
    float* zs = reinterpret_cast<float*>(smem_sp + Lo.o_z);
    uint64_t* roots = reinterpret_cast<uint64_t*>(smem_sp + Lo.o_roots);
    int* sc = reinterpret_cast<int*>(smem_sp + Lo.o_sc);
    unsigned long long* best = reinterpret_cast<unsigned long long*>(sc + SPS_BEST);
    unsigned long long* nodes = reinterpret_cast<unsigned long long*>(sc + SPS_NODES);
    const int wave = (int)threadIdx.x >> 6, lane = (int)threadIdx.x & 63;
    const float cs = pam_scale(P);

    const float* Rf = a.R + (size_t)frame * r_packed_size(n);
    const float* zf = a.z + (size_t)frame * n;
    for (int i = threadIdx.x; i < (int)r_packed_size(n); i += blockDim.x) Rs[i] = cs * Rf[i];
    for (int i = threadIdx.x; i < n; i += blockDim.x) zs[i] = zf[i];
    float r2init = INFINITY;
    if (!a.rerun) {
        if (a.radius2) r2init = a.radius2[frame];
        else if (a.redo) r2init = a.pd[frame] * (1.f + 1e-4f);  // the earlier search's best leaf stays inside
    }
    if (!(r2init >= 0.f)) r2init = INFINITY;  // NaN or negative: no radius
    if (threadIdx.x == 0) {
        sc[SPS_R2] = (int)__float_as_uint(r2init);
        sc[SPS_QHEAD] = 0;
        sc[SPS_NROOT] = 0;
        sc[SPS_STOP] = 0;
        sc[SPS_FLAGS] = 0;
        *best = ~0ull;
        *nodes = 0ull;
    }
    __syncthreads();

    // ---- sub-problems: the prefixes of the top d0 levels inside the radius, by pd
    int64_t exp_w = 0, eval_w = 0;  // this wave's node expansions and child evaluations
    if (wave == 0) {
        uint64_t key[SP_MAX_ROOTS / WAVE];
        bool bad = false;
#pragma unroll
        for (int e = 0; e < SP_MAX_ROOTS / WAVE; ++e) {
            const int r = e * WAVE + lane;
            key[e] = ~0ull;
            if (r >= a.nroot_all) continue;
            float pd = 0.f;
            int rem = r, div = a.nroot_all / P;
            int dig[12];  // digits, top level first (d0 <= 9)
            for (int t = 0; t < d0; ++t) {
                dig[t] = rem / div;
                rem -= dig[t] * div;
                div = div > 1 ? div / P : 1;
            }
            for (int t = 0; t < d0; ++t) {
                const int k = n - 1 - t;
                const float* rk = Rs + r_row_off(n, k);
                float acc = 0.f;
                for (int u = 0; u < t; ++u) acc = fmaf(rk[(n - 1 - u) - k], sp_amp<P>(dig[u]), acc);
                const float b = zs[k] - acc;
                const float ee = fmaf(-rk[0], sp_amp<P>(dig[t]), b);
                pd = fmaf(ee, ee, pd);
                if (!__builtin_isfinite(b) || !__builtin_isfinite(rk[0])) bad = true;
            }
            if (pd < r2init) key[e] = ((uint64_t)__float_as_uint(pd) << 32) | (uint32_t)r;
        }
        if (__ballot(bad)) {
            if (lane == 0) {
                sc[SPS_FLAGS] |= MIMO_FLAG_NONFINITE_INPUT;
                sc[SPS_STOP] = 1;
            }
        } else {
            bitonic_sort<SP_MAX_ROOTS / WAVE>(key, lane);
            int cnt = 0;
#pragma unroll
            for (int e = 0; e < SP_MAX_ROOTS / WAVE; ++e) {
                cnt += __popcll(__ballot(key[e] != ~0ull));
                roots[e * WAVE + lane] = key[e];
            }
            if (lane == 0) sc[SPS_NROOT] = cnt;
        }
        // the enumeration's own work: every prefix of the top levels expanded once
        int nodes_top = 0, evals_top = 0;
        for (int t = 0, pw = 1; t < d0; ++t, pw *= P) {
            nodes_top += pw;
            evals_top += pw * P;
        }
        exp_w = nodes_top;
        eval_w = evals_top;
    }
    __syncthreads();

    // ---- depth-first search of the sub-problems, one wave each at a time
    unsigned char* xw = smem_sp + Lo.o_wave + Lo.per_wave * (size_t)wave;
    unsigned char* bx = xw + SP_LEVELS;
    unsigned char* lo = bx + SP_LEVELS;
    unsigned char* hi = lo + SP_LEVELS;
    float* bw = reinterpret_cast<float*>(hi + SP_LEVELS);
    float* pp = bw + SP_LEVELS;
    float my_best = INFINITY;
    const int nroot = sc[SPS_NROOT];
    const int kr = n - d0;  // lowest level a prefix fixes

    // a leaf inside the radius: shrink the radius, record it, keep its path
    auto record = [&](float pd) {
        if (lane == 0) {
            atomicMin(reinterpret_cast<unsigned*>(sc + SPS_R2), __float_as_uint(pd));
            atomicMin(best, ((unsigned long long)__float_as_uint(pd) << 32) | (unsigned)wave);
        }
        if (pd < my_best) {
            my_best = pd;
            for (int j = lane; j < n; j += WAVE) bx[j] = xw[j];
        }
        sp_wave_sync();
    };

    for (;;) {
        if (sp_load(sc + SPS_STOP)) break;
        int qi = 0;
        if (lane == 0) qi = atomicAdd(sc + SPS_QHEAD, 1);
        qi = __builtin_amdgcn_readfirstlane(__shfl(qi, 0, WAVE));
        if (qi >= nroot) break;
        const uint64_t rk = roots[qi];
        const float pdr = __uint_as_float((uint32_t)(rk >> 32));
        if (!(pdr < __uint_as_float((uint32_t)sp_load(sc + SPS_R2)))) continue;  // pruned by a smaller radius since
        const int r = (int)(uint32_t)rk;
        if (lane < d0) {  // lane t sets level n-1-t
            int div = 1;
            for (int t = lane + 1; t < d0; ++t) div *= P;
            xw[n - 1 - lane] = (unsigned char)((r / div) % P);
        }
        sp_wave_sync();
        if (kr == 0) {  // the prefix is a whole leaf
            record(pdr);
            continue;
        }
        int k = kr - 1;
        float pdpar = pdr;
        bool down = true;
        for (;;) {
            if (sp_load(sc + SPS_STOP)) break;
            const float r2 = __uint_as_float((uint32_t)sp_load(sc + SPS_R2));
            if (down) {
                // centre of level k from the path above it
                const float* rkr = Rs + r_row_off(n, k);
                float acc = 0.f;
                for (int t = 1 + lane; t < n - k; t += WAVE) acc = fmaf(rkr[t], sp_amp<P>(xw[k + t]), acc);
                acc = wave_sum(acc);
                const float b = zs[k] - acc, rkk = rkr[0];
                if (!__builtin_isfinite(b) || !__builtin_isfinite(rkk)) {
                    if (lane == 0) {
                        atomicOr(sc + SPS_FLAGS, (int)MIMO_FLAG_NONFINITE_INPUT);
                        atomicExch(sc + SPS_STOP, 1);
                    }
                    break;
                }
                ++exp_w;
                if (a.budget > 0) {
                    unsigned long long old = 0;
                    if (lane == 0) old = atomicAdd(nodes, 1ull);
                    old = __shfl(old, 0, WAVE);
                    if (old >= (unsigned long long)a.budget) {
                        if (lane == 0) {
                            atomicOr(sc + SPS_FLAGS, (int)MIMO_FLAG_BUDGET_EXHAUSTED);
                            atomicExch(sc + SPS_STOP, 1);
                        }
                        break;
                    }
                }
                // the nearest child first (any child serves if rkk is 0)
                const float u = fminf(fmaxf(rintf(0.5f * (b / rkk + (float)(P - 1))), 0.f), (float)(P - 1));
                const int i0 = __builtin_isfinite(u) ? (int)u : 0;
                const float ee = fmaf(-rkk, sp_amp<P>(i0), b);
                const float pd = fmaf(ee, ee, pdpar);
                ++eval_w;
                if (pd < r2) {
                    if (lane == 0) xw[k] = (unsigned char)i0;
                    sp_wave_sync();
                    if (k == 0) {
                        // its siblings lie no closer: the level is done
                        record(pd);
                        k = 1;
                        down = false;
                    } else {
                        if (lane == 0) {
                            bw[k] = b;
                            pp[k] = pdpar;
                            lo[k] = (unsigned char)i0;
                            hi[k] = (unsigned char)i0;
                        }
                        sp_wave_sync();
                        pdpar = pd;
                        --k;
                    }
                } else {
                    ++k;  // the nearest child is outside: so are the others
                    down = false;
                }
            } else {
                if (k >= kr) break;  // back at the prefix: the sub-problem is searched
                // next sibling at level k in order of distance from the centre
                const float b = bw[k], pdp = pp[k], rkk = Rs[r_row_off(n, k)];
                const int l = lo[k], h = hi[k];
                int c = -1;
                if (l > 0 && h < P - 1) {
                    const float dl = fabsf(fmaf(-rkk, sp_amp<P>(l - 1), b));
                    const float dh = fabsf(fmaf(-rkk, sp_amp<P>(h + 1), b));
                    c = dh < dl ? h + 1 : l - 1;
                } else if (l > 0) {
                    c = l - 1;
                } else if (h < P - 1) {
                    c = h + 1;
                }
                if (c < 0) {
                    ++k;
                    continue;
                }
                const float ee = fmaf(-rkk, sp_amp<P>(c), b);
                const float pd = fmaf(ee, ee, pdp);
                ++eval_w;
                if (pd < r2) {
                    if (lane == 0) {
                        xw[k] = (unsigned char)c;
                        if (c < l) lo[k] = (unsigned char)c;
                        else hi[k] = (unsigned char)c;
                    }
                    sp_wave_sync();
                    pdpar = pd;
                    --k;
                    down = true;
                } else {
                    ++k;  // the nearer remaining sibling is outside: the level is done
                }
            }
        }
    }
    // per-wave counts into LDS, then the frame's outputs
    unsigned long long* cnt2 = reinterpret_cast<unsigned long long*>(smem_sp + Lo.o_roots);  // the roots are done
    __syncthreads();
    if (threadIdx.x < 2) cnt2[threadIdx.x] = 0ull;
    __syncthreads();
    if (lane == 0) {
        atomicAdd(cnt2, (unsigned long long)exp_w);
        atomicAdd(cnt2 + 1, (unsigned long long)eval_w);
    }
    __syncthreads();
    const unsigned long long bk = *best;
    const uint32_t fl = (uint32_t)sc[SPS_FLAGS];
    const bool found = bk != ~0ull && !(fl & MIMO_FLAG_NONFINITE_INPUT);
    const bool certified = !(fl & (MIMO_FLAG_BUDGET_EXHAUSTED | MIMO_FLAG_NONFINITE_INPUT));
    if (threadIdx.x == 0) {
        uint32_t out = fl;
        if (found) out |= MIMO_FLAG_FOUND;
        if (certified) out |= MIMO_FLAG_CERTIFIED;
        if (certified && !found) out |= MIMO_FLAG_EMPTY_SPHERE;  // searched again with r2 = +inf
        if (a.rerun) out |= MIMO_FLAG_EMPTY_SPHERE;
        a.flags[frame] = out;
        a.pd[frame] = found ? __uint_as_float((uint32_t)(bk >> 32)) : INFINITY;
        if (a.counters) {
            int64_t* c = a.counters + (size_t)frame * 4;
            if (a.redo || a.rerun) {
                c[0] += (int64_t)cnt2[0];
                c[1] += (int64_t)cnt2[1];
            } else {
                c[0] = (int64_t)cnt2[0];
                c[1] = (int64_t)cnt2[1];
                c[2] = 0;
                c[3] = 0;
            }
        }
    }
    // symbols of the winning wave's leaf
    const int nw = n / 2;
    const int win = found ? (int)(uint32_t)bk : 0;
    const unsigned char* bw_win = smem_sp + Lo.o_wave + Lo.per_wave * (size_t)win + SP_LEVELS;
    for (int i = threadIdx.x; i < nw; i += blockDim.x)
        a.sym[(size_t)frame * nw + i] = found ? (int)bw_win[2 * i] * P + (int)bw_win[2 * i + 1] : 0;
}

// waves per workgroup: as many (16 at most) as the LDS of a compute unit holds
static int sp_waves(int n)
{
    for (int w = 16; w >= 1; w >>= 1)
        if (SpLayout(n, w).total <= 160 * 1024) return w;
    return 0;
}

template <int P>
static int32_t launch_sp(const SpArgs& a0, int B, hipStream_t st)
{
    SpArgs a = a0;
    int d0 = 0, pw = 1;
    while (pw * P <= SP_MAX_ROOTS && d0 < a.n) {
        pw *= P;
        ++d0;
    }
    a.d0 = d0;
    a.nroot_all = pw;
    const int w = sp_waves(a.n);
    if (w == 0) return fail(MIMO_ERR_UNSUPPORTED, "sd_parallel_detect: n = %d does not fit the LDS", a.n);
    const size_t lds = SpLayout(a.n, w).total;
    const void* k = (const void*)sd_parallel_kernel<P>;
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute(k, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return fail(MIMO_ERR_HIP, "sd_parallel_detect: LDS attribute: %s", hipGetErrorString(e));
    }
    hipLaunchKernelGGL(sd_parallel_kernel<P>, dim3(B), dim3(w * WAVE), lds, st, a);
    return check_launch("sd_parallel_detect");
}

static int32_t dispatch_sp(const SpArgs& a, int pam, int B, hipStream_t st)
{
    switch (pam) {
    case 2: return launch_sp<2>(a, B, st);
    case 4: return launch_sp<4>(a, B, st);
    default: return launch_sp<8>(a, B, st);
    }
}

}  // namespace mimo

extern "C" int32_t sd_parallel_detect(const float* R, const float* z, int32_t B, int32_t n_tx, int32_t pam,
                                      const float* radius2, int64_t budget, int32_t redo, int32_t* sym, float* pd,
                                      uint32_t* flags, int64_t* counters, void* stream)
{
    using namespace mimo;
    const char* who = "sd_parallel_detect";
    if (B < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: B < 0", who);
    if (pam != 2 && pam != 4 && pam != 8) return fail(MIMO_ERR_INVALID_ARG, "%s: pam must be 2, 4 or 8", who);
    if (n_tx < 1) return fail(MIMO_ERR_INVALID_ARG, "%s: n_tx < 1", who);
    if (n_tx > MIMO_MAX_TX) return fail(MIMO_ERR_UNSUPPORTED, "%s: n_tx > %d", who, MIMO_MAX_TX);
    if (budget < 0) return fail(MIMO_ERR_INVALID_ARG, "%s: budget < 0", who);
    if (redo != 0 && redo != 1) return fail(MIMO_ERR_INVALID_ARG, "%s: redo must be 0 or 1", who);
    if (B == 0) return MIMO_OK;
    if (!R || !z || !sym || !pd || !flags) return fail(MIMO_ERR_INVALID_ARG, "%s: null pointer", who);
    SpArgs a{R, z, 2 * n_tx, 0, 0, radius2, budget, redo, 0, sym, pd, flags, counters};
    hipStream_t st = (hipStream_t)stream;
    int32_t rc = dispatch_sp(a, pam, B, st);
    if (rc) return rc;
    // frames whose finite radius held no leaf: searched again with r2 = +inf
    SpArgs r = a;
    r.radius2 = nullptr;
    r.redo = 0;
    r.rerun = 1;
    return dispatch_sp(r, pam, B, st);
}
