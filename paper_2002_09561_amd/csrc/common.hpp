// Shared device/host helpers of the gfx950 sphere-decoder library.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/mimo_sd.h"

namespace mimo {

constexpr int WAVE = 64;

// error reporting (thread-local text behind mimo_last_error)
int32_t fail(int32_t code, const char* fmt, ...);
int32_t check_launch(const char* what);

// PAM spacing scale c = sqrt(3 / (2 (P^2 - 1))) of a unit-energy square QAM.
__host__ __device__ inline float pam_scale(int P)
{
    return P == 2 ? 0.70710678118654752f : (P == 4 ? 0.31622776601683794f : 0.15430334996209191f);
}

// offset of row k of the packed level-order R (n real levels)
__host__ __device__ inline int64_t r_row_off(int n, int k)
{
    return (int64_t)(n - 1 - k) * (n - k) / 2;
}

__host__ __device__ inline int64_t r_packed_size(int n) { return (int64_t)n * (n + 1) / 2; }

// Exchange with lane ^ j for a compile-time j (after unrolling), without
// the LDS unit: DPP for j = 1, 2 (quad permutes), 4 (rotations by 12 and 4
// within a row of 16: lane + 4 for lanes with bit 2 clear, lane - 4 for the
// others) and 8 (rotation by 8 within a row); the gfx950 row swaps for 16
// (permlane16_swap of v with itself: rows 0 and 1, 2 and 3 exchanged) and 32
// (permlane32_swap: halves exchanged).  Any other j uses a permute.
__device__ __forceinline__ uint32_t xor_lanes(uint32_t v, int j, int lane)
{
    switch (j) {
    case 1: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0xB1, 0xF, 0xF, false);
    case 2: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x4E, 0xF, 0xF, false);
    case 4: {
        const uint32_t up = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x12C, 0xF, 0xF, false);
        const uint32_t dn = (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x124, 0xF, 0xF, false);
        return (lane & 4) ? dn : up;
    }
    case 8: return (uint32_t)__builtin_amdgcn_mov_dpp((int)v, 0x128, 0xF, 0xF, false);
    case 16: {
        const auto r = __builtin_amdgcn_permlane16_swap(v, v, false, false);
        return (lane & 16) ? r[0] : r[1];
    }
    case 32: {
        const auto r = __builtin_amdgcn_permlane32_swap(v, v, false, false);
        return (lane & 32) ? r[0] : r[1];
    }
    default: return (uint32_t)__builtin_amdgcn_ds_bpermute(((lane ^ j) & (WAVE - 1)) << 2, (int)v);
    }
}

__device__ __forceinline__ uint64_t xor_lanes_u64(uint64_t v, int j, int lane)
{
    const uint32_t lo = xor_lanes((uint32_t)v, j, lane), hi = xor_lanes((uint32_t)(v >> 32), j, lane);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline float shfl_f(float v, int src) { return __shfl(v, src, WAVE); }
// exchange with lane ^ m (all lanes active; DPP or swizzle when m is a
// compile-time power of two below 32)
__device__ __forceinline__ float shfl_xor_f(float v, int m)
{
    const int lane = __lane_id();
    return __builtin_bit_cast(float, xor_lanes(__builtin_bit_cast(uint32_t, v), m, lane));
}

__device__ inline uint64_t shfl_xor_u64(uint64_t v, int m)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl_xor(lo, m, WAVE);
    hi = __shfl_xor(hi, m, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline uint64_t shfl_u64(uint64_t v, int src)
{
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = __shfl(lo, src, WAVE);
    hi = __shfl(hi, src, WAVE);
    return ((uint64_t)hi << 32) | lo;
}

__device__ inline float wave_sum(float v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += shfl_xor_f(v, m);
    return v;
}

__device__ inline uint64_t wave_min_u64(uint64_t v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        uint64_t o = shfl_xor_u64(v, m);
        v = o < v ? o : v;
    }
    return v;
}

// Sort of one register of keys within groups of LIM lanes (LIM = 16, 32 or
// 64), ascending, or descending with DESC.  Two sorted runs are merged by
// comparing each lane with its mirror image in the block (lane ^ (size - 1))
// and then with lane ^ j for falling j, so which key a lane keeps depends on
// one lane bit per stage: six lane masks in all, where a network of
// alternating directions needs one per stage, more than the scalar registers
// hold beside the rest of a kernel (the spilled masks cost two lane reads per
// stage).  Mirrors within 4, 8 and 16 lanes are single DPP moves.  Beyond
// rows of 16 the run to be mirrored is reversed in place instead: the odd
// rows by a row mirror under a row mask before the 32-lane merge, and the
// upper 32 lanes by sorting their complements (the opposite order) before the
// 64-lane merge.  Stages across rows (lane ^ 16, lane ^ 32) take both keys of
// a pair from one row swap of each word, so no lane select is needed.
template <bool DESC>
__device__ __forceinline__ bool sn_before(uint64_t x, uint64_t y)  // x goes first
{
    return DESC ? y < x : x < y;
}

// lane bit m clear: the key that goes first of key and its partner's p
template <bool DESC>
__device__ __forceinline__ uint64_t sn_keep(uint64_t key, uint64_t p, int lane, int m)
{
    return (sn_before<DESC>(p, key) != ((lane & m) != 0)) ? p : key;
}

template <int CTRL>
__device__ __forceinline__ uint64_t sn_dpp(uint64_t v)
{
    const uint32_t lo = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)v, CTRL, 0xF, 0xF, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_mov_dpp((int)(uint32_t)(v >> 32), CTRL, 0xF, 0xF, false);
    return ((uint64_t)hi << 32) | lo;
}

// compare-exchange with lane ^ J, J = 16 or 32: after a row swap of a word
// with itself, its first result holds the pair's lower-lane word and its
// second the upper-lane word, in both lanes of the pair
template <int J, bool DESC>
__device__ __forceinline__ uint64_t sn_pair(uint64_t key, int lane)
{
    static_assert(J == 16 || J == 32, "row swaps exchange 16 or 32 lanes");
    const uint32_t lo = (uint32_t)key, hi = (uint32_t)(key >> 32);
    uint64_t a, b;
    if constexpr (J == 16) {
        const auto l = __builtin_amdgcn_permlane16_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane16_swap(hi, hi, false, false);
        a = ((uint64_t)h[0] << 32) | l[0];
        b = ((uint64_t)h[1] << 32) | l[1];
    } else {
        const auto l = __builtin_amdgcn_permlane32_swap(lo, lo, false, false);
        const auto h = __builtin_amdgcn_permlane32_swap(hi, hi, false, false);
        a = ((uint64_t)h[0] << 32) | l[0];
        b = ((uint64_t)h[1] << 32) | l[1];
    }
    return (sn_before<DESC>(b, a) != ((lane & J) != 0)) ? b : a;
}

// rows 1 and 3 reversed in place (row mirror written to those rows only)
__device__ __forceinline__ uint64_t sn_rev_odd_rows(uint64_t v)
{
    const int lo = (int)(uint32_t)v, hi = (int)(uint32_t)(v >> 32);
    const uint32_t rl = (uint32_t)__builtin_amdgcn_update_dpp(lo, lo, 0x140, 0xA, 0xF, false);
    const uint32_t rh = (uint32_t)__builtin_amdgcn_update_dpp(hi, hi, 0x140, 0xA, 0xF, false);
    return ((uint64_t)rh << 32) | rl;
}

// the half-cleaner stages lane ^ 8, 4, 2, 1 (in order within rows of 16
// when each row holds a bitonic sequence)
template <bool DESC>
__device__ __forceinline__ uint64_t sn_clean16(uint64_t key, int lane)
{
    key = sn_keep<DESC>(key, sn_dpp<0x128>(key), lane, 8);  // row rotation by 8 = lane ^ 8
    key = sn_keep<DESC>(key, xor_lanes_u64(key, 4, lane), lane, 4);
    key = sn_keep<DESC>(key, sn_dpp<0x4E>(key), lane, 2);
    return sn_keep<DESC>(key, sn_dpp<0xB1>(key), lane, 1);
}

template <int LIM, bool DESC = false>
__device__ __forceinline__ void sort_lanes(uint64_t& key, int lane)
{
    static_assert(LIM == 16 || LIM == 32 || LIM == 64, "groups of 16, 32 or 64 lanes");
    const uint64_t cm = (LIM == 64 && (lane & 32)) ? ~0ull : 0ull;
    key ^= cm;
    key = sn_keep<DESC>(key, sn_dpp<0xB1>(key), lane, 1);   // lane ^ 1
    key = sn_keep<DESC>(key, sn_dpp<0x1B>(key), lane, 2);   // lane ^ 3
    key = sn_keep<DESC>(key, sn_dpp<0xB1>(key), lane, 1);
    key = sn_keep<DESC>(key, sn_dpp<0x141>(key), lane, 4);  // lane ^ 7: half-row mirror
    key = sn_keep<DESC>(key, sn_dpp<0x4E>(key), lane, 2);   // lane ^ 2
    key = sn_keep<DESC>(key, sn_dpp<0xB1>(key), lane, 1);
    key = sn_keep<DESC>(key, sn_dpp<0x140>(key), lane, 8);  // lane ^ 15: row mirror
    key = sn_keep<DESC>(key, xor_lanes_u64(key, 4, lane), lane, 4);
    key = sn_keep<DESC>(key, sn_dpp<0x4E>(key), lane, 2);
    key = sn_keep<DESC>(key, sn_dpp<0xB1>(key), lane, 1);
    if constexpr (LIM >= 32) {
        key = sn_rev_odd_rows(key);
        key = sn_pair<16, DESC>(key, lane);
        key = sn_clean16<DESC>(key, lane);
    }
    if constexpr (LIM == 64) {
        key ^= cm;  // the upper half now runs the other way
        key = sn_pair<32, DESC>(key, lane);
        key = sn_pair<16, DESC>(key, lane);
        key = sn_clean16<DESC>(key, lane);
    }
}

// a bitonic register of 64 keys put in order (ascending, or descending with DESC)
template <bool DESC = false>
__device__ __forceinline__ uint64_t merge_lanes(uint64_t key, int lane)
{
    key = sn_pair<32, DESC>(key, lane);
    key = sn_pair<16, DESC>(key, lane);
    return sn_clean16<DESC>(key, lane);
}

// In-wave sort of 64*E keys, ascending by position e*64 + lane: every
// register sorted by sort_lanes (even ones ascending, odd ones descending),
// then bitonic merges of registers 2, 4, ... E wide: the stages between
// registers compare them whole, the stages within one are merge_lanes.
template <int E>
__device__ inline void bitonic_sort(uint64_t (&key)[E], int lane)
{
    constexpr int N = WAVE * E;
#pragma unroll
    for (int e = 0; e < E; ++e) {
        if (E > 1 && (e & 1)) sort_lanes<WAVE, true>(key[e], lane);
        else sort_lanes<WAVE, false>(key[e], lane);
    }
#pragma unroll
    for (int size = 2 * WAVE; size <= N; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j >= WAVE; j >>= 1) {
            const int je = j / WAVE;
#pragma unroll
            for (int e = 0; e < E; ++e) {
                const int pe = e ^ je;
                if (pe > e) {
                    const bool asc = ((e * WAVE) & size) == 0;
                    const uint64_t a = key[e], b = key[pe];
                    const bool sw = asc ? (a > b) : (a < b);
                    key[e] = sw ? b : a;
                    key[pe] = sw ? a : b;
                }
            }
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (((e * WAVE) & size) != 0) key[e] = merge_lanes<true>(key[e], lane);
            else key[e] = merge_lanes<false>(key[e], lane);
        }
    }
}

}  // namespace mimo
