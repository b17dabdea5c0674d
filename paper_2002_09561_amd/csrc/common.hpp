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

// In-wave bitonic sort of 64*E keys, ascending by position e*64 + lane.
template <int E>
__device__ inline void bitonic_sort(uint64_t (&key)[E], int lane)
{
    constexpr int N = WAVE * E;
#pragma unroll
    for (int size = 2; size <= N; size <<= 1) {
#pragma unroll
        for (int j = size >> 1; j > 0; j >>= 1) {
            if (j >= WAVE) {
                const int je = j / WAVE;
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const int pe = e ^ je;
                    if (pe > e) {
                        const bool asc = (((e * WAVE + lane) & size) == 0);
                        uint64_t a = key[e], b = key[pe];
                        bool sw = asc ? (a > b) : (a < b);
                        key[e] = sw ? b : a;
                        key[pe] = sw ? a : b;
                    }
                }
            } else {
#pragma unroll
                for (int e = 0; e < E; ++e) {
                    const uint64_t o = xor_lanes_u64(key[e], j, lane);
                    // keep the smaller key iff this lane's half and the block's
                    // direction agree; keys are distinct except the ~0 padding
                    const bool take_max = ((((e * WAVE + lane) & size) != 0) != ((lane & j) != 0));
                    const bool take_o = (o < key[e]) != take_max;
                    key[e] = take_o ? o : key[e];
                }
            }
        }
    }
}

}  // namespace mimo
