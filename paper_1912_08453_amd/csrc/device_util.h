// Device helpers shared by the HIP kernels of libpm (gfx950, wave64).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pm {

__device__ __forceinline__ int lane_id() { return (int)(threadIdx.x & 63u); }

__device__ __forceinline__ uint64_t ballot64(bool p) { return __ballot(p); }

// Lanes below this one in the wavefront.
__device__ __forceinline__ uint64_t lanemask_lt() {
    return (1ull << lane_id()) - 1ull;
}

__device__ __forceinline__ int32_t read_lane32(int32_t x, int l) {
    return __builtin_amdgcn_readlane(x, l);
}

__device__ __forceinline__ int64_t read_lane64(int64_t x, int l) {
    uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)x, l);
    uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)((uint64_t)x >> 32), l);
    return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ uint64_t read_lane_u64(uint64_t x, int l) {
    return (uint64_t)read_lane64((int64_t)x, l);
}

__device__ __forceinline__ int uniform(int x) { return __builtin_amdgcn_readfirstlane(x); }

__device__ __forceinline__ uint64_t shfl_xor_u64(uint64_t v, int mask, int width) {
    uint32_t lo = (uint32_t)v, hi = (uint32_t)(v >> 32);
    lo = (uint32_t)__shfl_xor((int)lo, mask, width);
    hi = (uint32_t)__shfl_xor((int)hi, mask, width);
    return ((uint64_t)hi << 32) | lo;
}

// Atomic OR of `bits` into element idx of an array of M (8/16/32/64-bit),
// through the naturally aligned 32- or 64-bit word that holds it.
template <typename M>
__device__ __forceinline__ void atomic_or_elem(M *base, int64_t idx, uint64_t bits) {
    if constexpr (sizeof(M) == 8) {
        atomicOr((unsigned long long *)(base + idx), (unsigned long long)bits);
    } else if constexpr (sizeof(M) == 4) {
        atomicOr((unsigned int *)(base + idx), (unsigned int)bits);
    } else {
        uintptr_t addr = (uintptr_t)(base + idx);
        unsigned int *word = (unsigned int *)(addr & ~(uintptr_t)3);
        unsigned int shift = (unsigned int)((addr & 3u) * 8u);
        atomicOr(word, (unsigned int)bits << shift);
    }
}

__device__ __forceinline__ void set_bit(uint64_t *bits, int64_t e) {
    atomicOr((unsigned long long *)(bits + (e >> 6)), 1ull << (e & 63));
}

// Bit e set for every lane with `valid`, with one atomic OR per run of
// lanes that target the same 64-bit word (a segmented OR over the lanes).
// All 64 lanes of the wavefront call it together; bit indices below 2^37.
// Lanes whose indices ascend with the lane number share the most atomics.
__device__ __forceinline__ void set_bits_wave(uint64_t *bits, int64_t e, bool valid) {
    const int lane = lane_id();
    const int32_t word = valid ? (int32_t)(e >> 6) : -1;
    const int b = (int)(e & 63);
    uint32_t lo = valid && b < 32 ? 1u << b : 0u;
    uint32_t hi = valid && b >= 32 ? 1u << (b - 32) : 0u;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const int32_t wu = __shfl_up(word, off);
        const uint32_t lu = __shfl_up(lo, off), hu = __shfl_up(hi, off);
        if (lane >= off && wu == word) {
            lo |= lu;
            hi |= hu;
        }
    }
    const int32_t wn = __shfl_down(word, 1);
    if (valid && (lane == 63 || wn != word))
        atomicOr((unsigned long long *)(bits + word), ((unsigned long long)hi << 32) | lo);
}

// Binary search of x in the sorted range col[lo, hi); returns index or -1.
__device__ __forceinline__ int64_t find_sorted(const int32_t *col, int64_t lo, int64_t hi,
                                               int32_t x) {
    while (lo < hi) {
        int64_t mid = lo + ((hi - lo) >> 1);
        int32_t y = col[mid];
        if (y == x) return mid;
        if (y < x) lo = mid + 1; else hi = mid;
    }
    return -1;
}

}  // namespace pm
