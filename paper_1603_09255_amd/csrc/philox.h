// Device Philox4x32-10 (Salmon, Moraes, Dror & Shaw, "Parallel random
// numbers: as easy as 1, 2, 3", SC'11): ten rounds, each two 32x32->64
// multiplications whose high halves are mixed with the other counter words
// and the round key; the key advances by the Weyl constants between rounds.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace spegg {

struct Words4 {
    uint32_t v[4];
};

__device__ __forceinline__ Words4 philox(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0,
                                         uint32_t k1) {
#pragma unroll
    for (int round = 0; round < 10; ++round) {
        // full 64-bit products: one v_mad_u64_u32 each instead of a
        // separate low and high multiply
        const uint64_t pa = (uint64_t)0xD2511F53u * c0, pb = (uint64_t)0xCD9E8D57u * c2;
        const uint32_t lo_a = (uint32_t)pa, hi_a = (uint32_t)(pa >> 32);
        const uint32_t lo_b = (uint32_t)pb, hi_b = (uint32_t)(pb >> 32);
        // From the third round on every counter word differs between lanes:
        // each three-way XOR is then one v_bitop3_b32 (truth table 0x96)
        // instead of two VALU XORs.  The first two rounds keep plain XORs,
        // so that words shared by the wave are combined on the scalar unit.
        uint32_t n0, n2;
        if (round >= 2) {
            n0 = __builtin_amdgcn_bitop3_b32(hi_b, c1, k0, 0x96);
            n2 = __builtin_amdgcn_bitop3_b32(hi_a, c3, k1, 0x96);
        } else {
            n0 = hi_b ^ c1 ^ k0;
            n2 = hi_a ^ c3 ^ k1;
        }
        c0 = n0;
        c1 = lo_b;
        c2 = n2;
        c3 = lo_a;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    Words4 w;
    w.v[0] = c0;
    w.v[1] = c1;
    w.v[2] = c2;
    w.v[3] = c3;
    return w;
}

// One random word of a replicate's stream: block `blk` of stream `stream`
// for individual/slot `index` in generation `gen`, component `comp`.
struct Rng {
    uint32_t k0, k1, c3;
    __device__ __forceinline__ Words4 block(uint32_t index, uint32_t stream, uint32_t blk, uint32_t gen) const {
        return philox(index, (stream << 24) | blk, gen, c3, k0, k1);
    }
    // word q of the stream read as one sequence (block q/4, component q%4)
    __device__ __forceinline__ uint32_t seq(uint32_t index, uint32_t stream, uint32_t q, uint32_t gen) const {
        const Words4 w = block(index, stream, q >> 2, gen);
        const uint32_t c = q & 3u;
        return c == 0 ? w.v[0] : c == 1 ? w.v[1] : c == 2 ? w.v[2] : w.v[3];
    }
};

// Uniform index in [0, n) from the 64-bit word lo | hi << 32.
__device__ __forceinline__ uint32_t uniform_index(uint32_t lo, uint32_t hi, uint32_t n) {
    return (uint32_t)__umul64hi(((uint64_t)hi << 32) | lo, (uint64_t)n);
}

// Smallest k with x < T[k]; T is nondecreasing and T[len-1] = 2^32.
__device__ __forceinline__ uint32_t table_draw(const uint64_t *__restrict__ T, uint32_t len, uint32_t x) {
    if ((uint64_t)x < T[0]) return 0;
    uint32_t lo = 1, hi = len - 1;  // answer in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if ((uint64_t)x < T[mid]) hi = mid; else lo = mid + 1;
    }
    return lo;
}

// Number of entries of the nondecreasing T[0..len) that are <= x.
__device__ __forceinline__ uint32_t table_count_le(const uint64_t *__restrict__ T, uint32_t len, uint32_t x) {
    uint32_t lo = 0, hi = len;
    while (lo < hi) {
        const uint32_t mid = (lo + hi) >> 1;
        if (T[mid] <= (uint64_t)x) lo = mid + 1; else hi = mid;
    }
    return lo;
}

}  // namespace spegg
