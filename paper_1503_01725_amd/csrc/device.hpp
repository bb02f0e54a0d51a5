// Device helpers for gfx950 kernels: the counter-based Philox4x32-10 generator
// (Salmon et al., SC'11), the per-particle uniform stream, and wave64 / block
// reductions.
#pragma once

#include "common.hpp"

namespace psl {
namespace dev {

constexpr uint32_t kTagSource = 1;     // sampling stream
constexpr uint32_t kTagTransport = 2;  // transport streams (sub 0 = source particle)

constexpr float kTwoPow24Inv = 5.9604644775390625e-8f;   // 2^-24

// Ten Philox4x32 rounds; the key is bumped by the Weyl constants between rounds.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t a0 = 0xD2511F53u * x0, b0 = __umulhi(0xD2511F53u, x0);
        const uint32_t a1 = 0xCD9E8D57u * x2, b1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t y0 = b1 ^ x1 ^ k0;
        const uint32_t y2 = b0 ^ x3 ^ k1;
        x0 = y0;
        x1 = a1;
        x2 = y2;
        x3 = a0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

// Uniform in [0, 1) from the top 24 bits; exact in FP32.
__device__ __forceinline__ float top24(uint32_t x) { return float(x >> 8) * kTwoPow24Inv; }

// The uniforms of one particle: key = seed, counter = (block, tag<<16 | sub,
// g_lo, g_hi); consumed four per block, in order.
struct Stream {
    uint32_t k0, k1, blk, tagsub, g0, g1;
    float u0, u1, u2, u3;
    int left;

    __device__ __forceinline__ void init(uint32_t seed_lo, uint32_t seed_hi, uint64_t g,
                                         uint32_t tag, uint32_t sub) {
        k0 = seed_lo;
        k1 = seed_hi;
        blk = 0;
        tagsub = (tag << 16) | (sub & 0xFFFFu);
        g0 = uint32_t(g);
        g1 = uint32_t(g >> 32);
        left = 0;
    }
    __device__ __forceinline__ void refill() {
        uint32_t x0 = blk, x1 = tagsub, x2 = g0, x3 = g1;
        philox4x32_10(x0, x1, x2, x3, k0, k1);
        u0 = top24(x0);
        u1 = top24(x1);
        u2 = top24(x2);
        u3 = top24(x3);
        ++blk;
        left = 4;
    }
    __device__ __forceinline__ float next() {
        if (left == 0) refill();
        const float r = u0;
        u0 = u1;
        u1 = u2;
        u2 = u3;
        --left;
        return r;
    }
};

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum(unsigned long long v) {
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Adds per-thread values of a whole block into global accumulators: one wave
// reduction, then lane 0 of every wave adds its partial (few waves per block).
template <int N>
__device__ __forceinline__ void block_add(double* dst, const double (&v)[N]) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int i = 0; i < N; ++i) {
        const double s = wave_sum(v[i]);
        if (lane == 0 && s != 0.0) atomicAdd(dst + i, s);
    }
}

__device__ __forceinline__ void block_add_u64(unsigned long long* dst, unsigned long long v) {
    const unsigned long long s = wave_sum(v);
    if ((threadIdx.x & 63) == 0 && s != 0ull) atomicAdd(dst, s);
}

// Reserves `want ? 1 : 0` slots per lane in a global stack with a single
// atomic per wave; returns the lane's slot (undefined if !want).
__device__ __forceinline__ uint32_t wave_reserve(bool want, uint32_t* counter) {
    const unsigned long long mask = __ballot(want);
    if (mask == 0ull) return 0u;
    const int lane = threadIdx.x & 63;
    const int leader = __ffsll((long long)mask) - 1;
    uint32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, uint32_t(__popcll(mask)));
    base = __shfl(base, leader, 64);
    const unsigned long long below = mask & ((1ull << lane) - 1ull);
    return base + uint32_t(__popcll(below));
}

}  // namespace dev
}  // namespace psl
