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
        // full 64-bit products: one v_mad_u64_u32 gives both halves
        const uint64_t p0 = uint64_t(0xD2511F53u) * x0, p1 = uint64_t(0xCD9E8D57u) * x2;
        const uint32_t a0 = uint32_t(p0), b0 = uint32_t(p0 >> 32);
        const uint32_t a1 = uint32_t(p1), b1 = uint32_t(p1 >> 32);
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

// The same per-particle stream with its uniforms buffered in LDS, so that the
// Philox blocks of a wavefront are generated together.  A lane that runs dry
// at its own draw site would call the generator with only itself active, and
// in a wavefront of 64 lanes some lane runs dry at almost every site; instead
// the whole wavefront tops its buffers up at one point of the loop (topup),
// where every lane with room generates at once, and the loop consumes at
// most what the top-up guarantees (pop), carrying unfinished work over to the
// next iteration.  The sequence of values each history consumes is unchanged.
//
// Lane t of a workgroup of kLanes threads owns the column pool[j * kLanes + t]
// for ring slots j < R (bank-conflict free for any per-lane slot).  The key is
// fixed for the launch, so it stays in scalar registers.
template <int R, int kLanes>
struct PoolStream {
    static_assert((R & (R - 1)) == 0 && R >= 8, "ring size must be a power of two >= 8");
    const uint32_t k0, k1;
    uint32_t blk, tagsub, g0, g1;
    uint32_t head, cnt;
    float* col;

    __device__ __forceinline__ PoolStream(float* pool, uint32_t seed_lo, uint32_t seed_hi)
        : k0(seed_lo), k1(seed_hi), blk(0), tagsub(0), g0(0), g1(0), head(0), cnt(0),
          col(pool + threadIdx.x) {}

    // Counter of the particle's stream: (block, tag<<16 | sub, g_lo, g_hi).
    __device__ __forceinline__ void init(uint64_t g, uint32_t tag, uint32_t sub) {
        blk = 0;
        tagsub = (tag << 16) | (sub & 0xFFFFu);
        g0 = uint32_t(g);
        g1 = uint32_t(g >> 32);
        head = 0;
        cnt = 0;
    }
    // Wave-uniform call: until no active lane holds fewer than `need`
    // uniforms, every active lane holding fewer than `fill` appends the next
    // block of four (need <= fill <= R - 3).
    __device__ __forceinline__ void topup(bool active, uint32_t need, uint32_t fill) {
        while (__ballot(active && cnt < need) != 0ull) {
            if (active && cnt < fill) {
                uint32_t x0 = blk, x1 = tagsub, x2 = g0, x3 = g1;
                philox4x32_10(x0, x1, x2, x3, k0, k1);
                ++blk;
                const uint32_t t = head + cnt;
                col[((t + 0u) & (R - 1)) * kLanes] = top24(x0);
                col[((t + 1u) & (R - 1)) * kLanes] = top24(x1);
                col[((t + 2u) & (R - 1)) * kLanes] = top24(x2);
                col[((t + 3u) & (R - 1)) * kLanes] = top24(x3);
                cnt += 4;
            }
        }
    }
    // Next uniform; the caller guarantees cnt > 0.
    __device__ __forceinline__ float pop() {
        const float r = col[head * kLanes];
        head = (head + 1u) & (R - 1);
        --cnt;
        return r;
    }
    // Next uniform for a lane on its own (no wave-wide call): an empty ring
    // takes the next block of four first.  For rare events whose number of
    // uniforms is not bounded in advance (rejection loops).
    __device__ __forceinline__ float next() {
        if (cnt == 0u) {
            uint32_t x0 = blk, x1 = tagsub, x2 = g0, x3 = g1;
            philox4x32_10(x0, x1, x2, x3, k0, k1);
            ++blk;
            col[((head + 0u) & (R - 1)) * kLanes] = top24(x0);
            col[((head + 1u) & (R - 1)) * kLanes] = top24(x1);
            col[((head + 2u) & (R - 1)) * kLanes] = top24(x2);
            col[((head + 3u) & (R - 1)) * kLanes] = top24(x3);
            cnt = 4u;
        }
        return pop();
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

// Per-thread ledger and event counters, flushed once per block at the end of
// a kernel.  The tally keeps kStripes copies of the accumulators and block b
// adds into copy b % kStripes, so that no address sees more than a handful of
// atomics per launch (same-address atomics serialise in the L2).
constexpr int kStripes = 64;
constexpr int kStatWords = L_N + C_N;

// Event counts are 32-bit per lane (a lane sees far fewer than 2^32 events in
// one launch) and widened to 64 bits in the flush.
struct LocalStats {
    double l[L_N];
    uint32_t c[C_N];
    __device__ LocalStats() {
#pragma unroll
        for (int i = 0; i < L_N; ++i) l[i] = 0.0;
#pragma unroll
        for (int i = 0; i < C_N; ++i) c[i] = 0u;
    }
};

// Every thread of the block must call this (it synchronises the block).
__device__ __forceinline__ void flush_stats(double* stats, const LocalStats& s) {
    __shared__ double red_l[L_N][16];
    __shared__ unsigned long long red_c[C_N][16];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < L_N; ++i) {
        const double v = wave_sum(s.l[i]);
        if (lane == 0) red_l[i][w] = v;
    }
#pragma unroll
    for (int i = 0; i < C_N; ++i) {
        const unsigned long long v = wave_sum(static_cast<unsigned long long>(s.c[i]));
        if (lane == 0) red_c[i][w] = v;
    }
    __syncthreads();
    double* mine = stats + (blockIdx.x % kStripes) * kStatWords;
    const int t = threadIdx.x;
    if (t < L_N) {
        double v = 0.0;
        for (int k = 0; k < nw; ++k) v += red_l[t][k];
        if (v != 0.0) atomicAdd(mine + t, v);
    } else if (t < L_N + C_N) {
        unsigned long long v = 0ull;
        for (int k = 0; k < nw; ++k) v += red_c[t - L_N][k];
        if (v != 0ull) atomicAdd(reinterpret_cast<unsigned long long*>(mine + L_N) + (t - L_N), v);
    }
    __syncthreads();
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
