// Learned 3D dose denoiser: a 4-level U-Net (two 3x3x3 conv + ReLU per level,
// 2x2x2 max pooling down, 2x2x2 stride-2 transposed conv up, skip
// concatenation, 1x1x1 head plus the scaled input dose) trained with Adam on
// MSE.  Activations and weights are BF16 in channels-last layout
// ([position][channel]), accumulation is FP32 on the MFMA units; weight
// gradients and the master weights are FP32.  3x3x3 convolutions run as
// direct brick kernels (input brick staged once in LDS for all 27 taps)
// where the grid and channels fit their tiles, everything else as an
// implicit GEMM.
#include <cmath>
#include <cstring>
#include <memory>
#include <vector>

#include "common.hpp"

namespace psl {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float floatx4 __attribute__((ext_vector_type(4)));

constexpr int kLevels = 4;
constexpr int kBK = 32;    // K of one MFMA (16 x 16 x 32)
constexpr int kKT = 64;    // K of one LDS tile (two MFMA K steps per barrier)
constexpr int kLdsPad = 8;

__device__ __forceinline__ float bf2f(uint16_t h) { return __uint_as_float(uint32_t(h) << 16); }
__device__ __forceinline__ uint16_t f2bf(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7F800000u) == 0x7F800000u) return uint16_t(u >> 16);   // inf / nan
    u += 0x7FFFu + ((u >> 16) & 1u);                                  // round to nearest even
    return uint16_t(u >> 16);
}

// A channels-last BF16 view: element (pos, c) at p[pos * stride + off + c].
// Positions are split into (z, y, x) by multiply-shift division by W and H
// (and by W/2, H/2 for the coarse grid under a transposed convolution): for
// n < 2^31, n / d = (umulhi(n, mul) + n) >> sh with sh = ceil(log2 d) and
// mul = floor(2^32 (2^sh - d) / d) + 1.  C is a power of two (cs = log2 C).
struct View {
    uint16_t* p;
    int D, H, W, C, stride, off;
    uint32_t wm, ws, hm, hs;       // division by W, H
    uint32_t w2m, w2s, h2m, h2s;   // division by W/2, H/2
    int cs;
};

enum Mode { kConvFwd = 0, kConvBwdData, kConvWgrad, kTconvFwd, kTconvBwdData, kTconvWgrad };

struct GemmArgs {
    View a;              // conv/tconv input (fwd, wgrad) or output gradient (bwd-data)
    View b;              // output (fwd, bwd-data) or output gradient (wgrad)
    const uint16_t* wt;  // packed weights B^T [N][K] (fwd / bwd-data)
    const uint16_t* wfrag;   // the same in the brick kernel's operand order (frag_elems)
    const float* bias;   // fwd: [C_out]
    View mask;           // bwd-data: multiply by (mask > 0) if mask.p
    float* wgrad;        // wgrad: FP32 gradient in the reference layout
    float* partial;      // wgrad: [splits][M][N] FP32 per-split sums (reduced afterwards)
    int M, N, K;
    int cin, cout;       // channels of the layer (real, not padded)
    int cout_sh;         // log2(cout) (cout is a power of two)
    int relu;
    int k_per_split;     // wgrad: positions per blockIdx.z
    View pool;           // direct conv fwd: 2x2x2 max-pooled output if pool.p
    uint8_t* arg;        //   and the index (0-7) of each maximum, [P/8][C]
    // direct conv fwd, one workgroup over all output channels: the 1x1x1 head
    // pred = dose + head_b + head_w . out per position if head_out (FP32 [P]);
    // with skip_store the layer's own output is not written
    const float* head_w;
    const float* head_b;
    const float* head_dose;
    float* head_out;
    int skip_store;
};

__device__ __forceinline__ void pos3(int m, int D, int H, int W, int& z, int& y, int& x) {
    x = m % W;
    const int t = m / W;
    y = t % H;
    z = t / H;
}

__device__ __forceinline__ uint32_t fdiv(uint32_t n, uint32_t mul, uint32_t sh) {
    return (__umulhi(n, mul) + n) >> sh;
}

// (z, y, x) of position m on the view's grid / on its half-resolution grid
__device__ __forceinline__ void pos3v(const View& v, int m, int& z, int& y, int& x) {
    const uint32_t q = fdiv(uint32_t(m), v.wm, v.ws);
    x = m - int(q) * v.W;
    const uint32_t r = fdiv(q, v.hm, v.hs);
    y = int(q) - int(r) * v.H;
    z = int(r);
}
__device__ __forceinline__ void pos3c(const View& v, int m, int& z, int& y, int& x) {
    const uint32_t q = fdiv(uint32_t(m), v.w2m, v.w2s);
    x = m - int(q) * (v.W >> 1);
    const uint32_t r = fdiv(q, v.h2m, v.h2s);
    y = int(q) - int(r) * (v.H >> 1);
    z = int(r);
}

__device__ __forceinline__ uint4 load8(const View& v, int pos, int c) {
    return *reinterpret_cast<const uint4*>(v.p + size_t(pos) * v.stride + v.off + c);
}

// 8 consecutive K values of row `row` (direct loads) ------------------------
template <int MODE>
__device__ __forceinline__ uint4 load_a_row(const GemmArgs& g, int m, int k) {
    const uint4 zero = {0u, 0u, 0u, 0u};
    if (m >= g.M || k >= g.K) return zero;
    const View& v = g.a;
    if (MODE == kConvFwd || MODE == kConvBwdData) {
        const int tap = k >> v.cs, c = k & (v.C - 1);
        int z, y, x;
        pos3v(v, m, z, y, x);
        z += tap / 9 - 1;
        y += (tap / 3) % 3 - 1;
        x += tap % 3 - 1;
        if (z < 0 || z >= v.D || y < 0 || y >= v.H || x < 0 || x >= v.W) return zero;
        return load8(v, (z * v.H + y) * v.W + x, c);
    } else if (MODE == kTconvFwd) {
        return load8(v, m, k);
    } else {   // kTconvBwdData: m is a coarse voxel, v the fine-grid gradient;
               // k = abc * cout + o picks child abc, channel o
        const int abc = k >> g.cout_sh, o = k & (g.cout - 1);
        int z, y, x;
        pos3c(v, m, z, y, x);
        const int cz = 2 * z + (abc >> 2), cy = 2 * y + ((abc >> 1) & 1), cx = 2 * x + (abc & 1);
        return load8(v, (cz * v.H + cy) * v.W + cx, o);
    }
}

// 8 consecutive rows at one K value (transposed loads, weight gradients) ----
// A rows: output channels (conv) / input channels (tconv) at position k.
template <int MODE>
__device__ __forceinline__ uint4 load_a_col(const GemmArgs& g, int row, int k) {
    const uint4 zero = {0u, 0u, 0u, 0u};
    if (row >= g.M || k >= g.K) return zero;
    if (MODE == kConvWgrad) return load8(g.b, k, row);     // dY[pos][o..o+7]
    return load8(g.a, k, row);                             // tconv: X[pos][c..c+7]
}

// B^T rows n..n+7 at position k.
template <int MODE>
__device__ __forceinline__ uint4 load_b_col(const GemmArgs& g, int n, int k) {
    const uint4 zero = {0u, 0u, 0u, 0u};
    if (n >= g.N || k >= g.K) return zero;
    int z, y, x;
    if (MODE == kConvWgrad) {
        const View& v = g.a;
        const int tap = n >> v.cs, c = n & (v.C - 1);
        pos3v(v, k, z, y, x);
        z += tap / 9 - 1;
        y += (tap / 3) % 3 - 1;
        x += tap % 3 - 1;
        if (z < 0 || z >= v.D || y < 0 || y >= v.H || x < 0 || x >= v.W) return zero;
        return load8(v, (z * v.H + y) * v.W + x, c);
    } else {   // kTconvWgrad: n = abc * cout + o, dY at the child voxel of position k
        const View& v = g.a;   // coarse grid
        const int abc = n >> g.cout_sh, o = n & (g.cout - 1);
        pos3v(v, k, z, y, x);
        const int cz = 2 * z + (abc >> 2), cy = 2 * y + ((abc >> 1) & 1), cx = 2 * x + (abc & 1);
        return load8(g.b, (cz * (2 * v.H) + cy) * (2 * v.W) + cx, o);
    }
}

// Tiles of BM x BN outputs per workgroup of four waves, each wave 32 x 32
// (2 x 2 MFMA tiles of 16 x 16): 64 x 64, or 128 x 32 / 32 x 128 when one
// GEMM dimension is only 32 (the outermost level's channels), so that no
// wave computes padding.
template <int MODE, int BM, int BN>
__global__ void __launch_bounds__(256) k_gemm(GemmArgs g) {
    static_assert(BM * BN == 4096 && BM % 32 == 0 && BN % 32 == 0, "four 32 x 32 wave tiles");
    constexpr int WN = BN / 32;   // waves along N
    __shared__ uint16_t As[BM][kKT + kLdsPad];
    __shared__ uint16_t Bs[BN][kKT + kLdsPad];
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int m0 = blockIdx.x * BM, n0 = blockIdx.y * BN;
    constexpr bool kWgrad = MODE == kConvWgrad || MODE == kTconvWgrad;
    int k_lo = 0, k_hi = g.K;
    if (kWgrad) {
        k_lo = blockIdx.z * g.k_per_split;
        k_hi = min(g.K, k_lo + g.k_per_split);
    }
    floatx4 acc[2][2];
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = floatx4{0.f, 0.f, 0.f, 0.f};
    const int wr = (w / WN) * 32, wc = (w % WN) * 32;

    // Staging: the next K tile is fetched into registers while the current
    // one is multiplied from LDS.  Direct operands: item = (row, 8 K values);
    // transposed operands: item = (8 rows, 2 consecutive K values), A's items
    // first, then B's, each written as 8 packed (K, K+1) pairs.
    constexpr int kDA = (BM * (kKT / 8) + 255) / 256, kDB = (BN * (kKT / 8) + 255) / 256;
    constexpr int kAT = (BM / 8) * (kKT / 2), kBT = (BN / 8) * (kKT / 2);
    constexpr int kTT = (kAT + kBT + 255) / 256;
    constexpr int kRegs = kWgrad ? 2 * kTT : kDA + kDB;
    uint4 reg[kRegs];
    auto fetch = [&](int k0) {
        const uint4 zero = {0u, 0u, 0u, 0u};
        if (!kWgrad) {
#pragma unroll
            for (int q = 0; q < kDA; ++q) {
                const int it = t + 256 * q;
                const int r = it >> 3, kc = (it & 7) << 3;
                reg[q] = it < BM * (kKT / 8) ? load_a_row<MODE>(g, m0 + r, k0 + kc) : zero;
            }
#pragma unroll
            for (int q = 0; q < kDB; ++q) {
                const int it = t + 256 * q;
                const int r = it >> 3, kc = (it & 7) << 3;
                uint4 bv = zero;
                if (it < BN * (kKT / 8) && n0 + r < g.N && k0 + kc < g.K)
                    bv = *reinterpret_cast<const uint4*>(g.wt + size_t(n0 + r) * g.K + k0 + kc);
                reg[kDA + q] = bv;
            }
        } else {
#pragma unroll
            for (int q = 0; q < kTT; ++q) {
                const int it = t + 256 * q;
                uint4 v0 = zero, v1 = zero;
                if (it < kAT + kBT) {
                    const bool isA = it < kAT;
                    const int x = isA ? it : it - kAT;
                    const int rows8 = isA ? BM / 8 : BN / 8;
                    const int rc = (x % rows8) << 3, kk = (x / rows8) << 1;
                    const int kpos = k0 + kk;
                    if (isA) {
                        if (kpos < k_hi) v0 = load_a_col<MODE>(g, m0 + rc, kpos);
                        if (kpos + 1 < k_hi) v1 = load_a_col<MODE>(g, m0 + rc, kpos + 1);
                    } else {
                        if (kpos < k_hi) v0 = load_b_col<MODE>(g, n0 + rc, kpos);
                        if (kpos + 1 < k_hi) v1 = load_b_col<MODE>(g, n0 + rc, kpos + 1);
                    }
                }
                reg[2 * q] = v0;
                reg[2 * q + 1] = v1;
            }
        }
    };
    auto stage = [&]() {
        if (!kWgrad) {
#pragma unroll
            for (int q = 0; q < kDA; ++q) {
                const int it = t + 256 * q;
                if (it < BM * (kKT / 8))
                    *reinterpret_cast<uint4*>(&As[it >> 3][(it & 7) << 3]) = reg[q];
            }
#pragma unroll
            for (int q = 0; q < kDB; ++q) {
                const int it = t + 256 * q;
                if (it < BN * (kKT / 8))
                    *reinterpret_cast<uint4*>(&Bs[it >> 3][(it & 7) << 3]) = reg[kDA + q];
            }
        } else {
#pragma unroll
            for (int q = 0; q < kTT; ++q) {
                const int it = t + 256 * q;
                if (it < kAT + kBT) {
                    const bool isA = it < kAT;
                    const int x = isA ? it : it - kAT;
                    const int rows8 = isA ? BM / 8 : BN / 8;
                    const int rc = (x % rows8) << 3, kk = (x / rows8) << 1;
                    const uint32_t* w0 = reinterpret_cast<const uint32_t*>(&reg[2 * q]);
                    const uint32_t* w1 = reinterpret_cast<const uint32_t*>(&reg[2 * q + 1]);
                    uint16_t (*dst)[kKT + kLdsPad] = isA ? As : Bs;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        // rows rc+2j (low halves) and rc+2j+1 (high halves): K pair (kk, kk+1)
                        const uint32_t lo = __builtin_amdgcn_perm(w1[j], w0[j], 0x05040100u);
                        const uint32_t hi = __builtin_amdgcn_perm(w1[j], w0[j], 0x07060302u);
                        *reinterpret_cast<uint32_t*>(&dst[rc + 2 * j][kk]) = lo;
                        *reinterpret_cast<uint32_t*>(&dst[rc + 2 * j + 1][kk]) = hi;
                    }
                }
            }
        }
    };

    if (k_lo < k_hi) fetch(k_lo);
    for (int k0 = k_lo; k0 < k_hi; k0 += kKT) {
        stage();
        __syncthreads();
        if (k0 + kKT < k_hi) fetch(k0 + kKT);   // in flight during the MFMAs below
        const int lr = lane & 15, kq = (lane >> 4) << 3;
#pragma unroll
        for (int ks = 0; ks < kKT; ks += kBK) {
#pragma unroll
            for (int i = 0; i < 2; ++i) {
                const uint4 araw = *reinterpret_cast<const uint4*>(&As[wr + 16 * i + lr][ks + kq]);
                const bf16x8 a = __builtin_bit_cast(bf16x8, araw);
#pragma unroll
                for (int j = 0; j < 2; ++j) {
                    const uint4 braw =
                        *reinterpret_cast<const uint4*>(&Bs[wc + 16 * j + lr][ks + kq]);
                    const bf16x8 b = __builtin_bit_cast(bf16x8, braw);
                    acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[i][j], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }

    // epilogue: lane holds rows 4*(lane/16)+e, column lane%16 of each 16x16 tile
    if constexpr (MODE == kTconvFwd && BM == 64 && BN == 64) {
        // Transposed convolution: the 64 x 64 tile (bias added, BF16) goes
        // through LDS (the A operand's buffer, free after the last barrier),
        // then each lane stores 8 consecutive channels of one child position
        // (16 bytes) instead of one 2-byte channel.  A tile's 64 columns are
        // whole 8-channel runs of one child (cout is a multiple of 8).
        uint16_t (*tile)[kKT + kLdsPad] = As;
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j)
#pragma unroll
                for (int e = 0; e < 4; ++e) {
                    const int ml = wr + 16 * i + 4 * (lane >> 4) + e;
                    const int nl = wc + 16 * j + (lane & 15);
                    const int o = (n0 + nl) & (g.cout - 1);
                    tile[ml][nl] = f2bf(acc[i][j][e] + g.bias[o]);
                }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int it = t + 256 * k;
            const int ml = it >> 3, nl = (it & 7) << 3;
            const int m = m0 + ml, n = n0 + nl;
            if (m >= g.M || n >= g.N) continue;
            const int abc = n >> g.cout_sh, o = n & (g.cout - 1);
            int z, y, x;
            pos3v(g.a, m, z, y, x);
            const int cz = 2 * z + (abc >> 2), cy = 2 * y + ((abc >> 1) & 1), cx = 2 * x + (abc & 1);
            const size_t child = (size_t(cz) * (2 * g.a.H) + cy) * (2 * g.a.W) + cx;
            *reinterpret_cast<uint4*>(g.b.p + child * g.b.stride + g.b.off + o) =
                *reinterpret_cast<const uint4*>(&tile[ml][nl]);
        }
        return;
    }
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j)
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int m = m0 + wr + 16 * i + 4 * (lane >> 4) + e;
                const int n = n0 + wc + 16 * j + (lane & 15);
                if (m >= g.M || n >= g.N) continue;
                float v = acc[i][j][e];
                if (MODE == kConvFwd) {
                    v += g.bias[n];
                    if (g.relu) v = fmaxf(v, 0.f);
                    g.b.p[size_t(m) * g.b.stride + g.b.off + n] = f2bf(v);
                } else if (MODE == kConvBwdData || MODE == kTconvBwdData) {
                    if (g.mask.p && !(bf2f(g.mask.p[size_t(m) * g.mask.stride + g.mask.off + n]) > 0.f))
                        v = 0.f;
                    g.b.p[size_t(m) * g.b.stride + g.b.off + n] = f2bf(v);
                } else if (MODE == kTconvFwd) {
                    const int abc = n >> g.cout_sh, o = n & (g.cout - 1);
                    int z, y, x;
                    pos3v(g.a, m, z, y, x);
                    const int cz = 2 * z + (abc >> 2), cy = 2 * y + ((abc >> 1) & 1),
                              cx = 2 * x + (abc & 1);
                    const size_t child = (size_t(cz) * (2 * g.a.H) + cy) * (2 * g.a.W) + cx;
                    g.b.p[child * g.b.stride + g.b.off + o] = f2bf(v + g.bias[o]);
                } else {
                    // weight gradients: this split's partial sum, reduced over
                    // the splits by k_wgrad_reduce (no atomics, fixed order)
                    g.partial[(size_t(blockIdx.z) * g.M + m) * g.N + n] = v;
                }
            }
}

// Bricks of the direct weight-gradient kernel: 4 x 8 x 8 positions.
constexpr int kDZ = 4, kDY = 8, kDX = 8;
constexpr int kHZ = kDZ + 2, kHY = kDY + 2, kHX = kDX + 2;
constexpr int kCC = 32;                    // input channels per staged chunk

typedef float floatx16 __attribute__((ext_vector_type(16)));

// Direct 3x3x3 convolution (forward, or input gradient as the forward
// convolution of the output gradient with the flipped packed weights) for
// bricks of 8 x 8 x 8 output positions and NT output channels.  The input
// brick with its one-voxel halo (10^3 positions) is staged in LDS one
// 32-channel chunk at a time and read by all 27 taps, instead of gathering
// every tap's operand from global memory.  v_mfma_f32_32x32x16_bf16: wave w
// computes brick layers w and w + 4 as four row tiles of 32 positions by
// NT / 32 column tiles, so that each weight operand (packed [N][27 C], read
// from the caches one tap ahead of its use) serves four MFMAs.  LDS bank
// conflicts, measured on gfx950: a 16-byte read serves 32 lanes at a time
// from 512 bytes of banks, a 16-byte write 8 lanes from 128 bytes.  With the
// 80-byte position pitch, the x-rows of a row tile lie 0, 8, 16 and 24
// (mod 32) positions apart, so the 32 lanes of a read hit distinct banks; a
// staging write covers 8 consecutive positions of one channel group.
constexpr int kFB = 8;                          // brick edge
constexpr int kFH = kFB + 2;                    // halo edge
constexpr int kFHalo = kFH * kFH * kFH;         // 1000 positions
constexpr int kFPitch = kCC + 8;                // BF16 per staged position

// (z, y, x) within the brick of row `row` of row tile i of wave w: the four
// x-rows (w, i), (w, i + 4), (w + 4, i), (w + 4, i + 4), 0, 40, 400 and 440
// halo positions apart
__device__ __forceinline__ void tile_pos(int w, int i, int row, int& z, int& y, int& x) {
    z = w + 4 * (row >> 4);
    y = i + 4 * ((row >> 3) & 1);
    x = row & 7;
}

// CC = 32: input channels in chunks of 32, two K steps of 16 per tap.
// CC = 8 (the network's 8-channel input): all channels in one chunk, one K
// step per two taps (lanes 0-31 tap 2s, lanes 32-63 tap 2s + 1), the
// operands of taps past the 27th zero.  blockIdx.z splits the input channels
// (CC = 32) over workgroups when the brick grid alone is too small for the
// chip: each split writes its FP32 partial sums and k_conv_split_reduce adds
// them in split order and applies the epilogue.
template <int MODE, int NT, int CC>
__global__ void __launch_bounds__(256, CC == 8 && NT == 32 ? 3 : 2) k_conv_direct(GemmArgs g) {
    static_assert(NT == 32 || NT == 64, "32 or 64 output channels per workgroup");
    static_assert(CC == 32 || CC == 8, "32 or 8 channels per staged chunk");
    constexpr int NJ = NT / 32;
    constexpr int kPitch = CC == 32 ? kFPitch : 8;
    // the output tile [512 positions][NT + 8] reuses the halo's LDS
    constexpr int kTP = NT + 8;
    constexpr int kLds = kFHalo * kPitch > 512 * kTP ? kFHalo * kPitch : 512 * kTP;
    __shared__ uint16_t halo[kLds];
    const View& v = g.a;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int bx_n = v.W / kFB, by_n = v.H / kFB;
    const int b = blockIdx.x;
    const int bx = b % bx_n, by = (b / bx_n) % by_n, bz = b / (bx_n * by_n);
    const int n0 = blockIdx.y * NT;
    const int C = v.C;
    const int c_per = C / int(gridDim.z);
    const int c_lo = int(blockIdx.z) * c_per, c_hi = c_lo + c_per;
    // independent accumulation chains: a 32x32x16 MFMA's result is not
    // ready for a dependent MFMA until several others have issued, so with
    // one column tile the even and odd K steps accumulate separately (eight
    // chains per wave either way), summed in the epilogue.  The 8-channel
    // input layer keeps four chains per wave instead: its 150 registers let
    // three workgroups share a CU (launch bounds above), whose staging and
    // stores then overlap more MFMA work than two could
    constexpr int KS = NJ == 1 && CC == 32 ? 2 : 1;
    floatx16 acc[4][NJ * KS];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < NJ * KS; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.f;
    const int r = lane & 31, kc = CC == 32 ? (lane >> 5) << 3 : 0;
    int qrow[4];   // halo position of this lane's row of tile i, centre tap
#pragma unroll
    for (int i = 0; i < 4; ++i) {
        int z, y, x;
        tile_pos(w, i, r, z, y, x);
        qrow[i] = ((z + 1) * kFH + y + 1) * kFH + x + 1;
    }
    // weights in operand order (k_frag): one contiguous 1 KB per wave and K
    // step, 512 values per step of a 32-row tile
    const int steps_all = CC == 32 ? (C / 32) * 54 : 15;
    const uint16_t* wrow[NJ];
#pragma unroll
    for (int j = 0; j < NJ; ++j)
        wrow[j] = g.wfrag + (size_t(n0 / 32 + j) * steps_all) * 512 + lane * 8;

    for (int c0 = c_lo; c0 < c_hi; c0 += CC) {
        // stage the halo brick of channels [c0, c0 + 32): item = (position, 8
        // channels), 8 consecutive positions per channel group.  A batch of
        // loads is issued before its first LDS write (addresses clamped into
        // the grid, outside values zeroed as they are written, so that no
        // branch separates the loads), which costs one memory latency per
        // batch instead of one per item.  The empty asm keeps the compiler
        // from holding every item's address across the chunk loop (registers
        // the accumulators need).
        constexpr int kItems = kFHalo * (CC / 8), kPer = (kItems + 255) / 256;
        // two batches where the registers allow (32 output channels), four
        // with 64 (its accumulators take the rest)
        constexpr int kBatch = CC == 32 ? (NT == 32 ? kPer / 2 : kPer / 4) : kPer;
#pragma unroll
        for (int k0 = 0; k0 < kPer; k0 += kBatch) {
            uint4 stg[kBatch];
            uint32_t outside = 0u;
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                int it = min(t + 256 * (k0 + k), kItems - 1);
                asm volatile("" : "+v"(it));
                const int q = CC == 32 ? ((it >> 5) << 3) + (it & 7) : it;
                const int cg = CC == 32 ? ((it >> 3) & 3) << 3 : 0;
                const int hz = q / (kFH * kFH), hy = (q / kFH) % kFH, hx = q % kFH;
                const int z = bz * kFB - 1 + hz, y = by * kFB - 1 + hy, x = bx * kFB - 1 + hx;
                const int zc = min(max(z, 0), v.D - 1), yc = min(max(y, 0), v.H - 1),
                          xc = min(max(x, 0), v.W - 1);
                stg[k] = load8(v, (zc * v.H + yc) * v.W + xc, c0 + cg);
                outside |= uint32_t(z != zc || y != yc || x != xc) << k;
            }
#pragma unroll
            for (int k = 0; k < kBatch; ++k) {
                const int it = t + 256 * (k0 + k);
                const int q = CC == 32 ? ((it >> 5) << 3) + (it & 7) : it;
                const int cg = CC == 32 ? ((it >> 3) & 3) << 3 : 0;
                const uint4 val = (outside >> k) & 1u ? uint4{0u, 0u, 0u, 0u} : stg[k];
                if (it < kItems) *reinterpret_cast<uint4*>(&halo[q * kPitch + cg]) = val;
            }
        }
        __syncthreads();
        // 54 K steps of 16 channels: step st is tap st / 2, channels
        // c0 + 16 (st % 2) .. + 15.  Software pipelined: the A operands of
        // step st + 1 are read from LDS while the MFMAs of step st run, and
        // the weights (from the L2: a layer's packed weights exceed the L1)
        // are loaded three steps ahead into a ring.  Past the last step the
        // addresses are clamped to it (loaded, never used), so that no
        // branch breaks the pipeline.
        // tap of step st for this lane, and the channel offset within it
        auto tap_of = [&](int st) {
            return CC == 32 ? st >> 1 : min(2 * st + (lane >> 5), 26);
        };
        auto a_ptr = [&](int st, int i) {
            const int tap = tap_of(st);
            const int dq = ((tap / 9 - 1) * kFH + (tap / 3) % 3 - 1) * kFH + tap % 3 - 1;
            const int co = CC == 32 ? 16 * (st & 1) + kc : 0;
            return reinterpret_cast<const uint4*>(&halo[(qrow[i] + dq) * kPitch + co]);
        };
        auto w_ptr = [&](int st, int j) {
            const int gs = CC == 32 ? (c0 / 32) * 54 + st : st;
            return reinterpret_cast<const uint4*>(wrow[j] + size_t(gs) * 512);
        };
        // the A operand of a step, zero for taps past the 27th (CC = 8)
        auto a_load = [&](int st, int i) {
            uint4 a = *a_ptr(st, i);
            if (CC == 8 && 2 * st + (lane >> 5) > 26) a = uint4{0u, 0u, 0u, 0u};
            return a;
        };
        // CC = 8: 14 steps padded to 15 (taps 27-29 zero) for an unroll of 3
        constexpr int kSteps = CC == 32 ? 54 : 15;
        constexpr int kUnroll = CC == 32 ? 6 : 3;
        uint4 ring[3][NJ], acur[4];
#pragma unroll
        for (int p = 0; p < 3; ++p)
#pragma unroll
            for (int j = 0; j < NJ; ++j) ring[p][j] = *w_ptr(p, j);
#pragma unroll
        for (int i = 0; i < 4; ++i) acur[i] = a_load(0, i);
#pragma unroll 1
        for (int s0 = 0; s0 < kSteps; s0 += kUnroll) {
#pragma unroll
            for (int u = 0; u < kUnroll; ++u) {
                const int st = s0 + u;
                uint4 anext[4];
#pragma unroll
                for (int i = 0; i < 4; ++i) anext[i] = a_load(min(st + 1, kSteps - 1), i);
                // keep the scheduler from sinking these reads to their use
                __builtin_amdgcn_sched_barrier(0);
#pragma unroll
                for (int i = 0; i < 4; ++i)
#pragma unroll
                    for (int j = 0; j < NJ; ++j) {
                        const int c = j * KS + (KS == 2 ? (u & 1) : 0);
                        acc[i][c] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(
                            __builtin_bit_cast(bf16x8, acur[i]), __builtin_bit_cast(bf16x8, ring[u % 3][j]),
                            acc[i][c], 0, 0, 0);
                    }
#pragma unroll
                for (int j = 0; j < NJ; ++j) ring[u % 3][j] = *w_ptr(min(st + 3, kSteps - 1), j);
#pragma unroll
                for (int i = 0; i < 4; ++i) acur[i] = anext[i];
            }
        }
        __syncthreads();
    }
    // epilogue: lane holds column lane % 32 and rows 8 (e / 4) + 4 (lane / 32) + e % 4
    if (gridDim.z > 1) {
        // a channel split: its FP32 partial sums
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                int z, y, x;
                tile_pos(w, i, 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3), z, y, x);
                const int m = ((bz * kFB + z) * v.H + by * kFB + y) * v.W + bx * kFB + x;
#pragma unroll
                for (int j = 0; j < NJ; ++j) {
                    float val = acc[i][j * KS][e];
                    if (KS == 2) val += acc[i][j * KS + 1][e];
                    g.partial[(size_t(blockIdx.z) * g.M + m) * g.N + n0 + 32 * j + (lane & 31)] = val;
                }
            }
        return;
    }
    // The output tile goes through LDS, so that each lane stores 16 bytes of
    // consecutive channels of one position (channels-last) instead of one
    // 2-byte channel: bias and ReLU (forward) before the BF16 rounding, as
    // in a direct store; the input gradient's mask (0 or 1) after it.  The
    // loop over chunks ended with a barrier, so the halo is free.
    uint16_t* tile = halo;
#pragma unroll
    for (int j = 0; j < NJ; ++j) {
        const int nl = 32 * j + (lane & 31);
        const float bias = MODE == kConvFwd ? g.bias[n0 + nl] : 0.f;
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
            for (int e = 0; e < 16; ++e) {
                int z, y, x;
                tile_pos(w, i, 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3), z, y, x);
                float val = acc[i][j * KS][e];
                if (KS == 2) val += acc[i][j * KS + 1][e];
                if (MODE == kConvFwd) {
                    val += bias;
                    if (g.relu) val = fmaxf(val, 0.f);
                }
                tile[((z * kFB + y) * kFB + x) * kTP + nl] = f2bf(val);
            }
    }
    __syncthreads();
    if (MODE == kConvFwd && g.head_out) {
        // the head from the tile: channels in ascending order, as k_head_fwd
        for (int p = t; p < 512; p += 256) {
            const int z = p >> 6, y = (p >> 3) & 7, x = p & 7;
            const int m = ((bz * kFB + z) * v.H + by * kFB + y) * v.W + bx * kFB + x;
            float sum = g.head_b[0] + g.head_dose[m];
#pragma unroll
            for (int c8 = 0; c8 < NT; c8 += 8) {
                const uint4 hv = *reinterpret_cast<const uint4*>(&tile[p * kTP + c8]);
                const uint16_t* he = reinterpret_cast<const uint16_t*>(&hv);
#pragma unroll
                for (int k = 0; k < 8; ++k) sum += g.head_w[c8 + k] * bf2f(he[k]);
            }
            g.head_out[m] = sum;
        }
        if (g.skip_store) return;
    }
    constexpr int kChunks = NT / 8;                 // 16-byte chunks per position
    constexpr int kOut = 512 * kChunks / 256;       // per thread
    const int ch = (t % kChunks) * 8;
#pragma unroll 4
    for (int k = 0; k < kOut; ++k) {
        const int p = (t + 256 * k) / kChunks;
        const int z = p >> 6, y = (p >> 3) & 7, x = p & 7;
        const int m = ((bz * kFB + z) * v.H + by * kFB + y) * v.W + bx * kFB + x;
        uint4 o = *reinterpret_cast<const uint4*>(&tile[p * kTP + ch]);
        if (MODE != kConvFwd && g.mask.p) {
            const uint4 mk = load8(g.mask, m, n0 + ch);
            const uint16_t* me = reinterpret_cast<const uint16_t*>(&mk);
            uint16_t* oe = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (!(bf2f(me[q]) > 0.f)) oe[q] = 0;
        }
        *reinterpret_cast<uint4*>(g.b.p + size_t(m) * g.b.stride + g.b.off + n0 + ch) = o;
    }
    if (MODE == kConvFwd && g.pool.p) {
        // 2x2x2 max pooling of the brick (4^3 coarse positions) from the same
        // tile: the first maximum in child order (z, y, x bits) wins, as in
        // k_pool_fwd
        for (int it = t; it < 64 * kChunks; it += 256) {
            const int cp = it / kChunks, c8 = (it % kChunks) * 8;
            const int cz = cp >> 4, cy = (cp >> 2) & 3, cx = cp & 3;
            float best[8];
            uint8_t bi[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                best[k] = -INFINITY;
                bi[k] = 0;
            }
#pragma unroll
            for (int a = 0; a < 8; ++a) {
                const int fz = 2 * cz + (a >> 2), fy = 2 * cy + ((a >> 1) & 1), fx = 2 * cx + (a & 1);
                const uint4 fv = *reinterpret_cast<const uint4*>(&tile[((fz * kFB + fy) * kFB + fx) * kTP + c8]);
                const uint16_t* fe = reinterpret_cast<const uint16_t*>(&fv);
#pragma unroll
                for (int k = 0; k < 8; ++k) {
                    const float f = bf2f(fe[k]);
                    if (f > best[k]) {
                        best[k] = f;
                        bi[k] = uint8_t(a);
                    }
                }
            }
            uint4 po;
            uint2 ab;
            uint16_t* pe = reinterpret_cast<uint16_t*>(&po);
            uint8_t* ae = reinterpret_cast<uint8_t*>(&ab);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                pe[k] = f2bf(best[k]);
                ae[k] = bi[k];
            }
            const int q = ((bz * 4 + cz) * (v.H >> 1) + by * 4 + cy) * (v.W >> 1) + bx * 4 + cx;
            *reinterpret_cast<uint4*>(g.pool.p + size_t(q) * g.pool.stride + g.pool.off + n0 + c8) = po;
            *reinterpret_cast<uint2*>(g.arg + size_t(q) * g.b.C + n0 + c8) = ab;
        }
    }
}

// Sum of the channel splits of k_conv_direct (in split order) and its
// epilogue: bias and ReLU (forward) or the ReLU mask (input gradient), BF16
// out.  8 output channels per thread: 16-byte stores.
template <int MODE>
__global__ void k_conv_split_reduce(GemmArgs g, int splits) {
    const int n8 = g.N >> 3;
    const int64_t total = int64_t(g.M) * n8;
    const size_t plane = size_t(g.M) * g.N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int m = int(i / n8), n = int(i - int64_t(m) * n8) << 3;
        const float* src = g.partial + size_t(m) * g.N + n;
        float4 a = *reinterpret_cast<const float4*>(src);
        float4 b = *reinterpret_cast<const float4*>(src + 4);
        for (int z = 1; z < splits; ++z) {
            const float4 pa = *reinterpret_cast<const float4*>(src + z * plane);
            const float4 pb = *reinterpret_cast<const float4*>(src + z * plane + 4);
            a.x += pa.x; a.y += pa.y; a.z += pa.z; a.w += pa.w;
            b.x += pb.x; b.y += pb.y; b.z += pb.z; b.w += pb.w;
        }
        float val[8] = {a.x, a.y, a.z, a.w, b.x, b.y, b.z, b.w};
        uint4 mk{0u, 0u, 0u, 0u};
        if (MODE != kConvFwd && g.mask.p) mk = load8(g.mask, m, n);
        const uint16_t* me = reinterpret_cast<const uint16_t*>(&mk);
        uint4 o;
        uint16_t* oe = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float x = val[k];
            if (MODE == kConvFwd) {
                x += g.bias[n + k];
                if (g.relu) x = fmaxf(x, 0.f);
            } else if (g.mask.p && !(bf2f(me[k]) > 0.f)) {
                x = 0.f;
            }
            oe[k] = f2bf(x);
        }
        *reinterpret_cast<uint4*>(g.b.p + size_t(m) * g.b.stride + g.b.off + n) = o;
    }
}

// Weight gradient of a 3x3x3 convolution by the same bricks:
// gW[o][tap][c] = sum over positions p of gz[p][o] * x[p + tap][c], with the
// positions as the GEMM's K.  A workgroup takes 32 output channels, 32 input
// channels and all 27 taps (a 32 x 864 tile of the [M][27 C] gradient) over a
// run of bricks, and writes its partial sum for k_wgrad_reduce.  Each input
// value is staged once per brick (with the halo, 600 / 256 times) instead of
// being gathered once per tap.  Both MFMA operands need 8 consecutive
// positions per lane, so the channels-last data is transposed while staged:
// the brick's gz as [x-row][o] -> 8 x values, the input with its halo as three
// copies [halo row][c] -> 8 x values shifted by dx = -1, 0, +1, so that every
// LDS read stays 16-byte aligned.  v_mfma_f32_32x32x16_bf16: one K step is two
// x-rows of 8 (lanes 0-31 the first, 32-63 the second); wave w owns taps
// 7w .. 7w + 6 (wave 3 six of them) and reuses its gz operand for each.
constexpr int kWRows = kDZ * kDY;          // x-rows of 8 positions per brick
constexpr int kHRows = kHZ * kHY;          // x-rows of 10 in the halo brick

// Column of element (row, col) in a [row][32] array of 16-byte entries: bits
// 0-2 of col are XORed with col's channel group (bits 3-4) and the row's
// parity, so that the 8 lanes of one staging write phase (2 rows x 4 channel
// groups) fall on 8 distinct entries modulo 8; a row keeps all its 32
// entries, so the MFMA operand reads (32 lanes on one 512-byte row) stay
// conflict-free.
__device__ __forceinline__ int swz(int row, int col) { return col ^ (((col >> 3) & 3) | ((row & 1) << 2)); }

// Channel j of 8 consecutive positions v[0..7] (8 channels each), packed.
__device__ __forceinline__ uint4 transpose_channel(const uint4* v, int j) {
    const uint32_t sel = (j & 1) ? 0x07060302u : 0x05040100u;
    uint32_t out[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        const uint32_t* lo = reinterpret_cast<const uint32_t*>(&v[2 * k]);
        const uint32_t* hi = reinterpret_cast<const uint32_t*>(&v[2 * k + 1]);
        out[k] = __builtin_amdgcn_perm(hi[j >> 1], lo[j >> 1], sel);
    }
    return uint4{out[0], out[1], out[2], out[3]};
}

__global__ void __launch_bounds__(256) k_conv_wgrad_direct(GemmArgs g, int bricks_per_split) {
    __shared__ uint4 gzT[kWRows][32];        // 16 KB
    __shared__ uint4 xT[3][kHRows][32];      // 90 KB
    const View& v = g.a;
    const View& gz = g.b;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    const int bx_n = v.W / kDX, by_n = v.H / kDY;
    const int nbricks = bx_n * by_n * (v.D / kDZ);
    const int o0 = blockIdx.y * 32, c0 = blockIdx.z * 32;
    const int b_lo = blockIdx.x * bricks_per_split;
    const int b_hi = min(nbricks, b_lo + bricks_per_split);
    const int tap0 = 7 * w, ntap = w == 3 ? 6 : 7;
    const uint4 zero = {0u, 0u, 0u, 0u};
    floatx16 acc[7];
#pragma unroll
    for (int i = 0; i < 7; ++i)
#pragma unroll
        for (int e = 0; e < 16; ++e) acc[i][e] = 0.f;

    // Staging items of this thread: item A = t (a halo row of the input if
    // t < 240, else an x-row of the output gradient), item B = t + 256 (an
    // x-row of the output gradient if t < 112).  The next brick's items are
    // loaded into registers while the current brick's MFMAs run; addresses
    // are clamped into the grid and outside values zeroed when written.
    constexpr int kXItems = kHRows * 4, kGItems = kWRows * 4;
    const bool a_is_x = t < kXItems;
    const int kA = t - kXItems, kB = t + 256 - kXItems;
    const bool has_b = kB < kGItems;
    uint4 ra[kHX], rb[kDX];
    uint32_t outside = 0u;
    auto fetch = [&](int b) {
        const int bx = b % bx_n, by = (b / bx_n) % by_n, bz = b / (bx_n * by_n);
        outside = 0u;
        if (a_is_x) {
            const int hr = t >> 2, cg = (t & 3) << 3;
            const int z = bz * kDZ - 1 + hr / kHY, y = by * kDY - 1 + hr % kHY;
            const int zc = min(max(z, 0), v.D - 1), yc = min(max(y, 0), v.H - 1);
            const bool row_out = z != zc || y != yc;
#pragma unroll
            for (int hx = 0; hx < kHX; ++hx) {
                const int x = bx * kDX - 1 + hx;
                const int xc = min(max(x, 0), v.W - 1);
                ra[hx] = load8(v, (zc * v.H + yc) * v.W + xc, c0 + cg);
                outside |= uint32_t(row_out || x != xc) << hx;
            }
        } else {
            const int r = kA >> 2, og = (kA & 3) << 3;
            const int z = bz * kDZ + r / kDY, y = by * kDY + r % kDY;
#pragma unroll
            for (int i = 0; i < kDX; ++i) ra[i] = load8(gz, (z * gz.H + y) * gz.W + bx * kDX + i, o0 + og);
        }
        if (has_b) {
            const int r = kB >> 2, og = (kB & 3) << 3;
            const int z = bz * kDZ + r / kDY, y = by * kDY + r % kDY;
#pragma unroll
            for (int i = 0; i < kDX; ++i) rb[i] = load8(gz, (z * gz.H + y) * gz.W + bx * kDX + i, o0 + og);
        }
    };
    auto stage = [&]() {
        if (a_is_x) {
            const int hr = t >> 2, cg = (t & 3) << 3;
#pragma unroll
            for (int hx = 0; hx < kHX; ++hx)
                if ((outside >> hx) & 1u) ra[hx] = zero;
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int j = 0; j < 8; ++j) xT[d][hr][swz(hr, cg + j)] = transpose_channel(ra + d, j);
        } else {
            const int r = kA >> 2, og = (kA & 3) << 3;
#pragma unroll
            for (int j = 0; j < 8; ++j) gzT[r][swz(r, og + j)] = transpose_channel(ra, j);
        }
        if (has_b) {
            const int r = kB >> 2, og = (kB & 3) << 3;
#pragma unroll
            for (int j = 0; j < 8; ++j) gzT[r][swz(r, og + j)] = transpose_channel(rb, j);
        }
    };

    if (b_lo < b_hi) fetch(b_lo);
    for (int b = b_lo; b < b_hi; ++b) {
        stage();
        __syncthreads();
        if (b + 1 < b_hi) fetch(b + 1);
        const int col = lane & 31;
#pragma unroll 2
        for (int ks = 0; ks < kWRows / 2; ++ks) {
            // K step ks: brick x-rows 2 ks (lanes 0-31) and 2 ks + 1 (lanes 32-63)
            const int row = 2 * ks + (lane >> 5);
            const int rz = row / kDY, ry = row % kDY;
            const bf16x8 a = __builtin_bit_cast(bf16x8, gzT[row][swz(row, col)]);
#pragma unroll
            for (int tt = 0; tt < 7; ++tt) {
                if (tt < ntap) {
                    const int tap = tap0 + tt;
                    const int hr = (rz + tap / 9) * kHY + ry + (tap / 3) % 3;
                    const bf16x8 bop = __builtin_bit_cast(bf16x8, xT[tap % 3][hr][swz(hr, col)]);
                    acc[tt] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, bop, acc[tt], 0, 0, 0);
                }
            }
        }
        __syncthreads();
    }
    // lane holds column lane % 32 and rows 8 (e / 4) + 4 (lane / 32) + e % 4
    float* out = g.partial + size_t(blockIdx.x) * g.M * g.N;
#pragma unroll
    for (int tt = 0; tt < 7; ++tt) {
        if (tt >= ntap) continue;
        const int n = (tap0 + tt) * v.C + c0 + (lane & 31);
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int m = o0 + 8 * (e >> 2) + 4 * (lane >> 5) + (e & 3);
            out[size_t(m) * g.N + n] = acc[tt][e];
        }
    }
}

// Sum of the split-K partials of a weight gradient, written in the reference
// layout: conv (MODE kConvWgrad) row m = output channel, column n = tap *
// C_in_padded + c; transposed conv: row m = input channel, column n =
// child * cout + o.
template <int MODE>
__global__ void k_wgrad_reduce(const float* partial, int splits, int M, int N, int c_pad, int cin,
                               int cout, float* wgrad) {
    const int64_t total = int64_t(M) * N;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        // eight independent partial sums keep eight loads in flight
        float v8[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
        int z = 0;
        for (; z + 8 <= splits; z += 8)
#pragma unroll
            for (int k = 0; k < 8; ++k) v8[k] += partial[size_t(z + k) * total + i];
        for (; z < splits; ++z) v8[0] += partial[size_t(z) * total + i];
        const float v = ((v8[0] + v8[1]) + (v8[2] + v8[3])) + ((v8[4] + v8[5]) + (v8[6] + v8[7]));
        const int m = int(i / N), n = int(i - int64_t(m) * N);
        if (MODE == kConvWgrad) {
            const int tap = n / c_pad, c = n - tap * c_pad;
            if (c < cin) wgrad[(size_t(m) * cin + c) * 27 + tap] = v;
        } else {
            const int abc = n / cout, o = n - abc * cout;
            wgrad[(size_t(m) * cout + o) * 8 + abc] = v;
        }
    }
}

// ---- element-wise / reduction kernels ---------------------------------------
// input [2][P] FP32 (scaled dose, density) -> x0 [P][8] BF16 (channels 2..7 zero)
__global__ void k_pack_input(const float* in, int P, uint16_t* x0) {
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        uint16_t v[8] = {f2bf(in[p]), f2bf(in[P + p]), 0, 0, 0, 0, 0, 0};
        *reinterpret_cast<uint4*>(x0 + size_t(p) * 8) = *reinterpret_cast<uint4*>(v);
    }
}

// 2x2x2 max pooling of view `in` (fine) into `out` (coarse); argmax = first
// maximum in (z, y, x) order of the block
__global__ void k_pool_fwd(View in, View out, uint8_t* arg) {
    // 8 channels per thread (C is a multiple of 8): 16-byte loads and stores
    const int C8 = in.C >> 3;
    const int total = out.D * out.H * out.W * C8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = (i % C8) << 3, q = i / C8;
        int z, y, x;
        pos3(q, out.D, out.H, out.W, z, y, x);
        float best[8];
        uint8_t bi[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            best[k] = -INFINITY;
            bi[k] = 0;
        }
#pragma unroll
        for (int a = 0; a < 8; ++a) {
            const int fz = 2 * z + (a >> 2), fy = 2 * y + ((a >> 1) & 1), fx = 2 * x + (a & 1);
            const uint4 v = load8(in, (fz * in.H + fy) * in.W + fx, c);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                const float f = bf2f(e[k]);
                if (f > best[k]) {
                    best[k] = f;
                    bi[k] = uint8_t(a);
                }
            }
        }
        uint4 o;
        uint2 ab;
        uint16_t* oe = reinterpret_cast<uint16_t*>(&o);
        uint8_t* ae = reinterpret_cast<uint8_t*>(&ab);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            oe[k] = f2bf(best[k]);
            ae[k] = bi[k];
        }
        *reinterpret_cast<uint4*>(out.p + size_t(q) * out.stride + out.off + c) = o;
        *reinterpret_cast<uint2*>(arg + size_t(q) * in.C + c) = ab;
    }
}

// gradient of the fine level: routed pool gradient + skip gradient, masked by
// the ReLU output `h` of that level; 8 channels per thread
__global__ void k_pool_bwd(View gcoarse, const uint8_t* arg, View gskip, View h, View gfine) {
    const int C = gfine.C, C8 = C >> 3;
    const int total = gfine.D * gfine.H * gfine.W * C8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int c = (i % C8) << 3, p = i / C8;
        int z, y, x;
        pos3(p, gfine.D, gfine.H, gfine.W, z, y, x);
        const int q = ((z >> 1) * gcoarse.H + (y >> 1)) * gcoarse.W + (x >> 1);
        const int a = ((z & 1) << 2) | ((y & 1) << 1) | (x & 1);
        const uint4 vs = load8(gskip, p, c), vh = load8(h, p, c), vc = load8(gcoarse, q, c);
        const uint2 av = *reinterpret_cast<const uint2*>(arg + size_t(q) * C + c);
        const uint16_t* es = reinterpret_cast<const uint16_t*>(&vs);
        const uint16_t* eh = reinterpret_cast<const uint16_t*>(&vh);
        const uint16_t* ec = reinterpret_cast<const uint16_t*>(&vc);
        const uint8_t* ea = reinterpret_cast<const uint8_t*>(&av);
        uint4 o;
        uint16_t* oe = reinterpret_cast<uint16_t*>(&o);
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            float v = bf2f(es[k]);
            if (ea[k] == a) v += bf2f(ec[k]);
            if (!(bf2f(eh[k]) > 0.f)) v = 0.f;
            oe[k] = f2bf(v);
        }
        *reinterpret_cast<uint4*>(gfine.p + size_t(p) * gfine.stride + gfine.off + c) = o;
    }
}

// head: pred = sum_c w[c] h[p][c] + b + dose[p]
__global__ void k_head_fwd(View h, const float* hw, const float* hb, const float* dose, int P,
                           float* pred) {
    // C is a multiple of 8: one 16-byte load per 8 channels
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        float s = hb[0] + dose[p];
        for (int c8 = 0; c8 < h.C; c8 += 8) {
            const uint4 v = load8(h, p, c8);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int k = 0; k < 8; ++k) s += hw[c8 + k] * bf2f(e[k]);
        }
        pred[p] = s;
    }
}

// loss = mean (pred - t)^2 (partial sums per block into striped slots),
// gy = 2 (pred - t) / P
__global__ void k_loss(const float* pred, const float* tgt, int P, float* gy, double* loss_parts) {
    double s = 0.0;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const float d = pred[p] - tgt[p];
        gy[p] = 2.f * d / float(P);
        s += double(d) * d;
    }
    for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
    if ((threadIdx.x & 63) == 0) atomicAdd(loss_parts + (blockIdx.x & 63), s / double(P));
}

// Head backward: per-position gradient into the last decoder output (masked
// by its ReLU) and the head's weight / bias gradients.  Each thread takes
// whole positions (C <= 32 channels, 8 per 16-byte load) and keeps its weight
// gradient in registers; waves reduce with shuffles, blocks through LDS.
__global__ void __launch_bounds__(256) k_head_bwd(View h, const float* hw, const float* gy, int P,
                                                  float* ghw, float* ghb, View g) {
    __shared__ float s_w[33];
    const int C = h.C;
    if (threadIdx.x < 33) s_w[threadIdx.x] = 0.f;
    __syncthreads();
    float acc[32], accb = 0.f;
#pragma unroll
    for (int c = 0; c < 32; ++c) acc[c] = 0.f;
    for (int p = blockIdx.x * blockDim.x + threadIdx.x; p < P; p += gridDim.x * blockDim.x) {
        const float gp = gy[p];
        accb += gp;
#pragma unroll
        for (int c8 = 0; c8 < 32; c8 += 8) {
            if (c8 < C) {
                const uint4 hv = load8(h, p, c8);
                const uint16_t* he = reinterpret_cast<const uint16_t*>(&hv);
                uint16_t out[8];
#pragma unroll
                for (int j = 0; j < 8; ++j) {
                    const float x = bf2f(he[j]);
                    acc[c8 + j] = fmaf(gp, x, acc[c8 + j]);
                    out[j] = f2bf(x > 0.f ? hw[c8 + j] * gp : 0.f);
                }
                *reinterpret_cast<uint4*>(g.p + size_t(p) * g.stride + g.off + c8) =
                    *reinterpret_cast<const uint4*>(out);
            }
        }
    }
    // wave sums, then one LDS add per wave and channel
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        float v = acc[c];
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
        acc[c] = v;
    }
    for (int off = 32; off >= 1; off >>= 1) accb += __shfl_xor(accb, off, 64);
    if ((threadIdx.x & 63) == 0) {
        for (int c = 0; c < C; ++c) atomicAdd(&s_w[c], acc[c]);
        atomicAdd(&s_w[32], accb);
    }
    __syncthreads();
    if (threadIdx.x < C) atomicAdd(ghw + threadIdx.x, s_w[threadIdx.x]);
    if (threadIdx.x == 32) atomicAdd(ghb, s_w[32]);
}

// bias gradient: column sums of a gradient view over all positions.  A
// thread sums 8 channels (one 16-byte load) over a strided set of positions;
// the block adds its partial sums in LDS, then once per channel globally.
__global__ void __launch_bounds__(256) k_bias_grad(View g, int P, float* gb) {
    __shared__ float s[256];
    const int C = g.C;                 // multiple of 8, at most 256
    const int groups = C >> 3;         // channel groups of 8
    for (int c = threadIdx.x; c < C; c += blockDim.x) s[c] = 0.f;
    __syncthreads();
    const int per_block = blockDim.x / groups;     // positions in flight per block
    const int grp = threadIdx.x % groups, row = threadIdx.x / groups;
    float acc[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (row < per_block) {
        // four loads in flight per pass; the sums keep the order of p
        const int step = gridDim.x * per_block;
        int p = blockIdx.x * per_block + row;
        for (; p + 3 * step < P; p += 4 * step) {
            uint4 v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = load8(g, p + u * step, grp * 8);
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const uint16_t* e = reinterpret_cast<const uint16_t*>(&v[u]);
#pragma unroll
                for (int j = 0; j < 8; ++j) acc[j] += bf2f(e[j]);
            }
        }
        for (; p < P; p += step) {
            const uint4 v = load8(g, p, grp * 8);
            const uint16_t* e = reinterpret_cast<const uint16_t*>(&v);
#pragma unroll
            for (int j = 0; j < 8; ++j) acc[j] += bf2f(e[j]);
        }
#pragma unroll
        for (int j = 0; j < 8; ++j) atomicAdd(&s[grp * 8 + j], acc[j]);
    }
    __syncthreads();
    for (int c = threadIdx.x; c < C; c += blockDim.x) atomicAdd(gb + c, s[c]);
}

__global__ void k_zero_f(float* p, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x)
        p[i] = 0.f;
}

__global__ void k_zero_d(double* p, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) p[i] = 0.0;
}

// Adam (Kingma & Ba) on the FP32 master parameters
__global__ void k_adam(float* p, const float* g, float* m, float* v, int64_t n, float lr, float b1,
                       float b2, float eps, float c1, float c2) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n;
         i += int64_t(gridDim.x) * blockDim.x) {
        const float gi = g[i];
        const float mi = b1 * m[i] + (1.f - b1) * gi;
        const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
        m[i] = mi;
        v[i] = vi;
        p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
    }
}

// conv weights [o][c][27] -> forward B^T [o][tap*cin_pad + c] and backward
// B^T [c][tap'*cout + o] with tap' = 26 - tap (flipped kernel)
__global__ void k_pack_conv(const float* w, int cout, int cin, int cin_pad, uint16_t* wf,
                            uint16_t* wb) {
    const int total = cout * cin_pad * 27;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int tap = i % 27, c = (i / 27) % cin_pad, o = i / (27 * cin_pad);
        const float v = c < cin ? w[(size_t(o) * cin + c) * 27 + tap] : 0.f;
        wf[size_t(o) * (27 * cin_pad) + tap * cin_pad + c] = f2bf(v);
        if (wb && c < cin) wb[size_t(c) * (27 * cout) + (26 - tap) * cout + o] = f2bf(v);
    }
}

// Elements of a [N][27 C] weight matrix in the brick kernel's operand order
// (0 where that kernel does not take it).
int64_t frag_elems(int N, int C) {
    if (N % 32 != 0 || !(C == 8 || C % 32 == 0)) return 0;
    const int64_t steps = C == 8 ? 15 : int64_t(C / 32) * 54;
    return int64_t(N / 32) * steps * 512;
}

// [N][27 C] weights (tap-major K) in k_conv_direct's operand order: for each
// 32-row tile and K step, the 64 lanes' 8 consecutive K values contiguous
// (lane l: row l % 32, K half l / 32).  C = 32 c: step s of chunk q covers
// tap s / 2, channels 32 q + 16 (s % 2) ..; C = 8: step s covers taps 2 s
// (lanes 0-31) and 2 s + 1 (lanes 32-63), clamped to the 27th (its operand
// is zeroed in the kernel).
__global__ void k_frag(const uint16_t* src, int N, int C, uint16_t* dst) {
    const int K = 27 * C;
    const int steps = C == 8 ? 15 : (C / 32) * 54;
    const int64_t total = int64_t(N / 32) * steps * 64;
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < total;
         i += int64_t(gridDim.x) * blockDim.x) {
        const int lane = int(i & 63);
        const int64_t q = i >> 6;
        const int st = int(q % steps), nt = int(q / steps);
        const int n = nt * 32 + (lane & 31), h = lane >> 5;
        int k;
        if (C == 8) {
            k = min(2 * st + h, 26) * 8;
        } else {
            const int chunk = st / 54, s = st % 54;
            k = (s >> 1) * C + chunk * 32 + 16 * (s & 1) + 8 * h;
        }
        *reinterpret_cast<uint4*>(dst + i * 8) =
            *reinterpret_cast<const uint4*>(src + size_t(n) * K + k);
    }
}

// tconv weights [c][o][8] -> forward B^T [abc*cout + o][c], backward B^T [c][abc*cout + o]
__global__ void k_pack_tconv(const float* w, int cin, int cout, uint16_t* wf, uint16_t* wb) {
    const int total = cin * cout * 8;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < total; i += gridDim.x * blockDim.x) {
        const int abc = i % 8, o = (i / 8) % cout, c = i / (8 * cout);
        const uint16_t v = f2bf(w[i]);
        wf[size_t(abc * cout + o) * cin + c] = v;
        wb[size_t(c) * (8 * cout) + abc * cout + o] = v;
    }
}

int grid1(int64_t n, int cap = 4096) {
    return int(std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, cap)));
}

}  // namespace

// ---------------------------------------------------------------------------
// Network object
// ---------------------------------------------------------------------------
struct UNet {
    int c = 32, D = 0, H = 0, W = 0;
    int64_t n_params = 0;
    // parameter offsets in the flat FP32 arrays (reference order)
    // wf / wb: forward [cout][27 cin_pad] and input-gradient [cin][27 cout]
    // packs; wff / wbf: the same in the brick kernel's operand order (or null)
    struct Conv {
        int64_t w, b;
        int cin, cout, cin_pad;
        uint16_t *wf, *wb, *wff, *wbf;
    };
    struct Tconv { int64_t w, b; int cin, cout; uint16_t* wf; uint16_t* wb; };
    Conv enc_a[kLevels], enc_b[kLevels], dec_a[kLevels], dec_b[kLevels];
    Tconv up[kLevels];
    int64_t head_w = 0, head_b = 0;
    DevBuf params, grads, adam_m, adam_v, packed;
    DevBuf wpart;          // split-K partial sums of the weight gradients
    // activations (BF16 channels-last) and gradients per level
    DevBuf x0, cat[kLevels], enc_a_out[kLevels], dec_a_out[kLevels], dec_b_out[kLevels],
        bottom_b, pooled[kLevels], arg[kLevels], g1[kLevels], g2[kLevels], gcat[kLevels], pred,
        gy, loss;
    int64_t step = 0;
    int dims[kLevels][3];
    int64_t P(int k) const { return int64_t(dims[k][0]) * dims[k][1] * dims[k][2]; }
    int ch(int k) const { return c << k; }
};

namespace {

// Multiply-shift constants for unsigned division by d >= 1 of n < 2^31.
void magic_div(uint32_t d, uint32_t& mul, uint32_t& sh) {
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    mul = uint32_t(((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1);
    sh = l;
}

View view(const DevBuf& b, const UNet& u, int level, int C, int stride, int off) {
    View v{b.as<uint16_t>(), u.dims[level][0], u.dims[level][1], u.dims[level][2], C, stride, off,
           0, 0, 0, 0, 0, 0, 0, 0, 0};
    PSL_CHECK(C > 0 && (C & (C - 1)) == 0, "channel counts must be powers of two");
    magic_div(uint32_t(v.W), v.wm, v.ws);
    magic_div(uint32_t(v.H), v.hm, v.hs);
    magic_div(uint32_t(std::max(1, v.W >> 1)), v.w2m, v.w2s);
    magic_div(uint32_t(std::max(1, v.H >> 1)), v.h2m, v.h2s);
    while ((1 << v.cs) < C) ++v.cs;
    return v;
}

// Tile of a GEMM: 128 x 32 for a direct GEMM with N <= 32, 32 x 128 for a
// weight gradient with M <= 32, else 64 x 64.
struct Tile { int bm, bn; };
Tile tile_for(int mode, int M, int N) {
    const bool wg = mode == kConvWgrad || mode == kTconvWgrad;
    if (!wg && N <= 32) return {128, 32};
    if (wg && M <= 32) return {32, 128};
    return {64, 64};
}

template <int MODE>
void launch_mode(const GemmArgs& g, dim3 grid, Tile tl, hipStream_t s) {
    if (tl.bm == 128) hipLaunchKernelGGL((k_gemm<MODE, 128, 32>), grid, dim3(256), 0, s, g);
    else if (tl.bm == 32) hipLaunchKernelGGL((k_gemm<MODE, 32, 128>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_gemm<MODE, 64, 64>), grid, dim3(256), 0, s, g);
}

void gemm_launch(int mode, const GemmArgs& g0, hipStream_t s, int splits = 1) {
    GemmArgs g = g0;
    if (mode == kTconvFwd || mode == kTconvBwdData || mode == kTconvWgrad) {
        PSL_CHECK(g.cout > 0 && (g.cout & (g.cout - 1)) == 0, "channel counts must be powers of two");
        g.cout_sh = 0;
        while ((1 << g.cout_sh) < g.cout) ++g.cout_sh;
    }
    const Tile tl = tile_for(mode, g.M, g.N);
    dim3 grid((g.M + tl.bm - 1) / tl.bm, (g.N + tl.bn - 1) / tl.bn, splits);
    switch (mode) {
        case kConvFwd: launch_mode<kConvFwd>(g, grid, tl, s); break;
        case kConvBwdData: launch_mode<kConvBwdData>(g, grid, tl, s); break;
        case kConvWgrad: launch_mode<kConvWgrad>(g, grid, tl, s); break;
        case kTconvFwd: launch_mode<kTconvFwd>(g, grid, tl, s); break;
        case kTconvBwdData: launch_mode<kTconvBwdData>(g, grid, tl, s); break;
        default: launch_mode<kTconvWgrad>(g, grid, tl, s); break;
    }
    PSL_HIP(hipGetLastError());
}

// Launch shape of the direct brick convolution of an input of C channels on
// a D x H x W grid into N output channels: output channels per workgroup
// (nt) and channel splits, so that the grid has about 512 workgroups (two
// per CU) where the bricks alone give fewer.  splits = 0: not direct.
struct ConvShape { int nt, splits; };
ConvShape conv_shape(int D, int H, int W, int C, int N) {
    if (D % kFB || H % kFB || W % kFB || N % 32 || !(C % kCC == 0 || C == 8)) return {0, 0};
    const int64_t bricks = int64_t(D / kFB) * (H / kFB) * (W / kFB);
    int nt = N % 64 == 0 ? 64 : 32;
    int splits = 1;
    if (C % kCC == 0) {
        const int chunks = C / kCC;
        if (nt == 64 && bricks * (N / 64) * chunks < 512) nt = 32;
        while (bricks * (N / nt) * splits < 512 && chunks % (2 * splits) == 0) splits *= 2;
    }
    return {nt, splits};
}

template <int MODE, int CC>
void launch_direct(dim3 grid, int nt, const GemmArgs& g, hipStream_t s) {
    if (nt == 64) hipLaunchKernelGGL((k_conv_direct<MODE, 64, CC>), grid, dim3(256), 0, s, g);
    else hipLaunchKernelGGL((k_conv_direct<MODE, 32, CC>), grid, dim3(256), 0, s, g);
}

// Convolution GEMM (forward or input gradient): the direct brick kernel
// where the grid and the channels fit its bricks, else the implicit GEMM.
// Channel splits use `scratch` (floats) for their partial sums.
// With g.pool.p set (forward only), the brick kernel also writes the 2x2x2
// max pooling of its output when it runs unsplit; the return value says
// whether it did (else the caller pools).
bool conv_launch(int mode, GemmArgs g, hipStream_t s, float* scratch, size_t scratch_floats) {
    const View& v = g.a;
    const ConvShape sh = conv_shape(v.D, v.H, v.W, v.C, g.N);
    if (sh.splits == 0 || g.K != 27 * v.C || int64_t(v.D) * v.H * v.W != g.M) {
        gemm_launch(mode, g, s);
        return false;
    }
    const bool pooled = mode == kConvFwd && g.pool.p && sh.splits == 1;
    if (!pooled) g.pool.p = nullptr;
    // the head needs every output channel of a position in one workgroup
    const bool headed = mode == kConvFwd && g.head_out && sh.splits == 1 && sh.nt == g.N;
    if (!headed) {
        g.head_out = nullptr;
        g.skip_store = 0;
    }
    PSL_CHECK(g.wfrag, "brick convolution without operand-ordered weights");
    dim3 grid((v.D / kFB) * (v.H / kFB) * (v.W / kFB), g.N / sh.nt, sh.splits);
    if (sh.splits > 1) {
        PSL_CHECK(scratch && scratch_floats >= size_t(sh.splits) * g.M * g.N,
                  "convolution split scratch too small");
        g.partial = scratch;
    }
    const bool c8 = v.C == 8;
    if (mode == kConvFwd) {
        if (c8) launch_direct<kConvFwd, 8>(grid, sh.nt, g, s);
        else launch_direct<kConvFwd, 32>(grid, sh.nt, g, s);
    } else {
        if (c8) launch_direct<kConvBwdData, 8>(grid, sh.nt, g, s);
        else launch_direct<kConvBwdData, 32>(grid, sh.nt, g, s);
    }
    PSL_HIP(hipGetLastError());
    if (sh.splits > 1) {
        const int64_t items = int64_t(g.M) * (g.N / 8);
        const int blocks = int(std::min<int64_t>((items + 255) / 256, 4096));
        if (mode == kConvFwd)
            hipLaunchKernelGGL(k_conv_split_reduce<kConvFwd>, dim3(blocks), dim3(256), 0, s, g,
                               sh.splits);
        else
            hipLaunchKernelGGL(k_conv_split_reduce<kConvBwdData>, dim3(blocks), dim3(256), 0, s, g,
                               sh.splits);
        PSL_HIP(hipGetLastError());
    }
    return pooled || headed;
}

// forward conv: in (cin_pad channels view) -> out view, bias, ReLU; with
// `pool`, also its 2x2x2 max pooling where the kernel can fuse it (returns
// whether it did)
struct HeadArgs {
    const float* w;
    const float* b;
    const float* dose;
    float* out;
    bool skip_store;
};

bool conv_fwd(const UNet& u, const UNet::Conv& L, View in, View out, hipStream_t s,
              const View* pool = nullptr, uint8_t* arg = nullptr, const HeadArgs* head = nullptr) {
    GemmArgs g{};
    g.a = in;
    g.b = out;
    g.wt = L.wf;
    g.wfrag = L.wff;
    g.bias = u.params.as<float>() + L.b;
    g.M = int(int64_t(in.D) * in.H * in.W);
    g.N = L.cout;
    g.K = 27 * L.cin_pad;
    g.cin = L.cin;
    g.cout = L.cout;
    g.relu = 1;
    if (pool) {
        g.pool = *pool;
        g.arg = arg;
    }
    if (head) {
        g.head_w = head->w;
        g.head_b = head->b;
        g.head_dose = head->dose;
        g.head_out = head->out;
        g.skip_store = head->skip_store ? 1 : 0;
    }
    return conv_launch(kConvFwd, g, s, u.wpart.as<float>(), u.wpart.bytes / 4);
}

// bias gradient over P positions: enough blocks that every thread sums a
// few dozen positions
void bias_grad(View g, int64_t P, float* gb, hipStream_t s) {
    const int64_t rows = 256 / (g.C / 8);
    const int blocks = int(std::max<int64_t>(1, std::min<int64_t>((P + 32 * rows - 1) / (32 * rows), 4096)));
    hipLaunchKernelGGL(k_bias_grad, dim3(blocks), dim3(256), 0, s, g, int(P), gb);
}

// Split-K of a weight gradient over `positions`: about 2048 workgroups in
// all, at least 1024 positions per split.
int wgrad_splits(int64_t positions, int M, int N) {
    const Tile tl = tile_for(kConvWgrad, M, N);
    const int64_t tiles = int64_t((M + tl.bm - 1) / tl.bm) * ((N + tl.bn - 1) / tl.bn);
    const int64_t by_grid = std::max<int64_t>(1, 2048 / tiles);
    return int(std::max<int64_t>(1, std::min<int64_t>(positions / 1024, by_grid)));
}

// Direct (brick) weight gradient of a convolution: the grid divides into
// bricks, and the input channels (c_pad) and output channels (M) into 32s.
bool wgrad_direct(int D, int H, int W, int c_pad, int M) {
    return D % kDZ == 0 && H % kDY == 0 && W % kDX == 0 && c_pad % 32 == 0 && M % 32 == 0;
}

// Bricks per workgroup of the direct weight gradient: about 512 workgroups
// in all (two rounds of one per CU; each takes 106 KB of LDS), at least 4
// bricks each.
int direct_bricks_per_split(int D, int H, int W, int c_pad, int M) {
    const int64_t bricks = int64_t(D / kDZ) * (H / kDY) * (W / kDX);
    const int64_t tiles = int64_t(M / 32) * (c_pad / 32);
    const int64_t splits = std::max<int64_t>(1, std::min<int64_t>(bricks / 4, 512 / tiles));
    return int((bricks + splits - 1) / splits);
}

int64_t direct_splits(int D, int H, int W, int c_pad, int M) {
    const int64_t bricks = int64_t(D / kDZ) * (H / kDY) * (W / kDX);
    const int per = direct_bricks_per_split(D, H, W, c_pad, M);
    return (bricks + per - 1) / per;
}

// Weight-gradient GEMM with split-K into the partial buffer, then the
// reduction into the gradient array.
void wgrad_launch(int mode, GemmArgs g, int64_t positions, int c_pad, const UNet& u,
                  hipStream_t s) {
    g.partial = u.wpart.as<float>();
    int splits = 0;
    const View& v = g.a;
    if (mode == kConvWgrad && wgrad_direct(v.D, v.H, v.W, c_pad, g.M)) {
        PSL_CHECK(v.C == c_pad && g.b.C == g.M && g.N == 27 * c_pad, "direct weight-gradient shapes");
        const int per = direct_bricks_per_split(v.D, v.H, v.W, c_pad, g.M);
        splits = int(direct_splits(v.D, v.H, v.W, c_pad, g.M));
        PSL_CHECK(u.wpart.bytes >= size_t(splits) * g.M * g.N * 4, "weight-gradient scratch too small");
        hipLaunchKernelGGL(k_conv_wgrad_direct, dim3(splits, g.M / 32, c_pad / 32), dim3(256), 0, s,
                           g, per);
        PSL_HIP(hipGetLastError());
    } else {
        const int splits0 = wgrad_splits(positions, g.M, g.N);
        g.k_per_split = int(((positions + splits0 - 1) / splits0 + kKT - 1) / kKT * kKT);
        splits = int((positions + g.k_per_split - 1) / g.k_per_split);
        PSL_CHECK(u.wpart.bytes >= size_t(splits) * g.M * g.N * 4, "weight-gradient scratch too small");
        gemm_launch(mode, g, s, splits);
    }
    const int64_t total = int64_t(g.M) * g.N;
    const int blocks = int(std::min<int64_t>((total + 255) / 256, 2048));
    if (mode == kConvWgrad)
        hipLaunchKernelGGL(k_wgrad_reduce<kConvWgrad>, dim3(blocks), dim3(256), 0, s, g.partial,
                           splits, g.M, g.N, c_pad, g.cin, g.cout, g.wgrad);
    else
        hipLaunchKernelGGL(k_wgrad_reduce<kTconvWgrad>, dim3(blocks), dim3(256), 0, s, g.partial,
                           splits, g.M, g.N, c_pad, g.cin, g.cout, g.wgrad);
    PSL_HIP(hipGetLastError());
}

// Floats of split-K scratch the largest weight gradient of the network needs.
size_t wpart_floats(const UNet& u) {
    size_t most = 0;
    auto need = [&](int64_t positions, int M, int N) {
        most = std::max(most, size_t(wgrad_splits(positions, M, N)) * M * N);
    };
    // channel splits of the direct convolution: forward (cin_pad -> cout),
    // input gradient (cout -> cin) and the decoder's unmasked half (C -> C)
    auto split = [&](int k, int C, int N) {
        const int* d = u.dims[k];
        const ConvShape sh = conv_shape(d[0], d[1], d[2], C, N);
        if (sh.splits > 1) most = std::max(most, size_t(sh.splits) * size_t(u.P(k)) * N);
    };
    auto conv = [&](int k, const UNet::Conv& L) {
        const int* d = u.dims[k];
        split(k, L.cin_pad, L.cout);
        split(k, L.cout, L.cin);
        split(k, L.cout, L.cout);
        need(u.P(k), L.cout, 27 * L.cin_pad);
        if (wgrad_direct(d[0], d[1], d[2], L.cin_pad, L.cout))
            most = std::max(most, size_t(direct_splits(d[0], d[1], d[2], L.cin_pad, L.cout)) *
                                      L.cout * 27 * L.cin_pad);
    };
    for (int k = 0; k < kLevels; ++k) {
        conv(k, u.enc_a[k]);
        conv(k, u.enc_b[k]);
    }
    for (int k = 0; k < kLevels - 1; ++k) {
        conv(k, u.dec_a[k]);
        conv(k, u.dec_b[k]);
        need(u.P(k + 1), u.ch(k + 1), 8 * u.ch(k));
    }
    return most;
}


// conv backward: gz (gradient at the conv output, ReLU already applied) ->
// weight and bias gradients, and (optional) gradient at the input masked by
// the input activation
void conv_bwd(const UNet& u, const UNet::Conv& L, View in, View gz, View* gin, hipStream_t s) {
    const int64_t P = int64_t(in.D) * in.H * in.W;
    GemmArgs g{};
    g.a = in;
    g.b = gz;
    g.wgrad = u.grads.as<float>() + L.w;
    g.M = L.cout;
    g.N = 27 * L.cin_pad;
    g.K = int(P);
    g.cin = L.cin;
    g.cout = L.cout;
    wgrad_launch(kConvWgrad, g, P, L.cin_pad, u, s);
    bias_grad(gz, P, u.grads.as<float>() + L.b, s);
    if (gin) {
        GemmArgs d{};
        d.a = gz;
        d.b = *gin;
        d.wt = L.wb;
        d.wfrag = L.wbf;
        d.mask = in;
        d.M = int(P);
        d.N = L.cin;
        d.K = 27 * L.cout;
        d.cin = L.cin;
        d.cout = L.cout;
        conv_launch(kConvBwdData, d, s, u.wpart.as<float>(), u.wpart.bytes / 4);
    }
}

void build_layout(UNet& u) {
    int64_t off = 0;
    auto conv = [&](UNet::Conv& L, int cin, int cout) {
        L.cin = cin;
        L.cout = cout;
        L.cin_pad = (cin + 7) / 8 * 8;
        L.w = off;
        off += int64_t(cout) * cin * 27;
        L.b = off;
        off += cout;
    };
    auto tconv = [&](UNet::Tconv& L, int cin, int cout) {
        L.cin = cin;
        L.cout = cout;
        L.w = off;
        off += int64_t(cin) * cout * 8;
        L.b = off;
        off += cout;
    };
    int prev = 2;
    for (int k = 0; k < kLevels; ++k) {
        conv(u.enc_a[k], prev, u.ch(k));
        conv(u.enc_b[k], u.ch(k), u.ch(k));
        prev = u.ch(k);
    }
    for (int k = kLevels - 2; k >= 0; --k) {
        tconv(u.up[k], u.ch(k + 1), u.ch(k));
        conv(u.dec_a[k], 2 * u.ch(k), u.ch(k));
        conv(u.dec_b[k], u.ch(k), u.ch(k));
    }
    u.head_w = off;
    off += u.c;
    u.head_b = off;
    off += 1;
    u.n_params = off;
}

void pack_all(UNet& u, hipStream_t s) {
    const float* p = u.params.as<float>();
    auto pc = [&](UNet::Conv& L) {
        hipLaunchKernelGGL(k_pack_conv, dim3(grid1(int64_t(L.cout) * L.cin_pad * 27)), dim3(256), 0,
                           s, p + L.w, L.cout, L.cin, L.cin_pad, L.wf, L.wb);
        if (L.wff)
            hipLaunchKernelGGL(k_frag, dim3(grid1(frag_elems(L.cout, L.cin_pad) / 8)), dim3(256), 0, s,
                               L.wf, L.cout, L.cin_pad, L.wff);
        if (L.wbf)
            hipLaunchKernelGGL(k_frag, dim3(grid1(frag_elems(L.cin, L.cout) / 8)), dim3(256), 0, s,
                               L.wb, L.cin, L.cout, L.wbf);
    };
    for (int k = 0; k < kLevels; ++k) {
        pc(u.enc_a[k]);
        pc(u.enc_b[k]);
    }
    for (int k = 0; k < kLevels - 1; ++k) {
        pc(u.dec_a[k]);
        pc(u.dec_b[k]);
        hipLaunchKernelGGL(k_pack_tconv, dim3(grid1(int64_t(u.up[k].cin) * u.up[k].cout * 8)),
                           dim3(256), 0, s, p + u.up[k].w, u.up[k].cin, u.up[k].cout, u.up[k].wf,
                           u.up[k].wb);
    }
    PSL_HIP(hipGetLastError());
}

// input [2][P0] FP32 -> pred [P0] FP32 (activations kept for the backward
// pass unless keep is false: then the last layer's output, which only the
// head reads, is not written where the head is fused into its convolution)
void forward(UNet& u, const float* input, hipStream_t s, bool keep = true, float* pred = nullptr) {
    float* const pred_out = pred ? pred : u.pred.as<float>();
    const int64_t P0 = u.P(0);
    hipLaunchKernelGGL(k_pack_input, dim3(grid1(P0)), dim3(256), 0, s, input, int(P0),
                       u.x0.as<uint16_t>());
    View h = view(u.x0, u, 0, 8, 8, 0);
    bool pooled_here = false;   // the previous level's conv wrote this level's pooling
    for (int k = 0; k < kLevels; ++k) {
        const int C = u.ch(k);
        if (k > 0) {
            View pooled = view(u.pooled[k], u, k, u.ch(k - 1), u.ch(k - 1), 0);
            if (!pooled_here)
                hipLaunchKernelGGL(k_pool_fwd, dim3(grid1(u.P(k) * u.ch(k - 1) / 8)), dim3(256), 0, s,
                                   h, pooled, u.arg[k].as<uint8_t>());
            h = pooled;
        }
        View a = view(u.enc_a_out[k], u, k, C, C, 0);
        conv_fwd(u, u.enc_a[k], h, a, s);
        // encoder output of levels < 3 goes straight into the first half of the
        // decoder's concatenation buffer (and is pooled for the next level)
        if (k < kLevels - 1) {
            View b = view(u.cat[k], u, k, C, 2 * C, 0);
            View pooled = view(u.pooled[k + 1], u, k + 1, C, C, 0);
            pooled_here = conv_fwd(u, u.enc_b[k], a, b, s, &pooled, u.arg[k + 1].as<uint8_t>());
            h = b;
        } else {
            View b = view(u.bottom_b, u, k, C, C, 0);
            conv_fwd(u, u.enc_b[k], a, b, s);
            h = b;
        }
    }
    for (int k = kLevels - 2; k >= 0; --k) {
        const int C = u.ch(k);
        View upv = view(u.cat[k], u, k, C, 2 * C, C);
        GemmArgs g{};
        g.a = h;
        g.b = upv;
        g.wt = u.up[k].wf;
        g.bias = u.params.as<float>() + u.up[k].b;
        g.M = int(u.P(k + 1));
        g.N = 8 * C;
        g.K = u.ch(k + 1);
        g.cin = u.ch(k + 1);
        g.cout = C;
        gemm_launch(kTconvFwd, g, s);
        View catv = view(u.cat[k], u, k, 2 * C, 2 * C, 0);
        View a = view(u.dec_a_out[k], u, k, C, C, 0);
        conv_fwd(u, u.dec_a[k], catv, a, s);
        View b = view(u.dec_b_out[k], u, k, C, C, 0);
        if (k == 0) {
            // the head in the last convolution's epilogue where it can go
            const HeadArgs head{u.params.as<float>() + u.head_w, u.params.as<float>() + u.head_b,
                                input, pred_out, !keep};
            if (!conv_fwd(u, u.dec_b[k], a, b, s, nullptr, nullptr, &head))
                hipLaunchKernelGGL(k_head_fwd, dim3(grid1(P0)), dim3(256), 0, s, b,
                                   u.params.as<float>() + u.head_w,
                                   u.params.as<float>() + u.head_b, input, int(P0), pred_out);
        } else {
            conv_fwd(u, u.dec_b[k], a, b, s);
        }
        h = b;
    }
    PSL_HIP(hipGetLastError());
}

// loss + gradients of every parameter into u.grads (zeroed here)
void backward(UNet& u, const float* input, const float* target, hipStream_t s) {
    const int64_t P0 = u.P(0);
    hipLaunchKernelGGL(k_zero_f, dim3(grid1(u.n_params)), dim3(256), 0, s, u.grads.as<float>(),
                       u.n_params);
    hipLaunchKernelGGL(k_zero_d, dim3(1), dim3(64), 0, s, u.loss.as<double>(), 64);
    hipLaunchKernelGGL(k_loss, dim3(grid1(P0, 1024)), dim3(256), 0, s, u.pred.as<float>(), target,
                       int(P0), u.gy.as<float>(), u.loss.as<double>());
    // head
    const int C0 = u.ch(0);
    View h0 = view(u.dec_b_out[0], u, 0, C0, C0, 0);
    View g = view(u.g1[0], u, 0, C0, C0, 0);
    hipLaunchKernelGGL(k_head_bwd, dim3(grid1(P0, 512)), dim3(256), 0, s, h0,
                       u.params.as<float>() + u.head_w, u.gy.as<float>(), int(P0),
                       u.grads.as<float>() + u.head_w, u.grads.as<float>() + u.head_b, g);
    // decoder, top level first; g holds the gradient at the ReLU output of
    // dec_b (already masked)
    View gz = g;
    for (int k = 0; k < kLevels - 1; ++k) {
        const int C = u.ch(k);
        View a = view(u.dec_a_out[k], u, k, C, C, 0);
        View ga = view(u.g2[k], u, k, C, C, 0);
        conv_bwd(u, u.dec_b[k], a, gz, &ga, s);            // ga masked by a > 0
        View catv = view(u.cat[k], u, k, 2 * C, 2 * C, 0);
        View gcat = view(u.gcat[k], u, k, 2 * C, 2 * C, 0);
        conv_bwd(u, u.dec_a[k], catv, ga, &gcat, s);       // masked by cat > 0
        // the up half of gcat was masked by the tconv output > 0, which is not a
        // ReLU output; recompute it unmasked below from the same product
        View gup = view(u.gcat[k], u, k, C, 2 * C, C);
        {
            GemmArgs d{};
            d.a = ga;
            d.b = gup;
            d.wt = u.dec_a[k].wb + size_t(C) * 27 * C;   // rows C..2C-1 of the backward pack
            d.wfrag = u.dec_a[k].wbf ? u.dec_a[k].wbf + size_t(C / 32) * ((C / 32) * 54) * 512
                                     : nullptr;          // the same rows (32-row tiles C / 32 ..)
            d.M = int(u.P(k));
            d.N = C;
            d.K = 27 * C;
            d.cin = 2 * C;
            d.cout = C;
            conv_launch(kConvBwdData, d, s, u.wpart.as<float>(), u.wpart.bytes / 4);
        }
        // tconv backward: weights, bias, gradient at its input (masked by the
        // lower level's ReLU output)
        View hin = k + 1 < kLevels - 1 ? view(u.dec_b_out[k + 1], u, k + 1, u.ch(k + 1), u.ch(k + 1), 0)
                                       : view(u.bottom_b, u, k + 1, u.ch(k + 1), u.ch(k + 1), 0);
        GemmArgs w{};
        w.a = hin;
        w.b = gup;
        w.wgrad = u.grads.as<float>() + u.up[k].w;
        w.M = u.ch(k + 1);
        w.N = 8 * C;
        w.K = int(u.P(k + 1));
        w.cin = u.ch(k + 1);
        w.cout = C;
        wgrad_launch(kTconvWgrad, w, u.P(k + 1), 0, u, s);
        bias_grad(gup, u.P(k), u.grads.as<float>() + u.up[k].b, s);
        View gh = view(u.g1[k + 1], u, k + 1, u.ch(k + 1), u.ch(k + 1), 0);
        GemmArgs d{};
        d.a = gup;
        d.b = gh;
        d.wt = u.up[k].wb;
        d.mask = hin;
        d.M = int(u.P(k + 1));
        d.N = u.ch(k + 1);
        d.K = 8 * C;
        d.cin = u.ch(k + 1);
        d.cout = C;
        gemm_launch(kTconvBwdData, d, s);
        gz = gh;
    }
    // encoder, bottom level first; gz = gradient at the ReLU output of enc_b[k]
    for (int k = kLevels - 1; k >= 0; --k) {
        const int C = u.ch(k);
        View a = view(u.enc_a_out[k], u, k, C, C, 0);
        View ga = view(u.g2[k], u, k, C, C, 0);
        conv_bwd(u, u.enc_b[k], a, gz, &ga, s);
        View hin = k == 0 ? view(u.x0, u, 0, 8, 8, 0) : view(u.pooled[k], u, k, u.ch(k - 1), u.ch(k - 1), 0);
        if (k == 0) {
            conv_bwd(u, u.enc_a[k], hin, ga, nullptr, s);
        } else {
            View gp = view(u.g1[k], u, k, u.ch(k - 1), u.ch(k - 1), 0);
            // pooled values are maxima of ReLU outputs: the mask hin > 0 is the
            // same as the mask of the selected fine value
            conv_bwd(u, u.enc_a[k], hin, ga, &gp, s);
            const int Cf = u.ch(k - 1);
            View gskip = view(u.gcat[k - 1], u, k - 1, Cf, 2 * Cf, 0);
            View hfine = view(u.cat[k - 1], u, k - 1, Cf, 2 * Cf, 0);
            View gfine = view(u.g1[k - 1], u, k - 1, Cf, Cf, 0);
            hipLaunchKernelGGL(k_pool_bwd, dim3(grid1(u.P(k - 1) * Cf / 8)), dim3(256), 0, s, gp,
                               u.arg[k].as<uint8_t>(), gskip, hfine, gfine);
            gz = gfine;
        }
    }
    PSL_HIP(hipGetLastError());
}

UNet* unet_cast(psl_unet* p) { return reinterpret_cast<UNet*>(p); }

// ---- error gate: a candidate dose judged by an independent plain dose -------
constexpr int kGateBlocks = 256;

__device__ double block_sum(double v, double* s) {
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// Mean of the candidate over block (kx, ky, kz) of b^3 voxels (clipped at the
// grid's edges).
__device__ double cand_block_mean(const float* cand, int nx, int ny, int nz, int b, int kx,
                                  int ky, int kz) {
    double sum = 0.0;
    int cnt = 0;
    for (int z = kz * b; z < min(nz, (kz + 1) * b); ++z)
        for (int y = ky * b; y < min(ny, (ky + 1) * b); ++y)
            for (int x = kx * b; x < min(nx, (kx + 1) * b); ++x) {
                sum += double(cand[(int64_t(z) * ny + y) * nx + x]);
                ++cnt;
            }
    return sum / cnt;
}

// Per-workgroup maxima of the candidate's block means: the candidate's
// maximum at the scale of a block, which a hot voxel does not set.
__global__ void __launch_bounds__(256) k_gate_max(const float* cand, int nx, int ny, int nz, int b,
                                                  double* part) {
    __shared__ double s[256];
    const int bx = (nx + b - 1) / b, by = (ny + b - 1) / b, bz = (nz + b - 1) / b;
    const int64_t nblk = int64_t(bx) * by * bz;
    double m = 0.0;
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < nblk;
         k += int64_t(gridDim.x) * blockDim.x)
        m = fmax(m, cand_block_mean(cand, nx, ny, nz, b, int(k % bx), int((k / bx) % by),
                                    int(k / (int64_t(bx) * by))));
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = blockDim.x / 2; off > 0; off >>= 1) {
        if (int(threadIdx.x) < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

constexpr double kGateTop = 0.95;   // the candidate's top region: >= 95 % of its maximum
constexpr int kGateSums = 9;

// One thread per b^3 block of voxels, with M the candidate's largest block
// mean: over the voxels where the candidate exceeds cutoff * M, the block's
// count n_b, sum of (c - p)^2, sum of sigma^2 and T_b = sum of
// ((c - p)^2 - sigma^2); the block-level sums T_b^2, T_b n_b and n_b^2 give a
// standard error of the mean of (c - p)^2 - sigma^2 that allows for noise
// correlated within a block (an electron track deposits in neighbouring
// voxels); and over the candidate's top region (blocks whose candidate mean
// is at least kGateTop M) the voxel count and the plain dose.
// The voxels are chosen by the candidate, which is independent of the plain
// dose's noise: a choice by the plain dose would favour its upward
// fluctuations, whose replica variance is large too, and bias the difference
// low.  part_max holds kGateBlocks maxima.
__global__ void __launch_bounds__(256) k_gate_sums(const float* cand, const double* plain,
                                                   const double* sig, int nx, int ny, int nz,
                                                   int b, const double* part_max, double cutoff,
                                                   double* part) {
    __shared__ double s[256];
    __shared__ double s_thr, s_top;
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int j = 0; j < kGateBlocks; ++j) m = fmax(m, part_max[j]);
        s_thr = cutoff * m;
        s_top = kGateTop * m;
    }
    __syncthreads();
    const double thr = s_thr, top = s_top;
    const int bx = (nx + b - 1) / b, by = (ny + b - 1) / b, bz = (nz + b - 1) / b;
    const int64_t nblk = int64_t(bx) * by * bz;
    double acc[kGateSums] = {};
    for (int64_t k = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; k < nblk;
         k += int64_t(gridDim.x) * blockDim.x) {
        const int kx = int(k % bx), ky = int((k / bx) % by), kz = int(k / (int64_t(bx) * by));
        const bool in_top = cand_block_mean(cand, nx, ny, nz, b, kx, ky, kz) >= top;
        double nb = 0.0, d2 = 0.0, v2 = 0.0, tb = 0.0, nt = 0.0, st = 0.0;
        for (int z = kz * b; z < min(nz, (kz + 1) * b); ++z)
            for (int y = ky * b; y < min(ny, (ky + 1) * b); ++y)
                for (int x = kx * b; x < min(nx, (kx + 1) * b); ++x) {
                    const int64_t i = (int64_t(z) * ny + y) * nx + x;
                    const double p = plain[i];
                    if (in_top) {
                        nt += 1.0;
                        st += p;
                    }
                    const double c = double(cand[i]);
                    if (!(c > thr)) continue;
                    const double d = c - p;
                    const double v = sig[i] * sig[i];
                    nb += 1.0;
                    d2 += d * d;
                    v2 += v;
                    tb += d * d - v;
                }
        acc[0] += nb;
        acc[1] += d2;
        acc[2] += v2;
        acc[3] += tb * tb;
        acc[4] += tb * nb;
        acc[5] += nb * nb;
        acc[6] += nt;
        acc[7] += st;
        acc[8] += nb > 0.0 ? 1.0 : 0.0;
    }
    double r[kGateSums];
    for (int q = 0; q < kGateSums; ++q) r[q] = block_sum(acc[q], s);
    if (threadIdx.x == 0)
        for (int q = 0; q < kGateSums; ++q) part[blockIdx.x * kGateSums + q] = r[q];
}
}  // namespace
}  // namespace psl

using namespace psl;

extern "C" int psl_unet_create(int32_t base_width, int32_t d, int32_t h, int32_t w, psl_unet** out) {
    return guarded([&] {
        PSL_CHECK(out, "null argument");
        PSL_CHECK(base_width == 8 || base_width == 16 || base_width == 32,
                  "base width must be 8, 16 or 32");
        PSL_CHECK(d >= 8 && h >= 8 && w >= 8 && d % 8 == 0 && h % 8 == 0 && w % 8 == 0,
                  "volume dimensions must be multiples of 8");
        PSL_CHECK(int64_t(d) * h * w < (int64_t(1) << 31) / 64, "volume too large");
        auto u = std::make_unique<UNet>();
        u->c = base_width;
        u->D = d;
        u->H = h;
        u->W = w;
        for (int k = 0; k < kLevels; ++k) {
            u->dims[k][0] = d >> k;
            u->dims[k][1] = h >> k;
            u->dims[k][2] = w >> k;
        }
        build_layout(*u);
        const size_t np = size_t(u->n_params);
        u->params.alloc(np * 4);
        u->grads.alloc(np * 4);
        u->adam_m.alloc(np * 4);
        u->adam_v.alloc(np * 4);
        // packed BF16 weights: forward + backward layouts of every layer
        size_t pk = 0;
        auto cnt_conv = [&](UNet::Conv& L) {
            pk += size_t(L.cout) * L.cin_pad * 27 + size_t(L.cin) * 27 * L.cout;
            pk += size_t(frag_elems(L.cout, L.cin_pad)) + size_t(frag_elems(L.cin, L.cout)) + 16;
        };
        for (int k = 0; k < kLevels; ++k) {
            cnt_conv(u->enc_a[k]);
            cnt_conv(u->enc_b[k]);
        }
        for (int k = 0; k < kLevels - 1; ++k) {
            cnt_conv(u->dec_a[k]);
            cnt_conv(u->dec_b[k]);
            pk += 2 * size_t(u->up[k].cin) * u->up[k].cout * 8;
        }
        u->packed.alloc(pk * 2 + 4096);
        uint16_t* q = u->packed.as<uint16_t>();
        auto take = [&](size_t n) { uint16_t* r = q; q += (n + 7) / 8 * 8; return r; };
        auto place_conv = [&](UNet::Conv& L) {
            L.wf = take(size_t(L.cout) * L.cin_pad * 27);
            L.wb = take(size_t(L.cin) * 27 * L.cout);
            const int64_t ff = frag_elems(L.cout, L.cin_pad), bf = frag_elems(L.cin, L.cout);
            L.wff = ff ? take(size_t(ff)) : nullptr;
            L.wbf = bf ? take(size_t(bf)) : nullptr;
        };
        for (int k = 0; k < kLevels; ++k) {
            place_conv(u->enc_a[k]);
            place_conv(u->enc_b[k]);
        }
        for (int k = 0; k < kLevels - 1; ++k) {
            place_conv(u->dec_a[k]);
            place_conv(u->dec_b[k]);
            u->up[k].wf = take(size_t(u->up[k].cin) * u->up[k].cout * 8);
            u->up[k].wb = take(size_t(u->up[k].cin) * u->up[k].cout * 8);
        }
        u->x0.alloc(size_t(u->P(0)) * 8 * 2);
        for (int k = 0; k < kLevels; ++k) {
            const size_t P = size_t(u->P(k)), C = size_t(u->ch(k));
            u->cat[k].alloc(P * 2 * C * 2);
            u->enc_a_out[k].alloc(P * C * 2);
            u->dec_a_out[k].alloc(P * C * 2);
            u->dec_b_out[k].alloc(P * C * 2);
            u->g1[k].alloc(P * 2 * C * 2);
            u->g2[k].alloc(P * 2 * C * 2);
            u->gcat[k].alloc(P * 2 * C * 2);
            if (k > 0) {
                u->pooled[k].alloc(P * size_t(u->ch(k - 1)) * 2);
                u->arg[k].alloc(P * size_t(u->ch(k - 1)));
            }
        }
        u->bottom_b.alloc(size_t(u->P(kLevels - 1)) * u->ch(kLevels - 1) * 2);
        u->pred.alloc(size_t(u->P(0)) * 4);
        u->gy.alloc(size_t(u->P(0)) * 4);
        u->loss.alloc(64 * 8);
        u->wpart.alloc(wpart_floats(*u) * 4);
        hipLaunchKernelGGL(k_zero_f, dim3(grid1(int64_t(np))), dim3(256), 0, nullptr,
                           u->adam_m.as<float>(), int64_t(np));
        hipLaunchKernelGGL(k_zero_f, dim3(grid1(int64_t(np))), dim3(256), 0, nullptr,
                           u->adam_v.as<float>(), int64_t(np));
        PSL_HIP(hipDeviceSynchronize());
        *out = reinterpret_cast<psl_unet*>(u.release());
    });
}

extern "C" void psl_unet_free(psl_unet* net) { delete unet_cast(net); }

extern "C" int psl_unet_param_count(const psl_unet* net, int64_t* n) {
    return guarded([&] {
        PSL_CHECK(net && n, "null argument");
        *n = reinterpret_cast<const UNet*>(net)->n_params;
    });
}

extern "C" int psl_unet_set_params(psl_unet* net, const float* host) {
    return guarded([&] {
        PSL_CHECK(net && host, "null argument");
        UNet& u = *unet_cast(net);
        PSL_HIP(hipMemcpy(u.params.p, host, size_t(u.n_params) * 4, hipMemcpyHostToDevice));
        hipLaunchKernelGGL(k_zero_f, dim3(grid1(u.n_params)), dim3(256), 0, nullptr,
                           u.adam_m.as<float>(), u.n_params);
        hipLaunchKernelGGL(k_zero_f, dim3(grid1(u.n_params)), dim3(256), 0, nullptr,
                           u.adam_v.as<float>(), u.n_params);
        u.step = 0;
        pack_all(u, nullptr);
        PSL_HIP(hipDeviceSynchronize());
    });
}

extern "C" int psl_unet_get_params(const psl_unet* net, float* host) {
    return guarded([&] {
        PSL_CHECK(net && host, "null argument");
        const UNet& u = *reinterpret_cast<const UNet*>(net);
        PSL_HIP(hipMemcpy(host, u.params.p, size_t(u.n_params) * 4, hipMemcpyDeviceToHost));
    });
}

extern "C" int psl_unet_forward(psl_unet* net, const float* input, float* pred, void* stream) {
    return guarded([&] {
        PSL_CHECK(net && input && pred, "null argument");
        UNet& u = *unet_cast(net);
        hipStream_t s = static_cast<hipStream_t>(stream);
        // inference only: the prediction straight into the caller's buffer,
        // the last layer's activations (read only by the backward pass) not kept
        forward(u, input, s, false, pred);
    });
}

extern "C" int psl_unet_gradients(psl_unet* net, const float* input, const float* target,
                                  float* grads_host, double* loss) {
    return guarded([&] {
        PSL_CHECK(net && input && target, "null argument");
        UNet& u = *unet_cast(net);
        forward(u, input, nullptr);
        backward(u, input, target, nullptr);
        PSL_HIP(hipDeviceSynchronize());
        if (grads_host)
            PSL_HIP(hipMemcpy(grads_host, u.grads.p, size_t(u.n_params) * 4, hipMemcpyDeviceToHost));
        if (loss) {
            double parts[64];
            PSL_HIP(hipMemcpy(parts, u.loss.p, sizeof parts, hipMemcpyDeviceToHost));
            double l = 0.0;
            for (double v : parts) l += v;
            *loss = l;
        }
    });
}

extern "C" int psl_unet_train_step(psl_unet* net, const float* input, const float* target, float lr,
                                   double* loss_dev, void* stream) {
    return guarded([&] {
        PSL_CHECK(net && input && target, "null argument");
        PSL_CHECK(lr > 0.f, "learning rate must be > 0");
        UNet& u = *unet_cast(net);
        hipStream_t s = static_cast<hipStream_t>(stream);
        forward(u, input, s);
        backward(u, input, target, s);
        u.step += 1;
        const float b1 = 0.9f, b2 = 0.999f;
        const float c1 = 1.f - std::pow(b1, float(u.step)), c2 = 1.f - std::pow(b2, float(u.step));
        hipLaunchKernelGGL(k_adam, dim3(grid1(u.n_params)), dim3(256), 0, s, u.params.as<float>(),
                           u.grads.as<float>(), u.adam_m.as<float>(), u.adam_v.as<float>(),
                           u.n_params, lr, b1, b2, 1e-8f, c1, c2);
        pack_all(u, s);
        if (loss_dev)
            PSL_HIP(hipMemcpyAsync(loss_dev, u.loss.p, 64 * 8, hipMemcpyDeviceToDevice, s));
    });
}

extern "C" int psl_dose_gate(const float* cand, const double* plain, const double* plain_sigma,
                             int32_t nx, int32_t ny, int32_t nz, int32_t block, double cutoff,
                             double* out, void* stream) {
    return guarded([&] {
        PSL_CHECK(cand && plain && plain_sigma && out, "null argument");
        PSL_CHECK(nx > 0 && ny > 0 && nz > 0, "empty dose");
        PSL_CHECK(int64_t(nx) * ny * nz < (int64_t(1) << 40), "dose grid too large");
        PSL_CHECK(block >= 1 && block <= 64, "block edge must lie in [1, 64]");
        PSL_CHECK(cutoff >= 0.0 && cutoff < 1.0, "cutoff must lie in [0, 1)");
        hipStream_t s = static_cast<hipStream_t>(stream);
        DevBuf part;
        part.alloc(size_t(kGateBlocks) * (1 + kGateSums) * sizeof(double));
        double* pmax = part.as<double>();
        double* psum = pmax + kGateBlocks;
        hipLaunchKernelGGL(k_gate_max, dim3(kGateBlocks), dim3(256), 0, s, cand, nx, ny, nz,
                           block, pmax);
        hipLaunchKernelGGL(k_gate_sums, dim3(kGateBlocks), dim3(256), 0, s, cand, plain,
                           plain_sigma, nx, ny, nz, block, pmax, cutoff, psum);
        PSL_HIP(hipGetLastError());
        std::vector<double> h(size_t(kGateBlocks) * (1 + kGateSums));
        PSL_HIP(hipMemcpyAsync(h.data(), part.p, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                               s));
        PSL_HIP(hipStreamSynchronize(s));
        double mx = 0.0, acc[kGateSums] = {};
        for (int j = 0; j < kGateBlocks; ++j) {
            mx = std::max(mx, h[j]);
            for (int k = 0; k < kGateSums; ++k) acc[k] += h[kGateBlocks + j * kGateSums + k];
        }
        out[0] = acc[0];
        out[1] = mx;
        for (int k = 1; k < kGateSums; ++k) out[k + 1] = acc[k];
    });
}
