// Measurement probes for the ceilings of the dose path: the rate of FP32
// atomic adds (no return) into a dose grid along a given address stream, and
// the streaming copy bandwidth of HBM.
#include "common.hpp"

namespace psl {
namespace {

constexpr int kProbeBlock = 256;

__global__ void __launch_bounds__(kProbeBlock) k_probe_atomics(float* grid, int64_t cells,
                                                               const int32_t* addr, int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t a = addr[i];
        if (a >= 0 && a < cells) atomicAdd(grid + a, 1.0f);
    }
}

__global__ void __launch_bounds__(kProbeBlock) k_probe_copy(float4* dst, const float4* src,
                                                            int64_t n) {
    const int64_t stride = int64_t(gridDim.x) * blockDim.x;
    for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += stride)
        dst[i] = src[i];
}

// Average milliseconds of `repeats` launches of `launch` on a private stream.
template <class F>
double time_launches(int repeats, F&& launch) {
    hipStream_t s;
    hipEvent_t e0, e1;
    PSL_HIP(hipStreamCreate(&s));
    PSL_HIP(hipEventCreate(&e0));
    PSL_HIP(hipEventCreate(&e1));
    launch(s);   // warm-up
    PSL_HIP(hipGetLastError());
    PSL_HIP(hipEventRecord(e0, s));
    for (int r = 0; r < repeats; ++r) launch(s);
    PSL_HIP(hipGetLastError());
    PSL_HIP(hipEventRecord(e1, s));
    PSL_HIP(hipEventSynchronize(e1));
    float ms = 0.f;
    PSL_HIP(hipEventElapsedTime(&ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipStreamDestroy(s);
    return double(ms) / repeats;
}

int probe_blocks(int64_t n) {
    return int(std::max<int64_t>(1, std::min<int64_t>((n + kProbeBlock - 1) / kProbeBlock, 8192)));
}

}  // namespace
}  // namespace psl

using namespace psl;

extern "C" int psl_probe_atomics(float* grid_dev, int64_t cells, const int32_t* addr_dev,
                                 int64_t n, int32_t repeats, double* ms_out) {
    return guarded([&] {
        PSL_CHECK(grid_dev && addr_dev && ms_out, "psl_probe_atomics: null argument");
        PSL_CHECK(cells > 0 && cells <= INT32_MAX && n > 0 && repeats >= 1,
                  "psl_probe_atomics: bad sizes");
        *ms_out = time_launches(repeats, [&](hipStream_t s) {
            hipLaunchKernelGGL(k_probe_atomics, dim3(probe_blocks(n)), dim3(kProbeBlock), 0, s,
                               grid_dev, cells, addr_dev, n);
        });
    });
}

extern "C" int psl_probe_copy(void* dst_dev, const void* src_dev, int64_t bytes, int32_t repeats,
                              double* ms_out) {
    return guarded([&] {
        PSL_CHECK(dst_dev && src_dev && ms_out, "psl_probe_copy: null argument");
        PSL_CHECK(bytes > 0 && bytes % 16 == 0 && repeats >= 1, "psl_probe_copy: bad sizes");
        PSL_CHECK((reinterpret_cast<uintptr_t>(dst_dev) | reinterpret_cast<uintptr_t>(src_dev)) % 16 == 0,
                  "psl_probe_copy: buffers must be 16-byte aligned");
        const int64_t n = bytes / 16;
        *ms_out = time_launches(repeats, [&](hipStream_t s) {
            hipLaunchKernelGGL(k_probe_copy, dim3(probe_blocks(n)), dim3(kProbeBlock), 0, s,
                               static_cast<float4*>(dst_dev), static_cast<const float4*>(src_dev), n);
        });
    });
}
