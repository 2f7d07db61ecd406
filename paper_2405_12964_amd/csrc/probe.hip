// Memory-bandwidth probe: the reference rate against which the walk kernels'
// BVH and primitive reads are priced.  A closest-point traversal fetches one
// pair node or one primitive at an address that depends on the query, so
// its reads are random gathers of short records rather than streams; this
// probe measures the rate of such gathers over a buffer of a chosen size
// (working sets of a few MB sit in the L2 and the Infinity Cache, large
// ones in HBM), and, for comparison, the rate of a plain streaming read.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>
#include <vector>

#include "host_common.hpp"

using dwos_host::fail;

namespace {

constexpr int kProbeBlock = 256;

__global__ void probe_fill_kernel(float4* buf, int64_t n4) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x)
        buf[i] = make_float4(1.0f, 2.0f, 3.0f, (float)(i & 1023));
}

// Random gathers: every thread reads `reads` records of `w4` float4 words at
// line indices drawn from a per-thread xorshift generator (addresses do not
// depend on loaded data, so many reads are in flight at once).  `flag` is 0
// at run time; the sum is stored only under it, which keeps the loads alive.
template <int W4>
__global__ void __launch_bounds__(kProbeBlock) probe_gather_kernel(const float4* buf, uint64_t n_lines,
                                                                   int reads, uint32_t seed, int flag,
                                                                   float* sink) {
    const uint32_t tid = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t h = (tid * 0x9E3779B9u) ^ seed;
    h = h ? h : 0x1234567u;
    float acc = 0.0f;
#pragma unroll 8
    for (int r = 0; r < reads; ++r) {
        h ^= h << 13;
        h ^= h >> 17;
        h ^= h << 5;
        const uint64_t line = ((uint64_t)h * n_lines) >> 32;
        const float4* p = buf + line * W4;
#pragma unroll
        for (int w = 0; w < W4; ++w) {
            const float4 v = p[w];
            acc += (v.x + v.y) + (v.z + v.w);
        }
    }
    if (flag) sink[tid] = acc;
}

// Streaming read: grid-stride over the whole buffer, coalesced 16-byte words.
__global__ void __launch_bounds__(kProbeBlock) probe_stream_kernel(const float4* buf, int64_t n4, int flag,
                                                                   float* sink) {
    float acc = 0.0f;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += (int64_t)gridDim.x * blockDim.x) {
        const float4 v = buf[i];
        acc += (v.x + v.y) + (v.z + v.w);
    }
    if (flag) sink[blockIdx.x * blockDim.x + threadIdx.x] = acc;
}

}  // namespace

extern "C" {

dwos_status dwos_probe_bandwidth(int64_t bytes, int32_t line_bytes, int32_t mode, double* gbps, double* ms) {
    if (!gbps) return fail(DWOS_EINVAL, "probe_bandwidth: NULL output");
    if (bytes < (1 << 16) || bytes > (int64_t(1) << 36))
        return fail(DWOS_EINVAL, "probe_bandwidth: buffer size must be in [64 KiB, 64 GiB]");
    if (mode != 0 && mode != 1) return fail(DWOS_EINVAL, "probe_bandwidth: mode must be 0 (gather) or 1 (stream)");
    if (mode == 0 && line_bytes != 16 && line_bytes != 32 && line_bytes != 48 && line_bytes != 64 &&
        line_bytes != 96 && line_bytes != 128)
        return fail(DWOS_EINVAL, "probe_bandwidth: line_bytes must be 16, 32, 48, 64, 96 or 128");
    int dev = 0, cus = 0;
    HIP_OK(hipGetDevice(&dev));
    HIP_OK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t n4 = bytes / 16;
    dwos_host::DevBuf buf, sink;
    HIP_OK(buf.reserve((size_t)n4 * 16));
    const unsigned grid = (unsigned)std::max(1, cus) * 32u;     // 32 blocks of 256 per CU
    HIP_OK(sink.reserve((size_t)grid * kProbeBlock * sizeof(float)));
    hipStream_t s = nullptr;
    HIP_OK(hipStreamCreate(&s));
    struct StreamGuard { hipStream_t s; ~StreamGuard() { (void)hipStreamDestroy(s); } } guard{s};
    hipLaunchKernelGGL(probe_fill_kernel, dim3(grid), dim3(kProbeBlock), 0, s, buf.as<float4>(), n4);
    HIP_OK(hipGetLastError());
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_OK(hipEventCreate(&e0));
    HIP_OK(hipEventCreate(&e1));
    struct EventGuard { hipEvent_t a, b; ~EventGuard() { (void)hipEventDestroy(a); (void)hipEventDestroy(b); } } eg{e0, e1};
    const int w4 = mode == 0 ? line_bytes / 16 : 1;
    const uint64_t n_lines = mode == 0 ? (uint64_t)(bytes / line_bytes) : 0;
    const int reads = 64;
    auto launch = [&](uint32_t seed) {
        if (mode == 1) {
            hipLaunchKernelGGL(probe_stream_kernel, dim3(grid), dim3(kProbeBlock), 0, s, buf.as<float4>(), n4, 0,
                               sink.as<float>());
            return;
        }
        const float4* b = buf.as<float4>();
        float* k = sink.as<float>();
        switch (w4) {
            case 1: hipLaunchKernelGGL(probe_gather_kernel<1>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
            case 2: hipLaunchKernelGGL(probe_gather_kernel<2>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
            case 3: hipLaunchKernelGGL(probe_gather_kernel<3>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
            case 4: hipLaunchKernelGGL(probe_gather_kernel<4>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
            case 6: hipLaunchKernelGGL(probe_gather_kernel<6>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
            default: hipLaunchKernelGGL(probe_gather_kernel<8>, dim3(grid), dim3(kProbeBlock), 0, s, b, n_lines, reads, seed, 0, k); break;
        }
    };
    // warm the caches with the same access pattern, then keep the fastest of
    // several timed launches
    launch(1u);
    HIP_OK(hipGetLastError());
    HIP_OK(hipStreamSynchronize(s));
    double best = 1e30;
    for (int rep = 0; rep < 8; ++rep) {
        HIP_OK(hipEventRecord(e0, s));
        launch(2u + (uint32_t)rep);
        HIP_OK(hipGetLastError());
        HIP_OK(hipEventRecord(e1, s));
        HIP_OK(hipEventSynchronize(e1));
        float t = 0.f;
        HIP_OK(hipEventElapsedTime(&t, e0, e1));
        best = std::min(best, (double)t);
    }
    const double moved = mode == 0 ? (double)grid * kProbeBlock * reads * w4 * 16.0 : (double)n4 * 16.0;
    *gbps = moved / (best * 1e-3) / 1e9;
    if (ms) *ms = best;
    return DWOS_OK;
}

}  // extern "C"
