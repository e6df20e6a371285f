// Streaming ceiling of the device: a plain copy with the access kinds the
// fused JPCG pass uses for the streams it does not re-read (16-byte vector
// loads and stores, optionally with the nontemporal hint). The benchmark
// times it beside the solver to price the solver's bandwidth against what a
// kernel with no arithmetic, no halo and no barrier reaches on the same GPU.
#include "pb_internal.hpp"

#include <algorithm>

namespace pb {
namespace {

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <bool NT>
__global__ __launch_bounds__(256) void k_stream_copy(const f32x4* __restrict__ src, f32x4* __restrict__ dst,
                                                     int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        if constexpr (NT) {
            __builtin_nontemporal_store(__builtin_nontemporal_load(src + i), dst + i);
        } else {
            dst[i] = src[i];
        }
    }
}

}  // namespace
}  // namespace pb

using namespace pb;

extern "C" pb_status pb_stream_copy(const void* src, void* dst, size_t bytes, int32_t nontemporal, void* stream) {
    PB_ARG(src && dst, "pb_stream_copy: null pointer");
    PB_ARG(((uintptr_t)src & 15) == 0 && ((uintptr_t)dst & 15) == 0 && bytes % 16 == 0,
           "pb_stream_copy: pointers and size must be multiples of 16 bytes");
    int dev = 0, cus = 0;
    PB_HIP(hipGetDevice(&dev));
    PB_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    const int64_t n = (int64_t)(bytes / 16);
    const unsigned grid = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, (int64_t)cus * 8));
    hipStream_t st = (hipStream_t)stream;
    if (nontemporal)
        hipLaunchKernelGGL(k_stream_copy<true>, dim3(grid), dim3(256), 0, st, (const f32x4*)src, (f32x4*)dst, n);
    else
        hipLaunchKernelGGL(k_stream_copy<false>, dim3(grid), dim3(256), 0, st, (const f32x4*)src, (f32x4*)dst, n);
    PB_HIP(hipGetLastError());
    return PB_OK;
}
