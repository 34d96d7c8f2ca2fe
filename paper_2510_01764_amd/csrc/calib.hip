// Roofline calibration kernels: a streaming HBM write of a known byte count
// (the attainable write bandwidth shown beside the 8 TB/s peak) and a plain
// device copy (its byte counters scale those of the step kernels), timed on
// the same device as the step kernels.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>

extern "C" {

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

// Each block writes one contiguous chunk of kCalibChunk x 4 KB with all of its
// stores issued back to back (no loop-carried work): of the store patterns
// measured on MI355X (grid-stride loops, persistent blocks, chunks of 16 KB to
// 1 MB, with and without the nontemporal hint) the fastest, about 6.1 TB/s.
constexpr uint32_t kCalibChunk = 64;   // 16-byte stores per thread
__global__ __launch_bounds__(256) void octax_calib_write_kernel(u32x4 *dst, uint64_t n16, uint32_t v) {
    const u32x4 val = {v, v, v, v};
    const uint64_t base = (uint64_t)blockIdx.x * 256 * kCalibChunk + threadIdx.x;
    if (base + 256ull * (kCalibChunk - 1) < n16) {
#pragma unroll
        for (uint32_t u = 0; u < kCalibChunk; u++) dst[base + 256ull * u] = val;
    } else {
        for (uint32_t u = 0; u < kCalibChunk; u++)
            if (base + 256ull * u < n16) dst[base + 256ull * u] = val;
    }
}

__global__ __launch_bounds__(256) void octax_calib_write_nt_kernel(u32x4 *dst, uint64_t n16, uint32_t v) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    const u32x4 val = {v, v, v, v};
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
        __builtin_nontemporal_store(val, dst + i);
}

__global__ __launch_bounds__(256) void octax_calib_copy_kernel(const uint4 *src, uint4 *dst, uint64_t n16) {
    const uint64_t stride = (uint64_t)gridDim.x * 256;
    for (uint64_t i = (uint64_t)blockIdx.x * 256 + threadIdx.x; i < n16; i += stride)
        dst[i] = src[i];
}

// Stream `bytes` (a multiple of 16) of the value v into d_dst; nontemporal
// != 0 uses stores with the nontemporal hint.
int32_t octax_calib_write(void *d_dst, uint64_t bytes, uint32_t v, uint32_t nontemporal, void *stream) {
    if (!d_dst || bytes % 16) return -1;
    if (bytes == 0) return 0;
    const uint64_t n16 = bytes / 16;
    if (nontemporal) {
        const uint32_t blocks = (uint32_t)std::min<uint64_t>(256 * 32, (n16 + 255) / 256);
        hipLaunchKernelGGL(octax_calib_write_nt_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                           (u32x4 *)d_dst, n16, v);
    } else {
        const uint64_t chunk = 256ull * kCalibChunk;
        const uint64_t blocks = (n16 + chunk - 1) / chunk;
        if (blocks > 0x7FFFFFFFull) return -1;
        hipLaunchKernelGGL(octax_calib_write_kernel, dim3((uint32_t)blocks), dim3(256), 0, (hipStream_t)stream,
                           (u32x4 *)d_dst, n16, v);
    }
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

// Copy `bytes` (a multiple of 16) from d_src to d_dst.
int32_t octax_calib_copy(const void *d_src, void *d_dst, uint64_t bytes, void *stream) {
    if (!d_src || !d_dst || bytes % 16) return -1;
    const uint64_t n16 = bytes / 16;
    const uint32_t blocks = (uint32_t)std::min<uint64_t>(256 * 32, (n16 + 255) / 256);
    hipLaunchKernelGGL(octax_calib_copy_kernel, dim3(blocks), dim3(256), 0, (hipStream_t)stream,
                       (const uint4 *)d_src, (uint4 *)d_dst, n16);
    return hipGetLastError() == hipSuccess ? 0 : -3;
}

}
