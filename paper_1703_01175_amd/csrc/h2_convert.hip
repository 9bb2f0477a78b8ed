// Storage-tier conversions of the block data and vectors.
//  - FP32 tier: round to nearest float (complex64 storage);
//  - BF16 hi+lo tier: hi = bf16_rne(v), lo = bf16_rne(v - hi) for the real and
//    imaginary parts; one complex packs into a 32-bit word (re in the low half).
#include <hip/hip_runtime.h>

#include "h2_api_internal.h"

namespace h2 {

__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
    uint32_t u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (u >> 16) | ((u & 0xffffu) ? 0x40u : 0u);  // inf / nan
    uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return u >> 16;
}

__device__ __forceinline__ float bf16_to_float(uint32_t b) { return __uint_as_float(b << 16); }

__global__ void k_convert_fp32(const double2* __restrict__ src, float2* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double2 v = src[i];
        dst[i] = make_float2((float)v.x, (float)v.y);
    }
}

__global__ void k_to_fp64(const float2* __restrict__ src, double2* __restrict__ dst, int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        float2 v = src[i];
        dst[i] = make_double2(v.x, v.y);
    }
}

__global__ void k_split_bf16(const double2* __restrict__ src, uint32_t* __restrict__ hi, uint32_t* __restrict__ lo,
                             int64_t n) {
    for (int64_t i = blockIdx.x * int64_t(blockDim.x) + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x) {
        double2 v = src[i];
        float re = (float)v.x, im = (float)v.y;
        uint32_t hr = bf16_rne_bits(re), hm = bf16_rne_bits(im);
        uint32_t lr = bf16_rne_bits(re - bf16_to_float(hr)), lm = bf16_rne_bits(im - bf16_to_float(hm));
        hi[i] = hr | (hm << 16);
        lo[i] = lr | (lm << 16);
    }
}

static int grid_for(int64_t n) {
    int64_t g = (n + 255) / 256;
    return int(g > 65536 ? 65536 : (g < 1 ? 1 : g));
}

hipError_t launch_convert_fp32(const double2* src, float2* dst, int64_t n, hipStream_t s) {
    k_convert_fp32<<<grid_for(n), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_vec_to_fp32(const double2* src, float2* dst, int64_t n, hipStream_t s) {
    return launch_convert_fp32(src, dst, n, s);
}

hipError_t launch_vec_to_fp64(const float2* src, double2* dst, int64_t n, hipStream_t s) {
    k_to_fp64<<<grid_for(n), 256, 0, s>>>(src, dst, n);
    return hipGetLastError();
}

hipError_t launch_split_bf16(const double2* src, uint32_t* hi, uint32_t* lo, int64_t n, hipStream_t s) {
    k_split_bf16<<<grid_for(n), 256, 0, s>>>(src, hi, lo, n);
    return hipGetLastError();
}

}  // namespace h2
