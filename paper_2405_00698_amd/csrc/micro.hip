// micro.hip -- roofline microbenchmarks: the LDS and VALU rates this chip
// actually delivers, measured with the same compiler and flags as the step
// kernels, as denominators for the step kernel's roofline fractions.
#include "internal.h"

namespace sr {

namespace {

constexpr int MB = 256;        // threads per workgroup
constexpr int LDS_F4 = 2048;   // 32 KB of float4 per workgroup

// Conflict-free LDS reads: each of the 8 unrolled reads per iteration hits a
// different float4 row; addresses move every iteration so nothing is hoisted.
template <int WORDS>
__global__ __launch_bounds__(MB) void k_lds_read(float *out, int iters) {
    __shared__ float4 buf[LDS_F4];
    for (int i = threadIdx.x; i < LDS_F4; i += MB) buf[i] = make_float4(i, i + 1, i + 2, i + 3);
    __syncthreads();
    float a0 = 0.f, a1 = 0.f, a2 = 0.f, a3 = 0.f;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            // a wave reads 64 consecutive rows; the window moves by one wave each iteration
            const int idx = (threadIdx.x + u * MB + it * 64) & (LDS_F4 - 1);
            const float4 *p = buf + idx;
            if (WORDS == 4) {
                const float4 v = *p;
                a0 += v.x;
                a1 += v.y;
                a2 += v.z;
                a3 += v.w;
            } else if (WORDS == 3) {
                typedef float f3v __attribute__((ext_vector_type(3)));
                const f3v v = *reinterpret_cast<const f3v *>(__builtin_assume_aligned(p, 16));
                a0 += v.x;
                a1 += v.y;
                a2 += v.z;
            } else {
                a0 += reinterpret_cast<const float *>(buf)[(threadIdx.x + u * MB + it * 64) & (4 * LDS_F4 - 1)];
            }
        }
    }
    out[blockIdx.x * MB + threadIdx.x] = a0 + a1 + a2 + a3;
}

// Eight independent FMA chains per lane.
__global__ __launch_bounds__(MB) void k_valu_fma(float *out, int iters, float a, float b) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = threadIdx.x * 1e-3f + j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = fmaf(x[j], a, b);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[blockIdx.x * MB + threadIdx.x] = s;
}

// Eight independent reciprocal-square-root chains per lane.
__global__ __launch_bounds__(MB) void k_valu_rsq(float *out, int iters) {
    float x[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) x[j] = 1.0f + threadIdx.x * 1e-3f + j;
    for (int it = 0; it < iters; ++it) {
#pragma unroll
        for (int j = 0; j < 8; ++j) x[j] = __builtin_amdgcn_rsqf(x[j]);
    }
    float s = 0.f;
#pragma unroll
    for (int j = 0; j < 8; ++j) s += x[j];
    out[blockIdx.x * MB + threadIdx.x] = s;
}

// Streaming device copy (16-byte loads and stores, grid-stride): the HBM rate
// a kernel can reach, read and written bytes together.
__global__ __launch_bounds__(MB) void k_hbm_copy(const float4 *__restrict__ src, float4 *__restrict__ dst, size_t n) {
    for (size_t i = (size_t)blockIdx.x * MB + threadIdx.x; i < n; i += (size_t)gridDim.x * MB) dst[i] = src[i];
}

}  // namespace

hipError_t launch_micro_hbm(const float4 *src, float4 *dst, size_t n, int grid, int passes, hipStream_t st,
                            double *units) {
    for (int p = 0; p < passes; ++p) hipLaunchKernelGGL(k_hbm_copy, dim3(grid), dim3(MB), 0, st, src, dst, n);
    *units = 2.0 * 16.0 * (double)n * passes;
    return hipGetLastError();
}

// which: 0 LDS read 16 B, 1 LDS read 12 B, 2 LDS read 4 B, 3 FP32 FMA, 4 rsq.
// Returns the work of one launch (bytes or lane operations) in *units.
hipError_t launch_micro(int which, int iters, int grid, float *out, hipStream_t st, double *units) {
    const double lanes = (double)grid * MB * (double)iters * 8.0;
    switch (which) {
        case 0: hipLaunchKernelGGL(k_lds_read<4>, dim3(grid), dim3(MB), 0, st, out, iters); *units = lanes * 16; break;
        case 1: hipLaunchKernelGGL(k_lds_read<3>, dim3(grid), dim3(MB), 0, st, out, iters); *units = lanes * 12; break;
        case 2: hipLaunchKernelGGL(k_lds_read<1>, dim3(grid), dim3(MB), 0, st, out, iters); *units = lanes * 4; break;
        case 3: hipLaunchKernelGGL(k_valu_fma, dim3(grid), dim3(MB), 0, st, out, iters, 0.999f, 1e-3f); *units = lanes; break;
        case 4: hipLaunchKernelGGL(k_valu_rsq, dim3(grid), dim3(MB), 0, st, out, iters); *units = lanes; break;
        default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

}  // namespace sr
