// Vector-FMA throughput kernel (measurement support; see calib.h).  Eight
// independent chains per lane keep the SIMD issuing one FMA per cycle
// without waiting on a result; the values stay bounded (x <- x a + b with
// a < 1) and nothing is written unless the sum equals a NaN, so neither
// memory traffic nor special values enter the measurement.  Built like the
// other kernels, with packed FP32 disabled, so the FP32 rate is that of
// v_fma_f32 / v_fmac_f32.
#include <hip/hip_runtime.h>

#include "calib.h"

namespace ps {

template <typename T>
__global__ __launch_bounds__(256) void fma_chain_kernel(int32_t iters, T a, T b, T never_equal, T* sink) {
    T x[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) x[k] = (T)(threadIdx.x & 63) * (T)1e-3 + (T)k;
#pragma unroll 4
    for (int32_t i = 0; i < iters; ++i) {
#pragma unroll
        for (int k = 0; k < 8; ++k) x[k] = fma(x[k], a, b);
    }
    T s = 0;
#pragma unroll
    for (int k = 0; k < 8; ++k) s += x[k];
    if (s == never_equal) sink[0] = s;
}

hipError_t launch_fma_chain(int precision, int64_t n_blocks, int32_t iters, double never_equal, void* sink,
                            hipStream_t st) {
    if (n_blocks <= 0 || n_blocks > 0x7fffffff || iters <= 0) return hipErrorInvalidValue;
    if (precision == 64)
        hipLaunchKernelGGL(fma_chain_kernel<double>, dim3((unsigned)n_blocks), dim3(256), 0, st, iters,
                           0.9999999, 1e-9, never_equal, reinterpret_cast<double*>(sink));
    else
        hipLaunchKernelGGL(fma_chain_kernel<float>, dim3((unsigned)n_blocks), dim3(256), 0, st, iters,
                           0.9999f, 1e-6f, (float)never_equal, reinterpret_cast<float*>(sink));
    return hipGetLastError();
}

}  // namespace ps
