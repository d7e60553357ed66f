// Kernel arguments and launchers (host side of kernels.hip).
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

#include "ps_ops.h"

namespace ps {

struct StepArgs {
    const float *x, *y, *z, *m0, *t1, *t2, *dw;  // device SoA object
    int64_t n_spins;
    const Op* ops;           // device, this time slice's operations
    int32_t n_ops;
    int32_t n_rows;          // shaped-pulse rotation rows (9 reals each)
    const void* rows;        // device, n_rows * 9 reals of the kernel precision
    void* partial;           // device, gridDim.x rows of row_stride reals
    int64_t row_stride;      // reals per workgroup row (2 per sample of the slice)
    void* state;             // device, 3 * n_spins reals (Mxy_a re, im, Mz_a), SoA
    int32_t load_state;      // resume from state instead of equilibrium
    int32_t save_state;      // write the anchors back at the end
};

// Spins handled by one workgroup for a given spins-per-lane choice.
int64_t spins_per_block_of(int spins_per_lane);

hipError_t launch_step(const StepArgs& a, int precision, int spins_per_lane, int64_t n_blocks,
                       hipStream_t st);
hipError_t launch_finalize(const void* partial, int precision, int64_t n_blocks, int64_t row_stride,
                           int64_t n_vals, double* out, hipStream_t st);
hipError_t launch_fill_zero(double* out, int64_t n, hipStream_t st);

}  // namespace ps
