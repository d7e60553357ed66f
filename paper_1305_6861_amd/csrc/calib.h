// Measurement support: a vector-FMA throughput kernel (not part of the
// simulation), used to state the attainable FP32 / FP64 FMA rate of the
// build's code generation next to the published peaks.
#pragma once
#include <hip/hip_runtime_api.h>
#include <stdint.h>

namespace ps {

// Launches n_blocks workgroups of 256 lanes; every lane runs 8 independent
// FMA chains for iters steps (2 * 8 * iters flops per lane) and writes
// nothing unless its sum equals never_equal (the caller passes a NaN).
hipError_t launch_fma_chain(int precision, int64_t n_blocks, int32_t iters, double never_equal, void* sink,
                            hipStream_t st);

}  // namespace ps
