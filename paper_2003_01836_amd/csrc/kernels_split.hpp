// kernels_split.hpp -- the sum of the partial potentials of plans whose
// targets take several lanes each (kernels_split.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bltc {

// phi[i] = sum over p < parts, in order, of buf[p n + i], i < n
hipError_t launch_sum_parts(const double* buf, int64_t n, int32_t parts, double* phi,
                            hipStream_t s);

}  // namespace bltc
