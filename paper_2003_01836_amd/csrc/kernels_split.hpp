// kernels_split.hpp -- plans whose targets take several lanes each
// (kernels_split.hip): the copies of the targets, and the sum of the partial
// potentials.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bltc {

// phi[i] = sum over p < parts, in order, of buf[p n + i], i < n
hipError_t launch_sum_parts(const double* buf, int64_t n, int32_t parts, double* phi,
                            hipStream_t s);

// parts copies of the n targets: tgt_t[p n + i] = tgt[i] and
// orig_t[p n + i] = p n + orig[i], p < parts
hipError_t launch_replicate_targets(double4* tgt_t, int64_t* orig_t, const double4* tgt,
                                    const int64_t* orig, int64_t n, int32_t parts, hipStream_t s);

}  // namespace bltc
