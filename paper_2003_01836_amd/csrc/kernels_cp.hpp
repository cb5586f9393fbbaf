// kernels_cp.hpp -- launch wrappers of the cluster-particle and cluster-cluster
// kernels (kernels_cp.hip).
#pragma once

#include "kernels.hpp"

namespace bltc {

// phi[tgt_orig[i]] += the interpolant of the proxy potentials phat[slot][P] of
// every slot listed for the target's leaf (path_off/path_slot per batch of d),
// grids slot_nodes[slot][3][n+1] (kernels_cp.hip)
hipError_t launch_interpolate_targets(const DevicePlan& d, const int32_t* path_off,
                                      const int32_t* path_slot, const double* slot_nodes,
                                      const double* phat, double* phi, hipStream_t s);

// tail[i].w = qhat[i] (and tail32[i].w when not NULL), i < n: modified charges
// as the charges of the source-grid points appended to the source array
hipError_t launch_proxy_charges(double4* tail, float4* tail32, const double* qhat, int64_t n,
                                hipStream_t s);

}  // namespace bltc
