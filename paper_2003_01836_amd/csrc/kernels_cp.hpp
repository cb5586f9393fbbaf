// kernels_cp.hpp -- launch wrappers of the cluster-particle kernels: proxy
// potentials, and the target interpolation shared with the cluster-cluster
// treecode (kernels_cp.hip).
#pragma once

#include "kernels.hpp"

namespace bltc {

// phi[tgt_orig[i]] += the interpolant of the proxy potentials phat[slot][P] of
// every slot listed for the target's leaf (path_off/path_slot per batch of d),
// grids slot_nodes[slot][3][n+1] (kernels_cp.hip)
hipError_t launch_interpolate_targets(const DevicePlan& d, const int32_t* path_off,
                                      const int32_t* path_slot, const double* slot_nodes,
                                      const double* phat, double* phi, hipStream_t s);

// Proxy potentials over the pieces of the slots' lists (d.chunk_slot, first
// entry d.chunk_begin, entries d.chunk_count, output row d.chunk_dst; entries
// d.near_begin/near_count/near_leaf): row r of `out` = sum over the piece's
// sources of G(t_k, y_j) q_j at its slot's Chebyshev points t_k (grids
// slot_nodes[slot][3][n+1]), FP64 or FP32-mixed as kp.precision; the caller
// sums the rows of a slot of several pieces (kernels_cp.hip)
hipError_t launch_proxy_potentials(const DevicePlan& d, const double* slot_nodes,
                                   const KernelParams& kp, double* out, hipStream_t s);

}  // namespace bltc
