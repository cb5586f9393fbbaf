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

// out[slot][k] = sum over the sources of the source batches listed for the
// slot (d.near_*) of G(t_k, y_j) q_j at the slot's Chebyshev points t_k
// (grids slot_nodes[slot][3][n+1]), FP64 or FP32-mixed as kp.precision.  The
// lists are cut into pieces d.chunk_slot/chunk_begin (first entry)/
// chunk_count (entries)/chunk_dst (output row); rows past d.nslots of `out`
// hold partial sums, added up per slot by slot_chunk_off (kernels_cp.hip)
hipError_t launch_proxy_potentials(const DevicePlan& d, const double* slot_nodes,
                                   const KernelParams& kp, double* out, hipStream_t s);

}  // namespace bltc
