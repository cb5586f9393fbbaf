// kernels_cp.hpp -- launch wrapper of the target interpolation kernel of the
// cluster-particle and cluster-cluster treecodes (kernels_cp.hip).
#pragma once

#include "kernels.hpp"

namespace bltc {

// phi[tgt_orig[i]] += the interpolant of the proxy potentials phat[slot][P] of
// every slot listed for the target's leaf (path_off/path_slot per batch of d),
// grids slot_nodes[slot][3][n+1] (kernels_cp.hip)
hipError_t launch_interpolate_targets(const DevicePlan& d, const int32_t* path_off,
                                      const int32_t* path_slot, const double* slot_nodes,
                                      const double* phat, double* phi, hipStream_t s);

}  // namespace bltc
