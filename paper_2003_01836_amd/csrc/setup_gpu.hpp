// setup_gpu.hpp -- setup phase on the GPU: cluster trees and interaction
// lists (setup_gpu.hip).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <functional>
#include <string>

#include "planner.hpp"

namespace bltc {

// Builds the tree of the n points (x, y, z: device arrays, caller order) with
// leaf capacity cap.  The node arrays of t are filled on the host and equal
// those of build_tree(); t.order, t.x, t.y, t.z stay empty.  Device outputs
// (n entries each, tree order): order[p] = caller index of tree position p,
// pos[p] = (x, y, z, 0), and when rel is not NULL the FP32 coordinates
// relative to the center of the leaf holding p.  The stream is synchronised
// before return.  Returns an empty string on success; a non-finite coordinate
// sets *bad_index to the lowest such caller index.
std::string build_tree_device(Tree& t, int64_t n, const double* x, const double* y,
                              const double* z, int64_t cap, int64_t* order, double4* pos,
                              float4* rel, hipStream_t s, int64_t* bad_index);

// Interaction lists on the device, in the host planner's layout and order.
struct DeviceLists {
    int32_t* far_slot = nullptr;
    int32_t* near_leaf = nullptr;
    int64_t* near_begin = nullptr;
    int64_t* near_count = nullptr;
    int32_t* item_batch = nullptr;     // items as found by the walk (for inspection)
    int32_t* item_cluster = nullptr;
    int32_t* item_kind = nullptr;
    int64_t n_items = 0;
};

// allocates device memory that the caller owns (bytes may be 0)
using DeviceAlloc = std::function<hipError_t(void** p, size_t bytes)>;

// Builds the lists of Alg. 1 for every batch on the GPU.  Needs hp.src, hp.tgt
// and plan_batches(hp); fills far_off, near_off, batch_cost, the slots and the
// pair/evaluation counts of hp, allocates the device lists through alloc and
// fills them.  plan_schedule(hp) completes the plan.  The stream is
// synchronised before return; returns an empty string on success.
std::string build_lists_device(HostPlan& hp, DeviceLists& out, const DeviceAlloc& alloc,
                               hipStream_t s);

}  // namespace bltc
