// kernels.hpp -- launch wrappers of the gfx950 kernels (internal to the library).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

namespace bltc {

constexpr int kMaxDegree = 16;
constexpr int kMaxHermiteDegree = 10;   // Hermite treecode: 8 (n+1)^3 charges per cluster
constexpr int kGroupSize = 256;      // targets (lanes) per interaction workgroup
constexpr int kGroupSizeSym = 64;    // the same for plans with mutual pairs (finer tail)

// The direct lists the single-vector interaction kernels walk: the plan's own,
// or, when mutual leaf pairs are evaluated by launch_near_pairs, the reduced
// lists plus per batch the unit results to add (pc_off == nullptr: none).
struct NearLists {
    const int32_t* off;
    const int64_t* begin;
    const int64_t* count;
    const int32_t* leaf;
    const int32_t* pc_off;
    const int64_t* pc_base;
    const double* pair_out;
    const int64_t* batch_begin;
};

// A sub-unit of a mutual pair of leaves (B, C) of a plan whose targets are
// its sources: nb of B's particles at tree positions [tb, tb + nb) against
// C's particles at [sb, sb + nc); row sums (potential at those B targets from
// C's sources) to out[roff + i], column sums (at C's targets from those B
// sources) to out[coff + j].
struct SymUnit {
    int64_t tb, sb, roff, coff;
    int32_t nb, nc;
    int32_t batch;    // B's batch (batch_info)
    int32_t leaf;     // C's node (node_info)
    int32_t apart;    // 1: no pair of the unit is at zero distance (SymPlan::apart)
    int32_t pad;
};

// Device-side view of a plan (all device pointers).
struct DevicePlan {
    int32_t degree = 0;
    int32_t hermite = 0;              // Hermite interpolation: 8 (n+1)^3 values per slot
    int64_t nt = 0, ns = 0, nslots = 0, nchunks = 0, ngroups = 0, nbatches = 0;
    // sources in tree order: x, y, z, charge of the current vector
    double4* src = nullptr;
    // targets in batch order: x, y, z, unused
    double4* tgt = nullptr;
    int64_t* tgt_orig = nullptr;      // caller index of each batch position
    const int64_t* src_order = nullptr; // caller index of each tree position
    // FP32-mixed path: sources relative to the center of their leaf
    float4* src32 = nullptr;          // x - c_x, y - c_y, z - c_z, q (tree order)
    double4* node_info = nullptr;     // per source node: box center, radius
    double4* batch_info = nullptr;    // per batch: box center, radius
    // lists
    int32_t* group_batch = nullptr;
    int64_t* group_first = nullptr;
    int64_t* batch_end = nullptr;
    int32_t* far_off = nullptr;
    int32_t* far_slot = nullptr;
    int32_t* near_off = nullptr;
    int64_t* near_begin = nullptr;
    int64_t* near_count = nullptr;
    int32_t* near_leaf = nullptr;
    // upward pass
    double* slot_nodes = nullptr;     // [slot][3][n+1]
    int32_t* chunk_slot = nullptr;
    int64_t* chunk_begin = nullptr;
    int64_t* chunk_count = nullptr;
    int32_t* slot_chunk_off = nullptr;
    int64_t* chunk_dst = nullptr;     // output row of each chunk (slot, or nslots + partial)
    double* qhat = nullptr;           // [slot][P] or [slot][P][16], then partial rows
    float* qhat32 = nullptr;          // [slot][P] (mixed precision; Hermite [slot][(n+1)^3][8])
    // several charge vectors at once (16 per pass)
    int32_t* slot_cluster = nullptr;  // cluster id of each slot
    double* qm = nullptr;             // [ns][16] charges in tree order
    float* qm32 = nullptr;            // [ns][16] (mixed precision)
    double* qhat16 = nullptr;         // [slot][P][16] (same storage as qhat)
    double4* proxies = nullptr;       // [slot][P] expanded Chebyshev grid (x, y, z, -)
    float4* proxies32 = nullptr;      // [slot][P] grid relative to the cluster center
    float* qhat16f = nullptr;         // [slot][P][16] (mixed precision)
    // Hermite: modified charges regrouped per grid point, [slot][(n+1)^3][8]
    double* qhat_h = nullptr;
    // symmetric near field (one charge vector): mutual leaf pairs evaluated once
    // by launch_near_pairs; the interaction kernels then take the reduced direct
    // lists and add, per target, the unit results listed in sym_pc_*
    int32_t sym = 0;
    int64_t sym_units = 0;            // sub-units
    // targets per workgroup of the single-vector interaction kernels (the plan's
    // group size: kGroupSize, or kGroupSizeSym for plans with mutual pairs)
    int32_t group_threads = 256;
    SymUnit* sym_unit = nullptr;
    double* sym_out = nullptr;
    int32_t* sym_near_off = nullptr;
    int64_t* sym_near_begin = nullptr;
    int64_t* sym_near_count = nullptr;
    int32_t* sym_near_leaf = nullptr;
    int32_t* sym_pc_off = nullptr;
    int64_t* sym_pc_base = nullptr;
    int64_t* batch_begin = nullptr;
    // results of the mutual pairs in several rounds through a bounded
    // workspace (sym_rounds > 1): each round's results are folded into
    // sym_acc (one FP64 value per target, tree order), and the interaction
    // kernels read sym_acc through one entry per batch
    int32_t sym_rounds = 0;
    double* sym_acc = nullptr;
};

// Constants of the kernel G passed to the interaction kernels: kappa of the
// Yukawa kernel and delta^2 of the regularized Coulomb kernel.
struct KernelConst {
    double kappa;
    double delta2;
};

// Everything the multi-vector interaction of one system needs (passed by value
// to a kernel, or as an array for the work-queue kernel).
struct MrhsDesc {
    const double4* tgt;
    const int64_t* tgt_orig;
    const double4* src;
    const float4* src32;
    const double* qm;
    const float* qm32;
    const double4* node_info;
    const double4* batch_info;
    const int32_t* group_batch;
    const int64_t* group_first;
    const int64_t* batch_end;
    const int32_t* far_off;
    const int32_t* far_slot;
    const int32_t* near_off;
    const int64_t* near_begin;
    const int64_t* near_count;
    const int32_t* near_leaf;
    const int32_t* slot_cluster;
    const double4* proxies;
    const float4* proxies32;
    const double* qhat16;
    const float* qhat16f;
    double* phi;
    int64_t phi_ld;
    int32_t np;
    int32_t mc;
    KernelConst kc;
};

struct KernelParams {
    int32_t kernel = 0;     // 0 Coulomb, 1 Yukawa, 2 regularized Coulomb
    int32_t precision = 0;  // 0 FP64, 1 FP32-mixed
    double kappa = 0.0;
    double delta = 0.0;
    KernelConst kconst() const { return KernelConst{kappa, delta * delta}; }
};

// src[j].w = q[order[j]] (and src32[j].w when present), j < ns: charges into tree order
hipError_t launch_gather_charges(const DevicePlan& d, const double* q, hipStream_t s);
// upward pass, eqs. 14-15, on the matrix cores (kernels_upward.hip): mw = 1 (charges in
// src[j].w, result buf[slot][k]) or 16 (charges in qm, result buf[slot][k][16]);
// buf holds nslots final rows followed by the partial rows of multi-chunk slots
hipError_t launch_upward_mfma(const DevicePlan& d, int32_t mw, double* buf, float* qhat32,
                              hipStream_t s);
// pieces of the same for many systems in one launch (unit = system, chunk)
struct UpwardDesc {
    const double4* src;
    const double* qm;
    const float* qm32;                // FP32 copies of the charges (FP32-mixed plans)
    const int32_t* chunk_slot;
    const int64_t* chunk_begin;
    const int64_t* chunk_count;
    const int64_t* chunk_dst;
    const double* slot_nodes;
    double* buf;
    int32_t np;
};
// nf: factors per dimension (np, or 2 np for the Hermite interpolation)
size_t upward_lds_bytes(int32_t np, int32_t mw, int32_t nf);
int32_t upward_passes(int32_t nf, int32_t mw);
hipError_t upward_prepare(size_t lds);
hipError_t launch_upward_many(const UpwardDesc* descs, const int2* units, int32_t nunits,
                              int32_t mw, int32_t passes, size_t lds, hipStream_t s);
// the 16-vector Lagrange kernel of n + 1 = np <= 9 for systems of one degree:
// whether it applies, and its launch (FP32 matrix-core products when f32)
bool upward_many_multi(int32_t np, int32_t mw);
hipError_t launch_upward_many_multi(const UpwardDesc* descs, const int2* units, int32_t nunits,
                                    int32_t np, bool f32, hipStream_t s);
hipError_t launch_upward_reduce(const DevicePlan& d, int32_t mw, double* buf, float* qhat32,
                                hipStream_t s);
// (with d.hermite the upward pass forms 8 (n+1)^3 charges per slot and the
// reduction writes them to d.qhat_h, [slot][k][a], and their FP32 copy to
// qhat32 when given; mw must be 1)
// Hermite approximation and direct sums (kernels_hermite.hip), FP64 or
// FP32-mixed as kp.precision, n <= 10
hipError_t launch_interact_hermite(const DevicePlan& d, const KernelParams& kp, double* phi,
                                   hipStream_t s);
inline NearLists near_lists(const DevicePlan& d)
{
    if (d.sym)
        return NearLists{d.sym_near_off, d.sym_near_begin, d.sym_near_count, d.sym_near_leaf,
                         d.sym_pc_off,   d.sym_pc_base,
                         d.sym_rounds > 1 ? d.sym_acc : d.sym_out,            d.batch_begin};
    return NearLists{d.near_off, d.near_begin, d.near_count, d.near_leaf,
                     nullptr,    nullptr,      nullptr,      nullptr};
}
// near field of the mutual leaf pairs (kernels_sym.hip): sub-units
// d.sym_unit[first .. first + count) into d.sym_out, FP64 or FP32-mixed as
// kp.precision
hipError_t launch_near_pairs(const DevicePlan& d, int64_t first, int64_t count,
                             const KernelParams& kp, hipStream_t s);
// one round of mutual-pair results folded into the per-target sums: for batch
// b (targets at [begin[b], end[b])) and target position p of the batch,
// acc[begin[b] + p] = (first ? 0 : acc[...]) + sum over e in [off[b], off[b + 1])
// of out[base[e] + p], in that order
hipError_t launch_fold_pairs(int64_t nbatches, const int64_t* begin, const int64_t* end,
                             const int32_t* off, const int64_t* base, const double* out,
                             double* acc, bool first, hipStream_t s);
// B targets per sub-unit of launch_near_pairs (one wave holds them all in
// registers, 64 per chunk): FP32-mixed and FP64
constexpr int64_t kSymTargetsMixed = 512;
constexpr int64_t kSymTargetsF64 = 512;
// the FP32-mixed path computes the kernel values of pairs closer than
// kMixedTauRel * (distance of the box centers + r_B + 2 r_C) from FP64 coordinates
constexpr double kMixedTauRel = 2.4e-2;
// side of the largest box of points the FP32-mixed path takes: squared FP32
// distances stay below 3 * 2^120, finite
constexpr double kMixedMaxExtent = 0x1p60;
// batch/cluster interactions: eqs. 9 and 11, phi written in caller order
hipError_t launch_interact(const DevicePlan& d, const KernelParams& kp, double* phi,
                           hipStream_t s);
// the same in FP32-mixed arithmetic (kernels_mixed.hip)
hipError_t launch_interact_mixed(const DevicePlan& d, const KernelParams& kp, double* phi,
                                 hipStream_t s);
// several charge vectors (kernels_mrhs.hip): charges of vectors m0..m0+mc-1
// into qm/qm32 (tree order, zero padded to 16), and the interactions of all
// mc vectors: phi[m * phi_ld + i], m < mc
hipError_t launch_gather_charges16(const DevicePlan& d, const double* q, int64_t q_ld, int32_t mc,
                                   hipStream_t s);
hipError_t launch_interact_mrhs(const DevicePlan& d, const KernelParams& kp, double* phi,
                                int64_t phi_ld, int32_t mc, hipStream_t s);
MrhsDesc make_mrhs_desc(const DevicePlan& d, const KernelParams& kp, double* phi, int64_t phi_ld,
                        int32_t mc);
// work queue over (system, group) units of many systems; counter reset first
hipError_t launch_reset_counter(int32_t* counter, hipStream_t s);
hipError_t launch_interact_queue(const MrhsDesc* descs, const int2* units, int32_t nunits,
                                 int32_t* counter, const KernelParams& kp, int32_t workgroups,
                                 hipStream_t s);
const void* interact_queue_symbol(const KernelParams& kp);
// GPU direct sum (eq. 1) of all targets against packed sources
hipError_t launch_pack_sources(int64_t ns, const double* x, const double* y, const double* z,
                               const double* q, double4* out, hipStream_t s);
hipError_t launch_direct(int64_t nt, const double* tx, const double* ty, const double* tz,
                         int64_t ns, const double4* src, const KernelParams& kp, double* phi,
                         hipStream_t s);

}  // namespace bltc
