// setup_gpu.hip -- the setup phase on the GPU: cluster trees (Sec. II-D) and
// the batch/cluster interaction lists of Alg. 1.
//
// The device build produces exactly the tree of the host planner: the same
// node numbering, ranges, boxes and particle order.  It runs level by level:
//
//  1. box:     minimal box of every open node (per-chunk min/max, then 64-bit
//              atomics on an order-preserving integer image of the doubles, so
//              the result is exact and independent of the reduction order);
//  2. decide:  the host reads the boxes back and applies the tree rules with
//              the planner's own functions (leaf test, aspect-ratio split);
//  3. count:   child code of every particle of a splitting node (comparisons
//              with the box midpoint only), per-chunk counts of the 8 codes;
//  4. offsets: per node, a scan of the chunk counts in (code, chunk) order;
//  5. scatter: stable partition by code -- within a chunk the rank of a
//              particle among equal codes comes from wave ballots, so the
//              permutation equals the host's stable counting sort.
//
// Particles live in two ping-pong buffer sets (x, y, z, caller index).  A
// finished leaf's range is never written again, so at the end each leaf is
// read from the set that was current when it became a leaf.  The final pass
// writes the caller index of every tree position, the positions as double4
// and, on request, FP32 coordinates relative to the leaf center.
//
// Floating-point work on the device is limited to min/max and comparisons;
// midpoints, radii and split decisions are computed on the host by the
// planner's functions, so both builds take every decision on identical values.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <string>
#include <vector>

#include "kernels.hpp"
#include "planner.hpp"
#include "setup_gpu.hpp"

namespace bltc {
namespace {

constexpr int kThreads = 256;           // threads per workgroup (4 waves)
constexpr int kWaves = kThreads / 64;
constexpr int64_t kChunk = 4096;        // particles per chunk (16 per thread)

struct Chunk {
    int64_t begin;      // first tree position of the chunk
    int32_t count;      // particles in the chunk
    int32_t node;       // index of the node in this level's node table
    int32_t j;          // chunk index within its node
    int32_t pad;
};

struct SplitNode {
    double ctr[3];      // box midpoint
    int64_t begin;      // first tree position of the node
    int64_t hist_base;  // first entry of the node's [code][chunk] counts
    int32_t nch;        // chunks of the node
    int32_t mask;       // bit l set: dimension l is cut
};

struct FinalChunk {
    int64_t begin;
    int32_t count;
    int32_t set;        // buffer set holding the leaf's particles
    double ctr[3];      // leaf center (FP32 local coordinates)
};

// order-preserving map of finite doubles to unsigned integers
__device__ __forceinline__ unsigned long long ordered_bits(double v)
{
    const unsigned long long u = static_cast<unsigned long long>(__double_as_longlong(v));
    return (u >> 63) ? ~u : (u | 0x8000000000000000ull);
}

double from_ordered_bits(unsigned long long e)
{
    const unsigned long long u = (e >> 63) ? (e & 0x7fffffffffffffffull) : ~e;
    double v;
    std::memcpy(&v, &u, sizeof(v));
    return v;
}

__global__ void __launch_bounds__(kThreads)
init_points(int64_t n, const double* __restrict__ x, const double* __restrict__ y,
            const double* __restrict__ z, double* __restrict__ bx, double* __restrict__ by,
            double* __restrict__ bz, int32_t* __restrict__ bo, unsigned long long* bad)
{
    const int64_t stride = static_cast<int64_t>(gridDim.x) * kThreads;
    for (int64_t i = static_cast<int64_t>(blockIdx.x) * kThreads + threadIdx.x; i < n; i += stride) {
        const double vx = x[i], vy = y[i], vz = z[i];
        bx[i] = vx;
        by[i] = vy;
        bz[i] = vz;
        bo[i] = static_cast<int32_t>(i);
        if (!isfinite(vx) || !isfinite(vy) || !isfinite(vz))
            atomicMin(bad, static_cast<unsigned long long>(i));
    }
}

__device__ __forceinline__ double wave_min(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v = fmin(v, __shfl_xor(v, m));
    return v;
}

__device__ __forceinline__ double wave_max(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1)
        v = fmax(v, __shfl_xor(v, m));
    return v;
}

// box[6 * node + l] (min of dimension l) and box[6 * node + 3 + l] (max)
__global__ void __launch_bounds__(kThreads)
node_boxes(const Chunk* __restrict__ chunks, const double* __restrict__ x,
           const double* __restrict__ y, const double* __restrict__ z,
           unsigned long long* __restrict__ box)
{
    __shared__ double part[kWaves][6];
    const Chunk c = chunks[blockIdx.x];
    const double* src[3] = {x + c.begin, y + c.begin, z + c.begin};
    double lo[3], hi[3];
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        lo[l] = INFINITY;
        hi[l] = -INFINITY;
    }
    for (int i = threadIdx.x; i < c.count; i += kThreads) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            const double v = src[l][i];
            lo[l] = fmin(lo[l], v);
            hi[l] = fmax(hi[l], v);
        }
    }
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
#pragma unroll
    for (int l = 0; l < 3; ++l) {
        lo[l] = wave_min(lo[l]);
        hi[l] = wave_max(hi[l]);
    }
    if (lane == 0) {
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            part[w][l] = lo[l];
            part[w][3 + l] = hi[l];
        }
    }
    __syncthreads();
    if (threadIdx.x < 6) {
        const int k = threadIdx.x;
        double v = part[0][k];
        for (int u = 1; u < kWaves; ++u)
            v = k < 3 ? fmin(v, part[u][k]) : fmax(v, part[u][k]);
        unsigned long long* dst = box + 6 * static_cast<int64_t>(c.node) + k;
        if (k < 3)
            atomicMin(dst, ordered_bits(v));
        else
            atomicMax(dst, ordered_bits(v));
    }
}

__device__ __forceinline__ int child_code(const SplitNode& s, double x, double y, double z)
{
    int k = 0;
    if ((s.mask & 1) && x >= s.ctr[0]) k |= 1;
    if ((s.mask & 2) && y >= s.ctr[1]) k |= 2;
    if ((s.mask & 4) && z >= s.ctr[2]) k |= 4;
    return k;
}

// hist[node.hist_base + code * node.nch + j] = particles of chunk j with that
// code; cnt[8 * node + code] accumulates the node totals
__global__ void __launch_bounds__(kThreads)
code_counts(const Chunk* __restrict__ chunks, const SplitNode* __restrict__ nodes,
            const double* __restrict__ x, const double* __restrict__ y,
            const double* __restrict__ z, int64_t* __restrict__ hist,
            unsigned long long* __restrict__ cnt)
{
    __shared__ int32_t wc[kWaves][8];
    const Chunk c = chunks[blockIdx.x];
    const SplitNode s = nodes[c.node];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    int32_t mine[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    const int passes = (c.count + kThreads - 1) / kThreads;
    for (int p = 0; p < passes; ++p) {
        const int i = p * kThreads + threadIdx.x;
        int code = 8;
        if (i < c.count)
            code = child_code(s, x[c.begin + i], y[c.begin + i], z[c.begin + i]);
#pragma unroll
        for (int k = 0; k < 8; ++k)
            mine[k] += __popcll(__ballot(code == k));
    }
    if (lane == 0)
        for (int k = 0; k < 8; ++k)
            wc[w][k] = mine[k];
    __syncthreads();
    if (threadIdx.x < 8) {
        const int k = threadIdx.x;
        int64_t t = 0;
        for (int u = 0; u < kWaves; ++u)
            t += wc[u][k];
        hist[s.hist_base + static_cast<int64_t>(k) * s.nch + c.j] = t;
        if (t)
            atomicAdd(cnt + 8 * static_cast<int64_t>(c.node) + k, static_cast<unsigned long long>(t));
    }
}

// one workgroup per splitting node: offs = first destination of each
// (code, chunk) run, i.e. begin + particles of lower codes + particles of the
// same code in earlier chunks
__global__ void __launch_bounds__(kThreads)
code_offsets(const SplitNode* __restrict__ nodes, const unsigned long long* __restrict__ cnt,
             const int64_t* __restrict__ hist, int64_t* __restrict__ offs)
{
    __shared__ int64_t part[kThreads];
    __shared__ int64_t code_base[8];
    const SplitNode s = nodes[blockIdx.x];
    if (threadIdx.x == 0) {
        int64_t run = s.begin;
        for (int k = 0; k < 8; ++k) {
            code_base[k] = run;
            run += static_cast<int64_t>(cnt[8 * static_cast<int64_t>(blockIdx.x) + k]);
        }
    }
    const int64_t per = (s.nch + kThreads - 1) / kThreads;
    const int64_t j0 = std::min<int64_t>(s.nch, per * threadIdx.x);
    const int64_t j1 = std::min<int64_t>(s.nch, j0 + per);
    for (int k = 0; k < 8; ++k) {
        const int64_t* h = hist + s.hist_base + static_cast<int64_t>(k) * s.nch;
        int64_t* o = offs + s.hist_base + static_cast<int64_t>(k) * s.nch;
        int64_t sum = 0;
        for (int64_t j = j0; j < j1; ++j)
            sum += h[j];
        part[threadIdx.x] = sum;
        __syncthreads();
        if (threadIdx.x == 0) {
            int64_t run = code_base[k];
            for (int t = 0; t < kThreads; ++t) {
                const int64_t v = part[t];
                part[t] = run;
                run += v;
            }
        }
        __syncthreads();
        int64_t run = part[threadIdx.x];
        for (int64_t j = j0; j < j1; ++j) {
            o[j] = run;
            run += h[j];
        }
        __syncthreads();
    }
}

// stable partition of every splitting node's range by child code
__global__ void __launch_bounds__(kThreads)
scatter_points(const Chunk* __restrict__ chunks, const SplitNode* __restrict__ nodes,
               const int64_t* __restrict__ offs, const double* __restrict__ x,
               const double* __restrict__ y, const double* __restrict__ z,
               const int32_t* __restrict__ o, double* __restrict__ x2, double* __restrict__ y2,
               double* __restrict__ z2, int32_t* __restrict__ o2)
{
    __shared__ int64_t base[8];
    __shared__ int32_t wc[kWaves][8];
    const Chunk c = chunks[blockIdx.x];
    const SplitNode s = nodes[c.node];
    const int w = threadIdx.x / 64, lane = threadIdx.x % 64;
    const unsigned long long below = (1ull << lane) - 1ull;
    if (threadIdx.x < 8)
        base[threadIdx.x] = offs[s.hist_base + static_cast<int64_t>(threadIdx.x) * s.nch + c.j];
    __syncthreads();
    const int passes = (c.count + kThreads - 1) / kThreads;
    for (int p = 0; p < passes; ++p) {
        const int i = p * kThreads + threadIdx.x;
        const bool valid = i < c.count;
        double vx = 0.0, vy = 0.0, vz = 0.0;
        int32_t vo = 0;
        int code = 8;
        if (valid) {
            vx = x[c.begin + i];
            vy = y[c.begin + i];
            vz = z[c.begin + i];
            vo = o[c.begin + i];
            code = child_code(s, vx, vy, vz);
        }
        int rank = 0;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const unsigned long long m = __ballot(code == k);
            if (code == k)
                rank = __popcll(m & below);
            if (lane == 0)
                wc[w][k] = __popcll(m);
        }
        __syncthreads();
        if (valid) {
            int64_t d = base[code] + rank;
            for (int u = 0; u < w; ++u)
                d += wc[u][code];
            x2[d] = vx;
            y2[d] = vy;
            z2[d] = vz;
            o2[d] = vo;
        }
        __syncthreads();
        if (threadIdx.x < 8) {
            int64_t t = 0;
            for (int u = 0; u < kWaves; ++u)
                t += wc[u][threadIdx.x];
            base[threadIdx.x] += t;
        }
        __syncthreads();
    }
}

struct Sets {
    const double* x[2];
    const double* y[2];
    const double* z[2];
    const int32_t* o[2];
};

__global__ void __launch_bounds__(kThreads)
finish_points(const FinalChunk* __restrict__ chunks, Sets sets, int64_t* __restrict__ order,
              double4* __restrict__ pos, float4* __restrict__ rel)
{
    const FinalChunk c = chunks[blockIdx.x];
    const double* x = sets.x[c.set];
    const double* y = sets.y[c.set];
    const double* z = sets.z[c.set];
    const int32_t* o = sets.o[c.set];
    for (int i = threadIdx.x; i < c.count; i += kThreads) {
        const int64_t p = c.begin + i;
        const double vx = x[p], vy = y[p], vz = z[p];
        order[p] = o[p];
        pos[p] = make_double4(vx, vy, vz, 0.0);
        if (rel)
            rel[p] = make_float4(static_cast<float>(vx - c.ctr[0]), static_cast<float>(vy - c.ctr[1]),
                                 static_cast<float>(vz - c.ctr[2]), 0.0f);
    }
}

// device buffer that grows on demand (the stream is idle whenever it grows)
template <class T>
struct Buf {
    T* p = nullptr;
    size_t cap = 0;
    ~Buf()
    {
        if (p)
            (void)hipFree(p);
    }
    hipError_t reserve(size_t n)
    {
        n = std::max<size_t>(n, 1);
        if (n <= cap)
            return hipSuccess;
        if (p)
            (void)hipFree(p);
        p = nullptr;
        cap = 0;
        hipError_t e = hipMalloc(reinterpret_cast<void**>(&p), n * sizeof(T));
        if (e == hipSuccess)
            cap = n;
        return e;
    }
    hipError_t put(const std::vector<T>& v, hipStream_t s)
    {
        hipError_t e = reserve(v.size());
        if (e == hipSuccess && !v.empty())
            e = hipMemcpyAsync(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice, s);
        return e;
    }
};

#define TB_TRY(call)                                                               \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess)                                                      \
            return std::string(#call) + ": " + hipGetErrorString(e_);              \
    } while (0)

}  // namespace

std::string build_tree_device(Tree& t, int64_t n, const double* x, const double* y,
                              const double* z, int64_t cap, int64_t* order, double4* pos,
                              float4* rel, hipStream_t s, int64_t* bad_index)
{
    t = Tree();
    t.n = n;
    *bad_index = -1;
    if (n == 0)
        return std::string();
    if (n > INT32_MAX)
        return "the device tree build takes at most 2^31 - 1 points";
    Buf<double> bx[2], by[2], bz[2];
    Buf<int32_t> bo[2];
    for (int k = 0; k < 2; ++k) {
        TB_TRY(bx[k].reserve(n));
        TB_TRY(by[k].reserve(n));
        TB_TRY(bz[k].reserve(n));
        TB_TRY(bo[k].reserve(n));
    }
    Buf<unsigned long long> bad, box, cnt;
    Buf<Chunk> chunks_d, split_chunks_d;
    Buf<SplitNode> split_d;
    Buf<int64_t> hist, offs;
    Buf<FinalChunk> final_d;
    const std::vector<unsigned long long> no_bad(1, ~0ull);
    TB_TRY(bad.put(no_bad, s));
    {
        const int64_t blocks = std::min<int64_t>((n + kThreads - 1) / kThreads, 8192);
        init_points<<<static_cast<uint32_t>(blocks), kThreads, 0, s>>>(
            n, x, y, z, bx[0].p, by[0].p, bz[0].p, bo[0].p, bad.p);
        TB_TRY(hipGetLastError());
    }

    t.add_node(0, n, 0, -1);
    std::vector<int32_t> open{0}, next;
    std::vector<int32_t> leaf_set;          // per node: buffer set of a finished leaf
    std::vector<Chunk> chunks, split_chunks;
    std::vector<SplitNode> split;
    std::vector<int32_t> split_node;        // tree id of each splitting node
    std::vector<unsigned long long> box_h, cnt_h;
    int cur = 0;
    bool first_level = true;
    while (!open.empty()) {
        // ---- boxes of the open nodes
        const int64_t nopen = static_cast<int64_t>(open.size());
        chunks.clear();
        for (int64_t i = 0; i < nopen; ++i) {
            const int32_t u = open[i];
            int32_t j = 0;
            for (int64_t off = 0; off < t.count[u]; off += kChunk, ++j)
                chunks.push_back({t.begin[u] + off,
                                  static_cast<int32_t>(std::min<int64_t>(kChunk, t.count[u] - off)),
                                  static_cast<int32_t>(i), j, 0});
        }
        box_h.assign(6 * nopen, 0ull);
        for (int64_t i = 0; i < nopen; ++i)
            for (int l = 0; l < 3; ++l)
                box_h[6 * i + l] = ~0ull;
        TB_TRY(chunks_d.put(chunks, s));
        TB_TRY(box.put(box_h, s));
        node_boxes<<<static_cast<uint32_t>(chunks.size()), kThreads, 0, s>>>(
            chunks_d.p, bx[cur].p, by[cur].p, bz[cur].p, box.p);
        TB_TRY(hipGetLastError());
        TB_TRY(hipMemcpyAsync(box_h.data(), box.p, box_h.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
        unsigned long long bad_h = ~0ull;
        if (first_level)
            TB_TRY(hipMemcpyAsync(&bad_h, bad.p, sizeof(bad_h), hipMemcpyDeviceToHost, s));
        TB_TRY(hipStreamSynchronize(s));
        if (first_level && bad_h != ~0ull) {
            *bad_index = static_cast<int64_t>(bad_h);
            return "coordinate is not finite";
        }
        first_level = false;

        // ---- decisions (planner rules, host arithmetic)
        if (static_cast<int64_t>(leaf_set.size()) < t.nodes())
            leaf_set.resize(t.nodes(), -1);
        split.clear();
        split_node.clear();
        std::vector<int32_t> split_of_open(nopen, -1);
        int64_t hist_total = 0;
        for (int64_t i = 0; i < nopen; ++i) {
            const int32_t u = open[i];
            double lo[3], hi[3];
            for (int l = 0; l < 3; ++l) {
                lo[l] = from_ordered_bits(box_h[6 * i + l]);
                hi[l] = from_ordered_bits(box_h[6 * i + 3 + l]);
            }
            t.set_box(u, lo, hi);
            bool cut[3];
            if (!node_split(t, u, cap, cut)) {
                leaf_set[u] = cur;
                continue;
            }
            SplitNode sn;
            for (int l = 0; l < 3; ++l)
                sn.ctr[l] = t.center[3 * u + l];
            sn.begin = t.begin[u];
            sn.nch = static_cast<int32_t>((t.count[u] + kChunk - 1) / kChunk);
            sn.hist_base = hist_total;
            sn.mask = (cut[0] ? 1 : 0) | (cut[1] ? 2 : 0) | (cut[2] ? 4 : 0);
            hist_total += 8 * static_cast<int64_t>(sn.nch);
            split_of_open[i] = static_cast<int32_t>(split.size());
            split.push_back(sn);
            split_node.push_back(u);
        }
        if (split.empty())
            break;
        split_chunks.clear();
        for (const Chunk& c : chunks)
            if (split_of_open[c.node] >= 0) {
                Chunk d = c;
                d.node = split_of_open[c.node];
                split_chunks.push_back(d);
            }

        // ---- counts, offsets, scatter into the other buffer set
        const int64_t nsplit = static_cast<int64_t>(split.size());
        cnt_h.assign(8 * nsplit, 0ull);
        TB_TRY(split_d.put(split, s));
        TB_TRY(split_chunks_d.put(split_chunks, s));
        TB_TRY(cnt.put(cnt_h, s));
        TB_TRY(hist.reserve(hist_total));
        TB_TRY(offs.reserve(hist_total));
        const uint32_t nsc = static_cast<uint32_t>(split_chunks.size());
        code_counts<<<nsc, kThreads, 0, s>>>(split_chunks_d.p, split_d.p, bx[cur].p, by[cur].p,
                                              bz[cur].p, hist.p, cnt.p);
        TB_TRY(hipGetLastError());
        code_offsets<<<static_cast<uint32_t>(nsplit), kThreads, 0, s>>>(split_d.p, cnt.p, hist.p,
                                                                         offs.p);
        TB_TRY(hipGetLastError());
        const int nxt = 1 - cur;
        scatter_points<<<nsc, kThreads, 0, s>>>(split_chunks_d.p, split_d.p, offs.p, bx[cur].p,
                                                 by[cur].p, bz[cur].p, bo[cur].p, bx[nxt].p,
                                                 by[nxt].p, bz[nxt].p, bo[nxt].p);
        TB_TRY(hipGetLastError());
        TB_TRY(hipMemcpyAsync(cnt_h.data(), cnt.p, cnt_h.size() * sizeof(unsigned long long),
                              hipMemcpyDeviceToHost, s));
        TB_TRY(hipStreamSynchronize(s));

        // ---- children (appended in node order: breadth-first numbering)
        next.clear();
        for (int64_t i = 0; i < nsplit; ++i) {
            const int32_t u = split_node[i];
            int nonempty = 0;
            for (int k = 0; k < 8; ++k)
                nonempty += cnt_h[8 * i + k] > 0;
            if (nonempty < 2) {
                // every particle in one child: a leaf (its range is unchanged)
                leaf_set[u] = cur;
                continue;
            }
            const int32_t first = static_cast<int32_t>(t.nodes());
            int64_t start = t.begin[u];
            int32_t nk = 0;
            for (int k = 0; k < 8; ++k) {
                const int64_t ck = static_cast<int64_t>(cnt_h[8 * i + k]);
                if (ck == 0)
                    continue;
                next.push_back(t.add_node(start, ck, t.level[u] + 1, u));
                start += ck;
                ++nk;
            }
            t.first_child[u] = first;
            t.nchild[u] = nk;
        }
        open.swap(next);
        cur = nxt;
    }

    // ---- tree order, positions, local coordinates
    leaf_set.resize(t.nodes(), -1);
    std::vector<FinalChunk> fin;
    for (int64_t u = 0; u < t.nodes(); ++u) {
        if (t.nchild[u] != 0)
            continue;
        for (int64_t off = 0; off < t.count[u]; off += kChunk) {
            FinalChunk f;
            f.begin = t.begin[u] + off;
            f.count = static_cast<int32_t>(std::min<int64_t>(kChunk, t.count[u] - off));
            f.set = leaf_set[u];
            for (int l = 0; l < 3; ++l)
                f.ctr[l] = t.center[3 * u + l];
            fin.push_back(f);
        }
    }
    TB_TRY(final_d.put(fin, s));
    Sets sets;
    for (int k = 0; k < 2; ++k) {
        sets.x[k] = bx[k].p;
        sets.y[k] = by[k].p;
        sets.z[k] = bz[k].p;
        sets.o[k] = bo[k].p;
    }
    finish_points<<<static_cast<uint32_t>(fin.size()), kThreads, 0, s>>>(final_d.p, sets, order,
                                                                           pos, rel);
    TB_TRY(hipGetLastError());
    // the scratch buffers are freed on return: finish first
    TB_TRY(hipStreamSynchronize(s));
    return std::string();
}

// ---------------------------------------------------------------------------
// Interaction lists (Alg. 1) on the GPU: one thread per batch walks the source
// tree depth first.  The walk is stackless: "skip" of a node is the node that
// follows its subtree in depth-first order (next sibling, else the parent's
// skip), so descending goes to the first child and accepting or summing a
// cluster directly goes to skip.  The visiting order equals the host's
// explicit-stack walk, hence the lists come out in the same order.  This file
// is compiled without floating-point contraction and the MAC uses the
// correctly rounded square root, so the decisions equal the host planner's.
// ---------------------------------------------------------------------------
namespace {

// one batch per lane; small workgroups spread the few waves over many CUs
constexpr int kListThreads = 64;

struct TravNode {
    double cx, cy, cz, r;   // box center and radius
    int64_t count;          // particles
    int32_t first_child;    // -1 for a leaf
    int32_t skip;           // next node after the subtree in depth-first order (-1: end)
};

struct TravBatch {
    double cx, cy, cz, r;
    int64_t count;
};

struct ListCounts {
    int32_t nfar, ndirect;
    int64_t nnear;          // leaf ranges of the direct clusters
    int64_t direct_particles;
};

__device__ __forceinline__ bool mac_geometric(const TravBatch& b, const TravNode& c, double theta)
{
    const double dx = b.cx - c.cx;
    const double dy = b.cy - c.cy;
    const double dz = b.cz - c.cz;
    const double R = __dsqrt_rn(dx * dx + dy * dy + dz * dz);
    return b.r + c.r < theta * R;
}

__global__ void __launch_bounds__(kListThreads)
count_lists(int64_t nb, const TravBatch* __restrict__ batches, const TravNode* __restrict__ nodes,
            double theta, int64_t P, const int64_t* __restrict__ run_len,
            ListCounts* __restrict__ counts, uint8_t* __restrict__ used)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kListThreads + threadIdx.x;
    if (b >= nb)
        return;
    const TravBatch tb = batches[b];
    ListCounts lc = {0, 0, 0, 0};
    int32_t c = 0;
    while (c >= 0) {
        const TravNode nd = nodes[c];
        const bool geometric = mac_geometric(tb, nd, theta);
        if (geometric && P < nd.count) {
            ++lc.nfar;
            used[c] = 1;
            c = nd.skip;
        } else if (!geometric && nd.first_child >= 0) {
            c = nd.first_child;
        } else {
            ++lc.ndirect;
            lc.nnear += run_len[c];
            lc.direct_particles += nd.count;
            c = nd.skip;
        }
    }
    counts[b] = lc;
}

struct ListOut {
    const int64_t* item_off;    // per batch: first item (approximations, then direct sums)
    const int32_t* far_off;
    const int32_t* near_off;
    const int32_t* cluster_slot;
    const int64_t* run_lo;
    const int64_t* run_hi;
    const int32_t* leaf_list;
    const int64_t* leaf_begin;  // per entry of leaf_list
    const int64_t* leaf_count;
    const ListCounts* counts;
    int32_t* far_slot;
    int32_t* near_leaf;
    int64_t* near_begin;
    int64_t* near_count;
    int32_t* item_batch;
    int32_t* item_cluster;
    int32_t* item_kind;
};

__global__ void __launch_bounds__(kListThreads)
fill_lists(int64_t nb, const TravBatch* __restrict__ batches, const TravNode* __restrict__ nodes,
           double theta, int64_t P, ListOut o)
{
    const int64_t b = static_cast<int64_t>(blockIdx.x) * kListThreads + threadIdx.x;
    if (b >= nb)
        return;
    const TravBatch tb = batches[b];
    int64_t ia = o.item_off[b];
    int64_t id = ia + o.counts[b].nfar;
    int64_t f = o.far_off[b];
    int64_t q = o.near_off[b];
    int32_t c = 0;
    while (c >= 0) {
        const TravNode nd = nodes[c];
        const bool geometric = mac_geometric(tb, nd, theta);
        if (geometric && P < nd.count) {
            o.item_batch[ia] = static_cast<int32_t>(b);
            o.item_cluster[ia] = c;
            o.item_kind[ia++] = 0;
            o.far_slot[f++] = o.cluster_slot[c];
            c = nd.skip;
        } else if (!geometric && nd.first_child >= 0) {
            c = nd.first_child;
        } else {
            o.item_batch[id] = static_cast<int32_t>(b);
            o.item_cluster[id] = c;
            o.item_kind[id++] = 1;
            for (int64_t r = o.run_lo[c]; r < o.run_hi[c]; ++r) {
                o.near_leaf[q] = o.leaf_list[r];
                o.near_begin[q] = o.leaf_begin[r];
                o.near_count[q++] = o.leaf_count[r];
            }
            c = nd.skip;
        }
    }
}

}  // namespace

std::string build_lists_device(HostPlan& hp, DeviceLists& out, const DeviceAlloc& alloc,
                               hipStream_t s)
{
    const Tree& S = hp.src;
    const Tree& T = hp.tgt;
    const int64_t nb = static_cast<int64_t>(hp.batch_node.size());
    const int64_t nn = S.nodes();
    out = DeviceLists();
    hp.far_off.assign(nb + 1, 0);
    hp.near_off.assign(nb + 1, 0);
    hp.batch_cost.assign(nb, 0);
    std::vector<uint8_t> used_h(std::max<int64_t>(nn, 1), 0);
    if (nb == 0 || nn == 0) {
        plan_slots(hp, used_h);
        return std::string();
    }
    // node and batch tables
    std::vector<TravNode> nodes(nn);
    std::vector<int32_t> skip(nn, -1);
    for (int64_t p = 0; p < nn; ++p)
        for (int32_t k = 0; k < S.nchild[p]; ++k) {
            const int32_t ch = S.first_child[p] + k;
            skip[ch] = k + 1 < S.nchild[p] ? ch + 1 : skip[p];
        }
    for (int64_t c = 0; c < nn; ++c)
        nodes[c] = {S.center[3 * c], S.center[3 * c + 1], S.center[3 * c + 2], S.radius[c],
                    S.count[c], S.nchild[c] > 0 ? S.first_child[c] : -1, skip[c]};
    std::vector<TravBatch> batches(nb);
    for (int64_t b = 0; b < nb; ++b) {
        const int32_t u = hp.batch_node[b];
        batches[b] = {T.center[3 * u], T.center[3 * u + 1], T.center[3 * u + 2], T.radius[u],
                      T.count[u]};
    }
    std::vector<int32_t> leaf_list;
    std::vector<int64_t> run_lo, run_hi;
    leaf_runs(S, leaf_list, run_lo, run_hi);
    std::vector<int64_t> run_len(nn), leaf_begin(leaf_list.size()), leaf_count(leaf_list.size());
    for (int64_t c = 0; c < nn; ++c)
        run_len[c] = run_hi[c] - run_lo[c];
    for (size_t i = 0; i < leaf_list.size(); ++i) {
        leaf_begin[i] = S.begin[leaf_list[i]];
        leaf_count[i] = S.count[leaf_list[i]];
    }

    Buf<TravNode> nodes_d;
    Buf<TravBatch> batches_d;
    Buf<int64_t> run_len_d, run_lo_d, run_hi_d, leaf_begin_d, leaf_count_d, item_off_d;
    Buf<int32_t> leaf_list_d, far_off_d, near_off_d, slot_d;
    Buf<ListCounts> counts_d;
    Buf<uint8_t> used_d;
    TB_TRY(nodes_d.put(nodes, s));
    TB_TRY(batches_d.put(batches, s));
    TB_TRY(run_len_d.put(run_len, s));
    TB_TRY(counts_d.reserve(nb));
    std::vector<uint8_t> zeros(nn, 0);
    TB_TRY(used_d.put(zeros, s));
    const uint32_t grid = static_cast<uint32_t>((nb + kListThreads - 1) / kListThreads);
    count_lists<<<grid, kListThreads, 0, s>>>(nb, batches_d.p, nodes_d.p, hp.prm.theta, hp.P,
                                          run_len_d.p, counts_d.p, used_d.p);
    TB_TRY(hipGetLastError());
    std::vector<ListCounts> counts(nb);
    TB_TRY(hipMemcpyAsync(counts.data(), counts_d.p, nb * sizeof(ListCounts),
                          hipMemcpyDeviceToHost, s));
    TB_TRY(hipMemcpyAsync(used_h.data(), used_d.p, nn, hipMemcpyDeviceToHost, s));
    TB_TRY(hipStreamSynchronize(s));

    // offsets, costs and statistics (host, per batch)
    std::vector<int64_t> item_off(nb + 1, 0), far_o(nb + 1, 0), near_o(nb + 1, 0);
    for (int64_t b = 0; b < nb; ++b) {
        const ListCounts& lc = counts[b];
        item_off[b + 1] = item_off[b] + lc.nfar + lc.ndirect;
        far_o[b + 1] = far_o[b] + lc.nfar;
        near_o[b + 1] = near_o[b] + lc.nnear;
        const int64_t nbt = batches[b].count;
        hp.batch_cost[b] = lc.nfar * hp.P + lc.direct_particles;
        hp.far_evals += nbt * hp.P * lc.nfar;
        hp.near_evals += nbt * lc.direct_particles;
        hp.approx_pairs += lc.nfar;
        hp.direct_pairs += lc.ndirect;
    }
    if (far_o[nb] > INT32_MAX || near_o[nb] > INT32_MAX)
        return "interaction lists exceed 2^31 entries";
    for (int64_t b = 0; b <= nb; ++b) {
        hp.far_off[b] = static_cast<int32_t>(far_o[b]);
        hp.near_off[b] = static_cast<int32_t>(near_o[b]);
    }
    plan_slots(hp, used_h);
    out.n_items = item_off[nb];

    // device lists, filled in place
    TB_TRY(alloc(reinterpret_cast<void**>(&out.far_slot), far_o[nb] * sizeof(int32_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.near_leaf), near_o[nb] * sizeof(int32_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.near_begin), near_o[nb] * sizeof(int64_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.near_count), near_o[nb] * sizeof(int64_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.item_batch), out.n_items * sizeof(int32_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.item_cluster), out.n_items * sizeof(int32_t)));
    TB_TRY(alloc(reinterpret_cast<void**>(&out.item_kind), out.n_items * sizeof(int32_t)));
    TB_TRY(item_off_d.put(item_off, s));
    TB_TRY(far_off_d.put(hp.far_off, s));
    TB_TRY(near_off_d.put(hp.near_off, s));
    TB_TRY(slot_d.put(hp.cluster_slot, s));
    TB_TRY(run_lo_d.put(run_lo, s));
    TB_TRY(run_hi_d.put(run_hi, s));
    TB_TRY(leaf_list_d.put(leaf_list, s));
    TB_TRY(leaf_begin_d.put(leaf_begin, s));
    TB_TRY(leaf_count_d.put(leaf_count, s));
    ListOut o;
    o.item_off = item_off_d.p;
    o.far_off = far_off_d.p;
    o.near_off = near_off_d.p;
    o.cluster_slot = slot_d.p;
    o.run_lo = run_lo_d.p;
    o.run_hi = run_hi_d.p;
    o.leaf_list = leaf_list_d.p;
    o.leaf_begin = leaf_begin_d.p;
    o.leaf_count = leaf_count_d.p;
    o.counts = counts_d.p;
    o.far_slot = out.far_slot;
    o.near_leaf = out.near_leaf;
    o.near_begin = out.near_begin;
    o.near_count = out.near_count;
    o.item_batch = out.item_batch;
    o.item_cluster = out.item_cluster;
    o.item_kind = out.item_kind;
    fill_lists<<<grid, kListThreads, 0, s>>>(nb, batches_d.p, nodes_d.p, hp.prm.theta, hp.P, o);
    TB_TRY(hipGetLastError());
    // the tables are freed on return: finish first
    TB_TRY(hipStreamSynchronize(s));
    return std::string();
}

}  // namespace bltc
