// kb_aux.hip -- small kernels around the search: where each pair's mapping
// starts in the output (exclusive prefix sum of the source orders), the
// per-pair statuses of a plan's set-aside pairs, the copy of database graphs
// into a serving arena, and the work lists of the allocation-free batched
// call.  None of them does any step of the search itself.
#include <hip/hip_runtime.h>

#include "ged_internal.h"

namespace gedk {
namespace {

constexpr int ST = 1024;   // threads of the single-workgroup scan
constexpr int SI = 4;      // pairs per thread and pass

// Inclusive prefix sum of v over the workgroup (Hillis-Steele in LDS).
__device__ int64_t block_incl_scan64(int64_t v, int64_t *s) {
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int d = 1; d < ST; d <<= 1) {
        const int64_t add = t >= d ? s[t - d] : 0;
        __syncthreads();
        s[t] += add;
        __syncthreads();
    }
    const int64_t r = s[t];
    __syncthreads();
    return r;
}

// off[p] = sum of n(src) over pairs q < p, in caller order; off[np] = the
// total.  A pair whose source id is outside [0, count) contributes 0.
__global__ __launch_bounds__(ST) void map_offsets_kernel(const GraphRec *graphs, int64_t count, const ged_pair *pairs,
                                                         int64_t np, int64_t *off) {
    __shared__ int64_t s[ST];
    int64_t carry = 0;
    for (int64_t base = 0; base < np; base += (int64_t)ST * SI) {
        int64_t v[SI];
        int64_t sum = 0;
#pragma unroll
        for (int q = 0; q < SI; ++q) {
            const int64_t idx = base + (int64_t)threadIdx.x * SI + q;
            int64_t n = 0;
            if (idx < np) {
                const int64_t src = pairs[idx].src;
                if (src >= 0 && src < count) n = graphs[src].n;
            }
            v[q] = n;
            sum += n;
        }
        const int64_t incl = block_incl_scan64(sum, s);
        int64_t run = carry + incl - sum;
#pragma unroll
        for (int q = 0; q < SI; ++q) {
            const int64_t idx = base + (int64_t)threadIdx.x * SI + q;
            if (idx < np) off[idx] = run;
            run += v[q];
        }
        // the last thread's inclusive sum is the pass total
        if (threadIdx.x == ST - 1) s[0] = incl;
        __syncthreads();
        carry += s[0];
        __syncthreads();
    }
    if (threadIdx.x == 0) off[np] = carry;
}

// status_out[p] = status[p] for every pair; each set-aside pair (item.out =
// its index, item.src = its mapping entries, item.map_off = the first)
// gets distance -1, mapping entries -1 and 0 children.
__global__ void pair_status_kernel(const int32_t *status, int64_t np, int32_t *status_out, const WorkItem *aside,
                                   int naside, int32_t *dist, int32_t *map, int64_t *cand) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (status_out)
        for (int64_t p = t0; p < np; p += stride) status_out[p] = status[p];
    for (int64_t k = t0; k < naside; k += stride) {
        const WorkItem w = aside[k];
        dist[w.out] = -1;
        if (cand) cand[w.out] = 0;
        for (int j = 0; j < w.src; ++j) map[w.map_off + j] = -1;
    }
}

// One workgroup per item (grid-stride): graph words and vertex labels from
// the database's pools into the arena's.
__global__ __launch_bounds__(256) void gather_graphs_kernel(const GatherItem *items, int nitems, const uint32_t *src_adj,
                                                            uint32_t *dst_adj, const int32_t *src_vlab,
                                                            int32_t *dst_vlab) {
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const GatherItem g = items[it];
        for (int64_t k = threadIdx.x; k < g.words; k += blockDim.x) dst_adj[g.dst_adj + k] = src_adj[g.src_adj + k];
        for (int64_t k = threadIdx.x; k < g.nv; k += blockDim.x) dst_vlab[g.dst_vlab + k] = src_vlab[g.src_vlab + k];
    }
}

// Work lists of the allocation-free call: pair p goes to bin
// pair_bin(n1, n2, K, directed) at the next free position of that bin's
// list (lists[base[bin] ..]); counters[bin] starts at 0.  The host counted
// the same bins with the same function, so every list is filled exactly.
__global__ void classify_pairs_kernel(const GraphRec *graphs, const ged_pair *pairs, int64_t np, const int64_t *off,
                                      int K, int directed, WorkItem *lists, BinBases base, int *counters) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < np; p += stride) {
        const int32_t s = (int32_t)pairs[p].src, d = (int32_t)pairs[p].dst;
        const int b = pair_bin(graphs[s].n, graphs[d].n, K, directed);
        const int slot = atomicAdd(&counters[b], 1);
        WorkItem w;
        w.src = s;
        w.dst = d;
        w.out = (int32_t)p;
        w.pad = 0;
        w.map_off = off[p];
        lists[base.at[b] + slot] = w;
    }
}

int grid_for(int64_t n, int threads) {
    const int64_t g = (n + threads - 1) / threads;
    return (int)(g < 1 ? 1 : (g > 4096 ? 4096 : g));
}

}  // namespace

hipError_t launch_map_offsets(const GraphRec *graphs, int64_t count, const ged_pair *pairs, int64_t np, int64_t *off,
                              hipStream_t stream) {
    hipLaunchKernelGGL(map_offsets_kernel, dim3(1), dim3(ST), 0, stream, graphs, count, pairs, np, off);
    return hipGetLastError();
}

hipError_t launch_pair_status(const int32_t *status, int64_t np, int32_t *status_out, const WorkItem *aside,
                              int naside, int32_t *dist, int32_t *map, int64_t *cand, hipStream_t stream) {
    if ((np <= 0 || !status_out) && naside <= 0) return hipSuccess;
    const int64_t n = (status_out && np > naside) ? np : naside;
    hipLaunchKernelGGL(pair_status_kernel, dim3(grid_for(n, 256)), dim3(256), 0, stream, status, np, status_out,
                       aside, naside, dist, map, cand);
    return hipGetLastError();
}

hipError_t launch_gather_graphs(const GatherItem *items, int nitems, const uint32_t *src_adj, uint32_t *dst_adj,
                                const int32_t *src_vlab, int32_t *dst_vlab, hipStream_t stream) {
    if (nitems <= 0) return hipSuccess;
    const int grid = nitems < 1024 ? nitems : 1024;
    hipLaunchKernelGGL(gather_graphs_kernel, dim3(grid), dim3(256), 0, stream, items, nitems, src_adj, dst_adj,
                       src_vlab, dst_vlab);
    return hipGetLastError();
}

hipError_t launch_classify_pairs(const GraphRec *graphs, const ged_pair *pairs, int64_t np, const int64_t *off, int K,
                                 int directed, WorkItem *lists, const BinBases &base, int *counters,
                                 hipStream_t stream) {
    if (np <= 0) return hipSuccess;
    hipLaunchKernelGGL(classify_pairs_kernel, dim3(grid_for(np, 256)), dim3(256), 0, stream, graphs, pairs, np, off, K,
                       directed, lists, base, counters);
    return hipGetLastError();
}

}  // namespace gedk
