// Internal declarations of the library: kernel entry points and shapes.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

#include "ged.h"
#include "ged_types.h"

namespace gedk {

// Block-per-pair kernel family: any n <= 512, K <= GED_MAX_K; beam state and
// the candidate matrix live in a per-block global workspace.  Workgroups of
// 256 threads, or 512 for bins too small to fill the device (two waves per
// SIMD on one pair instead of one).
constexpr int kBlockThreads = 256;
constexpr int kBlockThreadsWide = 512;
constexpr int kBlockThreadsXL = 1024;   // unlabelled 8- and 16-word rows, one pair per CU

struct BlockShape {
    int W;       // words per target row the instantiation handles (1,2,4,8,16)
    int PL;      // label planes the instantiation handles (0,2,4)
    int KS;      // slot stride: block_slot_stride(K, BT)
    int nmax1;   // largest source order in the bin
    int nmax2;   // largest target order in the bin
    int BT;      // threads per workgroup: kBlockThreads or kBlockThreadsWide
    int directed = 0;   // directed database: W covers an out-row and an in-row
};

// Slot stride of the workgroup kernel for beam width K and `threads` per
// workgroup (64, 128, 256, or K rounded up to a multiple of `threads`):
// BlockShape::KS must equal it.
int block_slot_stride(int K, int threads);
size_t block_workspace_bytes(const BlockShape &s);
// An instantiation exists for this shape (every shape at 256 and 512 threads).
bool block_shape_supported(const BlockShape &s);
hipError_t block_max_resident(const BlockShape &s, int *blocks_per_cu);
// last_complete: at the last level every child is completed (Sec. 4.4.1) and
// only the least total is kept, instead of the K of least partial distance
// (the same argument of every launch below).
hipError_t launch_block(const BlockShape &s, const DbView &src, const DbView &dst, const WorkItem *work, int nwork,
                        int *queue, Costs c, int K, int last_complete, void *workspace, size_t ws_stride,
                        Outputs out, int grid, hipStream_t stream);
hipError_t launch_fill_zero(int *p, int count, hipStream_t stream);

// Bipartite K-best-assignment bound, a workgroup of nwav (1 or 4) waves per
// pair (kb_bip.hip): n1 + n2 <= 256, K <= 256.  A launch's columns per lane
// (cpl = ceil((n1 + n2) / 64), 1..4), queue slots per lane (ceil(K / 64): 1,
// 2 or 4) and nwav pick the instantiation; `ws` holds grid x
// bip_workgroup_bytes(cpl, K) (a pool of K + 64 cpl queue nodes: potentials,
// assignment, fixed rows, forbidden pairs).
constexpr int kBipMaxM = 256;
constexpr int kBipMaxK = 256;
inline int bip_cols_per_lane(int m) { return m <= 64 ? 1 : (m + 63) / 64; }
inline int bip_queue_words(int K) { return K <= 64 ? 1 : (K <= 128 ? 2 : 4); }
inline size_t bip_node_bytes(int cpl, int K) {
    const size_t raw = 10 * 64 * (size_t)cpl + 8 * (size_t)cpl + 16 + 4 * (size_t)K;
    return (raw + 255) / 256 * 256;
}
inline size_t bip_workgroup_bytes(int cpl, int K) { return ((size_t)K + 64 * (size_t)cpl) * bip_node_bytes(cpl, K); }
hipError_t bip_max_resident(int PL, int cpl, int K, int nwav, int *blocks_per_cu);
hipError_t launch_bip(int PL, int cpl, int nwav, const DbView &src, const DbView &dst, const WorkItem *work,
                      int nwork, int *queue, Costs c, int K, void *ws, Outputs out, int grid, hipStream_t stream);

// Edit-path output (kb_path.hip): one workgroup per pair; cap_off[out] is
// the pair's first operation slot; directed: the view's rows hold out-arcs.
hipError_t launch_path(const DbView &view, const WorkItem *work, const int64_t *cap_off, int nwork, Costs c,
                       const int32_t *map, ged_edit_op *ops, int32_t *count, int directed, int grid,
                       hipStream_t stream);

// Whole-device search of one pair at large K (kb_wide.hip).
constexpr int kWideMaxK = GED_MAX_K_WIDE;

size_t wide_workspace_bytes(int n1, int n2, int w2, int planes, int K);
// Enqueue the search of pair (g1 of src, g2 of dst); `ws` holds at least
// wide_workspace_bytes bytes; dist[0], map[0..n1), cand[0] (may be null) are
// device outputs; `cus` sizes the grids.
hipError_t launch_wide(const DbView &src, const DbView &dst, const GraphRec &g1, const GraphRec &g2, Costs c, int K,
                       int last_complete, void *ws, size_t ws_bytes, int32_t *dist, int32_t *map, int64_t *cand,
                       int cus, hipStream_t stream);

// Wavefront family that fits a pair: 1 (n1, n2 <= 32 and K <= 64), 2 (else
// n1, n2 <= 64 and K <= 128), 3 (n2 <= 64, 64 < n1 <= 128 and K <= 128: the
// two-word kernel with a 128-vertex mapping), 0 none (K > 128 or a larger
// graph).
constexpr int kWaveFamilies = 3;
constexpr int kWave3MaxN1 = 128;
__host__ __device__ inline int wave_words_for(int n1, int n2, int K) {
    if (K > kWave2MaxK || n2 > kWave2MaxN) return 0;
    if (n1 > kWave2MaxN) return n1 <= kWave3MaxN1 ? 3 : 0;
    const int n = n1 > n2 ? n1 : n2;
    return (n <= kWaveMaxN && K <= kWaveMaxK) ? 1 : 2;
}
// Directed pairs of up to 32 vertices on the two-word wavefront kernel
// (kb_wave2.hip, DIR instantiations): a row word of out-arcs and one of
// in-arcs per vertex.
// family: 2 (sources of up to 64 vertices; directed: 32) or 3 (undirected
// sources of up to 128).
hipError_t wave2_max_resident_dir(int family, int PL, int K, int last_complete, int directed, int *blocks_per_cu);
hipError_t launch_wave2_dir(int family, int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork,
                            int *queue, Costs c, int K, int last_complete, int directed, Outputs out, int grid,
                            hipStream_t stream);
// Wavefront family of a directed pair: 2 when both orders are <= 32 and K <= 128.
__host__ __device__ inline int wave_words_for_directed(int n1, int n2, int K) {
    return (K <= kWave2MaxK && n1 <= kWaveMaxN && n2 <= kWaveMaxN) ? 2 : 0;
}

inline hipError_t wave_family_max_resident(int family, int PL, int K, int last_complete, int *blocks_per_cu,
                                           int directed = 0) {
    if (directed) return wave2_max_resident_dir(2, PL, K, last_complete, 1, blocks_per_cu);
    return family == 1 ? wave_max_resident(PL, last_complete, blocks_per_cu)
                       : wave2_max_resident_dir(family, PL, K, last_complete, 0, blocks_per_cu);
}
inline hipError_t launch_wave_family(int family, int PL, const DbView &src, const DbView &dst, const WorkItem *work,
                                     int nwork, int *queue, Costs c, int K, int last_complete, Outputs out, int grid,
                                     hipStream_t stream, int directed = 0) {
    if (directed)
        return launch_wave2_dir(2, PL, src, dst, work, nwork, queue, c, K, last_complete, 1, out, grid, stream);
    return family == 1 ? launch_wave(PL, src, dst, work, nwork, queue, c, K, last_complete, out, grid, stream)
                       : launch_wave2_dir(family, PL, src, dst, work, nwork, queue, c, K, last_complete, 0, out, grid,
                                          stream);
}

// Size bins of the default schedule of the tree search: 0 / 1 / 2 = the
// wavefront families 1 / 2 / 3 (n <= 32 and K <= 64 / the rest of n <= 64
// and K <= 128 / sources of 65..128 vertices against targets of up to 64;
// a directed pair of up to 32 vertices takes 1), 3 + log2(W) = the workgroup
// kernel whose rows have W words (target words rounded up to a power of two,
// doubled for a directed database's out and in rows).  The same function
// classifies pairs on the host and on the device.
constexpr int kPairBins = kWaveFamilies + 5;
__host__ __device__ inline int pair_bin(int n1, int n2, int K, int directed) {
    const int ww = directed ? wave_words_for_directed(n1, n2, K) : wave_words_for(n1, n2, K);
    if (ww > 0) return ww - 1;
    const int w2 = n2 > 32 ? (n2 + 31) / 32 : 1;
    int W = 1;
    while (W < w2) W <<= 1;
    if (directed) W <<= 1;
    int lg = 0;
    while ((1 << lg) < W) ++lg;
    return kWaveFamilies + lg;
}
// Row words of workgroup-kernel bin b (kWaveFamilies .. kPairBins - 1).
__host__ __device__ inline int bin_words(int b) { return 1 << (b - kWaveFamilies); }

// Start of each bin's work list in one array of work items.
struct BinBases {
    int64_t at[kPairBins];
};

// Copy of one database graph into a serving arena (word and label offsets
// into the two pools).
struct GatherItem {
    int64_t src_adj, dst_adj, words;
    int64_t src_vlab, dst_vlab, nv;
};

// kb_aux.hip.
// off[p] (p < np) = sum of n(src) over the pairs before p; off[np] = total.
hipError_t launch_map_offsets(const GraphRec *graphs, int64_t count, const ged_pair *pairs, int64_t np, int64_t *off,
                              hipStream_t stream);
// status_out[p] = status[p] (status_out may be null); set-aside pairs (out,
// src = mapping entries, map_off) get dist -1, mapping -1, cand 0.
hipError_t launch_pair_status(const int32_t *status, int64_t np, int32_t *status_out, const WorkItem *aside,
                              int naside, int32_t *dist, int32_t *map, int64_t *cand, hipStream_t stream);
hipError_t launch_gather_graphs(const GatherItem *items, int nitems, const uint32_t *src_adj, uint32_t *dst_adj,
                                const int32_t *src_vlab, int32_t *dst_vlab, hipStream_t stream);
// Work items of pairs[0..np) into lists[base.at[pair_bin(..)] + k] (counters
// zeroed beforehand; pair ids already validated).
hipError_t launch_classify_pairs(const GraphRec *graphs, const ged_pair *pairs, int64_t np, const int64_t *off, int K,
                                 int directed, WorkItem *lists, const BinBases &base, int *counters,
                                 hipStream_t stream);

}  // namespace gedk
