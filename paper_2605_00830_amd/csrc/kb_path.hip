// kb_path.hip -- edit-path output: the explicit edit operations a vertex
// mapping induces (Sec. 2.2-2.4), one workgroup per pair.
//
// For mapping phi of g1 into g2 (-1 = deleted), the operations, in order:
//   1. per g1 vertex v ascending: substitution (v, phi(v)) or deletion of v;
//   2. per g2 vertex u ascending outside the image: insertion of u;
//   3. per g1 edge (a < b) in lexicographic order: substitution by
//      (phi(a), phi(b)) when both ends are mapped onto a g2 edge, else
//      deletion;
//   4. per g2 edge (x < y) in lexicographic order that is no g1 edge's image:
//      insertion.
// Each carries its cost (0 for a substitution that keeps the label); the
// costs sum to the mapping's edit cost.  Thread t owns vertices 2t and 2t+1
// of each phase; a block exclusive scan of their operation counts places
// every operation.
// Directed graphs: phases 3 and 4 walk every arc (x, y) of the out-rows in
// lexicographic order, a substituted arc's image being (phi(x), phi(y)).
#include <hip/hip_runtime.h>

#include "ged.h"
#include "ged_internal.h"
#include "wave_common.h"

namespace gedk {
namespace {

using namespace wv;

constexpr int kPathThreads = 512;
static_assert(2 * kPathThreads >= GED_MAX_VERTICES, "two vertices per thread");

struct PathArgs {
    DbView view;
    const WorkItem *work;   // out = pair index, map_off = its first mapping entry
    const int64_t *cap_off; // first operation slot of each pair
    int nwork;
    Costs c;
    const int32_t *map;
    ged_edit_op *ops;
    int32_t *count;         // operations written per pair; -1 for an invalid mapping
    int directed;           // rows hold out-arcs; every arc is listed
};

__device__ __forceinline__ uint32_t row_word(const uint32_t *A, int w, int x, int y) {
    return A[(size_t)x * w + (y >> 5)];
}
__device__ __forceinline__ bool has_edge(const uint32_t *A, int w, int x, int y) {
    return (row_word(A, w, x, y) >> (y & 31)) & 1u;
}
__device__ __forceinline__ int edge_code(const uint32_t *A, int n, int w, int P, int x, int y) {
    int code = 0;
    for (int pl = 0; pl < P; ++pl) code |= (int)has_edge(A + (size_t)(1 + pl) * n * w, w, x, y) << pl;
    return code;
}

// the part of row word wd of vertex x the phases list: the bits above x
// (undirected: each edge once), or all of them (directed: rows hold out-arcs)
__device__ __forceinline__ uint32_t listed(uint32_t r, int wd, int x, int directed) {
    if (directed) return r;
    return r & (wd * 32 + 31 <= x ? 0u : (wd * 32 > x ? ~0u : ~((2u << (x & 31)) - 1u)));
}

// exclusive prefix of (v0 + v1) over the block's threads; *total = the sum
__device__ int block_excl_scan(int v, int *s_wave, int *total) {
    const int lane = threadIdx.x & 63, wv_ = threadIdx.x >> 6;
    const int ex = wave_excl_scan(v);
    if (lane == 63) s_wave[wv_] = ex + v;
    __syncthreads();
    int before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kPathThreads / 64; ++k) {
        const int t = s_wave[k];
        before += k < wv_ ? t : 0;
        all += t;
    }
    __syncthreads();
    *total = all;
    return before + ex;
}

__global__ __launch_bounds__(kPathThreads) void kb_path_kernel(PathArgs a) {
    __shared__ int s_phi[GED_MAX_VERTICES];
    __shared__ int s_pre[GED_MAX_VERTICES];
    __shared__ int s_wave[kPathThreads / 64];
    __shared__ int s_bad;
    const int t = threadIdx.x;
    const int P = a.view.planes;

    for (int item = blockIdx.x; item < a.nwork; item += gridDim.x) {
        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.view.graphs[wi.src];
        const GraphRec g2 = a.view.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n, w1 = g1.w, w2 = g2.w;
        const uint32_t *A1 = a.view.adj + g1.adj;
        const uint32_t *A2 = a.view.adj + g2.adj;
        const int32_t *vl1 = a.view.vlab + g1.vlab;
        const int32_t *vl2 = a.view.vlab + g2.vlab;
        ged_edit_op *out = a.ops + a.cap_off[wi.out];

        // ---------------- the mapping, checked: in range and injective
        if (t == 0) s_bad = 0;
        for (int u = t; u < n2; u += kPathThreads) s_pre[u] = -1;
        __syncthreads();
        for (int v = t; v < n1; v += kPathThreads) {
            const int f = a.map[wi.map_off + v];
            const bool ok = f >= -1 && f < n2;
            s_phi[v] = ok ? f : -1;
            if (!ok) s_bad = 1;
            else if (f >= 0 && atomicCAS(&s_pre[f], -1, v) != -1) s_bad = 1;
        }
        __syncthreads();
        if (s_bad) {
            if (t == 0) a.count[wi.out] = -1;
            __syncthreads();
            continue;
        }

        const int x0 = 2 * t, x1 = 2 * t + 1;   // this thread's vertices in every phase
        int base = 0;

        // ---------------- 1. g1 vertices: substitution or deletion
        for (int v = t; v < n1; v += kPathThreads) {
            const int f = s_phi[v];
            ged_edit_op op;
            op.kind = f >= 0 ? GED_OP_VSUB : GED_OP_VDEL;
            op.a = v;
            op.b = f;
            op.c = -1;
            op.d = -1;
            op.cost = f >= 0 ? (vl1[v] != vl2[f] ? a.c.vsub : 0) : a.c.vdel;
            out[v] = op;
        }
        base = n1;

        // ---------------- 2. g2 vertices outside the image: insertion
        {
            const int f0 = (x0 < n2 && s_pre[x0] < 0) ? 1 : 0;
            const int f1 = (x1 < n2 && s_pre[x1] < 0) ? 1 : 0;
            int nins = 0;
            const int pos = base + block_excl_scan(f0 + f1, s_wave, &nins);
            ged_edit_op op;
            op.kind = GED_OP_VINS;
            op.a = -1;
            op.c = -1;
            op.d = -1;
            op.cost = a.c.vins;
            if (f0) {
                op.b = x0;
                out[pos] = op;
            }
            if (f1) {
                op.b = x1;
                out[pos + f0] = op;
            }
            base += nins;
        }

        // ---------------- 3. g1 edges (a < b): substitution or deletion
        {
            int c0 = 0, c1 = 0;
            for (int wd = 0; wd < w1; ++wd) {
                if (x0 < n1) c0 += __popc(listed(A1[(size_t)x0 * w1 + wd], wd, x0, a.directed));
                if (x1 < n1) c1 += __popc(listed(A1[(size_t)x1 * w1 + wd], wd, x1, a.directed));
            }
            int m1 = 0;
            int pos = base + block_excl_scan(c0 + c1, s_wave, &m1);
            for (int h = 0; h < 2; ++h) {
                const int x = h == 0 ? x0 : x1;
                if (x >= n1) continue;
                const int fx = s_phi[x];
                for (int wd = 0; wd < w1; ++wd) {
                    uint32_t r = listed(A1[(size_t)x * w1 + wd], wd, x, a.directed);
                    while (r) {
                        const int y = 32 * wd + __builtin_ctz(r);
                        r &= r - 1u;
                        const int fy = s_phi[y];
                        ged_edit_op op;
                        op.a = x;
                        op.b = y;
                        if (fx >= 0 && fy >= 0 && has_edge(A2, w2, fx, fy)) {
                            op.kind = GED_OP_ESUB;
                            op.c = a.directed ? fx : min(fx, fy);
                            op.d = a.directed ? fy : max(fx, fy);
                            op.cost = edge_code(A1, n1, w1, P, x, y) != edge_code(A2, n2, w2, P, fx, fy) ? a.c.esub : 0;
                        } else {
                            op.kind = GED_OP_EDEL;
                            op.c = -1;
                            op.d = -1;
                            op.cost = a.c.edel;
                        }
                        out[pos++] = op;
                    }
                }
            }
            base += m1;
        }

        // ---------------- 4. g2 edges (x < y) that no g1 edge maps onto: insertion
        {
            auto covered = [&](int x, int y) -> bool {
                const int px = s_pre[x], py = s_pre[y];
                return px >= 0 && py >= 0 && has_edge(A1, w1, px, py);
            };
            int c0 = 0, c1 = 0;
            for (int h = 0; h < 2; ++h) {
                const int x = h == 0 ? x0 : x1;
                if (x >= n2) continue;
                int cnt = 0;
                for (int wd = 0; wd < w2; ++wd) {
                    uint32_t r = listed(A2[(size_t)x * w2 + wd], wd, x, a.directed);
                    while (r) {
                        const int y = 32 * wd + __builtin_ctz(r);
                        r &= r - 1u;
                        cnt += covered(x, y) ? 0 : 1;
                    }
                }
                if (h == 0) c0 = cnt;
                else c1 = cnt;
            }
            int nie = 0;
            int pos = base + block_excl_scan(c0 + c1, s_wave, &nie);
            for (int h = 0; h < 2; ++h) {
                const int x = h == 0 ? x0 : x1;
                if (x >= n2) continue;
                for (int wd = 0; wd < w2; ++wd) {
                    uint32_t r = listed(A2[(size_t)x * w2 + wd], wd, x, a.directed);
                    while (r) {
                        const int y = 32 * wd + __builtin_ctz(r);
                        r &= r - 1u;
                        if (covered(x, y)) continue;
                        ged_edit_op op;
                        op.kind = GED_OP_EINS;
                        op.a = -1;
                        op.b = -1;
                        op.c = x;
                        op.d = y;
                        op.cost = a.c.eins;
                        out[pos++] = op;
                    }
                }
            }
            base += nie;
        }
        if (t == 0) a.count[wi.out] = base;
        __syncthreads();
    }
}

}  // namespace

hipError_t launch_path(const DbView &view, const WorkItem *work, const int64_t *cap_off, int nwork, Costs c,
                       const int32_t *map, ged_edit_op *ops, int32_t *count, int directed, int grid,
                       hipStream_t stream) {
    if (grid <= 0 || nwork <= 0) return nwork == 0 ? hipSuccess : hipErrorInvalidValue;
    PathArgs a;
    a.view = view;
    a.work = work;
    a.cap_off = cap_off;
    a.nwork = nwork;
    a.c = c;
    a.map = map;
    a.ops = ops;
    a.count = count;
    a.directed = directed;
    void *args[] = {&a};
    return hipLaunchKernel(reinterpret_cast<const void *>(&kb_path_kernel), dim3(grid), dim3(kPathThreads), args,
                           0, stream);
}

}  // namespace gedk
