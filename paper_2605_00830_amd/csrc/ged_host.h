// Host-side internals shared by the C ABI's translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>
#include <vector>

#include "ged.h"
#include "ged_internal.h"

namespace gedh {

// Record `fmt` as the calling thread's last error and return `s`.
ged_status fail(ged_status s, const char *fmt, ...);
inline ged_status ok() { return GED_OK; }

#define GED_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return ::gedh::fail(GED_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

ged_status check_costs(const ged_costs &c);

// Shape checks of one host graph (index g for messages), host-only.
ged_status check_graph_shape(const ged_graph &G, int64_t g, bool directed = false);
// Words of the packed adjacency (rows plus label planes; twice that for a
// directed graph, whose in-arc rows and planes follow) of an n-vertex graph.
int64_t packed_words(int n, int planes, bool directed = false);
// Append graph G's packed rows, label planes and vertex labels to adj/vlab
// and describe them in R (offsets into adj/vlab).  `labels` is the sorted
// table of edge labels whose index is the label code; a label missing from
// it, a vertex out of range, a self-loop or a repeated edge is GED_EINVAL.
ged_status pack_graph(const ged_graph &G, int64_t g, const std::vector<int32_t> &labels, int planes,
                      std::vector<uint32_t> &adj, std::vector<int32_t> &vlab, gedk::GraphRec &R,
                      bool directed = false);

// Order the first `grid` items of a longest-first work list (the pairs the
// workgroups of a persistent launch take statically, workgroup b taking item
// b) so that the execution units share the work evenly.  A grid that fills
// the device evenly lands workgroup b on unit b mod `slots` (SIMDs for
// one-wave workgroups, CUs for workgroups of four waves), so unit u gets
// items u, u + slots, u + 2 slots, ...; dealing rounds of `slots` items in
// alternating directions gives each unit long and short pairs alike instead
// of the longest of every round.  Items past `grid` keep the longest-first
// order of the dynamic queue.
template <class T>
void deal_alternating(std::vector<T> &items, int64_t grid, int64_t slots) {
    const int64_t n = std::min<int64_t>((int64_t)items.size(), grid);
    if (slots <= 0) return;
    for (int64_t r = 1; r * slots < n; r += 2) {
        const int64_t lo = r * slots, hi = std::min(n, lo + slots);
        std::reverse(items.begin() + lo, items.begin() + hi);
    }
}

}  // namespace gedh

struct ged_db {
    int device = 0;
    int64_t count = 0;
    int32_t planes = 0;
    bool directed = false;          // arcs; rows then in-arc rows per graph
    std::vector<int32_t> elabels;   // sorted distinct edge labels; index = label code
    std::vector<gedk::GraphRec> h_graphs;
    gedk::GraphRec *d_graphs = nullptr;
    uint32_t *d_adj = nullptr;
    int32_t *d_vlab = nullptr;
    int64_t bytes = 0;
};

namespace gedh {
ged_status check_device(const ged_db *db);
}  // namespace gedh
