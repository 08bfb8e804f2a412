// Types shared by the host side of the library and its HIP kernels, and the
// wavefront kernels' entry points: everything kb_wave.hip and kb_wave2.hip
// compile against (nothing else of the library's internals).
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gedk {

// Graph record in the device database.  The adjacency pool holds, from
// word `adj` on: n rows of w 32-bit words (bit x of row v set iff {v,x} is
// an edge), then `planes` blocks of the same shape, block b holding bit b
// of the database-wide edge-label code at each edge position.
struct GraphRec {
    int32_t n;
    int32_t m;
    int32_t w;       // ceil(n / 32)
    int32_t pad;
    int64_t adj;     // word offset into the adjacency pool
    int64_t vlab;    // offset into the vertex-label pool
};

// A set of packed graphs: a database, or the staged queries of a serving
// batch.  Work items index graphs of a source view (g1) and a target view
// (g2); both use the same edge-label coding.
struct DbView {
    const GraphRec *graphs;
    const uint32_t *adj;
    const int32_t *vlab;
    int32_t planes;  // edge-label bit planes in this database (0..4)
};

// One pair of a batch, in schedule order.
struct WorkItem {
    int32_t src;     // g1 id
    int32_t dst;     // g2 id
    int32_t out;     // index of the pair in the caller's order
    int32_t pad;
    int64_t map_off; // first mapping entry of the pair in d_map
};

// Next item of a persistent launch for a workgroup that has finished one:
// items [0, grid) are the workgroups' own first items, the others come from
// the launch's queue counter.  Every workgroup pulls until it gets an item
// >= nwork, so a run takes exactly the values 0 .. nwork - 1 from the counter,
// and the workgroup that takes the last one puts it back to 0 for the next
// run (the counter starts at 0 when it is allocated): no reset between runs.
// A grid of at least nwork workgroups has no item to draw and leaves the
// counter alone: device-scope atomics on one address are serialised at the
// memory side, and a grid of thousands of short items would wait on them.
__device__ __forceinline__ int pull_item(int *queue, int nwork) {
    if ((int)gridDim.x >= nwork) return nwork;
    const int v = atomicAdd(queue, 1);
    if (v == nwork - 1) atomicExch(queue, 0);
    return (int)gridDim.x + v;
}

struct Costs {
    int32_t vsub, vdel, vins, esub, edel, eins;
};

struct Outputs {
    int32_t *dist;
    int32_t *map;
    int64_t *cand;   // may be null
};

// Wavefront-per-pair kernel family: n1, n2 <= 32 and K <= 64; the beam lives
// in registers (one slot per lane) and LDS.
constexpr int kWaveMaxN = 32;
constexpr int kWaveMaxK = 64;

hipError_t wave_max_resident(int PL, int last_complete, int *blocks_per_cu);
hipError_t launch_wave(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue, Costs c,
                       int K, int last_complete, Outputs out, int grid, hipStream_t stream);

// The same scheme for n1, n2 <= 64 (two-word vertex sets, children scored
// into bytes), K <= 128 (two beam slots per lane above 64).
constexpr int kWave2MaxN = 64;
constexpr int kWave2MaxK = 128;

hipError_t wave2_max_resident(int PL, int K, int last_complete, int *blocks_per_cu);
hipError_t launch_wave2(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue,
                        Costs c, int K, int last_complete, Outputs out, int grid, hipStream_t stream);

}  // namespace gedk
