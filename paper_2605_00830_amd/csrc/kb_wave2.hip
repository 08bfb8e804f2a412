// kb_wave2.hip -- the two-word wavefront kernel (kb_wave2.h) with one beam
// slot per lane (K <= 64), and the launch and occupancy functions of the
// kernel, which take the two-slot instantiations of kb_wave2_k128.hip for
// 64 < K <= 128 and those of kb_wave2_src128.hip for sources of 65..128
// vertices.
#include "kb_wave2.h"

namespace gedk {
namespace {

bool small_costs2(const Costs &c) {
    const int32_t lim = 1 << 22;
    return c.vsub < lim && c.vdel < lim && c.vins < lim && c.esub < lim && c.edel < lim && c.eins < lim;
}

// family 2: sources of up to 64 vertices (directed: 32); 3: undirected
// sources of up to 128
const void *select_wave2(int family, int K, int PL, bool small, bool complete, bool dir) {
    if (K < 1 || K > kWave2MaxK) return nullptr;
    if (family == 3) return dir ? nullptr : select_wave2_wide_source(K <= kWaveMaxK ? 1 : 2, PL, small, complete);
    if (family != 2) return nullptr;
    if (K <= kWaveMaxK) return w2::select_wave2_s<1>(PL, small, complete, dir);
    return select_wave2_two_slots(PL, small, complete, dir);
}

}  // namespace

hipError_t wave2_max_resident_dir(int family, int PL, int K, int last_complete, int directed, int *blocks_per_cu) {
    const void *k = select_wave2(family, K, PL, true, last_complete != 0, directed != 0);
    const void *k2 = select_wave2(family, K, PL, false, last_complete != 0, directed != 0);
    if (!k || !k2) return hipErrorInvalidValue;
    int x = 0, y = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&x, k, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&y, k2, 64, 0);
    *blocks_per_cu = x < y ? x : y;
    return e;
}

hipError_t wave2_max_resident(int PL, int K, int last_complete, int *blocks_per_cu) {
    return wave2_max_resident_dir(2, PL, K, last_complete, 0, blocks_per_cu);
}

hipError_t launch_wave2_dir(int family, int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork,
                            int *queue, Costs c, int K, int last_complete, int directed, Outputs out, int grid,
                            hipStream_t stream) {
    const void *k = select_wave2(family, K, PL, small_costs2(c), last_complete != 0, directed != 0);
    if (!k || grid <= 0) return hipErrorInvalidValue;
    w2::Wave2Args a;
    a.src = src;
    a.dst = dst;
    a.work = work;
    a.nwork = nwork;
    a.queue = queue;
    a.c = c;
    a.K = K;
    a.out = out;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, stream);
}

hipError_t launch_wave2(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue,
                        Costs c, int K, int last_complete, Outputs out, int grid, hipStream_t stream) {
    return launch_wave2_dir(2, PL, src, dst, work, nwork, queue, c, K, last_complete, 0, out, grid, stream);
}

}  // namespace gedk
