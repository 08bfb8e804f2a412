// ged_noalloc.hip -- ged_kbest_noalloc (include/ged.h): the batched K-Best
// search of ged_kbest (Alg. 1 for every pair) for callers that cannot
// allocate device memory.  All of its staging -- the pairs, their mapping
// offsets, the work lists and queue counters of the size bins, and the
// workgroup kernel's beam workspace -- lives in `scratch`, one array the
// library holds on every device until the process ends.  The searches are
// the same kernels as ged_kbest's, so the results are identical.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <mutex>

#include "ged.h"
#include "ged_host.h"
#include "ged_internal.h"

using gedh::fail;
using gedh::ok;
using gedk::GraphRec;
using gedk::WorkItem;

namespace {

constexpr size_t kScratchBytes = (size_t)GED_NOALLOC_SCRATCH_BYTES;

// The staging array.  Its name in host code is not a device address: host
// code only ever uses the address hipGetSymbolAddress returns for the
// current device (scratch_on).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {};

// Device address of the current device's copy of `scratch`, looked up once
// per device with that device current.
ged_status scratch_on(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(GED_EUNSUPPORTED, "device %d beyond the library's %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GED_EDEVICE, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = g_scratch[dev];
    return ok();
}

struct Carve {
    size_t off = 0;
    size_t take(size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    }
};

}  // namespace

extern "C" ged_status ged_kbest_noalloc(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs,
                                        int32_t K, int32_t *d_dist, int32_t *d_map, void *stream) {
    // ---- the checks of ged_kbest, on the host, without allocating
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (npairs < 0) return fail(GED_EINVAL, "npairs < 0");
    if (npairs > 0 && !h_pairs) return fail(GED_EINVAL, "pairs is NULL");
    if (npairs > (int64_t)std::numeric_limits<int32_t>::max()) return fail(GED_EUNSUPPORTED, "more than 2^31-1 pairs");
    if (K < 1) return fail(GED_EINVAL, "K must be >= 1 (got %d)", K);
    if (K > GED_MAX_K) return fail(GED_EUNSUPPORTED, "K = %d exceeds %d", K, GED_MAX_K);
    st = gedh::check_device(db);
    if (st != GED_OK) return st;
    const int directed = db->directed ? 1 : 0;
    const int64_t vmax = std::max({(int64_t)costs.vsub, (int64_t)costs.vdel, (int64_t)costs.vins});
    const int64_t emax = std::max({(int64_t)costs.esub, (int64_t)costs.edel, (int64_t)costs.eins});
    int64_t count[gedk::kPairBins] = {0};
    int nmax1[gedk::kPairBins] = {0}, nmax2[gedk::kPairBins] = {0};
    int64_t map_entries = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t s = h_pairs[i].src, d = h_pairs[i].dst;
        if (s < 0 || s >= db->count || d < 0 || d >= db->count)
            return fail(GED_EINVAL, "pair %lld: graph id out of range", (long long)i);
        const GraphRec &g1 = db->h_graphs[(size_t)s];
        const GraphRec &g2 = db->h_graphs[(size_t)d];
        if (directed && std::max(g1.n, g2.n) > GED_DIRECTED_MAX_ORDER)
            return fail(GED_EUNSUPPORTED, "pair %lld: directed graphs of more than %d vertices", (long long)i,
                        GED_DIRECTED_MAX_ORDER);
        if (std::max(g1.n, g2.n) > GED_MAX_VERTICES_BATCH)
            return fail(GED_EUNSUPPORTED, "pair %lld: a graph of %d vertices exceeds the batched search's %d",
                        (long long)i, std::max(g1.n, g2.n), GED_MAX_VERTICES_BATCH);
        if (vmax * ((int64_t)g1.n + g2.n) + emax * ((int64_t)g1.m + g2.m) > (int64_t)std::numeric_limits<int32_t>::max() - 1)
            return fail(GED_EINVAL, "costs may overflow int32 on pair %lld", (long long)i);
        const int b = gedk::pair_bin(g1.n, g2.n, K, directed);
        ++count[b];
        nmax1[b] = std::max(nmax1[b], g1.n);
        nmax2[b] = std::max(nmax2[b], g2.n);
        map_entries += g1.n;
    }
    if (npairs > 0 && !d_dist) return fail(GED_EINVAL, "d_dist is NULL");
    if (map_entries > 0 && !d_map) return fail(GED_EINVAL, "d_map is NULL");
    if (npairs == 0) return ok();

    int dev = 0, cus = 0;
    GED_HIP(hipGetDevice(&dev));
    GED_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    void *base = nullptr;
    st = scratch_on(dev, &base);
    if (st != GED_OK) return st;

    // ---- the scratch's layout: staging, then one workspace share per
    // workgroup-kernel bin
    const int PL = db->planes == 0 ? 0 : (db->planes <= 2 ? 2 : 4);
    Carve cv;
    const size_t o_pairs = cv.take(sizeof(ged_pair) * (size_t)npairs);
    const size_t o_off = cv.take(sizeof(int64_t) * (size_t)(npairs + 1));
    const size_t o_lists = cv.take(sizeof(WorkItem) * (size_t)npairs);
    const size_t o_cnt = cv.take(sizeof(int) * 2 * gedk::kPairBins);   // list fill counters, then queue counters
    gedk::BinBases lb{};
    int64_t at = 0;
    for (int b = 0; b < gedk::kPairBins; ++b) {
        lb.at[b] = at;
        at += count[b];
    }
    gedk::BlockShape shape[gedk::kPairBins];
    size_t stride[gedk::kPairBins] = {0}, o_ws[gedk::kPairBins] = {0};
    int grid[gedk::kPairBins] = {0};
    size_t reserve = 0;   // one workgroup's workspace for every workgroup bin
    for (int b = gedk::kWaveFamilies; b < gedk::kPairBins; ++b) {
        if (count[b] == 0) continue;
        const int threads = count[b] < 2 * (int64_t)cus ? gedk::kBlockThreadsWide : gedk::kBlockThreads;
        shape[b] = gedk::BlockShape{gedk::bin_words(b), PL, gedk::block_slot_stride(K, threads), nmax1[b], nmax2[b],
                                    threads, directed};
        stride[b] = gedk::block_workspace_bytes(shape[b]);
        reserve += (stride[b] + 255) & ~(size_t)255;
    }
    if (cv.off + reserve > kScratchBytes)
        return fail(GED_EUNSUPPORTED, "the batch needs %zu bytes of staging, more than the %zu-byte scratch",
                    cv.off + reserve, kScratchBytes);
    for (int b = 0; b < gedk::kPairBins; ++b) {
        if (count[b] == 0) continue;
        int per_cu = 0;
        hipError_t e = b < gedk::kWaveFamilies ? gedk::wave_family_max_resident(b + 1, PL, K, 0, &per_cu, directed)
                             : gedk::block_max_resident(shape[b], &per_cu);
        if (e != hipSuccess || per_cu <= 0)
            return fail(GED_EDEVICE, "occupancy query failed: %s", hipGetErrorString(e));
        int64_t g = std::min<int64_t>(count[b], (int64_t)per_cu * cus);
        if (b >= gedk::kWaveFamilies) {
            // as many workgroups as the scratch holds, keeping one for each later bin
            // (the reservation guarantees room for one, rounded up to 256 bytes)
            reserve -= (stride[b] + 255) & ~(size_t)255;
            const size_t avail = kScratchBytes - cv.off - reserve;
            g = std::min<int64_t>(g, (int64_t)(avail / stride[b]));
            while (g > 1 && ((stride[b] * (size_t)g + 255) & ~(size_t)255) > avail) --g;
            g = std::max<int64_t>(g, 1);
            o_ws[b] = cv.take(stride[b] * (size_t)g);
        }
        grid[b] = (int)std::max<int64_t>(1, g);
    }

    // ---- stage, classify, search; every step on `stream`
    const hipStream_t s = static_cast<hipStream_t>(stream);
    char *sp = static_cast<char *>(base);
    ged_pair *pairs = reinterpret_cast<ged_pair *>(sp + o_pairs);
    int64_t *moff = reinterpret_cast<int64_t *>(sp + o_off);
    WorkItem *lists = reinterpret_cast<WorkItem *>(sp + o_lists);
    int *cnt = reinterpret_cast<int *>(sp + o_cnt);
    GED_HIP(hipMemcpyAsync(pairs, h_pairs, sizeof(ged_pair) * (size_t)npairs, hipMemcpyHostToDevice, s));
    GED_HIP(gedk::launch_fill_zero(cnt, 2 * gedk::kPairBins, s));
    GED_HIP(gedk::launch_map_offsets(db->d_graphs, db->count, pairs, npairs, moff, s));
    GED_HIP(gedk::launch_classify_pairs(db->d_graphs, pairs, npairs, moff, K, directed, lists, lb, cnt, s));
    const gedk::DbView view{db->d_graphs, db->d_adj, db->d_vlab, db->planes};
    const gedk::Costs c{costs.vsub, costs.vdel, costs.vins, costs.esub, costs.edel, costs.eins};
    const gedk::Outputs out{d_dist, d_map, nullptr};
    int *queue = cnt + gedk::kPairBins;
    for (int b = 0; b < gedk::kPairBins; ++b) {
        if (count[b] == 0) continue;
        const WorkItem *work = lists + lb.at[b];
        if (b < gedk::kWaveFamilies) {
            GED_HIP(gedk::launch_wave_family(b + 1, PL, view, view, work, (int)count[b], queue + b, c, K, 0, out,
                                             grid[b], s, directed));
        } else {
            GED_HIP(gedk::launch_block(shape[b], view, view, work, (int)count[b], queue + b, c, K, 0, sp + o_ws[b],
                                       stride[b], out, grid[b], s));
        }
    }
    GED_HIP(hipStreamSynchronize(s));
    return ok();
}
