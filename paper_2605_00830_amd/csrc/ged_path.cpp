// ged_path.cpp -- edit-path output of the C ABI (include/ged.h): validates
// the pairs, stages the work list and capacity offsets on the device, runs
// kb_path_kernel and reports mappings the kernel rejected.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <vector>

#include "ged.h"
#include "ged_host.h"
#include "ged_internal.h"

using gedh::fail;
using gedh::ok;

namespace {

ged_status check_pairs(const ged_db *db, const ged_pair *h_pairs, int64_t npairs) {
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (npairs < 0) return fail(GED_EINVAL, "npairs < 0");
    if (npairs > 0 && !h_pairs) return fail(GED_EINVAL, "pairs is NULL");
    if (npairs > (int64_t)std::numeric_limits<int32_t>::max()) return fail(GED_EUNSUPPORTED, "more than 2^31-1 pairs");
    for (int64_t i = 0; i < npairs; ++i)
        if (h_pairs[i].src < 0 || h_pairs[i].src >= db->count || h_pairs[i].dst < 0 || h_pairs[i].dst >= db->count)
            return fail(GED_EINVAL, "pair %lld: graph id out of range", (long long)i);
    return ok();
}

}  // namespace

extern "C" {

ged_status ged_edit_path_capacity(const ged_db *db, const ged_pair *h_pairs, int64_t npairs, int64_t *h_offsets) {
    ged_status st = check_pairs(db, h_pairs, npairs);
    if (st != GED_OK) return st;
    if (!h_offsets) return fail(GED_EINVAL, "h_offsets is NULL");
    int64_t off = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        h_offsets[i] = off;
        const gedk::GraphRec &g1 = db->h_graphs[(size_t)h_pairs[i].src];
        const gedk::GraphRec &g2 = db->h_graphs[(size_t)h_pairs[i].dst];
        off += (int64_t)g1.n + g2.n + g1.m + g2.m;
    }
    h_offsets[npairs] = off;
    return ok();
}

ged_status ged_edit_path(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, const int32_t *d_map,
                         ged_edit_op *d_ops, int32_t *d_count, void *stream) {
    ged_status st = check_pairs(db, h_pairs, npairs);
    if (st != GED_OK) return st;
    st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    if (npairs == 0) return ok();
    if (!d_count || !d_ops) return fail(GED_EINVAL, "NULL output buffer");
    st = gedh::check_device(db);
    if (st != GED_OK) return st;
    std::vector<int64_t> cap((size_t)npairs + 1);
    st = ged_edit_path_capacity(db, h_pairs, npairs, cap.data());
    if (st != GED_OK) return st;
    std::vector<gedk::WorkItem> work((size_t)npairs);
    int64_t moff = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        work[(size_t)i].src = (int32_t)h_pairs[i].src;
        work[(size_t)i].dst = (int32_t)h_pairs[i].dst;
        work[(size_t)i].out = (int32_t)i;
        work[(size_t)i].pad = 0;
        work[(size_t)i].map_off = moff;
        moff += db->h_graphs[(size_t)h_pairs[i].src].n;
    }
    if (moff > 0 && !d_map) return fail(GED_EINVAL, "d_map is NULL");

    hipStream_t s = static_cast<hipStream_t>(stream);
    gedk::WorkItem *d_work = nullptr;
    int64_t *d_cap = nullptr;
    hipError_t e = hipMalloc((void **)&d_work, sizeof(gedk::WorkItem) * (size_t)npairs);
    if (e == hipSuccess) e = hipMalloc((void **)&d_cap, sizeof(int64_t) * (size_t)npairs);
    if (e != hipSuccess) {
        if (d_work) (void)hipFree(d_work);
        return fail(GED_ENOMEM, "edit-path staging allocation failed: %s", hipGetErrorString(e));
    }
    e = hipMemcpyAsync(d_work, work.data(), sizeof(gedk::WorkItem) * (size_t)npairs, hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(d_cap, cap.data(), sizeof(int64_t) * (size_t)npairs, hipMemcpyHostToDevice, s);
    int cus = 0, dev = 0;
    if (e == hipSuccess) e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e == hipSuccess) {
        const int grid = (int)std::min<int64_t>(npairs, (int64_t)cus * 8);
        const gedk::DbView view{db->d_graphs, db->d_adj, db->d_vlab, db->planes};
        const gedk::Costs c{costs.vsub, costs.vdel, costs.vins, costs.esub, costs.edel, costs.eins};
        e = gedk::launch_path(view, d_work, d_cap, (int)npairs, c, d_map, d_ops, d_count, db->directed ? 1 : 0, grid,
                              s);
    }
    std::vector<int32_t> h_count((size_t)npairs);
    if (e == hipSuccess)
        e = hipMemcpyAsync(h_count.data(), d_count, sizeof(int32_t) * (size_t)npairs, hipMemcpyDeviceToHost, s);
    const hipError_t es = hipStreamSynchronize(s);   // also before freeing after a failed enqueue
    if (e == hipSuccess) e = es;
    (void)hipFree(d_work);
    (void)hipFree(d_cap);
    if (e != hipSuccess) return fail(GED_EDEVICE, "edit-path run failed: %s", hipGetErrorString(e));
    for (int64_t i = 0; i < npairs; ++i)
        if (h_count[(size_t)i] < 0)
            return fail(GED_EINVAL, "pair %lld: mapping not injective or out of range", (long long)i);
    return ok();
}

}  // extern "C"
