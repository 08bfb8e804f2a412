// ged_wide.cpp -- the single-pair large-K search of the C ABI
// (include/ged.h): argument checks, the workspace, and the launch sequence
// of kb_wide.hip.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <limits>
#include <new>

#include "ged.h"
#include "ged_host.h"
#include "ged_internal.h"

using gedh::fail;
using gedh::ok;

struct ged_wide {
    ged_db *db = nullptr;
    int64_t src = 0, dst = 0;
    int32_t K = 0;
    int last_complete = 0;
    int cus = 0;
    void *d_ws = nullptr;
    size_t ws_bytes = 0;
};

extern "C" {

ged_status ged_wide_create(ged_db *db, int64_t src, int64_t dst, int32_t K, ged_wide **out) {
    return ged_wide_create_ex(db, src, dst, K, nullptr, out);
}

ged_status ged_wide_create_ex(ged_db *db, int64_t src, int64_t dst, int32_t K, const ged_plan_options *options,
                              ged_wide **out) {
    if (!out) return fail(GED_EINVAL, "out is NULL");
    const int last = options ? options->last_level : GED_LAST_SELECT;
    if (last != GED_LAST_SELECT && last != GED_LAST_COMPLETE) return fail(GED_EINVAL, "unknown last level %d", last);
    if (options && options->method != GED_METHOD_TREE)
        return fail(GED_EINVAL, "the single-pair search runs the tree method only");
    *out = nullptr;
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (src < 0 || src >= db->count || dst < 0 || dst >= db->count)
        return fail(GED_EINVAL, "graph id out of range");
    if (db->directed) return fail(GED_EUNSUPPORTED, "the single-pair search takes undirected graphs only");
    if (K < 1 || K > GED_MAX_K_WIDE) return fail(GED_EINVAL, "K must be in 1..%d (got %d)", GED_MAX_K_WIDE, K);
    ged_status st = gedh::check_device(db);
    if (st != GED_OK) return st;
    const gedk::GraphRec &g1 = db->h_graphs[(size_t)src];
    const gedk::GraphRec &g2 = db->h_graphs[(size_t)dst];
    ged_wide *w = new (std::nothrow) ged_wide;
    if (!w) return fail(GED_ENOMEM, "host allocation failed");
    w->db = db;
    w->src = src;
    w->dst = dst;
    w->K = K;
    w->last_complete = last == GED_LAST_COMPLETE ? 1 : 0;
    w->ws_bytes = gedk::wide_workspace_bytes(g1.n, g2.n, g2.w, db->planes, K);
    hipError_t e = hipDeviceGetAttribute(&w->cus, hipDeviceAttributeMultiprocessorCount, db->device);
    if (e != hipSuccess) {
        delete w;
        return fail(GED_EDEVICE, "device query failed: %s", hipGetErrorString(e));
    }
    e = hipMalloc(&w->d_ws, w->ws_bytes);
    if (e != hipSuccess) {
        delete w;
        return fail(GED_ENOMEM, "workspace of %zu bytes: %s", w->ws_bytes, hipGetErrorString(e));
    }
    *out = w;
    return ok();
}

ged_status ged_wide_bytes(const ged_wide *w, int64_t *bytes) {
    if (!w || !bytes) return fail(GED_EINVAL, "NULL argument");
    *bytes = (int64_t)w->ws_bytes;
    return ok();
}

ged_status ged_wide_run(ged_wide *w, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                        void *stream) {
    if (!w) return fail(GED_EINVAL, "handle is NULL");
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    st = gedh::check_device(w->db);
    if (st != GED_OK) return st;
    const gedk::GraphRec &g1 = w->db->h_graphs[(size_t)w->src];
    const gedk::GraphRec &g2 = w->db->h_graphs[(size_t)w->dst];
    if (!d_dist) return fail(GED_EINVAL, "d_dist is NULL");
    if (g1.n > 0 && !d_map) return fail(GED_EINVAL, "d_map is NULL");
    const int64_t vmax = std::max({(int64_t)costs.vsub, (int64_t)costs.vdel, (int64_t)costs.vins});
    const int64_t emax = std::max({(int64_t)costs.esub, (int64_t)costs.edel, (int64_t)costs.eins});
    const int64_t bound = vmax * ((int64_t)g1.n + g2.n) + emax * ((int64_t)g1.m + g2.m);
    if (bound > (int64_t)std::numeric_limits<int32_t>::max() - 1)
        return fail(GED_EINVAL, "costs may overflow int32 on this pair (bound %lld)", (long long)bound);
    const ged_db *db = w->db;
    const gedk::DbView view{db->d_graphs, db->d_adj, db->d_vlab, db->planes};
    const gedk::Costs c{costs.vsub, costs.vdel, costs.vins, costs.esub, costs.edel, costs.eins};
    GED_HIP(gedk::launch_wide(view, view, g1, g2, c, w->K, w->last_complete, w->d_ws, w->ws_bytes, d_dist, d_map,
                              d_cand, w->cus, static_cast<hipStream_t>(stream)));
    return ok();
}

ged_status ged_wide_destroy(ged_wide *w) {
    if (!w) return ok();
    if (w->d_ws) (void)hipFree(w->d_ws);
    delete w;
    return ok();
}

}  // extern "C"
