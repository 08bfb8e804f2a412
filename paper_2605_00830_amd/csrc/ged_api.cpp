// ged_api.cpp -- host side of the C ABI declared in include/ged.h.
//
// Validates every input on the host, packs graphs into the device database
// (adjacency bitsets plus edge-label bit planes), builds size-binned work
// lists and launches the kernels.  No computation of the search happens on
// the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ged.h"
#include "ged_internal.h"

using gedk::GraphRec;
using gedk::WorkItem;

namespace {

thread_local std::string g_last_error;

ged_status fail(ged_status s, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

ged_status ok() { return GED_OK; }

#define GED_HIP(call)                                                                     \
    do {                                                                                  \
        hipError_t e_ = (call);                                                           \
        if (e_ != hipSuccess)                                                             \
            return fail(GED_EDEVICE, "%s failed: %s", #call, hipGetErrorString(e_));      \
    } while (0)

int words_for(int n) { return (n + 31) / 32; }

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct ged_db {
    int device = 0;
    int64_t count = 0;
    int32_t planes = 0;
    std::vector<GraphRec> h_graphs;
    GraphRec *d_graphs = nullptr;
    uint32_t *d_adj = nullptr;
    int32_t *d_vlab = nullptr;
    int64_t bytes = 0;
};

namespace {

struct Bin {
    bool wave = false;           // wavefront-per-pair kernel (else workgroup-per-pair)
    gedk::BlockShape shape{};
    std::vector<WorkItem> h_work;
    WorkItem *d_work = nullptr;
    int *d_queue = nullptr;      // [1 + nwork]: batched counter, then one per pair
    void *d_ws = nullptr;
    size_t ws_stride = 0;
    int grid = 0;
};

}  // namespace

struct ged_plan {
    ged_db *db = nullptr;
    int64_t npairs = 0;
    int32_t K = 0;
    int64_t map_entries = 0;
    std::vector<int64_t> pair_n;   // n1 + n2 per pair, for the overflow bound
    std::vector<int64_t> pair_m;   // m1 + m2 per pair
    std::vector<Bin> bins;
    bool timing = false;
    bool timed_run = false;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    int64_t launches = 0;
};

namespace {

void free_plan(ged_plan *p) {
    if (!p) return;
    for (Bin &b : p->bins) {
        if (b.d_work) (void)hipFree(b.d_work);
        if (b.d_queue) (void)hipFree(b.d_queue);
        if (b.d_ws) (void)hipFree(b.d_ws);
    }
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    if (p->ev_stop) (void)hipEventDestroy(p->ev_stop);
    delete p;
}

void free_db(ged_db *db) {
    if (!db) return;
    if (db->d_graphs) (void)hipFree(db->d_graphs);
    if (db->d_adj) (void)hipFree(db->d_adj);
    if (db->d_vlab) (void)hipFree(db->d_vlab);
    delete db;
}

ged_status check_device(const ged_db *db) {
    int dev = -1;
    GED_HIP(hipGetDevice(&dev));
    if (dev != db->device)
        return fail(GED_EINVAL, "current HIP device %d differs from the database's device %d", dev,
                    db->device);
    return ok();
}

ged_status check_costs(const ged_costs &c) {
    const int32_t v[6] = {c.vsub, c.vdel, c.vins, c.esub, c.edel, c.eins};
    for (int k = 0; k < 6; ++k)
        if (v[k] < 0) return fail(GED_EINVAL, "costs must be >= 0 (cost %d is %d)", k, v[k]);
    return ok();
}

// Every partial edit distance and every completed cost of a pair is at most
// max_vertex_cost * (n1 + n2) + max_edge_cost * (m1 + m2); keep it below the
// kernels' sentinel INT32_MAX.
ged_status check_overflow(const ged_plan *p, const ged_costs &c) {
    const int64_t vmax = std::max({(int64_t)c.vsub, (int64_t)c.vdel, (int64_t)c.vins});
    const int64_t emax = std::max({(int64_t)c.esub, (int64_t)c.edel, (int64_t)c.eins});
    const int64_t lim = (int64_t)std::numeric_limits<int32_t>::max() - 1;
    for (int64_t i = 0; i < p->npairs; ++i) {
        const int64_t bound = vmax * p->pair_n[i] + emax * p->pair_m[i];
        if (bound > lim)
            return fail(GED_EINVAL, "costs may overflow int32 on pair %lld (bound %lld)",
                        (long long)i, (long long)bound);
    }
    return ok();
}

}  // namespace

extern "C" {

int32_t ged_abi_version(void) { return GED_ABI_VERSION; }

const char *ged_last_error(void) { return g_last_error.c_str(); }

const char *ged_status_name(int32_t s) {
    switch (s) {
        case GED_OK: return "GED_OK";
        case GED_EINVAL: return "GED_EINVAL";
        case GED_ENOMEM: return "GED_ENOMEM";
        case GED_EUNSUPPORTED: return "GED_EUNSUPPORTED";
        case GED_EDEVICE: return "GED_EDEVICE";
        case GED_EBUSY: return "GED_EBUSY";
        case GED_ETIMEOUT: return "GED_ETIMEOUT";
        case GED_ECANCELED: return "GED_ECANCELED";
        default: return "GED_UNKNOWN";
    }
}

ged_status ged_db_create(const ged_graph *graphs, int64_t count, ged_db **out) {
    if (!out) return fail(GED_EINVAL, "out is NULL");
    *out = nullptr;
    if (count < 0) return fail(GED_EINVAL, "count < 0");
    if (count > 0 && !graphs) return fail(GED_EINVAL, "graphs is NULL");
    if (count > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GED_EUNSUPPORTED, "more than 2^31-1 graphs");

    // pass 1: validate shapes, collect the distinct edge labels
    std::vector<int32_t> labels;
    int64_t total_words = 0, total_v = 0;
    for (int64_t g = 0; g < count; ++g) {
        const ged_graph &G = graphs[g];
        if (G.n < 0 || G.m < 0) return fail(GED_EINVAL, "graph %lld: negative n or m", (long long)g);
        if (G.n > GED_MAX_VERTICES)
            return fail(GED_EUNSUPPORTED, "graph %lld: n = %d exceeds %d", (long long)g, G.n,
                        GED_MAX_VERTICES);
        if (G.n > 0 && !G.vlabel) return fail(GED_EINVAL, "graph %lld: vlabel is NULL", (long long)g);
        if (G.m > 0 && (!G.eu || !G.ev))
            return fail(GED_EINVAL, "graph %lld: edge arrays are NULL", (long long)g);
        if ((int64_t)G.m > (int64_t)G.n * (G.n - 1) / 2)
            return fail(GED_EINVAL, "graph %lld: more edges than a simple graph allows", (long long)g);
        if (G.elabel)
            for (int k = 0; k < G.m; ++k) labels.push_back(G.elabel[k]);
        else if (G.m > 0)
            labels.push_back(0);
        total_v += G.n;
    }
    std::sort(labels.begin(), labels.end());
    labels.erase(std::unique(labels.begin(), labels.end()), labels.end());
    if ((int)labels.size() > GED_MAX_EDGE_LABELS)
        return fail(GED_EUNSUPPORTED, "%zu distinct edge labels exceed %d", labels.size(),
                    GED_MAX_EDGE_LABELS);
    int planes = 0;
    while ((1 << planes) < (int)labels.size()) ++planes;

    ged_db *db = new (std::nothrow) ged_db;
    if (!db) return fail(GED_ENOMEM, "host allocation failed");
    db->count = count;
    db->planes = planes;
    db->h_graphs.resize((size_t)count);
    for (int64_t g = 0; g < count; ++g) {
        const int w = words_for(graphs[g].n);
        total_words += (int64_t)graphs[g].n * w * (1 + planes);
    }

    // pass 2: pack rows and planes, rejecting self-loops, bad ids and repeats
    std::vector<uint32_t> adj((size_t)std::max<int64_t>(total_words, 1), 0u);
    std::vector<int32_t> vlab((size_t)std::max<int64_t>(total_v, 1), 0);
    int64_t wofs = 0, vofs = 0;
    for (int64_t g = 0; g < count; ++g) {
        const ged_graph &G = graphs[g];
        const int n = G.n, w = words_for(n);
        GraphRec &R = db->h_graphs[(size_t)g];
        R.n = n;
        R.m = G.m;
        R.w = w;
        R.pad = 0;
        R.adj = wofs;
        R.vlab = vofs;
        uint32_t *rows = adj.data() + wofs;
        const size_t plane = (size_t)n * w;
        for (int k = 0; k < G.m; ++k) {
            const int a = G.eu[k], b = G.ev[k];
            if (a < 0 || b < 0 || a >= n || b >= n) {
                free_db(db);
                return fail(GED_EINVAL, "graph %lld: edge %d has a vertex out of range", (long long)g, k);
            }
            if (a == b) {
                free_db(db);
                return fail(GED_EINVAL, "graph %lld: edge %d is a self-loop", (long long)g, k);
            }
            if (rows[(size_t)a * w + (b >> 5)] & (1u << (b & 31))) {
                free_db(db);
                return fail(GED_EINVAL, "graph %lld: edge %d repeats {%d,%d}", (long long)g, k, a, b);
            }
            rows[(size_t)a * w + (b >> 5)] |= 1u << (b & 31);
            rows[(size_t)b * w + (a >> 5)] |= 1u << (a & 31);
            const int32_t lab = G.elabel ? G.elabel[k] : 0;
            const int code = (int)(std::lower_bound(labels.begin(), labels.end(), lab) - labels.begin());
            for (int p = 0; p < planes; ++p) {
                if ((code >> p) & 1) {
                    uint32_t *pl = rows + (size_t)(1 + p) * plane;
                    pl[(size_t)a * w + (b >> 5)] |= 1u << (b & 31);
                    pl[(size_t)b * w + (a >> 5)] |= 1u << (a & 31);
                }
            }
        }
        for (int v = 0; v < n; ++v) vlab[(size_t)(vofs + v)] = G.vlabel[v];
        wofs += (int64_t)plane * (1 + planes);
        vofs += n;
    }

    // every check above is host-only; the device is touched from here on
    {
        hipError_t e = hipGetDevice(&db->device);
        if (e != hipSuccess) {
            free_db(db);
            return fail(GED_EDEVICE, "hipGetDevice failed: %s", hipGetErrorString(e));
        }
    }
    const size_t gbytes = sizeof(GraphRec) * (size_t)std::max<int64_t>(count, 1);
    const size_t abytes = sizeof(uint32_t) * adj.size();
    const size_t vbytes = sizeof(int32_t) * vlab.size();
    hipError_t e = hipMalloc((void **)&db->d_graphs, gbytes);
    if (e == hipSuccess) e = hipMalloc((void **)&db->d_adj, abytes);
    if (e == hipSuccess) e = hipMalloc((void **)&db->d_vlab, vbytes);
    if (e != hipSuccess) {
        free_db(db);
        return fail(GED_ENOMEM, "device allocation of the database failed: %s", hipGetErrorString(e));
    }
    if (count > 0) e = hipMemcpy(db->d_graphs, db->h_graphs.data(), sizeof(GraphRec) * (size_t)count,
                                 hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db->d_adj, adj.data(), abytes, hipMemcpyHostToDevice);
    if (e == hipSuccess) e = hipMemcpy(db->d_vlab, vlab.data(), vbytes, hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        free_db(db);
        return fail(GED_EDEVICE, "upload of the database failed: %s", hipGetErrorString(e));
    }
    db->bytes = (int64_t)(gbytes + abytes + vbytes);
    *out = db;
    return ok();
}

ged_status ged_db_destroy(ged_db *db) {
    free_db(db);
    return ok();
}

ged_status ged_db_count(const ged_db *db, int64_t *count) {
    if (!db || !count) return fail(GED_EINVAL, "NULL argument");
    *count = db->count;
    return ok();
}

ged_status ged_db_device_bytes(const ged_db *db, int64_t *bytes) {
    if (!db || !bytes) return fail(GED_EINVAL, "NULL argument");
    *bytes = db->bytes;
    return ok();
}

ged_status ged_db_order(const ged_db *db, int64_t id, int32_t *n) {
    if (!db || !n) return fail(GED_EINVAL, "NULL argument");
    if (id < 0 || id >= db->count) return fail(GED_EINVAL, "graph id %lld out of range", (long long)id);
    *n = db->h_graphs[(size_t)id].n;
    return ok();
}

ged_status ged_plan_create(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K,
                           ged_plan **out) {
    return ged_plan_create_ex(db, h_pairs, npairs, K, nullptr, out);
}

ged_status ged_plan_create_ex(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K,
                              const ged_plan_options *options, ged_plan **out) {
    ged_plan_options opt{GED_SCHED_AUTO, 0};
    if (options) opt = *options;
    if (opt.schedule != GED_SCHED_AUTO && opt.schedule != GED_SCHED_BLOCK)
        return fail(GED_EINVAL, "unknown schedule %d", opt.schedule);
    if (opt.groups_per_cu < 0) return fail(GED_EINVAL, "groups_per_cu < 0");
    if (!out) return fail(GED_EINVAL, "out is NULL");
    *out = nullptr;
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (npairs < 0) return fail(GED_EINVAL, "npairs < 0");
    if (npairs > 0 && !h_pairs) return fail(GED_EINVAL, "pairs is NULL");
    if (npairs > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GED_EUNSUPPORTED, "more than 2^31-1 pairs");
    if (K < 1) return fail(GED_EINVAL, "K must be >= 1 (got %d)", K);
    if (K > GED_MAX_K) return fail(GED_EUNSUPPORTED, "K = %d exceeds %d", K, GED_MAX_K);
    ged_status st = check_device(db);
    if (st != GED_OK) return st;

    ged_plan *p = new (std::nothrow) ged_plan;
    if (!p) return fail(GED_ENOMEM, "host allocation failed");
    p->db = db;
    p->npairs = npairs;
    p->K = K;
    p->pair_n.resize((size_t)npairs);
    p->pair_m.resize((size_t)npairs);

    // bins keyed by (target row words rounded up to a power of two, planes)
    const int PL = db->planes == 0 ? 0 : (db->planes <= 2 ? 2 : 4);
    std::map<int, Bin> bins;
    int64_t off = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t s = h_pairs[i].src, d = h_pairs[i].dst;
        if (s < 0 || s >= db->count || d < 0 || d >= db->count) {
            free_plan(p);
            return fail(GED_EINVAL, "pair %lld: graph id out of range", (long long)i);
        }
        const GraphRec &g1 = db->h_graphs[(size_t)s];
        const GraphRec &g2 = db->h_graphs[(size_t)d];
        p->pair_n[(size_t)i] = (int64_t)g1.n + g2.n;
        p->pair_m[(size_t)i] = (int64_t)g1.m + g2.m;
        const bool wave = opt.schedule == GED_SCHED_AUTO && g1.n <= gedk::kWaveMaxN &&
                          g2.n <= gedk::kWaveMaxN && K <= gedk::kWaveMaxK;
        const int W = pow2_at_least(std::max(1, g2.w));
        Bin &b = bins[wave ? 0 : W];
        b.wave = wave;
        b.shape.W = W;
        b.shape.PL = PL;
        b.shape.nmax1 = std::max(b.shape.nmax1, g1.n);
        b.shape.nmax2 = std::max(b.shape.nmax2, g2.n);
        WorkItem wi;
        wi.src = (int32_t)s;
        wi.dst = (int32_t)d;
        wi.out = (int32_t)i;
        wi.pad = 0;
        wi.map_off = off;
        b.h_work.push_back(wi);
        off += g1.n;
    }
    p->map_entries = off;

    int device = 0, cus = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        free_plan(p);
        return fail(GED_EDEVICE, "device query failed: %s", hipGetErrorString(e));
    }

    for (auto &kv : bins) {
        Bin b = kv.second;
        kv.second.h_work.clear();
        // longest first: work grows with n1 * (n2 + 1)
        std::stable_sort(b.h_work.begin(), b.h_work.end(), [&](const WorkItem &x, const WorkItem &y) {
            const int64_t cx = (int64_t)db->h_graphs[x.src].n * (db->h_graphs[x.dst].n + 1);
            const int64_t cy = (int64_t)db->h_graphs[y.src].n * (db->h_graphs[y.dst].n + 1);
            return cx > cy;
        });
        b.shape.KS = (K + gedk::kBlockThreads - 1) / gedk::kBlockThreads * gedk::kBlockThreads;
        int per_cu = 0;
        e = b.wave ? gedk::wave_max_resident(b.shape.PL, &per_cu) : gedk::block_max_resident(b.shape, &per_cu);
        if (e != hipSuccess || per_cu <= 0) {
            free_plan(p);
            return fail(GED_EDEVICE, "occupancy query failed: %s", hipGetErrorString(e));
        }
        if (opt.groups_per_cu > 0) per_cu = std::min(per_cu, opt.groups_per_cu);
        const int64_t nwork = (int64_t)b.h_work.size();
        b.grid = (int)std::min<int64_t>(nwork, (int64_t)per_cu * cus);
        b.ws_stride = b.wave ? 0 : gedk::block_workspace_bytes(b.shape);
        e = hipMalloc((void **)&b.d_work, sizeof(WorkItem) * (size_t)nwork);
        if (e == hipSuccess) e = hipMalloc((void **)&b.d_queue, sizeof(int) * (size_t)(nwork + 1));
        if (e == hipSuccess && !b.wave) e = hipMalloc(&b.d_ws, b.ws_stride * (size_t)b.grid);
        if (e == hipSuccess)
            e = hipMemcpy(b.d_work, b.h_work.data(), sizeof(WorkItem) * (size_t)nwork, hipMemcpyHostToDevice);
        p->bins.push_back(b);
        if (e != hipSuccess) {
            free_plan(p);
            return fail(GED_ENOMEM, "plan allocation failed: %s", hipGetErrorString(e));
        }
    }
    *out = p;
    return ok();
}

ged_status ged_plan_map_size(const ged_plan *plan, int64_t *entries) {
    if (!plan || !entries) return fail(GED_EINVAL, "NULL argument");
    *entries = plan->map_entries;
    return ok();
}

static ged_status plan_run(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                           int64_t *d_cand, void *stream, bool perpair) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    ged_status st = check_costs(costs);
    if (st != GED_OK) return st;
    if (plan->npairs > 0 && !d_dist) return fail(GED_EINVAL, "d_dist is NULL");
    if (plan->map_entries > 0 && !d_map) return fail(GED_EINVAL, "d_map is NULL");
    st = check_overflow(plan, costs);
    if (st != GED_OK) return st;
    st = check_device(plan->db);
    if (st != GED_OK) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const gedk::DbView view{plan->db->d_graphs, plan->db->d_adj, plan->db->d_vlab, plan->db->planes};
    const gedk::Costs c{costs.vsub, costs.vdel, costs.vins, costs.esub, costs.edel, costs.eins};
    const gedk::Outputs o{d_dist, d_map, d_cand};
    for (Bin &b : plan->bins) GED_HIP(gedk::launch_fill_zero(b.d_queue, (int)b.h_work.size() + 1, s));
    plan->timed_run = false;
    plan->launches = 0;
    if (plan->timing) GED_HIP(hipEventRecord(plan->ev_start, s));
    for (Bin &b : plan->bins) {
        const int nwork = (int)b.h_work.size();
        plan->launches += perpair ? nwork : 1;
        if (b.wave) {
            if (!perpair) {
                GED_HIP(gedk::launch_wave(b.shape.PL, view, b.d_work, nwork, b.d_queue, c, plan->K, o,
                                          b.grid, s));
            } else {
                for (int i = 0; i < nwork; ++i)
                    GED_HIP(gedk::launch_wave(b.shape.PL, view, b.d_work + i, 1, b.d_queue + 1 + i, c,
                                              plan->K, o, 1, s));
            }
        } else if (!perpair) {
            GED_HIP(gedk::launch_block(b.shape, view, b.d_work, nwork, b.d_queue, c, plan->K, b.d_ws,
                                       b.ws_stride, o, b.grid, s));
        } else {
            for (int i = 0; i < nwork; ++i)
                GED_HIP(gedk::launch_block(b.shape, view, b.d_work + i, 1, b.d_queue + 1 + i, c,
                                           plan->K, b.d_ws, b.ws_stride, o, 1, s));
        }
    }
    if (plan->timing) {
        GED_HIP(hipEventRecord(plan->ev_stop, s));
        plan->timed_run = true;
    }
    return ok();
}

ged_status ged_plan_set_timing(ged_plan *plan, int32_t enable) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    if (enable && !plan->ev_start) {
        GED_HIP(hipEventCreate(&plan->ev_start));
        GED_HIP(hipEventCreate(&plan->ev_stop));
    }
    plan->timing = enable != 0;
    plan->timed_run = false;
    return ok();
}

ged_status ged_plan_kernel_ms(ged_plan *plan, float *ms) {
    if (!plan || !ms) return fail(GED_EINVAL, "NULL argument");
    if (!plan->timing || !plan->timed_run) return fail(GED_EINVAL, "no timed run recorded");
    GED_HIP(hipEventElapsedTime(ms, plan->ev_start, plan->ev_stop));
    return ok();
}

ged_status ged_plan_bin_count(const ged_plan *plan, int32_t *count) {
    if (!plan || !count) return fail(GED_EINVAL, "NULL argument");
    *count = (int32_t)plan->bins.size();
    return ok();
}

ged_status ged_plan_bin_info(const ged_plan *plan, int32_t index, int32_t *kernel, int64_t *npairs,
                             int32_t *grid, int32_t *words) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    if (index < 0 || index >= (int32_t)plan->bins.size()) return fail(GED_EINVAL, "bin %d out of range", index);
    const Bin &b = plan->bins[(size_t)index];
    if (kernel) *kernel = b.wave ? GED_KERNEL_WAVE : GED_KERNEL_BLOCK;
    if (npairs) *npairs = (int64_t)b.h_work.size();
    if (grid) *grid = b.grid;
    if (words) *words = b.wave ? 1 : b.shape.W;
    return ok();
}

ged_status ged_plan_kernel_launches(const ged_plan *plan, int64_t *launches) {
    if (!plan || !launches) return fail(GED_EINVAL, "NULL argument");
    *launches = plan->launches;
    return ok();
}

ged_status ged_plan_run(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                        int64_t *d_cand, void *stream) {
    return plan_run(plan, costs, d_dist, d_map, d_cand, stream, false);
}

ged_status ged_plan_run_perpair(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                                int64_t *d_cand, void *stream) {
    return plan_run(plan, costs, d_dist, d_map, d_cand, stream, true);
}

ged_status ged_plan_destroy(ged_plan *plan) {
    free_plan(plan);
    return ok();
}

static ged_status oneshot(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs,
                          int32_t K, int32_t *d_dist, int32_t *d_map, void *stream, bool perpair) {
    ged_status st = check_costs(costs);
    if (st != GED_OK) return st;
    ged_plan *p = nullptr;
    st = ged_plan_create(db, h_pairs, npairs, K, &p);
    if (st != GED_OK) return st;
    st = plan_run(p, costs, d_dist, d_map, nullptr, stream, perpair);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_plan(p);
    if (st != GED_OK) return st;
    if (e != hipSuccess) return fail(GED_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return ok();
}

ged_status ged_kbest(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                     int32_t *d_dist, int32_t *d_map, void *stream) {
    return oneshot(db, h_pairs, npairs, costs, K, d_dist, d_map, stream, false);
}

ged_status ged_kbest_perpair(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs,
                             int32_t K, int32_t *d_dist, int32_t *d_map, void *stream) {
    return oneshot(db, h_pairs, npairs, costs, K, d_dist, d_map, stream, true);
}

}  // extern "C"
