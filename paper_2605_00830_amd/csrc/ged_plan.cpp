// ged_plan.cpp -- launch plans of the C ABI (include/ged.h): size bins,
// persistent work-queue launches, the per-pair baseline, HIP graph capture
// and the autotuner.  No step of the search runs on the host.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <limits>
#include <map>
#include <new>
#include <string>
#include <vector>

#include "ged.h"
#include "ged_host.h"
#include "ged_internal.h"

using gedh::fail;
using gedh::ok;
using gedk::GraphRec;
using gedk::WorkItem;

namespace {

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// One size bin: pairs sharing a kernel instantiation.
struct Bin {
    bool bip = false;            // bipartite method (its own kernel, queue-node workspace)
    int bip_cpl = 0;             // its columns per lane
    int bip_nwav = 1;            // its waves per pair (1 or 4)
    int bip_max_per_cu[2] = {0, 0};   // occupancy: 1 and 4 waves per workgroup
    bool wave_ok = false;        // every pair fits the wavefront kernel
    int wave_words = 0;          // its family: 1 (n <= 32), 2 (n <= 64), 3 (n1 <= 128, n2 <= 64)
    bool wave = false;           // current choice: wavefront kernel, else workgroup kernel
    gedk::BlockShape shape{};    // workgroup-kernel instantiation and workspace shape
    std::vector<WorkItem> h_sorted;   // longest first
    std::vector<WorkItem> h_work;     // launch order for the current grid (deal_alternating)
    WorkItem *d_work = nullptr;
    int *d_queue = nullptr;      // [1 + nwork]: batched counter, then one per pair
    void *d_ws = nullptr;        // workgroup-kernel workspace
    size_t ws_stride = 0;
    size_t ws_bytes = 0;         // workspace allocation
    int grid = 0;                // current persistent grid
    int groups_per_cu = 0;       // current resident workgroups per CU
    int max_wave_per_cu = 0;     // occupancy limits
    int max_block_per_cu[3] = {0, 0, 0};   // workgroups of 256, 512, 1024 threads (0: no such instantiation)
};

int bt_index(int threads) {
    return threads == gedk::kBlockThreadsXL ? 2 : (threads == gedk::kBlockThreadsWide ? 1 : 0);
}
int bt_of(int index) {
    return index == 2 ? gedk::kBlockThreadsXL : (index == 1 ? gedk::kBlockThreadsWide : gedk::kBlockThreads);
}

}  // namespace

struct ged_plan {
    ged_db *db = nullptr;
    int64_t npairs = 0;
    int32_t K = 0;
    int last_complete = 0;   // GED_LAST_COMPLETE
    int method = GED_METHOD_TREE;
    int64_t map_entries = 0;
    int cus = 0;
    std::vector<int64_t> pair_n;   // n1 + n2 per pair, for the overflow bound
    std::vector<int64_t> pair_m;   // m1 + m2 per pair
    std::vector<Bin> bins;
    bool timing = false;
    bool timed_run = false;
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    int64_t launches = 0;
    hipGraph_t graph = nullptr;
    hipGraphExec_t graph_exec = nullptr;
    uint32_t flags = 0;                 // GED_PLAN_* bits
    int32_t *d_status = nullptr;        // [npairs] GED_OK, or why the pair was set aside
    WorkItem *d_aside = nullptr;        // set-aside pairs: out, src = mapping entries, map_off
    int naside = 0;
    // bins after the first run on streams of their own, forked from and
    // joined to the caller's stream by events (parallel branches when captured)
    std::vector<hipStream_t> side;
    hipEvent_t ev_fork = nullptr;
    std::vector<hipEvent_t> ev_join;
};

namespace {

void drop_graph(ged_plan *p) {
    if (p->graph_exec) (void)hipGraphExecDestroy(p->graph_exec);
    if (p->graph) (void)hipGraphDestroy(p->graph);
    p->graph_exec = nullptr;
    p->graph = nullptr;
}

void free_plan(ged_plan *p) {
    if (!p) return;
    drop_graph(p);
    for (Bin &b : p->bins) {
        if (b.d_work) (void)hipFree(b.d_work);
        if (b.d_queue) (void)hipFree(b.d_queue);
        if (b.d_ws) (void)hipFree(b.d_ws);
    }
    if (p->ev_start) (void)hipEventDestroy(p->ev_start);
    if (p->ev_stop) (void)hipEventDestroy(p->ev_stop);
    if (p->d_status) (void)hipFree(p->d_status);
    if (p->d_aside) (void)hipFree(p->d_aside);
    for (hipStream_t st : p->side) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : p->ev_join) (void)hipEventDestroy(ev);
    if (p->ev_fork) (void)hipEventDestroy(p->ev_fork);
    delete p;
}

// Every partial edit distance and every completed cost of a pair is at most
// max_vertex_cost * (n1 + n2) + max_edge_cost * (m1 + m2); keep it below the
// kernels' sentinel INT32_MAX.
//
// The bipartite method also keeps its matrix entries, assignment costs and
// solver potentials in int32, and packs a reduced cost with an 8-bit column
// index: an entry is at most 2 vmax + 4 emax (n1 + n2), a reduced cost at
// most (n1 + n2 + 1) entries; the bound keeps that below 2^24.
ged_status check_overflow(const ged_plan *p, const ged_costs &c) {
    const int64_t vmax = std::max({(int64_t)c.vsub, (int64_t)c.vdel, (int64_t)c.vins});
    const int64_t emax = std::max({(int64_t)c.esub, (int64_t)c.edel, (int64_t)c.eins});
    const int64_t lim = (int64_t)std::numeric_limits<int32_t>::max() - 1;
    for (int64_t i = 0; i < p->npairs; ++i) {
        const int64_t bound = vmax * p->pair_n[i] + emax * p->pair_m[i];
        if (bound > lim)
            return fail(GED_EINVAL, "costs may overflow int32 on pair %lld (bound %lld)", (long long)i,
                        (long long)bound);
        if (p->method == GED_METHOD_BIPARTITE) {
            const int64_t entry = 2 * vmax + 4 * emax * p->pair_n[i];
            if ((p->pair_n[i] + 1) * entry >= ((int64_t)1 << 24))
                return fail(GED_EINVAL, "costs may overflow the bipartite solver on pair %lld", (long long)i);
        }
    }
    return ok();
}

// Default workgroup size of a workgroup-kernel bin: 512 threads when the
// bin cannot put two 256-thread workgroups on every CU, so each pair gets
// two waves per SIMD; otherwise 256.
int default_threads(const ged_plan *p, const Bin &b) {
    // the bipartite kernel: four waves per pair when every pair of the bin is
    // resident at once with one (the launch then lasts as long as its
    // slowest pair, which four waves shorten), else one
    if (b.bip) return (int64_t)b.h_sorted.size() <= (int64_t)b.bip_max_per_cu[0] * p->cus ? 256 : 64;
    // the workgroup kernel: four waves per SIMD on one pair when the bin has
    // at most one pair per CU (and the shape that instantiation), two when it
    // cannot fill every CU twice, else one
    const int64_t n = (int64_t)b.h_sorted.size();
    if (n <= (int64_t)p->cus && b.max_block_per_cu[2] > 0) return gedk::kBlockThreadsXL;
    return n < 2 * (int64_t)p->cus ? gedk::kBlockThreadsWide : gedk::kBlockThreads;
}

// Point bin `b` at one kernel family, workgroup size (workgroup kernel) and
// resident-workgroup count (groups_per_cu <= 0: the occupancy limit); grows
// the workspace as needed and uploads the work list in the launch order for
// that grid (blocking copy: no run of the plan may be in flight).
ged_status configure_bin(ged_plan *p, Bin &b, bool wave, int groups_per_cu, int threads) {
    if (b.bip) {
        // threads: 64 = one wave per pair, 256 = four
        const int nwav = threads >= 256 ? 4 : 1;
        const int limit = b.bip_max_per_cu[nwav == 4 ? 1 : 0];
        const int gpc = groups_per_cu > 0 ? std::min(groups_per_cu, limit) : limit;
        const int64_t nwork = (int64_t)b.h_work.size();
        const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nwork, (int64_t)gpc * p->cus));
        b.bip_nwav = nwav;
        b.ws_stride = gedk::bip_workgroup_bytes(b.bip_cpl, p->K);
        const size_t need = b.ws_stride * (size_t)grid;
        if (b.ws_bytes < need) {
            if (b.d_ws) GED_HIP(hipFree(b.d_ws));
            b.d_ws = nullptr;
            b.ws_bytes = 0;
            hipError_t e = hipMalloc(&b.d_ws, need);
            if (e != hipSuccess) return fail(GED_ENOMEM, "workspace allocation failed: %s", hipGetErrorString(e));
            b.ws_bytes = need;
        }
        b.h_work = b.h_sorted;
        gedh::deal_alternating(b.h_work, grid, (nwav == 1 ? 4 : 1) * (int64_t)p->cus);
        GED_HIP(hipMemcpy(b.d_work, b.h_work.data(), sizeof(WorkItem) * (size_t)nwork, hipMemcpyHostToDevice));
        b.wave = false;
        b.groups_per_cu = gpc;
        b.grid = grid;
        return ok();
    }
    if (wave && !b.wave_ok) return fail(GED_EINVAL, "bin does not fit the wavefront kernel");
    if (!wave) {
        b.shape.BT = threads;
        b.shape.KS = gedk::block_slot_stride(p->K, threads);
    }
    const int limit = wave ? b.max_wave_per_cu : b.max_block_per_cu[bt_index(threads)];
    const int gpc = groups_per_cu > 0 ? std::min(groups_per_cu, limit) : limit;
    const int64_t nwork = (int64_t)b.h_work.size();
    const int grid = (int)std::max<int64_t>(1, std::min<int64_t>(nwork, (int64_t)gpc * p->cus));
    if (!wave) {
        b.ws_stride = gedk::block_workspace_bytes(b.shape);
        const size_t need = b.ws_stride * (size_t)grid;
        if (b.ws_bytes < need) {
            if (b.d_ws) GED_HIP(hipFree(b.d_ws));
            b.d_ws = nullptr;
            b.ws_bytes = 0;
            hipError_t e = hipMalloc(&b.d_ws, need);
            if (e != hipSuccess) return fail(GED_ENOMEM, "workspace allocation failed: %s", hipGetErrorString(e));
            b.ws_bytes = need;
        }
    }
    b.h_work = b.h_sorted;
    gedh::deal_alternating(b.h_work, grid, wave ? 4 * (int64_t)p->cus : (int64_t)p->cus);
    GED_HIP(hipMemcpy(b.d_work, b.h_work.data(), sizeof(WorkItem) * (size_t)nwork, hipMemcpyHostToDevice));
    b.wave = wave;
    b.groups_per_cu = gpc;
    b.grid = grid;
    return ok();
}

struct RunCtx {
    gedk::DbView view;
    gedk::Costs c;
    gedk::Outputs o;
    hipStream_t s;
};

ged_status launch_bin(const ged_plan *p, const Bin &b, const RunCtx &r, bool perpair) {
    const int nwork = (int)b.h_work.size();
    if (nwork == 0) return ok();
    if (b.bip) {
        if (!perpair) {
            GED_HIP(gedk::launch_bip(b.shape.PL, b.bip_cpl, b.bip_nwav, r.view, r.view, b.d_work, nwork, b.d_queue,
                                     r.c, p->K, b.d_ws, r.o, b.grid, r.s));
        } else {
            for (int i = 0; i < nwork; ++i)
                GED_HIP(gedk::launch_bip(b.shape.PL, b.bip_cpl, b.bip_nwav, r.view, r.view, b.d_work + i, 1,
                                         b.d_queue + 1 + i, r.c, p->K, b.d_ws, r.o, 1, r.s));
        }
    } else if (b.wave) {
        if (!perpair) {
            GED_HIP(gedk::launch_wave_family(b.wave_words, b.shape.PL, r.view, r.view, b.d_work, nwork, b.d_queue, r.c,
                                             p->K, p->last_complete, r.o, b.grid, r.s, b.shape.directed));
        } else {
            for (int i = 0; i < nwork; ++i)
                GED_HIP(gedk::launch_wave_family(b.wave_words, b.shape.PL, r.view, r.view, b.d_work + i, 1,
                                                 b.d_queue + 1 + i, r.c, p->K, p->last_complete, r.o, 1, r.s,
                                                 b.shape.directed));
        }
    } else if (!perpair) {
        GED_HIP(gedk::launch_block(b.shape, r.view, r.view, b.d_work, nwork, b.d_queue, r.c, p->K, p->last_complete,
                                   b.d_ws, b.ws_stride, r.o, b.grid, r.s));
    } else {
        for (int i = 0; i < nwork; ++i)
            GED_HIP(gedk::launch_block(b.shape, r.view, r.view, b.d_work + i, 1, b.d_queue + 1 + i, r.c, p->K,
                                       p->last_complete, b.d_ws, b.ws_stride, r.o, 1, r.s));
    }
    return ok();
}

ged_status prepare_run(ged_plan *plan, const ged_costs &costs, int32_t *d_dist, int32_t *d_map,
                       int64_t *d_cand, void *stream, RunCtx *r) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    if (plan->npairs > 0 && !d_dist) return fail(GED_EINVAL, "d_dist is NULL");
    if (plan->map_entries > 0 && !d_map) return fail(GED_EINVAL, "d_map is NULL");
    st = check_overflow(plan, costs);
    if (st != GED_OK) return st;
    st = gedh::check_device(plan->db);
    if (st != GED_OK) return st;
    r->view = gedk::DbView{plan->db->d_graphs, plan->db->d_adj, plan->db->d_vlab, plan->db->planes};
    r->c = gedk::Costs{costs.vsub, costs.vdel, costs.vins, costs.esub, costs.edel, costs.eins};
    r->o = gedk::Outputs{d_dist, d_map, d_cand};
    r->s = static_cast<hipStream_t>(stream);
    return ok();
}

ged_status plan_run(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                    int32_t *d_status, void *stream, bool perpair, bool allow_timing) {
    RunCtx r;
    ged_status st = prepare_run(plan, costs, d_dist, d_map, d_cand, stream, &r);
    if (st != GED_OK) return st;
    GED_HIP(gedk::launch_pair_status(plan->d_status, plan->npairs, d_status, plan->d_aside, plan->naside, d_dist,
                                     d_map, d_cand, r.s));
    const bool timing = plan->timing && allow_timing;
    plan->timed_run = false;
    plan->launches = 0;
    if (timing) GED_HIP(hipEventRecord(plan->ev_start, r.s));
    // the bins are independent.  A bin whose persistent grid fills the device
    // (at least as many pairs as resident workgroups) runs on the caller's
    // stream, one after another; a bin with fewer pairs than the device
    // holds leaves CUs idle for its whole launch, so it runs on a stream of
    // its own beside the others, forked from and joined to the caller's
    // stream by events.  The per-pair baseline stays one launch after another.
    const bool fork = !perpair && plan->bins.size() > 1 && !plan->side.empty();
    if (fork) GED_HIP(hipEventRecord(plan->ev_fork, r.s));
    size_t nside = 0;
    for (size_t k = 0; k < plan->bins.size(); ++k) {
        Bin &b = plan->bins[k];
        plan->launches += perpair ? (int64_t)b.h_work.size() : 1;
        RunCtx rb = r;
        const bool beside = fork && (int64_t)b.grid < (int64_t)b.groups_per_cu * plan->cus;
        if (beside) {
            rb.s = plan->side[nside % plan->side.size()];
            GED_HIP(hipStreamWaitEvent(rb.s, plan->ev_fork, 0));
        }
        st = launch_bin(plan, b, rb, perpair);
        if (st != GED_OK) return st;
        if (beside) GED_HIP(hipEventRecord(plan->ev_join[nside++], rb.s));
    }
    for (size_t k = 0; k < nside; ++k) GED_HIP(hipStreamWaitEvent(r.s, plan->ev_join[k], 0));
    if (timing) {
        GED_HIP(hipEventRecord(plan->ev_stop, r.s));
        plan->timed_run = true;
    }
    return ok();
}

// ---------------------------------------------------------------- tuner cache

std::string device_key() {
    int dev = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return "unknown";
    char buf[160];
    snprintf(buf, sizeof buf, "%s:%dcu", prop.gcnArchName, prop.multiProcessorCount);
    for (char *c = buf; *c; ++c)
        if (*c == ' ' || *c == '|') *c = '_';
    return buf;
}

std::string bin_key(const std::string &dev, int K, int last_complete, const Bin &b) {
    int lg = 0;
    while ((1ll << (lg + 1)) <= (long long)b.h_work.size()) ++lg;
    char buf[256];
    snprintf(buf, sizeof buf, "%s|K%d%s%s%s|w%d|W%d|PL%d|n%d|m%d|p2^%d", dev.c_str(), K, last_complete ? "c" : "",
             b.bip ? "bip" : "", b.shape.directed ? "dir" : "", b.bip ? b.bip_cpl : (b.wave_ok ? b.wave_words : 0), b.shape.W, b.shape.PL,
             b.shape.nmax1, b.shape.nmax2, lg);
    return buf;
}

struct Choice {
    bool wave;
    int groups_per_cu;
    int threads;
};

// cache lines: "<key> <wave 0|1> <groups_per_cu> <threads>"
std::map<std::string, Choice> read_cache(const char *path) {
    std::map<std::string, Choice> m;
    if (!path) return m;
    FILE *f = fopen(path, "r");
    if (!f) return m;
    char line[768], key[512];
    while (fgets(line, sizeof line, f)) {
        int w = 0, g = 0, t = 0;
        if (sscanf(line, "%511s %d %d %d", key, &w, &g, &t) == 4 &&
            (t == gedk::kBlockThreads || t == gedk::kBlockThreadsWide || t == gedk::kBlockThreadsXL || t == 64))
            m[key] = Choice{w != 0, g, t};
    }
    fclose(f);
    return m;
}

}  // namespace

extern "C" {

ged_status ged_plan_create(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K, ged_plan **out) {
    return ged_plan_create_ex(db, h_pairs, npairs, K, nullptr, out);
}

ged_status ged_plan_create_ex(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K,
                              const ged_plan_options *options, ged_plan **out) {
    ged_plan_options opt{GED_SCHED_AUTO, 0, GED_LAST_SELECT, GED_METHOD_TREE, 0u};
    if (options) opt = *options;
    if (opt.flags & ~GED_PLAN_PAIR_STATUS) return fail(GED_EINVAL, "unknown plan flags 0x%x", opt.flags);
    const bool lenient = (opt.flags & GED_PLAN_PAIR_STATUS) != 0;
    if (opt.method != GED_METHOD_TREE && opt.method != GED_METHOD_BIPARTITE)
        return fail(GED_EINVAL, "unknown method %d", opt.method);
    const bool bip = opt.method == GED_METHOD_BIPARTITE;
    if (bip && opt.last_level != GED_LAST_SELECT)
        return fail(GED_EINVAL, "the bipartite method has no last-level option");
    if (opt.schedule != GED_SCHED_AUTO && opt.schedule != GED_SCHED_BLOCK)
        return fail(GED_EINVAL, "unknown schedule %d", opt.schedule);
    if (opt.last_level != GED_LAST_SELECT && opt.last_level != GED_LAST_COMPLETE)
        return fail(GED_EINVAL, "unknown last level %d", opt.last_level);
    if (opt.groups_per_cu < 0) return fail(GED_EINVAL, "groups_per_cu < 0");
    if (!out) return fail(GED_EINVAL, "out is NULL");
    *out = nullptr;
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (npairs < 0) return fail(GED_EINVAL, "npairs < 0");
    if (npairs > 0 && !h_pairs) return fail(GED_EINVAL, "pairs is NULL");
    if (npairs > (int64_t)std::numeric_limits<int32_t>::max()) return fail(GED_EUNSUPPORTED, "more than 2^31-1 pairs");
    if (K < 1) return fail(GED_EINVAL, "K must be >= 1 (got %d)", K);
    if (K > GED_MAX_K) return fail(GED_EUNSUPPORTED, "K = %d exceeds %d", K, GED_MAX_K);
    if (bip && K > GED_BIP_MAX_K)
        return fail(GED_EUNSUPPORTED, "K = %d exceeds the bipartite method's %d", K, GED_BIP_MAX_K);
    if (bip && db->directed) return fail(GED_EUNSUPPORTED, "the bipartite method takes undirected graphs only");
    ged_status st = gedh::check_device(db);
    if (st != GED_OK) return st;

    ged_plan *p = new (std::nothrow) ged_plan;
    if (!p) return fail(GED_ENOMEM, "host allocation failed");
    p->db = db;
    p->npairs = npairs;
    p->K = K;
    p->last_complete = opt.last_level == GED_LAST_COMPLETE ? 1 : 0;
    p->method = opt.method;
    p->flags = opt.flags;
    p->pair_n.resize((size_t)npairs);
    p->pair_m.resize((size_t)npairs);
    std::vector<int32_t> h_status((size_t)npairs, (int32_t)GED_OK);
    std::vector<WorkItem> h_aside;

    // bins keyed by kernel: -1 / -2 = wavefront kernel for n <= 32 / 64,
    // -3 .. -6 = bipartite kernel with 1 .. 4 columns per lane, else target
    // row words rounded up to a power of two (the workgroup kernel's
    // instantiation; twice that for a directed database, whose rows hold the
    // out-arcs and the in-arcs: only the workgroup kernel takes those)
    const int PL = db->planes == 0 ? 0 : (db->planes <= 2 ? 2 : 4);
    std::map<int, Bin> bins;
    int64_t off = 0;
    for (int64_t i = 0; i < npairs; ++i) {
        const int64_t s = h_pairs[i].src, d = h_pairs[i].dst;
        // a pair that cannot be searched: fail the plan, or set it aside
        // with its status (its mapping entries still take their place)
        auto refuse = [&](ged_status why, int n1) {
            WorkItem wi{};
            wi.src = n1;
            wi.out = (int32_t)i;
            wi.map_off = off;
            h_aside.push_back(wi);
            h_status[(size_t)i] = (int32_t)why;
            p->pair_n[(size_t)i] = 0;
            p->pair_m[(size_t)i] = 0;
            off += n1;
        };
        if (s < 0 || s >= db->count || d < 0 || d >= db->count) {
            if (lenient) {
                refuse(GED_EINVAL, (s >= 0 && s < db->count) ? db->h_graphs[(size_t)s].n : 0);
                continue;
            }
            free_plan(p);
            return fail(GED_EINVAL, "pair %lld: graph id out of range", (long long)i);
        }
        const GraphRec &g1 = db->h_graphs[(size_t)s];
        const GraphRec &g2 = db->h_graphs[(size_t)d];
        p->pair_n[(size_t)i] = (int64_t)g1.n + g2.n;
        p->pair_m[(size_t)i] = (int64_t)g1.m + g2.m;
        const char *beyond = nullptr;
        char why[160];
        if (db->directed && std::max(g1.n, g2.n) > GED_DIRECTED_MAX_ORDER) {
            snprintf(why, sizeof why, "directed graphs of more than %d vertices", GED_DIRECTED_MAX_ORDER);
            beyond = why;
        } else if (bip && g1.n + g2.n > GED_BIP_MAX_ORDER) {
            snprintf(why, sizeof why, "n1 + n2 = %d exceeds the bipartite method's %d", g1.n + g2.n,
                     GED_BIP_MAX_ORDER);
            beyond = why;
        } else if (std::max(g1.n, g2.n) > GED_MAX_VERTICES_BATCH) {
            snprintf(why, sizeof why, "a graph of %d vertices exceeds the batched search's %d (ged_wide_* takes it)",
                     std::max(g1.n, g2.n), GED_MAX_VERTICES_BATCH);
            beyond = why;
        }
        if (beyond) {
            if (lenient) {
                refuse(GED_EUNSUPPORTED, g1.n);
                continue;
            }
            free_plan(p);
            return fail(GED_EUNSUPPORTED, "pair %lld: %s", (long long)i, beyond);
        }
        const int ww = (bip || opt.schedule != GED_SCHED_AUTO) ? 0
                       : db->directed ? gedk::wave_words_for_directed(g1.n, g2.n, K)
                                      : gedk::wave_words_for(g1.n, g2.n, K);
        const bool wave = ww > 0;
        const int W = pow2_at_least(std::max(1, g2.w)) * (db->directed ? 2 : 1);
        const int cpl = bip ? gedk::bip_cols_per_lane(g1.n + g2.n) : 0;
        Bin &b = bins[bip ? -2 - cpl : (wave ? -ww : W)];
        b.bip = bip;
        b.bip_cpl = cpl;
        b.wave_ok = wave;
        b.wave = wave;
        b.wave_words = ww;
        b.shape.W = W;
        b.shape.PL = PL;
        b.shape.directed = db->directed ? 1 : 0;
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

    int device = 0;
    hipError_t e = hipGetDevice(&device);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&p->cus, hipDeviceAttributeMultiprocessorCount, device);
    if (e != hipSuccess) {
        free_plan(p);
        return fail(GED_EDEVICE, "device query failed: %s", hipGetErrorString(e));
    }
    // per-pair statuses and the set-aside pairs' output records
    p->naside = (int)h_aside.size();
    e = hipMalloc((void **)&p->d_status, sizeof(int32_t) * (size_t)std::max<int64_t>(npairs, 1));
    if (e == hipSuccess && npairs > 0)
        e = hipMemcpy(p->d_status, h_status.data(), sizeof(int32_t) * (size_t)npairs, hipMemcpyHostToDevice);
    if (e == hipSuccess && p->naside > 0) {
        e = hipMalloc((void **)&p->d_aside, sizeof(WorkItem) * h_aside.size());
        if (e == hipSuccess)
            e = hipMemcpy(p->d_aside, h_aside.data(), sizeof(WorkItem) * h_aside.size(), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) {
        free_plan(p);
        return fail(GED_ENOMEM, "plan allocation failed: %s", hipGetErrorString(e));
    }
    // streams and events for running bins side by side (default priority;
    // at most three extra streams, bins beyond share them in turn; one join
    // event per bin)
    const size_t nside = bins.size() > 1 ? std::min<size_t>(bins.size(), 3) : 0;
    for (size_t k = 0; k < nside && e == hipSuccess; ++k) {
        hipStream_t st = nullptr;
        e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
        if (e == hipSuccess) p->side.push_back(st);
    }
    if (e == hipSuccess && nside > 0) e = hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming);
    for (size_t k = 0; k < bins.size() && nside > 0 && e == hipSuccess; ++k) {
        hipEvent_t ev = nullptr;
        e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e == hipSuccess) p->ev_join.push_back(ev);
    }
    if (e != hipSuccess) {
        free_plan(p);
        return fail(GED_EDEVICE, "stream or event creation failed: %s", hipGetErrorString(e));
    }

    for (auto &kv : bins) {
        p->bins.push_back(Bin());
        Bin &b = p->bins.back();
        b.bip = kv.second.bip;
        b.bip_cpl = kv.second.bip_cpl;
        b.wave_ok = kv.second.wave_ok;
        b.wave_words = kv.second.wave_words;
        b.shape = kv.second.shape;
        b.h_work.swap(kv.second.h_work);
        // longest first: the tree search's work grows with n1 * (n2 + 1); the
        // bipartite method's with n1^2 (n1 + n2) (children per pop times
        // solver steps, measured by rank correlation with its step counts).
        // A wavefront pair's duration is n1 levels of a fixed part (reductions,
        // LDS round trips, the update) plus one that grows with n2, so those
        // bins go by n1 * (n2 + 24), so the pairs of most levels start first
        // (measured on the 4096-pair batches: 91.5 us against 99.7 with
        // n1 * (n2 + 1); constants from 16 to 32 are equally good)
        auto work_of = [&](const WorkItem &x) -> int64_t {
            const int64_t a = db->h_graphs[x.src].n, c = db->h_graphs[x.dst].n;
            return b.bip ? a * a * (a + c) : (b.wave_ok ? a * (c + 24) : a * (c + 1));
        };
        std::stable_sort(b.h_work.begin(), b.h_work.end(),
                         [&](const WorkItem &x, const WorkItem &y) { return work_of(x) > work_of(y); });
        b.h_sorted = b.h_work;
        if (b.bip) {
            e = gedk::bip_max_resident(b.shape.PL, b.bip_cpl, K, 1, &b.bip_max_per_cu[0]);
            if (e == hipSuccess) e = gedk::bip_max_resident(b.shape.PL, b.bip_cpl, K, 4, &b.bip_max_per_cu[1]);
            b.max_wave_per_cu = std::min(b.bip_max_per_cu[0], b.bip_max_per_cu[1]);
            b.max_block_per_cu[0] = b.max_block_per_cu[1] = 1;   // not used
        }
        for (int k = 0; k < 3 && e == hipSuccess && !b.bip; ++k) {
            gedk::BlockShape sh = b.shape;
            sh.BT = bt_of(k);
            sh.KS = gedk::block_slot_stride(K, sh.BT);
            if (k == 2 && !gedk::block_shape_supported(sh)) continue;   // 1024 threads: some shapes only
            e = gedk::block_max_resident(sh, &b.max_block_per_cu[k]);
        }
        if (e == hipSuccess && b.wave_ok)
            e = gedk::wave_family_max_resident(b.wave_words, b.shape.PL, K, p->last_complete, &b.max_wave_per_cu,
                                               b.shape.directed);
        if (e != hipSuccess || b.max_block_per_cu[0] <= 0 || b.max_block_per_cu[1] <= 0 ||
            ((b.wave_ok || b.bip) && b.max_wave_per_cu <= 0)) {
            free_plan(p);
            return fail(GED_EDEVICE, "occupancy query failed: %s", hipGetErrorString(e));
        }
        const int64_t nwork = (int64_t)b.h_work.size();
        e = hipMalloc((void **)&b.d_work, sizeof(WorkItem) * (size_t)nwork);
        if (e == hipSuccess) e = hipMalloc((void **)&b.d_queue, sizeof(int) * (size_t)(nwork + 1));
        // the queue counters start at 0; every run leaves them at 0 again
        if (e == hipSuccess) e = hipMemset(b.d_queue, 0, sizeof(int) * (size_t)(nwork + 1));
        if (e != hipSuccess) {
            free_plan(p);
            return fail(GED_ENOMEM, "plan allocation failed: %s", hipGetErrorString(e));
        }
        st = configure_bin(p, b, b.wave_ok, opt.groups_per_cu, default_threads(p, b));
        if (st != GED_OK) {
            free_plan(p);
            return st;
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

ged_status ged_plan_run(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                        void *stream) {
    return plan_run(plan, costs, d_dist, d_map, d_cand, nullptr, stream, false, true);
}

ged_status ged_plan_run_ex(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                           int32_t *d_status, void *stream) {
    return plan_run(plan, costs, d_dist, d_map, d_cand, d_status, stream, false, true);
}

ged_status ged_plan_run_perpair(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                                int64_t *d_cand, void *stream) {
    return plan_run(plan, costs, d_dist, d_map, d_cand, nullptr, stream, true, true);
}

ged_status ged_plan_destroy(ged_plan *plan) {
    free_plan(plan);
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

ged_status ged_plan_kernel_launches(const ged_plan *plan, int64_t *launches) {
    if (!plan || !launches) return fail(GED_EINVAL, "NULL argument");
    *launches = plan->launches;
    return ok();
}

ged_status ged_plan_bin_count(const ged_plan *plan, int32_t *count) {
    if (!plan || !count) return fail(GED_EINVAL, "NULL argument");
    *count = (int32_t)plan->bins.size();
    return ok();
}

ged_status ged_plan_bin_info(const ged_plan *plan, int32_t index, int32_t *kernel, int64_t *npairs, int32_t *grid,
                             int32_t *words) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    if (index < 0 || index >= (int32_t)plan->bins.size()) return fail(GED_EINVAL, "bin %d out of range", index);
    const Bin &b = plan->bins[(size_t)index];
    if (kernel) *kernel = b.bip ? GED_KERNEL_BIPARTITE : (b.wave ? GED_KERNEL_WAVE : GED_KERNEL_BLOCK);
    if (npairs) *npairs = (int64_t)b.h_work.size();
    if (grid) *grid = b.grid;
    if (words) *words = b.bip ? b.bip_cpl : (b.wave ? std::min(b.wave_words, 2) : b.shape.W);
    return ok();
}

ged_status ged_plan_capture(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                            void *stream) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    if (!stream) return fail(GED_EINVAL, "the null stream cannot be captured; pass a created stream");
    RunCtx r;
    ged_status st = prepare_run(plan, costs, d_dist, d_map, d_cand, stream, &r);
    if (st != GED_OK) return st;
    drop_graph(plan);
    GED_HIP(hipStreamBeginCapture(r.s, hipStreamCaptureModeThreadLocal));
    st = plan_run(plan, costs, d_dist, d_map, d_cand, nullptr, stream, false, false);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(r.s, &g);
    if (st != GED_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (e != hipSuccess) return fail(GED_EDEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(e));
    hipGraphExec_t x = nullptr;
    e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        (void)hipGraphDestroy(g);
        return fail(GED_EDEVICE, "hipGraphInstantiate failed: %s", hipGetErrorString(e));
    }
    plan->graph = g;
    plan->graph_exec = x;
    return ok();
}

ged_status ged_plan_replay(ged_plan *plan, void *stream) {
    if (!plan) return fail(GED_EINVAL, "plan is NULL");
    if (!plan->graph_exec) return fail(GED_EINVAL, "no captured graph");
    GED_HIP(hipGraphLaunch(plan->graph_exec, static_cast<hipStream_t>(stream)));
    return ok();
}

ged_status ged_plan_tune(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, void *stream,
                         const char *cache_path, int32_t *timed_bins) {
    RunCtx r;
    ged_status st = prepare_run(plan, costs, d_dist, d_map, nullptr, stream, &r);
    if (st != GED_OK) return st;
    // reconfiguring rewrites the plan's work lists: let earlier runs finish
    GED_HIP(hipDeviceSynchronize());
    drop_graph(plan);
    const std::string dev = device_key();
    std::map<std::string, Choice> cache = read_cache(cache_path);
    FILE *append = nullptr;
    int timed = 0;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    GED_HIP(hipEventCreate(&e0));
    GED_HIP(hipEventCreate(&e1));
    for (Bin &b : plan->bins) {
        const std::string key = bin_key(dev, plan->K, plan->last_complete, b);
        auto hit = cache.find(key);
        if (hit != cache.end() && (!hit->second.wave || b.wave_ok || b.bip) &&
            (b.bip || hit->second.wave || b.max_block_per_cu[bt_index(hit->second.threads)] > 0)) {
            st = configure_bin(plan, b, hit->second.wave, hit->second.groups_per_cu, hit->second.threads);
            if (st != GED_OK) break;
            continue;
        }
        // candidates: the wavefront kernel and the workgroup kernel (256 and
        // 512 threads), each at the occupancy limit and fractions of it; one
        // candidate per distinct grid
        std::vector<Choice> cands;
        const int64_t nwork = (int64_t)b.h_sorted.size();
        for (int fam = 0; fam < 4; ++fam) {
            const bool wave = fam == 0;
            if (b.bip && fam >= 2) continue;   // the bipartite kernel: one or four waves per pair
            if (wave && !b.wave_ok && !b.bip) continue;
            if (fam == 3 && b.max_block_per_cu[2] <= 0) continue;   // no 1024-thread instantiation
            const int threads = b.bip ? (fam == 0 ? 64 : 256) : bt_of(fam == 0 ? 0 : fam - 1);
            const int lim = b.bip ? b.bip_max_per_cu[fam] : (wave ? b.max_wave_per_cu : b.max_block_per_cu[bt_index(threads)]);
            int64_t last_grid = -1;
            for (int g = lim; g >= 1; g = g / 2) {
                const int64_t grid = std::min<int64_t>(nwork, (int64_t)g * plan->cus);
                if (grid != last_grid) cands.push_back(Choice{wave, g, threads});
                last_grid = grid;
                if (g == 1) break;
            }
        }
        float best_ms = 1e30f;
        Choice best = cands.front();
        for (const Choice &cd : cands) {
            st = configure_bin(plan, b, cd.wave, cd.groups_per_cu, cd.threads);
            if (st != GED_OK) break;
            float ms_sum[3] = {0, 0, 0};
            for (int rep = 0; rep < 4 && st == GED_OK; ++rep) {
                hipError_t he = gedk::launch_fill_zero(b.d_queue, (int)b.h_work.size() + 1, r.s);
                if (he == hipSuccess) he = hipEventRecord(e0, r.s);
                if (he != hipSuccess) {
                    st = fail(GED_EDEVICE, "tuning launch failed: %s", hipGetErrorString(he));
                    break;
                }
                st = launch_bin(plan, b, r, false);
                if (st != GED_OK) break;
                he = hipEventRecord(e1, r.s);
                if (he == hipSuccess) he = hipEventSynchronize(e1);
                float ms = 0.f;
                if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
                if (he != hipSuccess) {
                    st = fail(GED_EDEVICE, "tuning timing failed: %s", hipGetErrorString(he));
                    break;
                }
                if (rep > 0) ms_sum[rep - 1] = ms;   // first run warms up
            }
            if (st != GED_OK) break;
            std::sort(ms_sum, ms_sum + 3);
            if (ms_sum[1] < best_ms) {
                best_ms = ms_sum[1];
                best = cd;
            }
        }
        if (st != GED_OK) break;
        st = configure_bin(plan, b, best.wave, best.groups_per_cu, best.threads);
        if (st != GED_OK) break;
        ++timed;
        if (cache_path) {
            if (!append) append = fopen(cache_path, "a");
            if (append)
                fprintf(append, "%s %d %d %d\n", key.c_str(), best.wave ? 1 : 0, best.groups_per_cu, best.threads);
        }
    }
    if (append) fclose(append);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != GED_OK) return st;
    // leave the outputs holding a full result with the chosen configuration
    st = plan_run(plan, costs, d_dist, d_map, nullptr, nullptr, stream, false, false);
    if (st != GED_OK) return st;
    GED_HIP(hipStreamSynchronize(r.s));
    if (timed_bins) *timed_bins = timed;
    return ok();
}

ged_status ged_kbest(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                     int32_t *d_dist, int32_t *d_map, void *stream) {
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    ged_plan *p = nullptr;
    st = ged_plan_create(db, h_pairs, npairs, K, &p);
    if (st != GED_OK) return st;
    st = plan_run(p, costs, d_dist, d_map, nullptr, nullptr, stream, false, false);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_plan(p);
    if (st != GED_OK) return st;
    if (e != hipSuccess) return fail(GED_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return ok();
}

ged_status ged_kbest_ex(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                        const ged_plan_options *options, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                        int32_t *d_status, void *stream) {
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    ged_plan *p = nullptr;
    st = ged_plan_create_ex(db, h_pairs, npairs, K, options, &p);
    if (st != GED_OK) return st;
    st = plan_run(p, costs, d_dist, d_map, d_cand, d_status, stream, false, false);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_plan(p);
    if (st != GED_OK) return st;
    if (e != hipSuccess) return fail(GED_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return ok();
}

ged_status ged_map_offsets(ged_db *db, const ged_pair *d_pairs, int64_t npairs, int64_t *d_off, void *stream) {
    if (!db) return fail(GED_EINVAL, "db is NULL");
    if (!d_off) return fail(GED_EINVAL, "d_off is NULL");
    if (npairs < 0) return fail(GED_EINVAL, "npairs < 0");
    if (npairs > 0 && !d_pairs) return fail(GED_EINVAL, "d_pairs is NULL");
    ged_status st = gedh::check_device(db);
    if (st != GED_OK) return st;
    GED_HIP(gedk::launch_map_offsets(db->d_graphs, db->count, d_pairs, npairs, d_off,
                                     static_cast<hipStream_t>(stream)));
    return ok();
}

ged_status ged_kbest_perpair(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                             int32_t *d_dist, int32_t *d_map, void *stream) {
    ged_status st = gedh::check_costs(costs);
    if (st != GED_OK) return st;
    ged_plan *p = nullptr;
    st = ged_plan_create(db, h_pairs, npairs, K, &p);
    if (st != GED_OK) return st;
    st = plan_run(p, costs, d_dist, d_map, nullptr, nullptr, stream, true, false);
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    free_plan(p);
    if (st != GED_OK) return st;
    if (e != hipSuccess) return fail(GED_EDEVICE, "hipStreamSynchronize failed: %s", hipGetErrorString(e));
    return ok();
}

}  // extern "C"
