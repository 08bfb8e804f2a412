// ged_api.cpp -- status reporting and the device-resident graph database of
// the C ABI declared in include/ged.h.
//
// Validates every graph on the host and packs it into adjacency bitsets plus
// edge-label bit planes in device memory.  Plans and launches are in
// ged_plan.cpp.
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
#include "ged_host.h"
#include "ged_internal.h"

using gedk::GraphRec;
using gedk::WorkItem;

namespace gedh {

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

ged_status check_costs(const ged_costs &c) {
    const int32_t v[6] = {c.vsub, c.vdel, c.vins, c.esub, c.edel, c.eins};
    for (int k = 0; k < 6; ++k)
        if (v[k] < 0) return fail(GED_EINVAL, "costs must be >= 0 (cost %d is %d)", k, v[k]);
    return ok();
}

ged_status check_device(const ged_db *db) {
    int dev = -1;
    GED_HIP(hipGetDevice(&dev));
    if (dev != db->device)
        return fail(GED_EINVAL, "current HIP device %d differs from the database's device %d", dev,
                    db->device);
    return ok();
}


ged_status check_graph_shape(const ged_graph &G, int64_t g, bool directed) {
    if (G.n < 0 || G.m < 0) return fail(GED_EINVAL, "graph %lld: negative n or m", (long long)g);
    if (G.n > GED_MAX_VERTICES)
        return fail(GED_EUNSUPPORTED, "graph %lld: n = %d exceeds %d", (long long)g, G.n, GED_MAX_VERTICES);
    if (G.n > 0 && !G.vlabel) return fail(GED_EINVAL, "graph %lld: vlabel is NULL", (long long)g);
    if (G.m > 0 && (!G.eu || !G.ev)) return fail(GED_EINVAL, "graph %lld: edge arrays are NULL", (long long)g);
    if ((int64_t)G.m > (int64_t)G.n * (G.n - 1) / (directed ? 1 : 2))
        return fail(GED_EINVAL, "graph %lld: more edges than a simple graph allows", (long long)g);
    return ok();
}

int64_t packed_words(int n, int planes, bool directed) {
    return (int64_t)n * ((n + 31) / 32) * (1 + planes) * (directed ? 2 : 1);
}

// Undirected: row v holds the neighbours of v (both ends of every edge set).
// Directed: the first block's row v holds the heads of v's out-arcs, a second
// block of the same shape (rows, then planes) the tails of its in-arcs.
ged_status pack_graph(const ged_graph &G, int64_t g, const std::vector<int32_t> &labels, int planes,
                      std::vector<uint32_t> &adj, std::vector<int32_t> &vlab, gedk::GraphRec &R, bool directed) {
    const int n = G.n, w = (n + 31) / 32;
    const size_t base = adj.size();
    const size_t plane = (size_t)n * w;
    adj.resize(base + plane * (1 + planes) * (directed ? 2 : 1), 0u);
    R.n = n;
    R.m = G.m;
    R.w = w;
    R.pad = 0;
    R.adj = (int64_t)base;
    R.vlab = (int64_t)vlab.size();
    uint32_t *rows = adj.data() + base;
    uint32_t *rev = directed ? rows + plane * (1 + planes) : rows;   // where b's row gets a
    for (int k = 0; k < G.m; ++k) {
        const int a = G.eu[k], b = G.ev[k];
        if (a < 0 || b < 0 || a >= n || b >= n)
            return fail(GED_EINVAL, "graph %lld: edge %d has a vertex out of range", (long long)g, k);
        if (a == b) return fail(GED_EINVAL, "graph %lld: edge %d is a self-loop", (long long)g, k);
        if (rows[(size_t)a * w + (b >> 5)] & (1u << (b & 31)))
            return fail(GED_EINVAL, "graph %lld: edge %d repeats (%d,%d)", (long long)g, k, a, b);
        rows[(size_t)a * w + (b >> 5)] |= 1u << (b & 31);
        rev[(size_t)b * w + (a >> 5)] |= 1u << (a & 31);
        const int32_t lab = G.elabel ? G.elabel[k] : 0;
        const auto it = std::lower_bound(labels.begin(), labels.end(), lab);
        if (it == labels.end() || *it != lab)
            return fail(GED_EINVAL, "graph %lld: edge label %d is not in the database's label set", (long long)g, lab);
        const int code = (int)(it - labels.begin());
        for (int p = 0; p < planes; ++p) {
            if ((code >> p) & 1) {
                rows[(size_t)(1 + p) * plane + (size_t)a * w + (b >> 5)] |= 1u << (b & 31);
                rev[(size_t)(1 + p) * plane + (size_t)b * w + (a >> 5)] |= 1u << (a & 31);
            }
        }
    }
    for (int v = 0; v < n; ++v) vlab.push_back(G.vlabel[v]);
    return ok();
}

}  // namespace gedh

using gedh::fail;
using gedh::ok;

namespace {

int words_for(int n) { return (n + 31) / 32; }

}  // namespace

namespace {

void free_db(ged_db *db) {
    if (!db) return;
    if (db->d_graphs) (void)hipFree(db->d_graphs);
    if (db->d_adj) (void)hipFree(db->d_adj);
    if (db->d_vlab) (void)hipFree(db->d_vlab);
    delete db;
}

}  // namespace

extern "C" {

int32_t ged_abi_version(void) { return GED_ABI_VERSION; }

const char *ged_last_error(void) { return gedh::g_last_error.c_str(); }

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
    return ged_db_create_ex(graphs, count, 0u, out);
}

ged_status ged_db_create_ex(const ged_graph *graphs, int64_t count, uint32_t flags, ged_db **out) {
    if (!out) return fail(GED_EINVAL, "out is NULL");
    *out = nullptr;
    if (flags & ~(uint32_t)GED_DB_DIRECTED) return fail(GED_EINVAL, "unknown database flags 0x%x", flags);
    const bool directed = (flags & GED_DB_DIRECTED) != 0;
    if (count < 0) return fail(GED_EINVAL, "count < 0");
    if (count > 0 && !graphs) return fail(GED_EINVAL, "graphs is NULL");
    if (count > (int64_t)std::numeric_limits<int32_t>::max())
        return fail(GED_EUNSUPPORTED, "more than 2^31-1 graphs");

    // pass 1: validate shapes, collect the distinct edge labels
    std::vector<int32_t> labels;
    int64_t total_words = 0, total_v = 0;
    for (int64_t g = 0; g < count; ++g) {
        ged_status st = gedh::check_graph_shape(graphs[g], g, directed);
        if (st != GED_OK) return st;
        const ged_graph &G = graphs[g];
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
    for (int64_t g = 0; g < count; ++g) total_words += gedh::packed_words(graphs[g].n, planes, directed);

    ged_db *db = new (std::nothrow) ged_db;
    if (!db) return fail(GED_ENOMEM, "host allocation failed");
    db->count = count;
    db->planes = planes;
    db->directed = directed;
    db->elabels = labels;
    db->h_graphs.resize((size_t)count);

    // pass 2: pack rows and planes, rejecting self-loops, bad ids and repeats
    std::vector<uint32_t> adj;
    std::vector<int32_t> vlab;
    adj.reserve((size_t)std::max<int64_t>(total_words, 1));
    vlab.reserve((size_t)std::max<int64_t>(total_v, 1));
    for (int64_t g = 0; g < count; ++g) {
        ged_status st =
            gedh::pack_graph(graphs[g], g, labels, planes, adj, vlab, db->h_graphs[(size_t)g], directed);
        if (st != GED_OK) {
            free_db(db);
            return st;
        }
    }
    if (adj.empty()) adj.push_back(0u);
    if (vlab.empty()) vlab.push_back(0);

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

ged_status ged_db_flags(const ged_db *db, uint32_t *flags) {
    if (!db || !flags) return fail(GED_EINVAL, "NULL argument");
    *flags = db->directed ? (uint32_t)GED_DB_DIRECTED : 0u;
    return ok();
}

ged_status ged_db_order(const ged_db *db, int64_t id, int32_t *n) {
    if (!db || !n) return fail(GED_EINVAL, "NULL argument");
    if (id < 0 || id >= db->count) return fail(GED_EINVAL, "graph id %lld out of range", (long long)id);
    *n = db->h_graphs[(size_t)id].n;
    return ok();
}

}  // extern "C"
