// ged_server.cpp -- the serving loop of the C ABI (include/ged.h).
//
// Client threads submit (query graph, target id) requests; submit packs the
// query graph on the host with the database's edge-label coding.  One worker
// thread per server runs the loop:
//   1. completion: every stream whose batch event has fired hands its results
//      (already copied to pinned host memory on that stream) to the waiting
//      tickets and frees its slots and arena space;
//   2. admission: while a stream is idle, queued requests move into a batch
//      in arrival order as long as the in-flight slot limit and the stream's
//      arena (its share of the HBM budget) have room;
//   3. launch: the batch's query graphs and work lists are copied to the
//      device, the work-queue counters cleared by a kernel, the size bins
//      launched (wavefront kernels for pairs of up to 64 vertices, workgroup
//      kernel for the rest), results copied back and an event recorded -- all on that
//      stream, so batches on different streams overlap on the device.
// A query's search runs entirely inside one kernel launch, so its result
// does not depend on the other queries of its batch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "ged.h"
#include "ged_host.h"
#include "ged_internal.h"

using gedh::fail;
using gedh::ok;
using gedk::GraphRec;
using gedk::WorkItem;

namespace {

enum ReqState { QUEUED = 0, INFLIGHT = 1, DONE = 2, FAILED = 3, CANCELED = 4 };

// size classes: small (n <= 32) and mid (n <= 64) for the two wavefront
// kernels (K <= 64), medium (n <= 128) and large for the workgroup kernel;
// with the bipartite method, n1 + n2 <= 64, 128, 192, 256 (its kernel's
// columns per lane)
constexpr int kClasses = 4;
constexpr int kFirstBlockClass = 2;

struct Request {
    uint64_t ticket = 0;
    int cls = 0;
    int32_t n1 = 0;
    int32_t target = 0;
    GraphRec rec{};                 // adj / vlab offsets relative to this request's vectors
    std::vector<uint32_t> adj;      // packed rows and label planes (empty for a database query)
    std::vector<int32_t> vlab;
    int64_t words = 0;              // packed words of the query graph
    int64_t db_query = -1;          // the query is this database graph (copied on the device)
    int state = QUEUED;
    int32_t dist = -1;
    std::vector<int32_t> map;
    int64_t t_submit = 0, t_done = 0;   // monotonic clock, ns
};

int64_t now_ns() {
    return (int64_t)std::chrono::duration_cast<std::chrono::nanoseconds>(
               std::chrono::steady_clock::now().time_since_epoch()).count();
}

using ReqPtr = std::shared_ptr<Request>;

// Batch formation while a class already has a batch on the device: wait for
// this many queued queries, or until the oldest has waited this long.
constexpr int64_t kFillQueries = 64;
constexpr int64_t kHoldNs = 1'000'000;

// Resident workgroups per CU a batch of each class may hold (the wavefront
// classes are not capped): one 512-thread workgroup of the large class takes
// at most 288 of a SIMD lane's 512 VGPRs, leaving room for two waves of the
// wavefront kernels beside it.
constexpr int kBlockClassPerCu[4] = {1 << 20, 1 << 20, 2, 1};
constexpr int kLargeStreams = 2;

constexpr int kWaveBins = gedk::kWaveFamilies;   // wavefront bins: the three families
constexpr int kMaxBins = kWaveBins + 5;            // + workgroup bins W = 1, 2, 4, 8, 16

// Device and pinned-host buffers of one stream.  A batch's inputs are
// staged in one pinned buffer and reach the device in one copy: the queue
// counters (zeros), the work list, the database queries to gather, the query
// graph records, then the vertex labels and packed rows of the query graphs
// (the last two packed back to back, so the copy stops where the batch's
// data ends).  Its outputs come back in one copy as well: the distances, then
// the mappings.
struct Slab {
    int cls = 0;                    // size class this stream serves
    size_t ws_bytes = 0;            // its workgroup-kernel workspace
    int64_t cap_words = 0, cap_vlab = 0;   // arena capacity (mappings share cap_vlab)
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    size_t o_work = 0, o_gather = 0, o_recs = 0, o_var = 0, in_bytes = 0;   // input layout
    char *d_in = nullptr;           // device inputs
    char *h_in = nullptr;           // pinned staging of the inputs
    int32_t *d_out = nullptr;       // device outputs: dist[nq], then the mappings
    int32_t *h_out = nullptr;       // pinned copy of the outputs
    void *d_ws = nullptr;
    // the batch on the device
    bool busy = false;
    std::vector<ReqPtr> batch;
    std::vector<int64_t> map_off;
};

int pow2_at_least(int x) {
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

}  // namespace

struct ged_server {
    ged_db *db = nullptr;
    ged_server_config cfg{};
    gedk::Costs c{};
    int PL = 0;
    int cus = 0;
    int wave_per_cu[kWaveBins] = {0, 0, 0};   // the wavefront families' kernels
    int block_per_cu[2][5] = {};   // [256 | 512 threads][W = 1, 2, 4, 8, 16]
    bool bip = false;              // bipartite method
    bool directed = false;         // directed database: rows [out | in], W doubled
    int bip_per_cu[kClasses] = {0, 0, 0, 0};   // its kernel, 1..4 columns per lane
    int64_t device_bytes = 0;
    std::vector<Slab> slabs;

    std::mutex mu;
    std::condition_variable cv_work;   // worker: new requests or stop
    std::condition_variable cv_done;   // clients: results
    std::deque<ReqPtr> queue[kClasses];
    int64_t queued_total = 0;
    std::unordered_map<uint64_t, ReqPtr> tickets;
    uint64_t next_ticket = 1;
    bool stop = false;
    std::deque<uint64_t> done_order;   // finished tickets in completion order, for collect
    std::thread worker;
    int device = 0;

    ged_server_stats stats{};
};

namespace {

int w_index(int W) {
    int k = 0;
    while ((1 << k) < W) ++k;
    return k;
}

// Size class of a pair: 0 = small, 1 = mid (the wavefront kernels for
// n <= 32 and n <= 64), 2 = medium, 3 = large.
constexpr int kMediumMaxN = 128;

int server_class(const ged_server *s, int n1, int n2) {
    if (s->bip) return gedk::bip_cols_per_lane(n1 + n2) - 1;
    // directed pairs of up to 32 vertices take the two-word kernel (class 1);
    // sources of 65..128 vertices against targets of up to 64 are medium
    // queries, searched on the wavefront kernel's third family
    const int ww = s->directed ? gedk::wave_words_for_directed(n1, n2, s->cfg.K) : gedk::wave_words_for(n1, n2, s->cfg.K);
    if (ww == 3) return 2;
    if (ww > 0) return ww - 1;
    if (n1 <= kMediumMaxN && n2 <= kMediumMaxN) return 2;
    return 3;
}

gedk::BlockShape shape_for(const ged_server *s, int W, int nmax1, int nmax2, int threads) {
    gedk::BlockShape sh{};
    sh.W = W;
    sh.PL = s->PL;
    sh.BT = threads;
    sh.KS = gedk::block_slot_stride(s->cfg.K, threads);
    sh.nmax1 = nmax1;
    sh.nmax2 = nmax2;
    sh.directed = s->directed ? 1 : 0;
    return sh;
}

void free_slab(Slab &b) {
    if (b.d_in) (void)hipFree(b.d_in);
    if (b.d_out) (void)hipFree(b.d_out);
    if (b.d_ws) (void)hipFree(b.d_ws);
    if (b.h_in) (void)hipHostFree(b.h_in);
    if (b.h_out) (void)hipHostFree(b.h_out);
    if (b.done) (void)hipEventDestroy(b.done);
    if (b.stream) (void)hipStreamDestroy(b.stream);
    b = Slab();
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Launch the slab's batch; on error the caller fails the batch.
hipError_t launch_batch(ged_server *s, Slab &b) {
    const int nq = (int)b.batch.size();
    const int K = s->cfg.K;
    const auto &dbg = s->db->h_graphs;
    int *h_queue = reinterpret_cast<int *>(b.h_in);
    WorkItem *h_work = reinterpret_cast<WorkItem *>(b.h_in + b.o_work);
    gedk::GatherItem *h_gather = reinterpret_cast<gedk::GatherItem *>(b.h_in + b.o_gather);
    GraphRec *h_recs = reinterpret_cast<GraphRec *>(b.h_in + b.o_recs);
    int32_t *h_vlab = reinterpret_cast<int32_t *>(b.h_in + b.o_var);
    // vertex labels first; the rows start at the next 256-byte boundary
    int64_t nv = 0;
    for (int k = 0; k < nq; ++k) nv += b.batch[(size_t)k]->n1;
    const size_t o_adj = align256(b.o_var + sizeof(int32_t) * (size_t)nv);
    uint32_t *h_adj = reinterpret_cast<uint32_t *>(b.h_in + o_adj);
    // stage query graphs and map offsets; a database query's words are
    // copied from the database on the device after the staged ones arrive
    int64_t aw = 0, vo = 0, mo = 0;
    int ngather = 0;
    b.map_off.resize((size_t)nq);
    for (int k = 0; k < nq; ++k) {
        const Request &r = *b.batch[(size_t)k];
        if (r.db_query >= 0) {
            const GraphRec &q = dbg[(size_t)r.db_query];
            h_gather[ngather++] = gedk::GatherItem{q.adj, aw, r.words, q.vlab, vo, (int64_t)r.n1};
        } else {
            std::memcpy(h_adj + aw, r.adj.data(), sizeof(uint32_t) * r.adj.size());
            std::memcpy(h_vlab + vo, r.vlab.data(), sizeof(int32_t) * r.vlab.size());
        }
        GraphRec rec = r.rec;
        rec.adj = aw;
        rec.vlab = vo;
        h_recs[k] = rec;
        b.map_off[(size_t)k] = mo;
        aw += r.words;
        vo += r.n1;
        mo += r.n1;
    }
    for (int k = 0; k < kMaxBins; ++k) h_queue[k] = 0;
    const gedk::DbView src{reinterpret_cast<const GraphRec *>(b.d_in + b.o_recs),
                           reinterpret_cast<const uint32_t *>(b.d_in + o_adj),
                           reinterpret_cast<const int32_t *>(b.d_in + b.o_var), s->db->planes};
    const gedk::DbView dst{s->db->d_graphs, s->db->d_adj, s->db->d_vlab, s->db->planes};
    int *d_queue = reinterpret_cast<int *>(b.d_in);
    const WorkItem *d_work = reinterpret_cast<const WorkItem *>(b.d_in + b.o_work);
    const gedk::Outputs out{b.d_out, b.d_out + nq, nullptr};
    // one copy of everything staged, then the gather of database queries
    auto stage = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(b.d_in, b.h_in, o_adj + sizeof(uint32_t) * (size_t)aw, hipMemcpyHostToDevice,
                                      b.stream);
        if (e == hipSuccess && ngather > 0)
            e = gedk::launch_gather_graphs(reinterpret_cast<const gedk::GatherItem *>(b.d_in + b.o_gather), ngather,
                                           s->db->d_adj, reinterpret_cast<uint32_t *>(b.d_in + o_adj), s->db->d_vlab,
                                           reinterpret_cast<int32_t *>(b.d_in + b.o_var), b.stream);
        return e;
    };
    // one copy of the results, then the batch's event
    auto finish = [&]() -> hipError_t {
        hipError_t e = hipMemcpyAsync(b.h_out, b.d_out, sizeof(int32_t) * (size_t)(nq + mo), hipMemcpyDeviceToHost,
                                      b.stream);
        if (e == hipSuccess) e = hipEventRecord(b.done, b.stream);
        return e;
    };
    // the bipartite method: one launch of the class's instantiation
    if (s->bip) {
        for (int k = 0; k < nq; ++k) {
            WorkItem wi;
            wi.src = k;
            wi.dst = b.batch[(size_t)k]->target;
            wi.out = k;
            wi.pad = 0;
            wi.map_off = b.map_off[(size_t)k];
            h_work[k] = wi;
        }
        const int cpl = b.cls + 1;
        const size_t per_wave = gedk::bip_workgroup_bytes(cpl, K);
        const int fit = (int)std::min<size_t>(b.ws_bytes / per_wave, (size_t)std::numeric_limits<int>::max());
        const int grid = std::min({nq, s->bip_per_cu[b.cls] * s->cus, fit});
        if (grid <= 0) return hipErrorOutOfMemory;
        hipError_t e = stage();
        if (e == hipSuccess)
            e = gedk::launch_bip(s->PL, cpl, 1, src, dst, d_work, nq, d_queue, s->c, K, b.d_ws, out, grid, b.stream);
        if (e == hipSuccess) e = finish();
        return e;
    }
    // work items by bin: 0, 1 = wavefront kernels (n <= 32, n <= 64),
    // kWaveBins + log2(W) = workgroup kernel
    std::vector<WorkItem> bins[kMaxBins];
    int nmax1[kMaxBins] = {0}, nmax2[kMaxBins] = {0};
    for (int k = 0; k < nq; ++k) {
        const Request &r = *b.batch[(size_t)k];
        const GraphRec &g2 = dbg[(size_t)r.target];
        const int ww = s->directed ? gedk::wave_words_for_directed(r.n1, g2.n, K) : gedk::wave_words_for(r.n1, g2.n, K);
        const int bin =
            ww > 0 ? ww - 1 : kWaveBins + w_index(pow2_at_least(std::max(1, g2.w)) * (s->directed ? 2 : 1));
        WorkItem wi;
        wi.src = k;
        wi.dst = r.target;
        wi.out = k;
        wi.pad = 0;
        wi.map_off = b.map_off[(size_t)k];
        bins[bin].push_back(wi);
        nmax1[bin] = std::max(nmax1[bin], r.n1);
        nmax2[bin] = std::max(nmax2[bin], g2.n);
    }
    int64_t wo = 0;
    int start[kMaxBins], grid[kMaxBins];
    gedk::BlockShape shape[kMaxBins];
    size_t stride[kMaxBins];
    for (int bin = 0; bin < kMaxBins; ++bin) {
        const int cnt = (int)bins[bin].size();
        start[bin] = (int)wo;
        grid[bin] = 0;
        if (cnt == 0) continue;
        std::stable_sort(bins[bin].begin(), bins[bin].end(), [&](const WorkItem &x, const WorkItem &y) {
            return (int64_t)h_recs[x.src].n * (dbg[(size_t)x.dst].n + 1) >
                   (int64_t)h_recs[y.src].n * (dbg[(size_t)y.dst].n + 1);
        });
        if (bin < kWaveBins) {
            // in a workgroup class, as many waves per CU as its workgroups would hold
            const int per_cu = b.cls < kFirstBlockClass ? s->wave_per_cu[bin]
                                                        : std::min(s->wave_per_cu[bin], 4 * kBlockClassPerCu[b.cls]);
            grid[bin] = std::min(cnt, per_cu * s->cus);
        } else {
            // 512-thread workgroups when the bin cannot put two workgroups on
            // every CU: two waves per SIMD on each pair instead of one
            const int wide = cnt < 2 * s->cus ? 1 : 0;
            shape[bin] = shape_for(s, 1 << (bin - kWaveBins), nmax1[bin], nmax2[bin],
                                   wide ? gedk::kBlockThreadsWide : gedk::kBlockThreads);
            stride[bin] = gedk::block_workspace_bytes(shape[bin]);
            const int fit = (int)std::min<size_t>(b.ws_bytes / stride[bin], (size_t)std::numeric_limits<int>::max());
            // the workgroup classes hold at most kBlockClassPerCu[class]
            // workgroups per CU: a batch of large queries at full occupancy
            // would fill every SIMD's registers for tens of milliseconds and
            // keep the small and mid classes' waves off the device
            const int per_cu = std::min(s->block_per_cu[wide][bin - kWaveBins], kBlockClassPerCu[b.cls]);
            grid[bin] = std::min({cnt, per_cu * s->cus, fit});
            if (grid[bin] <= 0) return hipErrorOutOfMemory;
        }
        gedh::deal_alternating(bins[bin], grid[bin], bin < kWaveBins ? 4 * (int64_t)s->cus : (int64_t)s->cus);
        for (const WorkItem &wi : bins[bin]) h_work[wo++] = wi;
    }
    hipError_t e = stage();
    for (int bin = 0; bin < kMaxBins && e == hipSuccess; ++bin) {
        const int cnt = (int)bins[bin].size();
        if (cnt == 0) continue;
        if (bin < kWaveBins) {
            e = gedk::launch_wave_family(bin + 1, s->PL, src, dst, d_work + start[bin], cnt, d_queue + bin, s->c, K, 0,
                                         out, grid[bin], b.stream, s->directed ? 1 : 0);
        } else {
            e = gedk::launch_block(shape[bin], src, dst, d_work + start[bin], cnt, d_queue + bin, s->c, K, 0, b.d_ws,
                                   stride[bin], out, grid[bin], b.stream);
        }
    }
    if (e == hipSuccess) e = finish();
    return e;
}

// Called with s->mu held: results of a finished (or failed) batch.
void finish_batch(ged_server *s, Slab &b, bool failed) {
    const int64_t t = now_ns();
    for (size_t k = 0; k < b.batch.size(); ++k) {
        Request &r = *b.batch[k];
        r.t_done = t;
        s->done_order.push_back(r.ticket);
        if (failed) {
            r.state = FAILED;
        } else {
            const int32_t *maps = b.h_out + b.batch.size();
            r.dist = b.h_out[k];
            r.map.assign(maps + b.map_off[k], maps + b.map_off[k] + r.n1);
            r.state = DONE;
            r.adj.clear();
            r.adj.shrink_to_fit();
            r.vlab.clear();
            r.vlab.shrink_to_fit();
        }
    }
    // tickets taken with poll/wait stay in done_order until collect skips
    // them; keep the list within a constant factor of the live tickets
    if (s->done_order.size() > 2 * s->tickets.size() + 4096) {
        std::deque<uint64_t> live;
        for (uint64_t id : s->done_order)
            if (s->tickets.count(id)) live.push_back(id);
        s->done_order.swap(live);
    }
    s->stats.completed += (int64_t)b.batch.size();
    s->stats.inflight -= (int64_t)b.batch.size();
    b.batch.clear();
    b.busy = false;
}

void worker_loop(ged_server *s) {
    (void)hipSetDevice(s->device);
    std::unique_lock<std::mutex> lk(s->mu);
    for (;;) {
        // 1. completions
        bool any_busy = false;
        for (Slab &b : s->slabs) {
            if (!b.busy) continue;
            const hipError_t q = hipEventQuery(b.done);
            if (q == hipSuccess) {
                finish_batch(s, b, false);
                s->cv_done.notify_all();
            } else if (q != hipErrorNotReady) {
                (void)hipStreamSynchronize(b.stream);
                finish_batch(s, b, true);
                s->cv_done.notify_all();
            } else {
                any_busy = true;
            }
        }
        if (s->stop) {
            for (auto &q : s->queue) {
                for (ReqPtr &r : q) r->state = CANCELED;
                q.clear();
            }
            s->queued_total = 0;
            s->stats.queued = 0;
            s->cv_done.notify_all();
            if (!any_busy) break;
        }
        // 2. admission and launch: each idle stream takes from its class's queue.
        // A class with a batch on the device launches another only once the
        // queue holds a batch worth the launch (kFillQueries) or its oldest
        // query has waited kHoldNs: many tiny launches would cost more host
        // time per query than the device time they save.
        bool launched = false;
        if (!s->stop && s->queued_total > 0) {
            int class_busy[kClasses] = {0, 0, 0, 0};
            for (const Slab &b : s->slabs) class_busy[b.cls] += b.busy ? 1 : 0;
            const int64_t now = now_ns();
            for (Slab &b : s->slabs) {
                std::deque<ReqPtr> &queue = s->queue[b.cls];
                if (b.busy || queue.empty()) continue;
                if (s->stats.inflight >= s->cfg.max_inflight) break;
                if (class_busy[b.cls] > 0 && (int64_t)queue.size() < std::min<int64_t>(kFillQueries, s->cfg.max_batch) &&
                    now - queue.front()->t_submit < kHoldNs)
                    continue;
                int64_t aw = 0, vo = 0;
                while (!queue.empty() && (int)b.batch.size() < s->cfg.max_batch &&
                       s->stats.inflight + (int64_t)b.batch.size() < s->cfg.max_inflight) {
                    const Request &r = *queue.front();
                    if (aw + r.words > b.cap_words || vo + r.n1 > b.cap_vlab) break;
                    aw += r.words;
                    vo += r.n1;
                    queue.front()->state = INFLIGHT;
                    b.batch.push_back(queue.front());
                    queue.pop_front();
                }
                if (b.batch.empty()) continue;
                b.busy = true;
                class_busy[b.cls] += 1;
                s->queued_total -= (int64_t)b.batch.size();
                s->stats.queued = s->queued_total;
                s->stats.inflight += (int64_t)b.batch.size();
                s->stats.inflight_peak = std::max(s->stats.inflight_peak, s->stats.inflight);
                s->stats.batch_peak = std::max(s->stats.batch_peak, (int64_t)b.batch.size());
                s->stats.launches += 1;
                lk.unlock();
                const hipError_t e = launch_batch(s, b);
                lk.lock();
                if (e != hipSuccess) {
                    (void)hipStreamSynchronize(b.stream);
                    finish_batch(s, b, true);
                    s->cv_done.notify_all();
                }
                launched = true;
                any_busy = true;
            }
        }
        if (launched) continue;
        // 3. wait for work or poll the device
        if (any_busy) {
            s->cv_work.wait_for(lk, std::chrono::microseconds(20));
        } else {
            s->cv_work.wait(lk, [&] { return s->stop || s->queued_total > 0; });
        }
    }
}

}  // namespace

extern "C" {

ged_status ged_server_create(ged_db *db, const ged_server_config *config, ged_server **out) {
    if (!out) return fail(GED_EINVAL, "out is NULL");
    *out = nullptr;
    if (!db || !config) return fail(GED_EINVAL, "NULL argument");
    ged_server_config cfg = *config;
    if (cfg.K < 1) return fail(GED_EINVAL, "K must be >= 1 (got %d)", cfg.K);
    if (cfg.K > GED_MAX_K) return fail(GED_EUNSUPPORTED, "K = %d exceeds %d", cfg.K, GED_MAX_K);
    ged_status st = gedh::check_costs(cfg.costs);
    if (st != GED_OK) return st;
    if (cfg.hbm_budget < 0 || cfg.max_inflight < 0 || cfg.max_batch < 0 || cfg.streams < 0 || cfg.queue_capacity < 0)
        return fail(GED_EINVAL, "negative server limit");
    if (cfg.hbm_budget == 0) cfg.hbm_budget = (int64_t)2 << 30;
    if (cfg.max_inflight == 0) cfg.max_inflight = 4096;
    if (cfg.max_batch == 0) cfg.max_batch = 1024;
    if (cfg.streams == 0) cfg.streams = 1;
    if (cfg.queue_capacity == 0) cfg.queue_capacity = 1 << 20;
    if (cfg.streams > 4) return fail(GED_EINVAL, "streams (per size class) must be 1..4");
    if (cfg.method != GED_METHOD_TREE && cfg.method != GED_METHOD_BIPARTITE)
        return fail(GED_EINVAL, "unknown method %d", cfg.method);
    if (cfg.method == GED_METHOD_BIPARTITE && cfg.K > GED_BIP_MAX_K)
        return fail(GED_EUNSUPPORTED, "K = %d exceeds the bipartite method's %d", cfg.K, GED_BIP_MAX_K);
    if (cfg.method == GED_METHOD_BIPARTITE && db->directed)
        return fail(GED_EUNSUPPORTED, "the bipartite method takes undirected graphs only");
    st = gedh::check_device(db);
    if (st != GED_OK) return st;

    ged_server *s = new (std::nothrow) ged_server;
    if (!s) return fail(GED_ENOMEM, "host allocation failed");
    s->db = db;
    s->cfg = cfg;
    s->c = gedk::Costs{cfg.costs.vsub, cfg.costs.vdel, cfg.costs.vins, cfg.costs.esub, cfg.costs.edel, cfg.costs.eins};
    s->PL = db->planes == 0 ? 0 : (db->planes <= 2 ? 2 : 4);
    s->device = db->device;
    s->bip = cfg.method == GED_METHOD_BIPARTITE;
    s->directed = db->directed;
    hipError_t e = hipDeviceGetAttribute(&s->cus, hipDeviceAttributeMultiprocessorCount, s->device);
    const bool wave_classes = !s->bip && cfg.K <= gedk::kWave2MaxK;
    for (int k = 0; k < kWaveBins && e == hipSuccess && wave_classes; ++k)
        e = gedk::wave_family_max_resident(k + 1, s->PL, cfg.K, 0, &s->wave_per_cu[k], s->directed ? 1 : 0);
    // classes that can receive a query get streams: a directed database and a
    // beam above 64 slots have no one-word class (their pairs of up to 32
    // vertices take the two-word kernel)
    const int first_class =
        s->bip ? 0 : (wave_classes ? ((s->directed || cfg.K > gedk::kWaveMaxK) ? 1 : 0) : kFirstBlockClass);
    // streams per class: the configured number, and kLargeStreams times it for
    // the tree search's large class, whose batches last as long as their
    // slowest pair (tens of milliseconds): more of them in flight keep its
    // CUs busy while a batch's last pairs finish
    int nstr[kClasses];
    int nslabs = 0;
    for (int cls = 0; cls < kClasses; ++cls) {
        nstr[cls] = cls < first_class ? 0 : cfg.streams * ((!s->bip && cls == kClasses - 1) ? kLargeStreams : 1);
        nslabs += nstr[cls];
    }
    // every stream gets an equal share of the budget: its class's workspace
    // (at most half of the share; fewer resident workgroups when smaller),
    // then the arena
    const int64_t per_stream = cfg.hbm_budget / nslabs;
    size_t ws_class[kClasses] = {0, 0, 0, 0};
    // directed: class 0 takes no pair, class 1 the pairs of up to 32 vertices, class 3 up to 256
    const int max_n[kClasses] = {s->bip ? 64 : gedk::kWaveMaxN,
                                 s->bip ? 128 : (s->directed ? gedk::kWaveMaxN : gedk::kWave2MaxN),
                                 s->bip ? 192 : kMediumMaxN,
                                 s->bip ? 256 : (s->directed ? GED_DIRECTED_MAX_ORDER : GED_MAX_VERTICES_BATCH)};
    // bipartite classes: one queue slice per resident wave, at most half the share
    for (int cls = 0; cls < kClasses && e == hipSuccess && s->bip; ++cls) {
        e = gedk::bip_max_resident(s->PL, cls + 1, cfg.K, 1, &s->bip_per_cu[cls]);
        const size_t per_wave = gedk::bip_workgroup_bytes(cls + 1, cfg.K);
        const int64_t grid = std::min<int64_t>((int64_t)cfg.max_batch, (int64_t)s->bip_per_cu[cls] * s->cus);
        size_t ws = std::min<size_t>(per_wave * (size_t)grid, (size_t)std::max<int64_t>(per_stream / 2, 0));
        if (e == hipSuccess && ws < per_wave) {
            delete s;
            return fail(GED_ENOMEM, "hbm_budget %lld is too small: a stream needs %zu bytes for one wave's queue",
                        (long long)cfg.hbm_budget, per_wave);
        }
        ws_class[cls] = ws;
    }
    for (int cls = kFirstBlockClass; cls < kClasses && e == hipSuccess && !s->bip; ++cls) {
        size_t ws = 0, one_block = 0;
        // rows of W words cover 32 W vertices, or 16 W for a directed graph (out and in halves)
        const int per_word = s->directed ? 16 : 32;
        for (int k = s->directed ? 1 : 0; k < 5 && e == hipSuccess; ++k) {
            const int W = 1 << k;
            if (W > (s->directed ? 2 : 1) && per_word * W / 2 >= max_n[cls]) break;   // W / 2 words already cover it
            for (int wide = 0; wide < 2 && e == hipSuccess; ++wide) {
                const gedk::BlockShape sh = shape_for(s, W, max_n[cls], std::min(per_word * W, max_n[cls]),
                                                      wide ? gedk::kBlockThreadsWide : gedk::kBlockThreads);
                e = gedk::block_max_resident(sh, &s->block_per_cu[wide][k]);
                const int64_t grid =
                    std::min<int64_t>((int64_t)cfg.max_batch, (int64_t)s->block_per_cu[wide][k] * s->cus);
                one_block = std::max(one_block, gedk::block_workspace_bytes(sh));
                ws = std::max(ws, gedk::block_workspace_bytes(sh) * (size_t)grid);
            }
        }
        ws = std::min<size_t>(ws, (size_t)std::max<int64_t>(per_stream / 2, 0));
        if (e == hipSuccess && ws < one_block) {
            delete s;
            return fail(GED_ENOMEM, "hbm_budget %lld is too small: a stream needs %zu bytes for one workgroup's "
                                    "workspace", (long long)cfg.hbm_budget, one_block);
        }
        ws_class[cls] = ws;
    }
    if (e != hipSuccess) {
        delete s;
        return fail(GED_EDEVICE, "device query failed: %s", hipGetErrorString(e));
    }
    // arena of a stream: what its share leaves after the workspace, at most a
    // full batch of the class's largest queries (and 64 MiB of graph words)
    int64_t cap_words[kClasses], cap_vlab[kClasses];
    for (int cls = first_class; cls < kClasses; ++cls) {
        const int64_t fixed = (int64_t)ws_class[cls] +
                              (int64_t)cfg.max_batch * (int64_t)(sizeof(GraphRec) + sizeof(WorkItem) + 4 +
                                                                 sizeof(gedk::GatherItem)) + kMaxBins * 4;
        const int64_t rest = per_stream - fixed;
        const int64_t big = gedh::packed_words(max_n[cls], db->planes, s->directed);
        cap_words[cls] = std::min({rest / 4 * 8 / 10, (int64_t)cfg.max_batch * big, (int64_t)16 << 20});
        cap_vlab[cls] = std::min(rest / 4 / 20, (int64_t)cfg.max_batch * max_n[cls]);
        if (rest <= 0 || cap_words[cls] < big || cap_vlab[cls] < max_n[cls]) {
            delete s;
            return fail(GED_ENOMEM, "hbm_budget %lld is too small: each of %d streams needs %lld bytes of workspace "
                                    "plus room for one %d-vertex query", (long long)cfg.hbm_budget, nslabs,
                        (long long)fixed, max_n[cls]);
        }
    }
    s->slabs.resize((size_t)nslabs);
    for (int k = 0, cls = first_class, left = nstr[first_class]; k < nslabs; ++k, --left) {
        while (left == 0) left = nstr[++cls];
        Slab &b = s->slabs[(size_t)k];
        b.cls = cls;
        b.ws_bytes = ws_class[b.cls];
        b.cap_words = cap_words[b.cls];
        b.cap_vlab = cap_vlab[b.cls];
        e = hipStreamCreate(&b.stream);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        const size_t nb = (size_t)cfg.max_batch;
        b.o_work = align256(sizeof(int) * kMaxBins);
        b.o_gather = b.o_work + align256(sizeof(WorkItem) * nb);
        b.o_recs = b.o_gather + align256(sizeof(gedk::GatherItem) * nb);
        b.o_var = b.o_recs + align256(sizeof(GraphRec) * nb);
        b.in_bytes = b.o_var + align256(sizeof(int32_t) * (size_t)b.cap_vlab) + sizeof(uint32_t) * (size_t)b.cap_words;
        const size_t out_bytes = sizeof(int32_t) * (nb + (size_t)b.cap_vlab);
        if (e == hipSuccess) e = hipMalloc((void **)&b.d_in, b.in_bytes);
        if (e == hipSuccess) e = hipMalloc((void **)&b.d_out, out_bytes);
        if (e == hipSuccess && b.ws_bytes > 0) e = hipMalloc(&b.d_ws, b.ws_bytes);
        if (e == hipSuccess) e = hipHostMalloc((void **)&b.h_in, b.in_bytes, hipHostMallocDefault);
        if (e == hipSuccess) e = hipHostMalloc((void **)&b.h_out, out_bytes, hipHostMallocDefault);
        if (e != hipSuccess) break;
        s->device_bytes += (int64_t)(b.in_bytes + out_bytes + b.ws_bytes);
    }
    if (e != hipSuccess) {
        for (Slab &b : s->slabs) free_slab(b);
        delete s;
        return fail(GED_ENOMEM, "server allocation failed: %s", hipGetErrorString(e));
    }
    s->stats.device_bytes = s->device_bytes;
    s->worker = std::thread(worker_loop, s);
    *out = s;
    return ok();
}

// Limits and the overflow bound of query r (n1 = r->n1, m1 edges) against
// its target; sets its class.
static ged_status admit_pair(ged_server *srv, Request *r, int32_t m1) {
    const GraphRec &g2 = srv->db->h_graphs[(size_t)r->target];
    const int n1 = r->n1;
    if (srv->directed && std::max(n1, g2.n) > GED_DIRECTED_MAX_ORDER)
        return fail(GED_EUNSUPPORTED, "directed graphs of more than %d vertices", GED_DIRECTED_MAX_ORDER);
    if (srv->bip && n1 + g2.n > GED_BIP_MAX_ORDER)
        return fail(GED_EUNSUPPORTED, "n1 + n2 = %d exceeds the bipartite method's %d", n1 + g2.n,
                    GED_BIP_MAX_ORDER);
    if (std::max(n1, g2.n) > GED_MAX_VERTICES_BATCH)
        return fail(GED_EUNSUPPORTED, "a graph of %d vertices exceeds the server's %d", std::max(n1, g2.n),
                    GED_MAX_VERTICES_BATCH);
    r->cls = server_class(srv, n1, g2.n);
    const ged_costs &c = srv->cfg.costs;
    const int64_t vmax = std::max({(int64_t)c.vsub, (int64_t)c.vdel, (int64_t)c.vins});
    const int64_t emax = std::max({(int64_t)c.esub, (int64_t)c.edel, (int64_t)c.eins});
    if (vmax * ((int64_t)n1 + g2.n) + emax * ((int64_t)m1 + g2.m) > (int64_t)std::numeric_limits<int32_t>::max() - 1)
        return fail(GED_EINVAL, "costs may overflow int32 on this pair");
    // the bipartite solver's bound (as for plans): (n1 + n2 + 1) entries below 2^24
    const int64_t order = (int64_t)n1 + g2.n;
    if (srv->bip && (order + 1) * (2 * vmax + 4 * emax * order) >= ((int64_t)1 << 24))
        return fail(GED_EINVAL, "costs may overflow the bipartite solver on this pair");
    return ok();
}

static ged_status enqueue(ged_server *srv, std::shared_ptr<Request> r, uint64_t *ticket);

ged_status ged_server_submit(ged_server *srv, const ged_graph *query, int64_t target_id, uint64_t *ticket) {
    if (!srv || !query || !ticket) return fail(GED_EINVAL, "NULL argument");
    if (target_id < 0 || target_id >= srv->db->count) return fail(GED_EINVAL, "target id %lld out of range", (long long)target_id);
    ged_status st = gedh::check_graph_shape(*query, 0, srv->directed);
    if (st != GED_OK) return st;
    auto r = std::make_shared<Request>();
    r->n1 = query->n;
    r->target = (int32_t)target_id;
    st = gedh::pack_graph(*query, 0, srv->db->elabels, srv->db->planes, r->adj, r->vlab, r->rec, srv->directed);
    if (st != GED_OK) return st;
    r->words = (int64_t)r->adj.size();
    st = admit_pair(srv, r.get(), query->m);
    if (st != GED_OK) return st;
    return enqueue(srv, std::move(r), ticket);
}

ged_status ged_server_submit_id(ged_server *srv, int64_t query_id, int64_t target_id, uint64_t *ticket) {
    if (!srv || !ticket) return fail(GED_EINVAL, "NULL argument");
    if (query_id < 0 || query_id >= srv->db->count) return fail(GED_EINVAL, "query id %lld out of range", (long long)query_id);
    if (target_id < 0 || target_id >= srv->db->count) return fail(GED_EINVAL, "target id %lld out of range", (long long)target_id);
    const GraphRec &q = srv->db->h_graphs[(size_t)query_id];
    auto r = std::make_shared<Request>();
    r->n1 = q.n;
    r->target = (int32_t)target_id;
    r->db_query = query_id;
    r->rec = q;
    r->words = gedh::packed_words(q.n, srv->db->planes, srv->directed);
    ged_status st = admit_pair(srv, r.get(), q.m);
    if (st != GED_OK) return st;
    return enqueue(srv, std::move(r), ticket);
}

static ged_status enqueue(ged_server *srv, std::shared_ptr<Request> r, uint64_t *ticket) {
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        if (srv->stop) return fail(GED_ECANCELED, "server is shutting down");
        if (srv->queued_total >= srv->cfg.queue_capacity) {
            srv->stats.rejected_busy += 1;
            return fail(GED_EBUSY, "queue full (%d queued)", srv->cfg.queue_capacity);
        }
        r->ticket = srv->next_ticket++;
        r->t_submit = now_ns();
        srv->tickets[r->ticket] = r;
        srv->queue[r->cls].push_back(r);
        srv->queued_total += 1;
        srv->stats.submitted += 1;
        srv->stats.queued = srv->queued_total;
        *ticket = r->ticket;
    }
    srv->cv_work.notify_one();
    return ok();
}

static ged_status take_result(ged_server *srv, std::unordered_map<uint64_t, ReqPtr>::iterator it, int32_t *dist,
                              int32_t *map, int32_t map_capacity, int32_t *n1, int64_t *times_ns) {
    Request &r = *it->second;
    if (times_ns) {
        times_ns[0] = r.t_submit;
        times_ns[1] = r.t_done;
    }
    if (r.state == FAILED) {
        srv->tickets.erase(it);
        return fail(GED_EDEVICE, "the query's launch failed");
    }
    if (r.state == CANCELED) {
        srv->tickets.erase(it);
        return fail(GED_ECANCELED, "the server was destroyed before the query ran");
    }
    if (r.state != DONE) return GED_EBUSY;
    if (map_capacity < r.n1 || (r.n1 > 0 && !map)) return fail(GED_EINVAL, "map capacity %d < n1 = %d", map_capacity, r.n1);
    if (dist) *dist = r.dist;
    if (n1) *n1 = r.n1;
    if (r.n1 > 0) std::memcpy(map, r.map.data(), sizeof(int32_t) * (size_t)r.n1);
    srv->tickets.erase(it);
    return ok();
}

ged_status ged_server_poll(ged_server *srv, uint64_t ticket, int32_t *dist, int32_t *map, int32_t map_capacity,
                           int32_t *n1, int64_t *times_ns) {
    if (!srv) return fail(GED_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(GED_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    return take_result(srv, it, dist, map, map_capacity, n1, times_ns);
}

ged_status ged_server_wait(ged_server *srv, uint64_t ticket, int64_t timeout_us, int32_t *dist, int32_t *map,
                           int32_t map_capacity, int32_t *n1, int64_t *times_ns) {
    if (!srv) return fail(GED_EINVAL, "server is NULL");
    std::unique_lock<std::mutex> lk(srv->mu);
    auto it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(GED_EINVAL, "unknown ticket %llu", (unsigned long long)ticket);
    ReqPtr r = it->second;
    auto ready = [&] { return r->state != QUEUED && r->state != INFLIGHT; };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(GED_ETIMEOUT, "query not finished after %lld us", (long long)timeout_us);
    }
    it = srv->tickets.find(ticket);
    if (it == srv->tickets.end()) return fail(GED_EINVAL, "ticket %llu was taken by another caller", (unsigned long long)ticket);
    return take_result(srv, it, dist, map, map_capacity, n1, times_ns);
}

ged_status ged_server_submit_batch(ged_server *srv, const ged_graph *queries, const int64_t *targets,
                                   int64_t count, uint64_t *tickets, int64_t *accepted) {
    if (!srv || !accepted || (count > 0 && (!queries || !targets || !tickets))) return fail(GED_EINVAL, "NULL argument");
    *accepted = 0;
    for (int64_t k = 0; k < count; ++k) {
        const ged_status st = ged_server_submit(srv, &queries[k], targets[k], &tickets[k]);
        if (st != GED_OK) return st;
        *accepted = k + 1;
    }
    return ok();
}

ged_status ged_server_collect(ged_server *srv, int64_t timeout_us, int64_t max_count, uint64_t *tickets,
                              int32_t *dist, int64_t *times_ns, int32_t *maps, int64_t maps_capacity,
                              int64_t *count) {
    if (!srv || !tickets || !dist || !times_ns || !count || max_count < 1) return fail(GED_EINVAL, "bad argument");
    *count = 0;
    std::unique_lock<std::mutex> lk(srv->mu);
    auto ready = [&] {
        while (!srv->done_order.empty() && !srv->tickets.count(srv->done_order.front())) srv->done_order.pop_front();
        return !srv->done_order.empty();
    };
    if (timeout_us < 0) {
        srv->cv_done.wait(lk, ready);
    } else if (!srv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return fail(GED_ETIMEOUT, "no query finished within %lld us", (long long)timeout_us);
    }
    int64_t n = 0, mo = 0;
    while (n < max_count && !srv->done_order.empty()) {
        const uint64_t t = srv->done_order.front();
        auto it = srv->tickets.find(t);
        if (it == srv->tickets.end()) {   // already taken with poll/wait
            srv->done_order.pop_front();
            continue;
        }
        Request &r = *it->second;
        if (maps && mo + r.n1 > maps_capacity) break;
        srv->done_order.pop_front();
        tickets[n] = t;
        dist[n] = r.state == DONE ? r.dist : -1;
        times_ns[2 * n] = r.t_submit;
        times_ns[2 * n + 1] = r.t_done;
        if (maps && r.state == DONE && r.n1 > 0) std::memcpy(maps + mo, r.map.data(), sizeof(int32_t) * (size_t)r.n1);
        if (maps) mo += r.n1;
        srv->tickets.erase(it);
        ++n;
    }
    *count = n;
    return ok();
}

ged_status ged_server_stats_get(const ged_server *srv, ged_server_stats *out) {
    if (!srv || !out) return fail(GED_EINVAL, "NULL argument");
    ged_server *s = const_cast<ged_server *>(srv);
    std::lock_guard<std::mutex> lk(s->mu);
    *out = s->stats;
    return ok();
}

ged_status ged_server_destroy(ged_server *srv) {
    if (!srv) return ok();
    {
        std::lock_guard<std::mutex> lk(srv->mu);
        srv->stop = true;
    }
    srv->cv_work.notify_all();
    if (srv->worker.joinable()) srv->worker.join();
    for (Slab &b : srv->slabs) {
        if (b.stream) (void)hipStreamSynchronize(b.stream);
        free_slab(b);
    }
    delete srv;
    return ok();
}

}  // extern "C"
