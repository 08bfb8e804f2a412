/*
 * ged.h -- C ABI of the MI355X (gfx950) K-Best graph edit distance library.
 *
 * The library computes, for many pairs of labelled graphs at once, the
 * K-Best approximation of the graph edit distance (GED) described in
 * "Efficient Accelerated Graph Edit Distance Computation on GPU" (Dabah and
 * Herten): a level-by-level search over vertex mappings of the source graph
 * g1 onto the target graph g2 that keeps the K children of least partial
 * edit distance at every level (Alg. 1; branching Sec. 4.2.1, evaluation by
 * implied edge operations Sec. 2.3 and Alg. 2, selection Sec. 4.3), inserts
 * the unmatched target vertices at the end (Sec. 4.4.1) and returns the
 * cheapest complete edit path: an upper bound of the exact GED (Sec. 2.2).
 *
 * Conventions
 *   - Every function returns a ged_status.  Nothing aborts or throws across
 *     the ABI.  On failure ged_last_error() returns a message describing the
 *     most recent failure on the calling thread.
 *   - Pointers named h_* or documented as "host" are host memory owned by the
 *     caller; the library copies what it keeps before returning.
 *   - Pointers named d_* are device memory on the current HIP device,
 *     allocated and owned by the caller (for example torch tensors'
 *     data_ptr()).  Results written there are valid once the given HIP stream
 *     has been synchronized.
 *   - `stream` is a hipStream_t passed as void* (NULL = the null stream).
 *   - Graphs are undirected and simple (Sec. 2.1): no self-loops, no repeated
 *     edge; a database created with GED_DB_DIRECTED holds directed graphs
 *     instead (see ged_db_create_ex).  Vertex and edge labels are int32
 *     values compared for equality only (Sec. 2.4).
 *   - Costs are non-negative int32 (Sec. 2.4; the paper's default setting is
 *     vsub 2, vdel 4, vins 4, esub 1, edel 2, eins 2, Sec. 5).  A substitution
 *     costs 0 when the two labels are equal.  All arithmetic is exact int32.
 *
 * Readings fixed by this library where the paper leaves a choice open:
 *   - g1's vertices are edited in index order 0..n1-1 (the loop of Alg. 1).
 *   - A node's children are the substitutions by each unused g2 vertex in
 *     ascending index order, followed by the deletion (Sec. 4.2.1).
 *   - When several children share the K-th smallest partial edit distance,
 *     those generated first (parent by parent in beam order, then in child
 *     order) take the remaining places.  The surviving beam keeps
 *     generation order.  This makes every result deterministic.
 *   - Selection happens at every level including the last; insertion costs
 *     are added afterwards (Sec. 4.4.1); among leaves of equal total cost the
 *     first in beam order is returned.
 */
#ifndef GED_H
#define GED_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GED_ABI_VERSION 6

/* Limits of this version. */
#define GED_MAX_VERTICES 1024     /* per graph: databases, the single-pair search, edit paths */
#define GED_MAX_VERTICES_BATCH 512  /* per graph of a pair: batched plans, the per-pair path, serving */
#define GED_MAX_K 1024            /* beam width (batched plans, serving) */
#define GED_MAX_K_WIDE (1 << 21)  /* beam width of the single-pair large-K search */
#define GED_MAX_EDGE_LABELS 16    /* distinct edge labels in one database */
#define GED_BIP_MAX_ORDER 256     /* n1 + n2 of a pair, bipartite method */
#define GED_BIP_MAX_K 256         /* K of the bipartite method */

typedef enum {
    GED_OK = 0,
    GED_EINVAL = 1,        /* an argument or a graph violates the contract */
    GED_ENOMEM = 2,        /* host or device allocation failed */
    GED_EUNSUPPORTED = 3,  /* valid input beyond this version's limits */
    GED_EDEVICE = 4,       /* a HIP runtime call failed */
    GED_EBUSY = 5,
    GED_ETIMEOUT = 6,
    GED_ECANCELED = 7
} ged_status;

/* Edit operation costs (Sec. 2.4).  All must be >= 0. */
typedef struct {
    int32_t vsub, vdel, vins;  /* vertex substitution (labels differ), deletion, insertion */
    int32_t esub, edel, eins;  /* edge substitution (labels differ), deletion, insertion */
} ged_costs;

/* One graph G = (V, E, alpha, beta) (Sec. 2.1), host memory.
 * Vertices are 0..n-1.  vlabel[n] holds alpha.  Edge k joins eu[k] and ev[k]
 * (0 <= eu, ev < n, eu != ev, each unordered pair at most once); elabel[k]
 * is beta(e_k), or elabel == NULL when every edge has label 0. */
typedef struct {
    int32_t n, m;
    const int32_t *vlabel;
    const int32_t *eu;
    const int32_t *ev;
    const int32_t *elabel;
} ged_graph;

/* A pair of database graph ids: src is g1 (edited), dst is g2 (target). */
typedef struct {
    int64_t src, dst;
} ged_pair;

typedef struct ged_db ged_db;
typedef struct ged_plan ged_plan;

/* GED_ABI_VERSION of the loaded library. */
int32_t ged_abi_version(void);

/* Message for the most recent failure on this thread ("" if none).  The
 * string is owned by the library and valid until the next call on the same
 * thread. */
const char *ged_last_error(void);

/* Static name of a status code ("GED_OK", ...). */
const char *ged_status_name(int32_t status);

/* ------------------------------------------------------------------------
 * Device-resident graph database.
 *
 * ged_db_create validates `count` graphs (host memory, see ged_graph), packs
 * them into adjacency bitsets plus edge-label bit planes and copies them to
 * the current HIP device (synchronously).  The caller may free its arrays
 * once it returns.  Edge labels are re-coded database-wide; at most
 * GED_MAX_EDGE_LABELS distinct edge labels per database.
 * Errors: GED_EINVAL (count < 0, NULL pointers with n/m > 0, negative n or m,
 * vertex ids out of range, self-loop, repeated edge); GED_EUNSUPPORTED
 * (n > GED_MAX_VERTICES, too many edge labels); GED_ENOMEM; GED_EDEVICE.
 * On success *out owns device memory until ged_db_destroy.
 * ---------------------------------------------------------------------- */
ged_status ged_db_create(const ged_graph *graphs, int64_t count, ged_db **out);

/* Database flags.
 * GED_DB_DIRECTED: every graph is directed.  Edge k of a ged_graph is then
 * the arc eu[k] -> ev[k] (eu != ev, each ordered pair at most once, so a
 * pair of vertices may carry both arcs, with labels of their own; m <=
 * n(n-1)), and every arc is one edit operation: the implied operations of
 * Sec. 2.3 between the edited vertex and each earlier one are taken for
 * both arc directions.  A directed database serves the tree search
 * (ged_plan_create, ged_plan_create_ex with GED_METHOD_TREE, ged_kbest,
 * ged_kbest_perpair) and the server (ged_server_create; its queries are
 * then directed graphs too) for graphs of at most GED_DIRECTED_MAX_ORDER
 * vertices, and ged_edit_path; ged_wide_create and the bipartite method
 * return GED_EUNSUPPORTED for it. */
#define GED_DB_DIRECTED 1u
#define GED_DIRECTED_MAX_ORDER 256

/* ged_db_create with flags (0 or GED_DB_DIRECTED).  Errors as ged_db_create;
 * GED_EINVAL also for unknown flag bits. */
ged_status ged_db_create_ex(const ged_graph *graphs, int64_t count, uint32_t flags, ged_db **out);
/* The flags the database was created with. */
ged_status ged_db_flags(const ged_db *db, uint32_t *flags);
ged_status ged_db_destroy(ged_db *db);
ged_status ged_db_count(const ged_db *db, int64_t *count);
ged_status ged_db_device_bytes(const ged_db *db, int64_t *bytes);
/* n of graph `id` (host query), for sizing mapping outputs. */
ged_status ged_db_order(const ged_db *db, int64_t id, int32_t *n);

/* ------------------------------------------------------------------------
 * Batched K-Best search (Alg. 1 for every pair of a batch).
 *
 * ged_plan_create validates a batch of pairs (host array h_pairs[npairs],
 * ids in [0, count)) and the beam width K (1 <= K <= GED_MAX_K), bins the
 * pairs by size, orders each bin longest-first, uploads the work lists and
 * allocates the device workspace; the plan can then be run any number of
 * times (for example inside a captured HIP graph: ged_plan_run enqueues only
 * kernels).  The plan keeps a pointer to db, which must outlive it.
 *
 * ged_plan_run enqueues the search on `stream` and writes
 *   d_dist[p]  (int32 [npairs]) the K-Best distance of pair p;
 *   d_map[off(p) + v] (int32 [sum of n(src)]) the target vertex of source
 *              vertex v on the returned edit path, or -1 if v is deleted;
 *              off(p) = sum of n(src) over the pairs before p (caller order);
 *              target vertices absent from the mapping are inserted;
 *   d_cand[p]  (int64 [npairs], optional, NULL to skip) the number of
 *              children whose partial edit distance the search evaluated
 *              (sum over levels of the candidate count).
 * Errors (host-side, nothing enqueued): GED_EINVAL (negative cost, NULL
 * output with npairs > 0, costs that could overflow int32 on some pair of
 * the plan); GED_EDEVICE (launch failure).
 * ged_plan_create errors: GED_EINVAL (a graph id out of range, K < 1);
 * GED_EUNSUPPORTED (K > GED_MAX_K, a pair with a graph of more than
 * GED_MAX_VERTICES_BATCH vertices -- the single-pair search ged_wide_*
 * takes those); with GED_PLAN_PAIR_STATUS the per-pair ones become
 * statuses of their pairs instead.
 * ---------------------------------------------------------------------- */
ged_status ged_plan_create(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K,
                           ged_plan **out);

/* Kernel schedules.  GED_SCHED_AUTO lets the library choose per size bin:
 * a wavefront per pair (beam in registers) where n2 <= 64, n1 <= 128 and
 * K <= 128 (one kernel for n <= 32 at K <= 64, one for the rest, with two
 * beam slots per lane above K = 64), else a workgroup per pair.  GED_SCHED_BLOCK forces the
 * workgroup-per-pair kernel for every pair.  Every schedule computes the
 * same result bit for bit. */
#define GED_SCHED_AUTO 0
#define GED_SCHED_BLOCK 1

/* Last level of the search.  GED_LAST_SELECT (the default) keeps the K
 * children of least partial edit distance at every level, the last one
 * included, then completes them (Alg. 1 read literally).  GED_LAST_COMPLETE
 * completes every child of the last level with the insertions of Sec. 4.4.1
 * and keeps the least total (first in generation order on ties): never a
 * larger distance than GED_LAST_SELECT, and it skips the last selection. */
#define GED_LAST_SELECT 0
#define GED_LAST_COMPLETE 1

/* Method.  GED_METHOD_TREE (the default) is the paper's K-Best tree search
 * (Alg. 1).  GED_METHOD_BIPARTITE is the assignment-based variant, which the
 * paper does not contain: a node-assignment cost matrix (vertex operation
 * plus the least-cost assignment of the incident edges, Riesen and Bunke),
 * the K assignments of least cost enumerated by Murty's partitioning
 * (Hungarian solver, lowest index on ties, children re-solved from their
 * parent's potentials, subproblems popped by (cost, creation order)), and
 * the exact edit cost (Sec. 2.2-2.4) of each; the least, first popped among
 * equals, is the bound.  It needs n1 + n2 <= GED_BIP_MAX_ORDER for every
 * pair and K <= GED_BIP_MAX_K (else GED_EUNSUPPORTED), takes last_level =
 * GED_LAST_SELECT only, and d_cand then counts the assignment problems
 * solved (the first assignment included). */
#define GED_METHOD_TREE 0
#define GED_METHOD_BIPARTITE 1

/* Plan flags.
 * GED_PLAN_PAIR_STATUS: a pair that cannot be searched does not fail the
 * plan; it is set aside with a status of its own, which ged_plan_run_ex
 * reports per pair (the problem statement's result is per pair of graphs,
 * Alg. 1): GED_EINVAL for a graph id out of range, GED_EUNSUPPORTED for a
 * pair beyond the method's limits (a graph of more than
 * GED_MAX_VERTICES_BATCH vertices; directed graphs of more than
 * GED_DIRECTED_MAX_ORDER; the bipartite method's GED_BIP_MAX_ORDER).  A
 * set-aside pair's distance is -1, its mapping entries (n of its source
 * graph; none for a source id out of range) are -1 and its d_cand entry 0.
 * The other pairs' results are the same as without the flag. */
#define GED_PLAN_PAIR_STATUS 1u

typedef struct {
    int32_t schedule;        /* GED_SCHED_* */
    int32_t groups_per_cu;   /* resident workgroups per CU of a persistent launch;
                                0 = the occupancy limit, larger values are clamped to it */
    int32_t last_level;      /* GED_LAST_* */
    int32_t method;          /* GED_METHOD_* */
    uint32_t flags;          /* GED_PLAN_* bits, 0 = none */
} ged_plan_options;

/* ged_plan_create with options (NULL = defaults).  GED_EINVAL for an
 * unknown schedule, last level, method or flag bit, or groups_per_cu < 0. */
ged_status ged_plan_create_ex(ged_db *db, const ged_pair *h_pairs, int64_t npairs, int32_t K,
                              const ged_plan_options *options, ged_plan **out);
ged_status ged_plan_map_size(const ged_plan *plan, int64_t *entries);
ged_status ged_plan_run(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                        int64_t *d_cand, void *stream);
/* ged_plan_run with per-pair statuses: d_status[p] (int32 [npairs], device,
 * may be NULL) receives GED_OK for a searched pair and, in a plan created
 * with GED_PLAN_PAIR_STATUS, the status of each set-aside pair (whose
 * outputs are written as that flag states).  Enqueues only kernels.  Errors
 * as ged_plan_run: costs that could overflow int32 on a searched pair fail
 * the whole call (GED_EINVAL, nothing enqueued). */
ged_status ged_plan_run_ex(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                           int32_t *d_status, void *stream);
/* The plan's pairs again, as the per-pair baseline: one kernel launch per
 * pair, back to back on `stream`, same outputs as ged_plan_run. */
ged_status ged_plan_run_perpair(ged_plan *plan, ged_costs costs, int32_t *d_dist,
                                int32_t *d_map, int64_t *d_cand, void *stream);
ged_status ged_plan_destroy(ged_plan *plan);

/* Measurement hooks.  With timing enabled, ged_plan_run and
 * ged_plan_run_perpair record a HIP event on `stream` right before the
 * plan's first search-kernel launch and right after its last one; once that
 * stream has been synchronized, ged_plan_kernel_ms returns the elapsed
 * milliseconds between the two events of the most recent run (GED_EINVAL if
 * timing is off or nothing has run).  ged_plan_kernel_launches returns how
 * many search-kernel launches the most recent run made. */
ged_status ged_plan_set_timing(ged_plan *plan, int32_t enable);
ged_status ged_plan_kernel_ms(ged_plan *plan, float *ms);
ged_status ged_plan_kernel_launches(const ged_plan *plan, int64_t *launches);

/* The plan's size bins, in launch order.  For bin `index`: *kernel is
 * GED_KERNEL_WAVE (a wavefront per pair), GED_KERNEL_BLOCK (a workgroup
 * per pair) or GED_KERNEL_BIPARTITE (bipartite method; *words is then
 * its columns per lane, ceil((n1 + n2) / 64)), *npairs the pairs in the bin, *grid the persistent launch's
 * workgroups, *words the target-row words the instantiation handles (1
 * or 2 for the wavefront kernels: targets of up to 32 or 64 vertices).
 * Any output pointer may be NULL. */
/* HIP graphs.  ged_plan_capture records one ged_plan_run with these costs
 * and outputs into a HIP graph owned by the plan (replacing any previous
 * one); ged_plan_replay launches it on `stream`.  The graph holds only
 * kernel nodes (work-queue counters are cleared by a kernel, not a memset).
 * The output buffers must stay allocated while the graph is replayed.
 * `stream` must not be the null stream (HIP cannot capture it): GED_EINVAL.
 * ged_plan_replay without a captured graph: GED_EINVAL. */
ged_status ged_plan_capture(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                            int64_t *d_cand, void *stream);
ged_status ged_plan_replay(ged_plan *plan, void *stream);

/* Autotuner.  For every size bin, times the candidate schedules on the
 * plan's own pairs -- the wavefront kernel where the bin is eligible and
 * the workgroup kernel with 256- and 512-thread workgroups, each at several
 * resident-workgroup counts -- and
 * keeps the fastest; every candidate computes identical results, which are
 * written to the outputs.  With cache_path (may be NULL) the choices are
 * read from / appended to that text file, keyed by device, K and the bin's
 * shape, and a cached choice is applied without timing.  Waits for all
 * work on the device first (the plan's work lists are rewritten), and
 * synchronizes `stream`.  *timed_bins (may be NULL) gets the number of bins
 * that were timed rather than read from the cache.  A captured graph is
 * discarded. */
ged_status ged_plan_tune(ged_plan *plan, ged_costs costs, int32_t *d_dist, int32_t *d_map,
                         void *stream, const char *cache_path, int32_t *timed_bins);

#define GED_KERNEL_WAVE 0
#define GED_KERNEL_BLOCK 1
#define GED_KERNEL_BIPARTITE 2   /* the bipartite method's wavefront kernel */
ged_status ged_plan_bin_count(const ged_plan *plan, int32_t *count);
ged_status ged_plan_bin_info(const ged_plan *plan, int32_t index, int32_t *kernel, int64_t *npairs,
                             int32_t *grid, int32_t *words);

/* One-shot forms: create a plan, run it on `stream`, synchronize `stream`,
 * destroy the plan.  Same arguments and errors as above. */
ged_status ged_kbest(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs,
                     int32_t K, int32_t *d_dist, int32_t *d_map, void *stream);
ged_status ged_kbest_perpair(ged_db *db, const ged_pair *h_pairs, int64_t npairs,
                             ged_costs costs, int32_t K, int32_t *d_dist, int32_t *d_map,
                             void *stream);
/* One-shot form with options (NULL = defaults), the children evaluated
 * (d_cand, may be NULL) and per-pair statuses (d_status, may be NULL; see
 * ged_plan_run_ex and GED_PLAN_PAIR_STATUS). */
ged_status ged_kbest_ex(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                        const ged_plan_options *options, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                        int32_t *d_status, void *stream);

/* Mapping offsets on the device (the layout of every search's d_map: pair
 * p's mapping of its source graph g1, n1 entries, one per vertex of g1 as in
 * Alg. 1's edit path, starts at the sum of n1 over the pairs before it).
 * d_pairs: npairs pairs in device memory (caller's order); d_off: device,
 * npairs + 1 int64 entries: d_off[p] for p < npairs as above, d_off[npairs]
 * the total (the d_map entries the batch needs).  A pair whose source id is
 * outside the database contributes no entries (a search with
 * GED_PLAN_PAIR_STATUS reports it GED_EINVAL).  Enqueued on `stream` (one
 * kernel); allocates nothing.  Errors: GED_EINVAL (NULL db or d_off, NULL
 * d_pairs with npairs > 0, npairs < 0, a device other than the database's);
 * GED_EDEVICE. */
ged_status ged_map_offsets(ged_db *db, const ged_pair *d_pairs, int64_t npairs, int64_t *d_off, void *stream);

/* ------------------------------------------------------------------------
 * ged_kbest without device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same arguments, checks and results as ged_kbest (K-Best
 * search of every pair, default schedule and last level), bit for bit.
 *
 * Its staging (a device copy of the pairs, the mapping offsets, the work
 * lists and queue counters, the workgroup kernel's per-workgroup beam
 * workspace) lives in one device array of GED_NOALLOC_SCRATCH_BYTES that
 * the library holds on every device it runs on until the process ends, so
 * the call allocates no device memory.  Every call on a device shares that
 * device's array: calls that overlap on one device (from several host
 * threads or on several streams) race and must be serialized by the
 * caller.  The call enqueues its work on `stream` and synchronizes it.
 * Errors: as ged_kbest; GED_EUNSUPPORTED when the batch's staging (about
 * 48 bytes per pair) plus one workgroup's workspace for each of its
 * workgroup-kernel bins exceeds GED_NOALLOC_SCRATCH_BYTES (workgroup bins
 * otherwise run as many workgroups as the remaining scratch holds).
 * ---------------------------------------------------------------------- */
#define GED_NOALLOC_SCRATCH_BYTES (64ll << 20)
ged_status ged_kbest_noalloc(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, int32_t K,
                             int32_t *d_dist, int32_t *d_map, void *stream);

/* ------------------------------------------------------------------------
 * Edit paths.  A vertex mapping (as the searches return it) induces one edit
 * path (Sec. 2.2-2.4); ged_edit_path writes its operations explicitly.
 *
 * For each pair p the operations are, in this order:
 *   1. per g1 vertex v ascending: GED_OP_VSUB (a = v, b = map(v)) or
 *      GED_OP_VDEL (a = v, b = -1);
 *   2. per g2 vertex u ascending outside the mapping's image: GED_OP_VINS
 *      (a = -1, b = u);
 *   3. per g1 edge {a, b}, a < b, in lexicographic order: GED_OP_ESUB (c, d =
 *      the g2 edge {map(a), map(b)}, c < d) when both ends are mapped onto a
 *      g2 edge, else GED_OP_EDEL (c = d = -1);
 *   4. per g2 edge {c, d}, c < d, in lexicographic order that is no g1 edge's
 *      image: GED_OP_EINS (a = b = -1).
 * Directed database: steps 3 and 4 list every arc (a, b) in lexicographic
 * order of (a, b), and a substituted arc's image is (c, d) = (map(a), map(b))
 * as it stands.
 * cost is the operation's cost (0 for a substitution that keeps the label);
 * the costs of a pair sum to the edit cost of its mapping, i.e. to the
 * distance the search returned with it.
 *
 * ged_edit_path_capacity: h_offsets[0..npairs] (host, int64) receives the
 * exclusive prefix sum of n1 + n2 + m1 + m2 over the pairs, the most
 * operations each can take; pair p's operations start at h_offsets[p].
 * ged_edit_path: d_map is the mappings in the searches' layout (pair p at
 * the sum of n(src) of the pairs before it); d_ops holds h_offsets[npairs]
 * records; d_count[p] (int32, device) receives pair p's number of
 * operations.  Enqueued on `stream`, then synchronized.  Errors: GED_EINVAL
 * (ids out of range, NULL buffers, negative costs, or a mapping that is not
 * injective or has an entry outside [-1, n2): its d_count is -1 and the
 * message names the first such pair); GED_ENOMEM; GED_EDEVICE.
 * ---------------------------------------------------------------------- */
#define GED_OP_VSUB 0
#define GED_OP_VDEL 1
#define GED_OP_VINS 2
#define GED_OP_ESUB 3
#define GED_OP_EDEL 4
#define GED_OP_EINS 5

typedef struct {
    int32_t kind;   /* GED_OP_* */
    int32_t a, b;   /* vertex ops: g1 vertex, g2 vertex; edge ops: g1 edge ends */
    int32_t c, d;   /* edge ops: g2 edge ends */
    int32_t cost;
} ged_edit_op;

ged_status ged_edit_path_capacity(const ged_db *db, const ged_pair *h_pairs, int64_t npairs, int64_t *h_offsets);
ged_status ged_edit_path(ged_db *db, const ged_pair *h_pairs, int64_t npairs, ged_costs costs, const int32_t *d_map,
                         ged_edit_op *d_ops, int32_t *d_count, void *stream);

/* ------------------------------------------------------------------------
 * Single-pair search at large K (the paper's own regime, Sec. 5: K from
 * thousands to 1.2 million).  The whole device works on one pair: the beam
 * lives in device memory, and every level of Alg. 1 is a sequence of
 * grid-wide kernels -- every child's PED (Sec. 2.3) into a candidate matrix
 * with a histogram of the PEDs, the K-th smallest child by histogram select
 * (refined where the PED range needs it), stable compaction of the survivors
 * in generation order, and the beam update.  The result is the same as the
 * batched search's (ged_plan_run) at the same K, bit for bit.
 *
 * ged_wide_create sizes and allocates the workspace for pair (src, dst) of
 * `db` at beam width K (1 <= K <= GED_MAX_K_WIDE): about
 * K * (4 (n2 + 1) + 4 n1 + 24 + 4 w2 (3 + planes)) bytes (w2 = target words
 * of 32 vertices).  ged_wide_bytes returns what it holds.  ged_wide_run
 * enqueues the search on `stream` (NULL = the null stream); outputs are
 * device pointers: d_dist[0] the distance, d_map[0..n1) the target vertex
 * of each source vertex (-1 = deleted), d_cand[0] (may be NULL) the children
 * evaluated.  The workspace belongs to the handle, so runs of one handle must
 * not overlap; different handles are independent.
 *
 * Errors: GED_EINVAL (NULL arguments, graph id out of range, K out of range,
 * negative costs, costs that could overflow int32 on the pair, a device other
 * than the database's); GED_ENOMEM (workspace); GED_EDEVICE (launch failure).
 * ---------------------------------------------------------------------- */
typedef struct ged_wide ged_wide;

ged_status ged_wide_create(ged_db *db, int64_t src, int64_t dst, int32_t K, ged_wide **out);
/* With options: only last_level is used (GED_LAST_*; schedule and
 * groups_per_cu are ignored; method must be GED_METHOD_TREE).  GED_EINVAL
 * for an unknown last level or another method. */
ged_status ged_wide_create_ex(ged_db *db, int64_t src, int64_t dst, int32_t K, const ged_plan_options *options,
                              ged_wide **out);
ged_status ged_wide_bytes(const ged_wide *w, int64_t *bytes);
ged_status ged_wide_run(ged_wide *w, ged_costs costs, int32_t *d_dist, int32_t *d_map, int64_t *d_cand,
                        void *stream);
ged_status ged_wide_destroy(ged_wide *w);

/* ------------------------------------------------------------------------
 * Serving: a request loop over a device-resident database.
 *
 * Clients submit queries -- a query graph (host memory, copied and packed
 * with the database's edge-label coding) to be edited into database graph
 * `target_id` -- and poll for results.  Queries are sorted at submission
 * into four size classes with queues and streams of their own: small
 * (n1, n2 <= 32, K <= 64) and mid (n1, n2 <= 64, K <= 128; the wavefront
 * kernels), medium (n1, n2 <= 128) and large, so a small query never waits
 * for a larger one's batch.  A
 * worker thread owned by the server admits queued queries while device
 * slots and the HBM budget allow, packs them into a batch (query graphs
 * staged into a device arena) and launches the batch on a free stream of
 * its class; a batch can start while earlier ones still run, so queries
 * that arrive during a launch are admitted into the next one as slots and
 * memory free up (continuous batching).  Each
 * query's search state (its beam) lives on the device for the whole search;
 * results are copied back once the batch's stream reaches its event.  The
 * result of a query does not depend on the other queries of its batch.
 * ---------------------------------------------------------------------- */
typedef struct ged_server ged_server;

typedef struct {
    int32_t K;                /* beam width, 1..GED_MAX_K */
    ged_costs costs;          /* edit costs of every query */
    int64_t hbm_budget;       /* device bytes the server may hold (arenas, work
                                 lists, outputs, workspaces); 0 = 2 GiB */
    int32_t max_inflight;     /* queries admitted to the device at once; 0 = 4096 */
    int32_t max_batch;        /* queries per launch; 0 = 1024 */
    int32_t streams;          /* streams per size class (launches of a class that
                                 may overlap), 1..4; 0 = 1; the tree search's
                                 large class gets twice as many.  With more than
                                 one, a class's next batch starts while a slow
                                 one runs.  Streams beyond the process's hardware
                                 queues (HIP: GPU_MAX_HW_QUEUES, 4 by default)
                                 share queues, and a long launch then delays the
                                 others on its queue; give the process well
                                 over 5 * streams queues (other streams of the
                                 process take queues too).  While a class has a
                                 batch on the device, its next batch waits for
                                 64 queued queries or 1 ms; a batch of the
                                 medium / large class holds at most 2 / 1
                                 workgroups per CU. */
    int32_t queue_capacity;   /* queued (not yet admitted) queries before
                                 ged_server_submit returns GED_EBUSY; 0 = 1<<20 */
    int32_t method;           /* GED_METHOD_TREE (0) or GED_METHOD_BIPARTITE: the
                                 latter serves pairs with n1 + n2 <= GED_BIP_MAX_ORDER
                                 at K <= GED_BIP_MAX_K, in four size classes by
                                 ceil((n1 + n2) / 64) (submit: GED_EUNSUPPORTED
                                 for a larger pair) */
} ged_server_config;

typedef struct {
    int64_t submitted, completed, rejected_busy, launches;
    int64_t queued, inflight, inflight_peak;
    int64_t batch_peak;       /* largest batch launched */
    int64_t device_bytes;     /* device memory held */
} ged_server_stats;

/* The server's tree searches use the default last level (GED_LAST_SELECT).
 * Errors: GED_EINVAL (bad config, costs, K); GED_ENOMEM when the budget
 * cannot hold one batch of the configured size; GED_EDEVICE. */
ged_status ged_server_create(ged_db *db, const ged_server_config *config, ged_server **out);

/* Queue one query; *ticket identifies it.  GED_EINVAL for an invalid query
 * graph (as for ged_db_create; also an edge label absent from the database)
 * or target id, or costs that could overflow int32 on this pair;
 * GED_EUNSUPPORTED when the query or the target has more than
 * GED_MAX_VERTICES_BATCH vertices; GED_EBUSY when the queue is full
 * (backpressure: retry later). */
ged_status ged_server_submit(ged_server *srv, const ged_graph *query, int64_t target_id, uint64_t *ticket);

/* Queue one query whose graph is database graph `query_id` (Sec. 5's
 * query-versus-database setting: a database graph searched against another):
 * no host graph is passed, validated or packed; the batch copies the
 * graph's packed rows from the database on the device.  Same results and
 * errors as ged_server_submit with that graph (GED_EINVAL also for
 * query_id out of range). */
ged_status ged_server_submit_id(ged_server *srv, int64_t query_id, int64_t target_id, uint64_t *ticket);

/* Non-blocking: GED_OK writes the distance and the mapping (n1 entries,
 * -1 = deleted; *n1 gets n1) and releases the ticket; GED_EBUSY if the query
 * is not finished; GED_EINVAL for an unknown ticket or map_capacity < n1
 * (the ticket is kept); a query whose launch failed reports GED_EDEVICE.
 * times_ns (may be NULL) gets [submission, completion] on the monotonic
 * clock (CLOCK_MONOTONIC, nanoseconds); completion is when the worker saw
 * the batch's event. */
ged_status ged_server_poll(ged_server *srv, uint64_t ticket, int32_t *dist, int32_t *map,
                           int32_t map_capacity, int32_t *n1, int64_t *times_ns);
/* Blocking form of ged_server_poll; GED_ETIMEOUT after timeout_us
 * microseconds (< 0: wait without limit). */
ged_status ged_server_wait(ged_server *srv, uint64_t ticket, int64_t timeout_us, int32_t *dist,
                           int32_t *map, int32_t map_capacity, int32_t *n1, int64_t *times_ns);
/* Submit queries[0..count) in order (query k against targets[k]) until one
 * is refused; *accepted gets how many were queued (tickets[0..*accepted)).
 * Returns GED_OK if all were queued, else the refusal's status (GED_EBUSY
 * when the queue filled up). */
ged_status ged_server_submit_batch(ged_server *srv, const ged_graph *queries, const int64_t *targets,
                                   int64_t count, uint64_t *tickets, int64_t *accepted);
/* Collect finished queries in completion order (each once), releasing
 * their tickets: waits up to timeout_us microseconds (< 0: no limit) for
 * at least one, then moves up to max_count of them out: tickets[k],
 * dist[k] (-1 for a failed launch), times_ns[2k..2k+1] = submission and
 * completion (monotonic clock, ns), and, if maps is not NULL, the mappings
 * back to back in maps (stopping before one that would exceed
 * maps_capacity).  *count gets the number collected; GED_ETIMEOUT when none
 * finished in time.  A query taken with ged_server_poll/wait is not
 * reported again here. */
ged_status ged_server_collect(ged_server *srv, int64_t timeout_us, int64_t max_count, uint64_t *tickets,
                              int32_t *dist, int64_t *times_ns, int32_t *maps, int64_t maps_capacity,
                              int64_t *count);
ged_status ged_server_stats_get(const ged_server *srv, ged_server_stats *out);
/* Finishes every admitted query, cancels queued ones, frees everything. */
ged_status ged_server_destroy(ged_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* GED_H */
