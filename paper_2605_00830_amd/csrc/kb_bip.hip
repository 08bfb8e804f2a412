// kb_bip.hip -- the bipartite K-best-assignment bound of graph edit distance,
// one wavefront per pair (n1 + n2 <= 256, K <= 256).
//
// The variant: a node-assignment cost matrix (Riesen and Bunke's bipartite
// edit cost: vertex operation plus the least-cost assignment of the incident
// edges), the K assignments of least cost enumerated by Murty's partitioning,
// and the exact induced edit cost (Sec. 2.2-2.4) of each, the least of which
// is the bound.  The paper's own search is the tree search of kb_wave.hip;
// this kernel uses the paper's edit operations and costs only.
//
// Matrix: M = n1 + n2 columns (g2's vertices, then one deletion column per
// g1 vertex).  Row i < n1 holds, for column j < n2,
//     vsub [labels differ] + edel (d1 - mm) + eins (d2 - mm)
//       + min(esub, edel + eins) (mm - common) - ins(j) + D,
// mm = min(d1, d2), common = equal-label incident edge pairs, ins(j) = vins +
// eins d2(j), D = max_j ins(j); column n2 + i holds vdel + edel d1 + D; other
// deletion columns are closed.  Rows n1 .. M-1 are zero filler rows, so every
// column is always assigned.  No matrix is stored: a lane forms its columns'
// entries of the scanned row from the row's degree, label and incident-label
// counts (read once per step) and its columns' own.
//
// Lane layout, CPL = ceil(M / 64) slots per lane: lane l holds columns l,
// l + 64, ... (potential v, row p, search distance and predecessor) and rows
// l, l + 64, ... (potential u); QPL = ceil(K / 64) queue slots per lane hold
// the keys (assignment cost, creation number).  A row is inserted by a
// Dijkstra search over reduced costs: per step each lane relaxes its columns
// from the scanned row, one DPP minimum over (distance << 8 | column) gives
// the first column of least distance (reduced costs stay below (M + 1)
// entries, which the host keeps below 2^24), and the potentials of the
// tree's rows and columns are updated, branch-free per lane.  The matrix is
// square and every assigned pair tight, so an assignment's cost is the sum
// of all potentials.
//
// Murty's partitioning runs over g1's rows: a popped subproblem's free rows
// r_0 < r_1 < ... each give one child with r_0 .. r_{t-1} fixed to their
// columns and (r_t, its column) forbidden, solved from the parent's
// potentials with that one row re-inserted.  Queue nodes (potentials,
// assignment, fixed rows, forbidden pairs) live in a per-wave slice of the
// workspace; only the K - popped least keys can still be popped, so K slots
// suffice (a full queue evicts its largest key).  A popped node's forbidden
// pairs go into an LDS bitmap (row x column) with a per-row summary bit, read
// by a step only when its row has any.  Each popped mapping is scored by its
// induced cost: per g1 vertex, its earlier neighbours' images tested against
// the image's g2 row.
#include <hip/hip_runtime.h>

#include <type_traits>

#include "ged_internal.h"
#include "wave_common.h"

namespace gedk {
namespace {

using namespace wv;

constexpr uint32_t BINF = 0x7fffffffu;   // closed entry / unreached column

struct BipArgs {
    DbView src;
    DbView dst;
    const WorkItem *work;
    int nwork;
    int *queue;
    Costs c;
    int K;
    int pad;
    size_t node_bytes;
    unsigned char *ws;   // grid x K x node_bytes
    Outputs out;
};

// one of N per-lane slots, chosen by an index: an OR of masked values (a
// select chain over the array would be turned back into an indexed load of
// a stack copy)
template <int N, typename T>
__device__ __forceinline__ T pick(const T (&x)[N], int s) {
    using U = typename std::conditional<sizeof(T) == 8, uint64_t, uint32_t>::type;
    U r = 0;
#pragma unroll
    for (int k = 0; k < N; ++k) {
        U bits;
        __builtin_memcpy(&bits, &x[k], sizeof(T));
        r |= bits & (U)(0 - (U)(s == k));
    }
    T out;
    __builtin_memcpy(&out, &r, sizeof(T));
    return out;
}

__device__ __forceinline__ bool adj_bit(const uint32_t *A, int w, int x, int y) {
    return (A[(size_t)x * w + (y >> 5)] >> (y & 31)) & 1u;
}

template <int PL, int CPL, int QPL, int NWAV>
__global__ __launch_bounds__(64 * NWAV) void kb_bip_kernel(BipArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    constexpr int NL = PL > 0 ? (1 << PL) : 1;   // edge-label codes
    constexpr int NW = (NL + 3) / 4;             // words of byte counts
    constexpr int MAXM = 64 * CPL;
    constexpr int PWMAX = QPL + CPL;             // words of the node pool's free flags
    __shared__ int s_col[MAXM];                  // column of each row of the popped assignment
    __shared__ int s_phi[MAXM];                  // its mapping of g1's vertices
    __shared__ unsigned long long s_forb[MAXM][CPL];   // forbidden (row, column) bits
    __shared__ unsigned long long s_rowf[CPL];   // rows with any forbidden column
    __shared__ int s_res[MAXM];                  // per child: assignment cost, or ~0 (none)
    __shared__ int s_alloc[MAXM];                // per child: pool slot of its node
    __shared__ int s_item;

    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    const int32_t vsub = a.c.vsub, vdel = a.c.vdel, vins = a.c.vins;
    const int32_t esub = a.c.esub, edel = a.c.edel, eins = a.c.eins;
    const int32_t cross = min(esub, edel + eins);
    const int K = a.K;
    const int P = a.dst.planes;
    const size_t NB = a.node_bytes;
    // node layout (offsets inside a slot of NB bytes)
    const size_t oV = 4 * (size_t)MAXM, oP = 8 * (size_t)MAXM, oFix = 10 * (size_t)MAXM;
    const size_t oNf = oFix + 8 * CPL, oForb = oNf + 16;
    unsigned char *ws = a.ws + (size_t)blockIdx.x * (size_t)(K + MAXM) * NB;

    for (bool first = true;; first = false) {
        int item = (int)blockIdx.x;
        if (!first) {
            if (threadIdx.x == 0) s_item = pull_item(a.queue, a.nwork);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
        }
        if (item >= a.nwork) break;

        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.src.graphs[wi.src];
        const GraphRec g2 = a.dst.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n, M = n1 + n2;
        const int w1 = g1.w, w2 = g2.w;
        const uint32_t *A1 = a.src.adj + g1.adj;
        const uint32_t *A2 = a.dst.adj + g2.adj;

        // ---------------- per-vertex degree, label, incident-label counts
        int d1[CPL], l1[CPL], d2[CPL], l2[CPL];
        uint32_t c1[CPL][NW], c2[CPL][NW];
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            const int x = lane + 64 * k;
            d1[k] = d2[k] = 0;
            l1[k] = x < n1 ? a.src.vlab[g1.vlab + x] : 0;
            l2[k] = x < n2 ? a.dst.vlab[g2.vlab + x] : 0;
#pragma unroll
            for (int q = 0; q < NW; ++q) c1[k][q] = c2[k][q] = 0u;
            for (int wd = 0; wd < max(w1, w2); ++wd) {
                const uint32_t r1 = (x < n1 && wd < w1) ? A1[(size_t)x * w1 + wd] : 0u;
                const uint32_t r2 = (x < n2 && wd < w2) ? A2[(size_t)x * w2 + wd] : 0u;
                d1[k] += __popc(r1);
                d2[k] += __popc(r2);
                if (PL > 0) {
                    uint32_t q1[PLA], q2[PLA];
#pragma unroll
                    for (int b = 0; b < PLA; ++b) {
                        q1[b] = (b < P && x < n1 && wd < w1) ? A1[(size_t)(1 + b) * n1 * w1 + (size_t)x * w1 + wd] : 0u;
                        q2[b] = (b < P && x < n2 && wd < w2) ? A2[(size_t)(1 + b) * n2 * w2 + (size_t)x * w2 + wd] : 0u;
                    }
#pragma unroll
                    for (int L = 0; L < NL; ++L) {
                        uint32_t m1 = r1, m2 = r2;
#pragma unroll
                        for (int b = 0; b < PLA; ++b) {
                            m1 &= ((L >> b) & 1) ? q1[b] : ~q1[b];
                            m2 &= ((L >> b) & 1) ? q2[b] : ~q2[b];
                        }
                        c1[k][L >> 2] += (uint32_t)__popc(m1) << (8 * (L & 3));
                        c2[k][L >> 2] += (uint32_t)__popc(m2) << (8 * (L & 3));
                    }
                }
            }
        }
        int32_t ins[CPL];
        uint32_t dmax = 0u;
#pragma unroll
        for (int k = 0; k < CPL; ++k) {
            ins[k] = vins + eins * d2[k];
            dmax = max(dmax, lane + 64 * k < n2 ? (uint32_t)ins[k] : 0u);
        }
        const int32_t D = (int32_t)wave_umax(dmax);

        // entries of g1 row i for this lane's columns; BINF where closed
        auto row_entries = [&](int i, uint32_t (&e)[CPL]) __attribute__((always_inline)) {
            const int s = i >> 6, l = i & 63;
            const int d1i = __builtin_amdgcn_readlane(pick(d1, s), l);
            const int l1i = __builtin_amdgcn_readlane(pick(l1, s), l);
            uint32_t c1i[NW];
#pragma unroll
            for (int q = 0; q < NW; ++q) {
                uint32_t col[CPL];
#pragma unroll
                for (int k = 0; k < CPL; ++k) col[k] = c1[k][q];
                c1i[q] = (uint32_t)__builtin_amdgcn_readlane((int)pick(col, s), l);
            }
            const uint32_t del = (uint32_t)(vdel + edel * d1i + D);
            if (PL == 0) {
                // no edge labels (common = mm): the eins d2 terms cancel
                const int32_t base = edel * d1i - vins + D;
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const int j = lane + 64 * k;
                    const uint32_t sub = (uint32_t)(base + (l1i != l2[k] ? vsub : 0) - (edel + eins) * min(d1i, d2[k]));
                    e[k] = j < n2 ? sub : (j == n2 + i ? del : BINF);
                }
                return;
            }
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                const int j = lane + 64 * k;
                const int mm = min(d1i, d2[k]);
                int common = mm;
                if (PL > 0) {
                    common = 0;
#pragma unroll
                    for (int q = 0; q < NW; ++q)
#pragma unroll
                        for (int b = 0; b < 4; ++b)
                            common += (int)min(__builtin_amdgcn_ubfe(c1i[q], 8u * b, 8u),
                                               __builtin_amdgcn_ubfe(c2[k][q], 8u * b, 8u));
                }
                const uint32_t sub = (uint32_t)((l1i != l2[k] ? vsub : 0) + edel * (d1i - mm) + eins * (d2[k] - mm) +
                                                cross * (mm - common) - ins[k] + D);
                e[k] = j < n2 ? sub : (j == n2 + i ? del : BINF);
            }
        };

        // rows of the popped node with any forbidden column (wave-uniform copy)
        unsigned long long rowf[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) rowf[k] = 0ull;

        // ---------------- Hungarian row insertion (shortest augmenting path)
        // u: rows, v / p: columns (per-lane slots); open: column inside M and
        // not fixed to another row; (fr, fc): the child's own forbidden pair.
        auto augment = [&](int r, int32_t (&u)[CPL], int32_t (&v)[CPL], int (&p)[CPL], const bool (&open)[CPL], int fr,
                           int fc) __attribute__((always_inline)) -> bool {
            uint32_t minv[CPL];
            int way[CPL];
            bool used[CPL], live[CPL], intree[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                minv[k] = BINF;
                way[k] = -1;
                used[k] = false;
                live[k] = open[k];
                intree[k] = lane + 64 * k == r;
            }
            int i0 = r, j0 = -1;
            for (;;) {
                const int32_t ui0 = __builtin_amdgcn_readlane(pick(u, i0 >> 6), i0 & 63);
                uint32_t e[CPL];
                if (i0 < n1) {
                    row_entries(i0, e);
                } else {
#pragma unroll
                    for (int k = 0; k < CPL; ++k) e[k] = 0u;
                }
                const bool rf = (pick(rowf, i0 >> 6) >> (i0 & 63)) & 1ull;
                uint32_t key = 0xffffffffu;
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const int j = lane + 64 * k;
                    const bool forb = (rf && ((s_forb[i0][k] >> lane) & 1ull)) || (i0 == fr && j == fc);
                    const bool allow = live[k] && !forb && e[k] != BINF;
                    const uint32_t cur = (uint32_t)((int32_t)e[k] - ui0 - v[k]);
                    const bool better = allow && cur < minv[k];
                    minv[k] = better ? cur : minv[k];
                    way[k] = better ? j0 : way[k];
                    key = min(key, (live[k] && minv[k] != BINF) ? ((minv[k] << 8) | (uint32_t)j) : 0xffffffffu);
                }
                key = wave_umin(key);
                if (key == 0xffffffffu) return false;
                const uint32_t delta = key >> 8;
                const int j1 = (int)(key & 255u);
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const bool reach = live[k] && minv[k] != BINF;
                    u[k] += intree[k] ? (int32_t)delta : 0;
                    v[k] -= used[k] ? (int32_t)delta : 0;
                    minv[k] -= reach ? delta : 0u;
                    const bool hit = lane + 64 * k == j1;
                    used[k] = used[k] || hit;
                    live[k] = live[k] && !hit;
                }
                j0 = j1;
                const int pj = __builtin_amdgcn_readlane(pick(p, j1 >> 6), j1 & 63);
                if (pj < 0) break;
                i0 = pj;
#pragma unroll
                for (int k = 0; k < CPL; ++k) intree[k] = intree[k] || lane + 64 * k == i0;
            }
            // flip the path back to r
            while (j0 >= 0) {
                const int jp = __builtin_amdgcn_readlane(pick(way, j0 >> 6), j0 & 63);
                const int np = jp < 0 ? r : __builtin_amdgcn_readlane(pick(p, jp >> 6), jp & 63);
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if (lane + 64 * k == j0) p[k] = np;
                j0 = jp;
            }
            return true;
        };
        // cost of a complete assignment: every row and column assigned and
        // every assigned pair tight, so it is the sum of all potentials
        // (lanes past M keep zero potentials)
        auto assignment_cost = [&](const int32_t (&u)[CPL], const int32_t (&v)[CPL]) __attribute__((always_inline)) -> uint32_t {
            uint32_t s = 0u;
#pragma unroll
            for (int k = 0; k < CPL; ++k) s += (uint32_t)u[k] + (uint32_t)v[k];
            return wave_sum(s);
        };

        // ---------------- first assignment (wave 0): every row from zero potentials
        if (wv == 0) {
            int32_t u[CPL], v[CPL];
            int p[CPL];
            bool open0[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                u[k] = v[k] = 0;
                p[k] = -1;
                open0[k] = lane + 64 * k < M;
            }
            for (int r = 0; r < M; ++r) (void)augment(r, u, v, p, open0, -1, -1);   // a deletion column is always open
            const uint32_t c0 = assignment_cost(u, v);
            unsigned char *nb = ws;   // pool slot 0
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                reinterpret_cast<int32_t *>(nb)[lane + 64 * k] = u[k];
                reinterpret_cast<int32_t *>(nb + oV)[lane + 64 * k] = v[k];
                reinterpret_cast<int16_t *>(nb + oP)[lane + 64 * k] = (int16_t)p[k];
            }
            if (lane < CPL) reinterpret_cast<unsigned long long *>(nb + oFix)[lane] = 0ull;
            if (lane == 0) {
                *reinterpret_cast<int32_t *>(nb + oNf) = 0;
                s_res[0] = c0;
            }
        }
        __syncthreads();
        // the queue, identical in every wave: slot q = lane + 64 s holds
        // (assignment cost, creation number, pool slot of its node)
        uint32_t qcost[QPL], qseq[QPL];
        int qidx[QPL];
        bool qocc[QPL];
#pragma unroll
        for (int s = 0; s < QPL; ++s) {
            qcost[s] = qseq[s] = 0u;
            qidx[s] = 0;
            qocc[s] = false;
        }
        qocc[0] = lane == 0;
        qcost[0] = lane == 0 ? (uint32_t)s_res[0] : 0u;
        // node pool: K + MAXM slots (a full queue plus one pop's children);
        // slot x free <=> pfree[x >> 6] at lane x & 63
        const int PN = K + MAXM;
        bool pfree[PWMAX];
#pragma unroll
        for (int w = 0; w < PWMAX; ++w) pfree[w] = lane + 64 * w < PN && lane + 64 * w != 0;
        uint32_t seq = 1u;
        int popped = 0;
        int64_t solves = 1;
        uint32_t best = BINF;
        int bestphi[CPL];
#pragma unroll
        for (int k = 0; k < CPL; ++k) bestphi[k] = -1;
        auto set_free = [&](int x, bool f) __attribute__((always_inline)) {
#pragma unroll
            for (int w = 0; w < PWMAX; ++w) pfree[w] = (lane + 64 * w == x) ? f : pfree[w];
        };

        while (popped < K) {
            bool any = false;
#pragma unroll
            for (int s = 0; s < QPL; ++s) any = any || __ballot(qocc[s]) != 0ull;
            if (!any) break;
            // ---------------- pop the least (cost, creation number)
            uint32_t lc = 0xffffffffu;
#pragma unroll
            for (int s = 0; s < QPL; ++s) lc = min(lc, qocc[s] ? qcost[s] : 0xffffffffu);
            const uint32_t mc = wave_umin(lc);
            uint32_t ls = 0xffffffffu;
#pragma unroll
            for (int s = 0; s < QPL; ++s) ls = min(ls, (qocc[s] && qcost[s] == mc) ? qseq[s] : 0xffffffffu);
            const uint32_t ms = wave_umin(ls);
            int q = 0;
#pragma unroll
            for (int s = QPL - 1; s >= 0; --s) {
                const unsigned long long bl = __ballot(qocc[s] && qcost[s] == mc && qseq[s] == ms);
                q = bl ? 64 * s + (int)__builtin_ctzll(bl) : q;
            }
            const int pi = __builtin_amdgcn_readlane(pick(qidx, q >> 6), q & 63);
#pragma unroll
            for (int s = 0; s < QPL; ++s) qocc[s] = qocc[s] && lane + 64 * s != q;
            const unsigned char *nq = ws + (size_t)pi * NB;
            int32_t u_par[CPL], v_par[CPL];
            int p_par[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                u_par[k] = reinterpret_cast<const int32_t *>(nq)[lane + 64 * k];
                v_par[k] = reinterpret_cast<const int32_t *>(nq + oV)[lane + 64 * k];
                p_par[k] = lane + 64 * k < M ? (int)reinterpret_cast<const int16_t *>(nq + oP)[lane + 64 * k] : -1;
            }
            unsigned long long fixm[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) fixm[k] = reinterpret_cast<const unsigned long long *>(nq + oFix)[k];
            const int nf = *reinterpret_cast<const int32_t *>(nq + oNf);
            uint32_t fent[QPL];
#pragma unroll
            for (int s = 0; s < QPL; ++s)
                fent[s] = lane + 64 * s < nf ? reinterpret_cast<const uint32_t *>(nq + oForb)[lane + 64 * s] : 0u;
            set_free(pi, true);   // its children may reuse the slot once every wave has read it
            // forbidden bitmap, row -> column map and mapping of this node (every
            // wave stores the same values)
            for (int x = (int)threadIdx.x; x < MAXM * CPL; x += 64 * NWAV) (&s_forb[0][0])[x] = 0ull;
            if ((int)threadIdx.x < CPL) s_rowf[threadIdx.x] = 0ull;
            __syncthreads();
#pragma unroll
            for (int s = 0; s < QPL; ++s) {
                if (wv == 0 && lane + 64 * s < nf) {
                    const int fr = (int)(fent[s] & 0xffffu), fcol = (int)(fent[s] >> 16);
                    atomicOr(&s_forb[fr][fcol >> 6], 1ull << (fcol & 63));
                    atomicOr(&s_rowf[fr >> 6], 1ull << (fr & 63));
                }
            }
            if (wv == 0) {
#pragma unroll
                for (int k = 0; k < CPL; ++k)
                    if (p_par[k] >= 0) s_col[p_par[k]] = lane + 64 * k;
            }
            // the free rows (children, in ascending row order) and the pool
            // slot each child's node goes to: the lowest free slots, in order
            int m = 0;
            for (int w = 0; w < CPL; ++w) {
                const int base = 64 * w;
                unsigned long long fr = ~pick(fixm, w);
                fr &= n1 - base >= 64 ? ~0ull : (n1 > base ? ((1ull << (n1 - base)) - 1ull) : 0ull);
                m += __popcll(fr);
            }
            if (wv == 0) {
                int t = 0;
#pragma unroll
                for (int w = 0; w < PWMAX; ++w) {
                    unsigned long long bl = __ballot(pfree[w]);
                    while (bl && t < m) {
                        if (lane == 0) s_alloc[t] = 64 * w + (int)__builtin_ctzll(bl);
                        bl &= bl - 1ull;
                        ++t;
                    }
                }
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < CPL; ++k) rowf[k] = s_rowf[k];
            if (wv == 0) {
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const int x = lane + 64 * k;
                    if (x < n1) {
                        const int cx = s_col[x];
                        s_phi[x] = cx < n2 ? cx : -1;
                    }
                }
            }
            for (int t = 0; t < m; ++t) set_free(s_alloc[t], false);
            __syncthreads();

            // ---------------- its induced edit cost (wave 0)
            if (wv == 0) {
                uint32_t vc = 0u, matched = 0u, nsub = 0u;
#pragma unroll
                for (int k = 0; k < CPL; ++k) {
                    const int x = lane + 64 * k;
                    if (x >= n1) continue;
                    const int fx = s_phi[x];
                    if (fx < 0) {
                        vc += (uint32_t)vdel;
                    } else {
                        ++nsub;
                        vc += a.dst.vlab[g2.vlab + fx] != l1[k] ? (uint32_t)vsub : 0u;
                    }
                    // earlier neighbours b < x: kept (both mapped onto a g2
                    // edge, relabelled when a label plane differs) or deleted
                    for (int wd = 0; wd <= (x >> 5); ++wd) {
                        uint32_t row = A1[(size_t)x * w1 + wd];
                        if (wd == (x >> 5)) row &= (1u << (x & 31)) - 1u;
                        while (row) {
                            const int b = 32 * wd + __builtin_ctz(row);
                            row &= row - 1u;
                            const int fb = s_phi[b];
                            if (fx >= 0 && fb >= 0 && adj_bit(A2, w2, fx, fb)) {
                                ++matched;
                                if (PL > 0) {
                                    bool diff = false;
                                    for (int pl = 0; pl < P; ++pl)
                                        diff = diff || (adj_bit(A1 + (size_t)(1 + pl) * n1 * w1, w1, x, b) !=
                                                        adj_bit(A2 + (size_t)(1 + pl) * n2 * w2, w2, fx, fb));
                                    vc += diff ? (uint32_t)esub : 0u;
                                }
                            } else {
                                vc += (uint32_t)edel;
                            }
                        }
                    }
                }
                const uint32_t nsub_all = wave_sum(nsub);
                const uint32_t d = wave_sum(vc) + (uint32_t)vins * ((uint32_t)n2 - nsub_all) +
                                   (uint32_t)eins * ((uint32_t)g2.m - wave_sum(matched));
                if (d < best) {
                    best = d;
#pragma unroll
                    for (int k = 0; k < CPL; ++k) bestphi[k] = lane + 64 * k < n1 ? s_phi[lane + 64 * k] : -1;
                }
            }
            ++popped;
            if (popped == K) break;

            // ---------------- partition: one child per free row, ascending;
            // child t is solved by wave t mod NWAV
            unsigned long long cfix[CPL];
            bool blocked[CPL];
#pragma unroll
            for (int k = 0; k < CPL; ++k) {
                cfix[k] = fixm[k];
                const int pk = p_par[k];
                blocked[k] = pk >= 0 && pk < n1 && ((pick(fixm, pk >> 6) >> (pk & 63)) & 1ull);
            }
            int t = 0;
            for (int wsl = 0; wsl < CPL; ++wsl) {
                const int base = 64 * wsl;
                unsigned long long freem = ~pick(fixm, wsl);
                freem &= n1 - base >= 64 ? ~0ull : (n1 > base ? ((1ull << (n1 - base)) - 1ull) : 0ull);
                while (freem) {
                    const int r = base + (int)__builtin_ctzll(freem);
                    freem &= freem - 1ull;
                    const int c = s_col[r];   // uniform
                    if (t % NWAV == wv) {
                        int32_t cu[CPL], cv[CPL];
                        int cp[CPL];
                        bool open[CPL];
#pragma unroll
                        for (int k = 0; k < CPL; ++k) {
                            cu[k] = u_par[k];
                            cv[k] = v_par[k];
                            cp[k] = lane + 64 * k == c ? -1 : p_par[k];
                            open[k] = lane + 64 * k < M && !blocked[k];
                        }
                        uint32_t cost = 0xffffffffu;
                        if (augment(r, cu, cv, cp, open, r, c)) {
                            cost = assignment_cost(cu, cv);
                            unsigned char *nb = ws + (size_t)s_alloc[t] * NB;
#pragma unroll
                            for (int k = 0; k < CPL; ++k) {
                                reinterpret_cast<int32_t *>(nb)[lane + 64 * k] = cu[k];
                                reinterpret_cast<int32_t *>(nb + oV)[lane + 64 * k] = cv[k];
                                reinterpret_cast<int16_t *>(nb + oP)[lane + 64 * k] = (int16_t)cp[k];
                            }
                            if (lane < CPL) reinterpret_cast<unsigned long long *>(nb + oFix)[lane] = pick(cfix, lane);
                            if (lane == 0) *reinterpret_cast<int32_t *>(nb + oNf) = nf + 1;
#pragma unroll
                            for (int s = 0; s < QPL; ++s) {
                                const int x = lane + 64 * s;
                                if (x <= nf)
                                    reinterpret_cast<uint32_t *>(nb + oForb)[x] =
                                        x < nf ? fent[s] : ((uint32_t)r | ((uint32_t)c << 16));
                            }
                        }
                        if (lane == 0) s_res[t] = (int)cost;
                    }
                    // r is fixed for the later children
#pragma unroll
                    for (int k = 0; k < CPL; ++k) {
                        cfix[k] |= (r >> 6) == k ? (1ull << (r & 63)) : 0ull;
                        blocked[k] = blocked[k] || lane + 64 * k == c;
                    }
                    ++t;
                }
            }
            solves += m;
            __syncthreads();

            // ---------------- push the children in order (every wave alike)
            for (int tt = 0; tt < m; ++tt) {
                const uint32_t cost = (uint32_t)s_res[tt];
                const int x = s_alloc[tt];
                if (cost == 0xffffffffu) {   // no assignment: its slot returns to the pool
                    set_free(x, true);
                    continue;
                }
                const uint32_t cseq = seq++;
                const int cap = K - popped;
                int occn = 0;
#pragma unroll
                for (int s = 0; s < QPL; ++s) occn += __popcll(__ballot(qocc[s]));
                int slot = -1;
                if (occn < cap) {
#pragma unroll
                    for (int s = QPL - 1; s >= 0; --s) {
                        const unsigned long long bl = __ballot(!qocc[s] && lane + 64 * s < K);
                        slot = bl ? 64 * s + (int)__builtin_ctzll(bl) : slot;
                    }
                } else {
                    // the child's creation number exceeds every queued one, so
                    // it displaces the largest key only when cheaper
                    uint32_t xl = 0u;
#pragma unroll
                    for (int s = 0; s < QPL; ++s) xl = max(xl, qocc[s] ? qcost[s] : 0u);
                    const uint32_t xc = wave_umax(xl);
                    uint32_t sl = 0u;
#pragma unroll
                    for (int s = 0; s < QPL; ++s) sl = max(sl, (qocc[s] && qcost[s] == xc) ? qseq[s] : 0u);
                    const uint32_t xs = wave_umax(sl);
                    if (cost < xc) {
#pragma unroll
                        for (int s = QPL - 1; s >= 0; --s) {
                            const unsigned long long bl = __ballot(qocc[s] && qcost[s] == xc && qseq[s] == xs);
                            slot = bl ? 64 * s + (int)__builtin_ctzll(bl) : slot;
                        }
                        // the evicted node's slot returns to the pool
                        set_free(__builtin_amdgcn_readlane(pick(qidx, slot >> 6), slot & 63), true);
                    }
                }
                if (slot >= 0) {
#pragma unroll
                    for (int s = 0; s < QPL; ++s) {
                        const bool mine = lane + 64 * s == slot;
                        qocc[s] = qocc[s] || mine;
                        qcost[s] = mine ? cost : qcost[s];
                        qseq[s] = mine ? cseq : qseq[s];
                        qidx[s] = mine ? x : qidx[s];
                    }
                } else {
                    set_free(x, true);
                }
            }
            __syncthreads();
        }

        if (threadIdx.x == 0) {
            a.out.dist[wi.out] = (int32_t)best;
            if (a.out.cand) a.out.cand[wi.out] = solves;
        }
        if (wv == 0) {
#pragma unroll
            for (int k = 0; k < CPL; ++k)
                if (lane + 64 * k < n1) a.out.map[wi.map_off + lane + 64 * k] = bestphi[k];
        }
        __syncthreads();
    }
}

template <int PL, int CPL, int QPL>
const void *bip_ptr_w(int nwav) {
    if (nwav == 1) return reinterpret_cast<const void *>(&kb_bip_kernel<PL, CPL, QPL, 1>);
    if (nwav == 4) return reinterpret_cast<const void *>(&kb_bip_kernel<PL, CPL, QPL, 4>);
    return nullptr;
}

template <int PL, int CPL>
const void *bip_ptr_q(int qpl, int nwav) {
    if (qpl == 1) return bip_ptr_w<PL, CPL, 1>(nwav);
    if (qpl == 2) return bip_ptr_w<PL, CPL, 2>(nwav);
    if (qpl == 4) return bip_ptr_w<PL, CPL, 4>(nwav);
    return nullptr;
}

template <int PL>
const void *bip_ptr_c(int cpl, int qpl, int nwav) {
    if (cpl == 1) return bip_ptr_q<PL, 1>(qpl, nwav);
    if (cpl == 2) return bip_ptr_q<PL, 2>(qpl, nwav);
    if (cpl == 3) return bip_ptr_q<PL, 3>(qpl, nwav);
    if (cpl == 4) return bip_ptr_q<PL, 4>(qpl, nwav);
    return nullptr;
}

const void *select_bip(int PL, int cpl, int qpl, int nwav) {
    if (PL == 0) return bip_ptr_c<0>(cpl, qpl, nwav);
    if (PL == 2) return bip_ptr_c<2>(cpl, qpl, nwav);
    if (PL == 4) return bip_ptr_c<4>(cpl, qpl, nwav);
    return nullptr;
}

}  // namespace

hipError_t bip_max_resident(int PL, int cpl, int K, int nwav, int *blocks_per_cu) {
    const void *k = select_bip(PL, cpl, bip_queue_words(K), nwav);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64 * nwav, 0);
}

hipError_t launch_bip(int PL, int cpl, int nwav, const DbView &src, const DbView &dst, const WorkItem *work,
                      int nwork, int *queue, Costs c, int K, void *ws, Outputs out, int grid, hipStream_t stream) {
    const void *k = select_bip(PL, cpl, bip_queue_words(K), nwav);
    if (!k || grid <= 0 || K < 1 || K > kBipMaxK || !ws) return hipErrorInvalidValue;
    BipArgs a;
    a.src = src;
    a.dst = dst;
    a.work = work;
    a.nwork = nwork;
    a.queue = queue;
    a.c = c;
    a.K = K;
    a.pad = 0;
    a.node_bytes = bip_node_bytes(cpl, K);
    a.ws = static_cast<unsigned char *>(ws);
    a.out = out;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(grid), dim3(64 * nwav), args, 0, stream);
}

}  // namespace gedk
