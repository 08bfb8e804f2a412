// kb_bip.hip -- the bipartite K-best-assignment bound of graph edit distance,
// one wavefront per pair (n1 + n2 <= 64, K <= 64).
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
// column is always assigned.  Without edge labels a substitution entry
// simplifies to edel d1 - vins + D + vsub [labels differ] - (edel + eins) mm
// (the eins d2 terms cancel), so each lane computes its entry of the scanned
// row on the fly from the row's degree and label; with edge labels the
// matrix of g1's rows is built once in LDS, in 16-bit entries when the costs
// keep every entry below 2^16 (else 32-bit).
//
// Lane layout: lane j holds column j's potential v, its row p (-1 when free)
// and its forbidden-row mask; lane i holds row i's potential u; lane q holds
// queue slot q's key (assignment cost, creation number).  A row is inserted
// by a Dijkstra search over reduced costs: per step each lane forms its
// column's entry of the scanned row, then a DPP minimum and a ballot give the
// first column of least distance, and the potentials of the tree's rows and
// columns are updated, all lane-parallel.
//
// Murty's partitioning runs over g1's rows: a popped subproblem's free rows
// r_0 < r_1 < ... each give one child with r_0 .. r_{t-1} fixed to their
// columns and (r_t, its column) forbidden, solved from the parent's
// potentials with that one row re-inserted.  Queue nodes (potentials,
// assignment, fixed rows, forbidden pairs) live in a per-wave slice of the
// workspace; only the K - popped least keys can still be popped, so K slots
// suffice (a full queue evicts its largest key).  Each popped mapping is
// scored by its induced cost with bitset rows: the images of each vertex's
// earlier neighbours against the image's g2 row.
#include <algorithm>
#include <type_traits>

#include "ged_internal.h"
#include "wave_common.h"

namespace gedk {
namespace {

using namespace wv;

constexpr uint32_t BINF = 0x7fffffffu;   // closed entry / unreached column
constexpr uint32_t C16_CLOSED = 0xffffu;  // closed entry of the 16-bit matrix

// node layout inside a queue slot of kBipNodeBytes
constexpr int kNodeU = 0;       // int32 [64] row potentials
constexpr int kNodeV = 256;     // int32 [64] column potentials
constexpr int kNodeP = 512;     // int8 [64] row on each column
constexpr int kNodeFix = 576;   // uint64 fixed rows
constexpr int kNodeNf = 584;    // int32 forbidden pairs
constexpr int kNodeForb = 640;  // uint16 [64] forbidden (row | column << 8)
static_assert(kNodeForb + 128 <= kBipNodeBytes, "queue node layout");

struct BipArgs {
    DbView src;
    DbView dst;
    const WorkItem *work;
    int nwork;
    int *queue;
    Costs c;
    int K;
    unsigned char *ws;   // grid x K x kBipNodeBytes
    Outputs out;
};

__device__ __forceinline__ uint64_t load_row(const uint32_t *A, int w, int v) {
    const uint64_t lo = A[(size_t)v * w];
    const uint64_t hi = w > 1 ? A[(size_t)v * w + 1] : 0u;
    return lo | (hi << 32);
}

__device__ __forceinline__ uint64_t shfl64(uint64_t x, int l) {
    const uint32_t lo = (uint32_t)__shfl((int)(uint32_t)x, l);
    const uint32_t hi = (uint32_t)__shfl((int)(uint32_t)(x >> 32), l);
    return (uint64_t)lo | ((uint64_t)hi << 32);
}

__device__ __forceinline__ uint64_t low_bits(int n) { return n >= 64 ? ~0ull : ((1ull << n) - 1ull); }

template <int PL, bool C16>
__global__ __launch_bounds__(64) void kb_bip_kernel(BipArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    using Entry = typename std::conditional<C16, uint16_t, int32_t>::type;
    // rows of g1's vertices (edge labels only; one row otherwise, unused)
    __shared__ Entry s_C[PL > 0 ? 64 : 1][64];
    __shared__ int s_col[64];         // column of each row of the popped assignment
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const int32_t vsub = a.c.vsub, vdel = a.c.vdel, vins = a.c.vins;
    const int32_t esub = a.c.esub, edel = a.c.edel, eins = a.c.eins;
    const int32_t cross = min(esub, edel + eins);
    const int K = a.K;
    const int P = a.dst.planes;
    unsigned char *ws = a.ws + (size_t)blockIdx.x * (size_t)K * kBipNodeBytes;

    for (bool first = true;; first = false) {
        int item = (int)blockIdx.x;
        if (!first) {
            if (lane == 0) s_item = (int)gridDim.x + atomicAdd(a.queue, 1);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
        }
        if (item >= a.nwork) break;

        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.src.graphs[wi.src];
        const GraphRec g2 = a.dst.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n, M = n1 + n2;
        const uint32_t *A1 = a.src.adj + g1.adj;
        const uint32_t *A2 = a.dst.adj + g2.adj;
        const uint64_t r1 = lane < n1 ? load_row(A1, g1.w, lane) : 0ull;
        const uint64_t r2 = lane < n2 ? load_row(A2, g2.w, lane) : 0ull;
        const int l1 = lane < n1 ? a.src.vlab[g1.vlab + lane] : 0;
        const int l2 = lane < n2 ? a.dst.vlab[g2.vlab + lane] : 0;
        uint64_t p1[PLA], p2[PLA];
#pragma unroll
        for (int b = 0; b < PLA; ++b) {
            p1[b] = (PL > 0 && b < P && lane < n1) ? load_row(A1 + (size_t)(1 + b) * n1 * g1.w, g1.w, lane) : 0ull;
            p2[b] = (PL > 0 && b < P && lane < n2) ? load_row(A2 + (size_t)(1 + b) * n2 * g2.w, g2.w, lane) : 0ull;
        }
        const int d1 = __popcll(r1), d2 = __popcll(r2);

        // ---------------- cost matrix
        // incident-edge label counts, one byte per label code
        constexpr int NL = PL > 0 ? (1 << PL) : 1;
        uint32_t cnt1[(NL + 3) / 4], cnt2[(NL + 3) / 4];
#pragma unroll
        for (int k = 0; k < (NL + 3) / 4; ++k) cnt1[k] = cnt2[k] = 0u;
        if (PL > 0) {
#pragma unroll
            for (int L = 0; L < NL; ++L) {
                uint64_t m1 = r1, m2 = r2;
#pragma unroll
                for (int b = 0; b < PLA; ++b) {
                    m1 &= ((L >> b) & 1) ? p1[b] : ~p1[b];
                    m2 &= ((L >> b) & 1) ? p2[b] : ~p2[b];
                }
                cnt1[L >> 2] |= (uint32_t)__popcll(m1) << (8 * (L & 3));
                cnt2[L >> 2] |= (uint32_t)__popcll(m2) << (8 * (L & 3));
            }
        }
        const int32_t ins = vins + eins * d2;
        const int32_t D = (int32_t)wave_umax(lane < n2 ? (uint32_t)ins : 0u);
        for (int i = 0; i < (PL > 0 ? n1 : 0); ++i) {
            const int d1i = __builtin_amdgcn_readlane(d1, i);
            const int l1i = __builtin_amdgcn_readlane(l1, i);
            const int mm = min(d1i, d2);
            int common = mm;
            if (PL > 0) {
                common = 0;
#pragma unroll
                for (int k = 0; k < (NL + 3) / 4; ++k) {
                    const uint32_t c1 = (uint32_t)__builtin_amdgcn_readlane((int)cnt1[k], i);
#pragma unroll
                    for (int s = 0; s < 4; ++s)
                        common += (int)min(__builtin_amdgcn_ubfe(c1, 8u * s, 8u), __builtin_amdgcn_ubfe(cnt2[k], 8u * s, 8u));
                }
            }
            int32_t val = (int32_t)(C16 ? C16_CLOSED : BINF);
            if (lane < n2)
                val = (l1i != l2 ? vsub : 0) + edel * (d1i - mm) + eins * (d2 - mm) + cross * (mm - common) - ins + D;
            else if (lane == n2 + i)
                val = vdel + edel * d1i + D;
            s_C[i][lane] = (Entry)val;
        }
        __syncthreads();
        // entry (i, lane) of a g1 row; BINF where closed
        const int32_t rowbase_c = -vins + D;   // + edel d1(i): substitution entries without edge labels
        const int32_t ed_ei = edel + eins;
        auto entry = [&](int i) -> uint32_t {
            if (PL > 0) {
                const uint32_t e = (uint32_t)s_C[i][lane];
                return (C16 && e == C16_CLOSED) ? BINF : e;
            }
            const int d1i = __builtin_amdgcn_readlane(d1, i);
            const int l1i = __builtin_amdgcn_readlane(l1, i);
            const uint32_t sub = (uint32_t)(rowbase_c + edel * d1i + (l1i != l2 ? vsub : 0) - ed_ei * min(d1i, d2));
            const uint32_t del = lane == n2 + i ? (uint32_t)(vdel + edel * d1i + D) : BINF;
            return lane < n2 ? sub : del;
        };

        // ---------------- Hungarian row insertion (shortest augmenting path)
        // u: row potential of lane i; v, p: column lane j.  colfm: rows
        // forbidden on column lane j; blocked: column lane j belongs to a fixed
        // row.
        //
        // Reduced costs stay below (n1 + n2 + 1) times the largest entry
        // (potentials: u >= 0 grows, v <= 0 falls, |v| at most the assignment
        // cost), which the host keeps below 2^26; so (distance << 6 | column)
        // is one 32-bit key whose wave minimum gives both the least distance
        // and the lowest column holding it.  Per lane the step is branch-free.
        auto augment = [&](int r, int32_t &u, int32_t &v, int &p, uint64_t colfm, bool blocked) -> bool {
            uint32_t minv = BINF;
            int way = -1;
            bool used = false;
            bool live = lane < M && !blocked;   // may still be reached (not used, not closed)
            bool intree = lane == r;
            int i0 = r, j0 = -1;
            for (;;) {
                const int32_t ui0 = __builtin_amdgcn_readlane(u, i0);
                const uint32_t cst = i0 < n1 ? entry(i0) : 0u;
                const bool allow = live && !((colfm >> i0) & 1ull) && cst != BINF;
                const uint32_t cur = (uint32_t)((int32_t)cst - ui0 - v);
                const bool better = allow && cur < minv;
                minv = better ? cur : minv;
                way = better ? j0 : way;
                const bool reach = live && minv != BINF;
                const uint32_t key = wave_umin(reach ? ((minv << 6) | (uint32_t)lane) : 0xffffffffu);
                if (key == 0xffffffffu) return false;
                const uint32_t delta = key >> 6;
                const int j1 = (int)(key & 63u);
                u += intree ? (int32_t)delta : 0;
                v -= used ? (int32_t)delta : 0;
                minv -= reach ? delta : 0u;
                used = used || lane == j1;
                live = live && lane != j1;
                j0 = j1;
                const int pj = __builtin_amdgcn_readlane(p, j1);
                if (pj < 0) break;
                i0 = pj;
                intree = intree || lane == i0;
            }
            // flip the path back to r
            while (j0 >= 0) {
                const int jp = __builtin_amdgcn_readlane(way, j0);
                const int np = jp < 0 ? r : __builtin_amdgcn_readlane(p, jp);
                if (lane == j0) p = np;
                j0 = jp;
            }
            return true;
        };
        auto assignment_cost = [&](int p) -> uint32_t {
            const bool real = lane < M && p >= 0 && p < n1;
            uint32_t e = 0u;
            if (PL > 0) {
                e = real ? (uint32_t)s_C[p][lane] : 0u;
            } else {
                // every lane shuffles (sources outside the branch's lanes)
                const int pp = real ? p : 0;
                const int d1p = __shfl(d1, pp), l1p = __shfl(l1, pp);
                if (real)
                    e = lane < n2 ? (uint32_t)(rowbase_c + edel * d1p + (l1p != l2 ? vsub : 0) - ed_ei * min(d1p, d2))
                                  : (uint32_t)(vdel + edel * d1p + D);
            }
            return wave_sum(e);
        };

        // ---------------- first assignment: every row from zero potentials
        int32_t u = 0, v = 0;
        int p = -1;
        for (int r = 0; r < M; ++r) (void)augment(r, u, v, p, 0ull, false);   // a deletion column is always open
        uint32_t qcost = 0u, qseq = 0u;
        bool qocc = false;
        {
            unsigned char *nb = ws;
            if (lane < 64) {
                reinterpret_cast<int32_t *>(nb + kNodeU)[lane] = u;
                reinterpret_cast<int32_t *>(nb + kNodeV)[lane] = v;
                reinterpret_cast<int8_t *>(nb + kNodeP)[lane] = (int8_t)p;
            }
            if (lane == 0) {
                *reinterpret_cast<uint64_t *>(nb + kNodeFix) = 0ull;
                *reinterpret_cast<int32_t *>(nb + kNodeNf) = 0;
            }
            const uint32_t c0 = assignment_cost(p);
            if (lane == 0) {
                qocc = true;
                qcost = c0;
                qseq = 0u;
            }
        }
        uint32_t seq = 1u;
        int popped = 0;
        int64_t solves = 1;
        uint32_t best = BINF;
        int bestphi = -1;

        while (popped < K) {
            if (__ballot(qocc) == 0ull) break;
            // ---------------- pop the least (cost, creation number)
            const uint32_t mc = wave_umin(qocc ? qcost : 0xffffffffu);
            const uint32_t ms = wave_umin(qocc && qcost == mc ? qseq : 0xffffffffu);
            const int q = (int)__builtin_ctzll(__ballot(qocc && qcost == mc && qseq == ms));
            if (lane == q) qocc = false;
            const unsigned char *nq = ws + (size_t)q * kBipNodeBytes;
            const int32_t u_par = reinterpret_cast<const int32_t *>(nq + kNodeU)[lane];
            const int32_t v_par = reinterpret_cast<const int32_t *>(nq + kNodeV)[lane];
            const int p_par = lane < M ? (int)reinterpret_cast<const int8_t *>(nq + kNodeP)[lane] : -1;
            const uint64_t fixm = *reinterpret_cast<const uint64_t *>(nq + kNodeFix);
            const int nf = *reinterpret_cast<const int32_t *>(nq + kNodeNf);
            const uint32_t fent = lane < nf ? reinterpret_cast<const uint16_t *>(nq + kNodeForb)[lane] : 0u;
            uint64_t colfm = 0ull;
            for (int k = 0; k < nf; ++k) {
                const uint32_t e = (uint32_t)__builtin_amdgcn_readlane((int)fent, k);
                if (lane == (int)(e >> 8)) colfm |= 1ull << (e & 0xffu);
            }
            if (p_par >= 0) s_col[p_par] = lane;
            __syncthreads();
            const int colr = lane < n1 ? s_col[lane] : -1;
            __syncthreads();

            // ---------------- its mapping and induced edit cost
            const int phi = (lane < n1 && colr < n2) ? colr : -1;
            const int ph = phi >= 0 ? phi : 0;
            const int l2p = __shfl(l2, ph);
            const uint64_t R = shfl64(r2, ph);
            uint64_t Phi = 0ull, PhiB[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) PhiB[b] = 0ull;
            for (int b = 0; b < n1; ++b) {
                const int pb = __builtin_amdgcn_readlane(phi, b);
                if (pb < 0 || b >= lane || !((r1 >> b) & 1ull)) continue;
                Phi |= 1ull << pb;
#pragma unroll
                for (int pl = 0; pl < PLA; ++pl)
                    if (PL > 0 && ((p1[pl] >> b) & 1ull)) PhiB[pl] |= 1ull << pb;
            }
            const bool sub = phi >= 0;
            const uint32_t matched = sub ? (uint32_t)__popcll(Phi & R) : 0u;
            uint32_t mism = 0u;
            if (PL > 0) {
                uint64_t diff = 0ull;
#pragma unroll
                for (int pl = 0; pl < PLA; ++pl) diff |= PhiB[pl] ^ shfl64(p2[pl], ph);   // every lane shuffles
                mism = sub ? (uint32_t)__popcll(Phi & R & diff) : 0u;
            }
            const uint32_t early = lane < n1 ? (uint32_t)__popcll(r1 & low_bits(lane)) : 0u;
            uint32_t lc = 0u;
            if (lane < n1)
                lc = (sub ? (l1 != l2p ? (uint32_t)vsub : 0u) : (uint32_t)vdel) + (uint32_t)edel * (early - matched) +
                     (uint32_t)esub * mism;
            const uint32_t nsub = (uint32_t)__popcll(__ballot(lane < n1 && sub));
            const uint32_t d = wave_sum(lc) + (uint32_t)vins * ((uint32_t)n2 - nsub) +
                               (uint32_t)eins * ((uint32_t)g2.m - wave_sum(matched));
            ++popped;
            if (d < best) {
                best = d;
                bestphi = phi;
            }
            if (popped == K) break;

            // ---------------- partition: one child per free row, ascending
            uint64_t freem = low_bits(n1) & ~fixm;
            uint64_t cfix = fixm;
            bool blocked = p_par >= 0 && p_par < n1 && ((fixm >> p_par) & 1ull);
            while (freem) {
                const int r = (int)__builtin_ctzll(freem);
                freem &= freem - 1ull;
                const int c = __builtin_amdgcn_readlane(colr, r);
                int32_t cu = u_par, cv = v_par;
                int cp = lane == c ? -1 : p_par;
                const uint64_t cfm = colfm | (lane == c ? (1ull << r) : 0ull);
                ++solves;
                if (augment(r, cu, cv, cp, cfm, blocked)) {
                    const uint32_t cost = assignment_cost(cp);
                    const uint32_t cseq = seq++;
                    const int cap = K - popped;
                    const int occn = __popcll(__ballot(qocc));
                    int slot = -1;
                    if (occn < cap) {
                        slot = (int)__builtin_ctzll(__ballot(!qocc && lane < K));
                    } else {
                        // the child's creation number exceeds every queued one,
                        // so it displaces the largest key only when cheaper
                        const uint32_t xc = wave_umax(qocc ? qcost : 0u);
                        const uint32_t xs = wave_umax(qocc && qcost == xc ? qseq : 0u);
                        if (cost < xc) slot = (int)__builtin_ctzll(__ballot(qocc && qcost == xc && qseq == xs));
                    }
                    if (slot >= 0) {
                        unsigned char *nb = ws + (size_t)slot * kBipNodeBytes;
                        reinterpret_cast<int32_t *>(nb + kNodeU)[lane] = cu;
                        reinterpret_cast<int32_t *>(nb + kNodeV)[lane] = cv;
                        reinterpret_cast<int8_t *>(nb + kNodeP)[lane] = (int8_t)cp;
                        if (lane == 0) {
                            *reinterpret_cast<uint64_t *>(nb + kNodeFix) = cfix;
                            *reinterpret_cast<int32_t *>(nb + kNodeNf) = nf + 1;
                        }
                        if (lane <= nf)
                            reinterpret_cast<uint16_t *>(nb + kNodeForb)[lane] =
                                (uint16_t)(lane < nf ? fent : ((uint32_t)r | ((uint32_t)c << 8)));
                        if (lane == slot) {
                            qocc = true;
                            qcost = cost;
                            qseq = cseq;
                        }
                    }
                }
                cfix |= 1ull << r;
                if (lane == c) blocked = true;
            }
        }

        if (lane == 0) {
            a.out.dist[wi.out] = (int32_t)best;
            if (a.out.cand) a.out.cand[wi.out] = solves;
        }
        if (lane < n1) a.out.map[wi.map_off + lane] = bestphi;
        __syncthreads();
    }
}

template <int PL, bool C16>
const void *bip_ptr() {
    return reinterpret_cast<const void *>(&kb_bip_kernel<PL, C16>);
}

const void *select_bip(int PL, bool c16) {
    if (PL == 0) return bip_ptr<0, true>();   // no matrix: one instantiation
    if (PL == 2) return c16 ? bip_ptr<2, true>() : bip_ptr<2, false>();
    if (PL == 4) return c16 ? bip_ptr<4, true>() : bip_ptr<4, false>();
    return nullptr;
}

// every matrix entry below the 16-bit closed marker: an entry is at most
// max(vsub, vdel) + (edel + eins + cross) * 63 + (vins + eins * 63)
bool entries_fit_16(const Costs &c) {
    const int64_t cross = std::min<int64_t>(c.esub, (int64_t)c.edel + c.eins);
    const int64_t top = std::max<int64_t>(c.vsub, c.vdel) + ((int64_t)c.edel + c.eins + cross) * 63 + c.vins +
                        (int64_t)c.eins * 63;
    return top < (int64_t)C16_CLOSED;
}

}  // namespace

// grids are sized for the 16-bit matrix; with larger costs the 32-bit
// instantiation holds fewer waves and the rest start as others finish
hipError_t bip_max_resident(int PL, int *blocks_per_cu) {
    const void *k = select_bip(PL, true);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64, 0);
}

hipError_t launch_bip(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue,
                      Costs c, int K, void *ws, Outputs out, int grid, hipStream_t stream) {
    const void *k = select_bip(PL, entries_fit_16(c));
    if (!k || grid <= 0 || K < 1 || K > kBipMaxK || !ws) return hipErrorInvalidValue;
    BipArgs a;
    a.src = src;
    a.dst = dst;
    a.work = work;
    a.nwork = nwork;
    a.queue = queue;
    a.c = c;
    a.K = K;
    a.ws = static_cast<unsigned char *>(ws);
    a.out = out;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, stream);
}

}  // namespace gedk
