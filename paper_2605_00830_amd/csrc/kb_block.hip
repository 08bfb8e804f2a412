// kb_block.hip -- workgroup-per-pair K-Best search for gfx950 (any shape up
// to 512 vertices and K = 1024).
//
// One 256-thread workgroup searches one pair at a time: first the pair at
// its own index, then further pairs from a work queue (persistent launch).
// Beam slots are spread over the threads: G = min(KS, 256) slots per round,
// TPS = 256 / G threads per slot (thread t = slot-in-round * TPS + part),
// each part owning a contiguous range of the slot's children (substitutions
// by ascending free g2 vertex -- child j substitutes the slot's j-th unused
// vertex -- the deletion last), so thread order is generation order and only
// valid children are ever evaluated.
// Per level i (the loop of Alg. 1, g1 vertex v_i):
//   expand    every thread builds its slot's Phi = image of v_i's earlier
//             neighbours (one bit per g2 vertex, one set per edge-label
//             plane) and scores its children by the implied edge operations
//             of Sec. 2.3 / Alg. 2 as popcounts of word-wise ANDs against
//             g2's rows (staged in LDS):
//               kept   = |Phi & N2(u)|             edges kept (maybe relabelled)
//               del    = |P(v_i)| - kept           g1 edges deleted
//               ins    = |Img & N2(u)| - kept      g2 edges inserted
//               relab  = |Phi & N2(u) & label-mismatch|
//             The deletion child costs vdel + edel*|P(v_i)| (Sec. 4.2.1).
//             Each child also lands in an LDS histogram of 1024 bins above
//             the least parent PED (a lower bound of every child).
//   select    the K best children (Sec. 4.3) without sorting: T = K-th
//             smallest PED from the histogram (further windows from the
//             least value above it when needed), every child below T, and
//             the first (K - #below) children equal to T in generation order
//             (exclusive block scans).  Survivors are compacted in generation
//             order, so the beam stays ordered.
//   update    survivors copy their parent's mapping and add one entry (the
//             paper's update step, Sec. 4.4.2).
// At the end every slot adds the insertion costs of the unmatched g2
// vertices and edges (Sec. 4.4.1) and a block arg-min picks the result.
//
// LDS holds g2's rows padded to W words (read with vector loads, no bounds
// tests), its label planes when they fit, and the candidate matrix as
// cand[s][j] (child j of slot s; odd row stride, so the parts of a wave hit
// different banks) when everything fits 136 KB (CL); otherwise the candidate
// matrix lives in the per-block global workspace as cand[j][s] (consecutive
// slots coalesce).
// Beam state per slot in the workspace (slot-minor): PED, |Img|, g2 edges
// inside Img, Img bitset, mapping phi[j] (uint16, 0xffff = deleted).
//
// Directed graphs (each edge an arc, one edit operation per arc): the
// database holds a second block of rows and planes after the first, row v of
// it the in-arcs of v.  Here a vertex's row is its out-row in words
// [0, W/2) followed by its in-row in words [W/2, W), the image bitset holds
// Img in both halves, and an earlier neighbour of v_i reached by an in-arc
// sets its Phi bit in the upper half.  The same popcounts then count kept,
// deleted, inserted and relabelled arcs of both directions at once: the
// implied operations of Sec. 2.3 taken for each arc direction.
#include "ged_internal.h"

namespace gedk {
namespace {

constexpr int NBINS = 1024;
// beam-state loads a thread issues together: many for large graphs, whose
// beam state lives in HBM and whose levels are long; few for small ones,
// whose occupancy the extra registers would cut (and fewer again where the
// sets already take most registers)
template <int W, int PL, int BT>
constexpr int loads_together() { return W < 8 ? 2 : (BT >= 1024 ? 4 : (W * (1 + PL) >= 64 ? 8 : 16)); }
constexpr int SENT = 0x7fffffff;        // above every partial edit distance (empty minima)
constexpr uint16_t PHI_DEL = 0xffff;
constexpr size_t kDynLdsBytes = 136 * 1024;    // rows, staged planes, candidate matrix
constexpr size_t kPlaneLdsBytes = 48 * 1024;   // rows plus planes staged when they fit this

struct WsLayout {
    size_t ped, ein, nsub, img, phi, cand, stride;
    size_t phi_half;                     // elements per phi ping-pong half
};

struct BlockArgs {
    DbView src;    // graphs edited (g1)
    DbView dst;    // target graphs (g2); same edge-label coding as src
    const WorkItem *work;
    int nwork;
    int *queue;
    Costs c;
    int K;
    int last_complete;   // last level: complete every child, keep the least total
    int KS;        // slot stride
    int TPS;       // threads per slot
    int rows_words;   // LDS words per staged block of g2 rows (nmax2 x row_stride(W))
    int planes_lds;   // label planes staged in LDS after the rows
    char *ws;
    WsLayout L;
    Outputs out;
};

__device__ __forceinline__ int wave_min(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v = min(v, __shfl_xor(v, o));
    return v;
}

__device__ __forceinline__ int wave_sum(int v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int y = __shfl_up(v, o);
        if (lane >= o) v += y;
    }
    return v;
}

template <int NW>
__device__ __forceinline__ int block_min(int v, int *red) {
    v = wave_min(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = red[0];
#pragma unroll
    for (int k = 1; k < NW; ++k) r = min(r, red[k]);
    __syncthreads();
    return r;
}

template <int NW>
__device__ __forceinline__ int block_sum(int v, int *red) {
    v = wave_sum(v);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    int r = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) r += red[k];
    __syncthreads();
    return r;
}

// Exclusive scan over threads in index order; *total gets the block sum.
template <int NW>
__device__ __forceinline__ int block_excl_scan(int v, int *red, int *total) {
    const int incl = wave_incl_scan(v);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 63) red[w] = incl;
    __syncthreads();
    int base = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const int x = red[k];
        base += (k < w) ? x : 0;
        tot += x;
    }
    __syncthreads();
    *total = tot;
    return base + incl - v;
}

__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long v) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned lo = (unsigned)__shfl_xor((int)(unsigned)v, o);
        const unsigned hi = (unsigned)__shfl_xor((int)(unsigned)(v >> 32), o);
        const unsigned long long w = ((unsigned long long)hi << 32) | lo;
        v = w < v ? w : v;
    }
    return v;
}

__device__ __forceinline__ uint32_t below_mask(int i, int kw) {
    const int rem = i - kw * 32;
    return rem >= 32 ? 0xffffffffu : ((1u << rem) - 1u);
}

// The free g2 vertices of a slot -- vertices below n2 whose bit in the first
// NWF words of Img is clear -- in ascending order, from a given rank on.  A
// slot's substitution children are its free vertices in this order (the
// deletion child comes last), so child j substitutes the j-th free vertex.
// Word selection is unrolled: no register array is indexed dynamically.
// LDS stride of a staged row of W words: rows of 8 or more words are padded
// by four words, so that lanes reading the rows of different vertices (each
// lane visits its own slot's free vertices) start on different banks; the
// stride stays a multiple of four words for 16-byte loads.
__host__ __device__ constexpr int row_stride(int W) { return W >= 8 ? W + 4 : W; }

template <int W, int NWF>
struct FreeIter {
    uint32_t fr = 0u;   // free bits of word cw not yet visited
    int cw = 0;         // current word

    __device__ __forceinline__ static uint32_t free_word(const uint32_t (&img)[W], int k, int n2) {
        uint32_t w = 0u;
#pragma unroll
        for (int q = 0; q < NWF; ++q) w = (q == k) ? img[q] : w;
        const int rem = n2 - 32 * k;
        const uint32_t valid = rem >= 32 ? 0xffffffffu : (rem <= 0 ? 0u : ((1u << rem) - 1u));
        return ~w & valid;
    }
    // position before the free vertex of rank j0
    __device__ __forceinline__ void seek(const uint32_t (&img)[W], int n2, int j0) {
        cw = 0;
        fr = free_word(img, 0, n2);
        for (;;) {
            const int c = __popc(fr);
            if (j0 < c || cw >= NWF - 1) break;
            j0 -= c;
            ++cw;
            fr = free_word(img, cw, n2);
        }
        for (; j0 > 0 && fr; --j0) fr &= fr - 1u;
    }
    // the next free vertex (the caller asks only while one remains)
    __device__ __forceinline__ int next(const uint32_t (&img)[W], int n2) {
        while (fr == 0u && cw < NWF - 1) {
            ++cw;
            fr = free_word(img, cw, n2);
        }
        const int u = 32 * cw + (int)__builtin_ctzg(fr, 31);
        fr &= fr - 1u;
        return u;
    }
};

template <int W, int PL, bool CL, int BT, bool DIR>
__global__ __launch_bounds__(BT) void kb_block_kernel(BlockArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    constexpr int NW = BT / 64;
    extern __shared__ uint32_t s_dyn[];   // g2 rows, then (CL) the candidate matrix
    __shared__ int s_sel[GED_MAX_K];      // survivor: parent slot << 10 | child (n2 = deletion)
    __shared__ int s_selped[GED_MAX_K];   // survivor partial edit distance
    __shared__ int s_hist[NBINS];
    __shared__ uint16_t s_nbr[GED_MAX_VERTICES_BATCH];   // earlier neighbours of v_i
    __shared__ uint8_t s_nbl[GED_MAX_VERTICES_BATCH];    // their edge-label codes
    __shared__ int s_lc[GED_MAX_VERTICES_BATCH];         // vertex cost of substituting v_i by u
    __shared__ int s_red[NW];
    __shared__ unsigned long long s_red64[NW];
    __shared__ int s_bc[4];

    const int t = threadIdx.x;
    char *wsb = a.ws + (size_t)blockIdx.x * a.L.stride;
    int *ped_b = reinterpret_cast<int *>(wsb + a.L.ped);
    int *ein_b = reinterpret_cast<int *>(wsb + a.L.ein);
    int *nsub_b = reinterpret_cast<int *>(wsb + a.L.nsub);
    uint32_t *img_b = reinterpret_cast<uint32_t *>(wsb + a.L.img);
    uint16_t *phi_b = reinterpret_cast<uint16_t *>(wsb + a.L.phi);
    int *__restrict__ cand_g = reinterpret_cast<int *>(wsb + a.L.cand);
    constexpr int RS = row_stride(W);
    uint32_t *s_rows = s_dyn;             // row u at u * RS, padded with zero words
    uint32_t *s_planes = s_dyn + a.rows_words;
    int *cand_l = reinterpret_cast<int *>(s_dyn + a.rows_words * (1 + (a.planes_lds ? PL : 0)));
    const int KS = a.KS;
    const int TPS = a.TPS;
    const int G = BT / TPS;              // slots per round
    const int SPT = KS / G;              // rounds
    const int sg = t / TPS;              // slot within a round
    const int part = t % TPS;
    const int K = a.K;
    const Costs c = a.c;
    const int P = a.dst.planes;
    constexpr int DH = DIR ? W / 2 : 0;   // first word of the in-half (directed)
    constexpr int NWF = DIR ? W / 2 : W;  // words of Img that name g2 vertices
    constexpr int LB = loads_together<W, PL, BT>();
    // the keep, compaction and mapping-copy passes hold few other values: at
    // 1024 threads, where the expansion's registers keep LB at 4, they batch 8
    constexpr int LBK = BT >= 1024 ? 8 : LB;
    static_assert(!DIR || W >= 2, "a directed row has two halves");

    for (bool first = true;; first = false) {
        // the first pair is the workgroup's own index; later ones come from
        // the queue (taking every first pair from one shared counter would
        // serialise the grid's start on one atomic)
        int item = (int)blockIdx.x;
        if (!first) {
            if (t == 0) s_bc[0] = pull_item(a.queue, a.nwork);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_bc[0]);
            __syncthreads();
        }
        if (item >= a.nwork) break;

        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.src.graphs[wi.src];
        const GraphRec g2 = a.dst.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n, w1 = g1.w, w2 = g2.w;
        const uint32_t *A1 = a.src.adj + g1.adj;
        const uint32_t *A2 = a.dst.adj + g2.adj;
        const int *L1 = a.src.vlab + g1.vlab;
        const int *L2 = a.dst.vlab + g2.vlab;
        const size_t pl1 = (size_t)n1 * w1, pl2 = (size_t)n2 * w2;
        // directed: the in-arc rows and planes follow the out-arc ones
        const uint32_t *A1in = A1 + (size_t)(1 + a.src.planes) * pl1;
        const uint32_t *A2in = A2 + (size_t)(1 + P) * pl2;
        const int nc = n2 + 1;                       // most children of a slot (deletion last)
        const int CST = nc | 1;                      // LDS row stride of the candidate matrix
        // a slot with `ns` substitutions so far has n2 - ns + 1 children;
        // part `part` of its threads owns a contiguous range of them
        auto part_range = [&](int ns, int *jlo, int *jhi) {
            const int ncs = n2 - ns + 1;
            const int ch = (ncs + TPS - 1) / TPS;
            *jlo = min(part * ch, ncs);
            *jhi = min(*jlo + ch, ncs);
            return ncs;
        };

        for (int x = t; x < n2 * RS; x += BT) {
            const int u = x / RS, kk = x % RS;
            const bool hi = DH > 0 && kk >= DH;
            const int kr = hi ? kk - DH : kk;
            s_rows[x] = (kk < W && kr < w2) ? (hi ? A2in : A2)[(size_t)u * w2 + kr] : 0u;
        }
        if (PL > 0 && a.planes_lds) {
            for (int x = t; x < PL * n2 * RS; x += BT) {
                const int b = x / (n2 * RS), r = x % (n2 * RS), u = r / RS, kk = r % RS;
                const bool hi = DH > 0 && kk >= DH;
                const int kr = hi ? kk - DH : kk;
                s_planes[(size_t)b * a.rows_words + r] =
                    (b < P && kk < W && kr < w2) ? (hi ? A2in : A2)[(size_t)(1 + b) * pl2 + (size_t)u * w2 + kr] : 0u;
            }
        }
        if (t == 0) {
            ped_b[0] = 0;
            ein_b[0] = 0;
            nsub_b[0] = 0;
#pragma unroll
            for (int k = 0; k < W; ++k) img_b[(size_t)k * KS] = 0u;
        }
        int nb = 1, cur = 0;
        long long ce = 0;
        __syncthreads();

        for (int i = 0; i < n1; ++i) {
            const int lab1 = L1[i];
            int degP = 0;
            for (int kw = 0; kw * 32 < i; ++kw) degP += __popc(A1[(size_t)i * w1 + kw] & below_mask(i, kw));
            if (DH > 0)
                for (int kw = 0; kw * 32 < i; ++kw) degP += __popc(A1in[(size_t)i * w1 + kw] & below_mask(i, kw));
            const int del_cost = c.vdel + c.edel * degP;
            const bool coop = TPS > 1 && degP >= 2 * TPS;   // split the Phi lookups over a slot's parts
            // the earlier neighbours of v_i (the same for every slot), in index
            // order, with their edge-label codes: listed once per level by wave 0.
            // Directed: the out-arc neighbours, then the in-arc ones with bit 15 set.
            if (t < 64) {
                int base = 0;
                for (int dir = 0; dir < (DH > 0 ? 2 : 1); ++dir) {
                    const uint32_t *R1 = dir ? A1in : A1;
                    for (int kw = 0; kw * 32 < i; ++kw) {
                        const uint32_t bits = R1[(size_t)i * w1 + kw] & below_mask(i, kw);
                        const bool mine = t < 32 && ((bits >> t) & 1u);
                        const unsigned long long m = __ballot(mine);
                        if (mine) {
                            const int rank = (int)__builtin_amdgcn_mbcnt_hi(
                                (unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
                            int code = 0;
#pragma unroll
                            for (int b = 0; b < PLA; ++b)
                                if (PL > 0 && b < P)
                                    code |= (int)((R1[(size_t)(1 + b) * pl1 + (size_t)i * w1 + kw] >> t) & 1u) << b;
                            s_nbr[base + rank] = (uint16_t)((kw * 32 + t) | (dir << 15));
                            s_nbl[base + rank] = (uint8_t)code;
                        }
                        base += __popcll(m);
                    }
                }
            }

            const int *__restrict__ pedc = ped_b + cur * KS;
            const int *__restrict__ nsubc = nsub_b + cur * KS;
            const uint32_t *__restrict__ imgc = img_b + (size_t)cur * W * KS;
            const uint16_t *__restrict__ phic = phi_b + cur * a.L.phi_half;

            // lower bound of every child: the least parent PED
            int lpmin = SENT;
            for (int r = 0; r < SPT; ++r) {
                const int s = r * G + sg;
                if (s < nb && part == 0) lpmin = min(lpmin, pedc[s]);
            }
            for (int b = t; b < NBINS; b += BT) s_hist[b] = 0;
            for (int u = t; u < n2; u += BT) s_lc[u] = lab1 != L2[u] ? c.vsub : 0;
            // also orders the histogram reset, the neighbour list and the label costs
            const int m0 = block_min<NW>(lpmin, s_red);

            // ---------------- expand, evaluate, histogram
            int lcnt = 0, ovmin = SENT;
            for (int r = 0; r < SPT; ++r) {
                const int s = r * G + sg;
                if (s >= nb) break;
                const int pp = pedc[s];
                uint32_t img_r[W];
                uint32_t phi_r[W];
                uint32_t phib[PLA][W];
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    img_r[k] = imgc[(size_t)k * KS + s];
                    phi_r[k] = 0u;
#pragma unroll
                    for (int b = 0; b < PLA; ++b) phib[b][k] = 0u;
                }
                // with many earlier neighbours the slot's parts split them (each
                // part looks up every TPS-th one) and OR their sets together:
                // the parts of a slot are adjacent lanes of one wave
                // (the images are loaded LB at a time, so that many loads are
                // in flight before the first is used)
                const int q0 = coop ? part : 0, qs = coop ? TPS : 1;
                for (int qb = q0; qb < degP; qb += LB * qs) {
                    int xs[LB];
#pragma unroll
                    for (int k = 0; k < LB; ++k) {
                        const int q = qb + k * qs;
                        xs[k] = q < degP ? (int)phic[(size_t)(s_nbr[q] & 0x7fff) * KS + s] : (int)PHI_DEL;
                    }
#pragma unroll
                    for (int k = 0; k < LB; ++k) {
                        const int x = xs[k];
                        if (x == PHI_DEL) continue;   // deleted, or past the list
                        const int q = qb + k * qs;
                        const int nq = s_nbr[q];
                        const uint32_t bit = 1u << (x & 31);
                        const int xw = (x >> 5) + ((nq >> 15) ? DH : 0);
                        const int code = PL > 0 ? s_nbl[q] : 0;
#pragma unroll
                        for (int kk = 0; kk < W; ++kk) {
                            const uint32_t hit = (kk == xw) ? bit : 0u;
                            phi_r[kk] |= hit;
#pragma unroll
                            for (int b = 0; b < PLA; ++b)
                                phib[b][kk] |= ((code >> b) & 1) ? hit : 0u;
                        }
                    }
                }
                if (coop) {
                    for (int o = 1; o < TPS; o <<= 1) {
#pragma unroll
                        for (int k = 0; k < W; ++k) {
                            phi_r[k] |= (uint32_t)__shfl_xor((int)phi_r[k], o);
#pragma unroll
                            for (int b = 0; b < PLA; ++b)
                                if (PL > 0) phib[b][k] |= (uint32_t)__shfl_xor((int)phib[b][k], o);
                        }
                    }
                }
                // this part's children j = jlo .. jhi-1 in generation order: the
                // j-th free g2 vertex, the deletion last (j = ncs - 1); only free
                // vertices are evaluated
                int jlo, jhi;
                const int ncs = part_range(nsubc[s], &jlo, &jhi);
                const int jsub = min(jhi, ncs - 1);
                FreeIter<W, NWF> it;
                it.seek(img_r, n2, jlo);
#pragma unroll 2
                for (int j = jlo; j < jsub; ++j) {
                    const int u = it.next(img_r, n2);
                    const uint32_t *R = s_rows + u * RS;
                    uint32_t row[W];
#pragma unroll
                    for (int kk = 0; kk < W; ++kk) row[kk] = R[kk];
                    int kept = 0, inimg = 0, relab = 0;
#pragma unroll
                    for (int kk = 0; kk < W; ++kk) {
                        const uint32_t both = phi_r[kk] & row[kk];
                        kept += __popc(both);
                        inimg += __popc(img_r[kk] & row[kk]);
                        if (PL > 0) {
                            uint32_t diff = 0u;
                            if (a.planes_lds) {
#pragma unroll
                                for (int bb = 0; bb < PLA; ++bb)
                                    diff |= phib[bb][kk] ^ s_planes[(size_t)bb * a.rows_words + u * RS + kk];
                            } else {
                                const bool hi = DH > 0 && kk >= DH;
                                const int kr = hi ? kk - DH : kk;
                                if (kr < w2) {
                                    const uint32_t *B = hi ? A2in : A2;
#pragma unroll
                                    for (int bb = 0; bb < PLA; ++bb)
                                        if (bb < P) diff |= phib[bb][kk] ^ B[(size_t)(1 + bb) * pl2 + (size_t)u * w2 + kr];
                                }
                            }
                            relab += __popc(both & diff);
                        }
                    }
                    const int d = pp + s_lc[u] + c.edel * (degP - kept) +
                                  c.eins * (inimg - kept) + c.esub * relab;
                    if (CL) cand_l[s * CST + j] = d;
                    else cand_g[(size_t)j * KS + s] = d;
                    ++lcnt;
                    if (d - m0 < NBINS) atomicAdd(&s_hist[d - m0], 1);
                    else ovmin = min(ovmin, d);
                }
                if (jlo < jhi && jhi == ncs) {   // this part owns the deletion child
                    const int dd = pp + del_cost;
                    if (CL) cand_l[s * CST + ncs - 1] = dd;
                    else cand_g[(size_t)(ncs - 1) * KS + s] = dd;
                    ++lcnt;
                    if (dd - m0 < NBINS) atomicAdd(&s_hist[dd - m0], 1);
                    else ovmin = min(ovmin, dd);
                }
            }
            const int V = block_sum<NW>(lcnt, s_red);   // also orders the histogram updates
            ce += V;
            auto cand_at = [&](int s, int u) -> int {
                return CL ? cand_l[s * CST + u] : cand_g[(size_t)u * KS + s];
            };

            int nb_new;
            if (a.last_complete && i == n1 - 1) {
                // ---------------- complete-then-minimum last level: each
                // child's total (Sec. 4.4.1); the least, first in generation
                // order (slot, then column), is the one survivor
                // (key: total, then slot << 20 | child << 10 | vertex; the child
                // rank orders a slot's children as the vertex does)
                const int *einc = ein_b + cur * KS;
                unsigned long long bk = ~0ull;
                for (int r = 0; r < SPT; ++r) {
                    const int s = r * G + sg;
                    if (s >= nb) break;
                    uint32_t img_r[W];
#pragma unroll
                    for (int k = 0; k < W; ++k) img_r[k] = imgc[(size_t)k * KS + s];
                    const int e0 = einc[s], used0 = nsubc[s];
                    int jlo, jhi;
                    const int ncs = part_range(used0, &jlo, &jhi);
                    FreeIter<W, NWF> it;
                    it.seek(img_r, n2, jlo);
                    for (int j = jlo; j < jhi; ++j) {
                        const int v = cand_at(s, j);
                        const bool sub = j < ncs - 1;
                        const int u = sub ? it.next(img_r, n2) : n2;
                        int add_e = 0, used = used0;
                        if (sub) {
#pragma unroll
                            for (int k = 0; k < W; ++k) add_e += __popc(img_r[k] & s_rows[u * RS + k]);
                            ++used;
                        }
                        const int total = v + c.vins * (n2 - used) + c.eins * (g2.m - e0 - add_e);
                        const unsigned long long key = ((unsigned long long)(unsigned)total << 32) |
                                                       (unsigned)((s << 20) | (j << 10) | u);
                        bk = key < bk ? key : bk;
                    }
                }
                bk = wave_min_u64(bk);
                if ((t & 63) == 0) s_red64[t >> 6] = bk;
                __syncthreads();
                if (t == 0) {
                    unsigned long long m = s_red64[0];
#pragma unroll
                    for (int k = 1; k < NW; ++k) m = s_red64[k] < m ? s_red64[k] : m;
                    const int low = (int)(m & 0xffffffffu);
                    const int bs = low >> 20, bj = (low >> 10) & 1023, bu = low & 1023;
                    s_sel[0] = (bs << 10) | bu;
                    s_selped[0] = cand_at(bs, bj);
                }
                nb_new = 1;
            } else {
            // ---------------- threshold: K-th smallest partial edit distance
            int T = SENT, quota = 0;
            if (V > K) {
                int lo = m0, below = 0;
                int nxt = block_min<NW>(ovmin, s_red);
                for (;;) {
                    if (t < 64) {
                        constexpr int PER = NBINS / 64;
                        const int base = t * PER;
                        int sum = 0;
#pragma unroll
                        for (int k = 0; k < PER; ++k) sum += s_hist[base + k];
                        const int incl = wave_incl_scan(sum);
                        const unsigned long long hit = __ballot(below + incl >= K);
                        if (hit) {
                            const int Lh = __ffsll((long long)hit) - 1;
                            if (t == Lh) {
                                int cum = below + incl - sum;
                                for (int k = 0; k < PER; ++k) {
                                    const int h = s_hist[base + k];
                                    if (cum + h >= K) {
                                        s_bc[1] = 1;
                                        s_bc[2] = lo + base + k;
                                        s_bc[3] = cum;
                                        break;
                                    }
                                    cum += h;
                                }
                            }
                        } else if (t == 63) {
                            s_bc[1] = 0;
                            s_bc[3] = below + incl;
                        }
                    }
                    __syncthreads();
                    const int found = s_bc[1];
                    const int v2 = s_bc[2], v3 = s_bc[3];
                    __syncthreads();
                    if (found) {
                        T = v2;
                        quota = K - v3;
                        break;
                    }
                    // the K-th value lies above this window: the next window starts
                    // at the least value above it (one exists, since V > K)
                    below = v3;
                    lo = nxt;
                    for (int b = t; b < NBINS; b += BT) s_hist[b] = 0;
                    __syncthreads();
                    int nn = SENT;
                    for (int r = 0; r < SPT; ++r) {
                        const int s = r * G + sg;
                        if (s >= nb) break;
                        int jlo, jhi;
                        (void)part_range(nsubc[s], &jlo, &jhi);
#pragma unroll 16
                        for (int j = jlo; j < jhi; ++j) {
                            const int v = cand_at(s, j);
                            if (v < lo) continue;
                            if (v - lo < NBINS) atomicAdd(&s_hist[v - lo], 1);
                            else nn = min(nn, v);
                        }
                    }
                    nxt = block_min<NW>(nn, s_red);   // also orders the histogram writes
                }
            }

            // ---------------- keep flags, tie quota and compaction in generation order
            int eq_carry = 0, out_carry = 0;
            for (int r = 0; r < SPT; ++r) {
                const int s = r * G + sg;
                const bool live = s < nb;
                int lt = 0, eq = 0;
                int jlo = 0, jhi = 0, ncs = 0;
                if (live) {
                    ncs = part_range(nsubc[s], &jlo, &jhi);
                    for (int jb = jlo; jb < jhi; jb += LBK) {
                        int vv[LBK];
#pragma unroll
                        for (int k = 0; k < LBK; ++k) vv[k] = jb + k < jhi ? cand_at(s, jb + k) : 0;
#pragma unroll
                        for (int k = 0; k < LBK; ++k) {
                            const bool in = jb + k < jhi;
                            lt += (in && vv[k] < T) ? 1 : 0;
                            eq += (in && vv[k] == T) ? 1 : 0;
                        }
                    }
                }
                int tot;
                const int EQ = eq_carry + block_excl_scan<NW>(eq, s_red, &tot);
                eq_carry += tot;
                const int keep = lt + min(max(quota - EQ, 0), eq);
                const int OUT = out_carry + block_excl_scan<NW>(keep, s_red, &tot);
                out_carry += tot;
                if (live && keep > 0) {
                    int pos = OUT, e = EQ;
                    uint32_t img_r[W];
#pragma unroll
                    for (int k = 0; k < W; ++k) img_r[k] = imgc[(size_t)k * KS + s];
                    FreeIter<W, NWF> it;
                    it.seek(img_r, n2, jlo);
                    for (int jb = jlo; jb < jhi; jb += LBK) {
                        int vv[LBK];
#pragma unroll
                        for (int k = 0; k < LBK; ++k) vv[k] = jb + k < jhi ? cand_at(s, jb + k) : 0;
                        for (int k = 0; k < LBK && jb + k < jhi; ++k) {
                            const int j = jb + k;
                            const int v = vv[k];
                            const int u = j < ncs - 1 ? it.next(img_r, n2) : n2;
                            bool take = v < T;
                            if (v == T) {
                                take = e < quota;
                                ++e;
                            }
                            if (take) {
                                s_sel[pos] = (s << 10) | u;
                                s_selped[pos] = v;
                                ++pos;
                            }
                        }
                    }
                }
            }
            nb_new = out_carry;
            }
            __syncthreads();

            // ---------------- update: child = parent + (v_i -> u)
            const int nxt = cur ^ 1;
            int *pedn = ped_b + nxt * KS;
            int *einn = ein_b + nxt * KS;
            int *nsubn = nsub_b + nxt * KS;
            const int *einc = ein_b + cur * KS;
            uint32_t *__restrict__ imgn = img_b + (size_t)nxt * W * KS;
            uint16_t *__restrict__ phin = phi_b + nxt * a.L.phi_half;
            for (int r = 0; r < SPT; ++r) {
                const int s2 = r * G + sg;
                if (s2 >= nb_new) break;
                const int sel = s_sel[s2];
                const int p = sel >> 10, u = sel & 1023;
                const bool sub = u < n2;
                for (int jb = part; jb < i; jb += LBK * TPS) {
                    uint16_t x[LBK];
#pragma unroll
                    for (int k = 0; k < LBK; ++k) {
                        const int j = jb + k * TPS;
                        x[k] = j < i ? phic[(size_t)j * KS + p] : (uint16_t)0;
                    }
#pragma unroll
                    for (int k = 0; k < LBK; ++k) {
                        const int j = jb + k * TPS;
                        if (j < i) phin[(size_t)j * KS + s2] = x[k];
                    }
                }
                if (part == 0) {
                    phin[(size_t)i * KS + s2] = sub ? (uint16_t)u : PHI_DEL;
                    int add_e = 0;
#pragma unroll
                    for (int k = 0; k < W; ++k) {
                        const uint32_t ip = imgc[(size_t)k * KS + p];
                        const uint32_t row = sub ? s_rows[u * RS + k] : 0u;
                        add_e += __popc(ip & row);
                        const bool at = (u >> 5) == k || (DH > 0 && (u >> 5) + DH == k);
                        imgn[(size_t)k * KS + s2] = ip | ((sub && at) ? (1u << (u & 31)) : 0u);
                    }
                    pedn[s2] = s_selped[s2];
                    einn[s2] = einc[p] + add_e;
                    nsubn[s2] = nsubc[p] + (sub ? 1 : 0);
                }
            }
            __syncthreads();
            cur = nxt;
            nb = nb_new;
        }

        // ---------------- completion: insert what is left of g2, pick the best leaf
        unsigned long long best = ~0ull;
        {
            const int *pedc = ped_b + cur * KS;
            const int *einc = ein_b + cur * KS;
            const int *nsubc = nsub_b + cur * KS;
            for (int r = 0; r < SPT; ++r) {
                const int s = r * G + sg;
                if (s >= nb || part != 0) continue;
                const int total = pedc[s] + c.vins * (n2 - nsubc[s]) + c.eins * (g2.m - einc[s]);
                const unsigned long long key = ((unsigned long long)(unsigned)total << 32) | (unsigned)s;
                best = key < best ? key : best;
            }
        }
        best = wave_min_u64(best);
        if ((t & 63) == 0) s_red64[t >> 6] = best;
        __syncthreads();
        best = s_red64[0];
#pragma unroll
        for (int k = 1; k < NW; ++k) best = s_red64[k] < best ? s_red64[k] : best;
        const int bslot = (int)(best & 0xffffffffu);
        if (t == 0) {
            a.out.dist[wi.out] = (int)(best >> 32);
            if (a.out.cand) a.out.cand[wi.out] = ce;
        }
        const uint16_t *phic = phi_b + cur * a.L.phi_half;
        for (int j = t; j < n1; j += BT) {
            const int x = phic[(size_t)j * KS + bslot];
            a.out.map[wi.map_off + j] = (x == PHI_DEL) ? -1 : x;
        }
        __syncthreads();
    }
}

__global__ void fill_zero_kernel(int *p, int count) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = 0;
}

int cand_stride_max(const BlockShape &s) { return (s.nmax2 + 1) | 1; }

int rows_words(const BlockShape &s) { return s.nmax2 * row_stride(s.W); }

bool planes_in_lds(const BlockShape &s) {
    return s.PL > 0 && (size_t)(1 + s.PL) * (size_t)rows_words(s) * 4 <= kPlaneLdsBytes;
}

size_t staged_bytes(const BlockShape &s) {
    return (size_t)rows_words(s) * 4 * (1 + (planes_in_lds(s) ? s.PL : 0));
}

bool cand_in_lds(const BlockShape &s) {
    return staged_bytes(s) + (size_t)s.KS * (size_t)cand_stride_max(s) * 4 <= kDynLdsBytes;
}

WsLayout layout_for(const BlockShape &s) {
    WsLayout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~size_t(255);
        return o;
    };
    const size_t KS = (size_t)s.KS;
    const size_t n1 = (size_t)(s.nmax1 > 0 ? s.nmax1 : 1);
    L.ped = take(2 * KS * 4);
    L.ein = take(2 * KS * 4);
    L.nsub = take(2 * KS * 4);
    L.img = take(2 * (size_t)s.W * KS * 4);
    L.phi = take(2 * n1 * KS * 2);
    L.cand = take(cand_in_lds(s) ? 0 : ((size_t)s.nmax2 + 1) * KS * 4);
    L.stride = off;
    L.phi_half = n1 * KS;
    return L;
}

size_t dyn_lds_bytes(const BlockShape &s) {
    size_t b = staged_bytes(s);
    if (cand_in_lds(s)) b += (size_t)s.KS * (size_t)cand_stride_max(s) * 4;
    return b;
}

template <int W, int PL, bool CL, int BT, bool DIR>
const void *kernel_ptr() {
    return reinterpret_cast<const void *>(&kb_block_kernel<W, PL, CL, BT, DIR>);
}

// Directed instantiations exist for W = 2 .. 16 (graphs of up to 256
// vertices: out-row and in-row of 8 words each).
const void *select_kernel(int W, int PL, bool CL, int BT, bool DIR) {
#define GEDK_CASE(w, pl, cl, bt, d) \
    if (W == w && PL == pl && CL == cl && BT == bt && DIR == d) return kernel_ptr<w, pl, cl, bt, d>();
#define GEDK_ROW(w, cl, bt, d) GEDK_CASE(w, 0, cl, bt, d) GEDK_CASE(w, 2, cl, bt, d) GEDK_CASE(w, 4, cl, bt, d)
#define GEDK_ALL(bt)                                                                                        \
    GEDK_ROW(1, true, bt, false) GEDK_ROW(2, true, bt, false) GEDK_ROW(4, true, bt, false)                  \
    GEDK_ROW(8, true, bt, false) GEDK_ROW(16, true, bt, false) GEDK_ROW(1, false, bt, false)                \
    GEDK_ROW(2, false, bt, false) GEDK_ROW(4, false, bt, false) GEDK_ROW(8, false, bt, false)               \
    GEDK_ROW(16, false, bt, false) GEDK_ROW(2, true, bt, true) GEDK_ROW(4, true, bt, true)                   \
    GEDK_ROW(8, true, bt, true) GEDK_ROW(16, true, bt, true) GEDK_ROW(2, false, bt, true)                   \
    GEDK_ROW(4, false, bt, true) GEDK_ROW(8, false, bt, true) GEDK_ROW(16, false, bt, true)
    GEDK_ALL(256)
    GEDK_ALL(512)
    // four waves per SIMD on one pair: the largest rows without label planes
    GEDK_CASE(8, 0, false, 1024, false) GEDK_CASE(16, 0, false, 1024, false)
#undef GEDK_ALL
#undef GEDK_ROW
#undef GEDK_CASE
    return nullptr;
}

}  // namespace

int block_slot_stride(int K, int threads) {
    if (K <= 64) return 64;
    if (K <= 128) return 128;
    if (K <= 256) return 256;
    return (K + threads - 1) / threads * threads;
}

size_t block_workspace_bytes(const BlockShape &s) { return layout_for(s).stride; }

bool block_shape_supported(const BlockShape &s) {
    return select_kernel(s.W, s.PL, cand_in_lds(s), s.BT, s.directed != 0) != nullptr;
}

hipError_t block_max_resident(const BlockShape &s, int *blocks_per_cu) {
    const void *k = select_kernel(s.W, s.PL, cand_in_lds(s), s.BT, s.directed != 0);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, s.BT, dyn_lds_bytes(s));
}

hipError_t launch_block(const BlockShape &s, const DbView &src, const DbView &dst, const WorkItem *work, int nwork,
                        int *queue, Costs c, int K, int last_complete, void *workspace, size_t ws_stride,
                        Outputs out, int grid, hipStream_t stream) {
    const void *k = select_kernel(s.W, s.PL, cand_in_lds(s), s.BT, s.directed != 0);
    if (!k || grid <= 0 || s.KS != block_slot_stride(K, s.BT)) return hipErrorInvalidValue;
    BlockArgs a;
    a.src = src;
    a.dst = dst;
    a.work = work;
    a.nwork = nwork;
    a.queue = queue;
    a.c = c;
    a.K = K;
    a.last_complete = last_complete;
    a.KS = s.KS;
    a.TPS = s.KS >= s.BT ? 1 : s.BT / s.KS;
    a.rows_words = rows_words(s);
    a.planes_lds = planes_in_lds(s) ? 1 : 0;
    a.ws = static_cast<char *>(workspace);
    a.L = layout_for(s);
    if (a.L.stride != ws_stride) return hipErrorInvalidValue;
    a.out = out;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(grid), dim3(s.BT), args, dyn_lds_bytes(s), stream);
}

hipError_t launch_fill_zero(int *p, int count, hipStream_t stream) {
    if (count <= 0) return hipSuccess;
    const int threads = 256;
    const int blocks = (count + threads - 1) / threads;
    hipLaunchKernelGGL(fill_zero_kernel, dim3(blocks), dim3(threads), 0, stream, p, count);
    return hipGetLastError();
}

}  // namespace gedk
