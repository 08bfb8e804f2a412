// kb_wide.hip -- the K-Best search (Alg. 1) on ONE pair with the whole
// device: beam widths from thousands to millions, the regime of the paper's
// own experiments (Sec. 5: K up to 1.2 million).
//
// The beam lives in HBM, structure of arrays with the slot index fastest so
// that every per-slot access of a workgroup is coalesced:
//   ped[s], ein[s]        partial edit distance, g2 edges inside Img
//   img[k][s]             word k of Img (the g2 vertices in use)
//   phi[j][s]             image of g1 vertex j (uint16, 0xffff = deleted)
//   sets[b][k][s]         Phi for the current level (b = 0) and its edge-label
//                         planes Phi_b (b = 1..planes)
// ped/ein/img/phi are double-buffered by level parity.  The candidate
// columns u = 0..n2 (u = n2 is the deletion) are split into S chunks of
// whole 32-vertex words, so that a level with few parents (large graphs,
// small K) still spreads over the device: the per-parent kernels run one
// workgroup per (256 parents, chunk).  Per level i (g1 vertex v_i, in index
// order):
//   expand   every child's PED (Sec. 2.3, implied edge operations) into the
//            candidate matrix cand[u][p] (0xffffffff marks a used u), and an
//            LDS histogram of (PED - m0) >> shift, m0 the least parent PED and
//            shift chosen so that every child PED of the level fits 4096
//            bins; the workgroup histograms are summed in HBM.
//   select   one workgroup: the bin holding the K-th smallest child.  With
//            shift 0 that bin IS the threshold T; otherwise up to two refine
//            passes histogram the candidates inside the bin at finer shifts
//            (12 bits at a time) until the threshold is exact.
//   count    per (parent, chunk): children below T and equal to T.
//   scan     one workgroup: exclusive prefix sums over the workgroups.
//   compact  per (parent, chunk): its survivors in generation order (parent
//            slot, then target vertex ascending, then the deletion): every
//            child below T, and ties at T while the quota K - #below lasts,
//            counted from the first parent on, written as records
//            parent << 10 | column (and the child's PED) at their beam
//            position -- the new beam is again in generation order and never
//            needs sorting.
//   update   per (new slot, range of 64 mapping entries): the mapping copied
//            from the parent with u appended; the first range also sets Img
//            and e_in (compaction wrote the PED) and, when one range covers
//            the mapping, the next level's Phi sets.
//   sets     (mappings past 64 entries) per (new slot, range): the images of
//            the next vertex's earlier neighbours in the range, OR-ed into Phi.
// After the last level every leaf is completed (Sec. 4.4.1) and the first
// leaf of least total in beam order is returned.  With the complete-then-
// minimum option the last level skips selection: every child is completed
// and the least total (first in generation order) is the only survivor.
#include <algorithm>

#include "ged_internal.h"
#include "wave_common.h"

namespace gedk {
namespace {

using namespace wv;

constexpr uint32_t INVALID = 0xffffffffu;
constexpr uint32_t DEL16 = 0xffffu;
constexpr int WT = 256;          // threads of the per-parent kernels
constexpr int NWV = WT / 64;
constexpr int ST = 1024;         // threads of the single-workgroup kernels
constexpr int HBITS = 12;
constexpr int HB = 1 << HBITS;   // histogram bins
constexpr int CBITS = 11;        // survivor record: parent << CBITS | column (n2 < 2^11, K <= 2^21)
constexpr int MAXS = 16;         // column chunks (one per target word at most)
constexpr int MAXCW = 8;         // target words of a chunk when rows have more than 16 words

// Target words a chunk of the W-word instantiation can hold (its LDS rows).
template <int W>
constexpr int chunk_words() { return W > 16 ? MAXCW : W; }
constexpr int JR = 64;           // mapping entries per update workgroup

struct LevelState {
    uint32_t B;       // parents (beam slots) at this level
    uint32_t m0;      // least parent PED
    uint32_t mmax;    // largest parent PED
    uint32_t V;       // valid children of the level
    uint32_t shift;   // histogram shift of the expansion pass
    uint32_t T;       // threshold
    uint32_t quota;   // children equal to T that survive
    uint32_t refine;  // a refinement pass is pending
    uint32_t lo;      // refinement range [lo, lo + 2^rwidth)
    uint32_t rwidth;
    uint32_t rbin;    // refinement bin shift
    uint32_t need;    // rank of the threshold inside the refinement range
    uint32_t pad[4];
};

struct WideCtx {
    const uint32_t *a1;   // g1 rows, then its label planes
    const int32_t *l1;
    const uint32_t *a2;   // g2 rows, then its label planes
    const int32_t *l2;
    int n1, w1, n2, w2, m2, planes;
    Costs c;
    uint64_t pedmax;      // vmax n1 + emax (m1 + m2): no PED of the search exceeds it
    uint32_t K;
    uint32_t Kp;          // slot stride: K rounded up to WT
    uint32_t *ped[2];
    uint32_t *ein[2];
    uint32_t *img[2];
    uint16_t *phi[2];
    uint32_t *sets;
    uint32_t *cand;
    uint32_t *cnt;        // [MAXS][Kp]: below | equal << 16 per (chunk, parent)
    uint32_t *blk;        // [2][MAXS][Kp / WT]: per-workgroup sums of the counts
    uint32_t *pre;        // [2][Kp / WT]: their exclusive prefix over parent tiles
    uint32_t *rec;
    uint32_t *hist;
    LevelState *st;
    unsigned long long *ce;
    unsigned long long *best;   // least (total << 32 | slot) of the leaves
    int32_t *out_dist;
    int32_t *out_map;
    int64_t *out_cand;
};

__device__ __forceinline__ uint32_t sgpr(uint32_t v) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)v); }

// Exclusive prefix sum over a workgroup of NW waves; *total gets the sum.
template <int NW>
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t *s_tmp, uint32_t *total) {
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const uint32_t x = (uint32_t)wave_excl_scan((int)v);
    if (lane == 63) s_tmp[wid] = x + v;
    __syncthreads();
    uint32_t pre = 0, tot = 0;
#pragma unroll
    for (int k = 0; k < NW; ++k) {
        const uint32_t t = s_tmp[k];
        pre += k < wid ? t : 0u;
        tot += t;
    }
    __syncthreads();
    *total = tot;
    return pre + x;
}

// Earlier neighbours of g1 vertex v (bits below `lim`) in word k of its row.
__device__ __forceinline__ uint32_t earlier_word(const WideCtx &c, int v, int k, int lim) {
    const uint32_t r = c.a1[(size_t)v * c.w1 + k];
    const int lo = 32 * k;
    if (lim >= lo + 32) return r;
    if (lim <= lo) return 0u;
    return r & ((1u << (lim - lo)) - 1u);
}

// Candidate columns of chunk `chunk` of S: target words [k0, k1), i.e.
// vertices [u0, u1), plus the deletion column in the last chunk.
struct Cols {
    int u0, u1;
    bool del;
};
__device__ __forceinline__ Cols chunk_cols(const WideCtx &c, int chunk, int S) {
    const int k0 = chunk * c.w2 / S, k1 = (chunk + 1) * c.w2 / S;
    return Cols{32 * k0, min(32 * k1, c.n2), chunk == S - 1};
}

// ------------------------------------------------------------------ init
__global__ __launch_bounds__(WT) void wide_init(WideCtx c) {
    const int t = threadIdx.x;
    for (int l = t; l <= c.n1; l += WT) {
        LevelState s = {};
        s.m0 = l == 0 ? 0u : INVALID;
        s.B = l == 0 ? 1u : 0u;
        c.st[l] = s;
    }
    for (int b = t; b < HB; b += WT) c.hist[b] = 0u;
    for (int k = t; k < c.w2; k += WT) c.img[0][(size_t)k * c.Kp] = 0u;
    for (int k = t; k < (1 + c.planes) * c.w2; k += WT) c.sets[(size_t)k * c.Kp] = 0u;
    if (t == 0) {
        c.ped[0][0] = 0u;
        c.ein[0][0] = 0u;
        *c.ce = 0ull;
        *c.best = ~0ull;
    }
}

// ------------------------------------------------------------------ expand
// Persistent over the items (chunk, tile) of the level, chunk-major so that
// a workgroup restages its target rows only when its chunk changes.
template <int W, int PL, bool SMALL>
__global__ __launch_bounds__(WT) void wide_expand(WideCtx c, int i, int S, int tiles) {
    constexpr int PLA = PL > 0 ? PL : 1;
    constexpr int CW = chunk_words<W>();
    __shared__ uint32_t s_rows[32 * CW * W];  // N2(u) rows of the chunk, W words each
    __shared__ uint32_t s_lc[32 * CW];        // label cost of substituting v_i by u
    __shared__ uint32_t s_hist[HB];
    const int tid = threadIdx.x;
    const uint32_t B = sgpr(c.st[i].B);
    const uint32_t m0 = sgpr(c.st[i].m0), mmax = sgpr(c.st[i].mmax);
    const int n2 = c.n2, w2 = c.w2, P = c.planes;
    const uint32_t vsub = (uint32_t)c.c.vsub, vdel = (uint32_t)c.c.vdel, esub = (uint32_t)c.c.esub;
    const uint32_t edel = (uint32_t)c.c.edel, eins = (uint32_t)c.c.eins, nedel = 0u - edel;
    const uint32_t Kp = c.Kp;
    const int cur = i & 1;

    uint32_t deg = 0;
    for (int k = 0; k < c.w1; ++k) deg += (uint32_t)__popc(earlier_word(c, i, k, i));
    deg = sgpr(deg);
    const int lab1 = c.l1[i];
    // every child PED of the level lies in [m0, m0 + R] (and below pedmax:
    // a PED counts at most one operation per vertex of g1 and per edge of g1
    // and g2)
    const uint64_t inc_sub = (uint64_t)vsub + (uint64_t)max(edel, esub) * deg + (uint64_t)eins * (uint64_t)min(i, n2);
    const uint64_t inc_del = (uint64_t)vdel + (uint64_t)edel * deg;
    uint64_t R = (uint64_t)(mmax - m0) + (inc_sub > inc_del ? inc_sub : inc_del);
    R = R < c.pedmax ? R : c.pedmax;
    uint32_t shift = 0;
    while ((R >> shift) >= (uint64_t)HB) ++shift;
    const int nbins = (int)(R >> shift) + 1;   // bins that can be hit
    if (blockIdx.x == 0 && tid == 0) c.st[i].shift = shift;

    for (int b = tid; b < nbins; b += WT) s_hist[b] = 0u;
    const uint32_t *planes2 = c.a2 + (size_t)n2 * w2;
    int staged = -1;
    for (int w = blockIdx.x; w < tiles * S; w += gridDim.x) {
        const int chunk = w / tiles, tile = w % tiles;
        if ((uint32_t)tile * WT >= B) continue;
        const Cols cc = chunk_cols(c, chunk, S);
        const int k0 = cc.u0 >> 5, k1 = (cc.u1 + 31) >> 5;
        if (chunk != staged) {
            __syncthreads();
            for (int idx = tid; idx < (cc.u1 - cc.u0) * W; idx += WT) {
                const int uu = idx / W, k = idx % W;
                s_rows[idx] = k < w2 ? c.a2[(size_t)(cc.u0 + uu) * w2 + k] : 0u;
            }
            for (int uu = tid; uu < cc.u1 - cc.u0; uu += WT) s_lc[uu] = c.l2[cc.u0 + uu] != lab1 ? vsub : 0u;
            __syncthreads();
            staged = chunk;
        }
        const uint32_t p = (uint32_t)tile * WT + tid;
        const bool live = p < B;
        uint32_t ph[W], am[W], pb[PLA][W];
        uint32_t ped = 0u;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            ph[k] = 0u;
            am[k] = 0u;
#pragma unroll
            for (int b = 0; b < PLA; ++b) pb[b][k] = 0u;
        }
        if (live) {
            ped = c.ped[cur][p];
#pragma unroll
            for (int k = 0; k < W; ++k) {
                if (k < w2) {
                    ph[k] = c.sets[(size_t)k * Kp + p];
                    am[k] = c.img[cur][(size_t)k * Kp + p] & ~ph[k];
#pragma unroll
                    for (int b = 0; b < PLA; ++b)
                        if (PL > 0 && b < P) pb[b][k] = c.sets[(size_t)((1 + b) * w2 + k) * Kp + p];
                }
            }
        }
        const uint32_t basel = ped + mul_cost<SMALL>(deg, edel);
#pragma unroll
        for (int k = 0; k < W; ++k) {
            if (k < k0 || k >= k1) continue;
            const uint32_t used = ph[k] | am[k];
            const int ub = 32 * k;
            const int nb = min(32, n2 - ub);
            for (int bit = 0; bit < nb; ++bit) {
                const int u = ub + bit;
                const uint32_t *Rw = s_rows + (u - cc.u0) * W;
                uint32_t mt = 0u, at = 0u, rl = 0u;
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const uint32_t r = Rw[q];
                    mt += (uint32_t)__popc(ph[q] & r);
                    at += (uint32_t)__popc(am[q] & r);
                    if (PL > 0) {
                        uint32_t diff = 0u;
#pragma unroll
                        for (int b = 0; b < PLA; ++b)
                            if (b < P && q < w2) diff |= pb[b][q] ^ planes2[((size_t)b * n2 + u) * w2 + q];
                        rl += (uint32_t)__popc(ph[q] & r & diff);
                    }
                }
                uint32_t d = msub_cost<SMALL>(mt, nedel, mad_cost<SMALL>(at, eins, basel + s_lc[u - cc.u0]));
                if (PL > 0) d += mul_cost<SMALL>(rl, esub);
                const bool ok = live && !((used >> bit) & 1u);
                if (live) c.cand[(size_t)u * Kp + p] = ok ? d : INVALID;
                if (ok) atomicAdd(&s_hist[min((d - m0) >> shift, (uint32_t)HB - 1u)], 1u);
            }
        }
        if (cc.del && live) {
            const uint32_t d = basel + vdel;
            c.cand[(size_t)n2 * Kp + p] = d;
            atomicAdd(&s_hist[min((d - m0) >> shift, (uint32_t)HB - 1u)], 1u);
        }
    }
    __syncthreads();
    for (int b = tid; b < nbins; b += WT) {
        const uint32_t h = s_hist[b];
        if (h) atomicAdd(&c.hist[b], h);
    }
}

// ------------------------------------------------------------------ select
// round 0 reads the expansion histogram; rounds 1 and 2 read refinement
// histograms while a refinement is pending.  Clears the histogram it read.
// Round 0 also sets the next level's beam size and PED bounds: m0 from the
// least non-empty bin (the least child survives), mmax from the top of the
// threshold's bin (or of the last non-empty bin when every child survives).
__global__ __launch_bounds__(ST) void wide_select(WideCtx c, int i, int round) {
    __shared__ uint32_t s_tmp[ST / 64];
    __shared__ uint32_t s_res[2];
    __shared__ uint32_t s_first, s_last;
    LevelState *L = c.st + i;
    const int t = threadIdx.x;
    if (round > 0 && L->refine == 0u) return;
    const uint32_t K = c.K;
    if (t == 0) {
        s_first = HB;
        s_last = 0u;
    }
    uint32_t h[HB / ST];
    uint32_t sum = 0, first = HB, last = 0;
#pragma unroll
    for (int q = 0; q < HB / ST; ++q) {
        const uint32_t b = (uint32_t)(t * (HB / ST) + q);
        h[q] = c.hist[b];
        sum += h[q];
        if (h[q]) {
            first = min(first, b);
            last = max(last, b);
        }
    }
    const uint32_t target0 = round == 0 ? K : L->need;
    uint32_t V;   // children in the histogram
    const uint32_t pre = block_excl_scan<ST / 64>(sum, s_tmp, &V);
    if (round == 0) {
        if (first < (uint32_t)HB) atomicMin(&s_first, first);
        if (sum) atomicMax(&s_last, last);
    }
    const bool all = round == 0 && V <= K;   // every child survives
    if (!all && pre < target0 && target0 <= pre + sum) {
        uint32_t below = pre, bin = 0u;
        bool found = false;
#pragma unroll
        for (int q = 0; q < HB / ST; ++q) {
            if (!found && below + h[q] >= target0) {
                found = true;
                bin = (uint32_t)q;
            }
            if (!found) below += h[q];
        }
        s_res[0] = (uint32_t)(t * (HB / ST)) + bin;
        s_res[1] = below;
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < HB / ST; ++q) c.hist[t * (HB / ST) + q] = 0u;
    if (t != 0) return;
    if (round == 0) {
        const uint32_t m0 = L->m0, shift = L->shift, top = (1u << shift) - 1u;
        LevelState *N = c.st + i + 1;
        L->V = V;
        *c.ce += V;
        N->m0 = m0 + (s_first << shift);
        if (all) {
            L->T = INVALID;
            L->quota = 0u;
            L->refine = 0u;
            N->B = V;
            N->mmax = m0 + (s_last << shift) + top;
            return;
        }
        const uint32_t bin = s_res[0], below = s_res[1];
        N->B = K;
        N->mmax = m0 + (bin << shift) + top;
        if (shift == 0u) {
            L->T = m0 + bin;
            L->quota = K - below;
            L->refine = 0u;
        } else {
            L->lo = m0 + (bin << shift);
            L->rwidth = shift;
            L->rbin = shift > (uint32_t)HBITS ? shift - HBITS : 0u;
            L->need = K - below;
            L->refine = 1u;
        }
    } else {
        const uint32_t bin = s_res[0], below = s_res[1];
        const uint32_t rbin = L->rbin;
        if (rbin == 0u) {
            L->T = L->lo + bin;
            L->quota = L->need - below;
            L->refine = 0u;
            c.st[i + 1].mmax = L->T;
        } else {
            L->lo += bin << rbin;
            L->rwidth = rbin;
            L->rbin = rbin > (uint32_t)HBITS ? rbin - HBITS : 0u;
            L->need -= below;
        }
    }
}

// ------------------------------------------------------------------ refine
// One workgroup per (chunk, tile), chunk-major like every per-parent kernel.
__global__ __launch_bounds__(WT) void wide_refine(WideCtx c, int i, int S, int tiles) {
    __shared__ uint32_t s_hist[HB];
    const LevelState *L = c.st + i;
    if (sgpr(L->refine) == 0u) return;
    const int chunk = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const uint32_t B = sgpr(L->B);
    if ((uint32_t)tile * WT >= B) return;
    const uint32_t lo = sgpr(L->lo), rwidth = sgpr(L->rwidth), rbin = sgpr(L->rbin);
    const int tid = threadIdx.x;
    for (int b = tid; b < HB; b += WT) s_hist[b] = 0u;
    __syncthreads();
    const Cols cc = chunk_cols(c, chunk, S);
    const uint32_t p = (uint32_t)tile * WT + tid;
    if (p < B) {
        for (int u = cc.u0; u < cc.u1 + (cc.del ? 1 : 0); ++u) {
            const int col = u < cc.u1 ? u : c.n2;
            const uint32_t d = c.cand[(size_t)col * c.Kp + p];
            if (d != INVALID && d >= lo && ((d - lo) >> rwidth) == 0u)
                atomicAdd(&s_hist[min((d - lo) >> rbin, (uint32_t)HB - 1u)], 1u);
        }
    }
    __syncthreads();
    for (int b = tid; b < HB; b += WT) {
        const uint32_t h = s_hist[b];
        if (h) atomicAdd(&c.hist[b], h);
    }
}

// ------------------------------------------------------------------ count
__global__ __launch_bounds__(WT) void wide_count(WideCtx c, int i, int S, int tiles) {
    __shared__ uint32_t s_tmp[2][NWV];
    const LevelState *L = c.st + i;
    const uint32_t B = sgpr(L->B), T = sgpr(L->T);
    const int chunk = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const Cols cc = chunk_cols(c, chunk, S);
    const uint32_t p = (uint32_t)tile * WT + threadIdx.x;
    uint32_t lt = 0u, eq = 0u;
    if (p < B) {
        for (int u = cc.u0; u < cc.u1 + (cc.del ? 1 : 0); ++u) {
            const int col = u < cc.u1 ? u : c.n2;
            const uint32_t d = c.cand[(size_t)col * c.Kp + p];
            lt += d < T ? 1u : 0u;
            eq += d == T ? 1u : 0u;
        }
        c.cnt[(size_t)chunk * c.Kp + p] = lt | (eq << 16);
    }
    const uint32_t a = wave_sum(lt), b = wave_sum(eq);
    const int wid = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        s_tmp[0][wid] = a;
        s_tmp[1][wid] = b;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t sa = 0u, sb = 0u;
#pragma unroll
        for (int k = 0; k < NWV; ++k) {
            sa += s_tmp[0][k];
            sb += s_tmp[1][k];
        }
        c.blk[(size_t)chunk * tiles + tile] = sa;
        c.blk[(size_t)(S + chunk) * tiles + tile] = sb;
    }
}

// ------------------------------------------------------------------ scan
// pre[a][t] = sum over tiles before t and all chunks of blk[a][chunk][tile].
__global__ __launch_bounds__(ST) void wide_scan(WideCtx c, int S, int tiles) {
    __shared__ uint32_t s_tmp[ST / 64];
    const int t = threadIdx.x;
    const int per = (tiles + ST - 1) / ST;
    for (int a = 0; a < 2; ++a) {
        const uint32_t *x = c.blk + (size_t)a * S * tiles;
        uint32_t *y = c.pre + (size_t)a * tiles;
        uint32_t sum = 0u;
        for (int q = 0; q < per; ++q) {
            const int j = t * per + q;
            if (j < tiles)
                for (int ch = 0; ch < S; ++ch) sum += x[(size_t)ch * tiles + j];
        }
        uint32_t tot;
        uint32_t run = block_excl_scan<ST / 64>(sum, s_tmp, &tot);
        for (int q = 0; q < per; ++q) {
            const int j = t * per + q;
            if (j < tiles) {
                uint32_t v = 0u;
                for (int ch = 0; ch < S; ++ch) v += x[(size_t)ch * tiles + j];
                y[j] = run;
                run += v;
            }
        }
    }
}

// ------------------------------------------------------------------ compact
__global__ __launch_bounds__(WT) void wide_compact(WideCtx c, int i, int S, int tiles) {
    __shared__ uint32_t s_tmp[NWV];
    const LevelState *L = c.st + i;
    const uint32_t B = sgpr(L->B), T = sgpr(L->T), quota = sgpr(L->quota);
    const int chunk = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const uint32_t p = (uint32_t)tile * WT + threadIdx.x;
    const bool live = p < B;
    // the parent's counts: all chunks, chunks before this one, this chunk
    uint32_t lt = 0u, eq = 0u, ltb = 0u, eqb = 0u, ltc = 0u, eqc = 0u;
    if (live) {
        for (int ch = 0; ch < S; ++ch) {
            const uint32_t v = c.cnt[(size_t)ch * c.Kp + p];
            const uint32_t a = v & 0xffffu, b = v >> 16;
            lt += a;
            eq += b;
            if (ch < chunk) {
                ltb += a;
                eqb += b;
            }
            if (ch == chunk) {
                ltc = a;
                eqc = b;
            }
        }
    }
    uint32_t tot;
    const uint32_t LT = c.pre[tile] + block_excl_scan<NWV>(lt, s_tmp, &tot);
    const uint32_t EQ = c.pre[tiles + tile] + block_excl_scan<NWV>(eq, s_tmp, &tot);
    if (!live) return;
    // (every difference below is of a value and its own minimum with
    // something else, so none can wrap)
    const uint32_t eqk = min(EQ, quota);                 // ties kept before this parent
    const uint32_t keq = min(quota - eqk, eq);           // ties the parent keeps
    const uint32_t eqbk = min(eqb, keq);                 // ... in its earlier chunks
    uint32_t keqc = min(keq - eqbk, eqc);                // ... in this chunk
    uint32_t pos = LT + eqk + ltb + eqbk;
    const Cols cc = chunk_cols(c, chunk, S);
    for (int u = cc.u0; u < cc.u1 + (cc.del ? 1 : 0) && (ltc | keqc) != 0u; ++u) {
        const int col = u < cc.u1 ? u : c.n2;
        const uint32_t d = c.cand[(size_t)col * c.Kp + p];
        bool keep = false;
        if (d < T) {
            keep = true;
            --ltc;
        } else if (d == T && keqc > 0u) {
            keep = true;
            --keqc;
        }
        if (keep && pos < c.K) {
            c.rec[pos] = (p << CBITS) | (uint32_t)col;
            c.ped[(i + 1) & 1][pos] = d;
        }
        pos += keep ? 1u : 0u;
    }
}

// Parent slot and column of new slot s (records always name a parent of this
// level and a column <= n2; the clamps only keep accesses inside the beam).
__device__ __forceinline__ void read_record(const WideCtx &c, uint32_t s, uint32_t Bp, uint32_t *p, uint32_t *u) {
    const uint32_t r = c.rec[s];
    *p = min(r >> CBITS, Bp - 1u);
    *u = min(r & ((1u << CBITS) - 1u), (uint32_t)c.n2);
}

// ------------------------------------------------------------------ update
// Sets of the level's Phi handled per pass: all of them (Phi and its label
// planes) when they fit the update's LDS, else one (rows of more than 16
// words: 32 words x 256 slots is 32 KB per set).
template <int W, int PL>
constexpr int sets_per_pass() { return W > 16 ? 1 : 1 + PL; }

// Sets b0 .. b0 + NG - 1 (0 = Phi, 1 + b = label plane b) of level v for
// slot s from the images x(j) of v's earlier neighbours j in [j0, j1): bits
// OR-ed into this thread's LDS column of s_set.
template <int W, int NG, class GetX>
__device__ __forceinline__ void collect_phi(const WideCtx &c, int v, int j0, int j1, bool live, uint32_t *s_set,
                                            int b0, GetX getx) {
    constexpr int NS = NG * W;
    const int tid = threadIdx.x;
    const uint32_t *planes1 = c.a1 + (size_t)c.n1 * c.w1;
#pragma unroll
    for (int q = 0; q < NS; ++q) s_set[q * WT + tid] = 0u;
    for (int k = j0 >> 5; k < (j1 + 31) >> 5; ++k) {
        uint32_t nb = sgpr(earlier_word(c, v, k, j1));
        if (32 * k < j0) nb &= ~((1u << (j0 - 32 * k)) - 1u);
        while (nb) {
            const int j = 32 * k + __builtin_ctz(nb);
            nb &= nb - 1u;
            if (!live) continue;
            const uint32_t x = getx(j);
            if (x == DEL16) continue;
#pragma unroll
            for (int g = 0; g < NG; ++g) {
                const int b = b0 + g;   // set b: Phi (b = 0) or plane b - 1
                if (b == 0 || (b - 1 < c.planes &&
                               ((planes1[((size_t)(b - 1) * c.n1 + v) * c.w1 + (j >> 5)] >> (j & 31)) & 1u)))
                    atomicOr(&s_set[(g * W + (x >> 5)) * WT + tid], 1u << (x & 31u));
            }
        }
    }
}

// Store (whole) or OR in (partial) this thread's words of sets b0 ..
// b0 + NG - 1 for slot s.
template <int W, int NG>
__device__ __forceinline__ void store_phi(const WideCtx &c, uint32_t s, const uint32_t *s_set, bool whole, int b0) {
    const int tid = threadIdx.x;
    for (int g = 0; g < NG && b0 + g < 1 + c.planes; ++g) {
        const int b = b0 + g;
        for (int k = 0; k < c.w2; ++k) {
            const uint32_t word = s_set[(g * W + k) * WT + tid];
            uint32_t *dstw = &c.sets[(size_t)(b * c.w2 + k) * c.Kp + s];
            if (whole) *dstw = word;
            else if (word) atomicOr(dstw, word);
        }
    }
}

// All sets of level v for slot s, pass by pass.
template <int W, int PL, class GetX>
__device__ __forceinline__ void build_phi(const WideCtx &c, int v, int j0, int j1, bool live, uint32_t s,
                                          uint32_t *s_set, bool whole, GetX getx) {
    constexpr int NG = sets_per_pass<W, PL>();
    for (int b0 = 0; b0 < 1 + c.planes && b0 < 1 + PL; b0 += NG) {
        collect_phi<W, NG>(c, v, j0, j1, live, s_set, b0, getx);
        if (live) store_phi<W, NG>(c, s, s_set, whole, b0);
    }
}

// One workgroup per (mapping range jr, slot tile), range-major: the
// mapping copied from the parent with u appended.  The first range also
// sets Img and e_in (the PED came with the record); when one range holds
// the whole mapping it also builds the next level's Phi, else it clears
// Phi for the sets kernel.
template <int W, int PL>
__global__ __launch_bounds__(WT) void wide_update(WideCtx c, int i, int utiles, int nranges) {
    constexpr int NS = sets_per_pass<W, PL>() * W;
    __shared__ uint32_t s_set[NS * WT];
    const int jr = blockIdx.x / utiles, tile = blockIdx.x % utiles;
    const uint32_t Bn = sgpr(c.st[i + 1].B);
    if ((uint32_t)tile * WT >= Bn) return;
    const int tid = threadIdx.x;
    const uint32_t s = (uint32_t)tile * WT + tid;
    const bool live = s < Bn;
    const uint32_t Kp = c.Kp;
    const int cur = i & 1, nxt = cur ^ 1;
    const int n2 = c.n2, w2 = c.w2;
    uint32_t p = 0u, u = 0u;
    if (live) read_record(c, s, sgpr(c.st[i].B), &p, &u);
    const bool sub = (int)u < n2;
    const uint16_t *__restrict__ src = c.phi[cur];
    uint16_t *__restrict__ dst = c.phi[nxt];
    const int j0 = jr * JR, j1 = min(j0 + JR, i);
    if (live) {
        int j = j0;
        for (; j + 8 <= j1; j += 8) {
            uint16_t x[8];
#pragma unroll
            for (int q = 0; q < 8; ++q) x[q] = src[(size_t)(j + q) * Kp + p];
#pragma unroll
            for (int q = 0; q < 8; ++q) dst[(size_t)(j + q) * Kp + s] = x[q];
        }
        for (; j < j1; ++j) dst[(size_t)j * Kp + s] = src[(size_t)j * Kp + p];
        if (i >= j0 && i < j0 + JR) dst[(size_t)i * Kp + s] = (uint16_t)(sub ? u : DEL16);
    }
    if (jr != 0) return;
    if (live) {
        uint32_t e = c.ein[cur][p];
        for (int k = 0; k < w2; ++k) {
            uint32_t im = c.img[cur][(size_t)k * Kp + p];
            if (sub) {
                e += (uint32_t)__popc(im & c.a2[(size_t)u * w2 + k]);
                if (k == (int)(u >> 5)) im |= 1u << (u & 31u);
            }
            c.img[nxt][(size_t)k * Kp + s] = im;
        }
        c.ein[nxt][s] = e;
    }
    const int v = i + 1;
    if (v >= c.n1) return;
    if (nranges == 1) {
        build_phi<W, PL>(c, v, 0, v, live, s, s_set, true, [&](int j) -> uint32_t {
            return j < i ? (uint32_t)src[(size_t)j * Kp + p] : (sub ? u : DEL16);
        });
    } else if (live) {
        for (int k = 0; k < (1 + c.planes) * w2; ++k) c.sets[(size_t)k * Kp + s] = 0u;
    }
}

// ------------------------------------------------------------------ sets
// Phi of level v = i + 1 for the new slots when the mapping spans several
// ranges: the images of v's earlier neighbours in range jr, OR-ed into the
// sets the update cleared.
template <int W, int PL>
__global__ __launch_bounds__(WT) void wide_sets(WideCtx c, int i, int utiles) {
    constexpr int NS = sets_per_pass<W, PL>() * W;
    __shared__ uint32_t s_set[NS * WT];
    const int jr = blockIdx.x / utiles, tile = blockIdx.x % utiles;
    const uint32_t Bn = sgpr(c.st[i + 1].B);
    if ((uint32_t)tile * WT >= Bn) return;
    const uint32_t s = (uint32_t)tile * WT + threadIdx.x;
    const bool live = s < Bn;
    const int v = i + 1;
    const uint16_t *phin = c.phi[v & 1];
    const int j0 = jr * JR, j1 = min(j0 + JR, v);
    build_phi<W, PL>(c, v, j0, j1, live, s, s_set, false,
                     [&](int j) -> uint32_t { return (uint32_t)phin[(size_t)j * c.Kp + s]; });
}

// ------------------------------------------------------------------ complete-then-minimum
// Last level with the complete-then-minimum option: every child's total
// (Sec. 4.4.1: the unused g2 vertices and the g2 edges with an unused end
// inserted); the least (total, generation order) of the grid lands in *best.
__global__ __launch_bounds__(WT) void wide_complete(WideCtx c, int i, int S, int tiles) {
    __shared__ unsigned long long s_key[NWV];
    const uint32_t B = sgpr(c.st[i].B);
    const int chunk = blockIdx.x / tiles, tile = blockIdx.x % tiles;
    const Cols cc = chunk_cols(c, chunk, S);
    const uint32_t p = (uint32_t)tile * WT + threadIdx.x;
    const int cur = i & 1, w2 = c.w2;
    unsigned long long key = ~0ull;
    if (p < B) {
        uint32_t used = 0u;
        for (int k = 0; k < w2; ++k) used += (uint32_t)__popc(c.img[cur][(size_t)k * c.Kp + p]);
        const uint32_t e0 = c.ein[cur][p];
        for (int u = cc.u0; u < cc.u1 + (cc.del ? 1 : 0); ++u) {
            const int col = u < cc.u1 ? u : c.n2;
            const uint32_t d = c.cand[(size_t)col * c.Kp + p];
            if (d == INVALID) continue;
            uint32_t add = 0u, nu = (uint32_t)c.n2 - used;
            if (col < c.n2) {
                for (int k = 0; k < w2; ++k)
                    add += (uint32_t)__popc(c.img[cur][(size_t)k * c.Kp + p] & c.a2[(size_t)col * w2 + k]);
                --nu;
            }
            const uint64_t total = (uint64_t)d + (uint64_t)c.c.vins * nu + (uint64_t)c.c.eins * ((uint32_t)c.m2 - e0 - add);
            const unsigned long long k2 = (total << 32) | ((p << CBITS) | (uint32_t)col);
            key = k2 < key ? k2 : key;
        }
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long other = (unsigned long long)__shfl_xor((long long)key, o);
        key = other < key ? other : key;
    }
    if ((threadIdx.x & 63) == 0) s_key[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = s_key[0];
#pragma unroll
        for (int k = 1; k < NWV; ++k) m = s_key[k] < m ? s_key[k] : m;
        if (m != ~0ull) atomicMin(c.best, m);
    }
}

// The winner of wide_complete becomes the level's only survivor; the level's
// children (for the candidate count) come from the expansion histogram, which
// is cleared for the next use, as is *best.
__global__ __launch_bounds__(WT) void wide_pick(WideCtx c, int i) {
    __shared__ uint32_t s_tmp[NWV];
    const int t = threadIdx.x;
    uint32_t sum = 0u;
    for (int b = t; b < HB; b += WT) {
        sum += c.hist[b];
        c.hist[b] = 0u;
    }
    uint32_t V;
    (void)block_excl_scan<NWV>(sum, s_tmp, &V);
    if (t != 0) return;
    const unsigned long long best = *c.best;
    const uint32_t r = (uint32_t)(best & 0xffffffffull);
    const uint32_t p = r >> CBITS, col = r & ((1u << CBITS) - 1u);
    c.rec[0] = r;
    c.ped[(i + 1) & 1][0] = c.cand[(size_t)col * c.Kp + p];
    c.st[i].V = V;
    c.st[i + 1].B = 1u;
    *c.ce += V;
    *c.best = ~0ull;
}

// ------------------------------------------------------------------ final
// Every leaf's total (Sec. 4.4.1); the least (total, slot) wins.
__global__ __launch_bounds__(WT) void wide_final_keys(WideCtx c) {
    __shared__ unsigned long long s_key[NWV];
    const int n1 = c.n1, cur = n1 & 1;
    const uint32_t B = sgpr(c.st[n1].B);
    if ((uint32_t)blockIdx.x * WT >= B) return;
    const uint32_t s = blockIdx.x * WT + threadIdx.x;
    unsigned long long key = ~0ull;
    if (s < B) {
        uint32_t used = 0u;
        for (int k = 0; k < c.w2; ++k) used += (uint32_t)__popc(c.img[cur][(size_t)k * c.Kp + s]);
        const uint64_t total = (uint64_t)c.ped[cur][s] + (uint64_t)c.c.vins * (uint64_t)(c.n2 - (int)used) +
                               (uint64_t)c.c.eins * (uint64_t)(c.m2 - (int)c.ein[cur][s]);
        key = (total << 32) | s;
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) {
        const unsigned long long other = (unsigned long long)__shfl_xor((long long)key, o);
        key = other < key ? other : key;
    }
    if ((threadIdx.x & 63) == 0) s_key[threadIdx.x >> 6] = key;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long m = s_key[0];
#pragma unroll
        for (int k = 1; k < NWV; ++k) m = s_key[k] < m ? s_key[k] : m;
        atomicMin(c.best, m);
    }
}

__global__ __launch_bounds__(WT) void wide_final_map(WideCtx c) {
    const int n1 = c.n1, cur = n1 & 1;
    const unsigned long long best = *c.best;
    const uint32_t slot = (uint32_t)(best & 0xffffffffull);
    if (threadIdx.x == 0) {
        *c.out_dist = (int32_t)(best >> 32);
        if (c.out_cand) *c.out_cand = (int64_t)*c.ce;
    }
    for (int j = threadIdx.x; j < n1; j += WT) {
        const uint32_t x = c.phi[cur][(size_t)j * c.Kp + slot];
        c.out_map[j] = x == DEL16 ? -1 : (int32_t)x;
    }
}

// ------------------------------------------------------------------ host side

struct Layout {
    size_t ped[2], ein[2], img[2], phi[2], sets, cand, cnt, blk, pre, rec, hist, st, ce, best, total;
};

Layout layout(int n1, int n2, int w2, int planes, uint32_t Kp) {
    Layout L{};
    size_t off = 0;
    auto take = [&](size_t bytes) {
        const size_t o = off;
        off += (bytes + 255) & ~(size_t)255;
        return o;
    };
    const int S = w2 > 1 ? std::min(w2, MAXS) : 1;
    for (int k = 0; k < 2; ++k) {
        L.ped[k] = take((size_t)Kp * 4);
        L.ein[k] = take((size_t)Kp * 4);
        L.img[k] = take((size_t)w2 * Kp * 4);
        L.phi[k] = take((size_t)n1 * Kp * 2);
    }
    L.sets = take((size_t)(1 + planes) * w2 * Kp * 4);
    L.cand = take((size_t)(n2 + 1) * Kp * 4);
    L.cnt = take((size_t)S * Kp * 4);
    L.blk = take((size_t)2 * S * (Kp / WT) * 4);
    L.pre = take((size_t)2 * (Kp / WT) * 4);
    L.rec = take((size_t)Kp * 4);
    L.hist = take((size_t)HB * 4);
    L.st = take((size_t)(n1 + 1) * sizeof(LevelState));
    L.ce = take(8);
    L.best = take(8);
    L.total = off;
    return L;
}

uint32_t slot_stride(int K) { return (uint32_t)((K + WT - 1) / WT) * WT; }

// Column chunks for a level of `tiles` parent tiles: enough workgroups to
// cover the device twice over, at most one chunk per target word, and
// chunks of at most MAXCW words when the rows have more than 16 (the
// expansion's LDS rows of such instantiations hold MAXCW words of vertices).
int column_chunks(int tiles, int w2, int cus) {
    if (w2 <= 1) return 1;
    const int want = (2 * cus + tiles - 1) / tiles;
    const int least = w2 > 16 ? (w2 + MAXCW - 1) / MAXCW : 1;
    return std::max(least, std::min({want, w2, MAXS}));
}

template <int W, int PL>
hipError_t launch_levels(const WideCtx &c, bool refine_possible, bool last_complete, int cus, hipStream_t stream) {
    const bool small = c.c.vsub < (1 << 22) && c.c.vdel < (1 << 22) && c.c.vins < (1 << 22) &&
                       c.c.esub < (1 << 22) && c.c.edel < (1 << 22) && c.c.eins < (1 << 22);
    hipLaunchKernelGGL(wide_init, dim3(1), dim3(WT), 0, stream, c);
    uint64_t bound = 1;   // parents at level i are at most min(K, (n2 + 1)^i)
    for (int i = 0; i < c.n1; ++i) {
        const int tiles = (int)((bound + WT - 1) / WT);
        const int S = column_chunks(tiles, c.w2, cus);
        const int items = tiles * S;
        const int egrid = std::min(items, 8 * cus);
        if (small)
            hipLaunchKernelGGL((wide_expand<W, PL, true>), dim3(egrid), dim3(WT), 0, stream, c, i, S, tiles);
        else
            hipLaunchKernelGGL((wide_expand<W, PL, false>), dim3(egrid), dim3(WT), 0, stream, c, i, S, tiles);
        if (last_complete && i == c.n1 - 1) {
            // the last level keeps only its least completed child
            hipLaunchKernelGGL(wide_complete, dim3(items), dim3(WT), 0, stream, c, i, S, tiles);
            hipLaunchKernelGGL(wide_pick, dim3(1), dim3(WT), 0, stream, c, i);
            bound = 1;
            hipLaunchKernelGGL((wide_update<W, PL>), dim3(i / JR + 1), dim3(WT), 0, stream, c, i, 1, i / JR + 1);
            break;
        }
        hipLaunchKernelGGL(wide_select, dim3(1), dim3(ST), 0, stream, c, i, 0);
        if (refine_possible) {
            for (int r = 1; r <= 2; ++r) {
                hipLaunchKernelGGL(wide_refine, dim3(items), dim3(WT), 0, stream, c, i, S, tiles);
                hipLaunchKernelGGL(wide_select, dim3(1), dim3(ST), 0, stream, c, i, r);
            }
        }
        hipLaunchKernelGGL(wide_count, dim3(items), dim3(WT), 0, stream, c, i, S, tiles);
        hipLaunchKernelGGL(wide_scan, dim3(1), dim3(ST), 0, stream, c, S, tiles);
        hipLaunchKernelGGL(wide_compact, dim3(items), dim3(WT), 0, stream, c, i, S, tiles);
        const uint64_t grown = bound * (uint64_t)(c.n2 + 1);
        bound = grown < c.K ? grown : c.K;
        const int utiles = (int)((bound + WT - 1) / WT);
        // ranges of mapping entries 0..i (also of the next vertex's earlier neighbours)
        const int ranges = i / JR + 1;
        hipLaunchKernelGGL((wide_update<W, PL>), dim3(utiles * ranges), dim3(WT), 0, stream, c, i, utiles, ranges);
        if (i + 1 < c.n1 && ranges > 1)
            hipLaunchKernelGGL((wide_sets<W, PL>), dim3(utiles * ranges), dim3(WT), 0, stream, c, i, utiles);
    }
    const int ftiles = (int)((bound + WT - 1) / WT);
    hipLaunchKernelGGL(wide_final_keys, dim3(ftiles), dim3(WT), 0, stream, c);
    hipLaunchKernelGGL(wide_final_map, dim3(1), dim3(WT), 0, stream, c);
    return hipGetLastError();
}

template <int W>
hipError_t launch_pl(int PL, const WideCtx &c, bool refine_possible, bool last_complete, int cus,
                     hipStream_t stream) {
    if (PL == 0) return launch_levels<W, 0>(c, refine_possible, last_complete, cus, stream);
    if (PL == 2) return launch_levels<W, 2>(c, refine_possible, last_complete, cus, stream);
    if (PL == 4) return launch_levels<W, 4>(c, refine_possible, last_complete, cus, stream);
    return hipErrorInvalidValue;
}

}  // namespace

size_t wide_workspace_bytes(int n1, int n2, int w2, int planes, int K) {
    return layout(n1, n2, w2, planes, slot_stride(K)).total;
}

hipError_t launch_wide(const DbView &src, const DbView &dst, const GraphRec &g1, const GraphRec &g2, Costs costs,
                       int K, int last_complete, void *ws, size_t ws_bytes, int32_t *dist, int32_t *map,
                       int64_t *cand, int cus, hipStream_t stream) {
    const int planes = dst.planes;
    const int PL = planes == 0 ? 0 : (planes <= 2 ? 2 : 4);
    int W = 1;
    while (W < g2.w) W <<= 1;
    const uint32_t Kp = slot_stride(K);
    const Layout L = layout(g1.n, g2.n, g2.w, planes, Kp);
    if (K < 1 || K > kWideMaxK || L.total > ws_bytes || W > 32 || g1.n > GED_MAX_VERTICES ||
        g2.n > GED_MAX_VERTICES || cus < 1)
        return hipErrorInvalidValue;
    char *base = static_cast<char *>(ws);
    WideCtx c{};
    c.a1 = src.adj + g1.adj;
    c.l1 = src.vlab + g1.vlab;
    c.a2 = dst.adj + g2.adj;
    c.l2 = dst.vlab + g2.vlab;
    c.n1 = g1.n;
    c.w1 = g1.w;
    c.n2 = g2.n;
    c.w2 = g2.w;
    c.m2 = g2.m;
    c.planes = planes;
    c.c = costs;
    c.K = (uint32_t)K;
    c.Kp = Kp;
    for (int k = 0; k < 2; ++k) {
        c.ped[k] = reinterpret_cast<uint32_t *>(base + L.ped[k]);
        c.ein[k] = reinterpret_cast<uint32_t *>(base + L.ein[k]);
        c.img[k] = reinterpret_cast<uint32_t *>(base + L.img[k]);
        c.phi[k] = reinterpret_cast<uint16_t *>(base + L.phi[k]);
    }
    c.sets = reinterpret_cast<uint32_t *>(base + L.sets);
    c.cand = reinterpret_cast<uint32_t *>(base + L.cand);
    c.cnt = reinterpret_cast<uint32_t *>(base + L.cnt);
    c.blk = reinterpret_cast<uint32_t *>(base + L.blk);
    c.pre = reinterpret_cast<uint32_t *>(base + L.pre);
    c.rec = reinterpret_cast<uint32_t *>(base + L.rec);
    c.hist = reinterpret_cast<uint32_t *>(base + L.hist);
    c.st = reinterpret_cast<LevelState *>(base + L.st);
    c.ce = reinterpret_cast<unsigned long long *>(base + L.ce);
    c.best = reinterpret_cast<unsigned long long *>(base + L.best);
    c.out_dist = dist;
    c.out_map = map;
    c.out_cand = cand;
    // no PED of the search exceeds pedmax, so the expansion histogram needs a
    // shift (and refinement) only if pedmax does not fit its bins
    const int64_t vmax = std::max({(int64_t)costs.vsub, (int64_t)costs.vdel, (int64_t)costs.vins});
    const int64_t emax = std::max({(int64_t)costs.esub, (int64_t)costs.edel, (int64_t)costs.eins});
    c.pedmax = (uint64_t)(vmax * (int64_t)g1.n + emax * ((int64_t)g1.m + g2.m));
    const bool refine_possible = c.pedmax >= (uint64_t)HB;
    const bool lc = last_complete != 0;
    switch (W) {
        case 1: return launch_pl<1>(PL, c, refine_possible, lc, cus, stream);
        case 2: return launch_pl<2>(PL, c, refine_possible, lc, cus, stream);
        case 4: return launch_pl<4>(PL, c, refine_possible, lc, cus, stream);
        case 8: return launch_pl<8>(PL, c, refine_possible, lc, cus, stream);
        case 16: return launch_pl<16>(PL, c, refine_possible, lc, cus, stream);
        case 32: return launch_pl<32>(PL, c, refine_possible, lc, cus, stream);
        default: return hipErrorInvalidValue;
    }
}

}  // namespace gedk
