// kb_wave.hip -- wavefront-per-pair K-Best search for small pairs on gfx950.
//
// Handles pairs with n1 <= 32, n2 <= 32 and K <= 64: one 64-lane wavefront
// owns one pair for all its levels and pulls the next pair from a work queue
// (persistent launch, one wave per workgroup; the first pair is the
// workgroup's index).  Lane s holds beam slot s in
// registers: partial edit distance, the image Img (one 32-bit word: bit u
// set iff g2 vertex u is used), e_in (g2 edges inside Img) and the mapping
// phi as eight words of bytes (byte v = image of g1 vertex v, 0xff =
// deleted).  Lane u also holds g2's adjacency row N2(u), its label and its
// label-plane rows; lane v holds g1's row N1(v).
//
// Per level i (Alg. 1), with P = earlier neighbours of v_i:
//   expand   Phi = {phi(j) : j in P, not deleted} and A = Img \ Phi.  Since
//            Phi is a subset of Img, the implied edge operations of Sec. 2.3
//            for the child (v_i -> u) are
//              kept     = |Phi & N2(u)|
//              deleted  = |P| - kept
//              inserted = |Img & N2(u)| - kept = |A & N2(u)|
//            so PED' = (PED + edel |P|) + vsub [alpha1(v_i) != alpha2(u)]
//                      + eins |A & N2(u)| - edel |Phi & N2(u)|
//                      [+ esub |Phi & N2(u) & relabelled|].
//            Child j of a slot substitutes the slot's j-th free g2 vertex
//            (ascending, so j order is generation order): only free
//            vertices are visited, found with find-lowest-bit on the free
//            set, and (N2(u), vsub [labels differ]) comes from a per-level
//            LDS table.  Once a slot's free set is exhausted the lookup hits
//            a sentinel entry (empty row, label cost 0xffffffff, added with
//            unsigned saturation) whose child is 0xffffffff, the invalid
//            value, so no per-child validity test is needed.
//            Per child: two AND + popcount and two 24-bit multiply-adds (the
//            second with -edel).  The deletion child costs PED + vdel +
//            edel |P|.
//   select   T = K-th smallest PED.  As they are scored, children are
//            packed four to a word as bytes e = min(PED - base, 127), base =
//            least parent PED (no child costs less than its parent), and
//            count(PED <= base + t) for t < 127 is the sum over lanes of
//            popcount(((t * 0x01010101) | 0x80808080) - packed) & 0x80808080
//            (each byte's top bit is set iff e <= t; no borrow crosses a
//            byte).  The smallest t with count >= K is searched two
//            thresholds per reduction, starting from the previous level's
//            T - m0 (m0 = least child; galloping, then thirds).  When T lies 127 or more above the
//            base the exact count (wave ballots of full-width compares)
//            takes over.  Every child below T survives and the first
//            (K - #below) children equal to T in generation order (lane
//            order, then j, then the deletion), via per-lane bit masks
//            (gathered from the same byte flags by byte dot products) and
//            one exclusive scan of the per-lane (below, tie) counts in
//            16-bit halves; survivor (parent, j) pairs are written to LDS in
//            generation order.  With a full beam only V > K matters, which
//            one ballot decides.
//   update   new slot s reads its (parent, j) and the parent's child-j
//            vertex u (recorded in LDS during the expand), fetches the
//            parent's registers (PED + edel |P|, Phi, A, Img, e_in, the phi
//            words up to byte i) with ds_bpermute, and recomputes the child's
//            PED with the same integer formula, so the value is identical to
//            the candidate's.
// Completion adds vins (n2 - |Img|) + eins (m2 - e_in) (Sec. 4.4.1); the
// first lane of least total is the result.  The COMPLETE instantiation's last
// level instead completes every child and keeps only the least total (first
// in generation order), which then is the result.
//
// SMALL selects 24-bit multiplies, valid when every cost is below 2^22
// (counts are at most 32, and the plan's overflow bound keeps every sum in
// range); otherwise full 32-bit multiplies.  All sums are taken modulo 2^32;
// the true values are below 2^31, so they come out exact.
#include "ged_types.h"
#include "wave_common.h"

namespace gedk {
namespace {

using namespace wv;

constexpr uint32_t INVALID = 0xffffffffu;
constexpr uint32_t DEL8 = 0xffu;
constexpr int TBYTE = 127;        // byte-domain cap: e = min(PED - base, 127)

struct WaveArgs {
    DbView src;   // graphs edited (g1)
    DbView dst;   // target graphs (g2); same edge-label coding as src
    const WorkItem *work;
    int nwork;
    int *queue;
    Costs c;
    int K;
    Outputs out;
};

template <int PL, bool SMALL, bool COMPLETE>
__global__ __launch_bounds__(64) void kb_wave_kernel(WaveArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    __shared__ uint32_t s_sel[64];          // survivor: parent slot << 8 | j (0xff = deletion)
    __shared__ uint2 s_tab[33];             // per level: [1 + u] = (N2(u), vsub [labels differ]); [0] = sentinel
    __shared__ uint32_t s_uv[8][64];        // per level: [j / 4][slot] = g2 vertices of children j, bytes
    __shared__ uint32_t s_pl[PLA][33];      // label-plane rows of g2 at [1 + u]; [0] = 0
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const uint32_t vsub = (uint32_t)a.c.vsub, vdel = (uint32_t)a.c.vdel, vins = (uint32_t)a.c.vins;
    const uint32_t esub = (uint32_t)a.c.esub, edel = (uint32_t)a.c.edel, eins = (uint32_t)a.c.eins;
    const uint32_t nedel = 0u - edel;
    const int K = a.K;
    const int P = a.dst.planes;

    for (bool first = true;; first = false) {
        // the first pair is the workgroup's own index; later ones come from
        // the queue (one shared counter: taking every first pair from it would
        // serialise the whole grid's start on one atomic)
        int item = (int)blockIdx.x;
        if (!first) {
            if (lane == 0) s_item = pull_item(a.queue, a.nwork);
            __syncthreads();
            item = __builtin_amdgcn_readfirstlane(s_item);
            __syncthreads();
        }
        if (item >= a.nwork) break;

        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.src.graphs[wi.src];
        const GraphRec g2 = a.dst.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n;
        const uint32_t *A1 = a.src.adj + g1.adj;
        const uint32_t *A2 = a.dst.adj + g2.adj;
        const uint32_t r1 = lane < n1 ? A1[lane] : 0u;
        const uint32_t r2 = lane < n2 ? A2[lane] : 0u;
        const int l1 = lane < n1 ? a.src.vlab[g1.vlab + lane] : 0;
        const int l2 = lane < n2 ? a.dst.vlab[g2.vlab + lane] : 0;
        uint32_t p1[PLA], p2[PLA];
#pragma unroll
        for (int b = 0; b < PLA; ++b) {
            p1[b] = (PL > 0 && b < P && lane < n1) ? A1[(size_t)(1 + b) * n1 + lane] : 0u;
            p2[b] = (PL > 0 && b < P && lane < n2) ? A2[(size_t)(1 + b) * n2 + lane] : 0u;
        }
        const uint32_t umask = n2 >= 32 ? 0xffffffffu : ((1u << n2) - 1u);
        if (PL > 0 && lane <= 32) {
#pragma unroll
            for (int b = 0; b < PLA; ++b) s_pl[b][lane < 32 ? lane + 1 : 0] = lane < 32 ? p2[b] : 0u;
        }

        uint32_t ped = 0u, img = 0u, ein = 0u;
        uint32_t ph[8];
#pragma unroll
        for (int w = 0; w < 8; ++w) ph[w] = 0u;
        int nb = 1, hint = 0;
        uint32_t ce = 0u;   // this lane's evaluated children, summed over the wave at the end

        for (int i = 0; i < n1; ++i) {
            const uint32_t nbm = (uint32_t)__builtin_amdgcn_readlane((int)r1, i) & ((1u << i) - 1u);
            const int lab1 = __builtin_amdgcn_readlane(l1, i);
            const uint32_t degP = (uint32_t)__popc(nbm);
            uint32_t q[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) q[b] = (uint32_t)__builtin_amdgcn_readlane((int)p1[b], i) & nbm;
            const bool live = lane < nb;
            // entry 1 + u: (N2(u), label cost); entry 0 is the sentinel of an
            // exhausted free set (find-lowest-bit of an empty set is
            // 0xffffffff, one below entry 1): an empty row and a label cost
            // of 0xffffffff, which the saturating add below turns into an
            // invalid child
            if (lane <= 32) s_tab[lane < 32 ? lane + 1 : 0] = lane < 32 ? make_uint2(r2, l2 != lab1 ? vsub : 0u) : make_uint2(0u, INVALID);

            // ---------------- expand and evaluate
            uint32_t phi = 0u, phib[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) phib[b] = 0u;
            // word w of phi holds the images of g1 vertices 4w .. 4w+3: the
            // earlier neighbours are visited word by word (static register
            // indices), inside a word by a uniform loop over its set bits
#pragma unroll
            for (int w = 0; w < 8; ++w) {
                uint32_t nib = (nbm >> (4 * w)) & 0xfu;
                if (nib == 0u) continue;
                uint32_t qn[PLA];
#pragma unroll
                for (int b = 0; b < PLA; ++b) qn[b] = PL > 0 ? (q[b] >> (4 * w)) & 0xfu : 0u;
                do {
                    const uint32_t k = (uint32_t)__builtin_ctz(nib);
                    const uint32_t x = __builtin_amdgcn_ubfe(ph[w], k * 8u, 8u);
                    const uint32_t bit = x < 32u ? (1u << x) : 0u;
                    phi |= bit;
#pragma unroll
                    for (int b = 0; b < PLA; ++b)
                        if (PL > 0 && ((qn[b] >> k) & 1u)) phib[b] |= bit;
                    nib &= nib - 1u;
                } while (nib != 0u);
            }
            const uint32_t ai = img & ~phi;
            const uint32_t basel = live ? ped + mul_cost<SMALL>(degP, edel) : 0u;
            // child j of a slot substitutes its j-th free g2 vertex (free
            // vertices in ascending order: generation order)
            const uint32_t free = live ? (~img & umask) : 0u;
            const uint32_t nfree = (uint32_t)__popc(free);
            const int ngroups = (int)(wave_umax(nfree) + 3u) >> 2;   // children in groups of four
            // every child costs at least its parent (costs are
            // non-negative and |Phi & N2(u)| <= |P|), so the least parent
            // PED bounds every child from below: the byte-domain base
            const uint32_t base = wave_umin(live ? ped : INVALID);
            // the level's selection works on PEDs minus the base (candidates,
            // the deletion child, T), so a child's byte is min(value, 127)
            const uint32_t basel_r = basel - base;
            __syncthreads();
            uint32_t cand[32], pk[8];
            uint32_t lmin = INVALID;
            uint32_t fr = free;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                if (g < ngroups) {
                    uint32_t uw = 0u, e[4];
#pragma unroll
                    for (int j = 4 * g; j < 4 * g + 4; ++j) {
                        // 0xffffffff once exhausted: its byte and the later
                        // bytes of the word read 0xff, never selected
                        const uint32_t u = find_low(fr);
                        fr &= fr - 1u;
                        uw |= u << (8 * (j & 3));
                        const uint2 t = s_tab[u + 1u];
                        const uint32_t R = t.x;
                        // PED + label cost saturates only for the sentinel; its
                        // empty row keeps the edge terms at zero
                        uint32_t d = msub_cost<SMALL>((uint32_t)__popc(phi & R), nedel,
                                                      mad_cost<SMALL>((uint32_t)__popc(ai & R), eins,
                                                                      __builtin_elementwise_add_sat(basel_r, t.y)));
                        if (PL > 0) {
                            uint32_t diff = 0u;
#pragma unroll
                            for (int b = 0; b < PLA; ++b) diff |= phib[b] ^ s_pl[b][u + 1u];
                            d += mul_cost<SMALL>((uint32_t)__popc(phi & R & diff), esub);
                        }
                        cand[j] = d;
                        lmin = min(lmin, d);
                        // byte of the threshold search: min(PED - base, 127)
                        e[j & 3] = min(d, (uint32_t)TBYTE);
                    }
                    s_uv[g][lane] = uw;
                    pk[g] = pack4(e[0], e[1], e[2], e[3]);
                } else {
#pragma unroll
                    for (int j = 4 * g; j < 4 * g + 4; ++j) cand[j] = INVALID;
                    pk[g] = 0x7f7f7f7fu;   // 127s count below no threshold
                }
            }
            const uint32_t cdel = live ? basel_r + vdel : INVALID;
            // V = number of children; only V > K and min(V, K) are used, so
            // a full beam (every slot has its deletion child) needs one ballot
            ce += live ? nfree + 1u : 0u;
            int V;
            if (nb < K) V = (int)wave_sum(live ? nfree + 1u : 0u);
            else V = __ballot(nfree != 0u) != 0ull ? K + 1 : K;

            int nb_new;
            if (COMPLETE && i == n1 - 1) {
                // ---------------- complete-then-minimum last level: each
                // child's total (Sec. 4.4.1: the unused g2 vertices and the g2
                // edges with an unused end inserted); the least, first in
                // generation order, is the one survivor
                const uint32_t nu = (uint32_t)(n2 - __popc(img));
                const uint32_t mo = (uint32_t)g2.m - ein;   // g2 edges not inside Img
                uint32_t bt = INVALID, bj = DEL8;
#pragma unroll
                for (int g = 0; g < 8; ++g) {
                    if (g < ngroups) {
                        const uint32_t uw = s_uv[g][lane];
#pragma unroll
                        for (int k = 0; k < 4; ++k) {
                            const uint32_t d = cand[4 * g + k];
                            if (d == INVALID) continue;
                            const uint32_t R = s_tab[__builtin_amdgcn_ubfe(uw, (uint32_t)k * 8u, 8u) + 1u].x;
                            const uint32_t t = d + mul_cost<SMALL>(nu - 1u, vins) +
                                               mul_cost<SMALL>(mo - (uint32_t)__popc(img & R), eins);
                            if (t < bt) {
                                bt = t;
                                bj = (uint32_t)(4 * g + k);
                            }
                        }
                    }
                }
                if (live) {
                    const uint32_t t = cdel + mul_cost<SMALL>(nu, vins) + mul_cost<SMALL>(mo, eins);
                    if (t < bt) {
                        bt = t;
                        bj = DEL8;
                    }
                }
                const uint32_t wmin = wave_umin(bt);
                const int bl = (int)__builtin_ctzll(__ballot(bt == wmin));
                if (lane == bl) s_sel[0] = ((uint32_t)lane << 8) | bj;
                nb_new = 1;
            } else {
            // ---------------- threshold T: the K-th smallest PED
            uint32_t T = INVALID;
            int tbyte = -1;   // T - base when below 127
            const bool trim = V > K;
            const bool wide = ngroups > 4;
            if (trim) {
                // the least child m0 only steers the search: T - m0 (the
                // width of the kept window) changes little from level to
                // level, unlike T - base
                const uint32_t m0 = wave_umin(min(lmin, cdel));   // minus the base
                const int off = (int)min(m0, (uint32_t)TBYTE);   // count(t) = 0 for t < off
                const uint32_t pkd = 0x7f7f7f00u | min(cdel, (uint32_t)TBYTE);
                // count(PED <= base + ta) and count(PED <= base + tb), ta, tb
                // in [0, 126], summed in one reduction (low and high halves).
                // Words past the last group hold 127s and count nothing, so
                // the probe takes four or all eight words, straight-line.
                auto counts2 = [&](int ta, int tb) {
                    const uint32_t Ca = ((uint32_t)ta * 0x01010101u) | 0x80808080u;
                    const uint32_t Cb = ((uint32_t)tb * 0x01010101u) | 0x80808080u;
                    uint32_t ca = (uint32_t)__popc((Ca - pkd) & 0x80808080u);
                    uint32_t cb = (uint32_t)__popc((Cb - pkd) & 0x80808080u);
#pragma unroll
                    for (int g = 0; g < 4; ++g) {
                        ca += (uint32_t)__popc((Ca - pk[g]) & 0x80808080u);
                        cb += (uint32_t)__popc((Cb - pk[g]) & 0x80808080u);
                    }
                    if (wide) {
#pragma unroll
                        for (int g = 4; g < 8; ++g) {
                            ca += (uint32_t)__popc((Ca - pk[g]) & 0x80808080u);
                            cb += (uint32_t)__popc((Cb - pk[g]) & 0x80808080u);
                        }
                    }
                    return wave_sum(ca | (cb << 16));
                };
                // smallest t in [lo, hi] with count(t) >= K; hi = 127 stands
                // for "none below 127".  Two thresholds per round: first
                // m0 - base plus the previous level's T - m0, and the one
                // below it, then galloping up (no upper bound yet) or down
                // (no lower bound yet), then thirds of [lo, hi).
                int lo = off, hi = TBYTE;
                int ta = max(min(hint + off, TBYTE - 1) - 1, off);
                int tb = min(ta + 1, TBYTE - 1);
                for (int s = 1; lo < hi; s <<= 1) {
                    const uint32_t c2 = counts2(ta, tb);
                    if ((int)(c2 >> 16) >= K) hi = min(hi, tb);
                    else lo = max(lo, tb + 1);
                    if ((int)(c2 & 0xffffu) >= K) hi = min(hi, ta);
                    else lo = max(lo, ta + 1);
                    if (lo >= hi) break;
                    if (hi == TBYTE) {
                        ta = min(lo + s - 1, TBYTE - 1);
                        tb = min(lo + 2 * s, TBYTE - 1);
                    } else if (lo == off) {
                        tb = hi - 1;
                        ta = max(hi - 1 - s, off);
                    } else {
                        const int span = hi - lo;     // probe points lie in [lo, hi - 1]
                        ta = lo + (span - 1) / 3;
                        tb = lo + (2 * span - 1) / 3;
                    }
                }
                if (lo < TBYTE) {
                    T = (uint32_t)lo;
                    tbyte = lo;
                    hint = lo - off;
                } else {
                    // T >= base + 127: exact counts on the full values
                    auto count_le = [&](uint32_t t) {
                        int cnt = __popcll(__ballot(cdel <= t));
#pragma unroll
                        for (int g = 0; g < 8; ++g) {
                            if (g < ngroups) {
#pragma unroll
                                for (int u = 4 * g; u < 4 * g + 4; ++u) cnt += __popcll(__ballot(cand[u] <= t));
                            }
                        }
                        return cnt;
                    };
                    uint32_t l2o = (uint32_t)TBYTE, tt = l2o, step = 1, h2;
                    for (;;) {
                        if (count_le(tt) >= K) {
                            h2 = tt;
                            break;
                        }
                        l2o = tt + 1;
                        // count_le(INVALID - 1) = V > K, so the walk stops by then
                        tt = (tt > INVALID - 1u - step) ? INVALID - 1u : tt + step;
                        step = step < (1u << 29) ? step << 1 : step;
                    }
                    while (l2o < h2) {
                        const uint32_t mid = l2o + ((h2 - l2o) >> 1);
                        if (count_le(mid) >= K) h2 = mid;
                        else l2o = mid + 1;
                    }
                    T = l2o;
                    hint = TBYTE - 1;
                }
            }

            // ---------------- survivors in generation order
            // bit j of ltm / lem: child j below / at most T
            uint32_t ltm = 0u, lem = 0u;
            if (tbyte >= 0) {
                // from the bytes: the flag bits of byte b of word g (set iff
                // e <= t, as in the probes) are gathered by byte dot
                // products with the weights 2^b (even g) and 2^(4+b) (odd g)
                // into 128 x the mask byte of words g, g + 1
                const uint32_t Cle = ((uint32_t)tbyte * 0x01010101u) | 0x80808080u;
                const uint32_t Clt = tbyte > 0 ? (((uint32_t)tbyte - 1u) * 0x01010101u) | 0x80808080u : 0x7f7f7f7fu;
                auto byte_mask = [&](uint32_t C) {
                    uint32_t acc[4];
#pragma unroll
                    for (int h = 0; h < 4; ++h) {
                        if (h < 2 || wide) {
                            acc[h] = __builtin_amdgcn_udot4((C - pk[2 * h + 1]) & 0x80808080u, 0x80402010u, 0u, false);
                            acc[h] = __builtin_amdgcn_udot4((C - pk[2 * h]) & 0x80808080u, 0x08040201u, acc[h], false);
                        }
                    }
                    uint32_t m = (acc[0] >> 7) | (acc[1] << 1);
                    if (wide) m |= (acc[2] << 9) | (acc[3] << 17);
                    return m;
                };
                lem = byte_mask(Cle);
                ltm = byte_mask(Clt);
            } else {
                // full-width compares (every child kept, or T 127 or more
                // above the base), built high j first
#pragma unroll
                for (int g = 7; g >= 0; --g) {
                    if (g < ngroups) {
#pragma unroll
                        for (int u = 4 * g + 3; u >= 4 * g; --u) {
                            shift_in2(ltm, cand[u] < T, lem, cand[u] <= T);
                        }
                    }
                }
            }
            const uint32_t eqm = trim ? (lem & ~ltm) : 0u;
            const bool ltd = cdel < T;
            const bool eqd = trim && cdel == T;
            const int lt_l = __popc(ltm) + (ltd ? 1 : 0);
            const int eq_l = __popc(eqm) + (eqd ? 1 : 0);
            // one scan of (lt_l, eq_l) in 16-bit halves (sums <= 64 * 33):
            // the children below T in earlier lanes, the ties in earlier
            // lanes, and from the last lane the wave's total below T
            const int own = lt_l | (eq_l << 16);
            const int ex = wave_excl_scan(own);
            const int tot_lt = __builtin_amdgcn_readlane(ex + own, 63) & 0xffff;
            const int ex_lt = ex & 0xffff, ex_eq = (int)((uint32_t)ex >> 16);
            // quota > 0 under trim: fewer than K children lie below T
            const int quota = trim ? K - tot_lt : 0;
            int r = min(max(quota - ex_eq, 0), eq_l);
            uint32_t keepm = ltm;
            bool keepd = ltd;
            const int ne = __popc(eqm);
            if (r >= ne) {             // every tie of the slot is within the quota
                keepm |= eqm;
                r -= ne;
            } else {                   // the slot where the quota ends: its first r ties
                for (uint32_t e = eqm; r > 0; e &= e - 1u, --r) keepm |= e & (0u - e);
            }
            if (r > 0 && eqd) keepd = true;
            // earlier lanes keep all their children below T and the ties up
            // to the quota, in lane order
            int pos = ex_lt + min(quota, ex_eq);
            for (uint32_t mk = keepm; mk; mk &= mk - 1u) s_sel[pos++] = ((uint32_t)lane << 8) | (uint32_t)__builtin_ctz(mk);
            if (keepd) s_sel[pos] = ((uint32_t)lane << 8) | DEL8;
            nb_new = min(V, K);
            }
            __syncthreads();

            // ---------------- update: child = parent + (v_i -> u)
            const bool live2 = lane < nb_new;
            const uint32_t sel = live2 ? s_sel[lane] : 0u;
            const int p = (int)(sel >> 8);
            const uint32_t jc = sel & 0xffu;
            const bool sub = jc != DEL8;
            const uint32_t u = sub ? __builtin_amdgcn_ubfe(s_uv[(jc >> 2) & 7u][p], (jc & 3u) * 8u, 8u) : DEL8;
            const uint32_t us = sub ? u + 1u : 0u;   // table entry (0: the sentinel)
            const uint32_t basel_p = (uint32_t)__shfl((int)basel, p);
            const uint32_t phi_p = (uint32_t)__shfl((int)phi, p);
            const uint32_t ai_p = (uint32_t)__shfl((int)ai, p);
            const uint32_t img_p = (uint32_t)__shfl((int)img, p);
            const uint32_t ein_p = (uint32_t)__shfl((int)ein, p);
            const uint2 tu = s_tab[us];
            const uint32_t R = tu.x;
            const uint32_t vs_u = tu.y;
            uint32_t rp[PLA], phbp[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) {
                rp[b] = PL > 0 ? s_pl[b][us] : 0u;
                phbp[b] = PL > 0 ? (uint32_t)__shfl((int)phib[b], p) : 0u;
            }
            const int wl = i >> 2;
#pragma unroll
            for (int w = 0; w < 8; ++w)
                if (w <= wl) ph[w] = (uint32_t)__shfl((int)ph[w], p);
            if (live2) {
                if (sub) {
                    uint32_t d = msub_cost<SMALL>((uint32_t)__popc(phi_p & R), nedel,
                                                  mad_cost<SMALL>((uint32_t)__popc(ai_p & R), eins, basel_p + vs_u));
                    if (PL > 0) {
                        uint32_t diff = 0u;
#pragma unroll
                        for (int b = 0; b < PLA; ++b) diff |= phbp[b] ^ rp[b];
                        d += mul_cost<SMALL>((uint32_t)__popc(phi_p & R & diff), esub);
                    }
                    ped = d;
                    img = img_p | (1u << u);
                    ein = ein_p + (uint32_t)__popc(img_p & R);
                } else {
                    ped = basel_p + vdel;
                    img = img_p;
                    ein = ein_p;
                }
            }
            // byte i of the mapping
            const uint32_t sh = (uint32_t)(i & 3) * 8u;
#pragma unroll
            for (int w = 0; w < 8; ++w)
                if (w == wl) ph[w] = (ph[w] & ~(0xffu << sh)) | (u << sh);
            nb = nb_new;
        }

        // ---------------- completion and best leaf
        const uint32_t total = lane < nb ? ped + mul_cost<SMALL>((uint32_t)(n2 - __popc(img)), vins) +
                                               mul_cost<SMALL>((uint32_t)g2.m - ein, eins)
                                         : INVALID;
        const uint32_t best_total = wave_umin(total);
        const uint32_t ce_total = wave_sum(ce);
        const int best = (int)__builtin_ctzll(__ballot(total == best_total));
        if (lane == 0) {
            a.out.dist[wi.out] = (int)best_total;
            if (a.out.cand) a.out.cand[wi.out] = (long long)ce_total;
        }
        uint32_t word = 0u;
#pragma unroll
        for (int w = 0; w < 8; ++w) {
            const uint32_t bw = (uint32_t)__builtin_amdgcn_readlane((int)ph[w], best);
            word = (lane >> 2) == w ? bw : word;
        }
        if (lane < n1) {
            const uint32_t x = __builtin_amdgcn_ubfe(word, (uint32_t)(lane & 3) * 8u, 8u);
            a.out.map[wi.map_off + lane] = (x == DEL8) ? -1 : (int)x;
        }
        __syncthreads();
    }
}

template <int PL, bool SMALL, bool COMPLETE>
const void *wave_ptr() {
    return reinterpret_cast<const void *>(&kb_wave_kernel<PL, SMALL, COMPLETE>);
}

// the complete-then-minimum last level is a kernel of its own, so that the
// default search keeps its register budget
template <bool COMPLETE>
const void *select_wave_c(int PL, bool small) {
    if (PL == 0) return small ? wave_ptr<0, true, COMPLETE>() : wave_ptr<0, false, COMPLETE>();
    if (PL == 2) return small ? wave_ptr<2, true, COMPLETE>() : wave_ptr<2, false, COMPLETE>();
    if (PL == 4) return small ? wave_ptr<4, true, COMPLETE>() : wave_ptr<4, false, COMPLETE>();
    return nullptr;
}

const void *select_wave(int PL, bool small, bool complete) {
    return complete ? select_wave_c<true>(PL, small) : select_wave_c<false>(PL, small);
}

bool small_costs(const Costs &c) {
    const int32_t lim = 1 << 22;
    return c.vsub < lim && c.vdel < lim && c.vins < lim && c.esub < lim && c.edel < lim && c.eins < lim;
}

}  // namespace

hipError_t wave_max_resident(int PL, int last_complete, int *blocks_per_cu) {
    const void *k = select_wave(PL, true, last_complete != 0);
    const void *k2 = select_wave(PL, false, last_complete != 0);
    if (!k || !k2) return hipErrorInvalidValue;
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k2, 64, 0);
    *blocks_per_cu = a < b ? a : b;
    return e;
}

hipError_t launch_wave(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue, Costs c,
                       int K, int last_complete, Outputs out, int grid, hipStream_t stream) {
    const void *k = select_wave(PL, small_costs(c), last_complete != 0);
    if (!k || grid <= 0 || K > kWaveMaxK) return hipErrorInvalidValue;
    WaveArgs a;
    a.src = src;
    a.dst = dst;
    a.work = work;
    a.nwork = nwork;
    a.queue = queue;
    a.c = c;
    a.K = K;
    a.out = out;
    void *args[] = {&a};
    return hipLaunchKernel(k, dim3(grid), dim3(64), args, 0, stream);
}

}  // namespace gedk
