// kb_wave2.h -- wavefront-per-pair K-Best search for targets of up to 64
// vertices on gfx950 (the kernel template; kb_wave2.hip instantiates one
// beam slot per lane, kb_wave2_k128.hip two, kb_wave2_src128.hip sources of
// up to 128 vertices).
//
// The same scheme as kb_wave.hip (one 64-lane wavefront per pair, persistent
// over a work queue whose first pair is the workgroup's index) for n2 <= 64:
// target vertex sets are 64-bit (two words), the mapping phi is M words of
// bytes (M = 16: sources of up to 64 vertices, a lane holding g1's row of
// its own index; M = 32: up to 128, row v_i read once per level), and a
// slot has up to 64 substitution children, too many to keep as 32-bit
// values.  A lane holds S beam slots (S = 1: K <= 64; S = 2: K <= 128);
// slot s lives in lane s / S, register set s % S, so the slots of one lane
// are neighbours in the beam's order and every scan over lanes gives the
// slots' order directly.  Children are scored straight into bytes relative
// to a base b:
//   x = 0 if PED < b, else min((PED - b) >> sh, 126) + 1,
// four to a register, and the threshold search, the keep masks and the tie
// quota all work on those bytes:
//   fast pass   b = the least PED of the beam's slots (every child's PED is at
//               least its parent's, so nothing lies below b) and sh = 0: the
//               bytes are exact offsets for PEDs below b + 126.  This holds
//               whenever the K-th smallest child is within 125 of the least
//               parent, which is the common case.
//   otherwise   the children are scored again with b = that least PED + 126
//               and sh = 24 (buckets of 2^24 cover every valid PED), the
//               bucket holding the K-th smallest child becomes the new base
//               and sh drops by 7, until sh = 0 and the threshold is exact
//               (at most five more passes).
// count(x <= t) for 1 <= t <= 126 is a popcount of byte-wise compares
// (((t * 0x01010101) | 0x80808080) - packed) & 0x80808080, summed over the
// wave; two thresholds per reduction, starting from the previous level's t.
// With T = b + t* - 1 found in the final pass, a child is below T iff its
// byte is below t* and equal to T iff its byte is t*; children below b have
// byte 0 and are below T.
//
// Per level i (Alg. 1), with P = earlier neighbours of v_i, Phi = images of
// P, A = Img \ Phi: the child (v_i -> u) costs
//   (PED + edel |P|) + vsub [alpha1(v_i) != alpha2(u)] + eins |A & N2(u)|
//   - edel |Phi & N2(u)| [+ esub |Phi & N2(u) & relabelled|]      (Sec. 2.3)
// and child j of a slot substitutes its j-th free g2 vertex (ascending, so
// j order is generation order), with N2(u) and the label cost from a
// per-level LDS table whose entry 64 is a sentinel for exhausted free sets
// (empty row, label cost 0xffffffff, saturating add: the invalid value
// 0xffffffff).  The deletion child costs PED + vdel + edel |P|.  Survivors:
// every child below T and the first (K - #below) children equal to T in
// generation order (slot, then j, then the deletion) -- bit masks gathered
// from the bytes' flags by byte dot products, and one exclusive scan of the
// per-lane (below, tie) counts in 16-bit halves for the quota and the
// positions -- written to LDS as (parent slot, j); a new slot finds its
// vertex and recomputes its PED with the same formula.  With a full beam
// only V > K matters (the number of children), which one ballot decides.  With one slot per lane the parent's state comes over
// the wave's lane permute and the child's vertex from a per-level LDS table;
// with two, every parent's mapping words, PED, edge count and Img go through
// LDS, the new slot rebuilds the parent's Phi from them and finds its vertex
// as the j-th free one.  Completion adds vins (n2 - |Img|) + eins (m2 -
// e_in) (Sec. 4.4.1); the first slot of least total is the result.  The
// COMPLETE instantiation's last level instead completes every child and
// keeps only the least total (first in generation order).
//
// The DIR instantiation takes directed pairs of up to 32 vertices (each edge
// an arc, one edit operation per arc): a vertex's 64-bit row is its out-arc
// row in the low word and its in-arc row in the high word, Img holds the
// image in both words, and an earlier neighbour j + 32 of the g1 row (an
// in-arc of v_i from j) sets its Phi bit in the high word.  The formulas
// above then count kept, deleted, inserted and relabelled arcs of both
// directions at once (the implied operations of Sec. 2.3 per arc direction);
// only |Img| reads the low word alone.
#pragma once

#include "ged_internal.h"
#include "wave_common.h"

namespace gedk {
namespace w2 {

using namespace wv;

constexpr uint32_t INVALID = 0xffffffffu;
constexpr uint32_t DEL8 = 0xffu;
constexpr int TOP = 127;          // byte above every threshold (126 is the largest)

struct Wave2Args {
    DbView src;   // graphs edited (g1)
    DbView dst;   // target graphs (g2); same edge-label coding as src
    const WorkItem *work;
    int nwork;
    int *queue;
    Costs c;
    int K;
    Outputs out;
};

__device__ __forceinline__ uint64_t u64(uint32_t lo, uint32_t hi) { return ((uint64_t)hi << 32) | lo; }

__device__ __forceinline__ uint64_t readlane64(uint64_t v, int l) {
    return u64((uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, l),
               (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), l));
}

__device__ __forceinline__ uint64_t shfl64(uint64_t v, int l) {
    return u64((uint32_t)__shfl((int)(uint32_t)v, l), (uint32_t)__shfl((int)(uint32_t)(v >> 32), l));
}

__device__ __forceinline__ uint32_t popc64(uint64_t v) { return (uint32_t)__popcll(v); }

// byte of a child's PED against base b and shift sh (see above)
__device__ __forceinline__ uint32_t to_byte(uint32_t d, uint32_t b, int sh) {
    return d < b ? 0u : min((d - b) >> sh, 126u) + 1u;
}

// position of the j-th set bit of m (j < popcount(m)), by halving
__device__ __forceinline__ uint32_t nth_bit64(uint64_t m, uint32_t j) {
    const uint32_t lo = (uint32_t)m;
    const uint32_t c32 = (uint32_t)__popc(lo);
    const bool up = j >= c32;
    uint32_t x = up ? (uint32_t)(m >> 32) : lo;
    uint32_t pos = up ? 32u : 0u;
    j = up ? j - c32 : j;
#pragma unroll
    for (int half = 16; half >= 1; half >>= 1) {
        const uint32_t c = (uint32_t)__popc(x & ((1u << half) - 1u));
        const bool hi = j >= c;
        j = hi ? j - c : j;
        x = hi ? x >> half : x;
        pos = hi ? pos + (uint32_t)half : pos;
    }
    return pos;
}

template <int S, int M, int PL, bool SMALL, bool COMPLETE, bool DIR>
__global__ __launch_bounds__(64) void kb_wave2_kernel(Wave2Args a) {
    static_assert(M == 16 || (M == 32 && !DIR), "mapping of 64 source vertices, or 128 undirected");
    constexpr int PLA = PL > 0 ? PL : 1;
    constexpr int NS = 64 * S;              // beam slots
    constexpr int PW = 20;                  // parent words (S = 2): 16 of phi, PED, e_in, Img lo, Img hi
    __shared__ uint32_t s_sel[NS];          // survivor: parent slot << 8 | j (0xff = deletion)
    __shared__ uint4 s_tab[65];             // per level: (N2(u) lo, hi, label cost, 0); [64] = sentinel
    // S = 1: [j / 4 * 64 + slot] = g2 vertices of children j, bytes;
    // S = 2: [w * NS + slot] = parent word w (16 mapping words -- a 32-word
    // mapping goes through in two halves -- then PED, e_in, Img)
    __shared__ __align__(16) uint32_t s_aux[S == 1 ? 16 * 64 : PW * NS];
    __shared__ uint2 s_pl[PLA][65];         // label-plane rows of g2; [64] = 0
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const uint32_t vsub = (uint32_t)a.c.vsub, vdel = (uint32_t)a.c.vdel, vins = (uint32_t)a.c.vins;
    const uint32_t esub = (uint32_t)a.c.esub, edel = (uint32_t)a.c.edel, eins = (uint32_t)a.c.eins;
    const uint32_t nedel = 0u - edel;
    const int K = a.K;
    const int P = a.dst.planes;

    for (bool first = true;; first = false) {
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
        const int n1 = g1.n, n2 = g2.n, w1 = g1.w, w2 = g2.w;
        const uint32_t *A1 = a.src.adj + g1.adj;
        const uint32_t *A2 = a.dst.adj + g2.adj;
        // directed (n <= 32, one row word): the in-arc rows and planes follow the out-arc ones
        const uint32_t *A1in = A1 + (size_t)(1 + a.src.planes) * n1 * w1;
        const uint32_t *A2in = A2 + (size_t)(1 + P) * n2 * w2;
        // M = 16: lane v holds g1's row v and its label; M = 32 loads row v_i per level
        const uint64_t r1 = M == 16 && lane < n1 ? u64(A1[(size_t)lane * w1], DIR ? A1in[(size_t)lane * w1]
                                                                     : (w1 > 1 ? A1[(size_t)lane * w1 + 1] : 0u))
                                      : 0ull;
        const uint64_t r2 = lane < n2 ? u64(A2[(size_t)lane * w2], DIR ? A2in[(size_t)lane * w2]
                                                                     : (w2 > 1 ? A2[(size_t)lane * w2 + 1] : 0u))
                                      : 0ull;
        const int l1 = M == 16 && lane < n1 ? a.src.vlab[g1.vlab + lane] : 0;
        const int l2 = lane < n2 ? a.dst.vlab[g2.vlab + lane] : 0;
        uint64_t p1[PLA];
#pragma unroll
        for (int b = 0; b < PLA; ++b) {
            p1[b] = 0ull;
            if (PL > 0 && M == 16 && b < P && lane < n1) {
                const uint32_t *B1 = A1 + (size_t)(1 + b) * n1 * w1 + (size_t)lane * w1;
                const uint32_t *B1in = A1in + (size_t)(1 + b) * n1 * w1 + (size_t)lane * w1;
                p1[b] = u64(B1[0], DIR ? B1in[0] : (w1 > 1 ? B1[1] : 0u));
            }
            if (PL > 0 && lane <= 64) {
                uint2 v = make_uint2(0u, 0u);
                if (b < P && lane < n2) {
                    const uint32_t *B2 = A2 + (size_t)(1 + b) * n2 * w2 + (size_t)lane * w2;
                    const uint32_t *B2in = A2in + (size_t)(1 + b) * n2 * w2 + (size_t)lane * w2;
                    v = make_uint2(B2[0], DIR ? B2in[0] : (w2 > 1 ? B2[1] : 0u));
                }
                s_pl[b][lane] = v;
            }
        }
        if (PL > 0 && lane == 0) {
#pragma unroll
            for (int b = 0; b < PLA; ++b) s_pl[b][64] = make_uint2(0u, 0u);
        }
        const uint64_t umask = n2 >= 64 ? ~0ull : ((1ull << n2) - 1ull);

        // the lane's beam slots S * lane + h
        uint32_t ped[S], ein[S];
        uint64_t img[S];
        uint32_t ph[S][M];
#pragma unroll
        for (int h = 0; h < S; ++h) {
            ped[h] = 0u;
            ein[h] = 0u;
            img[h] = 0ull;
#pragma unroll
            for (int w = 0; w < M; ++w) ph[h][w] = 0u;
        }
        int nb = 1, hint = 1;
        uint32_t ce = 0u;   // this lane's evaluated children, summed over the wave at the end

        for (int i = 0; i < n1; ++i) {
            // earlier neighbours of v_i (nlo: vertices 0..63, nhi: 64..127) and
            // their label-plane bits
            uint64_t nlo, nhi = 0ull, qlo[PLA], qhi[PLA];
            int lab1;
            if constexpr (M == 16) {
                const uint64_t below = DIR ? (((1ull << i) - 1ull) * 0x100000001ull)   // i < 32: both words
                                           : (i >= 64 ? ~0ull : ((1ull << i) - 1ull));
                nlo = readlane64(r1, i) & below;
                lab1 = __builtin_amdgcn_readlane(l1, i);
#pragma unroll
                for (int b = 0; b < PLA; ++b) {
                    qlo[b] = PL > 0 ? readlane64(p1[b], i) & nlo : 0ull;
                    qhi[b] = 0ull;
                }
            } else {
                // row v_i of g1 (w1 <= 4 words) and its planes, the same address in every lane
                auto word = [&](const uint32_t *r, int k) -> uint32_t {
                    return k < w1 ? (uint32_t)__builtin_amdgcn_readfirstlane((int)r[k]) : 0u;
                };
                const uint32_t *row = A1 + (size_t)i * w1;
                const uint64_t blo = i >= 64 ? ~0ull : ((1ull << i) - 1ull);
                const uint64_t bhi = i <= 64 ? 0ull : ((1ull << (i - 64)) - 1ull);
                nlo = u64(word(row, 0), word(row, 1)) & blo;
                nhi = u64(word(row, 2), word(row, 3)) & bhi;
                lab1 = __builtin_amdgcn_readfirstlane(a.src.vlab[g1.vlab + i]);
#pragma unroll
                for (int b = 0; b < PLA; ++b) {
                    qlo[b] = 0ull;
                    qhi[b] = 0ull;
                    if (PL > 0 && b < P) {
                        const uint32_t *pr = A1 + (size_t)(1 + b) * n1 * w1 + (size_t)i * w1;
                        qlo[b] = u64(word(pr, 0), word(pr, 1)) & nlo;
                        qhi[b] = u64(word(pr, 2), word(pr, 3)) & nhi;
                    }
                }
            }
            const uint32_t degP = popc64(nlo) + popc64(nhi);
            const uint32_t edP = mul_cost<SMALL>(degP, edel);
            // lane u: (N2(u), label cost); entry 64: the exhausted-set sentinel
            s_tab[lane] = make_uint4((uint32_t)r2, (uint32_t)(r2 >> 32), l2 != lab1 ? vsub : 0u, 0u);
            if (lane == 0) s_tab[64] = make_uint4(0u, 0u, INVALID, 0u);

            // Phi (and its label-plane sets) of a slot whose mapping words are m:
            // word by word, the earlier neighbours in it by a loop over the
            // word's bits (uniform), so that no per-bit condition outlives it
            auto build_phi = [&](const uint32_t (&m)[M], uint64_t &phi, uint64_t (&phib)[PLA]) {
                phi = 0ull;
#pragma unroll
                for (int b = 0; b < PLA; ++b) phib[b] = 0ull;
#pragma unroll
                for (int w = 0; w < M; ++w) {
                    const uint64_t nw = w < 16 ? nlo : nhi;   // a constant choice once unrolled
                    uint32_t nib = (uint32_t)(nw >> (4 * (w & 15))) & 0xfu;
                    if (nib == 0u) continue;
                    // directed: bits 32..63 (words 8..15) are in-arcs from vertices j - 32
                    const uint32_t mw = m[DIR && w >= 8 ? w - 8 : w];   // a constant index once unrolled
                    const uint32_t up = DIR && w >= 8 ? 32u : 0u;
                    uint32_t qn[PLA];
#pragma unroll
                    for (int b = 0; b < PLA; ++b)
                        qn[b] = PL > 0 ? (uint32_t)((w < 16 ? qlo[b] : qhi[b]) >> (4 * (w & 15))) & 0xfu : 0u;
                    do {
                        const uint32_t k = (uint32_t)__builtin_ctz(nib);
                        const uint32_t x = __builtin_amdgcn_ubfe(mw, k * 8u, 8u);
                        const uint64_t bit = x < 64u ? (1ull << (x + up)) : 0ull;
                        phi |= bit;
#pragma unroll
                        for (int b = 0; b < PLA; ++b)
                            if (PL > 0 && ((qn[b] >> k) & 1u)) phib[b] |= bit;
                        nib &= nib - 1u;
                    } while (nib != 0u);
                }
            };

            // ---------------- Phi and the children of every slot
            bool live[S];
            uint64_t phi[S], phib[S][PLA], ai[S], free[S];
            uint32_t basel[S], basel_r[S], nfree[S], cdel[S];
            uint32_t nfmax = 0u, vl = 0u;
#pragma unroll
            for (int h = 0; h < S; ++h) {
                live[h] = S * lane + h < nb;
                build_phi(ph[h], phi[h], phib[h]);
                ai[h] = img[h] & ~phi[h];
                basel[h] = live[h] ? ped[h] + edP : 0u;
                free[h] = live[h] ? (~img[h] & umask) : 0ull;
                nfree[h] = popc64(free[h]);
                nfmax = max(nfmax, nfree[h]);
                vl += live[h] ? nfree[h] + 1u : 0u;
                cdel[h] = live[h] ? basel[h] + vdel : INVALID;
            }
            const int ngroups = (int)(wave_umax(nfmax) + 3u) >> 2;   // children in groups of four
            // V = number of children; only V > K and min(V, K) are used, so
            // a full beam (every slot has its deletion child) needs one ballot
            ce += vl;
            int V;
            if (nb < K) V = (int)wave_sum(vl);
            else V = __ballot(nfmax != 0u) != 0ull ? K + 1 : K;
            const bool trim = V > K;
            __syncthreads();

            // PED of the child of slot h substituting v_i by u (u = 64: the
            // exhausted-set sentinel, whose label cost saturates the sum to
            // 0xffffffff)
            auto score = [&](int h, uint32_t u) -> uint32_t {
                const uint4 t = s_tab[u];
                const uint64_t R = u64(t.x, t.y);
                uint32_t d = msub_cost<SMALL>(popc64(phi[h] & R), nedel,
                                              mad_cost<SMALL>(popc64(ai[h] & R), eins,
                                                              __builtin_elementwise_add_sat(basel_r[h], t.z)));
                if (PL > 0) {
                    uint64_t diff = 0ull;
#pragma unroll
                    for (int b = 0; b < PLA; ++b) {
                        const uint2 pl = s_pl[b][u];
                        diff |= phib[h][b] ^ u64(pl.x, pl.y);
                    }
                    d += mul_cost<SMALL>(popc64(phi[h] & R & diff), esub);
                }
                return d;
            };
            // one pass: every child's byte against (base, sh) into pk; the
            // first pass (base 0, sh 0: a child's byte is min(value, 126) + 1,
            // nothing lies below) of a one-slot wave also records each
            // child's vertex.  Values are PEDs minus the least parent PED.
            uint32_t pk[S][16];
            auto pass = [&](uint32_t base, int sh, bool record) {
#pragma unroll
                for (int h = 0; h < S; ++h) {
                    uint64_t fr = free[h];
#pragma unroll
                    for (int g = 0; g < 16; ++g) {
                        if (g < ngroups) {
                            uint32_t w = 0u, uw = 0u;
#pragma unroll
                            for (int k = 0; k < 4; ++k) {
                                const uint32_t u = (uint32_t)__builtin_ctzg(fr, 64);   // 64 once exhausted
                                fr &= fr - 1ull;
                                uw |= u << (8 * k);
                                const uint32_t d = score(h, u);
                                w |= (record ? min(d, 126u) : to_byte(d, base, sh)) << (8 * k);
                            }
                            pk[h][g] = record ? w + 0x01010101u : w;   // bytes <= 127: no carry
                            if constexpr (S == 1)
                                if (record) s_aux[g * 64 + lane] = uw;
                        } else {
                            pk[h][g] = 0x7f7f7f7fu;
                        }
                    }
                }
            };
            // the deletion children's bytes, one per slot, the rest 127
            auto del_bytes = [&](uint32_t base, int sh) {
                uint32_t v = 0x7f7f7f7fu;
#pragma unroll
                for (int h = 0; h < S; ++h) v = (v & ~(0xffu << (8 * h))) | (to_byte(cdel[h], base, sh) << (8 * h));
                return v;
            };
            // count(byte <= ta) and count(byte <= tb), summed over the wave in
            // the low and high halves of one word
            auto counts2 = [&](uint32_t pkd, int ta, int tb) {
                const uint32_t Ca = ((uint32_t)ta * 0x01010101u) | 0x80808080u;
                const uint32_t Cb = ((uint32_t)tb * 0x01010101u) | 0x80808080u;
                uint32_t ca = (uint32_t)__popc((Ca - pkd) & 0x80808080u);
                uint32_t cb = (uint32_t)__popc((Cb - pkd) & 0x80808080u);
                // words past the last group hold 127s and count nothing:
                // guards per four words
#pragma unroll
                for (int h = 0; h < S; ++h) {
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        if (4 * q < ngroups) {
#pragma unroll
                            for (int g = 4 * q; g < 4 * q + 4; ++g) {
                                ca += (uint32_t)__popc((Ca - pk[h][g]) & 0x80808080u);
                                cb += (uint32_t)__popc((Cb - pk[h][g]) & 0x80808080u);
                            }
                        }
                    }
                }
                return wave_sum(ca | (cb << 16));
            };
            // smallest t in [1, 126] with count(byte <= t) >= K (127 = none),
            // two thresholds per round starting at `start`
            auto search = [&](uint32_t pkd, int start) {
                int lo = 1, hi = TOP;
                int ta = max(min(start, TOP - 1) - 1, 1);
                int tb = min(ta + 1, TOP - 1);
                for (int s = 1;; s <<= 1) {
                    const uint32_t c2 = counts2(pkd, ta, tb);
                    if ((int)(c2 >> 16) >= K) hi = min(hi, tb);
                    else lo = max(lo, tb + 1);
                    if ((int)(c2 & 0xffffu) >= K) hi = min(hi, ta);
                    else lo = max(lo, ta + 1);
                    if (lo >= hi) break;
                    if (hi == TOP) {
                        ta = min(lo + s - 1, TOP - 1);
                        tb = min(lo + 2 * s, TOP - 1);
                    } else if (lo == 1) {
                        tb = hi - 1;
                        ta = max(hi - 1 - s, 1);
                    } else {
                        const int span = hi - lo;   // probe points lie in [lo, hi - 1]
                        ta = lo + (span - 1) / 3;
                        tb = lo + (2 * span - 1) / 3;
                    }
                }
                return lo;
            };

            // ---------------- threshold T (byte t_T in the final pass)
            uint32_t mp = INVALID;
#pragma unroll
            for (int h = 0; h < S; ++h) mp = min(mp, live[h] ? ped[h] : INVALID);
            const uint32_t m0 = wave_umin(mp);   // no child lies below
            // the level's selection works on PEDs minus m0
#pragma unroll
            for (int h = 0; h < S; ++h) {
                basel_r[h] = basel[h] - m0;
                cdel[h] = live[h] ? cdel[h] - m0 : INVALID;
            }
            pass(0u, 0, true);
            int nb_new;
            if (COMPLETE && i == n1 - 1) {
                // ---------------- complete-then-minimum last level: each
                // child's total (Sec. 4.4.1); the least, first in generation
                // order, is the one survivor
                uint32_t bt = INVALID, bsel = 0u;
#pragma unroll
                for (int h = 0; h < S; ++h) {
                    const uint32_t slot = (uint32_t)(S * lane + h);
                    const uint32_t nu = (uint32_t)n2 - (DIR ? (uint32_t)__popc((uint32_t)img[h]) : popc64(img[h]));
                    const uint32_t mo = (uint32_t)g2.m - ein[h];   // g2 edges not inside Img
                    uint64_t fr = free[h];
                    for (uint32_t j = 0; fr; ++j, fr &= fr - 1ull) {
                        const uint32_t u = (uint32_t)__builtin_ctzll(fr);
                        const uint4 tu = s_tab[u];
                        const uint32_t t = score(h, u) + mul_cost<SMALL>(nu - 1u, vins) +
                                           mul_cost<SMALL>(mo - popc64(img[h] & u64(tu.x, tu.y)), eins);
                        if (t < bt) {
                            bt = t;
                            bsel = (slot << 8) | j;
                        }
                    }
                    if (live[h]) {
                        const uint32_t t = cdel[h] + mul_cost<SMALL>(nu, vins) + mul_cost<SMALL>(mo, eins);
                        if (t < bt) {
                            bt = t;
                            bsel = (slot << 8) | DEL8;
                        }
                    }
                }
                const uint32_t wmin = wave_umin(bt);
                const int bl = (int)__builtin_ctzll(__ballot(bt == wmin));
                if (lane == bl) s_sel[0] = bsel;
                nb_new = 1;
            } else {
            uint32_t T = INVALID;
            int tT = TOP;   // no trimming: every child with a byte below 127 survives
            if (trim) {
                uint32_t base = 0u;
                int sh = 0;
                int t = search(del_bytes(base, sh), hint);
                if (t < TOP) {
                    hint = t;
                } else {
                    // the K-th child lies 126 or more above the least parent:
                    // bucket passes from 2^24 down to exact offsets
                    base = 126u;
                    sh = 24;
                    for (;;) {
                        pass(base, sh, false);
                        t = search(del_bytes(base, sh), 63);
                        if (sh == 0 && t < TOP) break;
                        if (t < TOP) {
                            base += (uint32_t)(t - 1) << sh;
                            sh = sh > 7 ? sh - 7 : 0;
                        } else {
                            base += 126u << sh;   // only while sh = 0: coarse buckets cover every PED
                        }
                    }
                    hint = TOP - 1;
                }
                T = base + (uint32_t)t - 1u;
                tT = t;
            }

            // ---------------- survivors in generation order
            uint64_t keepm[S], eqm[S];
            bool keepd[S], eqd[S];
            int eqc[S];
            uint32_t lt_l = 0u;
            const uint32_t uT = (uint32_t)tT;
            // bit j set iff byte j <= t, for C = (t * 0x01010101) | 0x80808080
            // (t <= 126): the flag bits of byte b of word g (as in the
            // probes) are gathered by byte dot products with the weights 2^b
            // (even g) and 2^(4+b) (odd g) into 128 x the mask byte of words
            // g, g + 1; words past the last group hold 127s and give none
            auto byte_mask = [&](int h, uint32_t C) {
                uint32_t acc[8];
#pragma unroll
                for (int q = 0; q < 8; ++q) {
                    acc[q] = 0u;
                    if (2 * q < ngroups) {
                        acc[q] = __builtin_amdgcn_udot4((C - pk[h][2 * q + 1]) & 0x80808080u, 0x80402010u, 0u, false);
                        acc[q] = __builtin_amdgcn_udot4((C - pk[h][2 * q]) & 0x80808080u, 0x08040201u, acc[q], false);
                    }
                }
                const uint32_t lo = (acc[0] >> 7) | (acc[1] << 1) | (acc[2] << 9) | (acc[3] << 17);
                const uint32_t hi = (acc[4] >> 7) | (acc[5] << 1) | (acc[6] << 9) | (acc[7] << 17);
                return u64(lo, hi);
            };
#pragma unroll
            for (int h = 0; h < S; ++h) {
                // bit j of ltm / lem: child j below / at most T
                uint64_t ltm = 0ull, lem = 0ull;
                if (trim) {
                    lem = byte_mask(h, (uT * 0x01010101u) | 0x80808080u);
                    ltm = byte_mask(h, ((uT - 1u) * 0x01010101u) | 0x80808080u);
                } else {
                    // without trimming T is not set: every valid child survives
                    const uint64_t all = nfree[h] >= 64 ? ~0ull : ((1ull << nfree[h]) - 1ull);
                    ltm = live[h] ? all : 0ull;
                    lem = ltm;
                }
                eqm[h] = trim ? (lem & ~ltm) : 0ull;
                const bool ltd = trim ? cdel[h] < T : live[h];
                eqd[h] = trim && cdel[h] == T;
                keepm[h] = ltm;
                keepd[h] = ltd;
                lt_l += popc64(ltm) + (ltd ? 1u : 0u);
                eqc[h] = (int)popc64(eqm[h]) + (eqd[h] ? 1 : 0);
            }
            int eq_l = 0;
#pragma unroll
            for (int h = 0; h < S; ++h) eq_l += eqc[h];
            // one scan of (below, ties) per lane in 16-bit halves (sums <=
            // 64 * 130): the children below T in earlier lanes, the ties in
            // earlier lanes, and from the last lane the wave's total below T
            const int own = (int)lt_l | (eq_l << 16);
            const int exs = wave_excl_scan(own);
            const int tot_lt = __builtin_amdgcn_readlane(exs + own, 63) & 0xffff;
            // quota > 0 under trim: fewer than K children lie below T
            const int quota = trim ? K - tot_lt : 0;
            const int ex_eq = (int)((uint32_t)exs >> 16);
            int ex = ex_eq;
#pragma unroll
            for (int h = 0; h < S; ++h) {
                int r = min(max(quota - ex, 0), eqc[h]);
                ex += eqc[h];
                const int ne = (int)popc64(eqm[h]);
                if (r >= ne) {
                    keepm[h] |= eqm[h];
                    r -= ne;
                } else {
                    for (uint64_t e = eqm[h]; r > 0; e &= e - 1ull, --r) keepm[h] |= e & (0ull - e);
                }
                if (r > 0 && eqd[h]) keepd[h] = true;
            }
            // earlier lanes keep all their children below T and the ties up
            // to the quota, in lane order
            int pos = (exs & 0xffff) + min(quota, ex_eq);
#pragma unroll
            for (int h = 0; h < S; ++h) {
                const uint32_t slot = (uint32_t)(S * lane + h);
                for (uint64_t mk = keepm[h]; mk; mk &= mk - 1ull)
                    s_sel[pos++] = (slot << 8) | (uint32_t)__builtin_ctzll(mk);
                if (keepd[h]) s_sel[pos++] = (slot << 8) | DEL8;
            }
            nb_new = min(V, K);
            }
            const int wl = i >> 2;
            if constexpr (S > 1) {
                // every slot's mapping words up to word wl (the first 16), PED,
                // edge count and Img for the update
#pragma unroll
                for (int w = 0; w < 16; ++w)
                    if (w <= wl) *reinterpret_cast<uint2 *>(&s_aux[w * NS + S * lane]) = make_uint2(ph[0][w], ph[S - 1][w]);
                *reinterpret_cast<uint2 *>(&s_aux[16 * NS + S * lane]) = make_uint2(ped[0], ped[S - 1]);
                *reinterpret_cast<uint2 *>(&s_aux[17 * NS + S * lane]) = make_uint2(ein[0], ein[S - 1]);
                *reinterpret_cast<uint2 *>(&s_aux[18 * NS + S * lane]) =
                    make_uint2((uint32_t)img[0], (uint32_t)img[S - 1]);
                *reinterpret_cast<uint2 *>(&s_aux[19 * NS + S * lane]) =
                    make_uint2((uint32_t)(img[0] >> 32), (uint32_t)(img[S - 1] >> 32));
            }
            __syncthreads();

            // ---------------- update: child = parent + (v_i -> u)
            const uint32_t sh8 = (uint32_t)(i & 3) * 8u;
            if constexpr (S == 1) {
                const bool live2 = lane < nb_new;
                const uint32_t sel = live2 ? s_sel[lane] : 0u;
                const int p = (int)(sel >> 8);
                const uint32_t jc = sel & 0xffu;
                const bool sub = jc != DEL8;
                const uint32_t u = sub ? __builtin_amdgcn_ubfe(s_aux[((jc >> 2) & 15u) * 64 + p], (jc & 3u) * 8u, 8u)
                                       : DEL8;
                const uint32_t us = sub ? min(u, 64u) : 0u;
                const uint32_t basel_p = (uint32_t)__shfl((int)basel[0], p);
                const uint64_t phi_p = shfl64(phi[0], p);
                const uint64_t ai_p = shfl64(ai[0], p);
                const uint64_t img_p = shfl64(img[0], p);
                const uint32_t ein_p = (uint32_t)__shfl((int)ein[0], p);
                const uint4 tu = s_tab[us];
                const uint64_t R = u64(tu.x, tu.y);
                uint64_t phbp[PLA], rp[PLA];
#pragma unroll
                for (int b = 0; b < PLA; ++b) {
                    phbp[b] = PL > 0 ? shfl64(phib[0][b], p) : 0ull;
                    const uint2 pl = PL > 0 ? s_pl[b][us] : make_uint2(0u, 0u);
                    rp[b] = u64(pl.x, pl.y);
                }
#pragma unroll
                for (int w = 0; w < M; ++w)
                    if (w <= wl) ph[0][w] = (uint32_t)__shfl((int)ph[0][w], p);
                if (live2) {
                    if (sub) {
                        uint32_t d = msub_cost<SMALL>(popc64(phi_p & R), nedel,
                                                      mad_cost<SMALL>(popc64(ai_p & R), eins, basel_p + tu.z));
                        if (PL > 0) {
                            uint64_t diff = 0ull;
#pragma unroll
                            for (int b = 0; b < PLA; ++b) diff |= phbp[b] ^ rp[b];
                            d += mul_cost<SMALL>(popc64(phi_p & R & diff), esub);
                        }
                        ped[0] = d;
                        img[0] = img_p | (1ull << (us & 63u)) | (DIR ? (1ull << ((us + 32u) & 63u)) : 0ull);
                        ein[0] = ein_p + popc64(img_p & R);
                    } else {
                        ped[0] = basel_p + vdel;
                        img[0] = img_p;
                        ein[0] = ein_p;
                    }
                }
                // byte i of the mapping
#pragma unroll
                for (int w = 0; w < M; ++w)
                    if (w == wl) ph[0][w] = (ph[0][w] & ~(0xffu << sh8)) | (u << sh8);
            } else {
                // the new slots' parents: first their mapping words 0..15 (read
                // straight into the slot's words, whose old values are in LDS
                // already), PED, edge count and Img; a 32-word mapping's upper
                // half then goes through the same LDS rows in a second round
                int pp[S];
                uint32_t jcs[S], ped_ps[S], ein_ps[S];
                uint64_t img_ps[S];
#pragma unroll
                for (int h = 0; h < S; ++h) {
                    const bool live2 = S * lane + h < nb_new;
                    const uint32_t sel = live2 ? s_sel[S * lane + h] : 0u;
                    pp[h] = (int)(sel >> 8);
                    jcs[h] = sel & 0xffu;
                    ped_ps[h] = s_aux[16 * NS + pp[h]];
                    ein_ps[h] = s_aux[17 * NS + pp[h]];
                    img_ps[h] = u64(s_aux[18 * NS + pp[h]], s_aux[19 * NS + pp[h]]);
#pragma unroll
                    for (int w = 0; w < 16; ++w) ph[h][w] = w <= wl ? s_aux[w * NS + pp[h]] : 0u;
                }
                if constexpr (M > 16) {
                    if (wl >= 16) {
                        __syncthreads();   // every read of the first half is done
#pragma unroll
                        for (int w = 0; w < 16; ++w)
                            if (16 + w <= wl)
                                *reinterpret_cast<uint2 *>(&s_aux[w * NS + S * lane]) =
                                    make_uint2(ph[0][16 + w], ph[S - 1][16 + w]);
                        __syncthreads();
#pragma unroll
                        for (int h = 0; h < S; ++h) {
#pragma unroll
                            for (int w = 0; w < 16; ++w) ph[h][16 + w] = 16 + w <= wl ? s_aux[w * NS + pp[h]] : 0u;
                        }
                    }
                }
#pragma unroll
                for (int h = 0; h < S; ++h) {
                    const bool live2 = S * lane + h < nb_new;
                    const bool sub = jcs[h] != DEL8;
                    const uint64_t img_p = img_ps[h];
                    // the parent's j-th free vertex (a survivor is never an exhausted child)
                    const uint32_t u = sub ? nth_bit64(~img_p & umask, jcs[h]) : DEL8;
                    const uint32_t us = sub ? min(u, 64u) : 0u;
                    // ph[h] holds the parent's mapping (byte i not yet set)
                    uint64_t phi_p, phbp[PLA];
                    build_phi(ph[h], phi_p, phbp);
                    const uint64_t ai_p = img_p & ~phi_p;
                    const uint32_t basel_p = ped_ps[h] + edP;
                    const uint4 tu = s_tab[us];
                    const uint64_t R = u64(tu.x, tu.y);
                    if (live2) {
                        if (sub) {
                            uint32_t d = msub_cost<SMALL>(popc64(phi_p & R), nedel,
                                                          mad_cost<SMALL>(popc64(ai_p & R), eins, basel_p + tu.z));
                            if (PL > 0) {
                                uint64_t diff = 0ull;
#pragma unroll
                                for (int b = 0; b < PLA; ++b) {
                                    const uint2 pl = s_pl[b][us];
                                    diff |= phbp[b] ^ u64(pl.x, pl.y);
                                }
                                d += mul_cost<SMALL>(popc64(phi_p & R & diff), esub);
                            }
                            ped[h] = d;
                            img[h] = img_p | (1ull << (us & 63u)) | (DIR ? (1ull << ((us + 32u) & 63u)) : 0ull);
                            ein[h] = ein_ps[h] + popc64(img_p & R);
                        } else {
                            ped[h] = basel_p + vdel;
                            img[h] = img_p;
                            ein[h] = ein_ps[h];
                        }
                    }
#pragma unroll
                    for (int w = 0; w < M; ++w)
                        if (w == wl) ph[h][w] = (ph[h][w] & ~(0xffu << sh8)) | (u << sh8);
                }
            }
            nb = nb_new;
        }

        // ---------------- completion and best leaf
        uint32_t tot[S], tmin = INVALID;
#pragma unroll
        for (int h = 0; h < S; ++h) {
            const uint32_t nimg = DIR ? (uint32_t)__popc((uint32_t)img[h]) : popc64(img[h]);
            tot[h] = S * lane + h < nb ? ped[h] + mul_cost<SMALL>((uint32_t)n2 - nimg, vins) +
                                             mul_cost<SMALL>((uint32_t)g2.m - ein[h], eins)
                                       : INVALID;
            tmin = min(tmin, tot[h]);
        }
        const uint32_t best_total = wave_umin(tmin);
        const uint32_t ce_total = wave_sum(ce);
        const int best = (int)__builtin_ctzll(__ballot(tmin == best_total));
        // the slot of the best lane that holds it (the first one)
        const int hb = S == 1 ? 0 : __builtin_amdgcn_readlane(tot[0] == best_total ? 0 : 1, best);
        if (lane == 0) {
            a.out.dist[wi.out] = (int)best_total;
            if (a.out.cand) a.out.cand[wi.out] = (long long)ce_total;
        }
        // lane v writes the images of source vertices v and v + 64
#pragma unroll
        for (int half = 0; half < M / 16; ++half) {
            uint32_t word = 0u;
#pragma unroll
            for (int w = 0; w < 16; ++w) {
                const uint32_t v = hb == 0 ? ph[0][16 * half + w] : ph[S - 1][16 * half + w];
                const uint32_t bw = (uint32_t)__builtin_amdgcn_readlane((int)v, best);
                word = (lane >> 2) == w ? bw : word;
            }
            const int v1 = 64 * half + lane;
            if (v1 < n1) {
                const uint32_t x = __builtin_amdgcn_ubfe(word, (uint32_t)(lane & 3) * 8u, 8u);
                a.out.map[wi.map_off + v1] = (x == DEL8) ? -1 : (int)x;
            }
        }
        __syncthreads();
    }
}

template <int S, int M, int PL, bool SMALL, bool COMPLETE, bool DIR>
const void *wave2_ptr() {
    return reinterpret_cast<const void *>(&kb_wave2_kernel<S, M, PL, SMALL, COMPLETE, DIR>);
}

// the complete-then-minimum last level is a kernel of its own, so that the
// default search keeps its register budget; so are directed pairs
template <int S, int M, bool COMPLETE, bool DIR>
const void *select_wave2_c(int PL, bool small) {
    if (PL == 0) return small ? wave2_ptr<S, M, 0, true, COMPLETE, DIR>() : wave2_ptr<S, M, 0, false, COMPLETE, DIR>();
    if (PL == 2) return small ? wave2_ptr<S, M, 2, true, COMPLETE, DIR>() : wave2_ptr<S, M, 2, false, COMPLETE, DIR>();
    if (PL == 4) return small ? wave2_ptr<S, M, 4, true, COMPLETE, DIR>() : wave2_ptr<S, M, 4, false, COMPLETE, DIR>();
    return nullptr;
}

template <int S>
const void *select_wave2_s(int PL, bool small, bool complete, bool dir) {
    if (dir) return complete ? select_wave2_c<S, 16, true, true>(PL, small) : select_wave2_c<S, 16, false, true>(PL, small);
    return complete ? select_wave2_c<S, 16, true, false>(PL, small) : select_wave2_c<S, 16, false, false>(PL, small);
}

template <int S>
const void *select_wave2_wide_src(int PL, bool small, bool complete) {
    return complete ? select_wave2_c<S, 32, true, false>(PL, small) : select_wave2_c<S, 32, false, false>(PL, small);
}

}  // namespace w2

// kb_wave2_k128.hip: the two-slot instantiations (64 < K <= 128)
const void *select_wave2_two_slots(int PL, bool small, bool complete, bool dir);
// kb_wave2_src128.hip: sources of 65..128 vertices (undirected), slots = 1 or 2 per lane
const void *select_wave2_wide_source(int slots, int PL, bool small, bool complete);

}  // namespace gedk
