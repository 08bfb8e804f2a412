// kb_wave.hip -- wavefront-per-pair K-Best search for small pairs on gfx950.
//
// Handles pairs with n1 <= 32, n2 <= 32 and K <= 64: one 64-lane wavefront
// owns one pair for all its levels and pulls the next pair from a work queue
// (persistent launch, one wave per workgroup so a barrier is one s_barrier).
// Lane s holds beam slot s in registers: partial edit distance, the image
// Img (one 32-bit word: bit u set iff g2 vertex u is used) and e_in (g2
// edges inside Img).  Lane u also holds g2's adjacency row N2(u), its label
// and its label-plane rows, and lane v holds g1's row N1(v).  The mapping
// phi of each slot lives in LDS, one byte per g1 vertex (0xff = deleted).
//
// Per level i (Alg. 1), with P = earlier neighbours of v_i:
//   expand   Phi = {phi(j) : j in P, not deleted}; for every g2 vertex u
//            (a compile-time unrolled loop; N2(u) broadcast from lane u):
//              PED' = PED + [alpha1(v_i) != alpha2(u)] vsub + edel (|P| - kept)
//                     + eins (|Img & N2(u)| - kept) + esub relabelled,
//              kept = |Phi & N2(u)|  (implied edge operations, Sec. 2.3);
//            the deletion child costs PED + vdel + edel |P|.  Children held
//            as unsigned values; an invalid child (u used, u >= n2, or an
//            empty slot) is 0xffffffff, obtained by OR-ing the sign-extended
//            bit u of (Img | invalid-u mask).
//   select   T = K-th smallest PED by counting probes: count(PED <= t) is a
//            sum of popcounts of wave ballots, galloping then bisection from
//            the wave minimum.  Every child below T survives and the first
//            (K - #below) children equal to T in generation order (lane
//            order, then u, then the deletion), via per-lane bit masks and
//            ballot/mbcnt exclusive scans; survivor (parent, u) pairs are
//            written to LDS in generation order.
//   update   new slot s reads its (parent, u), copies the parent's phi
//            words, fetches the parent's registers with ds_bpermute and
//            recomputes the child's PED from the parent (the same integer
//            formula, so the value is identical to the candidate's).
// Completion adds vins (n2 - |Img|) + eins (m2 - e_in) (Sec. 4.4.1); the
// first lane of least total is the result.
//
// SMALL selects 24-bit multiply-adds, valid when every cost is below 2^22
// (counts are at most 32, and the plan's overflow bound keeps every sum in
// range); otherwise full 32-bit multiplies.
#include "ged_internal.h"

namespace gedk {
namespace {

constexpr uint32_t INVALID = 0xffffffffu;
constexpr uint32_t DEL8 = 0xffu;

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

// DPP row rotations (row_ror:k) reduce inside each 16-lane row; the four
// row results are combined with readlane.
template <int CTRL>
__device__ __forceinline__ uint32_t dpp_ror(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v) {
    v += dpp_ror<0x121>(v);
    v += dpp_ror<0x122>(v);
    v += dpp_ror<0x124>(v);
    v += dpp_ror<0x128>(v);
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 0) + (uint32_t)__builtin_amdgcn_readlane((int)v, 16) +
           (uint32_t)__builtin_amdgcn_readlane((int)v, 32) + (uint32_t)__builtin_amdgcn_readlane((int)v, 48);
}

__device__ __forceinline__ uint32_t wave_umin(uint32_t v) {
    v = min(v, dpp_ror<0x121>(v));
    v = min(v, dpp_ror<0x122>(v));
    v = min(v, dpp_ror<0x124>(v));
    v = min(v, dpp_ror<0x128>(v));
    const uint32_t a = min((uint32_t)__builtin_amdgcn_readlane((int)v, 0), (uint32_t)__builtin_amdgcn_readlane((int)v, 16));
    const uint32_t b = min((uint32_t)__builtin_amdgcn_readlane((int)v, 32), (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
    return min(a, b);
}

__device__ __forceinline__ int lanes_below(unsigned long long m) {
    return (int)__builtin_amdgcn_mbcnt_hi((unsigned)(m >> 32), __builtin_amdgcn_mbcnt_lo((unsigned)m, 0u));
}

// Exclusive prefix sum over lanes of v in [0, 63], bit-sliced with ballots.
__device__ __forceinline__ int wave_excl_scan6(int v) {
    int r = 0;
#pragma unroll
    for (int b = 0; b < 6; ++b) r += lanes_below(__ballot((v >> b) & 1)) << b;
    return r;
}

__device__ __forceinline__ uint32_t phi_byte(const uint32_t *plane, int j, int slot) {
    return (plane[(j >> 2) * 64 + slot] >> ((j & 3) * 8)) & 0xffu;
}

// bit u of m, sign-extended: 0 or 0xffffffff
__device__ __forceinline__ uint32_t bit_mask(uint32_t m, int u) {
    return (uint32_t)__builtin_amdgcn_sbfe((int)m, u, 1);
}

template <bool SMALL>
__device__ __forceinline__ uint32_t mul_cost(uint32_t count, uint32_t cost) {
    return SMALL ? __umul24(count, cost) : count * cost;
}

template <int PL, bool SMALL>
__global__ __launch_bounds__(64) void kb_wave_kernel(WaveArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    __shared__ uint32_t s_phi[2][8 * 64];   // [half][word j/4][slot]: bytes of phi
    __shared__ uint32_t s_sel[64];          // survivor: parent slot << 8 | u (0xff = deletion)
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const uint32_t vsub = (uint32_t)a.c.vsub, vdel = (uint32_t)a.c.vdel, vins = (uint32_t)a.c.vins;
    const uint32_t esub = (uint32_t)a.c.esub, edel = (uint32_t)a.c.edel, eins = (uint32_t)a.c.eins;
    const uint32_t kc = edel + eins;
    const int K = a.K;
    const int P = a.dst.planes;

    for (;;) {
        if (lane == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
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
        const int ngroups = (n2 + 3) >> 2;     // u is processed in groups of four

        uint32_t ped = 0u, img = 0u, ein = 0u;
        int nb = 1, cur = 0;
        long long ce = 0;

        for (int i = 0; i < n1; ++i) {
            const uint32_t nbm = (uint32_t)__builtin_amdgcn_readlane((int)r1, i) & ((1u << i) - 1u);
            const int lab1 = __builtin_amdgcn_readlane(l1, i);
            const uint32_t degP = (uint32_t)__popc(nbm);
            uint32_t q[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) q[b] = (uint32_t)__builtin_amdgcn_readlane((int)p1[b], i) & nbm;
            const uint32_t vsm = (uint32_t)__ballot(l2 != lab1) & umask;
            const bool live = lane < nb;
            const uint32_t *phic = s_phi[cur];

            // ---------------- expand and evaluate
            uint32_t phi = 0u, phib[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) phib[b] = 0u;
            for (uint32_t bits = nbm; bits; bits &= bits - 1u) {
                const int j = __builtin_ctz(bits);
                const uint32_t x = phi_byte(phic, j, lane);
                const uint32_t bit = (x != DEL8) ? (1u << (x & 31u)) : 0u;
                phi |= bit;
#pragma unroll
                for (int b = 0; b < PLA; ++b)
                    if (PL > 0 && ((q[b] >> j) & 1u)) phib[b] |= bit;
            }
            const uint32_t base = ped + mul_cost<SMALL>(degP, edel);
            const uint32_t blocked = live ? (img | ~umask) : 0xffffffffu;
            uint32_t cand[32];
            uint32_t lmin = INVALID;
#pragma unroll
            for (int g = 0; g < 8; ++g) {
                if (g < ngroups) {
#pragma unroll
                    for (int u = 4 * g; u < 4 * g + 4; ++u) {
                        const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)r2, u);
                        const uint32_t vs = ((vsm >> u) & 1u) ? vsub : 0u;
                        const uint32_t kp = phi & R;
                        uint32_t d = base + vs + mul_cost<SMALL>((uint32_t)__popc(img & R), eins) -
                                     mul_cost<SMALL>((uint32_t)__popc(kp), kc);
                        if (PL > 0) {
                            uint32_t diff = 0u;
#pragma unroll
                            for (int b = 0; b < PLA; ++b)
                                diff |= phib[b] ^ (uint32_t)__builtin_amdgcn_readlane((int)p2[b], u);
                            d += mul_cost<SMALL>((uint32_t)__popc(kp & diff), esub);
                        }
                        d |= bit_mask(blocked, u);
                        cand[u] = d;
                        lmin = min(lmin, d);
                    }
                } else {
#pragma unroll
                    for (int u = 4 * g; u < 4 * g + 4; ++u) cand[u] = INVALID;
                }
            }
            const uint32_t cdel = live ? base + vdel : INVALID;
            lmin = min(lmin, cdel);
            const int V = (int)wave_sum(live ? (uint32_t)(n2 - __popc(img) + 1) : 0u);
            ce += V;

            // ---------------- threshold T: the K-th smallest PED
            uint32_t T = INVALID;
            const bool trim = V > K;
            if (trim) {
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
                uint32_t lo = wave_umin(lmin), t = lo, step = 1, hi;
                for (;;) {
                    if (count_le(t) >= K) {
                        hi = t;
                        break;
                    }
                    lo = t + 1;
                    // count_le(INVALID - 1) = V > K, so the walk stops by then
                    t = (t > INVALID - 1u - step) ? INVALID - 1u : t + step;
                    step = step < (1u << 29) ? step << 1 : step;
                }
                while (lo < hi) {
                    const uint32_t mid = lo + ((hi - lo) >> 1);
                    if (count_le(mid) >= K) hi = mid;
                    else lo = mid + 1;
                }
                T = lo;
            }

            // ---------------- survivors in generation order
            // bit u of ltm / lem: child u below / at most T (built high u first)
            uint32_t ltm = 0u, lem = 0u;
#pragma unroll
            for (int g = 7; g >= 0; --g) {
                if (g < ngroups) {
#pragma unroll
                    for (int u = 4 * g + 3; u >= 4 * g; --u) {
                        ltm = ltm + ltm + (cand[u] < T ? 1u : 0u);
                        lem = lem + lem + (cand[u] <= T ? 1u : 0u);
                    }
                }
            }
            const uint32_t eqm = trim ? (lem & ~ltm) : 0u;
            const bool ltd = cdel < T;
            const bool eqd = trim && cdel == T;
            const int lt_l = __popc(ltm) + (ltd ? 1 : 0);
            const int eq_l = __popc(eqm) + (eqd ? 1 : 0);
            const int quota = trim ? K - (int)wave_sum((uint32_t)lt_l) : 0;
            int r = min(max(quota - wave_excl_scan6(eq_l), 0), eq_l);
            uint32_t keepm = ltm;
            bool keepd = ltd;
            for (uint32_t e = eqm; r > 0 && e; e &= e - 1u, --r) keepm |= e & (0u - e);
            if (r > 0 && eqd) keepd = true;
            int pos = wave_excl_scan6(__popc(keepm) + (keepd ? 1 : 0));
            for (uint32_t mk = keepm; mk; mk &= mk - 1u) s_sel[pos++] = ((uint32_t)lane << 8) | (uint32_t)__builtin_ctz(mk);
            if (keepd) s_sel[pos] = ((uint32_t)lane << 8) | DEL8;
            const int nb_new = min(V, K);
            __syncthreads();

            // ---------------- update: child = parent + (v_i -> u)
            const int nxt = cur ^ 1;
            uint32_t *phin = s_phi[nxt];
            const bool live2 = lane < nb_new;
            const uint32_t sel = live2 ? s_sel[lane] : 0u;
            const int p = (int)(sel >> 8);
            const uint32_t u = sel & 0xffu;
            const bool sub = u != DEL8;
            const int us = sub ? (int)u : 0;
            const uint32_t ped_p = (uint32_t)__shfl((int)ped, p);
            const uint32_t img_p = (uint32_t)__shfl((int)img, p);
            const uint32_t ein_p = (uint32_t)__shfl((int)ein, p);
            const uint32_t R = (uint32_t)__shfl((int)r2, us);
            const int lab2u = __shfl(l2, us);
            uint32_t rp[PLA];
#pragma unroll
            for (int b = 0; b < PLA; ++b) rp[b] = PL > 0 ? (uint32_t)__shfl((int)p2[b], us) : 0u;
            if (live2) {
                // copy the parent's phi bytes 0..i-1 and append byte i
                const int wi_last = i >> 2;
                for (int jw = 0; jw <= wi_last; ++jw) {
                    uint32_t wv = phic[jw * 64 + p];
                    if (jw == wi_last) {
                        const int sh = (i & 3) * 8;
                        wv = (wv & ((1u << sh) - 1u)) | (u << sh);
                    }
                    phin[jw * 64 + lane] = wv;
                }
                uint32_t php = 0u, phbp[PLA];
#pragma unroll
                for (int b = 0; b < PLA; ++b) phbp[b] = 0u;
                for (uint32_t bits = nbm; bits; bits &= bits - 1u) {
                    const int j = __builtin_ctz(bits);
                    const uint32_t x = phi_byte(phic, j, p);
                    const uint32_t bit = (x != DEL8) ? (1u << (x & 31u)) : 0u;
                    php |= bit;
#pragma unroll
                    for (int b = 0; b < PLA; ++b)
                        if (PL > 0 && ((q[b] >> j) & 1u)) phbp[b] |= bit;
                }
                const uint32_t pbase = ped_p + mul_cost<SMALL>(degP, edel);
                if (sub) {
                    const uint32_t kp = php & R;
                    const uint32_t inimg = (uint32_t)__popc(img_p & R);
                    uint32_t d = pbase + (lab1 != lab2u ? vsub : 0u) + mul_cost<SMALL>(inimg, eins) -
                                 mul_cost<SMALL>((uint32_t)__popc(kp), kc);
                    if (PL > 0) {
                        uint32_t diff = 0u;
#pragma unroll
                        for (int b = 0; b < PLA; ++b) diff |= phbp[b] ^ rp[b];
                        d += mul_cost<SMALL>((uint32_t)__popc(kp & diff), esub);
                    }
                    ped = d;
                    img = img_p | (1u << u);
                    ein = ein_p + inimg;
                } else {
                    ped = pbase + vdel;
                    img = img_p;
                    ein = ein_p;
                }
            }
            __syncthreads();
            cur = nxt;
            nb = nb_new;
        }

        // ---------------- completion and best leaf
        const uint32_t total = lane < nb ? ped + mul_cost<SMALL>((uint32_t)(n2 - __popc(img)), vins) +
                                               mul_cost<SMALL>((uint32_t)g2.m - ein, eins)
                                         : INVALID;
        const uint32_t best_total = wave_umin(total);
        const int best = (int)__builtin_ctzll(__ballot(total == best_total));
        if (lane == 0) {
            a.out.dist[wi.out] = (int)best_total;
            if (a.out.cand) a.out.cand[wi.out] = ce;
        }
        if (lane < n1) {
            const uint32_t x = phi_byte(s_phi[cur], lane, best);
            a.out.map[wi.map_off + lane] = (x == DEL8) ? -1 : (int)x;
        }
        __syncthreads();
    }
}

template <int PL, bool SMALL>
const void *wave_ptr() {
    return reinterpret_cast<const void *>(&kb_wave_kernel<PL, SMALL>);
}

const void *select_wave(int PL, bool small) {
    if (PL == 0) return small ? wave_ptr<0, true>() : wave_ptr<0, false>();
    if (PL == 2) return small ? wave_ptr<2, true>() : wave_ptr<2, false>();
    if (PL == 4) return small ? wave_ptr<4, true>() : wave_ptr<4, false>();
    return nullptr;
}

bool small_costs(const Costs &c) {
    const int32_t lim = 1 << 22;
    return c.vsub < lim && c.vdel < lim && c.vins < lim && c.esub < lim && c.edel < lim && c.eins < lim;
}

}  // namespace

hipError_t wave_max_resident(int PL, int *blocks_per_cu) {
    const void *k = select_wave(PL, true);
    const void *k2 = select_wave(PL, false);
    if (!k || !k2) return hipErrorInvalidValue;
    int a = 0, b = 0;
    hipError_t e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&a, k, 64, 0);
    if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&b, k2, 64, 0);
    *blocks_per_cu = a < b ? a : b;
    return e;
}

hipError_t launch_wave(int PL, const DbView &src, const DbView &dst, const WorkItem *work, int nwork, int *queue, Costs c,
                       int K, Outputs out, int grid, hipStream_t stream) {
    const void *k = select_wave(PL, small_costs(c));
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
