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
//            the deletion child costs PED + vdel + edel |P|; used u -> SENT.
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
#include "ged_internal.h"

namespace gedk {
namespace {

constexpr int SENT = 0x7fffffff;
constexpr uint32_t DEL8 = 0xffu;

struct WaveArgs {
    DbView db;
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
__device__ __forceinline__ int dpp_ror(int v) {
    return __builtin_amdgcn_update_dpp(0, v, CTRL, 0xf, 0xf, false);
}

__device__ __forceinline__ int wave_sum(int v) {
    v += dpp_ror<0x121>(v);
    v += dpp_ror<0x122>(v);
    v += dpp_ror<0x124>(v);
    v += dpp_ror<0x128>(v);
    return __builtin_amdgcn_readlane(v, 0) + __builtin_amdgcn_readlane(v, 16) +
           __builtin_amdgcn_readlane(v, 32) + __builtin_amdgcn_readlane(v, 48);
}

__device__ __forceinline__ int wave_min(int v) {
    v = min(v, dpp_ror<0x121>(v));
    v = min(v, dpp_ror<0x122>(v));
    v = min(v, dpp_ror<0x124>(v));
    v = min(v, dpp_ror<0x128>(v));
    return min(min(__builtin_amdgcn_readlane(v, 0), __builtin_amdgcn_readlane(v, 16)),
               min(__builtin_amdgcn_readlane(v, 32), __builtin_amdgcn_readlane(v, 48)));
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

template <int PL>
__global__ __launch_bounds__(64) void kb_wave_kernel(WaveArgs a) {
    constexpr int PLA = PL > 0 ? PL : 1;
    __shared__ uint32_t s_phi[2][8 * 64];   // [half][word j/4][slot]: bytes of phi
    __shared__ uint32_t s_sel[64];          // survivor: parent slot << 8 | u (0xff = deletion)
    __shared__ int s_item;

    const int lane = threadIdx.x;
    const Costs c = a.c;
    const int K = a.K;
    const int P = a.db.planes;

    for (;;) {
        if (lane == 0) s_item = atomicAdd(a.queue, 1);
        __syncthreads();
        const int item = __builtin_amdgcn_readfirstlane(s_item);
        __syncthreads();
        if (item >= a.nwork) break;

        const WorkItem wi = a.work[item];
        const GraphRec g1 = a.db.graphs[wi.src];
        const GraphRec g2 = a.db.graphs[wi.dst];
        const int n1 = g1.n, n2 = g2.n;
        const uint32_t *A1 = a.db.adj + g1.adj;
        const uint32_t *A2 = a.db.adj + g2.adj;
        const uint32_t r1 = lane < n1 ? A1[lane] : 0u;
        const uint32_t r2 = lane < n2 ? A2[lane] : 0u;
        const int l1 = lane < n1 ? a.db.vlab[g1.vlab + lane] : 0;
        const int l2 = lane < n2 ? a.db.vlab[g2.vlab + lane] : 0;
        uint32_t p1[PLA], p2[PLA];
#pragma unroll
        for (int b = 0; b < PLA; ++b) {
            p1[b] = (PL > 0 && b < P && lane < n1) ? A1[(size_t)(1 + b) * n1 + lane] : 0u;
            p2[b] = (PL > 0 && b < P && lane < n2) ? A2[(size_t)(1 + b) * n2 + lane] : 0u;
        }
        const uint32_t umask = n2 >= 32 ? 0xffffffffu : ((1u << n2) - 1u);

        int ped = 0, ein = 0;
        uint32_t img = 0u;
        int nb = 1, cur = 0;
        long long ce = 0;

        for (int i = 0; i < n1; ++i) {
            const uint32_t nbm = (uint32_t)__builtin_amdgcn_readlane((int)r1, i) & ((1u << i) - 1u);
            const int lab1 = __builtin_amdgcn_readlane(l1, i);
            const int degP = __popc(nbm);
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
            const int base = ped + c.edel * degP;
            const int kc = c.edel + c.eins;
            int cand[32];
            int lmin = SENT;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                cand[u] = SENT;
                if (u < n2) {
                    const uint32_t R = (uint32_t)__builtin_amdgcn_readlane((int)r2, u);
                    const int vs = ((vsm >> u) & 1u) ? c.vsub : 0;
                    const uint32_t kp = phi & R;
                    int d = base + vs + c.eins * __popc(img & R) - kc * __popc(kp);
                    if (PL > 0) {
                        uint32_t diff = 0u;
#pragma unroll
                        for (int b = 0; b < PLA; ++b)
                            diff |= phib[b] ^ (uint32_t)__builtin_amdgcn_readlane((int)p2[b], u);
                        d += c.esub * __popc(kp & diff);
                    }
                    d = (live && !((img >> u) & 1u)) ? d : SENT;
                    cand[u] = d;
                    lmin = min(lmin, d);
                }
            }
            const int cdel = live ? ped + c.vdel + c.edel * degP : SENT;
            lmin = min(lmin, cdel);
            const int V = wave_sum(live ? n2 - __popc(img) + 1 : 0);
            ce += V;

            // ---------------- threshold T: the K-th smallest PED
            int T = SENT;
            const bool trim = V > K;
            if (trim) {
                auto count_le = [&](int t) {
                    int cnt = __popcll(__ballot(cdel <= t));
#pragma unroll
                    for (int u = 0; u < 32; ++u)
                        if (u < n2) cnt += __popcll(__ballot(cand[u] <= t));
                    return cnt;
                };
                int lo = wave_min(lmin), t = lo, step = 1, hi;
                for (;;) {
                    if (count_le(t) >= K) {
                        hi = t;
                        break;
                    }
                    lo = t + 1;
                    // count_le(SENT - 1) = V > K, so the walk stops by then
                    t = (t > SENT - 1 - step) ? SENT - 1 : t + step;
                    step = step < (1 << 29) ? step << 1 : step;
                }
                while (lo < hi) {
                    const int mid = lo + ((hi - lo) >> 1);
                    if (count_le(mid) >= K) hi = mid;
                    else lo = mid + 1;
                }
                T = lo;
            }

            // ---------------- survivors in generation order
            uint32_t ltm = 0u, eqm = 0u;
#pragma unroll
            for (int u = 0; u < 32; ++u) {
                if (u < n2) {
                    ltm |= (cand[u] < T) ? (1u << u) : 0u;
                    eqm |= (trim && cand[u] == T) ? (1u << u) : 0u;
                }
            }
            const bool ltd = cdel < T;
            const bool eqd = trim && cdel == T;
            const int lt_l = __popc(ltm) + (ltd ? 1 : 0);
            const int eq_l = __popc(eqm) + (eqd ? 1 : 0);
            const int quota = trim ? K - wave_sum(lt_l) : 0;
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
            const int ped_p = __shfl(ped, p);
            const uint32_t img_p = (uint32_t)__shfl((int)img, p);
            const int ein_p = __shfl(ein, p);
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
                if (sub) {
                    const uint32_t kp = php & R;
                    const int inimg = __popc(img_p & R);
                    int d = ped_p + c.edel * degP + (lab1 != lab2u ? c.vsub : 0) + c.eins * inimg - kc * __popc(kp);
                    if (PL > 0) {
                        uint32_t diff = 0u;
#pragma unroll
                        for (int b = 0; b < PLA; ++b) diff |= phbp[b] ^ rp[b];
                        d += c.esub * __popc(kp & diff);
                    }
                    ped = d;
                    img = img_p | (1u << u);
                    ein = ein_p + inimg;
                } else {
                    ped = ped_p + c.vdel + c.edel * degP;
                    img = img_p;
                    ein = ein_p;
                }
            }
            __syncthreads();
            cur = nxt;
            nb = nb_new;
        }

        // ---------------- completion and best leaf
        const int total = lane < nb ? ped + c.vins * (n2 - __popc(img)) + c.eins * (g2.m - ein) : SENT;
        const int best_total = wave_min(total);
        const int best = (int)__builtin_ctzll(__ballot(total == best_total));
        if (lane == 0) {
            a.out.dist[wi.out] = best_total;
            if (a.out.cand) a.out.cand[wi.out] = ce;
        }
        if (lane < n1) {
            const uint32_t x = phi_byte(s_phi[cur], lane, best);
            a.out.map[wi.map_off + lane] = (x == DEL8) ? -1 : (int)x;
        }
        __syncthreads();
    }
}

template <int PL>
const void *wave_ptr() {
    return reinterpret_cast<const void *>(&kb_wave_kernel<PL>);
}

const void *select_wave(int PL) {
    if (PL == 0) return wave_ptr<0>();
    if (PL == 2) return wave_ptr<2>();
    if (PL == 4) return wave_ptr<4>();
    return nullptr;
}

}  // namespace

hipError_t wave_max_resident(int PL, int *blocks_per_cu) {
    const void *k = select_wave(PL);
    if (!k) return hipErrorInvalidValue;
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, k, 64, 0);
}

hipError_t launch_wave(int PL, const DbView &db, const WorkItem *work, int nwork, int *queue, Costs c,
                       int K, Outputs out, int grid, hipStream_t stream) {
    const void *k = select_wave(PL);
    if (!k || grid <= 0 || K > kWaveMaxK) return hipErrorInvalidValue;
    WaveArgs a;
    a.db = db;
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
