// Device helpers shared by the wavefront-per-pair kernels (kb_wave.hip,
// kb_wave2.hip): wave-wide reductions and scans on DPP, the carry-chain mask
// builder, and the cost multiply-adds.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>

namespace gedk {
namespace wv {

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

__device__ __forceinline__ uint32_t wave_umax(uint32_t v) {
    v = max(v, dpp_ror<0x121>(v));
    v = max(v, dpp_ror<0x122>(v));
    v = max(v, dpp_ror<0x124>(v));
    v = max(v, dpp_ror<0x128>(v));
    const uint32_t a = max((uint32_t)__builtin_amdgcn_readlane((int)v, 0), (uint32_t)__builtin_amdgcn_readlane((int)v, 16));
    const uint32_t b = max((uint32_t)__builtin_amdgcn_readlane((int)v, 32), (uint32_t)__builtin_amdgcn_readlane((int)v, 48));
    return max(a, b);
}

// DPP move with out-of-row sources and rows outside ROWS reading 0.
template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_zero(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWS, 0xf, true);
}

// Exclusive prefix sum over lanes: shifted adds inside each 16-lane row,
// then the last lane of row 0 (row 2) is broadcast into row 1 (row 3), and
// the last lane of row 1 into rows 2 and 3.
__device__ __forceinline__ int wave_excl_scan(int v) {
    uint32_t x = (uint32_t)v;
    x += dpp_zero<0x111, 0xf>(x);   // row_shr:1
    x += dpp_zero<0x112, 0xf>(x);   // row_shr:2
    x += dpp_zero<0x114, 0xf>(x);   // row_shr:4
    x += dpp_zero<0x118, 0xf>(x);   // row_shr:8
    x += dpp_zero<0x142, 0xa>(x);   // row_bcast:15
    x += dpp_zero<0x143, 0xc>(x);   // row_bcast:31
    return (int)x - v;
}

// m1 = 2 m1 + [c1], m2 = 2 m2 + [c2]: each condition's wave mask (one
// compare into a scalar pair) is the carry-in of one add; both compares are
// issued before the adds
__device__ __forceinline__ void shift_in2(uint32_t &m1, bool c1, uint32_t &m2, bool c2) {
    const unsigned long long b1 = __ballot(c1);
    const unsigned long long b2 = __ballot(c2);
    uint32_t r1, r2;
    unsigned long long co1, co2;
    asm("v_addc_co_u32 %0, %2, %4, %4, %6\n\tv_addc_co_u32 %1, %3, %5, %5, %7"
        : "=&v"(r1), "=&v"(r2), "=&s"(co1), "=&s"(co2)
        : "v"(m1), "v"(m2), "s"(b1), "s"(b2));
    m1 = r1;
    m2 = r2;
}

template <bool SMALL>
__device__ __forceinline__ uint32_t mul_cost(uint32_t count, uint32_t cost) {
    return SMALL ? __umul24(count, cost) : count * cost;
}

// count * cost + acc (one v_mad_u32_u24 under SMALL)
template <bool SMALL>
__device__ __forceinline__ uint32_t mad_cost(uint32_t count, uint32_t cost, uint32_t acc) {
    if (SMALL) {
        uint32_t r;
        asm("v_mad_u32_u24 %0, %1, %2, %3" : "=v"(r) : "v"(count), "s"(cost), "v"(acc));
        return r;
    }
    return count * cost + acc;
}

// acc - count * cost (one v_mad_i32_i24 with the negated cost under SMALL;
// modulo 2^32)
template <bool SMALL>
__device__ __forceinline__ uint32_t msub_cost(uint32_t count, uint32_t neg_cost, uint32_t acc) {
    if (SMALL) {
        uint32_t r;
        asm("v_mad_i32_i24 %0, %1, %2, %3" : "=v"(r) : "v"(count), "s"(neg_cost), "v"(acc));
        return r;
    }
    return count * neg_cost + acc;
}

// Index of the lowest set bit, 0xffffffff for 0 (the hardware's find-first-
// bit, whose result for an empty word the compiler does not model).
__device__ __forceinline__ uint32_t find_low(uint32_t x) {
    uint32_t r;
    asm("v_ffbl_b32 %0, %1" : "=v"(r) : "v"(x));
    return r;
}

__device__ __forceinline__ uint32_t pack4(uint32_t e0, uint32_t e1, uint32_t e2, uint32_t e3) {
    return e0 | (e1 << 8) | (e2 << 16) | (e3 << 24);
}


}  // namespace wv
}  // namespace gedk
