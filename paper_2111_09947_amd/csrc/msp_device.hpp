// Device-side building blocks for the masked SpGEMM kernels (gfx950, wave64).
//
// - wave-level primitives (ballot rank, shuffle scans) used by the row
//   streams and the ordered emission,
// - semiring traits: how a product a (x) b is formed and how it is folded
//   into an LDS accumulator slot with a single atomic where possible,
// - small binary searches over sorted CSR rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "msp.h"

namespace mspk {

constexpr int WAVE = 64;

__device__ __forceinline__ int lane() { return (int)__lane_id(); }

// Number of set bits of `m` below the calling lane.
__device__ __forceinline__ int rank_below(uint64_t m) {
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
}

// Orders LDS accesses of one wavefront: LDS operations of a wave execute in
// issue order, so a compiler barrier plus a wave scheduling barrier is what a
// lane needs before reading what another lane of its wave wrote.
__device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    __builtin_amdgcn_wave_barrier();
}

__device__ __forceinline__ int64_t wave_incl_scan(int64_t v) {
    const int l = lane();
#pragma unroll
    for (int d = 1; d < WAVE; d <<= 1) {
        const int64_t t = __shfl_up(v, d, WAVE);
        if (l >= d) v += t;
    }
    return v;
}

__device__ __forceinline__ int64_t wave_sum(int64_t v) {
#pragma unroll
    for (int d = WAVE / 2; d >= 1; d >>= 1) v += __shfl_xor(v, d, WAVE);
    return v;
}

// Exclusive scan over a block of NW waves; `tmp` is NW int64 of LDS.
// Every thread of the block must call it. Returns the exclusive prefix and
// the block total.
template <int NW>
__device__ __forceinline__ int64_t block_excl_scan(int64_t v, int64_t* tmp, int64_t& total) {
    const int64_t inc = wave_incl_scan(v);
    if (NW == 1) {
        total = __shfl(inc, WAVE - 1, WAVE);
        return inc - v;
    }
    const int w = threadIdx.x / WAVE;
    if (lane() == WAVE - 1) tmp[w] = inc;
    __syncthreads();
    int64_t off = 0, tot = 0;
#pragma unroll
    for (int x = 0; x < NW; ++x) {
        const int64_t s = tmp[x];
        off += (x < w) ? s : 0;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return off + inc - v;
}

// First position p in [lo, hi) with a[p] >= key (a sorted ascending).
__device__ __forceinline__ int64_t lower_bound_g(const int32_t* __restrict__ a, int64_t lo, int64_t hi,
                                                 int64_t key) {
    while (lo < hi) {
        const int64_t mid = lo + ((hi - lo) >> 1);
        if ((int64_t)a[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// Semirings. acc_t is the LDS accumulator slot. For PAIR, I32 and BOOL the
// slot also records whether anything was inserted (nonzero <=> inserted), so
// one LDS atomic per admitted product suffices:
//  PAIR: count of products (never wraps to 0 in practice: 2^64 products)
//  I32:  (count << 32) + sum; the low word is the sum mod 2^32, carries only
//        reach the high word, which stays >= 1 once anything was inserted
//  BOOL: bit 1 = inserted, bit 0 = OR of (a && b)
// F64 and I64 keep a separate inserted flag (a plain byte store, races are
// benign since every writer stores 1). F64 starts from -0.0, the identity of
// IEEE addition, so an atomic add of the first product returns it exactly.
template <int SR> struct SRT;

// A value in global memory at a byte address (kept in the global address
// space, so that the load is a global rather than a flat one).
template <class V>
__device__ __forceinline__ V gload(uint64_t addr) {
    return *reinterpret_cast<const __attribute__((address_space(1))) V*>(addr);
}

template <> struct SRT<MSP_PLUS_TIMES_F64> {
    using in_t = double;
    using acc_t = double;
    using out_t = double;
    static constexpr bool needs_values = true;
    static constexpr bool sep_flag = true;
    __device__ static in_t one() { return 1.0; }
    __device__ static in_t load(const void* v, int64_t p) {
        return v ? static_cast<const double*>(v)[p] : 1.0;
    }
    static constexpr int vbytes = 8;  // width of a stored value
    __device__ static in_t load_at(uint64_t addr) { return gload<double>(addr); }
    __device__ static acc_t identity() { return -0.0; }
    // each product and each sum is rounded on its own: no fused multiply-add
    // is formed across term() and add()
    __device__ static acc_t term(in_t a, in_t b) {
#pragma clang fp contract(off)
        return a * b;
    }
    __device__ static void lds_add(acc_t* slot, acc_t t) { atomicAdd(slot, t); }
    __device__ static void merge(acc_t* slot, acc_t part) { atomicAdd(slot, part); }
    __device__ static acc_t add(acc_t x, acc_t t) {
#pragma clang fp contract(off)
        return x + t;
    }
    __device__ static bool is_set(acc_t) { return false; }
    __device__ static out_t finish(acc_t x) { return x; }
};

template <> struct SRT<MSP_PLUS_PAIR_I64> {
    using in_t = int32_t;  // unused: pair ignores values
    using acc_t = unsigned long long;
    using out_t = int64_t;
    static constexpr bool needs_values = false;
    static constexpr bool sep_flag = false;
    __device__ static in_t one() { return 1; }
    __device__ static in_t load(const void*, int64_t) { return 1; }
    static constexpr int vbytes = 4;
    __device__ static in_t load_at(uint64_t) { return 1; }
    __device__ static acc_t identity() { return 0ull; }
    __device__ static acc_t term(in_t, in_t) { return 1ull; }
    __device__ static void lds_add(acc_t* slot, acc_t) { atomicAdd(slot, 1ull); }
    __device__ static void merge(acc_t* slot, acc_t part) { atomicAdd(slot, part); }
    __device__ static acc_t add(acc_t x, acc_t) { return x + 1ull; }
    __device__ static bool is_set(acc_t x) { return x != 0ull; }
    __device__ static out_t finish(acc_t x) { return (int64_t)x; }
};

template <> struct SRT<MSP_LOR_LAND_BOOL> {
    using in_t = uint32_t;
    using acc_t = unsigned int;
    using out_t = uint8_t;
    static constexpr bool needs_values = true;
    static constexpr bool sep_flag = false;
    __device__ static in_t one() { return 1u; }
    // the raw byte: any nonzero byte is true (tested in term(), so that a load
    // is not waited for until the product is formed)
    __device__ static in_t load(const void* v, int64_t p) {
        return v ? (uint32_t)static_cast<const uint8_t*>(v)[p] : 1u;
    }
    static constexpr int vbytes = 1;
    __device__ static in_t load_at(uint64_t addr) { return (uint32_t)gload<uint8_t>(addr); }
    __device__ static acc_t identity() { return 0u; }
    __device__ static acc_t term(in_t a, in_t b) { return 2u | (uint32_t)((a != 0u) & (b != 0u)); }
    __device__ static void lds_add(acc_t* slot, acc_t t) { atomicOr(slot, t); }
    __device__ static void merge(acc_t* slot, acc_t part) { atomicOr(slot, part); }
    __device__ static acc_t add(acc_t x, acc_t t) { return x | t; }
    __device__ static bool is_set(acc_t x) { return x != 0u; }
    __device__ static out_t finish(acc_t x) { return (uint8_t)(x & 1u); }
};

template <> struct SRT<MSP_PLUS_TIMES_I32> {
    using in_t = uint32_t;
    using acc_t = unsigned long long;
    using out_t = int32_t;
    static constexpr bool needs_values = true;
    static constexpr bool sep_flag = false;
    __device__ static in_t one() { return 1u; }
    __device__ static in_t load(const void* v, int64_t p) {
        return v ? (uint32_t)static_cast<const int32_t*>(v)[p] : 1u;
    }
    static constexpr int vbytes = 4;
    __device__ static in_t load_at(uint64_t addr) { return gload<uint32_t>(addr); }
    __device__ static acc_t identity() { return 0ull; }
    __device__ static acc_t term(in_t a, in_t b) { return (1ull << 32) | (unsigned long long)(a * b); }
    __device__ static void lds_add(acc_t* slot, acc_t t) { atomicAdd(slot, t); }
    __device__ static void merge(acc_t* slot, acc_t part) { atomicAdd(slot, part); }
    __device__ static acc_t add(acc_t x, acc_t t) { return x + t; }
    __device__ static bool is_set(acc_t x) { return x != 0ull; }
    __device__ static out_t finish(acc_t x) { return (int32_t)(uint32_t)x; }
};

template <> struct SRT<MSP_PLUS_TIMES_I64> {
    using in_t = unsigned long long;
    using acc_t = unsigned long long;
    using out_t = int64_t;
    static constexpr bool needs_values = true;
    static constexpr bool sep_flag = true;
    __device__ static in_t one() { return 1ull; }
    __device__ static in_t load(const void* v, int64_t p) {
        return v ? (unsigned long long)static_cast<const int64_t*>(v)[p] : 1ull;
    }
    static constexpr int vbytes = 8;
    __device__ static in_t load_at(uint64_t addr) { return gload<unsigned long long>(addr); }
    __device__ static acc_t identity() { return 0ull; }
    __device__ static acc_t term(in_t a, in_t b) { return a * b; }
    __device__ static void lds_add(acc_t* slot, acc_t t) { atomicAdd(slot, t); }
    __device__ static void merge(acc_t* slot, acc_t part) { atomicAdd(slot, part); }
    __device__ static acc_t add(acc_t x, acc_t t) { return x + t; }
    __device__ static bool is_set(acc_t) { return false; }
    __device__ static out_t finish(acc_t x) { return (int64_t)x; }
};

}  // namespace mspk
