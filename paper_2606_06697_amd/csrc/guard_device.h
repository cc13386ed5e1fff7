// Device-side data layout and helpers shared by the guard kernels (gfx950, wave64).
//
// Table image (built on the host from the sorted range list, uploaded in stream order):
//   radix[r]    u32  search index over the LDS-resident splitters (see DevTable)
//   nrec[b]     16 B the bucket's record with bit-packed offsets (see DevTable), when they fit
//   split64[b]  u64  base of the first range of bucket b (buckets hold 2 consecutive
//                    ranges in address order), nb = ceil(n/2) entries
//   split32[b]  u32  (split64[b] - gmin) >> shift, present when every bucket base is a
//                    multiple of 2^shift above gmin and the keys fit 32 bits; a query key
//                    (addr - gmin) >> shift then orders exactly like the address
//   rec[b]      32 B {base of the 2nd range (U64 max if none), end of 1st, end of 2nd,
//                    meta of 1st, meta of 2nd}, meta = id << 2 | kind
//   backed[b]   u8   bit 0 / bit 1: the first / second range was inserted as backed memory
// A lookup finds the last bucket whose base is <= addr, then reads one 32-byte record to
// pick the range inside the bucket and to get its end, id and kind.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "guard_arith.h"

namespace agile {

constexpr uint32_t KIND_USER = 0;
constexpr uint8_t V_ALLOW = 0, V_PROTECTED = 1, V_STRADDLE = 2, V_UNMAPPED = 3,
                  V_CROSS_ALLOC = 4, V_INEXACT = 5;
constexpr uint64_t U64MAX = ~0ull;

struct alignas(32) PairRec {
    uint64_t base1;
    uint64_t end0;
    uint64_t end1;
    uint32_t meta0;
    uint32_t meta1;
};
static_assert(sizeof(PairRec) == 32, "PairRec is one 32-byte sector");

struct DevTable {
    const uint64_t* split64;
    const uint32_t* split32;
    const PairRec* rec;
    const uint32_t* radix;  // validation search index, see below
    const uint8_t* backed;  // per bucket: bit 0 / bit 1 = first / second range is backed memory
    uint64_t gmin;
    uint32_t nb;          // number of buckets (0 for an empty table)
    uint32_t shift;
    uint32_t compressed;  // split32 valid
    // Validation search geometry. The LDS holds top[k] = splitter(k << rlog2), k < ntop, then
    // `pad` sentinels of the largest key value, then radix[r] = number of top entries below
    // gmin + (r << rsh), r <= nr (radix[nr] = ntop): an address with offset d = addr - gmin
    // has its answer among top[radix[r] ..], r = min(d >> rsh, nr - 1), at most 2^rlevels - 1
    // entries on. With compressed keys, r = min(key >> xs, nr - 1) (xs = rsh - shift, capped at
    // 31; nr == 1 whenever it would exceed 31). pad = 2^lift, lift >= rlevels.
    uint32_t ntop;
    uint32_t rlog2;
    uint32_t nr;
    uint32_t rsh;
    uint32_t xs;
    uint32_t rlevels;
    uint32_t lift;
    uint32_t pad;
    uint32_t lds_bytes;   // LDS one validation workgroup needs (top + sentinels + radix)
    // Packed records (validation only, present when narrow != 0; then rlog2 == 0): per bucket
    // 16 bytes {u32 lo, u32 hi, u32 meta0, u32 meta1} with offsets relative to the bucket base:
    // lo = (second range's base >> sb) | (first range's end << w1), hi = second range's end.
    const uint4* nrec;
    uint32_t narrow;
    uint32_t sb;
    uint32_t w1;
    uint32_t pad2;
};

// Device copy of the public fault log (same field order as agile_fault) + per-launch scratch.
struct DevLog {
    unsigned long long count;
    unsigned long long first_seq;
    unsigned long long first_elem;
    unsigned long long first_addr;
    uint32_t first_width;
    uint32_t first_op;
    uint32_t first_operand;
    uint32_t first_verdict;
    int32_t first_owner;
    uint32_t reserved;
    // scratch of one guarded launch, returned to its idle state by the launch's finishing kernel
    unsigned long long s_minkey;   // min over (elem << 2 | operand) of this launch's denials
    unsigned long long s_count;    // denials of this launch
};

// Classification of `a` inside bucket b (split64[b] <= a is known): verdict + owner for a
// length-L query (L >= 1).
__device__ __forceinline__ void classify_in_bucket(const PairRec& r, uint64_t a, uint64_t L,
                                                   uint8_t& v, int32_t& owner) {
    const bool second = r.base1 <= a;
    const uint64_t end = second ? r.end1 : r.end0;
    const uint32_t meta = second ? r.meta1 : r.meta0;
    if (a >= end) {
        v = V_UNMAPPED;
        owner = -1;
        return;
    }
    owner = (int32_t)(meta >> 2);
    if ((meta & 3u) != KIND_USER) {
        v = V_PROTECTED;
    } else {
        v = (L <= end - a) ? V_ALLOW : V_STRADDLE;
    }
}

__device__ __forceinline__ PairRec load_rec(const PairRec* p) {
    const ulonglong2* q = reinterpret_cast<const ulonglong2*>(p);
    ulonglong2 x = q[0];
    ulonglong2 y = q[1];
    PairRec r;
    r.base1 = x.x;
    r.end0 = x.y;
    r.end1 = y.x;
    r.meta0 = (uint32_t)y.y;
    r.meta1 = (uint32_t)(y.y >> 32);
    return r;
}

// Last bucket with split64[b] <= a, or -1. One lane, binary search over global memory
// (used for single lookups in fault records).
__device__ inline int64_t bucket_search_lane(const DevTable& t, uint64_t a) {
    if (t.nb == 0 || t.split64[0] > a) return -1;
    uint32_t base = 0, len = t.nb;
    while (len > 1) {
        uint32_t half = len >> 1;
        base = (t.split64[base + half] <= a) ? base + half : base;
        len -= half;
    }
    return base;
}

__device__ inline void verdict_lane(const DevTable& t, uint64_t a, uint64_t len, uint8_t& v,
                                    int32_t& owner) {
    int64_t b = bucket_search_lane(t, a);
    if (b < 0) {
        v = V_UNMAPPED;
        owner = -1;
        return;
    }
    classify_in_bucket(load_rec(t.rec + b), a, len < 1 ? 1 : len, v, owner);
}

// Move a wave-uniform 64-bit value into scalar registers (readfirstlane works on 32-bit
// halves and returns int: widen through uint32_t so no sign bits leak into the high half).
__device__ __forceinline__ uint64_t uniform_u64(uint64_t x) {
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)x);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readfirstlane((int)(uint32_t)(x >> 32));
    return ((uint64_t)hi << 32) | lo;
}

// Reason recorded for a denied access at address a (already known to lie in [0, 2^64)).
__device__ inline void reason_lane(const DevTable& t, uint64_t a, uint32_t w, uint32_t& v,
                                   int32_t& owner) {
    uint8_t vv;
    verdict_lane(t, a, w, vv, owner);
    v = (vv == V_ALLOW) ? V_CROSS_ALLOC : vv;
}

// Write the first-fault record if the log has none yet (launches of one handle are ordered,
// so an earlier launch's record always wins).
__device__ inline void log_record(DevLog* log, unsigned long long seq, unsigned long long elem,
                                  uint32_t operand, uint64_t addr, uint32_t width, uint32_t op,
                                  uint32_t verdict, int32_t owner) {
    if (log->first_seq != ~0ull) return;
    log->first_elem = elem;
    log->first_addr = addr;
    log->first_width = width;
    log->first_op = op;
    log->first_operand = operand;
    log->first_verdict = verdict;
    log->first_owner = owner;
    __threadfence();
    log->first_seq = seq;
}

// Wave reductions (wave64).
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}
__device__ __forceinline__ unsigned long long wave_min_u64(unsigned long long x) {
    for (int o = 32; o > 0; o >>= 1) {
        unsigned long long y = __shfl_xor(x, o, 64);
        x = y < x ? y : x;
    }
    return x;
}

// ---- denial accounting shared by the data-dependent guarded kernels ----
struct FaultAcc {
    unsigned long long cnt = 0;
    unsigned long long mk = ~0ull;
    __device__ __forceinline__ void note(unsigned long long key) {
        ++cnt;
        mk = key < mk ? key : mk;
    }
};

// Fold per-lane denials into the launch's scratch: one atomic pair per wave that saw a denial
// (no workgroup-wide step, so waves and workgroups finish independently). The record of the
// smallest key is written afterwards by the launch's finishing kernel.
__device__ inline void fold_faults(FaultAcc acc, DevLog* log) {
    const unsigned long long c = wave_sum_u64(acc.cnt);
    const unsigned long long m = wave_min_u64(acc.mk);
    if ((threadIdx.x & 63u) == 0 && c) {
        atomicAdd(&log->s_count, c);
        atomicMin(&log->s_minkey, m);
    }
}

__device__ inline void record_at(const DevTable& t, DevLog* log, unsigned long long seq,
                                 unsigned long long elem, uint32_t operand, __int128 A, uint32_t w,
                                 uint32_t op) {
    uint32_t v = V_UNMAPPED;
    int32_t o = -1;
    const bool in_space = A >= 0 && A <= (__int128)U64MAX;
    if (in_space) reason_lane(t, (uint64_t)A, w, v, o);
    log_record(log, seq, elem, operand, (uint64_t)A, w, op, v, o);
}

// Where the denials of a row kernel (gather, scatter, scatter-add) live: a key's element e is
// row i = e / D, column e % D; operand 0 is the index load at idx + 8 i, the contiguous operand is
// at cont + e * w and the row-addressed one at rowp + idx[i] * rb + column * w.
struct FaultSite {
    uint32_t op;           // AGILE_OP_* of the call
    uint32_t w;            // element width
    uint32_t row_operand;  // operand number of the row-addressed pointer (1 gather, 2 scatter)
    uint32_t pad;
    uint64_t D, rb, ki;    // elements per row, row bytes, readable index prefix
    uint64_t idx, cont, rowp;
};

}  // namespace agile
