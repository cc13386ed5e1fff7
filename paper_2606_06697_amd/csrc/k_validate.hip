// Batched pointer validation (the API-time classification rule of AgileOS Sections IV-E and
// V-C, applied to many (addr, len) queries at once).
//
// Each workgroup (16 waves, one per CU: the LDS holds the whole search index) stages the
// table's splitters (every 2^rlog2-th bucket base; 32-bit keys when the table allows exact
// compression), a run of largest-value sentinels and a radix index over the splitters into LDS
// once. Every lane then classifies its queries: the radix entry of the address offset gives the
// start of a short run of candidate splitters, binary lifting over that run finds the last
// splitter <= addr (reading past the run is harmless: later splitters and the sentinels compare
// greater, so the predicate stays monotone and needs no bound checks), and one bucket record
// read resolves the range inside the bucket with its end, id and kind.
//
// With DMA set the same search answers the DMA registration check (Section V-C: only an exact
// live user allocation is accepted): an allowed range that is not the whole allocation, from
// its base with its full size, is reported INEXACT.
//
// Two record formats: packed 16-byte records (one load per query; offsets relative to the
// bucket base, used whenever the table's offsets fit) and general 32-byte records. Queries
// stream in with coalesced 16-byte loads, the next chunk's queries are in flight while the
// current chunk is searched, and verdict bytes and owner ids are stored coalesced.
#include <cstdlib>
#include <type_traits>

#include "launch.h"

namespace agile {

constexpr int VBLOCK = 1024;
typedef unsigned long long uint64x2 __attribute__((ext_vector_type(2)));

template <bool COMP>
struct KeyT {
    using T = uint64_t;
};
template <>
struct KeyT<true> {
    using T = uint32_t;
};

// Stage the search index into LDS: splitters, sentinels, radix entries.
template <bool COMP>
__device__ __forceinline__ const uint32_t* stage_index(const DevTable& t, unsigned char* lds_raw) {
    using K = typename KeyT<COMP>::T;
    const uint32_t ntop = t.ntop, npad = ntop + t.pad;
    K* top = reinterpret_cast<K*>(lds_raw);
    uint32_t* ri = reinterpret_cast<uint32_t*>(lds_raw + (((size_t)npad * sizeof(K) + 15) & ~15ull));
    const K* gsplit = COMP ? reinterpret_cast<const K*>(t.split32)
                           : reinterpret_cast<const K*>(t.split64);
    for (uint32_t k = threadIdx.x; k < npad; k += VBLOCK)
        top[k] = k < ntop ? gsplit[(uint64_t)k << t.rlog2] : (K)~(K)0;
    for (uint32_t k = threadIdx.x; k <= t.nr; k += VBLOCK) ri[k] = t.radix[k];
    __syncthreads();
    return ri;
}

template <int QPT, bool TAIL>
__device__ __forceinline__ void load_chunk(const ulonglong2* __restrict__ q, uint64_t n,
                                           uint64_t c0, uint32_t lane, ulonglong2 (&x)[QPT]) {
    const uint64x2* qp = reinterpret_cast<const uint64x2*>(q) + c0 + lane;
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        uint64x2 v;
        if (TAIL) {
            const uint64_t i = c0 + (uint64_t)j * 64u + lane;
            v = __builtin_nontemporal_load(reinterpret_cast<const uint64x2*>(q) + (i < n ? i : n - 1));
        } else {
            v = __builtin_nontemporal_load(qp + j * 64);
        }
        x[j] = make_ulonglong2(v.x, v.y);
    }
}

// Search key and radix start of each query.
template <bool COMP, int QPT>
__device__ __forceinline__ void keys_and_starts(const DevTable& t, const uint32_t* ri,
                                                const ulonglong2 (&x)[QPT],
                                                typename KeyT<COMP>::T (&key)[QPT],
                                                uint32_t (&p)[QPT]) {
    const uint32_t nr1 = t.nr - 1;
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const uint64_t d = x[j].x - t.gmin;
        uint32_t r;
        if (COMP) {
            const uint64_t kk = d >> t.shift;
            key[j] = (uint32_t)(kk > 0xFFFFFFFFull ? 0xFFFFFFFFull : kk);
            r = (uint32_t)key[j] >> t.xs;
        } else {
            key[j] = x[j].x;
            const uint64_t rr = d >> t.rsh;
            r = rr > 0xFFFFFFFFull ? 0xFFFFFFFFu : (uint32_t)rr;
        }
        p[j] = ri[r < nr1 ? r : nr1];
    }
}

// ---------------------------------------------------------------- general (32-byte records)
template <bool COMP, int QPT, bool TAIL, bool DMA>
__device__ __forceinline__ void chunk_wide(const DevTable& t, const unsigned char* lds_raw,
                                           const uint32_t* ri, const ulonglong2 (&x)[QPT],
                                           uint64_t n, uint8_t* __restrict__ verdict,
                                           int32_t* __restrict__ owner, uint64_t c0, uint32_t lane) {
    using K = typename KeyT<COMP>::T;
    const K* top = reinterpret_cast<const K*>(lds_raw);
    const uint32_t ntop = t.ntop;
    K key[QPT];
    uint32_t p[QPT];  // number of splitters known to be <= key
    keys_and_starts<COMP, QPT>(t, ri, x, key, p);
    for (uint32_t step = t.rlevels ? 1u << (t.rlevels - 1) : 0u; step; step >>= 1) {
        K v[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) v[j] = top[p[j] + step - 1];
#pragma unroll
        for (int j = 0; j < QPT; ++j) p[j] = v[j] <= key[j] ? p[j] + step : p[j];
    }
    const uint32_t rlog2 = t.rlog2, nb = t.nb;
    bool found[QPT];
    uint32_t b[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const uint32_t cnt = p[j] < ntop ? p[j] : ntop;
        found[j] = cnt > 0 && x[j].x >= t.gmin;
        b[j] = (cnt > 0 ? cnt - 1 : 0) << rlog2;
    }
    if (rlog2 > 0) {
        // the 2^rlog2 buckets under the chosen LDS splitter (global, L2 resident)
        const K* gsplit = COMP ? reinterpret_cast<const K*>(t.split32)
                               : reinterpret_cast<const K*>(t.split64);
        const uint32_t R = 1u << rlog2;
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            uint32_t len = nb - b[j] < R ? nb - b[j] : R;
            uint32_t base = b[j];
            while (len > 1) {
                const uint32_t half = len >> 1;
                base = (gsplit[base + half] <= key[j]) ? base + half : base;
                len -= half;
            }
            b[j] = base;
        }
    }
    PairRec rec[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) rec[j] = load_rec(t.rec + b[j]);
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        uint8_t v = V_UNMAPPED;
        int32_t o = -1;
        const uint64_t L = x[j].y;
        if (found[j]) classify_in_bucket(rec[j], x[j].x, L < 1 ? 1 : L, v, o);
        if (DMA && v == V_ALLOW) {
            // the first range of a bucket starts at the bucket's splitter
            const bool second = rec[j].base1 <= x[j].x;
            const uint64_t st = second ? rec[j].base1 : t.split64[b[j]];
            const uint64_t en = second ? rec[j].end1 : rec[j].end0;
            if (x[j].x != st || L != en - st) v = V_INEXACT;
        }
        const uint64_t i = c0 + (uint64_t)j * 64u + lane;
        if (!TAIL || i < n) {
            verdict[i] = v;
            owner[i] = o;
        }
    }
}

// ---------------------------------------------------------------- packed 16-byte records
// Offsets inside a bucket (the second range's base, both ends) are below 2^32 whenever packed
// records are built, so after one 64-bit subtraction the classification runs on 32-bit values.
template <bool COMP, int LEVELS, int QPT, bool TAIL, bool DMA>
__device__ __forceinline__ void chunk_packed(const DevTable& t, const unsigned char* lds_raw,
                                             const uint32_t* ri, const ulonglong2 (&x)[QPT],
                                             uint64_t n, uint8_t* __restrict__ verdict,
                                             int32_t* __restrict__ owner, uint64_t c0,
                                             uint32_t lane) {
    using K = typename KeyT<COMP>::T;
    const uint32_t ntop = t.ntop;
    K key[QPT];
    uint32_t p[QPT];
    keys_and_starts<COMP, QPT>(t, ri, x, key, p);
    // unrolled lifting: every step is a constant, so the LDS reads use immediate offsets
    const K* top = reinterpret_cast<const K*>(lds_raw);
#pragma unroll
    for (int lv = LEVELS - 1; lv >= 0; --lv) {
        const uint32_t step = 1u << lv;
        K v[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) v[j] = (top + step - 1)[p[j]];
#pragma unroll
        for (int j = 0; j < QPT; ++j) p[j] += v[j] <= key[j] ? step : 0u;
    }
    uint32_t b[QPT];
    bool found[QPT];
    K sp[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        const uint32_t cnt = p[j] < ntop ? p[j] : ntop;
        found[j] = cnt > 0 && x[j].x >= t.gmin;
        b[j] = cnt > 0 ? cnt - 1 : 0;
        sp[j] = top[b[j]];
    }
    uint4 r[QPT];
#pragma unroll
    for (int j = 0; j < QPT; ++j) r[j] = t.nrec[b[j]];
    const uint32_t m1 = t.w1 >= 32 ? 0xFFFFFFFFu : (1u << t.w1) - 1u;
    const uint32_t sb = t.sb, w1 = t.w1;
    uint8_t* vp = verdict + c0 + lane;
    int32_t* op = owner + c0 + lane;
#pragma unroll
    for (int j = 0; j < QPT; ++j) {
        // offset from the bucket base; an address 2^32 or more past it is in no range of it
        const uint64_t rel64 = COMP ? (x[j].x - t.gmin) - ((uint64_t)sp[j] << t.shift)
                                    : x[j].x - (uint64_t)sp[j];
        const bool near = (uint32_t)(rel64 >> 32) == 0u;
        const uint32_t rel = (uint32_t)rel64;
        const uint32_t ob1 = (r[j].x & m1) << sb;
        const uint32_t oe0 = w1 >= 32 ? 0u : r[j].x >> w1;
        const bool second = rel >= ob1;
        const uint32_t oend = second ? r[j].y : oe0;
        const uint32_t meta = second ? r[j].w : r[j].z;
        const bool inside = found[j] && near && rel < oend;
        // inside a range, oend - rel >= 1, so max(len, 1) <= oend - rel iff len <= oend - rel
        const bool fits = (uint32_t)(x[j].y >> 32) == 0u && (uint32_t)x[j].y <= oend - rel;
        // DMA: the range starts at offset 0 (first) or ob1 (second) and must be taken whole
        const uint32_t ost = second ? ob1 : 0u;
        const bool exact = !DMA || (rel == ost && (uint32_t)x[j].y == oend - ost);
        const uint8_t v = !inside ? V_UNMAPPED
                                  : ((meta & 3u) != KIND_USER
                                         ? V_PROTECTED
                                         : (fits ? (exact ? V_ALLOW : V_INEXACT) : V_STRADDLE));
        const int32_t o = inside ? (int32_t)(meta >> 2) : -1;
        if (TAIL) {
            const uint64_t i = c0 + (uint64_t)j * 64u + lane;
            if (i < n) {
                verdict[i] = v;
                owner[i] = o;
            }
        } else {
            __builtin_nontemporal_store(v, vp + j * 64);  // written once, not read back
            __builtin_nontemporal_store(o, op + j * 64);
        }
    }
}

// Grid-stride loop over chunks of 64*QPT queries per wave, full chunks software-pipelined.
template <bool COMP, bool PACKED, int LEVELS, int QPT, bool DMA>
__global__ __launch_bounds__(VBLOCK) void k_validate(DevTable t, const ulonglong2* __restrict__ q,
                                                      uint64_t n, uint8_t* __restrict__ verdict,
                                                      int32_t* __restrict__ owner) {
    extern __shared__ __align__(16) unsigned char lds_raw[];
    const uint32_t* ri = stage_index<COMP>(t, lds_raw);
    if (t.nb == 0) {
        // empty table: everything is unmapped
        for (uint64_t i = (uint64_t)blockIdx.x * VBLOCK + threadIdx.x; i < n;
             i += (uint64_t)gridDim.x * VBLOCK) {
            verdict[i] = V_UNMAPPED;
            owner[i] = -1;
        }
        return;
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * VBLOCK + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * VBLOCK) >> 6;
    constexpr uint64_t CHUNK = 64u * QPT;
    const uint64_t nfull = n / CHUNK * CHUNK;
    const uint64_t stride = nwaves * CHUNK;
    uint64_t c0 = wave * CHUNK;
    ulonglong2 x[QPT];
    if (c0 < nfull) load_chunk<QPT, false>(q, n, c0, lane, x);
    for (; c0 < nfull; c0 += stride) {
        ulonglong2 cur[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) cur[j] = x[j];
        if (c0 + stride < nfull) load_chunk<QPT, false>(q, n, c0 + stride, lane, x);
        if (PACKED)
            chunk_packed<COMP, LEVELS, QPT, false, DMA>(t, lds_raw, ri, cur, n, verdict, owner, c0,
                                                        lane);
        else
            chunk_wide<COMP, QPT, false, DMA>(t, lds_raw, ri, cur, n, verdict, owner, c0, lane);
    }
    if (c0 < n) {
        load_chunk<QPT, true>(q, n, c0, lane, x);
        if (PACKED)
            chunk_packed<COMP, LEVELS, QPT, true, DMA>(t, lds_raw, ri, x, n, verdict, owner, c0, lane);
        else
            chunk_wide<COMP, QPT, true, DMA>(t, lds_raw, ri, x, n, verdict, owner, c0, lane);
    }
}

template <bool COMP, bool PACKED, int LEVELS, int QPT, bool DMA>
static hipError_t launch_v(const DevTable& t, const DevInfo& d, const void* q, uint64_t n,
                           uint8_t* verdict, int32_t* owner, hipStream_t s) {
    const void* fn = reinterpret_cast<const void*>(&k_validate<COMP, PACKED, LEVELS, QPT, DMA>);
    const size_t lds = t.lds_bytes;
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(lds > 0 ? lds : 16));
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, VBLOCK, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const uint64_t chunks = (n + 64u * QPT - 1) / (64u * QPT);
    const uint64_t want = (chunks + (VBLOCK / 64) - 1) / (VBLOCK / 64);
    uint64_t grid = (uint64_t)d.num_cu * per_cu;
    if (want < grid) grid = want;
    hipLaunchKernelGGL((k_validate<COMP, PACKED, LEVELS, QPT, DMA>), dim3((uint32_t)grid), dim3(VBLOCK),
                       lds, s, t, reinterpret_cast<const ulonglong2*>(q), n, verdict, owner);
    return hipGetLastError();
}

template <bool COMP, bool DMA>
static hipError_t launch_c(const DevTable& t, const DevInfo& d, const void* q, uint64_t n,
                           uint8_t* verdict, int32_t* owner, hipStream_t s) {
    constexpr int QW = 6;  // queries per lane, general records
    constexpr int QP = 6;  // queries per lane, packed records
    if (t.narrow && t.rlog2 == 0) {
        switch (t.lift) {
            case 2: return launch_v<COMP, true, 2, QP, DMA>(t, d, q, n, verdict, owner, s);
            case 4: return launch_v<COMP, true, 4, QP, DMA>(t, d, q, n, verdict, owner, s);
            case 6: return launch_v<COMP, true, 6, QP, DMA>(t, d, q, n, verdict, owner, s);
            case 8: return launch_v<COMP, true, 8, QP, DMA>(t, d, q, n, verdict, owner, s);
            default: break;
        }
    }
    return launch_v<COMP, false, 0, QW, DMA>(t, d, q, n, verdict, owner, s);
}

hipError_t launch_validate(const DevTable& t, const DevInfo& d, const void* q, uint64_t n,
                           uint8_t* verdict, int32_t* owner, bool dma, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (dma) {
        if (t.compressed) return launch_c<true, true>(t, d, q, n, verdict, owner, s);
        return launch_c<false, true>(t, d, q, n, verdict, owner, s);
    }
    if (t.compressed) return launch_c<true, false>(t, d, q, n, verdict, owner, s);
    return launch_c<false, false>(t, d, q, n, verdict, owner, s);
}

}  // namespace agile
