// Batched pointer validation (the API-time classification rule of AgileOS Sections IV-E and
// V-C, applied to many (addr, len) queries at once).
//
// Each workgroup stages the table's splitters (every 2^rlog2-th bucket base; 32-bit keys when
// the table allows exact compression) into LDS once, then every lane classifies its queries:
// a branchless binary search over the LDS splitters, an optional short search over the global
// splitters (only when the table is too large for the LDS budget), and one 32-byte record read
// that resolves the range inside the bucket and supplies its end, id and kind. Queries are
// streamed with coalesced 16-byte loads; verdict bytes and owner ids are stored coalesced.
#include <type_traits>

#include "launch.h"

namespace agile {

constexpr int VBLOCK = 256;
constexpr int QPT = 4;  // queries in flight per lane

template <bool COMP>
__global__ __launch_bounds__(VBLOCK) void k_validate(DevTable t, const ulonglong2* __restrict__ q,
                                                      uint64_t n, uint8_t* __restrict__ verdict,
                                                      int32_t* __restrict__ owner, uint32_t ntop,
                                                      uint32_t rlog2) {
    using K = typename std::conditional<COMP, uint32_t, uint64_t>::type;
    extern __shared__ __align__(16) unsigned char lds_raw[];
    K* top = reinterpret_cast<K*>(lds_raw);
    const K* gsplit = COMP ? reinterpret_cast<const K*>(t.split32)
                           : reinterpret_cast<const K*>(t.split64);
    for (uint32_t k = threadIdx.x; k < ntop; k += VBLOCK) top[k] = gsplit[(uint64_t)k << rlog2];
    __syncthreads();

    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * VBLOCK + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * VBLOCK) >> 6;
    constexpr uint64_t CHUNK = 64u * QPT;
    const uint32_t nb = t.nb;

    for (uint64_t c0 = wave * CHUNK; c0 < n; c0 += nwaves * CHUNK) {
        uint64_t a[QPT], L[QPT];
        K key[QPT];
        bool live[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            const uint64_t i = c0 + (uint64_t)j * 64u + lane;
            live[j] = i < n;
            ulonglong2 x = live[j] ? q[i] : make_ulonglong2(0, 0);
            a[j] = x.x;
            L[j] = x.y < 1 ? 1 : x.y;
        }
        bool below[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            if (COMP) {
                below[j] = a[j] < t.gmin;
                uint64_t d = (a[j] - t.gmin) >> t.shift;
                key[j] = (K)(d > 0xFFFFFFFFull ? 0xFFFFFFFFull : d);
            } else {
                below[j] = false;
                key[j] = (K)a[j];
            }
        }
        // level 1: branchless search over the LDS splitters (uniform trip count)
        uint32_t pos[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) pos[j] = 0;
        for (uint32_t len = ntop; len > 1;) {
            const uint32_t half = len >> 1;
#pragma unroll
            for (int j = 0; j < QPT; ++j) pos[j] = (top[pos[j] + half] <= key[j]) ? pos[j] + half : pos[j];
            len -= half;
        }
        bool found[QPT];
        uint32_t b[QPT];
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            found[j] = ntop > 0 && !below[j] && top[pos[j]] <= key[j];
            b[j] = pos[j] << rlog2;
        }
        // level 2: the 2^rlog2 buckets under the chosen LDS splitter (global, L2 resident)
        if (rlog2 > 0) {
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
        // record: pick the range inside the bucket, classify
#pragma unroll
        for (int j = 0; j < QPT; ++j) {
            uint8_t v = V_UNMAPPED;
            int32_t o = -1;
            if (found[j]) classify_in_bucket(load_rec(t.rec + b[j]), a[j], L[j], v, o);
            const uint64_t i = c0 + (uint64_t)j * 64u + lane;
            if (live[j]) {
                verdict[i] = v;
                owner[i] = o;
            }
        }
    }
}

SearchGeom validate_geometry(const DevTable& t, const DevInfo& d, size_t lds_budget) {
    SearchGeom g{0, 0, 0};
    if (t.nb == 0) return g;
    const size_t ks = t.compressed ? 4 : 8;
    size_t budget = lds_budget < d.lds_per_block ? lds_budget : d.lds_per_block;
    size_t cap = budget / ks;
    if (cap < 1) cap = 1;
    uint32_t rlog2 = 0;
    while (((uint64_t)t.nb + (1ull << rlog2) - 1) >> rlog2 > cap) ++rlog2;
    g.rlog2 = rlog2;
    g.ntop = (uint32_t)(((uint64_t)t.nb + (1ull << rlog2) - 1) >> rlog2);
    g.lds_bytes = (size_t)g.ntop * ks;
    return g;
}

hipError_t launch_validate(const DevTable& t, const DevInfo& d, size_t lds_budget, const void* q,
                           uint64_t n, uint8_t* verdict, int32_t* owner, hipStream_t s) {
    if (n == 0) return hipSuccess;
    SearchGeom g = validate_geometry(t, d, lds_budget);
    const void* fn = t.compressed ? reinterpret_cast<const void*>(&k_validate<true>)
                                  : reinterpret_cast<const void*>(&k_validate<false>);
    hipError_t e = hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)(g.lds_bytes > 0 ? g.lds_bytes : 16));
    if (e != hipSuccess) return e;
    int per_cu = 0;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, fn, VBLOCK, g.lds_bytes);
    if (e != hipSuccess) return e;
    if (per_cu < 1) per_cu = 1;
    const uint64_t chunks = (n + 64u * QPT - 1) / (64u * QPT);
    const uint64_t want = (chunks + (VBLOCK / 64) - 1) / (VBLOCK / 64);
    uint64_t grid = (uint64_t)d.num_cu * per_cu;
    if (want < grid) grid = want;
    if (t.compressed)
        hipLaunchKernelGGL(k_validate<true>, dim3((uint32_t)grid), dim3(VBLOCK), g.lds_bytes, s, t,
                           reinterpret_cast<const ulonglong2*>(q), n, verdict, owner, g.ntop,
                           g.rlog2);
    else
        hipLaunchKernelGGL(k_validate<false>, dim3((uint32_t)grid), dim3(VBLOCK), g.lds_bytes, s, t,
                           reinterpret_cast<const ulonglong2*>(q), n, verdict, owner, g.ntop,
                           g.rlog2);
    return hipGetLastError();
}

}  // namespace agile
