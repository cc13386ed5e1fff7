// Guarded scatter-add dst[idx[i], :] += src[i, :] (kernel memory guard of AgileOS Section V-E),
// organised so that heavily repeated destination rows (the hot rows of a Zipf-distributed
// embedding gradient) do not serialize on atomics.
//
// Each workgroup takes a chunk of 2048 consecutive indices, sorts (destination key, position)
// pairs in LDS with a bitonic network, and cuts the sorted chunk into pieces of at most 32
// equal keys. A wave sums one piece's source rows in position order (fixed order, fp32 or fp64
// registers) and adds the sum to the destination row with one atomic per element, so a row
// repeated r times in a chunk costs ceil(r/32) atomic row-updates instead of r. The guard binds
// the three pointer arguments once per wave: index loads and source elements are prefix-bounded,
// destination rows inside the binding's row interval take the fast path, every other row is
// checked per element with exact arithmetic. Denials are counted and the smallest (element,
// operand) key is recorded as in the other data-dependent guarded kernels.
#include <type_traits>

#include "launch.h"

namespace agile {

constexpr int SABLOCK = 256;
constexpr int SACHUNK = 2048;
constexpr int SAPIECE = 32;
constexpr uint64_t SA_SLOW = ~0ull;  // key of rows outside the destination's row interval

template <int W>
struct FloatOf;
template <>
struct FloatOf<4> {
    using F = float;
    using E = uint32_t;
};
template <>
struct FloatOf<8> {
    using F = double;
    using E = uint64_t;
};

// Exclusive block-wide prefix sum of one value per thread (SABLOCK threads); returns the total.
__device__ inline uint32_t block_exscan(uint32_t v, uint32_t& excl, uint32_t* wsum) {
    const uint32_t lane = threadIdx.x & 63u, wv = threadIdx.x >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0, total = 0;
    for (int k = 0; k < SABLOCK / 64; ++k) {
        const uint32_t s = wsum[k];
        if ((uint32_t)k < wv) before += s;
        total += s;
    }
    excl = before + inc - v;
    __syncthreads();
    return total;
}

template <bool GUARD, int W, int EPL>
__global__ __launch_bounds__(SABLOCK) void k_scatter_add(DevTable t, DevLog* log, uint8_t* dst,
                                                         uint64_t rb, const int64_t* idx,
                                                         const uint8_t* src, uint64_t n,
                                                         RowsGuard rg, unsigned long long seq,
                                                         int logon) {
    using F = typename FloatOf<W>::F;
    __shared__ uint64_t skey[SACHUNK];
    __shared__ uint16_t spos[SACHUNK];
    __shared__ uint16_t sstart[SACHUNK + 1];
    __shared__ uint32_t wsum[SABLOCK / 64];
    __shared__ uint32_t snp;

    const uint64_t D = rb / W;
    const uint64_t Ki = rg.ki, Ks = rg.kc;
    const RowGuard g = rg.g;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    constexpr uint32_t NWV = SABLOCK / 64;
    FaultAcc acc;

    for (uint64_t c0 = (uint64_t)blockIdx.x * SACHUNK; c0 < n; c0 += (uint64_t)gridDim.x * SACHUNK) {
        const uint32_t cnt = (uint32_t)(n - c0 < SACHUNK ? n - c0 : SACHUNK);
        // 1. destination keys: offset of the row inside the binding's row interval, or SA_SLOW
        for (uint32_t k = tid; k < SACHUNK; k += SABLOCK) {
            uint64_t key = SA_SLOW;
            if (k < cnt) {
                const uint64_t i = c0 + k;
                const bool iok = !GUARD || i < Ki;
                const int64_t iv = iok ? idx[i] : 0;
                if (!iok) acc.note((i * D) << 2);
                if (GUARD && g.rlo <= iv && iv <= g.rhi) key = (uint64_t)iv - (uint64_t)g.rlo;
                if (!GUARD) key = (uint64_t)iv ^ 0x8000000000000000ull;  // order-preserving
            }
            skey[k] = key;
            spos[k] = (uint16_t)k;
        }
        __syncthreads();
        // 2. bitonic sort of (key, position), ascending; padding (position >= cnt) sorts last
        for (uint32_t size = 2; size <= SACHUNK; size <<= 1) {
            for (uint32_t stride = size >> 1; stride > 0; stride >>= 1) {
                for (uint32_t x = tid; x < SACHUNK / 2; x += SABLOCK) {
                    const uint32_t a = 2 * x - (x & (stride - 1));
                    const uint32_t b = a + stride;
                    const bool asc = (a & size) == 0;
                    const uint64_t ka = skey[a], kb = skey[b];
                    const uint16_t pa = spos[a], pb = spos[b];
                    const bool gt = ka > kb || (ka == kb && pa > pb);
                    if (gt == asc) {
                        skey[a] = kb;
                        skey[b] = ka;
                        spos[a] = pb;
                        spos[b] = pa;
                    }
                }
                __syncthreads();
            }
        }
        // 3. pieces: runs of equal keys, cut every SAPIECE positions
        constexpr uint32_t PER = SACHUNK / SABLOCK;
        uint32_t flags = 0, c = 0;
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q) {
            const uint32_t k = tid * PER + q;
            const bool f = k < cnt && (k == 0 || k % SAPIECE == 0 || skey[k] != skey[k - 1]);
            flags |= (uint32_t)f << q;
            c += f;
        }
        uint32_t excl;
        const uint32_t np = block_exscan(c, excl, wsum);
#pragma unroll
        for (uint32_t q = 0; q < PER; ++q)
            if ((flags >> q) & 1u) sstart[excl++] = (uint16_t)(tid * PER + q);
        if (tid == 0) {
            sstart[np] = (uint16_t)cnt;
            snp = np;
        }
        __syncthreads();
        // 4. one wave per piece: sum the piece's source rows, add once to the destination row
        const uint32_t npieces = snp;
        for (uint32_t p = wv; p < npieces; p += NWV) {
            const uint32_t s = sstart[p], e = sstart[p + 1];
            const uint64_t key = skey[s];
            if (key != SA_SLOW) {
                const int64_t r = GUARD ? (int64_t)(key + (uint64_t)g.rlo)
                                        : (int64_t)(key ^ 0x8000000000000000ull);
                uint8_t* drow = dst + (uint64_t)r * rb;
                for (uint64_t col0 = (uint64_t)lane * EPL; col0 < D; col0 += 64u * EPL) {
                    F sum[EPL];
#pragma unroll
                    for (int q = 0; q < EPL; ++q) sum[q] = (F)-0.0;
                    for (uint32_t k = s; k < e; ++k) {
                        const uint64_t pos = c0 + spos[k];
                        const uint64_t es = pos * D + col0;
                        if (!GUARD || es + EPL <= Ks) {
                            const F* sp = reinterpret_cast<const F*>(src) + es;
#pragma unroll
                            for (int q = 0; q < EPL; ++q) sum[q] += sp[q];
                        } else {
#pragma unroll
                            for (int q = 0; q < EPL; ++q) {
                                if (es + q < Ks) sum[q] += reinterpret_cast<const F*>(src)[es + q];
                                else {
                                    sum[q] += (F)0.0;
                                    acc.note(((es + q) << 2) | 1u);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int q = 0; q < EPL; ++q)
                        unsafeAtomicAdd(reinterpret_cast<F*>(drow) + col0 + q, sum[q]);
                }
            } else {
                // rows outside the destination's row interval: exact per-element checks
                for (uint32_t k = s; k < e; ++k) {
                    const uint64_t pos = c0 + spos[k];
                    const bool iok = !GUARD || pos < Ki;
                    const int64_t iv = iok ? idx[pos] : 0;
                    uint8_t* drow = dst + (uint64_t)iv * rb;
                    for (uint64_t col = lane; col < D; col += 64) {
                        const uint64_t es = pos * D + col;
                        F v = (F)0.0;
                        if (!GUARD || es < Ks) v = reinterpret_cast<const F*>(src)[es];
                        else acc.note((es << 2) | 1u);
                        if (!GUARD || elem_ok(g, iv, rb, col, W))
                            unsafeAtomicAdd(reinterpret_cast<F*>(drow + col * W), v);
                        else
                            acc.note((es << 2) | 2u);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (GUARD && logon) {
        fold_faults(acc, log, [&](unsigned long long k) {
            const unsigned long long elem = k >> 2;
            const uint32_t operand = (uint32_t)(k & 3u);
            const uint64_t i = elem / D, col = elem % D;
            __int128 A;
            uint32_t w = W;
            if (operand == 0) {
                A = (__int128)(uint64_t)idx + (__int128)(8 * i);
                w = 8;
            } else if (operand == 1) {
                A = (__int128)(uint64_t)src + (__int128)elem * W;
            } else {
                const int64_t v = i < Ki ? idx[i] : 0;
                A = (__int128)(uint64_t)dst + (__int128)v * (__int128)rb + (__int128)(col * W);
            }
            record_at(t, log, seq, elem, operand, A, w, 5 /*OP_SCATTER_ADD*/);
        });
    }
}

template <bool G, int W>
static void scatter_add_w(const DevTable& t, DevLog* log, void* dst, uint64_t rb,
                          const int64_t* idx, const void* src, uint64_t n, const RowsGuard& rg,
                          unsigned long long seq, int logon, const DevInfo& d, hipStream_t s) {
    uint64_t grid = (n + SACHUNK - 1) / SACHUNK;
    const uint64_t cap = (uint64_t)d.num_cu * 4;
    if (grid > cap) grid = cap;
    const bool v4 = W == 4 && (rb / W) % 4 == 0 && ((uint64_t)src & 15) == 0;
    if (v4)
        hipLaunchKernelGGL((k_scatter_add<G, W, 4>), dim3((uint32_t)grid), dim3(SABLOCK), 0, s, t, log,
                           (uint8_t*)dst, rb, idx, (const uint8_t*)src, n, rg, seq, logon);
    else
        hipLaunchKernelGGL((k_scatter_add<G, W, 1>), dim3((uint32_t)grid), dim3(SABLOCK), 0, s, t, log,
                           (uint8_t*)dst, rb, idx, (const uint8_t*)src, n, rg, seq, logon);
}

hipError_t launch_scatter_add(bool guard, const DevTable& t, DevLog* log, const Bind* binds,
                              void* dst, uint64_t rb, const int64_t* idx, const void* src,
                              uint64_t n, uint32_t w, unsigned long long seq, int logon,
                              const DevInfo& d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (guard) {
        const RowsGuard rg = rows_guard(binds[0], binds[1], binds[2], (uint64_t)idx, (uint64_t)src,
                                        (uint64_t)dst, n, rb, w);
        if (w == 4) scatter_add_w<true, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_add_w<true, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    } else {
        const RowsGuard rg = rows_open(n, rb, w);
        if (w == 4) scatter_add_w<false, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_add_w<false, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    }
    return hipGetLastError();
}

}  // namespace agile
