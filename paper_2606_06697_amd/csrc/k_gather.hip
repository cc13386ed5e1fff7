// Guarded gather and scatter(-add) over rows (kernel memory guard of AgileOS Section V-E).
//
// out[i,:] = T[idx[i],:]  /  dst[idx[i],:] (+)= src[i,:], rows of `rb` bytes, elements of W bytes.
// Every wave binds the three pointer arguments once (wave-cooperative table search, bounds in
// scalar registers). The index and the contiguous operand have prefix-shaped allowed sets; for
// the row-addressed operand the binding becomes an index interval [rlo, rhi] of rows that lie
// wholly inside the allocation, so the per-row guard is two signed compares of the loaded
// index against scalars. Rows outside it (hostile indices, or a table pointer that is not
// row-aligned with its allocation's ends) take an exact 128-bit per-element path. Denials are
// counted per lane, reduced per wave, and folded into the handle's log: the smallest
// (element, operand) key wins, and the last workgroup to finish writes that denial's record.
// GUARD=false compiles the same loops with no binding and no compare (the unguarded twin).
#include "launch.h"

namespace agile {

constexpr int GBLOCK = 256;
constexpr int GROWS = 4;  // rows in flight per lane group

template <int B>
struct Word;
template <>
struct Word<4> {
    using T = uint32_t;
};
template <>
struct Word<8> {
    using T = uint64_t;
};
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
template <>
struct Word<16> {
    using T = u32x4;
};

template <bool GUARD, int CW, int W>
__global__ __launch_bounds__(GBLOCK) void k_gather(DevTable t, DevLog* log, uint8_t* out,
                                                    const uint8_t* T, uint64_t rb,
                                                    const int64_t* idx, uint64_t n,
                                                    unsigned long long seq, int logon,
                                                    uint32_t glog2) {
    using V = typename Word<CW>::T;
    using E = typename Word<W>::T;
    constexpr uint32_t EPC = CW / W;  // elements per chunk
    const uint64_t D = rb / W;
    const uint64_t nch = rb / CW;
    uint64_t Ki = n, Ko = n * D;
    RowGuard g{INT64_MIN, INT64_MAX, 0, 0, true};
    if (GUARD) {
        const Bind bi = bind_wave(t, (uint64_t)idx);
        const Bind bt = bind_wave(t, (uint64_t)T);
        const Bind bo = bind_wave(t, (uint64_t)out);
        Ki = clip_prefix(bi, (uint64_t)idx, n, 8);
        Ko = clip_prefix(bo, (uint64_t)out, n * D, W);
        g = row_guard(bt, (uint64_t)T, rb);
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t G = 1u << glog2;
    const uint32_t lir = lane & (G - 1);
    const uint32_t riw = lane >> glog2;
    const uint64_t rpw = 64u >> glog2;  // rows per wave
    const uint64_t wave = ((uint64_t)blockIdx.x * GBLOCK + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * GBLOCK) >> 6;
    FaultAcc acc;
    for (uint64_t r0 = wave * rpw * GROWS; r0 < n; r0 += nwaves * rpw * GROWS) {
        int64_t iv[GROWS];
        bool live[GROWS];
#pragma unroll
        for (int u = 0; u < GROWS; ++u) {
            const uint64_t i = r0 + u * rpw + riw;
            live[u] = i < n;
            const bool iok = !GUARD || i < Ki;
            iv[u] = (live[u] && iok) ? idx[i] : 0;
            if (GUARD && live[u] && !iok && lir == 0) acc.note((i * D) << 2);
        }
#pragma unroll
        for (int u = 0; u < GROWS; ++u) {
            if (!live[u]) continue;
            const uint64_t i = r0 + u * rpw + riw;
            const bool full = !GUARD || (g.rlo <= iv[u] && iv[u] <= g.rhi);
            const uint8_t* trow = T + (uint64_t)iv[u] * rb;
            uint8_t* orow = out + i * rb;
            for (uint64_t ch = lir; ch < nch; ch += G) {
                const uint64_t e0 = i * D + ch * EPC;
                if (full && (!GUARD || e0 + EPC <= Ko)) {
                    *reinterpret_cast<V*>(orow + ch * CW) = *reinterpret_cast<const V*>(trow + ch * CW);
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < EPC; ++k) {
                        const uint64_t col = ch * EPC + k;
                        const uint64_t e = e0 + k;
                        E val = 0;
                        if (full || elem_ok(g, iv[u], rb, col, W)) {
                            val = *reinterpret_cast<const E*>(trow + col * W);
                        } else {
                            acc.note((e << 2) | 1u);
                        }
                        if (e < Ko) *reinterpret_cast<E*>(orow + col * W) = val;
                        else acc.note((e << 2) | 2u);
                    }
                }
            }
        }
    }
    if (GUARD && logon) {
        fold_faults(acc, log, [&](unsigned long long key) {
            const unsigned long long elem = key >> 2;
            const uint32_t operand = (uint32_t)(key & 3u);
            const uint64_t i = elem / D, col = elem % D;
            __int128 A;
            uint32_t w = W;
            if (operand == 0) {
                A = (__int128)(uint64_t)idx + (__int128)(8 * i);
                w = 8;
            } else if (operand == 1) {
                const int64_t v = i < Ki ? idx[i] : 0;
                A = (__int128)(uint64_t)T + (__int128)v * (__int128)rb + (__int128)(col * W);
            } else {
                A = (__int128)(uint64_t)out + (__int128)elem * W;
            }
            record_at(t, log, seq, elem, operand, A, w, 3 /*OP_GATHER*/);
        });
    }
}

template <bool GUARD, int CW, int W, bool ACC>
__global__ __launch_bounds__(GBLOCK) void k_scatter(DevTable t, DevLog* log, uint8_t* dst,
                                                     uint64_t rb, const int64_t* idx,
                                                     const uint8_t* src, uint64_t n,
                                                     unsigned long long seq, int logon,
                                                     uint32_t glog2) {
    using V = typename Word<CW>::T;
    using E = typename Word<W>::T;
    using F = typename std::conditional<W == 4, float, double>::type;
    constexpr uint32_t EPC = CW / W;
    const uint64_t D = rb / W;
    const uint64_t nch = rb / CW;
    uint64_t Ki = n, Ks = n * D;
    RowGuard g{INT64_MIN, INT64_MAX, 0, 0, true};
    if (GUARD) {
        const Bind bi = bind_wave(t, (uint64_t)idx);
        const Bind bs = bind_wave(t, (uint64_t)src);
        const Bind bd = bind_wave(t, (uint64_t)dst);
        Ki = clip_prefix(bi, (uint64_t)idx, n, 8);
        Ks = clip_prefix(bs, (uint64_t)src, n * D, W);
        g = row_guard(bd, (uint64_t)dst, rb);
    }
    const uint32_t lane = threadIdx.x & 63u;
    const uint32_t G = 1u << glog2;
    const uint32_t lir = lane & (G - 1);
    const uint32_t riw = lane >> glog2;
    const uint64_t rpw = 64u >> glog2;
    const uint64_t wave = ((uint64_t)blockIdx.x * GBLOCK + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * GBLOCK) >> 6;
    FaultAcc acc;
    for (uint64_t r0 = wave * rpw * GROWS; r0 < n; r0 += nwaves * rpw * GROWS) {
        int64_t iv[GROWS];
        bool live[GROWS];
#pragma unroll
        for (int u = 0; u < GROWS; ++u) {
            const uint64_t i = r0 + u * rpw + riw;
            live[u] = i < n;
            const bool iok = !GUARD || i < Ki;
            iv[u] = (live[u] && iok) ? idx[i] : 0;
            if (GUARD && live[u] && !iok && lir == 0) acc.note((i * D) << 2);
        }
#pragma unroll
        for (int u = 0; u < GROWS; ++u) {
            if (!live[u]) continue;
            const uint64_t i = r0 + u * rpw + riw;
            const bool full = !GUARD || (g.rlo <= iv[u] && iv[u] <= g.rhi);
            uint8_t* drow = dst + (uint64_t)iv[u] * rb;
            const uint8_t* srow = src + i * rb;
            for (uint64_t ch = lir; ch < nch; ch += G) {
                const uint64_t e0 = i * D + ch * EPC;
                if (!ACC && full && (!GUARD || e0 + EPC <= Ks)) {
                    *reinterpret_cast<V*>(drow + ch * CW) = *reinterpret_cast<const V*>(srow + ch * CW);
                } else {
#pragma unroll
                    for (uint32_t k = 0; k < EPC; ++k) {
                        const uint64_t col = ch * EPC + k;
                        const uint64_t e = e0 + k;
                        E val = 0;
                        if (!GUARD || e < Ks) val = *reinterpret_cast<const E*>(srow + col * W);
                        else acc.note((e << 2) | 1u);
                        if (full || elem_ok(g, iv[u], rb, col, W)) {
                            if (ACC) {
                                F fv;
                                __builtin_memcpy(&fv, &val, W);
                                unsafeAtomicAdd(reinterpret_cast<F*>(drow + col * W), fv);
                            } else {
                                *reinterpret_cast<E*>(drow + col * W) = val;
                            }
                        } else {
                            acc.note((e << 2) | 2u);
                        }
                    }
                }
            }
        }
    }
    if (GUARD && logon) {
        fold_faults(acc, log, [&](unsigned long long key) {
            const unsigned long long elem = key >> 2;
            const uint32_t operand = (uint32_t)(key & 3u);
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
            record_at(t, log, seq, elem, operand, A, w, ACC ? 5 : 4);
        });
    }
}

__global__ void k_log_reset(DevLog* log) {
    log->count = 0;
    log->first_seq = ~0ull;
    log->first_elem = 0;
    log->first_addr = 0;
    log->first_width = 0;
    log->first_op = 0;
    log->first_operand = 0;
    log->first_verdict = 0;
    log->first_owner = -1;
    log->reserved = 0;
    log->s_minkey = ~0ull;
    log->s_count = 0;
    log->s_done = 0;
    log->s_pad = 0;
}

hipError_t launch_log_reset(DevLog* log, hipStream_t s) {
    hipLaunchKernelGGL(k_log_reset, dim3(1), dim3(1), 0, s, log);
    return hipGetLastError();
}

// Lanes per row: enough to cover the row's chunks, at most a wave.
static uint32_t lanes_log2(uint64_t nch) {
    uint32_t l = 0;
    while (l < 6 && (1ull << l) < nch) ++l;
    return l;
}

static uint32_t rows_grid(uint64_t n, uint32_t glog2, const DevInfo& d) {
    const uint64_t rows_per_block = (uint64_t)(GBLOCK / 64) * (64u >> glog2) * GROWS;
    uint64_t want = (n + rows_per_block - 1) / rows_per_block;
    const uint64_t cap = (uint64_t)d.num_cu * 8;
    if (want < 1) want = 1;
    return (uint32_t)(want < cap ? want : cap);
}

template <bool G, int W>
static void gather_w(const DevTable& t, DevLog* log, void* out, const void* tab, uint64_t rb,
                     const int64_t* idx, uint64_t n, unsigned long long seq, int logon,
                     const DevInfo& d, hipStream_t s) {
    const bool v16 = rb % 16 == 0 && (((uint64_t)out | (uint64_t)tab) & 15) == 0;
    const uint64_t nch = v16 ? rb / 16 : rb / W;
    const uint32_t gl = lanes_log2(nch);
    const dim3 grid(rows_grid(n, gl, d)), block(GBLOCK);
    if (v16)
        hipLaunchKernelGGL((k_gather<G, 16, W>), grid, block, 0, s, t, log, (uint8_t*)out,
                           (const uint8_t*)tab, rb, idx, n, seq, logon, gl);
    else
        hipLaunchKernelGGL((k_gather<G, W, W>), grid, block, 0, s, t, log, (uint8_t*)out,
                           (const uint8_t*)tab, rb, idx, n, seq, logon, gl);
}

hipError_t launch_gather(bool guard, const DevTable& t, DevLog* log, void* out, const void* tab,
                         uint64_t rb, const int64_t* idx, uint64_t n, uint32_t w,
                         unsigned long long seq, int logon, const DevInfo& d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (guard) {
        if (w == 4) gather_w<true, 4>(t, log, out, tab, rb, idx, n, seq, logon, d, s);
        else gather_w<true, 8>(t, log, out, tab, rb, idx, n, seq, logon, d, s);
    } else {
        if (w == 4) gather_w<false, 4>(t, log, out, tab, rb, idx, n, seq, logon, d, s);
        else gather_w<false, 8>(t, log, out, tab, rb, idx, n, seq, logon, d, s);
    }
    return hipGetLastError();
}

template <bool G, int W, bool ACC>
static void scatter_w(const DevTable& t, DevLog* log, void* dst, uint64_t rb, const int64_t* idx,
                      const void* src, uint64_t n, unsigned long long seq, int logon,
                      const DevInfo& d, hipStream_t s) {
    const bool v16 = !ACC && rb % 16 == 0 && (((uint64_t)dst | (uint64_t)src) & 15) == 0;
    const uint64_t nch = v16 ? rb / 16 : rb / W;
    const uint32_t gl = lanes_log2(nch);
    const dim3 grid(rows_grid(n, gl, d)), block(GBLOCK);
    if (v16)
        hipLaunchKernelGGL((k_scatter<G, 16, W, ACC>), grid, block, 0, s, t, log, (uint8_t*)dst, rb,
                           idx, (const uint8_t*)src, n, seq, logon, gl);
    else
        hipLaunchKernelGGL((k_scatter<G, W, W, ACC>), grid, block, 0, s, t, log, (uint8_t*)dst, rb,
                           idx, (const uint8_t*)src, n, seq, logon, gl);
}

hipError_t launch_scatter(bool guard, const DevTable& t, DevLog* log, void* dst, uint64_t rb,
                          const int64_t* idx, const void* src, uint64_t n, uint32_t w,
                          int accumulate, unsigned long long seq, int logon, const DevInfo& d,
                          hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (accumulate)
        return launch_scatter_add(guard, t, log, dst, rb, idx, src, n, w, seq, logon, d, s);
    if (guard) {
        if (w == 4) scatter_w<true, 4, false>(t, log, dst, rb, idx, src, n, seq, logon, d, s);
        else scatter_w<true, 8, false>(t, log, dst, rb, idx, src, n, seq, logon, d, s);
    } else {
        if (w == 4) scatter_w<false, 4, false>(t, log, dst, rb, idx, src, n, seq, logon, d, s);
        else scatter_w<false, 8, false>(t, log, dst, rb, idx, src, n, seq, logon, d, s);
    }
    return hipGetLastError();
}

}  // namespace agile
