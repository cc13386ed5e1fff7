// Guarded gather and scatter(-add) over rows (kernel memory guard of AgileOS Section V-E).
//
// out[i,:] = T[idx[i],:]  /  dst[idx[i],:] (+)= src[i,:], rows of `rb` bytes, elements of W bytes.
// The three pointer arguments are bound once per call (host lookup in the table the launch is
// ordered after) and reach the kernel as scalars. The index and the contiguous operand have
// prefix-shaped allowed sets; for the row-addressed operand the binding becomes an index
// interval [rlo, rhi] of rows that lie wholly inside the allocation, so the per-row guard is
// two signed compares of the loaded index against scalars. Rows outside it (hostile indices, or a table pointer that is not
// row-aligned with its allocation's ends) take an exact 128-bit per-element path. Denials are
// counted per lane, reduced per wave and folded into the handle's log (count and smallest
// (element, operand) key); a one-thread kernel after the launch writes that denial's record.
// GUARD=false compiles the same loops with no binding and no compare (the unguarded twin).
#include "launch.h"

namespace agile {

constexpr int GBLOCK = 256;

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

// Lane layout shared by both kernels: a row is covered by G = 2^glog2 lanes (one CW-byte chunk
// each per pass), a wave covers 64/G rows, and each lane keeps R rows in flight. WIDE kernels
// give a whole wave to each row (G = 64), so a row's index is wave-uniform and its guard test
// runs on scalar registers.
struct RowLanes {
    uint32_t G, lir, riw;
    uint64_t rpw, wave, nwaves;
    __device__ explicit RowLanes(uint32_t glog2) {
        const uint32_t lane = threadIdx.x & 63u;
        G = 1u << glog2;
        lir = lane & (G - 1);
        riw = lane >> glog2;
        rpw = 64u >> glog2;
        wave = ((uint64_t)blockIdx.x * GBLOCK + threadIdx.x) >> 6;
        nwaves = ((uint64_t)gridDim.x * GBLOCK) >> 6;
    }
};

// Per pass, every lane first issues the loads of all its rows that pass the fast test, then the
// matching stores, and only then runs the exact per-element path for the rest, so the guard
// adds no wait between the R independent loads. The fast test of row i is i < nfast (its index
// is readable and its contiguous-operand row is wholly allowed: both are prefixes) and
// rlo <= idx[i] <= rhi (its row-addressed row is wholly inside the binding).
template <bool GUARD, bool WIDE, int R>
__device__ __forceinline__ void load_rows(const RowLanes& L, uint64_t r0, uint64_t nfast,
                                          const int64_t* idx, int64_t (&iv)[R]) {
#pragma unroll
    for (int u = 0; u < R; ++u) {
        const uint64_t i = r0 + u * L.rpw + L.riw;
        // narrow rows: each index is read once, non-temporally (kept out of L2 and the MALL,
        // which then hold more table lines); wide rows read one index per wave
        int64_t x = i < nfast ? (WIDE ? idx[i] : __builtin_nontemporal_load(idx + i)) : 0;
        if (WIDE) x = (int64_t)uniform_u64((uint64_t)x);
        iv[u] = x;
    }
}

template <bool GUARD, int CW, int W, int R, bool WIDE>
__global__ __launch_bounds__(GBLOCK) void k_gather(DevTable t, DevLog* log, uint8_t* out,
                                                    const uint8_t* T, uint64_t rb,
                                                    const int64_t* idx, uint64_t n, RowsGuard rg,
                                                    unsigned long long seq, int logon,
                                                    uint32_t glog2) {
    using V = typename Word<CW>::T;
    using E = typename Word<W>::T;
    constexpr uint32_t EPC = CW / W;  // elements per chunk
    const uint64_t D = rb / W;
    const uint64_t nch = rb / CW;
    const uint64_t Ki = rg.ki, Ko = rg.kc, nfast = rg.nfast;
    const RowGuard g = rg.g;
    const RowLanes L(WIDE ? 6u : glog2);
    FaultAcc acc;
    for (uint64_t r0 = L.wave * L.rpw * R; r0 < n; r0 += L.nwaves * L.rpw * R) {
        int64_t iv[R];
        load_rows<GUARD, WIDE, R>(L, r0, nfast, idx, iv);
        for (uint64_t c0 = 0; c0 < nch; c0 += L.G) {
            const uint64_t ch = c0 + L.lir;
            V v[R];
            uint32_t slow = 0;  // rows of this lane whose chunk takes the exact path
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint64_t i = r0 + u * L.rpw + L.riw;
                const bool on = i < n && ch < nch;
                const bool fast = on && (!GUARD || (i < nfast && g.rlo <= iv[u] && iv[u] <= g.rhi));
                if (fast) v[u] = *reinterpret_cast<const V*>(T + (uint64_t)iv[u] * rb + ch * CW);
                if (on && !fast) slow |= 1u << u;
            }
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint64_t i = r0 + u * L.rpw + L.riw;
                if (i < n && ch < nch && !((slow >> u) & 1u))
                    __builtin_nontemporal_store(v[u], reinterpret_cast<V*>(out + i * rb + ch * CW));
            }
            if (!GUARD || slow == 0) continue;
#pragma unroll 1
            for (int u = 0; u < R; ++u) {
                if (!((slow >> u) & 1u)) continue;
                const uint64_t i = r0 + u * L.rpw + L.riw;
                const bool iok = i < Ki;
                if (!iok && ch == 0) acc.note((i * D) << 2);  // one 8-byte index load per row
                const int64_t x = iok ? idx[i] : 0;
                const bool full = g.rlo <= x && x <= g.rhi;
                const uint8_t* trow = T + (uint64_t)x * rb;
                uint8_t* orow = out + i * rb;
#pragma unroll 1
                for (uint32_t k = 0; k < EPC; ++k) {
                    const uint64_t col = ch * EPC + k;
                    const uint64_t e = i * D + col;
                    E val = 0;
                    if (full || elem_ok(g, x, rb, col, W)) {
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
    if (GUARD && logon) fold_faults(acc, log);
}

// Plain scatter (no accumulation): with duplicate indices one of the writers wins.
template <bool GUARD, int CW, int W, int R, bool WIDE>
__global__ __launch_bounds__(GBLOCK) void k_scatter(DevTable t, DevLog* log, uint8_t* dst,
                                                     uint64_t rb, const int64_t* idx,
                                                     const uint8_t* src, uint64_t n, RowsGuard rg,
                                                     unsigned long long seq, int logon,
                                                     uint32_t glog2) {
    using V = typename Word<CW>::T;
    using E = typename Word<W>::T;
    constexpr uint32_t EPC = CW / W;
    const uint64_t D = rb / W;
    const uint64_t nch = rb / CW;
    const uint64_t Ki = rg.ki, Ks = rg.kc, nfast = rg.nfast;
    const RowGuard g = rg.g;
    const RowLanes L(WIDE ? 6u : glog2);
    FaultAcc acc;
    for (uint64_t r0 = L.wave * L.rpw * R; r0 < n; r0 += L.nwaves * L.rpw * R) {
        int64_t iv[R];
        load_rows<GUARD, WIDE, R>(L, r0, nfast, idx, iv);
        for (uint64_t c0 = 0; c0 < nch; c0 += L.G) {
            const uint64_t ch = c0 + L.lir;
            V v[R];
            uint32_t slow = 0;
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint64_t i = r0 + u * L.rpw + L.riw;
                const bool on = i < n && ch < nch;
                const bool fast = on && (!GUARD || (i < nfast && g.rlo <= iv[u] && iv[u] <= g.rhi));
                if (fast) v[u] = *reinterpret_cast<const V*>(src + i * rb + ch * CW);
                if (on && !fast) slow |= 1u << u;
            }
#pragma unroll
            for (int u = 0; u < R; ++u) {
                const uint64_t i = r0 + u * L.rpw + L.riw;
                if (i < n && ch < nch && !((slow >> u) & 1u))
                    *reinterpret_cast<V*>(dst + (uint64_t)iv[u] * rb + ch * CW) = v[u];
            }
            if (!GUARD || slow == 0) continue;
#pragma unroll 1
            for (int u = 0; u < R; ++u) {
                if (!((slow >> u) & 1u)) continue;
                const uint64_t i = r0 + u * L.rpw + L.riw;
                const bool iok = i < Ki;
                if (!iok && ch == 0) acc.note((i * D) << 2);
                const int64_t x = iok ? idx[i] : 0;
                const bool full = g.rlo <= x && x <= g.rhi;
                uint8_t* drow = dst + (uint64_t)x * rb;
                const uint8_t* srow = src + i * rb;
#pragma unroll 1
                for (uint32_t k = 0; k < EPC; ++k) {
                    const uint64_t col = ch * EPC + k;
                    const uint64_t e = i * D + col;
                    E val = 0;
                    if (e < Ks) val = *reinterpret_cast<const E*>(srow + col * W);
                    else acc.note((e << 2) | 1u);
                    if (full || elem_ok(g, x, rb, col, W)) {
                        *reinterpret_cast<E*>(drow + col * W) = val;
                    } else {
                        acc.note((e << 2) | 2u);
                    }
                }
            }
        }
    }
    if (GUARD && logon) fold_faults(acc, log);
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
}

hipError_t launch_log_reset(DevLog* log, hipStream_t s) {
    hipLaunchKernelGGL(k_log_reset, dim3(1), dim3(1), 0, s, log);
    return hipGetLastError();
}

// Finishing step of a row kernel's launch: adds the launch's denial count to the log and, if
// the log holds no record yet, records the smallest key (its address and reason).
__global__ void k_fault_finish(DevTable t, DevLog* log, FaultSite f, unsigned long long seq) {
    // device-scope atomics: the launch's waves folded into these from every XCD
    const unsigned long long total = atomicAdd(&log->s_count, 0ull);
    if (total == 0) return;
    const unsigned long long key = atomicMin(&log->s_minkey, ~0ull);
    atomicAdd(&log->count, total);
    const unsigned long long elem = key >> 2;
    const uint32_t operand = (uint32_t)(key & 3u);
    const uint64_t i = elem / f.D, col = elem % f.D;
    const int64_t* idx = reinterpret_cast<const int64_t*>(f.idx);
    __int128 A;
    uint32_t w = f.w;
    if (operand == 0) {
        A = (__int128)f.idx + (__int128)(8 * i);
        w = 8;
    } else if (operand == f.row_operand) {
        const int64_t v = i < f.ki ? idx[i] : 0;
        A = (__int128)f.rowp + (__int128)v * (__int128)f.rb + (__int128)(col * f.w);
    } else {
        A = (__int128)f.cont + (__int128)elem * f.w;
    }
    record_at(t, log, seq, elem, operand, A, w, f.op);
    atomicExch(&log->s_count, 0ull);
    atomicExch(&log->s_minkey, ~0ull);
}

hipError_t launch_fault_finish(const DevTable& t, DevLog* log, const FaultSite& f,
                               unsigned long long seq, hipStream_t s) {
    hipLaunchKernelGGL(k_fault_finish, dim3(1), dim3(1), 0, s, t, log, f, seq);
    return hipGetLastError();
}

FaultSite rows_fault_site(uint32_t op, uint32_t w, uint32_t row_operand, uint64_t rb, uint64_t ki,
                          const void* idx, const void* cont, const void* rowp) {
    FaultSite f{};
    f.op = op;
    f.w = w;
    f.row_operand = row_operand;
    f.D = rb / w;
    f.rb = rb;
    f.ki = ki;
    f.idx = (uint64_t)idx;
    f.cont = (uint64_t)cont;
    f.rowp = (uint64_t)rowp;
    return f;
}

// Lanes per row: enough to cover the row's chunks, at most a wave.
static uint32_t lanes_log2(uint64_t nch) {
    uint32_t l = 0;
    while (l < 6 && (1ull << l) < nch) ++l;
    return l;
}

// Rows in flight per lane: more for narrow rows, where each load is a lone random access, and
// for rows that take a whole wave, where the row's index and guard live in scalar registers.
constexpr int R_NARROW = 8, R_WIDE = 4, R_ROWWAVE = 8;

// Grid: 4 workgroups per CU, the measured best of 1-16 for rows of a wave or more. Narrow rows
// (the random-access case) go in one pass instead, with as many workgroups as the rows need:
// 1.437 ms against 1.458 ms for 2^26 four-byte rows. The same change made the embedding's
// whole-wave rows slower (0.240 ms against 0.216 ms), so those keep the cap.
static uint32_t rows_grid(uint64_t n, uint32_t glog2, int R, const DevInfo& d,
                          bool one_pass = false) {
    const uint64_t rows_per_block = (uint64_t)(GBLOCK / 64) * (64u >> glog2) * R;
    uint64_t want = (n + rows_per_block - 1) / rows_per_block;
    const uint64_t cap = one_pass ? (1ull << 30) : (uint64_t)d.num_cu * 4;
    if (want < 1) want = 1;
    return (uint32_t)(want < cap ? want : cap);
}

template <bool G, int CW, int W>
static void gather_cw(const DevTable& t, DevLog* log, void* out, const void* tab, uint64_t rb,
                      const int64_t* idx, uint64_t n, const RowsGuard& rg, unsigned long long seq,
                      int logon, const DevInfo& d, hipStream_t s) {
    const uint32_t gl = lanes_log2(rb / CW);
    const dim3 block(GBLOCK);
    if (gl == 6)
        hipLaunchKernelGGL((k_gather<G, CW, W, R_ROWWAVE, true>), dim3(rows_grid(n, gl, R_ROWWAVE, d)),
                           block, 0, s, t, log, (uint8_t*)out, (const uint8_t*)tab, rb, idx, n, rg, seq,
                           logon, gl);
    else if (rb <= 16)
        hipLaunchKernelGGL((k_gather<G, CW, W, R_NARROW, false>), dim3(rows_grid(n, gl, R_NARROW, d, true)),
                           block, 0, s, t, log, (uint8_t*)out, (const uint8_t*)tab, rb, idx, n, rg, seq,
                           logon, gl);
    else
        hipLaunchKernelGGL((k_gather<G, CW, W, R_WIDE, false>), dim3(rows_grid(n, gl, R_WIDE, d)),
                           block, 0, s, t, log, (uint8_t*)out, (const uint8_t*)tab, rb, idx, n, rg, seq,
                           logon, gl);
}

template <bool G, int W>
static void gather_w(const DevTable& t, DevLog* log, void* out, const void* tab, uint64_t rb,
                     const int64_t* idx, uint64_t n, const RowsGuard& rg, unsigned long long seq,
                     int logon, const DevInfo& d, hipStream_t s) {
    if (rb % 16 == 0 && (((uint64_t)out | (uint64_t)tab) & 15) == 0)
        gather_cw<G, 16, W>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
    else
        gather_cw<G, W, W>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
}

hipError_t launch_gather(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* out,
                         const void* tab, uint64_t rb, const int64_t* idx, uint64_t n, uint32_t w,
                         unsigned long long seq, int logon, const DevInfo& d, hipStream_t s,
                         bool finish) {
    if (n == 0) return hipSuccess;
    if (guard) {
        const RowsGuard rg = rows_guard(binds[0], binds[2], binds[1], (uint64_t)idx, (uint64_t)out,
                                        (uint64_t)tab, n, rb, w);
        if (w == 4) gather_w<true, 4>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
        else gather_w<true, 8>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
        if (logon && finish)
            return launch_fault_finish(t, log, rows_fault_site(3 /*OP_GATHER*/, w, 1, rb, rg.ki, idx,
                                                                 out, tab), seq, s);
    } else {
        const RowsGuard rg = rows_open(n, rb, w);
        if (w == 4) gather_w<false, 4>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
        else gather_w<false, 8>(t, log, out, tab, rb, idx, n, rg, seq, logon, d, s);
    }
    return hipGetLastError();
}

template <bool G, int CW, int W>
static void scatter_cw(const DevTable& t, DevLog* log, void* dst, uint64_t rb, const int64_t* idx,
                       const void* src, uint64_t n, const RowsGuard& rg, unsigned long long seq,
                       int logon, const DevInfo& d, hipStream_t s) {
    const uint32_t gl = lanes_log2(rb / CW);
    const dim3 block(GBLOCK);
    if (gl == 6)
        hipLaunchKernelGGL((k_scatter<G, CW, W, R_ROWWAVE, true>), dim3(rows_grid(n, gl, R_ROWWAVE, d)),
                           block, 0, s, t, log, (uint8_t*)dst, rb, idx, (const uint8_t*)src, n, rg, seq,
                           logon, gl);
    else if (rb <= 16)
        hipLaunchKernelGGL((k_scatter<G, CW, W, R_NARROW, false>), dim3(rows_grid(n, gl, R_NARROW, d)),
                           block, 0, s, t, log, (uint8_t*)dst, rb, idx, (const uint8_t*)src, n, rg, seq,
                           logon, gl);
    else
        hipLaunchKernelGGL((k_scatter<G, CW, W, R_WIDE, false>), dim3(rows_grid(n, gl, R_WIDE, d)),
                           block, 0, s, t, log, (uint8_t*)dst, rb, idx, (const uint8_t*)src, n, rg, seq,
                           logon, gl);
}

template <bool G, int W>
static void scatter_w(const DevTable& t, DevLog* log, void* dst, uint64_t rb, const int64_t* idx,
                      const void* src, uint64_t n, const RowsGuard& rg, unsigned long long seq,
                      int logon, const DevInfo& d, hipStream_t s) {
    if (rb % 16 == 0 && (((uint64_t)dst | (uint64_t)src) & 15) == 0)
        scatter_cw<G, 16, W>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    else
        scatter_cw<G, W, W>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
}

hipError_t launch_scatter(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* dst,
                          uint64_t rb, const int64_t* idx, const void* src, uint64_t n, uint32_t w,
                          int accumulate, unsigned long long seq, int logon, void* scratch,
                          const DevInfo& d, hipStream_t s, bool finish) {
    if (n == 0) return hipSuccess;
    if (accumulate)
        return launch_scatter_add(guard, t, log, binds, dst, rb, idx, src, n, w, seq, logon,
                                  scratch, d, s, finish, accumulate == 2);
    if (guard) {
        const RowsGuard rg = rows_guard(binds[0], binds[1], binds[2], (uint64_t)idx, (uint64_t)src,
                                        (uint64_t)dst, n, rb, w);
        if (w == 4) scatter_w<true, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_w<true, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        if (logon && finish)
            return launch_fault_finish(t, log, rows_fault_site(4 /*OP_SCATTER*/, w, 2, rb, rg.ki, idx,
                                                                 src, dst), seq, s);
    } else {
        const RowsGuard rg = rows_open(n, rb, w);
        if (w == 4) scatter_w<false, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_w<false, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    }
    return hipGetLastError();
}

}  // namespace agile
