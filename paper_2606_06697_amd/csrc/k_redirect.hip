// Redirecting guard policies (the paper's "sink", "report" and "remap_or", Section V-E): a pass
// after a guarded kernel that gives each denied access its redirected effect.
//
// The guarded kernels run unchanged (denied loads read zero, denied stores are dropped, every
// denial counted). For SINK, REPORT and REMAP the library then runs one of these kernels on the
// same stream:
//  * SINK: a denied access of width w at exact address A goes to the quarantine slot
//    q + ((A mod 2^64) mod qsize), rounded down to a multiple of w (qsize a power of two);
//  * REPORT: a denied access is performed at A itself when [A, A+w) lies inside one registered
//    range of the handle's table (any kind) that was inserted as backed memory, and stays
//    suppressed otherwise;
//  * REMAP ("remap_or", kept safe: the target is a live user allocation, its own argument's):
//    with lo' = lo rounded up to w and m the largest multiple of w not above hi - lo', the
//    access goes to lo' + ((A - lo') mod m) rounded down to w; no binding leaves it suppressed.
// Copy and triad deny a suffix of their elements, so the pass walks that suffix. Row kernels
// ran on the rows whose index is readable (a prefix); the pass re-runs every element of those
// rows that had a denied access, with the redirects, and runs the remaining rows completely,
// counting their denials into the launch's scratch (the finishing kernel then writes the log).
#include "launch.h"

#pragma clang fp contract(off)

namespace agile {

constexpr int XBLOCK = 256;

// Where a denied access of the argument bound to b goes, or null when it stays suppressed.
__device__ inline uint8_t* redirect_to(const DevTable& t, const Redirect& r, Bind b, __int128 A,
                                       uint32_t w) {
    if (r.mode == REDIRECT_SINK) return r.q + (((uint64_t)A & r.qmask) & ~(uint64_t)(w - 1));
    if (r.mode == REDIRECT_REMAP) {
        if (b.hi <= b.lo) return nullptr;
        const __int128 lo = ((__int128)b.lo + (w - 1)) / w * w;
        if (lo >= (__int128)b.hi) return nullptr;
        const __int128 m = ((__int128)b.hi - lo) / w * w;
        if (m == 0) return nullptr;
        __int128 off = (A - lo) % m;
        if (off < 0) off += m;
        return reinterpret_cast<uint8_t*>((uint64_t)(lo + off / w * w));
    }
    if (A < 0 || A + (__int128)w > ((__int128)1 << 64)) return nullptr;
    const uint64_t a = (uint64_t)A;
    const int64_t bk = bucket_search_lane(t, a);
    if (bk < 0) return nullptr;
    const PairRec rec = load_rec(t.rec + bk);
    const bool second = rec.base1 <= a;
    const uint64_t end = second ? rec.end1 : rec.end0;
    if (a >= end || (uint64_t)w > end - a) return nullptr;
    if (!((t.backed[bk] >> (second ? 1 : 0)) & 1u)) return nullptr;  // no memory promised there
    return reinterpret_cast<uint8_t*>(a);
}

template <typename E>
__device__ __forceinline__ E rload(const DevTable& t, const Redirect& r, Bind b, __int128 A) {
    const uint8_t* p = redirect_to(t, r, b, A, sizeof(E));
    return p ? *reinterpret_cast<const E*>(p) : E(0);
}

template <typename E>
__device__ __forceinline__ void rstore(const DevTable& t, const Redirect& r, Bind b, __int128 A,
                                       E v) {
    uint8_t* p = redirect_to(t, r, b, A, sizeof(E));
    if (p) *reinterpret_cast<E*>(p) = v;
}

template <typename F>
__device__ __forceinline__ void radd(const DevTable& t, const Redirect& r, Bind b, __int128 A,
                                     F v) {
    uint8_t* p = redirect_to(t, r, b, A, sizeof(F));
    if (p) atomicAdd(reinterpret_cast<F*>(p), v);
}

// Copy: bytes k >= min(Ks, Kd). Below Kd the destination is allowed (the kernel wrote zero
// where the source was denied); from Kd on the store is redirected.
__global__ __launch_bounds__(XBLOCK) void k_copy_fix(DevTable t, Redirect r, Bind bs, Bind bd,
                                                     uint8_t* dst, const uint8_t* src, uint64_t n,
                                                     uint64_t Ks, uint64_t Kd) {
    const uint64_t k0 = Ks < Kd ? Ks : Kd;
    for (uint64_t k = k0 + (uint64_t)blockIdx.x * XBLOCK + threadIdx.x; k < n;
         k += (uint64_t)gridDim.x * XBLOCK) {
        const uint8_t v = k < Ks ? src[k] : rload<uint8_t>(t, r, bs, (__int128)(uint64_t)src + k);
        if (k < Kd) dst[k] = v;
        else rstore<uint8_t>(t, r, bd, (__int128)(uint64_t)dst + k, v);
    }
}

__global__ __launch_bounds__(XBLOCK) void k_triad_fix(DevTable t, Redirect r, Bind ba, Bind bb,
                                                      Bind bc, float* a, const float* b,
                                                      const float* c, float s, uint64_t n,
                                                      uint64_t Ka, uint64_t Kb, uint64_t Kc) {
    uint64_t i0 = Ka < Kb ? Ka : Kb;
    i0 = i0 < Kc ? i0 : Kc;
    for (uint64_t i = i0 + (uint64_t)blockIdx.x * XBLOCK + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * XBLOCK) {
        const float bv = i < Kb ? b[i] : rload<float>(t, r, bb, (__int128)(uint64_t)b + 4 * i);
        const float cv = i < Kc ? c[i] : rload<float>(t, r, bc, (__int128)(uint64_t)c + 4 * i);
        const float v = __fadd_rn(bv, __fmul_rn(s, cv));
        if (i < Ka) a[i] = v;
        else rstore<float>(t, r, ba, (__int128)(uint64_t)a + 4 * i, v);
    }
}

// Row kernels. OP: 0 gather (table row-addressed, out contiguous), 1 scatter, 2 scatter-add
// (src contiguous, dst row-addressed). rg: the call's guard over all n rows; rows below
// nmain = rg.ki were run by the guarded kernel.
template <int OP, typename F>
__global__ __launch_bounds__(XBLOCK) void k_rows_fix(DevTable t, DevLog* log, Redirect r,
                                                     RowBinds bb, uint8_t* cont, uint8_t* rowp,
                                                     uint64_t rb, const int64_t* idx, uint64_t n,
                                                     RowsGuard rg) {
    constexpr uint32_t W = sizeof(F);
    const uint64_t D = rb / W;
    const uint64_t nmain = rg.ki, Kc = rg.kc;
    FaultAcc acc;
    for (uint64_t i = (uint64_t)blockIdx.x * XBLOCK + threadIdx.x; i < n;
         i += (uint64_t)gridDim.x * XBLOCK) {
        const bool ran = i < nmain;
        int64_t iv;
        if (ran) {
            iv = idx[i];
            // nothing was denied in this row
            if ((i + 1) * D <= Kc && rg.g.rlo <= iv && iv <= rg.g.rhi) continue;
        } else {
            acc.note((i * D) << 2);  // the index load
            iv = rload<int64_t>(t, r, bb.idx, (__int128)(uint64_t)idx + (__int128)(8 * i));
        }
        for (uint64_t col = 0; col < D; ++col) {
            const uint64_t e = i * D + col;
            const bool cok = e < Kc;
            const bool rok = elem_ok(rg.g, iv, rb, col, W);
            if (ran && cok && rok) continue;  // done by the guarded kernel
            const __int128 Ac = (__int128)(uint64_t)cont + (__int128)(e * W);
            const __int128 Ar = (__int128)(uint64_t)rowp + (__int128)iv * (__int128)rb +
                                (__int128)(col * W);
            if (OP == 0) {
                // load table (operand 1), store out (operand 2)
                if (!ran && !rok) acc.note((e << 2) | 1u);
                const F v = rok ? *reinterpret_cast<const F*>(rowp + (uint64_t)iv * rb + col * W)
                                : rload<F>(t, r, bb.row, Ar);
                if (!ran && !cok) acc.note((e << 2) | 2u);
                if (cok) *reinterpret_cast<F*>(cont + e * W) = v;
                else rstore<F>(t, r, bb.cont, Ac, v);
            } else {
                // load src (operand 1), store or add into dst (operand 2)
                if (!ran && !cok) acc.note((e << 2) | 1u);
                const F v = cok ? *reinterpret_cast<const F*>(cont + e * W)
                                : rload<F>(t, r, bb.cont, Ac);
                if (!ran && !rok) acc.note((e << 2) | 2u);
                F* dp = reinterpret_cast<F*>(rowp + (uint64_t)iv * rb + col * W);
                if (OP == 1) {
                    if (rok) *dp = v;
                    else rstore<F>(t, r, bb.row, Ar, v);
                } else if (rok) {
                    // the guarded kernel added zero for the denied source element (a row that
                    // it did not run adds its whole value here)
                    atomicAdd(dp, v);
                } else {
                    radd<F>(t, r, bb.row, Ar, v);
                }
            }
        }
    }
    fold_faults(acc, log);
}

static uint32_t fix_grid(uint64_t n, const DevInfo& d) {
    uint64_t g = (n + XBLOCK - 1) / XBLOCK;
    const uint64_t cap = (uint64_t)d.num_cu * 8;
    if (g > cap) g = cap;
    return (uint32_t)(g ? g : 1);
}

hipError_t launch_copy_fix(const DevTable& t, const Redirect& r, Bind bs, Bind bd, void* dst,
                           const void* src, uint64_t n, uint64_t Ks, uint64_t Kd, const DevInfo& d,
                           hipStream_t s) {
    const uint64_t k0 = Ks < Kd ? Ks : Kd;
    if (k0 >= n) return hipSuccess;
    hipLaunchKernelGGL(k_copy_fix, dim3(fix_grid(n - k0, d)), dim3(XBLOCK), 0, s, t, r, bs, bd,
                       (uint8_t*)dst, (const uint8_t*)src, n, Ks, Kd);
    return hipGetLastError();
}

hipError_t launch_triad_fix(const DevTable& t, const Redirect& r, Bind ba, Bind bb, Bind bc,
                            float* a, const float* b, const float* c, float sc, uint64_t n,
                            uint64_t Ka, uint64_t Kb, uint64_t Kc, const DevInfo& d,
                            hipStream_t s) {
    uint64_t i0 = Ka < Kb ? Ka : Kb;
    i0 = i0 < Kc ? i0 : Kc;
    if (i0 >= n) return hipSuccess;
    hipLaunchKernelGGL(k_triad_fix, dim3(fix_grid(n - i0, d)), dim3(XBLOCK), 0, s, t, r, ba, bb,
                       bc, a, b, c, sc, n, Ka, Kb, Kc);
    return hipGetLastError();
}

hipError_t launch_rows_fix(int op, const DevTable& t, DevLog* log, const Redirect& r,
                           const RowBinds& bb, void* cont, void* rowp, uint64_t rb,
                           const int64_t* idx, uint64_t n, const RowsGuard& rg, uint32_t w,
                           const DevInfo& d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    const dim3 grid(fix_grid(n, d)), block(XBLOCK);
    uint8_t* c = (uint8_t*)cont;
    uint8_t* p = (uint8_t*)rowp;
    if (w == 4) {
        if (op == 0) hipLaunchKernelGGL((k_rows_fix<0, float>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
        else if (op == 1) hipLaunchKernelGGL((k_rows_fix<1, float>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
        else hipLaunchKernelGGL((k_rows_fix<2, float>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
    } else {
        if (op == 0) hipLaunchKernelGGL((k_rows_fix<0, double>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
        else if (op == 1) hipLaunchKernelGGL((k_rows_fix<1, double>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
        else hipLaunchKernelGGL((k_rows_fix<2, double>), grid, block, 0, s, t, log, r, bb, c, p, rb, idx, n, rg);
    }
    return hipGetLastError();
}

}  // namespace agile
