// Guarded streaming kernels: copy and the fp32 triad a = b + s*c (kernel memory guard of
// AgileOS Section V-E, with the suppress-and-record policies).
//
// Each pointer argument is bound once per call to the USER range containing it (a host lookup
// in the table the launch is ordered after), which turns the guard into an allowed prefix
// length per argument, passed in kernel arguments and so held in scalar registers. The vector
// loop compares each lane's vector offset with that bound before touching memory; vectors past
// a bound take the per-element path (denied loads read zero, denied stores are dropped). The
// denial count and the first denial follow in closed form from the prefix lengths and are
// logged by one thread. GUARD=false compiles the same loop with no compare (the unguarded twin).
#include "launch.h"

#pragma clang fp contract(off)

namespace agile {

constexpr int SBLOCK = 128;
constexpr int SUNROLL = 1;  // vectors per thread per pass

typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int VW>
struct VecT;
template <>
struct VecT<16> {
    using T = u32x4;
    static __device__ __forceinline__ T zero() { return T{0u, 0u, 0u, 0u}; }
};
template <>
struct VecT<4> {
    using T = uint32_t;
    static __device__ __forceinline__ T zero() { return 0u; }
};
template <>
struct VecT<1> {
    using T = uint8_t;
    static __device__ __forceinline__ T zero() { return 0; }
};

__device__ inline void copy_bytes_slow(uint8_t* dst, const uint8_t* src, uint64_t b0, uint64_t b1,
                                       uint64_t Ks, uint64_t Kd) {
    for (uint64_t k = b0; k < b1; ++k) {
        uint8_t v = k < Ks ? src[k] : (uint8_t)0;
        if (k < Kd) dst[k] = v;
    }
}

// Ks, Kd: allowed byte prefixes of src and dst (n and n for the unguarded twin).
template <bool GUARD, int VW>
__global__ __launch_bounds__(SBLOCK) void k_copy(DevTable t, DevLog* log, uint8_t* __restrict__ dst,
                                                  const uint8_t* __restrict__ src, uint64_t n,
                                                  uint64_t Ks, uint64_t Kd,
                                                  unsigned long long seq, int logon) {
    using V = typename VecT<VW>::T;
    const uint64_t K = Ks < Kd ? Ks : Kd;
    const uint64_t nv = n / VW;
    const uint64_t tid = (uint64_t)blockIdx.x * SBLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * SBLOCK;
    const V* sv = reinterpret_cast<const V*>(src);
    V* dv = reinterpret_cast<V*>(dst);
    // Main loop: every vector of the pass lies inside both allowed prefixes (they are prefixes,
    // so one scalar bound covers the pass), so the loads issue unconditionally, back to back.
    const uint64_t lim = GUARD ? (K / VW < nv ? K / VW : nv) : nv;
    uint64_t v0 = tid;
    for (; v0 + (SUNROLL - 1) * stride < lim; v0 += SUNROLL * stride) {
        V x[SUNROLL];
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u) x[u] = __builtin_nontemporal_load(sv + v0 + u * stride);
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u) __builtin_nontemporal_store(x[u], dv + v0 + u * stride);
    }
    // Last pass of this thread: per-vector bounds, and the guard's per-element path.
    for (; v0 < nv; v0 += SUNROLL * stride) {
        V x[SUNROLL];
        bool m[SUNROLL];
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u) {
            const uint64_t v = v0 + u * stride;
            m[u] = v < nv && (!GUARD || (v + 1) * VW <= K);
            if (m[u]) x[u] = __builtin_nontemporal_load(sv + v);
        }
#pragma unroll
        for (int u = 0; u < SUNROLL; ++u)
            if (m[u]) __builtin_nontemporal_store(x[u], dv + (v0 + u * stride));
        if (GUARD) {
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                const uint64_t v = v0 + u * stride;
                if (v < nv && !m[u]) {
                    const uint64_t b0 = v * VW;
                    if (b0 >= Ks && b0 + VW <= Kd) {
                        dv[v] = VecT<VW>::zero();
                    } else if (b0 < Kd) {
                        copy_bytes_slow(dst, src, b0, b0 + VW, Ks, Kd);
                    }
                }
            }
        }
    }
    // tail bytes
    const uint64_t tb = nv * VW + tid;
    if (tb < n) {
        if (!GUARD) dst[tb] = src[tb];
        else copy_bytes_slow(dst, src, tb, tb + 1, Ks, Kd);
    }
    if (GUARD && logon && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t cnt = (n - Ks) + (n - Kd);
        if (cnt) {
            atomicAdd(&log->count, (unsigned long long)cnt);
            const uint32_t operand = Ks <= Kd ? 0u : 1u;
            const uint64_t k = operand ? Kd : Ks;
            const uint64_t A = (operand ? (uint64_t)dst : (uint64_t)src) + k;
            uint32_t v;
            int32_t o;
            reason_lane(t, A, 1, v, o);
            log_record(log, seq, k, operand, A, 1, 1 /*OP_COPY*/, v, o);
        }
    }
}

__device__ __forceinline__ float triad1(float b, float s, float c) {
    return __fadd_rn(b, __fmul_rn(s, c));
}

__device__ inline void triad_slow(float* a, const float* b, const float* c, float s, uint64_t i0,
                                  uint64_t i1, uint64_t Ka, uint64_t Kb, uint64_t Kc) {
    for (uint64_t i = i0; i < i1; ++i) {
        const float bv = i < Kb ? b[i] : 0.0f;
        const float cv = i < Kc ? c[i] : 0.0f;
        const float r = triad1(bv, s, cv);
        if (i < Ka) a[i] = r;
    }
}

// Ka, Kb, Kc: allowed element prefixes of the three operands (all n for the unguarded twin).
template <bool GUARD, int VE>
__global__ __launch_bounds__(SBLOCK) void k_triad(DevTable t, DevLog* log, float* a, const float* b,
                                                   const float* c, float s, uint64_t n,
                                                   uint64_t Ka, uint64_t Kb, uint64_t Kc,
                                                   unsigned long long seq, int logon) {
    uint64_t K = Ka < Kb ? Ka : Kb;
    K = K < Kc ? K : Kc;
    const uint64_t nv = n / VE;
    const uint64_t tid = (uint64_t)blockIdx.x * SBLOCK + threadIdx.x;
    const uint64_t stride = (uint64_t)gridDim.x * SBLOCK;
    // Main loop: every vector of the pass is inside all three allowed prefixes.
    const uint64_t lim = GUARD ? (K / VE < nv ? K / VE : nv) : nv;
    uint64_t v0 = tid;
    if (VE == 4) {
        const f32x4* b4 = reinterpret_cast<const f32x4*>(b);
        const f32x4* c4 = reinterpret_cast<const f32x4*>(c);
        f32x4* a4 = reinterpret_cast<f32x4*>(a);
        for (; v0 + (SUNROLL - 1) * stride < lim; v0 += SUNROLL * stride) {
            f32x4 xb[SUNROLL], xc[SUNROLL];
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                xb[u] = __builtin_nontemporal_load(b4 + v0 + u * stride);
                xc[u] = __builtin_nontemporal_load(c4 + v0 + u * stride);
            }
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                f32x4 r;
                r.x = triad1(xb[u].x, s, xc[u].x);
                r.y = triad1(xb[u].y, s, xc[u].y);
                r.z = triad1(xb[u].z, s, xc[u].z);
                r.w = triad1(xb[u].w, s, xc[u].w);
                __builtin_nontemporal_store(r, a4 + v0 + u * stride);
            }
        }
    }
    // Last pass of this thread (and the whole range for unaligned operands).
    for (; v0 < nv; v0 += SUNROLL * stride) {
        bool m[SUNROLL];
        if (VE == 4) {
            f32x4 xb[SUNROLL], xc[SUNROLL];
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                const uint64_t v = v0 + u * stride;
                m[u] = v < nv && (!GUARD || (v + 1) * 4 <= K);
                if (m[u]) {
                    xb[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(b) + v);
                    xc[u] = __builtin_nontemporal_load(reinterpret_cast<const f32x4*>(c) + v);
                }
            }
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                if (m[u]) {
                    f32x4 r;
                    r.x = triad1(xb[u].x, s, xc[u].x);
                    r.y = triad1(xb[u].y, s, xc[u].y);
                    r.z = triad1(xb[u].z, s, xc[u].z);
                    r.w = triad1(xb[u].w, s, xc[u].w);
                    __builtin_nontemporal_store(r, reinterpret_cast<f32x4*>(a) + (v0 + u * stride));
                }
            }
        } else {
            float xb[SUNROLL], xc[SUNROLL];
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                const uint64_t v = v0 + u * stride;
                m[u] = v < nv && (!GUARD || v + 1 <= K);
                if (m[u]) {
                    xb[u] = b[v];
                    xc[u] = c[v];
                }
            }
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u)
                if (m[u]) a[v0 + u * stride] = triad1(xb[u], s, xc[u]);
        }
        if (GUARD) {
#pragma unroll
            for (int u = 0; u < SUNROLL; ++u) {
                const uint64_t v = v0 + u * stride;
                if (v < nv && !m[u]) triad_slow(a, b, c, s, v * VE, v * VE + VE, Ka, Kb, Kc);
            }
        }
    }
    const uint64_t ti = nv * VE + tid;
    if (ti < n) triad_slow(a, b, c, s, ti, ti + 1, Ka, Kb, Kc);
    if (GUARD && logon && blockIdx.x == 0 && threadIdx.x == 0) {
        const uint64_t cnt = (n - Kb) + (n - Kc) + (n - Ka);
        if (cnt) {
            atomicAdd(&log->count, (unsigned long long)cnt);
            uint64_t k = Kb;
            uint32_t operand = 0;
            uint64_t p = (uint64_t)b;
            if (Kc < k) { k = Kc; operand = 1; p = (uint64_t)c; }
            if (Ka < k) { k = Ka; operand = 2; p = (uint64_t)a; }
            const uint64_t A = p + 4 * k;
            uint32_t v;
            int32_t o;
            reason_lane(t, A, 4, v, o);
            log_record(log, seq, k, operand, A, 4, 2 /*OP_TRIAD*/, v, o);
        }
    }
}

// One pass: as many 128-thread blocks as the vectors need, each thread one vector. Measured on
// MI355X for 2^28 fp32 (triad) and 1 GiB (copy): 0.492 ms and 0.339 ms, against 0.540 ms and
// 0.382 ms with one persistent 256-thread workgroup per CU looping over 4 vectors per thread
// per pass (the hardware's block dispatch balances the end of the launch better than a fixed
// split), and against 0.51-0.60 ms for the triad with blocks of 64-256 threads and 2-4 vectors.
static uint32_t stream_grid(uint64_t nv, const DevInfo& d) {
    (void)d;
    uint64_t want = (nv + (uint64_t)SBLOCK * SUNROLL - 1) / ((uint64_t)SBLOCK * SUNROLL);
    const uint64_t cap = 1ull << 30;  // beyond 2^37 vectors the loop takes further passes
    if (want < 1) want = 1;
    return (uint32_t)(want < cap ? want : cap);
}

template <bool G>
static void copy_dispatch(const DevTable& t, DevLog* log, void* dst, const void* src, uint64_t n,
                          uint64_t Ks, uint64_t Kd, unsigned long long seq, int logon,
                          const DevInfo& d, hipStream_t s) {
    const uint64_t ad = (uint64_t)dst | (uint64_t)src;
    if ((ad & 15) == 0)
        hipLaunchKernelGGL((k_copy<G, 16>), dim3(stream_grid(n / 16, d)), dim3(SBLOCK), 0, s, t, log,
                           (uint8_t*)dst, (const uint8_t*)src, n, Ks, Kd, seq, logon);
    else if ((ad & 3) == 0)
        hipLaunchKernelGGL((k_copy<G, 4>), dim3(stream_grid(n / 4, d)), dim3(SBLOCK), 0, s, t, log,
                           (uint8_t*)dst, (const uint8_t*)src, n, Ks, Kd, seq, logon);
    else
        hipLaunchKernelGGL((k_copy<G, 1>), dim3(stream_grid(n, d)), dim3(SBLOCK), 0, s, t, log,
                           (uint8_t*)dst, (const uint8_t*)src, n, Ks, Kd, seq, logon);
}

hipError_t launch_copy(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* dst,
                       const void* src, uint64_t n, unsigned long long seq, int logon,
                       const DevInfo& d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (guard)
        copy_dispatch<true>(t, log, dst, src, n, clip_prefix(binds[0], (uint64_t)src, n, 1),
                            clip_prefix(binds[1], (uint64_t)dst, n, 1), seq, logon, d, s);
    else
        copy_dispatch<false>(t, log, dst, src, n, n, n, seq, logon, d, s);
    return hipGetLastError();
}

template <bool G>
static void triad_dispatch(const DevTable& t, DevLog* log, float* a, const float* b, const float* c,
                           float sc, uint64_t n, uint64_t Ka, uint64_t Kb, uint64_t Kc,
                           unsigned long long seq, int logon, const DevInfo& d, hipStream_t s) {
    const uint64_t ad = (uint64_t)a | (uint64_t)b | (uint64_t)c;
    if ((ad & 15) == 0)
        hipLaunchKernelGGL((k_triad<G, 4>), dim3(stream_grid(n / 4, d)), dim3(SBLOCK), 0, s, t, log,
                           a, b, c, sc, n, Ka, Kb, Kc, seq, logon);
    else
        hipLaunchKernelGGL((k_triad<G, 1>), dim3(stream_grid(n, d)), dim3(SBLOCK), 0, s, t, log, a,
                           b, c, sc, n, Ka, Kb, Kc, seq, logon);
}

hipError_t launch_triad(bool guard, const DevTable& t, DevLog* log, const Bind* binds, float* a,
                        const float* b, const float* c, float sc, uint64_t n,
                        unsigned long long seq, int logon, const DevInfo& d, hipStream_t s) {
    if (n == 0) return hipSuccess;
    if (guard)
        triad_dispatch<true>(t, log, a, b, c, sc, n, clip_prefix(binds[2], (uint64_t)a, n, 4),
                             clip_prefix(binds[0], (uint64_t)b, n, 4),
                             clip_prefix(binds[1], (uint64_t)c, n, 4), seq, logon, d, s);
    else
        triad_dispatch<false>(t, log, a, b, c, sc, n, n, n, n, seq, logon, d, s);
    return hipGetLastError();
}

}  // namespace agile
