// Guarded scatter-add dst[idx[i], :] += src[i, :] (kernel memory guard of AgileOS Section V-E),
// organised so that heavily repeated destination rows (the hot rows of a Zipf-distributed
// embedding gradient) neither serialize on atomics nor pay one atomic row-update per index.
//
// Sorted path (large calls). Rows that pass the guard's fast test (index readable, source row
// wholly inside its allowed prefix, destination row inside the binding's row interval) get a
// 32-bit key, their destination row's offset inside that interval; every other row gets the
// largest key. A stable LSD radix sort (8-bit digits; per pass: per-tile digit histograms, their
// exclusive scan, a stable scatter that ranks a tile's keys with wave ballots and regroups them
// by digit in LDS, so that each digit's keys leave the tile as one contiguous run; a pass whose
// digit is the same for every key is skipped on the device) orders (key, position) pairs by
// destination row, position ascending. Each wave then walks a tile of 256 sorted entries and sums the source rows
// of each run of equal keys in position order; a run that lies wholly inside the tile owns its
// destination row and adds with a plain read-modify-write, a run that crosses a tile boundary
// adds with one atomic per element. When the caller promises a destination of +0.0 rows (scatter-
// add into zeros), an owned run stores (+0.0 + its sum) without reading the row. Rows that failed the fast test follow in a separate kernel
// that checks every element exactly (denied loads read zero, denied stores are dropped) and
// counts denials as the other data-dependent guarded kernels do; a one-thread kernel after the
// launch records the smallest key.
//
// Chunk path (small calls, or destination intervals too large for 32-bit keys): each workgroup
// takes 2048 consecutive indices, sorts (key, position) pairs in LDS with a bitonic network,
// cuts the sorted chunk into pieces of at most 32 equal keys, sums each piece in position order
// and adds the sum with one atomic per element; rows outside the interval are checked per element.
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
    if (GUARD && logon) fold_faults(acc, log);
}

// ================================================================ sorted path
constexpr int SRT_BLOCK = 256;
constexpr uint32_t SRT_TILE = 4096;   // keys per histogram / scatter tile (16 per thread)
constexpr uint32_t SRT_TB = 1024;      // threads of the histogram and scatter workgroups
constexpr uint32_t SRT_SENT = 0xFFFFFFFFu;
constexpr uint32_t RED_TILE = 256;    // sorted entries per reduce wave
// ctl[p] (p < 4): pass p was skipped (one digit value only); ctl[4 + p]: the buffer pass p reads
// (ctl[4 + npasses]: the buffer holding the sorted result, which the reduce reads)
constexpr int CTL_WORDS = 16;

struct SortBufs {
    uint32_t* keys[2];
    uint32_t* vals[2];
    uint32_t* hist;  // [256 * ntiles], scanned in place
    uint32_t* ctl;   // [CTL_WORDS]
    uint32_t* dstart;  // [256]: the current pass's digit totals
    uint64_t* slow;  // [ceil(n / 64)]: bit l of word w marks row 64 w + l as failing the fast test
};

static inline uint64_t srt_ntiles(uint64_t n) { return (n + SRT_TILE - 1) / SRT_TILE; }

size_t scatter_add_scratch_bytes(uint64_t n) {
    const uint64_t a = ((n * 4 + 255) / 256) * 256;
    return 4 * a + srt_ntiles(n) * 256 * 4 + 256 + 1024 + ((n + 63) / 64) * 8;
}

static SortBufs sort_bufs(void* scratch, uint64_t n) {
    const uint64_t a = ((n * 4 + 255) / 256) * 256;
    uint8_t* p = static_cast<uint8_t*>(scratch);
    SortBufs b;
    b.keys[0] = reinterpret_cast<uint32_t*>(p);
    b.keys[1] = reinterpret_cast<uint32_t*>(p + a);
    b.vals[0] = reinterpret_cast<uint32_t*>(p + 2 * a);
    b.vals[1] = reinterpret_cast<uint32_t*>(p + 3 * a);
    b.hist = reinterpret_cast<uint32_t*>(p + 4 * a);
    b.ctl = reinterpret_cast<uint32_t*>(p + 4 * a + srt_ntiles(n) * 256 * 4);
    b.dstart = reinterpret_cast<uint32_t*>(p + 4 * a + srt_ntiles(n) * 256 * 4 + 256);
    b.slow = reinterpret_cast<uint64_t*>(p + 4 * a + srt_ntiles(n) * 256 * 4 + 256 + 1024);
    return b;
}

// Keys: guarded rows that pass the fast test get (idx - rlo); the others the sentinel. The
// unguarded twin keys every row by idx + 2^31 (its indices must lie in [-2^31, 2^31 - 1)). One
// workgroup per tile of SRT_TILE rows, which also counts the tile's digits of the first pass, so
// the sort's first histogram needs no pass over the keys of its own.
template <bool GUARD>
__global__ __launch_bounds__(SRT_TB) void k_srt_keys(const int64_t* __restrict__ idx, uint64_t n,
                                                     RowsGuard rg, SortBufs b) {
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < CTL_WORDS) b.ctl[tid] = 0;  // every pass starts from buffer 0
    if (tid < 256) h[tid] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * SRT_TILE;
#pragma unroll
    for (uint32_t r = 0; r < SRT_TILE / SRT_TB; ++r) {
        // a wave covers 64 consecutive rows (i0 is its first), so its ballot is one bitmask word
        const uint64_t i0 = t0 + r * SRT_TB + (tid & ~63u);
        const uint64_t i = i0 + (tid & 63u);
        uint32_t key = SRT_SENT;
        bool slow = false;
        if (i < n) {
            if (GUARD) {
                const int64_t x = i < rg.nfast ? idx[i] : 0;
                const bool fast = i < rg.nfast && rg.g.rlo <= x && x <= rg.g.rhi;
                key = fast ? (uint32_t)((uint64_t)x - (uint64_t)rg.g.rlo) : SRT_SENT;
                slow = !fast;
            } else {
                key = (uint32_t)((uint64_t)idx[i] + 0x80000000ull);
            }
            b.keys[0][i] = key;
            b.vals[0][i] = (uint32_t)i;
            atomicAdd(&h[key & 255u], 1u);
        }
        if (GUARD) {
            const uint64_t m = __ballot(slow);
            if ((tid & 63u) == 0 && i0 < n) b.slow[i0 >> 6] = m;
        }
    }
    __syncthreads();
    if (tid < 256) b.hist[(uint64_t)tid * gridDim.x + blockIdx.x] = h[tid];
}

// Digit histogram of one pass per tile of SRT_TILE keys, stored digit-major (hist[d * ntiles + t]).
__global__ __launch_bounds__(SRT_TB) void k_srt_hist(SortBufs b, uint64_t n, uint32_t pass) {
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x, shift = 8 * pass;
    const uint32_t* keys = b.keys[b.ctl[4 + pass]];
    if (tid < 256) h[tid] = 0;
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * SRT_TILE;
    uint32_t k[SRT_TILE / SRT_TB];
#pragma unroll
    for (uint32_t r = 0; r < SRT_TILE / SRT_TB; ++r) {
        const uint64_t i = t0 + r * SRT_TB + tid;
        k[r] = i < n ? keys[i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < SRT_TILE / SRT_TB; ++r)
        if (t0 + r * SRT_TB + tid < n) atomicAdd(&h[(k[r] >> shift) & 255u], 1u);
    __syncthreads();
    if (tid < 256) b.hist[(uint64_t)tid * gridDim.x + blockIdx.x] = h[tid];
}

// Offsets of a pass. k_srt_scan_rows: one workgroup per digit turns the digit's per-tile counts
// into exclusive prefixes and records the digit's total; the scatter's workgroups then turn the
// 256 totals into each digit's first output position themselves.
template <uint32_t NT>
__device__ inline uint32_t block_scan(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint32_t inc = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(inc, o, 64);
        if (lane >= (uint32_t)o) inc += y;
    }
    if (lane == 63) wsum[wv] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
    for (uint32_t k = 0; k < NT / 64; ++k) {
        if (k < wv) before += wsum[k];
        total += wsum[k];
    }
    __syncthreads();
    return before + inc - v;
}

__global__ __launch_bounds__(SRT_BLOCK) void k_srt_scan_rows(SortBufs b, uint32_t ntiles) {
    __shared__ uint32_t wsum[SRT_BLOCK / 64];
    uint32_t* row = b.hist + (uint64_t)blockIdx.x * ntiles;
    uint32_t carry = 0;
    for (uint32_t t0 = 0; t0 < ntiles; t0 += SRT_BLOCK) {
        const uint32_t t = t0 + threadIdx.x;
        const uint32_t v = t < ntiles ? row[t] : 0u;
        uint32_t total;
        const uint32_t ex = block_scan<SRT_BLOCK>(v, wsum, total);
        if (t < ntiles) row[t] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) b.dstart[blockIdx.x] = carry;
}

// Stable scatter of one pass over a tile of SRT_TILE keys. The workgroup first turns the 256 digit
// totals into each digit's first output position (a pass whose digit is the same for all n keys is
// skipped; workgroup 0 records that, and which buffer the next pass reads). Each wave then ranks
// its SRT_TILE / 16 consecutive keys by digit in rounds of 64: wave ballots rank equal digits by
// lane, and a per-wave running count per digit carries the order from round to round (a wave's
// LDS reads and writes take effect in program order, so no barrier is needed between rounds).
// The tile's keys are regrouped by digit in LDS, in position order within a digit, and each
// digit's group is written to its place in the output as one contiguous run.
__global__ __launch_bounds__(SRT_TB) void k_srt_scatter(SortBufs b, uint64_t n, uint32_t pass) {
    constexpr uint32_t NW = SRT_TB / 64;
    constexpr uint32_t R = SRT_TILE / SRT_TB;  // rounds per wave
    __shared__ uint32_t wc[NW][256];  // keys per wave and digit, then each wave's offset in the digit
    __shared__ uint32_t lstart[256];  // first slot of each digit in the regrouped tile
    __shared__ uint32_t gstart[256];  // output position of the tile's first key of each digit
    __shared__ uint32_t sk[SRT_TILE], sv[SRT_TILE];
    __shared__ uint32_t wsum[NW];
    __shared__ uint32_t skip;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6, shift = 8 * pass;
    const uint32_t src = b.ctl[4 + pass];
    if (tid == 0) skip = 0;
    const uint32_t tot = tid < 256 ? b.dstart[tid] : 0u;
    __syncthreads();
    if (tid < 256 && (uint64_t)tot == n) skip = 1;
    uint32_t all;
    const uint32_t dfirst = block_scan<SRT_TB>(tot, wsum, all);
    if (blockIdx.x == 0 && tid == 0) {
        b.ctl[pass] = skip;
        b.ctl[4 + pass + 1] = skip ? src : 1u - src;
    }
    if (skip) return;
    const uint32_t* kin = b.keys[src];
    const uint32_t* vin = b.vals[src];
    uint32_t* kout = b.keys[1u - src];
    uint32_t* vout = b.vals[1u - src];
    if (tid < 256) {
#pragma unroll
        for (uint32_t w = 0; w < NW; ++w) wc[w][tid] = 0;
        gstart[tid] = dfirst + b.hist[(uint64_t)tid * gridDim.x + blockIdx.x];
    }
    __syncthreads();
    const uint64_t t0 = (uint64_t)blockIdx.x * SRT_TILE;
    const uint64_t w0 = t0 + (uint64_t)wv * (SRT_TILE / NW);
    const uint64_t below = lane ? (~0ull >> (64 - lane)) : 0ull;
    uint32_t key[R], val[R], pre[R];
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const uint64_t i = w0 + r * 64 + lane;
        key[r] = i < n ? kin[i] : 0u;
        val[r] = i < n ? vin[i] : 0u;
    }
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        const bool valid = w0 + r * 64 + lane < n;
        const uint32_t d = (key[r] >> shift) & 255u;
        uint64_t match = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t bb = __ballot((d >> bit) & 1u);
            match &= ((d >> bit) & 1u) ? bb : ~bb;
        }
        const uint32_t rank = (uint32_t)__popcll(match & below);
        pre[r] = wc[wv][d] + rank;
        if (valid && rank == 0) wc[wv][d] = pre[r] + (uint32_t)__popcll(match);
    }
    __syncthreads();
    // thread tid < 256 owns digit tid: the tile's count, and each wave's offset inside the digit
    uint32_t cnt = 0;
    if (tid < 256) {
#pragma unroll
        for (uint32_t w = 0; w < NW; ++w) {
            const uint32_t c = wc[w][tid];
            wc[w][tid] = cnt;
            cnt += c;
        }
    }
    const uint32_t lfirst = block_scan<SRT_TB>(cnt, wsum, all);
    if (tid < 256) lstart[tid] = lfirst;
    __syncthreads();
#pragma unroll
    for (uint32_t r = 0; r < R; ++r) {
        if (w0 + r * 64 + lane < n) {
            const uint32_t d = (key[r] >> shift) & 255u;
            const uint32_t slot = lstart[d] + wc[wv][d] + pre[r];
            sk[slot] = key[r];
            sv[slot] = val[r];
        }
    }
    __syncthreads();
    const uint32_t m = (uint32_t)(n - t0 < SRT_TILE ? n - t0 : SRT_TILE);
    for (uint32_t q = tid; q < m; q += SRT_TB) {
        const uint32_t k = sk[q];
        const uint32_t d = (k >> shift) & 255u;
        const uint32_t pos = gstart[d] + (q - lstart[d]);
        kout[pos] = k;
        vout[pos] = sv[q];
    }
}

template <int W, int EPL>
struct RowVec {
    typename FloatOf<W>::F v[EPL];
};

// NT: a row read once (a source row of the sum): non-temporal, so it does not push the
// destination rows, which are read, summed and written back, out of the caches.
template <int W, int EPL, bool NT = false>
__device__ __forceinline__ RowVec<W, EPL> load_row(const uint8_t* src, uint64_t rb, uint32_t row,
                                                   uint64_t col0) {
    using F = typename FloatOf<W>::F;
    RowVec<W, EPL> r;
    const F* sp = reinterpret_cast<const F*>(src + (uint64_t)row * rb) + col0;
    if (EPL == 4) {
        typedef F f4 __attribute__((ext_vector_type(4)));
        const f4* vp = reinterpret_cast<const f4*>(sp);
        const f4 v = NT ? __builtin_nontemporal_load(vp) : *vp;
        r.v[0] = v.x;
        r.v[EPL > 1 ? 1 : 0] = v.y;
        r.v[EPL > 2 ? 2 : 0] = v.z;
        r.v[EPL > 3 ? 3 : 0] = v.w;
    } else {
#pragma unroll
        for (int q = 0; q < EPL; ++q) r.v[q] = NT ? __builtin_nontemporal_load(sp + q) : sp[q];
    }
    return r;
}

// End of a run: an owned destination row gets (its value loaded when the run started + the
// run's sum) stored back; a shared one gets atomic adds.
template <int W, int EPL>
__device__ __forceinline__ void srt_flush(uint8_t* dst, uint64_t rb, int64_t row, uint64_t col0,
                                          bool owned, const RowVec<W, EPL>& old,
                                          const typename FloatOf<W>::F (&acc)[EPL]) {
    using F = typename FloatOf<W>::F;
    F* d = reinterpret_cast<F*>(dst + (uint64_t)row * rb) + col0;
    if (owned) {
        if (EPL == 4) {
            typedef F f4 __attribute__((ext_vector_type(4)));
            f4 v;
            v.x = old.v[0] + acc[0];
            v.y = old.v[EPL > 1 ? 1 : 0] + acc[EPL > 1 ? 1 : 0];
            v.z = old.v[EPL > 2 ? 2 : 0] + acc[EPL > 2 ? 2 : 0];
            v.w = old.v[EPL > 3 ? 3 : 0] + acc[EPL > 3 ? 3 : 0];
            *reinterpret_cast<f4*>(d) = v;
        } else {
#pragma unroll
            for (int q = 0; q < EPL; ++q) d[q] = old.v[q] + acc[q];
        }
    } else {
#pragma unroll
        for (int q = 0; q < EPL; ++q) unsafeAtomicAdd(d + q, acc[q]);
    }
}

// Each wave walks RED_TILE sorted entries (their keys and positions held one per lane, read out
// wave-uniformly) with RED_U rows in flight: the source rows of the next RED_U entries are loaded
// together with the destination row of every run that starts among them, then the rows are
// summed in order. A run the tile owns ends with a plain store of (destination + sum); a run
// shared with a neighbouring tile ends with one atomic add per element.
constexpr int RED_U = 8;
// zero_dst: the destination rows are +0.0 before the call (the caller's promise), so the rows are
// not read: an owned run stores (+0.0 + sum), exactly what the read-modify-write would.
template <bool GUARD, int W, int EPL>
__global__ __launch_bounds__(256) void k_srt_reduce(uint8_t* dst, uint64_t rb,
                                                    const uint8_t* __restrict__ src, uint64_t n,
                                                    SortBufs b, uint32_t npasses, int64_t rlo,
                                                    uint32_t zero_dst) {
    using F = typename FloatOf<W>::F;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * 256) >> 6;
    const uint32_t buf = b.ctl[4 + npasses];
    const uint32_t* __restrict__ keys = b.keys[buf];
    const uint32_t* __restrict__ vals = b.vals[buf];
    const uint64_t D = rb / W;
    const int64_t base = GUARD ? rlo : -(int64_t)0x80000000ll;
    const uint64_t ncb = (D + 64 * EPL - 1) / (64 * EPL);
    for (uint64_t e0 = wave * RED_TILE; e0 < n; e0 += nwaves * RED_TILE) {
        const uint64_t e1 = e0 + RED_TILE < n ? e0 + RED_TILE : n;
        const uint32_t k0 = keys[e0];
        if (k0 == SRT_SENT) continue;
        // does the tile's first run continue a run of the previous tile, its last run the next?
        const bool head_shared = e0 > 0 && keys[e0 - 1] == k0;
        const uint32_t klast = keys[e1 - 1];
        const bool tail_shared = e1 < n && klast != SRT_SENT && keys[e1] == klast;
        // the tile's keys and positions, one per lane per group of 64 (sentinel past the tile)
        uint32_t tk[RED_TILE / 64], tv[RED_TILE / 64];
#pragma unroll
        for (int j = 0; j < RED_TILE / 64; ++j) {
            const uint64_t e = e0 + (uint64_t)j * 64 + lane;
            tk[j] = e < e1 ? keys[e] : SRT_SENT;
            tv[j] = e < e1 ? vals[e] : 0u;
        }
        for (uint64_t cb = 0; cb < ncb; ++cb) {
            const uint64_t col0 = cb * 64 * EPL + (uint64_t)lane * EPL;
            const bool on = col0 < D;
            F acc[EPL];
#pragma unroll
            for (int q = 0; q < EPL; ++q) acc[q] = (F)-0.0;
            uint32_t cur = k0;
            bool first = true, stop = false;
            RowVec<W, EPL> dcur;
#pragma unroll
            for (int q = 0; q < EPL; ++q) dcur.v[q] = (F)0.0;
            if (on && !head_shared && !zero_dst)
                dcur = load_row<W, EPL>(dst + (uint64_t)(base + (int64_t)k0) * rb, rb, 0, col0);
#pragma unroll
            for (int j = 0; j < RED_TILE / 64; ++j) {
                for (uint32_t l = 0; l < 64 && !stop; l += RED_U) {
                    uint32_t kk[RED_U], vv[RED_U];
                    RowVec<W, EPL> rv[RED_U], dv[RED_U];
#pragma unroll
                    for (int u = 0; u < RED_U; ++u) {
                        kk[u] = (uint32_t)__builtin_amdgcn_readlane((int)tk[j], (int)(l + u));
                        vv[u] = (uint32_t)__builtin_amdgcn_readlane((int)tv[j], (int)(l + u));
                    }
#pragma unroll
                    for (int u = 0; u < RED_U; ++u) {
                        if (kk[u] != SRT_SENT && on) {
                            rv[u] = load_row<W, EPL, true>(src, rb, vv[u], col0);
                            const uint32_t prev = u == 0 ? cur : kk[u - 1];
                            if (kk[u] != prev) {
                                if (zero_dst) {
#pragma unroll
                                    for (int q = 0; q < EPL; ++q) dv[u].v[q] = (F)0.0;
                                } else {
                                    dv[u] = load_row<W, EPL>(
                                        dst + (uint64_t)(base + (int64_t)kk[u]) * rb, rb, 0, col0);
                                }
                            }
                        }
                    }
#pragma unroll
                    for (int u = 0; u < RED_U; ++u) {
                        if (kk[u] == SRT_SENT) {
                            stop = true;
                            break;
                        }
                        if (kk[u] != cur) {
                            if (on) srt_flush<W, EPL>(dst, rb, base + (int64_t)cur, col0,
                                                      !(first && head_shared), dcur, acc);
#pragma unroll
                            for (int q = 0; q < EPL; ++q) acc[q] = (F)-0.0;
                            cur = kk[u];
                            dcur = dv[u];
                            first = false;
                        }
                        if (on) {
#pragma unroll
                            for (int q = 0; q < EPL; ++q) acc[q] += rv[u].v[q];
                        }
                    }
                }
            }
            // the last run of the tile: shared with the next tile only if it reaches the tile end
            const bool last_shared = tail_shared && cur == klast;
            if (on) srt_flush<W, EPL>(dst, rb, base + (int64_t)cur, col0,
                                      !((first && head_shared) || last_shared), dcur, acc);
        }
    }
}

// Rows that failed the fast test: every element checked exactly, atomics for the allowed ones.
template <int W>
__global__ __launch_bounds__(256) void k_srt_slow(DevTable t, DevLog* log, uint8_t* dst, uint64_t rb,
                                                  const int64_t* idx, const uint8_t* src,
                                                  uint64_t n, RowsGuard rg, SortBufs b,
                                                  unsigned long long seq, int logon) {
    using F = typename FloatOf<W>::F;
    const uint32_t lane = threadIdx.x & 63u;
    const uint64_t wave = ((uint64_t)blockIdx.x * 256 + threadIdx.x) >> 6;
    const uint64_t nwaves = ((uint64_t)gridDim.x * 256) >> 6;
    const uint64_t D = rb / W;
    const uint64_t Ki = rg.ki, Ks = rg.kc;
    const RowGuard g = rg.g;
    FaultAcc acc;
    for (uint64_t r0 = wave * 64; r0 < n; r0 += nwaves * 64) {
        uint64_t m = uniform_u64(b.slow[r0 >> 6]);
        while (m) {
            const uint32_t l = (uint32_t)__builtin_ctzll(m);
            m &= m - 1;
            const uint64_t r = r0 + l;
            const bool iok = r < Ki;
            if (!iok && lane == 0) acc.note((r * D) << 2);
            const int64_t iv = iok ? idx[r] : 0;
            uint8_t* drow = dst + (uint64_t)iv * rb;
            for (uint64_t col = lane; col < D; col += 64) {
                const uint64_t es = r * D + col;
                F v = (F)0.0;
                if (es < Ks) v = reinterpret_cast<const F*>(src)[es];
                else acc.note((es << 2) | 1u);
                if (elem_ok(g, iv, rb, col, W))
                    unsafeAtomicAdd(reinterpret_cast<F*>(drow + col * W), v);
                else
                    acc.note((es << 2) | 2u);
            }
        }
    }
    if (logon) fold_faults(acc, log);
}

template <bool G, int W>
static void scatter_add_sorted(const DevTable& t, DevLog* log, void* dst, uint64_t rb,
                               const int64_t* idx, const void* src, uint64_t n,
                               const RowsGuard& rg, uint32_t npasses, void* scratch,
                               unsigned long long seq, int logon, const DevInfo& d,
                               hipStream_t s, bool zero_dst) {
    const SortBufs b = sort_bufs(scratch, n);
    const uint32_t ntiles = (uint32_t)srt_ntiles(n);
    // the key pass also writes the first pass's per-tile histograms
    hipLaunchKernelGGL((k_srt_keys<G>), dim3(ntiles), dim3(SRT_TB), 0, s, idx, n, rg, b);
    for (uint32_t p = 0; p < npasses; ++p) {
        if (p > 0) hipLaunchKernelGGL(k_srt_hist, dim3(ntiles), dim3(SRT_TB), 0, s, b, n, p);
        hipLaunchKernelGGL(k_srt_scan_rows, dim3(256), dim3(SRT_BLOCK), 0, s, b, ntiles);
        hipLaunchKernelGGL(k_srt_scatter, dim3(ntiles), dim3(SRT_TB), 0, s, b, n, p);
    }
    const uint64_t waves = (n + RED_TILE - 1) / RED_TILE;
    const uint64_t rg_blocks = (waves + 3) / 4;
    const uint32_t rgrid = (uint32_t)(rg_blocks < (uint64_t)d.num_cu * 8 ? rg_blocks : (uint64_t)d.num_cu * 8);
    const bool v4 = W == 4 && (rb / W) % 4 == 0 && (((uint64_t)src | (uint64_t)dst | rb) & 15) == 0;
    if (v4)
        hipLaunchKernelGGL((k_srt_reduce<G, W, 4>), dim3(rgrid), dim3(256), 0, s, (uint8_t*)dst, rb,
                           (const uint8_t*)src, n, b, npasses, rg.g.rlo, (uint32_t)zero_dst);
    else
        hipLaunchKernelGGL((k_srt_reduce<G, W, 1>), dim3(rgrid), dim3(256), 0, s, (uint8_t*)dst, rb,
                           (const uint8_t*)src, n, b, npasses, rg.g.rlo, (uint32_t)zero_dst);
    if (G) {
        const uint64_t sw = (n + 63) / 64;
        const uint64_t sb = (sw + 3) / 4;
        const uint32_t sgrid = (uint32_t)(sb < (uint64_t)d.num_cu * 4 ? sb : (uint64_t)d.num_cu * 4);
        hipLaunchKernelGGL((k_srt_slow<W>), dim3(sgrid), dim3(256), 0, s, t, log, (uint8_t*)dst, rb,
                           idx, (const uint8_t*)src, n, rg, b, seq, logon);
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
                              void* scratch, const DevInfo& d, hipStream_t s, bool finish,
                              bool zero_dst) {
    if (n == 0) return hipSuccess;
    const RowsGuard rg = guard ? rows_guard(binds[0], binds[1], binds[2], (uint64_t)idx,
                                            (uint64_t)src, (uint64_t)dst, n, rb, w)
                               : rows_open(n, rb, w);
    // sorted path: 32-bit keys (guarded: the destination's row interval minus the sentinel;
    // unguarded: idx + 2^31), positions below 2^32
    uint32_t npasses = 0;
    bool sorted = scratch != nullptr && n >= SORT_MIN_N && n < (1ull << 32);
    if (sorted && guard) {
        if (!rg.g.bound || rg.g.rhi < rg.g.rlo) {
            npasses = 1;  // no fast rows: every key is the sentinel, the sort is trivial
        } else {
            const uint64_t span = (uint64_t)rg.g.rhi - (uint64_t)rg.g.rlo;
            if (span >= SRT_SENT) sorted = false;
            // enough bits for span + 1, so that no key equals the sentinel in the sorted bits
            // (the largest key of a 2^16-row table is all ones in 16 bits)
            uint32_t bits = 0;
            while (bits < 32 && ((span + 1) >> bits)) ++bits;
            npasses = (bits + 7) / 8;
            if (npasses == 0) npasses = 1;
        }
    } else if (sorted) {
        npasses = 4;
    }
    if (sorted) {
        if (guard) {
            if (w == 4) scatter_add_sorted<true, 4>(t, log, dst, rb, idx, src, n, rg, npasses, scratch, seq, logon, d, s, zero_dst);
            else scatter_add_sorted<true, 8>(t, log, dst, rb, idx, src, n, rg, npasses, scratch, seq, logon, d, s, zero_dst);
        } else {
            if (w == 4) scatter_add_sorted<false, 4>(t, log, dst, rb, idx, src, n, rg, npasses, scratch, seq, logon, d, s, zero_dst);
            else scatter_add_sorted<false, 8>(t, log, dst, rb, idx, src, n, rg, npasses, scratch, seq, logon, d, s, zero_dst);
        }
    } else if (guard) {
        if (w == 4) scatter_add_w<true, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_add_w<true, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    } else {
        if (w == 4) scatter_add_w<false, 4>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
        else scatter_add_w<false, 8>(t, log, dst, rb, idx, src, n, rg, seq, logon, d, s);
    }
    if (guard && logon && finish)
        return launch_fault_finish(t, log, rows_fault_site(5 /*OP_SCATTER_ADD*/, w, 2, rb, rg.ki, idx,
                                                             src, dst), seq, s);
    return hipGetLastError();
}

}  // namespace agile
