// Batched multi-client requests in one persistent launch.
//
// The paper's runtime assigns each client to a worker, and the worker checks every pointer
// argument of a mediated request against that client's own allocations before the real call
// (AgileOS Sections IV-B, IV-C, IV-F; a pointer valid for another client is not valid here,
// Section III). Here one launch serves many requests of many clients: every request is cut
// into tiles (pointer validation, guarded copy, guarded gather), workgroups pull tiles from an
// atomic counter until none are left (every workgroup exits once the counter passes the last
// tile), and the workgroup that finishes a request's last tile writes the request's result:
// the lowest failing pointer argument and the request's fault record.
#include "launch.h"

namespace agile {

constexpr int BBLOCK = 512;  // 8 waves per CU: 1.42 ms for the 512-request launch (256: 1.55)
constexpr uint64_t TILE_PTRS = 2048;       // pointers per validation tile (4 per thread)
constexpr uint64_t TILE_COPY_MAX = 2ull << 20;  // bytes per copy tile, large launches
constexpr int COPY_U = 8;                 // 16-byte vectors in flight per thread
constexpr uint64_t COPY_CHUNK = (uint64_t)BBLOCK * COPY_U * 16;  // one pass of a workgroup
constexpr uint64_t TILE_ROWS_MAX = 16384;  // rows per gather tile, large launches
constexpr uint64_t TILE_ROWS_MIN = 512;
constexpr int VQ = 4;  // pointer queries per lane
static_assert(TILE_PTRS == (uint64_t)VQ * BBLOCK, "a validation tile is one pass of the block");
constexpr uint32_t LDS_SPLIT = 4096;       // bucket splitters staged in LDS for the search

__device__ inline void tiles_of(const BatchReq& q, uint64_t tile_copy, uint64_t& vt,
                                uint64_t& ct) {
    vt = (q.nptr + TILE_PTRS - 1) / TILE_PTRS;
    ct = (q.copy_bytes + tile_copy - 1) / tile_copy;
}

// VQ pointer queries per lane, searched together (uniform trip count over the client table).
// Tables of up to LDS_SPLIT buckets have their splitters staged in LDS first (one round of
// coalesced loads instead of a chain of dependent global loads per query); larger ones are
// searched in global memory (L2-resident).
__device__ inline void validate_tile(const DevTable& t, const ulonglong2* ptrs, uint64_t p0,
                                     uint64_t k0, uint64_t k1, uint8_t* pv, int32_t* po,
                                     uint32_t& minfail, uint64_t* s_split) {
    const bool staged = t.nb <= LDS_SPLIT;
    if (staged) {
        for (uint32_t k = threadIdx.x; k < t.nb; k += BBLOCK) s_split[k] = t.split64[k];
        __syncthreads();
    }
    const uint64_t* sp = staged ? s_split : t.split64;
    uint64_t a[VQ], L[VQ];
    uint32_t base[VQ];
    bool live[VQ];
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
        const uint64_t k = k0 + (uint64_t)q * BBLOCK + threadIdx.x;
        live[q] = k < k1;
        const ulonglong2 x = live[q] ? ptrs[p0 + k] : make_ulonglong2(0, 0);
        a[q] = x.x;
        L[q] = x.y < 1 ? 1 : x.y;
        base[q] = 0;
    }
    for (uint32_t len = t.nb; len > 1;) {
        const uint32_t half = len >> 1;
#pragma unroll
        for (int q = 0; q < VQ; ++q) base[q] = sp[base[q] + half] <= a[q] ? base[q] + half : base[q];
        len -= half;
    }
#pragma unroll
    for (int q = 0; q < VQ; ++q) {
        if (!live[q]) continue;
        const uint64_t k = k0 + (uint64_t)q * BBLOCK + threadIdx.x;
        uint8_t v = V_UNMAPPED;
        int32_t o = -1;
        if (t.nb > 0 && sp[base[q]] <= a[q]) classify_in_bucket(load_rec(t.rec + base[q]), a[q], L[q], v, o);
        pv[p0 + k] = v;
        po[p0 + k] = o;
        if (v != V_ALLOW && (uint32_t)k < minfail) minfail = (uint32_t)k;
    }
}

// Bytes [o0, o1) of a guarded copy whose arguments allow the prefixes Ks (src) and Kd (dst).
__device__ inline void copy_tile(uint8_t* dst, const uint8_t* src, uint64_t o0, uint64_t o1,
                                 uint64_t Ks, uint64_t Kd) {
    const uint64_t K = Ks < Kd ? Ks : Kd;
    const bool vec = (((uint64_t)dst | (uint64_t)src | o0) & 15) == 0;
    uint64_t done = o0;
    typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));
    if (vec && o1 <= K) {
        // the whole range lies inside both allowed prefixes: CU vectors in flight per thread
        constexpr int CU = COPY_U;
        // global-address-space pointers: the request's addresses arrive as integers, and generic
        // pointers would give flat accesses (1.42 against 1.46 ms for the 512-request launch)
        typedef __attribute__((address_space(1))) const u32x4 gcv;
        typedef __attribute__((address_space(1))) u32x4 gv;
        const gcv* sv = (const gcv*)(uintptr_t)src;
        gv* dv = (gv*)(uintptr_t)dst;
        const uint64_t v0 = o0 / 16, v1 = o1 / 16;
        for (uint64_t v = v0 + threadIdx.x; v < v1; v += (uint64_t)BBLOCK * CU) {
            u32x4 x[CU];
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const uint64_t w = v + (uint64_t)u * BBLOCK;
                if (w < v1) x[u] = __builtin_nontemporal_load(sv + w);
            }
#pragma unroll
            for (int u = 0; u < CU; ++u) {
                const uint64_t w = v + (uint64_t)u * BBLOCK;
                if (w < v1) __builtin_nontemporal_store(x[u], dv + w);
            }
        }
        done = v1 * 16;
    } else if (vec) {
        const uint64_t v0 = o0 / 16, v1 = o1 / 16;
        for (uint64_t v = v0 + threadIdx.x; v < v1; v += BBLOCK) {
            const uint64_t b0 = v * 16;
            if (b0 + 16 <= K) {
                reinterpret_cast<u32x4*>(dst)[v] = reinterpret_cast<const u32x4*>(src)[v];
            } else if (b0 >= Ks && b0 + 16 <= Kd) {
                reinterpret_cast<u32x4*>(dst)[v] = u32x4{0u, 0u, 0u, 0u};
            } else if (b0 < Kd) {
                for (uint64_t k = b0; k < b0 + 16; ++k) {
                    const uint8_t x = k < Ks ? src[k] : (uint8_t)0;
                    if (k < Kd) dst[k] = x;
                }
            }
        }
        done = v1 * 16;
    }
    for (uint64_t k = done + threadIdx.x; k < o1; k += BBLOCK) {
        const uint8_t x = k < Ks ? src[k] : (uint8_t)0;
        if (k < Kd) dst[k] = x;
    }
}

__device__ inline void gather_tile(const BatchReq& q, const RowsGuard& rg, uint64_t i0, uint64_t i1,
                                   FaultAcc& acc) {
    const uint64_t rb = q.gather_row_bytes, D = rb / 4;
    const int64_t* idx = reinterpret_cast<const int64_t*>(q.gather_idx);
    const uint8_t* T = reinterpret_cast<const uint8_t*>(q.gather_table);
    uint8_t* out = reinterpret_cast<uint8_t*>(q.gather_out);
    const uint64_t Ki = rg.ki, Ko = rg.kc;
    const RowGuard g = rg.g;
    for (uint64_t i = i0 + threadIdx.x; i < i1; i += BBLOCK) {
        const bool iok = i < Ki;
        const int64_t iv = iok ? idx[i] : 0;
        if (!iok) acc.note((i * D) << 2);
        const bool full = g.rlo <= iv && iv <= g.rhi;
        const uint8_t* trow = T + (uint64_t)iv * rb;
        for (uint64_t col = 0; col < D; ++col) {
            const uint64_t e = i * D + col;
            uint32_t val = 0;
            if (full || elem_ok(g, iv, rb, col, 4)) val = *reinterpret_cast<const uint32_t*>(trow + col * 4);
            else acc.note((e << 2) | 1u);
            if (e < Ko) *reinterpret_cast<uint32_t*>(out + e * 4) = val;
            else acc.note((e << 2) | 2u);
        }
    }
}

// Result of request r, written by the workgroup that finished its last tile (one thread).
__device__ inline void finish_request(const BatchArgs& A, uint32_t r) {
    const BatchReq& q = A.reqs[r];
    const DevTable& t = A.tables[q.client];
    BatchScratch* s = A.scratch + r;
    agile_req_result_dev* res = A.result + r;
    const uint32_t mf = atomicAdd(&s->minfail, 0u);
    if (mf != 0xFFFFFFFFu) {
        res->verdict = A.pv[q.ptr_off + mf];
        res->arg = (int32_t)mf;
        res->owner = A.po[q.ptr_off + mf];
    } else {
        res->verdict = V_ALLOW;
        res->arg = -1;
        res->owner = -1;
    }
    DevLog f{};
    f.first_seq = ~0ull;
    f.first_owner = -1;
    if (q.copy_bytes) {
        const uint64_t n = q.copy_bytes;
        const uint64_t Ks = A.guards[r].copy_ks, Kd = A.guards[r].copy_kd;
        const uint64_t cnt = (n - Ks) + (n - Kd);
        if (cnt) {
            f.count += cnt;
            const uint32_t operand = Ks <= Kd ? 0u : 1u;
            const uint64_t k = operand ? Kd : Ks;
            const uint64_t Aaddr = (operand ? q.copy_dst : q.copy_src) + k;
            uint32_t v;
            int32_t o;
            reason_lane(t, Aaddr, 1, v, o);
            f.first_seq = r;
            f.first_elem = k;
            f.first_addr = Aaddr;
            f.first_width = 1;
            f.first_op = 1;
            f.first_operand = operand;
            f.first_verdict = v;
            f.first_owner = o;
        }
    }
    const unsigned long long gc = atomicAdd(&s->gcount, 0ull);
    if (gc) {
        f.count += gc;
        if (f.first_seq == ~0ull) {
            const unsigned long long key = atomicMin(&s->gminkey, ~0ull);
            const uint64_t D = q.gather_row_bytes / 4;
            const unsigned long long elem = key >> 2;
            const uint32_t operand = (uint32_t)(key & 3u);
            const uint64_t i = elem / D, col = elem % D;
            __int128 Aa;
            uint32_t w = 4;
            if (operand == 0) {
                Aa = (__int128)q.gather_idx + (__int128)(8 * i);
                w = 8;
            } else if (operand == 1) {
                const uint64_t Ki = A.guards[r].gather.ki;
                const int64_t v = i < Ki ? reinterpret_cast<const int64_t*>(q.gather_idx)[i] : 0;
                Aa = (__int128)q.gather_table + (__int128)v * (__int128)q.gather_row_bytes +
                     (__int128)(col * 4);
            } else {
                Aa = (__int128)q.gather_out + (__int128)elem * 4;
            }
            uint32_t v = V_UNMAPPED;
            int32_t o = -1;
            if (Aa >= 0 && Aa <= (__int128)U64MAX) reason_lane(t, (uint64_t)Aa, w, v, o);
            f.first_seq = r;
            f.first_elem = elem;
            f.first_addr = (uint64_t)Aa;
            f.first_width = w;
            f.first_op = 3;
            f.first_operand = operand;
            f.first_verdict = v;
            f.first_owner = o;
        }
    }
    res->fault_count = f.count;
    res->fault_seq = f.first_seq;
    res->fault_elem = f.first_elem;
    res->fault_addr = f.first_addr;
    res->fault_width = f.first_width;
    res->fault_op = f.first_op;
    res->fault_operand = f.first_operand;
    res->fault_verdict = f.first_verdict;
    res->fault_owner = f.first_owner;
    res->fault_reserved = 0;
    __threadfence();
    res->done = 1;
}

__global__ __launch_bounds__(BBLOCK) void k_batch(BatchArgs A) {
    __shared__ uint32_t s_tile, s_next;
    __shared__ uint32_t s_minfail;
    __shared__ uint64_t s_split[LDS_SPLIT];
    const uint32_t tid = threadIdx.x;
    if (tid == 0) s_next = atomicAdd(&A.ctl->next, 1u);
    while (true) {
        __syncthreads();
        if (tid == 0) {
            s_tile = s_next;
            s_minfail = 0xFFFFFFFFu;
        }
        __syncthreads();
        const uint64_t tile = s_tile;
        if (tile >= A.ntiles) break;  // uniform: every wave of the block leaves together
        // claim the next tile now, so the counter's latency overlaps this tile's work (a
        // claimed tile is always processed: the loop only ends on an index past the last tile)
        if (tid == 0) s_next = atomicAdd(&A.ctl->next, 1u);
        const uint32_t r = A.tile_req[tile];
        const BatchReq q = A.reqs[r];
        const DevTable& t = A.tables[q.client];
        uint64_t vt, ct;
        tiles_of(q, A.tile_copy, vt, ct);
        const uint64_t local = tile - A.tstart[r];
        if (local < vt) {
            const uint64_t k0 = local * TILE_PTRS;
            const uint64_t k1 = k0 + TILE_PTRS < q.nptr ? k0 + TILE_PTRS : q.nptr;
            uint32_t mf = 0xFFFFFFFFu;
            validate_tile(t, A.ptrs, q.ptr_off, k0, k1, A.pv, A.po, mf, s_split);
            atomicMin(&s_minfail, mf);
            __syncthreads();
            if (tid == 0 && s_minfail != 0xFFFFFFFFu) atomicMin(&A.scratch[r].minfail, s_minfail);
        } else if (local < vt + ct) {
            // copy tile j of ct takes chunks j, j + ct, j + 2 ct, ... of COPY_CHUNK bytes, so the
            // workgroups working on one request at the same time read one contiguous window
            const uint64_t j = local - vt;
            for (uint64_t o0 = j * COPY_CHUNK; o0 < q.copy_bytes; o0 += ct * COPY_CHUNK) {
                const uint64_t o1 = o0 + COPY_CHUNK < q.copy_bytes ? o0 + COPY_CHUNK : q.copy_bytes;
                copy_tile(reinterpret_cast<uint8_t*>(q.copy_dst),
                          reinterpret_cast<const uint8_t*>(q.copy_src), o0, o1,
                          A.guards[r].copy_ks, A.guards[r].copy_kd);
            }
        } else if (q.gather_n) {
            const uint64_t i0 = (local - vt - ct) * A.tile_rows;
            const uint64_t i1 = i0 + A.tile_rows < q.gather_n ? i0 + A.tile_rows : q.gather_n;
            FaultAcc acc;
            gather_tile(q, A.guards[r].gather, i0, i1, acc);
            const unsigned long long c = wave_sum_u64(acc.cnt);
            const unsigned long long m = wave_min_u64(acc.mk);
            if ((tid & 63u) == 0 && c) {
                atomicAdd(&A.scratch[r].gcount, c);
                atomicMin(&A.scratch[r].gminkey, m);
            }
        }
        __syncthreads();
        if (tid == 0) {
            __threadfence();
            if (atomicSub(&A.scratch[r].remaining, 1u) == 1u) {
                __threadfence();
                finish_request(A, r);
            }
        }
    }
}

hipError_t launch_batch(const BatchArgs& A, const DevInfo& d, hipStream_t s) {
    if (A.ntiles == 0) return hipSuccess;
    uint64_t grid = (uint64_t)d.num_cu;
    if (grid > A.ntiles) grid = A.ntiles;
    hipLaunchKernelGGL(k_batch, dim3((uint32_t)grid), dim3(BBLOCK), 0, s, A);
    return hipGetLastError();
}

void batch_tile_sizes(uint64_t copy_bytes, uint64_t gather_rows, const DevInfo& d,
                      uint64_t& tile_copy, uint64_t& tile_rows) {
    // about two tiles per CU for each kind of work, within [one workgroup pass, the maximum]
    const uint64_t want = 2ull * (uint64_t)(d.num_cu > 0 ? d.num_cu : 1);
    uint64_t tc = copy_bytes / want;
    tc = (tc + COPY_CHUNK - 1) / COPY_CHUNK * COPY_CHUNK;
    tile_copy = tc < COPY_CHUNK ? COPY_CHUNK : (tc > TILE_COPY_MAX ? TILE_COPY_MAX : tc);
    uint64_t tr = gather_rows / want;
    tile_rows = tr < TILE_ROWS_MIN ? TILE_ROWS_MIN : (tr > TILE_ROWS_MAX ? TILE_ROWS_MAX : tr);
}

uint64_t batch_tiles(const BatchReq& q, uint64_t tile_copy, uint64_t tile_rows) {
    const uint64_t vt = (q.nptr + TILE_PTRS - 1) / TILE_PTRS;
    const uint64_t ct = (q.copy_bytes + tile_copy - 1) / tile_copy;
    const uint64_t gt = (q.gather_n + tile_rows - 1) / tile_rows;
    const uint64_t all = vt + ct + gt;
    return all ? all : 1;
}

}  // namespace agile
