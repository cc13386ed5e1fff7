// Client handle tokens: a worker-owned slot table behind opaque 64-bit tokens, so that forged,
// stale and cross-client handles are refused (AgileOS Section IV-C, the CUDA virtualization
// boundary), with a batched device check.
//
// Token = slot << 40 | gen << 16 | tag. The slot (24 bits) indexes the table; gen (24 bits) is
// the slot's generation when the token was minted; tag (16 bits) is the top of SplitMix64
// (Steele, Lea and Flood, 2014: state advanced by the golden gamma, then the published
// finalizer) of key ^ (slot << 24 | gen), under the table's secret key. Minting takes the
// lowest free slot; releasing advances the slot's generation, and a slot released in its last
// generation is retired.
//
// Device record per slot (8 bytes): {owner client, or FREE / RETIRED; gen << 8 | kind}. The
// host keeps the authoritative copy and uploads the dirty slot range in stream order before a
// check that follows a change.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <new>
#include <set>
#include <vector>

#include "device_guard.h"
#include "agile_guard.h"

namespace agile {

constexpr uint32_t SLOT_MAX = 1u << 24;
constexpr uint32_t GEN_MASK = (1u << 24) - 1;
constexpr uint32_t OWNER_FREE = 0xFFFFFFFFu, OWNER_RETIRED = 0xFFFFFFFEu;
constexpr int TBLOCK = 256, TPT = 4;  // tokens per thread per pass

static __host__ __device__ inline uint64_t splitmix64(uint64_t x) {
    uint64_t z = x + 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static __host__ __device__ inline uint32_t token_tag(uint64_t key, uint32_t slot, uint32_t gen) {
    return (uint32_t)(splitmix64(key ^ (((uint64_t)slot << 24) | gen)) >> 48);
}

// One verdict; `rec` is the slot's record (read only when the slot is in range).
static __device__ __forceinline__ uint8_t token_verdict(uint64_t tok, uint32_t slot, uint2 rec, uint64_t key,
                                         uint32_t client, uint32_t want) {
    const uint32_t gen = (uint32_t)(tok >> 16) & GEN_MASK;
    if ((uint32_t)(tok & 0xFFFFu) != token_tag(key, slot, gen)) return AGILE_TOKEN_FORGED;
    const uint32_t rgen = rec.y >> 8, rkind = rec.y & 0xFFu;
    if (gen < rgen || rec.x == OWNER_RETIRED) return AGILE_TOKEN_STALE;
    if (gen > rgen || rec.x == OWNER_FREE) return AGILE_TOKEN_FORGED;
    if (rec.x != client) return AGILE_TOKEN_CROSS_CLIENT;
    if (want != AGILE_TOKEN_ANY_KIND && rkind != want) return AGILE_TOKEN_WRONG_KIND;
    return AGILE_TOKEN_VALID;
}

// Grid-stride over groups of TPT tokens per thread: the token, client and kind loads are
// coalesced, the TPT slot-record loads of a thread are issued together (random 8-byte reads of
// an L2-resident table), then each token gets its verdict.
__global__ __launch_bounds__(TBLOCK) void k_tokens_check(
    const uint2* __restrict__ recs, uint32_t cap, uint64_t key, const uint64_t* __restrict__ tok,
    const uint32_t* __restrict__ cli, const uint8_t* __restrict__ kinds, uint64_t n,
    uint8_t* __restrict__ verdict, int32_t* __restrict__ slot_out) {
    const uint64_t nth = (uint64_t)gridDim.x * TBLOCK;
    for (uint64_t i0 = (uint64_t)blockIdx.x * TBLOCK + threadIdx.x; i0 < n; i0 += nth * TPT) {
        uint64_t t[TPT];
        uint32_t c[TPT], w[TPT], s[TPT];
        uint2 r[TPT];
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            const uint64_t i = i0 + (uint64_t)j * nth;
            const bool in = i < n;
            // streamed once: non-temporal, so they do not push the slot records out of L2
            t[j] = in ? __builtin_nontemporal_load(tok + i) : 0;
            c[j] = in ? __builtin_nontemporal_load(cli + i) : 0;
            w[j] = (in && kinds) ? kinds[i] : AGILE_TOKEN_ANY_KIND;
            s[j] = (uint32_t)(t[j] >> 40);
        }
#pragma unroll
        for (int j = 0; j < TPT; ++j) r[j] = s[j] < cap ? recs[s[j]] : make_uint2(OWNER_FREE, 0);
#pragma unroll
        for (int j = 0; j < TPT; ++j) {
            const uint64_t i = i0 + (uint64_t)j * nth;
            if (i >= n) break;
            const uint8_t v = s[j] < cap ? token_verdict(t[j], s[j], r[j], key, c[j], w[j])
                                         : (uint8_t)AGILE_TOKEN_FORGED;
            __builtin_nontemporal_store(v, verdict + i);
            __builtin_nontemporal_store(v == AGILE_TOKEN_VALID ? (int32_t)s[j] : -1, slot_out + i);
        }
    }
}

}  // namespace agile

namespace {
using agile::DeviceGuard;
}  // namespace

using agile::GEN_MASK;
using agile::OWNER_FREE;
using agile::OWNER_RETIRED;
using agile::SLOT_MAX;
using agile::TBLOCK;
using agile::TPT;
using agile::token_tag;

struct agile_tokens {
    int device = 0;
    uint32_t cap = 0;
    uint64_t key = 0;
    std::vector<uint2> rec;           // authoritative slot records
    std::set<uint32_t> free_slots;    // released, reusable
    uint32_t next_new = 0;
    uint32_t dlo = 0, dhi = 0;        // dirty slot range [dlo, dhi)
    uint2* d_rec = nullptr;
    uint2* h_stage = nullptr;         // pinned staging of the upload
    hipEvent_t upload_done = nullptr;
    bool upload_pending = false;
    hipStream_t upload_stream = nullptr;
    bool uploaded = false;
    std::vector<hipStream_t> streams_used;  // streams that checked since the last upload
};

static void mark_dirty(agile_tokens* ts, uint32_t s) {
    if (ts->dlo >= ts->dhi) {
        ts->dlo = s;
        ts->dhi = s + 1;
    } else {
        ts->dlo = std::min(ts->dlo, s);
        ts->dhi = std::max(ts->dhi, s + 1);
    }
}

int agile_tokens_create(agile_tokens** out, uint32_t capacity, uint64_t key, int device) {
    if (!out || capacity < 1 || capacity > SLOT_MAX) return AGILE_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return AGILE_EDEVICE;
    if (device < 0 || device >= ndev) return AGILE_EINVAL;
    DeviceGuard dg(device);
    if (!dg.ok) return AGILE_EDEVICE;
    agile_tokens* ts = new (std::nothrow) agile_tokens();
    if (!ts) return AGILE_ENOMEM;
    ts->device = device;
    ts->cap = capacity;
    ts->key = key;
    ts->rec.assign(capacity, make_uint2(OWNER_FREE, 0u));
    if (hipMalloc(&ts->d_rec, (size_t)capacity * sizeof(uint2)) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&ts->h_stage), (size_t)capacity * sizeof(uint2),
                      hipHostMallocDefault) != hipSuccess ||
        hipEventCreateWithFlags(&ts->upload_done, hipEventDisableTiming) != hipSuccess) {
        agile_tokens_destroy(ts);
        return AGILE_ENOMEM;
    }
    ts->dlo = 0;
    ts->dhi = capacity;  // the first check uploads every (free) slot
    *out = ts;
    return AGILE_OK;
}

int agile_tokens_destroy(agile_tokens* ts) {
    if (!ts) return AGILE_OK;
    DeviceGuard dg(ts->device);
    int rc = AGILE_OK;
    if (hipDeviceSynchronize() != hipSuccess) rc = AGILE_EDEVICE;
    if (ts->upload_done) (void)hipEventDestroy(ts->upload_done);
    if (ts->h_stage) (void)hipHostFree(ts->h_stage);
    if (ts->d_rec) (void)hipFree(ts->d_rec);
    delete ts;
    return rc;
}

int agile_token_mint(agile_tokens* ts, uint32_t client, uint32_t kind, uint64_t* out_token) {
    if (!ts || !out_token || client >= OWNER_RETIRED || kind >= AGILE_TOKEN_ANY_KIND)
        return AGILE_EINVAL;
    uint32_t s;
    if (!ts->free_slots.empty()) {
        s = *ts->free_slots.begin();
        ts->free_slots.erase(ts->free_slots.begin());
    } else if (ts->next_new < ts->cap) {
        s = ts->next_new++;
    } else {
        return AGILE_ENOSPC;
    }
    const uint32_t gen = ts->rec[s].y >> 8;
    ts->rec[s] = make_uint2(client, (gen << 8) | kind);
    mark_dirty(ts, s);
    *out_token = ((uint64_t)s << 40) | ((uint64_t)gen << 16) | token_tag(ts->key, s, gen);
    return AGILE_OK;
}

// Host-side verdict of one token (the same rule as the device check).
static int host_token_verdict(const agile_tokens* ts, uint64_t tok, uint32_t client, uint32_t* slot) {
    const uint32_t s = (uint32_t)(tok >> 40);
    if (s >= ts->cap) return AGILE_TOKEN_FORGED;
    *slot = s;
    const uint2 r = ts->rec[s];
    const uint32_t gen = (uint32_t)(tok >> 16) & GEN_MASK;
    if ((uint32_t)(tok & 0xFFFFu) != token_tag(ts->key, s, gen)) return AGILE_TOKEN_FORGED;
    if (gen < (r.y >> 8) || r.x == OWNER_RETIRED) return AGILE_TOKEN_STALE;
    if (gen > (r.y >> 8) || r.x == OWNER_FREE) return AGILE_TOKEN_FORGED;
    if (r.x != client) return AGILE_TOKEN_CROSS_CLIENT;
    return AGILE_TOKEN_VALID;
}

int agile_token_release(agile_tokens* ts, uint64_t token, uint32_t client) {
    if (!ts) return AGILE_EINVAL;
    uint32_t s = 0;
    if (host_token_verdict(ts, token, client, &s) != AGILE_TOKEN_VALID) return AGILE_ENOENT;
    const uint32_t gen = ts->rec[s].y >> 8;
    if (gen == GEN_MASK) {
        ts->rec[s] = make_uint2(OWNER_RETIRED, gen << 8);
    } else {
        ts->rec[s] = make_uint2(OWNER_FREE, (gen + 1) << 8);
        ts->free_slots.insert(s);
    }
    mark_dirty(ts, s);
    return AGILE_OK;
}

// Bring the device records up to date on stream s (in stream order).
static int tokens_prepare(agile_tokens* ts, hipStream_t s) {
    if (ts->dlo < ts->dhi) {
        // checks queued on other streams read the records about to be overwritten
        for (hipStream_t o : ts->streams_used) {
            if (o == s) continue;
            hipEvent_t ev;
            if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return AGILE_EDEVICE;
            const bool ok = hipEventRecord(ev, o) == hipSuccess && hipStreamWaitEvent(s, ev, 0) == hipSuccess;
            (void)hipEventDestroy(ev);
            if (!ok) return AGILE_EDEVICE;
        }
        ts->streams_used.clear();
        // the staging buffer may still feed the previous upload
        if (ts->upload_pending && hipEventSynchronize(ts->upload_done) != hipSuccess)
            return AGILE_EDEVICE;
        const size_t lo = ts->dlo, cnt = (size_t)ts->dhi - ts->dlo;
        std::copy(ts->rec.begin() + lo, ts->rec.begin() + lo + cnt, ts->h_stage + lo);
        if (hipMemcpyAsync(ts->d_rec + lo, ts->h_stage + lo, cnt * sizeof(uint2),
                           hipMemcpyHostToDevice, s) != hipSuccess ||
            hipEventRecord(ts->upload_done, s) != hipSuccess)
            return AGILE_EDEVICE;
        ts->upload_pending = true;
        ts->upload_stream = s;
        ts->uploaded = true;
        ts->dlo = ts->dhi = 0;
    } else if (ts->uploaded && ts->upload_stream != s) {
        if (hipStreamWaitEvent(s, ts->upload_done, 0) != hipSuccess) return AGILE_EDEVICE;
    }
    if (std::find(ts->streams_used.begin(), ts->streams_used.end(), s) == ts->streams_used.end())
        ts->streams_used.push_back(s);
    return AGILE_OK;
}

int agile_tokens_check(agile_tokens* ts, const uint64_t* d_tokens, const uint32_t* d_clients,
                       const uint8_t* d_kinds, uint64_t n, uint8_t* d_verdict, int32_t* d_slot,
                       void* stream) {
    if (!ts) return AGILE_EINVAL;
    if (n == 0) return AGILE_OK;
    if (!d_tokens || !d_clients || !d_verdict || !d_slot || ((uint64_t)d_tokens & 7) ||
        ((uint64_t)d_clients & 3) || ((uint64_t)d_slot & 3))
        return AGILE_EINVAL;
    DeviceGuard dg(ts->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int rc = tokens_prepare(ts, s);
    if (rc != AGILE_OK) return rc;
    const uint64_t per_block = (uint64_t)TBLOCK * TPT;
    uint64_t grid = (n + per_block - 1) / per_block;
    // one pass (0.603 ms for 2^26 tokens, against 0.628 ms with 8 workgroups per CU looping)
    const uint64_t cap = 1ull << 30;
    if (grid > cap) grid = cap;
    hipLaunchKernelGGL(agile::k_tokens_check, dim3((uint32_t)grid), dim3(TBLOCK), 0, s, ts->d_rec,
                       ts->cap, ts->key, d_tokens, d_clients, d_kinds, n, d_verdict, d_slot);
    return hipGetLastError() == hipSuccess ? AGILE_OK : AGILE_EDEVICE;
}
