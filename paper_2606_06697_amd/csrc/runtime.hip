// Host runtime of libagile_guard.so: the C ABI declared in include/agile_guard.h.
//
// A handle keeps the allocation table (AgileOS Section V-A/V-C: base and live size of every
// range, plus its kind from the Table I layout) as a sorted host mirror with stable ids, and a
// device image rebuilt from it when the table changed. The image is uploaded lazily by the next
// launch, on that launch's stream, after every other stream that used the handle has been made
// to wait for its earlier work; the pinned staging buffer is reused only after its previous
// upload completed. Guarded calls take consecutive sequence numbers (the first-fault order).
#include <algorithm>
#include <atomic>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <unordered_map>
#include <vector>

#include "device_guard.h"
#include "agile_guard.h"
#include "agile_aperture.h"
#include "launch.h"

using namespace agile;

namespace {

struct Entry {
    uint64_t base, end;
    int32_t id;
    uint8_t kind;
    uint8_t backed;  // inserted with AGILE_RANGE_BACKED (mapped memory, REPORT may touch it)
};

using agile::DeviceGuard;

constexpr uint32_t MAX_CAPACITY = 1u << 26;
constexpr int32_t MAX_ID = (1 << 30) - 1;

// One device copy of the table image (layout below) and its upload state.
struct Image {
    uint64_t* split64 = nullptr;
    uint32_t* split32 = nullptr;
    PairRec* rec = nullptr;
    uint32_t* radix = nullptr;
    uint4* nrec = nullptr;
    uint8_t* backed = nullptr;       // per bucket: bit 0 first range backed, bit 1 second
    void* stage = nullptr;           // pinned staging the upload copies from
    hipEvent_t ready = nullptr;      // recorded after the upload into this image
    hipStream_t ready_stream = nullptr;
    bool uploaded = false;
    bool ready_done = false;         // the upload is known to have completed
    // Recorded, when this image stopped being current, on every stream that had launched with
    // it: the next upload into it waits for these (that is, for its last readers) only.
    std::vector<hipEvent_t> retired;
};

void drop_events(std::vector<hipEvent_t>& v) {
    for (hipEvent_t e : v) (void)hipEventDestroy(e);
    v.clear();
}

// Device scratch of the sorted scatter-add, grown on demand and released in stream order: the
// stream of the call that grows it first waits (on the device) for every other stream that used
// the old buffer, then frees it and allocates the new one on that stream. Nothing waits on the
// host, and launches on unrelated streams are not held up.
struct StreamScratch {
    void* buf = nullptr;
    size_t cap = 0;
    std::vector<hipStream_t> users;  // streams that launched with buf

    // null when it cannot grow (the caller then takes a path without scratch)
    void* get(size_t need, hipStream_t s) {
        if (need <= cap) {
            if (std::find(users.begin(), users.end(), s) == users.end()) users.push_back(s);
            return buf;
        }
        if (buf) {
            for (hipStream_t o : users) {
                if (o == s) continue;
                hipEvent_t e;
                if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) return nullptr;
                const bool ok = hipEventRecord(e, o) == hipSuccess && hipStreamWaitEvent(s, e, 0) == hipSuccess;
                (void)hipEventDestroy(e);
                if (!ok) return nullptr;
            }
            if (hipFreeAsync(buf, s) != hipSuccess) return nullptr;
            buf = nullptr;
            cap = 0;
            users.clear();
        }
        const size_t want = need + need / 4;
        if (hipMallocAsync(&buf, want, s) != hipSuccess) {
            (void)hipGetLastError();
            buf = nullptr;
            return nullptr;
        }
        cap = want;
        users.assign(1, s);
        return buf;
    }

    // once no queued work can use it any more
    void release() {
        if (buf) (void)hipFreeAsync(buf, nullptr);
        buf = nullptr;
        cap = 0;
        users.clear();
    }
};

}  // namespace

struct agile_rt {
    int device = 0;
    uint32_t capacity = 0;
    uint32_t cap_nb = 0;
    std::vector<Entry> entries;                 // sorted by base
    std::unordered_map<int32_t, uint64_t> by_id;  // id -> base
    int32_t next_id = 0;
    bool dirty = true;
    unsigned long long seq = 0;
    DevInfo info{};
    size_t lds_budget = 0;
    bool wide_only = false;  // never build narrow records (AGILE_WIDE_RECORDS=1)
    uint32_t min_lift = 0;   // least unrolled lifting depth of the search (AGILE_MIN_LIFT)
    // two device images with their pinned staging: a table change is built into the image that
    // is not current, so launches still reading the current one are not waited for
    void* dmem = nullptr;
    Image img[2];
    int cur = 0;
    DevLog* d_log = nullptr;
    DevTable tab{};
    size_t stage_bytes = 0;
    agile_fault* hlog = nullptr;
    unsigned long long* htrap = nullptr;  // log count before / after a TRAP-policy call
    uint8_t* q_ptr = nullptr;             // quarantine of the SINK policy (caller-owned)
    uint64_t q_bytes = 0;
    bool retired = false;                 // retired by a TRAP-policy violation
    std::vector<hipStream_t> streams_used;  // streams that launched with the current image
    StreamScratch sa;  // sort scratch of the scatter-add (grown on demand)
};

// Image layout: split64 | split32 | (64-byte aligned) rec | radix
static size_t rec_offset(uint32_t cap_nb) {
    return (((size_t)cap_nb * 12 + 63) / 64) * 64;
}
static size_t radix_offset(uint32_t cap_nb) {
    return rec_offset(cap_nb) + (size_t)cap_nb * sizeof(PairRec);
}
static size_t nrec_offset(uint32_t cap_nb) {
    return radix_offset(cap_nb) + (((size_t)MAX_RADIX * 4 + 63) / 64) * 64;
}
static size_t backed_offset(uint32_t cap_nb) {
    return nrec_offset(cap_nb) + (size_t)cap_nb * 16;
}
static size_t image_bytes(uint32_t cap_nb) {
    return backed_offset(cap_nb) + (((size_t)cap_nb + 63) / 64) * 64;
}

static uint32_t bitlen(uint64_t x) {
    uint32_t b = 0;
    while (x) {
        ++b;
        x >>= 1;
    }
    return b;
}

static uint32_t ctz64(uint64_t x) {
    uint32_t c = 0;
    while (c < 64 && !((x >> c) & 1)) ++c;
    return c;
}

// Packed 16-byte records: relative to the bucket base, the second range's base in units of 2^sb
// and the first range's end share one 32-bit word, the second range's end takes another.
static void build_narrow(DevTable& t, const uint64_t* s64, const PairRec* rec, uint32_t* nrec) {
    t.narrow = 0;
    const uint32_t nb = t.nb;
    if (nb == 0 || t.rlog2 != 0 || t.rlevels > 8) return;
    uint32_t sb = 32;
    uint64_t me0 = 0, me1 = 0;
    for (uint32_t b = 0; b < nb; ++b) {
        me0 = std::max(me0, rec[b].end0 - s64[b]);
        if (rec[b].base1 != U64MAX) {
            sb = std::min(sb, ctz64(rec[b].base1 - s64[b]));
            me1 = std::max(me1, rec[b].end1 - s64[b]);
        }
    }
    if (sb >= 32) sb = 0;  // no bucket holds a second range
    // a missing second range gets a base at or past the first end and an end of 0, so an
    // address past the first range classifies as unmapped either way
    auto ob1 = [&](uint32_t b) -> uint64_t {
        return rec[b].base1 != U64MAX ? (rec[b].base1 - s64[b]) >> sb
                                      : ((rec[b].end0 - s64[b]) + (1ull << sb) - 1) >> sb;
    };
    uint64_t mb1 = 0;
    for (uint32_t b = 0; b < nb; ++b) mb1 = std::max(mb1, ob1(b));
    const uint32_t w1 = bitlen(mb1), w2 = bitlen(me0), w3 = bitlen(me1);
    if (w1 + w2 > 32 || w3 > 32) return;
    // the kernel rebuilds the second base as a 32-bit value (field << sb)
    if (sb >= 32 || (mb1 << sb) > 0xFFFFFFFFull) return;
    for (uint32_t b = 0; b < nb; ++b) {
        const bool two = rec[b].base1 != U64MAX;
        nrec[4 * b + 0] = (uint32_t)(ob1(b) | ((rec[b].end0 - s64[b]) << w1));
        nrec[4 * b + 1] = two ? (uint32_t)(rec[b].end1 - s64[b]) : 0u;
        nrec[4 * b + 2] = rec[b].meta0;
        nrec[4 * b + 3] = two ? rec[b].meta1 : 0u;
    }
    t.narrow = 1;
    t.sb = sb;
    t.w1 = w1;
}


// Validation search geometry for nb buckets with first bases s64[]: how many splitters the LDS
// holds (every 2^rlog2-th) and a radix index over them that bounds each lookup to a run of at
// most 2^rlevels - 1 splitters; the LDS array carries 2^rlevels sentinels after the splitters.
static uint32_t lift_levels(uint32_t rlevels) {
    // the unrolled lifting exists for 2, 4, 6 and 8 levels; reading more levels than needed
    // stays correct (the predicate is monotone over the sentinel padding)
    if (rlevels <= 8) return rlevels <= 2 ? 2 : (rlevels + 1) & ~1u;
    return rlevels;
}

// min_lift (2, 4, 6 or 8; 0 for none) raises the unrolled lifting depth for tests
// (AGILE_MIN_LIFT): every depth variant of the packed-record search is then reachable on any table.
static void search_geometry(DevTable& t, const uint64_t* s64, uint32_t* radix, size_t budget,
                            uint32_t min_lift) {
    const uint32_t nb = t.nb;
    const size_t ks = t.compressed ? 4 : 8;
    t.rlog2 = 0;
    if (nb == 0) {
        t.ntop = 0;
        t.nr = 1;
        t.rsh = t.shift;
        t.xs = 0;
        t.rlevels = 0;
        t.lift = 0;
        t.pad = 1;
        radix[0] = radix[1] = 0;
        t.lds_bytes = 16 + 8;
        return;
    }
    const uint64_t gmin = s64[0];
    for (uint32_t rlog2 = 0; rlog2 < 32; ++rlog2) {
        const uint32_t ntop = (uint32_t)(((uint64_t)nb + (1ull << rlog2) - 1) >> rlog2);
        const uint64_t span = s64[(uint64_t)(ntop - 1) << rlog2] - gmin;
        const uint32_t bits = bitlen(span);
        for (int R = 14; R >= 0; --R) {
            if (R > 0 && (1ull << (R - 1)) >= ntop) continue;  // no more radix bins than splitters
            const uint32_t rsh = std::max<uint32_t>(bits > (uint32_t)R ? bits - R : 0, t.shift);
            const uint32_t nr = (uint32_t)(span >> rsh) + 1;
            if ((size_t)(nr + 1) * 4 + (size_t)ntop * ks > budget) continue;
            uint32_t k = 0, maxm = 0;
            for (uint32_t r = 0; r < nr; ++r) {
                const uint64_t bound = gmin + ((uint64_t)r << rsh);
                while (k < ntop && s64[(uint64_t)k << rlog2] < bound) ++k;
                radix[r] = k;
            }
            radix[nr] = ntop;
            for (uint32_t r = 0; r < nr; ++r) maxm = std::max(maxm, radix[r + 1] - radix[r]);
            const uint32_t rlevels = bitlen(maxm);
            const uint32_t lift = rlevels <= 8 ? std::max(lift_levels(rlevels), min_lift)
                                               : lift_levels(rlevels);
            const size_t top_bytes = ((((size_t)ntop + (1ull << lift)) * ks + 15) / 16) * 16;
            const size_t need = top_bytes + (size_t)(nr + 1) * 4;
            if (need > budget) continue;
            t.rlog2 = rlog2;
            t.ntop = ntop;
            t.nr = nr;
            t.rsh = rsh;
            t.xs = std::min<uint32_t>(rsh - t.shift, 31);
            t.rlevels = rlevels;
            t.lift = lift;
            t.pad = 1u << lift;
            t.lds_bytes = (uint32_t)need;
            return;
        }
    }
}

static void note_stream(agile_rt* rt, hipStream_t s) {
    for (hipStream_t x : rt->streams_used)
        if (x == s) return;
    rt->streams_used.push_back(s);
}

// Build the table into the image that is not current and queue its upload on stream s; that
// image then becomes current. The upload waits on the device for the launches that read this
// image while it was last current (two versions ago), not for those reading the current one.
static int upload(agile_rt* rt, hipStream_t s) {
    if (!rt->dirty) return AGILE_OK;
    const int x = 1 - rt->cur;
    Image& im = rt->img[x];
    // the staging buffer may still feed this image's previous upload
    if (im.uploaded && hipEventSynchronize(im.ready) != hipSuccess) return AGILE_EDEVICE;
    const uint32_t n = (uint32_t)rt->entries.size();
    const uint32_t nb = (n + 1) / 2;
    uint8_t* h = static_cast<uint8_t*>(im.stage);
    uint64_t* s64 = reinterpret_cast<uint64_t*>(h);
    uint32_t* s32 = reinterpret_cast<uint32_t*>(h + (size_t)rt->cap_nb * 8);
    PairRec* rec = reinterpret_cast<PairRec*>(h + rec_offset(rt->cap_nb));
    uint32_t* radix = reinterpret_cast<uint32_t*>(h + radix_offset(rt->cap_nb));
    uint32_t* nrec = reinterpret_cast<uint32_t*>(h + nrec_offset(rt->cap_nb));
    uint8_t* bk = h + backed_offset(rt->cap_nb);
    const auto& E = rt->entries;
    for (uint32_t b = 0; b < nb; ++b) {
        const Entry& e0 = E[2 * b];
        s64[b] = e0.base;
        bk[b] = (uint8_t)(e0.backed | ((2 * b + 1 < n ? E[2 * b + 1].backed : 0) << 1));
        PairRec r;
        r.end0 = e0.end;
        r.meta0 = ((uint32_t)e0.id << 2) | e0.kind;
        if (2 * b + 1 < n) {
            const Entry& e1 = E[2 * b + 1];
            r.base1 = e1.base;
            r.end1 = e1.end;
            r.meta1 = ((uint32_t)e1.id << 2) | e1.kind;
        } else {
            r.base1 = U64MAX;
            r.end1 = 0;
            r.meta1 = 0;
        }
        rec[b] = r;
    }
    DevTable t{};
    t.split64 = im.split64;
    t.split32 = im.split32;
    t.rec = im.rec;
    t.radix = im.radix;
    t.backed = im.backed;
    t.nb = nb;
    t.compressed = 0;
    if (nb > 0) {
        const uint64_t gmin = s64[0];
        t.gmin = gmin;
        const uint64_t span = s64[nb - 1] - gmin;
        uint32_t sh = 0;
        while (sh < 63 && (span >> sh) > 0xFFFFFFFEull) ++sh;
        const uint64_t mask = (sh == 0) ? 0 : ((1ull << sh) - 1);
        bool ok = (span >> sh) <= 0xFFFFFFFEull;
        for (uint32_t b = 0; ok && b < nb; ++b) ok = ((s64[b] - gmin) & mask) == 0;
        if (ok) {
            for (uint32_t b = 0; b < nb; ++b) s32[b] = (uint32_t)((s64[b] - gmin) >> sh);
            t.compressed = 1;
            t.shift = sh;
        }
    }
    search_geometry(t, s64, radix, std::min(rt->lds_budget, rt->info.lds_per_block), rt->min_lift);
    t.nrec = im.nrec;
    if (!rt->wide_only) build_narrow(t, s64, rec, nrec);
    // the last readers of image x
    for (hipEvent_t e : im.retired)
        if (hipStreamWaitEvent(s, e, 0) != hipSuccess) return AGILE_EDEVICE;
    drop_events(im.retired);
    // retire the current image: mark the end of every launch that reads it
    Image& old = rt->img[rt->cur];
    drop_events(old.retired);
    for (hipStream_t o : rt->streams_used) {
        hipEvent_t ev;
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) return AGILE_EDEVICE;
        old.retired.push_back(ev);
        if (hipEventRecord(ev, o) != hipSuccess) return AGILE_EDEVICE;
    }
    rt->streams_used.clear();
    if (nb > 0) {
        if (hipMemcpyAsync(im.split64, s64, (size_t)nb * 8, hipMemcpyHostToDevice, s) != hipSuccess)
            return AGILE_EDEVICE;
        if (t.compressed &&
            hipMemcpyAsync(im.split32, s32, (size_t)nb * 4, hipMemcpyHostToDevice, s) != hipSuccess)
            return AGILE_EDEVICE;
        if (hipMemcpyAsync(im.rec, rec, (size_t)nb * sizeof(PairRec), hipMemcpyHostToDevice, s) !=
                hipSuccess ||
            hipMemcpyAsync(im.backed, bk, nb, hipMemcpyHostToDevice, s) != hipSuccess)
            return AGILE_EDEVICE;
    }
    if (t.narrow &&
        hipMemcpyAsync(im.nrec, nrec, (size_t)nb * 16, hipMemcpyHostToDevice, s) != hipSuccess)
        return AGILE_EDEVICE;
    if (hipMemcpyAsync(im.radix, radix, (size_t)(t.nr + 1) * 4, hipMemcpyHostToDevice, s) !=
            hipSuccess ||
        hipEventRecord(im.ready, s) != hipSuccess)
        return AGILE_EDEVICE;
    im.uploaded = true;
    im.ready_done = false;
    im.ready_stream = s;
    rt->cur = x;
    rt->tab = t;
    rt->dirty = false;
    return AGILE_OK;
}

// Every launch with the table: bring the image up to date, and make sure a launch on another
// stream than the one that uploaded the current image waits for that upload.
static int prepare(agile_rt* rt, hipStream_t s) {
    int rc = upload(rt, s);
    if (rc != AGILE_OK) return rc;
    Image& im = rt->img[rt->cur];
    if (im.uploaded && !im.ready_done && im.ready_stream != s) {
        const hipError_t q = hipEventQuery(im.ready);
        if (q == hipSuccess) {
            im.ready_done = true;
        } else if (q != hipErrorNotReady || hipStreamWaitEvent(s, im.ready, 0) != hipSuccess) {
            return AGILE_EDEVICE;
        }
    }
    note_stream(rt, s);
    return AGILE_OK;
}

extern "C" {

const char* agile_strerror(int code) {
    switch (code) {
        case AGILE_OK: return "ok";
        case AGILE_EINVAL: return "invalid argument";
        case AGILE_ENOMEM: return "out of memory";
        case AGILE_EOVERLAP: return "range overlaps an existing range";
        case AGILE_ENOENT: return "no such range id";
        case AGILE_ENOSPC: return "range table full";
        case AGILE_EDEVICE: return "HIP runtime error";
        case AGILE_EFAULTED: return "guarded access denied (fault log not empty)";
        case AGILE_ETRAPPED: return "handle retired by a violation under the trap policy";
        case AGILE_ENOTSUP: return "the device does not support virtual memory management";
        case AGILE_E2BIG: return "more rows than the no-allocation scatter-add's fixed scratch holds";
        default: return "unknown status";
    }
}

}  // extern "C"

// ---- fixed scratch of the no-allocation scatter-add ------------------------------------
// One copy per GPU (a device global, held until the process ends). In host code the name only
// stands in for the symbol: kernels get the address hipGetSymbolAddress reports for the device.
static __device__ __align__(256) unsigned char scratch[AGILE_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
std::atomic<void*> g_scratch_ptr[NOALLOC_MAX_DEVICES];  // device address of `scratch`, per device
}  // namespace

// The device address of `scratch` on `device`, looked up once with that device current (the
// caller makes it current); null if the lookup failed.
static void* noalloc_scratch(int device) {
    if (device < 0 || device >= NOALLOC_MAX_DEVICES) return nullptr;
    void* p = g_scratch_ptr[device].load(std::memory_order_acquire);
    if (p) return p;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    p = g_scratch_ptr[device].load(std::memory_order_relaxed);
    if (p) return p;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
        (void)hipGetLastError();
        return nullptr;
    }
    g_scratch_ptr[device].store(p, std::memory_order_release);
    return p;
}

extern "C" {

int agile_rt_create(agile_rt** out, uint32_t capacity, int device) {
    if (!out || capacity < 1 || capacity > MAX_CAPACITY) return AGILE_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return AGILE_EDEVICE;
    if (device < 0 || device >= ndev) return AGILE_EINVAL;
    DeviceGuard dg(device);
    if (!dg.ok) return AGILE_EDEVICE;
    agile_rt* rt = new (std::nothrow) agile_rt();
    if (!rt) return AGILE_ENOMEM;
    rt->device = device;
    rt->capacity = capacity;
    rt->cap_nb = (capacity + 1) / 2;
    hipDeviceProp_t p;
    if (hipGetDeviceProperties(&p, device) != hipSuccess) {
        delete rt;
        return AGILE_EDEVICE;
    }
    rt->info.num_cu = p.multiProcessorCount;
    rt->info.lds_per_block = p.sharedMemPerBlock;
    rt->info.lds_per_cu = p.maxSharedMemoryPerMultiProcessor;
    // set-up of the device: the no-allocation scatter-add's scratch address (looked up again by
    // that entry point if this fails)
    (void)noalloc_scratch(device);
    rt->lds_budget = 160 * 1024;
    if (const char* e = std::getenv("AGILE_LDS_BUDGET")) {
        long v = std::strtol(e, nullptr, 10);
        if (v >= 1024) rt->lds_budget = (size_t)v;
    }
    if (const char* e = std::getenv("AGILE_WIDE_RECORDS")) rt->wide_only = std::atoi(e) != 0;
    if (const char* e = std::getenv("AGILE_MIN_LIFT")) {
        const int v = std::atoi(e);
        if (v == 2 || v == 4 || v == 6 || v == 8) rt->min_lift = (uint32_t)v;
    }
    rt->stage_bytes = image_bytes(rt->cap_nb);
    const size_t img_bytes = ((rt->stage_bytes + 255) / 256) * 256;
    const size_t dev_bytes = 2 * img_bytes + sizeof(DevLog);
    if (hipMalloc(&rt->dmem, dev_bytes) != hipSuccess) {
        delete rt;
        return AGILE_ENOMEM;
    }
    for (int k = 0; k < 2; ++k) {
        uint8_t* d = static_cast<uint8_t*>(rt->dmem) + k * img_bytes;
        Image& im = rt->img[k];
        im.split64 = reinterpret_cast<uint64_t*>(d);
        im.split32 = reinterpret_cast<uint32_t*>(d + (size_t)rt->cap_nb * 8);
        im.rec = reinterpret_cast<PairRec*>(d + rec_offset(rt->cap_nb));
        im.radix = reinterpret_cast<uint32_t*>(d + radix_offset(rt->cap_nb));
        im.nrec = reinterpret_cast<uint4*>(d + nrec_offset(rt->cap_nb));
        im.backed = d + backed_offset(rt->cap_nb);
        if (hipHostMalloc(&im.stage, rt->stage_bytes, hipHostMallocDefault) != hipSuccess ||
            hipEventCreateWithFlags(&im.ready, hipEventDisableTiming) != hipSuccess) {
            agile_rt_destroy(rt);
            return AGILE_ENOMEM;
        }
    }
    rt->d_log = reinterpret_cast<DevLog*>(static_cast<uint8_t*>(rt->dmem) + 2 * img_bytes);
    if (
        hipHostMalloc(reinterpret_cast<void**>(&rt->hlog), sizeof(agile_fault),
                      hipHostMallocDefault) != hipSuccess ||
        hipHostMalloc(reinterpret_cast<void**>(&rt->htrap), 2 * sizeof(unsigned long long),
                      hipHostMallocDefault) != hipSuccess) {
        agile_rt_destroy(rt);
        return AGILE_ENOMEM;
    }
    if (launch_log_reset(rt->d_log, nullptr) != hipSuccess ||
        hipDeviceSynchronize() != hipSuccess) {
        agile_rt_destroy(rt);
        return AGILE_EDEVICE;
    }
    *out = rt;
    return AGILE_OK;
}

int agile_rt_destroy(agile_rt* rt) {
    if (!rt) return AGILE_OK;
    DeviceGuard dg(rt->device);
    int rc = AGILE_OK;
    if (hipDeviceSynchronize() != hipSuccess) rc = AGILE_EDEVICE;
    for (Image& im : rt->img) {
        if (im.ready) (void)hipEventDestroy(im.ready);
        if (im.stage) (void)hipHostFree(im.stage);
        drop_events(im.retired);
    }
    if (rt->hlog) (void)hipHostFree(rt->hlog);
    if (rt->htrap) (void)hipHostFree(rt->htrap);
    if (rt->dmem) (void)hipFree(rt->dmem);
    const bool had_scratch = rt->sa.buf != nullptr;
    rt->sa.release();  // the device is idle (synchronized above)
    if (had_scratch && hipStreamSynchronize(nullptr) != hipSuccess) rc = AGILE_EDEVICE;
    delete rt;
    return rc;
}

// kind: an AGILE_KIND_* value, optionally with AGILE_RANGE_BACKED
static int check_range(uint64_t base, uint64_t size, uint32_t kind) {
    const uint32_t k = kind & ~(uint32_t)AGILE_RANGE_BACKED;
    if (k > AGILE_KIND_MMIO || size < 1 || size > U64MAX - base) return AGILE_EINVAL;
    return AGILE_OK;
}
static Entry make_entry(uint64_t base, uint64_t size, int32_t id, uint32_t kind) {
    return Entry{base, base + size, id, (uint8_t)(kind & ~(uint32_t)AGILE_RANGE_BACKED),
                 (uint8_t)((kind & AGILE_RANGE_BACKED) ? 1 : 0)};
}

int agile_rt_insert(agile_rt* rt, uint64_t base, uint64_t size, uint32_t kind, int32_t* out_id) {
    if (!rt) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    int rc = check_range(base, size, kind);
    if (rc != AGILE_OK) return rc;
    if (rt->entries.size() >= rt->capacity || rt->next_id > MAX_ID) return AGILE_ENOSPC;
    const uint64_t end = base + size;
    auto& E = rt->entries;
    auto it = std::upper_bound(E.begin(), E.end(), base,
                               [](uint64_t v, const Entry& e) { return v < e.base; });
    if (it != E.begin() && std::prev(it)->end > base) return AGILE_EOVERLAP;
    if (it != E.end() && it->base < end) return AGILE_EOVERLAP;
    const int32_t id = rt->next_id++;
    E.insert(it, make_entry(base, size, id, kind));
    rt->by_id[id] = base;
    rt->dirty = true;
    if (out_id) *out_id = id;
    return AGILE_OK;
}

int agile_rt_insert_many(agile_rt* rt, const uint64_t* base, const uint64_t* size,
                         const uint8_t* kind, uint32_t n, int32_t* out_ids) {
    if (!rt) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    if (n == 0) return AGILE_OK;
    if (!base || !size || !kind) return AGILE_EINVAL;
    for (uint32_t i = 0; i < n; ++i) {
        int rc = check_range(base[i], size[i], kind[i]);
        if (rc != AGILE_OK) return rc;
    }
    if ((uint64_t)rt->entries.size() + n > rt->capacity ||
        (int64_t)rt->next_id + (int64_t)n - 1 > MAX_ID)
        return AGILE_ENOSPC;
    std::vector<Entry> add(n);
    for (uint32_t i = 0; i < n; ++i)
        add[i] = make_entry(base[i], size[i], rt->next_id + (int32_t)i, kind[i]);
    std::vector<Entry> merged;
    merged.reserve(rt->entries.size() + n);
    std::vector<Entry> sorted_add = add;
    std::sort(sorted_add.begin(), sorted_add.end(),
              [](const Entry& a, const Entry& b) { return a.base < b.base; });
    std::merge(rt->entries.begin(), rt->entries.end(), sorted_add.begin(), sorted_add.end(),
               std::back_inserter(merged),
               [](const Entry& a, const Entry& b) { return a.base < b.base; });
    for (size_t i = 1; i < merged.size(); ++i)
        if (merged[i - 1].end > merged[i].base) return AGILE_EOVERLAP;
    rt->entries.swap(merged);
    for (uint32_t i = 0; i < n; ++i) {
        rt->by_id[add[i].id] = add[i].base;
        if (out_ids) out_ids[i] = add[i].id;
    }
    rt->next_id += (int32_t)n;
    rt->dirty = true;
    return AGILE_OK;
}

int agile_rt_remove(agile_rt* rt, int32_t id) {
    if (!rt) return AGILE_EINVAL;
    auto f = rt->by_id.find(id);
    if (f == rt->by_id.end()) return AGILE_ENOENT;
    const uint64_t b = f->second;
    auto& E = rt->entries;
    auto it = std::lower_bound(E.begin(), E.end(), b,
                               [](const Entry& e, uint64_t v) { return e.base < v; });
    if (it == E.end() || it->base != b) return AGILE_ENOENT;
    E.erase(it);
    rt->by_id.erase(f);
    rt->dirty = true;
    return AGILE_OK;
}

int agile_rt_set_quarantine(agile_rt* rt, void* d_quarantine, uint64_t bytes) {
    if (!rt) return AGILE_EINVAL;
    if (!d_quarantine && bytes == 0) {
        rt->q_ptr = nullptr;
        rt->q_bytes = 0;
        return AGILE_OK;
    }
    if (!d_quarantine || bytes < 256 || bytes > (1ull << 40) || (bytes & (bytes - 1)) ||
        ((uint64_t)d_quarantine & 255))
        return AGILE_EINVAL;
    rt->q_ptr = static_cast<uint8_t*>(d_quarantine);
    rt->q_bytes = bytes;
    return AGILE_OK;
}

int agile_rt_clear(agile_rt* rt) {
    if (!rt) return AGILE_EINVAL;
    rt->entries.clear();
    rt->by_id.clear();
    rt->dirty = true;
    return AGILE_OK;
}

int agile_rt_count(const agile_rt* rt, uint32_t* out_n) {
    if (!rt || !out_n) return AGILE_EINVAL;
    *out_n = (uint32_t)rt->entries.size();
    return AGILE_OK;
}

int agile_rt_sync(agile_rt* rt, void* stream) {
    if (!rt) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    return prepare(rt, static_cast<hipStream_t>(stream));
}

static int validate_common(agile_rt* rt, const agile_ptr* d_q, uint64_t n, uint8_t* d_verdict,
                           int32_t* d_owner, bool dma, void* stream) {
    if (!rt) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    if (n == 0) return AGILE_OK;
    if (!d_q || !d_verdict || !d_owner || ((uint64_t)d_q & 15)) return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = prepare(rt, s);
    if (rc != AGILE_OK) return rc;
    if (launch_validate(rt->tab, rt->info, d_q, n, d_verdict, d_owner, dma, s) != hipSuccess)
        return AGILE_EDEVICE;
    return AGILE_OK;
}

int agile_validate_ptrs(agile_rt* rt, const agile_ptr* d_q, uint64_t n, uint8_t* d_verdict,
                        int32_t* d_owner, void* stream) {
    return validate_common(rt, d_q, n, d_verdict, d_owner, false, stream);
}

int agile_validate_dma(agile_rt* rt, const agile_ptr* d_q, uint64_t n, uint8_t* d_verdict,
                       int32_t* d_owner, void* stream) {
    return validate_common(rt, d_q, n, d_verdict, d_owner, true, stream);
}

static bool policy_ok(int policy) {
    return policy == AGILE_POLICY_SUPPRESS_LOG || policy == AGILE_POLICY_SUPPRESS_ONLY ||
           policy == AGILE_POLICY_TRAP || policy == AGILE_POLICY_SINK ||
           policy == AGILE_POLICY_REPORT || policy == AGILE_POLICY_REMAP;
}

static bool redirecting(int policy) {
    return policy == AGILE_POLICY_SINK || policy == AGILE_POLICY_REPORT ||
           policy == AGILE_POLICY_REMAP;
}

// The redirect of a SINK, REPORT or REMAP call (EINVAL: SINK without a quarantine).
static int redirect_of(const agile_rt* rt, int policy, Redirect* r) {
    *r = Redirect{};
    if (policy == AGILE_POLICY_SINK) {
        if (!rt->q_ptr) return AGILE_EINVAL;
        r->mode = REDIRECT_SINK;
        r->q = rt->q_ptr;
        r->qmask = rt->q_bytes - 1;
    } else {
        r->mode = policy == AGILE_POLICY_REMAP ? REDIRECT_REMAP : REDIRECT_REPORT;
    }
    return AGILE_OK;
}

// Whether a call's denials go to the log (every policy but SUPPRESS_ONLY).
static int log_on(int policy) { return policy != AGILE_POLICY_SUPPRESS_ONLY; }

// Trap policy, before the call's kernels: queue a copy of the log's denial count.
static int trap_begin(agile_rt* rt, int policy, hipStream_t s) {
    if (policy != AGILE_POLICY_TRAP) return AGILE_OK;
    return hipMemcpyAsync(&rt->htrap[0], &rt->d_log->count, sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, s) == hipSuccess
               ? AGILE_OK
               : AGILE_EDEVICE;
}

// Trap policy, after the call's kernels: wait for them; if the count grew, the call denied an
// access, so the handle is retired.
static int trap_end(agile_rt* rt, int policy, hipStream_t s) {
    if (policy != AGILE_POLICY_TRAP) return AGILE_OK;
    if (hipMemcpyAsync(&rt->htrap[1], &rt->d_log->count, sizeof(unsigned long long),
                       hipMemcpyDeviceToHost, s) != hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AGILE_EDEVICE;
    if (rt->htrap[1] == rt->htrap[0]) return AGILE_OK;
    rt->retired = true;
    return AGILE_ETRAPPED;
}

// Binding of a pointer argument of a guarded call: the USER range containing p, from the host
// copy of the table (the state the launch is ordered after), or the empty interval.
static Bind host_bind(const agile_rt* rt, uint64_t p) {
    const auto& e = rt->entries;
    auto it = std::upper_bound(e.begin(), e.end(), p,
                               [](uint64_t a, const Entry& x) { return a < x.base; });
    if (it == e.begin()) return Bind{0, 0};
    --it;
    if (p < it->end && it->kind == AGILE_KIND_USER) return Bind{it->base, it->end};
    return Bind{0, 0};
}

int agile_guarded_copy(agile_rt* rt, void* d_dst, const void* d_src, uint64_t nbytes, int policy,
                       void* stream) {
    if (!rt || !policy_ok(policy)) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    Redirect rd;
    if (redirecting(policy) && redirect_of(rt, policy, &rd) != AGILE_OK) return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = prepare(rt, s);
    if (rc != AGILE_OK) return rc;
    rc = trap_begin(rt, policy, s);
    if (rc != AGILE_OK) return rc;
    const unsigned long long seq = rt->seq++;
    const Bind b[2] = {host_bind(rt, (uint64_t)d_src), host_bind(rt, (uint64_t)d_dst)};
    if (launch_copy(true, rt->tab, rt->d_log, b, d_dst, d_src, nbytes, seq,
                    log_on(policy), rt->info, s) != hipSuccess)
        return AGILE_EDEVICE;
    if (redirecting(policy) &&
        launch_copy_fix(rt->tab, rd, b[0], b[1], d_dst, d_src, nbytes,
                        clip_prefix(b[0], (uint64_t)d_src, nbytes, 1),
                        clip_prefix(b[1], (uint64_t)d_dst, nbytes, 1), rt->info, s) != hipSuccess)
        return AGILE_EDEVICE;
    return trap_end(rt, policy, s);
}

int agile_guarded_triad(agile_rt* rt, float* d_a, const float* d_b, const float* d_c, float s_,
                        uint64_t n, int policy, void* stream) {
    if (!rt || !policy_ok(policy)) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    Redirect rd;
    if (redirecting(policy) && redirect_of(rt, policy, &rd) != AGILE_OK) return AGILE_EINVAL;
    if ((((uint64_t)d_a | (uint64_t)d_b | (uint64_t)d_c) & 3) || n > (U64MAX >> 3))
        return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int rc = prepare(rt, s);
    if (rc != AGILE_OK) return rc;
    rc = trap_begin(rt, policy, s);
    if (rc != AGILE_OK) return rc;
    const unsigned long long seq = rt->seq++;
    const Bind b[3] = {host_bind(rt, (uint64_t)d_b), host_bind(rt, (uint64_t)d_c),
                       host_bind(rt, (uint64_t)d_a)};
    if (launch_triad(true, rt->tab, rt->d_log, b, d_a, d_b, d_c, s_, n, seq,
                     log_on(policy), rt->info, s) != hipSuccess)
        return AGILE_EDEVICE;
    if (redirecting(policy) &&
        launch_triad_fix(rt->tab, rd, b[2], b[0], b[1], d_a, d_b, d_c, s_, n,
                         clip_prefix(b[2], (uint64_t)d_a, n, 4),
                         clip_prefix(b[0], (uint64_t)d_b, n, 4),
                         clip_prefix(b[1], (uint64_t)d_c, n, 4), rt->info, s) != hipSuccess)
        return AGILE_EDEVICE;
    return trap_end(rt, policy, s);
}

static int rows_args_ok(uint64_t row_bytes, uint64_t n, int dtype, const void* a, const void* b,
                        uint32_t* w) {
    if (dtype != AGILE_DTYPE_F32 && dtype != AGILE_DTYPE_F64) return AGILE_EINVAL;
    *w = dtype == AGILE_DTYPE_F32 ? 4 : 8;
    if (row_bytes == 0 || row_bytes % *w || row_bytes > (1ull << 40)) return AGILE_EINVAL;
    const uint64_t D = row_bytes / *w;
    if (n > 0 && D > ((1ull << 62) - 1) / n) return AGILE_EINVAL;
    if ((((uint64_t)a | (uint64_t)b) & (*w - 1))) return AGILE_EINVAL;
    return AGILE_OK;
}

int agile_guarded_gather(agile_rt* rt, void* d_out, const void* d_table, uint64_t row_bytes,
                         const int64_t* d_idx, uint64_t n, int dtype, int policy, void* stream) {
    if (!rt || !policy_ok(policy)) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    Redirect rd;
    if (redirecting(policy) && redirect_of(rt, policy, &rd) != AGILE_OK) return AGILE_EINVAL;
    uint32_t w;
    int rc = rows_args_ok(row_bytes, n, dtype, d_out, d_table, &w);
    if (rc != AGILE_OK) return rc;
    if ((uint64_t)d_idx & 7) return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    rc = prepare(rt, s);
    if (rc != AGILE_OK) return rc;
    rc = trap_begin(rt, policy, s);
    if (rc != AGILE_OK) return rc;
    const unsigned long long seq = rt->seq++;
    const Bind b[3] = {host_bind(rt, (uint64_t)d_idx), host_bind(rt, (uint64_t)d_table),
                       host_bind(rt, (uint64_t)d_out)};
    if (redirecting(policy)) {
        // the guarded kernel runs the rows whose index is readable, the redirect pass the rest
        const RowsGuard full = rows_guard(b[0], b[2], b[1], (uint64_t)d_idx, (uint64_t)d_out,
                                          (uint64_t)d_table, n, row_bytes, w);
        if (launch_gather(true, rt->tab, rt->d_log, b, d_out, d_table, row_bytes, d_idx, full.ki,
                          w, seq, 1, rt->info, s, false) != hipSuccess ||
            launch_rows_fix(0, rt->tab, rt->d_log, rd, RowBinds{b[0], b[2], b[1]}, d_out,
                            const_cast<void*>(d_table),
                            row_bytes, d_idx, n, full, w, rt->info, s) != hipSuccess ||
            launch_fault_finish(rt->tab, rt->d_log,
                                rows_fault_site(AGILE_OP_GATHER, w, 1, row_bytes, full.ki, d_idx,
                                                d_out, d_table),
                                seq, s) != hipSuccess)
            return AGILE_EDEVICE;
    } else if (launch_gather(true, rt->tab, rt->d_log, b, d_out, d_table, row_bytes, d_idx, n, w,
                             seq, log_on(policy), rt->info, s) != hipSuccess) {
        return AGILE_EDEVICE;
    }
    return trap_end(rt, policy, s);
}

// Guarded scatter / scatter-add. noalloc: the sort scratch is the fixed device array `scratch`
// (the caller checked that n fits it) instead of the handle's growing buffer.
static int scatter_impl(agile_rt* rt, void* d_dst, uint64_t row_bytes, const int64_t* d_idx,
                        const void* d_src, uint64_t n, int dtype, int accumulate, int policy,
                        void* stream, bool noalloc) {
    if (!rt || !policy_ok(policy) || accumulate < 0 || accumulate > 2) return AGILE_EINVAL;
    if (rt->retired) return AGILE_ETRAPPED;
    Redirect rd;
    if (redirecting(policy) && redirect_of(rt, policy, &rd) != AGILE_OK) return AGILE_EINVAL;
    uint32_t w;
    int rc = rows_args_ok(row_bytes, n, dtype, d_dst, d_src, &w);
    if (rc != AGILE_OK) return rc;
    if ((uint64_t)d_idx & 7) return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const bool sort = accumulate && n >= SORT_MIN_N;
    void* fixed = nullptr;
    if (noalloc && sort) {
        if (scatter_add_scratch_bytes(n) > AGILE_NOALLOC_SCRATCH_BYTES) return AGILE_E2BIG;
        fixed = noalloc_scratch(rt->device);
        if (!fixed) return AGILE_EDEVICE;
    }
    rc = prepare(rt, s);
    if (rc != AGILE_OK) return rc;
    rc = trap_begin(rt, policy, s);
    if (rc != AGILE_OK) return rc;
    const unsigned long long seq = rt->seq++;
    const Bind b[3] = {host_bind(rt, (uint64_t)d_idx), host_bind(rt, (uint64_t)d_src),
                       host_bind(rt, (uint64_t)d_dst)};
    void* scr = !sort ? nullptr : (noalloc ? fixed : rt->sa.get(scatter_add_scratch_bytes(n), s));
    if (redirecting(policy)) {
        const RowsGuard full = rows_guard(b[0], b[1], b[2], (uint64_t)d_idx, (uint64_t)d_src,
                                          (uint64_t)d_dst, n, row_bytes, w);
        if (launch_scatter(true, rt->tab, rt->d_log, b, d_dst, row_bytes, d_idx, d_src, full.ki, w,
                           accumulate, seq, 1, scr, rt->info, s, false) != hipSuccess ||
            launch_rows_fix(accumulate ? 2 : 1, rt->tab, rt->d_log, rd,
                            RowBinds{b[0], b[1], b[2]}, const_cast<void*>(d_src), d_dst,
                            row_bytes, d_idx, n, full, w, rt->info, s) != hipSuccess ||
            launch_fault_finish(rt->tab, rt->d_log,
                                rows_fault_site(accumulate ? AGILE_OP_SCATTER_ADD : AGILE_OP_SCATTER,
                                                w, 2, row_bytes, full.ki, d_idx, d_src, d_dst),
                                seq, s) != hipSuccess)
            return AGILE_EDEVICE;
    } else if (launch_scatter(true, rt->tab, rt->d_log, b, d_dst, row_bytes, d_idx, d_src, n, w,
                              accumulate, seq, log_on(policy), scr, rt->info, s) != hipSuccess) {
        return AGILE_EDEVICE;
    }
    return trap_end(rt, policy, s);
}

int agile_guarded_scatter(agile_rt* rt, void* d_dst, uint64_t row_bytes, const int64_t* d_idx,
                          const void* d_src, uint64_t n, int dtype, int accumulate, int policy,
                          void* stream) {
    return scatter_impl(rt, d_dst, row_bytes, d_idx, d_src, n, dtype, accumulate, policy, stream,
                        false);
}

int agile_guarded_scatter_add_noalloc(agile_rt* rt, void* d_dst, uint64_t row_bytes,
                                      const int64_t* d_idx, const void* d_src, uint64_t n,
                                      int dtype, int policy, void* stream) {
    if (!rt) return AGILE_EINVAL;
    if (n > AGILE_NOALLOC_MAX_ROWS) return AGILE_E2BIG;
    return scatter_impl(rt, d_dst, row_bytes, d_idx, d_src, n, dtype, 1, policy, stream, true);
}

int agile_fault_log_read(agile_rt* rt, agile_fault* out, int clear, void* stream) {
    if (!rt || !out) return AGILE_EINVAL;
    DeviceGuard dg(rt->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemcpyAsync(rt->hlog, rt->d_log, sizeof(agile_fault), hipMemcpyDeviceToHost, s) !=
            hipSuccess ||
        hipStreamSynchronize(s) != hipSuccess)
        return AGILE_EDEVICE;
    *out = *rt->hlog;
    if (clear && launch_log_reset(rt->d_log, s) != hipSuccess) return AGILE_EDEVICE;
    if (rt->retired) return AGILE_ETRAPPED;
    return out->count ? AGILE_EFAULTED : AGILE_OK;
}

// ---- batched multi-client requests -----------------------------------------------------
namespace {
constexpr int BATCH_SLOTS = 8;
struct BatchSlot {
    void* dmem = nullptr;
    size_t dcap = 0;
    void* hstage = nullptr;
    size_t hcap = 0;
    hipEvent_t done = nullptr;
    bool used = false;
};
size_t align64(size_t x) { return (x + 63) & ~(size_t)63; }
}  // namespace

struct agile_clients {
    int device = 0;
    std::vector<agile_rt*> tables;
    BatchSlot slot[BATCH_SLOTS];
    int next = 0;
};

int agile_clients_create(agile_clients** out, agile_rt* const* tables, uint32_t n, int device) {
    if (!out || !tables || n == 0) return AGILE_EINVAL;
    for (uint32_t i = 0; i < n; ++i)
        if (!tables[i] || tables[i]->device != device) return AGILE_EINVAL;
    DeviceGuard dg(device);
    if (!dg.ok) return AGILE_EDEVICE;
    agile_clients* cs = new (std::nothrow) agile_clients();
    if (!cs) return AGILE_ENOMEM;
    cs->device = device;
    cs->tables.assign(tables, tables + n);
    for (auto& sl : cs->slot) {
        if (hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess) {
            agile_clients_destroy(cs);
            return AGILE_EDEVICE;
        }
    }
    *out = cs;
    return AGILE_OK;
}

int agile_clients_destroy(agile_clients* cs) {
    if (!cs) return AGILE_OK;
    DeviceGuard dg(cs->device);
    int rc = AGILE_OK;
    for (auto& sl : cs->slot) {
        if (sl.done) {
            if (sl.used && hipEventSynchronize(sl.done) != hipSuccess) rc = AGILE_EDEVICE;
            (void)hipEventDestroy(sl.done);
        }
        if (sl.dmem) (void)hipFree(sl.dmem);
        if (sl.hstage) (void)hipHostFree(sl.hstage);
    }
    delete cs;
    return rc;
}

int agile_batch_run(agile_clients* cs, const agile_request* reqs, uint32_t nreq,
                    const agile_ptr* d_ptrs, uint64_t nptrs, uint8_t* d_ptr_verdict,
                    int32_t* d_ptr_owner, agile_req_result* d_result, void* stream) {
    static_assert(sizeof(agile_request) == sizeof(BatchReq), "request layout");
    static_assert(sizeof(agile_req_result) == sizeof(agile_req_result_dev), "result layout");
    if (!cs) return AGILE_EINVAL;
    if (nreq == 0) return AGILE_OK;
    if (!reqs || !d_result) return AGILE_EINVAL;
    if (nptrs && (!d_ptrs || !d_ptr_verdict || !d_ptr_owner || ((uint64_t)d_ptrs & 15)))
        return AGILE_EINVAL;
    const uint32_t ncl = (uint32_t)cs->tables.size();
    uint64_t total_copy = 0, total_rows = 0;
    for (uint32_t r = 0; r < nreq; ++r) {
        const agile_request& q = reqs[r];
        if (q.client >= ncl || q.ptr_off > nptrs || q.nptr > nptrs - q.ptr_off) return AGILE_EINVAL;
        if (cs->tables[q.client]->retired) return AGILE_ETRAPPED;
        if (q.nptr > 0xFFFFFFFEull) return AGILE_EINVAL;
        if (q.gather_n && (q.gather_row_bytes == 0 || q.gather_row_bytes % 4 ||
                           ((q.gather_out | q.gather_table) & 3) || (q.gather_idx & 7) ||
                           q.gather_n > ((1ull << 62) - 1) / (q.gather_row_bytes / 4)))
            return AGILE_EINVAL;
        total_copy = q.copy_bytes > U64MAX - total_copy ? U64MAX : total_copy + q.copy_bytes;
        total_rows = q.gather_n > U64MAX - total_rows ? U64MAX : total_rows + q.gather_n;
    }
    uint64_t tile_copy, tile_rows;
    batch_tile_sizes(total_copy, total_rows, cs->tables[0]->info, tile_copy, tile_rows);
    uint64_t ntiles = 0;
    for (uint32_t r = 0; r < nreq; ++r)
        ntiles += batch_tiles(reinterpret_cast<const BatchReq&>(reqs[r]), tile_copy, tile_rows);
    DeviceGuard dg(cs->device);
    if (!dg.ok) return AGILE_EDEVICE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    for (agile_rt* rt : cs->tables) {
        const int rc = prepare(rt, s);
        if (rc != AGILE_OK) return rc;
    }
    // layout: ctl | tstart[nreq+1] | reqs | scratch | tables | guards[nreq] | tile_req[ntiles]
    if (ntiles > 0xFFFFFFFFull) return AGILE_EINVAL;
    const size_t o_ts = align64(sizeof(BatchCtl));
    const size_t o_rq = o_ts + align64((size_t)(nreq + 1) * 8);
    const size_t o_sc = o_rq + align64((size_t)nreq * sizeof(BatchReq));
    const size_t o_tb = o_sc + align64((size_t)nreq * sizeof(BatchScratch));
    const size_t o_gd = o_tb + align64((size_t)ncl * sizeof(DevTable));
    const size_t o_tr = o_gd + align64((size_t)nreq * sizeof(BatchGuard));
    const size_t bytes = o_tr + align64((size_t)ntiles * 4);
    // a staging slot whose last launch has finished (launches complete out of order): the
    // first one already large enough, else the first free one (it grows); with none free, the
    // next one in turn, waited for
    int fit = -1, any = -1;
    for (int j = 0; j < BATCH_SLOTS && fit < 0; ++j) {
        BatchSlot& c = cs->slot[j];
        if (c.used) {
            const hipError_t q = hipEventQuery(c.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return AGILE_EDEVICE;
            c.used = false;
        }
        if (c.dcap >= bytes) fit = j;
        else if (any < 0) any = j;
    }
    int pick = fit >= 0 ? fit : any;
    if (pick < 0) {
        pick = cs->next;
        cs->next = (cs->next + 1) % BATCH_SLOTS;
    }
    BatchSlot& sl = cs->slot[pick];
    if (sl.used) {
        if (hipEventSynchronize(sl.done) != hipSuccess) return AGILE_EDEVICE;
        sl.used = false;
    }
    if (sl.dcap < bytes) {
        if (sl.dmem) (void)hipFree(sl.dmem);
        if (sl.hstage) (void)hipHostFree(sl.hstage);
        sl.dmem = sl.hstage = nullptr;
        sl.dcap = sl.hcap = 0;
        const size_t cap = bytes * 2;
        if (hipMalloc(&sl.dmem, cap) != hipSuccess) return AGILE_ENOMEM;
        if (hipHostMalloc(&sl.hstage, cap, hipHostMallocDefault) != hipSuccess) {
            (void)hipFree(sl.dmem);
            sl.dmem = nullptr;
            return AGILE_ENOMEM;
        }
        sl.dcap = sl.hcap = cap;
    }
    uint8_t* h = static_cast<uint8_t*>(sl.hstage);
    std::memset(h, 0, o_ts);
    uint64_t* ts = reinterpret_cast<uint64_t*>(h + o_ts);
    BatchReq* rq = reinterpret_cast<BatchReq*>(h + o_rq);
    BatchScratch* sc = reinterpret_cast<BatchScratch*>(h + o_sc);
    DevTable* tb = reinterpret_cast<DevTable*>(h + o_tb);
    BatchGuard* gd = reinterpret_cast<BatchGuard*>(h + o_gd);
    uint32_t* tr = reinterpret_cast<uint32_t*>(h + o_tr);
    uint64_t acc = 0;
    for (uint32_t r = 0; r < nreq; ++r) {
        std::memcpy(&rq[r], &reqs[r], sizeof(BatchReq));
        const uint64_t k = batch_tiles(rq[r], tile_copy, tile_rows);
        for (uint64_t j = 0; j < k; ++j) tr[acc + j] = r;
        ts[r] = acc;
        acc += k;
        // the request's arguments bound against its own client's table (host lookup)
        const agile_rt* crt = cs->tables[rq[r].client];
        const BatchReq& q = rq[r];
        gd[r].copy_ks = clip_prefix(host_bind(crt, q.copy_src), q.copy_src, q.copy_bytes, 1);
        gd[r].copy_kd = clip_prefix(host_bind(crt, q.copy_dst), q.copy_dst, q.copy_bytes, 1);
        gd[r].gather = q.gather_n
                           ? rows_guard(host_bind(crt, q.gather_idx), host_bind(crt, q.gather_out),
                                        host_bind(crt, q.gather_table), q.gather_idx, q.gather_out,
                                        q.gather_table, q.gather_n, q.gather_row_bytes, 4)
                           : rows_open(0, 4, 4);
        sc[r].minfail = 0xFFFFFFFFu;
        sc[r].remaining = (unsigned int)k;
        sc[r].gcount = 0;
        sc[r].gminkey = ~0ull;
        sc[r].pad = 0;
    }
    ts[nreq] = acc;
    for (uint32_t c = 0; c < ncl; ++c) tb[c] = cs->tables[c]->tab;
    if (hipMemcpyAsync(sl.dmem, h, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
        return AGILE_EDEVICE;
    uint8_t* d = static_cast<uint8_t*>(sl.dmem);
    BatchArgs A{};
    A.ctl = reinterpret_cast<BatchCtl*>(d);
    A.tstart = reinterpret_cast<const uint64_t*>(d + o_ts);
    A.reqs = reinterpret_cast<const BatchReq*>(d + o_rq);
    A.scratch = reinterpret_cast<BatchScratch*>(d + o_sc);
    A.tables = reinterpret_cast<const DevTable*>(d + o_tb);
    A.guards = reinterpret_cast<const BatchGuard*>(d + o_gd);
    A.tile_req = reinterpret_cast<const uint32_t*>(d + o_tr);
    A.ptrs = reinterpret_cast<const ulonglong2*>(d_ptrs);
    A.pv = d_ptr_verdict;
    A.po = d_ptr_owner;
    A.result = reinterpret_cast<agile_req_result_dev*>(d_result);
    A.ntiles = ntiles;
    A.tile_copy = tile_copy;
    A.tile_rows = tile_rows;
    A.nreq = nreq;
    if (launch_batch(A, cs->tables[0]->info, s) != hipSuccess) return AGILE_EDEVICE;
    if (hipEventRecord(sl.done, s) != hipSuccess) return AGILE_EDEVICE;
    sl.used = true;
    return AGILE_OK;
}

// ---- unguarded twins ------------------------------------------------------------------
static DevInfo current_info() {
    static thread_local int cached_dev = -1;
    static thread_local DevInfo cached{};
    int dev = 0;
    (void)hipGetDevice(&dev);
    if (dev != cached_dev) {
        hipDeviceProp_t p;
        if (hipGetDeviceProperties(&p, dev) == hipSuccess) {
            cached.num_cu = p.multiProcessorCount;
            cached.lds_per_block = p.sharedMemPerBlock;
            cached.lds_per_cu = p.maxSharedMemoryPerMultiProcessor;
            cached_dev = dev;
        } else {
            cached.num_cu = 1;
        }
    }
    return cached;
}

int agile_unguarded_copy(void* d_dst, const void* d_src, uint64_t nbytes, void* stream) {
    if (nbytes && (!d_dst || !d_src)) return AGILE_EINVAL;
    return launch_copy(false, DevTable{}, nullptr, nullptr, d_dst, d_src, nbytes, 0, 0, current_info(),
                       static_cast<hipStream_t>(stream)) == hipSuccess
               ? AGILE_OK
               : AGILE_EDEVICE;
}

int agile_unguarded_triad(float* d_a, const float* d_b, const float* d_c, float s_, uint64_t n,
                          void* stream) {
    if (n && (!d_a || !d_b || !d_c)) return AGILE_EINVAL;
    if (((uint64_t)d_a | (uint64_t)d_b | (uint64_t)d_c) & 3) return AGILE_EINVAL;
    return launch_triad(false, DevTable{}, nullptr, nullptr, d_a, d_b, d_c, s_, n, 0, 0, current_info(),
                        static_cast<hipStream_t>(stream)) == hipSuccess
               ? AGILE_OK
               : AGILE_EDEVICE;
}

int agile_unguarded_gather(void* d_out, const void* d_table, uint64_t row_bytes,
                           const int64_t* d_idx, uint64_t n, int dtype, void* stream) {
    uint32_t w;
    int rc = rows_args_ok(row_bytes, n, dtype, d_out, d_table, &w);
    if (rc != AGILE_OK) return rc;
    if (n && (!d_out || !d_table || !d_idx)) return AGILE_EINVAL;
    return launch_gather(false, DevTable{}, nullptr, nullptr, d_out, d_table, row_bytes, d_idx, n, w, 0, 0,
                         current_info(), static_cast<hipStream_t>(stream)) == hipSuccess
               ? AGILE_OK
               : AGILE_EDEVICE;
}

int agile_unguarded_scatter(void* d_dst, uint64_t row_bytes, const int64_t* d_idx,
                            const void* d_src, uint64_t n, int dtype, int accumulate,
                            void* stream) {
    uint32_t w;
    if (accumulate < 0 || accumulate > 2) return AGILE_EINVAL;
    int rc = rows_args_ok(row_bytes, n, dtype, d_dst, d_src, &w);
    if (rc != AGILE_OK) return rc;
    if (n && (!d_dst || !d_src || !d_idx)) return AGILE_EINVAL;
    void* scr = nullptr;
    if (accumulate && n >= SORT_MIN_N) {
        // one scratch buffer per device for the unguarded twin, kept until the process ends
        static std::mutex mu;
        static std::vector<StreamScratch> per_dev;
        int dev = 0;
        (void)hipGetDevice(&dev);
        std::lock_guard<std::mutex> lk(mu);
        if ((size_t)dev >= per_dev.size()) per_dev.resize(dev + 1);
        scr = per_dev[dev].get(scatter_add_scratch_bytes(n), static_cast<hipStream_t>(stream));
    }
    return launch_scatter(false, DevTable{}, nullptr, nullptr, d_dst, row_bytes, d_idx, d_src, n, w,
                          accumulate, 0, 0, scr, current_info(),
                          static_cast<hipStream_t>(stream)) == hipSuccess
               ? AGILE_OK
               : AGILE_EDEVICE;
}

}  // extern "C"
