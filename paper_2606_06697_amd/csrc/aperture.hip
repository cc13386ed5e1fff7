// Fixed address apertures (AgileOS Section IV-E, Table I), built with HIP's virtual memory calls
// the way Section V-A builds them with CUDA's: read the allocation granularity, reserve the I/O,
// module and user apertures back to back in Table I's order, and attach physical memory to each
// allocation as it is made (create a handle, map it into its aperture, grant the device
// read/write access), recording the allocation's base and requested size in a range table.
//
// Reservations. Every free run of an aperture is one reservation, and so is every allocation:
// an allocation releases the free run it is taken from and reserves, at the same addresses, its
// own range and what is left of the run; a release merges its range back with its free
// neighbours the same way. The aperture's addresses therefore stay reserved at all times, and
// each reservation holds at most one mapping. Inside one large reservation this runtime refuses
// device access to some mappings depending on what was mapped before them (in a 1 TiB
// reservation, 4 KiB mapped right after 1 MiB + 4 KiB or after 2 MiB: hipMemMap succeeds,
// hipMemSetAccess fails with invalid argument and hipMemGetAccess reports no access; the same
// pair in a 1 GiB reservation works). Every allocation's access is also read back (first and
// last page) before the allocation is handed out, so memory without access never reaches a
// kernel.
//
// The coarse check of the Fig. 2 guard then needs only the four aperture bounds: a streaming
// kernel classifies (addr, len) queries with a few compares each. It reads 16 bytes and writes
// 1 (+4 with the aperture index) per query, all coalesced and non-temporal, so it runs at the
// HBM roofline whatever the number of allocations.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <map>
#include <new>

#include "agile_aperture.h"
#include "agile_guard.h"
#include "device_guard.h"
#include "va_ranges.h"

using agile::DeviceGuard;

struct agile_aperture {
    struct Alloc {
        uint64_t bytes;  // mapped and reserved bytes (the request rounded up to the granularity)
        int region;
        agile_rt* rt;    // table the allocation is registered in, or null
        int32_t id;
        hipMemGenericAllocationHandle_t h;
    };
    int device = 0;
    uint64_t gran = 0;   // the runtime's minimum allocation granularity
    bool user_hint = false;  // placed at a base address the caller asked for
    bool broken = false;     // a failed re-reservation left part of an aperture unreserved
    uint64_t b[4] = {0, 0, 0, 0};
    uint64_t budget[3] = {0, 0, 0};  // most physical bytes each aperture may hold mapped
    uint64_t mapped[3] = {0, 0, 0};  // physical bytes mapped now
    hipMemAllocationProp prop{};
    agile::VaRanges va[3];  // free runs, each one reservation
    std::map<uint64_t, Alloc> allocs;  // by address
};

namespace agile {

// 128-thread blocks of 2 queries per thread measured best for 2^28 queries (0.876 ms), against
// 256 x 4 (0.929 ms), 512 x 2 (0.892 ms), 1024 x 4 (0.979 ms) and 64 x 2 (0.925 ms)
constexpr int ABLOCK = 128, AQPT = 2;  // threads per block, queries per thread per pass
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

struct ApBounds {
    uint64_t b0, b1, b2, b3;
};

// A block covers ABLOCK * AQPT consecutive queries per pass, lane-contiguous for each of its
// AQPT loads; the loads of a pass are issued before any query is classified. The grid covers
// the queries in one pass (the loop only matters beyond 2^40 queries).
template <bool REGION>
__global__ __launch_bounds__(ABLOCK) void k_validate_aperture(ApBounds B, const u64x2* __restrict__ q,
                                                              uint64_t n, uint8_t* __restrict__ verdict,
                                                              int32_t* __restrict__ region) {
    const uint64_t step = (uint64_t)gridDim.x * (ABLOCK * AQPT);
    for (uint64_t i0 = (uint64_t)blockIdx.x * (ABLOCK * AQPT) + threadIdx.x; i0 < n; i0 += step) {
        u64x2 x[AQPT];
#pragma unroll
        for (int j = 0; j < AQPT; ++j) {
            const uint64_t i = i0 + (uint64_t)j * ABLOCK;
            x[j] = i < n ? __builtin_nontemporal_load(q + i) : u64x2{0, 0};
        }
#pragma unroll
        for (int j = 0; j < AQPT; ++j) {
            const uint64_t i = i0 + (uint64_t)j * ABLOCK;
            if (i >= n) break;
            const uint64_t a = x[j].x, len = x[j].y;
            const uint64_t L = len ? len : 1;
            const bool in = a >= B.b0 && a < B.b3;
            const bool user = a >= B.b2;
            uint8_t v;
            int32_t r;
            if (!in) {
                v = AGILE_V_UNMAPPED;
                r = -1;
            } else if (!user) {
                v = AGILE_V_PROTECTED;
                r = a < B.b1 ? AGILE_AP_IO : AGILE_AP_MODULE;
            } else {
                v = L <= B.b3 - a ? AGILE_ALLOW : AGILE_V_STRADDLE;
                r = AGILE_AP_USER;
            }
            __builtin_nontemporal_store(v, verdict + i);
            if (REGION) __builtin_nontemporal_store(r, region + i);
        }
    }
}

static hipMemAllocationProp device_prop(int device) {
    hipMemAllocationProp p = {};
    p.type = hipMemAllocationTypePinned;
    p.requestedHandleType = hipMemHandleTypeNone;
    p.location.type = hipMemLocationTypeDevice;
    p.location.id = device;
    return p;
}

static uint32_t kind_of(int region) {
    return region == AGILE_AP_USER ? AGILE_KIND_USER
                                   : region == AGILE_AP_MODULE ? AGILE_KIND_PROTECTED
                                                               : AGILE_KIND_MMIO;
}

// Unmap and release one allocation's memory (the device must be done with it).
static bool unmap_alloc(const agile_aperture::Alloc& a, uint64_t addr) {
    bool ok = hipMemUnmap(reinterpret_cast<void*>(addr), a.bytes) == hipSuccess;
    ok &= hipMemRelease(a.h) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    return ok;
}

// Reserve exactly [s, e): true when the runtime grants that address.
static bool reserve_exact(uint64_t s, uint64_t e, uint64_t align) {
    void* p = nullptr;
    const hipError_t r = hipMemAddressReserve(&p, e - s, align, reinterpret_cast<void*>(s), 0);
    if (r == hipSuccess && reinterpret_cast<uint64_t>(p) == s) return true;
    if (r == hipSuccess) (void)hipMemAddressFree(p, e - s);
    (void)hipGetLastError();
    return false;
}

static bool release(uint64_t s, uint64_t e) {
    const bool ok = hipMemAddressFree(reinterpret_cast<void*>(s), e - s) == hipSuccess;
    if (!ok) (void)hipGetLastError();
    return ok;
}

// Replace the reservations [s, e) by the reservations [s, m) and [m, e) (s < m <= e; an empty
// piece is not reserved). On failure the original reservation is restored if the runtime still
// grants it; otherwise the aperture is marked broken.
static bool split_run(agile_aperture* ap, uint64_t s, uint64_t m, uint64_t e) {
    if (!release(s, e)) return false;
    const bool a = reserve_exact(s, m, ap->gran);
    const bool b = a && (m == e || reserve_exact(m, e, ap->gran));
    if (b) return true;
    if (a) (void)release(s, m);
    if (!reserve_exact(s, e, ap->gran)) ap->broken = true;
    return false;
}

// Free the reservations create made. Failures are cleared from the runtime's last-error state,
// which later launch checks read; the return value says whether everything was released.
static bool teardown(agile_aperture* ap) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        // The HIP runtime may refuse to release a reservation placed at an address the caller
        // asked for; that address range then stays reserved (no memory) until the process ends.
        for (const auto& [fs, fe] : ap->va[k].free_) ok &= release(fs, fe) || ap->user_hint;
        ap->va[k].free_.clear();
    }
    (void)hipGetLastError();
    return ok;
}

// Reserve the three apertures back to back from b0 (each at its requested address, each one
// free run); false, with nothing left reserved, when the runtime places any of them elsewhere.
static bool reserve_at(agile_aperture* ap, uint64_t b0, const uint64_t* sz) {
    uint64_t at = b0;
    for (int k = 0; k < 3; ++k) {
        if (!reserve_exact(at, at + sz[k], ap->gran)) {
            for (int j = 0; j < k; ++j) (void)release(ap->b[j], ap->b[j + 1]);
            (void)hipGetLastError();
            return false;
        }
        ap->b[k] = at;
        ap->b[k + 1] = at + sz[k];
        at += sz[k];
    }
    for (int k = 0; k < 3; ++k) ap->va[k].reset(ap->b[k], ap->b[k + 1]);
    return true;
}

}  // namespace agile

using namespace agile;

extern "C" {

int agile_aperture_create(agile_aperture** out, int device, const uint64_t* sizes,
                          const uint64_t* budget, uint64_t base_hint) {
    constexpr uint64_t MAXB = 1ull << 48;
    if (!out || !sizes) return AGILE_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (sizes[k] == 0 || sizes[k] > MAXB) return AGILE_EINVAL;
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess) return AGILE_EDEVICE;
    if (device < 0 || device >= ndev) return AGILE_EINVAL;
    DeviceGuard dg(device);
    if (!dg.ok) return AGILE_EDEVICE;
    int vmm = 0;
    if (hipDeviceGetAttribute(&vmm, hipDeviceAttributeVirtualMemoryManagementSupported, device) !=
        hipSuccess)
        return AGILE_EDEVICE;
    if (!vmm) return AGILE_ENOTSUP;
    const hipMemAllocationProp prop = device_prop(device);
    size_t g = 0;
    if (hipMemGetAllocationGranularity(&g, &prop, hipMemAllocationGranularityMinimum) !=
            hipSuccess ||
        g == 0 || (g & (g - 1)))
        return AGILE_EDEVICE;
    if (base_hint % g) return AGILE_EINVAL;
    auto up = [g](uint64_t x) { return (x + g - 1) / g * g; };
    const uint64_t sz[3] = {up(sizes[0]), up(sizes[1]), up(sizes[2])};
    const uint64_t total = sz[0] + sz[1] + sz[2];
    agile_aperture* ap = new (std::nothrow) agile_aperture;
    if (!ap) return AGILE_ENOMEM;
    ap->device = device;
    ap->gran = g;
    ap->prop = prop;
    for (int k = 0; k < 3; ++k) ap->budget[k] = budget ? budget[k] : ~0ull;
    // Placement: at the caller's base if the runtime grants it; otherwise one reservation of
    // the whole layout shows where it fits, is released, and the three apertures are reserved
    // back to back at that address.
    bool placed = base_hint && base_hint <= ~0ull - 1 - total && reserve_at(ap, base_hint, sz);
    ap->user_hint = placed;
    // (another thread may take the released range first: a few attempts)
    for (int attempt = 0; attempt < 4 && !placed; ++attempt) {
        void* p = nullptr;
        if (hipMemAddressReserve(&p, total, g, nullptr, 0) == hipSuccess && p) {
            const uint64_t b0 = reinterpret_cast<uint64_t>(p);
            placed = hipMemAddressFree(p, total) == hipSuccess && b0 <= ~0ull - 1 - total &&
                     reserve_at(ap, b0, sz);
        }
        (void)hipGetLastError();
    }
    if (!placed) {
        delete ap;
        return AGILE_ENOMEM;
    }
    *out = ap;
    return AGILE_OK;
}

int agile_aperture_destroy(agile_aperture* ap) {
    if (!ap) return AGILE_OK;
    int rc = AGILE_OK;
    {
        DeviceGuard dg(ap->device);
        if (!dg.ok || hipDeviceSynchronize() != hipSuccess) rc = AGILE_EDEVICE;
        for (auto& [addr, a] : ap->allocs) {
            if (a.rt) (void)agile_rt_remove(a.rt, a.id);
            if (!unmap_alloc(a, addr)) rc = AGILE_EDEVICE;
            if (!release(addr, addr + a.bytes) && !ap->user_hint) rc = AGILE_EDEVICE;
        }
        ap->allocs.clear();
        if (!teardown(ap)) rc = AGILE_EDEVICE;
    }
    delete ap;
    return rc;
}

int agile_aperture_info(const agile_aperture* ap, uint64_t* bounds, uint64_t* mapped,
                        uint64_t* granularity) {
    if (!ap) return AGILE_EINVAL;
    if (bounds)
        for (int k = 0; k < 4; ++k) bounds[k] = ap->b[k];
    if (mapped)
        for (int k = 0; k < 3; ++k) mapped[k] = ap->mapped[k];
    if (granularity) *granularity = ap->gran;
    return AGILE_OK;
}

int agile_aperture_alloc(agile_aperture* ap, int region, uint64_t bytes, agile_rt* rt,
                         void** out_ptr, int32_t* out_id) {
    if (!ap || !out_ptr || region < AGILE_AP_IO || region > AGILE_AP_USER || bytes == 0 ||
        bytes > ap->b[region + 1] - ap->b[region])
        return AGILE_EINVAL;
    if (ap->broken) return AGILE_EDEVICE;
    const uint64_t n = (bytes + ap->gran - 1) / ap->gran * ap->gran;
    if (n > ap->budget[region] - ap->mapped[region]) return AGILE_ENOSPC;
    uint64_t s = 0, e = 0;
    if (!ap->va[region].first_fit(n, &s, &e)) return AGILE_ENOSPC;
    DeviceGuard dg(ap->device);
    if (!dg.ok) return AGILE_EDEVICE;
    // the free run [s, e) becomes the allocation's reservation [s, s + n) and the rest
    if (!split_run(ap, s, s + n, e)) return AGILE_EDEVICE;
    uint64_t addr = 0;
    (void)ap->va[region].take(n, &addr);  // == s: the same lowest fit
    auto undo_va = [&]() {  // merge [s, s + n) back into the free run
        uint64_t ms, me;
        ap->va[region].merged(s, n, &ms, &me);
        bool ok = release(s, s + n);
        if (me > s + n) ok &= release(s + n, me);
        if (ok && !reserve_exact(ms, me, ap->gran)) ap->broken = true;
        ap->va[region].give(s, n);
    };
    // physical memory for this allocation alone, mapped in its own reservation, read/write
    agile_aperture::Alloc a{n, region, rt, -1, {}};
    if (hipMemCreate(&a.h, n, &ap->prop, 0) != hipSuccess) {
        (void)hipGetLastError();
        undo_va();
        return AGILE_ENOMEM;
    }
    void* p = reinterpret_cast<void*>(addr);
    if (hipMemMap(p, n, 0, a.h, 0) != hipSuccess) {
        (void)hipGetLastError();
        (void)hipMemRelease(a.h);
        undo_va();
        return AGILE_EDEVICE;
    }
    hipMemAccessDesc acc = {};
    acc.location = ap->prop.location;
    acc.flags = hipMemAccessFlagsProtReadWrite;
    unsigned long long f0 = 0, f1 = 0;
    const bool granted =
        hipMemSetAccess(p, n, &acc, 1) == hipSuccess &&
        hipMemGetAccess(&f0, &acc.location, p) == hipSuccess &&
        hipMemGetAccess(&f1, &acc.location, reinterpret_cast<void*>(addr + n - ap->gran)) ==
            hipSuccess &&
        f0 == hipMemAccessFlagsProtReadWrite && f1 == hipMemAccessFlagsProtReadWrite;
    if (!granted) {  // never hand out memory the device may not touch
        (void)hipGetLastError();
        (void)unmap_alloc(a, addr);
        undo_va();
        return AGILE_EDEVICE;
    }
    if (rt) {
        // its own mapped memory: a kernel may touch it
        const int rc = agile_rt_insert(rt, addr, bytes, kind_of(region) | AGILE_RANGE_BACKED, &a.id);
        if (rc != AGILE_OK) {
            (void)unmap_alloc(a, addr);
            undo_va();
            return rc;
        }
    }
    ap->mapped[region] += n;
    ap->allocs.emplace(addr, a);
    *out_ptr = p;
    if (out_id) *out_id = a.id;
    return AGILE_OK;
}

int agile_aperture_free(agile_aperture* ap, void* ptr) {
    if (!ap || !ptr) return AGILE_EINVAL;
    auto it = ap->allocs.find(reinterpret_cast<uint64_t>(ptr));
    if (it == ap->allocs.end()) return AGILE_ENOENT;
    DeviceGuard dg(ap->device);
    // wait first: on a failure nothing has changed
    if (!dg.ok || hipDeviceSynchronize() != hipSuccess) return AGILE_EDEVICE;
    const agile_aperture::Alloc a = it->second;
    const uint64_t s = it->first;
    if (!unmap_alloc(a, s)) return AGILE_EDEVICE;
    if (a.rt) (void)agile_rt_remove(a.rt, a.id);
    ap->mapped[a.region] -= a.bytes;
    ap->allocs.erase(it);
    // the allocation's reservation and its free neighbours become one free run
    uint64_t ms, me;
    ap->va[a.region].merged(s, a.bytes, &ms, &me);
    bool ok = release(s, s + a.bytes);
    if (ms < s) ok &= release(ms, s);
    if (me > s + a.bytes) ok &= release(s + a.bytes, me);
    ap->va[a.region].give(s, a.bytes);
    if (!ok || !reserve_exact(ms, me, ap->gran)) {
        ap->broken = true;
        return AGILE_EDEVICE;
    }
    return AGILE_OK;
}

int agile_validate_aperture(const agile_aperture* ap, const agile_ptr* d_q, uint64_t n,
                            uint8_t* d_verdict, int32_t* d_region, void* stream) {
    if (!ap) return AGILE_EINVAL;
    if (n == 0) return AGILE_OK;
    if (!d_q || !d_verdict || ((uint64_t)d_q & 15) || ((uint64_t)d_region & 3) ||
        n > (1ull << 48))
        return AGILE_EINVAL;
    DeviceGuard dg(ap->device);
    if (!dg.ok) return AGILE_EDEVICE;
    const ApBounds B{ap->b[0], ap->b[1], ap->b[2], ap->b[3]};
    // one pass per block: a grid-stride loop over a CU-sized grid measured 1.3x slower here
    const uint64_t per = (uint64_t)ABLOCK * AQPT;
    uint64_t grid = (n + per - 1) / per;
    if (grid > (1ull << 30)) grid = 1ull << 30;
    hipStream_t s = static_cast<hipStream_t>(stream);
    const u64x2* q = reinterpret_cast<const u64x2*>(d_q);
    if (d_region)
        hipLaunchKernelGGL(k_validate_aperture<true>, dim3((uint32_t)grid), dim3(ABLOCK), 0, s, B,
                           q, n, d_verdict, d_region);
    else
        hipLaunchKernelGGL(k_validate_aperture<false>, dim3((uint32_t)grid), dim3(ABLOCK), 0, s, B,
                           q, n, d_verdict, d_region);
    return hipGetLastError() == hipSuccess ? AGILE_OK : AGILE_EDEVICE;
}

}  // extern "C"
