// Fixed address apertures (AgileOS Section IV-E, Table I), built with HIP's virtual memory calls
// the way Section V-A builds them with CUDA's: read the minimum allocation granularity, reserve
// the I/O, module and user apertures back to back in Table I's order, attach physical memory
// (create a handle, map it, grant the device read/write access), and record each allocation
// (base, requested size) in a range table.
//
// The paper attaches memory per allocation. This HIP runtime resolves a second live mapping
// inside one reservation to the first mapping's handle, so granting access to it fails or
// would not reach it. Each aperture is therefore its own reservation with at most one mapping:
// a backing of a size fixed at creation, mapped at the aperture's start, from which
// allocations are carved (lowest fit, in granules). Allocation and release make no HIP call
// other than the release's device synchronization.
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
        uint64_t bytes;  // carved bytes (the request rounded up to the granularity)
        int region;
        agile_rt* rt;  // table the allocation is registered in, or null
        int32_t id;
    };
    int device = 0;
    uint64_t gran = 0;
    bool user_hint = false;  // placed at a base address the caller asked for
    uint64_t b[4] = {0, 0, 0, 0};
    bool reserved[3] = {false, false, false};
    uint64_t backed[3] = {0, 0, 0};  // bytes mapped at the start of each aperture
    hipMemGenericAllocationHandle_t h[3] = {};
    agile::VaRanges va[3];
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

// Undo what create set up: unmap and release each aperture's backing, then free its
// reservation. Failures are cleared from the runtime's last-error state, which later launch
// checks read; the return value says whether everything was released.
static bool teardown(agile_aperture* ap) {
    bool ok = true;
    for (int k = 0; k < 3; ++k) {
        void* p = reinterpret_cast<void*>(ap->b[k]);
        if (ap->backed[k]) {
            ok &= hipMemUnmap(p, ap->backed[k]) == hipSuccess;
            ok &= hipMemRelease(ap->h[k]) == hipSuccess;
            ap->backed[k] = 0;
        }
        if (ap->reserved[k]) {
            // The HIP runtime may refuse to release a reservation placed at an address the
            // caller asked for; that address range then stays reserved (no memory) until the
            // process ends.
            const bool freed = hipMemAddressFree(p, ap->b[k + 1] - ap->b[k]) == hipSuccess;
            ok &= freed || ap->user_hint;
            ap->reserved[k] = false;
        }
    }
    (void)hipGetLastError();
    return ok;
}

// Reserve the three apertures back to back from b0 (each at its requested address); false,
// with nothing left reserved, when the runtime places any of them elsewhere.
static bool reserve_at(agile_aperture* ap, uint64_t b0, const uint64_t* sz) {
    uint64_t at = b0;
    for (int k = 0; k < 3; ++k) {
        void* p = nullptr;
        const hipError_t e = hipMemAddressReserve(&p, sz[k], ap->gran, reinterpret_cast<void*>(at), 0);
        if (e == hipSuccess && reinterpret_cast<uint64_t>(p) != at) (void)hipMemAddressFree(p, sz[k]);
        if (e != hipSuccess || reinterpret_cast<uint64_t>(p) != at) {
            (void)hipGetLastError();
            for (int j = 0; j < k; ++j) {
                (void)hipMemAddressFree(reinterpret_cast<void*>(ap->b[j]), sz[j]);
                ap->reserved[j] = false;
            }
            (void)hipGetLastError();
            return false;
        }
        ap->b[k] = at;
        ap->reserved[k] = true;
        at += sz[k];
    }
    ap->b[3] = at;
    return true;
}

}  // namespace agile

using namespace agile;

extern "C" {

int agile_aperture_create(agile_aperture** out, int device, const uint64_t* sizes,
                          const uint64_t* backed, uint64_t base_hint) {
    constexpr uint64_t MAXB = 1ull << 48;
    if (!out || !sizes) return AGILE_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (sizes[k] == 0 || sizes[k] > MAXB || (backed && backed[k] > sizes[k]))
            return AGILE_EINVAL;
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
    // Backing: one physical allocation mapped at the start of each aperture (the runtime grants
    // access reliably to one mapping per reservation only).
    hipMemAccessDesc acc = {};
    acc.location = prop.location;
    acc.flags = hipMemAccessFlagsProtReadWrite;
    for (int k = 0; k < 3; ++k) {
        const uint64_t n = backed ? up(backed[k]) : 0;
        ap->va[k].reset(ap->b[k], ap->b[k] + n);
        if (n == 0) continue;
        void* p = reinterpret_cast<void*>(ap->b[k]);
        if (hipMemCreate(&ap->h[k], n, &prop, 0) != hipSuccess) {
            (void)hipGetLastError();
            teardown(ap);
            delete ap;
            return AGILE_ENOMEM;
        }
        if (hipMemMap(p, n, 0, ap->h[k], 0) != hipSuccess) {
            (void)hipMemRelease(ap->h[k]);
            (void)hipGetLastError();
            teardown(ap);
            delete ap;
            return AGILE_EDEVICE;
        }
        ap->backed[k] = n;
        if (hipMemSetAccess(p, n, &acc, 1) != hipSuccess) {
            (void)hipGetLastError();
            teardown(ap);
            delete ap;
            return AGILE_EDEVICE;
        }
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
        for (auto& [addr, a] : ap->allocs)
            if (a.rt) (void)agile_rt_remove(a.rt, a.id);
        ap->allocs.clear();
        if (!teardown(ap)) rc = AGILE_EDEVICE;
    }
    delete ap;
    return rc;
}

int agile_aperture_info(const agile_aperture* ap, uint64_t* bounds, uint64_t* backed,
                        uint64_t* granularity) {
    if (!ap) return AGILE_EINVAL;
    if (bounds)
        for (int k = 0; k < 4; ++k) bounds[k] = ap->b[k];
    if (backed)
        for (int k = 0; k < 3; ++k) backed[k] = ap->backed[k];
    if (granularity) *granularity = ap->gran;
    return AGILE_OK;
}

int agile_aperture_alloc(agile_aperture* ap, int region, uint64_t bytes, agile_rt* rt,
                         void** out_ptr, int32_t* out_id) {
    if (!ap || !out_ptr || region < AGILE_AP_IO || region > AGILE_AP_USER || bytes == 0 ||
        bytes > ap->b[region + 1] - ap->b[region])
        return AGILE_EINVAL;
    const uint64_t n = (bytes + ap->gran - 1) / ap->gran * ap->gran;
    uint64_t addr = 0;
    if (!ap->va[region].take(n, &addr)) return AGILE_ENOSPC;
    int32_t id = -1;
    if (rt) {
        // carved from the aperture's mapped backing: memory a kernel may touch
        const int rc = agile_rt_insert(rt, addr, bytes, kind_of(region) | AGILE_RANGE_BACKED, &id);
        if (rc != AGILE_OK) {
            ap->va[region].give(addr, n);
            return rc;
        }
    }
    ap->allocs.emplace(addr, agile_aperture::Alloc{n, region, rt, id});
    *out_ptr = reinterpret_cast<void*>(addr);
    if (out_id) *out_id = id;
    return AGILE_OK;
}

int agile_aperture_free(agile_aperture* ap, void* ptr) {
    if (!ap || !ptr) return AGILE_EINVAL;
    auto it = ap->allocs.find(reinterpret_cast<uint64_t>(ptr));
    if (it == ap->allocs.end()) return AGILE_ENOENT;
    DeviceGuard dg(ap->device);
    // wait first: on a failure nothing has changed
    if (!dg.ok || hipDeviceSynchronize() != hipSuccess) return AGILE_EDEVICE;
    if (it->second.rt) (void)agile_rt_remove(it->second.rt, it->second.id);
    ap->va[it->second.region].give(it->first, it->second.bytes);
    ap->allocs.erase(it);
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
