/*
 * agile_aperture.h - fixed address apertures (part of libagile_guard.so; conventions as in
 * agile_guard.h).
 *
 * Section IV-E (Table I) lays the GPU address space out as three fixed apertures, back to
 * back: a protected I/O aperture for MMIO mappings, a protected aperture for kernel/module and
 * imported service memory, and the user aperture that user allocations are carved from.
 * Section V-A builds the layout with the virtual memory API: it reads the allocation
 * granularity, reserves the address ranges, and attaches physical memory (create a handle, map
 * it into the aperture, grant the device access), recording each allocation's base and
 * requested size in the allocation table. An aperture object does the same with HIP's virtual
 * memory calls on one device, and answers the coarse pointer check of the Fig. 2 guard in a
 * few compares per query, whatever the number of allocations.
 *
 * Each allocation gets physical memory of its own, mapped in a reservation of its own at its
 * place in the aperture (the aperture's free runs are reservations too, so its addresses stay
 * reserved), and its access is read back before the allocation is returned: inside one large
 * reservation the HIP runtime refuses device access to some mappings depending on what was
 * mapped before them.
 */
#ifndef AGILE_APERTURE_H
#define AGILE_APERTURE_H

#include <stdint.h>

#include "agile_guard.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct agile_aperture agile_aperture; /* opaque, library-owned */

/* Returned by agile_aperture_create when the device has no virtual memory management. */
enum { AGILE_ENOTSUP = -9 };

/* Aperture indices, in address order (Table I). */
enum { AGILE_AP_IO = 0, AGILE_AP_MODULE = 1, AGILE_AP_USER = 2 };

/* Reserve the I/O, module and user apertures on HIP device `device`, back to back in that
 * order: sizes[k] bytes for aperture k (AGILE_AP_*; each >= 1, rounded up to the device's
 * minimum allocation granularity; at most 2^48 bytes each). No memory is attached yet.
 * budget[k] (NULL: no limit) caps the device memory aperture k may hold mapped at once.
 * `base_hint` (0, or a multiple of the granularity) asks for the layout to
 * start there, as Table I fixes 0xF0000000000; if the runtime cannot place it there, it goes
 * where the runtime has room, and agile_aperture_info reports where. The runtime may refuse to
 * release address ranges it placed at a caller's base: allocations in such a layout then fail
 * with EDEVICE (the layout still answers agile_validate_aperture). *out receives the handle.
 * Errors: EINVAL, ENOTSUP (no virtual memory management on the device), ENOMEM (no room for
 * the layout), EDEVICE. */
int agile_aperture_create(agile_aperture** out, int device, const uint64_t* sizes,
                          const uint64_t* budget, uint64_t base_hint);

/* Wait for all work on the device, remove every allocation still live from the table it was
 * registered in (which must still exist), unmap and release their memory and free the
 * reservations. The HIP runtime may refuse to release a reservation placed at the caller's
 * base_hint: that address range (address space only, no memory) then stays reserved until the
 * process ends, a later create with the same hint is placed elsewhere, and it is not reported
 * as an error. NULL is accepted. */
int agile_aperture_destroy(agile_aperture* ap);

/* bounds[0..3] = the I/O aperture's start, the module aperture's start, the user aperture's
 * start and the user aperture's end; mapped[0..2] = the device memory each aperture holds
 * mapped now (its live allocations, each rounded up to the granularity); *granularity = the
 * mapping unit in bytes. Any output may be NULL. */
int agile_aperture_info(const agile_aperture* ap, uint64_t* bounds, uint64_t* mapped,
                        uint64_t* granularity);

/* Allocate `bytes` (>= 1, at most the aperture's size) of device memory in aperture `region`
 * (AGILE_AP_*), as Section V-A does for every allocation: physical memory of bytes rounded up
 * to the granularity is created, mapped at the lowest free address of the aperture with room
 * for it, in an address reservation of its own, and made readable and writable by the device,
 * which is read back before the call returns. When `rt` is not NULL, the allocation
 * [ptr, ptr + bytes) (the requested size, not the rounded one) is inserted into it with kind
 * USER, PROTECTED or MMIO for the user, module or I/O aperture, marked backed, and *out_id (may
 * be NULL) receives its id (-1 without a table). The memory's contents are undefined. The table
 * must outlive the allocation. Errors: EINVAL, ENOSPC (no free run of the aperture is long
 * enough, or the aperture's budget would be exceeded), ENOMEM (no device memory), EDEVICE (the
 * runtime refused a reservation, the mapping or the access), and the table insertion's errors
 * (nothing is kept on any error). */
int agile_aperture_alloc(agile_aperture* ap, int region, uint64_t bytes, agile_rt* rt,
                         void** out_ptr, int32_t* out_id);

/* Release an allocation made by agile_aperture_alloc (`ptr` exactly as returned): all work on
 * the device is waited for, its memory is unmapped and released, its range is removed from the
 * table it was registered in, and its addresses join the aperture's free run around them.
 * Errors: EINVAL, ENOENT (not a live allocation of this aperture), EDEVICE. */
int agile_aperture_free(agile_aperture* ap, void* ptr);

/* Classify n queries d_q[i] = (addr, len) against the three apertures alone (the coarse check
 * of the Fig. 2 guard; it knows nothing of individual allocations, so a hole or a freed
 * allocation inside the user aperture reads ALLOW). The aperture holding the first byte
 * decides: none -> AGILE_V_UNMAPPED; I/O or module -> AGILE_V_PROTECTED; user -> AGILE_ALLOW
 * if max(len, 1) <= user end - addr, else AGILE_V_STRADDLE. d_verdict[i] receives the verdict
 * (uint8), d_region[i] (int32; may be NULL) the aperture index or -1. Device arrays of n
 * elements owned by the caller; d_q 16-byte aligned, d_region 4-byte aligned. n == 0 is a
 * no-op. Errors: EINVAL, EDEVICE. */
int agile_validate_aperture(const agile_aperture* ap, const agile_ptr* d_q, uint64_t n,
                            uint8_t* d_verdict, int32_t* d_region, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* AGILE_APERTURE_H */
