/*
 * agile_guard.h - C ABI of the MI355X (gfx950) range guard library (libagile_guard.so).
 *
 * Implements the data-parallel part of the protected GPU memory model of AgileOS
 * (arXiv 2606.06697): an allocation table that separates user allocations from protected
 * module and MMIO ranges (Section IV-E, Table I; Section V-A records each allocation's base
 * and live size), batched API-time pointer validation and the DMA registration check
 * (Section IV-E, V-C), and guarded kernels whose every global access is checked before it
 * happens, with the paper's poison (record, fail later), sink (to a zero page or a
 * quarantine), report, remap_or (restricted to the argument's own allocation) and trap
 * (retire) policies (Section V-E). Around them: client handle tokens (Section IV-C), a batched
 * multi-client launch and a native serving loop with revocation (Sections IV-B, IV-D).
 * agile_aperture.h adds Table I's fixed apertures and their coarse check (Sections IV-E, V-A).
 *
 * Conventions for every entry point
 *  - Return value: AGILE_OK (0) or a negative AGILE_E* code; nothing is thrown across the
 *    ABI. Invalid arguments are rejected before any device work is queued (unsupported
 *    requests fail closed, Section IV-C). Out-parameters are written only on AGILE_OK,
 *    except agile_fault_log_read, which also fills its record when it returns
 *    AGILE_EFAULTED.
 *  - Ownership: the library owns each table handle, its device image and its fault log.
 *    The caller owns every data, query and output buffer (device pointers) and every
 *    stream; the library never frees caller memory.
 *  - Streams: `stream` is a hipStream_t (NULL = the legacy default stream). Device work is
 *    queued asynchronously on it. Table mutations take effect for work queued after them
 *    (the device image is refreshed lazily, in stream order, by the next launch; the handle
 *    keeps two images, so a change does not wait for launches, on any stream, that still
 *    read the previous table).
 *  - Threading: one handle must not be used from two host threads at once, and guarded
 *    calls on one handle that run concurrently on different streams race on its fault
 *    scratch; order them (one stream, or events).
 *  - Guard denials are not errors: validation reports them as verdicts, guarded kernels
 *    suppress them (loads read zero bits, stores are dropped) and count them in the log.
 *  - Overlap: a guarded kernel's output must not alias its inputs except an elementwise
 *    output identical to an input (a == b in the triad); otherwise results are unspecified
 *    (the guard still never writes outside the output's own allocation).
 */
#ifndef AGILE_GUARD_H
#define AGILE_GUARD_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct agile_rt agile_rt; /* opaque, library-owned range-table handle */

enum {
    AGILE_OK = 0,
    AGILE_EINVAL = -1,    /* null handle/pointer, unknown enum value, bad size or alignment */
    AGILE_ENOMEM = -2,    /* device or pinned host allocation failed */
    AGILE_EOVERLAP = -3,  /* inserted range intersects an existing range */
    AGILE_ENOENT = -4,    /* unknown or already removed range id */
    AGILE_ENOSPC = -5,    /* table at capacity, or the id space (2^30 ids) is used up */
    AGILE_EDEVICE = -6,   /* a HIP runtime call or kernel launch failed */
    AGILE_EFAULTED = -7,  /* fault log is non-empty ("poison" surfaces here) */
    AGILE_ETRAPPED = -8,  /* the handle was retired by a violation under AGILE_POLICY_TRAP */
    AGILE_E2BIG = -10     /* more rows than agile_guarded_scatter_add_noalloc's fixed scratch holds */
};

/* Range kinds (Table I): user allocations, protected module/service memory, MMIO. */
enum { AGILE_KIND_USER = 0, AGILE_KIND_PROTECTED = 1, AGILE_KIND_MMIO = 2 };

/* Flag OR-ed into a kind at insertion: the caller states that every byte of the range is
 * mapped device memory that a kernel may touch. Only the REPORT policy reads it (it performs a
 * denied access only inside such a range); classification ignores it. */
enum { AGILE_RANGE_BACKED = 0x80 };

/* Verdicts. The owner of the first byte decides: no owner -> UNMAPPED; a protected or
 * MMIO owner -> PROTECTED; a USER owner -> ALLOW if max(len,1) <= end - addr, else
 * STRADDLE (the byte range must stay inside one live allocation, Section V-C).
 * CROSS_ALLOC only appears as a fault reason: a guarded access that lands in a different
 * user allocation than its argument's. INEXACT only comes from agile_validate_dma. */
enum {
    AGILE_ALLOW = 0,
    AGILE_V_PROTECTED = 1,
    AGILE_V_STRADDLE = 2,
    AGILE_V_UNMAPPED = 3,
    AGILE_V_CROSS_ALLOC = 4,
    AGILE_V_INEXACT = 5
};

/* Guard policies (Section V-E): SUPPRESS_LOG = sink to a zero page + poison record;
 * SUPPRESS_ONLY = sink without a record; TRAP = stop on a violation and retire the context
 * (Section V-E "trap"; Section IV-D: a worker whose context can no longer be trusted is
 * retired). A GPU trap instruction would end every kernel of the process, so TRAP is realized
 * at call granularity: the call runs as under SUPPRESS_LOG (no denied access happens, every
 * denial is counted and the smallest key recorded), then waits for its stream; if it denied
 * at least one access, the handle is retired and the call returns AGILE_ETRAPPED. A TRAP call
 * therefore synchronizes its stream (it cannot be captured in a graph). A retired handle
 * accepts no further work: validation, guarded calls, insertions, agile_rt_sync and batches
 * naming it return AGILE_ETRAPPED before queuing anything; agile_rt_remove (revocation),
 * agile_rt_count, agile_fault_log_read (which then returns AGILE_ETRAPPED) and
 * agile_rt_destroy still work. Retirement lasts until the handle is destroyed. */
enum {
    AGILE_POLICY_SUPPRESS_LOG = 0,
    AGILE_POLICY_SUPPRESS_ONLY = 1,
    AGILE_POLICY_TRAP = 2,
    AGILE_POLICY_SINK = 3,
    AGILE_POLICY_REPORT = 4,
    AGILE_POLICY_REMAP = 5
};
/* SINK (Section V-E "sink": redirect to quarantine memory, for debugging, without isolation
 * between violations): a denied access of width w at exact address A goes to the handle's
 * quarantine (agile_rt_set_quarantine) at offset (A mod 2^64) mod qsize, rounded down to a
 * multiple of w: denied loads read it, denied stores write it, denied scatter-adds add into it
 * (atomically). REPORT (Section V-E "report": log would-be violations without enforcing): a
 * denied access is performed at A when [A, A+w) lies inside one registered range of the table
 * (any kind) that was inserted with AGILE_RANGE_BACKED; everywhere else (outside every range,
 * or in a range not declared backed, which may have no memory behind it) it stays suppressed.
 * Both log every denial as SUPPRESS_LOG does, and both run a second pass after the guarded
 * kernel on the same stream. Denied accesses of one call that reach the same quarantine slot
 * or address are unordered (like duplicate indices of a plain scatter). SINK without a
 * quarantine is EINVAL.
 * REMAP (Section V-E "remap_or", restricted to a safe target): a denied access of width w at
 * exact address A through a pointer argument whose USER range is [lo, hi) is rewritten into
 * that range: with lo' = lo rounded up to a multiple of w and m the largest multiple of w not
 * above hi - lo', it goes to lo' + ((A - lo') mod m) rounded down to a multiple of w (mod taken
 * non-negative). A pointer with no USER range (or with m == 0) leaves the access suppressed.
 * It is logged and run like SINK and REPORT; a remapped store can overwrite data that other
 * elements of the same call read or write, in no defined order. */

/* Guarded operations, as recorded in a fault record. */
enum {
    AGILE_OP_COPY = 1,
    AGILE_OP_TRIAD = 2,
    AGILE_OP_GATHER = 3,
    AGILE_OP_SCATTER = 4,
    AGILE_OP_SCATTER_ADD = 5
};

/* Element types of gather/scatter (element width 4 or 8 bytes). */
enum { AGILE_DTYPE_F32 = 0, AGILE_DTYPE_F64 = 1 };

/* One pointer query: 16 bytes, array-of-structs in device memory. */
typedef struct {
    uint64_t addr;
    uint64_t len;
} agile_ptr;

/* Fault log (56 bytes). `count` is the exact number of denied accesses since the last
 * clear (one per denied element access of its operand's width). The record describes the
 * denial with the smallest key (first_seq, first_elem, first_operand): first_seq numbers
 * the handle's guarded calls in call order from 0, first_elem is the flat element index
 * (byte for copy, element for triad, row*D+col for gather/scatter, row*D for an index
 * load), first_operand the operand's position in its op's access order (copy: src 0,
 * dst 1; triad: b 0, c 1, a 2; gather: idx 0, table 1, out 2; scatter: idx 0, src 1,
 * dst 2). first_addr is the access address mod 2^64, first_verdict the classification
 * of [addr, addr+width) with ALLOW reported as CROSS_ALLOC (UNMAPPED if the exact
 * address lies outside [0, 2^64)), first_owner that range's id or -1.
 * first_seq == UINT64_MAX means no record. */
typedef struct {
    uint64_t count;
    uint64_t first_seq;
    uint64_t first_elem;
    uint64_t first_addr;
    uint32_t first_width;
    uint32_t first_op;
    uint32_t first_operand;
    uint32_t first_verdict;
    int32_t first_owner;
    uint32_t reserved;
} agile_fault;

/* ---- range table (the allocation table of Section V-A / V-C) --------------------- */

/* Create an empty table for up to `capacity` ranges (1 <= capacity <= 2^26) on HIP device
 * `device`; allocates its device image, fault log and pinned staging. *out receives the
 * handle. Errors: EINVAL, ENOMEM, EDEVICE.
 * Three environment variables, read here once per handle, choose among equivalent search
 * layouts (for tests and measurement; no verdict, owner or fault record depends on them):
 * AGILE_LDS_BUDGET=<bytes, at least 1024> caps the LDS the validation's search index may use
 * (default 160 KiB; a smaller budget stages fewer splitters); AGILE_WIDE_RECORDS=1 uses the
 * general 32-byte bucket records even where packed 16-byte ones fit; AGILE_MIN_LIFT=2|4|6|8
 * searches at least that many unrolled levels. Other values are ignored. */
int agile_rt_create(agile_rt** out, uint32_t capacity, int device);

/* Destroy a handle after all work queued with it has completed (the call synchronizes the
 * handle's device before freeing). Removing a client's state revokes its ranges (Section
 * IV-D, lifetime and revocation). NULL is accepted. */
int agile_rt_destroy(agile_rt* rt);

/* Insert the half-open range [base, base+size) of `kind` (an AGILE_KIND_*, optionally OR-ed
 * with AGILE_RANGE_BACKED; any other bit is EINVAL). Requires size >= 1 and
 * base + size <= 2^64 - 1. Adjacent ranges are legal; any intersection gives EOVERLAP.
 * *out_id (may be NULL) receives the new stable id: 0, 1, 2, ... in insertion order,
 * never reused. Errors: EINVAL, EOVERLAP, ENOSPC. */
int agile_rt_insert(agile_rt* rt, uint64_t base, uint64_t size, uint32_t kind,
                    int32_t* out_id);

/* Insert n ranges (host arrays) as one all-or-nothing batch, in array order; ids are
 * assigned in that order. kind[i] as for agile_rt_insert. out_ids (may be NULL) receives n
 * ids. */
int agile_rt_insert_many(agile_rt* rt, const uint64_t* base, const uint64_t* size,
                         const uint8_t* kind, uint32_t n, int32_t* out_ids);

/* Remove range `id` (a freed allocation): its bytes become a hole, so later validation
 * reports UNMAPPED there (freed allocations are rejected, Section IV-E, V-C).
 * Errors: EINVAL, ENOENT. */
int agile_rt_remove(agile_rt* rt, int32_t id);

/* Set the quarantine of the SINK policy: caller-owned device memory of `bytes` bytes (a power
 * of two, 256 .. 2^40, 256-byte aligned), used by later SINK calls until replaced; NULL and 0
 * remove it. The library never frees it. Errors: EINVAL. */
int agile_rt_set_quarantine(agile_rt* rt, void* d_quarantine, uint64_t bytes);

/* Remove every range: the end of a client's assignment revokes all of its allocations
 * (Section IV-D, lifetime and revocation). Ids are not reused afterwards. Launches queued
 * before the call keep the table they were queued with. Works on a retired handle. */
int agile_rt_clear(agile_rt* rt);

/* Number of live ranges. */
int agile_rt_count(const agile_rt* rt, uint32_t* out_n);

/* Upload pending table changes now on `stream` (optional: every launch does it lazily). */
int agile_rt_sync(agile_rt* rt, void* stream);

/* ---- batched API-time pointer validation (Section IV-E, V-C) ----------------------- */

/* Classify n queries d_q[i] = (addr, len) against the table: d_verdict[i] (uint8, AGILE_ALLOW
 * .. AGILE_V_UNMAPPED) and d_owner[i] (int32 range id, -1 when unmapped). All three arrays
 * are caller-owned device memory of n elements; d_q must be 16-byte aligned. n == 0 is a
 * no-op. Errors: EINVAL, EDEVICE. */
int agile_validate_ptrs(agile_rt* rt, const agile_ptr* d_q, uint64_t n, uint8_t* d_verdict,
                        int32_t* d_owner, void* stream);

/* DMA registration check (Section V-C: a module may register a user buffer for device DMA
 * only if it is an exact live user allocation). Same arguments, layout and errors as
 * agile_validate_ptrs; each query gets the pointer verdict, except that an ALLOW range which is
 * not a whole USER range (addr != base or len != size; len is taken as given, so 0 is never
 * exact) gets AGILE_V_INEXACT. The owner is reported as in agile_validate_ptrs. */
int agile_validate_dma(agile_rt* rt, const agile_ptr* d_q, uint64_t n, uint8_t* d_verdict,
                       int32_t* d_owner, void* stream);

/* ---- guarded kernels (kernel memory guard, Section V-E) ----------------------------
 * Each pointer argument is bound once per call to the USER range that contains it (empty if
 * none), looked up in the table as it stands when the call is made (the state the launch is
 * ordered after); every element access is then allowed only if it lies wholly inside its
 * argument's range. Each call takes the next sequence number of the handle. Calls on one
 * handle must be ordered (one stream, or streams the caller synchronizes): they share the
 * handle's fault-log scratch and, for scatter-add, its sort scratch. */

/* dst[k] = src[k] for bytes k < nbytes. Denied src bytes read 0, denied dst bytes are left
 * unchanged. Any alignment; 16-byte-aligned pointers take the vector path. */
int agile_guarded_copy(agile_rt* rt, void* d_dst, const void* d_src, uint64_t nbytes,
                       int policy, void* stream);

/* a[i] = b[i] + s*c[i] for i < n, fp32, rounded twice (no fused multiply-add), denormals
 * kept. 4-byte-aligned pointers required (EINVAL otherwise). */
int agile_guarded_triad(agile_rt* rt, float* d_a, const float* d_b, const float* d_c, float s,
                        uint64_t n, int policy, void* stream);

/* out[i, :] = table[idx[i], :] for i < n, rows of row_bytes bytes (a multiple of the
 * element width of dtype), the row address table + idx[i]*row_bytes computed exactly (an
 * index never wraps around the address space). idx is int64. Requires n*row_bytes/width
 * < 2^62. Pointers must be aligned to the element width. */
int agile_guarded_gather(agile_rt* rt, void* d_out, const void* d_table, uint64_t row_bytes,
                         const int64_t* d_idx, uint64_t n, int dtype, int policy,
                         void* stream);

/* dst[idx[i], :] = src[i, :] (accumulate == 0; with duplicate indices one writer wins) or
 * dst[idx[i], :] += src[i, :] (accumulate == 1). accumulate == 2 is accumulate == 1 for a
 * destination whose rows are all +0.0 before the call (a fresh gradient, for instance): the
 * result is the same bit for bit, and large calls then write each row's sum without reading
 * the row; on any other destination the result is unspecified. Other values: AGILE_EINVAL.
 * With accumulate, calls of at least 32,768
 * rows sort the destination rows (scratch owned by the handle, grown on demand with
 * hipMalloc, freed by agile_rt_destroy; ENOMEM never results: without scratch the call takes
 * the chunk path) and sum each run of equal rows in index order; the order in which partial
 * sums of one row from different parts of the call are added is unspecified, as is the
 * order in smaller calls (per-chunk sums, then atomic adds). */
int agile_guarded_scatter(agile_rt* rt, void* d_dst, uint64_t row_bytes, const int64_t* d_idx,
                          const void* d_src, uint64_t n, int dtype, int accumulate, int policy,
                          void* stream);

/* Read the fault log (queues a device-to-host copy on `stream` and synchronizes it).
 * *out receives the log; clear != 0 then resets it on `stream`. Returns AGILE_ETRAPPED when
 * the handle is retired, else AGILE_EFAULTED when the log holds at least one denial (the
 * paper's "poison" policy reports a violation at a later synchronization boundary, Section
 * V-E), AGILE_OK when it is empty. */
int agile_fault_log_read(agile_rt* rt, agile_fault* out, int clear, void* stream);

/* ---- unguarded twins (same kernels with the guard compiled out; measurement only) ----
 * Every access is performed as addressed: the caller guarantees the arguments are valid.
 * agile_unguarded_scatter with accumulate (1 or 2, as above) and n >= 32,768 sorts 32-bit
 * keys idx + 2^31, so its indices must lie in [-2^31, 2^31 - 1); its sort scratch is one buffer per device
 * (grown on demand), so such calls on one device must be ordered. */
int agile_unguarded_copy(void* d_dst, const void* d_src, uint64_t nbytes, void* stream);
int agile_unguarded_triad(float* d_a, const float* d_b, const float* d_c, float s, uint64_t n,
                          void* stream);
int agile_unguarded_gather(void* d_out, const void* d_table, uint64_t row_bytes,
                           const int64_t* d_idx, uint64_t n, int dtype, void* stream);
int agile_unguarded_scatter(void* d_dst, uint64_t row_bytes, const int64_t* d_idx,
                            const void* d_src, uint64_t n, int dtype, int accumulate,
                            void* stream);

/* ---- batched multi-client requests (Section IV-B: a scheduler assigns each client to a worker;
 * Section IV-C/IV-F: every pointer argument of a mediated request is checked against the
 * calling client's own allocations before the real call). Many requests of many clients run in
 * one persistent launch; each request is judged only against its own client's table. -------- */

typedef struct agile_clients agile_clients; /* opaque: a fixed set of client tables */

/* One request (host memory, 96 bytes). Every part is optional (a zero count skips it):
 *  - validate: nptr pointer arguments at d_ptrs[ptr_off .. ptr_off + nptr) of the launch;
 *  - copy:     guarded copy of copy_bytes bytes from copy_src to copy_dst;
 *  - gather:   guarded gather of gather_n rows of gather_row_bytes bytes (fp32 elements) from
 *              gather_table by the int64 indices at gather_idx into gather_out.
 * All addresses are device addresses judged against client `client`'s table. */
typedef struct {
    uint32_t client;
    uint32_t reserved0;
    uint64_t ptr_off;
    uint64_t nptr;
    uint64_t copy_dst;
    uint64_t copy_src;
    uint64_t copy_bytes;
    uint64_t gather_out;
    uint64_t gather_table;
    uint64_t gather_idx;
    uint64_t gather_n;
    uint32_t gather_row_bytes;
    uint32_t reserved1;
    uint64_t reserved2;
} agile_request;

/* Per-request result (device memory, 72 bytes), written when the request completes:
 * verdict/arg/owner: the verdict of the lowest-index pointer argument that is not ALLOW, its
 * index within the request and its owner (ALLOW, -1, -1 if all pass). fault: the denials of
 * the request's copy and gather (count, and the smallest key; first_seq = the request's index
 * in the launch; a copy's denials precede its gather's). done is set to 1 last. */
typedef struct {
    uint32_t verdict;
    int32_t arg;
    int32_t owner;
    uint32_t done;
    agile_fault fault;
} agile_req_result;

/* Gather `n` table handles (client i = tables[i]) into a client set on `device`. The tables
 * stay owned by the caller and must outlive the set; their later changes are picked up by
 * the next batch. Errors: EINVAL, ENOMEM, EDEVICE. */
int agile_clients_create(agile_clients** out, agile_rt* const* tables, uint32_t n, int device);
int agile_clients_destroy(agile_clients* cs);

/* Run `nreq` requests (host array) in one persistent launch on `stream`. d_ptrs holds the
 * pointer arguments of all requests (device, 16-byte aligned); d_ptr_verdict / d_ptr_owner
 * (device, one entry per pointer) receive each pointer's verdict and owner; d_result (device
 * memory, or pinned host memory from hipHostMalloc; nreq entries) receives each request's
 * result. The request array is copied before the call
 * returns. Requests must not write into each other's inputs or outputs. Errors: EINVAL (bad
 * client index, sizes, alignment), ENOMEM, EDEVICE. */
int agile_batch_run(agile_clients* cs, const agile_request* reqs, uint32_t nreq,
                    const agile_ptr* d_ptrs, uint64_t nptrs, uint8_t* d_ptr_verdict,
                    int32_t* d_ptr_owner, agile_req_result* d_result, void* stream);

/* ---- client handle tokens (Section IV-C: client-visible objects are tokens backed by tables
 * the worker owns, so fabricated, stale and cross-client handles are refused) --------------
 * A token is 64 bits: slot << 40 | gen << 16 | tag. slot (24 bits) indexes the worker's slot
 * table, gen (24 bits) is the slot's generation when the token was minted, and tag (16 bits)
 * is the top 16 bits of SplitMix64(key ^ (slot << 24 | gen)) for the table's secret key
 * (SplitMix64: Steele, Lea and Flood, 2014; state + 0x9e3779b97f4a7c15, then the published
 * finalizer). Minting takes the lowest free slot; releasing advances the slot's generation,
 * which makes every copy of the token stale; a slot released in its last generation is
 * retired. */
typedef struct agile_tokens agile_tokens; /* opaque, library-owned slot table */

enum {
    AGILE_TOKEN_VALID = 0,
    AGILE_TOKEN_FORGED = 1,       /* never minted: bad slot, bad tag, or a generation not issued */
    AGILE_TOKEN_STALE = 2,        /* minted, then released */
    AGILE_TOKEN_CROSS_CLIENT = 3, /* live, but owned by another client */
    AGILE_TOKEN_WRONG_KIND = 4    /* live and owned, but names another kind of object */
};
enum { AGILE_TOKEN_ANY_KIND = 255 };

/* Create a table of `capacity` slots (1 <= capacity <= 2^24) on `device` with secret `key`.
 * Errors: EINVAL, ENOMEM, EDEVICE. */
int agile_tokens_create(agile_tokens** out, uint32_t capacity, uint64_t key, int device);
/* Destroy (synchronizes the device first). NULL is accepted. */
int agile_tokens_destroy(agile_tokens* ts);
/* Mint a token for a new object of `kind` (0..254) owned by `client` (< 0xFFFFFFFE).
 * Errors: EINVAL, ENOSPC (no free slot). */
int agile_token_mint(agile_tokens* ts, uint32_t client, uint32_t kind, uint64_t* out_token);
/* Release the object of a live token owned by `client`. Errors: EINVAL, ENOENT (the token is
 * not a live token of this client; nothing changes). */
int agile_token_release(agile_tokens* ts, uint64_t token, uint32_t client);
/* Check n presented tokens in device memory: d_tokens[i] (uint64, 8-byte aligned) presented by
 * client d_clients[i] (uint32), expecting kind d_kinds[i] (uint8, AGILE_TOKEN_ANY_KIND for any;
 * d_kinds may be NULL: any kind). Writes d_verdict[i] (uint8, AGILE_TOKEN_*) and d_slot[i]
 * (int32: the slot of a VALID token, else -1). Verdict order: FORGED, STALE, CROSS_CLIENT,
 * WRONG_KIND, VALID. Mints and releases made before the call are seen by it (the slot records
 * are refreshed in stream order). n == 0 is a no-op. Errors: EINVAL, EDEVICE. */
int agile_tokens_check(agile_tokens* ts, const uint64_t* d_tokens, const uint32_t* d_clients,
                       const uint8_t* d_kinds, uint64_t n, uint8_t* d_verdict, int32_t* d_slot,
                       void* stream);

/* ---- native serving loop (Section IV-B: a worker executes its clients' mediated requests;
 * Sections IV-C, IV-E: each pointer argument is checked against the calling client's table
 * first; Section IV-D: revocation when a client's assignment ends) -----------------------
 * Open-loop continuous batching over agile_batch_run: requests arrive at given times, wait in
 * a FIFO, are admitted while their output fits the client's output ring and the in-flight HBM
 * budget, and run as persistent batches on up to max_inflight streams, so new batches overlap
 * the ones still on the device. */
typedef struct agile_server agile_server; /* opaque */

typedef struct {
    uint32_t max_batch;     /* requests per launch, 1..65536 */
    uint32_t max_inflight;  /* launches on the device at once (one stream each), 1..16 */
    uint64_t hbm_budget;    /* bytes of outputs in flight, all clients together */
} agile_server_config;

enum { AGILE_SERVER_MAX_REVOKE = 16 };

typedef struct {
    double elapsed_s;
    uint64_t launches;
    uint64_t served;
    uint64_t refused;       /* revoked client, or an output larger than its ring or the budget */
    uint64_t max_inflight_bytes;  /* most output bytes in flight at once (at most hbm_budget) */
    uint64_t max_concurrent;      /* most launches in flight at once (at most max_inflight) */
    uint64_t budget_waits;  /* requests that reached the FIFO head and waited for budget */
    uint64_t ring_waits;    /* requests that reached the FIFO head and waited for ring space */
    double revoked_at_s[AGILE_SERVER_MAX_REVOKE]; /* when each revocation took effect */
} agile_server_stats;

/* A server for client set cs (whose client i is tables[i]), with client i's output ring at
 * device address ring_base[i] (256-byte aligned) of ring_bytes[i] bytes (registered in its
 * table by the caller). d_ptrs / d_ptr_verdict / d_ptr_owner: the pointer pool and its outputs,
 * as in agile_batch_run. Everything stays owned by the caller. Errors: EINVAL, ENOMEM. */
int agile_server_create(agile_server** out, agile_clients* cs, agile_rt* const* tables,
                        uint32_t nclients, const uint64_t* ring_base, const uint64_t* ring_bytes,
                        const agile_server_config* cfg, const agile_ptr* d_ptrs, uint64_t nptrs,
                        uint8_t* d_ptr_verdict, int32_t* d_ptr_owner, int device);
int agile_server_destroy(agile_server* sv);

/* Serve n requests (host arrays). reqs[i] arrives arrival_s[i] seconds after the call starts
 * (non-decreasing); its output slice (out_bytes[i] bytes, 0 for validation) is taken from its
 * client's ring and written into reqs[i].copy_dst or gather_out (reqs is in/out). Client
 * revoke_client[k] is revoked (agile_rt_clear) at revoke_s[k]: launches made before keep the
 * table they were made with, and its requests from then on are refused. Outputs per request:
 * latency_s (completion seen by the loop minus arrival, NaN if refused), launch_s (NaN if
 * refused), results (may be NULL: agile_req_result per request). record (may be NULL): for
 * requests with record[i] != 0, at completion the output bytes and then, for validation, the
 * nptr verdict bytes and nptr owner int32s are copied to rec_buf + rec_off[i]. Returns when
 * every request completed or was refused. Errors: EINVAL, EDEVICE, or those of
 * agile_batch_run. */
int agile_server_run(agile_server* sv, agile_request* reqs, const uint64_t* out_bytes,
                     const double* arrival_s, uint64_t n, const uint32_t* revoke_client,
                     const double* revoke_s, uint32_t nrevoke, const uint8_t* record,
                     uint8_t* rec_buf, const uint64_t* rec_off, double* latency_s,
                     double* launch_s, agile_req_result* results, agile_server_stats* stats);

/* ---- scatter-add without allocation ---------------------------------------------------
 * For callers that cannot allocate device memory: code under HIP graph capture, tight serving
 * loops, harnesses that forbid hipMalloc. Same operation, arguments, policies and errors as
 * agile_guarded_scatter with accumulate = 1, but the sort scratch of its large calls is a fixed
 * array inside the library (AGILE_NOALLOC_SCRATCH_BYTES, one copy per GPU, held until the
 * process ends) instead of a buffer the handle grows with hipMallocAsync; the call allocates no
 * device memory. n above AGILE_NOALLOC_MAX_ROWS returns AGILE_E2BIG before anything is queued.
 * Every call on one GPU shares that GPU's array and leaves its contents behind (each call sets
 * up what it reads): calls that may overlap on one GPU (other streams, other threads) race on
 * it and give wrong sums, so order them on one stream. */
#define AGILE_NOALLOC_MAX_ROWS (1u << 20)
#define AGILE_NOALLOC_SCRATCH_BYTES (17u << 20)
int agile_guarded_scatter_add_noalloc(agile_rt* rt, void* d_dst, uint64_t row_bytes,
                                      const int64_t* d_idx, const void* d_src, uint64_t n,
                                      int dtype, int policy, void* stream);

/* Static text for a status code. */
const char* agile_strerror(int code);

#ifdef __cplusplus
}
#endif

#endif /* AGILE_GUARD_H */
