// Host-side launchers of the guard kernels (internal to libagile_guard.so).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "guard_device.h"

namespace agile {

struct DevInfo {
    int num_cu;
    size_t lds_per_block;  // largest dynamic LDS one workgroup may take
    size_t lds_per_cu;
};

// Maximum number of radix entries (plus one) the validation index may use.
constexpr uint32_t MAX_RADIX = (1u << 14) + 1;

// dma: answer the DMA registration check (only a whole USER range is ALLOW, else INEXACT).
hipError_t launch_validate(const DevTable& t, const DevInfo& d, const void* q, uint64_t n,
                           uint8_t* verdict, int32_t* owner, bool dma, hipStream_t s);

// Guarded launches take the bindings of their pointer arguments, looked up on the host from the
// table the launch is ordered after (`binds` in the operand order of the operation: copy src,
// dst; triad b, c, a; gather idx, table, out; scatter idx, src, dst). With guard == false
// `binds` is ignored and may be null.
hipError_t launch_copy(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* dst,
                       const void* src, uint64_t n, unsigned long long seq, int logon,
                       const DevInfo& d, hipStream_t s);

hipError_t launch_triad(bool guard, const DevTable& t, DevLog* log, const Bind* binds, float* a,
                        const float* b, const float* c, float sc, uint64_t n,
                        unsigned long long seq, int logon, const DevInfo& d, hipStream_t s);

// finish == false leaves the launch's denials in the log scratch for a later kernel (the
// redirecting policies' pass) and the finishing kernel.
hipError_t launch_gather(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* out,
                         const void* tab, uint64_t row_bytes, const int64_t* idx, uint64_t n,
                         uint32_t w, unsigned long long seq, int logon, const DevInfo& d,
                         hipStream_t s, bool finish = true);

// Scatter with accumulate = 1 uses `scratch` (device memory of at least
// scatter_add_scratch_bytes(n) bytes, or null for the chunk path) for its sort; calls that share
// a scratch buffer must be ordered on one stream.
hipError_t launch_scatter(bool guard, const DevTable& t, DevLog* log, const Bind* binds, void* dst,
                          uint64_t row_bytes, const int64_t* idx, const void* src, uint64_t n,
                          uint32_t w, int accumulate, unsigned long long seq, int logon,
                          void* scratch, const DevInfo& d, hipStream_t s, bool finish = true);

// zero_dst: the destination rows are +0.0 before the call (scatter-add mode 2); the sorted path
// then writes each row's sum without reading the row.
hipError_t launch_scatter_add(bool guard, const DevTable& t, DevLog* log, const Bind* binds,
                              void* dst, uint64_t rb, const int64_t* idx, const void* src,
                              uint64_t n, uint32_t w, unsigned long long seq, int logon,
                              void* scratch, const DevInfo& d, hipStream_t s, bool finish = true,
                              bool zero_dst = false);

size_t scatter_add_scratch_bytes(uint64_t n);

// Scatter-add calls of at least this many rows sort their destination keys (when given scratch).
constexpr uint64_t SORT_MIN_N = 1u << 15;

hipError_t launch_log_reset(DevLog* log, hipStream_t s);

// Redirecting policies (sink to a quarantine, report): the pass after a guarded kernel.
constexpr uint32_t REDIRECT_SINK = 1, REDIRECT_REPORT = 2, REDIRECT_REMAP = 3;
struct Redirect {
    uint32_t mode;
    uint32_t pad;
    uint8_t* q;      // quarantine (SINK)
    uint64_t qmask;  // its size - 1 (a power of two)
};
// The bindings (REMAP rewrites into them) come in operand order.
struct RowBinds {
    Bind idx, cont, row;  // index array, contiguous operand (out / src), row-addressed operand
};
hipError_t launch_copy_fix(const DevTable& t, const Redirect& r, Bind bs, Bind bd, void* dst,
                           const void* src, uint64_t n, uint64_t Ks, uint64_t Kd, const DevInfo& d,
                           hipStream_t s);
hipError_t launch_triad_fix(const DevTable& t, const Redirect& r, Bind ba, Bind bb, Bind bc,
                            float* a, const float* b, const float* c, float sc, uint64_t n,
                            uint64_t Ka, uint64_t Kb, uint64_t Kc, const DevInfo& d,
                            hipStream_t s);
// op 0 gather (cont = out, rowp = table), 1 scatter, 2 scatter-add (cont = src, rowp = dst);
// rg: the guard over all n rows; the guarded kernel ran rows below rg.ki.
hipError_t launch_rows_fix(int op, const DevTable& t, DevLog* log, const Redirect& r,
                           const RowBinds& bb, void* cont, void* rowp, uint64_t rb,
                           const int64_t* idx, uint64_t n, const RowsGuard& rg, uint32_t w,
                           const DevInfo& d, hipStream_t s);

// After a guarded row kernel: folds the launch's denial count into the log and records the
// smallest key if the log is empty.
hipError_t launch_fault_finish(const DevTable& t, DevLog* log, const FaultSite& f,
                               unsigned long long seq, hipStream_t s);
FaultSite rows_fault_site(uint32_t op, uint32_t w, uint32_t row_operand, uint64_t rb, uint64_t ki,
                          const void* idx, const void* cont, const void* rowp);

// ---- batched multi-client launch (device images of the public request/result layouts) ----
struct BatchReq {
    uint32_t client, reserved0;
    uint64_t ptr_off, nptr;
    uint64_t copy_dst, copy_src, copy_bytes;
    uint64_t gather_out, gather_table, gather_idx, gather_n;
    uint32_t gather_row_bytes, reserved1;
    uint64_t reserved2;
};
static_assert(sizeof(BatchReq) == 96, "BatchReq mirrors agile_request");

struct BatchScratch {
    unsigned int minfail;      // lowest failing pointer index of the request (or ~0)
    unsigned int remaining;    // tiles of the request not finished yet
    unsigned long long gcount; // gather denials
    unsigned long long gminkey;
    unsigned long long pad;
};
static_assert(sizeof(BatchScratch) == 32, "BatchScratch is 32 bytes");

struct BatchCtl {
    unsigned int next;  // next tile to hand out
    unsigned int pad[15];
};

struct agile_req_result_dev {
    uint32_t verdict;
    int32_t arg;
    int32_t owner;
    uint32_t done;
    unsigned long long fault_count, fault_seq, fault_elem, fault_addr;
    uint32_t fault_width, fault_op, fault_operand, fault_verdict;
    int32_t fault_owner;
    uint32_t fault_reserved;
};
static_assert(sizeof(agile_req_result_dev) == 72, "mirrors agile_req_result");

// Guard of one request, computed on the host from its client's table at launch time (the
// bindings of its copy and gather arguments as allowed prefixes and a row interval).
struct BatchGuard {
    uint64_t copy_ks, copy_kd;  // allowed byte prefixes of copy_src and copy_dst
    RowsGuard gather;           // gather: index / out prefixes and the table's row interval
};

struct BatchArgs {
    BatchCtl* ctl;
    const uint64_t* tstart;  // nreq + 1 entries: first tile of each request, then the total
    const uint32_t* tile_req;  // ntiles entries: the request each tile belongs to
    const BatchGuard* guards;  // nreq entries
    const BatchReq* reqs;
    BatchScratch* scratch;
    const DevTable* tables;
    const ulonglong2* ptrs;
    uint8_t* pv;
    int32_t* po;
    agile_req_result_dev* result;
    uint64_t ntiles;
    uint64_t tile_copy;  // bytes per copy tile of this launch
    uint64_t tile_rows;  // rows per gather tile of this launch
    uint32_t nreq;
    uint32_t pad;
};

// Tile sizes of one launch: small launches get small tiles, so that even one request spreads
// over the whole chip; large launches get the largest tiles (fewer claims, longer streams).
void batch_tile_sizes(uint64_t copy_bytes, uint64_t gather_rows, const DevInfo& d,
                      uint64_t& tile_copy, uint64_t& tile_rows);
uint64_t batch_tiles(const BatchReq& q, uint64_t tile_copy, uint64_t tile_rows);
hipError_t launch_batch(const BatchArgs& a, const DevInfo& d, hipStream_t s);

}  // namespace agile
