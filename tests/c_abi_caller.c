/* A C caller of libagile_guard.so (no Python): a table with two user allocations and a
 * protected range, batched validation of four queries, and a guarded copy that runs past its
 * source and destination. Prints "c abi ok" when every result is the expected one. */
#include <stdint.h>
#include <stdio.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "agile_guard.h"

#define CHECK(cond, what)                                  \
    do {                                                   \
        if (!(cond)) {                                     \
            printf("FAIL %s (line %d)\n", what, __LINE__); \
            return 1;                                      \
        }                                                  \
    } while (0)

int main(void) {
    const uint64_t NB = 16384;
    uint8_t *a = NULL, *b = NULL, *prot = NULL, *dv = NULL;
    int32_t* dow = NULL;
    agile_ptr* dq = NULL;
    CHECK(hipMalloc((void**)&a, NB) == hipSuccess, "hipMalloc a");
    CHECK(hipMalloc((void**)&b, NB) == hipSuccess, "hipMalloc b");
    CHECK(hipMalloc((void**)&prot, 65536) == hipSuccess, "hipMalloc prot");
    CHECK(hipMalloc((void**)&dq, 4 * sizeof(agile_ptr)) == hipSuccess, "hipMalloc q");
    CHECK(hipMalloc((void**)&dv, 4) == hipSuccess, "hipMalloc verdict");
    CHECK(hipMalloc((void**)&dow, 4 * sizeof(int32_t)) == hipSuccess, "hipMalloc owner");

    agile_rt* rt = NULL;
    int32_t ia = -1, ib = -1, ip = -1;
    CHECK(agile_rt_create(&rt, 16, 0) == AGILE_OK, "create");
    CHECK(agile_rt_insert(rt, (uint64_t)(uintptr_t)a, NB, AGILE_KIND_USER, &ia) == AGILE_OK, "insert a");
    CHECK(agile_rt_insert(rt, (uint64_t)(uintptr_t)b, NB, AGILE_KIND_USER, &ib) == AGILE_OK, "insert b");
    CHECK(agile_rt_insert(rt, (uint64_t)(uintptr_t)prot, 65536, AGILE_KIND_PROTECTED, &ip) == AGILE_OK,
          "insert prot");
    CHECK(agile_rt_insert(rt, (uint64_t)(uintptr_t)a + 8, 8, AGILE_KIND_USER, NULL) == AGILE_EOVERLAP,
          "overlap refused");

    /* validation: whole allocation, one byte too long, inside the protected range, and an
       address below every range of this table */
    const uint64_t lowest = (uint64_t)(uintptr_t)(a < b ? (a < prot ? a : prot) : (b < prot ? b : prot));
    agile_ptr hq[4] = {{(uint64_t)(uintptr_t)a, NB}, {(uint64_t)(uintptr_t)a, NB + 1},
                       {(uint64_t)(uintptr_t)prot + 8, 8}, {lowest - 1, 1}};
    CHECK(hipMemcpy(dq, hq, sizeof(hq), hipMemcpyHostToDevice) == hipSuccess, "copy queries");
    CHECK(agile_validate_ptrs(rt, dq, 4, dv, dow, NULL) == AGILE_OK, "validate");
    uint8_t v[4];
    int32_t o[4];
    CHECK(hipMemcpy(v, dv, 4, hipMemcpyDeviceToHost) == hipSuccess, "read verdicts");
    CHECK(hipMemcpy(o, dow, sizeof(o), hipMemcpyDeviceToHost) == hipSuccess, "read owners");
    CHECK(v[0] == AGILE_ALLOW && o[0] == ia, "whole allocation allowed");
    CHECK(v[1] == AGILE_V_STRADDLE && o[1] == ia, "one byte too long straddles");
    CHECK(v[2] == AGILE_V_PROTECTED && o[2] == ip, "protected");
    CHECK(v[3] == AGILE_V_UNMAPPED && o[3] == -1, "unmapped");

    /* guarded copy b <- a of NB + 64 bytes: the first NB move, the last 64 are denied twice
       (source load and destination store) */
    CHECK(hipMemset(a, 0x5A, NB) == hipSuccess, "fill a");
    CHECK(hipMemset(b, 0, NB) == hipSuccess, "clear b");
    CHECK(agile_guarded_copy(rt, b, a, NB + 64, AGILE_POLICY_SUPPRESS_LOG, NULL) == AGILE_OK, "copy");
    static uint8_t hb[16384];
    CHECK(hipMemcpy(hb, b, NB, hipMemcpyDeviceToHost) == hipSuccess, "read b");
    for (uint64_t k = 0; k < NB; ++k) CHECK(hb[k] == 0x5A, "copied bytes");
    agile_fault f;
    memset(&f, 0, sizeof(f));
    CHECK(agile_fault_log_read(rt, &f, 1, NULL) == AGILE_EFAULTED, "log non-empty");
    CHECK(f.count == 128 && f.first_seq == 0 && f.first_elem == NB && f.first_operand == 0 &&
              f.first_op == AGILE_OP_COPY && f.first_width == 1,
          "first fault");
    CHECK(agile_fault_log_read(rt, &f, 0, NULL) == AGILE_OK && f.count == 0, "log cleared");

    CHECK(agile_rt_destroy(rt) == AGILE_OK, "destroy");
    hipFree(a);
    hipFree(b);
    hipFree(prot);
    hipFree(dq);
    hipFree(dv);
    hipFree(dow);
    (void)ib;
    printf("c abi ok\n");
    return 0;
}
