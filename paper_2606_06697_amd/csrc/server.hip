// Native worker-side request loop with continuous batching (AgileOS Section IV-B: a worker owns
// the device context and executes its clients' mediated requests; Sections IV-C and IV-E: every
// pointer argument is checked against the calling client's own table before the real work).
//
// Host code only; every request runs in the persistent batch kernel through agile_batch_run.
// The loop polls, in order:
//  1. retire: launches whose completion event has fired give their requests' latencies and
//     results (written by the batch kernel straight into pinned host memory) and return their
//     output space;
//  2. revoke: clients whose assignment ends now lose every range (agile_rt_clear); launches
//     already queued keep the table they were made with;
//  3. arrive: requests whose arrival time has passed join a FIFO;
//  4. admit + launch: from the FIFO head, requests are admitted while their output fits the
//     client's output ring and the in-flight HBM budget (a revoked client's requests are
//     refused), then launched as one batch on a free stream.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <new>
#include <thread>
#include <vector>

#include "device_guard.h"
#include "agile_guard.h"
#include "ring.h"

namespace {

using agile::DeviceGuard;

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    void* h_res = nullptr;       // agile_req_result[max_batch], pinned host memory that the
                                 // batch kernel writes directly (read after its event fires)
    bool busy = false;
    std::vector<uint64_t> rids;
    std::vector<std::pair<uint32_t, uint64_t>> allocs;  // (client, ring start)
    uint64_t nbytes = 0;
};

}  // namespace

struct agile_server {
    int device = 0;
    agile_clients* cs = nullptr;
    std::vector<agile_rt*> tables;
    std::vector<agile::Ring> rings;
    agile_server_config cfg{};
    const agile_ptr* d_ptrs = nullptr;
    uint64_t nptrs = 0;
    uint8_t* d_pv = nullptr;
    int32_t* d_po = nullptr;
    std::vector<Slot> slots;
};

int agile_server_create(agile_server** out, agile_clients* cs, agile_rt* const* tables,
                        uint32_t nclients, const uint64_t* ring_base, const uint64_t* ring_bytes,
                        const agile_server_config* cfg, const agile_ptr* d_ptrs, uint64_t nptrs,
                        uint8_t* d_ptr_verdict, int32_t* d_ptr_owner, int device) {
    if (!out || !cs || !tables || nclients == 0 || !ring_base || !ring_bytes || !cfg ||
        cfg->max_batch == 0 || cfg->max_batch > (1u << 16) || cfg->max_inflight == 0 ||
        cfg->max_inflight > 16)
        return AGILE_EINVAL;
    if (nptrs && (!d_ptrs || !d_ptr_verdict || !d_ptr_owner)) return AGILE_EINVAL;
    for (uint32_t c = 0; c < nclients; ++c)
        if (!tables[c] || ring_bytes[c] < 256 || (ring_base[c] & 255)) return AGILE_EINVAL;
    DeviceGuard dg(device);
    if (!dg.ok) return AGILE_EDEVICE;
    agile_server* sv = new (std::nothrow) agile_server();
    if (!sv) return AGILE_ENOMEM;
    sv->device = device;
    sv->cs = cs;
    sv->tables.assign(tables, tables + nclients);
    sv->rings.resize(nclients);
    for (uint32_t c = 0; c < nclients; ++c) {
        sv->rings[c].base = ring_base[c];
        sv->rings[c].size = ring_bytes[c];
    }
    sv->cfg = *cfg;
    sv->d_ptrs = d_ptrs;
    sv->nptrs = nptrs;
    sv->d_pv = d_ptr_verdict;
    sv->d_po = d_ptr_owner;
    sv->slots.resize(cfg->max_inflight);
    const size_t rbytes = (size_t)cfg->max_batch * sizeof(agile_req_result);
    for (Slot& sl : sv->slots) {
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc(&sl.h_res, rbytes, hipHostMallocDefault) != hipSuccess) {
            agile_server_destroy(sv);
            return AGILE_ENOMEM;
        }
    }
    *out = sv;
    return AGILE_OK;
}

int agile_server_destroy(agile_server* sv) {
    if (!sv) return AGILE_OK;
    DeviceGuard dg(sv->device);
    int rc = AGILE_OK;
    for (Slot& sl : sv->slots) {
        if (sl.stream && hipStreamSynchronize(sl.stream) != hipSuccess) rc = AGILE_EDEVICE;
        if (sl.done) (void)hipEventDestroy(sl.done);
        if (sl.h_res) (void)hipHostFree(sl.h_res);
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
    }
    delete sv;
    return rc;
}

int agile_server_run(agile_server* sv, agile_request* reqs, const uint64_t* out_bytes,
                     const double* arrival_s, uint64_t n, const uint32_t* revoke_client,
                     const double* revoke_s, uint32_t nrevoke, const uint8_t* record,
                     uint8_t* rec_buf, const uint64_t* rec_off, double* latency_s,
                     double* launch_s, agile_req_result* results, agile_server_stats* stats) {
    if (!sv || (n && (!reqs || !out_bytes || !arrival_s || !latency_s || !launch_s)))
        return AGILE_EINVAL;
    if (nrevoke && (!revoke_client || !revoke_s || nrevoke > AGILE_SERVER_MAX_REVOKE))
        return AGILE_EINVAL;
    if (record && (!rec_buf || !rec_off)) return AGILE_EINVAL;
    const uint32_t ncl = (uint32_t)sv->tables.size();
    for (uint64_t i = 0; i < n; ++i) {
        if (reqs[i].client >= ncl) return AGILE_EINVAL;
        if (i && arrival_s[i] < arrival_s[i - 1]) return AGILE_EINVAL;
    }
    for (uint32_t k = 0; k < nrevoke; ++k)
        if (revoke_client[k] >= ncl) return AGILE_EINVAL;
    DeviceGuard dg(sv->device);
    if (!dg.ok) return AGILE_EDEVICE;
    for (uint64_t i = 0; i < n; ++i) {
        latency_s[i] = NAN;
        launch_s[i] = NAN;
    }
    std::vector<std::pair<double, uint32_t>> due;
    for (uint32_t k = 0; k < nrevoke; ++k) due.emplace_back(revoke_s[k], revoke_client[k]);
    std::sort(due.begin(), due.end());
    size_t next_due = 0;
    std::vector<char> revoked(ncl, 0);
    std::vector<double> revoked_at(ncl, NAN);
    std::deque<uint64_t> pending;
    std::vector<agile_request> batch;
    batch.reserve(sv->cfg.max_batch);
    uint64_t nxt = 0, done = 0, launches = 0, refused = 0, inflight_bytes = 0;
    uint64_t max_inflight_bytes = 0, max_concurrent = 0, budget_waits = 0, ring_waits = 0;
    // why the FIFO head last waited (1 budget, 2 ring), so each request is counted once
    std::vector<uint8_t> waited(n, 0);
    auto note_wait = [&](uint64_t r, uint8_t why) {
        if (waited[r] & why) return;
        waited[r] |= why;
        if (why == 1) ++budget_waits;
        else ++ring_waits;
    };
    const auto t0 = std::chrono::steady_clock::now();
    auto clock = [&]() {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    };
    while (done < n) {
        double now = clock();
        // 1. retire finished launches
        for (Slot& sl : sv->slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipErrorNotReady) continue;
            if (q != hipSuccess) return AGILE_EDEVICE;
            const double fin = clock();
            const agile_req_result* hr = static_cast<const agile_req_result*>(sl.h_res);
            for (size_t k = 0; k < sl.rids.size(); ++k) {
                const uint64_t r = sl.rids[k];
                latency_s[r] = fin - arrival_s[r];
                if (results) results[r] = hr[k];
                if (record && record[r]) {
                    const agile_request& rq = reqs[r];
                    const uint64_t addr = rq.copy_bytes ? rq.copy_dst : rq.gather_out;
                    uint8_t* dst = rec_buf + rec_off[r];
                    if (out_bytes[r] &&
                        hipMemcpyAsync(dst, reinterpret_cast<const void*>(addr), out_bytes[r],
                                       hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
                        return AGILE_EDEVICE;
                    if (rq.nptr) {
                        uint8_t* pv = dst + out_bytes[r];
                        if (hipMemcpyAsync(pv, sv->d_pv + rq.ptr_off, rq.nptr, hipMemcpyDeviceToHost,
                                           sl.stream) != hipSuccess ||
                            hipMemcpyAsync(pv + rq.nptr, sv->d_po + rq.ptr_off, rq.nptr * 4,
                                           hipMemcpyDeviceToHost, sl.stream) != hipSuccess)
                            return AGILE_EDEVICE;
                    }
                    if (hipStreamSynchronize(sl.stream) != hipSuccess) return AGILE_EDEVICE;
                }
            }
            done += sl.rids.size();
            for (auto& a : sl.allocs) sv->rings[a.first].free(a.second);
            inflight_bytes -= sl.nbytes;
            sl.busy = false;
        }
        // 2. revocations that are due, while other launches may still be on the device
        while (next_due < due.size() && due[next_due].first <= now) {
            const uint32_t c = due[next_due++].second;
            if (!revoked[c]) {
                const int rc = agile_rt_clear(sv->tables[c]);
                if (rc != AGILE_OK) return rc;
                revoked[c] = 1;
                revoked_at[c] = now;
            }
        }
        // 3. arrivals
        while (nxt < n && arrival_s[nxt] <= now) pending.push_back(nxt++);
        // 4. admission and launch on a free stream
        Slot* free_slot = nullptr;
        for (Slot& sl : sv->slots)
            if (!sl.busy) {
                free_slot = &sl;
                break;
            }
        if (!pending.empty() && free_slot) {
            Slot& sl = *free_slot;
            sl.rids.clear();
            sl.allocs.clear();
            batch.clear();
            uint64_t nbytes = 0;
            while (!pending.empty() && sl.rids.size() < sv->cfg.max_batch) {
                const uint64_t r = pending.front();
                agile_request& rq = reqs[r];
                if (revoked[rq.client]) {
                    pending.pop_front();
                    ++refused;
                    ++done;
                    continue;
                }
                const uint64_t need = out_bytes[r];
                if (need > sv->rings[rq.client].size || need > sv->cfg.hbm_budget) {
                    pending.pop_front();  // can never be admitted
                    ++refused;
                    ++done;
                    continue;
                }
                if (inflight_bytes + nbytes + need > sv->cfg.hbm_budget) {
                    note_wait(r, 1);  // admitted once earlier launches return their bytes
                    break;
                }
                if (need) {
                    uint64_t start, addr;
                    if (!sv->rings[rq.client].alloc(need, &start, &addr)) {
                        note_wait(r, 2);  // admitted once the client's ring drains
                        break;
                    }
                    if (rq.copy_bytes) rq.copy_dst = addr;
                    else rq.gather_out = addr;
                    sl.allocs.emplace_back(rq.client, start);
                }
                pending.pop_front();
                sl.rids.push_back(r);
                batch.push_back(rq);
                nbytes += need;
            }
            if (!batch.empty()) {
                int rc = agile_batch_run(sv->cs, batch.data(), (uint32_t)batch.size(), sv->d_ptrs,
                                         sv->nptrs, sv->d_pv, sv->d_po,
                                         static_cast<agile_req_result*>(sl.h_res), sl.stream);
                if (rc != AGILE_OK) return rc;
                if (hipEventRecord(sl.done, sl.stream) != hipSuccess) return AGILE_EDEVICE;
                for (uint64_t r : sl.rids) launch_s[r] = now;
                sl.nbytes = nbytes;
                inflight_bytes += nbytes;
                sl.busy = true;
                ++launches;
                uint64_t busy = 0;
                for (const Slot& o : sv->slots) busy += o.busy ? 1 : 0;
                max_concurrent = std::max(max_concurrent, busy);
                max_inflight_bytes = std::max(max_inflight_bytes, inflight_bytes);
                continue;
            }
        }
        // idle: nothing on the device and nothing waiting until the next arrival
        bool any_busy = false;
        for (const Slot& sl : sv->slots) any_busy = any_busy || sl.busy;
        if (!any_busy && pending.empty() && nxt < n) {
            const double wait = arrival_s[nxt] - clock();
            if (wait > 200e-6)
                std::this_thread::sleep_for(std::chrono::duration<double>(wait - 100e-6));
        }
    }
    if (stats) {
        std::memset(stats, 0, sizeof(*stats));
        stats->elapsed_s = clock();
        stats->launches = launches;
        stats->refused = refused;
        stats->served = n - refused;
        stats->max_inflight_bytes = max_inflight_bytes;
        stats->max_concurrent = max_concurrent;
        stats->budget_waits = budget_waits;
        stats->ring_waits = ring_waits;
    }
    // revocation times, for the caller (NaN where a revocation was not reached)
    if (stats)
        for (uint32_t k = 0; k < nrevoke; ++k) stats->revoked_at_s[k] = revoked_at[revoke_client[k]];
    return AGILE_OK;
}
