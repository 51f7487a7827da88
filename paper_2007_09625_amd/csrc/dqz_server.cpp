// dqz_server.cpp -- continuous batching of compression and decompression
// requests on one GPU.
//
// Clients submit requests (any thread); one dispatcher thread admits them in
// arrival order as soon as a slot is free and the request's device footprint
// (its input, its output capacity and its workspace) fits the server's HBM
// budget beside the requests already running, enqueues the request's kernels
// on the slot's stream (the same launch sequences as dqz_compress_async /
// dqz_decompress_async, on a workspace carved from a resident arena), and
// polls the slots' completion events.  Requests that arrive while others run
// are admitted the moment a slot and memory free up, and their kernels
// overlap the running ones on the device.  Nothing is allocated per request:
// the arena, the slots' streams, events and pinned status blocks are made
// once, when the server is created.
#include "dqz_host.h"

#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <unordered_map>
#include <unordered_set>

using namespace dqz;
using namespace dqz::host;

namespace {

using Clock = std::chrono::steady_clock;

double us_since(Clock::time_point t0, Clock::time_point t) {
    return std::chrono::duration<double, std::micro>(t - t0).count();
}

// First-fit allocator over [0, size) in 256-byte units, coalescing on free.
class Arena {
public:
    void reset(uint64_t size) {
        free_.clear();
        if (size) free_[0] = size;
    }
    bool alloc(uint64_t bytes, uint64_t &off) {
        bytes = (bytes + 255) / 256 * 256;
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) / 256 * 256;
        auto next = free_.lower_bound(off);
        if (next != free_.end() && off + bytes == next->first) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
private:
    std::map<uint64_t, uint64_t> free_;
};

struct Job {
    uint64_t ticket = 0;
    dqz_request req;
    Plan P;
    WsLayout W;
    HeaderInfo H;
    uint64_t ws_need = 0;      // workspace bytes to carve for it
    uint64_t footprint = 0;    // input + output capacity + workspace
    Clock::time_point t_submit, t_admit;
    uint32_t attempts = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    Readback *h_rb = nullptr;   // pinned, written by the kernels
    Readback *d_rb = nullptr;
    bool busy = false;
    Job job;
    uint64_t ws_off = 0, ws_bytes = 0;
};

}  // namespace

struct dqz_server {
    int device = 0;
    int ncu = 256;
    dqz_server_config cfg;
    void *arena_mem = nullptr;
    Arena arena;
    std::vector<Slot> slots;
    std::thread worker;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    bool stop = false;
    std::deque<Job> incoming;                                  // submitted, not yet seen by the dispatcher
    std::deque<Job> pending;                                   // dispatcher's FIFO (admission order)
    std::unordered_map<uint64_t, dqz_completion> finished;     // ticket -> completion
    std::unordered_set<uint64_t> outstanding;                  // submitted, not yet collected
    uint64_t next_ticket = 1;
    uint64_t in_flight_bytes = 0;
    dqz_server_stats stats;
    Clock::time_point t0;
};

namespace {

// Record a request's completion (with the archive header of a compression,
// or NULL) and wake its waiters.
void complete(dqz_server *sv, const Job &job, int32_t status, uint64_t out_bytes, Clock::time_point t_done,
              const uint8_t *header) {
    dqz_completion c;
    memset(&c, 0, sizeof(c));
    c.status = status;
    c.output_bytes = out_bytes;
    c.footprint = job.footprint;
    c.t_submit_us = us_since(sv->t0, job.t_submit);
    c.t_admit_us = job.attempts ? us_since(sv->t0, job.t_admit) : c.t_submit_us;
    c.t_done_us = us_since(sv->t0, t_done);
    if (header) memcpy(c.header, header, DQZ_HEADER_BYTES);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->finished[job.ticket] = c;
    sv->stats.completed++;
    if (status != DQZ_OK) sv->stats.failed++;
    sv->cv_done.notify_all();
}

// Enqueue a job's kernels on a slot (dispatcher thread only).
void launch(dqz_server *sv, Slot &s) {
    Job &j = s.job;
    uint8_t *ws = static_cast<uint8_t *>(sv->arena_mem) + s.ws_off;
    s.h_rb->bits = 0xFFFFFFFFu;
    s.h_rb->code = 0;
    if (j.req.kind == DQZ_REQ_COMPRESS) {
        enqueue_compress(nullptr, ws, s.ws_bytes, sv->ncu, static_cast<const float *>(j.req.d_input), &j.req.params,
                         static_cast<uint8_t *>(j.req.d_output), j.P, j.W, s.d_rb, s.stream);
    } else {
        launch_publish(s.stream, s.d_rb, 0u, j.H.archive_bytes);
        if (j.H.nelem)
            enqueue_decompress(nullptr, ws, sv->ncu, static_cast<const uint8_t *>(j.req.d_input),
                               static_cast<float *>(j.req.d_output), j.H, j.P, j.W, s.d_rb, s.stream);
    }
    (void)hipEventRecord(s.done, s.stream);
}

void dispatcher(dqz_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        bool busy_any = false;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            for (const Slot &s : sv->slots) busy_any = busy_any || s.busy;
            if (!busy_any && sv->incoming.empty() && sv->pending.empty()) {
                if (sv->stop) return;
                sv->cv_work.wait(lk, [&] { return sv->stop || !sv->incoming.empty(); });
                if (sv->stop && sv->incoming.empty()) return;
            }
            while (!sv->incoming.empty()) {
                sv->pending.push_back(std::move(sv->incoming.front()));
                sv->incoming.pop_front();
            }
        }
        // completions
        for (Slot &s : sv->slots) {
            if (!s.busy) continue;
            const hipError_t e = hipEventQuery(s.done);
            if (e == hipErrorNotReady) continue;
            const Clock::time_point t = Clock::now();
            int32_t st = e == hipSuccess ? s.h_rb->code : DQZ_EHIP;
            if (e == hipSuccess && s.job.req.kind == DQZ_REQ_COMPRESS && s.h_rb->bits == 0xFFFFFFFFu) st = DQZ_EINTERNAL;
            const uint64_t need = s.h_rb->workspace_need;
            const uint64_t out = s.job.req.kind == DQZ_REQ_COMPRESS ? s.h_rb->archive_bytes : s.job.H.nelem * 4;
            sv->arena.release(s.ws_off, s.ws_bytes);
            sv->in_flight_bytes -= s.job.footprint;
            s.busy = false;
            if (st == DQZ_ENOMEM && need > s.ws_bytes && s.job.attempts < 3) {
                // the exception records overflowed the workspace: run it again
                // first in line with the size the device reported
                Job again = s.job;
                again.footprint += need - again.ws_need;
                again.ws_need = need;
                {
                    std::lock_guard<std::mutex> lk(sv->mu);
                    sv->stats.retried++;
                }
                sv->pending.push_front(std::move(again));
                continue;
            }
            const bool hdr = st == DQZ_OK && s.job.req.kind == DQZ_REQ_COMPRESS;
            complete(sv, s.job, st, out, t, hdr ? s.h_rb->header : nullptr);
        }
        // admissions, in arrival order: the head waits until it fits
        uint32_t running = 0;
        for (Slot &s : sv->slots) running += s.busy ? 1u : 0u;
        while (!sv->pending.empty()) {
            Slot *free_slot = nullptr;
            for (Slot &s : sv->slots)
                if (!s.busy) { free_slot = &s; break; }
            if (!free_slot) break;
            Job &j = sv->pending.front();
            if (sv->in_flight_bytes + j.footprint > sv->cfg.hbm_budget && running > 0) break;
            uint64_t off = 0;
            if (!sv->arena.alloc(j.ws_need, off)) {
                if (running > 0) break;
                // nothing runs and it still does not fit: it never will
                Job dead = std::move(j);
                sv->pending.pop_front();
                complete(sv, dead, DQZ_ENOMEM, 0, Clock::now(), nullptr);
                continue;
            }
            Slot &s = *free_slot;
            s.job = std::move(j);
            sv->pending.pop_front();
            s.ws_off = off;
            s.ws_bytes = (s.job.ws_need + 255) / 256 * 256;
            s.job.t_admit = Clock::now();
            s.job.attempts++;
            s.busy = true;
            sv->in_flight_bytes += s.job.footprint;
            running++;
            launch(sv, s);
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stats.admitted++;
            if (running > sv->stats.max_running) sv->stats.max_running = running;
            if (sv->in_flight_bytes > sv->stats.max_in_flight_bytes) sv->stats.max_in_flight_bytes = sv->in_flight_bytes;
        }
        // while kernels run, poll the slots at a short interval
        if (running > 0) std::this_thread::sleep_for(std::chrono::microseconds(5));
    }
}

}  // namespace

extern "C" {

dqz_status dqz_server_create(int device, const dqz_server_config *cfg, dqz_server **out) {
    if (!cfg || !out) return DQZ_EINVAL;
    *out = nullptr;
    if (cfg->slots < 1 || cfg->slots > DQZ_MAX_LANES || cfg->workspace_bytes == 0 || cfg->hbm_budget == 0)
        return DQZ_EINVAL;
    int count = 0;
    if (hipGetDeviceCount(&count) != hipSuccess || device < 0 || device >= count) {
        (void)hipGetLastError();
        return DQZ_EINVAL;
    }
    if (hipSetDevice(device) != hipSuccess) return DQZ_EHIP;
    if (decode_kernel_attributes() != hipSuccess) {
        (void)hipGetLastError();
        return DQZ_EHIP;
    }
    dqz_server *sv = new (std::nothrow) dqz_server;
    if (!sv) return DQZ_ENOMEM;
    sv->device = device;
    sv->cfg = *cfg;
    memset(&sv->stats, 0, sizeof(sv->stats));
    int ncu = 0;
    if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, device) == hipSuccess && ncu > 0)
        sv->ncu = ncu;
    dqz_status st = DQZ_OK;
    if (hipMalloc(&sv->arena_mem, cfg->workspace_bytes) != hipSuccess) {
        (void)hipGetLastError();
        sv->arena_mem = nullptr;
        st = DQZ_ENOMEM;
    }
    sv->arena.reset(cfg->workspace_bytes / 256 * 256);
    sv->slots.resize(cfg->slots);
    for (Slot &s : sv->slots) {
        if (st != DQZ_OK) break;
        if (hipStreamCreateWithFlags(&s.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&s.done, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&s.h_rb, sizeof(Readback), hipHostMallocDefault) != hipSuccess ||
            hipHostGetDevicePointer((void **)&s.d_rb, s.h_rb, 0) != hipSuccess) {
            (void)hipGetLastError();
            st = DQZ_EHIP;
        }
    }
    if (st != DQZ_OK) {
        dqz_server_destroy(sv);
        return st;
    }
    sv->t0 = Clock::now();
    sv->worker = std::thread(dispatcher, sv);
    *out = sv;
    return DQZ_OK;
}

void dqz_server_destroy(dqz_server *sv) {
    if (!sv) return;
    if (sv->worker.joinable()) {
        {
            std::lock_guard<std::mutex> lk(sv->mu);
            sv->stop = true;
        }
        sv->cv_work.notify_all();
        sv->worker.join();   // returns once every submitted request has completed
    }
    (void)hipSetDevice(sv->device);
    for (Slot &s : sv->slots) {
        if (s.stream) (void)hipStreamSynchronize(s.stream);
        if (s.done) (void)hipEventDestroy(s.done);
        if (s.stream) (void)hipStreamDestroy(s.stream);
        if (s.h_rb) (void)hipHostFree(s.h_rb);
    }
    if (sv->arena_mem) (void)hipFree(sv->arena_mem);
    delete sv;
}

dqz_status dqz_server_submit(dqz_server *sv, const dqz_request *req, uint64_t *ticket) {
    if (!sv || !req || !ticket) return DQZ_EINVAL;
    Job j;
    j.req = *req;
    std::string why;
    dqz_status st;
    if (req->kind == DQZ_REQ_COMPRESS) {
        st = plan_compress_args(static_cast<const float *>(req->d_input), &req->shape, &req->params, req->d_output,
                                req->output_capacity, j.P, j.W, why);
        if (st != DQZ_OK) return st;
        // the fixed layout plus room for exception records past the tiles'
        // slots: one record per element, enough for every element an outlier
        // (a request that also needs many patches runs again with what the
        // device reports)
        j.ws_need = j.W.fixed + 8ull * j.P.g.nelem;
        j.footprint = 4ull * j.P.g.nelem + req->output_capacity + j.ws_need;
    } else if (req->kind == DQZ_REQ_DECOMPRESS) {
        if (!req->d_input) return DQZ_EINVAL;
        st = plan_decompress_args(req->header, req->input_bytes, static_cast<float *>(req->d_output),
                                  req->output_capacity / 4, j.H, j.P, j.W, why);
        if (st != DQZ_OK) return st;
        j.ws_need = j.H.nelem ? j.W.total : 256;
        j.footprint = req->input_bytes + 4ull * j.H.nelem + j.ws_need;
    } else {
        return DQZ_EINVAL;
    }
    if (j.ws_need > sv->cfg.workspace_bytes) return DQZ_ENOMEM;   // could never be admitted
    j.t_submit = Clock::now();
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        j.ticket = sv->next_ticket++;
        *ticket = j.ticket;
        sv->stats.submitted++;
        sv->outstanding.insert(j.ticket);
        sv->incoming.push_back(std::move(j));
    }
    sv->cv_work.notify_one();
    return DQZ_OK;
}

dqz_status dqz_server_wait(dqz_server *sv, uint64_t ticket, int64_t timeout_us, dqz_completion *out) {
    if (!sv || !out) return DQZ_EINVAL;
    std::unique_lock<std::mutex> lk(sv->mu);
    if (!sv->outstanding.count(ticket)) return DQZ_EINVAL;   // unknown or already collected
    auto ready = [&] { return sv->finished.count(ticket) != 0; };
    if (timeout_us < 0) {
        sv->cv_done.wait(lk, ready);
    } else if (!sv->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
        return DQZ_EAGAIN;
    }
    *out = sv->finished[ticket];
    sv->finished.erase(ticket);
    sv->outstanding.erase(ticket);
    return DQZ_OK;
}

dqz_status dqz_server_get_stats(dqz_server *sv, dqz_server_stats *out) {
    if (!sv || !out) return DQZ_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    *out = sv->stats;
    return DQZ_OK;
}

}  // extern "C"
