// Request-serving runtime over resident device graphs (gpm_server_* in
// gpm.h).  One scheduler thread owns all HIP work of the server:
//   - completions: each busy slot's event is polled; its pinned result copy
//     is then complete, the workspace returns to the pool;
//   - admissions: the queue head is admitted when a slot is free and its
//     workspace fits in the pool (first fit over a free list), so work that
//     arrives while others run is started as soon as slots and memory free
//     up, and runs concurrently on its own stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <new>
#include <thread>
#include <vector>

#include "gpm_internal.h"

namespace {

double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

// First-fit allocator over [0, size) in 256-byte units.
class Pool {
public:
    explicit Pool(uint64_t size) { free_[0] = size & ~uint64_t(255); }
    bool alloc(uint64_t bytes, uint64_t &off) {
        bytes = (bytes + 255) & ~uint64_t(255);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= bytes) {
                off = it->first;
                const uint64_t rest = it->second - bytes;
                free_.erase(it);
                if (rest) free_[off + bytes] = rest;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes) {
        bytes = (bytes + 255) & ~uint64_t(255);
        auto it = free_.emplace(off, bytes).first;
        auto nx = std::next(it);
        if (nx != free_.end() && it->first + it->second == nx->first) {
            it->second += nx->second;
            free_.erase(nx);
        }
        if (it != free_.begin()) {
            auto pv = std::prev(it);
            if (pv->first + pv->second == it->first) {
                pv->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t largest() const {
        uint64_t b = 0;
        for (auto &f : free_) b = std::max(b, f.second);
        return b;
    }

private:
    std::map<uint64_t, uint64_t> free_;
};

struct Job {
    gpm_request req;
    gpm_response resp;
    gpm_pattern pat;
    uint64_t ws_bytes = 0, ws_off = 0;
    uint64_t ws_alloc = 0;   // bytes taken from the pool (at least 256)
};

}  // namespace

struct gpm_server {
    gpm_server_config cfg;
    uint64_t result_bytes = 0;     // per-slot device result area at the pool's start
    Pool *pool = nullptr;
    std::vector<hipStream_t> streams;
    std::vector<hipEvent_t> events;
    // per slot: timing events recorded on the slot's stream before and after
    // a request's work, read against `ref` (recorded once at creation)
    std::vector<hipEvent_t> ev_start, ev_end;
    hipEvent_t ref = nullptr;
    std::vector<Job *> slot_job;
    uint64_t *pinned = nullptr;    // per slot: 8 words
    std::mutex mu;
    std::condition_variable cv;
    std::deque<Job *> queue;
    std::vector<gpm_response> done;
    uint64_t next_id = 1;
    int64_t pending = 0;
    bool stop = false;
    std::thread worker;
    int dev = 0;
    int cu_limit = 0;              // compute units one request's grids are sized for
};

namespace {

gpm_status job_workspace(Job *j) {
    if (j->req.kind == GPM_QUERY_CLIQUE) {
        gpm_status rc = gpm_pattern_clique(j->req.k, GPM_VERTEX_INDUCED, &j->pat);
        if (rc) return rc;
        return gpm_workspace_bytes(j->req.graph, &j->pat, &j->ws_bytes);
    }
    if (j->req.kind == GPM_QUERY_MOTIF)
        return gpm_motif_workspace_bytes(j->req.graph, j->req.k, &j->ws_bytes);
    return gpm::fail(GPM_INVALID_ARGUMENT, "unknown query kind");
}

// Enqueues a job on slot i (scheduler thread, lock held).
gpm_status launch(gpm_server *s, int i, Job *j) {
    char *pool = static_cast<char *>(s->cfg.d_pool);
    uint64_t *d_res = reinterpret_cast<uint64_t *>(pool + (uint64_t)i * 256);
    void *ws = pool + s->result_bytes + j->ws_off;
    hipStream_t st = s->streams[i];
    gpm_status rc;
    GPM_HIP(hipEventRecord(s->ev_start[i], st));
    // size this request's persistent grids for its share of the device
    gpm::set_cu_limit(s->cu_limit);
    if (j->req.kind == GPM_QUERY_CLIQUE)
        rc = gpm_count(j->req.graph, &j->pat, ws, j->ws_bytes, d_res, st);
    else
        rc = gpm_motif_count(j->req.graph, j->req.k, ws, j->ws_bytes, d_res, st);
    gpm::set_cu_limit(0);
    if (rc) return rc;
    GPM_HIP(hipEventRecord(s->ev_end[i], st));
    GPM_HIP(hipMemcpyAsync(s->pinned + 8 * i, d_res, 64, hipMemcpyDeviceToHost, st));
    GPM_HIP(hipEventRecord(s->events[i], st));
    return GPM_OK;
}

void finish(gpm_server *s, Job *j) {
    s->done.push_back(j->resp);
    s->pending--;
    delete j;
}

void run(gpm_server *s) {
    // without the device every request fails rather than running elsewhere
    const bool dev_ok = hipSetDevice(s->dev) == hipSuccess;
    const int slots = s->cfg.max_slots;
    std::unique_lock<std::mutex> lock(s->mu);
    for (;;) {
        bool progress = false;
        for (int i = 0; i < slots; i++) {
            Job *j = s->slot_job[i];
            if (!j) continue;
            hipError_t q = hipEventQuery(s->events[i]);
            if (q == hipErrorNotReady) continue;
            j->resp.t_done = now_s();
            if (q != hipSuccess) {
                j->resp.status = GPM_DEVICE_ERROR;
            } else {
                for (int v = 0; v < 7; v++) j->resp.values[v] = s->pinned[8 * i + v];
                float a = 0.f, b = 0.f;
                if (hipEventElapsedTime(&a, s->ref, s->ev_start[i]) == hipSuccess &&
                    hipEventElapsedTime(&b, s->ref, s->ev_end[i]) == hipSuccess) {
                    j->resp.d_start = 1e-3 * a;
                    j->resp.d_end = 1e-3 * b;
                } else {
                    j->resp.d_start = j->resp.d_end = -1.0;
                }
            }
            s->pool->release(j->ws_off, j->ws_alloc);
            s->slot_job[i] = nullptr;
            finish(s, j);
            progress = true;
        }
        while (!s->queue.empty()) {
            int free_slot = -1;
            for (int i = 0; i < slots; i++)
                if (!s->slot_job[i]) { free_slot = i; break; }
            if (free_slot < 0) break;
            Job *j = s->queue.front();
            uint64_t off;
            j->ws_alloc = std::max<uint64_t>(j->ws_bytes, 256);
            if (!s->pool->alloc(j->ws_alloc, off)) break;  // wait for memory
            s->queue.pop_front();
            j->ws_off = off;
            j->resp.t_admit = now_s();
            gpm_status rc = dev_ok ? launch(s, free_slot, j) : GPM_DEVICE_ERROR;
            if (rc) {
                j->resp.status = rc;
                j->resp.t_done = now_s();
                s->pool->release(off, j->ws_alloc);
                finish(s, j);
            } else {
                s->slot_job[free_slot] = j;
            }
            progress = true;
        }
        bool busy = false;
        for (int i = 0; i < slots; i++) busy |= s->slot_job[i] != nullptr;
        if (s->stop && !busy && s->queue.empty()) break;
        if (!progress) {
            if (busy)
                s->cv.wait_for(lock, std::chrono::microseconds(20));
            else
                s->cv.wait_for(lock, std::chrono::milliseconds(5));
        }
    }
}

}  // namespace

extern "C" {

double gpm_server_now(void) { return now_s(); }

gpm_status gpm_server_create(const gpm_server_config *cfg, gpm_server **out) {
    if (!cfg || !out) return gpm::fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (cfg->max_slots < 1 || cfg->max_slots > 64)
        return gpm::fail(GPM_INVALID_ARGUMENT, "max_slots must be in [1, 64]");
    if (cfg->cu_percent < 0 || cfg->cu_percent > 100)
        return gpm::fail(GPM_INVALID_ARGUMENT, "cu_percent must be in [0, 100]");
    if (!cfg->d_pool || ((uintptr_t)cfg->d_pool & 255))
        return gpm::fail(GPM_INVALID_ARGUMENT, "pool NULL or not 256-byte aligned");
    const uint64_t result_bytes = (uint64_t)cfg->max_slots * 256;
    if (cfg->pool_bytes <= result_bytes + 256)
        return gpm::fail(GPM_OUT_OF_MEMORY, "pool too small");
    gpm_server *s = new (std::nothrow) gpm_server;
    if (!s) return gpm::fail(GPM_OUT_OF_MEMORY, "host allocation failed");
    s->cfg = *cfg;
    s->result_bytes = result_bytes;
    s->pool = new Pool(cfg->pool_bytes - result_bytes);
    if (hipGetDevice(&s->dev) != hipSuccess) {
        delete s->pool;
        delete s;
        return gpm::fail(GPM_DEVICE_ERROR, "no current HIP device");
    }
    {
        const int pct = cfg->cu_percent > 0 ? cfg->cu_percent : 50;
        s->cu_limit = std::max(1, gpm::cu_count() * pct / 100);
    }
    for (int i = 0; i < cfg->max_slots; i++) {
        hipStream_t st;
        hipEvent_t ev;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess) {
            gpm_server_destroy(s);
            return gpm::fail(GPM_DEVICE_ERROR, "stream creation failed");
        }
        if (hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            (void)hipStreamDestroy(st);
            gpm_server_destroy(s);
            return gpm::fail(GPM_DEVICE_ERROR, "event creation failed");
        }
        s->streams.push_back(st);
        s->events.push_back(ev);
        s->slot_job.push_back(nullptr);
        hipEvent_t ea, eb;
        if (hipEventCreate(&ea) != hipSuccess) {
            gpm_server_destroy(s);
            return gpm::fail(GPM_DEVICE_ERROR, "event creation failed");
        }
        if (hipEventCreate(&eb) != hipSuccess) {
            (void)hipEventDestroy(ea);
            gpm_server_destroy(s);
            return gpm::fail(GPM_DEVICE_ERROR, "event creation failed");
        }
        s->ev_start.push_back(ea);
        s->ev_end.push_back(eb);
    }
    if (hipEventCreate(&s->ref) != hipSuccess) {
        s->ref = nullptr;
        gpm_server_destroy(s);
        return gpm::fail(GPM_DEVICE_ERROR, "event creation failed");
    }
    if (hipEventRecord(s->ref, s->streams[0]) != hipSuccess ||
        hipEventSynchronize(s->ref) != hipSuccess) {
        gpm_server_destroy(s);
        return gpm::fail(GPM_DEVICE_ERROR, "reference event failed");
    }
    void *pin = nullptr;
    if (hipHostMalloc(&pin, (size_t)cfg->max_slots * 64, hipHostMallocDefault) != hipSuccess) {
        gpm_server_destroy(s);
        return gpm::fail(GPM_DEVICE_ERROR, "pinned host buffer allocation failed");
    }
    s->pinned = static_cast<uint64_t *>(pin);
    s->worker = std::thread(run, s);
    *out = s;
    return GPM_OK;
}

gpm_status gpm_server_submit(gpm_server *s, const gpm_request *r, uint64_t *id) {
    if (!s || !r || !id) return gpm::fail(GPM_INVALID_ARGUMENT, "NULL argument");
    if (!r->graph) return gpm::fail(GPM_INVALID_ARGUMENT, "request without a graph");
    Job *j = new (std::nothrow) Job;
    if (!j) return gpm::fail(GPM_OUT_OF_MEMORY, "host allocation failed");
    std::memset(&j->resp, 0, sizeof(j->resp));
    j->req = *r;
    j->resp.t_submit = now_s();
    j->resp.tag = r->tag;
    j->resp.n_values = r->kind == GPM_QUERY_MOTIF ? (r->k == 3 ? 2 : 6) : 1;
    gpm_status rc = job_workspace(j);
    if (rc) {
        delete j;
        return rc;
    }
    std::lock_guard<std::mutex> lock(s->mu);
    if (std::max<uint64_t>(j->ws_bytes, 256) > s->cfg.pool_bytes - s->result_bytes) {
        delete j;
        return gpm::fail(GPM_OUT_OF_MEMORY, "request workspace larger than the whole pool");
    }
    j->resp.id = s->next_id++;
    *id = j->resp.id;
    s->queue.push_back(j);
    s->pending++;
    s->cv.notify_one();
    return GPM_OK;
}

gpm_status gpm_server_poll(gpm_server *s, gpm_response *out, int32_t max, int32_t *n) {
    if (!s || !n || (max > 0 && !out)) return gpm::fail(GPM_INVALID_ARGUMENT, "NULL argument");
    std::lock_guard<std::mutex> lock(s->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(max, 0), s->done.size());
    for (int32_t i = 0; i < k; i++) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n = k;
    return GPM_OK;
}

int64_t gpm_server_pending(gpm_server *s) {
    if (!s) return 0;
    std::lock_guard<std::mutex> lock(s->mu);
    return s->pending;
}

void gpm_server_destroy(gpm_server *s) {
    if (!s) return;
    {
        std::lock_guard<std::mutex> lock(s->mu);
        s->stop = true;
        s->cv.notify_one();
    }
    if (s->worker.joinable()) s->worker.join();
    for (auto st : s->streams) (void)hipStreamDestroy(st);
    for (auto ev : s->events) (void)hipEventDestroy(ev);
    for (auto ev : s->ev_start) (void)hipEventDestroy(ev);
    for (auto ev : s->ev_end) (void)hipEventDestroy(ev);
    if (s->ref) (void)hipEventDestroy(s->ref);
    if (s->pinned) (void)hipHostFree(s->pinned);
    for (auto *j : s->queue) delete j;
    delete s->pool;
    delete s;
}

}  // extern "C"
