// spect_server.hip - reconstruction server: continuous admission of OSEM
// requests onto concurrent HIP streams, with workspaces carved from one
// device memory pool (admission by memory footprint).
//
// A request is a whole reconstruction (osem_reconstruct).  Requests queue in
// arrival order; the head of the queue is admitted as soon as a slot (a HIP
// stream) is idle and the pool has a free block of the request's workspace
// size, so requests that arrive while others run start without waiting for
// them, and their kernels overlap on the device.  Completion is detected by
// polling an event recorded after the request's launches.  A request's
// launches wait (on the device) for an event recorded on the caller's stream
// when it was submitted, so inputs the caller produced asynchronously are
// complete before the reconstruction reads them.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <deque>
#include <string>
#include <unordered_map>
#include <vector>

#include "spect.h"
#include "spect_internal.h"

using spect_internal::clear_error;
using spect_internal::set_error;

namespace {

struct Request {
    const spect_plan *plan = nullptr;
    float *f = nullptr;
    const float *mu = nullptr, *g = nullptr, *s = nullptr;
    int iters = 0, subsets = 1;
    size_t ws = 0, off = 0;
    hipEvent_t ready = nullptr;  // recorded on the caller's stream at submission
    int state = SPECT_REQ_QUEUED;
    int slot = -1;
    int err = SPECT_OK;
    std::string msg;
};

struct Block {
    size_t off, size;
};

size_t round256(size_t x) { return (x + 255) & ~size_t(255); }

int failf(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
int failf(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    return set_error(code, buf);
}

}  // namespace

struct spect_server {
    int device = 0;
    std::vector<hipStream_t> slots;
    std::vector<hipEvent_t> done;
    std::vector<int64_t> busy;  // request per slot, -1 when idle
    char *pool = nullptr;
    size_t pool_bytes = 0, in_use = 0;
    std::vector<Block> free_list;  // sorted by offset, coalesced
    std::deque<int64_t> queue;
    std::unordered_map<int64_t, Request> reqs;
    int64_t next_id = 1;
    int peak_running = 0;

    bool alloc(size_t n, size_t *off)
    {
        for (size_t i = 0; i < free_list.size(); ++i)
            if (free_list[i].size >= n) {
                *off = free_list[i].off;
                free_list[i].off += n;
                free_list[i].size -= n;
                if (free_list[i].size == 0) free_list.erase(free_list.begin() + i);
                in_use += n;
                return true;
            }
        return false;
    }

    void release(size_t off, size_t n)
    {
        in_use -= n;
        auto it = std::lower_bound(free_list.begin(), free_list.end(), off,
                                   [](const Block &b, size_t o) { return b.off < o; });
        it = free_list.insert(it, Block{off, n});
        const size_t i = it - free_list.begin();
        if (i + 1 < free_list.size() && free_list[i].off + free_list[i].size == free_list[i + 1].off) {
            free_list[i].size += free_list[i + 1].size;
            free_list.erase(free_list.begin() + i + 1);
        }
        if (i > 0 && free_list[i - 1].off + free_list[i - 1].size == free_list[i].off) {
            free_list[i - 1].size += free_list[i].size;
            free_list.erase(free_list.begin() + i);
        }
    }

    static void drop_ready(Request &r)
    {
        if (r.ready) (void)hipEventDestroy(r.ready);
        r.ready = nullptr;
    }

    int running() const
    {
        int n = 0;
        for (int64_t r : busy) n += r >= 0;
        return n;
    }

    // Retire finished requests, then admit from the head of the queue.
    void progress()
    {
        for (size_t k = 0; k < slots.size(); ++k) {
            if (busy[k] < 0) continue;
            const hipError_t e = hipEventQuery(done[k]);
            if (e == hipErrorNotReady) continue;
            Request &r = reqs[busy[k]];
            if (e == hipSuccess) {
                r.state = SPECT_REQ_DONE;
            } else {
                r.state = SPECT_REQ_FAILED;
                r.err = SPECT_EHIP;
                r.msg = hipGetErrorString(e);
            }
            release(r.off, r.ws);
            drop_ready(r);
            r.slot = -1;
            busy[k] = -1;
        }
        while (!queue.empty()) {
            int k = -1;
            for (size_t i = 0; i < slots.size(); ++i)
                if (busy[i] < 0) {
                    k = (int)i;
                    break;
                }
            if (k < 0) break;
            Request &r = reqs[queue.front()];
            size_t off = 0;
            if (!alloc(r.ws, &off)) break;  // the head waits for memory; arrival order is kept
            const int64_t id = queue.front();
            queue.pop_front();
            int st = SPECT_OK;
            if (hipStreamWaitEvent(slots[k], r.ready, 0) != hipSuccess) {
                st = set_error(SPECT_EHIP, "slot stream could not wait for the submission event");
            } else {
                st = osem_reconstruct(r.plan, r.f, r.mu, r.g, r.s, r.iters, r.subsets, pool + off, r.ws, slots[k]);
                if (st == SPECT_OK && hipEventRecord(done[k], slots[k]) != hipSuccess) st = SPECT_EHIP;
            }
            if (st != SPECT_OK) {
                r.state = SPECT_REQ_FAILED;
                r.err = st;
                r.msg = spect_last_error();
                release(off, r.ws);
                // the slot stream may hold the wait on the event: destroy it
                // only once the stream has drained
                (void)hipStreamSynchronize(slots[k]);
                drop_ready(r);
                continue;
            }
            r.off = off;
            r.slot = k;
            r.state = SPECT_REQ_RUNNING;
            busy[k] = id;
            peak_running = std::max(peak_running, running());
        }
    }
};

extern "C" {

int spect_server_create(int32_t n_slots, size_t pool_bytes, spect_server **out)
{
    if (!out) return set_error(SPECT_EINVAL, "out is NULL");
    *out = nullptr;
    if (n_slots < 1 || n_slots > 64) return failf(SPECT_EINVAL, "n_slots = %d outside [1, 64]", n_slots);
    if (pool_bytes < 256) return set_error(SPECT_EINVAL, "pool_bytes must be at least 256");
    spect_server *s = new spect_server();
    if (hipGetDevice(&s->device) != hipSuccess) {
        delete s;
        return set_error(SPECT_EHIP, "no HIP device");
    }
    s->pool_bytes = pool_bytes & ~size_t(255);
    if (hipMalloc(reinterpret_cast<void **>(&s->pool), s->pool_bytes) != hipSuccess) {
        delete s;
        return failf(SPECT_ENOMEM, "hipMalloc of a %zu-byte pool failed", pool_bytes);
    }
    s->free_list.push_back(Block{0, s->pool_bytes});
    for (int k = 0; k < n_slots; ++k) {
        hipStream_t st = nullptr;
        hipEvent_t ev = nullptr;
        if (hipStreamCreateWithFlags(&st, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) {
            if (st) (void)hipStreamDestroy(st);
            spect_server_destroy(s);
            return set_error(SPECT_EHIP, "stream or event creation failed");
        }
        s->slots.push_back(st);
        s->done.push_back(ev);
        s->busy.push_back(-1);
    }
    *out = s;
    return clear_error();
}

int spect_server_destroy(spect_server *s)
{
    if (!s) return clear_error();
    for (size_t k = 0; k < s->slots.size(); ++k) (void)hipStreamSynchronize(s->slots[k]);
    for (hipStream_t st : s->slots) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : s->done) (void)hipEventDestroy(ev);
    for (auto &kv : s->reqs) spect_server::drop_ready(kv.second);
    if (s->pool) (void)hipFree(s->pool);
    delete s;
    return clear_error();
}

int spect_server_submit(spect_server *s, const spect_plan *plan, float *f, const float *mu, const float *g,
                        const float *s_add, int32_t n_iters, int32_t n_subsets, void *stream,
                        int64_t *request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    if (!request_id) return set_error(SPECT_EINVAL, "request_id is NULL");
    if (!plan || !f || !g) return set_error(SPECT_EINVAL, "plan, f and g must not be NULL");
    if (n_iters < 0) return failf(SPECT_EINVAL, "n_iters = %d is negative", n_iters);
    size_t ws = 0;
    int st = spect_workspace_size(plan, SPECT_OP_RECON, n_subsets, mu != nullptr, &ws);
    if (st) return st;
    ws = round256(std::max<size_t>(ws, 256));
    if (ws > s->pool_bytes)
        return failf(SPECT_EINVAL, "request needs %zu workspace bytes, the pool has %zu", ws, s->pool_bytes);
    Request r;
    r.plan = plan;
    r.f = f;
    r.mu = mu;
    r.g = g;
    r.s = s_add;
    r.iters = n_iters;
    r.subsets = n_subsets;
    r.ws = ws;
    if (hipEventCreateWithFlags(&r.ready, hipEventDisableTiming) != hipSuccess)
        return set_error(SPECT_EHIP, "event creation failed");
    if (hipEventRecord(r.ready, static_cast<hipStream_t>(stream)) != hipSuccess) {
        (void)hipEventDestroy(r.ready);
        return set_error(SPECT_EHIP, "could not record the submission event on the caller's stream");
    }
    const int64_t id = s->next_id++;
    s->reqs[id] = r;
    s->queue.push_back(id);
    *request_id = id;
    s->progress();
    return clear_error();
}

int spect_server_progress(spect_server *s, int32_t *n_running, int32_t *n_queued)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    s->progress();
    if (n_running) *n_running = s->running();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    return clear_error();
}

int spect_server_status(spect_server *s, int64_t request_id, int32_t *state)
{
    if (!s || !state) return set_error(SPECT_EINVAL, "server and state must not be NULL");
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    *state = it->second.state;
    if (it->second.state == SPECT_REQ_FAILED) return set_error(it->second.err, it->second.msg.c_str());
    return clear_error();
}

int spect_server_wait(spect_server *s, int64_t request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    for (;;) {
        s->progress();
        const Request &r = s->reqs[request_id];
        if (r.state == SPECT_REQ_DONE) return clear_error();
        if (r.state == SPECT_REQ_FAILED) return set_error(r.err, r.msg.c_str());
        // wait for the request itself, or for any running one to free its slot and memory
        int k = r.slot;
        if (k < 0)
            for (size_t i = 0; i < s->busy.size(); ++i)
                if (s->busy[i] >= 0) {
                    k = (int)i;
                    break;
                }
        if (k < 0) return set_error(SPECT_EINVAL, "request cannot be admitted: nothing running, head blocked");
        const hipError_t e = hipEventSynchronize(s->done[k]);
        if (e != hipSuccess && e != hipErrorNotReady) return failf(SPECT_EHIP, "wait: %s", hipGetErrorString(e));
    }
}

int spect_server_stats(const spect_server *s, int32_t *n_running, int32_t *n_queued, int32_t *peak_running,
                       size_t *pool_in_use)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    if (n_running) *n_running = s->running();
    if (n_queued) *n_queued = (int32_t)s->queue.size();
    if (peak_running) *peak_running = s->peak_running;
    if (pool_in_use) *pool_in_use = s->in_use;
    return clear_error();
}

int spect_server_forget(spect_server *s, int64_t request_id)
{
    if (!s) return set_error(SPECT_EINVAL, "server is NULL");
    auto it = s->reqs.find(request_id);
    if (it == s->reqs.end()) return failf(SPECT_EINVAL, "unknown request %lld", (long long)request_id);
    if (it->second.state != SPECT_REQ_DONE && it->second.state != SPECT_REQ_FAILED)
        return set_error(SPECT_EINVAL, "request is still queued or running");
    s->reqs.erase(it);
    return clear_error();
}

}  // extern "C"
