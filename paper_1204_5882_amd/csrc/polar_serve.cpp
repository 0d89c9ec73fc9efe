// libpolar serving loop: requests (one frame each) are admitted against a
// device arena, gathered into batches and decoded by the persistent batch
// decoder on up to kStreams streams at once, so that new requests start while
// earlier batches still run (continuous batching).
//
// Admission: a batch takes requests from the head of the queue in arrival
// order while its workspace fits a free range of the arena.  One stream is
// kept for small requests (at most 2^kSmallLog2N bits, about a millisecond of
// decoding): a batch holding a large frame keeps its stream for tens of
// milliseconds while using a few compute units, and would otherwise make the
// small requests behind it wait for a stream.  The small stream takes the
// small requests in arrival order, the others take every request.  Each request is
// charged its own footprint: a descriptor and a scratch slot sized for its
// own N (per-frame slots), so admission follows the frames' sizes, not the
// largest frame of the batch.  A request that cannot fit even an empty arena
// completes with POLAR_E_NOMEM.
//
// Completion is per request: the decoder writes a ticket into a
// host-coherent flag once the frame's u-hat is globally visible, and a poll
// that finds the ticket completes the request, even while the rest of its
// batch is still decoding.  A batch's arena range is released when its
// stream event fires.  Latency is host time from submit to that poll.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "host_internal.h"
#include "polar.h"

using namespace polar_host;

namespace {

// Streams of the server.  HIP gives a process four hardware queues by
// default, and the caller's own stream holds one: a fourth server stream
// would share a queue with another stream, and a small request's kernel
// would then wait behind a large batch's (measured: 2^16 requests at 5-13 ms
// p50 with four streams, 0.6-1.2 ms with three).
constexpr int kStreams = 3;
constexpr int kSmallLog2N = 17;  // stream 0 takes only requests of at most 2^17 bits
constexpr size_t kQueueCap = 1 << 16;

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Req {
    uint64_t id;
    polar_frame f;
    double t_submit;
    uint32_t flag = 0xffffffffu;  // completion flag index while running
    uint32_t ticket = 0;
    bool finished = false;
};

struct Batch {
    bool active = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;    // the batch's work has finished
    hipEvent_t inputs = nullptr;  // inputs produced on the caller's stream
    Stager stager;
    size_t off = 0, bytes = 0;
    std::vector<Req> reqs;
};

}  // namespace

struct polar_server {
    polar_ctx* ctx = nullptr;
    uint8_t* arena = nullptr;
    size_t arena_bytes = 0;
    int max_batch = 0;
    int poll_us = 50;
    hipStream_t input_stream = nullptr;
    std::deque<Req> queue;
    Batch batch[kStreams];
    std::vector<polar_completion> ready;
    uint32_t* flags = nullptr;  // host-coherent completion flags, one per running request
    std::vector<uint32_t> free_flags;
    uint32_t ticket = 0;
};

namespace {

// First-fit over the arena, given the ranges held by active batches.
bool arena_find(const polar_server* s, size_t need, size_t* off) {
    std::vector<std::pair<size_t, size_t>> used;
    for (const auto& b : s->batch)
        if (b.active) used.push_back({b.off, b.off + b.bytes});
    std::sort(used.begin(), used.end());
    size_t cur = 0;
    for (const auto& u : used) {
        if (u.first >= cur + need) {
            *off = cur;
            return true;
        }
        cur = std::max(cur, align256(u.second));
    }
    if (cur + need <= s->arena_bytes) {
        *off = cur;
        return true;
    }
    return false;
}

// Workspace of a growing batch with per-frame slots: the same total
// make_plan computes, kept per launch group so that adding a frame costs no
// re-planning.
struct BatchSize {
    SizeHist g[kGroupKeys];  // f_kind * 2 + leaf dump
    int n = 0;
    static int key(const polar_frame& f) { return f.f_kind * 2 + (f.leaf_llr ? 1 : 0); }
    size_t total(const polar_ctx* c, const SizeHist* h, int nf) const {
        int64_t slots = 0;
        for (int k = 0; k < kGroupKeys; ++k) {
            if (!h[k].count) continue;
            const LaunchCfg cfg = group_cfg(c, k >> 1, (k & 1) != 0, h[k], false, nullptr, false);
            slots += group_slot_bytes(h[k], cfg, true, nullptr);
        }
        return align256(256 + sizeof(FrameDesc) * (size_t)nf) + (size_t)slots;
    }
    size_t total_with(const polar_ctx* c, const polar_frame& f) const {
        SizeHist h[kGroupKeys];
        for (int k = 0; k < kGroupKeys; ++k) h[k] = g[k];
        h[key(f)].add(f.log2n);
        return total(c, h, n + 1);
    }
    void add(const polar_frame& f) {
        g[key(f)].add(f.log2n);
        ++n;
    }
};

void complete(polar_server* s, uint64_t id, int status, double t_submit) {
    polar_completion c{};
    c.req_id = id;
    c.status = status;
    c.latency_s = now_s() - t_submit;
    s->ready.push_back(c);
}

void finish_req(polar_server* s, Req& r, int status) {
    if (r.finished) return;
    r.finished = true;
    complete(s, r.id, status, r.t_submit);
}

void release_batch(polar_server* s, Batch& b) {
    for (const auto& r : b.reqs)
        if (r.flag != 0xffffffffu) s->free_flags.push_back(r.flag);
    b.reqs.clear();
    b.active = false;
}

// Complete requests whose frames are done, and collect finished batches.
// Every batch is examined; the first device error is returned after all of
// them have been reported with their own status.
int reap(polar_server* s) {
    int rc = POLAR_OK;
    for (auto& b : s->batch) {
        if (!b.active) continue;
        for (auto& r : b.reqs)
            if (!r.finished && r.flag != 0xffffffffu &&
                __atomic_load_n(s->flags + r.flag, __ATOMIC_ACQUIRE) == r.ticket)
                finish_req(s, r, POLAR_OK);
        hipError_t e = hipEventQuery(b.done);
        if (e == hipErrorNotReady) continue;
        const int status = e == hipSuccess ? POLAR_OK : POLAR_E_DEVICE;
        for (auto& r : b.reqs) finish_req(s, r, status);
        release_batch(s, b);
        if (e != hipSuccess && rc == POLAR_OK) rc = hip_fail(e, "serving batch");
    }
    return rc;
}

// Start batches on idle streams while requests wait and fit.
int launch(polar_server* s) {
    polar_ctx* c = s->ctx;
    for (int si = 0; si < kStreams; ++si) {
        Batch& b = s->batch[si];
        if (b.active || s->queue.empty()) continue;
        // requests that cannot fit even an empty arena
        while (!s->queue.empty()) {
            if (BatchSize().total_with(c, s->queue.front().f) <= s->arena_bytes) break;
            complete(s, s->queue.front().id, POLAR_E_NOMEM, s->queue.front().t_submit);
            s->queue.pop_front();
        }
        if (s->queue.empty()) break;
        const bool small_only = si == 0;
        // the largest free range bounds the batch
        size_t free_max = 0;
        {
            size_t lo = 0, hi = s->arena_bytes;
            while (lo < hi) {  // largest size that arena_find accepts
                const size_t mid = lo + (hi - lo + 1) / 2;
                size_t o;
                if (arena_find(s, mid, &o)) lo = mid; else hi = mid - 1;
            }
            free_max = lo;
        }
        std::vector<polar_frame> fr;
        std::vector<size_t> taken;  // queue positions, increasing
        BatchSize bs;
        size_t need = 0, off = 0;
        const int limit = std::min<int>(s->max_batch, (int)s->free_flags.size());
        for (size_t qi = 0; qi < s->queue.size() && (int)taken.size() < limit; ++qi) {
            const Req& r = s->queue[qi];
            if (small_only && r.f.log2n > kSmallLog2N) continue;
            const size_t nb = bs.total_with(c, r.f);
            if (nb > free_max) break;
            bs.add(r.f);
            fr.push_back(r.f);
            taken.push_back(qi);
            need = nb;
        }
        if (taken.empty()) {
            if (small_only) continue;  // no small request waits
            break;                     // the head waits for memory
        }
        if (!arena_find(s, need, &off)) break;
        const int take = (int)taken.size();
        Plan p;
        make_plan(c, fr.data(), take, false, p, nullptr, true);
        std::vector<Req> reqs;
        reqs.reserve(taken.size());
        for (size_t qi : taken) reqs.push_back(s->queue[qi]);
        // the requests left in the queue, in arrival order
        const auto drop_taken = [&]() {
            std::deque<Req> rest;
            size_t t = 0;
            for (size_t qi = 0; qi < s->queue.size(); ++qi) {
                if (t < taken.size() && taken[t] == qi) {
                    ++t;
                    continue;
                }
                rest.push_back(s->queue[qi]);
            }
            s->queue.swap(rest);
        };
        for (size_t k = 0; k < p.descs.size(); ++k) {
            Req& r = reqs[(size_t)p.order[k]];
            r.flag = s->free_flags.back();
            s->free_flags.pop_back();
            if (++s->ticket == 0) ++s->ticket;
            r.ticket = s->ticket;
            p.descs[k].done_idx = r.flag;
            p.descs[k].done_val = r.ticket;
        }
        // the batch starts after the work already enqueued on the input stream
        TraceRange tr("polar_serve batch");
        log_line("serve: batch of %zu requests on stream %d, %zu workspace bytes", p.descs.size(), si, need);
        hipError_t e = hipEventRecord(b.inputs, s->input_stream);
        if (e == hipSuccess) e = hipStreamWaitEvent(b.stream, b.inputs, 0);
        int rc = e == hipSuccess ? run_plan(c, p, s->arena + off, need, b.stream, b.stager, false, s->flags)
                                 : hip_fail(e, "serving input dependency");
        if (rc) {
            for (auto& r : reqs) {
                if (r.flag != 0xffffffffu) s->free_flags.push_back(r.flag);
                complete(s, r.id, rc, r.t_submit);
            }
            drop_taken();
            return rc;
        }
        e = hipEventRecord(b.done, b.stream);
        b.active = true;
        b.off = off;
        b.bytes = need;
        b.reqs = std::move(reqs);
        drop_taken();
        if (e != hipSuccess) return hip_fail(e, "serving event");
    }
    return ok();
}

}  // namespace

extern "C" int polar_serve_open(polar_ctx* c, const polar_serve_cfg* cfg, polar_server** out) {
    if (!out) return fail(POLAR_E_INVAL, "out is NULL");
    *out = nullptr;
    if (!c || !cfg) return fail(POLAR_E_INVAL, "NULL argument");
    if (!cfg->arena || cfg->arena_bytes < 4096) return fail(POLAR_E_INVAL, "arena missing or smaller than 4 KiB");
    if (((uintptr_t)cfg->arena & 255) != 0) return fail(POLAR_E_INVAL, "arena must be 256-byte aligned");
    if (cfg->max_slots < 0 || cfg->poll_us < 0) return fail(POLAR_E_INVAL, "negative max_slots or poll_us");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    polar_server* s = new polar_server();
    s->ctx = c;
    s->arena = (uint8_t*)cfg->arena;
    s->arena_bytes = cfg->arena_bytes;
    // default batch: the workgroups of the default decoder that can be resident at once
    s->max_batch = cfg->max_slots ? cfg->max_slots : c->n_cu * occupancy(c, 12, 0, false, 8, true);
    s->poll_us = cfg->poll_us;
    s->input_stream = (hipStream_t)cfg->input_stream;
    const size_t n_flags = (size_t)s->max_batch * kStreams;
    hipError_t e = hipHostMalloc((void**)&s->flags, n_flags * sizeof(uint32_t), hipHostMallocCoherent);
    if (e != hipSuccess) {
        s->flags = nullptr;
        polar_serve_close(s);
        return hip_fail(e, "serving completion flags");
    }
    for (size_t i = 0; i < n_flags; ++i) s->flags[i] = 0;
    for (size_t i = n_flags; i-- > 0;) s->free_flags.push_back((uint32_t)i);
    for (auto& b : s->batch) {
        e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.inputs, hipEventDisableTiming);
        if (e != hipSuccess) {
            polar_serve_close(s);
            return hip_fail(e, "serving streams");
        }
    }
    *out = s;
    return ok();
}

extern "C" int polar_serve_submit(polar_server* s, const polar_frame* req, uint64_t req_id) {
    if (!s || !req) return fail(POLAR_E_INVAL, "NULL argument");
    int rc = validate_frames(req, 1);
    if (rc) return rc;
    if (s->queue.size() >= kQueueCap) return fail(POLAR_E_BUSY, "serving queue full (%zu requests)", kQueueCap);
    Req r;
    r.id = req_id;
    r.f = *req;
    r.t_submit = now_s();
    s->queue.push_back(r);
    return ok();
}

extern "C" int polar_serve_poll(polar_server* s, polar_completion* out, int max_out, int* n_out) {
    if (!s || !n_out || max_out < 0 || (max_out > 0 && !out)) return fail(POLAR_E_INVAL, "bad argument");
    *n_out = 0;
    DeviceGuard g(s->ctx->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", s->ctx->device);
    int rc = reap(s);
    int rc2 = launch(s);
    const int n = std::min<int>(max_out, (int)s->ready.size());
    std::copy(s->ready.begin(), s->ready.begin() + n, out);
    s->ready.erase(s->ready.begin(), s->ready.begin() + n);
    *n_out = n;
    return rc ? rc : rc2;
}

extern "C" int polar_serve_pending(const polar_server* s, int* queued, int* running, int* completed) {
    if (!s) return fail(POLAR_E_INVAL, "NULL server");
    int run = 0;
    for (const auto& b : s->batch)
        for (const auto& r : b.reqs) run += r.finished ? 0 : 1;
    if (queued) *queued = (int)s->queue.size();
    if (running) *running = run;
    if (completed) *completed = (int)s->ready.size();
    return ok();
}

extern "C" int polar_serve_stats(const polar_server* s, int* batches_running, size_t* arena_used) {
    if (!s) return fail(POLAR_E_INVAL, "NULL server");
    int nb = 0;
    size_t used = 0;
    for (const auto& b : s->batch)
        if (b.active) {
            ++nb;
            used += b.bytes;
        }
    if (batches_running) *batches_running = nb;
    if (arena_used) *arena_used = used;
    return ok();
}

extern "C" int polar_serve_cancel(polar_server* s, uint64_t req_id) {
    if (!s) return fail(POLAR_E_INVAL, "NULL server");
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it) {
        if (it->id == req_id) {
            complete(s, it->id, POLAR_E_CANCELLED, it->t_submit);
            s->queue.erase(it);
            return ok();
        }
    }
    for (const auto& b : s->batch)
        for (const auto& r : b.reqs)
            if (r.id == req_id && !r.finished)
                return fail(POLAR_E_BUSY, "request %llu is already running", (unsigned long long)req_id);
    return fail(POLAR_E_INVAL, "request %llu is not queued", (unsigned long long)req_id);
}

extern "C" int polar_serve_close(polar_server* s) {
    if (!s) return ok();
    int rc = POLAR_OK;
    {
        DeviceGuard g(s->ctx->device);
        for (auto& b : s->batch) {
            if (b.active && b.done) {
                hipError_t e = hipEventSynchronize(b.done);
                if (e != hipSuccess && rc == POLAR_OK) rc = hip_fail(e, "serving batch");
            }
            b.stager.release();
            if (b.done) (void)hipEventDestroy(b.done);
            if (b.inputs) (void)hipEventDestroy(b.inputs);
            if (b.stream) (void)hipStreamDestroy(b.stream);
        }
        if (s->flags) (void)hipHostFree(s->flags);
    }
    delete s;
    return rc;
}

extern "C" int polar_serve(polar_ctx* c, const polar_serve_cfg* cfg, polar_next_fn next, polar_done_fn done,
                           void* user) {
    if (!next || !done) return fail(POLAR_E_INVAL, "NULL callback");
    polar_server* s = nullptr;
    int rc = polar_serve_open(c, cfg, &s);
    if (rc) return rc;
    bool ended = false;
    std::vector<polar_completion> comp(256);
    while (true) {
        bool progressed = false;
        while (!ended) {
            polar_frame f{};
            uint64_t id = 0;
            const int r = next(user, &f, &id);
            if (r == 0) {
                const int sr = polar_serve_submit(s, &f, id);
                if (sr) done(user, id, sr, 0.0);
                progressed = true;
            } else if (r == 2) {
                ended = true;
            } else {
                break;
            }
        }
        int n = 0;
        rc = polar_serve_poll(s, comp.data(), (int)comp.size(), &n);
        for (int k = 0; k < n; ++k) done(user, comp[(size_t)k].req_id, comp[(size_t)k].status, comp[(size_t)k].latency_s);
        if (rc) break;
        progressed |= n > 0;
        int q = 0, run = 0, fin = 0;
        (void)polar_serve_pending(s, &q, &run, &fin);
        if (ended && q == 0 && run == 0 && fin == 0) {
            int nb = 0;
            (void)polar_serve_stats(s, &nb, nullptr);
            if (nb == 0) break;  // every request reported and every batch's range released
        }
        if (!progressed && s->poll_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(s->poll_us));
    }
    // A device error ends the loop.  Requests still on the device are reported
    // only after their batch has stopped touching their buffers.
    if (rc) {
        for (auto& b : s->batch) {
            if (!b.active) continue;
            const hipError_t e = hipEventSynchronize(b.done);
            for (auto& r : b.reqs)
                if (!r.finished) {
                    r.finished = true;
                    done(user, r.id, e == hipSuccess ? POLAR_OK : rc, now_s() - r.t_submit);
                }
            release_batch(s, b);
        }
        for (const auto& r : s->ready) done(user, r.req_id, r.status, r.latency_s);
        s->ready.clear();
        for (const auto& r : s->queue) done(user, r.id, POLAR_E_CANCELLED, now_s() - r.t_submit);
        s->queue.clear();
    }
    const int rc2 = polar_serve_close(s);
    return rc ? rc : rc2;
}
