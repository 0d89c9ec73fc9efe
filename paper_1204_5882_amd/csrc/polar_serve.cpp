// libpolar serving loop: requests (one frame each) are admitted against a
// device arena, gathered into batches and decoded by the persistent batch
// decoder on up to kStreams streams at once, so that new requests start while
// earlier batches finish (continuous batching at batch granularity).
//
// Admission: a batch takes requests from the head of the queue in arrival
// order while its workspace (descriptors + per-frame scratch, see
// polar_workspace_bytes) fits a free range of the arena; a request that
// cannot fit even an empty arena completes with POLAR_E_NOMEM.  Latency is
// measured on the host from submit to the poll that sees the batch finished.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <deque>
#include <thread>
#include <vector>

#include "host_internal.h"
#include "polar.h"

using namespace polar_host;

namespace {

constexpr int kStreams = 4;
constexpr size_t kQueueCap = 1 << 16;

double now_s() {
    using clk = std::chrono::steady_clock;
    return std::chrono::duration<double>(clk::now().time_since_epoch()).count();
}

struct Req {
    uint64_t id;
    polar_frame f;
    double t_submit;
};

struct Batch {
    bool active = false;
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
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
    std::deque<Req> queue;
    Batch batch[kStreams];
    std::vector<polar_completion> ready;
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

// Workspace of a growing batch, the same total make_plan computes, updated
// per added frame without re-planning.
struct BatchSize {
    struct G { int count = 0, maxlog = 0; };
    G g[4];  // f_kind * 2 + leaf dump
    int n = 0;
    size_t total_with(const polar_ctx* c, const polar_frame& f) const {
        G h[4];
        for (int k = 0; k < 4; ++k) h[k] = g[k];
        const int key = f.f_kind * 2 + (f.leaf_llr ? 1 : 0);
        h[key].count++;
        h[key].maxlog = std::max(h[key].maxlog, (int)f.log2n);
        int slots = 0;
        int64_t slot_bytes = 0;
        for (int k = 0; k < 4; ++k) {
            if (!h[k].count) continue;
            const LaunchCfg cfg = group_cfg(c, k >> 1, h[k].maxlog, h[k].count, (k & 1) != 0, false);
            slots = std::max(slots, cfg.slots);
            slot_bytes = std::max(slot_bytes, polar_dev_slot_bytes(h[k].maxlog, cfg.cutover));
        }
        const size_t slot_off = align256(256 + sizeof(FrameDesc) * (size_t)(n + 1));
        return slot_off + (size_t)slots * (size_t)slot_bytes;
    }
    void add(const polar_frame& f) {
        const int key = f.f_kind * 2 + (f.leaf_llr ? 1 : 0);
        g[key].count++;
        g[key].maxlog = std::max(g[key].maxlog, (int)f.log2n);
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

// Collect finished batches.
int reap(polar_server* s) {
    for (auto& b : s->batch) {
        if (!b.active) continue;
        hipError_t e = hipEventQuery(b.done);
        if (e == hipErrorNotReady) continue;
        const int status = e == hipSuccess ? POLAR_OK : POLAR_E_DEVICE;
        for (const auto& r : b.reqs) complete(s, r.id, status, r.t_submit);
        b.reqs.clear();
        b.active = false;
        if (e != hipSuccess) return hip_fail(e, "serving batch");
    }
    return ok();
}

// Start batches on idle streams while requests wait and fit.
int launch(polar_server* s) {
    polar_ctx* c = s->ctx;
    for (auto& b : s->batch) {
        if (b.active || s->queue.empty()) continue;
        // requests that cannot fit even an empty arena
        while (!s->queue.empty()) {
            if (BatchSize().total_with(c, s->queue.front().f) <= s->arena_bytes) break;
            complete(s, s->queue.front().id, POLAR_E_NOMEM, s->queue.front().t_submit);
            s->queue.pop_front();
        }
        if (s->queue.empty()) break;
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
        BatchSize bs;
        size_t need = 0, off = 0;
        int take = 0;
        for (const auto& r : s->queue) {
            if (take >= s->max_batch) break;
            const size_t nb = bs.total_with(c, r.f);
            if (nb > free_max) break;
            bs.add(r.f);
            fr.push_back(r.f);
            need = nb;
            ++take;
        }
        if (take == 0) break;  // the head waits for memory
        if (!arena_find(s, need, &off)) break;
        Plan p;
        make_plan(c, fr.data(), take, false, p);
        int rc = run_plan(c, p, s->arena + off, need, b.stream, b.stager, false);
        if (rc) {
            for (int k = 0; k < take; ++k) {
                complete(s, s->queue.front().id, rc, s->queue.front().t_submit);
                s->queue.pop_front();
            }
            return rc;
        }
        hipError_t e = hipEventRecord(b.done, b.stream);
        b.active = true;
        b.off = off;
        b.bytes = need;
        for (int k = 0; k < take; ++k) {
            b.reqs.push_back(s->queue.front());
            s->queue.pop_front();
        }
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
    s->max_batch = cfg->max_slots ? cfg->max_slots : 2 * c->n_cu;
    s->poll_us = cfg->poll_us;
    for (auto& b : s->batch) {
        hipError_t e = hipStreamCreateWithFlags(&b.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&b.done, hipEventDisableTiming);
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
    s->queue.push_back({req_id, *req, now_s()});
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
    for (const auto& b : s->batch) run += (int)b.reqs.size();
    if (queued) *queued = (int)s->queue.size();
    if (running) *running = run;
    if (completed) *completed = (int)s->ready.size();
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
            if (r.id == req_id) return fail(POLAR_E_BUSY, "request %llu is already running", (unsigned long long)req_id);
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
            if (b.stream) (void)hipStreamDestroy(b.stream);
        }
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
        if (ended && q == 0 && run == 0 && fin == 0) break;
        if (!progressed && s->poll_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(s->poll_us));
    }
    // a device error ends the loop: report what is left
    if (rc) {
        int n = 0;
        for (auto& b : s->batch) {
            for (const auto& r : b.reqs) done(user, r.id, rc, now_s() - r.t_submit);
            b.reqs.clear();
        }
        for (const auto& r : s->queue) done(user, r.id, POLAR_E_CANCELLED, now_s() - r.t_submit);
        s->queue.clear();
        (void)n;
    }
    const int rc2 = polar_serve_close(s);
    return rc ? rc : rc2;
}
