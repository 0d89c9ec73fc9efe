// Allocation-free batch decoding: polar_sc_decode_batch_static decodes with
// the library's own static device buffer as its workspace (counters, frame
// descriptors, per-workgroup LLR-level and partial-sum slots) and performs no
// device, pinned or host heap allocation, for callers that cannot allocate.
//
// The buffer is a file-scope __device__ array: each device the library runs
// on holds its own copy until the process ends.  In host code the array's
// name is only a host-side stand-in, so its device address is looked up once
// per device (hipGetSymbolAddress, with that device current) when a context
// is created there, and that address is what the kernels are given.  Every
// call on a device shares the device's buffer: calls that overlap on one
// device race, and each call resets the work counter it uses (a kernel, not
// a memset) before decoding.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>

#include "host_internal.h"
#include "polar.h"

using namespace polar_host;

namespace {

static __device__ __align__(256) uint8_t scratch[POLAR_STATIC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_mutex;
void* g_scratch[kMaxDevices] = {};  // device address of scratch, per device

}  // namespace

namespace polar_host {

// Called by polar_ctx_create with c->device current: finds the device's copy
// of the static buffer (once per device) and reserves the context's host
// tables for the allocation-free path.
int static_setup(polar_ctx* c) {
    if (c->device < 0 || c->device >= kMaxDevices) return fail(POLAR_E_INVAL, "device %d out of range", c->device);
    {
        std::lock_guard<std::mutex> lock(g_mutex);
        if (!g_scratch[c->device]) {
            void* ptr = nullptr;
            const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return hip_fail(e, "static scratch address");
            g_scratch[c->device] = ptr;
        }
        c->static_scratch = g_scratch[c->device];
    }
    c->static_bytes = POLAR_STATIC_SCRATCH_BYTES;
    int rc = c->static_stager.reserve(POLAR_STATIC_MAX_FRAMES);
    if (rc) return rc;
    c->static_plan.descs.reserve(POLAR_STATIC_MAX_FRAMES);
    c->static_plan.order.reserve(POLAR_STATIC_MAX_FRAMES);
    c->static_plan.groups.reserve(4);
    c->static_descs.reserve(POLAR_STATIC_MAX_FRAMES);
    return ok();
}

}  // namespace polar_host

extern "C" int polar_sc_decode_batch_static(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream) {
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    int rc = validate_frames(frames, n_frames);
    if (rc) return rc;
    if (n_frames > POLAR_STATIC_MAX_FRAMES)
        return fail(POLAR_E_INVAL, "%d frames exceed the %d of the allocation-free path", n_frames,
                    POLAR_STATIC_MAX_FRAMES);
    if (n_frames == 0) return ok();
    if (!c->static_scratch) return fail(POLAR_E_DEVICE, "static scratch buffer not set up");
    Plan& p = c->static_plan;
    make_plan(c, frames, n_frames, false, p);
    // per-workgroup slots: as many workgroups as the buffer holds slots for
    if (p.total > c->static_bytes) {
        const size_t room = c->static_bytes > p.slot_off ? c->static_bytes - p.slot_off : 0;
        const int64_t fit = p.slot_bytes > 0 ? (int64_t)(room / (size_t)p.slot_bytes) : 0;
        if (fit < 1)
            return fail(POLAR_E_NOMEM, "batch needs %zu bytes of slots and descriptors, beyond the %zu-byte static buffer",
                        p.slot_off + (size_t)p.slot_bytes, c->static_bytes);
        for (auto& g : p.groups) g.cfg.slots = std::min<int>(g.cfg.slots, (int)fit);
        p.slots = std::min<int>(p.slots, (int)fit);
        p.total = p.slot_off + (size_t)p.slots * (size_t)p.slot_bytes;
    }
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    bind_descs(p, c->static_scratch, c->static_descs);
    rc = c->static_stager.upload(c->static_descs.data(), c->static_descs.size(),
                                 (uint8_t*)c->static_scratch + p.desc_off, s, false);
    if (rc) return rc;
    return enqueue_launches(c, p, c->static_scratch, s, false, nullptr);
}
