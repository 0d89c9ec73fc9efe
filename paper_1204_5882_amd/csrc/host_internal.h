// Internal host-side interface shared by the libpolar C ABI translation units
// (decode and options, autotuner, serving loop).  Not part of the public API.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <map>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "polar.h"
#include "sc_device.h"

namespace polar_host {

int fail(int code, const char* fmt, ...);
int ok();
int hip_fail(hipError_t e, const char* what);

// A roctx range for the lifetime of the object (shown by rocprofv3
// --marker-trace around each library call's host work and launches).
struct TraceRange {
    explicit TraceRange(const char* name);
    ~TraceRange();
};

// Diagnostic log to stderr, on when the environment variable POLAR_LOG is
// set to a non-empty value other than 0 (read once).
bool log_on();
void log_line(const char* fmt, ...);

// Keeps the caller's current device unchanged across a call.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev);
    ~DeviceGuard();
};

size_t align256(size_t x);

// Launch parameters of one group of frames.
struct LaunchCfg {
    int cutover = 12;
    int waves = 8;
    int slots = 0;  // workgroups (frames above 2^cutover in flight)
    int fwg = 0;    // frames per workgroup for frames of at most 2^cutover leaves (0 = automatic)
    int prune = -1; // exact node shortcuts: 0 / 1, or -1 = the context's option
    int small_slots = 0;  // workgroups of the per-wavefront launch (computed, not tuned)
    int helpers = 0;      // sweep helpers beside the frame workgroups (computed, not tuned)
};

// Launch-group keys: f_kind * 2 + leaf dump, for every check-update kind.
constexpr int kGroupKeys = (POLAR_F_MINSUM_Q8 + 1) * 2;

// Frame sizes of one launch group: count per log2 N.
struct SizeHist {
    int n[POLAR_MAX_LOG2N + 1] = {};
    int count = 0, maxlog = 0;
    void add(int log2n) {
        ++n[log2n];
        ++count;
        if (log2n > maxlog) maxlog = log2n;
    }
};

// A pinned host buffer for descriptor uploads; the event guards its reuse.
struct Stager {
    FrameDesc* buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    // may_grow = false: refuse (POLAR_E_INVAL) rather than allocate when n
    // exceeds the reserved capacity
    int upload(const FrameDesc* d, size_t n, void* dst, hipStream_t s, bool may_grow = true);
    int reserve(size_t n);  // pinned buffer for n descriptors and the event, allocated now
    void release();
};

// Frames grouped per launch (same f_kind and leaf-dump flag), longest first,
// and the workspace layout [counters | descriptors | slots].  Slots are
// either one per workgroup, sized for the largest frame (batch decoding), or
// one per frame above the cutover, sized for that frame (serving: a request
// is charged its own footprint); descs[k].slot is then an offset from the
// slot area until the plan is bound to a workspace.
struct Plan {
    std::vector<FrameDesc> descs;
    std::vector<int> order;  // descs[k] is frames[order[k]]
    struct Group {
        int fk, dump, first, count, maxlog;
        SizeHist hist;
        LaunchCfg cfg;
    };
    std::vector<Group> groups;
    bool per_frame = false;
    int slots = 0;
    int64_t slot_bytes = 0;
    size_t desc_off = 0, box_off = 0, slot_off = 0, total = 0;
    int boxes = 0;  // sweep mailboxes (frame workgroups of the largest launch with helpers)
};

struct GraphEntry {
    std::vector<uint8_t> key;      // exact bytes the graph was built for
    hipGraphExec_t exec = nullptr;
    FrameDesc* pinned = nullptr;   // descriptor table read by the graph's copy node
    uint64_t last_use = 0;
};

}  // namespace polar_host

struct polar_ctx {
    int device = 0;
    int n_cu = 256;
    void* ws = nullptr;
    size_t ws_bytes = 0;
    int prune = 1;
    int cutover = 0;    // 0 = automatic
    int waves = 0;      // 0 = automatic
    int max_slots = 0;  // 0 = automatic
    int fwg = 0;        // 0 = automatic
    int graph = 0;      // replay batches through cached HIP graphs
    int helpers = 1;    // spare resident workgroups help with the sweeps of large frames
    unsigned long long* prof = nullptr;  // optional device timing counters
    polar_host::Stager stager;
    // resident workgroups per compute unit, per decoder variant and size
    // (fixed size, filled on first use: lookups never allocate)
    mutable std::vector<int> occ_cache = std::vector<int>(5 * 5 * 2 * 2 * 26 * 8, 0);
    // autotuned launch configurations, key (f_kind, log2n of the largest frame)
    std::map<std::pair<int, int>, polar_host::LaunchCfg> tuned;
    // allocation-free decoding (polar_sc_decode_batch_static): host tables
    // reserved at creation, the device's static scratch buffer
    polar_host::Stager static_stager;
    polar_host::Plan static_plan;
    std::vector<FrameDesc> static_descs;
    void* static_scratch = nullptr;
    size_t static_bytes = 0;
    // graph cache
    std::unordered_map<uint64_t, polar_host::GraphEntry> graphs;
    uint64_t graph_clock = 0;
    hipStream_t capture_stream = nullptr;
};

namespace polar_host {

int validate_frames(const polar_frame* frames, int n_frames);
// Resident workgroups per compute unit of a decoder variant (at least 1).
// small_log2n >= 0: the per-wavefront kernel with `waves` wavefronts for
// frames of at most 2^small_log2n leaves.
int occupancy(const polar_ctx* c, int cutover, int fk, bool dump, int waves, bool prune, int small_log2n = -1);
// Launch configuration of a group: explicit options first, then the tuned
// table, then defaults; force replaces both (autotuner).  Leaf-dump and
// unpruned groups always use cutover 12.  Workgroups are capped at what can
// be resident at once; frames of at most 2^cutover leaves are shared out
// fwg per workgroup.
LaunchCfg group_cfg(const polar_ctx* c, int fk, bool dump, const SizeHist& h, bool plain,
                    const LaunchCfg* force = nullptr, bool helpers = true);
// Slot bytes of one group under cfg: per workgroup (slots x largest frame)
// or per frame (sum over the frames above the cutover).
int64_t group_slot_bytes(const SizeHist& h, const LaunchCfg& cfg, bool per_frame, int64_t* per_wg);
// per_frame: every frame gets its own slot (serving); it also keeps the
// launches free of sweep helpers, so that batches can share the device.
void make_plan(const polar_ctx* c, const polar_frame* frames, int n_frames, bool plain, Plan& p,
               const LaunchCfg* force = nullptr, bool per_frame = false);
// Enqueue the decode of a planned batch on stream s using workspace ws;
// done: completion flags for descriptors with a done index (or null).
int run_plan(polar_ctx* c, const Plan& p, void* ws, size_t ws_bytes, hipStream_t s, Stager& st, bool plain,
             uint32_t* done = nullptr);
int decode_impl(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream, bool plain);
// Descriptors of a plan bound to a workspace (per-frame slot offsets become
// pointers); writes into out without reallocating when it has the capacity.
void bind_descs(const Plan& p, void* ws, std::vector<FrameDesc>& out);
int enqueue_launches(polar_ctx* c, const Plan& p, void* ws, hipStream_t s, bool plain, uint32_t* done);
// Sets up the allocation-free path for a new context (its device current).
int static_setup(polar_ctx* c);

}  // namespace polar_host
