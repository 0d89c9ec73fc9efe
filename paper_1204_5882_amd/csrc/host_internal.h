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
    int slots = 0;  // workgroups (frames in flight)
};

// A pinned host buffer for descriptor uploads; the event guards its reuse.
struct Stager {
    FrameDesc* buf = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool pending = false;
    int upload(const FrameDesc* d, size_t n, void* dst, hipStream_t s);
    void release();
};

// Frames grouped per launch (same f_kind and leaf-dump flag), longest first,
// and the workspace layout [counters | descriptors | slots].
struct Plan {
    std::vector<FrameDesc> descs;
    struct Group {
        int fk, dump, first, count, maxlog;
        LaunchCfg cfg;
    };
    std::vector<Group> groups;
    int slots = 0;
    int64_t slot_bytes = 0;
    size_t desc_off = 0, slot_off = 0, total = 0;
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
    int graph = 0;      // replay batches through cached HIP graphs
    unsigned long long* prof = nullptr;  // optional device timing counters
    polar_host::Stager stager;
    // autotuned launch configurations, key (f_kind, log2n of the largest frame)
    std::map<std::pair<int, int>, polar_host::LaunchCfg> tuned;
    // graph cache
    std::unordered_map<uint64_t, polar_host::GraphEntry> graphs;
    uint64_t graph_clock = 0;
    hipStream_t capture_stream = nullptr;
};

namespace polar_host {

int validate_frames(const polar_frame* frames, int n_frames);
// Launch configuration of a group: explicit options first, then the tuned
// table, then defaults.  Leaf-dump and unpruned groups always use cutover 12.
LaunchCfg group_cfg(const polar_ctx* c, int fk, int maxlog, int count, bool dump, bool plain);
void make_plan(const polar_ctx* c, const polar_frame* frames, int n_frames, bool plain, Plan& p,
               const LaunchCfg* force = nullptr);
// Enqueue the decode of a planned batch on stream s using workspace ws.
int run_plan(polar_ctx* c, const Plan& p, void* ws, size_t ws_bytes, hipStream_t s, Stager& st, bool plain);
int decode_impl(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream, bool plain);

}  // namespace polar_host
