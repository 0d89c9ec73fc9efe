// libpolar C ABI: argument validation, the host-side frozen-set builder,
// context / workspace management and kernel launches.  Device code lives in
// sc_device.hip.
#include "polar.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <numeric>
#include <string>
#include <vector>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "host_internal.h"
#include "sc_device.h"

using namespace polar_host;

namespace polar_host {

thread_local std::string g_err;

int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int ok() { return POLAR_OK; }

TraceRange::TraceRange(const char* name) { roctxRangePushA(name); }
TraceRange::~TraceRange() { roctxRangePop(); }

bool log_on() {
    static const bool on = [] {
        const char* v = std::getenv("POLAR_LOG");
        return v != nullptr && v[0] != 0 && !(v[0] == '0' && v[1] == 0);
    }();
    return on;
}

void log_line(const char* fmt, ...) {
    if (!log_on()) return;
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    std::fprintf(stderr, "[libpolar] %s\n", buf);
}

int hip_fail(hipError_t e, const char* what) {
    return fail(POLAR_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

DeviceGuard::DeviceGuard(int dev) {
    if (hipGetDevice(&prev) != hipSuccess) prev = -1;
    if (prev != dev) ok = hipSetDevice(dev) == hipSuccess;
}

DeviceGuard::~DeviceGuard() {
    int cur = -1;
    if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
}

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

namespace {
int64_t words_of(int log2n) { return log2n >= 5 ? ((int64_t)1 << (log2n - 5)) : 1; }
}  // namespace

}  // namespace polar_host

// ---------------------------------------------------------------------------
// Frozen set (Section 3): Bhattacharyya parameters of the synthetic channels,
// carried as (ln Z, ln(1 - Z)) so that Z does not saturate at 1 in double.
// ---------------------------------------------------------------------------
namespace {

// ln(1 - e^x) for x < 0 (Maechler's two-branch evaluation).
double ln_one_minus_exp(double x) { return x > -M_LN2 ? std::log(-std::expm1(x)) : std::log1p(-std::exp(x)); }

// In-place expansion: after step t, entries [0, 2^t) hold the channels of a
// length-2^t code; entry j spawns 2j (first-decoded, Z' = 2Z - Z^2) and
// 2j + 1 (Z' = Z^2).  Walking j downwards keeps the parents intact.
void bhattacharyya_pairs(int log2n, double z0, std::vector<double>& lz, std::vector<double>& lw) {
    const int64_t n = (int64_t)1 << log2n;
    lz.assign((size_t)n, 0.0);
    lw.assign((size_t)n, 0.0);
    lz[0] = std::log(z0);
    lw[0] = std::log1p(-z0);
    for (int t = 0; t < log2n; ++t) {
        const int64_t cnt = (int64_t)1 << t;
        for (int64_t j = cnt - 1; j >= 0; --j) {
            const double a = lz[(size_t)j], b = lw[(size_t)j];
            const bool z_small = std::exp(a) < 0.5;
            // 1 - Z^- = (1 - Z)^2 ;  Z^- = Z (2 - Z) = Z (1 + (1 - Z))
            const double wm = 2.0 * b;
            const double zm = z_small ? a + std::log1p(std::exp(b)) : ln_one_minus_exp(wm);
            // Z^+ = Z^2 ;  1 - Z^+ = (1 - Z)(1 + Z)
            const double zp = 2.0 * a;
            const double wp = std::exp(a) > 0.5 ? b + std::log1p(std::exp(a)) : ln_one_minus_exp(zp);
            lz[(size_t)(2 * j)] = zm;
            lw[(size_t)(2 * j)] = wm;
            lz[(size_t)(2 * j + 1)] = zp;
            lw[(size_t)(2 * j + 1)] = wp;
        }
    }
}

}  // namespace

extern "C" const char* polar_last_error(void) { return g_err.c_str(); }

extern "C" const char* polar_version(void) { return "libpolar 0.1 (gfx950)"; }

extern "C" int polar_build_frozen_set(int log2n, double z0, int64_t n_frozen, double fer_bound,
                                      uint32_t* frozen_mask, double* r_out, int64_t* n_frozen_out) {
    if (log2n < 1 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 1..%d", log2n, POLAR_MAX_LOG2N);
    if (!(z0 > 0.0 && z0 < 1.0)) return fail(POLAR_E_INVAL, "z0 must lie in (0, 1)");
    if (!frozen_mask) return fail(POLAR_E_INVAL, "frozen_mask is NULL");
    const int64_t n = (int64_t)1 << log2n;
    if (n_frozen > n || n_frozen < -1) return fail(POLAR_E_INVAL, "n_frozen %lld outside -1..N", (long long)n_frozen);
    if (n_frozen == -1 && !(fer_bound >= 0.0)) return fail(POLAR_E_INVAL, "fer_bound must be >= 0");

    std::vector<double> lz, lw;
    bhattacharyya_pairs(log2n, z0, lz, lw);
    std::vector<double> r((size_t)n);
    for (int64_t i = 0; i < n; ++i) r[(size_t)i] = lw[(size_t)i] - lz[(size_t)i];
    if (r_out) std::memcpy(r_out, r.data(), sizeof(double) * (size_t)n);

    // total order: ascending reliability, ties by index
    std::vector<int64_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), 0);
    auto less = [&](int64_t a, int64_t b) { return r[(size_t)a] < r[(size_t)b] || (r[(size_t)a] == r[(size_t)b] && a < b); };
    int64_t nf = n_frozen;
    if (nf == -1) {
        std::sort(idx.begin(), idx.end(), less);
        double sum = 0.0;
        int64_t k = 0;
        for (; k < n; ++k) {
            const double z = std::exp(lz[(size_t)idx[(size_t)(n - 1 - k)]]);
            if (sum + z > fer_bound) break;
            sum += z;
        }
        nf = n - k;
    } else if (nf > 0 && nf < n) {
        std::nth_element(idx.begin(), idx.begin() + nf, idx.end(), less);
    }
    const int64_t nw = log2n >= 5 ? ((int64_t)1 << (log2n - 5)) : 1;
    std::memset(frozen_mask, 0, sizeof(uint32_t) * (size_t)nw);
    for (int64_t t = 0; t < nf; ++t) {
        const int64_t i = idx[(size_t)t];
        frozen_mask[i >> 5] |= 1u << (i & 31);
    }
    if (n_frozen_out) *n_frozen_out = nf;
    return ok();
}

// ---------------------------------------------------------------------------
// Encoder.
// ---------------------------------------------------------------------------
extern "C" int polar_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, void* stream) {
    if (log2n < 0 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 0..%d", log2n, POLAR_MAX_LOG2N);
    if (n_frames < 0) return fail(POLAR_E_INVAL, "n_frames < 0");
    if (n_frames == 0) return ok();
    if (!u || !x) return fail(POLAR_E_INVAL, "NULL buffer");
    hipError_t e = polar_dev_encode(log2n, n_frames, u, x, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "encode launch");
    return ok();
}

// ---------------------------------------------------------------------------
// Batches: plan, descriptor upload, launches, optional graph replay.
// ---------------------------------------------------------------------------
namespace polar_host {

namespace {
constexpr size_t kHeaderBytes = 256;  // work counters
constexpr size_t kMaxGraphs = 16;
}  // namespace

int Stager::reserve(size_t n) {
    if (!ev) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (n <= cap) return ok();
    if (pending) {
        hipError_t e = hipEventSynchronize(ev);
        if (e != hipSuccess) return hip_fail(e, "descriptor staging");
        pending = false;
    }
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    hipError_t e = hipHostMalloc((void**)&buf, n * sizeof(FrameDesc), hipHostMallocDefault);
    if (e != hipSuccess) return hip_fail(e, "pinned descriptor buffer");
    cap = n;
    return ok();
}

int Stager::upload(const FrameDesc* d, size_t n, void* dst, hipStream_t s, bool may_grow) {
    if (n == 0) return ok();
    if (!may_grow && (n > cap || !ev))
        return fail(POLAR_E_INVAL, "%zu descriptors exceed the %zu reserved for this call", n, cap);
    if (!ev) {
        hipError_t e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        if (e != hipSuccess) return hip_fail(e, "hipEventCreate");
    }
    if (pending) {
        hipError_t e = hipEventSynchronize(ev);
        if (e != hipSuccess) return hip_fail(e, "descriptor staging");
        pending = false;
    }
    if (n > cap) {
        if (buf) (void)hipHostFree(buf);
        buf = nullptr;
        cap = 0;
        const size_t want = std::max(n, (size_t)1024);
        hipError_t e = hipHostMalloc((void**)&buf, want * sizeof(FrameDesc), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "pinned descriptor buffer");
        cap = want;
    }
    std::memcpy(buf, d, n * sizeof(FrameDesc));
    hipError_t e = hipMemcpyAsync(dst, buf, n * sizeof(FrameDesc), hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload");
    e = hipEventRecord(ev, s);
    if (e != hipSuccess) return hip_fail(e, "descriptor upload event");
    pending = true;
    return ok();
}

void Stager::release() {
    if (ev) {
        (void)hipEventSynchronize(ev);
        (void)hipEventDestroy(ev);
        ev = nullptr;
    }
    if (buf) (void)hipHostFree(buf);
    buf = nullptr;
    cap = 0;
    pending = false;
}

int validate_frames(const polar_frame* frames, int n_frames) {
    if (n_frames < 0) return fail(POLAR_E_INVAL, "n_frames < 0");
    if (n_frames > 0 && !frames) return fail(POLAR_E_INVAL, "frames is NULL");
    for (int i = 0; i < n_frames; ++i) {
        const polar_frame& f = frames[i];
        if (f.log2n < 1 || f.log2n > POLAR_MAX_LOG2N)
            return fail(POLAR_E_INVAL, "frame %d: log2n %d outside 1..%d", i, f.log2n, POLAR_MAX_LOG2N);
        if (f.f_kind < POLAR_F_MINSUM || f.f_kind > POLAR_F_MINSUM_Q8)
            return fail(POLAR_E_INVAL, "frame %d: unknown f_kind %d", i, f.f_kind);
        if (!f.llr || !f.frozen_mask || !f.frozen_vals || !f.u_hat)
            return fail(POLAR_E_INVAL, "frame %d: NULL buffer", i);
        if ((uintptr_t)f.llr & 15) return fail(POLAR_E_INVAL, "frame %d: llr must be 16-byte aligned", i);
        if (((uintptr_t)f.frozen_mask & 3) || ((uintptr_t)f.frozen_vals & 3) || ((uintptr_t)f.u_hat & 3) ||
            ((uintptr_t)f.leaf_llr & 3))
            return fail(POLAR_E_INVAL, "frame %d: bit vectors and leaf_llr must be 4-byte aligned", i);
    }
    return ok();
}

int occupancy(const polar_ctx* c, int cutover, int fk, bool dump, int waves, bool prune, int small_log2n) {
    // cache slot: cutover 8..12, f_kind 0..4, dump, prune, small_log2n -1..24, waves 1..8
    const int key = (((((cutover - 8) * 5 + fk) * 2 + (dump ? 1 : 0)) * 2 + (prune ? 1 : 0)) * 26 + small_log2n + 1) *
                        8 + (waves - 1);
    const bool cacheable = cutover >= 8 && cutover <= 12 && waves >= 1 && waves <= 8 && small_log2n >= -1 &&
                           small_log2n <= POLAR_MAX_LOG2N && key >= 0 && key < (int)c->occ_cache.size();
    if (cacheable && c->occ_cache[(size_t)key] > 0) return c->occ_cache[(size_t)key];
    DeviceGuard g(c->device);
    int occ = g.ok ? polar_dev_occupancy(cutover, fk, prune ? 1 : 0, dump ? 1 : 0, waves, small_log2n) : 0;
    occ = std::max(1, occ);
    if (cacheable) c->occ_cache[(size_t)key] = occ;
    return occ;
}

LaunchCfg group_cfg(const polar_ctx* c, int fk, bool dump, const SizeHist& h, bool plain, const LaunchCfg* force,
                    bool helpers) {
    LaunchCfg cfg;
    if (plain) {
        cfg.cutover = 12;
        cfg.waves = 4;
        cfg.slots = 1;
        cfg.fwg = 1;
        cfg.prune = 0;
        return cfg;
    }
    cfg.slots = 0;
    cfg.waves = 8;  // the level sweeps are bound by the bytes in flight per workgroup
    if (force) {
        cfg = *force;
    } else {
        auto it = c->tuned.find({fk, h.maxlog});
        if (it != c->tuned.end()) cfg = it->second;
        if (c->cutover) cfg.cutover = c->cutover;
        if (c->waves) cfg.waves = c->waves;
        if (c->max_slots) cfg.slots = c->max_slots;
        if (c->fwg) cfg.fwg = c->fwg;
    }
    // pruning switched off in the context wins over a tuned choice
    if (!c->prune) cfg.prune = 0;
    else if (cfg.prune < 0) cfg.prune = 1;
    if (dump || !cfg.prune) cfg.cutover = 12;
    // variants other than cutover 12 are built for the FP32 check updates only
    if (!polar_dev_variant_built(cfg.cutover, fk, cfg.prune, dump ? 1 : 0)) cfg.cutover = 12;
    // at most the workgroups that can be resident at once
    const int cap = c->n_cu * occupancy(c, cfg.cutover, fk, dump, cfg.waves, cfg.prune != 0);
    const int asked = cfg.slots;
    if (cfg.slots <= 0 || cfg.slots > cap) cfg.slots = cap;
    int n_small = 0, lg_small = 0;
    for (int l = 0; l <= std::min(cfg.cutover, (int)POLAR_MAX_LOG2N); ++l)
        if (h.n[l]) {
            n_small += h.n[l];
            lg_small = l;
        }
    const int n_big = h.count - n_small;
    cfg.slots = std::max(1, std::min(cfg.slots, n_big));
    // spare resident workgroups share the large frames' sweeps (not when the
    // caller limited the workgroups with POLAR_OPT_MAX_SLOTS)
    cfg.helpers = (helpers && c->helpers && n_big > 0 && c->max_slots <= 0) ? std::max(0, cap - cfg.slots) : 0;
    if (!n_small) {
        cfg.fwg = 1;
        cfg.small_slots = 1;
        return cfg;
    }
    // small frames: fwg wavefronts (one frame each) per workgroup; the
    // default holds the most frames in flight (resident workgroups x fwg,
    // up to the frames there are), the smallest such fwg on ties
    const int f_max = std::max(1, polar_dev_max_fwg(cfg.cutover, lg_small, cfg.waves));
    auto small_cap = [&](int fw) {
        int sc = c->n_cu * occupancy(c, cfg.cutover, fk, dump, fw, cfg.prune != 0, lg_small);
        return std::max(1, asked > 0 ? std::min(sc, asked) : sc);
    };
    if (cfg.fwg <= 0) {
        cfg.fwg = 1;
        int64_t best = 0;
        for (int fw = 1; fw <= f_max; ++fw) {
            const int64_t inflight = std::min<int64_t>((int64_t)small_cap(fw) * fw, n_small);
            if (inflight > best) {
                best = inflight;
                cfg.fwg = fw;
            }
        }
    }
    cfg.fwg = std::max(1, std::min(cfg.fwg, f_max));
    cfg.small_slots = std::max(1, std::min(small_cap(cfg.fwg), (n_small + cfg.fwg - 1) / cfg.fwg));
    return cfg;
}

int64_t group_slot_bytes(const SizeHist& h, const LaunchCfg& cfg, bool per_frame, int64_t* per_wg) {
    int64_t sum = 0, big = 0;
    for (int l = cfg.cutover + 1; l <= POLAR_MAX_LOG2N; ++l)
        if (h.n[l]) {
            const int64_t b = polar_dev_slot_bytes(l, cfg.cutover);
            sum += b * h.n[l];
            big = std::max(big, b);
        }
    if (per_wg) *per_wg = big;
    return per_frame ? sum : big * cfg.slots;
}

void make_plan(const polar_ctx* c, const polar_frame* frames, int n_frames, bool plain, Plan& p,
               const LaunchCfg* force, bool per_frame) {
    // order: by (f_kind, leaf dump), inside a group most work (largest N)
    // first, ties in submission order: a stable counting sort over the
    // kGroupKeys x 25 keys (no allocation once the plan's vectors have the
    // capacity)
    constexpr int NL = POLAR_MAX_LOG2N + 1;
    auto key = [&](int i) { return frames[i].f_kind * 2 + (frames[i].leaf_llr ? 1 : 0); };
    auto bucket = [&](int i) { return key(i) * NL + (POLAR_MAX_LOG2N - frames[i].log2n); };
    int start[kGroupKeys * NL + 1] = {};
    for (int i = 0; i < n_frames; ++i) ++start[bucket(i) + 1];
    for (int b = 0; b < kGroupKeys * NL; ++b) start[b + 1] += start[b];
    std::vector<int>& order = p.order;
    order.resize((size_t)n_frames);
    for (int i = 0; i < n_frames; ++i) order[(size_t)start[bucket(i)]++] = i;
    p.descs.clear();
    p.groups.clear();
    p.per_frame = per_frame && !plain;
    for (int k = 0; k < n_frames; ++k) {
        const polar_frame& f = frames[order[(size_t)k]];
        FrameDesc d{};
        d.llr = f.llr;
        d.mask = f.frozen_mask;
        d.vals = f.frozen_vals;
        d.uhat = f.u_hat;
        d.leaf = f.leaf_llr;
        d.log2n = f.log2n;
        d.fkind = f.f_kind;
        d.slot = nullptr;
        d.done_idx = 0xffffffffu;
        d.done_val = 0;
        p.descs.push_back(d);
        if (p.groups.empty() || key(order[(size_t)k]) != p.groups.back().fk * 2 + p.groups.back().dump)
            p.groups.push_back({f.f_kind, f.leaf_llr ? 1 : 0, k, 0, (int)f.log2n, SizeHist{}, LaunchCfg{}});
        p.groups.back().count++;
        p.groups.back().hist.add(f.log2n);
    }
    p.slots = 0;
    p.slot_bytes = 0;
    int64_t frame_bytes = 0;  // per-frame slots: running offset
    for (auto& g : p.groups) {
        g.cfg = group_cfg(c, g.fk, g.dump != 0, g.hist, plain, force, !p.per_frame);
        int64_t per_wg = 0;
        (void)group_slot_bytes(g.hist, g.cfg, p.per_frame, &per_wg);
        p.slots = std::max(p.slots, g.cfg.slots);
        p.slot_bytes = std::max(p.slot_bytes, per_wg);
        if (p.per_frame)
            for (int k = g.first; k < g.first + g.count; ++k)
                if (p.descs[(size_t)k].log2n > g.cfg.cutover) {
                    p.descs[(size_t)k].slot = reinterpret_cast<uint8_t*>((uintptr_t)frame_bytes);
                    frame_bytes += polar_dev_slot_bytes(p.descs[(size_t)k].log2n, g.cfg.cutover);
                }
    }
    p.boxes = 0;
    for (const auto& g : p.groups)
        if (g.cfg.helpers > 0) p.boxes = std::max(p.boxes, g.cfg.slots);
    p.desc_off = kHeaderBytes;
    p.box_off = align256(p.desc_off + sizeof(FrameDesc) * (size_t)n_frames);
    p.slot_off = align256(p.box_off + sizeof(SweepBox) * (size_t)p.boxes);
    p.total = p.slot_off + (p.per_frame ? (size_t)frame_bytes : (size_t)p.slots * (size_t)p.slot_bytes);
}

// Descriptors of a plan bound to a workspace: per-frame slot offsets become
// device pointers.
void bind_descs(const Plan& p, void* ws, std::vector<FrameDesc>& out) {
    out.assign(p.descs.begin(), p.descs.end());
    if (!p.per_frame) return;
    uint8_t* slots = (uint8_t*)ws + p.slot_off;
    for (const auto& g : p.groups)
        for (int k = g.first; k < g.first + g.count; ++k)
            if (out[(size_t)k].log2n > g.cfg.cutover) out[(size_t)k].slot = slots + (uintptr_t)out[(size_t)k].slot;
}

int enqueue_launches(polar_ctx* c, const Plan& p, void* ws, hipStream_t s, bool plain, uint32_t* done) {
    uint8_t* base = (uint8_t*)ws;
    unsigned* counter = (unsigned*)base;
    const FrameDesc* dtab = (const FrameDesc*)(base + p.desc_off);
    uint8_t* slots = base + p.slot_off;
    SweepBox* boxes = p.boxes > 0 ? reinterpret_cast<SweepBox*>(base + p.box_off) : nullptr;
    for (const auto& gr : p.groups) {
        DecodeLaunch a{};
        a.cutover = gr.cfg.cutover;
        a.fk = gr.fk;
        a.prune = plain ? 0 : gr.cfg.prune;
        a.dump = gr.dump;
        a.waves = gr.cfg.waves;
        a.counter = counter;
        a.slots = slots;
        a.slot_bytes = p.slot_bytes;
        a.prof = c->prof;
        a.done = done;
        a.stream = s;
        // frames above the cutover come first (longest first); the rest go
        // to the per-wavefront kernel
        int n_big = 0;
        while (n_big < gr.count && p.descs[(size_t)(gr.first + n_big)].log2n > gr.cfg.cutover) ++n_big;
        if (plain) {
            for (int k = 0; k < gr.count; ++k) {
                a.descs = dtab + gr.first + k;
                a.n_frames = 1;
                a.grid = 1;
                a.small = k >= n_big;
                a.small_log2n = p.descs[(size_t)(gr.first + k)].log2n;
                a.fwg = 1;
                hipError_t e = polar_dev_launch_decode(&a);
                if (e != hipSuccess) return hip_fail(e, "decode launch");
            }
            continue;
        }
        if (n_big > 0) {
            a.descs = dtab + gr.first;
            a.n_frames = n_big;
            a.grid = gr.cfg.slots;
            a.small = 0;
            a.helpers = boxes ? gr.cfg.helpers : 0;
            a.boxes = boxes;
            hipError_t e = polar_dev_launch_decode(&a);
            if (e != hipSuccess) return hip_fail(e, "decode launch");
        }
        if (n_big < gr.count) {
            a.descs = dtab + gr.first + n_big;
            a.n_frames = gr.count - n_big;
            a.grid = gr.cfg.small_slots;
            a.small = 1;
            a.small_log2n = p.descs[(size_t)(gr.first + n_big)].log2n;
            a.fwg = gr.cfg.fwg;
            hipError_t e = polar_dev_launch_decode(&a);
            if (e != hipSuccess) return hip_fail(e, "decode launch (per-wavefront frames)");
        }
    }
    return ok();
}

namespace {

uint64_t fnv1a(const std::vector<uint8_t>& v) {
    uint64_t h = 1469598103934665603ull;
    for (uint8_t b : v) h = (h ^ b) * 1099511628211ull;
    return h;
}

template <class T>
void put(std::vector<uint8_t>& v, const T& x) {
    const uint8_t* p = reinterpret_cast<const uint8_t*>(&x);
    v.insert(v.end(), p, p + sizeof(T));
}

// Replays the batch through a cached graph: [descriptor copy, counter reset,
// decode launch] per group, captured once for these exact descriptors,
// launch parameters and workspace.
int run_graph(polar_ctx* c, const Plan& p, void* ws, hipStream_t s) {
    std::vector<FrameDesc> descs;
    bind_descs(p, ws, descs);
    std::vector<uint8_t> key;
    put(key, ws);
    put(key, c->prof);
    for (const auto& g : p.groups) {
        put(key, g.cfg.prune);
        put(key, g.first);
        put(key, g.count);
        put(key, g.cfg.cutover);
        put(key, g.cfg.waves);
        put(key, g.cfg.slots);
        put(key, g.cfg.fwg);
    }
    put(key, p.slot_bytes);
    const uint8_t* d = reinterpret_cast<const uint8_t*>(descs.data());
    key.insert(key.end(), d, d + descs.size() * sizeof(FrameDesc));
    const uint64_t h = fnv1a(key);
    auto it = c->graphs.find(h);
    if (it != c->graphs.end() && it->second.key != key) {
        // hash collision: drop the old entry, which may still be running
        hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return hip_fail(e, "graph cache collision");
        (void)hipGraphExecDestroy(it->second.exec);
        (void)hipHostFree(it->second.pinned);
        c->graphs.erase(it);
        it = c->graphs.end();
    }
    if (it == c->graphs.end()) {
        if (c->graphs.size() >= kMaxGraphs) {
            auto victim = c->graphs.begin();
            for (auto j = c->graphs.begin(); j != c->graphs.end(); ++j)
                if (j->second.last_use < victim->second.last_use) victim = j;
            // the victim may still be running on some stream
            hipError_t e = hipDeviceSynchronize();
            if (e != hipSuccess) return hip_fail(e, "graph cache eviction");
            (void)hipGraphExecDestroy(victim->second.exec);
            (void)hipHostFree(victim->second.pinned);
            c->graphs.erase(victim);
        }
        if (!c->capture_stream) {
            hipError_t e = hipStreamCreateWithFlags(&c->capture_stream, hipStreamNonBlocking);
            if (e != hipSuccess) return hip_fail(e, "capture stream");
        }
        GraphEntry ge;
        ge.key = key;
        const size_t nb = descs.size() * sizeof(FrameDesc);
        hipError_t e = hipHostMalloc((void**)&ge.pinned, std::max(nb, (size_t)64), hipHostMallocDefault);
        if (e != hipSuccess) return hip_fail(e, "pinned graph descriptors");
        std::memcpy(ge.pinned, descs.data(), nb);
        hipStream_t cs = c->capture_stream;
        e = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
        if (e != hipSuccess) {
            (void)hipHostFree(ge.pinned);
            return hip_fail(e, "begin graph capture");
        }
        e = hipMemcpyAsync((uint8_t*)ws + p.desc_off, ge.pinned, nb, hipMemcpyHostToDevice, cs);
        int rc = e == hipSuccess ? enqueue_launches(c, p, ws, cs, false, nullptr) : hip_fail(e, "captured copy");
        hipGraph_t graph = nullptr;
        hipError_t e2 = hipStreamEndCapture(cs, &graph);
        if (rc == POLAR_OK && e2 != hipSuccess) rc = hip_fail(e2, "end graph capture");
        if (rc == POLAR_OK) {
            e = hipGraphInstantiate(&ge.exec, graph, nullptr, nullptr, 0);
            if (e != hipSuccess) rc = hip_fail(e, "graph instantiate");
        }
        if (graph) (void)hipGraphDestroy(graph);
        if (rc != POLAR_OK) {
            (void)hipHostFree(ge.pinned);
            return rc;
        }
        it = c->graphs.emplace(h, std::move(ge)).first;
    }
    it->second.last_use = ++c->graph_clock;
    hipError_t e = hipGraphLaunch(it->second.exec, s);
    if (e != hipSuccess) return hip_fail(e, "graph launch");
    return ok();
}

}  // namespace

int run_plan(polar_ctx* c, const Plan& p, void* ws, size_t ws_bytes, hipStream_t s, Stager& st, bool plain,
             uint32_t* done) {
    if (!ws || ws_bytes < p.total)
        return fail(POLAR_E_NOMEM, "workspace of %zu bytes < %zu required", ws ? ws_bytes : (size_t)0, p.total);
    if (((uintptr_t)ws & 255) != 0) return fail(POLAR_E_INVAL, "workspace must be 256-byte aligned");
    std::vector<FrameDesc> descs;
    bind_descs(p, ws, descs);
    int rc = st.upload(descs.data(), descs.size(), (uint8_t*)ws + p.desc_off, s);
    if (rc) return rc;
    return enqueue_launches(c, p, ws, s, plain, done);
}

int decode_impl(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream, bool plain) {
    TraceRange tr(plain ? "polar_sc_decode_plain" : "polar_sc_decode_batch");
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    int rc = validate_frames(frames, n_frames);
    if (rc) return rc;
    if (n_frames == 0) return ok();
    Plan p;
    make_plan(c, frames, n_frames, plain, p);
    if (log_on())
        for (const auto& g : p.groups)
            log_line("decode: f_kind %d dump %d, %d frames (largest 2^%d): cutover %d, %d waves, %d slots + %d "
                     "helpers, %d frames per small workgroup, prune %d; workspace %zu bytes",
                     g.fk, g.dump, g.count, g.hist.maxlog, g.cfg.cutover, g.cfg.waves, g.cfg.slots, g.cfg.helpers,
                     g.cfg.fwg, g.cfg.prune, p.total);
    if (!c->ws || c->ws_bytes < p.total)
        return fail(POLAR_E_NOMEM, "workspace of %zu bytes < %zu required", c->ws_bytes, p.total);
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    if (c->graph && !plain) return run_graph(c, p, c->ws, s);
    return run_plan(c, p, c->ws, c->ws_bytes, s, c->stager, plain);
}

}  // namespace polar_host

extern "C" int polar_ctx_create(polar_ctx** out, int device, void* workspace, size_t ws_bytes) {
    if (!out) return fail(POLAR_E_INVAL, "out is NULL");
    *out = nullptr;
    int ndev = 0;
    hipError_t e = hipGetDeviceCount(&ndev);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceCount");
    if (device < 0 || device >= ndev) return fail(POLAR_E_INVAL, "device %d outside 0..%d", device, ndev - 1);
    DeviceGuard g(device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", device);
    polar_ctx* c = new polar_ctx();
    c->device = device;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess && prop.multiProcessorCount > 0)
        c->n_cu = prop.multiProcessorCount;
    c->ws = workspace;
    c->ws_bytes = workspace ? ws_bytes : 0;
    const int rc = static_setup(c);
    if (rc) {
        c->static_stager.release();
        delete c;
        return rc;
    }
    *out = c;
    return ok();
}

extern "C" int polar_ctx_destroy(polar_ctx* c) {
    if (!c) return ok();
    {
        DeviceGuard g(c->device);
        c->stager.release();
        c->static_stager.release();
        if (!c->graphs.empty()) (void)hipDeviceSynchronize();
        for (auto& kv : c->graphs) {
            (void)hipGraphExecDestroy(kv.second.exec);
            (void)hipHostFree(kv.second.pinned);
        }
        c->graphs.clear();
        if (c->capture_stream) (void)hipStreamDestroy(c->capture_stream);
    }
    delete c;
    return ok();
}

extern "C" int polar_ctx_set_workspace(polar_ctx* c, void* workspace, size_t ws_bytes) {
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    if (((uintptr_t)workspace & 255) != 0) return fail(POLAR_E_INVAL, "workspace must be 256-byte aligned");
    c->ws = workspace;
    c->ws_bytes = workspace ? ws_bytes : 0;
    return ok();
}

extern "C" int polar_ctx_set_option(polar_ctx* c, int option, int64_t value) {
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    switch (option) {
        case POLAR_OPT_PRUNE:
            if (value != 0 && value != 1) return fail(POLAR_E_INVAL, "prune must be 0 or 1");
            c->prune = (int)value;
            return ok();
        case POLAR_OPT_CUTOVER:
            if (value != 0 && !polar_dev_cutover_supported((int)value))
                return fail(POLAR_E_INVAL, "cutover %lld not built", (long long)value);
            c->cutover = (int)value;
            return ok();
        case POLAR_OPT_WG_WAVES:
            if (value != 0 && !polar_dev_waves_supported((int)value))
                return fail(POLAR_E_INVAL, "waves per workgroup %lld not built", (long long)value);
            c->waves = (int)value;
            return ok();
        case POLAR_OPT_MAX_SLOTS:
            if (value < 0 || value > (1 << 20)) return fail(POLAR_E_INVAL, "max_slots out of range");
            c->max_slots = (int)value;
            return ok();
        case POLAR_OPT_TIMING:
            if (value & 7) return fail(POLAR_E_INVAL, "timing buffer must be 8-byte aligned");
            c->prof = reinterpret_cast<unsigned long long*>((uintptr_t)value);
            return ok();
        case POLAR_OPT_GRAPH:
            if (value != 0 && value != 1) return fail(POLAR_E_INVAL, "graph must be 0 or 1");
            c->graph = (int)value;
            return ok();
        case POLAR_OPT_FWG:
            if (value < 0 || value > 8) return fail(POLAR_E_INVAL, "frames per workgroup must be 0 .. 8");
            c->fwg = (int)value;
            return ok();
        case POLAR_OPT_HELPERS:
            if (value != 0 && value != 1) return fail(POLAR_E_INVAL, "helpers must be 0 or 1");
            c->helpers = (int)value;
            return ok();
        default:
            return fail(POLAR_E_INVAL, "unknown option %d", option);
    }
}

extern "C" int polar_ctx_get_option(polar_ctx* c, int option, int64_t* value) {
    if (!c || !value) return fail(POLAR_E_INVAL, "NULL argument");
    switch (option) {
        case POLAR_OPT_PRUNE: *value = c->prune; return ok();
        case POLAR_OPT_CUTOVER: *value = c->cutover; return ok();
        case POLAR_OPT_WG_WAVES: *value = c->waves; return ok();
        case POLAR_OPT_MAX_SLOTS: *value = c->max_slots; return ok();
        case POLAR_OPT_TIMING: *value = (int64_t)(uintptr_t)c->prof; return ok();
        case POLAR_OPT_GRAPH: *value = c->graph; return ok();
        case POLAR_OPT_FWG: *value = c->fwg; return ok();
        case POLAR_OPT_HELPERS: *value = c->helpers; return ok();
        default: return fail(POLAR_E_INVAL, "unknown option %d", option);
    }
}

extern "C" size_t polar_workspace_bytes(const polar_ctx* c, const polar_frame* frames, int n_frames) {
    if (!c || n_frames < 0 || (n_frames > 0 && !frames)) return 0;
    for (int i = 0; i < n_frames; ++i)
        if (frames[i].log2n < 1 || frames[i].log2n > POLAR_MAX_LOG2N) return 0;
    Plan p;
    make_plan(c, frames, n_frames, false, p);
    Plan q;
    make_plan(c, frames, n_frames, true, q);
    return std::max(p.total, q.total);
}

extern "C" int polar_sc_decode_batch(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream) {
    return decode_impl(c, frames, n_frames, stream, false);
}

extern "C" int polar_sc_decode_plain(polar_ctx* c, const polar_frame* frames, int n_frames, void* stream) {
    return decode_impl(c, frames, n_frames, stream, true);
}

extern "C" int polar_debug_phi_table(float* out, void* stream) {
    if (!out) return fail(POLAR_E_INVAL, "out is NULL");
    hipError_t e = polar_dev_phi_table(out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "phi table launch");
    return ok();
}

extern "C" int polar_debug_lane_selftest(uint32_t* out, void* stream) {
    if (!out) return fail(POLAR_E_INVAL, "out is NULL");
    hipError_t e = polar_dev_lane_selftest(out, (hipStream_t)stream);
    if (e != hipSuccess) return hip_fail(e, "selftest launch");
    return ok();
}
