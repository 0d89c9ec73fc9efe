// libpolar autotuner: picks the launch configuration (register-resident
// subtree size, wavefronts per workgroup, frames in flight) per
// (f_kind, log2 N of the largest frame) by timing the built variants on the
// caller's frames, and keeps the table in the context (saved / loaded as
// JSON).  Every configuration decodes to identical results; only speed
// differs.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "host_internal.h"
#include "polar.h"

using namespace polar_host;

namespace {

struct Candidate {
    LaunchCfg cfg;
    double median_ms = 0.0;
};

int time_candidate(polar_ctx* c, const polar_frame* frames, int n_frames, const LaunchCfg& cfg, int reps,
                   hipStream_t s, double* median_ms) {
    Plan p;
    make_plan(c, frames, n_frames, false, p, &cfg);
    if (!c->ws || c->ws_bytes < p.total) return POLAR_E_NOMEM;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    if (e != hipSuccess) {
        if (e0) (void)hipEventDestroy(e0);
        return hip_fail(e, "tuner events");
    }
    std::vector<double> ms;
    int rc = POLAR_OK;
    // one untimed run, then reps timed runs
    for (int r = -1; r < reps && rc == POLAR_OK; ++r) {
        e = hipEventRecord(e0, s);
        if (e != hipSuccess) { rc = hip_fail(e, "tuner event"); break; }
        rc = run_plan(c, p, c->ws, c->ws_bytes, s, c->stager, false);
        if (rc) break;
        e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        if (e != hipSuccess) { rc = hip_fail(e, "tuner run"); break; }
        float t = 0.0f;
        e = hipEventElapsedTime(&t, e0, e1);
        if (e != hipSuccess) { rc = hip_fail(e, "tuner timing"); break; }
        if (r >= 0) ms.push_back(t);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (rc) return rc;
    std::sort(ms.begin(), ms.end());
    *median_ms = ms[ms.size() / 2];
    return POLAR_OK;
}

}  // namespace

extern "C" int polar_autotune(polar_ctx* c, const polar_frame* frames, int n_frames, int reps, void* stream,
                              int* best_cutover, int* best_waves, int* best_slots, int* best_fwg, int* best_prune,
                              double* best_ms, int* n_candidates) {
    TraceRange tr("polar_autotune");
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    int rc = validate_frames(frames, n_frames);
    if (rc) return rc;
    if (n_frames < 1) return fail(POLAR_E_INVAL, "autotune needs at least one frame");
    if (reps < 1 || reps > 1000) return fail(POLAR_E_INVAL, "reps must be in 1..1000");
    const int fk = frames[0].f_kind;
    int maxlog = 0;
    for (int i = 0; i < n_frames; ++i) {
        if (frames[i].f_kind != fk) return fail(POLAR_E_INVAL, "autotune frames must share one f_kind");
        if (frames[i].leaf_llr) return fail(POLAR_E_INVAL, "autotune frames must not request leaf LLRs");
        maxlog = std::max(maxlog, (int)frames[i].log2n);
    }
    if (!c->prune) return fail(POLAR_E_INVAL, "autotune applies to the pruned decoder");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;

    SizeHist hist;
    for (int i = 0; i < n_frames; ++i) hist.add(frames[i].log2n);
    std::vector<LaunchCfg> grid;
    auto push = [&](const LaunchCfg& cfg) {
        for (const auto& q : grid)
            if (q.cutover == cfg.cutover && q.waves == cfg.waves && q.slots == cfg.slots && q.fwg == cfg.fwg &&
                q.prune == cfg.prune)
                return;
        grid.push_back(cfg);
    };
    for (int cut = 8; cut <= 12; ++cut) {
        if (!polar_dev_cutover_supported(cut) || !polar_dev_variant_built(cut, fk, 1, 0)) continue;
        int lg_small = 0, n_small = 0;
        for (int l = 1; l <= cut; ++l)
            if (hist.n[l]) {
                lg_small = l;
                n_small += hist.n[l];
            }
        for (int w : {4, 8}) {
            if (!polar_dev_waves_supported(w)) continue;
            const int cap = c->n_cu * occupancy(c, cut, fk, false, w, true);
            const int f_max = n_small ? polar_dev_max_fwg(cut, lg_small, w) : 1;
            for (int sl : {c->n_cu / 2, c->n_cu, cap}) {
                if (sl < 1 || sl > cap) continue;
                for (int fw : {1, 2, 4, 8}) {
                    if (fw > f_max) continue;
                    LaunchCfg cfg;
                    cfg.cutover = cut;
                    cfg.waves = w;
                    cfg.slots = sl;
                    cfg.fwg = fw;
                    cfg.prune = 1;
                    push(cfg);
                }
            }
        }
    }
    {  // the unpruned decoder (same results, every node visited)
        LaunchCfg cfg;
        cfg.cutover = 12;
        cfg.waves = 8;
        cfg.slots = c->n_cu * occupancy(c, 12, fk, false, 8, false);
        cfg.fwg = 1;
        cfg.prune = 0;
        push(cfg);
    }
    Candidate best;
    bool have = false;
    for (const auto& cfg : grid) {
        double ms = 0.0;
        rc = time_candidate(c, frames, n_frames, cfg, reps, s, &ms);
        if (rc == POLAR_E_NOMEM) continue;  // does not fit the workspace
        if (rc) return rc;
        if (!have || ms < best.median_ms) {
            best.cfg = cfg;
            best.median_ms = ms;
            have = true;
        }
    }
    if (!have) return fail(POLAR_E_NOMEM, "no candidate configuration fits the workspace");
    c->tuned[{fk, maxlog}] = best.cfg;
    // what a batch of these frames now runs with (workgroups capped by the batch)
    const LaunchCfg used = group_cfg(c, fk, false, hist, false, &best.cfg);
    if (best_cutover) *best_cutover = used.cutover;
    if (best_waves) *best_waves = used.waves;
    if (best_slots) *best_slots = used.slots;
    if (best_fwg) *best_fwg = used.fwg;
    if (best_prune) *best_prune = used.prune;
    if (best_ms) *best_ms = best.median_ms;
    if (n_candidates) *n_candidates = (int)grid.size();
    return ok();
}

extern "C" int polar_query_launch(const polar_ctx* c, int f_kind, int log2n, int n_frames, int* cutover,
                                  int* waves, int* slots, int* fwg, int* prune) {
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    if (log2n < 1 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 1..%d", log2n, POLAR_MAX_LOG2N);
    if (f_kind < POLAR_F_MINSUM || f_kind > POLAR_F_MINSUM_Q8) return fail(POLAR_E_INVAL, "unknown f_kind");
    if (n_frames < 1) return fail(POLAR_E_INVAL, "n_frames < 1");
    SizeHist h;
    for (int i = 0; i < n_frames; ++i) h.add(log2n);
    const LaunchCfg cfg = group_cfg(c, f_kind, false, h, false);
    if (cutover) *cutover = cfg.cutover;
    if (waves) *waves = cfg.waves;
    if (slots) *slots = cfg.slots;
    if (fwg) *fwg = cfg.fwg;
    if (prune) *prune = cfg.prune;
    return ok();
}

extern "C" int polar_tune_clear(polar_ctx* c) {
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    c->tuned.clear();
    return ok();
}

extern "C" int polar_tune_save(const polar_ctx* c, const char* path) {
    if (!c || !path) return fail(POLAR_E_INVAL, "NULL argument");
    FILE* f = std::fopen(path, "w");
    if (!f) return fail(POLAR_E_INVAL, "cannot write %s", path);
    std::fprintf(f, "{\"libpolar_tune\": 1, \"entries\": [");
    bool first = true;
    for (const auto& kv : c->tuned) {
        std::fprintf(f,
                     "%s\n  {\"f_kind\": %d, \"log2n\": %d, \"cutover\": %d, \"waves\": %d, \"slots\": %d, "
                     "\"fwg\": %d, \"prune\": %d}",
                     first ? "" : ",", kv.first.first, kv.first.second, kv.second.cutover, kv.second.waves,
                     kv.second.slots, kv.second.fwg, kv.second.prune);
        first = false;
    }
    std::fprintf(f, "\n]}\n");
    const bool bad = std::ferror(f) != 0;
    if (std::fclose(f) != 0 || bad) return fail(POLAR_E_INVAL, "write error on %s", path);
    return ok();
}

namespace {

// Reads the integer after "key": inside [p, end).
bool read_int(const std::string& obj, const char* key, long* out) {
    const std::string k = std::string("\"") + key + "\"";
    size_t i = obj.find(k);
    if (i == std::string::npos) return false;
    i = obj.find(':', i + k.size());
    if (i == std::string::npos) return false;
    char* endp = nullptr;
    const long v = std::strtol(obj.c_str() + i + 1, &endp, 10);
    if (endp == obj.c_str() + i + 1) return false;
    *out = v;
    return true;
}

}  // namespace

extern "C" int polar_tune_load(polar_ctx* c, const char* path) {
    if (!c || !path) return fail(POLAR_E_INVAL, "NULL argument");
    FILE* f = std::fopen(path, "r");
    if (!f) return fail(POLAR_E_INVAL, "cannot read %s", path);
    std::string text;
    char buf[4096];
    size_t n;
    while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
    std::fclose(f);
    if (text.find("\"libpolar_tune\"") == std::string::npos) return fail(POLAR_E_INVAL, "%s: not a tune file", path);
    std::map<std::pair<int, int>, LaunchCfg> table;
    size_t pos = text.find('[');
    while (pos != std::string::npos) {
        const size_t a = text.find('{', pos);
        if (a == std::string::npos) break;
        const size_t b = text.find('}', a);
        if (b == std::string::npos) return fail(POLAR_E_INVAL, "%s: unterminated entry", path);
        const std::string obj = text.substr(a, b - a + 1);
        long fk, lg, cut, w, sl, fw = 0, pr = -1;
        if (!read_int(obj, "f_kind", &fk) || !read_int(obj, "log2n", &lg) || !read_int(obj, "cutover", &cut) ||
            !read_int(obj, "waves", &w) || !read_int(obj, "slots", &sl))
            return fail(POLAR_E_INVAL, "%s: entry lacks a field", path);
        (void)read_int(obj, "fwg", &fw);    // optional
        (void)read_int(obj, "prune", &pr);  // optional
        if (fk < POLAR_F_MINSUM || fk > POLAR_F_MINSUM_Q8 || lg < 1 || lg > POLAR_MAX_LOG2N ||
            !polar_dev_cutover_supported((int)cut) || !polar_dev_waves_supported((int)w) || sl < 1 ||
            sl > (1 << 20) || fw < 0 || fw > w || pr < -1 || pr > 1 || (pr == 0 && cut != 12))
            return fail(POLAR_E_INVAL, "%s: entry out of range", path);
        LaunchCfg cfg;
        cfg.cutover = (int)cut;
        cfg.waves = (int)w;
        cfg.slots = (int)sl;
        cfg.fwg = (int)fw;
        cfg.prune = (int)pr;
        table[{(int)fk, (int)lg}] = cfg;
        pos = b + 1;
    }
    for (const auto& kv : table) c->tuned[kv.first] = kv.second;
    return ok();
}
