// The library's host code (plans, frozen-set builders, argument checks, the
// tune-file parser) under AddressSanitizer and UndefinedBehaviorSanitizer, on
// a machine without a GPU.  The device layer is replaced by stubs that answer
// what the host code asks of it (which variants exist, slot sizes) and fail
// every launch; device queries fail on their own (no device).  Prints "ok"
// when every check passes; a sanitizer report aborts first.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <random>
#include <string>
#include <vector>

#include "host_internal.h"

// ---------------------------------------------------------------------------
// Device-layer stubs.
// ---------------------------------------------------------------------------
extern "C" {
int polar_dev_cutover_supported(int c) { return c >= 8 && c <= 12; }
int polar_dev_waves_supported(int w) { return w == 4 || w == 8; }
int polar_dev_variant_built(int cutover, int fk, int prune, int dump) {
    if (fk < 0 || fk > 4 || cutover < 8 || cutover > 12) return 0;
    if (cutover == 12) return 1;
    return (fk == 0 || fk == 1) && prune && !dump;
}
int polar_dev_max_fwg(int cutover, int log2n, int waves) { return log2n > cutover ? 1 : waves; }
int polar_dev_occupancy(int, int, int, int, int, int) { return 1; }
int64_t polar_dev_slot_bytes(int log2n, int cutover) {
    return log2n > cutover ? ((int64_t)8 << log2n) + 4096 : 0;
}
hipError_t polar_dev_launch_decode(const DecodeLaunch*) { return hipErrorNoDevice; }
hipError_t polar_dev_encode(int, int, const uint32_t*, uint32_t*, hipStream_t) { return hipErrorNoDevice; }
hipError_t polar_dev_phi_table(float*, hipStream_t) { return hipErrorNoDevice; }
hipError_t polar_dev_lane_selftest(uint32_t*, hipStream_t) { return hipErrorNoDevice; }
}
namespace polar_host {
int static_setup(polar_ctx*) { return fail(POLAR_E_DEVICE, "no device"); }
}  // namespace polar_host

static int g_fail = 0;
#define CHECK(cond)                                                        \
    do {                                                                   \
        if (!(cond)) {                                                     \
            std::fprintf(stderr, "check failed at line %d: %s\n", __LINE__, #cond); \
            ++g_fail;                                                      \
        }                                                                  \
    } while (0)

// Fake, aligned device addresses: the host code never dereferences them.
static const void* fake(uintptr_t k) { return reinterpret_cast<const void*>((uintptr_t)0x100000 + k * 4096); }

static polar_frame frame_of(int log2n, int fk, bool dump, uintptr_t k) {
    polar_frame f{};
    f.log2n = log2n;
    f.f_kind = fk;
    f.llr = (const float*)fake(4 * k);
    f.frozen_mask = (const uint32_t*)fake(4 * k + 1);
    f.frozen_vals = (const uint32_t*)fake(4 * k + 2);
    f.u_hat = (uint32_t*)fake(4 * k + 3);
    f.leaf_llr = dump ? (float*)fake(4 * k + 3) : nullptr;
    return f;
}

static void frozen_sets() {
    std::vector<uint32_t> mask;
    std::vector<double> r;
    for (int log2n = 1; log2n <= 16; ++log2n) {
        const int64_t n = (int64_t)1 << log2n;
        mask.assign((size_t)std::max<int64_t>(1, n / 32), 0u);
        r.assign((size_t)n, 0.0);
        for (double z0 : {1e-9, 0.05, 0.341174, 0.5, 0.9, 1.0 - 1e-9}) {
            for (int64_t nf : {(int64_t)-1, (int64_t)0, n / 3, n}) {
                int64_t got = -2;
                const int rc = polar_build_frozen_set(log2n, z0, nf, 0.1, mask.data(), r.data(), &got);
                CHECK(rc == POLAR_OK);
                if (nf >= 0) CHECK(got == nf);
                int64_t ones = 0;
                for (int64_t i = 0; i < n; ++i) ones += (mask[(size_t)(i >> 5)] >> (i & 31)) & 1u;
                CHECK(ones == got);
            }
        }
        CHECK(polar_build_frozen_set(log2n, 0.3, n + 1, 0.1, mask.data(), nullptr, nullptr) != POLAR_OK);
    }
    CHECK(polar_build_frozen_set(0, 0.3, 0, 0.1, mask.data(), nullptr, nullptr) != POLAR_OK);
    CHECK(polar_build_frozen_set(25, 0.3, 1, 0.1, mask.data(), nullptr, nullptr) != POLAR_OK);
    CHECK(polar_build_frozen_set(4, std::nan(""), 1, 0.1, mask.data(), nullptr, nullptr) != POLAR_OK);
    CHECK(polar_build_frozen_set(4, 0.3, 1, 0.1, nullptr, nullptr, nullptr) != POLAR_OK);

    std::mt19937_64 g(7);
    std::uniform_real_distribution<double> u01(0.0, 1.0);
    for (int log2n = 0; log2n <= 14; ++log2n) {
        const int64_t n = (int64_t)1 << log2n;
        std::vector<double> pe((size_t)n);
        for (auto& p : pe) p = g() % 4 == 0 ? 0.25 : u01(g) * 0.5;  // ties included
        mask.assign((size_t)std::max<int64_t>(1, n / 32), 0u);
        for (int64_t nf : {(int64_t)-1, (int64_t)0, n / 2, n}) {
            int64_t got = -2;
            CHECK(polar_frozen_from_pe(log2n, pe.data(), nf, 0.1, mask.data(), &got) == POLAR_OK);
            if (nf >= 0) CHECK(got == nf);
        }
        pe[0] = 1.5;
        CHECK(polar_frozen_from_pe(log2n, pe.data(), 1, 0.1, mask.data(), nullptr) != POLAR_OK);
    }
}

static void plans() {
    polar_ctx c;
    c.n_cu = 256;
    std::mt19937_64 g(11);
    polar_host::Plan p;
    std::vector<polar_frame> frames;
    for (int trial = 0; trial < 60; ++trial) {
        const int n = trial == 0 ? 0 : 1 + (int)(g() % (trial < 30 ? 40 : 700));
        frames.clear();
        for (int k = 0; k < n; ++k) {
            const int fk = (int)(g() % (POLAR_F_MINSUM_Q8 + 1));
            const int log2n = 1 + (int)(g() % POLAR_MAX_LOG2N);
            frames.push_back(frame_of(log2n, fk, g() % 5 == 0, (uintptr_t)k));
        }
        CHECK(polar_host::validate_frames(frames.data(), n) == POLAR_OK);
        for (int plain = 0; plain < 2; ++plain)
            for (int per_frame = 0; per_frame < 2; ++per_frame) {
                polar_host::make_plan(&c, frames.data(), n, plain != 0, p, nullptr, per_frame != 0);
                CHECK((int)p.descs.size() == n);
                int counted = 0;
                for (const auto& gr : p.groups) {
                    counted += gr.count;
                    CHECK(gr.cfg.slots >= 1);
                }
                CHECK(counted == n);
                // grouped by (f_kind, dump), largest first inside a group
                for (const auto& gr : p.groups)
                    for (int k = gr.first + 1; k < gr.first + gr.count; ++k)
                        CHECK(p.descs[(size_t)k].log2n <= p.descs[(size_t)k - 1].log2n &&
                              p.descs[(size_t)k].fkind == gr.fk);
            }
        CHECK(n == 0 || polar_workspace_bytes(&c, frames.data(), n) > 0);
    }
    // every option the plan reads
    c.cutover = 10;
    c.waves = 4;
    c.max_slots = 3;
    c.fwg = 2;
    c.prune = 0;
    frames.clear();
    for (int k = 0; k < 9; ++k) frames.push_back(frame_of(1 + 2 * k, k % 5, k % 3 == 0, (uintptr_t)k));
    polar_host::make_plan(&c, frames.data(), 9, false, p, nullptr, false);
    CHECK((int)p.descs.size() == 9);

    // argument errors
    polar_frame bad = frame_of(10, 0, false, 1);
    bad.f_kind = POLAR_F_MINSUM_Q8 + 1;
    CHECK(polar_host::validate_frames(&bad, 1) != POLAR_OK);
    bad = frame_of(25, 0, false, 1);
    CHECK(polar_host::validate_frames(&bad, 1) != POLAR_OK);
    bad = frame_of(10, 0, false, 1);
    bad.llr = (const float*)((uintptr_t)bad.llr + 4);
    CHECK(polar_host::validate_frames(&bad, 1) != POLAR_OK);
    bad = frame_of(10, 0, false, 1);
    bad.u_hat = nullptr;
    CHECK(polar_host::validate_frames(&bad, 1) != POLAR_OK);
    CHECK(polar_host::validate_frames(nullptr, 1) != POLAR_OK);
    CHECK(polar_workspace_bytes(nullptr, frames.data(), 1) == 0);
}

static void tune_files(const char* dir) {
    polar_ctx c;
    c.n_cu = 256;
    const std::string path = std::string(dir) + "/tune.json";
    auto write = [&](const std::string& text) {
        FILE* f = std::fopen(path.c_str(), "wb");
        std::fwrite(text.data(), 1, text.size(), f);
        std::fclose(f);
    };
    const std::string head = "{\"libpolar_tune\": 1, \"entries\": [";
    write(head + "{\"f_kind\": 0, \"log2n\": 20, \"cutover\": 12, \"waves\": 8, \"slots\": 256, \"fwg\": 1, "
                 "\"prune\": 1}, {\"f_kind\": 4, \"log2n\": 16, \"cutover\": 12, \"waves\": 4, \"slots\": 9}]}");
    CHECK(polar_tune_load(&c, path.c_str()) == POLAR_OK);
    CHECK(c.tuned.size() == 2);
    const std::string saved = std::string(dir) + "/saved.json";
    CHECK(polar_tune_save(&c, saved.c_str()) == POLAR_OK);
    polar_ctx d;
    CHECK(polar_tune_load(&d, saved.c_str()) == POLAR_OK);
    CHECK(d.tuned.size() == 2);
    const char* bad[] = {
        "",
        "{\"entries\": []}",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": 0, \"log2n\": 20",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": 9, \"log2n\": 20, \"cutover\": 12, \"waves\": 8, \"slots\": 1}]}",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": 0, \"log2n\": 20, \"cutover\": 7, \"waves\": 8, \"slots\": 1}]}",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": 0, \"log2n\": 20, \"cutover\": 12, \"waves\": 8, "
        "\"slots\": 99999999999999999999999}]}",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": 0, \"log2n\": 20, \"cutover\": 12, \"waves\": 8}]}",
        "{\"libpolar_tune\": 1, \"entries\": [{\"f_kind\": -, \"log2n\": :, \"cutover\": , \"waves\": 8, \"slots\": 1}]}",
    };
    for (const char* t : bad) {
        write(t);
        polar_ctx e;
        CHECK(polar_tune_load(&e, path.c_str()) != POLAR_OK);
        CHECK(e.tuned.empty());
    }
    CHECK(polar_tune_load(&c, (std::string(dir) + "/missing.json").c_str()) != POLAR_OK);
    CHECK(polar_tune_load(&c, nullptr) != POLAR_OK);
}

static void options() {
    polar_ctx c;
    for (int opt = 0; opt <= 10; ++opt)
        for (int64_t v : {(int64_t)-5, (int64_t)0, (int64_t)1, (int64_t)4, (int64_t)12, (int64_t)1 << 40}) {
            (void)polar_ctx_set_option(&c, opt, v);
            int64_t got = 0;
            (void)polar_ctx_get_option(&c, opt, &got);
        }
    // a long error message is kept whole and NUL-terminated
    std::string big(5000, 'x');
    (void)polar_host::fail(POLAR_E_INVAL, "%s", big.c_str());
    CHECK(std::strlen(polar_last_error()) >= 1);
}

int main(int argc, char** argv) {
    frozen_sets();
    plans();
    tune_files(argc > 1 ? argv[1] : ".");
    options();
    if (g_fail) {
        std::fprintf(stderr, "%d checks failed\n", g_fail);
        return 1;
    }
    std::printf("ok\n");
    return 0;
}
