// Internal interface between the libpolar C ABI (host code) and its device
// code.  Not part of the public API.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

// One frame as the device sees it (64 bytes, built by the host from a
// polar_frame).
struct FrameDesc {
    const float* llr;
    const uint32_t* mask;
    const uint32_t* vals;
    uint32_t* uhat;
    float* leaf;
    int32_t log2n;
    int32_t fkind;
    int64_t pad[2];
};
static_assert(sizeof(FrameDesc) == 64, "descriptor layout");

// Everything one persistent decode launch needs.
struct DecodeLaunch {
    int cutover;               // log2 of the register-resident subtree
    int fk;                    // 0 min-sum, 1 box-plus
    int prune;                 // exact rate-0 / rate-1 shortcuts
    int dump;                  // write leaf LLRs
    int waves;                 // wavefronts per workgroup
    int grid;                  // workgroups (frames in flight)
    const FrameDesc* descs;    // device descriptor table
    int n_frames;
    unsigned* counter;         // device work counter (reset by the launch)
    uint8_t* slots;            // per-workgroup scratch, slot_bytes each
    int64_t slot_bytes;
    unsigned long long* prof;  // optional timing counters (device, 8 words) or null
    hipStream_t stream;
};

extern "C" {
hipError_t polar_dev_launch_decode(const DecodeLaunch* a);
// decoder variants (one translation unit each)
hipError_t polar_dec_c12_ms(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c11_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c11_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c10_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c10_bp_prune(const DecodeLaunch* a);

int polar_dev_cutover_supported(int c);
int polar_dev_waves_supported(int w);
int64_t polar_dev_slot_bytes(int log2n, int cutover);
hipError_t polar_dev_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, hipStream_t s);
hipError_t polar_dev_lane_selftest(uint32_t* out, hipStream_t s);
}
