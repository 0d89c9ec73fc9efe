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

extern "C" {
hipError_t polar_dev_launch_decode(int cutover, int fk, int prune, int dump, int waves, const FrameDesc* descs,
                                   int n_frames, unsigned* counter, uint8_t* slots, int64_t slot_bytes, int grid,
                                   hipStream_t s);
int polar_dev_cutover_supported(int c);
int polar_dev_waves_supported(int w);
int64_t polar_dev_slot_bytes(int log2n, int cutover);
hipError_t polar_dev_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, hipStream_t s);
hipError_t polar_dev_lane_selftest(uint32_t* out, hipStream_t s);
}
