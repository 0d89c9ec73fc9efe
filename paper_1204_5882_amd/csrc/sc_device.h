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
    uint8_t* slot;      // the frame's own scratch slot, or null: the workgroup's slot
    uint32_t done_idx;  // completion flag index (with DecodeLaunch::done), or ~0u
    uint32_t done_val;  // value written to done[done_idx] once the frame's u-hat is out
};
static_assert(sizeof(FrameDesc) == 64, "descriptor layout");

// Mailbox of one frame workgroup for cooperative level sweeps (128 bytes,
// one per frame workgroup of a launch, zeroed before the launch).
struct SweepBox {
    unsigned long long claim;  // seq << 32 | partitions << 16 | next partition
    uint32_t done;             // partitions finished by other workgroups for seq
    int32_t op;                // 1: sweep2 with g first, 0: sweep2 with f first
    const float* in;
    const uint64_t* beta;
    float* mid;
    float* out;
    int64_t half;
    uint64_t pad[9];
};
static_assert(sizeof(SweepBox) == 128, "mailbox layout");

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
    uint32_t* done;            // completion flags (host-coherent memory) or null
    int small;                 // 1: every frame has at most 2^cutover leaves (per-wavefront kernel)
    int small_log2n;           // small: log2 N of the largest (first) frame
    int fwg;                   // small: frames per workgroup = its wavefronts
    int helpers;               // large frames: workgroups beyond grid that only help with sweeps
    SweepBox* boxes;           // large frames: grid mailboxes (zeroed by the launch), or null
    hipStream_t stream;
};

extern "C" {
hipError_t polar_dev_launch_decode(const DecodeLaunch* a);
// decoder variants (one translation unit each)
hipError_t polar_dec_c10_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c10_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c11_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c11_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_bp_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_ms_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_phi(const DecodeLaunch* a);
hipError_t polar_dec_c12_phi_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_phi_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_phi_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_q16(const DecodeLaunch* a);
hipError_t polar_dec_c12_q16_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_q16_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_q16_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_q8(const DecodeLaunch* a);
hipError_t polar_dec_c12_q8_dump(const DecodeLaunch* a);
hipError_t polar_dec_c12_q8_prune(const DecodeLaunch* a);
hipError_t polar_dec_c12_q8_prune_dump(const DecodeLaunch* a);
hipError_t polar_dec_c8_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c8_ms_prune(const DecodeLaunch* a);
hipError_t polar_dec_c9_bp_prune(const DecodeLaunch* a);
hipError_t polar_dec_c9_ms_prune(const DecodeLaunch* a);
int polar_dec_c10_bp_prune_occupancy(int waves, int small_log2n);
int polar_dec_c10_ms_prune_occupancy(int waves, int small_log2n);
int polar_dec_c11_bp_prune_occupancy(int waves, int small_log2n);
int polar_dec_c11_ms_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_bp_occupancy(int waves, int small_log2n);
int polar_dec_c12_bp_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_bp_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_bp_prune_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_ms_occupancy(int waves, int small_log2n);
int polar_dec_c12_ms_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_ms_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_ms_prune_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_phi_occupancy(int waves, int small_log2n);
int polar_dec_c12_phi_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_phi_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_phi_prune_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_q16_occupancy(int waves, int small_log2n);
int polar_dec_c12_q16_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_q16_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_q16_prune_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_q8_occupancy(int waves, int small_log2n);
int polar_dec_c12_q8_dump_occupancy(int waves, int small_log2n);
int polar_dec_c12_q8_prune_occupancy(int waves, int small_log2n);
int polar_dec_c12_q8_prune_dump_occupancy(int waves, int small_log2n);
int polar_dec_c8_bp_prune_occupancy(int waves, int small_log2n);
int polar_dec_c8_ms_prune_occupancy(int waves, int small_log2n);
int polar_dec_c9_bp_prune_occupancy(int waves, int small_log2n);
int polar_dec_c9_ms_prune_occupancy(int waves, int small_log2n);

int polar_dev_cutover_supported(int c);
// 1 if the decoder variant (cutover, check-update kind, pruning, leaf dump) is built.
int polar_dev_variant_built(int cutover, int fk, int prune, int dump);
// Frames per workgroup a workgroup of `waves` wavefronts can decode at once,
// one per wavefront, for frames of 2^log2n <= 2^cutover leaves (LDS bound).
int polar_dev_max_fwg(int cutover, int log2n, int waves);
// Resident workgroups per compute unit for a decoder variant (0 on error):
// its large-frame kernel with `waves` wavefronts (small_log2n < 0), or its
// per-wavefront kernel with `waves` wavefronts for frames of at most
// 2^small_log2n leaves.
int polar_dev_occupancy(int cutover, int fk, int prune, int dump, int waves, int small_log2n);
int polar_dev_waves_supported(int w);
int64_t polar_dev_slot_bytes(int log2n, int cutover);
hipError_t polar_dev_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, hipStream_t s);
hipError_t polar_dev_lane_selftest(uint32_t* out, hipStream_t s);
hipError_t polar_dev_phi_table(float* out, hipStream_t s);
}
