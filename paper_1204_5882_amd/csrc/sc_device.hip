// Device code of libpolar outside the decoder variants: the polar encoder,
// the cross-lane self-test and the dispatch to the decoder variants (each
// compiled in its own translation unit, see sc_kernels.h).
#include "sc_kernels.h"

namespace polar_dev {

// ---------------------------------------------------------------------------
// Encoder x = u G_N on packed words.
// Local stages (distance < 2^LOCAL bits) run on a chunk of 2^LOCAL bits in
// registers/LDS; the remaining stages are word-level XOR passes.
// ---------------------------------------------------------------------------
constexpr int ENC_LOCAL = 14;  // 16384 bits = 512 words per chunk

__global__ __launch_bounds__(256) void k_encode_local(const uint32_t* __restrict__ u, uint32_t* __restrict__ x,
                                                      int log2n, int64_t words_per_frame, int64_t n_chunks) {
    __shared__ uint32_t sw[512];
    const int64_t chunk = blockIdx.x;  // over frames * chunks
    const int tid = threadIdx.x;
    const int lg = log2n < ENC_LOCAL ? log2n : ENC_LOCAL;
    const int nbits = 1 << lg;
    const int nwords = nbits >= 32 ? nbits / 32 : 1;
    const int64_t frame = chunk / n_chunks;
    const int64_t c = chunk % n_chunks;
    const uint32_t* src = u + frame * words_per_frame + c * nwords;
    uint32_t* dst = x + frame * words_per_frame + c * nwords;
    for (int i = tid; i < nwords; i += blockDim.x) {
        uint32_t w = src[i];
        if (nbits < 32) w &= (1u << nbits) - 1u;
        // in-word stages h = 1 .. 16
#pragma unroll
        for (int h = 1; h < 32; h <<= 1)
            if (h < nbits) w ^= (w >> h) & (uint32_t)low_mask64(h);
        sw[i] = w;
    }
    __syncthreads();
    for (int hw = 1; hw < nwords; hw <<= 1) {  // word distance
        for (int i = tid; i < nwords; i += blockDim.x)
            if (!(i & hw)) sw[i] ^= sw[i + hw];
        __syncthreads();
    }
    for (int i = tid; i < nwords; i += blockDim.x) dst[i] = sw[i];
}

__global__ __launch_bounds__(256) void k_encode_stage(uint32_t* __restrict__ x, int64_t words_per_frame,
                                                      int64_t hw, int64_t total_pairs) {
    // one thread per (frame, lower-half word): x[i] ^= x[i + hw]
    int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= total_pairs) return;
    const int64_t per_frame = words_per_frame / 2;
    const int64_t frame = p / per_frame;
    const int64_t q = p % per_frame;
    const int64_t blk = q / hw, off = q % hw;
    const int64_t i = frame * words_per_frame + blk * 2 * hw + off;
    x[i] ^= x[i + hw];
}

// Self-test of the cross-lane primitives used above (diagnostics only).
__global__ void k_lane_selftest(uint32_t* out) {
    const int l = lane_id();
    uint32_t x = 1000u + (uint32_t)l;
    out[0 * 64 + l] = lane_down<1>(x);
    out[1 * 64 + l] = lane_down<2>(x);
    out[2 * 64 + l] = lane_down<4>(x);
    out[3 * 64 + l] = lane_down<8>(x);
    out[4 * 64 + l] = lane_down<16>(x);
    out[5 * 64 + l] = lane_down<32>(x);
    out[6 * 64 + l] = lane_up<1>(x);
    out[7 * 64 + l] = lane_up<2>(x);
    out[8 * 64 + l] = lane_up<4>(x);
    out[9 * 64 + l] = lane_up<8>(x);
    out[10 * 64 + l] = lane_up<16>(x);
    out[11 * 64 + l] = lane_up<32>(x);
    uint64_t w = (uint64_t)(l * 2654435761u) ^ ((uint64_t)(l + 17) << 40);
    uint64_t t = transpose64(w);
    out[12 * 64 + l] = (uint32_t)t;
    out[13 * 64 + l] = (uint32_t)(t >> 32);
    uint64_t lt = lane_transform(w);
    out[14 * 64 + l] = (uint32_t)lt;
    out[15 * 64 + l] = (uint32_t)(lt >> 32);
}

// The phi table of the fixed-point check update, as every workgroup of a
// FK = 3 decoder builds it (diagnostics).
__global__ void k_phi_table(float* out) {
    phi_table_init();
    __syncthreads();
    for (int i = (int)threadIdx.x; i < PHI_LEN; i += (int)blockDim.x) out[i] = g_phi[i];
}

}  // namespace polar_dev

using namespace polar_dev;

extern "C" hipError_t polar_dev_phi_table(float* out, hipStream_t s) {
    hipLaunchKernelGGL(k_phi_table, dim3(1), dim3(256), 0, s, out);
    return hipGetLastError();
}

namespace {

// Every built decoder variant: (cutover, check-update kind, pruning, leaf
// dump) and its launch and occupancy functions.
struct Variant {
    int cutover, fk, prune, dump;
    hipError_t (*launch)(const DecodeLaunch*);
    int (*occupancy)(int, int);
};

constexpr Variant kVariants[] = {
    {10, 1, 1, 0, polar_dec_c10_bp_prune, polar_dec_c10_bp_prune_occupancy},
    {10, 0, 1, 0, polar_dec_c10_ms_prune, polar_dec_c10_ms_prune_occupancy},
    {11, 1, 1, 0, polar_dec_c11_bp_prune, polar_dec_c11_bp_prune_occupancy},
    {11, 0, 1, 0, polar_dec_c11_ms_prune, polar_dec_c11_ms_prune_occupancy},
    {12, 1, 0, 0, polar_dec_c12_bp, polar_dec_c12_bp_occupancy},
    {12, 1, 0, 1, polar_dec_c12_bp_dump, polar_dec_c12_bp_dump_occupancy},
    {12, 1, 1, 0, polar_dec_c12_bp_prune, polar_dec_c12_bp_prune_occupancy},
    {12, 1, 1, 1, polar_dec_c12_bp_prune_dump, polar_dec_c12_bp_prune_dump_occupancy},
    {12, 0, 0, 0, polar_dec_c12_ms, polar_dec_c12_ms_occupancy},
    {12, 0, 0, 1, polar_dec_c12_ms_dump, polar_dec_c12_ms_dump_occupancy},
    {12, 0, 1, 0, polar_dec_c12_ms_prune, polar_dec_c12_ms_prune_occupancy},
    {12, 0, 1, 1, polar_dec_c12_ms_prune_dump, polar_dec_c12_ms_prune_dump_occupancy},
    {12, 3, 0, 0, polar_dec_c12_phi, polar_dec_c12_phi_occupancy},
    {12, 3, 0, 1, polar_dec_c12_phi_dump, polar_dec_c12_phi_dump_occupancy},
    {12, 3, 1, 0, polar_dec_c12_phi_prune, polar_dec_c12_phi_prune_occupancy},
    {12, 3, 1, 1, polar_dec_c12_phi_prune_dump, polar_dec_c12_phi_prune_dump_occupancy},
    {12, 2, 0, 0, polar_dec_c12_q16, polar_dec_c12_q16_occupancy},
    {12, 2, 0, 1, polar_dec_c12_q16_dump, polar_dec_c12_q16_dump_occupancy},
    {12, 2, 1, 0, polar_dec_c12_q16_prune, polar_dec_c12_q16_prune_occupancy},
    {12, 2, 1, 1, polar_dec_c12_q16_prune_dump, polar_dec_c12_q16_prune_dump_occupancy},
    {12, 4, 0, 0, polar_dec_c12_q8, polar_dec_c12_q8_occupancy},
    {12, 4, 0, 1, polar_dec_c12_q8_dump, polar_dec_c12_q8_dump_occupancy},
    {12, 4, 1, 0, polar_dec_c12_q8_prune, polar_dec_c12_q8_prune_occupancy},
    {12, 4, 1, 1, polar_dec_c12_q8_prune_dump, polar_dec_c12_q8_prune_dump_occupancy},
    {8, 1, 1, 0, polar_dec_c8_bp_prune, polar_dec_c8_bp_prune_occupancy},
    {8, 0, 1, 0, polar_dec_c8_ms_prune, polar_dec_c8_ms_prune_occupancy},
    {9, 1, 1, 0, polar_dec_c9_bp_prune, polar_dec_c9_bp_prune_occupancy},
    {9, 0, 1, 0, polar_dec_c9_ms_prune, polar_dec_c9_ms_prune_occupancy},
};

const Variant* find_variant(int cutover, int fk, int prune, int dump) {
    for (const Variant& v : kVariants)
        if (v.cutover == cutover && v.fk == fk && v.prune == (prune ? 1 : 0) && v.dump == (dump ? 1 : 0)) return &v;
    return nullptr;
}

}  // namespace

extern "C" hipError_t polar_dev_launch_decode(const DecodeLaunch* a) {
    if (a->waves != 4 && a->waves != 8) return hipErrorInvalidValue;
    const Variant* v = find_variant(a->cutover, a->fk, a->prune, a->dump);
    return v ? v->launch(a) : hipErrorInvalidValue;
}

extern "C" int polar_dev_occupancy(int cutover, int fk, int prune, int dump, int waves, int small_log2n) {
    const Variant* v = find_variant(cutover, fk, prune, dump);
    return v ? v->occupancy(waves, small_log2n) : 0;
}

extern "C" int polar_dev_variant_built(int cutover, int fk, int prune, int dump) {
    return find_variant(cutover, fk, prune, dump) != nullptr;
}

extern "C" int polar_dev_max_fwg(int cutover, int log2n, int waves) {
    if (log2n > cutover) return 1;
    switch (cutover) {
        case 12: return max_fwg<12>(log2n, waves);
        case 11: return max_fwg<11>(log2n, waves);
        case 10: return max_fwg<10>(log2n, waves);
        case 9: return max_fwg<9>(log2n, waves);
        case 8: return max_fwg<8>(log2n, waves);
    }
    return 1;
}

extern "C" int polar_dev_cutover_supported(int c) { return c >= 8 && c <= 12; }
extern "C" int polar_dev_waves_supported(int w) { return w == 4 || w == 8; }

extern "C" int64_t polar_dev_slot_bytes(int log2n, int cutover) {
    if (log2n <= cutover) return 256;
    const int D = log2n - cutover;
    int64_t levels = slot_level_offset(log2n, D);            // levels 1 .. D-1
    int64_t beta = ((int64_t)1 << D) * 64 * 8;                // lane-packed partial sums
    int64_t total = levels + beta;
    return (total + 255) & ~(int64_t)255;
}

extern "C" hipError_t polar_dev_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, hipStream_t s) {
    if (n_frames <= 0) return hipSuccess;
    const int64_t n = (int64_t)1 << log2n;
    const int64_t wpf = n >= 32 ? n / 32 : 1;
    const int lg = log2n < ENC_LOCAL ? log2n : ENC_LOCAL;
    const int64_t chunk_words = lg >= 5 ? ((int64_t)1 << lg) / 32 : 1;
    const int64_t n_chunks = wpf / chunk_words;
    hipLaunchKernelGGL(k_encode_local, dim3((unsigned)(n_chunks * n_frames)), dim3(256), 0, s, u, x, log2n, wpf,
                       n_chunks);
    for (int64_t hw = chunk_words; hw < wpf; hw <<= 1) {
        const int64_t pairs = (wpf / 2) * n_frames;
        const unsigned blocks = (unsigned)((pairs + 255) / 256);
        hipLaunchKernelGGL(k_encode_stage, dim3(blocks), dim3(256), 0, s, x, wpf, hw, pairs);
    }
    return hipGetLastError();
}

extern "C" hipError_t polar_dev_lane_selftest(uint32_t* out, hipStream_t s) {
    hipLaunchKernelGGL(k_lane_selftest, dim3(1), dim3(64), 0, s, out);
    return hipGetLastError();
}
