// Frame-error-rate harness on the device: synthetic BSC frames, SC decoding,
// error counting, all on the GPU.
//
// The paper reports SC decoding at a frame error rate (Table 1, FER and
// efficiency columns), uses the FER in the secret key rate (Section 2.1,
// eq. (5)) and sizes frozen sets for FER 0.1 (Section 3).  This harness
// measures it by Monte Carlo.  Frames are drawn from a counter-based
// generator, Philox4x32-10 (Salmon, Moraes, Dror and Shaw, SC'11), so a
// frame depends only on (seed, frame index) and any frame can be rebuilt
// anywhere:
//   key = (seed mod 2^32, frame index mod 2^32)
//   u word w            = Philox((w >> 2, 0, 0, 0), key)[w & 3]
//   channel error, bit i = Philox((i >> 2, 1, 0, 0), key)[i & 3] < floor(p 2^32)
//   x = u G_N, L_i = +L0 if x_i = e_i else -L0, L0 = float32(ln((1 - p)/p))
//   (16-bit fixed-point check updates: L0 in units of 2^-4, rounded half to
//   even; the 8-bit kind: in units of 2^-2, rounded half to even, capped at 127)
//   frozen values = u on the frozen set
// A frame is in error when its u-hat differs from u anywhere.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>

#include "host_internal.h"
#include "polar.h"
#include "sc_device.h"

using namespace polar_host;

namespace {

// ---------------------------------------------------------------------------
// Philox4x32-10: ten rounds of two 32 x 32 -> 64-bit products whose halves
// are swapped and mixed with the other counter words and the key; the key is
// bumped by two Weyl increments between rounds.
// ---------------------------------------------------------------------------
struct U4 {
    uint32_t x, y, z, w;
};

__device__ __forceinline__ U4 philox4x32_10(U4 c, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * c.x;
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * c.z;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        c = U4{hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0};
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

// u words of n_frames frames (frame k at u + k * wpf) and their frozen
// values; one thread per Philox block of four words.
__global__ __launch_bounds__(256) void k_gen_u(uint32_t seed, uint32_t frame0, int n_frames, int log2n, int64_t wpf,
                                               const uint32_t* __restrict__ mask, uint32_t* __restrict__ u,
                                               uint32_t* __restrict__ vals) {
    const int64_t blocks_per_frame = (wpf + 3) / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= blocks_per_frame * n_frames) return;
    const int64_t f = t / blocks_per_frame;
    const int64_t b = t % blocks_per_frame;
    const U4 r = philox4x32_10(U4{(uint32_t)b, 0u, 0u, 0u}, seed, frame0 + (uint32_t)f);
    const uint32_t out[4] = {r.x, r.y, r.z, r.w};
    const uint32_t low = log2n < 5 ? (1u << (1 << log2n)) - 1u : 0xFFFFFFFFu;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t w = b * 4 + j;
        if (w < wpf) {
            const uint32_t word = out[j] & low;
            u[f * wpf + w] = word;
            vals[f * wpf + w] = word & mask[w];
        }
    }
}

// Channel LLRs from x = u G_N and the BSC error indicators: one thread per
// Philox block of stream 1 (four consecutive bits, one 16-byte store).
__global__ __launch_bounds__(256) void k_gen_llr_bsc(uint32_t seed, uint32_t frame0, int n_frames, int log2n,
                                                     int64_t wpf, uint32_t thresh, float l0,
                                                     const uint32_t* __restrict__ x, float* __restrict__ llr) {
    const int64_t n = (int64_t)1 << log2n;
    const int64_t quads = (n + 3) / 4;
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= quads * n_frames) return;
    const int64_t f = t / quads;
    const int64_t q = t % quads;
    const U4 r = philox4x32_10(U4{(uint32_t)q, 1u, 0u, 0u}, seed, frame0 + (uint32_t)f);
    const uint32_t ev[4] = {r.x, r.y, r.z, r.w};
    float o[4];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = q * 4 + j;
        const uint32_t xb = i < n ? (x[f * wpf + (i >> 5)] >> (i & 31)) & 1u : 0u;
        const uint32_t y = xb ^ (ev[j] < thresh ? 1u : 0u);
        o[j] = y ? -l0 : l0;
    }
    float* dst = llr + f * n + q * 4;
    if (n >= 4) {
        *reinterpret_cast<float4*>(dst) = make_float4(o[0], o[1], o[2], o[3]);
    } else {
        for (int j = 0; j < n; ++j) dst[j] = o[j];
    }
}

// Bit errors of each frame: popcount(u xor u-hat) over its words, reduced
// in the workgroup (blockIdx.y = frame, blockIdx.x = chunk of words), one
// atomic per workgroup.
__global__ __launch_bounds__(256) void k_count_errors(const uint32_t* __restrict__ u,
                                                      const uint32_t* __restrict__ uhat, int64_t wpf,
                                                      uint32_t* __restrict__ bit_err) {
    __shared__ uint32_t part[256];
    const int64_t f = blockIdx.y;
    const int64_t chunk = (wpf + gridDim.x - 1) / gridDim.x;
    const int64_t lo = blockIdx.x * chunk;
    const int64_t hi = lo + chunk < wpf ? lo + chunk : wpf;
    uint32_t s = 0;
    for (int64_t w = lo + threadIdx.x; w < hi; w += blockDim.x) s += __popc(u[f * wpf + w] ^ uhat[f * wpf + w]);
    part[threadIdx.x] = s;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) part[threadIdx.x] += part[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part[0]) atomicAdd(bit_err + f, part[0]);
}

__global__ void k_zero_u32(uint32_t* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0u;
}

// totals[0] += frames with errors, totals[1] += bit errors (one workgroup)
__global__ __launch_bounds__(256) void k_sum_errors(const uint32_t* __restrict__ bit_err, int64_t n,
                                                    unsigned long long* totals) {
    __shared__ unsigned long long fr[256], bi[256];
    unsigned long long a = 0, b = 0;
    for (int64_t i = threadIdx.x; i < n; i += blockDim.x) {
        a += bit_err[i] ? 1ull : 0ull;
        b += bit_err[i];
    }
    fr[threadIdx.x] = a;
    bi[threadIdx.x] = b;
    __syncthreads();
    for (int h = 128; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            fr[threadIdx.x] += fr[threadIdx.x + h];
            bi[threadIdx.x] += bi[threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        totals[0] = fr[0];
        totals[1] = bi[0];
    }
}

int64_t wpf_of(int log2n) { return log2n >= 5 ? ((int64_t)1 << (log2n - 5)) : 1; }

unsigned grid_of(int64_t threads) { return (unsigned)((threads + 255) / 256); }

int check_cfg(const polar_fer_cfg* cfg) {
    if (!cfg) return fail(POLAR_E_INVAL, "cfg is NULL");
    if (cfg->log2n < 1 || cfg->log2n > POLAR_MAX_LOG2N)
        return fail(POLAR_E_INVAL, "log2n %d outside 1..%d", cfg->log2n, POLAR_MAX_LOG2N);
    if (cfg->f_kind < POLAR_F_MINSUM || cfg->f_kind > POLAR_F_MINSUM_Q8) return fail(POLAR_E_INVAL, "unknown f_kind");
    if (!(cfg->p > 0.0 && cfg->p < 0.5)) return fail(POLAR_E_INVAL, "p must lie in (0, 1/2)");
    if (!cfg->frozen_mask) return fail(POLAR_E_INVAL, "frozen_mask is NULL");
    if (cfg->n_frames < 0 || cfg->frame0 < 0 || cfg->frame0 + cfg->n_frames > ((int64_t)1 << 32))
        return fail(POLAR_E_INVAL, "frame indices must lie in 0 .. 2^32 - 1");
    if (cfg->batch < 0) return fail(POLAR_E_INVAL, "batch < 0");
    return ok();
}

// Frames per generate-decode-count step.
int batch_of(const polar_ctx* c, const polar_fer_cfg* cfg) {
    if (cfg->batch > 0) return cfg->batch;
    // every resident workgroup busy (small frames go one per wavefront), at
    // most 32 GiB of channel LLRs per step
    const int per = cfg->log2n > 12 ? 1 : 8 * 4;
    const int64_t by_mem = ((int64_t)32 << 30) / ((int64_t)4 << cfg->log2n);
    return (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)c->n_cu * per, by_mem));
}

struct FerLayout {
    int batch;
    size_t totals, llr, u, x, vals, uhat, dec, total;
    size_t dec_bytes;
};

FerLayout layout(const polar_ctx* c, const polar_fer_cfg* cfg) {
    FerLayout L{};
    L.batch = batch_of(c, cfg);
    const int64_t n = (int64_t)1 << cfg->log2n;
    const size_t wb = (size_t)wpf_of(cfg->log2n) * 4 * (size_t)L.batch;
    // decode workspace of a full batch
    std::vector<polar_frame> fr((size_t)L.batch);
    for (auto& f : fr) {
        f = polar_frame{};
        f.log2n = cfg->log2n;
        f.f_kind = cfg->f_kind;
    }
    L.dec_bytes = polar_workspace_bytes(c, fr.data(), L.batch);
    L.totals = 0;
    L.llr = 256;
    L.u = align256(L.llr + (size_t)n * 4 * (size_t)L.batch);
    L.x = align256(L.u + wb);
    L.vals = align256(L.x + wb);
    L.uhat = align256(L.vals + wb);
    L.dec = align256(L.uhat + wb);
    L.total = L.dec + L.dec_bytes;
    return L;
}

}  // namespace

extern "C" int polar_fer_generate_bsc(int log2n, double p, int fixed_point, const uint32_t* frozen_mask,
                                      uint64_t seed, int64_t frame0, int n_frames, uint32_t* u,
                                      uint32_t* frozen_vals, uint32_t* x_scratch, float* llr, void* stream) {
    if (log2n < 1 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 1..%d", log2n, POLAR_MAX_LOG2N);
    if (!(p > 0.0 && p < 0.5)) return fail(POLAR_E_INVAL, "p must lie in (0, 1/2)");
    if (fixed_point < 0 || fixed_point > 2) return fail(POLAR_E_INVAL, "fixed_point must be 0, 1 or 2");
    if (n_frames < 0 || frame0 < 0 || frame0 + n_frames > ((int64_t)1 << 32))
        return fail(POLAR_E_INVAL, "frame indices must lie in 0 .. 2^32 - 1");
    if (n_frames == 0) return ok();
    if (!frozen_mask || !u || !frozen_vals || !x_scratch || !llr) return fail(POLAR_E_INVAL, "NULL buffer");
    if ((uintptr_t)llr & 15) return fail(POLAR_E_INVAL, "llr must be 16-byte aligned");
    hipStream_t s = (hipStream_t)stream;
    const int64_t wpf = wpf_of(log2n);
    const int64_t n = (int64_t)1 << log2n;
    const uint32_t th = (uint32_t)std::floor(p * 4294967296.0);
    // fixed point: L0 in units of 2^-4 (8-bit: 2^-2), rounded half to even, saturated
    const double l0d = std::log((1.0 - p) / p);
    const float l0 = fixed_point == 1 ? (float)std::min(std::nearbyint(l0d * (1 << POLAR_FIXED_FRAC)), (double)POLAR_FIXED_MAX)
                     : fixed_point == 2
                         ? (float)std::min(std::nearbyint(l0d * (1 << POLAR_FIXED8_FRAC)), (double)POLAR_FIXED8_MAX)
                         : (float)l0d;
    hipLaunchKernelGGL(k_gen_u, dim3(grid_of((wpf + 3) / 4 * n_frames)), dim3(256), 0, s, (uint32_t)seed,
                       (uint32_t)frame0, n_frames, log2n, wpf, frozen_mask, u, frozen_vals);
    hipError_t e = polar_dev_encode(log2n, n_frames, u, x_scratch, s);
    if (e != hipSuccess) return hip_fail(e, "encode");
    hipLaunchKernelGGL(k_gen_llr_bsc, dim3(grid_of((n + 3) / 4 * n_frames)), dim3(256), 0, s, (uint32_t)seed,
                       (uint32_t)frame0, n_frames, log2n, wpf, th, l0, x_scratch, llr);
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "frame generation");
    return ok();
}

extern "C" size_t polar_fer_workspace_bytes(const polar_ctx* c, const polar_fer_cfg* cfg) {
    if (!c || check_cfg(cfg)) return 0;
    return layout(c, cfg).total;
}

extern "C" int polar_fer_bsc(polar_ctx* c, const polar_fer_cfg* cfg, void* workspace, size_t ws_bytes,
                             uint32_t* bit_errors, polar_fer_result* out, void* stream) {
    TraceRange tr("polar_fer_bsc");
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    int rc = check_cfg(cfg);
    if (rc) return rc;
    if (!bit_errors || !out) return fail(POLAR_E_INVAL, "NULL output");
    if (((uintptr_t)workspace & 255) != 0) return fail(POLAR_E_INVAL, "workspace must be 256-byte aligned");
    const FerLayout L = layout(c, cfg);
    if (!workspace || ws_bytes < L.total)
        return fail(POLAR_E_NOMEM, "workspace of %zu bytes < %zu required", ws_bytes, L.total);
    std::memset(out, 0, sizeof *out);
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    uint8_t* ws = (uint8_t*)workspace;
    const int log2n = cfg->log2n;
    const int64_t n = (int64_t)1 << log2n;
    const int64_t wpf = wpf_of(log2n);
    float* llr = (float*)(ws + L.llr);
    uint32_t* u = (uint32_t*)(ws + L.u);
    uint32_t* x = (uint32_t*)(ws + L.x);
    uint32_t* vals = (uint32_t*)(ws + L.vals);
    uint32_t* uhat = (uint32_t*)(ws + L.uhat);
    if (cfg->n_frames > 0)
        hipLaunchKernelGGL(k_zero_u32, dim3(grid_of(cfg->n_frames)), dim3(256), 0, s, bit_errors, cfg->n_frames);
    std::vector<polar_frame> fr;
    Plan p;
    for (int64_t done = 0; done < cfg->n_frames; done += L.batch) {
        const int nb = (int)std::min<int64_t>(L.batch, cfg->n_frames - done);
        const int fixed = cfg->f_kind == POLAR_F_MINSUM_Q8 ? 2 : (cfg->f_kind >= POLAR_F_MINSUM_Q16 ? 1 : 0);
        rc = polar_fer_generate_bsc(log2n, cfg->p, fixed, cfg->frozen_mask, cfg->seed,
                                    cfg->frame0 + done, nb, u, vals, x, llr, stream);
        if (rc) return rc;
        fr.assign((size_t)nb, polar_frame{});
        for (int k = 0; k < nb; ++k) {
            fr[(size_t)k].log2n = log2n;
            fr[(size_t)k].f_kind = cfg->f_kind;
            fr[(size_t)k].llr = llr + (int64_t)k * n;
            fr[(size_t)k].frozen_mask = cfg->frozen_mask;
            fr[(size_t)k].frozen_vals = vals + (int64_t)k * wpf;
            fr[(size_t)k].u_hat = uhat + (int64_t)k * wpf;
        }
        make_plan(c, fr.data(), nb, false, p);
        rc = run_plan(c, p, ws + L.dec, L.dec_bytes, s, c->stager, false);
        if (rc) return rc;
        const unsigned chunks = (unsigned)std::max<int64_t>(1, std::min<int64_t>(64, wpf / 2048));
        hipLaunchKernelGGL(k_count_errors, dim3(chunks, (unsigned)nb), dim3(256), 0, s, u, uhat, wpf,
                           bit_errors + done);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return hip_fail(e, "error count");
    }
    unsigned long long* totals = (unsigned long long*)(ws + L.totals);
    hipLaunchKernelGGL(k_sum_errors, dim3(1), dim3(256), 0, s, bit_errors, cfg->n_frames, totals);
    unsigned long long host[2] = {0, 0};
    hipError_t e = hipMemcpyAsync(host, totals, sizeof host, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "FER totals");
    out->frames = cfg->n_frames;
    out->frame_errors = (int64_t)host[0];
    out->bit_errors = (int64_t)host[1];
    return ok();
}
