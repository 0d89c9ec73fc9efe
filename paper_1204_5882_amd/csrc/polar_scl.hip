// SC list decoding on the device.
//
// Section 4 names list decoders (Tal and Vardy; Li, Shen and Tang; Chen,
// Niu and Lin) as the improvement over SC.  This file decodes each frame
// with up to L paths, FP32 min-sum f and g as in the SC decoder, and the
// LLR form of the path metric (Balatsoukas-Stimming, Bastani Parizi, Burg):
//   frozen leaf:  u = frozen value; PM += |lambda| if u != [lambda < 0]
//   info leaf:    each path p offers u = b with PM_p + (b != [lambda < 0] ?
//                 |lambda| : 0), b = 0, 1; candidates are ordered by
//                 (metric, p, b) and the first min(L, count) become the new
//                 paths, in that order
// and returns the path of least metric (ties to the lower path).
//
// Layout: one wavefront per frame, every path's state in LDS.  A path owns a
// slot: the LLRs of its current node at every depth (depth d at offset
// N - (N >> (d - 1)), N >> d floats) and its decided bits (one byte each).
// The partial sums a g needs are the left sibling's decisions re-encoded
// into a per-slot scratch.  Each level update runs over all paths at once
// (lane = path x element), so small nodes still fill the wavefront.  At an
// information leaf the ranks of the 2L candidates come from one comparison
// per candidate pair across lanes; a surviving path keeps its parent's slot
// for its first child and copies it into a free slot for the second.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <vector>

#include "host_internal.h"
#include "polar.h"
#include "sc_device.h"

using namespace polar_host;

namespace {

__device__ __forceinline__ float scl_f(float a, float b) {
    const float m = fminf(fabsf(a), fabsf(b));
    const uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(m) | s);
}

__device__ __forceinline__ float lane_readf(float x, int l) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

__device__ __forceinline__ int depth_off(int n_leaves, int d) { return n_leaves - (n_leaves >> (d - 1)); }

// LDS of one frame, in this order: LLRs [list][N] floats, frozen mask and
// value words [2][W], slot table [list] ints, decided bits [list][W] words,
// partial-sum scratch [list][max(1, N/2)] bytes; W = max(1, N/32).
__host__ __device__ inline size_t scl_lds_bytes(int log2n, int list) {
    const size_t n = (size_t)1 << log2n;
    const size_t half = n > 1 ? n / 2 : 1;
    const size_t words = n >= 32 ? n / 32 : 1;
    return (size_t)list * n * 4 + 2 * words * 4 + 4 * (size_t)list + (size_t)list * words * 4 + (size_t)list * half;
}

__global__ __launch_bounds__(64) void k_scl_decode(const FrameDesc* __restrict__ descs, int n_frames, int list,
                                                   float* __restrict__ pm_out) {
    extern __shared__ float lds[];
    const int f = (int)blockIdx.x;
    if (f >= n_frames) return;
    const FrameDesc fd = descs[f];
    const int n = fd.log2n;
    const int N = 1 << n;
    const int NB = N > 1 ? N / 2 : 1;
    const int W = N >= 32 ? N / 32 : 1;
    float* A = lds;
    uint32_t* mw = reinterpret_cast<uint32_t*>(A + (size_t)list * N);
    uint32_t* vw = mw + W;
    int* phys = reinterpret_cast<int*>(vw + W);
    uint32_t* U = reinterpret_cast<uint32_t*>(phys + list);  // bit i of word i/32: decision of leaf i
    uint8_t* Bt = reinterpret_cast<uint8_t*>(U + (size_t)list * W);
    const int lane = (int)threadIdx.x;

    for (int w = lane; w < W; w += 64) {
        mw[w] = fd.mask[w];
        vw[w] = fd.vals[w];
    }
    // logical path k (lane k) lives in slot phys[k]; phys is a permutation of
    // the slots whose first `active` entries are the live paths
    if (lane < list) phys[lane] = lane;
    float pm = 0.0f;  // lane k: metric of path k
    int active = 1;

    // f (g_op false) or g at depth d for every live path: out[j] = op(par[j], par[j + h])
    auto level = [&](int d, bool g_op) {
        const int th = n - d;
        const int h = 1 << th;
        const int total = active << th;
        for (int base = 0; base < total; base += 64) {
            const int idx = base + lane;
            if (idx < total) {
                const int k = idx >> th, j = idx & (h - 1);
                const int s = phys[k];
                const float* par = d == 1 ? fd.llr : A + (size_t)s * N + depth_off(N, d - 1);
                const float a = par[j], b = par[j + h];
                float r;
                if (g_op) r = Bt[(size_t)s * NB + j] ? b - a : b + a;
                else r = scl_f(a, b);
                A[(size_t)s * N + depth_off(N, d) + j] = r;
            }
        }
    };

    for (int i = 0; i < N; ++i) {
        int top = 1;
        if (i > 0) {
            const int t = __builtin_ctz((unsigned)i);
            const int h = 1 << t;
            top = n - t;
            const int total = active << t;
            // partial sums of the left sibling (leaves i-h .. i-1), re-encoded:
            // x[j] ^= x[j + q] for every j without bit q, q = 1, 2, .., h/2
            for (int base = 0; base < total; base += 64) {
                const int idx = base + lane;
                if (idx < total) {
                    const int s = phys[idx >> t], j = idx & (h - 1);
                    const int e = i - h + j;
                    Bt[(size_t)s * NB + j] = (uint8_t)((U[(size_t)s * W + (e >> 5)] >> (e & 31)) & 1u);
                }
            }
            for (int q = 1; q < h; q <<= 1)
                for (int base = 0; base < total; base += 64) {
                    const int idx = base + lane;
                    if (idx < total) {
                        const int s = phys[idx >> t], j = idx & (h - 1);
                        if ((j & q) == 0) Bt[(size_t)s * NB + j] ^= Bt[(size_t)s * NB + j + q];
                    }
                }
            level(top, true);
            ++top;
        }
        for (int d = top; d <= n; ++d) level(d, false);

        // leaf LLR of path k on lane k
        float lam = 0.0f;
        if (lane < active) lam = n == 0 ? fd.llr[0] : A[(size_t)phys[lane] * N + depth_off(N, n)];
        const bool hard = lam < 0.0f;

        if ((mw[i >> 5] >> (i & 31)) & 1u) {
            const int b = (int)((vw[i >> 5] >> (i & 31)) & 1u);
            if (lane < active) {
                if ((b != 0) != hard) pm = pm + fabsf(lam);
                uint32_t* w = U + (size_t)phys[lane] * W + (i >> 5);
                *w = (*w & ~(1u << (i & 31))) | ((uint32_t)b << (i & 31));
            }
            continue;
        }

        // candidates c = 2k + b on lanes c < 2 active
        const int nc = 2 * active;
        const int kc = lane >> 1, bc = lane & 1;
        const float lam_k = __shfl(lam, kc);
        const float pm_k = __shfl(pm, kc);
        const bool hard_k = lam_k < 0.0f;
        float pmc = pm_k;
        if ((bc != 0) != hard_k) pmc = pm_k + fabsf(lam_k);
        int rank = 0;
        for (int c2 = 0; c2 < nc; ++c2) {
            const float o = lane_readf(pmc, c2);
            rank += (o < pmc || (o == pmc && c2 < lane)) ? 1 : 0;
        }
        const int keep = nc < list ? nc : list;
        const bool survives = lane < nc && rank < keep;

        // new paths in rank order: r -> candidate lane cand_of[r]
        int new_slot = -1, new_parent = 0, new_bit = 0;  // lane r: its path's slot, parent, bit
        float new_pm = 0.0f;
        uint32_t claimed = 0u;  // parents whose slot went to their first surviving child
        int pending = 0;        // bit r: rank r needs a fresh slot
        for (int r = 0; r < keep; ++r) {
            const uint64_t hit = __ballot(survives && rank == r);
            const int c = hit ? (int)__builtin_ctzll(hit) : 0;  // (a NaN metric only: inputs are finite)
            const int p = c >> 1;
            const int slot_p = phys[p];
            const float pmr = lane_readf(pmc, c);
            if (lane == r) {
                new_parent = p;
                new_bit = c & 1;
                new_pm = pmr;
                new_slot = (claimed >> p) & 1u ? -1 : slot_p;
            }
            if (((claimed >> p) & 1u) == 0u) claimed |= 1u << p;
            else pending |= 1 << r;
        }
        // free slots: those of parents left without a child, and the unused ones
        uint32_t used = 0u;
        for (int k = 0; k < active; ++k)
            if ((claimed >> k) & 1u) used |= 1u << phys[k];
        uint32_t free_slots = ((list >= 32 ? 0xffffffffu : ((1u << list) - 1u))) & ~used;
        for (int r = 0; r < keep; ++r) {
            if (((pending >> r) & 1) == 0) continue;
            const int s = __builtin_ctz(free_slots);
            free_slots &= free_slots - 1u;
            const int p = __shfl(new_parent, r);
            const int src = phys[p];
            if (lane == r) new_slot = s;
            // copy what the new path will read of its parent: the node LLRs at
            // the depths d whose node holds leaf i in its left half (their
            // right child's g is still to come; the other depths are
            // rewritten before they are read), and the decisions 0 .. i-1
            for (int d = 1; d < n; ++d) {
                if ((i >> (n - 1 - d)) & 1) continue;
                const int off = depth_off(N, d), sz = N >> d;
                for (int e = lane; e < sz; e += 64) A[(size_t)s * N + off + e] = A[(size_t)src * N + off + e];
            }
            for (int e = lane; e <= (i >> 5); e += 64) U[(size_t)s * W + e] = U[(size_t)src * W + e];
        }
        // new slot table: ranks first, then the free slots
        uint32_t rest = free_slots;
        int slot_here = new_slot;
        for (int r = keep; r < list; ++r) {
            const int s = __builtin_ctz(rest);
            rest &= rest - 1u;
            if (lane == r) slot_here = s;
        }
        if (lane < list) phys[lane] = slot_here;
        if (lane < keep) {
            uint32_t* w = U + (size_t)slot_here * W + (i >> 5);
            *w = (*w & ~(1u << (i & 31))) | ((uint32_t)new_bit << (i & 31));
        }
        pm = lane < keep ? new_pm : 0.0f;
        active = keep;
    }

    // the path of least metric, ties to the lower index
    int best = 0;
    float best_pm = lane_readf(pm, 0);
    for (int k = 1; k < active; ++k) {
        const float o = lane_readf(pm, k);
        if (o < best_pm) {
            best_pm = o;
            best = k;
        }
    }
    const int sb = phys[best];
    const uint32_t low = N < 32 ? (1u << N) - 1u : 0xffffffffu;
    for (int e = lane; e < W; e += 64) fd.uhat[e] = U[(size_t)sb * W + e] & low;
    if (pm_out && lane == 0) pm_out[f] = best_pm;
}

}  // namespace

extern "C" size_t polar_scl_workspace_bytes(int n_frames) {
    if (n_frames < 0) return 0;
    return align256(256 + sizeof(FrameDesc) * (size_t)std::max(1, n_frames));
}

extern "C" int polar_scl_decode_batch(polar_ctx* c, const polar_frame* frames, int n_frames, int list_size,
                                      float* path_metric, void* stream) {
    TraceRange tr("polar_scl_decode_batch");
    if (!c) return fail(POLAR_E_INVAL, "ctx is NULL");
    if (list_size < 1 || list_size > POLAR_SCL_MAX_LIST)
        return fail(POLAR_E_INVAL, "list size %d outside 1..%d", list_size, POLAR_SCL_MAX_LIST);
    int rc = validate_frames(frames, n_frames);
    if (rc) return rc;
    int max_log = 0;
    for (int k = 0; k < n_frames; ++k) {
        const polar_frame& f = frames[k];
        if (f.f_kind != POLAR_F_MINSUM) return fail(POLAR_E_INVAL, "frame %d: list decoding uses min-sum only", k);
        if (f.leaf_llr) return fail(POLAR_E_INVAL, "frame %d: no leaf-LLR dump in list decoding", k);
        if (((int64_t)list_size << f.log2n) > POLAR_SCL_MAX_NL)
            return fail(POLAR_E_INVAL, "frame %d: N x list size %lld exceeds %d", k,
                        (long long)((int64_t)list_size << f.log2n), POLAR_SCL_MAX_NL);
        max_log = std::max(max_log, (int)f.log2n);
    }
    if (path_metric && ((uintptr_t)path_metric & 3)) return fail(POLAR_E_INVAL, "path_metric must be 4-byte aligned");
    if (n_frames == 0) return ok();
    const size_t need = polar_scl_workspace_bytes(n_frames);
    if (!c->ws || c->ws_bytes < need) return fail(POLAR_E_NOMEM, "workspace of %zu bytes < %zu required", c->ws_bytes, need);
    if (((uintptr_t)c->ws & 255) != 0) return fail(POLAR_E_INVAL, "workspace must be 256-byte aligned");
    DeviceGuard g(c->device);
    if (!g.ok) return fail(POLAR_E_DEVICE, "cannot select device %d", c->device);
    hipStream_t s = (hipStream_t)stream;
    std::vector<FrameDesc> d((size_t)n_frames);
    for (int k = 0; k < n_frames; ++k) {
        const polar_frame& f = frames[k];
        FrameDesc x{};
        x.llr = f.llr;
        x.mask = f.frozen_mask;
        x.vals = f.frozen_vals;
        x.uhat = f.u_hat;
        x.leaf = nullptr;
        x.log2n = f.log2n;
        x.fkind = f.f_kind;
        x.slot = nullptr;
        x.done_idx = 0xffffffffu;
        d[(size_t)k] = x;
    }
    FrameDesc* dtab = reinterpret_cast<FrameDesc*>((uint8_t*)c->ws + 256);
    rc = c->stager.upload(d.data(), d.size(), dtab, s);
    if (rc) return rc;
    // one wavefront per frame; LDS sized for the largest frame of the batch
    const size_t smem = scl_lds_bytes(max_log, list_size);
    if (smem > 160 * 1024) return fail(POLAR_E_INVAL, "list decoder needs %zu bytes of LDS", smem);
    if (smem > 65536) {
        hipError_t e = hipFuncSetAttribute((const void*)k_scl_decode, hipFuncAttributeMaxDynamicSharedMemorySize,
                                           (int)smem);
        if (e != hipSuccess) return hip_fail(e, "list decoder LDS size");
    }
    hipLaunchKernelGGL(k_scl_decode, dim3((unsigned)n_frames), dim3(64), smem, s, dtab, n_frames, list_size,
                       path_metric);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "list decoder launch");
    return ok();
}
