// Frozen-set construction by channel degradation, on the device.
//
// Section 3 freezes the synthetic channels of lowest capacity; the paper's
// frozen sets come from the density-evolution construction it cites [MT09].
// This file computes an upper bound on the error probability of every
// synthetic channel by carrying each one as a finite binary-input symmetric
// channel and degrading it to at most mu outputs after every polarization
// step (Tal and Vardy, "How to construct polar codes", IEEE Trans. IT 2013),
// merging outputs by binning them on the binary entropy of their posterior
// (Pedarsani, Hassani, Tal and Telatar, ISIT 2011).
//
// A channel is a list of output pairs (a, b), a >= b >= 0, a = W(y|0),
// b = W(y|1) for one output y of a conjugate pair, summing to 1; its error
// probability is the sum of the b.  Child 2c of channel c is its minus
// ("first decoded") channel and child 2c + 1 its plus channel; over the
// ordered output pairs (i, j) of the parent
//   minus  (a_i a_j + b_i b_j, a_i b_j + b_i a_j)              output i m + j
//   plus   (a_i a_j, b_i b_j)                                  output 2(i m + j)
//          (max(a_i b_j, b_i a_j), min(a_i b_j, b_i a_j))      output 2(i m + j) + 1
// Merge: an output with a + b > 0 goes to bin min(mu - 1, floor(mu h2(b / (a + b)))),
// each bin sums its outputs in output order, and the occupied bins are kept
// in ascending order.  Every product and sum is rounded on its own (the build
// disables contraction), so the result does not depend on the schedule.
//
// Layout: one wavefront per parent channel; lane k holds the accumulator of
// bin k of each child.  Outputs are formed one row i at a time (lane j: the
// pair (i, j)), then folded into their bins one lane after the other, which
// keeps every bin's sum in output order without atomics.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "host_internal.h"
#include "polar.h"

using namespace polar_host;

namespace {

__device__ __forceinline__ double lane_read(double x, int j) {
    const uint64_t u = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)u, j);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(u >> 32), j);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Bin of one output, or -1 for an output of zero mass.
__device__ __forceinline__ int bin_of(double a, double b, int mu) {
    const double tot = a + b;
    if (!(tot > 0.0)) return -1;
    const double q = b / tot;
    double h = 0.0;
    if (q > 0.0 && q < 1.0) h = (-q) * log2(q) - (1.0 - q) * log2(1.0 - q);
    const int k = (int)floor((double)mu * h);
    return k < mu - 1 ? k : mu - 1;
}

struct Acc {
    double a = 0.0, b = 0.0;
};

// Folds the outputs of lanes 0 .. count-1 (pair (oa, ob), bin) into the bin
// accumulators, lane order.
__device__ __forceinline__ void fold(Acc& acc, double oa, double ob, int bin, int count, int lane) {
    for (int j = 0; j < count; ++j) {
        const int bj = __builtin_amdgcn_readlane(bin, j);
        if (bj < 0) continue;
        const double xa = lane_read(oa, j), xb = lane_read(ob, j);
        if (lane == bj) {
            acc.a += xa;
            acc.b += xb;
        }
    }
}

// As fold, with two outputs per lane taken in the order (lane j first, lane j second).
__device__ __forceinline__ void fold2(Acc& acc, double pa, double pb, int bp, double qa, double qb, int bq,
                                      int count, int lane) {
    for (int j = 0; j < count; ++j) {
        const int b1 = __builtin_amdgcn_readlane(bp, j);
        if (b1 >= 0) {
            const double xa = lane_read(pa, j), xb = lane_read(pb, j);
            if (lane == b1) {
                acc.a += xa;
                acc.b += xb;
            }
        }
        const int b2 = __builtin_amdgcn_readlane(bq, j);
        if (b2 >= 0) {
            const double xa = lane_read(qa, j), xb = lane_read(qb, j);
            if (lane == b2) {
                acc.a += xa;
                acc.b += xb;
            }
        }
    }
}

// Stores a merged channel (occupied bins, ascending) and/or its error
// probability (the b of the occupied bins added in ascending order; an
// unoccupied bin adds +0, which leaves the sum unchanged).
__device__ __forceinline__ void emit(const Acc& acc, int mu, int lane, double2* out, int* out_cnt, double* pe,
                                     int64_t ch) {
    if (out) {
        const bool occ = lane < mu && (acc.a + acc.b) > 0.0;
        const uint64_t m = __ballot(occ);
        const int pos = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(m >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)m, 0u));
        if (occ) out[ch * mu + pos] = make_double2(acc.a, acc.b);
        if (lane == 0) out_cnt[ch] = __popcll(m);
    }
    if (pe) {
        double s = 0.0;
        for (int k = 0; k < mu; ++k) s += lane_read(acc.b, k);
        if (lane == 0) pe[ch] = s;
    }
}

// The channel at the root: w0 merged.  One wavefront.
__global__ __launch_bounds__(64) void k_merge_root(const double2* __restrict__ w0, int m0, int mu,
                                                   double2* __restrict__ out, int* __restrict__ out_cnt,
                                                   double* __restrict__ pe) {
    const int lane = threadIdx.x;
    Acc acc;
    for (int c0 = 0; c0 < m0; c0 += 64) {
        const int k = c0 + lane;
        double oa = 0.0, ob = 0.0;
        int bin = -1;
        if (k < m0) {
            const double2 v = w0[k];
            oa = v.x;
            ob = v.y;
            bin = bin_of(oa, ob, mu);
        }
        fold(acc, oa, ob, bin, min(64, m0 - c0), lane);
    }
    emit(acc, mu, lane, out, out_cnt, pe, 0);
}

// One polarization step of every channel of a level: parent c -> children 2c, 2c + 1.
// out == nullptr at the last level, where only the error probabilities are kept.
__global__ __launch_bounds__(256) void k_degrade_level(const double2* __restrict__ in, const int* __restrict__ in_cnt,
                                                      double2* __restrict__ out, int* __restrict__ out_cnt,
                                                      double* __restrict__ pe, int64_t n_par, int mu) {
    const int lane = threadIdx.x & 63;
    const int64_t wave0 = (int64_t)blockIdx.x * (blockDim.x >> 6) + __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int64_t n_waves = (int64_t)gridDim.x * (blockDim.x >> 6);
    for (int64_t c = wave0; c < n_par; c += n_waves) {
        const int m = __builtin_amdgcn_readfirstlane(in_cnt[c]);
        double wa = 0.0, wb = 0.0;
        if (lane < m) {
            const double2 v = in[c * mu + lane];
            wa = v.x;
            wb = v.y;
        }
        Acc am, ap;
        for (int i = 0; i < m; ++i) {
            const double ai = lane_read(wa, i), bi = lane_read(wb, i);
            double ma = 0.0, mb = 0.0, p1a = 0.0, p1b = 0.0, p2a = 0.0, p2b = 0.0;
            int bm = -1, b1 = -1, b2 = -1;
            if (lane < m) {
                ma = ai * wa + bi * wb;
                mb = ai * wb + bi * wa;
                p1a = ai * wa;
                p1b = bi * wb;
                const double x = ai * wb, y = bi * wa;
                p2a = x > y ? x : y;
                p2b = x > y ? y : x;
                bm = bin_of(ma, mb, mu);
                b1 = bin_of(p1a, p1b, mu);
                b2 = bin_of(p2a, p2b, mu);
            }
            fold(am, ma, mb, bm, m, lane);
            fold2(ap, p1a, p1b, b1, p2a, p2b, b2, m, lane);
        }
        emit(am, mu, lane, out, out_cnt, pe, 2 * c);
        emit(ap, mu, lane, out, out_cnt, pe, 2 * c + 1);
    }
}

// Workspace: w0 | level buffer 0 (2^(n-1) channels) | level buffer 1
// (2^(n-2) channels) | their output counts.  Level l lives in buffer
// (n - 1 - l) & 1, so the last stored level (n - 1) gets the larger buffer.
struct Layout {
    size_t w0, buf[2], cnt[2], total;
    int64_t cap[2];
};

Layout layout_of(int log2n, int mu, int m0) {
    Layout L{};
    L.cap[0] = log2n >= 1 ? ((int64_t)1 << (log2n - 1)) : 1;
    L.cap[1] = log2n >= 2 ? ((int64_t)1 << (log2n - 2)) : 1;
    L.w0 = 0;
    L.buf[0] = align256((size_t)m0 * sizeof(double2));
    L.buf[1] = align256(L.buf[0] + (size_t)L.cap[0] * (size_t)mu * sizeof(double2));
    L.cnt[0] = align256(L.buf[1] + (size_t)L.cap[1] * (size_t)mu * sizeof(double2));
    L.cnt[1] = align256(L.cnt[0] + (size_t)L.cap[0] * sizeof(int));
    L.total = align256(L.cnt[1] + (size_t)L.cap[1] * sizeof(int));
    return L;
}

bool args_ok(int log2n, int mu, int m0) {
    return log2n >= 0 && log2n <= POLAR_MAX_LOG2N && mu >= 2 && mu <= POLAR_CONSTRUCT_MAX_MU && m0 >= 1 &&
           m0 <= POLAR_CONSTRUCT_MAX_OUTPUTS;
}

}  // namespace

extern "C" size_t polar_construct_workspace_bytes(int log2n, int mu, int m0) {
    if (!args_ok(log2n, mu, m0)) return 0;
    return layout_of(log2n, mu, m0).total;
}

extern "C" int polar_construct_degrade(int log2n, const double* w0, int m0, int mu, void* workspace,
                                       size_t ws_bytes, double* pe, void* stream) {
    TraceRange tr("polar_construct_degrade");
    if (log2n < 0 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 0..%d", log2n, POLAR_MAX_LOG2N);
    if (mu < 2 || mu > POLAR_CONSTRUCT_MAX_MU) return fail(POLAR_E_INVAL, "mu %d outside 2..%d", mu, POLAR_CONSTRUCT_MAX_MU);
    if (m0 < 1 || m0 > POLAR_CONSTRUCT_MAX_OUTPUTS)
        return fail(POLAR_E_INVAL, "m0 %d outside 1..%d", m0, POLAR_CONSTRUCT_MAX_OUTPUTS);
    if (!w0 || !pe || !workspace) return fail(POLAR_E_INVAL, "NULL buffer");
    if (((uintptr_t)workspace & 255) != 0) return fail(POLAR_E_INVAL, "workspace must be 256-byte aligned");
    if (((uintptr_t)pe & 7) != 0) return fail(POLAR_E_INVAL, "pe must be 8-byte aligned");
    double sum = 0.0;
    for (int k = 0; k < m0; ++k) {
        const double a = w0[2 * k], b = w0[2 * k + 1];
        if (!(std::isfinite(a) && std::isfinite(b) && b >= 0.0 && a >= b))
            return fail(POLAR_E_INVAL, "w0 pair %d must satisfy a >= b >= 0", k);
        sum += a + b;
    }
    if (!(std::fabs(sum - 1.0) <= 1e-12)) return fail(POLAR_E_INVAL, "w0 must sum to 1 (sums to %.17g)", sum);
    const Layout L = layout_of(log2n, mu, m0);
    if (ws_bytes < L.total) return fail(POLAR_E_NOMEM, "workspace %zu bytes, need %zu", ws_bytes, L.total);

    hipStream_t s = (hipStream_t)stream;
    int dev = 0, n_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e == hipSuccess) e = hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return hip_fail(e, "device query");
    uint8_t* ws = (uint8_t*)workspace;
    double2* w0d = (double2*)(ws + L.w0);
    double2* buf[2] = {(double2*)(ws + L.buf[0]), (double2*)(ws + L.buf[1])};
    int* cnt[2] = {(int*)(ws + L.cnt[0]), (int*)(ws + L.cnt[1])};

    // w0 is the caller's (possibly pageable) memory: copy it and wait, so it
    // may be reused as soon as this call returns.
    e = hipMemcpyAsync(w0d, w0, (size_t)m0 * sizeof(double2), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "w0 upload");

    const int top = (log2n - 1) & 1;  // buffer of level 0 (n >= 1)
    hipLaunchKernelGGL(k_merge_root, dim3(1), dim3(64), 0, s, w0d, m0, mu, log2n >= 1 ? buf[top] : nullptr,
                       log2n >= 1 ? cnt[top] : nullptr, log2n == 0 ? pe : nullptr);
    for (int l = 0; l < log2n; ++l) {
        const int bi = (log2n - 1 - l) & 1, bo = bi ^ 1;
        const bool last = l == log2n - 1;
        const int64_t n_par = (int64_t)1 << l;
        const int64_t blocks = std::min<int64_t>((n_par + 3) / 4, (int64_t)n_cu * 16);
        hipLaunchKernelGGL(k_degrade_level, dim3((unsigned)blocks), dim3(256), 0, s, buf[bi], cnt[bi],
                           last ? nullptr : buf[bo], last ? nullptr : cnt[bo], last ? pe : nullptr, n_par, mu);
    }
    e = hipGetLastError();
    if (e != hipSuccess) return hip_fail(e, "construction launch");
    return ok();
}

extern "C" int polar_frozen_from_pe(int log2n, const double* pe, int64_t n_frozen, double fer_bound,
                                    uint32_t* frozen_mask, int64_t* n_frozen_out) {
    if (log2n < 0 || log2n > POLAR_MAX_LOG2N) return fail(POLAR_E_INVAL, "log2n %d outside 0..%d", log2n, POLAR_MAX_LOG2N);
    if (!pe || !frozen_mask) return fail(POLAR_E_INVAL, "NULL buffer");
    const int64_t n = (int64_t)1 << log2n;
    if (n_frozen > n || n_frozen < -1) return fail(POLAR_E_INVAL, "n_frozen %lld outside -1..N", (long long)n_frozen);
    if (n_frozen == -1 && !(fer_bound >= 0.0)) return fail(POLAR_E_INVAL, "fer_bound must be >= 0");
    for (int64_t i = 0; i < n; ++i)
        if (!(pe[i] >= 0.0 && pe[i] <= 1.0)) return fail(POLAR_E_INVAL, "pe[%lld] outside [0, 1]", (long long)i);

    // total order, least reliable first: descending error probability, ties by index
    std::vector<int64_t> idx((size_t)n);
    std::iota(idx.begin(), idx.end(), 0);
    auto worse = [&](int64_t a, int64_t b) { return pe[a] > pe[b] || (pe[a] == pe[b] && a < b); };
    int64_t nf = n_frozen;
    if (nf == -1) {
        std::sort(idx.begin(), idx.end(), worse);
        double sum = 0.0;
        int64_t k = 0;
        for (; k < n; ++k) {
            const double p = pe[idx[(size_t)(n - 1 - k)]];
            if (sum + p > fer_bound) break;
            sum += p;
        }
        nf = n - k;
    } else if (nf > 0 && nf < n) {
        std::nth_element(idx.begin(), idx.begin() + nf, idx.end(), worse);
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
