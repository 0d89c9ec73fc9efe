// Device code of libpolar: polar encoding and successive-cancellation (SC)
// decoding for gfx950 (CDNA4, wave64).
//
// SC decoding (Section 4 of the paper; Arikan's construction cited in
// Section 3) visits the binary tree of a length-N code depth first.  A node
// of size M with input LLRs alpha computes
//     alpha_L[j] = f(alpha[j], alpha[j + M/2])                 (left child)
//     alpha_R[j] = alpha[j + M/2] + (1 - 2 beta_L[j]) alpha[j]  (right child)
//     beta       = [beta_L ^ beta_R, beta_R]                    (partial sums)
// and a leaf decides u = frozen value, or [alpha < 0] for an information bit.
// Section 4 notes that SC is inherently sequential, so only parallelism
// across frames and across the elements of one node is available.  This file
// maps the tree onto the GPU as follows:
//
//   * one workgroup decodes one frame at a time, taking frames from a device
//     queue (persistent launch);
//   * nodes larger than 2^C (C <= 12) are processed by wide, coalesced sweeps
//     of the whole workgroup over HBM-resident LLR levels;
//   * every 2^C-leaf subtree is decoded by a single wavefront entirely in
//     registers: lane l holds elements k*64 + l, so for node sizes >= 128 the
//     pair (j, j + M/2) sits in one lane and f/g need no data movement;
//   * each 64-leaf block is decoded with one element per lane: the half
//     shift of a node of size M is a DPP row shift (M <= 16) or a gfx950
//     permlane16/32 swap (M = 32, 64), decisions come from a ballot, and the
//     partial sums live in one 64-bit scalar word;
//   * exact pruning: a node whose leaves are all frozen (rate 0) takes
//     beta = v G_M without any LLR work; a node without frozen leaves
//     (rate 1) takes beta from the sign / zero state of its LLRs by the
//     three-state rule, which equals SC even when LLRs are exactly zero.
//
// Arithmetic follows the FP32 definitions exactly (no FMA contraction is
// possible in min-sum: f is a min and a sign, g one addition), so the
// min-sum decoder is bit-exact against any correct FP32 implementation.

#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "sc_device.h"

namespace polar_dev {

// ---------------------------------------------------------------------------
// Cross-lane moves inside a wavefront.
//   lane_down<H>(x): lane l receives x from lane l + H
//   lane_up<H>(x):   lane l receives x from lane l - H
// Only lanes whose partner lies in the same aligned group of 2H lanes are
// meaningful; callers never read the others.  They must be called with the
// whole wavefront active (never inside a lane-divergent branch), since an
// inactive partner lane supplies no data.
// ---------------------------------------------------------------------------
template <int H>
__device__ __forceinline__ uint32_t lane_down(uint32_t x) {
    if constexpr (H <= 8) {
        // lanes without a source read 0 (bound_ctrl); the move can then be
        // folded into the instruction that consumes it
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x100 + H, 0xf, 0xf, true);
    } else if constexpr (H == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return r[1];
    } else {
        static_assert(H == 32, "lane distance");
        auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return r[1];
    }
}

template <int H>
__device__ __forceinline__ uint32_t lane_up(uint32_t x) {
    if constexpr (H <= 8) {
        return (uint32_t)__builtin_amdgcn_mov_dpp((int)x, 0x110 + H, 0xf, 0xf, true);
    } else if constexpr (H == 16) {
        auto r = __builtin_amdgcn_permlane16_swap(x, x, false, false);
        return r[0];
    } else {
        static_assert(H == 32, "lane distance");
        auto r = __builtin_amdgcn_permlane32_swap(x, x, false, false);
        return r[0];
    }
}

template <int H>
__device__ __forceinline__ float lane_downf(float x) {
    return __uint_as_float(lane_down<H>(__float_as_uint(x)));
}
template <int H>
__device__ __forceinline__ float lane_upf(float x) {
    return __uint_as_float(lane_up<H>(__float_as_uint(x)));
}
template <int H>
__device__ __forceinline__ uint64_t lane_down64(uint64_t x) {
    return (uint64_t)lane_down<H>((uint32_t)x) | ((uint64_t)lane_down<H>((uint32_t)(x >> 32)) << 32);
}
template <int H>
__device__ __forceinline__ uint64_t lane_up64(uint64_t x) {
    return (uint64_t)lane_up<H>((uint32_t)x) | ((uint64_t)lane_up<H>((uint32_t)(x >> 32)) << 32);
}

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

__device__ __forceinline__ uint64_t ballot(bool p) { return __builtin_amdgcn_ballot_w64(p); }

__device__ __forceinline__ uint32_t readlane(uint32_t x, int l) {
    return (uint32_t)__builtin_amdgcn_readlane((int)x, l);
}
__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
    return (uint64_t)readlane((uint32_t)x, l) | ((uint64_t)readlane((uint32_t)(x >> 32), l) << 32);
}

// Bits with (bit index & h) == 0, i.e. the lower half of every 2h block.
__host__ __device__ constexpr uint64_t low_mask64(int h) {
    return h == 1    ? 0x5555555555555555ull
           : h == 2  ? 0x3333333333333333ull
           : h == 4  ? 0x0F0F0F0F0F0F0F0Full
           : h == 8  ? 0x00FF00FF00FF00FFull
           : h == 16 ? 0x0000FFFF0000FFFFull
                     : 0x00000000FFFFFFFFull;
}

__host__ __device__ constexpr uint64_t ones64(int m) { return m >= 64 ? ~0ull : ((1ull << m) - 1ull); }

// x = u G_m on a word whose bit i is u_i, for a block of m <= 64 bits
// starting at bit 0: stage h applies x[j] ^= x[j + h] to the lower half of
// every 2h block.
__device__ __forceinline__ uint64_t word_transform(uint64_t x, int m) {
#pragma unroll
    for (int h = 1; h < 64; h <<= 1)
        if (h < m) x ^= (x >> h) & low_mask64(h);
    return x;
}

// Polar transform across the 64 lanes of a wavefront, applied independently
// to every bit position of a per-lane word: element index = lane.
__device__ __forceinline__ uint64_t lane_transform(uint64_t w) {
    const int l = lane_id();
    uint64_t p;
    p = lane_down64<1>(w);  if (!(l & 1))  w ^= p;
    p = lane_down64<2>(w);  if (!(l & 2))  w ^= p;
    p = lane_down64<4>(w);  if (!(l & 4))  w ^= p;
    p = lane_down64<8>(w);  if (!(l & 8))  w ^= p;
    p = lane_down64<16>(w); if (!(l & 16)) w ^= p;
    p = lane_down64<32>(w); if (!(l & 32)) w ^= p;
    return w;
}

// 64 x 64 bit-matrix transpose: on entry lane r holds row r (bit c = M[r][c]);
// on exit lane c holds column c (bit r = M[r][c]).  Cross-lane reads only see
// active lanes, so both partners are fetched with the whole wave active and
// the result is selected afterwards.
template <int S>
__device__ __forceinline__ uint64_t transpose_stage(uint64_t w) {
    const uint64_t m = low_mask64(S);
    const uint64_t pu = lane_up64<S>(w);
    const uint64_t pd = lane_down64<S>(w);
    const uint64_t from_lo = (w & ~m) | ((pu >> S) & m);  // lanes with bit S set
    const uint64_t from_hi = (w & m) | ((pd << S) & ~m);  // lanes with bit S clear
    return (lane_id() & S) ? from_lo : from_hi;
}
__device__ __forceinline__ uint64_t transpose64(uint64_t w) {
    w = transpose_stage<32>(w);
    w = transpose_stage<16>(w);
    w = transpose_stage<8>(w);
    w = transpose_stage<4>(w);
    w = transpose_stage<2>(w);
    w = transpose_stage<1>(w);
    return w;
}

// ---------------------------------------------------------------------------
// LLR updates.
// ---------------------------------------------------------------------------
// Min-sum check update: sign(a) sign(b) min(|a|, |b|), signs from the IEEE
// sign bits.
__device__ __forceinline__ float f_minsum(float a, float b) {
    float m = fminf(fabsf(a), fabsf(b));
    uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(m) | s);
}

// Exact check update 2 atanh(tanh(a/2) tanh(b/2)) (the phi = log tanh(x/2)
// form of Section 4) in FP32, on magnitudes A = |a|, B = |b|, m = min(A, B):
//   m <= 1:  r = log1p(2t / (1 - t)),  t = tanh(A/2) tanh(B/2) <= tanh(1/2)^2,
//            which with tanh(x/2) = E / (E + 2), E = expm1(x), is exactly
//            r = log1p(Ea Eb / (Ea + Eb + 2))  (no 1 - t cancellation);
//   m >  1:  r = m + log1p(e^-(A+B)) - log1p(e^-|A-B|)   (r >= 1 - ln 2).
// Each form is accurate where it is selected.  Everything is straight-line
// code on the hardware exp2 / log2 / reciprocal (no library calls, no IEEE
// division sequence: the reciprocal is within 1 ulp, far inside the 1e-5
// LLR tolerance): both forms are evaluated and one is selected, so the
// wavefront never diverges here (the decoder's ballots and lane shifts need a
// fully active wavefront).
__device__ __forceinline__ float hw_exp(float x) {   // e^x
    return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
}
__device__ __forceinline__ float hw_log(float x) {   // ln x
    return __builtin_amdgcn_logf(x) * 0.693147180559945309f;
}
__device__ __forceinline__ float hw_rcp(float x) {   // 1 / x, normal x
    return __builtin_amdgcn_rcpf(x);
}
// expm1(x) for x >= 0: Taylor series to x^9/9! below 1/2 (truncation error
// < 3e-9 relative), e^x - 1 above (no cancellation there).
__device__ __forceinline__ float expm1_pos(float x) {
    float p = 1.0f / 362880.0f;
    p = fmaf(p, x, 1.0f / 40320.0f);
    p = fmaf(p, x, 1.0f / 5040.0f);
    p = fmaf(p, x, 1.0f / 720.0f);
    p = fmaf(p, x, 1.0f / 120.0f);
    p = fmaf(p, x, 1.0f / 24.0f);
    p = fmaf(p, x, 1.0f / 6.0f);
    p = fmaf(p, x, 0.5f);
    p = fmaf(p, x, 1.0f);
    const float small = p * x;
    const float large = hw_exp(x) - 1.0f;
    return x < 0.5f ? small : large;
}
// log1p(z) for z >= 0 (Goldberg: ln(u) z / (u - 1) with u = 1 + z).
__device__ __forceinline__ float log1p_pos(float z) {
    const float u = 1.0f + z;
    const float d = u - 1.0f;
    const float r = hw_log(u) * (z * hw_rcp(d));  // d = 0 or d >= 2^-24: normal
    return d == 0.0f ? z : r;
}
// The two forms on magnitudes A, B.  tanh form: argument clamped (tanh(x/2)
// is 1 in FP32 beyond x = 40).
__device__ __forceinline__ float boxplus_tanh_form(float A, float B) {
    const float ea = expm1_pos(fminf(A, 40.0f));
    const float eb = expm1_pos(fminf(B, 40.0f));
    return log1p_pos(ea * eb * hw_rcp(ea + eb + 2.0f));
}
__device__ __forceinline__ float boxplus_log_form(float A, float B) {
    return fminf(A, B) + log1p_pos(hw_exp(-(A + B))) - log1p_pos(hw_exp(-fabsf(A - B)));
}
__device__ __forceinline__ float f_boxplus(float a, float b) {
    const float A = fabsf(a), B = fabsf(b);
    const float m = fminf(A, B);
    const float r_small = boxplus_tanh_form(A, B);
    const float r_large = boxplus_log_form(A, B);
    const float r = (m <= 1.0f) ? r_small : r_large;
    const uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(r) | s);
}
// The same update on the lanes of one node of the block decoder (lanes: the
// lanes whose result is used; the wavefront is fully active there).  The
// tanh form is evaluated only when one of those lanes selects it, so a node
// whose smaller inputs all exceed 1 pays for the log form alone.  (Skipping
// the log form too where every lane selects the tanh form measured slower.)
// Results on those lanes are f_boxplus's.
__device__ __forceinline__ float f_boxplus_on(float a, float b, uint64_t lanes) {
    const float A = fabsf(a), B = fabsf(b);
    const float m = fminf(A, B);
    float r = boxplus_log_form(A, B);
    if ((ballot(m <= 1.0f) & lanes) != 0) {
        const float r_small = boxplus_tanh_form(A, B);
        r = (m <= 1.0f) ? r_small : r;
    }
    const uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(r) | s);
}

// Fixed point (Section 4: the paper's decoder keeps LLRs in fixed point and
// takes the check update from a table of phi(x) = -ln tanh(x/2), its main
// optimization).  LLRs are integers in units of 2^-4, saturated to +-32767,
// held in FP32 registers (exact: every value is an integer below 2^24, and
// min, add and compare of such floats are the integer operations).
//   FK = 2, saturating min-sum:  f = sign(a) sign(b) min(|a|, |b|)
//   FK = 3, phi table:           f = sign(a) sign(b) min(T[min(T[|a|] + T[|b|], 255)], |a|, |b|)
//                                (T[i] = 0 from i = 67 on, so beyond the table
//                                the lookup is 0; the min with |a|, |b| holds
//                                because the exact update never exceeds either
//                                magnitude, and stands in for T[0] = phi(0))
//   both: g = sat(b + (1 - 2u) a)
constexpr float FIXED_MAX = 32767.0f;
constexpr int PHI_LEN = 256;

// FK = 4, saturating min-sum on 8-bit integers: f as FK = 2, g saturated to
// +-127 (values in whatever units the caller quantized to: min-sum is the same
// at every scale but for the saturation).
constexpr float FIXED8_MAX = 127.0f;

// Kinds whose check update is min-sum (FP32, and both saturating kinds).
template <int FK>
constexpr bool minsum_kind() { return FK == 0 || FK == 2 || FK == 4; }

template <int FK>
constexpr float fixed_max() { return FK == 4 ? FIXED8_MAX : FIXED_MAX; }

// The workgroup's copy of T (kernels with FK = 3 only: LDS is allocated only
// in kernels that use it).
static __shared__ float g_phi[PHI_LEN];

// T[i] = round(phi(i / 16) * 16) (half up), capped at 32767, T[0] = 32767,
// with phi(x) = log1p(2 / expm1(x)) (the same function as -ln tanh(x/2),
// without cancellation for large x), in FP64.  Every thread of the workgroup
// must call it; the caller synchronises before use.
__device__ __forceinline__ void phi_table_init() {
    for (int i = (int)threadIdx.x; i < PHI_LEN; i += (int)blockDim.x) {
        float t = FIXED_MAX;
        if (i > 0) {
            const double r = floor(log1p(2.0 / expm1((double)i * 0.0625)) * 16.0 + 0.5);
            t = r > 32767.0 ? FIXED_MAX : (float)r;
        }
        g_phi[i] = t;
    }
}

__device__ __forceinline__ float f_phi(float a, float b) {
    const float A = fabsf(a), B = fabsf(b);
    const float m = fminf(A, B);
    const int ia = min((int)A, PHI_LEN - 1), ib = min((int)B, PHI_LEN - 1);
    const int is = (int)fminf(g_phi[ia] + g_phi[ib], (float)(PHI_LEN - 1));
    const float r = fminf(g_phi[is], m);
    const uint32_t s = (__float_as_uint(a) ^ __float_as_uint(b)) & 0x80000000u;
    return __uint_as_float(__float_as_uint(r) | s);
}

template <int FK>
__device__ __forceinline__ float fupd(float a, float b) {
    if constexpr (minsum_kind<FK>()) return f_minsum(a, b);
    else if constexpr (FK == 1) return f_boxplus(a, b);
    else return f_phi(a, b);
}

// f whose result is used on the given lanes only (the block decoder's nodes).
template <int FK>
__device__ __forceinline__ float fupd_on(float a, float b, uint64_t lanes) {
    if constexpr (FK == 1) return f_boxplus_on(a, b, lanes);
    else return fupd<FK>(a, b);
}

// The variable update's sum, saturated for the fixed-point kinds.
template <int FK>
__device__ __forceinline__ float gsat(float x) {
    if constexpr (FK >= 2) return __builtin_amdgcn_fmed3f(x, -fixed_max<FK>(), fixed_max<FK>());
    else return x;
}

// g = b + (1 - 2u) a with the sign of a flipped by sgn (0 or 0x80000000).
template <int FK>
__device__ __forceinline__ float gupd(float a, float b, uint32_t sgn) {
    return gsat<FK>(b + __uint_as_float(__float_as_uint(a) ^ sgn));
}

// Rate-1 nodes (no frozen leaf).  In a rate-1 node SC's partial sums equal
// the hard decisions of the node's LLRs whenever no LLR anywhere inside the
// node is zero: f keeps the sign product, and g = b + (1 - 2u) a then adds
// two terms of the sign of b.  (With exact zeros the hard decision is not SC:
// alpha = (0, -1) gives x-hat = (1, 1).)
//   min-sum: an LLR inside the node is zero only if the node has an input
//            that is zero, so "no input LLR is zero" suffices (floor 0);
//   box-plus: f of small inputs is tiny (f(x, x) ~ x^2 / 2) and can round
//            to zero.  f grows with both magnitudes and g adds them in a
//            rate-1 node, so the smallest LLR of a node of size 2^L whose
//            inputs are all at least F is at least f applied L times along
//            the left spine, x -> f(x, x) from F.  The floor F_L is the
//            least F (rounded up) for which that exceeds 1e-5 in exact
//            arithmetic: then every exact LLR of the node is at least 1e-5
//            with the sign the hard decisions assume, so SC decides them
//            (in exact arithmetic, in the FP64 reference, and in FP32, whose
//            deviation stays far inside the margin).
// Below the floor the decoder descends into the node like any other, which
// is SC by construction; its children are checked again.
//   saturating min-sum (FK = 2, 4): as min-sum (a saturated sum of two terms
//            of the sign of b keeps that sign and is nonzero);
//   phi table (FK = 3): the update can round a nonzero result to 0 (f of
//            1 and -1 is -0), but T[i] = 0 for every i >= 67 (phi(67/16) 16
//            = 0.486 rounds to 0), so for |a|, |b| >= 67 the sum of lookups
//            is 0 and the update is min(T[0], |a|, |b|) = min(|a|, |b|): f is
//            min-sum there and keeps the bound, as g does, so inputs of 67
//            and above (floor 66, any L) make the hard decisions SC.  67 is
//            the least bound closed under f: T[T[66] + T[66]] = T[2] = 44.
constexpr float BOXPLUS_FLOOR[13] = {0.0f,  0.01f, 0.10f, 0.45f, 1.02f, 1.68f, 2.37f,
                                     3.06f, 3.75f, 4.44f, 5.13f, 5.83f, 6.52f};

template <int FK>
__host__ __device__ constexpr float rate1_floor(int L) {
    return minsum_kind<FK>()    ? 0.0f
           : FK == 1            ? BOXPLUS_FLOOR[L]
                                : 66.0f;
}

// |x| <= floor, evaluated on the magnitude bits (non-negative floats order
// like their bit patterns), as one integer compare against a literal.
template <int FK, int L>
__device__ __forceinline__ bool below_rate1_floor(float x) {
    constexpr uint32_t fb = __builtin_bit_cast(uint32_t, rate1_floor<FK>(L));
    return (__float_as_uint(x) & 0x7fffffffu) <= fb;
}

__device__ __forceinline__ bool lane_bit(uint64_t mask) { return __builtin_amdgcn_inverse_ballot_w64(mask); }

// ---------------------------------------------------------------------------
// 64-leaf block decoder.  The node of size M at lane offset O holds its LLRs
// in lanes [O, O + M) of a single VGPR.  Partial sums are kept per lane as a
// sign word (0 or 0x80000000), so f, g and the combine are pure vector code:
//   f:       a_L = f(a, down_H(a))
//   g:       a_R = a + up_H(a ^ beta)      (beta of the left child flips a_lo)
//   combine: beta[j] ^= beta[j + H] for j in [O, O + H)
// The node type (rate 0, rate 1, repetition, mixed) is a function of the
// block's frozen mask alone, so it is decided on the scalar unit without
// waiting for vector results; only the rate-1 floor test and the repetition
// decision read a ballot.
// ---------------------------------------------------------------------------
constexpr uint32_t SIGN = 0x80000000u;

template <int M>
constexpr int ilog2() { return M <= 1 ? 0 : 1 + ilog2<M / 2>(); }

struct Blk {
    uint64_t F;       // frozen mask of the block (bit i = leaf i), wave-uniform
    uint64_t V;       // frozen values of the block (zero outside F), wave-uniform
    uint32_t fv;      // lane i: SIGN if leaf i is frozen with value 1
    uint32_t w[7];    // lane i: SIGN if bit i of the frozen values re-encoded
                      // inside every aligned 2^t-block (w[0] = fv)
    uint32_t beta;    // lane i: partial sum of element i, as a sign word
    float leaf;       // lane i: decision LLR of leaf i
    bool has_leaf;    // lane i: leaf i was reached (not inside a pruned node)
};

// Decision of a leaf as a sign word: SIGN iff a < 0, so that -0 decides 0.
// Integer form: a & (a - 1) has its sign bit set exactly for negative nonzero
// a; no compare, so no scalar mask and no wait before the select.
__device__ __forceinline__ uint32_t dec_sign(float a) {
    const uint32_t b = __float_as_uint(a);
    return b & (b - 1u) & SIGN;
}

__device__ __forceinline__ uint32_t sel_lanes(uint64_t lanes, uint32_t x, uint32_t y) {
    return lane_bit(lanes) ? x : y;
}

// Repetition node: every leaf frozen except the last.  SC never needs the
// f values here (the frozen decisions do not read LLRs): the last leaf's LLR
// is the chain of g updates down the right spine, each left sibling of size h
// being a rate-0 node whose partial sums are w[log h] on its lanes.  The node's
// partial sums are the frozen values re-encoded (w[log M]), all flipped when
// the last bit is 1 (row M-1 of G_M is all ones).
template <int H, int M, int FK>
__device__ __forceinline__ float rep_chain(float x, const Blk& B) {
    if constexpr (H == 0) {
        return x;
    } else {
        const float y = gsat<FK>(x + __uint_as_float(lane_up<H>(__float_as_uint(x) ^ B.w[ilog2<H>()])));
        return rep_chain<H / 2, M, FK>(y, B);
    }
}

template <int M, int FK, bool DUMP>
__device__ __forceinline__ void rep_node(float a, int O, Blk& B) {
    const float last = rep_chain<M / 2, M, FK>(a, B);
    const int il = O + M - 1;
    if (DUMP && lane_id() == il) {
        B.leaf = last;
        B.has_leaf = true;
    }
    const bool u = (ballot(last < 0.0f) >> il) & 1ull;
    B.beta = sel_lanes(ones64(M) << O, B.w[ilog2<M>()] ^ (u ? SIGN : 0u), B.beta);
}

// ---------------------------------------------------------------------------
// Small nodes with a known frozen pattern.  Moving a 1 of a channel index to
// a less significant place, or dropping it, never lowers the Bhattacharyya
// parameter, so in a code built from those parameters the frozen pattern of
// every aligned node is closed under that order: an 8-leaf node has one of
// only ten patterns.  Such a node is decoded by straight-line code generated
// for its pattern at compile time (no per-node type tests, no loop); any
// other pattern takes the generic path below.
// ---------------------------------------------------------------------------
#ifndef POLAR_SPEC_M
#define POLAR_SPEC_M 16
#endif
constexpr int SPEC_M = POLAR_SPEC_M;
static_assert(SPEC_M == 8 || SPEC_M == 16, "specialized node size");

template <int M>
constexpr uint32_t ones32() { return M >= 32 ? ~0u : (1u << M) - 1u; }

// Rate-1 node under min-sum: partial sums from the sign (S) and exact-zero
// (Z) words of its LLRs by the three-state recursion
//   left:  S_L = S_lo ^ S_hi,  Z_L = Z_lo | Z_hi
//   right: Z_R = Z_lo & Z_hi,  S_R = Z_hi ? (S_lo ^ beta_L) : S_hi
//   beta = [beta_L ^ beta_R, beta_R];  no zeros: beta = S
// (hard decisions alone are not SC once an LLR is exactly zero).
template <int M, bool CHECK = true>
__device__ __forceinline__ uint32_t r1_bits(uint32_t S, uint32_t Z) {
    if constexpr (M == 1) {
        return S & ~Z & 1u;
    } else {
        if (CHECK && Z == 0) return S;
        // children of 4 leaves or fewer take no zero test: straight-line
        // scalar code is cheaper there than the branches
        constexpr bool SUB = M > 4;
        constexpr int H = M / 2;
        constexpr uint32_t LO = ones32<H>();
        const uint32_t bl = r1_bits<H, SUB>((S ^ (S >> H)) & LO, (Z | (Z >> H)) & LO);
        const uint32_t zhi = Z >> H, shi = S >> H;
        const uint32_t zr = Z & zhi & LO;
        const uint32_t sr = ((zhi & (S ^ bl)) | (~zhi & shi)) & LO;
        const uint32_t br = r1_bits<H, SUB>(sr, zr);
        return (bl ^ br) | (br << H);
    }
}

// Lanes whose index has bit H clear: the left halves of all aligned nodes of
// size 2H.
template <int H>
constexpr uint64_t left_lanes() {
    uint64_t m = 0;
    for (int l = 0; l < 64; ++l)
        if ((l & H) == 0) m |= 1ull << l;
    return m;
}

// Node of size M at lane offset O with frozen pattern P (bit j = leaf j
// frozen).  Returns the node's partial sums as sign words, meaningful on the
// node's lanes [O, O + M) only: values on other lanes are left undefined, so
// leaves and rate-0 / repetition nodes need no lane selects, and a combine
// picks its halves with a constant lane mask.  Decisions stay in vector
// registers except where a ballot is inherent (rate-1 zero test, repetition
// decision).
template <int M, uint64_t P, int FK, bool DUMP>
__device__ __forceinline__ uint32_t sl_node(float a, int O, Blk& B) {
    constexpr uint64_t ALL = ones64(M);
    constexpr int LG = ilog2<M>();
    if constexpr (P == ALL) {
        return B.w[LG];  // rate 0 (a frozen leaf: its revealed value)
    } else if constexpr (M == 1) {
        if (DUMP && lane_id() == O) {
            B.leaf = a;
            B.has_leaf = true;
        }
        return dec_sign(a);
    } else if constexpr (P == 0 && minsum_kind<FK>() && M > 2) {
        // (a 2-leaf rate-1 node is cheaper as plain f, g and two decisions
        // in vector registers than as two ballots and a scalar round trip)
        static_assert(M <= 32, "three-state words are 32 bits");
        const uint32_t S = (uint32_t)((ballot(a < 0.0f) >> O) & ALL);
        const uint32_t Z = (uint32_t)((ballot(a == 0.0f) >> O) & ALL);
        const uint64_t bits = (uint64_t)r1_bits<M>(S, Z) << O;
        return lane_bit(bits) ? SIGN : 0u;
    } else if constexpr (P == 0 && (FK == 1 || FK == 3) && M >= 2) {
        // the exact updates have no three-state rule: hard decisions when no
        // input is at or under the floor, else the node's plain recursion
        constexpr int H = M / 2;
        const uint64_t low = ballot(below_rate1_floor<FK, LG>(a));
        uint32_t bn;
        if (((low >> O) & ALL) == 0) {
            bn = dec_sign(a);
        } else {
            const float c = fupd_on<FK>(a, lane_downf<H>(a), ones64(H) << O);
            const uint32_t bl = sl_node<H, 0, FK, DUMP>(c, O, B);
            const float d = gsat<FK>(a + __uint_as_float(lane_up<H>(__float_as_uint(a) ^ bl)));
            const uint32_t br = sl_node<H, 0, FK, DUMP>(d, O + H, B);
            bn = sel_lanes(left_lanes<H>(), bl ^ lane_down<H>(br), br);
        }
        return bn;
    } else if constexpr (P == (ALL >> 1)) {
        const float last = rep_chain<M / 2, M, FK>(a, B);  // repetition
        const int il = O + M - 1;
        if (DUMP && lane_id() == il) {
            B.leaf = last;
            B.has_leaf = true;
        }
        const uint32_t u = (uint32_t)(ballot(last < 0.0f) >> il) & 1u;
        return B.w[LG] ^ (u << 31);
    } else {
        constexpr int H = M / 2;
        constexpr uint64_t LO = ones64(H);
        const float c = fupd_on<FK>(a, lane_downf<H>(a), ones64(H) << O);
        const uint32_t bl = sl_node<H, (P & LO), FK, DUMP>(c, O, B);
        const float d = gsat<FK>(a + __uint_as_float(lane_up<H>(__float_as_uint(a) ^ bl)));
        const uint32_t br = sl_node<H, (P >> H), FK, DUMP>(d, O + H, B);
        return sel_lanes(left_lanes<H>(), bl ^ lane_down<H>(br), br);
    }
}

template <int M, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void blk_generic(float a, int O, Blk& B);

// Size-SPEC_M node: straight-line code for each closed pattern (10 of 8
// leaves, 27 of 16 leaves).
template <int FK, bool DUMP>
__device__ __forceinline__ uint32_t spec_local(float a, int O, Blk& B) {
    constexpr int M = SPEC_M;
    const uint32_t p = (uint32_t)(B.F >> O) & ones32<M>();
    uint32_t bn;
    if constexpr (M == 16) {
        // Two levels: the five patterns that make up over 90% of the 16-leaf
        // nodes of Bhattacharyya-built codes first, then the rest.  The
        // selector of the second switch is made opaque so that the compiler
        // does not fold both into one deeper branch tree (a data-dependent
        // multiway branch is a chain of scalar tests and taken branches).
        switch (p) {
            case 0x177f: bn = sl_node<M, 0x177f, FK, DUMP>(a, O, B); break;
            case 0x117: bn = sl_node<M, 0x117, FK, DUMP>(a, O, B); break;
            case 0x1: bn = sl_node<M, 0x1, FK, DUMP>(a, O, B); break;
            case 0x7fff: bn = sl_node<M, 0x7fff, FK, DUMP>(a, O, B); break;
            case 0x0: bn = sl_node<M, 0x0, FK, DUMP>(a, O, B); break;
            default: {
                uint32_t q = __builtin_amdgcn_readfirstlane(p);
                asm volatile("" : "+s"(q));
                switch (q) {
                    case 0x3: bn = sl_node<M, 0x3, FK, DUMP>(a, O, B); break;
                    case 0x7: bn = sl_node<M, 0x7, FK, DUMP>(a, O, B); break;
                    case 0xf: bn = sl_node<M, 0xf, FK, DUMP>(a, O, B); break;
                    case 0x17: bn = sl_node<M, 0x17, FK, DUMP>(a, O, B); break;
                    case 0x1f: bn = sl_node<M, 0x1f, FK, DUMP>(a, O, B); break;
                    case 0x3f: bn = sl_node<M, 0x3f, FK, DUMP>(a, O, B); break;
                    case 0x7f: bn = sl_node<M, 0x7f, FK, DUMP>(a, O, B); break;
                    case 0xff: bn = sl_node<M, 0xff, FK, DUMP>(a, O, B); break;
                    case 0x11f: bn = sl_node<M, 0x11f, FK, DUMP>(a, O, B); break;
                    case 0x13f: bn = sl_node<M, 0x13f, FK, DUMP>(a, O, B); break;
                    case 0x17f: bn = sl_node<M, 0x17f, FK, DUMP>(a, O, B); break;
                    case 0x1ff: bn = sl_node<M, 0x1ff, FK, DUMP>(a, O, B); break;
                    case 0x33f: bn = sl_node<M, 0x33f, FK, DUMP>(a, O, B); break;
                    case 0x37f: bn = sl_node<M, 0x37f, FK, DUMP>(a, O, B); break;
                    case 0x3ff: bn = sl_node<M, 0x3ff, FK, DUMP>(a, O, B); break;
                    case 0x77f: bn = sl_node<M, 0x77f, FK, DUMP>(a, O, B); break;
                    case 0x7ff: bn = sl_node<M, 0x7ff, FK, DUMP>(a, O, B); break;
                    case 0xfff: bn = sl_node<M, 0xfff, FK, DUMP>(a, O, B); break;
                    case 0x17ff: bn = sl_node<M, 0x17ff, FK, DUMP>(a, O, B); break;
                    case 0x1fff: bn = sl_node<M, 0x1fff, FK, DUMP>(a, O, B); break;
                    case 0x3fff: bn = sl_node<M, 0x3fff, FK, DUMP>(a, O, B); break;
                    case 0xffff: bn = sl_node<M, 0xffff, FK, DUMP>(a, O, B); break;
                    default:
                        blk_generic<M, FK, true, DUMP>(a, O, B);
                        bn = B.beta;
                        break;
                }
                break;
            }
        }
    } else {
        switch (p) {
            case 0x0: bn = sl_node<M, 0x0, FK, DUMP>(a, O, B); break;
            case 0x1: bn = sl_node<M, 0x1, FK, DUMP>(a, O, B); break;
            case 0x3: bn = sl_node<M, 0x3, FK, DUMP>(a, O, B); break;
            case 0x7: bn = sl_node<M, 0x7, FK, DUMP>(a, O, B); break;
            case 0xf: bn = sl_node<M, 0xf, FK, DUMP>(a, O, B); break;
            case 0x17: bn = sl_node<M, 0x17, FK, DUMP>(a, O, B); break;
            case 0x1f: bn = sl_node<M, 0x1f, FK, DUMP>(a, O, B); break;
            case 0x3f: bn = sl_node<M, 0x3f, FK, DUMP>(a, O, B); break;
            case 0x7f: bn = sl_node<M, 0x7f, FK, DUMP>(a, O, B); break;
            case 0xff: bn = sl_node<M, 0xff, FK, DUMP>(a, O, B); break;
            default:
                blk_generic<M, FK, true, DUMP>(a, O, B);
                bn = B.beta;
                break;
        }
    }
    return bn;
}

template <int FK, bool DUMP>
__device__ __forceinline__ void blk_spec(float a, int O, Blk& B) {
    const uint32_t bn = spec_local<FK, DUMP>(a, O, B);
    B.beta = sel_lanes(ones64(SPEC_M) << O, bn, B.beta);
}

// Node of size M at lane offset O (runtime), used at 32 and 64 leaves (and
// for patterns outside the specialized set).  The two children are visited
// by an unrolled two-pass loop: the pattern-specialized 16-leaf code is then
// inlined four times per block, which measured faster than the rolled loop's
// branches despite the larger code.
//
// Both ballots of a node are taken unconditionally at its top and only read
// inside the shortcut branches: with a ballot placed under the rate-1 test
// (or an early return nested in that test) this toolchain's -O2/-O3 code
// returned corrupted partial sums after a failed test, exact at -O1.
// The most frequent mixed 64- and 32-leaf patterns of Bhattacharyya-built
// codes (each a composition of frequent 16-leaf patterns) get straight-line
// code too: one dispatch replaces the generic node's type test and the
// dispatches of its children.  Other patterns take the generic node.
template <int M, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void blk_node(float a, int O, Blk& B) {
    // (64-leaf cases only for min-sum without the leaf dump: with box-plus's
    // longer f, or the dump, they exceed the register budget)
    if constexpr (PRUNE && M == 64 && minsum_kind<FK>() && !DUMP) {
        uint32_t bn;
        bool known = true;
        switch (B.F) {
            case 0x177f7fff7fffffffull: bn = sl_node<64, 0x177f7fff7fffffffull, FK, DUMP>(a, 0, B); break;
            case 0x0117177f177f7fffull: bn = sl_node<64, 0x0117177f177f7fffull, FK, DUMP>(a, 0, B); break;
            case 0x000101170117177full: bn = sl_node<64, 0x000101170117177full, FK, DUMP>(a, 0, B); break;
            case 0x0000000100010117ull: bn = sl_node<64, 0x0000000100010117ull, FK, DUMP>(a, 0, B); break;
            case 0x0000000000000001ull: bn = sl_node<64, 0x0000000000000001ull, FK, DUMP>(a, 0, B); break;
            case 0x7fffffffffffffffull: bn = sl_node<64, 0x7fffffffffffffffull, FK, DUMP>(a, 0, B); break;
            default: known = false; bn = 0; break;
        }
        if (known) B.beta = bn;
        else blk_generic<M, FK, PRUNE, DUMP>(a, O, B);
    } else if constexpr (PRUNE && M == 32) {
        uint32_t bn;
        bool known = true;
        switch ((uint32_t)(B.F >> O)) {
            case 0x177f7fffu: bn = sl_node<32, 0x177f7fffu, FK, DUMP>(a, O, B); break;
            case 0x0117177fu: bn = sl_node<32, 0x0117177fu, FK, DUMP>(a, O, B); break;
            case 0x00010117u: bn = sl_node<32, 0x00010117u, FK, DUMP>(a, O, B); break;
            case 0x00000001u: bn = sl_node<32, 0x00000001u, FK, DUMP>(a, O, B); break;
            case 0x7fffffffu: bn = sl_node<32, 0x7fffffffu, FK, DUMP>(a, O, B); break;
            case 0xffffffffu: bn = sl_node<32, 0xffffffffu, FK, DUMP>(a, O, B); break;
            case 0x00000000u: bn = sl_node<32, 0x00000000u, FK, DUMP>(a, O, B); break;
            default: known = false; bn = 0; break;
        }
        if (known) B.beta = sel_lanes(ones64(32) << O, bn, B.beta);
        else blk_generic<M, FK, PRUNE, DUMP>(a, O, B);
    } else if constexpr (PRUNE && M == SPEC_M) {
        blk_spec<FK, DUMP>(a, O, B);
    } else {
        blk_generic<M, FK, PRUNE, DUMP>(a, O, B);
    }
}

template <int M, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void blk_generic(float a, int O, Blk& B) {
    if constexpr (M == 1) {
        if (DUMP && lane_id() == O) {
            B.leaf = a;
            B.has_leaf = true;
        }
        // frozen: the revealed value; information bit: [alpha < 0].  Lane O
        // reads its own frozen bit, so the choice is a lane select.
        const uint32_t d = lane_bit(B.F) ? B.fv : dec_sign(a);
        B.beta = sel_lanes(1ull << O, d, B.beta);
    } else {
        constexpr int LG = ilog2<M>();
        int type = 0;
        uint64_t low = 0;
        if constexpr (PRUNE) {
            low = ballot(below_rate1_floor<FK, LG>(a));
            // node type from its frozen pattern: 1 rate 0, 2 rate 1, 3 repetition
            const uint64_t fm = (B.F >> O) & ones64(M);
            type = fm == ones64(M) ? 1 : fm == 0 ? 2 : fm == (ones64(M) >> 1) ? 3 : 0;
            // rate-1 node with an LLR at or under the floor (an exact zero
            // under min-sum): hard decisions need not be SC there, decode it
            if (type == 2 && (low & (ones64(M) << O)) != 0) type = 0;
        }
        if (type == 0) {
            constexpr int H = M / 2;
#pragma unroll
            for (int side = 0; side < 2; ++side) {
                float c;
                if (side == 0) {
                    c = fupd_on<FK>(a, lane_downf<H>(a), ones64(H) << O);  // left child, lanes [O, O + H)
                } else {
                    c = gsat<FK>(a + __uint_as_float(lane_up<H>(__float_as_uint(a) ^ B.beta)));  // right child
                }
                blk_node<H, FK, PRUNE, DUMP>(c, O + side * H, B);
            }
            B.beta = sel_lanes(ones64(H) << O, B.beta ^ lane_down<H>(B.beta), B.beta);
        } else if (type == 1) {
            B.beta = sel_lanes(ones64(M) << O, B.w[LG], B.beta);
        } else if (type == 3) {
            rep_node<M, FK, DUMP>(a, O, B);
        } else {
            B.beta = sel_lanes(ones64(M) << O, dec_sign(a), B.beta);
        }
    }
}

// Block set-up from its frozen mask F and frozen values V (wave-uniform).
__device__ __forceinline__ void blk_init(Blk& B, uint64_t F, uint64_t V) {
    B.F = F;
    B.V = V & F;
    uint64_t W = V & F;
    B.w[0] = lane_bit(W) ? SIGN : 0u;
#pragma unroll
    for (int t = 1; t < 7; ++t) {
        const int h = 1 << (t - 1);
        W ^= (W >> h) & low_mask64(h);
        B.w[t] = lane_bit(W) ? SIGN : 0u;
    }
    B.fv = B.w[0];
    B.beta = 0;
    B.leaf = 0.0f;
    B.has_leaf = false;
}

// ---------------------------------------------------------------------------
// Subtree of 2^C leaves (C <= 12) decoded by one wavefront.  Level L keeps the
// LLRs of the current node of size 2^L as elements k*64 + lane,
// k < 2^(L-6): levels above R in LDS (they are used rarely), levels R and
// below in registers.  Partial sums of the whole subtree sit in one 64-bit
// word per lane, bit k = element k*64 + lane (the "lane-packed" layout),
// which is also how they are exchanged with HBM.
// ---------------------------------------------------------------------------
template <int C>
struct SubCfg {
    static constexpr int R = C < 9 ? C : 9;  // highest register level
    // LDS floats a subtree of 2^lg leaves keeps its levels above R in: level
    // L (R < L <= lg) at offset 2^(lg+1) - 2^(L+1) from the subtree's base,
    // so the subtree's own input level sits at the base.
    __host__ __device__ static constexpr int floats(int lg) { return lg > R ? (1 << (lg + 1)) - (1 << (R + 1)) : 0; }
    __host__ __device__ static constexpr int off(int lg, int L) { return (1 << (lg + 1)) - (1 << (L + 1)); }
    static constexpr int lds_floats = floats(C);
    static constexpr int NL = C > R ? C - R : 1;  // LDS-resident levels
};

template <int C>
struct Lv {
    float* lp[SubCfg<C>::NL];  // level L > R at lp[L - R - 1] (wave-uniform)
    float a9[8];
    float a8[4];
    float a7[2];
    float a6;
};

template <int L, int C>
__device__ __forceinline__ float lv_get(Lv<C>& v, int k) {
    if constexpr (L > SubCfg<C>::R) return v.lp[L - SubCfg<C>::R - 1][k * 64 + lane_id()];
    else if constexpr (L == 9) return v.a9[k];
    else if constexpr (L == 8) return v.a8[k];
    else if constexpr (L == 7) return v.a7[k];
    else return v.a6;
}

template <int L, int C>
__device__ __forceinline__ void lv_set(Lv<C>& v, int k, float x) {
    if constexpr (L > SubCfg<C>::R) v.lp[L - SubCfg<C>::R - 1][k * 64 + lane_id()] = x;
    else if constexpr (L == 9) v.a9[k] = x;
    else if constexpr (L == 8) v.a8[k] = x;
    else if constexpr (L == 7) v.a7[k] = x;
    else v.a6 = x;
}

enum { OP_NONE = 0, OP_F = 1, OP_G = 2 };

// Compute the node of size 2^L from its parent (size 2^(L+1)) by f or g.
// For g the left sibling covers blocks [b - E, b), E = 2^(L-6).
template <int L, int C, int FK>
__device__ __forceinline__ void level_step(Lv<C>& v, int op, int b, uint64_t acc) {
    constexpr int E = 1 << (L - 6);
    if (op == OP_F) {
#pragma unroll
        for (int k = 0; k < E; ++k) lv_set<L, C>(v, k, fupd<FK>(lv_get<L + 1, C>(v, k), lv_get<L + 1, C>(v, k + E)));
    } else {
        const uint64_t x = acc >> (b - E);
#pragma unroll
        for (int k = 0; k < E; ++k) {
            const uint32_t sgn = (uint32_t)((x >> k) & 1ull) << 31;
            lv_set<L, C>(v, k, gupd<FK>(lv_get<L + 1, C>(v, k), lv_get<L + 1, C>(v, k + E), sgn));
        }
    }
}

// Rate-1 shortcut at level L >= 7 (see rate1_floor): on success the partial
// sums are the hard decisions, bit k of the lane word.
template <int L, int C, int FK>
__device__ __forceinline__ bool level_rate1(Lv<C>& v, uint64_t& bits) {
    constexpr int E = 1 << (L - 6);
    bool z = false;
    uint64_t s = 0;
#pragma unroll
    for (int k = 0; k < E; ++k) {
        const float x = lv_get<L, C>(v, k);
        z |= below_rate1_floor<FK, L>(x);
        s |= (uint64_t)(x < 0.0f) << k;
    }
    if (ballot(z) != 0) return false;
    bits = s;
    return true;
}

template <int L, int C>
__device__ __forceinline__ void level_load_global(Lv<C>& v, const float* src) {
    constexpr int E = 1 << (L - 6);
#pragma unroll
    for (int k = 0; k < E; ++k) lv_set<L, C>(v, k, src[k * 64 + lane_id()]);
}

struct SubIO {
    const uint32_t* mask;      // frozen mask words of the subtree
    const uint32_t* vals;      // frozen value words of the subtree
    uint32_t* uhat;            // u-hat words of the subtree (out)
    float* leaf;               // leaf LLRs of the subtree (out) or null
    uint64_t* beta_out;        // lane-packed partial sums (out) or null
    uint64_t* beta_lds;        // second copy of the partial sums (LDS) or null
};

// State of one subtree decode shared by its node visits.
struct SubCtx {
    uint64_t mw, vw;  // lane l: frozen mask / values of block l
    uint64_t A0, A1;  // bit b: block b is all frozen / has no frozen leaf
    uint64_t vT;      // lane l, bit k: frozen value of leaf k*64 + l
    uint64_t acc;     // lane-packed partial sums, bit k = element k*64 + lane
};

// One 64-leaf block (level 6 of the subtree): its LLRs are v.a6.
template <int C, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void sub_block(Lv<C>& v, SubCtx& x, const SubIO& io, int b) {
    if (PRUNE && ((x.A0 >> b) & 1ull)) {
        // rate 0: the block's frozen values re-encoded across the lanes
        x.acc |= (lane_transform(x.vT >> b) & 1ull) << b;
    } else {
        Blk B;
        blk_init(B, readlane64(x.mw, b), readlane64(x.vw, b));
        blk_node<64, FK, PRUNE, DUMP>(v.a6, 0, B);
        x.acc |= (uint64_t)(B.beta >> 31) << b;
        if (DUMP && B.has_leaf) io.leaf[b * 64 + lane_id()] = B.leaf;
    }
}

// Node of 2^L leaves (L >= 7) covering blocks [b, b + 2^(L-6)); its LLRs are
// level L of v.  Each level has one copy of its code (the two children are
// visited by a rolled loop, and a subtree smaller than 2^C passes through
// the levels above its root), and every level keeps its LLRs in its own
// registers or LDS area.
template <int L, int C, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void sub_node(Lv<C>& v, SubCtx& x, const SubIO& io, int b, int lg) {
    constexpr int EB = 1 << (L - 6);  // blocks covered
    constexpr int EH = EB / 2;        // blocks per child
    const bool above = L > lg;        // above the subtree's root: pass through
    bool done = above;
    if (!above) {
        const uint64_t rng = ones64(EB) << b;
        if (PRUNE && (x.A0 & rng) == rng) {
            // rate 0: beta = v G over the node, lane-packed
            uint64_t w = (x.vT >> b) & ones64(EB);
            w = word_transform(w, EB);
            x.acc |= lane_transform(w) << b;
            done = true;
        } else if (PRUNE && (x.A1 & rng) == rng) {
            uint64_t bits = 0;
            done = level_rate1<L, C, FK>(v, bits);
            if (done) x.acc |= bits << b;
        }
    }
    if (above || !done) {
        const int sides = above ? 1 : 2;
#pragma clang loop unroll(disable)
        for (int side = 0; side < sides; ++side) {
            const int bc = b + side * EH;
            if (!above) level_step<L - 1, C, FK>(v, side ? OP_G : OP_F, bc, x.acc);
            if constexpr (L - 1 == 6) sub_block<C, FK, PRUNE, DUMP>(v, x, io, bc);
            else sub_node<L - 1, C, FK, PRUNE, DUMP>(v, x, io, bc, lg);
        }
        if (!above) x.acc ^= (x.acc >> EH) & (ones64(EH) << b);  // beta = [beta_L ^ beta_R, beta_R]
    }
}

// u-hat = x-hat G over a subtree of nb blocks, from its lane-packed partial
// sums: G over k inside the lane word, then across lanes; transposed so that
// lane k holds leaves [64k, 64k + 64).
__device__ __forceinline__ void emit_uhat(uint64_t acc, int nb, uint32_t* uhat) {
    const int l = lane_id();
    uint64_t u = word_transform(acc, nb);
    u = lane_transform(u);
    u = transpose64(u);
    if (l < nb) {
        uhat[2 * l] = (uint32_t)u;
        uhat[2 * l + 1] = (uint32_t)(u >> 32);
    }
}

// Decode a subtree of 2^lg leaves, 6 <= lg <= C, on one wavefront.  Input
// LLRs: at lds (the subtree's LDS base) when lg > R, else at gsrc (global).
template <int C, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void subtree_decode(const SubIO io, int lg, float* lds, const float* gsrc) {
    constexpr int R = SubCfg<C>::R;
    const int l = lane_id();
    const int nb = 1 << (lg - 6);  // 64-leaf blocks
    Lv<C> v;
#pragma unroll
    for (int L = R + 1; L <= C; ++L)  // levels above lg are never touched
        v.lp[L - R - 1] = lds + (L <= lg ? SubCfg<C>::off(lg, L) : 0);

    SubCtx x;
    // Block words: lane l holds block l's mask and values.
    x.mw = 0;
    x.vw = 0;
    if (l < nb) {
        x.mw = (uint64_t)io.mask[2 * l] | ((uint64_t)io.mask[2 * l + 1] << 32);
        x.vw = (uint64_t)io.vals[2 * l] | ((uint64_t)io.vals[2 * l + 1] << 32);
    }
    x.A0 = ballot(l < nb && x.mw == ~0ull);  // all-frozen blocks
    x.A1 = ballot(l < nb && x.mw == 0ull);   // frozen-free blocks
    x.vT = 0;                                // lane l, bit k = value of leaf k*64 + l
    if (PRUNE && x.A0 != 0) x.vT = transpose64(x.vw);
    x.acc = 0;

    if (lg <= R) {
        switch (lg) {
            case 9: if constexpr (R >= 9) level_load_global<9, C>(v, gsrc); break;
            case 8: if constexpr (R >= 8) level_load_global<8, C>(v, gsrc); break;
            case 7: level_load_global<7, C>(v, gsrc); break;
            default: v.a6 = gsrc[l]; break;
        }
    }
    sub_node<C, C, FK, PRUNE, DUMP>(v, x, io, 0, lg);
    const uint64_t acc = x.acc;

    if (io.beta_out) io.beta_out[l] = acc;
    if (io.beta_lds) io.beta_lds[l] = acc;
    if (io.uhat) emit_uhat(acc, nb, io.uhat);
}

// Frames with N < 64: a single block decoder with the node at offset 0.
template <int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void tiny_decode(const FrameDesc& fd) {
    const int l = lane_id();
    const int n = 1 << fd.log2n;
    float a = l < n ? fd.llr[l] : 0.0f;
    Blk B;
    blk_init(B, fd.mask[0] & (uint32_t)ones64(n), fd.vals[0]);
    switch (fd.log2n) {
        case 1: blk_node<2, FK, PRUNE, DUMP>(a, 0, B); break;
        case 2: blk_node<4, FK, PRUNE, DUMP>(a, 0, B); break;
        case 3: blk_node<8, FK, PRUNE, DUMP>(a, 0, B); break;
        case 4: blk_node<16, FK, PRUNE, DUMP>(a, 0, B); break;
        case 5: blk_node<32, FK, PRUNE, DUMP>(a, 0, B); break;
        default: blk_node<1, FK, PRUNE, DUMP>(a, 0, B); break;
    }
    uint64_t u = word_transform(ballot(B.beta != 0u) & ones64(n), n);
    if (l == 0) fd.uhat[0] = (uint32_t)u;
    if (DUMP && l < n && B.has_leaf) fd.leaf[l] = B.leaf;
}

// ---------------------------------------------------------------------------
// Workgroup-wide sweeps over the LLR levels of nodes larger than 2^C (in HBM,
// or in the LDS tier).  Each lane handles 4 consecutive elements with 16-byte
// accesses, rows of 256 elements per wave instruction, SWEEP_UNROLL rows in
// flight per wave: these sweeps are bound by the bytes one workgroup keeps in
// flight, not by instruction count.
// ---------------------------------------------------------------------------
constexpr int SWEEP_UNROLL = 8;  // rows in flight per wave

__device__ __forceinline__ float4 ld4(const float* p) { return *reinterpret_cast<const float4*>(p); }

// The sweeps sit in the same loop as the register-hungry leaf decoder: their
// per-lane offsets, if hoisted out of that loop, would stay live across it
// and force spills.  An empty volatile asm makes the lane index and the first
// row opaque at every call, so the offsets are recomputed where used.
__device__ __forceinline__ int lane_id_here() {
    int x = lane_id();
    asm volatile("" : "+v"(x));
    return x;
}
__device__ __forceinline__ int64_t row_here(int wave) {
    int r = __builtin_amdgcn_readfirstlane(wave);
    asm volatile("" : "+s"(r));
    return r;
}
__device__ __forceinline__ void st4(float* p, float4 v) { *reinterpret_cast<float4*>(p) = v; }

// Level storage.  The FP32 kinds keep every level as float.  The fixed-point
// kinds keep the levels that live in HBM as int16 (int8 for the 8-bit kind),
// which is exact (every value is an integer within the kind's saturation) and
// halves (quarters) the bytes of the sweeps that HBM bounds; the channel input
// and the LDS levels stay float.  (A zero loses its sign in an integer, which
// no decision or later update depends on: decisions test L < 0, f and g give
// zeros of equal magnitude either way.)
// Raw loads (4 elements: a float4, or 4 int16 in an int2) and their
// conversion to float, kept apart so that a sweep converts only where it uses
// the values and holds the narrow form while its loads are in flight.
__device__ __forceinline__ float4 ldraw(const float* p) { return ld4(p); }
__device__ __forceinline__ int2 ldraw(const int16_t* p) { return *reinterpret_cast<const int2*>(p); }
__device__ __forceinline__ uint32_t ldraw(const int8_t* p) { return *reinterpret_cast<const uint32_t*>(p); }
__device__ __forceinline__ float4 cvt4(float4 v) { return v; }
__device__ __forceinline__ float4 cvt4(int2 w) {
    return make_float4((float)(((int32_t)((uint32_t)w.x << 16)) >> 16), (float)(w.x >> 16),
                       (float)(((int32_t)((uint32_t)w.y << 16)) >> 16), (float)(w.y >> 16));
}
__device__ __forceinline__ float4 cvt4(uint32_t w) {
    return make_float4((float)((int32_t)(w << 24) >> 24), (float)((int32_t)(w << 16) >> 24),
                       (float)((int32_t)(w << 8) >> 24), (float)((int32_t)w >> 24));
}
template <typename T>
__device__ __forceinline__ float4 ldv(const T* p) { return cvt4(ldraw(p)); }
__device__ __forceinline__ void stv(float* p, float4 v) { st4(p, v); }
__device__ __forceinline__ void stv(int16_t* p, float4 v) {
    const uint32_t a = (uint32_t)(int32_t)v.x & 0xffffu, b = (uint32_t)(int32_t)v.y;
    const uint32_t c = (uint32_t)(int32_t)v.z & 0xffffu, d = (uint32_t)(int32_t)v.w;
    *reinterpret_cast<int2*>(p) = make_int2((int32_t)(a | (b << 16)), (int32_t)(c | (d << 16)));
}
__device__ __forceinline__ void stv(int8_t* p, float4 v) {
    const uint32_t a = (uint32_t)(int32_t)v.x & 0xffu, b = (uint32_t)(int32_t)v.y & 0xffu;
    const uint32_t c = (uint32_t)(int32_t)v.z & 0xffu, d = (uint32_t)(int32_t)v.w;
    *reinterpret_cast<uint32_t*>(p) = a | (b << 8) | (c << 16) | (d << 24);
}

// Element type of the fixed-point kinds' HBM levels.
template <int FK>
using narrow_t = typename std::conditional<FK == 4, int8_t, int16_t>::type;

// Element types of a two-level sweep's input, middle and output levels, one
// bit each (set: the kind's integer type): LV_IN, LV_MID, LV_OUT.
enum : uint32_t { LV_IN = 1u, LV_MID = 2u, LV_OUT = 4u };

template <int FK>
__device__ __forceinline__ float4 f4(float4 a, float4 b) {
    return make_float4(fupd<FK>(a.x, b.x), fupd<FK>(a.y, b.y), fupd<FK>(a.z, b.z), fupd<FK>(a.w, b.w));
}

template <int FK>
__device__ __forceinline__ void sweep_f(const float* __restrict__ in, int64_t half, float* __restrict__ out,
                                        int wave, int nw) {
    const int l4 = lane_id_here() * 4;
    const int64_t rows = half >> 8;
    int64_t r = row_here(wave);
    for (; r + (SWEEP_UNROLL - 1) * nw < rows; r += SWEEP_UNROLL * nw) {
        float4 x[SWEEP_UNROLL], y[SWEEP_UNROLL];
#pragma unroll
        for (int i = 0; i < SWEEP_UNROLL; ++i) {
            const int64_t j = (r + i * nw) * 256 + l4;
            x[i] = ld4(in + j);
            y[i] = ld4(in + j + half);
        }
#pragma unroll
        for (int i = 0; i < SWEEP_UNROLL; ++i) st4(out + (r + i * nw) * 256 + l4, f4<FK>(x[i], y[i]));
    }
    for (; r < rows; r += nw) {
        const int64_t j = r * 256 + l4;
        st4(out + j, f4<FK>(ld4(in + j), ld4(in + j + half)));
    }
}

// beta: lane-packed partial sums of the left child (subtrees of 2^C leaves,
// 64 words each, bit k of word (s, lane) = element s*2^C + k*64 + lane).
// Element j reads bit (j >> 6) mod 2^(C-6) of word (j >> C)*64 + (j & 63);
// the 4 elements of a lane use 4 consecutive words.
template <int C, int FK>
__device__ __forceinline__ float4 g4(float4 a, float4 b, const uint64_t* __restrict__ beta, int64_t j) {
    constexpr int E = 1 << (C - 6);
    const uint64_t* w = beta + (j >> C) * 64 + (j & 63);
    const ulonglong2 w01 = *reinterpret_cast<const ulonglong2*>(w);
    const ulonglong2 w23 = *reinterpret_cast<const ulonglong2*>(w + 2);
    const int k = (int)((j >> 6) & (E - 1));
    const auto sg = [k](uint64_t x) { return (uint32_t)((x >> k) & 1ull) << 31; };
    return make_float4(gupd<FK>(a.x, b.x, sg(w01.x)), gupd<FK>(a.y, b.y, sg(w01.y)),
                       gupd<FK>(a.z, b.z, sg(w23.x)), gupd<FK>(a.w, b.w, sg(w23.y)));
}

template <int C, int FK>
__device__ __forceinline__ void sweep_g(const float* __restrict__ in, int64_t half,
                                        const uint64_t* __restrict__ beta, float* __restrict__ out,
                                        int wave, int nw) {
    const int l4 = lane_id_here() * 4;
    const int64_t rows = half >> 8;
    int64_t r = row_here(wave);
    for (; r + (SWEEP_UNROLL - 1) * nw < rows; r += SWEEP_UNROLL * nw) {
        float4 x[SWEEP_UNROLL], y[SWEEP_UNROLL];
#pragma unroll
        for (int i = 0; i < SWEEP_UNROLL; ++i) {
            const int64_t j = (r + i * nw) * 256 + l4;
            x[i] = ld4(in + j);
            y[i] = ld4(in + j + half);
        }
#pragma unroll
        for (int i = 0; i < SWEEP_UNROLL; ++i) {
            const int64_t j = (r + i * nw) * 256 + l4;
            st4(out + j, g4<C, FK>(x[i], y[i], beta, j));
        }
    }
    for (; r < rows; r += nw) {
        const int64_t j = r * 256 + l4;
        st4(out + j, g4<C, FK>(ld4(in + j), ld4(in + j + half), beta, j));
    }
}

// Two levels in one pass.  The first level (f, or g with partial sums beta)
// maps in[0 .. 2h) to mid[0 .. h); the second (f) maps mid to out[0 .. h/2).
// Each lane takes elements j .. j+3 of out and produces mid[j], mid[j + h/2]
// (and their 4-wide neighbours) from in[j], in[j + h], in[j + h/2],
// in[j + h/2 + h]: mid is written for its later g but not read back.
template <int C, int FK, bool G, typename TI = float, typename TM = float, typename TO = float>
__device__ __forceinline__ void sweep2(const TI* __restrict__ in, int64_t h, const uint64_t* __restrict__ beta,
                                       TM* __restrict__ mid, TO* __restrict__ out, int wave, int nw) {
    // rows in flight: a narrow input moves fewer bytes per row, so more rows
    // keep more of its bytes in flight (twice the rows at most: four times
    // made the 8-bit kernels spill)
    constexpr int U = SWEEP_UNROLL / 4 * (sizeof(TI) < 4 ? 2 : 1);
    const int l4 = lane_id_here() * 4;
    const int64_t q = h >> 1;
    const int64_t rows = q >> 8;
    const auto first = [&](float4 a, float4 b, int64_t j) -> float4 {
        if constexpr (G) return g4<C, FK>(a, b, beta, j);
        else return f4<FK>(a, b);
    };
    int64_t r = row_here(wave);
    using Raw = decltype(ldraw(in));
    for (; r + (U - 1) * nw < rows; r += U * nw) {
        Raw a0[U], b0[U], a1[U], b1[U];
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int64_t j = (r + i * nw) * 256 + l4;
            a0[i] = ldraw(in + j);
            b0[i] = ldraw(in + j + h);
            a1[i] = ldraw(in + j + q);
            b1[i] = ldraw(in + j + q + h);
        }
#pragma unroll
        for (int i = 0; i < U; ++i) {
            const int64_t j = (r + i * nw) * 256 + l4;
            const float4 m0 = first(cvt4(a0[i]), cvt4(b0[i]), j);
            const float4 m1 = first(cvt4(a1[i]), cvt4(b1[i]), j + q);
            stv(mid + j, m0);
            stv(mid + j + q, m1);
            stv(out + j, f4<FK>(m0, m1));
        }
    }
    for (; r < rows; r += nw) {
        const int64_t j = r * 256 + l4;
        const float4 m0 = first(ldv(in + j), ldv(in + j + h), j);
        const float4 m1 = first(ldv(in + j + q), ldv(in + j + q + h), j + q);
        stv(mid + j, m0);
        stv(mid + j + q, m1);
        stv(out + j, f4<FK>(m0, m1));
    }
}

// sweep2 on levels of the element types given by the LV_ bits (only the
// fixed-point kinds have int16 levels; the combinations are those of three
// consecutive depths: input or int16, then int16 or float).
template <int C, int FK, bool G>
__device__ __forceinline__ void sweep2_lv(uint32_t types, const float* in, int64_t h, const uint64_t* beta, float* mid,
                                          float* out, int wave, int nw) {
    if constexpr (FK >= 2) {
        using I = narrow_t<FK>;
        switch (types) {
            case LV_IN | LV_MID | LV_OUT:
                sweep2<C, FK, G, I, I, I>((const I*)in, h, beta, (I*)mid, (I*)out, wave, nw);
                return;
            case LV_IN | LV_MID:
                sweep2<C, FK, G, I, I, float>((const I*)in, h, beta, (I*)mid, out, wave, nw);
                return;
            case LV_IN:
                sweep2<C, FK, G, I, float, float>((const I*)in, h, beta, mid, out, wave, nw);
                return;
            case LV_MID | LV_OUT:
                sweep2<C, FK, G, float, I, I>(in, h, beta, (I*)mid, (I*)out, wave, nw);
                return;
            case LV_MID:
                sweep2<C, FK, G, float, I, float>(in, h, beta, (I*)mid, out, wave, nw);
                return;
            default:
                break;
        }
    }
    sweep2<C, FK, G>(in, h, beta, mid, out, wave, nw);
}

// beta[0 .. words) ^= beta[words .. 2 words)
__device__ __forceinline__ void combine_words(uint64_t* beta, int64_t words, int tid, int nt) {
    for (int64_t i = tid; i < words; i += nt) beta[i] ^= beta[i + words];
}

// ---------------------------------------------------------------------------
// Cooperative level sweeps.  A launch may hold more resident workgroups than
// it has frames: the extra workgroups, and those whose frames are done, help
// the frames' workgroups with their large two-level sweeps over HBM.  A
// frame's workgroup posts the sweep in its mailbox, split into partitions
// (partition p runs the sweep as waves p W .. p W + W - 1 of a virtual
// workgroup of P W waves); every workgroup, the poster included, claims
// partitions by a compare-and-swap on the mailbox's claim word (sequence
// number, partition count, next partition).  The poster waits only for
// partitions that others have already claimed, so no workgroup ever waits
// for one that has not started, and with no helper the poster runs every
// partition itself.  Data crosses compute units (and their L2 caches)
// through device-scope release fences before the post and before each
// partition's completion count, and acquire fences after the claim and
// after the wait.
// ---------------------------------------------------------------------------
// Optional timing: wave 0 accumulates, in s_memrealtime ticks (100 MHz), the
// time spent in register-resident subtree decoding.
__device__ __forceinline__ uint64_t now_ticks() { return __builtin_amdgcn_s_memrealtime(); }

constexpr uint64_t HELP_IDLE_TICKS = 100000000ull;  // 1 s of the 100 MHz clock
constexpr int COOP_MIN_ROWS = 128;  // rows of 256 outputs below which a sweep is not shared
constexpr int COOP_MAX_PARTS = 64;

__device__ __forceinline__ void fence_release_dev() { __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent"); }
__device__ __forceinline__ void fence_acquire_dev() { __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent"); }

__device__ __forceinline__ unsigned long long claim_load(SweepBox* b) {
    return __hip_atomic_load(&b->claim, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Claims the next partition of the sweep with sequence number seq (seq = 0:
// whatever sweep is open).  Returns the partition, or -1 when none is left.
__device__ __forceinline__ int claim_part(SweepBox* b, uint32_t seq, int* parts_out) {
    unsigned long long w = claim_load(b);
    while (true) {
        const uint32_t sq = (uint32_t)(w >> 32);
        const int parts = (int)((w >> 16) & 0xffffu), next = (int)(w & 0xffffu);
        if (sq == 0 || (seq != 0 && sq != seq) || next >= parts) return -1;
        if (__hip_atomic_compare_exchange_strong(&b->claim, &w, w + 1ull, __ATOMIC_ACQUIRE, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT)) {
            *parts_out = parts;
            return next;
        }
    }
}

// op: bit 0 set for a g first, bits 1..3 the levels' LV_ bits.
template <int C, int FK>
__device__ __forceinline__ void run_part(int op, const float* in, int64_t h, const uint64_t* beta, float* mid,
                                         float* out, int part, int parts, int wave, int W) {
    const uint32_t types = (uint32_t)op >> 1;
    if (op & 1) sweep2_lv<C, FK, true>(types, in, h, beta, mid, out, part * W + wave, parts * W);
    else sweep2_lv<C, FK, false>(types, in, h, nullptr, mid, out, part * W + wave, parts * W);
}

// Per-workgroup state of the cooperative sweeps, kept in LDS and read
// through volatile loads where used, so that it holds no registers across
// the leaf decoder.
struct CoopState {
    SweepBox* box;    // this frame workgroup's mailbox, or null (no helpers)
    SweepBox* boxes;  // the launch's mailboxes (one per frame workgroup), or null
    int n_main;       // frame workgroups of the launch
    uint32_t seq;     // sequence number of its last posted sweep
    int cmd[3];       // claim broadcast: mailbox, partition, partitions
};

// Variants that take helpers.  The pruned cutover-12 min-sum variants (the
// straight-line 64-leaf patterns) already use every register the leaf
// decoder can have; the cooperative code tips them into spilling, so they
// decode their frames alone.
template <int C, int FK, bool PRUNE, bool DUMP>
constexpr bool coop_variant() {
    return !(C == 12 && PRUNE && !DUMP && minsum_kind<FK>());
}

// sweep2 over the whole workgroup, shared with helpers when it is large and
// the workgroup has a mailbox.  Ends with the workgroup synchronised and the
// outputs visible to it.
template <int C, int FK, bool G, bool COOP>
__device__ __forceinline__ void coop_sweep2(bool shareable, CoopState* cs, uint32_t types, const float* in, int64_t h,
                                            const uint64_t* beta, float* mid, float* out, int wave, int W) {
    const int64_t rows = (h >> 1) >> 8;
    SweepBox* box = COOP && shareable ? *(SweepBox* volatile*)&cs->box : nullptr;
    if (!COOP || box == nullptr || rows < COOP_MIN_ROWS) {
        sweep2_lv<C, FK, G>(types, in, h, beta, mid, out, wave, W);
        __syncthreads();
        return;
    }
    int parts = (int)(rows / (SWEEP_UNROLL * W));
    parts = parts < COOP_MAX_PARTS ? parts : COOP_MAX_PARTS;
    // everything this workgroup wrote (levels, partial sums) is read by others
    fence_release_dev();
    __syncthreads();
    const uint32_t seq = *(volatile uint32_t*)&cs->seq + 1u;
    int* s_part = &cs->cmd[0];
    __syncthreads();  // every thread has read seq before thread 0 advances it
    if (threadIdx.x == 0) {
        cs->seq = seq;
        box->op = (int32_t)((G ? 1u : 0u) | (types << 1));
        box->in = in;
        box->beta = beta;
        box->mid = mid;
        box->out = out;
        box->half = h;
        __hip_atomic_store(&box->done, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&box->claim, ((unsigned long long)seq << 32) | ((unsigned long long)parts << 16),
                           __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
    int own = 0;
    while (true) {
        if (threadIdx.x == 0) {
            int pp = 0;
            *s_part = claim_part(box, seq, &pp);
        }
        __syncthreads();
        const int p = *s_part;
        __syncthreads();
        if (p < 0) break;
        ++own;
        run_part<C, FK>((int)((G ? 1u : 0u) | (types << 1)), in, h, beta, mid, out, p, parts, wave, W);
    }
    if (threadIdx.x == 0) {
        // partitions claimed by other workgroups are running and end on their
        // own; the bound (2^28 polls, seconds) only keeps a broken count
        // from hanging the device
        const uint32_t others = (uint32_t)(parts - own);
        for (uint32_t it = 0; it < (1u << 28); ++it) {
            if (__hip_atomic_load(&box->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= others) break;
            __builtin_amdgcn_s_sleep(1);
        }
    }
    __syncthreads();
    fence_acquire_dev();
}

// A workgroup without a frame: claims partitions of any open sweep of the
// launch until every frame is done (frames_done reaches n_frames), or until
// it has found nothing to do for a second (a helper that leaves only costs
// speed: frame workgroups never wait for unclaimed partitions).

template <int C, int FK>
__device__ __forceinline__ void help_sweeps(SweepBox* boxes, int n_boxes, const unsigned* frames_done, int n_frames,
                                            int* s_cmd) {
    const int W = (int)(blockDim.x >> 6);
    const int wave = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    // each helper watches its own frame workgroup's mailbox and looks at all
    // of them every 8th poll (the polls are device-scope loads)
    const int home = (int)(blockIdx.x % (unsigned)n_boxes);
    unsigned poll = 0;
    uint64_t idle_since = now_ticks();
    while (true) {
        if (threadIdx.x == 0) {
            s_cmd[0] = -1;
            const int span = (poll & 7u) == 7u ? n_boxes : 1;
            for (int k = 0; k < span; ++k) {
                const int b = home + k < n_boxes ? home + k : home + k - n_boxes;
                int parts = 0;
                const int p = claim_part(boxes + b, 0u, &parts);
                if (p >= 0) {
                    s_cmd[0] = b;
                    s_cmd[1] = p;
                    s_cmd[2] = parts;
                    break;
                }
            }
            if (s_cmd[0] < 0) {
                ++poll;
                if (__hip_atomic_load(frames_done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) >= (unsigned)n_frames ||
                    now_ticks() - idle_since > HELP_IDLE_TICKS)
                    s_cmd[0] = -2;
                else
                    __builtin_amdgcn_s_sleep(32);
            } else {
                idle_since = now_ticks();
            }
        }
        __syncthreads();
        const int b = __builtin_amdgcn_readfirstlane(s_cmd[0]);
        const int p = __builtin_amdgcn_readfirstlane(s_cmd[1]);
        const int parts = __builtin_amdgcn_readfirstlane(s_cmd[2]);
        __syncthreads();
        if (b == -2) break;
        if (b < 0) continue;
        fence_acquire_dev();
        SweepBox* x = boxes + b;
        const auto uptr = [](const void* q) {
            const uint64_t v = (uint64_t)q;
            const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
            const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
            return ((uint64_t)hi << 32) | lo;
        };
        const int op = __builtin_amdgcn_readfirstlane(x->op);
        const float* in = (const float*)uptr(x->in);
        const uint64_t* beta = (const uint64_t*)uptr(x->beta);
        float* mid = (float*)uptr(x->mid);
        float* out = (float*)uptr(x->out);
        const int64_t h = (int64_t)uptr((const void*)x->half);
        run_part<C, FK>(op, in, h, beta, mid, out, p, parts, wave, W);
        fence_release_dev();
        __syncthreads();
        if (threadIdx.x == 0) __hip_atomic_fetch_add(&x->done, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Byte offsets inside one frame slot of the workspace.
__host__ __device__ inline int64_t slot_level_offset(int log2n, int d) {
    // level d (1 <= d) holds N >> d floats; levels are packed from d = 1
    const int64_t n = (int64_t)1 << log2n;
    return (n - (n >> (d - 1))) * 4;
}


// A frame of 2^n > 2^C leaves, decoded by the whole workgroup: sweeps over
// the levels above the cutover, one wavefront per subtree.
template <int C, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void decode_frame(const FrameDesc& fd, uint8_t* slot, float* lds, float* tier,
                                             uint32_t* words, uint64_t* lbeta, uint64_t& sub_ticks, CoopState* cs) {
    const int W = (int)(blockDim.x >> 6);  // wavefronts in the workgroup
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);  // wave-uniform: keeps sweep offsets scalar
    const int n = fd.log2n;  // > C: frames of at most 2^C leaves go to decode_small
    const int D = n - C;
    const int64_t N = (int64_t)1 << n;
    uint64_t* beta = reinterpret_cast<uint64_t*>(slot + slot_level_offset(n, D));
    // Levels of the two depths above the cutover live in LDS (the "tier"),
    // so that most subtree steps make no HBM round trip; deeper-up levels
    // are in the frame's slot in HBM.
    auto level = [&](int d) -> float* {
        if (d == 0) return const_cast<float*>(fd.llr);
        if (d == D - 1) return tier;
        if (d == D - 2) return tier + (2 << C);
        return reinterpret_cast<float*>(slot + slot_level_offset(n, d));
    };
    // LV_ bits of a sweep whose input, middle and output levels are at depths
    // d, d + 1, d + 2 (the last in LDS when it is the cutover depth): the
    // fixed-point kinds' HBM levels, depths 1 .. D - 3, are int16
    const auto lv_types = [&](int d) -> uint32_t {
        if constexpr (FK >= 2) {
            const auto hbm = [&](int e) { return e >= 1 && e <= D - 3; };
            return (hbm(d) ? LV_IN : 0u) | (hbm(d + 1) ? LV_MID : 0u) | (hbm(d + 2) ? LV_OUT : 0u);
        } else {
            return 0u;
        }
    };
    const int64_t nsub = (int64_t)1 << D;
    // mask and value words of subtree s: LDS buffer s & 1, filled by wave 1
    // while wave 0 decodes the subtree before it
    constexpr int NW = 1 << (C - 5);
    const auto stage = [&](int64_t s2) {
        uint32_t* dst = words + (s2 & 1) * 2 * NW;
        const int64_t wb = (s2 << C) >> 5;
        for (int i = tid & 63; i < 2 * NW; i += 64) dst[i] = i < NW ? fd.mask[wb + i] : fd.vals[wb + i - NW];
    };
    if (wave == 1) stage(0);
    for (int64_t s = 0; s < nsub; ++s) {
        int t;
        if (s == 0) {
            t = D;
        } else {
            t = __builtin_ctzll((unsigned long long)s);
            for (int q = 1; q <= t; ++q) {
                combine_words(beta + (s - (1ll << q)) * 64, (1ll << (q - 1)) * 64, tid, W * 64);
                if (q == 1 && tid < 64) lbeta[tid] ^= lbeta[64 + tid];  // the LDS copy too
                __syncthreads();
            }
            // g: parent at depth D - t - 1, right child at depth D - t; when
            // the f chain continues, the first f rides in the same pass
            const int dp = D - t - 1;
            const int64_t half = N >> (dp + 1);
            const uint64_t* bl = beta + (s - (1ll << t)) * 64;
            // (for the two deepest g levels the left sibling's partial sums
            // are the last one or two subtrees', read from their LDS copy)
            if (t == 0) {
                sweep_g<C, FK>(level(dp), half, lbeta, lds, wave, W);
                __syncthreads();
            } else if (t == 1) {
                sweep2<C, FK, true>(level(dp), half, lbeta, level(D - t), lds, wave, W);
                __syncthreads();
            } else {
                // both outputs in HBM (t >= 4) can be shared with helpers
                coop_sweep2<C, FK, true, coop_variant<C, FK, PRUNE, DUMP>()>(
                    t >= 4, cs, lv_types(dp), level(dp), half, bl, level(D - t), level(D - t + 1), wave, W);
            }
        }
        // rest of the f chain down to the cutover depth (the cutover node goes
        // to LDS), two levels per pass
        int d = (s == 0) ? 1 : D - t + 2;
        for (; d + 1 <= D; d += 2) {
            // outputs at depths d, d + 1 <= D - 3 are in HBM: shareable
            coop_sweep2<C, FK, false, coop_variant<C, FK, PRUNE, DUMP>()>(
                d + 1 <= D - 3, cs, lv_types(d - 1), level(d - 1), N >> d, nullptr, level(d),
                d + 1 == D ? lds : level(d + 1), wave, W);
        }
        if (d == D) {
            sweep_f<FK>(level(d - 1), N >> d, lds, wave, W);
            __syncthreads();
        }
        if (wave == 0) {
            const uint64_t t0 = now_ticks();
            const int64_t base = s << C;
            SubIO io{words + (s & 1) * 2 * NW, words + (s & 1) * 2 * NW + NW, nullptr,
                     DUMP ? fd.leaf + base : nullptr, beta + s * 64, lbeta + (s & 1) * 64};
            // (a cutover node that fits the registers is loaded from LDS
            // through a generic pointer)
            subtree_decode<C, FK, PRUNE, DUMP>(io, C, lds, C <= SubCfg<C>::R ? lds : nullptr);
            sub_ticks += now_ticks() - t0;
        } else if (wave == 1 && s + 1 < nsub) {
            stage(s + 1);
        } else if (wave == 2 && s > 0) {
            // u-hat of the previous subtree, from its partial sums' LDS copy
            // (slot (s - 1) & 1 is not written again before the next barrier)
            emit_uhat(lbeta[((s - 1) & 1) * 64 + lane_id()], 1 << (C - 6), fd.uhat + (((s - 1) << C) >> 5));
        }
        __syncthreads();
    }
    if (wave == 2) emit_uhat(lbeta[((nsub - 1) & 1) * 64 + lane_id()], 1 << (C - 6), fd.uhat + (((nsub - 1) << C) >> 5));
}

template <int C>
constexpr int TIER_FLOATS = (2 << C) + (4 << C);

// All LDS LLR storage of a workgroup: the subtree levels of a large frame,
// then its tier; or, for frames of at most 2^C leaves, one region per
// wavefront decoding its own frame.
template <int C>
constexpr int LDS_FLOATS = (SubCfg<C>::lds_floats > (1 << C) ? SubCfg<C>::lds_floats : (1 << C)) + TIER_FLOATS<C>;

// Frames of 2^lg <= 2^C leaves one workgroup of W wavefronts decodes at once
// (one per wavefront), bounded by the LDS their subtree levels need.
template <int C>
__host__ __device__ inline int max_fwg(int lg, int W) {
    const int need = SubCfg<C>::floats(lg);
    const int by_lds = need > 0 ? LDS_FLOATS<C> / need : W;
    return by_lds < W ? by_lds : W;
}

// Completion flag of a frame: written (system scope, host-coherent memory)
// once every u-hat word of the frame is globally visible.  Call with the
// whole wavefront active; lane 0 stores.
__device__ __forceinline__ void signal_done(const FrameDesc& fd, uint32_t* done) {
    if (done == nullptr || fd.done_idx == 0xffffffffu) return;
    __threadfence_system();
    if (lane_id() == 0) __hip_atomic_store(done + fd.done_idx, fd.done_val, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

// A frame of 2^n <= 2^C leaves decoded by one wavefront on its own LDS
// region (no workgroup barrier).  The channel LLRs are staged in the
// region's input level by the lane that later reads each element.
template <int C, int FK, bool PRUNE, bool DUMP>
__device__ __forceinline__ void decode_small(const FrameDesc& fd, float* lds) {
    constexpr int R = SubCfg<C>::R;
    const int n = fd.log2n;
    if (n < 6) {
        tiny_decode<FK, PRUNE, DUMP>(fd);
        return;
    }
    if (n > R)
        for (int i = lane_id(); i < (1 << n); i += 64) lds[i] = fd.llr[i];
    SubIO io{fd.mask, fd.vals, fd.uhat, fd.leaf, nullptr, nullptr};
    subtree_decode<C, FK, PRUNE, DUMP>(io, n, lds, fd.llr);
}

// Next frame index from the work counter, for one wavefront.
__device__ __forceinline__ int wave_draw(unsigned* counter) {
    unsigned f = 0;
    if (lane_id() == 0) f = atomicAdd(counter, 1u);
    return (int)__builtin_amdgcn_readfirstlane(f);
}

// One kernel serves every workgroup size up to MAXW wavefronts (its register
// budget is the one of MAXW).  Workgroups take frames from a device counter
// in the host's order (longest first); every frame has more than 2^C leaves
// (smaller ones go to k_sc_decode_small) and is decoded by the whole
// workgroup.
template <int C, int FK, bool PRUNE, bool DUMP, int MAXW>
__global__ __launch_bounds__(MAXW * 64) void k_sc_decode(const FrameDesc* __restrict__ descs, int n_frames,
                                                       unsigned* __restrict__ counter, uint8_t* slots,
                                                       int64_t slot_bytes, unsigned long long* prof,
                                                       uint32_t* done, SweepBox* boxes, int n_main) {
    __shared__ float lds_all[LDS_FLOATS<C>];
    __shared__ int s_frame;
    __shared__ CoopState s_coop;
    __shared__ uint32_t s_words[2][2 << (C - 5)];  // staged mask and value words of the next subtree
    __shared__ uint64_t s_beta[2][64];  // partial sums of the last two subtrees (slot s & 1)
    constexpr int LDS_SUB = LDS_FLOATS<C> - TIER_FLOATS<C>;
    float* lds = lds_all;
    float* tier = lds_all + LDS_SUB;  // LLR levels of sizes 2^(C+1) and 2^(C+2)
    // workgroups 0 .. n_main-1 decode frames (then help); the rest only help.
    // The cooperative state goes to LDS at once, so that none of it holds
    // registers across the frame loop.
    // (the fixed-point kinds take the workgroup index as a scalar, which keeps
    // their slot address out of vector registers: their int16 sweeps need those)
    const unsigned wg = FK >= 2 ? (unsigned)__builtin_amdgcn_readfirstlane((int)blockIdx.x) : blockIdx.x;
    const bool main_wg = (int)wg < n_main;
    uint8_t* wg_slot = slots + (int64_t)wg * slot_bytes;
    if (threadIdx.x == 0) {
        s_coop.box = boxes != nullptr && main_wg ? boxes + wg : nullptr;
        s_coop.boxes = boxes;
        s_coop.n_main = n_main;
        s_coop.seq = 0;
    }
    if constexpr (FK == 3) phi_table_init();
    __syncthreads();
    while (main_wg) {
        if (threadIdx.x == 0) s_frame = (int)atomicAdd(counter, 1u);
        __syncthreads();
        const int f = s_frame;
        __syncthreads();
        if (f >= n_frames) break;
        const FrameDesc fd = descs[f];
        if (fd.log2n <= C) continue;  // never sent here by the host
        uint64_t sub_ticks = 0;
        const uint64_t t0 = prof ? now_ticks() : 0;
        decode_frame<C, FK, PRUNE, DUMP>(fd, fd.slot ? fd.slot : wg_slot, lds, tier, &s_words[0][0], &s_beta[0][0],
                                         sub_ticks, &s_coop);
        __syncthreads();
        if (threadIdx.x < 64) signal_done(fd, done);
        if (threadIdx.x == 0 && *(SweepBox* volatile*)&s_coop.box != nullptr)
            __hip_atomic_fetch_add(counter + 32, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);  // frames done
        if (prof && threadIdx.x == 0) {
            atomicAdd(prof + 0, (unsigned long long)sub_ticks);
            atomicAdd(prof + 1, (unsigned long long)(now_ticks() - t0));
            atomicAdd(prof + 2, 1ull);
        }
    }
    if constexpr (coop_variant<C, FK, PRUNE, DUMP>()) {
        SweepBox* const all = *(SweepBox* volatile*)&s_coop.boxes;
        const int nm = *(volatile int*)&s_coop.n_main;
        if (all != nullptr && (int)gridDim.x > nm) help_sweeps<C, FK>(all, nm, counter + 32, n_frames, &s_coop.cmd[0]);
    }
}

// Frames of at most 2^C leaves: each wavefront of a workgroup (fwg of them)
// decodes frames on its own (its own LDS region, no workgroup barrier),
// drawing them from the device counter one at a time.  region: LDS floats
// per wavefront, for the largest frame of the launch (frames come longest
// first, so later frames fit too); the launch gives fwg * region floats of
// dynamic LDS.
template <int C, int FK, bool PRUNE, bool DUMP, int MAXW>
__global__ __launch_bounds__(MAXW * 64) void k_sc_decode_small(const FrameDesc* __restrict__ descs, int n_frames,
                                                             unsigned* __restrict__ counter,
                                                             unsigned long long* prof, uint32_t* done, int region) {
    extern __shared__ float lds_dyn[];
    if constexpr (FK == 3) {
        phi_table_init();
        __syncthreads();
    }
    const int wave = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    float* mine = lds_dyn + wave * region;
    for (int g = wave_draw(counter); g < n_frames; g = wave_draw(counter)) {
        const FrameDesc d = descs[g];
        const uint64_t t0 = prof ? now_ticks() : 0;
        decode_small<C, FK, PRUNE, DUMP>(d, mine);
        signal_done(d, done);
        if (prof && lane_id() == 0) {
            const unsigned long long dt = now_ticks() - t0;
            atomicAdd(prof + 0, dt);
            atomicAdd(prof + 1, dt);
            atomicAdd(prof + 2, 1ull);
        }
    }
}

// Work-counter reset (a kernel rather than a memset, so that the launch can
// be captured into a graph).
static __global__ void k_reset_counter(unsigned* counter, SweepBox* boxes, int n_boxes) {
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        counter[0] = 0u;   // work counter
        counter[32] = 0u;  // frames done (cooperative sweeps)
    }
    uint64_t* w = reinterpret_cast<uint64_t*>(boxes);
    const int64_t words = (int64_t)n_boxes * (int64_t)(sizeof(SweepBox) / 8);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += (int64_t)gridDim.x * blockDim.x)
        w[i] = 0ull;
}

// Every variant fits the register budget of 8 wavefronts per workgroup.
constexpr int MAX_WAVES = 8;

template <int C, int FK, bool PRUNE, bool DUMP>
hipError_t launch_decode(const DecodeLaunch& a) {
    constexpr int MAXW = MAX_WAVES;
    if (a.waves < 1 || a.waves > MAXW) return hipErrorInvalidValue;
    const int waves = a.waves;
    // (without helpers a frame's workgroup would run its shared sweeps as
    // partitions one after another: no mailboxes then)
    SweepBox* boxes = a.small || a.helpers <= 0 || !coop_variant<C, FK, PRUNE, DUMP>() ? nullptr : a.boxes;
    const int n_boxes = boxes ? a.grid : 0;
    hipLaunchKernelGGL(k_reset_counter, dim3(n_boxes > 16 ? (n_boxes + 15) / 16 : 1), dim3(256), 0, a.stream,
                       a.counter, boxes, n_boxes);
    if (a.small) {
        // every frame of the launch has at most 2^C leaves, the first one the
        // most; one wavefront per frame in flight, each with its LDS region
        const int region = SubCfg<C>::floats(a.small_log2n);
        if (a.small_log2n > C || a.fwg < 1 || a.fwg > MAXW || a.fwg * region > LDS_FLOATS<C>)
            return hipErrorInvalidValue;
        const size_t smem = (size_t)a.fwg * (size_t)region * sizeof(float);
        auto kern = k_sc_decode_small<C, FK, PRUNE, DUMP, MAXW>;
        if (smem > 65536) {
            const hipError_t e =
                hipFuncSetAttribute((const void*)kern, hipFuncAttributeMaxDynamicSharedMemorySize, (int)smem);
            if (e != hipSuccess) return e;
        }
        hipLaunchKernelGGL(kern, dim3(a.grid), dim3(a.fwg * 64), smem, a.stream, a.descs, a.n_frames, a.counter,
                           a.prof, a.done, region);
    } else {
        if (a.helpers < 0 || (a.helpers > 0 && a.boxes == nullptr)) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_sc_decode<C, FK, PRUNE, DUMP, MAXW>), dim3(a.grid + (boxes ? a.helpers : 0)),
                           dim3(waves * 64), 0,
                           a.stream, a.descs, a.n_frames, a.counter, a.slots, a.slot_bytes, a.prof, a.done, boxes,
                           a.grid);
    }
    return hipGetLastError();
}

// Resident workgroups per compute unit: the large-frame kernel with `waves`
// wavefronts (small_log2n < 0), or the per-wavefront kernel with `waves`
// wavefronts decoding frames of at most 2^small_log2n leaves.
template <int C, int FK, bool PRUNE, bool DUMP>
int occupancy_decode(int waves, int small_log2n) {
    int blocks = 0;
    hipError_t e;
    if (small_log2n >= 0) {
        const size_t smem = (size_t)waves * (size_t)SubCfg<C>::floats(small_log2n < C ? small_log2n : C) * 4;
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sc_decode_small<C, FK, PRUNE, DUMP, MAX_WAVES>,
                                                         waves * 64, smem);
    } else {
        e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&blocks, k_sc_decode<C, FK, PRUNE, DUMP, MAX_WAVES>,
                                                         waves * 64, 0);
    }
    return e == hipSuccess ? blocks : 0;
}

}  // namespace polar_dev

// One translation unit per decoder variant, so that the variants compile in
// parallel: NAME launches k_sc_decode<C, FK, PRUNE, DUMP>; NAME_occupancy
// reports the resident workgroups per compute unit of its large-frame (small
// = 0) or per-wavefront (small = 1) kernel.
#define POLAR_DECODE_VARIANT(NAME, C, FK, PRUNE, DUMP)                                  \
    extern "C" hipError_t NAME(const DecodeLaunch* a) {                                \
        return polar_dev::launch_decode<C, FK, PRUNE, DUMP>(*a);                       \
    }                                                                                  \
    extern "C" int NAME##_occupancy(int waves, int small_log2n) {                      \
        return polar_dev::occupancy_decode<C, FK, PRUNE, DUMP>(waves, small_log2n);    \
    }
