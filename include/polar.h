/*
 * libpolar: successive-cancellation (SC) decoding of long polar codes on
 * AMD Instinct MI355X (gfx950).
 *
 * The decoding problem is the one of Section 1 and Section 3 of Jouguet and
 * Kunz-Jacques, "High performance error correction for quantum key
 * distribution using polar codes": Alice's string is the polar codeword
 * (no encoding step), the values of the frozen bits of u = x G_N are
 * revealed over the classical channel, and Bob recovers u-hat from the LLRs
 * of his own string with the recursive SC decoder of Section 4.
 *
 * Conventions for every call:
 *   - Return value: POLAR_OK (0) or a negative POLAR_E_* code; the message of
 *     the last failing call on this thread is available from
 *     polar_last_error().  Nothing aborts the process.
 *   - Bit vectors are packed little-endian into uint32 words: bit i of a
 *     length-N vector is bit (i & 31) of word (i >> 5).  A vector of N < 32
 *     bits occupies one word whose unused high bits are zero on output and
 *     ignored on input.
 *   - LLRs are float32, L = ln P(bit = 0 | y) / P(bit = 1 | y).
 *   - Pointers documented as "device" must point to memory of the device the
 *     context (or the call) runs on; "host" pointers to host memory.  The
 *     caller owns every buffer; the library frees nothing it did not
 *     allocate.
 *   - "stream" is a hipStream_t passed as void* (NULL = the null stream).
 *     Device work is enqueued asynchronously; outputs are valid once the
 *     stream has been synchronised.  Argument errors are reported
 *     synchronously with nothing enqueued; errors raised by the device show
 *     up as POLAR_E_DEVICE from a later call.
 */
#ifndef POLAR_H
#define POLAR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POLAR_OK 0
#define POLAR_E_INVAL (-1)     /* bad argument (size, pointer, option)            */
#define POLAR_E_NOMEM (-2)     /* workspace / arena too small                     */
#define POLAR_E_DEVICE (-3)    /* HIP runtime or device error                     */
#define POLAR_E_BUSY (-4)      /* serving queue full                              */
#define POLAR_E_CANCELLED (-5) /* serving request cancelled before it ran         */

/* Check-node update used by SC decoding (Section 4). */
#define POLAR_F_MINSUM 0  /* sign(a) sign(b) min(|a|,|b|), FP32, bit-exact        */
#define POLAR_F_BOXPLUS 1 /* 2 atanh(tanh(a/2) tanh(b/2)) (the phi-function form), FP32 */
/* Fixed point (Section 4: fixed-point LLRs, check update from a phi table).
   The frame's llr array holds integers in units of 2^-POLAR_FIXED_FRAC with
   |L| <= POLAR_FIXED_MAX, stored as float (exact); every variable update
   g = b +- a saturates to +-POLAR_FIXED_MAX; leaf LLRs come out in the same
   units.  Results are bit-exact against integer arithmetic.  Other llr values
   give undefined results (the decoder keeps its large LLR levels in the
   workspace as 16-bit integers). */
#define POLAR_F_MINSUM_Q16 2 /* saturating min-sum                               */
#define POLAR_F_PHI_Q16 3    /* sign(a) sign(b) min(T[min(T[|a|] + T[|b|], 255)], |a|, |b|),
                                T[i] = round(phi(i 2^-4) 2^4), phi(x) = -ln tanh(x/2),
                                T[0] = 32767; T is 0 from index 67 on            */
#define POLAR_FIXED_FRAC 4
#define POLAR_FIXED_MAX 32767
/* Saturating min-sum on 8-bit integers (the second step of Section 4's
   fixed point): llr holds integers with |L| <= POLAR_FIXED8_MAX, stored as
   float, in whatever units the caller quantized to (min-sum decides the same
   at every scale but for the saturation); g saturates to +-POLAR_FIXED8_MAX.
   Results are bit-exact against integer arithmetic; other llr values give
   undefined results (the decoder keeps its large LLR levels as 8-bit
   integers). */
#define POLAR_F_MINSUM_Q8 4
#define POLAR_FIXED8_MAX 127
#define POLAR_FIXED8_FRAC 2  /* units of the FER generator's 8-bit LLRs */

#define POLAR_MAX_LOG2N 24

/* List decoding: paths per frame, and the largest N x paths (state on chip). */
#define POLAR_SCL_MAX_LIST 16
#define POLAR_SCL_MAX_NL 32768  /* every path's state in the 160 KiB of LDS */

/* Degrading construction: outputs kept per channel, and outputs of the
   channel it starts from. */
#define POLAR_CONSTRUCT_MAX_MU 64
#define POLAR_CONSTRUCT_MAX_OUTPUTS 65536

/* Message describing the last failing call made by this thread ("" if none). */
const char* polar_last_error(void);

/* Library version string. */
const char* polar_version(void);

/*
 * Frozen set from the Bhattacharyya parameters of the synthetic channels
 * (Section 3: the lowest-capacity bits are frozen; the frozen set can be
 * chosen so that the bound on the frame error rate is 0.1).  Host only.
 *
 * One polarisation step maps Z to 2Z - Z^2 for the first-decoded ("minus")
 * channel and to Z^2 for the other; index i applies the step selected by its
 * most significant bit first.  Z is carried as (ln Z, ln(1 - Z)) in double so
 * that it does not saturate at 1.  Channels are ranked by
 * r_i = ln((1 - Z_i) / Z_i); the least reliable are frozen, exact ties
 * freezing the lower index first.
 *
 *   log2n        1 .. POLAR_MAX_LOG2N
 *   z0           Bhattacharyya parameter of the channel, 0 < z0 < 1
 *                (BSC(p): 2 sqrt(p(1-p)); BPSK/AWGN(sigma): exp(-1/(2 sigma^2)))
 *   n_frozen     >= 0: freeze exactly this many (<= N);
 *                -1: union-bound rule, the largest information set whose
 *                sum of Z_i is <= fer_bound
 *   fer_bound    used only when n_frozen == -1 (e.g. 0.1)
 *   frozen_mask  host out, max(1, N/32) words, 1 = frozen
 *   r_out        host out, N doubles, or NULL
 *   n_frozen_out host out, or NULL
 */
int polar_build_frozen_set(int log2n, double z0, int64_t n_frozen, double fer_bound,
                           uint32_t* frozen_mask, double* r_out, int64_t* n_frozen_out);

/*
 * Frozen-set construction by channel degradation, on the device (Section 3
 * freezes the least reliable synthetic channels; the paper's sets come from
 * the density-evolution construction it cites [MT09], which it does not
 * describe).  Every synthetic channel is carried as a finite binary-input
 * symmetric channel and degraded to at most mu outputs after each
 * polarization step (Tal and Vardy), merging outputs by binning the binary
 * entropy of their posterior (Pedarsani, Hassani, Tal and Telatar).  Merging
 * degrades, so each pe[i] is an upper bound on the error probability of the
 * ML decision of u_i given y and u_0 .. u_{i-1}; on the BEC it is exact
 * (Z_i / 2).
 *
 * A channel is a list of pairs (a_k, b_k), a_k = W(y_k|0) >= b_k = W(y_k|1)
 * >= 0, one per conjugate output pair {y_k, y_k'} (W(y_k'|0) = b_k), summing
 * to 1; BSC(p): {(1-p, p)}; BEC(e): {(1-e, 0), (e/2, e/2)}.  Index i applies
 * the polarization step selected by its most significant bit first (as in
 * polar_build_frozen_set): minus (a_i a_j + b_i b_j, a_i b_j + b_i a_j) over
 * the ordered output pairs (i, j); plus (a_i a_j, b_i b_j) and
 * (max(a_i b_j, b_i a_j), min(a_i b_j, b_i a_j)).  Merge: output k goes to
 * bin min(mu-1, floor(mu h2(b_k / (a_k + b_k)))), bins sum their outputs in
 * output order (minus: i m + j; plus: the two outputs of (i, j) at
 * 2(i m + j) and 2(i m + j) + 1), occupied bins kept ascending; w0 itself is
 * merged first.  pe[i] = the b of channel i's occupied bins added in
 * ascending order.  Double precision, every product and sum rounded alone.
 *
 *   log2n      0 .. POLAR_MAX_LOG2N
 *   w0         host, m0 pairs (a, b) as 2 m0 doubles, a >= b >= 0, summing
 *              to 1 within 1e-12 (used as given: each step squares a
 *              channel's total mass, so a w0 off 1 by d scales level-n
 *              values by about 1 + 2^n d); copied before the call returns
 *              (the call waits for the stream to reach the copy)
 *   m0         1 .. POLAR_CONSTRUCT_MAX_OUTPUTS
 *   mu         2 .. POLAR_CONSTRUCT_MAX_MU outputs kept per channel
 *   workspace  device, 256-byte aligned, polar_construct_workspace_bytes
 *              (2^(n-1) + 2^(n-2) channels of mu pairs: 12 GiB at n = 24,
 *              mu = 64)
 *   pe         device out, N doubles
 * Work on the device is asynchronous on stream.  Errors: POLAR_E_INVAL
 * (arguments, w0 not a channel), POLAR_E_NOMEM (workspace too small),
 * POLAR_E_DEVICE.
 */
size_t polar_construct_workspace_bytes(int log2n, int mu, int m0); /* 0 on invalid arguments */
int polar_construct_degrade(int log2n, const double* w0, int m0, int mu, void* workspace, size_t ws_bytes,
                            double* pe, void* stream);

/*
 * Frozen set from per-channel error probabilities (host).  Channels are
 * ranked by pe, largest first, exact ties freezing the lower index first.
 *   n_frozen  >= 0: freeze exactly this many (<= N); -1: the union-bound rule
 *             of Section 3, the largest information set whose pe add up
 *             (best first, one at a time) to at most fer_bound
 *   pe        host, N doubles in [0, 1]
 *   frozen_mask host out, max(1, N/32) words, 1 = frozen; n_frozen_out host out or NULL
 */
int polar_frozen_from_pe(int log2n, const double* pe, int64_t n_frozen, double fer_bound,
                         uint32_t* frozen_mask, int64_t* n_frozen_out);

/*
 * x = u G_N over GF(2) with G_N the n-fold Kronecker power of [[1,0],[1,1]],
 * natural index order (Arikan's construction, cited in Section 3).  Used to
 * re-encode u-hat (x-hat = u-hat G_N) and to build test frames; G_N G_N = I,
 * so the same call also inverts it.
 *
 *   log2n     0 .. POLAR_MAX_LOG2N
 *   n_frames  >= 0; frame k uses words [k W, (k+1) W), W = max(1, N/32)
 *   u, x      device, n_frames * W words each; x may equal u (in place)
 */
int polar_encode(int log2n, int n_frames, const uint32_t* u, uint32_t* x, void* stream);

/* One frame to decode.  All pointers are device pointers; llr is 16-byte
   aligned, the other buffers 4-byte aligned. */
typedef struct polar_frame {
    int32_t log2n;                /* 1 .. POLAR_MAX_LOG2N                              */
    int32_t f_kind;               /* POLAR_F_MINSUM, _BOXPLUS, _MINSUM_Q16, _PHI_Q16 or
                                     _MINSUM_Q8                                        */
    const float* llr;             /* N channel LLRs, 16-byte aligned (fixed-point
                                     kinds: integers, see above)                      */
    const uint32_t* frozen_mask;  /* max(1, N/32) words, 1 = frozen; may be shared      */
    const uint32_t* frozen_vals;  /* max(1, N/32) words, revealed values of u_F;
                                     bits outside the mask are ignored                 */
    uint32_t* u_hat;              /* out, max(1, N/32) words; frozen positions hold
                                     frozen_vals                                       */
    float* leaf_llr;              /* out, N floats (decision LLR of every leaf), or
                                     NULL.  Leaves inside nodes skipped by pruning
                                     are left unwritten.                              */
} polar_frame;

typedef struct polar_ctx polar_ctx;

/* Options for polar_ctx_set_option. */
#define POLAR_OPT_PRUNE 1       /* 0/1: exact rate-0 / rate-1 node shortcuts (default 1) */
#define POLAR_OPT_CUTOVER 2     /* log2 of the subtree decoded by one wavefront from
                                   LDS / registers (larger nodes stream through HBM):
                                   8 .. 12; 0 = automatic (default: the tuned
                                   value, else 12).  Leaf-LLR dumps and unpruned
                                   decoding always use 12.                                */
#define POLAR_OPT_WG_WAVES 3    /* wavefronts per workgroup: 4 or 8; 0 = automatic (8) */
#define POLAR_OPT_MAX_SLOTS 4   /* max workgroups of a launch; 0 = automatic (the tuned
                                   value, else every workgroup that can be resident at
                                   once: compute units x the variant's occupancy).
                                   Never more than can be resident.                     */
#define POLAR_OPT_TIMING 5      /* device pointer (as an integer) to 8 zeroed uint64
                                   counters, or 0 = off.  Decoding then adds, per frame:
                                   [0] ticks spent in register-resident subtree decoding
                                   (the serial leaf region), [1] ticks for the whole
                                   frame, [2] 1.  Ticks are the 100 MHz s_memrealtime
                                   clock, summed over frames in flight.              */
#define POLAR_OPT_FWG 7         /* frames per workgroup for frames of at most 2^cutover
                                   leaves, each decoded by its own wavefront: 1 .. waves
                                   (capped by the LDS the frames' subtree levels need:
                                   4 at 2^12 with cutover 12); 0 = automatic (the tuned
                                   value, else enough to spread the small frames over
                                   every workgroup).  Frames above 2^cutover are decoded
                                   by a whole workgroup each.                          */
#define POLAR_OPT_HELPERS 8     /* 0/1 (default 1): when a batch has fewer frames above
                                   the cutover than workgroups that can be resident,
                                   polar_sc_decode_batch (and the FER harness) launches
                                   the spare ones as helpers that share each frame's
                                   large HBM level sweeps (Section 4's internal
                                   parallelism over the node's elements, across
                                   compute units).  The serving loop never uses them
                                   (its batches share the device).                     */
#define POLAR_OPT_GRAPH 6       /* 0/1: polar_sc_decode_batch replays each distinct batch
                                   (same descriptors, options and workspace) through a
                                   cached HIP graph [descriptor copy, counter reset,
                                   decode].  The host descriptor array is still read at
                                   every call; up to 16 graphs are kept per context.    */

/*
 * Create a decoding context on a device.  The context owns only host-side
 * state (options, a pinned staging buffer for frame descriptors); device
 * scratch is the caller's workspace, attached with polar_ctx_set_workspace.
 * Every call that runs in that workspace (polar_sc_decode_batch, _plain,
 * polar_scl_decode_batch, polar_autotune) reuses it from its start: the
 * caller orders such calls on the device (one stream, or events).  Calls
 * given their own workspace (polar_fer_bsc, polar_construct_degrade) or
 * arena (serving) are independent of it.
 *   device     HIP device ordinal
 *   workspace  device pointer or NULL (attach later)
 *   ws_bytes   size of workspace in bytes
 */
int polar_ctx_create(polar_ctx** out, int device, void* workspace, size_t ws_bytes);
int polar_ctx_destroy(polar_ctx* ctx);
int polar_ctx_set_workspace(polar_ctx* ctx, void* workspace, size_t ws_bytes);
int polar_ctx_set_option(polar_ctx* ctx, int option, int64_t value);
int polar_ctx_get_option(polar_ctx* ctx, int option, int64_t* value);

/*
 * Workspace bytes polar_sc_decode_batch needs for these frames under the
 * context's current options (host array of n_frames descriptors; only log2n
 * and f_kind are read).  Roughly 4N + N/8 bytes per frame in flight.
 * Returns 0 on invalid arguments.
 */
size_t polar_workspace_bytes(const polar_ctx* ctx, const polar_frame* frames, int n_frames);

/*
 * Decode a batch of frames (Section 4's SC rule; Section 4 also notes that SC
 * admits only "external" parallelism across frames, which is how the batch is
 * spread over the GPU).  Frames may differ in N, rate, mask and f_kind.  One
 * persistent launch per f_kind: workgroups take frames from a device queue,
 * longest first.  Results depend only on the frame, not on the batch.
 *   frames    host array of n_frames descriptors (copied before return)
 *   n_frames  >= 0
 * Errors: POLAR_E_INVAL (descriptor), POLAR_E_NOMEM (workspace too small),
 * POLAR_E_DEVICE.
 */
int polar_sc_decode_batch(polar_ctx* ctx, const polar_frame* frames, int n_frames, void* stream);

/*
 * Allocation-free batch decoding, for callers that cannot allocate (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc).  Same frames, options and results as polar_sc_decode_batch,
 * but the workspace is the library's own static device buffer of
 * POLAR_STATIC_SCRATCH_BYTES per device (held by each device the library
 * runs on until the process ends; the context needs no workspace), and the
 * call performs no device, pinned or host heap allocation: its host tables
 * and pinned descriptor buffer are reserved by polar_ctx_create.
 *   n_frames  0 .. POLAR_STATIC_MAX_FRAMES (POLAR_E_INVAL beyond)
 * Frames above 2^cutover leaves need a slot of about 4N + N/8 bytes per
 * workgroup in flight; the call runs as many workgroups as the buffer holds
 * slots for (fewer than polar_sc_decode_batch for large frames) and returns
 * POLAR_E_NOMEM if not even one fits.  Every call on a device shares that
 * device's buffer, which keeps the last call's contents: calls that overlap
 * on one device (two streams, two threads, two contexts) race, so the
 * caller orders them (one stream, or events).
 */
#define POLAR_STATIC_SCRATCH_BYTES ((size_t)256 << 20)
#define POLAR_STATIC_MAX_FRAMES 16384
int polar_sc_decode_batch_static(polar_ctx* ctx, const polar_frame* frames, int n_frames, void* stream);

/*
 * Plain per-frame GPU decoder, kept as the baseline the batched decoder is
 * measured against: one launch per frame, one workgroup, no pruning, frames
 * serially on the stream.  Same arguments, workspace and results.
 */
int polar_sc_decode_plain(polar_ctx* ctx, const polar_frame* frames, int n_frames, void* stream);

/*
 * Autotuner.  Times the built launch configurations on these frames with the
 * context's workspace (configurations that do not fit it are skipped):
 * cutover 8 .. 12, 4 or 8 wavefronts per workgroup, workgroups per launch
 * (half the compute units, all of them, every resident slot), frames per
 * workgroup 1 / 2 / 4 / 8 for frames of at most 2^cutover leaves, and the
 * unpruned decoder; median of reps runs after one warm-up each.  Records the
 * fastest for (f_kind, largest log2n of the frames); later batches whose
 * largest frame has that size use it unless an option is set explicitly.
 * Every configuration gives the same results (the shortcuts are exact).
 * Frames must share one f_kind, must not request leaf LLRs, and pruning must
 * be on in the context.  The frames' u_hat buffers are overwritten.  The
 * best_* outputs describe the launch a batch of these frames now gets;
 * n_candidates the number of configurations timed.  Outputs may be NULL.
 */
int polar_autotune(polar_ctx* ctx, const polar_frame* frames, int n_frames, int reps, void* stream,
                   int* best_cutover, int* best_waves, int* best_slots, int* best_fwg, int* best_prune,
                   double* best_ms, int* n_candidates);

/* Launch configuration a batch of n_frames frames of f_kind, each of 2^log2n
   leaves, would use under the context's options and tuned table. */
int polar_query_launch(const polar_ctx* ctx, int f_kind, int log2n, int n_frames, int* cutover, int* waves,
                       int* slots, int* fwg, int* prune);

/* Tuned table: forget it, or save / load it as JSON
   {"libpolar_tune": 1, "entries": [{"f_kind", "log2n", "cutover", "waves", "slots",
   "fwg", "prune"}, ...]} ("fwg" and "prune" optional on load).  Loading merges
   into the table and rejects out-of-range entries. */
int polar_tune_clear(polar_ctx* ctx);
int polar_tune_save(const polar_ctx* ctx, const char* path);
int polar_tune_load(polar_ctx* ctx, const char* path);

/*
 * Serving (Section 4: frames are independent, so requests are decoded side by
 * side).  Requests (one frame each, caller-owned device buffers that must
 * stay valid until the request completes) are queued, admitted against a
 * caller-provided device arena and decoded in batches by the batch decoder on
 * up to three internal streams at once: a new batch starts on an idle stream
 * with the requests that have arrived, in arrival order, as many as fit the
 * free arena (and at most max_slots), while earlier batches still run.  One
 * of the streams takes only requests of at most 2^17 bits, so that small
 * requests never wait for a stream behind batches of large frames.  Each
 * request is charged its own footprint in the arena: a 64-byte descriptor
 * plus, above 2^12 leaves, a scratch slot of about 4N + N/8 bytes for its own
 * N (256 bytes of counters per batch).  A request too large for the whole
 * arena completes with POLAR_E_NOMEM.
 *
 * Ordering: a batch starts only after all work enqueued on input_stream
 * before the batch was formed, so request inputs (LLRs, frozen words, and
 * any fill of u_hat) produced on that stream before submit are complete when
 * they are read.  Inputs produced on other streams must be synchronised by
 * the caller before submit.
 *
 * Completion is per request: the decoder flags a frame as soon as its u_hat
 * is written and globally visible, and the next poll reports it, while the
 * rest of its batch may still run.  Results equal those of decoding the
 * frame alone.  Latency is host time from submit to the poll that sees the
 * request's flag.  A server is used from one host thread.
 */
typedef struct polar_serve_cfg {
    size_t arena_bytes;  /* >= 4096                                             */
    void* arena;         /* device, 256-byte aligned, caller-owned               */
    int max_slots;       /* max requests per batch; 0 = the workgroups of the
                            default decoder that can be resident at once        */
    int poll_us;         /* idle sleep of polar_serve between polls (0 = spin)   */
    void* input_stream;  /* stream the request inputs are produced on (NULL =
                            the null stream); see Ordering above                */
} polar_serve_cfg;

typedef struct polar_completion {
    uint64_t req_id;
    int32_t status;      /* POLAR_OK, POLAR_E_NOMEM, POLAR_E_CANCELLED, POLAR_E_DEVICE */
    int32_t reserved;
    double latency_s;
} polar_completion;

typedef struct polar_server polar_server;

int polar_serve_open(polar_ctx* ctx, const polar_serve_cfg* cfg, polar_server** out);
/* Queue a request (copied).  POLAR_E_BUSY when 65536 requests are queued. */
int polar_serve_submit(polar_server* srv, const polar_frame* req, uint64_t req_id);
/* Reap finished batches, start new ones, and return up to max_out completions. */
int polar_serve_poll(polar_server* srv, polar_completion* out, int max_out, int* n_out);
/* Requests waiting, running, and completed but not yet returned by a poll. */
int polar_serve_pending(const polar_server* srv, int* queued, int* running, int* completed);
/* Batches on the device (at most four) and the arena bytes they hold; a
   batch is counted until the poll that finds its last work finished. */
int polar_serve_stats(const polar_server* srv, int* batches_running, size_t* arena_used);
/* Cancel a queued request (it completes with POLAR_E_CANCELLED); POLAR_E_BUSY
   if it is already running, POLAR_E_INVAL if unknown. */
int polar_serve_cancel(polar_server* srv, uint64_t req_id);
/* Wait for running batches and free the server; queued requests are dropped. */
int polar_serve_close(polar_server* srv);

/*
 * Blocking loop over the calls above: next() is asked for requests until it
 * returns 1 (none yet) or 2 (no more); done() is called once per request
 * (also for requests refused at submit, with latency 0).  Returns when next()
 * has returned 2 and every request has completed.
 */
typedef int (*polar_next_fn)(void* user, polar_frame* req, uint64_t* req_id); /* 0 ok, 1 none yet, 2 end */
typedef void (*polar_done_fn)(void* user, uint64_t req_id, int status, double latency_s);
int polar_serve(polar_ctx* ctx, const polar_serve_cfg* cfg, polar_next_fn next, polar_done_fn done, void* user);

/*
 * Frame-error-rate harness (Table 1's FER at a code rate; Section 2.1 eq. (5)
 * puts the FER into the key rate; Section 3 sizes frozen sets for FER 0.1):
 * synthetic BSC frames generated on the device, decoded by the batch decoder
 * and checked against the transmitted u, all on the GPU.
 *
 * Frames come from the counter-based generator Philox4x32-10 (Salmon et al.,
 * SC'11), so frame f depends only on (seed, f):
 *   key = (seed mod 2^32, f)
 *   u word w             = Philox((w >> 2, 0, 0, 0), key)[w & 3]
 *                          (N < 32: the low N bits of word 0)
 *   channel error, bit i = Philox((i >> 2, 1, 0, 0), key)[i & 3] < floor(p 2^32)
 *   x = u G_N; L_i = +L0 where x_i equals the error bit, else -L0, with
 *   L0 = ln((1 - p) / p) computed in double and rounded once to float32
 *   (fixed_point = 1, and the 16-bit fixed-point f_kinds of polar_fer_bsc: L0
 *   in units of 2^-POLAR_FIXED_FRAC, rounded half to even; fixed_point = 2,
 *   and POLAR_F_MINSUM_Q8: in units of 2^-POLAR_FIXED8_FRAC, rounded half to
 *   even and capped at POLAR_FIXED8_MAX)
 *   frozen values = u on the frozen set
 * A frame is in error when its u-hat differs from u in any position.
 *
 * polar_fer_generate_bsc writes frames frame0 .. frame0 + n_frames - 1:
 *   u, frozen_vals, x_scratch  device, n_frames * max(1, N/32) words each
 *   llr                        device, n_frames * N floats, 16-byte aligned
 * polar_fer_bsc generates, decodes (under the context's options) and counts
 * cfg->n_frames frames in steps of cfg->batch, in caller memory: workspace of
 * polar_fer_workspace_bytes (256-byte aligned), bit_errors (device, one
 * uint32 per frame: u-hat bits that differ from u).  It synchronises the
 * stream before filling *out (host).
 */
typedef struct polar_fer_cfg {
    int32_t log2n;                /* 1 .. POLAR_MAX_LOG2N                              */
    int32_t f_kind;               /* any POLAR_F_* check update                        */
    double p;                     /* BSC crossover probability, 0 < p < 1/2            */
    const uint32_t* frozen_mask;  /* device, max(1, N/32) words, 1 = frozen            */
    uint64_t seed;                /* low 32 bits used                                  */
    int64_t frame0;               /* first frame index; frame indices < 2^32           */
    int64_t n_frames;             /* >= 0                                              */
    int32_t batch;                /* frames per step; 0 = automatic                    */
    int32_t reserved;
} polar_fer_cfg;

typedef struct polar_fer_result {
    int64_t frames;
    int64_t frame_errors;
    int64_t bit_errors;
} polar_fer_result;

int polar_fer_generate_bsc(int log2n, double p, int fixed_point, const uint32_t* frozen_mask, uint64_t seed,
                           int64_t frame0, int n_frames, uint32_t* u, uint32_t* frozen_vals,
                           uint32_t* x_scratch, float* llr, void* stream);
/* Returns 0 on invalid arguments. */
size_t polar_fer_workspace_bytes(const polar_ctx* ctx, const polar_fer_cfg* cfg);
int polar_fer_bsc(polar_ctx* ctx, const polar_fer_cfg* cfg, void* workspace, size_t ws_bytes,
                  uint32_t* bit_errors, polar_fer_result* out, void* stream);

/*
 * SC list decoding (Section 4 names list decoders as the improvement over
 * SC).  Each frame keeps up to list_size paths; f and g are the FP32 min-sum
 * updates of POLAR_F_MINSUM, and each path carries the LLR path metric:
 *   frozen leaf:  u = frozen value; PM += |lambda| if u != [lambda < 0]
 *   info leaf:    path p offers u = b, b = 0, 1, with PM_p + |lambda| when
 *                 b != [lambda < 0] (else PM_p); candidates ordered by
 *                 (metric, p, b), the first min(list_size, count) are the
 *                 new paths in that order
 * u_hat receives the path of least metric (ties to the lower path).  With
 * min-sum updates the metric of a complete path equals the correlation
 * discrepancy sum_j |L_j| [x_j != (L_j < 0)] of its codeword, so with
 * list_size >= 2^K the result is a max-log maximum-likelihood codeword.
 *
 *   frames       host array as for polar_sc_decode_batch; f_kind must be
 *                POLAR_F_MINSUM, leaf_llr NULL, and N x list_size <=
 *                POLAR_SCL_MAX_NL (every path's state is on chip)
 *   list_size    1 .. POLAR_SCL_MAX_LIST (1 is SC)
 *   path_metric  device, n_frames floats (the chosen path's metric), or NULL
 * Uses the context's workspace for the descriptor table
 * (polar_scl_workspace_bytes).  Asynchronous on stream.  Errors:
 * POLAR_E_INVAL, POLAR_E_NOMEM (workspace), POLAR_E_DEVICE.
 */
size_t polar_scl_workspace_bytes(int n_frames);
int polar_scl_decode_batch(polar_ctx* ctx, const polar_frame* frames, int n_frames, int list_size,
                           float* path_metric, void* stream);

/*
 * Diagnostics: exercises the cross-lane moves (DPP row shifts, permlane
 * swaps), the bit-matrix transpose and the cross-lane polar transform the
 * decoder is built from.  out: device, 1024 words.
 */
int polar_debug_lane_selftest(uint32_t* out, void* stream);

/* Diagnostics: the 256-entry phi table T of POLAR_F_PHI_Q16 as the decoder
   builds it on the device (FP64 on the GPU), as floats.  out: device, 256
   floats. */
int polar_debug_phi_table(float* out, void* stream);

#ifdef __cplusplus
}
#endif

#endif /* POLAR_H */
