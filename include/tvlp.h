/*
 * tvlp.h — C ABI of the MI355X (gfx950) time-varying linear-prediction filter.
 *
 * The operation (paper Sec. 3.2, Eq. 6): for every sequence b,
 *     s(t) = e(t) - sum_{i=1..M} a_i(t) s(t-i),      t = 0 .. T-1,
 * with zero initial conditions s(t) = e(t) = 0 for t < 0 (Sec. 2.2), unless an
 * initial state zi is given.  The coefficient row a(t) belongs to the output
 * time t.  Its adjoint (Eqs. 12-13): with g(t) = dL/ds(t),
 *     ghat(t) = g(t) - sum_{i=1..M} a_i(t+i) ghat(t+i),   ghat(t >= T) = 0,
 *     dL/de(t) = ghat(t),      dL/da_i(t) = -ghat(t) s(t-i).
 *
 * Layout (all row-major, contiguous):
 *   e, s, g, grad_e  float32 [B][T]        (packed [N] for the varlen calls)
 *   a, grad_a        float32 [B][T][M]     (packed [N][M])
 *   zi, zf, grad_zi  float64 [B][M]        zi[b][j-1] = s(-j), zf[b][j-1] = s(T-j)
 *   offsets          int64   [B+1]         device array, offsets[0] = 0, non-decreasing
 * Every pointer passed to lp_forward* / lp_backward* is a DEVICE pointer on the
 * plan's device; `stream` is a hipStream_t (NULL = default stream).  Results
 * are float32; all internal arithmetic (recursions, chunk transitions, carried
 * states) is float64.
 *
 * Ownership: the caller owns every buffer it passes; the library never frees
 * caller memory.  A plan owns a device workspace that grows on demand
 * (lp_plan_reserve sizes it up front, which callers that capture launches into
 * a hipGraph must do).  Calls are asynchronous on `stream`.
 *
 * Errors: every call returns an int status (LP_OK = 0, negative on error) and
 * never throws.  lp_last_error() returns a thread-local message for the most
 * recent failure.  Invalid arguments (B < 1, T < 1, M outside [1, 64], NULL
 * required pointers, an unsupported order for the chunked kernels) give
 * LP_EINVAL and launch nothing; device failures give LP_EDEVICE.  Non-finite
 * inputs are not errors: they propagate through the recursion, and
 * lp_forward / lp_backward report per sequence whether any output is
 * non-finite (their `nonfinite` argument).
 */
#ifndef TVLP_H
#define TVLP_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct lp_plan lp_plan;
typedef struct lp_graph lp_graph;

enum {
    LP_OK = 0,
    LP_PENDING = 1,
    LP_EINVAL = -1,
    LP_ENOMEM = -2,
    LP_EDEVICE = -3,
    LP_ENOTFOUND = -4,
    LP_EBUDGET = -5
};

/* Plan flags.
 * LP_FLAG_CHAINED_CARRY: the chunk-to-chunk carry applies each chunk's
 *   transition to the carried state in turn (one group of chunks after the
 *   other) instead of composing transitions into group matrices first.  The
 *   composed products can lose accuracy on strongly resonant, fast-varying
 *   filters (time-varying pole radii near 1, where single transitions already
 *   have entries in the thousands); the chained carry keeps the rounding error
 *   at the level of one transition, at the cost of a serial dependency between
 *   consecutive groups of a sequence.
 * LP_FLAG_HIGH_RADIUS: for inputs whose frozen poles come close to the unit
 *   circle (radius above about 0.99, or tracks that are briefly unstable
 *   within frames).  Implies LP_FLAG_CHAINED_CARRY, makes the plan's default
 *   chunk length the longest its order supports (at most 2048), and restricts
 *   lp_plan_autotune to chunk lengths of at least 1536 (or that longest one):
 *   over short chunks single transitions of such filters have entries in the
 *   thousands, and chaining many of them loses the result; over long chunks the
 *   transient dies out inside the chunk.  lp_plan_set_chunk still accepts any
 *   length. */
enum {
    LP_FLAG_NONE = 0,
    LP_FLAG_CHAINED_CARRY = 1,
    LP_FLAG_HIGH_RADIUS = 2
};

/* Library version string, e.g. "tvlp 0.1 gfx950". */
const char *lp_version(void);

/* Thread-local description of the last non-OK return on this thread. */
const char *lp_last_error(void);

/* Orders M for which the chunked kernels are compiled (1, 2, 3, 4, 6, 8, 10,
 * 12, 16, 20, 22, 24, 32: every order the paper's configurations use, with
 * a register and LDS mapping tuned per order); returns the count and writes
 * up to `cap` of them to `out` (which may be NULL).  The sequential kernels
 * (lp_forward_plain / lp_backward_plain) take any M in [1, 64]. */
int lp_supported_orders(int *out, int cap);

/* Create a plan for filter order M on `device`.  The plan selects the chunk
 * length L (a multiple of M, at least M) used by the chunked kernels.  `flags`
 * is a combination of the LP_FLAG_* values (others: LP_EINVAL).  M outside
 * [1, 64], or an order with no compiled chunked kernels (lp_supported_orders),
 * gives LP_EINVAL with the reason in lp_last_error. */
int lp_plan_create(lp_plan **out, int device, int M, int flags);
/* Frees the plan and its workspace (after a device synchronisation).  LP_EINVAL,
 * and nothing freed, while a captured graph of the plan exists. */
int lp_plan_destroy(lp_plan *p);

/* Override / query the chunk length.  L must be a positive multiple of M and
 * at most 2048 (at most about 1200 for M < 8, where the adjoint kernel keeps 16
 * chunks per wave in LDS); LP_EINVAL otherwise. */
int lp_plan_set_chunk(lp_plan *p, int L);
int lp_plan_get_chunk(const lp_plan *p);

/* Carry mode: 1 for the chained carry (LP_FLAG_CHAINED_CARRY), 0 for group
 * maps.  Setting 0 or 1 fixes the mode for the autotuner; -1 keeps the current
 * mode and leaves the choice to the autotuner again.  A high-radius plan
 * accepts only 1; other values give LP_EINVAL.  Both modes use the same
 * workspace and saved state, so a forward and its adjoint may run in
 * different modes.  lp_plan_get_carry returns -1 for a NULL plan. */
int lp_plan_set_carry(lp_plan *p, int mode);
int lp_plan_get_carry(const lp_plan *p);

/* Chunk-length autotuner (the launch mapping: chunk length L, hence the
 * number of chunks and of waves per sequence, and the carry mode): times one
 * forward + recompute-adjoint step of a B x T batch (B capped so that the
 * timed batch holds about 32 M samples) for candidate chunk lengths near
 * 64 .. 1024 samples (multiples of M) and, unless the caller fixed the carry
 * mode (a carry flag at creation, or lp_plan_set_carry), both carry modes;
 * `reps` timed repetitions each after one warm-up; keeps the fastest on the
 * plan.  Allocates and frees its own buffers, filled with deterministic
 * stand-in data (e and g uniform in [-1, 1), coefficients of a stable filter
 * below 0.9/M in magnitude: the kernels' time depends on the values through
 * their power draw, so zeros would favour the wrong candidates), and
 * synchronises the device.  Writes the chosen L and
 * its best step time in ms (either pointer may be NULL; the carry mode is read
 * back with lp_plan_get_carry).  On error the plan keeps its previous chunk
 * length and carry mode. */
int lp_plan_autotune(lp_plan *p, int64_t B, int64_t T, int reps, int *chosen, double *best_ms);

/* Per-kernel timing.  When on, every kernel the plan launches is bracketed by
 * hipEvents recorded on the launch stream.  lp_plan_timings waits for the
 * recorded events, adds their durations to per-kernel totals and writes up to
 * `cap` entries: names (cap x name_len chars, NUL-terminated), total
 * milliseconds and launch counts.  Returns the number of kernels seen. */
int lp_plan_set_timing(lp_plan *p, int on);
int lp_plan_timings(lp_plan *p, char *names, int name_len, double *ms, int64_t *launches, int cap);
int lp_plan_reset_timings(lp_plan *p);

/* Synchronises the device and reports whether a segment table of this plan
 * (lp_forward_segments) held more samples than its total_bound since the last
 * check.  Returns LP_OK, or LP_EINVAL and clears the flag; LP_EDEVICE if the
 * device reports an error. */
int lp_plan_status(lp_plan *p);

/* Grow the plan's workspace for a batch of B sequences of length T (or, for
 * varlen use, a total of N samples in B sequences: pass T = ceil(N / B) + L). */
int lp_plan_reserve(lp_plan *p, int64_t B, int64_t T);

/*
 * lp_forward without any device allocation, for callers that cannot allocate:
 * code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  Same arguments, kernels and results as lp_forward, except:
 *   - `saved` is required (lp_saved_bytes(p, B, T) bytes, caller-owned);
 *   - the workspace (chunk offsets, group maps and carries, the zero block the
 *     row DMA reads) is the library's static per-device scratch of 16 MiB
 *     (16 << 20 bytes), looked up and cleared when a plan is created on that
 *     device, not the plan's own allocation; a call whose workspace exceeds it
 *     returns LP_EINVAL and launches nothing (64 x 48000 samples at M = 22
 *     need about 8.3 MB at the default chunk length, 5.4 MB at 418);
 *   - no timing events are recorded for it.
 * Every call on one GPU shares that GPU's scratch, which keeps the last call's
 * contents: calls that overlap on one GPU (on different streams or threads)
 * race and must be serialised by the caller.  No hipMalloc, hipFree or other
 * allocating routine is called.
 */
int lp_forward_noalloc(lp_plan *p, int64_t B, int64_t T, const float *e, const float *a,
                       const double *zi, float *s, double *zf, void *saved, uint32_t *nonfinite,
                       void *stream);

/* Bytes of the `saved` buffer that lp_forward fills for lp_backward: the
 * float64 chunk-entry states and chunk transition matrices (Sec. 3.2 method,
 * chunked form; the backward recomputes s(t) per chunk from them). */
size_t lp_saved_bytes(const lp_plan *p, int64_t B, int64_t T);
size_t lp_saved_bytes_varlen(const lp_plan *p, int64_t B, int64_t N);

/*
 * Chunked forward (Eq. 6).  e [B,T], a [B,T,M] -> s [B,T].
 * zi: optional [B,M] initial state (NULL = zero initial conditions).
 * zf: optional [B,M] final state out.
 * saved: optional, lp_saved_bytes(p,B,T) bytes, filled for lp_backward; when
 *        NULL the plan's workspace holds the intermediates.
 * nonfinite: optional [B] device array of uint32 flags: the call sets
 *        nonfinite[b] = 1 when some s(t) of sequence b is Inf or NaN (a
 *        non-finite input, or a recursion that overflows), else 0.  Non-finite
 *        values are not an error: they propagate, and other sequences are not
 *        affected.
 */
int lp_forward(lp_plan *p, int64_t B, int64_t T,
               const float *e, const float *a, const double *zi,
               float *s, double *zf, void *saved, uint32_t *nonfinite, void *stream);

/*
 * Chunked adjoint (Eqs. 12-13).  g [B,T] = dL/ds; a, e, zi as given to the
 * lp_forward call that filled `saved` (required).  s: the forward output, or
 * NULL to recompute s(t) chunk by chunk from `saved`.  Outputs (each may be
 * NULL if not wanted): grad_e [B,T], grad_a [B,T,M], grad_zi [B,M], and
 * nonfinite [B] (uint32): 1 when some dL/de(t) or dL/da_i(t) of sequence b is
 * Inf or NaN, else 0 (as for lp_forward, not an error).
 */
int lp_backward(lp_plan *p, int64_t B, int64_t T,
                const float *g, const float *a, const float *e, const double *zi,
                const float *s, const void *saved,
                float *grad_e, float *grad_a, double *grad_zi, uint32_t *nonfinite, void *stream);

/*
 * Time-invariant coefficients (the all-pole filter of Sec. 2.2, Eqs. 2-4, with
 * one coefficient row per sequence): the same chunked forward and adjoint, with
 * a [B,M] (row b used at every sample of sequence b) instead of [B,T,M].
 * Everything else as for lp_forward / lp_backward: the saved buffer, zi, zf,
 * stored or recomputed s, grad_e [B,T], grad_zi [B,M].  grad_a is [B,M]:
 * dL/da_i = -sum_t ghat(t) s(t-i) (Eq. 4, from the single backward filter of
 * Sec. 3.2), accumulated per chunk in float64 and summed per sequence.
 * Uniform batches only.  Error behaviour as for lp_forward / lp_backward.
 */
int lp_forward_ti(lp_plan *p, int64_t B, int64_t T,
                  const float *e, const float *a, const double *zi,
                  float *s, double *zf, void *saved, void *stream);
int lp_backward_ti(lp_plan *p, int64_t B, int64_t T,
                   const float *g, const float *a, const float *e,
                   const double *zi, const float *s, const void *saved,
                   float *grad_e, float *grad_a, double *grad_zi, void *stream);

/*
 * Frame-rate coefficients (the pipeline of Sec. 4.3: LP coefficients produced
 * once per analysis frame and linearly upsampled to the sample rate).  A
 * [B,F,M] holds one row per frame, frame q at sample q*hop of its sequence, F =
 * lp_coef_frames_count(T, hop) = (T - 1) / hop + 2 (the last sample has a right
 * neighbour).  Sample t = q*hop + n (0 <= n < hop) uses
 *   a(t) = A[q] + n (A[q+1] - A[q]) / hop,
 * interpolated inside the kernels (evaluated in float64, rounded once to
 * float32, the precision of the per-sample rows), so no [B,T,M] array is read
 * or written.  lp_forward_frames is lp_forward with those rows (same saved buffer,
 * zi, zf); lp_backward_frames is lp_backward with grad_A [B,F,M] = dL/dA in place
 * of grad_a: each sample hands (1 - n/hop) of dL/da(t) = -ghat(t) s(t-i) (Eq. 13)
 * to frame q and n/hop to frame q + 1, accumulated per chunk in float64 and
 * summed per frame.  Uniform batches only; hop in [1, 2^20].  Errors: LP_EINVAL
 * for bad sizes or pointers, or when hop is so short against the plan's chunk
 * length that the frame rows one chunk touches ((L - 1) / hop + 3 of them) do not
 * fit in LDS; otherwise as for lp_forward / lp_backward.
 */
int64_t lp_coef_frames_count(int64_t T, int64_t hop);
int lp_forward_frames(lp_plan *p, int64_t B, int64_t T, int64_t hop,
                      const float *e, const float *A, const double *zi,
                      float *s, double *zf, void *saved, void *stream);
int lp_backward_frames(lp_plan *p, int64_t B, int64_t T, int64_t hop,
                       const float *g, const float *A, const float *e,
                       const double *zi, const float *s, const void *saved,
                       float *grad_e, float *grad_A, double *grad_zi, void *stream);

/*
 * Source-filter synthesiser around the LP filter (Eq. 5, S = (G + N C) H, with
 * the trainable output FIR): the pieces that wrap lp_forward_frames /
 * lp_backward_frames.  Signals are [B,T] float32; frames as for the frame-rate
 * coefficients (frame q at sample q*hop, F = lp_coef_frames_count(T, hop));
 * device pointers, caller-owned; enqueued on `stream`.  Errors: LP_EINVAL for
 * sizes out of range (B <= 65535, 1 <= hop <= 4096, 1 <= K <= 1024) or null
 * pointers, LP_EDEVICE for a failed launch; the message is lp_sf_last_error().
 *
 * lp_sf_source: u(t) = p(t) + sum_k C[q(t-k)][k] n(t-k), the noise n filtered
 * frame-wise (each hop-sample input frame q convolved with its own K taps
 * C[q] from C [B,F,K], results overlap-added) plus the pulse source p; and the
 * LP input x(t) = gamma(t) u(t), gamma linearly upsampled from gain [B,F].
 * lp_sf_source_adjoint: from gx = dL/dx: gu = dL/du = dL/dp [B,T] (written),
 * gC = dL/dC [B,F,K], ggain = dL/dgain [B,F].
 * lp_fir: y(t) = sum_k h[k] s(t-k), h [K] shared by all sequences.
 * lp_fir_adjoint: gs = dL/ds [B,T] and gh = dL/dh [K] (each may be NULL);
 * gh needs `work`, lp_fir_adjoint_work_bytes(B, T, K) bytes of device memory
 * (per-tile partial sums, summed in float64 in a fixed order).
 */
const char *lp_sf_last_error(void);
int lp_sf_source(int64_t B, int64_t T, int64_t hop, int64_t K, const float *p, const float *n,
                 const float *C, const float *gain, float *u, float *x, void *stream);
int lp_sf_source_adjoint(int64_t B, int64_t T, int64_t hop, int64_t K, const float *gx, const float *u,
                         const float *n, const float *gain, float *gu, float *gC, float *ggain, void *stream);
int lp_fir(int64_t B, int64_t T, int64_t K, const float *s, const float *h, float *y, void *stream);
size_t lp_fir_adjoint_work_bytes(int64_t B, int64_t T, int64_t K);
int lp_fir_adjoint(int64_t B, int64_t T, int64_t K, const float *gy, const float *s, const float *h,
                   float *gs, float *gh, void *work, void *stream);

/*
 * Frame-wise approximation (the comparator of Sec. 3.2: time-invariant filtering
 * of short overlapping frames, overlap-added; 75 % overlap as in Sec. 5).  Frames
 * have length W = 4 hop; frame f of a sequence starts at sample (f - 3) hop and
 * there are F = lp_frames_count(T, hop) = ceil(T / hop) + 3 of them, so every
 * sample lies in exactly four frames.  With weighting on, a frame value at
 * position n is multiplied by w(n) / 2, w the periodic Hann window
 * sin^2(pi n / W) (the four shifted windows sum to 2).
 *
 * lp_frames_gather: xf [B,F,W] <- x [B,T] (zero outside the signal).
 * lp_frames_overlap_add: x [B,T] <- sum over the four frames holding each
 * sample of xf [B,F,W] (the adjoint of lp_frames_gather with the same weighting).
 *
 * The frame-wise filter is gather (unweighted) -> lp_forward_ti over the B*F
 * frames with their coefficient rows af [B*F,M] -> overlap-add (weighted); its
 * adjoint is gather (weighted) of dL/ds -> lp_backward_ti -> overlap-add
 * (unweighted) of the frames' dL/de.  Device pointers, caller-owned; errors:
 * LP_EINVAL for sizes < 1 or missing pointers.
 */
int64_t lp_frames_count(int64_t T, int64_t hop);
int lp_frames_gather(int64_t B, int64_t T, int64_t hop, const float *x, float *xf, int weighted, void *stream);
int lp_frames_overlap_add(int64_t B, int64_t T, int64_t hop, const float *xf, float *x, int weighted,
                          void *stream);

/* Variable-length batches: sequence b occupies samples [offsets[b], offsets[b+1])
 * of the packed arrays e [N], a [N,M], s [N] (N = offsets[B]).  `offsets` is a
 * device array; `N` must equal offsets[B].  Chunk boundaries are relative to
 * each sequence's own start, so a sequence's result does not depend on what
 * else is in the batch. */
int lp_forward_varlen(lp_plan *p, int64_t B, const int64_t *offsets, int64_t N,
                      const float *e, const float *a, const double *zi,
                      float *s, double *zf, void *saved, void *stream);
int lp_backward_varlen(lp_plan *p, int64_t B, const int64_t *offsets, int64_t N,
                       const float *g, const float *a, const float *e, const double *zi,
                       const float *s, const void *saved,
                       float *grad_e, float *grad_a, double *grad_zi, void *stream);

/* Segment tables: sequence b occupies samples [starts[b], starts[b] + lens[b])
 * of arrays with N samples (device int64 arrays; segments need not be packed
 * or ordered but must not overlap; lens[b] may be 0, which leaves zf[b]
 * untouched).  total_bound > 0 is an upper bound on sum(lens) that sizes the
 * launch (0: N); if the table holds more, the excess is not computed and the
 * next lp_plan_status returns LP_EINVAL.  zi / zf are [B][M] and may alias
 * (every state is read before any is written), which lets a caller continue
 * sequences slice by slice from device-resident state; the result then
 * differs from one call over the whole sequence only by the rounding of the
 * float64 chunk states.  Forward only (serving path). */
int lp_forward_segments(lp_plan *p, int64_t B, const int64_t *starts, const int64_t *lens, int64_t N,
                        int64_t total_bound, const float *e, const float *a, const double *zi,
                        float *s, double *zf, void *stream);

/*
 * Harmonic-plus-noise filter pair (Eq. 1: S = G H + N C with two LP filters per
 * item): both filters of every item run in one launch per direction as a
 * stacked batch of 2B sequences.
 *   e2 [2][B][T], a2 [2][B][T][M]: filter 0 (e.g. H on the glottal pulses)
 *   then filter 1 (C on the noise); s2 [2][B][T] receives both outputs and
 *   y [B][T] = s2[0] + s2[1].  saved: lp_saved_bytes_pair(p, B, T) bytes.
 * The adjoint takes the single upstream gradient g = dL/dy [B][T] (shared by
 * both filters) and writes ge2 [2][B][T], ga2 [2][B][T][M] (either may be
 * NULL); s2 may be passed to skip recomputing s, or NULL.
 */
size_t lp_saved_bytes_pair(const lp_plan *p, int64_t B, int64_t T);
int lp_forward_pair(lp_plan *p, int64_t B, int64_t T, const float *e2, const float *a2,
                    float *y, float *s2, void *saved, void *stream);
int lp_backward_pair(lp_plan *p, int64_t B, int64_t T, const float *g, const float *a2,
                     const float *e2, const float *s2, const void *saved,
                     float *ge2, float *ga2, void *stream);

/*
 * hipGraph capture of one full pair step (forward, sum, adjoint) with fixed
 * buffers; the plan's workspace is reserved before capture, so replays launch
 * kernels only (no allocation, no memset).  Replays reuse the captured
 * pointers: refill the input buffers between replays.  store_s != 0 makes the
 * adjoint read s2 instead of recomputing it.  A plan must not be used by
 * other calls while one of its graphs is running.
 * A graph keeps the address of its plan's workspace.  Until every graph of a
 * plan is destroyed the plan refuses, with LP_EINVAL and nothing launched or
 * freed, whatever would move or free that workspace or change the layout the
 * graph was captured with: a call that needs a larger workspace, a change of
 * chunk length (lp_plan_set_chunk, lp_plan_autotune) and lp_plan_destroy.
 * Calls that fit the reserved workspace remain allowed between replays.
 * lp_graph_destroy releases the graph's hold on the plan.
 */
int lp_graph_capture_pair_step(lp_plan *p, int64_t B, int64_t T, const float *e2, const float *a2,
                               float *y, float *s2, void *saved, const float *g,
                               float *ge2, float *ga2, int store_s, lp_graph **out);
int lp_graph_launch(lp_graph *g, void *stream);
int lp_graph_destroy(lp_graph *g);

/*
 * Serving runtime (continuous batching of forward-filter jobs, Sec. 3.2's
 * filter applied per request).  A server owns an HBM arena of
 * hbm_budget_bytes for the inputs and outputs of admitted jobs
 * ((M + 2) * 4 bytes per sample), max_slots device-resident float64 filter
 * states, and a scheduler thread.  Jobs are admitted in submission order while
 * a slot and arena space are free; every scheduler iteration advances each
 * running job by up to slice_len samples (rounded up to a multiple of the
 * chunk length; <= 0 picks 48 chunks) with one lp_forward_segments launch over
 * all slots, so short jobs finish while long ones keep running.  Inputs are
 * uploaded and outputs downloaded on their own streams, overlapping compute.
 *
 * lp_serve_submit copies nothing at call time: e_host [T], a_host [T][M] must
 * stay valid and s_host_out [T] must stay writable until the job completes
 * (pinned host memory makes the copies asynchronous).  Zero initial state.
 * A job's result does not depend on the other jobs in flight (bit-identical to
 * running it alone through a server with the same slice_len).
 * Returns: submit LP_EBUDGET if T exceeds the whole arena; poll / wait
 * LP_PENDING while the job runs, LP_OK once s_host_out holds the result (the
 * ticket is then retired: a second poll gives LP_ENOTFOUND), LP_EDEVICE if it
 * failed; latency_ms_out (may be NULL) receives submit-to-completion time
 * (host clock: queueing, upload, compute and download); lp_serve_wait's
 * device_ms_out (may be NULL) receives the job's time on the device, from the
 * launch of its first slice to the end of its last one (shared with the other
 * jobs in flight; no queueing, no copies).
 * lp_serve_destroy finishes every admitted and queued job, then frees all.
 * All functions are thread-safe.
 */
typedef struct lp_server lp_server;
int lp_serve_create(lp_server **out, int device, int M, size_t hbm_budget_bytes, int max_slots,
                    int64_t slice_len, int flags);
int lp_serve_submit(lp_server *srv, int64_t T, const float *e_host, const float *a_host,
                    float *s_host_out, uint64_t *ticket);
int lp_serve_poll(lp_server *srv, uint64_t ticket, double *latency_ms_out);
int lp_serve_wait(lp_server *srv, uint64_t ticket, double timeout_s, double *latency_ms_out,
                  double *device_ms_out);
int lp_serve_stats(lp_server *srv, int64_t *iterations, int64_t *samples, int64_t *jobs_done,
                   int64_t *queued, int64_t *active);
int lp_serve_destroy(lp_server *srv);

/*
 * Sequential baseline: one GPU thread per sequence runs Eq. 6 (forward) and
 * the adjoint of Eqs. 12-13 (backward, which reads the stored forward output
 * s) straight through, float64 arithmetic, float32 I/O.  Same layouts as above.
 */
int lp_forward_plain(int M, int64_t B, int64_t T, const float *e, const float *a,
                     const double *zi, float *s, double *zf, void *stream);
int lp_backward_plain(int M, int64_t B, int64_t T, const float *g, const float *a,
                      const double *zi, const float *s,
                      float *grad_e, float *grad_a, double *grad_zi, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* TVLP_H */
