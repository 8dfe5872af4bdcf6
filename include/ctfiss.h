/*
 * ctfiss.h -- C ABI of the MI355X (gfx950) CTF-MNMF-ISS separation library.
 *
 * Blind source separation by convolutive-transfer-function multichannel NMF
 * (Xie et al., APSIPA ASC 2025).  Given the STFT of an M-channel mixture, the
 * library minimises the negative log-likelihood of Eq. (5) over the
 * per-bin extended demixing matrices W_f and the NMF source model
 * lambda_{n,f,t} = sum_k b_{n,f,k} v_{n,k,t} (Sec. II, problem statement
 * Eq. (6)), and returns the separated source images of Sec. III-B.
 *
 * Shapes and layouts (all device buffers are dense, row-major, caller-owned):
 *   X  [M][F][T]       observed STFT, complex, interleaved (re, im)
 *   W  [F][Mbar][Mbar] extended demixing matrices; row r of W_f holds w_r^H
 *                      (Sec. II, demixing Eq. (4)), Mbar = M * D
 *   B  [N][F][K]       NMF bases b_{n,f,k} (real)
 *   V  [N][K][T]       NMF activations v_{n,k,t} (real)
 *   C  [N][M][F][T]    source images (complex)
 * Scalar type: precision CTFISS_FP32 uses complex64 / float32 for every
 * buffer above, CTFISS_FP64 uses complex128 / float64.  CTFISS_MIXED (ISS
 * rule only, single contexts) takes the FP32 buffers and kernels, except that
 * the ISS sweep updates the rows of W in FP64 registers (each row of W_f gets
 * Mbar rank-one updates per iteration; holding them in FP64 leaves one FP32
 * rounding of W per iteration instead of Mbar).  Same layout and workspace as
 * CTFISS_FP32.  CTFISS_MIXED_BF16 (also ISS, single contexts) is CTFISS_MIXED
 * with the contractions of the source model -- lambda = b v and the sums of the
 * multiplicative updates of Eqs. (17) and (18) -- on bfloat16 matrix cores
 * (operands rounded to bfloat16, products accumulated in FP32); the weights,
 * square roots and everything else stay FP32.
 *
 * Rows of W: r = L_0 + ... + L_{n-1} + l is tap l of source n (source-major,
 * tap-minor, the flattened index of Sec. III-A-1).  The observation may stack
 * D delayed frames, xbar_{f,t}[d*M + m] = x_{m,f,t-d} (zero before the first
 * frame); D = 1 is the paper's square model with sum_n L_n = M.
 *
 * Ownership: the caller allocates X, W, B, V, C and one device workspace of
 * ctfiss_workspace_size() bytes (256-byte aligned).  The library allocates and
 * frees no device memory; a context holds host metadata and pointers only.
 * X must stay alive and unchanged while a context may read it.
 *
 * Errors and ordering: argument and shape errors are returned synchronously,
 * before any HIP call.  Every other call enqueues work on the context's stream
 * (hipStream_t passed as void*, NULL = the null stream) and returns without
 * waiting, except where stated.  Numeric faults found on the device (a
 * non-positive or non-finite ISS denominator, a singular IP system, a singular
 * W_f in the output stage, a non-finite multiplicative update) are latched in
 * a device status word and reported by ctfiss_sync_status(); so is a team of
 * workgroups sharing a bin whose members did not all publish their partial
 * sums within the wait bound (code 6; the launch still completes, its results
 * are not valid).  Team launches (ctfiss_get_plan reports team > 1) size their
 * grid so that all members of a bin are resident at once on an otherwise idle
 * device; kernels of other streams occupying the device meanwhile can delay
 * members past that bound, so run team contexts where they do not share the
 * device with long-running work, or check the status.  No exceptions cross
 * this interface.  One context per stream; calls on one context must not
 * overlap from several host threads.
 */
#ifndef CTFISS_H
#define CTFISS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Status codes: 0 on success, negative on error. */
#define CTFISS_OK 0
#define CTFISS_E_ARG (-1)          /* null pointer, bad enum, negative count        */
#define CTFISS_E_SHAPE (-2)        /* inconsistent shape, e.g. sum(taps) != M*D    */
#define CTFISS_E_UNSUPPORTED (-3)  /* valid shape beyond this build's kernel limits */
#define CTFISS_E_WORKSPACE (-4)    /* workspace too small or not 256-byte aligned  */
#define CTFISS_E_ORDER (-5)        /* input or state not set before use            */
#define CTFISS_E_HIP (-6)          /* a HIP runtime call failed                    */
#define CTFISS_E_NUMERIC (-7)      /* a device numeric fault was latched           */
#define CTFISS_E_TOO_LARGE (-8)    /* workspace beyond the static scratch (noalloc) */

/* Limits of this build (CTFISS_E_UNSUPPORTED beyond them). */
#define CTFISS_MAX_ROWS 64         /* Mbar = M * D                                  */
#define CTFISS_MAX_SOURCES 8       /* N                                             */
#define CTFISS_MAX_BASES 64        /* K                                             */

typedef enum { CTFISS_FP32 = 0, CTFISS_FP64 = 1, CTFISS_MIXED = 2, CTFISS_MIXED_BF16 = 3 } ctfiss_precision;

/* Demixing-matrix update: ISS rank-1 steering, Eqs. (11) and (16), or the
 * iterative-projection baseline, Eqs. (9) and (10). */
typedef enum { CTFISS_RULE_ISS = 0, CTFISS_RULE_IP = 1 } ctfiss_rule;

/* Activation update: ALL_TAPS sums every tap of a source (the exact
 * majorise-minimise step of Eq. (5)); PAPER_TAP0 is Eq. (18) as printed,
 * tap 0 only.  Bases always follow Eq. (17). */
typedef enum { CTFISS_VRULE_ALL_TAPS = 0, CTFISS_VRULE_PAPER_TAP0 = 1 } ctfiss_vrule;

typedef struct {
  int32_t F;            /* frequency bins                                */
  int32_t T;            /* frames                                        */
  int32_t M;            /* microphones                                   */
  int32_t D;            /* stacked delayed frames (1 = paper's model)    */
  int32_t N;            /* sources                                       */
  int32_t K;            /* NMF bases per source                          */
  const int32_t* taps;  /* host pointer, N entries L_n >= 1, sum = M * D */
} ctfiss_shape;

typedef struct ctfiss_ctx ctfiss_ctx;

/* Bytes of device workspace a context of this shape and precision needs: the
 * state (W, B, V), the per-iteration intermediates (1/lambda, tap-aligned
 * powers, activation partial sums, row power sums, scales) and the demixed
 * rows Y = W xbar [F][Mbar][T], which the ISS rule carries from one iteration
 * to the next instead of recomputing (the sweep and the rescale apply the same
 * row operations to W and Y, so the two agree up to rounding).  Shapes whose
 * bins do not fit one workgroup (e.g. Mbar = 64 with T ~ 1000) split each bin's
 * frames over a team of up to 8 workgroups; their workspace also holds the
 * exchange words of the team's partial sums (F * team_words 64-bit words, a
 * few percent of Y).  The size depends on CTFISS_PLAN in the environment, as
 * the launch shape chosen at create does. */
int ctfiss_workspace_size(const ctfiss_shape* shape, int precision, size_t* bytes);

/* Create a context.  rule: ctfiss_rule; vrule: ctfiss_vrule; floor >= 0 is
 * the lower clamp applied to b and v after every multiplicative update
 * (0 = the printed update; 1e-8 is the recommended value).  workspace must
 * hold ctfiss_workspace_size() bytes, 256-byte aligned; it belongs to the
 * context until ctfiss_destroy().  stream: hipStream_t or NULL. */
int ctfiss_create(const ctfiss_shape* shape, int precision, int rule, int vrule, double floor,
                  void* workspace, size_t workspace_bytes, void* stream, ctfiss_ctx** out);

/* Bind the observation X [M][F][T] (device, complex of the context's precision). */
int ctfiss_set_input(ctfiss_ctx* ctx, const void* X);

/* Copy an initial state into the context (device-to-device on its stream).
 * W [F][Mbar][Mbar] may be NULL for identity matrices (the paper's
 * initialisation, Sec. V-A); B [N][F][K] and V [N][K][T] must be positive.
 * Clears the device status word. */
int ctfiss_set_state(ctfiss_ctx* ctx, const void* W, const void* B, const void* V);

/* Enqueue n_iter >= 0 iterations.  One iteration is: W update for every row r
 * in ascending order (ISS or IP), multiplicative update of b (Eq. (17)), of v
 * (Eq. (18) or ALL_TAPS), each followed by the floor clamp, and the scale
 * normalisation of Eqs. (19)-(21).  Requires set_input and set_state.
 * nll_host: NULL, or a host array of n_iter doubles that receives the
 * negative log-likelihood of Eq. (5) (constant dropped, as ctfiss_nll) at the
 * state each iteration leaves, rescale applied; computed on the device in
 * FP64.  A traced call synchronises the stream (once per 256 iterations and
 * at its end), runs eagerly in graph mode, and leaves the same state, bit for
 * bit, as an untraced call. */
int ctfiss_iterate(ctfiss_ctx* ctx, int32_t n_iter, double* nll_host);

/* Graph mode (enable != 0): ctfiss_iterate captures the launches of an
 * n_iter-iteration call once into a HIP graph (one per n_iter and per
 * whether the carried Y is valid at the start, up to 8 kept) and replays it
 * on later calls; the results are those of the launches it was captured from.
 * Useful where launches dominate (small bins, few frames).  Not with profiling
 * (such calls run eagerly), not for contexts on the NULL stream or with team
 * launches (CTFISS_E_UNSUPPORTED).  Disabling synchronises the stream and
 * frees the graphs. */
int ctfiss_set_graph(ctfiss_ctx* ctx, int enable);

/* Launch shape of the context's W update: lanes per row group (G), frames per
 * lane (cpl), rows per group (rpl) and workgroups per bin (team, 1 = one). */
int ctfiss_get_plan(ctfiss_ctx* ctx, int32_t* G, int32_t* cpl, int32_t* rpl, int32_t* team);

/* How the context runs the source-model steps (Eqs. (17)-(19)) of an iteration.
 * fused: 0 = 1/lambda and the basis update are launches of their own; 1 = each
 * bin of the W update forms them, the activations held in LDS; 2 = likewise,
 * the activations read from device memory.  v_one_launch: 1 = the activation
 * update and the row scales are one launch, 0 = partial sums over bin chunks
 * and a final launch.  Either pointer may be null. */
int ctfiss_get_nmf_path(ctfiss_ctx* ctx, int32_t* fused, int32_t* v_one_launch);

/* Measured choice of the W update's launch shape: every instantiated shape that
 * fits the context's shape (team shapes where the default plan is a team plan)
 * runs the W update `trials` times on the context's input and state (after
 * one warm-up run), timed with events; the fastest becomes the context's plan
 * and is cached for the process, per (precision, rule, Mbar, M, D, N, largest
 * tap count, T rounded up to 32), so that contexts created later for such a
 * shape start with it (CTFISS_PLAN in the environment still overrides).
 * scratch: caller-owned device buffer of ctfiss_autotune_scratch_size() bytes
 * (256-byte aligned) that holds a copy of the state (W, B, V) during the call;
 * the state is restored from it afterwards.  Synchronises; allocates nothing.
 * If a device fault is already latched when it is called, it returns
 * CTFISS_E_NUMERIC, times nothing and leaves the fault latched; a candidate
 * whose runs latch a fault is skipped (and that fault cleared).  Not in graph
 * mode (CTFISS_E_UNSUPPORTED). */
int ctfiss_autotune_scratch_size(ctfiss_ctx* ctx, size_t* bytes);
int ctfiss_autotune(ctfiss_ctx* ctx, int32_t trials, void* scratch, size_t scratch_bytes);

/* Forget every plan ctfiss_autotune cached (contexts created afterwards take
 * the built-in rule again; existing contexts keep their plans). */
int ctfiss_clear_tuned_plans(void);

/* Copy the current state out (device-to-device on the context's stream).
 * Any of W, B, V may be NULL to skip it. */
int ctfiss_get_state(ctfiss_ctx* ctx, void* W, void* B, void* V);

/* Source images C [N][M][F][T] of the current state: multichannel Wiener
 * filter of Eq. (24), which with H_f = W_f^{-1} square reduces to
 * c_{n,f,t} = sum_{l < L_n} H_f[:, (n,l)] y_{(n,l),f,t}; the M undelayed rows
 * are returned.  The inverse and projection run in FP64 for both precisions. */
int ctfiss_source_images(ctfiss_ctx* ctx, void* C);

/* Negative log-likelihood of Eq. (5) (constant dropped) at the current state,
 * written to *out.  Computed on the device in FP64; synchronises the stream. */
int ctfiss_nll(ctfiss_ctx* ctx, double* out);

/* Reverse mode (gradients) of the unrolled separation: the forward is W = I
 * (Sec. V-A), B = B0, V = V0, n_iter iterations as in ctfiss_iterate, then
 * the source images C = ctfiss_source_images (Eq. (24) by projection back).
 * Given gC = dL/dC for a real loss L (complex [N][M][F][T], gradient
 * convention dL/dRe + i dL/dIm), writes gX = dL/dX [M][F][T] (the bound
 * input), gB0 = dL/dB0 [N][F][K] and gV0 = dL/dV0 [N][K][T] (either may be
 * NULL).  The factor floor is treated as a clamp: where a factor is clamped,
 * its update passes no gradient.  The forward is run again inside the call
 * with the state saved before every iteration; each iteration is then
 * reversed from its saved state (hand-written adjoint kernels of the rescale,
 * activation and basis updates, the ISS sweep row by row and the demix).
 * ISS contexts in FP32 (complex64, the kernels' arithmetic in FP32), FP64 or
 * mixed precision (the forward as ctfiss_iterate runs it, the adjoint kernels
 * in FP32; not the bfloat16 NMF path), under either activation rule (the
 * context's) and any plan, team launches included; every Mbar in FP32 and
 * mixed precision, Mbar <= 56 in FP64 (the per-bin images adjoint must fit
 * LDS), else CTFISS_E_UNSUPPORTED.  aws: device workspace of
 * ctfiss_adjoint_workspace_size() bytes (256-byte aligned), scratch for the
 * call.  The context ends in the forward's final state, as after
 * ctfiss_iterate.  Enqueued on the context's stream without waiting (so that
 * the reverse passes of several contexts on several streams overlap): the
 * status word is cleared where the forward restarts from (I, B0, V0), and a
 * numeric fault of the forward or the reverse pass stays latched for
 * ctfiss_sync_status, which the caller must read before using gX, gB0, gV0. */
int ctfiss_adjoint_workspace_size(const ctfiss_shape* shape, int precision, int32_t n_iter, size_t* bytes);
int ctfiss_backward(ctfiss_ctx* ctx, int32_t n_iter, const void* B0, const void* V0, const void* gC, void* gX,
                    void* gB0, void* gV0, void* aws, size_t aws_bytes);

/* Synchronise the stream and return CTFISS_E_NUMERIC if a device fault was
 * latched since the last set_state, CTFISS_E_HIP on a HIP error, else 0.
 * *fault_code (nullable) receives the raw device code (0 = none). */
int ctfiss_sync_status(ctfiss_ctx* ctx, int32_t* fault_code);

/* Release the context (does not touch the workspace or any device buffer).
 * Does not wait for work already enqueued on the context's stream (unless
 * profiling launches are pending): the workspace and the buffers the context
 * used must stay allocated until that work has completed, e.g. freed in
 * stream order or after a synchronisation. */
int ctfiss_destroy(ctfiss_ctx* ctx);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): one whole
 * separation -- ctfiss_create, set_input(X), set_state(W0, B0, V0),
 * iterate(n_iter), source_images(C) and get_state(W, B, V) -- with the
 * context's workspace in the library's own static device scratch of 96 MiB
 * instead of a caller buffer (enough for FP32 at F = 1025, T = 313, Mbar = 24,
 * 72.5 MiB).  Arguments as in those calls; W0 may be NULL (identity); C, W, B,
 * V may each be NULL to skip that output; status (device int32, nullable)
 * receives the latched device fault code (0 = none) by a stream-ordered copy.
 * Results equal those of the calls above on a caller workspace, bit for bit.
 * Enqueued on `stream` without waiting; allocates nothing (no device memory;
 * the context lives on the call's stack).  A shape whose workspace
 * (ctfiss_workspace_size) exceeds the scratch returns CTFISS_E_TOO_LARGE
 * before any HIP call.  The scratch is one per GPU and keeps the last call's
 * contents (each call clears what must start at zero): calls that overlap on
 * one GPU, from several streams or host threads, race and must be serialised
 * by the caller. */
int ctfiss_separate_noalloc(const ctfiss_shape* shape, int precision, int rule, int vrule, double floor,
                            const void* X, const void* W0, const void* B0, const void* V0, int32_t n_iter, void* C,
                            void* W, void* B, void* V, int32_t* status, void* stream);

/* Static description of a status code. */
const char* ctfiss_status_string(int status);

/* Kernel timing: ctfiss_set_profiling(ctx, mask) records HIP events around
 * every launch of each kernel class whose bit is set in mask (0 disables,
 * -1 times every class) on the context's stream, in ctfiss_iterate and
 * ctfiss_source_images.  Kernel classes: 0 = W update [ISS or IP sweep],
 * 1 = activation partial sums (bfloat16 contexts and CTFISS_UNFUSED_NMF only;
 * elsewhere class 2 is one launch), 2 = activation update and scale, 3 = final
 * rescale, 4 = source images, 5 = source-variance product lambda = b v,
 * 6 = basis update.  ctfiss_kernel_stats synchronises and returns, for class
 * `which`, the launches and summed milliseconds since the last
 * ctfiss_set_profiling call. */
int ctfiss_set_profiling(ctfiss_ctx* ctx, int mask);
int ctfiss_kernel_stats(ctfiss_ctx* ctx, int which, int64_t* launches, double* total_ms);

/* ---------------------------------------------------------------- batches
 * Many independent mixtures of uneven shape (T, M, D, N, taps, K may differ)
 * separated together.  Every mixture gets the same iteration as a single
 * context of the same shape and precision (the same results bit for bit as one
 * created with CTFISS_UNFUSED_NMF in the environment, whose bins leave lambda
 * and the basis update to separate launches; the default single context sums
 * those in another order), but
 * an iteration is a handful of launches over all mixtures: the W update is
 * one persistent launch per launch shape over the (mixture, bin) items of
 * every mixture of that shape (the shapes' launches overlap on up to three
 * side streams of the batch, forked from and joined to its stream within the
 * iteration, also in a captured graph), and each NMF step is one launch over
 * the workgroups of all mixtures.  The IP rule is accepted and runs mixture by
 * mixture.  Mixture i uses its own device buffers exactly as a context does
 * (X[i] [M_i][F_i][T_i], W[i], B[i], V[i], C[i]: same layouts and types). */
typedef struct ctfiss_batch ctfiss_batch;

/* Workspace bytes for n >= 1 mixtures of the given shapes (host array). */
int ctfiss_batch_workspace_size(const ctfiss_shape* shapes, int32_t n, int precision, size_t* bytes);

/* Create a batch; arguments as ctfiss_create, with one shape per mixture.
 * The workspace (ctfiss_batch_workspace_size bytes, 256-byte aligned) holds
 * every mixture's context workspace and the work tables. */
int ctfiss_batch_create(const ctfiss_shape* shapes, int32_t n, int precision, int rule, int vrule, double floor,
                        void* workspace, size_t workspace_bytes, void* stream, ctfiss_batch** out);

/* X: host array of n device pointers.  Writes the work tables (device copies
 * on the batch's stream) and synchronises the stream. */
int ctfiss_batch_set_input(ctfiss_batch* b, const void* const* X);

/* Host arrays of n device pointers; W may be NULL (identity for every
 * mixture) and so may any of its entries. */
int ctfiss_batch_set_state(ctfiss_batch* b, const void* const* W, const void* const* B, const void* const* V);

/* n_iter iterations of every mixture (as ctfiss_iterate). */
int ctfiss_batch_iterate(ctfiss_batch* b, int32_t n_iter);

/* Graph mode for the batch (enable != 0; ISS rule): ctfiss_batch_iterate
 * captures the launches of an n_iter-iteration call once into a HIP graph (one
 * per n_iter and per whether the carried Y is valid at the start, up to 8
 * kept) and replays it on later calls; a replay is the captured work, with the
 * same results bit for bit.  The launches read every mixture's buffers through
 * the batch's device work tables, so graphs stay valid across set_input and
 * set_state.  Needs a batch created on a non-NULL stream
 * (CTFISS_E_UNSUPPORTED).  Disabling synchronises the stream and frees them. */
int ctfiss_batch_set_graph(ctfiss_batch* b, int enable);

/* Source images of every mixture into C[i] (host array of device pointers). */
int ctfiss_batch_source_images(ctfiss_batch* b, void* const* C);

/* Synchronise; CTFISS_E_NUMERIC if any mixture latched a device fault, with
 * the first such mixture's index in *mixture and its code in *fault_code
 * (both nullable). */
int ctfiss_batch_sync_status(ctfiss_batch* b, int32_t* mixture, int32_t* fault_code);

/* Release the batch (not the workspace or any device buffer). */
int ctfiss_batch_destroy(ctfiss_batch* b);

#ifdef __cplusplus
}
#endif

#endif /* CTFISS_H */
