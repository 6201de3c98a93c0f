/*
 * csmri.h -- C ABI of the MI355X (gfx950) ADMM reconstruction library for
 * Cartesian-sampled dynamic parallel MRI.
 *
 * Method: Bilen, Wang & Selesnick, "High Speed Compressed Sensing
 * Reconstruction in Dynamic Parallel MRI Using Augmented Lagrangian and
 * Parallel Processing".  The library computes
 *   - the measurement operator H and its adjoint (Sec. II-A,
 *     eqs. mri_mcoil2, mri_csmcoill2, H_2, H_1, S, F),
 *   - Algorithm 2 (ADMM_Analysis, Sec. IV-B) with R = temporal TV (eq. TV),
 *   - Algorithm 1 (ADMM_Synthesis, Sec. IV-A) with Psi = unitary temporal DFT,
 *   - the exact x-update (mu I + H'H)^{-1} using the per-(column, frame)
 *     block structure of H'H (Sec. IV-C, eqs. HconjH, separate_x, eigen_mu).
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 *  * Complex values are interleaved single precision (cs_c64 = {re, im}),
 *    bit-compatible with torch.complex64 / numpy.complex64.
 *  * Every array pointer is a DEVICE pointer on the plan's GPU unless the
 *    comment says otherwise.  Arrays are dense, C order, last index fastest:
 *        image  x    [nt][nv][nh]
 *        k-space y   [nt][nc][nv][nh]   (row ky of frame t is one readout line)
 *        coil   s    [nc][nv][nh]
 *        mask        [nt][nv]  uint8, nonzero = phase-encode line ky acquired
 *    j / ky index the vertical (phase-encode, subsampled) axis and i / kx the
 *    horizontal (readout) axis, as in eq. x_def.  Only ky is subsampled, and
 *    the pattern may differ per frame (eq. mri_csmcoill2).
 *  * Transforms are unitary with DC at index 0 (no fftshift); the forward
 *    2D DFT uses exp(-2 pi i (ky j / nv + kx i / nh)).
 *  * Sizes: nv and nh must be 2^a 3^b with 2 <= n <= 512; 1 <= nc <= 64;
 *    2 <= nt <= 64 for the TV prior and 1 <= nt <= 64 for the DFT prior.
 *  * Streams: `stream` is a hipStream_t (NULL = the null stream).  Calls are
 *    asynchronous with respect to the host unless stated; results are ready
 *    when the stream has drained.  A plan must not be used by two streams at
 *    once (its workspaces are shared between calls).
 *  * Errors: every call returns a cs_status.  No C++ exception crosses the
 *    ABI.  On error the outputs are unspecified and the plan stays valid.
 *    cs_last_error() returns a thread-local message for the last failure.
 */
#ifndef CSMRI_H
#define CSMRI_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct { float re, im; } cs_c64;
typedef struct cs_plan cs_plan;   /* opaque: factor store, tables, workspaces */
typedef void* cs_stream;          /* hipStream_t */

typedef enum {
  CS_OK = 0,
  CS_EINVAL = 1,          /* null pointer, size out of range, mu <= 0, lambda < 0, iters < 0 */
  CS_EUNSUPPORTED = 2,    /* size outside the supported set (see above) */
  CS_ENOMEM = 3,          /* the allocator returned NULL */
  CS_EDEVICE = 4,         /* a HIP runtime or rocSOLVER error; detail in cs_last_error() */
  CS_EMU_MISMATCH = 5,    /* solve asked for another mu and CS_FLAG_NO_REFACTOR is set */
} cs_status;

typedef enum {
  CS_PRIOR_TEMPORAL_TV = 0,   /* Algorithm 2 with R = D_t (eq. TV) */
  CS_PRIOR_TEMPORAL_DFT = 1,  /* Algorithm 1 with Psi = unitary DFT along frames */
  CS_PRIOR_TEMPORAL_FRAME = 2, /* Algorithm 1 with the overcomplete tight frame Psi = [I; F] / sqrt(2)
                                  (identity and unitary DFT along frames; Psi'Psi = I, Psi Psi' != I),
                                  including the (1/mu)(I - Psi Psi') term of the w-update (Sec. IV-A).
                                  Coefficients have 2 nt frames (identity part first).  J(k) is taken
                                  at the coefficients w_k, lambda ||w_k||_1 + ||y - H Psi' w_k||^2
                                  (eq. L1unconst).  No column-resident form. */
} cs_prior;

enum {
  CS_FLAG_NO_REFACTOR = 1u << 0,     /* cs_admm_solve with a different mu fails instead of refactoring */
  CS_FLAG_GRAPH = 1u << 1,           /* phase-kernel form: capture the iteration loop once per distinct
                                        (iters, lambda, mu, J_trace) as a hipGraph, cache it in the plan
                                        and replay it (not while cs_kernel_timing is on) */
  CS_FLAG_COLUMN_RESIDENT = 1u << 2, /* run all iterations in one launch, one workgroup per readout
                                        column, instead of two launches per iteration; same results */
  CS_FLAG_XU_WAVE = 1u << 3,         /* phase form, even nv: one 64-lane wave solves a block, or two
                                        blocks when nv = 64 or 192 (nv/2 row pairs do not fill whole
                                        waves, nv pairs do) */
  CS_FLAG_XU_GROUP = 1u << 4,        /* phase form, even nv: a workgroup of nv/2 lanes (rounded up to
                                        whole waves) solves a block.  With neither XU flag the wave
                                        form is used when nv/2 is a multiple of 64 and for nv = 64 and
                                        192.  All x-update forms give bit-identical results. */
  CS_FLAG_EIGEN = 1u << 5,           /* set at cs_plan_create only (cs_plan_set_flags keeps it as it
                                        is): store every block in the paper's eigen form
                                        G = U diag(e) U' (Sec. IV-C, eq. eigen_mu; complex64 U, float e,
                                        from an FP64 eigendecomposition) instead of the packed inverse,
                                        and apply (mu I + G)^{-1} b = U diag(1/(mu + e)) U' b.  Any mu
                                        then runs without refactoring (CS_FLAG_NO_REFACTOR has no
                                        effect).  U is kept twice (conjugated rows and columns, so
                                        both products stream it), which is 4x the packed inverse's
                                        memory and HBM bytes per x-update; the execution-form flags
                                        (COLUMN_RESIDENT, XU_WAVE, XU_GROUP) have no effect.  Results
                                        agree with the packed inverse to rounding, not bit for bit.
                                        The eigendecomposition is rocSOLVER's batched zheevd, on the
                                        plan's stream; its failure is CS_EDEVICE.  Its FP64 matrices and
                                        the library's own device workspace (sized by rocBLAS's size
                                        query) both come from the plan's allocator and are released
                                        before cs_plan_create returns; the rocBLAS handle runs on that
                                        caller-allocated workspace (CS_EDEVICE if it would not). */
  CS_FLAG_CHECK_FINITE = 1u << 6,    /* reject non-finite inputs with CS_EINVAL before any work: the
                                        coil maps (cs_plan_create), the sampled rows of y (cs_apply_AH,
                                        cs_admm_solve, cs_admm_solve_until, cs_batch_solve,
                                        cs_admm_forward_ckpt; unsampled rows are ignored as always),
                                        x (cs_apply_A), b (cs_apply_block_inverse) and grad_x
                                        (cs_admm_backward).  lambda and mu are checked whatever the
                                        flags.  Each check reads one int back and synchronises the
                                        stream, so a checked call cannot be recorded under stream
                                        capture (CS_EINVAL). */
};

/* Device-memory allocator used for everything the plan owns.  alloc returns
 * NULL on failure (the call then returns CS_ENOMEM).  Passing NULL for the
 * whole struct selects hipMalloc / hipFree. */
typedef struct {
  void* (*alloc)(size_t bytes, void* ctx);
  void (*free)(void* ptr, void* ctx);
  void* ctx;
} cs_allocator;

typedef struct {
  int32_t nv, nh, nt, nc;  /* rows (phase-encode), columns (readout), frames, coils */
  int32_t prior;           /* cs_prior */
  float mu_ratio;          /* rho = mu_2 / mu_1 of Algorithm 2 (Sec. V uses 0.5 or 0.25);
                              must be > 0; ignored for the DFT prior */
  uint32_t flags;          /* CS_FLAG_* */
} cs_plan_desc;

/* Solver state, caller-owned device arrays in the image layout.
 *   TV : s0 = m [nt], s1 = d1 [nt-1], s2 = x [nt], s3 = d2 [nt]   (Algorithm 2)
 *   DFT: s0 = w [nt], s1 = v  [nt],   s2 = d [nt], s3 unused       (Algorithm 1)
 * (each [k] means k frames of nv*nh values).  iter = iterations already
 * done: 0 means "start from the algorithm's initialisation", > 0 means "warm
 * start from these arrays".  On return the arrays hold the state after the
 * call and iter has been advanced by the number of iterations run. */
typedef struct {
  cs_c64* s0;
  cs_c64* s1;
  cs_c64* s2;
  cs_c64* s3;
  int32_t iter;
} cs_state;

/* Build a plan for one slice: copies the coil maps and mask, forms every
 * per-(column i, frame t) block G = sum_c S' F~' F~ S of H'H (eq. HconjH, with
 * the coil product taken as conj(s_j) s_k) and stores (mu I + G)^{-1} for the
 * exact x-update (Sec. IV-C).  The factor is computed in FP64 and stored in
 * complex64, packed Hermitian: nv(nv+1)/2 values per block, nh*nt blocks.
 * Synchronises `stream` before returning; `coil` and `mask` may be freed
 * afterwards.  Returns CS_EINVAL / CS_EUNSUPPORTED / CS_ENOMEM / CS_EDEVICE. */
int cs_plan_create(const cs_plan_desc* desc, const cs_c64* coil, const uint8_t* mask,
                   float mu, const cs_allocator* alloc, cs_stream stream, cs_plan** out);

/* Release everything the plan owns (through its allocator).  NULL is a no-op. */
int cs_plan_destroy(cs_plan* plan);

/* Bytes of device memory the plan holds (factor + tables + workspaces). */
int cs_plan_bytes(const cs_plan* plan, size_t* bytes);

/* y = H x (eq. mri_csmcoill2): y[t,c] = M_t F (s_c . x_t).  Writes every
 * element of y; rows ky that frame t does not sample are set to zero. */
int cs_apply_A(cs_plan* plan, const cs_c64* x, cs_c64* y, cs_stream stream);

/* x = H' y, the adjoint of cs_apply_A (H' = S' F~' of the stacked operator
 * H = F~ S, Sec. II-A, eqs. H_1, S, F; H'y is the initial x of Algorithm 2
 * and the constant part of every x-update, Sec. IV-B):
 * x_t = sum_c conj(s_c) . F' M_t y_{t,c}.  Reads only the sampled rows of y
 * (other rows are ignored and may hold anything). */
int cs_apply_AH(cs_plan* plan, const cs_c64* y, cs_c64* x, cs_stream stream);

/* cs_apply_AH without a plan, for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): x = H'y for the operator that desc (nv, nh, nt, nc; prior,
 * mu_ratio and flags are ignored), coil [nc][nv][nh] and mask [nt][nv] define,
 * with the same layouts, conventions and kernels as cs_apply_AH.  It makes no
 * allocation and no host round trip: every intermediate (the sampled-row
 * tables built on the device from mask, the twiddles, the coil maps in
 * column-major order, the hybrid-space rows and the column-major image of a
 * chunk of frames) lives in one fixed 64 MiB device array of the library,
 * which each GPU the call runs on holds until the process ends.  Frames are
 * processed in chunks that fit it; the tables, the coil maps and one frame
 * must fit (about 8 nv nh (2 nc + 1) bytes), else CS_EUNSUPPORTED.  Runs on
 * the current device.  Every call on a GPU shares that GPU's array: calls that
 * overlap on one GPU (two streams, two threads) race and give undefined
 * results; calls ordered on one stream are safe.  Nothing left in the array by
 * an earlier call is read.  Errors: CS_EINVAL (NULL pointer, size < 1),
 * CS_EUNSUPPORTED (sizes as for cs_plan_create, or beyond the array). */
int cs_apply_AH_noalloc(const cs_plan_desc* desc, const cs_c64* coil, const uint8_t* mask, const cs_c64* y,
                        cs_c64* x, cs_stream stream);

/* x = (mu I + H'H)^{-1} b with the plan's mu (eq. eigen_mu), b and x images
 * [nt][nv][nh]; x may alias b.  The plan's mu is the one it was created with,
 * or the mu of its latest solve or forward pass if that one differed (a
 * packed plan refactored for it; a CS_FLAG_EIGEN plan just takes it over). */
int cs_apply_block_inverse(cs_plan* plan, const cs_c64* b, cs_c64* x, cs_stream stream);

/* Run `iters` ADMM iterations on data y (Algorithm 2 for the TV prior,
 * Algorithm 1 for the DFT prior) and write the image series to x_out.
 *   lambda >= 0 weights the l1 term; mu > 0 is mu (Algorithm 1) or mu_2
 *   (Algorithm 2, with mu_1 = mu / mu_ratio).  If mu differs from the plan's
 *   mu the factor is rebuilt first (FP64, not cheap) unless the plan has
 *   CS_FLAG_NO_REFACTOR, which makes the call return CS_EMU_MISMATCH.
 *   state may be NULL (fresh start, nothing returned) -- see cs_state.
 *   J_trace, if not NULL, is a device float[iters] that receives the
 *   objective J(k) after each iteration (lambda ||D_t x||_1 + ||y - Hx||^2,
 *   lambda ||Psi x||_1 + ||y - Hx||^2, or for the frame lambda ||w||_1 +
 *   ||y - H Psi' w||^2), used for Delta(k) of eq. r_ratio.  On the frame prior
 *   each evaluation also completes w and d, which leaves results bit-identical.
 * iters == 0 writes H'y (the algorithms' initial x) to x_out.
 * Execution: two launches per iteration (temporal step, x-update).  With
 * CS_FLAG_COLUMN_RESIDENT, even nv and no J_trace, all iterations run in one
 * launch in which a workgroup owns one readout column (temporal priors never
 * couple columns).  Both forms give bit-identical results. */
int cs_admm_solve(cs_plan* plan, const cs_c64* y, float lambda, float mu, int32_t iters,
                  cs_c64* x_out, cs_state* state, float* J_trace, cs_stream stream);

/* Read or replace the plan's flags (any CS_FLAG_* combination that
 * cs_plan_create accepts).  The form flags only choose how iterations are
 * launched, never what they compute. */
int cs_plan_flags(const cs_plan* plan, uint32_t* flags);
int cs_plan_set_flags(cs_plan* plan, uint32_t flags);

/* FFT tiles of the SENSE passes: readout columns per wave of the vertical
 * (phase-encode) FFTs and sampled rows per workgroup of the horizontal ones.
 * cs_plan_fft_tiles returns the values in use; cs_plan_set_fft_tiles sets
 * them.  0 selects the default: as many columns as fit 256 values (one when
 * nv > 256) and as many rows as fit 4096 values.  Larger values are clipped to
 * 512 values per column group and 4096 per row group.  Results do not depend
 * on them.  At n_v = 16 M (M = 4, 6, 8, 9, 12, 16: 64 ... 256) the vertical
 * passes, and at n_h = 16 M the horizontal ones, run register transforms with
 * fixed tiles (4 columns per wave, 16 rows per workgroup) and ignore the
 * corresponding value. */
int cs_plan_fft_tiles(const cs_plan* plan, int32_t* cols, int32_t* rows);
int cs_plan_set_fft_tiles(cs_plan* plan, int32_t cols, int32_t rows);

/* Autotuner: first picks the FFT tiles (every pair from the largest tiles down
 * to 1/16 of their columns and 1/4 of their rows, timed on H'y of y plus the
 * vertical forward pass; a value the passes ignore is not swept), then times `iters` iterations (after as many
 * untimed ones) of every execution form the plan supports -- phase form with
 * each x-update form (graph-replayed), and the column-resident form -- on the
 * data y, in three interleaved rounds, and keeps the form with the fastest
 * round in the plan's flags (CS_FLAG_NO_REFACTOR is preserved).  entries
 * (host array of `cap`, may be NULL) receives the flags and fastest measured
 * ms per iteration of each candidate; *count (may be NULL) their number.
 * Synchronises `stream`.  The plan's solver workspaces are overwritten. */
typedef struct {
  uint32_t flags;
  float ms_per_iter;
} cs_tune_entry;
int cs_plan_tune(cs_plan* plan, const cs_c64* y, float lambda, int32_t iters, cs_tune_entry* entries,
                 int32_t cap, int32_t* count, cs_stream stream);

/* The paper's stopping rule (Sec. V, eq. r_ratio): iterate until
 * |Delta(k)| < tol, Delta(k) = (J(k-1) - J(k)) / J(k), or max_iters
 * iterations.  The magnitude is compared because ADMM does not decrease J
 * monotonically: a check at which J rose by more than tol does not stop the
 * solve (tol <= 0 never stops it before max_iters).  Delta is
 * checked every `check_every` iterations (J is evaluated at the last two
 * iterations of each block of check_every, or at every iteration when
 * check_every == 1, J(0) being taken at the initial iterate), so the solve
 * stops at the first multiple of check_every (or at max_iters) where the
 * test holds.  *iters_done (host) receives the number of iterations run and
 * *delta (host, nullable) the last Delta evaluated.  Same arguments otherwise
 * as cs_admm_solve (without J_trace); x_out and state equal what
 * cs_admm_solve returns for *iters_done iterations, bit for bit.  The phase
 * form is used whatever the plan's flags.  Synchronises `stream` once per
 * block to read J back. */
int cs_admm_solve_until(cs_plan* plan, const cs_c64* y, float lambda, float mu, int32_t max_iters, float tol,
                        int32_t check_every, cs_c64* x_out, cs_state* state, int32_t* iters_done, float* delta,
                        cs_stream stream);

/* ---------------------------------------------------------------- batches
 * Many independent slices (uneven sizes, coil counts, sampling, priors) solved
 * together.  Each slice is one plan (as cs_plan_create); cs_batch_solve runs
 * every slice's whole solve -- H'y setup and `iters` iterations -- as one
 * hipGraph launch of two concurrent chains of slices (dealt largest factor
 * first, each to the chain with less work so far), so the GPU overlaps one
 * slice's short steps with another's factor stream and the host pays one
 * launch per call.  The graph is recorded on the first call and replayed
 * while the pointers, lambdas, iteration count and each slice's mu, form and
 * FFT tiles stay the same.  Results equal cs_admm_solve on each slice bit for
 * bit. */
typedef struct cs_batch cs_batch;

typedef struct {
  cs_plan_desc desc;    /* sizes, prior, mu_ratio of this slice; CS_FLAG_GRAPH is ignored */
  const cs_c64* coil;   /* device [nc][nv][nh] */
  const uint8_t* mask;  /* device [nt][nv] */
  float mu;
} cs_slice_desc;

/* slices: host array of `count` descriptors.  Builds every plan (synchronous,
 * like cs_plan_create).  On error no batch is returned. */
int cs_batch_create(const cs_slice_desc* slices, int32_t count, const cs_allocator* alloc, cs_stream stream,
                    cs_batch** out);
int cs_batch_destroy(cs_batch* batch);
int cs_batch_size(const cs_batch* batch, int32_t* count);
/* The plan of slice `index` (owned by the batch: do not destroy it).  It may
 * be used on its own (cs_apply_A, cs_plan_tune, ...); changing its flags makes
 * the next cs_batch_solve record the graph again. */
int cs_batch_plan(cs_batch* batch, int32_t index, cs_plan** plan);

/* y, x_out: host arrays of `count` device pointers (k-space and image of each
 * slice, layouts as for cs_admm_solve); lambda: host array of `count` values.
 * Each slice runs with its plan's mu, from the algorithm's initialisation. */
int cs_batch_solve(cs_batch* batch, const cs_c64* const* y, const float* lambda, int32_t iters,
                   cs_c64* const* x_out, cs_stream stream);

/* ---------------------------------------------------------------- gradients
 * Reverse-mode derivative of K unrolled iterations of Algorithm 2 (temporal TV
 * prior, Sec. IV-B) or Algorithm 1 (temporal DFT prior, Sec. IV-A) from its
 * initialisation, for training or tuning through the reconstruction: given
 * dL/dx_K of a real loss L, returns dL/dy, dL/dlambda and dL/dmu (for TV
 * mu = mu_2 and rho = mu_ratio is held fixed).  Complex gradients use the
 * convention g = dL/dRe z + i dL/dIm z (that of torch.autograd).
 *
 * The forward keeps the solver state every `ckpt_every` iterations, and the
 * per-iteration values the adjoint needs (the tape) of its last segment; the
 * backward sweeps the segments last first, recomputing each one's tape from
 * its checkpoint except the one the forward kept (so ckpt_every >= iters
 * recomputes nothing), and applies the transposed Jacobian of each line of the
 * algorithm in reverse (the x-update kernel applies the Hermitian
 * (mu I + H'H)^{-1}; one kernel over 16-pixel tiles does the transposed
 * temporal step on the matrix cores, the soft threshold and the dual updates).  Memory: about 4 images per checkpoint plus 3 per
 * iteration of a segment plus 7.
 * dL/dy = A(dL/dH'y) is zero on rows the mask does not sample.  Where some
 * |D m + d1| equals tau exactly the map is not differentiable; the derivative
 * of the inactive side is returned. */
typedef struct cs_grad cs_grad;

/* Workspace for `iters` unrolled iterations on `plan` (TV or DFT prior; the
 * overcomplete frame prior returns CS_EUNSUPPORTED), allocated through the
 * plan's allocator; it must be destroyed before the plan.  ckpt_every >= 1. */
int cs_grad_create(cs_plan* plan, int32_t iters, int32_t ckpt_every, cs_grad** out);
int cs_grad_destroy(cs_grad* grad);

/* x_out = x_K of cs_admm_solve(plan, y, lambda, mu, iters) (bit-identical),
 * keeping checkpoints and H'y in the workspace for one cs_admm_backward. */
int cs_admm_forward_ckpt(cs_grad* grad, const cs_c64* y, float lambda, float mu, cs_c64* x_out,
                         cs_stream stream);

/* grad_x: device image dL/dx_K; grad_y: device k-space [nt][nc][nv][nh]
 * receiving dL/dy; grad_lambda_mu: device float[2] receiving dL/dlambda and
 * dL/dmu (FP64 accumulation).  Uses the lambda and mu of the last
 * cs_admm_forward_ckpt (CS_EINVAL if there was none); overwrites the plan's
 * solver workspaces. */
int cs_admm_backward(cs_grad* grad, const cs_c64* grad_x, cs_c64* grad_y, float* grad_lambda_mu,
                     cs_stream stream);

/* Per-kernel device timing, a profiling aid for callers that report kernel
 * throughput.  cs_kernel_timing(plan, 1) starts bracketing every launch of
 * the per-iteration kernels made by cs_admm_solve with a pair of hipEvents on
 * the solve's stream (0 stops; either call clears the accumulated times).
 * cs_kernel_times waits for those events and fills up to `max` records, one
 * per kernel kind, with the number of launches and their summed device time;
 * *count receives the number of kinds seen.  Kinds: "tv_step", "dft_step"
 * (also the frame prior's step), "x_update", "objective", "frame_finish" (the
 * pass that completes the frame prior's w and d before each objective
 * evaluation) (phase-kernel form) and "column_solve" (one launch running all
 * iterations, one workgroup per readout column).  Event records add a few microseconds of host
 * work per launch and nothing to the kernels themselves. */
typedef struct {
  char name[24];
  int32_t launches;
  double ms;
} cs_kernel_time;

int cs_kernel_timing(cs_plan* plan, int enable);
int cs_kernel_times(cs_plan* plan, cs_kernel_time* out, int max, int* count);

/* Measurement aid, not part of the method: reads `bytes` of device memory at
 * `buf` with a streaming kernel (each of `blocks` workgroups of 256 threads,
 * 0 selecting 8192, reads contiguous 32 KB tiles with 16-byte non-temporal
 * loads, eight in flight per thread) and writes nothing, except that *sink (device float) would receive
 * the sum of the values read if it equalled one fixed improbable number.
 * Timed around a launch it gives the HBM read rate the chip sustains for a
 * pure read stream, the practical ceiling of the read-bound x-update.
 * Asynchronous on `stream`.  Errors: CS_EINVAL (NULL pointer, bytes not a
 * positive multiple of 16, buf not 16-byte aligned, blocks outside
 * [0, 65535]). */
int cs_read_stream(const void* buf, size_t bytes, int32_t blocks, float* sink, cs_stream stream);

/* Static description of a status code. */
const char* cs_status_string(int status);

/* Thread-local text of the last error raised on this thread ("" if none). */
const char* cs_last_error(void);

/* Library version as major*10000 + minor*100 + patch. */
int cs_version(void);

#ifdef __cplusplus
}
#endif
#endif /* CSMRI_H */
