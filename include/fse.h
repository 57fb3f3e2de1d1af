/*
 * fse.h - C ABI of the MI355X (gfx950) complex-valued Frequency Selective
 * Extrapolation library (libfse.so).
 *
 * The library conceals lost rectangular blocks of 8-bit frames. For every
 * lost block B it cuts the extrapolation area L = A u B (B grown by `border`
 * pixels on each side; Seiler & Kaup, Section II and Fig. 1), weights the
 * received pixels with the isotropic window of eq. (3), and runs the
 * frequency-domain cFSE iteration of Section III / Algorithm 1:
 *   R_w = DFT(s*w), W = DFT(w)                          (eq. (11))
 *   repeat I times:
 *     (u,v) = argmax |R_w[k,l]|^2, lowest k*F+l on ties  (eq. (12))
 *     c = gamma * R_w[u,v] / W[0,0]                      (eq. (13))
 *     G[u,v] += F*F*c                                     (eq. (15))
 *     R_w[k,l] -= c * W[(k-u) mod F, (l-v) mod F]  all k,l (eq. (18))
 *   g = IDFT(G); B <- Re{g}                               (Algorithm 1)
 * on an F x F zero-padded transform grid (F in {32, 64, 128}; the paper uses
 * a 48x48 area in a 64x64 transform, Section IV).
 *
 * Beside plain cFSE the library offers a learned warm start (fse_cnn_*,
 * fse_warm_*), mask-driven loss areas (FSE_PLAN_MASKED_B), real-valued FSE
 * (FSE_PLAN_REAL), a bit-exact fixed-point encoding (FSE_PLAN_FIXED), 3-D
 * video concealment of lost volumes (fse_batch3d_*, plain and warm-started)
 * and an LDS bandwidth probe for roofline accounting.
 *
 * Conventions used by every entry point:
 *  - Pointers prefixed d_ are device memory on the current HIP device and
 *    are owned by the caller; h_ pointers are host memory owned by the
 *    caller. The library never frees caller memory.
 *  - Frames are row-major uint8 [n_frames][H][pitch]; the availability mask
 *    has the same layout (nonzero = received, 0 = lost). The output is
 *    float32 [n_frames][H][out_pitch]; only pixels of the blocks' B regions
 *    are written, everything else is left untouched.
 *  - Inside the area, pixels outside the frame, lost pixels (mask 0) and B
 *    itself carry zero weight; blocks are therefore independent.
 *  - Errors found on the host are returned before anything is launched.
 *    Launch-time HIP errors return FSE_ERR_HIP. Per-block conditions are
 *    written to d_status once the stream reaches them.
 *  - Entry points are thread-safe for distinct handles. One batch handle
 *    must not run on two streams at once (its work queue is shared).
 */
#ifndef FSE_H_
#define FSE_H_

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  FSE_OK = 0,
  FSE_ERR_INVALID_ARG = -1,  /* null pointer, bad size, bad parameter        */
  FSE_ERR_UNSUPPORTED = -2,  /* F not in {32,64,128}, area larger than F ... */
  FSE_ERR_OOM = -3,          /* device or host allocation failed             */
  FSE_ERR_HIP = -4,          /* a HIP runtime call failed                    */
  FSE_ERR_OVERLAP = -5,      /* two blocks' loss areas B overlap             */
  FSE_ERR_WORKSPACE = -6     /* caller's workspace too small or misplaced    */
} fse_status_t;

/* Per-block result codes written to d_status[i] for block i. */
enum {
  FSE_BLOCK_OK = 0,
  FSE_BLOCK_EMPTY_SUPPORT = 1, /* W[0,0] == 0: no received pixel; B untouched */
  FSE_BLOCK_NONFINITE = 2      /* a coefficient was not finite; B untouched   */
};

/* One lost block: B is the bh x bw rectangle with top-left (y0, x0) in frame
 * `frame`; its area extends `border` pixels beyond B on every side, so the
 * area is M x N = (bh + 2*border) x (bw + 2*border) and must fit the
 * transform: M <= fft and N <= fft. `iters` is the iteration count I.
 * 24 bytes, natural alignment. */
typedef struct {
  int32_t frame;
  int32_t y0, x0;
  int16_t bh, bw;
  int16_t border;
  int16_t fft;
  int32_t iters;
} fse_block_t;

/* One lost volume of a video clip (three dimensions): B is bh x bw pixels
 * at (y0, x0) in frames frame .. frame + bt - 1; its area extends `border`
 * pixels and `tborder` frames beyond B on every side (M x N x T =
 * (bh + 2 border) x (bw + 2 border) x (bt + 2 tborder)), transformed on an
 * fft x fft x fft_t grid (64 x 64 x 8 in this library). `pad` must be 0.
 * 32 bytes, natural alignment. */
typedef struct {
  int32_t frame;
  int32_t y0, x0;
  int16_t bt, bh, bw;
  int16_t border, tborder;
  int16_t fft, fft_t;
  int16_t pad;
  int32_t iters;
} fse_volume_t;

/* Plan parameters shared by every block run with the plan. */
typedef struct {
  float rho;          /* window decay rho in (0, 1], eq. (3)                  */
  float gamma;        /* orthogonality deficiency compensation, [0, 1], eq. (13) */
  int32_t max_iters;  /* largest per-block iteration count accepted (<= 4096) */
  uint32_t flags;     /* FSE_PLAN_* bits; others must be 0                    */
} fse_plan_desc_t;

/* Mask-driven loss areas (arbitrary loss shapes, the concealment and
 * inpainting setting of Section I): a block's bh x bw rectangle only bounds
 * its loss; B is the set of the rectangle's pixels with avail == 0, the
 * rectangle's received pixels belong to the support A (eq. (3)), and only
 * the pixels of B are written. Plain FSE only (the warm start refuses such
 * plans). See fse_blocks_from_mask for covering an arbitrary mask. */
#define FSE_PLAN_MASKED_B 1u

/* Plan flag: real-valued FSE (rFSE, the model of eq. (2), Section II)
 * instead of cFSE. Every iteration adds a basis function and its complex
 * conjugate: the pair is the weighted least-squares fit of the residual on
 * the real span of phi_(k,l) and phi_(-k,-l), selected by the largest
 * decrease of the weighted residual energy and scaled by gamma. Blocks
 * must use fft = 64; the plan cannot be combined with FSE_PLAN_MASKED_B;
 * the warm start and the 3-D path refuse it. Trace records name the
 * pair's lower-index bin and its coefficient c (model increment
 * Re{c phi*}); r2 is the selection criterion (the decrease, or |R_w|^2
 * with FSE_PLAN_REAL_POWER). */
#define FSE_PLAN_REAL 2u

/* Modifier of FSE_PLAN_REAL (invalid without it): the pair constants,
 * divisions by W0^2 - |W[2k,2l]|^2 included, are recomputed for every bin in
 * every iteration instead of once per block, the formulation whose cost
 * the paper's runtime comparison describes (Section II). Same results up
 * to FP32 rounding. */
#define FSE_PLAN_REAL_INLOOP 8u

/* Modifier of FSE_PLAN_REAL (invalid without it, exclusive with
 * FSE_PLAN_REAL_INLOOP): the other reading of rFSE's selection, the pair
 * holding the bin of largest |R_w|^2 (the criterion of eq. (12)), with the
 * same least-squares estimate. */
#define FSE_PLAN_REAL_POWER 16u

/* Plan flag: fixed-point cFSE (the integer form the paper's conclusion
 * argues for: the loop has no division). Every value is an integer with a
 * fixed scale and every sum is exact in int64, so results are reproducible
 * bit for bit: window round(2^15 rho^d), twiddles round(2^14 e^{-j2pi q/64}),
 * z = s w + j 2^7 w, a direct separable transform rounded after each pass
 * (by 2^14, then 2^23), R2 = 2^7 R_w and W2 = 2^14 W by the conjugate
 * split, one division per block G = floor(round(2^16 gamma) 2^33 / W2[0,0]),
 * then per iteration the exact argmax of R2x^2 + R2y^2 (lowest index on
 * ties), c = round(R2[u,v] G / 2^26) (units 2^-16 pixel) and
 * R2 -= round(c W2[k-u, l-v] / 2^23); B receives
 * round(sum Re{c e^{j theta}} 2^14 / 2^22) / 2^8, a float32 holding a
 * multiple of 2^-8. round(x / 2^s) = (x + 2^(s-1)) >> s. Blocks must use
 * fft = 64 with areas of at most 64 x 64 pixels; the flag excludes
 * FSE_PLAN_MASKED_B and FSE_PLAN_REAL; the warm start and the 3-D path
 * refuse it. Trace records carry c / 2^16 (exact in FP32) and the score. */
#define FSE_PLAN_FIXED 4u

/* One record per block and iteration when tracing: selected bin (u, v),
 * coefficient c of eq. (13) and |R_w[u,v]|^2 as seen by the argmax. For a
 * volume, u = k and v = l * fft_t + s for the selected bin (k, l, s). */
typedef struct {
  uint16_t u, v;
  float c_re, c_im;
  float r2;
} fse_trace_t;

typedef struct fse_plan_s* fse_plan_t;
typedef struct fse_batch_s* fse_batch_t;

/* Create a plan: validates the descriptor and builds the window table
 * rho^(distance) (eq. (3)) and the DFT twiddle tables in FP64 on the host,
 * rounded to FP32. Host-only: no device memory is touched until the first
 * batch is created. Returns FSE_ERR_INVALID_ARG for rho outside (0,1], gamma
 * outside [0,1], max_iters outside [0,4096], unknown flags or null
 * pointers or FSE_PLAN_REAL_INLOOP without FSE_PLAN_REAL,
 * FSE_ERR_UNSUPPORTED when more than one of FSE_PLAN_MASKED_B, FSE_PLAN_REAL
 * and FSE_PLAN_FIXED is set. */
fse_status_t fse_plan_create(const fse_plan_desc_t* desc, fse_plan_t* out_plan);

/* Destroy a plan and the device tables it uploaded. Batches created from it
 * must be destroyed first. Null is ignored. */
void fse_plan_destroy(fse_plan_t plan);

/* Host-only check of a block list against frames of n_frames x H x W:
 * fft in {32,64,128}; bh, bw >= 1; border >= 0; M, N <= fft; 0 <= iters <=
 * max_iters; frame in range; B inside the frame; no two B overlapping.
 * Returns FSE_OK, FSE_ERR_UNSUPPORTED, FSE_ERR_OVERLAP or
 * FSE_ERR_INVALID_ARG. *bad_index (if not null) receives the first offending
 * block index, or -1. */
fse_status_t fse_validate_blocks(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                                 int32_t n_frames, int32_t H, int32_t W, int32_t* bad_index);

/* Cover the lost pixels of an availability mask with blocks, host-side:
 * frame f of h_avail (uint8 [n_frames][H][pitch], 0 = lost) is cut into
 * cell x cell tiles from (0, 0), clipped at the right and bottom edges, and
 * every tile holding a lost pixel becomes one block {f, y0, x0, bh, bw,
 * border, fft, iters}, frame-major then row-major, for a plan with
 * FSE_PLAN_MASKED_B. Writes the first min(count, cap) blocks to h_out (may be
 * null when cap = 0) and the count to *n_out. FSE_ERR_INVALID_ARG for a null
 * mask or n_out, non-positive sizes, pitch < W, cell < 1 or border < 0;
 * FSE_ERR_UNSUPPORTED when cell + 2*border exceeds fft or fft is not 32, 64
 * or 128. */
fse_status_t fse_blocks_from_mask(const uint8_t* h_avail, int32_t n_frames, int32_t H, int32_t W, int64_t pitch,
                                  int32_t cell, int32_t border, int32_t fft, int32_t iters, fse_block_t* h_out,
                                  int32_t cap, int32_t* n_out);

/* Prepare a batch: validates h_blocks (as fse_validate_blocks), groups the
 * blocks by transform size, orders each group longest-first by F*F*I,
 * uploads descriptors, the schedule and the plan tables to the current
 * device and allocates the work-queue counters. Synchronous. After this
 * call h_blocks may be freed. With an FSE_PLAN_REAL or FSE_PLAN_FIXED plan
 * every block must have fft = 64 (FSE_ERR_UNSUPPORTED otherwise). */
fse_status_t fse_batch_create(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                              int32_t n_frames, int32_t H, int32_t W, fse_batch_t* out_batch);

/* Release a batch's device memory (none for a batch made by
 * fse_batch_create_in: its workspace stays the caller's). Synchronises the
 * device. Null is ignored. */
void fse_batch_destroy(fse_batch_t batch);

/* Flag of fse_batch_workspace_size and fse_batch_create_in: the workspace
 * also holds the staging of the warm start's two-kernel form
 * (fse_warm_extrapolate_batch, n_blocks x (16896 + 4096) bytes). */
#define FSE_WS_WARM 1u

/* Bytes of device workspace that fse_batch_create_in needs for n_blocks
 * blocks under `plan`: the block descriptors and their schedule, the
 * work-queue counters, a copy of the plan's window table of eq. (3) and its
 * twiddles (and, for FSE_PLAN_FIXED, their integer forms), each array
 * 256-byte aligned, plus the warm staging when ws_flags has FSE_WS_WARM.
 * Host-only. FSE_ERR_INVALID_ARG for a null argument, n_blocks < 0 or an
 * unknown flag; FSE_ERR_UNSUPPORTED for FSE_WS_WARM with a plan the warm
 * start does not take. */
fse_status_t fse_batch_workspace_size(fse_plan_t plan, int32_t n_blocks, uint32_t ws_flags, size_t* bytes);

/* fse_batch_create with caller-owned device memory: every device array of
 * the batch (those of fse_batch_workspace_size) lies in
 * [d_workspace, d_workspace + ws_bytes), so neither this call, the launches
 * nor fse_batch_destroy allocate or free device memory, and the plan's
 * tables are not shared with other batches. d_workspace must be 256-byte
 * aligned device memory of the current device, ws_bytes at least
 * fse_batch_workspace_size(plan, n_blocks, ws_flags) and the whole range
 * inside one allocation; it must stay allocated, and must not be written
 * by anyone else, until fse_batch_destroy. Results are those of
 * fse_batch_create's batch, bit for bit. Synchronous (uploads). Errors as
 * fse_batch_create, plus FSE_ERR_INVALID_ARG for a null, misaligned or
 * non-device workspace and FSE_ERR_WORKSPACE for one that is too small or
 * runs past its allocation. A batch made without FSE_WS_WARM returns
 * FSE_ERR_WORKSPACE from the warm-start calls that need the staging. */
fse_status_t fse_batch_create_in(fse_plan_t plan, const fse_block_t* h_blocks, int32_t n_blocks,
                                 int32_t n_frames, int32_t H, int32_t W, void* d_workspace, size_t ws_bytes,
                                 uint32_t ws_flags, fse_batch_t* out_batch);

/* Largest iteration count among the batch's blocks (the trace stride). */
int32_t fse_batch_max_iters(fse_batch_t batch);

/* Run cFSE (rFSE with an FSE_PLAN_REAL plan, fixed-point cFSE with an
 * FSE_PLAN_FIXED plan) on every block of the batch:
 * kernel launches only, on `stream`
 * (a hipStream_t; null = default stream), asynchronous, no allocation and no
 * host-device copies, so the call may be captured into a HIP graph.
 *   d_image, d_avail : uint8 [n_frames][H][pitch] (pitch >= W, in bytes)
 *   d_out            : float32 [n_frames][H][out_pitch]; B pixels written
 *   d_status         : int32 [n_blocks], FSE_BLOCK_* per block (required)
 *   d_trace          : null, or fse_trace_t [n_blocks][fse_batch_max_iters]
 *                      receiving every block's selections in order
 * Block i of the list given to fse_batch_create writes d_status[i] and
 * trace row i. Results do not depend on the other blocks of the batch. */
fse_status_t fse_extrapolate_batch(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                   int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                   fse_trace_t* d_trace, void* stream);

/* Launch configuration chosen for transform size F (32, 64 or 128): threads
 * per workgroup, workgroups resident per CU, persistent grid size and
 * dynamic LDS bytes per workgroup. Any output pointer may be null. Returns
 * FSE_ERR_INVALID_ARG if the batch has no block of that size. With an
 * FSE_PLAN_REAL or FSE_PLAN_FIXED plan it describes that kernel. */
fse_status_t fse_batch_launch_info(fse_batch_t batch, int32_t F, int32_t* threads, int32_t* wg_per_cu,
                                   int32_t* grid, int32_t* lds_bytes);

/* Run the blocks of transform size F with the compiled kernel variant that
 * has `threads` threads per workgroup (F=32: 64, 128, 256; F=64: 128, 256,
 * 512; F=128: 512, 1024). Every variant computes bit-identical results;
 * they differ in speed only. Returns FSE_ERR_UNSUPPORTED if no such variant
 * is compiled or it does not fit a compute unit, FSE_ERR_INVALID_ARG if the
 * batch has no block of that size, FSE_ERR_UNSUPPORTED for an FSE_PLAN_REAL
 * or FSE_PLAN_FIXED plan. Host-side; affects later fse_extrapolate_batch
 * calls. */
fse_status_t fse_batch_set_variant(fse_batch_t batch, int32_t F, int32_t threads);

/* Autotuner: for every transform size present in the batch, launch every
 * compiled variant once untimed and `reps` times timed (HIP events on
 * `stream`) on the given inputs, and keep the fastest. Synchronous.
 * Arguments as for fse_extrapolate_batch (d_out and d_status receive the
 * results of the last launch). If `report` is not null, up to report_len
 * bytes of text are written to it, one line "F threads microseconds" per
 * variant timed. FSE_ERR_UNSUPPORTED for an FSE_PLAN_REAL or FSE_PLAN_FIXED
 * plan. */
fse_status_t fse_batch_autotune(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail, int64_t pitch,
                                float* d_out, int64_t out_pitch, int32_t* d_status, int32_t reps, void* stream,
                                char* report, size_t report_len);

/* The autotuner with a decision cache: a text file of lines "key threads
 * microseconds", where the key names the device (architecture name and
 * compute-unit count) and the class (transform size, rectangular or
 * mask-driven loss areas, block count and largest iteration count rounded
 * up to powers of two). A class whose key the file holds, with a compiled
 * variant that fits, is configured from it without timing (report line "F
 * threads cached"); every other class is timed as by fse_batch_autotune
 * and its decision appended to the file (created if absent; an unreadable
 * or unwritable path acts as an empty cache). cache_path null: exactly
 * fse_batch_autotune. Synchronous when it times; a fully cached call
 * launches nothing. */
fse_status_t fse_batch_autotune_cached(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                       int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                       int32_t reps, void* stream, char* report, size_t report_len,
                                       const char* cache_path);

/* Kernel timing, a profiling hook. fse_batch_set_timing(batch, max_records)
 * makes every later kernel launch of this batch (fse_extrapolate_batch,
 * fse_warm_extrapolate_batch; not the autotuner) record a HIP event on its
 * stream before and after the kernel, for up to max_records kernels;
 * further launches run untimed. max_records = 0 switches timing off and
 * frees the events; calling it again restarts the record. Host-side.
 * fse_batch_kernel_times waits for the recorded kernels and writes, for
 * the first min(count, cap) of them in launch order, the duration in ms,
 * the kernel kind (FSE_KERNEL_*) and the transform size; returns the number
 * recorded (negative fse_status_t on error). */
enum {
  FSE_KERNEL_PLAIN = 0,       /* persistent kernel, plain FSE                     */
  FSE_KERNEL_WARM_FUSED = 1,  /* warm start, restricted and full phases in one    */
  FSE_KERNEL_WARM_PREP = 2,   /* warm start, transform and staging (split form)   */
  FSE_KERNEL_RESTRICTED = 3,  /* warm start, restricted iterations (split form)   */
  FSE_KERNEL_REAL = 4,        /* rFSE (plan flag FSE_PLAN_REAL)                   */
  FSE_KERNEL_FIXED = 5        /* fixed-point cFSE (plan flag FSE_PLAN_FIXED)      */
};
fse_status_t fse_batch_set_timing(fse_batch_t batch, int32_t max_records);
int32_t fse_batch_kernel_times(fse_batch_t batch, float* ms, int32_t* kind, int32_t* fft, int32_t cap);

/* ------------------------------------------------------------------------
 * Learned warm start. Not part of the paper's method: a small network reads
 * each 48x48 area and scores every bin of the 64x64 transform; the K best
 * bins become a candidate set. FSE iterations restricted to the candidates
 * (argmax and update over those bins only, eqs. (12), (13), (18)) produce
 * the first coefficients, which are then applied to the whole spectrum
 * (eq. (18) once per distinct bin), and the usual FSE iterations over all
 * bins continue from there. Plain FSE is the fallback.
 *
 * Network: input [B][48][48][2] BF16 (channel 0: (s - mean over A)/64 on
 * the support area A, channel 1: indicator of A); four 3x3 stride-2
 * convolutions with bias and ReLU, 2->32->32->32->32 channels
 * (48->24->12->6->3 pixels); a dense head from the 288 features to 4096
 * logits (bin k*64+l). BF16 weights and activations, FP32 accumulation.
 * Parameters are one flat FP32 vector (fse_cnn_num_params elements, in the
 * order conv1..conv4 weight [32][3][3][Cin] and bias [32], head weight
 * [4096][288] and bias [4096]).
 * ---------------------------------------------------------------------- */
typedef struct fse_cnn_s* fse_cnn_t;

/* Number of parameters of the network (1212096). */
int64_t fse_cnn_num_params(void);

/* Create the network on the current device for batches of up to max_batch
 * samples: FP32 master parameters (He-uniform weights drawn from `seed`,
 * zero biases), their BF16 working copy and the Adam state. Training
 * buffers are allocated by the first forward that keeps activations. */
fse_status_t fse_cnn_create(int32_t max_batch, uint64_t seed, fse_cnn_t* out);
void fse_cnn_destroy(fse_cnn_t net);

/* Host copies of the FP32 master parameters: set (also refreshes the BF16
 * copy) and get; get may also fetch the accumulated gradient (h_grads not
 * null). Synchronous. */
fse_status_t fse_cnn_set_params(fse_cnn_t net, const float* h_params);
fse_status_t fse_cnn_get_params(fse_cnn_t net, float* h_params, float* h_grads);

/* Network inputs for every block of a batch whose areas are all 48x48:
 * d_x [n_blocks][48][48][2] BF16, row i for block i of the caller's list.
 * Returns FSE_ERR_UNSUPPORTED for other area sizes. Asynchronous. */
fse_status_t fse_cnn_patches(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail, int64_t pitch,
                             uint16_t* d_x, void* stream);

/* Forward pass for every block of a batch whose areas are all 48x48, the
 * network inputs built on the fly from the frames (the inputs
 * fse_cnn_patches would write): d_logits [n_blocks][4096] FP32, row i for
 * block i of the caller's list, the same values as fse_cnn_patches followed
 * by fse_cnn_forward. n_blocks must not exceed the network's max_batch; no
 * activations are kept. Returns FSE_ERR_UNSUPPORTED for other area sizes.
 * Asynchronous. */
fse_status_t fse_cnn_forward_blocks(fse_cnn_t net, fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                    int64_t pitch, float* d_logits, void* stream);

/* Forward pass: d_logits [B][4096] FP32. keep_activations != 0 stores what
 * fse_cnn_backward needs. Asynchronous. */
fse_status_t fse_cnn_forward(fse_cnn_t net, const uint16_t* d_x, int32_t B, float* d_logits,
                             int32_t keep_activations, void* stream);

/* Loss and gradient of the last forward (same d_x and B, activations kept):
 * binary cross-entropy of d_logits against the target bits
 * d_target_bits [B][128] (bit l%32 of word l/32 = bin l selected), positives
 * weighted by pos_weight, averaged over B*4096 terms; adds the loss to
 * *d_loss and writes the gradient into the network's gradient buffer
 * (cleared by fse_cnn_adam). B must be a multiple of 16. Asynchronous. */
fse_status_t fse_cnn_backward(fse_cnn_t net, const uint16_t* d_x, const float* d_logits,
                              const uint32_t* d_target_bits, int32_t B, float pos_weight, float* d_loss,
                              void* stream);

/* One Adam step on the FP32 master parameters with bias correction, then
 * the BF16 copy is refreshed and the gradient cleared. Asynchronous. */
fse_status_t fse_cnn_adam(fse_cnn_t net, float lr, float beta1, float beta2, float eps, void* stream);

/* Candidate sets: for each of B rows of d_logits [B][4096], the K bins with
 * the largest logits (ties to the lower bin), written in ascending bin order
 * to d_cand [B][K]; d_flags[b] = 1 if row b holds a NaN (the block then
 * falls back to plain FSE), else 0. Asynchronous. */
fse_status_t fse_cnn_topk(const float* d_logits, int32_t B, int32_t K, int16_t* d_cand, int32_t* d_flags,
                          void* stream);

/* Warm-started cFSE for a batch whose blocks all use F = 64. For block i
 * with d_flags[i] == 0: restricted_iters iterations over the kc candidates
 * d_cand[i][0..kc) (ascending bins), their distinct coefficients applied
 * to the whole spectrum, then the block's `iters` full iterations. A block
 * with d_flags[i] != 0 runs fallback_iters plain iterations instead
 * (bit-identical to fse_extrapolate_batch with that count). When every
 * block's `iters` is 0 the work runs as two kernels (transform and staging
 * of W rows 0..32 and of R_w at the candidates, then one workgroup per
 * block for the restricted iterations) with kc in {128, 256, 384, 512};
 * otherwise as one kernel with kc in {128, 256, 512}. Both forms give the
 * same results. Output, status and threading as fse_extrapolate_batch;
 * d_trace (optional) rows have fse_warm_trace_stride(...) entries: the
 * restricted selections first. The staging buffer of the two-kernel form
 * (n_blocks x (16896 + 4096) bytes, room for any compiled kc) is allocated
 * by fse_warm_prepare, or by the first call here if that was not called,
 * and kept by the batch until fse_batch_destroy; a batch made by
 * fse_batch_create_in with FSE_WS_WARM takes it from its workspace instead
 * (without the flag: FSE_ERR_WORKSPACE). After fse_warm_prepare
 * with the same (kc, restricted_iters, fallback_iters) this call allocates
 * nothing and may be captured into a HIP graph; a call with other counts
 * reconfigures the batch (host state only), which a graph captured before
 * does not see. */
fse_status_t fse_warm_extrapolate_batch(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                        int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                        fse_trace_t* d_trace, const int16_t* d_cand, const int32_t* d_flags,
                                        int32_t kc, int32_t restricted_iters, int32_t fallback_iters,
                                        void* stream);

/* Set-up of the warm start (Algorithm 1 started from a candidate set; same
 * arguments as fse_warm_extrapolate_batch): chooses the kernels and their
 * launch shape for (kc, restricted_iters, fallback_iters) and allocates the
 * batch's staging buffer if the two-kernel form needs one. Synchronous, host
 * side plus one allocation; call it before capturing warm-started launches
 * into a graph or in a loop that must not allocate. Errors as
 * fse_warm_extrapolate_batch. */
fse_status_t fse_warm_prepare(fse_batch_t batch, int32_t kc, int32_t restricted_iters, int32_t fallback_iters);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * warm-started cFSE of fse_warm_extrapolate_batch, same arguments, same
 * kernels and the same bits, but it allocates nothing. The two-kernel
 * form's staging lives in a static array of 48 MiB that the library holds
 * on every device it runs on until the process ends; the batch's blocks run
 * in consecutive ranges of at most fse_warm_noalloc_max_blocks(kc) blocks
 * that reuse it in stream order. Every call on a device shares that
 * device's array: calls that overlap on one device (other streams, other
 * threads) race and give undefined results. kc beyond the array
 * (fse_warm_noalloc_max_blocks(kc) == 0) is FSE_ERR_UNSUPPORTED. A change of
 * (kc, restricted_iters, fallback_iters) reconfigures the batch's host
 * state only (no allocation). Other errors as fse_warm_extrapolate_batch. */
fse_status_t fse_warm_extrapolate_batch_noalloc(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail,
                                                int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                                fse_trace_t* d_trace, const int16_t* d_cand, const int32_t* d_flags,
                                                int32_t kc, int32_t restricted_iters, int32_t fallback_iters,
                                                void* stream);

/* Blocks per staging range of fse_warm_extrapolate_batch_noalloc for kc
 * candidates (0 when kc < 1 or kc > 512). Host only. */
size_t fse_warm_noalloc_max_blocks(int32_t kc);

/* Step of the warm start's restricted iterations: the gamma of eq. (13)
 * used while the argmax and update run over the candidates (the full
 * iterations after them and every fallback keep the plan's gamma). A value
 * in (0, 1]; a negative value restores the plan's gamma (the default). Host
 * state of the batch, read by later warm-started launches (a graph captured
 * before the change keeps the old step). */
fse_status_t fse_warm_set_restricted_gamma(fse_batch_t batch, float gamma_r);

/* Squared magnitudes of the first transform, |R_w[k, l]|^2 = |DFT(s w)|^2
 * (eq. (11), the criterion of eq. (12) before the first selection), for
 * every block of a batch whose blocks all use F = 64: d_power [n_blocks][4096]
 * FP32 in the caller's block order, bin k*64 + l; the same FP32 values the
 * iterations compare. Candidate sets that do not come from the network (the
 * top-K of this spectrum, fse_cnn_topk on d_power) serve as the comparison
 * for the learned ones. Asynchronous on `stream`; errors as
 * fse_warm_extrapolate_batch. */
fse_status_t fse_initial_power(fse_batch_t batch, const uint8_t* d_image, const uint8_t* d_avail, int64_t pitch,
                               float* d_power, void* stream);

/* restricted_iters + max(largest block iteration count, fallback_iters). */
int32_t fse_warm_trace_stride(fse_batch_t batch, int32_t restricted_iters, int32_t fallback_iters);

/* ------------------------------------------------------------------------
 * Three dimensions (video). cFSE extends to more dimensions (Section II and
 * the Conclusion): the same iteration on an F x F x Ft grid, the window
 * rho^(distance) in pixel and frame units, B a lost volume. One workgroup
 * of 1024 threads per volume: R_w in registers (32 bins per thread), the
 * half of W with l <= 32 in LDS (132 KB), the transform as Ft-point DFTs
 * per pixel followed by the 2-D FFTs of the Ft slices in LDS; nothing but
 * the output is written to device memory.
 *
 * fse_batch3d_create validates h_volumes (fft = 64, fft_t = 8, area within
 * the transform, B inside the clip, 0 <= iters <= the plan's max_iters, no
 * two B overlapping; the plan must not have FSE_PLAN_MASKED_B,
 * FSE_PLAN_REAL or FSE_PLAN_FIXED), uploads
 * them and the 3-D window table to the current device. Synchronous.
 * *bad_index (if not null)
 * receives the first offending volume or -1. */
typedef struct fse_batch3d_s* fse_batch3d_t;
fse_status_t fse_batch3d_create(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes,
                                int32_t n_frames, int32_t H, int32_t W, fse_batch3d_t* out_batch,
                                int32_t* bad_index);
void fse_batch3d_destroy(fse_batch3d_t batch);

/* Bytes of device workspace fse_batch3d_create_in needs for n_volumes
 * volumes: the volume descriptors, the 3-D window table of eq. (3) and the
 * 64-point twiddles, each 256-byte aligned. Host-only. FSE_ERR_INVALID_ARG
 * for a null argument or n_volumes < 0. */
fse_status_t fse_batch3d_workspace_size(fse_plan_t plan, int32_t n_volumes, size_t* bytes);

/* fse_batch3d_create with caller-owned device memory, under the conditions
 * of fse_batch_create_in (256-byte aligned device memory of the current
 * device, at least fse_batch3d_workspace_size bytes inside one allocation,
 * kept and untouched until fse_batch3d_destroy, which frees nothing).
 * Same results as fse_batch3d_create's batch; errors as fse_batch3d_create
 * plus FSE_ERR_INVALID_ARG and FSE_ERR_WORKSPACE as fse_batch_create_in. */
fse_status_t fse_batch3d_create_in(fse_plan_t plan, const fse_volume_t* h_volumes, int32_t n_volumes,
                                   int32_t n_frames, int32_t H, int32_t W, void* d_workspace, size_t ws_bytes,
                                   fse_batch3d_t* out_batch, int32_t* bad_index);

/* Conceal every volume of the batch: frames and avail are uint8
 * [n_frames][H][pitch], d_out float32 [n_frames][H][out_pitch] (only the
 * voxels of each B are written), d_status int32 [n_volumes] (FSE_BLOCK_*),
 * d_trace null or fse_trace_t [n_volumes][max iters of the batch].
 * Asynchronous on `stream`; no allocation. */
fse_status_t fse_extrapolate3d_batch(fse_batch3d_t batch, const uint8_t* d_frames, const uint8_t* d_avail,
                                     int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                     fse_trace_t* d_trace, void* stream);

/* Warm-started 3-D cFSE: the iterations of fse_extrapolate3d_batch with the
 * argmax and the update restricted to candidate bins (a restriction of the
 * dictionary; every equation unchanged). d_cand2 is int16 [n_volumes][k2]:
 * for each volume k2 = 128 distinct columns k * 64 + l in ascending order
 * (for instance the top-128 bins of the 2-D warm-start network run on the
 * volume's first lost frame, fse_cnn_forward_blocks + fse_cnn_topk); the
 * candidates are those columns with every s, 1024 bins. d_flags int32
 * [n_volumes] as written by fse_cnn_topk: a volume whose flag is nonzero is
 * not concealed (status FSE_BLOCK_NONFINITE, B untouched; run it with
 * fse_extrapolate3d_batch). Other arguments, results and errors as for
 * fse_extrapolate3d_batch; FSE_ERR_UNSUPPORTED for k2 != 128. */
fse_status_t fse_warm3d_extrapolate_batch(fse_batch3d_t batch, const uint8_t* d_frames, const uint8_t* d_avail,
                                          int64_t pitch, float* d_out, int64_t out_pitch, int32_t* d_status,
                                          fse_trace_t* d_trace, const int16_t* d_cand2, const int32_t* d_flags,
                                          int32_t k2, void* stream);

/* Measurement (roofline accounting): the LDS read bandwidth of the current
 * device, measured by a kernel in which every workgroup (5 per compute
 * unit, 32 KiB of LDS each) streams `iters` x 8 conflict-free 16-byte reads
 * per thread (64 consecutive lanes read 1 KiB of consecutive entries).
 * Launches three times to warm up, then times five launches with HIP events on
 * `stream`; writes the aggregate bytes/s of the median to *bytes_per_s. Synchronous;
 * allocates and frees a small device buffer. FSE_ERR_INVALID_ARG for a null
 * pointer or iters outside [1, 2^20]. */
fse_status_t fse_measure_lds_bandwidth(int32_t iters, void* stream, double* bytes_per_s);

/* Static description of the most recent error on this thread (never null). */
const char* fse_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* FSE_H_ */
