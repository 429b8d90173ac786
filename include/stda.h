/*
 * stda.h -- C ABI of the MI355X (gfx950) Radar-STDA hot path.
 *
 * Radar-STDA (arXiv 2307.09063) is a spatial-temporal denoising autoencoder: three consecutive
 * interfered range-Doppler (RD) maps in, the clean RD map of the latest frame out
 * (Sec. IV-A, Eq. (encoder_stda), Eq. (decoder_stda)).  This library runs its forward pass,
 * its hand-written training backward pass, an SGD step, the reconstruction loss, the SINR
 * metric and the FMCW RD-map synthesizer that produces its inputs, all as hand-written HIP
 * kernels.
 *
 * Conventions shared by every entry point
 *  - Memory.  Every pointer named *_dev, and every tensor argument, is DEVICE memory owned by
 *    the caller; host arrays are marked host.  The library never allocates or frees device
 *    memory: scratch comes in through `ws` (and, between a training forward and its backward,
 *    `saved`), sized by the matching *_size query.
 *  - Streams.  Work is enqueued on `stream` (0 = the null stream) and the call returns without
 *    waiting.  Results are valid once the stream has been synchronised.
 *  - Errors.  Arguments are validated before anything is enqueued; on error nothing runs and a
 *    negative stda_status is returned.  STDA_E_HIP carries the HIP error, retrievable with
 *    stda_last_hip_error().  No C++ exception crosses the ABI.
 *  - Threads.  Entry points are re-entrant; two calls that share `ws` or `saved` on different
 *    streams race.
 *  - Layout.  Boundary maps are FP32, planar: x is [clips][3][H][W] with channel 0 = frame t,
 *    1 = frame t-1, 2 = frame t-2 (Sec. IV-B, Eq. (concat_operation)); z, y, dz are
 *    [clips][1][H][W].  H = range bins (samples per chirp), W = Doppler bins (chirps).
 *    Internally activations are NHWC, FP32 or BF16.
 */
#ifndef STDA_H
#define STDA_H

#include <stddef.h>
#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  STDA_OK = 0,
  STDA_E_INVALID = -1,     /* null pointer, unknown enum, bad count                      */
  STDA_E_SHAPE = -2,       /* H or W not a multiple of 4, below 8, or above 4096          */
  STDA_E_WORKSPACE = -3,   /* ws / saved smaller than the size query says                 */
  STDA_E_HIP = -4,         /* a HIP runtime call or launch failed                         */
  STDA_E_NONFINITE = -5    /* stda_autotune: a timed step's loss was NaN / Inf            */
} stda_status;

typedef enum { STDA_FP32 = 0, STDA_BF16 = 1 } stda_dtype;  /* activation / weight storage  */
typedef enum { STDA_EVAL = 0, STDA_TRAIN = 1 } stda_mode;    /* BN running vs batch stats   */

/*
 * A segment is a group of clips of one map size.  Batch-norm statistics in TRAIN mode are
 * taken over one segment (its clips x H x W); a batch of uneven map sizes is a list of
 * segments.  x_off / z_off are element offsets of the segment's first clip in the packed x
 * (3*H*W floats per clip) and z / y / dz (H*W floats per clip).
 */
typedef struct {
  int32_t n;        /* clips in the segment, >= 1                                          */
  int32_t H, W;     /* range bins, Doppler bins: multiples of 4 in [8, 4096]                */
  int64_t x_off;
  int64_t z_off;
} stda_segment;

/* One entry of the flat FP32 parameter buffer (137,469 floats). */
typedef struct {
  char name[40];
  int64_t offset;   /* element offset into the flat buffer                                 */
  int32_t ndim;
  int32_t shape[4]; /* conv: [Cout, Cin/groups, k, k]; deconv: [Cin, Cout/groups, k, k]      */
  int32_t fan_in;   /* (Cin/groups) * k * k for conv and deconv weights; 0 otherwise        */
} stda_param_desc;

const char* stda_status_string(int status);
int stda_last_hip_error(void);

/* Parameter layout (the network of Sec. IV; readings of unstated sizes are fixed here). */
size_t stda_param_count(void);
/* Writes min(cap, count) descriptors to host `out`; returns the total count. */
int stda_param_table(stda_param_desc* out, int cap);
/* BN layers: 17; running buffer = per layer C means then C variances (1,184 floats). */
int stda_bn_layer_count(void);
size_t stda_running_count(void);

/* ------------------------------------------------------------------ architecture readings
 * Three places where the text of Sec. IV-C leaves the network open are selectable, process-wide
 * (the default, 0, is the network described above):
 *   STDA_ARCH_RES3    decoder long residual of Eq. (mobile_decoder_stage2) as DeConv3x3-s2-p1
 *                     with output padding 1 (weight [Cin][Cout][3][3]) instead of DeConv4x4-s2-p1;
 *                     the parameter count drops to 119,549.
 *   STDA_ARCH_SIGMOID logistic sigmoid on the output module: z = sigma(Conv3x3(d1) + b).  TRAIN
 *                     saves a copy of z (4 bytes per pixel) for the backward.
 *   STDA_ARCH_PW_DW   stage-1 1x1 branch of Eq. (mobile_encoder_stage1) / (mobile_decoder_stage1)
 *                     depthwise (weight [C][1][1][1]) instead of dense; 6,256 parameters fewer.
 * The setting is read by every call: the parameter table and count, workspace sizes, and the
 * launches.  A parameter vector, `saved` buffer or captured graph made under one setting must not
 * be used under another.  Not synchronised: change it only while no other thread is inside the
 * library.  Returns STDA_E_INVALID for unknown bits.
 */
#define STDA_ARCH_RES3 1
#define STDA_ARCH_SIGMOID 2
#define STDA_ARCH_PW_DW 4
int stda_set_arch(int flags);
int stda_get_arch(void);

/*
 * Byte sizes of `saved` (kept from a TRAIN forward to its backward) and `ws` (scratch of a
 * single call; one size serves forward, backward and loss).  `recompute` != 0 keeps the
 * block-boundary checkpoints and each block's output before ECA (with its stage-2 ReLU decisions)
 * in `saved` and recomputes the other block internals (stage-1 output, stage-2 pre-BN) during the
 * backward.
 */
int stda_workspace_size(const stda_segment* segs /*host*/, int n_segs, int dtype, int mode,
                        int recompute, size_t* saved_bytes /*host out*/,
                        size_t* ws_bytes /*host out*/);

/*
 * Forward pass of Radar-STDA (Sec. IV, Eq. (decoder_stda)): z = f(h(x_t, x_t-1, x_t-2)).
 *   x       [sum 3*H*W]  FP32 boundary maps (segment layout above).
 *   w       [137,469]    FP32 master parameters; BF16 mode rounds them to nearest-even.
 *   running [1,184]      BN running mean / variance; read in EVAL, updated in TRAIN
 *                        (momentum 0.1, unbiased variance), one update per segment in order.
 *   z       [sum H*W]    FP32 restored map of frame t.
 *   saved   TRAIN: filled for stda_backward (may be NULL in EVAL).
 * Returns STDA_OK or an error (nothing enqueued on error).
 */
int stda_forward(const stda_segment* segs /*host*/, int n_segs, const float* x, const float* w,
                 float* running, float* z, void* saved, size_t saved_bytes, void* ws,
                 size_t ws_bytes, int dtype, int mode, int recompute, hipStream_t stream);

/*
 * EVAL forward without a caller workspace, for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid hipMalloc).  Same result as
 * stda_forward in EVAL mode with the same arguments; the kernels' scratch is a library-owned
 * static device array of STDA_NOALLOC_WS_MAX bytes (32 MiB) on each GPU the library runs on,
 * held until the process ends.  The call allocates nothing.
 *   segs, x, w, z, dtype: as stda_forward; running: read only (EVAL statistics).
 *   stream: must belong to the current device (STDA_E_INVALID otherwise).
 * Batches whose EVAL workspace (stda_workspace_size, mode EVAL) exceeds STDA_NOALLOC_WS_MAX are
 * refused with STDA_E_WORKSPACE before anything is enqueued (one clip of 256 x 128 needs 29 MiB
 * in FP32, 18 MiB in BF16; the paper's single 128 x 64 clip 13 MiB).  Every call on one GPU shares its array and nothing in it has to
 * start at any value: calls that overlap on one GPU (other streams, other threads) race and must
 * be serialised by the caller.  The first call on a device looks up the array's address there.
 */
#define STDA_NOALLOC_WS_MAX (32u << 20)
int stda_forward_noalloc(const stda_segment* segs /*host*/, int n_segs, const float* x, const float* w,
                         const float* running, float* z, int dtype, hipStream_t stream);

/* ------------------------------------------------------------------ folded EVAL inference
 * In EVAL mode every batch normalisation is a fixed per-channel affine map, which folds into the
 * adjacent weights (the re-parameterisation the mobile block of Sec. IV-C takes from MobileOne):
 * stage 1 becomes ReLU(PW'(x) + DW'(x) + b1) with the identity branch on the 1x1 weight's
 * diagonal, stage 2 ReLU(conv'(x1) + b) + conv_res(x), the input module ReLU(conv'(x) + b').
 * stda_eval_fold computes the folded parameters once, from the FP32 master parameters w and the
 * running statistics, into the caller's device buffer `folded` (stda_eval_fold_size bytes; for
 * `dtype`, whose stage-2 weights it also arranges for the matrix cores).  stda_forward_folded then
 * runs the EVAL forward on it: per mobile block one stage-1 launch, one launch for all of stage 2
 * (both convolutions, bias, ReLU and the residual sum) and one for ECA and the skip; z equals
 * stda_forward's EVAL result up to rounding.  ws: stda_workspace_size's ws bytes for these
 * segments in EVAL mode.  The main architecture reading and the sigmoid output are supported;
 * STDA_ARCH_RES3 and STDA_ARCH_PW_DW give STDA_E_INVALID.  A folded buffer is valid until w or
 * the running statistics change.
 */
int stda_eval_fold_size(int dtype, size_t* bytes /*host out*/);
int stda_eval_fold(const float* w, const float* running, void* folded, size_t folded_bytes, int dtype,
                   hipStream_t stream);
int stda_forward_folded(const stda_segment* segs /*host*/, int n_segs, const float* x, const void* folded,
                        size_t folded_bytes, float* z, void* ws, size_t ws_bytes, int dtype, hipStream_t stream);

/*
 * Hand-written adjoint of the TRAIN forward that filled `saved` (same segs, x, w, dtype,
 * recompute; x is read again for the input-module weight gradient).  dz = dL/dz; writes dw (all
 * 137,469 gradients, summed over segments; no zero initialisation needed) and, if dx is not NULL,
 * dL/dx.  Weight-gradient partials are reduced across blocks in FP64.
 * Every TRAIN forward records, on the host, the layout key of the `saved` it filled (segments,
 * dtype, recompute, architecture reading); a `saved` that no TRAIN forward of this process filled
 * under the same key is refused with STDA_E_INVALID (the layout would not match).
 */
int stda_backward(const stda_segment* segs /*host*/, int n_segs, const float* x, const float* dz,
                  const float* w, const void* saved, size_t saved_bytes, float* dw, float* dx,
                  void* ws, size_t ws_bytes, int dtype, int recompute, hipStream_t stream);

/*
 * Reconstruction loss (a reading: the paper names none): per segment the mean of (z - y)^2
 * over its clips x H x W, summed over segments, reduced in FP64 into loss_dev[0];
 * dz = 2 (z - y) / (n_s H W).  ws must hold stda_workspace_size's ws bytes for these segs.
 */
int stda_mse_loss(const stda_segment* segs /*host*/, int n_segs, const float* z, const float* y,
                  double* loss_dev, float* dz, void* ws, size_t ws_bytes, hipStream_t stream);

/*
 * SGD with L2 weight decay over the flat master buffer: w <- w - lr (g + weight_decay w).
 * If w_bf16 is not NULL it receives the round-to-nearest-even BF16 copy of the new w.
 */
int stda_sgd_step(float* w, const float* dw, int64_t n, float lr, float weight_decay,
                  uint16_t* w_bf16, hipStream_t stream);

/*
 * AdamW (Table 5 names AdamW with weight decay and step annealing; moment coefficients and the
 * annealing period are not given, so they are parameters here).  State in DEVICE memory, owned
 * by the caller and initialised once (t = 0; m and v zero):
 *   lr_t = lr * gamma^floor(t / step_size) (step_size 0: constant), t = steps already taken;
 *   m <- b1 m + (1 - b1) g;  v <- b2 v + (1 - b2) g^2;
 *   w <- w (1 - lr_t weight_decay) - lr_t (m / (1 - b1^(t+1))) / (sqrt(v / (1 - b2^(t+1))) + eps);
 * then t <- t + 1 on the device (so a captured graph replays consecutive steps).  m, v: [n] FP32
 * (device); w_bf16 as in stda_sgd_step.
 */
typedef struct {
  double lr, beta1, beta2, eps, weight_decay, gamma;  /* FP64 so that 1 - beta is exact enough */
  int32_t step_size;
  int32_t t;
} stda_adamw_state;
int stda_adamw_step(float* w, const float* dw, float* m, float* v, int64_t n,
                    stda_adamw_state* state_dev, uint16_t* w_bf16, hipStream_t stream);

/*
 * SINR of Sec. V-B over a batch of maps: per map 10 log10(mean_O m^2 / mean_N m^2) where the
 * O and N cells are given by the byte masks o_mask / n_mask ([n_maps][H][W], 1 = member).
 * Sums are FP64; out_dev[n_maps] receives the dB values.
 */
int stda_sinr(const float* maps, const uint8_t* o_mask, const uint8_t* n_mask, int n_maps, int H,
              int W, double* out_dev, hipStream_t stream);

/* ------------------------------------------------------------------ detection step */
/*
 * CA-CFAR peak detection on restored maps (Sec. V-B names a cell-averaging CFAR as the peak
 * detector whose hits the average precision of Eq. (21) counts; its parameters are a reading).
 * Square-law statistic p = m^2 of each map value m.  The training cells of a cell are those of
 * the (2(guard_r+train_r)+1) x (2(guard_d+train_d)+1) window around it (rows = range, columns =
 * Doppler) outside the (2 guard_r+1) x (2 guard_d+1) guard window; columns wrap around (the
 * Doppler axis is circular), rows outside the map do not count.  With N training cells summing to
 * S (FP64), the cell is detected when p > alpha(N) S / N, alpha(N) = N (pfa^(-1/N) - 1).
 *   maps     [n_maps][H][W] FP32 (device)
 *   det      [n_maps][H][W] bytes out, 1 = detection (device)
 *   o_mask   [n_maps][H][W] reference-peak cells, 1 = member, or NULL (device)
 *   counts   [n_maps][2] int32 out or NULL (device): detections, detections on o_mask cells
 * guard_r + train_r and guard_d + train_d must not exceed STDA_CFAR_MAX_HALO and the windows
 * must fit the map (STDA_E_SHAPE); at least one training extent must be positive and
 * 0 < pfa < 1 (STDA_E_INVALID).
 */
#define STDA_CFAR_MAX_HALO 8
int stda_cfar(const float* maps, int n_maps, int H, int W, int guard_r, int guard_d, int train_r,
              int train_d, double pfa, uint8_t* det, const uint8_t* o_mask, int32_t* counts,
              hipStream_t stream);

/*
 * EVM of Sec. V-B, Eq. (20), per map: the mean over the o_mask cells of |clean - est| / |clean|,
 * FP64 sums, into out_dev[n_maps]; a map without o_mask cells gives 0.  All arrays are
 * [n_maps][H][W] on the device.
 */
int stda_evm(const float* est, const float* clean, const uint8_t* o_mask, int n_maps, int H, int W,
             double* out_dev, hipStream_t stream);

/* ------------------------------------------------------------------ captured training step */
/*
 * One training step -- stda_forward (TRAIN), stda_mse_loss against y, stda_backward (dx not
 * computed), stda_sgd_step -- captured once from the given arguments into a hipGraph and
 * instantiated.  Every later stda_graph_launch replays exactly those kernels on those buffers
 * (one host call per step; the buffers' contents may change between launches, their addresses
 * may not).  `stream` must be a non-null stream (capture is per-thread; nothing is executed while
 * capturing).  Arguments are validated first; on error nothing is captured and *graph is NULL.
 * The timing hook must be off while capturing.  Uneven batches are captured as their segment
 * list, so one launch runs every segment of the step.
 */
typedef struct stda_graph_s* stda_graph;
int stda_train_step_graph_create(const stda_segment* segs /*host*/, int n_segs, const float* x,
                                 const float* y, float* w, float* running, float* z,
                                 double* loss_dev, float* dz, float* dw, void* saved,
                                 size_t saved_bytes, void* ws, size_t ws_bytes, int dtype,
                                 int recompute, float lr, float weight_decay, uint16_t* w_bf16,
                                 hipStream_t stream, stda_graph* graph /*host out*/);
/*
 * Inference form of the forward (Sec. IV; the paper reports throughput for one clip at a time):
 * one EVAL (or TRAIN) forward captured into a graph on the caller's (non-null) stream, for
 * replay with stda_graph_launch at low latency.  Arguments as stda_forward; the buffers are
 * bound at capture time.
 */
int stda_forward_graph_create(const stda_segment* segs /*host*/, int n_segs, const float* x,
                              const float* w, float* running, float* z, void* saved,
                              size_t saved_bytes, void* ws, size_t ws_bytes, int dtype, int mode,
                              hipStream_t stream, stda_graph* graph /*host out*/);
/* The folded EVAL forward (stda_forward_folded) captured the same way. */
int stda_forward_folded_graph_create(const stda_segment* segs /*host*/, int n_segs, const float* x,
                                     const void* folded, size_t folded_bytes, float* z, void* ws,
                                     size_t ws_bytes, int dtype, hipStream_t stream,
                                     stda_graph* graph /*host out*/);
int stda_graph_launch(stda_graph graph, hipStream_t stream);
/* Frees the graph and its handle (NULL is a no-op); STDA_E_HIP if HIP reports an error, the
 * handle is freed in any case. */
int stda_graph_destroy(stda_graph graph);

/* ------------------------------------------------------------------ measurement hooks */
/*
 * Per-kernel timing.  After stda_profile_select(tag) every launch carrying that tag (for example
 * "dense_fwd_main.dec1", "wgrad_main.dec0", "s1_bwd_apply.enc0", "stem_bwd_apply") is bracketed
 * by two HIP events recorded on its launch stream; NULL or "" turns the hook off.  Selecting
 * resets the record.  stda_profile_read waits for the recorded events and returns the summed
 * kernel time in milliseconds and the number of bracketed launches.  Tags are listed next to
 * the launches in the library source; an unknown tag simply records nothing.
 */
int stda_profile_select(const char* tag);
int stda_profile_read(double* total_ms /*host out*/, int* count /*host out*/);
/*
 * With the tag "*" every tagged launch is recorded.  stda_profile_report writes one line per
 * tag, "tag<TAB>launches<TAB>total_ms", into host buf (NUL-terminated, truncated to cap) and the
 * size it needs into *needed.
 */
int stda_profile_report(char* buf /*host out*/, size_t cap, size_t* needed /*host out*/);

/* ------------------------------------------------------------------ tile-shape autotuning
 * The stage-2 dense layers (Conv3x3-s2 / DeConv4x4-s2, their input and weight gradients) and the
 * fused stage-1 adjoint have several tilings each.  A tunable launch is (kind, dtype, block):
 * kind 0 = stage-2 forward (main and residual convolution), 1 = stage-2 input gradient (both),
 * 2 = stage-2 weight gradient (both), 3 = stage-1 adjoint (tile shape and registers per thread);
 * block 0..3 = encoder 0, encoder 1, decoder 0, decoder 1.  The choice is process-wide and read
 * when a launch is enqueued (a captured graph keeps the choice it was captured with).
 */
int stda_tune_count(int kind);  /* number of variants of `kind`, or a negative status */
int stda_tune_set(int kind, int dtype, int block, int variant);
int stda_tune_get(int kind, int dtype, int block, int* variant /*host out*/);

/*
 * Upper bound on the workgroups of every tiled network kernel (0, the default, = no bound beyond
 * the kernel's own).  Those kernels hand their tiles to a persistent grid and carry accumulators
 * (batch-norm partial sums, weight-gradient products) from one tile to the next; a small bound
 * makes a small batch take the same multi-tile paths a large one does.  A bound that is a multiple
 * of 8 keeps the XCD-contiguous tile schedule, any other the plain grid stride.  Process-wide, read
 * when a launch is enqueued (a captured graph keeps its grid).  Negative: STDA_E_INVALID.
 */
int stda_set_grid_cap(int cap);
int stda_get_grid_cap(void);

/*
 * Autotuner: for every variant v, sets all tunable launches of `dtype` to v, runs one untimed
 * training forward + loss + backward on the given buffers and then `reps` timed ones (HIP events
 * around each tunable launch), and finally sets every tunable launch to its fastest variant
 * (variant 0, the default, unless another is at least 3 % faster).
 * Arguments are those of stda_forward / stda_mse_loss / stda_backward; `running` is updated by
 * every trial step (pass a scratch copy), w is not modified, z / loss / dz / dw are overwritten.
 * The per-variant times and the choice are written as text lines
 * "kind<TAB>block<TAB>ms_v0<TAB>ms_v1...<TAB>chosen" into host `report` (NUL-terminated,
 * truncated to cap; may be NULL) and the size needed into *needed (may be NULL).  Blocks the
 * host until the trials are done.  The per-kernel timing hook must be off.  Returns
 * STDA_E_NONFINITE (with the previous choice restored) when a variant's last timed step ends with
 * a NaN / Inf loss.  The choice table is process-wide: other threads' calls may run during the
 * trials with whichever variants are set at the time.
 */
int stda_autotune(const stda_segment* segs /*host*/, int n_segs, const float* x, const float* y,
                  const float* w, float* running, float* z, double* loss_dev, float* dz, float* dw,
                  void* saved, size_t saved_bytes, void* ws, size_t ws_bytes, int dtype,
                  int recompute, int reps, hipStream_t stream, char* report /*host out*/,
                  size_t cap, size_t* needed /*host out*/);

/* ------------------------------------------------------------------ RD-map synthesizer */
#define RD_MAX_TONES 48
#define RD_MAX_INTF 4

/* Target or clutter tone of one frame: a exp(j 2 pi (fr n + fd m + ph) / 2^32). */
typedef struct {
  uint32_t fr;      /* range frequency, cycles/sample in 32-bit fixed point (mod 1)          */
  uint32_t fd;      /* Doppler frequency, cycles/chirp in 32-bit fixed point (mod 1)         */
  uint32_t ph;      /* phase at n = m = 0, cycles in 32-bit fixed point                      */
  float amp;
} rd_tone;

/*
 * FMCW interferer of one frame after dechirping (Sec. III-A, Eq. (IF signal)).  All frequencies
 * are signed 2^-32 cycles/sample.  The start beat frequency of victim chirp m is
 *   g(m) = f0 + m dl                          (wrap == 0)
 *   g(m) = f0 + ((s0 + m dl) mod wrap)        (wrap > 0, the remainder in [0, wrap)): the
 *          aggressor's own ramp, sampled at each victim chirp start, is a sawtooth of span wrap;
 * the beat frequency is F(n, m) = 2 q n + g(m) and the term a exp(j 2 pi (g(m) n + q n^2 + phi_m)
 * / 2^32) is present while |F| < 2^31 (an ideal IF low-pass at half the sampling rate).
 * phi_m = word 0 of Philox4x32-10(counter = (m, i, frame, 1), key = (seed, clip)) when
 * coherent == 0, else ph0 + m phd (mod 2^32; oscillators coherent from chirp to chirp).
 */
typedef struct {
  int64_t q;
  int64_t f0;
  int64_t dl;
  int64_t s0;
  int64_t wrap;
  uint32_t ph0;
  uint32_t phd;
  float amp;
  uint32_t coherent;
} rd_intf;

typedef struct {
  int32_t n_tones[3];                  /* per frame t, t-1, t-2                             */
  int32_t n_intf[3];
  rd_tone tone[3][RD_MAX_TONES];
  rd_intf intf[3][RD_MAX_INTF];
} rd_scene;

size_t rd_synth_workspace_size(int n_clips, int N, int M);

/*
 * RD-map synthesis (Sec. III-A, Eq. (discrete signal), Eq. (IF signal); Sec. III-B,
 * Eq. (column transform), Eq. (row transform)).  For each clip c and frame f:
 *   s(n, m) = tones + interferers + noise, noise = sigma/sqrt(2) (g0 + j g1) with g0, g1 from
 *   Box-Muller on words 0, 1 of Philox4x32-10(counter = (n, m, f, 0), key = (seed, clip_base + c));
 *   periodic Hann windows on n and m; N-point DFT over n, M-point DFT over m; zero Doppler
 *   moved to column M/2; 20 log10 |Y| floored at (max - 80 dB); min-max scaled to [0, 1].
 * scenes: DEVICE array of n_clips rd_scene.  N, M: powers of two in [8, 1024].
 * x_out [n_clips][3][N][M]: frames t, t-1, t-2 with interference.
 * clean_out [n_clips][1][N][M] (may be NULL): frame t without interferers, same noise.
 */
int rd_synth(const rd_scene* scenes, int n_clips, int N, int M, uint32_t seed, float noise_sigma,
             int clip_base, float* x_out, float* clean_out, void* ws, size_t ws_bytes,
             hipStream_t stream);

/*
 * rd_synth with the scene table in HOST memory (n_clips rd_scene): the table is copied into the
 * end of the workspace and the stream synchronized before the synthesis is enqueued, so the host
 * array may be reused as soon as the call returns (not capturable into a graph).  ws must hold
 * rd_synth_host_workspace_size(n_clips, N, M) bytes; outputs, statuses and the synthesis itself
 * as rd_synth (the same results).
 */
size_t rd_synth_host_workspace_size(int n_clips, int N, int M);
int rd_synth_host(const rd_scene* scenes_host, int n_clips, int N, int M, uint32_t seed,
                  float noise_sigma, int clip_base, float* x_out, float* clean_out, void* ws,
                  size_t ws_bytes, hipStream_t stream);

#ifdef __cplusplus
}
#endif
#endif /* STDA_H */
