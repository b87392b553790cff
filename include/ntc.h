/*
 * ntc.h — C ABI of the MI355X (gfx950) neural texture compression hot path.
 *
 * Method: Vaidyanathan et al., "Random-Access Neural Compression of Material
 * Textures" (arXiv 2305.17105).  A texture set of W x H x C texels with its mip
 * chain is represented by a pyramid of quantized latent grid pairs (section 4.1)
 * and one small per-material MLP (section 4.4).  Decoding a texel samples the
 * grids of the level that serves its mip (four G0 neighbours concatenated, G1
 * bilinear; section 4.3.1), appends a tiled positional encoding (section 4.3.2)
 * and runs the MLP, which outputs all C channels.  Training optimises latents and
 * MLP jointly with L2 loss and Adam (section 4.5), with simulated quantization
 * noise and a post-update clamp (section 4.2).
 *
 * Conventions for every entry point:
 *  - Pointers are DEVICE pointers unless marked (host).  All memory is owned and
 *    allocated by the caller; no entry point allocates device memory.
 *  - `stream` is a hipStream_t (NULL = the null stream).  Work is enqueued
 *    asynchronously; nothing synchronises the host.
 *  - Every argument is validated before anything is enqueued, so a call that
 *    returns an error has no side effect.  Errors never abort the process;
 *    ntc_last_error() gives a message for the calling thread.
 *  - Per-element device data (query coordinates) is never an error: u, v are
 *    clamped to the texture (NaN -> 0), lod is clamped to [0, num_mips-1].
 *  - Calls on the same buffers from different streams are not synchronised
 *    against each other; the caller orders them.
 */
#ifndef NTC_H
#define NTC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  NTC_OK = 0,
  NTC_E_INVALID = 1,      /* bad argument or descriptor */
  NTC_E_UNSUPPORTED = 2,  /* valid, but no kernel is built for this shape */
  NTC_E_WORKSPACE = 3,    /* workspace missing or too small */
  NTC_E_HIP = 4           /* HIP runtime error (also asynchronous errors of earlier work) */
} ntc_status;

typedef enum { NTC_F32 = 0, NTC_F16 = 1, NTC_FP8_E4M3 = 2 } ntc_dtype;

typedef enum { NTC_ACT_RELU = 0, NTC_ACT_HARDGELU = 1 } ntc_activation;

/* Positional encoding (section 4.3.2): per axis, at the texel-centre phase
 * t = ((i mod 8) + 1/2) / 8 and frequencies f = 1, 2, 4 per 8-texel tile, the pair
 * (S(f t), K(f t)).  NTC_PE_SINCOS: S = sin 2 pi x, K = cos 2 pi x.  NTC_PE_TRIANGLE
 * (the paper's triangular waves): S(x) = 4 |frac(x - 1/4) - 1/2| - 1, K(x) =
 * 4 |frac(x) - 1/2| - 1, the piecewise-linear waves with the zeros and extrema of sin
 * and cos.  Either way the last value per axis is identically 0 at texel centres. */
typedef enum { NTC_PE_SINCOS = 0, NTC_PE_TRIANGLE = 1 } ntc_posenc;

/* One texel query: u, v in [0, 1) over the whole texture, integer mip level. 12 bytes. */
typedef struct {
  float u, v;
  int32_t lod;
} ntc_query;

#define NTC_MAX_LEVELS 8
#define NTC_MAX_MIPS 16

/*
 * Material descriptor (host struct, passed by pointer and copied by the callee).
 * The caller sets the first block, then ntc_material_init() validates it and
 * fills the derived geometry (section 4.1, Table 1):
 *   level j: G0 = (W, H) >> (grid_shift + 2 j), G1 = G0 / 2; levels are added
 *   while G1 has at least one cell and the mip chain still reaches them;
 *   mip l is served by level clamp(floor((l - grid_shift) / 2), 0, J - 1).
 * Buffer layouts fixed by the descriptor:
 *   latents (FP32): for each level j ascending, G0^j then G1^j, each [h][w][c].
 *   packed latents: same grid order, each grid a dense LSB-first bitstream of
 *     B-bit codes in cell-major, channel-minor order, padded to 16 bytes; the
 *     unpadded size is the paper's w*h*C*B/8 (Appendix 'Storage Cost').
 *   MLP (FP32, canonical): W1[K][Hd], b1[Hd], W2[Hd][Hd], b2[Hd], W3[Hd][C], b3[C],
 *     K = 4 c0 + c1 + 12 + lod_input (section 4.4).  Input order: G0 neighbours
 *     (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1) each c0 wide, G1 bilinear (c1),
 *     positional encoding (x: the two waves at 1, 2, 4 cycles per 8 texels, then
 *     y), and with lod_input the decoded texel's mip l / (M - 1) (0 when M = 1).
 *   targets (FP32): mips 0..M-1 concatenated, each [H_l][W_l][C].
 */
typedef struct {
  /* set by the caller */
  int32_t width, height;   /* powers of two */
  int32_t channels;        /* C, 1..16 */
  int32_t num_mips;        /* M; 0 selects the full chain down to 1x1 */
  int32_t c0, c1;          /* latent channels of G0 (1..16) and G1 (1..32); kernels exist for
                              c0 = c1 = C in {8, 10, 12, 16} and for Table 3's profiles on
                              C = 9: (c0 x b0, c1 x b1) = (8x2, 12x4), (12x4, 20x4),
                              (12x2, 10x4), (16x4, 12x4) (ntc_shape_supported) */
  int32_t b0, b1;          /* bits per latent: 1, 2, 4 or 8 */
  int32_t grid_shift;      /* G0 at level 0 is the texture size >> grid_shift (2: W/4) */
  int32_t hidden;          /* Hd: 32 or 64 */
  int32_t activation;      /* ntc_activation */
  int32_t posenc;          /* ntc_posenc */
  int32_t lod_input;       /* 1: the normalized mip l / (M - 1) is a network input (section 4.4) */
  /* filled by ntc_material_init */
  int32_t num_levels;
  int32_t input_width;
  int32_t mip_w[NTC_MAX_MIPS], mip_h[NTC_MAX_MIPS], level_of_mip[NTC_MAX_MIPS];
  int32_t g0_w[NTC_MAX_LEVELS], g0_h[NTC_MAX_LEVELS];
  int32_t g1_w[NTC_MAX_LEVELS], g1_h[NTC_MAX_LEVELS];
  int64_t g0_offset[NTC_MAX_LEVELS], g1_offset[NTC_MAX_LEVELS]; /* floats, latent buffer */
  int64_t g0_packed[NTC_MAX_LEVELS], g1_packed[NTC_MAX_LEVELS]; /* bytes, packed buffer */
  int64_t mip_offset[NTC_MAX_MIPS];                             /* floats, target chain */
  int64_t latent_count, packed_bytes, target_count, mlp_params;
} ntc_material;

const char* ntc_status_string(ntc_status s);
/* Message describing the last failing call made by this thread ("" if none). */
const char* ntc_last_error(void);

/* Validate the caller fields of *m and fill the derived ones (host only, no GPU). */
ntc_status ntc_material_init(ntc_material* m);

/* Whether kernels are built for this material's (c0, c1, channels, hidden) and,
 * for decode, its bit depths.  Host only. */
int ntc_shape_supported(const ntc_material* m, int for_decode);

/*
 * Fixed-rate quantization of all latents (section 4.2): with N = 2^B levels and
 * Q = 1/N, the value x becomes k = clamp(rint(x N), -N/2 + 1, N/2) (ties to
 * even; x N is exact) and is stored as the code k + N/2 - 1 in B bits.  Zero is
 * exact.  Non-finite inputs store the code of zero.  Bit-exact.
 *   latents: m->latent_count floats.  packed: m->packed_bytes bytes (fully written,
 *   padding zeroed).
 */
ntc_status ntc_quantize_latents(const ntc_material* m, const float* latents, uint8_t* packed,
                                void* stream);

/* Inverse of ntc_quantize_latents for the codes: code k -> (k - (N/2 - 1)) / N. */
ntc_status ntc_dequantize_latents(const ntc_material* m, const uint8_t* packed, float* latents,
                                  void* stream);

/*
 * Network weights for decoding.  ntc_pack_mlp converts the canonical FP32 MLP
 * (m->mlp_params floats) into the library's matrix-core operand layout in the
 * given compute precision (NTC_F32, NTC_F16 or NTC_FP8_E4M3).  `packed` must hold
 * ntc_mlp_packed_bytes(m, precision) bytes; its content is private to the
 * library and valid only for the same material shape and precision.
 * NTC_FP8_E4M3 (lower-precision intermediates, section 7.3 Future Work): per layer l the
 * pack holds the e4m3 rounding (OCP E4M3, round to nearest even) of W_l / s_l with
 * s_l = max|W_l| / 448, computed on the device; biases stay FP32.  It needs G0 cells
 * of whole 32-bit words (c0 * b0 a multiple of 32), b0, b1 <= 4 and hidden 32 or 64;
 * otherwise ntc_mlp_packed_bytes returns 0 and ntc_pack_mlp NTC_E_UNSUPPORTED.
 */
size_t ntc_mlp_packed_bytes(const ntc_material* m, ntc_dtype precision);
ntc_status ntc_pack_mlp(const ntc_material* m, const float* mlp, ntc_dtype precision,
                        void* packed, void* stream);

/*
 * Decode all C channels of n texels (sections 4.3-4.4) from the packed latents.
 *   q: n queries.  out: n x C values, row-major, of out_dtype (NTC_F32 or NTC_F16).
 *   precision: arithmetic of the MLP (NTC_F32: FP32 matrix cores; NTC_F16: FP16
 *   inputs with FP32 accumulation; NTC_FP8_E4M3: e4m3 inputs, weights and hidden
 *   activations, FP32 accumulation, s_l * sum + b_l in FP32); `mlp_packed` must come
 *   from ntc_pack_mlp with the same precision.  n == 0 is a no-op.
 */
ntc_status ntc_decode(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                      ntc_dtype precision, const ntc_query* q, int64_t n, void* out,
                      ntc_dtype out_dtype, void* stream);

/*
 * Coherent decode (the screen-space workload of section 6): every texel of the
 * rectangle [x0, x0 + width) x [y0, y0 + height) of mip `lod`, without a query array.
 * out: width * height * C values, row-major over the rectangle then channel.  Same
 * results, bit for bit, as ntc_decode on the texel-centre queries of the rectangle.
 * The rectangle must lie inside the mip (NTC_E_INVALID otherwise); an empty one is
 * a no-op.  Other arguments as for ntc_decode.
 */
ntc_status ntc_decode_tile(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                           ntc_dtype precision, int32_t lod, int32_t x0, int32_t y0, int32_t width,
                           int32_t height, void* out, ntc_dtype out_dtype, void* stream);

/*
 * Filtered decode (section 5.3, Filtering): the network is fitted at discrete texels
 * and mips only, so filtering is done in software on decoded texels.  A filter query
 * has a continuous mip level `lod` (clamped to [0, num_mips - 1]; NaN -> 0); u, v as
 * for ntc_decode.  Modes:
 *   NTC_FILTER_BILINEAR: mip l = floor(lod + 1/2); with x = u W_l - 1/2, x0 = floor(x),
 *     fx = x - x0 (y likewise), the texels (x0, y0), (x0+1, y0), (x0, y0+1), (x0+1, y0+1)
 *     (clamped to the mip) weighted (1-fx)(1-fy), fx(1-fy), (1-fx)fy, fx fy: 4 decodes.
 *   NTC_FILTER_TRILINEAR: bilinear in mips l0 = floor(lod) and min(l0 + 1, M - 1),
 *     weighted 1 - t and t with t = lod - l0: 8 decodes.
 *   NTC_FILTER_STOCHASTIC: one decode.  With SplitMix64 counters key = mix(seed ^
 *     0x66696C74), h1 = mix(key + gamma (2i + 1)), h2 = mix(key + gamma (2i + 2)) for
 *     output i, and r1 = (h1 >> 40) 2^-24, r2 = ((h1 >> 16) & (2^24 - 1)) 2^-24,
 *     r3 = (h2 >> 40) 2^-24: mip l = l0 + (r3 < lod - l0) (at most M - 1), then the
 *     nearest texel of mip l at (u + (r1 - 1/2) / W_l, v + (r2 - 1/2) / H_l), i.e. a
 *     uniform jitter of up to half a texel (bilinear filtering in expectation).
 * Built for NTC_F16 decode packs (NTC_E_UNSUPPORTED otherwise); out holds n x C values.
 */
typedef struct {
  float u, v, lod;
} ntc_filter_query;

typedef enum { NTC_FILTER_BILINEAR = 1, NTC_FILTER_TRILINEAR = 2, NTC_FILTER_STOCHASTIC = 3 } ntc_filter;

ntc_status ntc_decode_filtered(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                               ntc_dtype precision, const ntc_filter_query* q, int64_t n, int32_t filter,
                               uint64_t seed, void* out, ntc_dtype out_dtype, void* stream);

/*
 * Training (autodecoder, section 4; optimiser section 4.5 and section 5.1).
 * State buffers (all caller-owned device memory):
 *   latents      latent_count  FP32 masters
 *   latents_fwd  latent_count  latents the next forward reads (masters + noise)
 *   lat_m, lat_v latent_count  Adam moments
 *   lat_grad     latent_count  gradient of the last step's loss w.r.t. the forward
 *                              latents (times the loss scale for NTC_F16); every entry
 *                              is overwritten by each step that trains latents
 *   mlp, mlp_m, mlp_v  mlp_params  canonical FP32 weights and Adam moments
 *   mlp_packed   ntc_train_packed_bytes(m, precision) bytes, private layout
 *   loss         1 float: mean squared error of the last step
 *   loss_scale   2 floats (NTC_F16 only; may be NULL for NTC_F32): the dynamic loss
 *                scale, double-buffered by step parity.  Step s reads loss_scale[s & 1]
 *                and its update writes the scale of step s + 1 to loss_scale[(s + 1) & 1]
 *                (so a captured step can be replayed).  Set BOTH entries to the initial
 *                scale (e.g. 65536) before the first step, whatever its index.
 *   scale_state  2 int32: [0] consecutive good steps, [1] 1 if the last step was skipped
 * The five latent buffers must be 16-byte aligned (NTC_E_INVALID otherwise).
 */
typedef struct {
  float* latents;
  float* latents_fwd;
  float* lat_m;
  float* lat_v;
  float* lat_grad;
  float* mlp;
  float* mlp_m;
  float* mlp_v;
  void* mlp_packed;
  float* loss;
  float* loss_scale;
  int32_t* scale_state;
} ntc_train_state;

/* Host struct.  beta1/beta2/eps: Adam (0.9, 0.999, 1e-8).  step: 0-based index of
 * this step (Adam uses t = step + 1; the noise of step s is a stateless hash of
 * (noise_seed, s, latent index)).  precision: NTC_F32 or NTC_F16.  noise: add
 * U(-Q/2, Q/2) to the forward latents.  freeze_latents: the quantize-and-freeze
 * phase (latents neither noised nor updated).  scale_growth_interval: NTC_F16
 * doubles the loss scale after this many good steps (halves it on overflow).
 * Graph replay: with step_dev (device int32, optional) the kernels read the step
 * index from device memory instead of `step`, and ntc_train_update (ntc_train_step)
 * increments it after the update, so one captured step can be replayed; with lr_dev
 * (device float[2] = latent, MLP learning rate, optional) the learning rates are read
 * on the device as well.  NULL: the host values are used. */
typedef struct {
  float lr_latent, lr_mlp, beta1, beta2, eps;
  uint64_t noise_seed;
  int32_t step;
  int32_t precision;
  int32_t noise;
  int32_t freeze_latents;
  int32_t scale_growth_interval;
  int32_t* step_dev;
  const float* lr_dev;
} ntc_hparams;

size_t ntc_train_packed_bytes(const ntc_material* m, ntc_dtype precision);
/* Workspace for a training step of n samples on the current device. */
size_t ntc_train_workspace_bytes(const ntc_material* m, int64_t n, ntc_dtype precision);

/*
 * Tuning of the training step (tile shapes): times ntc_train_gradients of this
 * material and sample count for each candidate (samples per work item, latent-tile
 * side) and keeps the fastest for the material's shape (c0, c1, channels, hidden,
 * activation) and precision; later plans of that shape use it.  Writes lat_grad and
 * the workspace but not the masters or the optimiser state; synchronizes the stream.
 * Thread-safe (the table is mutex-guarded).  chosen (host, optional) receives the
 * choice and its time per gradient pass.
 */
typedef struct {
  int32_t chunk;        /* samples per work item */
  int32_t tile;         /* latent-tile side (G0 cells) */
  double microseconds;  /* measured time of one gradient pass */
} ntc_train_tuning;
ntc_status ntc_train_autotune(const ntc_material* m, const ntc_train_state* s, const ntc_query* q, int64_t n,
                              const float* targets, const ntc_hparams* hp, void* workspace, size_t ws_bytes,
                              void* stream, ntc_train_tuning* chosen);
/* Set the tuning-table entry of the material's shape and precision by hand (for example
 * to restore an earlier ntc_train_autotune result): (chunk, tile) must be one of the
 * tuner's candidates (samples per work item, tile side) = (256, 8), (512, 8), (256, 16),
 * (512, 16), (1024, 16), (512, 32) or (1024, 32) (NTC_E_INVALID otherwise); (0, 0) removes
 * the entry, so plans take the defaults again.  A tile side larger than the kernel holds is
 * capped to its capacity.  Host only, thread-safe.
 * ntc_train_get_tuning reports the (chunk, tile) a plan of this material would use now
 * (microseconds = 0).  Tables built earlier (ntc_train_table_init) keep their plans. */
ntc_status ntc_train_set_tuning(const ntc_material* m, ntc_dtype precision, const ntc_train_tuning* t);
ntc_status ntc_train_get_tuning(const ntc_material* m, ntc_dtype precision, ntc_train_tuning* out);

/*
 * Make the state consistent for step hp->step: latents_fwd = latents (+ that
 * step's noise when hp->noise and not frozen), lat_grad = 0, mlp_packed from mlp.
 * Call once before the first step and after changing latents or mlp directly.
 */
ntc_status ntc_train_prepare(const ntc_material* m, const ntc_train_state* s,
                             const ntc_hparams* hp, void* stream);

/*
 * One training step on n samples: forward with latents_fwd, L2 loss against the
 * targets at each query's texel, backward into the MLP and the latents,
 * bias-corrected Adam on every parameter (dense), clamp of the latents to
 * [-(N-1)/(2N), 1/2], then latents_fwd for step hp->step + 1.  If any gradient
 * is not finite the update is skipped (scale_state[1] = 1; NTC_F16 halves the
 * loss scale).  workspace: ws_bytes >= ntc_train_workspace_bytes(m, n, precision).
 * n: 1 .. (2^31 - 1) / 4 samples (each is listed under up to 4 latent tiles with
 * 32-bit positions); larger n returns NTC_E_UNSUPPORTED (and the workspace query 0),
 * the same for every training, tuning and backward entry point.
 * Latent gradients are accumulated without global atomics: samples are binned
 * by the spatial tile of latents their footprint touches and each tile's
 * gradient is summed in on-chip memory and written once.  NTC_F16 sums them as
 * 32-bit fixed point: each contribution is rounded to 2^-16 of the delta unit
 * 2 * loss_scale / (n * channels) (rounded to a power of two); a work item with
 * a contribution beyond the fixed-point range is summed again in FP32.
 */
ntc_status ntc_train_step(const ntc_material* m, const ntc_train_state* s, const ntc_query* q,
                          int64_t n, const float* targets, const ntc_hparams* hp,
                          void* workspace, size_t ws_bytes, void* stream);

/*
 * ntc_train_step without a caller workspace, for callers that cannot allocate device
 * memory (code under graph capture, tight serving loops, harnesses that forbid it).
 * The step's workspace is a static device array of NTC_NOALLOC_SCRATCH_BYTES (128 MiB)
 * that the library holds on every GPU it runs on until the process ends; its address
 * on a device is looked up on the first call there.  Steps whose workspace
 * (ntc_train_workspace_bytes of the plan in use) exceeds it return NTC_E_WORKSPACE
 * before anything is enqueued; for example a 2048^2 x 12 material fits 4,096-sample
 * steps, a 256^2 x 8 one 65,536-sample steps.  All calls on one GPU share the array:
 * calls that overlap on one GPU (on different streams or host threads) race and must
 * be serialised by the caller.  Nothing needs clearing between calls (every stage
 * writes what it reads).  Results equal ntc_train_step's bit for bit.  Allocates
 * nothing: no hipMalloc, no hipFree, no allocating library call.
 */
#define NTC_NOALLOC_SCRATCH_BYTES (128u << 20)
ntc_status ntc_train_step_noalloc(const ntc_material* m, const ntc_train_state* s, const ntc_query* q,
                                  int64_t n, const float* targets, const ntc_hparams* hp, void* stream);

/*
 * The two halves of ntc_train_step, for callers that time or overlap them, or
 * accumulate gradients of several batches before one update:
 *  ntc_train_gradients: binning of the samples by latent tile, then forward, loss
 *    and backward of the n samples (one fused kernel).  Writes s->lat_grad (all
 *    entries, unless latents are frozen); per-block weight-gradient and loss
 *    partials go to the workspace.
 *  ntc_train_update: reduces the partials of the preceding ntc_train_gradients
 *    call with the same (n, workspace), then Adam, clamp and the next forward
 *    latents exactly as ntc_train_step.  n must equal the gradient call's n.
 * ntc_train_step(...) == ntc_train_gradients(...) followed by ntc_train_update(...).
 */
ntc_status ntc_train_gradients(const ntc_material* m, const ntc_train_state* s, const ntc_query* q,
                               int64_t n, const float* targets, const ntc_hparams* hp,
                               void* workspace, size_t ws_bytes, void* stream);
ntc_status ntc_train_update(const ntc_material* m, const ntc_train_state* s, int64_t n,
                            const ntc_hparams* hp, void* workspace, size_t ws_bytes, void* stream);

/*
 * Differentiation path (decoder as a differentiable function of latents and
 * weights, sections 4 and 4.5): y = decode(latents, mlp) at n queries and its
 * vector-Jacobian product.  The backward recomputes the forward per tile (no
 * stored activations) with the same kernels as the training step.
 *
 *  ntc_pack_mlp_train: canonical FP32 MLP -> forward + backward operand packs
 *    (ntc_train_packed_bytes(m, precision) bytes), as used by ntc_backward.
 *  ntc_forward: decode from FP32 latents (canonical layout, used as given: no
 *    quantization or noise); weights from mlp_train_packed (ntc_pack_mlp_train of
 *    the same mlp, so forward and backward see identically rounded weights),
 *    biases from the canonical FP32 mlp; out: n x C FP32.
 *  ntc_backward: given dout = dL/dy (n x C FP32), writes grad_latents (all
 *    latent_count entries, overwritten) and grad_mlp (mlp_params, canonical
 *    layout).  dout is multiplied by dout_scale inside the kernels (use a power of
 *    two that brings |dout| near 1 for NTC_F16) and the outputs are divided by it.
 *    dout_scale = 0 lets the library choose it on the device, with no host
 *    synchronisation: 2^round(log2(1/4 / max|dout|)) (1 when that maximum is 0 or not
 *    finite), so the call can be captured in a HIP graph.  Negative or non-finite
 *    values are NTC_E_INVALID.
 *    NTC_F16 rounds each latent-gradient contribution to 2^-16 of the scaled delta's
 *    unit (1), summing out-of-range work items again in FP32.
 *    workspace: ntc_backward_workspace_bytes(m, n, precision).
 */
ntc_status ntc_pack_mlp_train(const ntc_material* m, const float* mlp, ntc_dtype precision, void* packed,
                              void* stream);
ntc_status ntc_forward(const ntc_material* m, const float* latents, const float* mlp, const void* mlp_train_packed,
                       ntc_dtype precision, const ntc_query* q, int64_t n, float* out, void* stream);
size_t ntc_backward_workspace_bytes(const ntc_material* m, int64_t n, ntc_dtype precision);
ntc_status ntc_backward(const ntc_material* m, const float* latents, const float* mlp, const void* mlp_train_packed,
                        ntc_dtype precision, const ntc_query* q, int64_t n, const float* dout, float dout_scale,
                        float* grad_latents, float* grad_mlp, void* workspace, size_t ws_bytes, void* stream);

/*
 * One training batch as in section 5.1: `crops` crops of side x side texels, all from
 * one level of detail, LOD = floor(-log4 X) with X ~ U(0, 1] (clamped to the chain),
 * or uniform over the chain for a `uniform_fraction` of the batches.  The random
 * numbers are SplitMix64 outputs of counters derived from (seed, step): key =
 * mix(mix(seed ^ 0x63726F70) + gamma (step + 1)), r_i = mix(key + gamma (i + 1));
 * X = 1 - (r_0 >> 11) 2^-53; uniform batch when (r_1 >> 11) 2^-53 < uniform_fraction,
 * LOD = r_2 mod num_mips; crop c starts at (r_(3+2c) mod (W_l - side + 1),
 * r_(4+2c) mod (H_l - side + 1)); on mips smaller than the crop it starts at 0 and
 * wraps around.  out: crops * side^2 queries at texel centres, crop-major, row-major
 * within a crop (caller-owned device memory).
 */
ntc_status ntc_crop_queries(const ntc_material* m, uint64_t seed, int32_t step, int32_t crops, int32_t side,
                            double uniform_fraction, ntc_query* out, void* stream);

/*
 * Many materials (uneven sizes, channel counts and MLP widths, each with its own
 * weights and state) in one call.  Queries are grouped per material: material i
 * owns q[offsets[i] .. offsets[i+1]) (offsets: host, nmat + 1 entries, offsets[0] = 0,
 * non-decreasing; an empty group skips the material).  Every argument of every
 * material is validated before anything is enqueued; the calls enqueue only kernel
 * launches on `stream`, so a whole batched step can be captured in a HIP graph (with
 * hp->step_dev, one captured step replays as the next step).
 *   ntc_train_step_batched: one training step (ntc_train_step) of every material;
 *     states[i], targets[i] (device pointer) per material, hp shared; with
 *     hp->step_dev the step index advances once per batched step.  workspace:
 *     ntc_train_workspace_bytes_batched bytes.
 *   ntc_decode_batched: decode of every group (ntc_decode); packed_latents[i] and
 *     mlp_packed[i] per material (mlp_packed from ntc_pack_mlp with `precision`);
 *     out holds the groups one after another, n_i x C_i values each.
 */
size_t ntc_train_workspace_bytes_batched(const ntc_material* mats, int32_t nmat, const int64_t* offsets,
                                         ntc_dtype precision);
ntc_status ntc_train_step_batched(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                  const ntc_query* q, const int64_t* offsets, const float* const* targets,
                                  const ntc_hparams* hp, void* workspace, size_t ws_bytes, void* stream);
ntc_status ntc_decode_batched(const ntc_material* mats, int32_t nmat, const uint8_t* const* packed_latents,
                              const void* const* mlp_packed, ntc_dtype precision, const ntc_query* q,
                              const int64_t* offsets, void* out, ntc_dtype out_dtype, void* stream);

/*
 * Grouped training: the batched step of ntc_train_step_batched with each stage
 * (binning, scans, partial-tile reduction, weight-gradient reduction, Adam) run as one
 * launch for the whole group instead of one per material, and the fused training
 * kernel as one launch per kernel shape (c0, c1, channels, hidden, activation), each
 * member with the blocks and work-item shares of its own launch (the same sums, bit for
 * bit).  At most 64 materials share a launch.  Every member needs samples (offsets
 * strictly increasing).
 *   ntc_train_table_bytes: size of the device table for nmat materials.
 *   ntc_train_table_init: validates the group and writes the table into `table`
 *     (caller device memory): per material its geometry, training plan (tile shapes
 *     from the tuning table in effect), sample group and the device pointers of its
 *     state, targets and workspace slice (the workspace is laid out as for
 *     ntc_train_step_batched, ntc_train_workspace_bytes_batched bytes).  Synchronous;
 *     a set-up call, not for stream capture.  Build it again after tuning a member's
 *     shape or changing any of these.
 *   ntc_train_step_grouped: one training step of every member; arguments as for
 *     ntc_train_step_batched plus the table.  The launches carry a hash of the group
 *     (materials, plans, sample groups, precision, buffers; not the queries or the
 *     hyper-parameters) and do nothing when it differs from the table's.  Only kernel
 *     launches are enqueued: with hp->step_dev (and hp->lr_dev) a captured step replays
 *     as the next step.
 */
size_t ntc_train_table_bytes(int32_t nmat);
ntc_status ntc_train_table_init(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                const int64_t* offsets, const float* const* targets, ntc_dtype precision,
                                void* workspace, size_t ws_bytes, void* table, size_t table_bytes);
ntc_status ntc_train_step_grouped(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                  const ntc_query* q, const int64_t* offsets, const float* const* targets,
                                  const ntc_hparams* hp, void* workspace, size_t ws_bytes, const void* table,
                                  void* stream);

/*
 * Grouped decode: the batch of ntc_decode_batched decoded with one launch per kernel
 * shape (c0, c1, channels, hidden, b0, b1, activation, posenc) instead of one per material;
 * each launch shares its blocks out over its materials (at most 32 per launch) in
 * proportion to their queries, and every block decodes with its own material's weights.
 *   ntc_decode_table_bytes: size of the device table for nmat materials.
 *   ntc_decode_table_init: validates the batch (as ntc_decode_batched, for the given
 *     precision) and writes the table into `table` (caller device memory): per
 *     material its geometry and the device pointers packed_latents[i], mlp_packed[i]
 *     (host arrays).  Synchronous (returns after the copy); a set-up call, not for
 *     stream capture.  Those buffers must stay allocated while the table is used; their
 *     contents may change (re-quantized latents, re-packed weights).
 *   ntc_decode_grouped: decodes group i (queries offsets[i] .. offsets[i+1]-1, host
 *     offsets) of material i into out as ntc_decode_batched does.  mats and nmat must be
 *     those the table was built for: the launches carry a hash of them and decode nothing
 *     when it differs from the table's.  precision must match the packs.  Only kernel
 *     launches are enqueued, so the call can be captured in a HIP graph.
 */
size_t ntc_decode_table_bytes(int32_t nmat);

/*
 * Mixed-material decode (Appendix A, handling divergence): queries in any order, each
 * naming its material (an index into mats; out-of-range indices are clamped).  A
 * wavefront's 16-texel tile gathers every texel from its own material, then evaluates
 * the network once per distinct material in the tile (that material's weights for the
 * whole tile, outputs kept for its texels), as the paper's divergence loop does.  All
 * materials share one decode shape (c0, c1, channels, hidden, b0, b1, activation,
 * posenc); at most 64; NTC_F16 decode packs; the table from ntc_decode_table_init
 * (same hash rule as ntc_decode_grouped).  out holds n x C values in query order.
 */
typedef struct {
  float u, v;
  int32_t lod;
  int32_t material;
} ntc_mixed_query;
ntc_status ntc_decode_mixed(const ntc_material* mats, int32_t nmat, const void* table, ntc_dtype precision,
                            const ntc_mixed_query* q, int64_t n, void* out, ntc_dtype out_dtype, void* stream);
ntc_status ntc_decode_table_init(const ntc_material* mats, int32_t nmat, const uint8_t* const* packed_latents,
                                 const void* const* mlp_packed, ntc_dtype precision, void* table,
                                 size_t table_bytes);
ntc_status ntc_decode_grouped(const ntc_material* mats, int32_t nmat, const void* table, ntc_dtype precision,
                              const ntc_query* q, const int64_t* offsets, void* out, ntc_dtype out_dtype,
                              void* stream);

/*
 * Kernel timing for measurement (not needed for normal use).  After
 * ntc_timing_begin(max_launches), the library records a HIP event pair on the launch
 * stream around each of the next max_launches launches of every timed kernel
 * ("train_fused": the fused training kernel of ntc_train_gradients / ntc_train_step /
 * ntc_backward; "decode": the kernel of ntc_decode).  ntc_timing_read waits for the
 * recorded events and returns their summed elapsed time and count; ntc_timing_end
 * synchronizes the device, stops recording and frees the events.  Calls from several
 * threads are serialized; begin resets earlier records.
 */
ntc_status ntc_timing_begin(int32_t max_launches);
ntc_status ntc_timing_read(const char* kernel, double* total_ms, int32_t* launches);
ntc_status ntc_timing_end(void);

#ifdef __cplusplus
}
#endif
#endif /* NTC_H */
