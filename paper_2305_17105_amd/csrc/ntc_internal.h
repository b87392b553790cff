// Host-side internals shared by the C ABI layer and the kernel launchers.
#pragma once
#include <hip/hip_runtime.h>

#include <string>

#include "../../include/ntc.h"
#include "ntc_device.h"

namespace ntc {

// Optional launch timing (ntc_timing_begin / _read / _end): a slot >= 0 when a start
// event was recorded, to be closed by timing_after on the same stream.
enum TimedKernel { TK_TRAIN_FUSED = 0, TK_DECODE = 1, TK_COUNT = 2 };
int timing_before(TimedKernel k, hipStream_t s);
void timing_after(TimedKernel k, hipStream_t s, int slot);

// Thread-local error message for ntc_last_error().
void set_error(const std::string& msg);

// ntc_material (validated) -> kernel view.
DevMat dev_mat(const ntc_material& m);
PeTable pe_table(const ntc_material& m);

// Number of CUs of the current device (cached per device).
int device_cus();

// Resident blocks per CU of a kernel at the given block size and dynamic LDS (at least
// 1).  Launchers keep the result in a function-local static initialised by one call,
// which C++ guarantees to run once even when several threads launch for the first time.
template <typename K>
int blocks_per_cu(K kern, int threads, size_t lds) {
  int v = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, threads, lds) != hipSuccess || v < 1) v = 1;
  return v;
}

// Launchers: return hipSuccess or the launch error.  Shapes are validated by the caller.
hipError_t launch_quantize(const ntc_material& m, const float* lat, uint8_t* packed, hipStream_t s);
hipError_t launch_dequantize(const ntc_material& m, const uint8_t* packed, float* lat, hipStream_t s);
// Scatter canonical FP32 weights into operand packs (forward only, or forward + backward).
hipError_t launch_pack_mlp(const ntc_material& m, const float* mlp, bool f16, bool with_backward,
                           void* packed, hipStream_t s);
// FP8-e4m3 decode pack (weights, per-layer scales, FP32 biases) and its weight-part size.
size_t fp8_pack_weight_bytes(const ntc_material& m);
hipError_t launch_pack_mlp_fp8(const ntc_material& m, const float* mlp, void* packed, hipStream_t s);
// Decode launchers: rect == nullptr decodes the n queries of q; otherwise the n texels
// of the rectangle, row-major (q unused).
hipError_t launch_decode_fp8(const ntc_material& m, const uint8_t* packed, const void* wpack, const ntc_query* q,
                             long long n, const TexelRect* rect, void* out, bool out_f16, hipStream_t s);
hipError_t launch_decode(const ntc_material& m, const uint8_t* packed, const void* wpack, bool f16,
                         const ntc_query* q, long long n, const TexelRect* rect, void* out, bool out_f16,
                         hipStream_t s);

// Mixed-material decode (FP16 decode packs of one shape, at most kMixedMax materials).
hipError_t launch_decode_mixed(const ntc_material* mats, int nmat, const void* table, const ntc_mixed_query* q,
                               long long n, void* out, bool out_f16, hipStream_t s);
// Filtered decode (FP16 decode packs): filter 1 bilinear, 2 trilinear, 3 stochastic.
hipError_t launch_decode_filtered(const ntc_material& m, const uint8_t* packed, const void* wpack,
                                  const ntc_filter_query* q, long long n, int filter, uint64_t seed, void* out,
                                  bool out_f16, hipStream_t s);

// Grouped decode: table entries, the hash that ties a table to its materials, and the
// launches (one per kernel shape, at most kGroupSegs materials each).
void fill_group_entry(const ntc_material& m, const void* packed, const void* wpack, GroupEntry& e);
unsigned long long group_hash(const ntc_material* mats, int nmat);
hipError_t launch_decode_grouped(const ntc_material* mats, int nmat, const void* table, int precision,
                                 const ntc_query* q, const int64_t* offsets, void* out, bool out_f16,
                                 hipStream_t s);

// Tunable plan parameters: samples per work item and largest latent-tile side
// (0: the kernel's capacity).
struct TrainTune {
  int chunk, tile;
};
void set_train_tune(const ntc_material& m, bool f16, const TrainTune& t);
void clear_train_tune(const ntc_material& m, bool f16);
TrainTune get_train_tune(const ntc_material& m, bool f16);
const TrainTune* train_tune_candidates(int* count);

// Launch plan of a training step: tile geometry, grids and workspace layout (bytes).
struct TrainPlan {
  TileGeom tg;
  TrainTune tune;  // the parameters in effect
  int nbins, ntiles, region_max, nbb, per_bin_block, grid;
  long long max_items;
  bool supported_bins;
  size_t off_counts, off_offsets, off_total, off_base, off_tstart, off_ttotal, off_ibase, off_itile, off_misc;
  size_t off_list;
  size_t off_part_lat;
  size_t off_part_dw, off_part_loss, off_grad, off_dscale, total;
};
// tune == nullptr: the tuning table's entry for the material's shape (or the defaults)
TrainPlan train_plan(const ntc_material& m, bool f16, long long n, const TrainTune* tune = nullptr);

struct TrainLaunch {
  const float* lat_fwd;
  const void* wpack;
  const float* mlp;
  const ntc_query* q;
  long long n;
  const float* targets;
  float* lat_grad;          // dense latent gradient (overwritten)
  void* workspace;
  const float* loss_scale;  // device, 2 entries, or nullptr (scale 1)
  int scale_slot;
  const int* step_dev;      // device step index (graph replay) or nullptr: scale_slot
  int32_t* overflow_flag;   // reset by the fused kernel
  bool scatter_latents;     // false: latents frozen, samples processed in query order
  const float* dout;        // external output gradient, or nullptr (L2 loss against targets)
  float dout_scale;
  float out_scale;          // multiplies the latent gradient written to lat_grad
  const float* dscale = nullptr;  // device (dout_scale, out_scale) replacing the two above
  const unsigned long long* table_hash = nullptr;  // grouped step: the table's hash (kernel no-ops on mismatch)
  unsigned long long hash = 0;
};
hipError_t launch_train_gradients(const ntc_material& m, bool f16, const TrainPlan& p, const TrainLaunch& a,
                                  hipStream_t s);
hipError_t launch_train_reduce(const ntc_material& m, const TrainPlan& p, void* workspace, float* loss_out,
                               float loss_norm, int32_t* overflow_flag, hipStream_t s, float* grad_out = nullptr,
                               float out_scale = 1.f, const float* dscale = nullptr);
// Device-chosen output-gradient scale of the differentiation path: writes (scale, 1 /
// scale) to work[0..1], using work[2 ..] (kScaleBlocks floats) for block maxima.
hipError_t launch_dout_scale(const float* dout, long long count, float* work, hipStream_t s);
hipError_t launch_forward(const ntc_material& m, const float* latents, const float* mlp, const void* wpack, bool f16,
                          const ntc_query* q, long long n, float* out, hipStream_t s);

struct AdamLaunch {
  float* latents;
  float* latents_fwd;
  float* lat_m;
  float* lat_v;
  float* lat_grad;
  float* mlp;
  float* mlp_m;
  float* mlp_v;
  const float* mlp_grad;
  void* wpack;
  float* loss_scale;   // 2 entries or nullptr
  int32_t* scale_state;
  float lr_lat, lr_mlp, beta1, beta2, eps, bc1, bc2;
  uint64_t next_key;   // noise key of step + 1
  int step, noise, freeze, growth, f16;
  int* step_dev;        // device step index or nullptr (then step, bc1, bc2, next_key)
  const float* lr_dev;  // device (lr_lat, lr_mlp) or nullptr
  uint64_t seed;        // noise seed (device-step mode derives the key on the device)
  bool advance;         // device-step mode: advance the step index after the update
  float* loss_out = nullptr;  // grouped step: the member's loss
};
hipError_t launch_crop_queries(const ntc_material& m, uint64_t seed, int step, int crops, int side, double fraction,
                               ntc_query* out, hipStream_t s);
hipError_t launch_adam(const ntc_material& m, const AdamLaunch& a, hipStream_t s);
hipError_t launch_step_advance(int* step_dev, hipStream_t s);

// Grouped training step (one launch per stage for a group of materials; the fused
// kernel per material): device-table size, the hash tying a table to its group, the
// table's host image, and the step's launches.  fused[i] / adam[i]: the member's
// buffers; hot: the step-dependent Adam scalars shared by the group.
size_t train_table_bytes(int nmat);
unsigned long long train_group_hash(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16,
                                    const TrainLaunch* fused, const AdamLaunch* adam);
void fill_train_table(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16, const TrainLaunch* fused,
                      const AdamLaunch* adam, unsigned long long hash, void* host_table);
hipError_t launch_train_grouped(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16,
                                const void* table, unsigned long long hash, const ntc_query* q, bool scatter,
                                const TrainLaunch* fused, const AdamLaunch& hot, hipStream_t s);
hipError_t launch_prepare(const ntc_material& m, const float* latents, float* latents_fwd, float* lat_grad,
                          uint64_t key, int noise, hipStream_t s);

}  // namespace ntc
