// C ABI of the library: argument validation, geometry, workspace layout and the
// launch sequence of each entry point.  No entry point allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <vector>
#include <mutex>
#include <string>

#include "ntc_internal.h"

namespace ntc {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

int device_cus() {
  static std::mutex mu;
  static int cache[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  std::lock_guard<std::mutex> lock(mu);
  if (cache[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus <= 0) cus = 256;
    cache[dev] = cus;
  }
  return cache[dev];
}

DevMat dev_mat(const ntc_material& m) {
  DevMat d;
  std::memset(&d, 0, sizeof d);
  d.W = m.width; d.H = m.height; d.C = m.channels; d.M = m.num_mips;
  d.C0 = m.c0; d.C1 = m.c1; d.B0 = m.b0; d.B1 = m.b1; d.shift = m.grid_shift;
  d.Hd = m.hidden; d.act = m.activation; d.pe = m.posenc; d.lod_in = m.lod_input; d.J = m.num_levels; d.K = m.input_width;
  for (int l = 0; l < kMaxMips; ++l) {
    d.mip_w[l] = m.mip_w[l]; d.mip_h[l] = m.mip_h[l]; d.level_of_mip[l] = m.level_of_mip[l];
    d.mip_off[l] = m.mip_offset[l];
  }
  for (int j = 0; j < kMaxLevels; ++j) {
    d.g0_w[j] = m.g0_w[j]; d.g0_h[j] = m.g0_h[j]; d.g1_w[j] = m.g1_w[j]; d.g1_h[j] = m.g1_h[j];
    d.g0_off[j] = m.g0_offset[j]; d.g1_off[j] = m.g1_offset[j];
    d.g0_pk[j] = m.g0_packed[j]; d.g1_pk[j] = m.g1_packed[j];
    if (j < m.num_levels) {
      d.g0_pk_end[j] = (m.g1_packed[j]) / 4 - 1;
      const long long next = (j + 1 < m.num_levels) ? m.g0_packed[j + 1] : m.packed_bytes;
      d.g1_pk_end[j] = next / 4 - 1;
    }
  }
  d.latent_count = m.latent_count;
  return d;
}

PeTable pe_table(const ntc_material& m) {
  PeTable p;
  const double two_pi = 6.283185307179586476925286766559;
  auto frac = [](double x) { return x - std::floor(x); };
  for (int i = 0; i < 8; ++i) {
    const double t = (i + 0.5) / 8.0;
    for (int f = 0; f < 3; ++f) {
      const double x = (double)(1 << f) * t;
      if (m.posenc == NTC_PE_TRIANGLE) {
        p.v[i][2 * f] = (float)(4.0 * std::fabs(frac(x - 0.25) - 0.5) - 1.0);
        p.v[i][2 * f + 1] = (float)(4.0 * std::fabs(frac(x) - 0.5) - 1.0);
      } else {
        p.v[i][2 * f] = (float)std::sin(two_pi * x);
        p.v[i][2 * f + 1] = (float)std::cos(two_pi * x);
      }
    }
  }
  return p;
}

bool decode_shape_supported(int c0, int c1, int c, int hd, int b0, int b1);
bool train_shape_supported(int c0, int c1, int c, int hd);

}  // namespace ntc

using namespace ntc;

static long long grid_bytes(long long cells, int ch, int bits) {
  const long long raw = (cells * ch * bits + 7) / 8;
  return (raw + 15) / 16 * 16;
}

static bool pow2(int v) { return v > 0 && (v & (v - 1)) == 0; }

static ntc_status fail(ntc_status s, const std::string& msg) {
  set_error(msg);
  return s;
}

static ntc_status hip_status(hipError_t e, const char* where) {
  if (e == hipSuccess) return NTC_OK;
  return fail(NTC_E_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

// Re-check a descriptor the caller passes back (it must come from ntc_material_init).
static ntc_status check_material(const ntc_material* m) {
  if (!m) return fail(NTC_E_INVALID, "material is NULL");
  ntc_material copy = *m;
  if (ntc_material_init(&copy) != NTC_OK) return NTC_E_INVALID;
  if (std::memcmp(&copy, m, sizeof copy) != 0)
    return fail(NTC_E_INVALID, "material descriptor was modified after ntc_material_init");
  return NTC_OK;
}

// Training and backward calls bin each sample under at most 4 latent tiles with 32-bit
// list positions and sample indices: n is limited to INT32_MAX / 4.
static const int64_t kMaxTrainSamples = 0x7fffffffLL / 4;

static long long mlp_params(int K, int Hd, int C) {
  return (long long)K * Hd + Hd + (long long)Hd * Hd + Hd + (long long)Hd * C + C;
}

extern "C" {

const char* ntc_status_string(ntc_status s) {
  switch (s) {
    case NTC_OK: return "ok";
    case NTC_E_INVALID: return "invalid argument";
    case NTC_E_UNSUPPORTED: return "unsupported shape";
    case NTC_E_WORKSPACE: return "workspace too small";
    case NTC_E_HIP: return "HIP runtime error";
  }
  return "unknown status";
}

const char* ntc_last_error(void) { return g_err.c_str(); }

ntc_status ntc_material_init(ntc_material* m) {
  if (!m) return fail(NTC_E_INVALID, "material is NULL");
  if (!pow2(m->width) || !pow2(m->height) || m->width > 32768 || m->height > 32768)
    return fail(NTC_E_INVALID, "width and height must be powers of two <= 32768");
  if (m->channels < 1 || m->channels > 16) return fail(NTC_E_INVALID, "channels must be in 1..16");
  if (m->c0 < 1 || m->c0 > 16 || m->c1 < 1 || m->c1 > 32)
    return fail(NTC_E_INVALID, "c0 must be in 1..16 and c1 in 1..32");
  auto okbits = [](int b) { return b == 1 || b == 2 || b == 4 || b == 8; };
  if (!okbits(m->b0) || !okbits(m->b1)) return fail(NTC_E_INVALID, "b0, b1 must be 1, 2, 4 or 8");
  if (m->grid_shift < 0 || m->grid_shift > 8) return fail(NTC_E_INVALID, "grid_shift must be in 0..8");
  if (m->hidden != 16 && m->hidden != 32 && m->hidden != 48 && m->hidden != 64)
    return fail(NTC_E_INVALID, "hidden must be 16, 32, 48 or 64");
  if (m->activation != NTC_ACT_RELU && m->activation != NTC_ACT_HARDGELU)
    return fail(NTC_E_INVALID, "unknown activation");
  if (m->posenc != NTC_PE_SINCOS && m->posenc != NTC_PE_TRIANGLE) return fail(NTC_E_INVALID, "unknown posenc");
  if (m->lod_input != 0 && m->lod_input != 1) return fail(NTC_E_INVALID, "lod_input must be 0 or 1");
  const int W = m->width, H = m->height, sh = m->grid_shift;
  int full = 1;
  while ((std::max(W, H) >> (full - 1)) > 1) ++full;
  const int M = m->num_mips == 0 ? full : m->num_mips;
  if (M < 1 || M > full || M > NTC_MAX_MIPS) return fail(NTC_E_INVALID, "num_mips out of range");
  int jmax = 0;
  while (jmax < 30 && (W >> (sh + 2 * jmax + 1)) >= 1 && (H >> (sh + 2 * jmax + 1)) >= 1) ++jmax;
  if (jmax == 0) return fail(NTC_E_INVALID, "texture too small for grid_shift (G1 would be empty)");
  const int raw_last = std::max(0, (M - 1 - sh) >= 0 ? (M - 1 - sh) / 2 : 0);
  const int J = std::min(jmax, raw_last + 1);
  if (J > NTC_MAX_LEVELS) return fail(NTC_E_INVALID, "too many feature levels");
  m->num_mips = M;
  m->num_levels = J;
  m->input_width = 4 * m->c0 + m->c1 + 12 + m->lod_input;
  std::memset(m->mip_w, 0, sizeof m->mip_w);
  std::memset(m->mip_h, 0, sizeof m->mip_h);
  std::memset(m->level_of_mip, 0, sizeof m->level_of_mip);
  std::memset(m->mip_offset, 0, sizeof m->mip_offset);
  long long toff = 0;
  for (int l = 0; l < M; ++l) {
    m->mip_w[l] = std::max(1, W >> l);
    m->mip_h[l] = std::max(1, H >> l);
    const int d = l - sh;
    const int lv = d < 0 ? 0 : d / 2;
    m->level_of_mip[l] = std::min(lv, J - 1);
    m->mip_offset[l] = toff;
    toff += (long long)m->mip_w[l] * m->mip_h[l] * m->channels;
  }
  m->target_count = toff;
  std::memset(m->g0_w, 0, sizeof m->g0_w);
  std::memset(m->g0_h, 0, sizeof m->g0_h);
  std::memset(m->g1_w, 0, sizeof m->g1_w);
  std::memset(m->g1_h, 0, sizeof m->g1_h);
  std::memset(m->g0_offset, 0, sizeof m->g0_offset);
  std::memset(m->g1_offset, 0, sizeof m->g1_offset);
  std::memset(m->g0_packed, 0, sizeof m->g0_packed);
  std::memset(m->g1_packed, 0, sizeof m->g1_packed);
  long long off = 0, pk = 0;
  for (int j = 0; j < J; ++j) {
    const int w0 = W >> (sh + 2 * j), h0 = H >> (sh + 2 * j);
    m->g0_w[j] = w0; m->g0_h[j] = h0; m->g1_w[j] = w0 / 2; m->g1_h[j] = h0 / 2;
    m->g0_offset[j] = off;
    m->g0_packed[j] = pk;
    off += (long long)w0 * h0 * m->c0;
    pk += grid_bytes((long long)w0 * h0, m->c0, m->b0);
    m->g1_offset[j] = off;
    m->g1_packed[j] = pk;
    off += (long long)(w0 / 2) * (h0 / 2) * m->c1;
    pk += grid_bytes((long long)(w0 / 2) * (h0 / 2), m->c1, m->b1);
  }
  if (off >= (1ll << 31)) return fail(NTC_E_INVALID, "latent count exceeds 2^31");
  m->latent_count = off;
  m->packed_bytes = pk;
  m->mlp_params = mlp_params(m->input_width, m->hidden, m->channels);
  return NTC_OK;
}

int ntc_shape_supported(const ntc_material* m, int for_decode) {
  if (!m) return 0;
  if (for_decode) return decode_shape_supported(m->c0, m->c1, m->channels, m->hidden, m->b0, m->b1) ? 1 : 0;
  return train_shape_supported(m->c0, m->c1, m->channels, m->hidden) ? 1 : 0;
}

ntc_status ntc_quantize_latents(const ntc_material* m, const float* latents, uint8_t* packed, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (!latents || !packed) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_quantize(*m, latents, packed, (hipStream_t)stream), "ntc_quantize_latents");
}

ntc_status ntc_dequantize_latents(const ntc_material* m, const uint8_t* packed, float* latents, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (!latents || !packed) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_dequantize(*m, packed, latents, (hipStream_t)stream), "ntc_dequantize_latents");
}

static size_t round16(size_t b) { return (b + 15) / 16 * 16; }

static bool fp8_supported(const ntc_material* m) {
  return fp8_layout(m->c0, m->c1, m->b0, m->b1, m->hidden) &&
         decode_shape_supported(m->c0, m->c1, m->channels, m->hidden, m->b0, m->b1);
}

size_t ntc_mlp_packed_bytes(const ntc_material* m, ntc_dtype precision) {
  if (m && precision == NTC_FP8_E4M3)
    return fp8_supported(m) ? fp8_pack_weight_bytes(*m) + 16 + round16((size_t)(2 * m->hidden + m->channels) * 4) : 0;
  if (!m || (precision != NTC_F32 && precision != NTC_F16)) return 0;
  const bool f16 = precision == NTC_F16;
  const PackGeom pg = pack_geom_decode(m->c0, m->c1, m->b0, m->b1, m->hidden, f16);
  const size_t w = round16((size_t)pg.fwd_end * (f16 ? 2 : 4));
  return w + round16((size_t)(2 * m->hidden + m->channels) * 4);
}

size_t ntc_train_packed_bytes(const ntc_material* m, ntc_dtype precision) {
  if (!m || (precision != NTC_F32 && precision != NTC_F16)) return 0;
  const bool f16 = precision == NTC_F16;
  const PackGeom pg = pack_geom(m->c0, m->c1, m->hidden, f16);
  return round16((size_t)pg.train_end * (f16 ? 2 : 4));
}

ntc_status ntc_pack_mlp(const ntc_material* m, const float* mlp, ntc_dtype precision, void* packed, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision == NTC_FP8_E4M3) {
    if (!fp8_supported(m))
      return fail(NTC_E_UNSUPPORTED, "FP8 decode needs whole-dword G0 cells, b0, b1 <= 4 and a decode shape");
    if (!mlp || !packed) return fail(NTC_E_INVALID, "NULL buffer");
    return hip_status(launch_pack_mlp_fp8(*m, mlp, packed, (hipStream_t)stream), "ntc_pack_mlp");
  }
  if (precision != NTC_F32 && precision != NTC_F16)
    return fail(NTC_E_UNSUPPORTED, "pack precision must be F32, F16 or FP8_E4M3");
  if (!mlp || !packed) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_pack_mlp(*m, mlp, precision == NTC_F16, false, packed, (hipStream_t)stream), "ntc_pack_mlp");
}

static ntc_status check_decode(const ntc_material* m, ntc_dtype precision, ntc_dtype out_dtype) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16 && precision != NTC_FP8_E4M3)
    return fail(NTC_E_UNSUPPORTED, "decode precision must be F32, F16 or FP8_E4M3");
  if (out_dtype != NTC_F32 && out_dtype != NTC_F16) return fail(NTC_E_UNSUPPORTED, "output dtype must be F32 or F16");
  if (!decode_shape_supported(m->c0, m->c1, m->channels, m->hidden, m->b0, m->b1))
    return fail(NTC_E_UNSUPPORTED, "no decode kernel for this (c0, c1, channels, hidden, b0, b1)");
  if (precision == NTC_FP8_E4M3 && !fp8_supported(m))
    return fail(NTC_E_UNSUPPORTED, "FP8 decode needs whole-dword G0 cells and b0, b1 <= 4");
  if (m->packed_bytes >= ((int64_t)1 << 32)) return fail(NTC_E_UNSUPPORTED, "packed latents of 4 GiB or more");
  return NTC_OK;
}

static ntc_status run_decode(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                             ntc_dtype precision, const ntc_query* q, int64_t n, const TexelRect* rect, void* out,
                             ntc_dtype out_dtype, void* stream, const char* where) {
  if (precision == NTC_FP8_E4M3)
    return hip_status(launch_decode_fp8(*m, packed_latents, mlp_packed, q, n, rect, out, out_dtype == NTC_F16,
                                        (hipStream_t)stream), where);
  return hip_status(launch_decode(*m, packed_latents, mlp_packed, precision == NTC_F16, q, n, rect, out,
                                  out_dtype == NTC_F16, (hipStream_t)stream), where);
}

ntc_status ntc_decode(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                      ntc_dtype precision, const ntc_query* q, int64_t n, void* out, ntc_dtype out_dtype,
                      void* stream) {
  ntc_status st = check_decode(m, precision, out_dtype);
  if (st != NTC_OK) return st;
  if (n < 0) return fail(NTC_E_INVALID, "n < 0");
  if (n == 0) return NTC_OK;
  if (!packed_latents || !mlp_packed || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  return run_decode(m, packed_latents, mlp_packed, precision, q, n, nullptr, out, out_dtype, stream, "ntc_decode");
}

ntc_status ntc_decode_tile(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                           ntc_dtype precision, int32_t lod, int32_t x0, int32_t y0, int32_t width, int32_t height,
                           void* out, ntc_dtype out_dtype, void* stream) {
  ntc_status st = check_decode(m, precision, out_dtype);
  if (st != NTC_OK) return st;
  if (lod < 0 || lod >= m->num_mips) return fail(NTC_E_INVALID, "lod outside the mip chain");
  const int wl = m->mip_w[lod], hl = m->mip_h[lod];
  if (width < 0 || height < 0 || x0 < 0 || y0 < 0 || (int64_t)x0 + width > wl || (int64_t)y0 + height > hl)
    return fail(NTC_E_INVALID, "rectangle outside the mip");
  const int64_t n = (int64_t)width * height;
  if (n == 0) return NTC_OK;
  if (!packed_latents || !mlp_packed || !out) return fail(NTC_E_INVALID, "NULL buffer");
  TexelRect r;
  r.lod = lod;
  r.x0 = x0;
  r.y0 = y0;
  r.w = width;
  r.h = height;
  r.inv_w = 1.f / (float)wl;  // powers of two: exact
  r.inv_h = 1.f / (float)hl;
  return run_decode(m, packed_latents, mlp_packed, precision, nullptr, n, &r, out, out_dtype, stream,
                    "ntc_decode_tile");
}

ntc_status ntc_decode_filtered(const ntc_material* m, const uint8_t* packed_latents, const void* mlp_packed,
                               ntc_dtype precision, const ntc_filter_query* q, int64_t n, int32_t filter,
                               uint64_t seed, void* out, ntc_dtype out_dtype, void* stream) {
  ntc_status st = check_decode(m, precision, out_dtype);
  if (st != NTC_OK) return st;
  if (precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "filtered decode is built for F16 decode packs");
  if (filter != NTC_FILTER_BILINEAR && filter != NTC_FILTER_TRILINEAR && filter != NTC_FILTER_STOCHASTIC)
    return fail(NTC_E_INVALID, "unknown filter");
  if (n < 0 || n > ((int64_t)1 << 40)) return fail(NTC_E_INVALID, "n outside [0, 2^40]");
  if (n == 0) return NTC_OK;
  if (!packed_latents || !mlp_packed || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_decode_filtered(*m, packed_latents, mlp_packed, q, n, filter, seed, out,
                                           out_dtype == NTC_F16, (hipStream_t)stream),
                    "ntc_decode_filtered");
}

size_t ntc_train_workspace_bytes(const ntc_material* m, int64_t n, ntc_dtype precision) {
  if (!m || n <= 0 || n > kMaxTrainSamples || (precision != NTC_F32 && precision != NTC_F16)) return 0;
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden)) return 0;
  // large enough for every tuning candidate, so a tuned plan always fits
  const bool f16 = precision == NTC_F16;
  const TrainPlan base = train_plan(*m, f16, n);
  if (!base.supported_bins) return 0;  // more latent tiles than the binning kernels hold
  size_t total = base.total;
  int nc = 0;
  const TrainTune* c = train_tune_candidates(&nc);
  for (int i = 0; i < nc; ++i) total = std::max(total, train_plan(*m, f16, n, &c[i]).total);
  return total;
}

static ntc_status check_state(const ntc_train_state* s, bool f16) {
  if (!s) return fail(NTC_E_INVALID, "state is NULL");
  if (!s->latents || !s->latents_fwd || !s->lat_m || !s->lat_v || !s->lat_grad || !s->mlp || !s->mlp_m ||
      !s->mlp_v || !s->mlp_packed || !s->loss || !s->scale_state)
    return fail(NTC_E_INVALID, "NULL state buffer");
  if (f16 && !s->loss_scale) return fail(NTC_E_INVALID, "loss_scale is required for F16 training");
  for (const float* p : {s->latents, s->latents_fwd, s->lat_m, s->lat_v, s->lat_grad})
    if (reinterpret_cast<uintptr_t>(p) % 16 != 0) return fail(NTC_E_INVALID, "latent buffers must be 16-byte aligned");
  return NTC_OK;
}

static ntc_status check_hparams(const ntc_hparams* hp) {
  if (!hp) return fail(NTC_E_INVALID, "hparams is NULL");
  if (hp->precision != NTC_F32 && hp->precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  if (hp->step < 0) return fail(NTC_E_INVALID, "step < 0");
  if (!(hp->beta1 >= 0.f && hp->beta1 < 1.f && hp->beta2 >= 0.f && hp->beta2 < 1.f && hp->eps > 0.f))
    return fail(NTC_E_INVALID, "bad Adam constants");
  if (!std::isfinite(hp->lr_latent) || !std::isfinite(hp->lr_mlp)) return fail(NTC_E_INVALID, "bad learning rate");
  return NTC_OK;
}

ntc_status ntc_train_prepare(const ntc_material* m, const ntc_train_state* s, const ntc_hparams* hp, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if ((st = check_hparams(hp)) != NTC_OK) return st;
  const bool f16 = hp->precision == NTC_F16;
  if ((st = check_state(s, f16)) != NTC_OK) return st;
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no training kernel for this (c0, c1, channels, hidden)");
  hipStream_t hs = (hipStream_t)stream;
  const bool noise = hp->noise && !hp->freeze_latents;
  hipError_t e = launch_prepare(*m, s->latents, s->latents_fwd, s->lat_grad, noise_key(hp->noise_seed, hp->step),
                                noise ? 1 : 0, hs);
  if (e == hipSuccess) e = launch_pack_mlp(*m, s->mlp, f16, true, s->mlp_packed, hs);
  return hip_status(e, "ntc_train_prepare");
}

static ntc_status check_train(const ntc_material* m, const ntc_train_state* s, const ntc_hparams* hp, int64_t n) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if ((st = check_hparams(hp)) != NTC_OK) return st;
  if ((st = check_state(s, hp->precision == NTC_F16)) != NTC_OK) return st;
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no training kernel for this (c0, c1, channels, hidden)");
  if (n <= 0) return fail(NTC_E_INVALID, "n must be positive");
  if (n > kMaxTrainSamples) return fail(NTC_E_UNSUPPORTED, "n exceeds 2^31 / 4 samples per training call");
  return NTC_OK;
}

ntc_status ntc_train_gradients(const ntc_material* m, const ntc_train_state* s, const ntc_query* q, int64_t n,
                               const float* targets, const ntc_hparams* hp, void* workspace, size_t ws_bytes,
                               void* stream) {
  ntc_status st = check_train(m, s, hp, n);
  if (st != NTC_OK) return st;
  if (!q || !targets) return fail(NTC_E_INVALID, "NULL queries or targets");
  const bool f16 = hp->precision == NTC_F16;
  const TrainPlan plan = train_plan(*m, f16, n);
  if (!plan.supported_bins) return fail(NTC_E_UNSUPPORTED, "too many latent tiles for this material");
  if (!workspace || ws_bytes < plan.total) return fail(NTC_E_WORKSPACE, "workspace too small");
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "ntc_train_gradients (earlier asynchronous error)");
  TrainLaunch a;
  a.lat_fwd = s->latents_fwd;
  a.wpack = s->mlp_packed;
  a.mlp = s->mlp;
  a.q = q;
  a.n = n;
  a.targets = targets;
  a.lat_grad = s->lat_grad;
  a.workspace = workspace;
  a.loss_scale = f16 ? s->loss_scale : nullptr;
  a.scale_slot = hp->step & 1;
  a.step_dev = hp->step_dev;
  a.overflow_flag = s->scale_state + 1;
  a.scatter_latents = !hp->freeze_latents;
  a.dout = nullptr;
  a.dout_scale = 1.f;
  a.out_scale = 1.f;
  return hip_status(launch_train_gradients(*m, f16, plan, a, (hipStream_t)stream), "ntc_train_gradients");
}

ntc_status ntc_train_autotune(const ntc_material* m, const ntc_train_state* s, const ntc_query* q, int64_t n,
                              const float* targets, const ntc_hparams* hp, void* workspace, size_t ws_bytes,
                              void* stream, ntc_train_tuning* chosen) {
  ntc_status st = check_train(m, s, hp, n);
  if (st != NTC_OK) return st;
  if (!q || !targets) return fail(NTC_E_INVALID, "NULL queries or targets");
  if (hp->freeze_latents) return fail(NTC_E_INVALID, "tuning needs the latent scatter (freeze_latents = 0)");
  const bool f16 = hp->precision == NTC_F16;
  if (!workspace || ws_bytes < ntc_train_workspace_bytes(m, n, (ntc_dtype)hp->precision))
    return fail(NTC_E_WORKSPACE, "workspace too small");
  hipStream_t hs = (hipStream_t)stream;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return hip_status(hipGetLastError(), "ntc_train_autotune");
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return hip_status(hipGetLastError(), "ntc_train_autotune");
  }
  TrainLaunch a;
  a.lat_fwd = s->latents_fwd;
  a.wpack = s->mlp_packed;
  a.mlp = s->mlp;
  a.q = q;
  a.n = n;
  a.targets = targets;
  a.lat_grad = s->lat_grad;
  a.workspace = workspace;
  a.loss_scale = f16 ? s->loss_scale : nullptr;
  a.scale_slot = hp->step & 1;
  a.step_dev = hp->step_dev;
  a.overflow_flag = s->scale_state + 1;
  a.scatter_latents = true;
  a.dout = nullptr;
  a.dout_scale = 1.f;
  a.out_scale = 1.f;
  int nc = 0;
  const TrainTune* cand = train_tune_candidates(&nc);
  float best = 1e30f;
  TrainTune best_t{0, 0};
  hipError_t e = hipSuccess;
  for (int i = 0; i < nc && e == hipSuccess; ++i) {
    const TrainPlan plan = train_plan(*m, f16, n, &cand[i]);
    if (!plan.supported_bins || plan.total > ws_bytes) continue;
    if (i > 0 && plan.tune.chunk == best_t.chunk && plan.tune.tile == best_t.tile) continue;
    e = launch_train_gradients(*m, f16, plan, a, hs);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(e0, hs);
    for (int r = 0; r < 3 && e == hipSuccess; ++r) e = launch_train_gradients(*m, f16, plan, a, hs);
    if (e == hipSuccess) e = hipEventRecord(e1, hs);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    if (e == hipSuccess && ms < best) {
      best = ms;
      best_t = plan.tune;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_status(e, "ntc_train_autotune");
  if (best_t.chunk == 0) return fail(NTC_E_UNSUPPORTED, "no tuning candidate fits this material");
  set_train_tune(*m, f16, best_t);
  if (chosen) {
    chosen->chunk = best_t.chunk;
    chosen->tile = best_t.tile;
    chosen->microseconds = best * 1000.0 / 3.0;
  }
  return NTC_OK;
}

ntc_status ntc_train_set_tuning(const ntc_material* m, ntc_dtype precision, const ntc_train_tuning* t) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no training kernel for this (c0, c1, channels, hidden)");
  if (!t) return fail(NTC_E_INVALID, "tuning is NULL");
  if (t->chunk == 0 && t->tile == 0) {
    clear_train_tune(*m, precision == NTC_F16);
    return NTC_OK;
  }
  int nc = 0;
  const TrainTune* c = train_tune_candidates(&nc);
  for (int i = 0; i < nc; ++i)
    if (c[i].chunk == t->chunk && c[i].tile == t->tile) {
      set_train_tune(*m, precision == NTC_F16, c[i]);
      return NTC_OK;
    }
  return fail(NTC_E_INVALID, "(chunk, tile) is not one of the tuning candidates");
}

ntc_status ntc_train_get_tuning(const ntc_material* m, ntc_dtype precision, ntc_train_tuning* out) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no training kernel for this (c0, c1, channels, hidden)");
  if (!out) return fail(NTC_E_INVALID, "output is NULL");
  const TrainPlan p = train_plan(*m, precision == NTC_F16, 1);
  out->chunk = p.tune.chunk;
  out->tile = p.tune.tile;
  out->microseconds = 0.0;
  return NTC_OK;
}

static ntc_status train_update_impl(const ntc_material* m, const ntc_train_state* s, int64_t n,
                                    const ntc_hparams* hp, void* workspace, size_t ws_bytes, void* stream,
                                    bool advance_step);

ntc_status ntc_train_update(const ntc_material* m, const ntc_train_state* s, int64_t n, const ntc_hparams* hp,
                            void* workspace, size_t ws_bytes, void* stream) {
  return train_update_impl(m, s, n, hp, workspace, ws_bytes, stream, true);
}

static ntc_status train_update_impl(const ntc_material* m, const ntc_train_state* s, int64_t n,
                                    const ntc_hparams* hp, void* workspace, size_t ws_bytes, void* stream,
                                    bool advance_step) {
  ntc_status st = check_train(m, s, hp, n);
  if (st != NTC_OK) return st;
  const bool f16 = hp->precision == NTC_F16;
  const TrainPlan plan = train_plan(*m, f16, n);
  if (!workspace || ws_bytes < plan.total) return fail(NTC_E_WORKSPACE, "workspace too small");
  hipStream_t hs = (hipStream_t)stream;
  char* ws = (char*)workspace;
  hipError_t e = launch_train_reduce(*m, plan, workspace, s->loss, 1.0f / (float)((double)n * m->channels),
                                     s->scale_state + 1, hs);
  if (e == hipSuccess) {
    AdamLaunch ad;
    ad.latents = s->latents;
    ad.latents_fwd = s->latents_fwd;
    ad.lat_m = s->lat_m;
    ad.lat_v = s->lat_v;
    ad.lat_grad = s->lat_grad;
    ad.mlp = s->mlp;
    ad.mlp_m = s->mlp_m;
    ad.mlp_v = s->mlp_v;
    ad.mlp_grad = (const float*)(ws + plan.off_grad);
    ad.wpack = s->mlp_packed;
    ad.loss_scale = f16 ? s->loss_scale : nullptr;
    ad.scale_state = s->scale_state;
    ad.lr_lat = hp->lr_latent;
    ad.lr_mlp = hp->lr_mlp;
    ad.beta1 = hp->beta1;
    ad.beta2 = hp->beta2;
    ad.eps = hp->eps;
    const double t = (double)hp->step + 1.0;
    ad.bc1 = (float)(1.0 - std::pow((double)hp->beta1, t));
    ad.bc2 = (float)(1.0 - std::pow((double)hp->beta2, t));
    ad.next_key = noise_key(hp->noise_seed, hp->step + 1);
    ad.step = hp->step;
    ad.noise = hp->noise ? 1 : 0;
    ad.freeze = hp->freeze_latents ? 1 : 0;
    ad.growth = hp->scale_growth_interval > 0 ? hp->scale_growth_interval : 2000;
    ad.f16 = f16 ? 1 : 0;
    ad.step_dev = hp->step_dev;
    ad.lr_dev = hp->lr_dev;
    ad.seed = hp->noise_seed;
    ad.advance = advance_step;
    e = launch_adam(*m, ad, hs);
  }
  return hip_status(e, "ntc_train_update");
}

ntc_status ntc_pack_mlp_train(const ntc_material* m, const float* mlp, ntc_dtype precision, void* packed,
                              void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "pack precision must be F32 or F16");
  if (!mlp || !packed) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_pack_mlp(*m, mlp, precision == NTC_F16, true, packed, (hipStream_t)stream),
                    "ntc_pack_mlp_train");
}

ntc_status ntc_forward(const ntc_material* m, const float* latents, const float* mlp, const void* mlp_train_packed,
                       ntc_dtype precision, const ntc_query* q, int64_t n, float* out, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  if (n < 0) return fail(NTC_E_INVALID, "n < 0");
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no kernel for this (c0, c1, channels, hidden)");
  if (n == 0) return NTC_OK;
  if (!latents || !mlp || !mlp_train_packed || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(
      launch_forward(*m, latents, mlp, mlp_train_packed, precision == NTC_F16, q, n, out, (hipStream_t)stream),
      "ntc_forward");
}

size_t ntc_backward_workspace_bytes(const ntc_material* m, int64_t n, ntc_dtype precision) {
  return ntc_train_workspace_bytes(m, n, precision);
}

ntc_status ntc_backward(const ntc_material* m, const float* latents, const float* mlp, const void* mlp_train_packed,
                        ntc_dtype precision, const ntc_query* q, int64_t n, const float* dout, float dout_scale,
                        float* grad_latents, float* grad_mlp, void* workspace, size_t ws_bytes, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  if (!train_shape_supported(m->c0, m->c1, m->channels, m->hidden))
    return fail(NTC_E_UNSUPPORTED, "no kernel for this (c0, c1, channels, hidden)");
  if (n <= 0) return fail(NTC_E_INVALID, "n must be positive");
  if (n > kMaxTrainSamples) return fail(NTC_E_UNSUPPORTED, "n exceeds 2^31 / 4 samples per backward call");
  if (!latents || !mlp || !mlp_train_packed || !q || !dout || !grad_latents || !grad_mlp)
    return fail(NTC_E_INVALID, "NULL buffer");
  if (!(dout_scale >= 0.f) || !std::isfinite(dout_scale))
    return fail(NTC_E_INVALID, "dout_scale must be positive (or 0: chosen on the device)");
  const bool f16 = precision == NTC_F16;
  const TrainPlan plan = train_plan(*m, f16, n);
  if (!plan.supported_bins) return fail(NTC_E_UNSUPPORTED, "too many latent tiles for this material");
  if (!workspace || ws_bytes < plan.total) return fail(NTC_E_WORKSPACE, "workspace too small");
  hipStream_t hs = (hipStream_t)stream;
  char* ws = (char*)workspace;
  TrainLaunch a;
  a.lat_fwd = latents;
  a.wpack = mlp_train_packed;
  a.mlp = mlp;
  a.q = q;
  a.n = n;
  a.targets = nullptr;
  a.lat_grad = grad_latents;
  a.workspace = workspace;
  a.loss_scale = nullptr;
  a.scale_slot = 0;
  a.step_dev = nullptr;
  a.overflow_flag = (int32_t*)(ws + plan.off_misc + 16);
  a.scatter_latents = true;
  a.dout = dout;
  const bool auto_scale = dout_scale == 0.f;
  a.dout_scale = auto_scale ? 1.f : dout_scale;
  a.out_scale = 1.f / a.dout_scale;
  float* dscale = auto_scale ? (float*)(ws + plan.off_dscale) : nullptr;
  a.dscale = dscale;
  hipError_t e = auto_scale ? launch_dout_scale(dout, n * (int64_t)m->channels, dscale, hs) : hipSuccess;
  if (e == hipSuccess) e = launch_train_gradients(*m, f16, plan, a, hs);
  if (e == hipSuccess)
    e = launch_train_reduce(*m, plan, workspace, nullptr, 0.f, nullptr, hs, grad_mlp, a.out_scale, dscale);
  return hip_status(e, "ntc_backward");
}

ntc_status ntc_train_step(const ntc_material* m, const ntc_train_state* s, const ntc_query* q, int64_t n,
                          const float* targets, const ntc_hparams* hp, void* workspace, size_t ws_bytes,
                          void* stream) {
  ntc_status st = ntc_train_gradients(m, s, q, n, targets, hp, workspace, ws_bytes, stream);
  if (st != NTC_OK) return st;
  return ntc_train_update(m, s, n, hp, workspace, ws_bytes, stream);
}

// ------------------------------------------------------------------ training without a workspace
// The step's workspace as a file-scope device array: each GPU the library runs on holds
// one copy until the process ends.  In host code `scratch` names a host-side stand-in;
// its device address on the current device comes from hipGetSymbolAddress, taken once
// per device on the first call there and kept.
static __device__ __align__(256) unsigned char scratch[NTC_NOALLOC_SCRATCH_BYTES];

static ntc_status scratch_on_current_device(void** out) {
  static std::mutex mu;
  static void* ptr[64] = {nullptr};
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return hip_status(e, "ntc_train_step_noalloc (hipGetDevice)");
  if (dev < 0 || dev >= 64) return fail(NTC_E_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(mu);
  if (!ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return hip_status(e != hipSuccess ? e : hipErrorInvalidSymbol,
                                                  "ntc_train_step_noalloc (hipGetSymbolAddress)");
    ptr[dev] = p;
  }
  *out = ptr[dev];
  return NTC_OK;
}

ntc_status ntc_train_step_noalloc(const ntc_material* m, const ntc_train_state* s, const ntc_query* q, int64_t n,
                                  const float* targets, const ntc_hparams* hp, void* stream) {
  ntc_status st = check_train(m, s, hp, n);
  if (st != NTC_OK) return st;
  if (!q || !targets) return fail(NTC_E_INVALID, "NULL queries or targets");
  const TrainPlan plan = train_plan(*m, hp->precision == NTC_F16, n);
  if (!plan.supported_bins) return fail(NTC_E_UNSUPPORTED, "too many latent tiles for this material");
  if (plan.total > (size_t)NTC_NOALLOC_SCRATCH_BYTES)
    return fail(NTC_E_WORKSPACE, "this step needs " + std::to_string(plan.total) +
                                     " bytes of scratch, more than the static array's " +
                                     std::to_string((size_t)NTC_NOALLOC_SCRATCH_BYTES) +
                                     " (call ntc_train_step with a workspace)");
  void* ws = nullptr;
  if ((st = scratch_on_current_device(&ws)) != NTC_OK) return st;
  return ntc_train_step(m, s, q, n, targets, hp, ws, (size_t)NTC_NOALLOC_SCRATCH_BYTES, stream);
}

ntc_status ntc_crop_queries(const ntc_material* m, uint64_t seed, int32_t step, int32_t crops, int32_t side,
                            double uniform_fraction, ntc_query* out, void* stream) {
  ntc_status st = check_material(m);
  if (st != NTC_OK) return st;
  if (crops < 1 || side < 1 || side > 32768 || (int64_t)crops * side * side > ((int64_t)1 << 31))
    return fail(NTC_E_INVALID, "crops and side must be positive, crops * side^2 < 2^31");
  if (!(uniform_fraction >= 0.0 && uniform_fraction <= 1.0)) return fail(NTC_E_INVALID, "fraction outside [0, 1]");
  if (step < 0) return fail(NTC_E_INVALID, "step < 0");
  if (!out) return fail(NTC_E_INVALID, "NULL output");
  return hip_status(launch_crop_queries(*m, seed, step, crops, side, uniform_fraction, out, (hipStream_t)stream),
                    "ntc_crop_queries");
}

// ------------------------------------------------------------------ many materials
static ntc_status check_batch(const ntc_material* mats, int32_t nmat, const int64_t* offsets) {
  if (!mats || !offsets) return fail(NTC_E_INVALID, "NULL materials or offsets");
  if (nmat < 1) return fail(NTC_E_INVALID, "nmat must be positive");
  if (offsets[0] != 0) return fail(NTC_E_INVALID, "offsets[0] must be 0");
  for (int i = 0; i < nmat; ++i) {
    ntc_status st = check_material(mats + i);
    if (st != NTC_OK) return st;
    if (offsets[i + 1] < offsets[i]) return fail(NTC_E_INVALID, "offsets must be non-decreasing");
  }
  return NTC_OK;
}

size_t ntc_train_workspace_bytes_batched(const ntc_material* mats, int32_t nmat, const int64_t* offsets,
                                         ntc_dtype precision) {
  if (check_batch(mats, nmat, offsets) != NTC_OK) return 0;
  size_t total = 0;
  for (int i = 0; i < nmat; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n <= 0) continue;
    const size_t b = ntc_train_workspace_bytes(mats + i, n, precision);
    if (b == 0) return 0;
    total += (b + 255) / 256 * 256;
  }
  return total;
}

ntc_status ntc_train_step_batched(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                  const ntc_query* q, const int64_t* offsets, const float* const* targets,
                                  const ntc_hparams* hp, void* workspace, size_t ws_bytes, void* stream) {
  ntc_status st = check_batch(mats, nmat, offsets);
  if (st != NTC_OK) return st;
  if (!states || !q || !targets) return fail(NTC_E_INVALID, "NULL states, queries or targets");
  for (int i = 0; i < nmat; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n <= 0) continue;
    if ((st = check_train(mats + i, states + i, hp, n)) != NTC_OK) return st;
    if (!targets[i]) return fail(NTC_E_INVALID, "NULL targets");
    if (!train_plan(mats[i], hp->precision == NTC_F16, n).supported_bins)
      return fail(NTC_E_UNSUPPORTED, "too many latent tiles for a material");
  }
  const size_t need = ntc_train_workspace_bytes_batched(mats, nmat, offsets, (ntc_dtype)hp->precision);
  if (!workspace || need == 0 || ws_bytes < need) return fail(NTC_E_WORKSPACE, "workspace too small");
  char* ws = (char*)workspace;
  size_t off = 0;
  for (int i = 0; i < nmat; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n <= 0) continue;
    const size_t b = (ntc_train_workspace_bytes(mats + i, n, (ntc_dtype)hp->precision) + 255) / 256 * 256;
    st = ntc_train_gradients(mats + i, states + i, q + offsets[i], n, targets[i], hp, ws + off, b, stream);
    if (st == NTC_OK)
      st = train_update_impl(mats + i, states + i, n, hp, ws + off, b, stream, /*advance_step=*/false);
    if (st != NTC_OK) return st;
    off += b;
  }
  if (hp->step_dev)  // one step for the whole batch
    return hip_status(launch_step_advance(hp->step_dev, (hipStream_t)stream), "ntc_train_step_batched");
  return NTC_OK;
}

ntc_status ntc_decode_batched(const ntc_material* mats, int32_t nmat, const uint8_t* const* packed_latents,
                              const void* const* mlp_packed, ntc_dtype precision, const ntc_query* q,
                              const int64_t* offsets, void* out, ntc_dtype out_dtype, void* stream) {
  ntc_status st = check_batch(mats, nmat, offsets);
  if (st != NTC_OK) return st;
  if (!packed_latents || !mlp_packed || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  for (int i = 0; i < nmat; ++i) {
    if ((st = check_decode(mats + i, precision, out_dtype)) != NTC_OK) return st;
    if (offsets[i + 1] > offsets[i] && (!packed_latents[i] || !mlp_packed[i]))
      return fail(NTC_E_INVALID, "NULL latents or weights");
  }
  const size_t esz = out_dtype == NTC_F16 ? 2 : 4;
  size_t o = 0;
  for (int i = 0; i < nmat; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    if (n > 0) {
      st = run_decode(mats + i, packed_latents[i], mlp_packed[i], precision, q + offsets[i], n, nullptr,
                      (char*)out + o * esz, out_dtype, stream, "ntc_decode_batched");
      if (st != NTC_OK) return st;
    }
    o += (size_t)n * mats[i].channels;
  }
  return NTC_OK;
}

// ------------------------------------------------------------------ grouped training
// Validates a grouped-training group and builds each member's buffer view (fused[i],
// with the queries of `q`, and adam[i], pointers only).
static ntc_status group_members(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                const ntc_query* q, const int64_t* offsets, const float* const* targets,
                                ntc_dtype precision, void* workspace, size_t ws_bytes,
                                std::vector<TrainLaunch>& fused, std::vector<AdamLaunch>& adam) {
  ntc_status st = check_batch(mats, nmat, offsets);
  if (st != NTC_OK) return st;
  if (!states || !targets) return fail(NTC_E_INVALID, "NULL states or targets");
  if (precision != NTC_F32 && precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "precision must be F32 or F16");
  const bool f16 = precision == NTC_F16;
  for (int i = 0; i < nmat; ++i) {
    if ((st = check_state(states + i, f16)) != NTC_OK) return st;
    if (!train_shape_supported(mats[i].c0, mats[i].c1, mats[i].channels, mats[i].hidden))
      return fail(NTC_E_UNSUPPORTED, "no training kernel for a material's (c0, c1, channels, hidden)");
    if (offsets[i + 1] <= offsets[i]) return fail(NTC_E_INVALID, "every member of a group needs samples");
    if (!targets[i]) return fail(NTC_E_INVALID, "NULL targets");
    if (!train_plan(mats[i], f16, offsets[i + 1] - offsets[i]).supported_bins)
      return fail(NTC_E_UNSUPPORTED, "too many latent tiles for a material");
  }
  const size_t need = ntc_train_workspace_bytes_batched(mats, nmat, offsets, precision);
  if (!workspace || need == 0 || ws_bytes < need) return fail(NTC_E_WORKSPACE, "workspace too small");
  fused.assign(nmat, TrainLaunch{});
  adam.assign(nmat, AdamLaunch{});
  size_t off = 0;
  for (int i = 0; i < nmat; ++i) {
    const int64_t n = offsets[i + 1] - offsets[i];
    const ntc_train_state* sp = states + i;
    TrainLaunch& a = fused[i];
    a.lat_fwd = sp->latents_fwd;
    a.wpack = sp->mlp_packed;
    a.mlp = sp->mlp;
    a.q = q ? q + offsets[i] : nullptr;
    a.n = n;
    a.targets = targets[i];
    a.lat_grad = sp->lat_grad;
    a.workspace = (char*)workspace + off;
    a.loss_scale = f16 ? sp->loss_scale : nullptr;
    a.scale_slot = 0;
    a.step_dev = nullptr;
    a.overflow_flag = sp->scale_state + 1;
    a.scatter_latents = true;
    a.dout = nullptr;
    a.dout_scale = 1.f;
    a.out_scale = 1.f;
    AdamLaunch& d = adam[i];
    d.latents = sp->latents;
    d.latents_fwd = sp->latents_fwd;
    d.lat_m = sp->lat_m;
    d.lat_v = sp->lat_v;
    d.lat_grad = sp->lat_grad;
    d.mlp = sp->mlp;
    d.mlp_m = sp->mlp_m;
    d.mlp_v = sp->mlp_v;
    d.mlp_grad = nullptr;  // the member's workspace (set with the table)
    d.wpack = sp->mlp_packed;
    d.loss_scale = f16 ? sp->loss_scale : nullptr;
    d.scale_state = sp->scale_state;
    d.f16 = f16 ? 1 : 0;
    d.loss_out = sp->loss;
    off += (ntc_train_workspace_bytes(mats + i, n, precision) + 255) / 256 * 256;
  }
  return NTC_OK;
}

size_t ntc_train_table_bytes(int32_t nmat) { return nmat < 1 ? 0 : train_table_bytes(nmat); }

ntc_status ntc_train_table_init(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                const int64_t* offsets, const float* const* targets, ntc_dtype precision,
                                void* workspace, size_t ws_bytes, void* table, size_t table_bytes) {
  std::vector<TrainLaunch> fused;
  std::vector<AdamLaunch> adam;
  ntc_status st = group_members(mats, nmat, states, nullptr, offsets, targets, precision, workspace, ws_bytes, fused,
                                adam);
  if (st != NTC_OK) return st;
  if (!table) return fail(NTC_E_INVALID, "NULL table");
  if (table_bytes < train_table_bytes(nmat)) return fail(NTC_E_WORKSPACE, "training table too small");
  const bool f16 = precision == NTC_F16;
  const unsigned long long h = train_group_hash(mats, nmat, offsets, f16, fused.data(), adam.data());
  std::vector<char> host(train_table_bytes(nmat));
  fill_train_table(mats, nmat, offsets, f16, fused.data(), adam.data(), h, host.data());
  return hip_status(hipMemcpy(table, host.data(), host.size(), hipMemcpyHostToDevice), "ntc_train_table_init");
}

ntc_status ntc_train_step_grouped(const ntc_material* mats, int32_t nmat, const ntc_train_state* states,
                                  const ntc_query* q, const int64_t* offsets, const float* const* targets,
                                  const ntc_hparams* hp, void* workspace, size_t ws_bytes, const void* table,
                                  void* stream) {
  ntc_status st = check_hparams(hp);
  if (st != NTC_OK) return st;
  if (!q || !table) return fail(NTC_E_INVALID, "NULL queries or table");
  std::vector<TrainLaunch> fused;
  std::vector<AdamLaunch> adam;
  st = group_members(mats, nmat, states, q, offsets, targets, (ntc_dtype)hp->precision, workspace, ws_bytes, fused,
                     adam);
  if (st != NTC_OK) return st;
  const bool f16 = hp->precision == NTC_F16;
  const unsigned long long h = train_group_hash(mats, nmat, offsets, f16, fused.data(), adam.data());
  for (auto& a : fused) {
    a.scale_slot = hp->step & 1;
    a.step_dev = hp->step_dev;
    a.scatter_latents = !hp->freeze_latents;
  }
  AdamLaunch hot{};
  hot.lr_lat = hp->lr_latent;
  hot.lr_mlp = hp->lr_mlp;
  hot.beta1 = hp->beta1;
  hot.beta2 = hp->beta2;
  hot.eps = hp->eps;
  const double t = (double)hp->step + 1.0;
  hot.bc1 = (float)(1.0 - std::pow((double)hp->beta1, t));
  hot.bc2 = (float)(1.0 - std::pow((double)hp->beta2, t));
  hot.next_key = noise_key(hp->noise_seed, hp->step + 1);
  hot.seed = hp->noise_seed;
  hot.step = hp->step;
  hot.noise = hp->noise ? 1 : 0;
  hot.freeze = hp->freeze_latents ? 1 : 0;
  hot.growth = hp->scale_growth_interval > 0 ? hp->scale_growth_interval : 2000;
  hot.step_dev = hp->step_dev;
  hot.lr_dev = hp->lr_dev;
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_status(e, "ntc_train_step_grouped (earlier asynchronous error)");
  return hip_status(launch_train_grouped(mats, nmat, offsets, f16, table, h, q, !hp->freeze_latents, fused.data(), hot,
                                         (hipStream_t)stream),
                    "ntc_train_step_grouped");
}

size_t ntc_decode_table_bytes(int32_t nmat) {
  if (nmat < 1) return 0;
  return (size_t)kGroupHeaderBytes + (size_t)nmat * sizeof(GroupEntry);
}

ntc_status ntc_decode_table_init(const ntc_material* mats, int32_t nmat, const uint8_t* const* packed_latents,
                                 const void* const* mlp_packed, ntc_dtype precision, void* table,
                                 size_t table_bytes) {
  if (!mats || nmat < 1) return fail(NTC_E_INVALID, "NULL materials or nmat < 1");
  if (!packed_latents || !mlp_packed || !table) return fail(NTC_E_INVALID, "NULL buffer");
  if (table_bytes < ntc_decode_table_bytes(nmat)) return fail(NTC_E_WORKSPACE, "decode table too small");
  for (int i = 0; i < nmat; ++i) {
    ntc_status st = check_decode(mats + i, precision, NTC_F16);
    if (st != NTC_OK) return st;
    if (!packed_latents[i] || !mlp_packed[i]) return fail(NTC_E_INVALID, "NULL latents or weights");
  }
  std::vector<char> host(ntc_decode_table_bytes(nmat), 0);
  const unsigned long long h = group_hash(mats, nmat);
  std::memcpy(host.data(), &h, sizeof h);
  GroupEntry* e = reinterpret_cast<GroupEntry*>(host.data() + kGroupHeaderBytes);
  for (int i = 0; i < nmat; ++i) fill_group_entry(mats[i], packed_latents[i], mlp_packed[i], e[i]);
  return hip_status(hipMemcpy(table, host.data(), host.size(), hipMemcpyHostToDevice), "ntc_decode_table_init");
}

ntc_status ntc_decode_mixed(const ntc_material* mats, int32_t nmat, const void* table, ntc_dtype precision,
                            const ntc_mixed_query* q, int64_t n, void* out, ntc_dtype out_dtype, void* stream) {
  if (!mats || nmat < 1 || nmat > kMixedMax) return fail(NTC_E_INVALID, "nmat must be in 1..64");
  ntc_status st = NTC_OK;
  for (int i = 0; i < nmat; ++i) {
    if ((st = check_decode(mats + i, precision, out_dtype)) != NTC_OK) return st;
    const ntc_material& a = mats[0];
    const ntc_material& b = mats[i];
    if (a.c0 != b.c0 || a.c1 != b.c1 || a.channels != b.channels || a.hidden != b.hidden || a.b0 != b.b0 ||
        a.b1 != b.b1 || a.activation != b.activation || a.posenc != b.posenc)
      return fail(NTC_E_UNSUPPORTED, "mixed decode needs materials of one decode shape");
  }
  if (precision != NTC_F16) return fail(NTC_E_UNSUPPORTED, "mixed decode is built for F16 decode packs");
  if (n < 0) return fail(NTC_E_INVALID, "n < 0");
  if (n == 0) return NTC_OK;
  if (!table || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  return hip_status(launch_decode_mixed(mats, nmat, table, q, n, out, out_dtype == NTC_F16, (hipStream_t)stream),
                    "ntc_decode_mixed");
}

ntc_status ntc_decode_grouped(const ntc_material* mats, int32_t nmat, const void* table, ntc_dtype precision,
                              const ntc_query* q, const int64_t* offsets, void* out, ntc_dtype out_dtype,
                              void* stream) {
  ntc_status st = check_batch(mats, nmat, offsets);
  if (st != NTC_OK) return st;
  if (!table || !q || !out) return fail(NTC_E_INVALID, "NULL buffer");
  for (int i = 0; i < nmat; ++i)
    if ((st = check_decode(mats + i, precision, out_dtype)) != NTC_OK) return st;
  return hip_status(launch_decode_grouped(mats, nmat, table, precision, q, offsets, out, out_dtype == NTC_F16,
                                          (hipStream_t)stream),
                    "ntc_decode_grouped");
}

}  // extern "C"
