// Single-material decode launchers: random queries (ntc_decode), texel rectangles
// (ntc_decode_tile) and the FP32-latent forward of the differentiation path.
#include <algorithm>

#include "decode_impl.h"

namespace ntc {

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
static hipError_t decode_fp8_t1(const ntc_material& mm, const uint8_t* packed, const void* wpack, const ntc_query* q,
                                long long n, const TexelRect& rect, void* out, bool out_f16, hipStream_t s) {
  constexpr PackGeom pg = pack_geom_fp8(C0, C1, B0, B1, HD);
  constexpr int WB = ((int)pg.fwd_end + 15) / 16 * 16;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4 + kMaxLevels * sizeof(LevelBytes) +
                     DecodeLayout<_Float16, C0, C1, HD, B0, B1, true>::SLAB;
  const float* scales = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wpack) + WB);
  auto kern = decode_fp8_kernel<C0, C1, C, HD, B0, B1, ACT>;
  static const int per_cu = blocks_per_cu(kern, 256, lds);
  const long long tiles = (n + 15) / 16;
  long long grid = (tiles + 3) / 4;
  const long long cap = (long long)device_cus() * per_cu;
  if (grid > cap) grid = cap;
  const int slot = timing_before(TK_DECODE, s);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, dev_mat(mm), pe_table(mm),
                     reinterpret_cast<const uint32_t*>(packed), reinterpret_cast<const uint8_t*>(wpack), scales,
                     scales + 4, q, n, rect, out, out_f16 ? 1 : 0);
  timing_after(TK_DECODE, s, slot);
  return hipGetLastError();
}

// mlp: canonical FP32 parameters supplying the biases, or nullptr when the biases
// follow the weights in the pack (decode packs)
template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED, int ACT>
static hipError_t decode_t1(const ntc_material& mm, const void* src, const void* wpack, const float* mlp,
                           const ntc_query* q, long long n, const TexelRect& rect, void* out, bool out_f16,
                           hipStream_t s) {
  using DL = DecodeLayout<T, C0, C1, HD, B0, B1, PACKED>;
  constexpr int WB = DL::WB;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4 + kMaxLevels * sizeof(LevelBytes) + DL::SLAB;
  const float *b1, *b2, *b3;
  if (mlp) {
    const long long K = mm.input_width;
    b1 = mlp + K * HD;
    b2 = b1 + HD + (long long)HD * HD;
    b3 = b2 + HD + (long long)HD * C;
  } else {
    b1 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wpack) + WB);
    b2 = b1 + HD;
    b3 = b2 + HD;
  }
  auto kern = decode_kernel<T, C0, C1, C, HD, B0, B1, PACKED, ACT>;
  static const int per_cu = blocks_per_cu(kern, 256, lds);
  const long long tiles = (n + 15) / 16;
  long long grid = (tiles + 3) / 4;
  const long long cap = (long long)device_cus() * per_cu;
  if (grid > cap) grid = cap;
  const int slot = PACKED ? timing_before(TK_DECODE, s) : -1;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, dev_mat(mm), pe_table(mm), src,
                     reinterpret_cast<const T*>(wpack), b1, b2, b3, q, n, rect, out, out_f16 ? 1 : 0);
  timing_after(TK_DECODE, s, slot);
  return hipGetLastError();
}

template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED>
static hipError_t decode_t(const ntc_material& mm, const void* src, const void* wpack, const float* mlp,
                           const ntc_query* q, long long n, const TexelRect& rect, void* out, bool out_f16,
                           hipStream_t s) {
  return mm.activation
             ? decode_t1<T, C0, C1, C, HD, B0, B1, PACKED, 1>(mm, src, wpack, mlp, q, n, rect, out, out_f16, s)
             : decode_t1<T, C0, C1, C, HD, B0, B1, PACKED, 0>(mm, src, wpack, mlp, q, n, rect, out, out_f16, s);
}

bool decode_shape_supported(int c0, int c1, int c, int hd, int b0, int b1) {
#define NTC_X(a, b, cc, h, x0, x1) \
  if (c0 == a && c1 == b && c == cc && hd == h && b0 == x0 && b1 == x1) return true;
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return false;
}

// rect: nullptr for query-array decode, else the texel rectangle to decode (q unused)
static TexelRect make_rect(const ntc_material& m, const TexelRect* rect) {
  if (rect) return *rect;
  TexelRect r{};
  return r;
}

hipError_t launch_decode(const ntc_material& m, const uint8_t* packed, const void* wpack, bool f16, const ntc_query* q,
                         long long n, const TexelRect* rect, void* out, bool out_f16, hipStream_t s) {
  const TexelRect r = make_rect(m, rect);
#define NTC_X(a, b, cc, h, x0, x1)                                                                             \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h && m.b0 == x0 && m.b1 == x1)                \
    return f16 ? decode_t<_Float16, a, b, cc, h, x0, x1, true>(m, packed, wpack, nullptr, q, n, r, out, out_f16, s) \
               : decode_t<float, a, b, cc, h, x0, x1, true>(m, packed, wpack, nullptr, q, n, r, out, out_f16, s);
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

hipError_t launch_decode_fp8(const ntc_material& m, const uint8_t* packed, const void* wpack, const ntc_query* q,
                             long long n, const TexelRect* rect, void* out, bool out_f16, hipStream_t s) {
  const TexelRect r = make_rect(m, rect);
#define NTC_X(a, b, cc, h, x0, x1)                                                                      \
  if constexpr (fp8_layout(a, b, x0, x1, h))                                                            \
    if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h && m.b0 == x0 && m.b1 == x1)       \
      return m.activation ? decode_fp8_t1<a, b, cc, h, x0, x1, 1>(m, packed, wpack, q, n, r, out, out_f16, s) \
                          : decode_fp8_t1<a, b, cc, h, x0, x1, 0>(m, packed, wpack, q, n, r, out, out_f16, s);
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

// Forward from FP32 latents (the differentiation path) with the training pack, whose
// forward part leads it, and the biases of the canonical parameters; shapes as for training.
#define NTC_FORWARD_SHAPES(X)                                                          \
  X(8, 8, 8, 64) X(10, 10, 10, 64) X(12, 12, 12, 64) X(16, 16, 16, 64) X(8, 8, 8, 32) \
  X(10, 10, 10, 32) X(12, 12, 12, 32) X(16, 16, 16, 32)                              \
  X(8, 12, 9, 64) X(12, 20, 9, 64) X(12, 10, 9, 64) X(16, 12, 9, 64)

hipError_t launch_forward(const ntc_material& m, const float* latents, const float* mlp, const void* wpack, bool f16,
                          const ntc_query* q, long long n, float* out, hipStream_t s) {
#define NTC_X(a, b, cc, h)                                                                                   \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h)                                           \
    return f16 ? decode_t<_Float16, a, b, cc, h, 4, 4, false>(m, latents, wpack, mlp, q, n, TexelRect{}, out,  \
                                                                 false, s)                                     \
               : decode_t<float, a, b, cc, h, 4, 4, false>(m, latents, wpack, mlp, q, n, TexelRect{}, out, false, s);
  NTC_FORWARD_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

}  // namespace ntc
