// Filtered decode launchers (bilinear, trilinear, stochastic; section 5.3) for the
// FP16 decoder: the filter's taps are decoded like point queries, TAPS lanes of a
// 16-texel tile per output, and their weighted sum is reduced across those lanes.
#include <algorithm>

#include "decode_impl.h"

namespace ntc {

namespace {

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT, int FILT>
hipError_t filtered_t(const ntc_material& mm, const uint8_t* packed, const void* wpack, const ntc_filter_query* q,
                      long long n, uint64_t key, void* out, bool out_f16, hipStream_t s) {
  constexpr int WB = DecodeLayout<_Float16, C0, C1, HD, B0, B1, true>::WB;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4 + kMaxLevels * sizeof(LevelBytes);
  auto kern = decode_filtered_kernel<_Float16, C0, C1, C, HD, B0, B1, ACT, FILT>;
  static const int per_cu = blocks_per_cu(kern, 256, lds);
  const long long tiles = (n * filter_taps<FILT>() + 15) / 16;
  const long long grid = std::min((tiles + 3) / 4, (long long)device_cus() * per_cu);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, dev_mat(mm), pe_table(mm), packed,
                     reinterpret_cast<const _Float16*>(wpack), q, n, key, out, out_f16 ? 1 : 0);
  return hipGetLastError();
}

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
hipError_t filtered_mode(const ntc_material& m, const uint8_t* packed, const void* wpack, const ntc_filter_query* q,
                         long long n, int filter, uint64_t key, void* out, bool out_f16, hipStream_t s) {
  switch (filter) {
    case NTC_FILTER_BILINEAR:
      return filtered_t<C0, C1, C, HD, B0, B1, ACT, 1>(m, packed, wpack, q, n, key, out, out_f16, s);
    case NTC_FILTER_TRILINEAR:
      return filtered_t<C0, C1, C, HD, B0, B1, ACT, 2>(m, packed, wpack, q, n, key, out, out_f16, s);
    case NTC_FILTER_STOCHASTIC:
      return filtered_t<C0, C1, C, HD, B0, B1, ACT, 3>(m, packed, wpack, q, n, key, out, out_f16, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_decode_filtered(const ntc_material& m, const uint8_t* packed, const void* wpack,
                                  const ntc_filter_query* q, long long n, int filter, uint64_t seed, void* out,
                                  bool out_f16, hipStream_t s) {
  const uint64_t key = mix64(seed ^ kFilterTag);
#define NTC_X(a, b, cc, h, x0, x1)                                                                            \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h && m.b0 == x0 && m.b1 == x1)              \
    return m.activation ? filtered_mode<a, b, cc, h, x0, x1, 1>(m, packed, wpack, q, n, filter, key, out, out_f16, s) \
                        : filtered_mode<a, b, cc, h, x0, x1, 0>(m, packed, wpack, q, n, filter, key, out, out_f16, s);
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

}  // namespace ntc
