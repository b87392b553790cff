// Random-access decode (sections 4.3-4.4): packed latents -> all C channels per texel.
//
// Persistent kernel, 4 wavefronts per block, one 16-texel tile per wavefront
// iteration.  Each of the 4 lane groups of a texel fetches one G0 neighbour cell
// (a contiguous C0*B0-bit window), a quarter of the G1 bilinear channels and 3 of
// the 12 positional-encoding values, so the MLP input is assembled directly in the
// B-operand layout of the matrix cores.  The three layers chain through registers;
// weights are staged once per block in LDS.
#include <algorithm>

#include "ntc_internal.h"

namespace ntc {

// PACKED: latents come as bit-packed codes (ntc_decode); otherwise as FP32 values
// in the canonical latent layout (ntc_forward, the differentiation path).
template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED>
__global__ __launch_bounds__(256) void decode_kernel(DevMat m, PeTable pe, const void* __restrict__ src,
                                                     const T* __restrict__ wpack, const float* __restrict__ bias,
                                                     const ntc_query* __restrict__ q, long long n,
                                                     void* __restrict__ out, int out_f16) {
  const uint32_t* __restrict__ packed = reinterpret_cast<const uint32_t*>(src);
  const float* __restrict__ lat = reinterpret_cast<const float*>(src);
  using IS = InSlots<C0, C1>;
  constexpr PackGeom pg = pack_geom(C0, C1, HD, sizeof(T) == 2);
  constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT;
  constexpr int WB = ((int)pg.fwd_end * (int)sizeof(T) + 15) / 16 * 16;
  extern __shared__ __align__(16) char smem[];
  T* w_lds = reinterpret_cast<T*>(smem);
  float* pe_lds = reinterpret_cast<float*>(smem + WB);
  float* b_lds = pe_lds + 48;  // b1 (HD), b2 (HD), b3 (C, zero-padded to 16)

  for (int i = threadIdx.x; i < WB / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(smem)[i] = reinterpret_cast<const uint4*>(wpack)[i];
  for (int i = threadIdx.x; i < 48; i += blockDim.x) pe_lds[i] = pe.v[i / 6][i % 6];
  for (int i = threadIdx.x; i < 2 * HD + 16; i += blockDim.x) b_lds[i] = (i < 2 * HD + C) ? bias[i] : 0.f;
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const long long tiles = (n + 15) / 16;
  for (long long tile = (long long)blockIdx.x * 4 + wave; tile < tiles; tile += (long long)gridDim.x * 4) {
    const long long s = tile * 16 + r;
    const bool valid = s < n;
    float u = 0.f, v = 0.f;
    int lod = 0;
    if (valid) {
      u = q[s].u;
      v = q[s].v;
      lod = q[s].lod;
    }
    const Footprint f = locate(m, u, v, lod, g);
    T xs[S1];
    if constexpr (PACKED) {
      {  // G0: this group's neighbour, all C0 channels (learned interpolation input)
        constexpr int NB = C0 * B0, NW = (NB + 31) / 32;
        uint32_t win[NW];
        load_bits<NW, NB % 32 == 0>(packed, m.g0_pk[f.j] * 8 + (long long)f.g0_cell * NB, m.g0_pk_end[f.j], win);
#pragma unroll
        for (int t = 0; t < C0; ++t) xs[t] = (T)dequant<B0>(code_at<B0>(win, t));
      }
      {  // G1: bilinear over 4 taps, channels g, g+4, ...
        constexpr int NB = C1 * B1, NW = (NB + 31) / 32;
        float acc[IS::n1max];
#pragma unroll
        for (int i = 0; i < IS::n1max; ++i) acc[i] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
          uint32_t win[NW];
          load_bits<NW, NB % 32 == 0>(packed, m.g1_pk[f.j] * 8 + (long long)f.g1_cell[k] * NB, m.g1_pk_end[f.j], win);
#pragma unroll
          for (int i = 0; i < IS::n1max; ++i) {
            const int ch = min(g + 4 * i, C1 - 1);
            acc[i] += f.g1_w[k] * dequant<B1>(code_at_dyn<B1>(win, ch));
          }
        }
#pragma unroll
        for (int i = 0; i < IS::n1max; ++i) xs[C0 + i] = (g + 4 * i < C1) ? (T)acc[i] : (T)0.f;
      }
    } else {
      const long long g0base = m.g0_off[f.j] + (long long)f.g0_cell * C0;
      const long long g1base = m.g1_off[f.j];
#pragma unroll
      for (int t = 0; t < C0; ++t) xs[t] = (T)lat[g0base + t];
#pragma unroll
      for (int i = 0; i < IS::n1max; ++i) {
        const int ch = g + 4 * i;
        float acc = 0.f;
        if (ch < C1) {
#pragma unroll
          for (int k = 0; k < 4; ++k) acc += f.g1_w[k] * lat[g1base + (long long)f.g1_cell[k] * C1 + ch];
        }
        xs[C0 + i] = (T)acc;
      }
    }
    {
      float pv[3];
      pe_values(pe_lds, f.ix, f.iy, g, pv);
#pragma unroll
      for (int k = 0; k < 3; ++k) xs[IS::T_lat + k] = (T)pv[k];
#pragma unroll
      for (int t = IS::T_used; t < S1; ++t) xs[t] = (T)0.f;
    }
    // layer 1
    f32x4 acc[MT];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + 16 * mo + 4 * g);
      acc[mo] = mma_slots<S1>(acc[mo], w_lds + pg.L1 + mo * S1 * 64, xs, lane);
    }
    T h[SH];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo)
#pragma unroll
      for (int i = 0; i < 4; ++i) h[4 * mo + i] = (T)act_fn(acc[mo][i], m.act);
    // layer 2
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + HD + 16 * mo + 4 * g);
      acc[mo] = mma_slots<SH>(acc[mo], w_lds + pg.L2 + mo * SH * 64, h, lane);
    }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo)
#pragma unroll
      for (int i = 0; i < 4; ++i) h[4 * mo + i] = (T)act_fn(acc[mo][i], m.act);
    // layer 3 (no activation): lane group g holds channels 4g .. 4g+3
    f32x4 y = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
    y = mma_slots<SH>(y, w_lds + pg.L3, h, lane);
    if (valid && 4 * g < C) {
      if (out_f16) {
        _Float16* o = reinterpret_cast<_Float16*>(out) + s * C + 4 * g;
        if constexpr (C % 4 == 0) {
          f16x4 hv = {(_Float16)y[0], (_Float16)y[1], (_Float16)y[2], (_Float16)y[3]};
          *reinterpret_cast<f16x4*>(o) = hv;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (4 * g + i < C) o[i] = (_Float16)y[i];
        }
      } else {
        float* o = reinterpret_cast<float*>(out) + s * C + 4 * g;
        if constexpr (C % 4 == 0) {
          *reinterpret_cast<f32x4*>(o) = y;
        } else {
#pragma unroll
          for (int i = 0; i < 4; ++i)
            if (4 * g + i < C) o[i] = y[i];
        }
      }
    }
  }
}

template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED>
static hipError_t decode_t(const ntc_material& mm, const void* src, const void* wpack, const ntc_query* q,
                           long long n, void* out, bool out_f16, hipStream_t s) {
  constexpr PackGeom pg = pack_geom(C0, C1, HD, sizeof(T) == 2);
  constexpr int WB = ((int)pg.fwd_end * (int)sizeof(T) + 15) / 16 * 16;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4;
  const float* bias = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wpack) + WB);
  auto kern = decode_kernel<T, C0, C1, C, HD, B0, B1, PACKED>;
  static int per_cu = 0;
  if (per_cu == 0) {
    int v = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&v, kern, 256, lds) != hipSuccess || v < 1) v = 1;
    per_cu = v;
  }
  const long long tiles = (n + 15) / 16;
  long long grid = (tiles + 3) / 4;
  const long long cap = (long long)device_cus() * per_cu;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, dev_mat(mm), pe_table(), src,
                     reinterpret_cast<const T*>(wpack), bias, q, n, out, out_f16 ? 1 : 0);
  return hipGetLastError();
}

#define NTC_DECODE_SHAPES(X)                                                                     \
  X(8, 8, 8, 64, 4, 4) X(10, 10, 10, 64, 4, 4) X(12, 12, 12, 64, 4, 4) X(16, 16, 16, 64, 4, 4)  \
  X(8, 8, 8, 32, 4, 4) X(10, 10, 10, 32, 4, 4) X(12, 12, 12, 32, 4, 4) X(16, 16, 16, 32, 4, 4)  \
  X(16, 16, 16, 64, 2, 4)

bool decode_shape_supported(int c0, int c1, int c, int hd, int b0, int b1) {
#define NTC_X(a, b, cc, h, x0, x1) \
  if (c0 == a && c1 == b && c == cc && hd == h && b0 == x0 && b1 == x1) return true;
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return false;
}

hipError_t launch_decode(const ntc_material& m, const uint8_t* packed, const void* wpack, bool f16, const ntc_query* q,
                         long long n, void* out, bool out_f16, hipStream_t s) {
#define NTC_X(a, b, cc, h, x0, x1)                                                                   \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h && m.b0 == x0 && m.b1 == x1)      \
    return f16 ? decode_t<_Float16, a, b, cc, h, x0, x1, true>(m, packed, wpack, q, n, out, out_f16, s)   \
               : decode_t<float, a, b, cc, h, x0, x1, true>(m, packed, wpack, q, n, out, out_f16, s);
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

// Forward from FP32 latents (the differentiation path); shapes as for training.
#define NTC_FORWARD_SHAPES(X)                                                          \
  X(8, 8, 8, 64) X(10, 10, 10, 64) X(12, 12, 12, 64) X(16, 16, 16, 64) X(8, 8, 8, 32) \
  X(10, 10, 10, 32) X(12, 12, 12, 32) X(16, 16, 16, 32)

hipError_t launch_forward(const ntc_material& m, const float* latents, const void* wpack, bool f16, const ntc_query* q,
                          long long n, float* out, hipStream_t s) {
#define NTC_X(a, b, cc, h)                                                                                  \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h)                                          \
    return f16 ? decode_t<_Float16, a, b, cc, h, 4, 4, false>(m, latents, wpack, q, n, out, false, s)       \
               : decode_t<float, a, b, cc, h, 4, 4, false>(m, latents, wpack, q, n, out, false, s);
  NTC_FORWARD_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

}  // namespace ntc
