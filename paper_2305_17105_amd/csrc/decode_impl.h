// Random-access decode kernels (sections 4.3-4.4): packed latents -> all C channels
// per texel, shared by the single-material and grouped launchers.
//
// Persistent kernel, 4 wavefronts per block, one 16-texel tile per wavefront
// iteration.  Each of the 4 lane groups of a texel fetches one G0 neighbour cell
// (a contiguous C0*B0-bit window), a quarter of the G1 bilinear channels and 3 of
// the 12 positional-encoding values, so the MLP input is assembled directly in the
// B-operand layout of the matrix cores.  The three layers chain through registers;
// weights are staged once per block in LDS.
#pragma once
#include "ntc_internal.h"

namespace ntc {

// Shapes (c0, c1, channels, hidden, b0, b1) with decode kernels: the configurations' shapes
// and Table 3's four profiles on a 9-channel texture set (NTC 0.2, 0.5, 1.0, 2.25).
#define NTC_DECODE_SHAPES(X)                                                                     \
  X(8, 8, 8, 64, 4, 4) X(10, 10, 10, 64, 4, 4) X(12, 12, 12, 64, 4, 4) X(16, 16, 16, 64, 4, 4)  \
  X(8, 8, 8, 32, 4, 4) X(10, 10, 10, 32, 4, 4) X(12, 12, 12, 32, 4, 4) X(16, 16, 16, 32, 4, 4)  \
  X(16, 16, 16, 64, 2, 4)                                                                        \
  X(8, 12, 9, 64, 2, 4) X(12, 20, 9, 64, 4, 4) X(12, 10, 9, 64, 2, 4) X(16, 12, 9, 64, 4, 4)

// Input layout of the decoder for a material: packed codes in FP16 use the paired
// layout where it applies; everything else (and the forward of the differentiation
// path, which shares the training pack) the plain one.
template <typename T, int C0, int C1, int HD, int B0, int B1, bool PACKED>
struct DecodeLayout {
  static constexpr bool paired = PACKED && paired_layout(C0, C1, B0, B1, sizeof(T) == 2);
  static constexpr PackGeom pg = PACKED ? pack_geom_decode(C0, C1, B0, B1, HD, sizeof(T) == 2)
                                        : pack_geom(C0, C1, HD, sizeof(T) == 2);
  static constexpr int WB = ((int)pg.fwd_end * (int)sizeof(T) + 15) / 16 * 16;
  // Point decode of the paired layout locates each texel once: every lane of a wavefront
  // takes one texel of a 64-texel group, gathers its four G0 neighbour windows and four
  // G1 taps, forms the G1 pairs of all four lane groups and leaves them in a per-wavefront
  // slab of LDS, SW words per texel (odd: consecutive texels fall in different banks).
  static constexpr int NW0 = (C0 * B0 + 31) / 32, NW1 = (C1 * B1 + 31) / 32;
  static constexpr int NP = paired ? NW1 * (4 / B1) : 0;  // G1 pairs of one lane group
  static constexpr int GW = NW0 + NP;                     // words of one lane group
  static constexpr int SW = (4 * GW + 1) | 1;             // + the texel's PE / LOD word
  static constexpr int SLAB = paired ? 4 * 64 * SW * 4 : 0;  // bytes, 4 wavefronts
};

// Two codes of one 32-bit word (bit offsets s and s + 16) as FP16 values 1024 + code:
// OR-ing the exponent of 1024 over a code of at most 10 bits is the exact conversion.
template <int B>
__device__ inline f16x2 code_pair(uint32_t w, int s) {
  constexpr uint32_t cm = (1u << B) - 1u, pm = cm | (cm << 16);
  return __builtin_bit_cast(f16x2, ((w >> s) & pm) | 0x64006400u);
}

// Byte offsets of one feature level's packed grids and of their last dwords (the
// packed latents of a decodable material are below 4 GiB, see ntc_decode), kept in
// LDS so a per-lane level index reads them directly.
struct LevelBytes {
  uint32_t g0, g1, g0_last, g1_last;
};
__device__ inline void fill_level_bytes(const DevMat& m, LevelBytes* lb, int tid, int nthreads) {
  for (int j = tid; j < kMaxLevels; j += nthreads) {
    LevelBytes b;
    b.g0 = (uint32_t)m.g0_pk[j];
    b.g1 = (uint32_t)m.g1_pk[j];
    b.g0_last = (uint32_t)(m.g0_pk_end[j] * 4);
    b.g1_last = (uint32_t)(m.g1_pk_end[j] * 4);
    lb[j] = b;
  }
}

// NW dwords of the code window of `cell` (NB bits per cell) in a grid at byte `base`,
// with 32-bit byte offsets from the packed-latent pointer (loads through a scalar base).
// The packed latents are global memory: the explicit address space keeps the loads
// global (not flat) even when the pointer came from a table in memory.
typedef const __attribute__((address_space(1))) char gbyte;
template <typename W>
__device__ inline W gload(gbyte* p) {
  return *reinterpret_cast<const __attribute__((address_space(1))) W*>(p);
}
template <int NW, int NB>
__device__ inline void load_window(gbyte* __restrict__ packed, uint32_t base, uint32_t cell, uint32_t last,
                                   uint32_t (&out)[NW]) {
  if constexpr (NB % 64 == 0) {  // whole 8-byte units (grid bases are 16-byte aligned)
    const uint32_t b0 = base + cell * (uint32_t)(NB / 8);
#pragma unroll
    for (int k = 0; k < NW / 2; ++k) {
      const unsigned long long w = gload<unsigned long long>(packed + (b0 + 8u * k));
      out[2 * k] = (uint32_t)w;
      out[2 * k + 1] = (uint32_t)(w >> 32);
    }
  } else if constexpr (NB % 32 == 0) {
    const uint32_t b0 = base + cell * (uint32_t)(NB / 8);
#pragma unroll
    for (int k = 0; k < NW; ++k) out[k] = gload<uint32_t>(packed + (b0 + 4u * k));
  } else {
    const uint64_t bit = (uint64_t)cell * NB;
    const uint32_t b0 = base + (uint32_t)(bit >> 5) * 4u, s = (uint32_t)bit & 31u;
    uint32_t w[NW + 1];
#pragma unroll
    for (int k = 0; k <= NW; ++k) w[k] = gload<uint32_t>(packed + min(b0 + 4u * k, last));
#pragma unroll
    for (int k = 0; k < NW; ++k) out[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], s);
  }
}

// The bit-packed code words one texel's lane group needs (its G0 neighbour cell and
// the four G1 taps) plus what the input assembly needs from the footprint.
template <int C0, int C1, int B0, int B1>
struct CodeWindow {
  static constexpr int NB0 = C0 * B0, NW0 = (NB0 + 31) / 32, NB1 = C1 * B1, NW1 = (NB1 + 31) / 32;
  int ix, iy, l;
  float fx, fy, w[4];
  uint32_t g0[NW0];
  uint32_t g1[4][NW1];
  __device__ inline void fetch(const DevMat& m, const LevelBytes* __restrict__ lb, const uint32_t* __restrict__ packed,
                               float u, float v, int lod, int g) {
    const Footprint f = locate(m, u, v, lod, g);
    ix = f.ix;
    iy = f.iy;
    l = f.l;
    fx = f.fx;
    fy = f.fy;
#pragma unroll
    for (int k = 0; k < 4; ++k) w[k] = f.g1_w[k];
    const LevelBytes b = lb[f.j];
    gbyte* pk = (gbyte*)reinterpret_cast<const char*>(packed);
    load_window<NW0, NB0>(pk, b.g0, (uint32_t)f.g0_cell, b.g0_last, g0);
#pragma unroll
    for (int k = 0; k < 4; ++k) load_window<NW1, NB1>(pk, b.g1, (uint32_t)f.g1_cell[k], b.g1_last, g1[k]);
  }
};

// G1 bilinear of the paired layout: pair p = d * (4/B1) + kk holds channels
// d*32/B1 + g + 4kk and that + 16/B1.  Separable, in centred code units: the row steps
// are exact, the column step rounds once, the power-of-two scale is exact, so the
// result equals the FP16 rounding of the exact bilinear value.
template <int NW1, int B1>
__device__ inline void g1_pairs_words(const uint32_t (&w1)[4][NW1], float gfx, float gfy, int g,
                                      f16x2 (&out)[NW1 * (4 / B1)]) {
  constexpr int KP = 4 / B1, N1 = 1 << B1;
  const f16x2 fx = {(_Float16)gfx, (_Float16)gfx}, fy = {(_Float16)gfy, (_Float16)gfy};
  const _Float16 o = (_Float16)(-(1024.f + N1 / 2 - 1));
  const f16x2 of = {o, o};
  const f16x2 sc = {(_Float16)(1.f / N1), (_Float16)(1.f / N1)};
#pragma unroll
  for (int d = 0; d < NW1; ++d)
#pragma unroll
    for (int kk = 0; kk < KP; ++kk) {
      const int sh = B1 * (g + 4 * kk);
      const f16x2 x0 = code_pair<B1>(w1[0][d], sh), x1 = code_pair<B1>(w1[1][d], sh);
      const f16x2 x2 = code_pair<B1>(w1[2][d], sh), x3 = code_pair<B1>(w1[3][d], sh);
      const f16x2 r0 = __builtin_elementwise_fma(fx, x1 - x0, x0 + of);
      const f16x2 r1 = __builtin_elementwise_fma(fx, x3 - x2, x2 + of);
      out[d * KP + kk] = __builtin_elementwise_fma(fy, r1 - r0, r0) * sc;
    }
}
template <int C0, int C1, int B0, int B1>
__device__ inline void g1_pairs(const CodeWindow<C0, C1, B0, B1>& R, int g,
                                f16x2 (&out)[CodeWindow<C0, C1, B0, B1>::NW1 * (4 / B1)]) {
  g1_pairs_words<CodeWindow<C0, C1, B0, B1>::NW1, B1>(R.g1, R.fx, R.fy, g, out);
}

// The code words of one texel for the grouped gather: the four G0 neighbour windows
// (order (x0,y0), (x0+1,y0), (x0,y0+1), (x0+1,y0+1)) and the four G1 taps, plus what the
// input assembly needs from the footprint.
template <int C0, int C1, int B0, int B1>
struct TexelCodes {
  static constexpr int NB0 = C0 * B0, NW0 = (NB0 + 31) / 32, NB1 = C1 * B1, NW1 = (NB1 + 31) / 32;
  int ix, iy, l;
  float fx, fy;
  uint32_t g0[4][NW0];
  uint32_t g1[4][NW1];
  __device__ inline void fetch(const DevMat& m, const LevelBytes* __restrict__ lb, const uint32_t* __restrict__ packed,
                               float u, float v, int lod) {
    const Footprint f = locate(m, u, v, lod, 0);
    ix = f.ix;
    iy = f.iy;
    l = f.l;
    fx = f.fx;
    fy = f.fy;
    const int w0 = m.W >> (m.shift + 2 * f.j);
    const LevelBytes b = lb[f.j];
    gbyte* pk = (gbyte*)reinterpret_cast<const char*>(packed);
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int cell = ((g >> 1) ? f.by : f.ay) * w0 + ((g & 1) ? f.bx : f.ax);
      load_window<NW0, NB0>(pk, b.g0, (uint32_t)cell, b.g0_last, g0[g]);
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) load_window<NW1, NB1>(pk, b.g1, (uint32_t)f.g1_cell[k], b.g1_last, g1[k]);
  }
};

// Latent slots of the paired FP16 layout from a code window: G0 two channels per
// instruction ((1024 + code) / N - (N/2 - 1 + 1024) / N is exact), then the G1 pairs.
template <int NW0, int B0, int S1>
__device__ inline void paired_g0(const uint32_t (&w0)[NW0], _Float16 (&xs)[S1]) {
  constexpr int HALF = 16 / B0, N0 = 1 << B0;
  const f16x2 sc = {(_Float16)(1.f / N0), (_Float16)(1.f / N0)};
  const _Float16 o = (_Float16)(-(1024.f + N0 / 2 - 1) / N0);
  const f16x2 of = {o, o};
#pragma unroll
  for (int d = 0; d < NW0; ++d)
#pragma unroll
    for (int c = 0; c < HALF; ++c) {
      const f16x2 x = __builtin_elementwise_fma(code_pair<B0>(w0[d], B0 * c), sc, of);
      xs[2 * (d * HALF + c)] = x[0];
      xs[2 * (d * HALF + c) + 1] = x[1];
    }
}
template <int C0, int C1, int B0, int B1, int S1>
__device__ inline void paired_inputs(const CodeWindow<C0, C1, B0, B1>& R, int g, _Float16 (&xs)[S1]) {
  using Raw = CodeWindow<C0, C1, B0, B1>;
  paired_g0<Raw::NW0, B0>(R.g0, xs);
  f16x2 v[Raw::NW1 * (4 / B1)];
  g1_pairs(R, g, v);
  constexpr int G0S = paired_g0_slots(C0, B0);
#pragma unroll
  for (int p = 0; p < Raw::NW1 * (4 / B1); ++p) {
    xs[G0S + 2 * p] = v[p][0];
    xs[G0S + 2 * p + 1] = v[p][1];
  }
}

// Lane group g's four output channels 4g .. 4g+3 of texel s.
template <int C>
__device__ inline void store_out(void* __restrict__ out, int out_f16, long long s, long long n, int g, f32x4 y) {
  if (s >= n || 4 * g >= C) return;
  if (out_f16) {
    _Float16* o = reinterpret_cast<_Float16*>(out) + s * C + 4 * g;
    if constexpr (C % 4 == 0) {
      *reinterpret_cast<f16x4*>(o) = __builtin_convertvector(y, f16x4);
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

// Filtered decode (section 5.3): texel filtering done in software by decoding the
// texels it combines.  FILT 1: bilinear, the 4 texels around (u, v) in the nearest mip;
// FILT 2: trilinear, bilinear in the two mips around lod blended by its fraction (8
// texels); FILT 3: stochastic, one texel after a uniform jitter of (u, v) by up to half
// a texel and a random choice between the two mips around lod.  TAPS texels feed one
// output; tap k of output s at position (u, v), integer mip lod, weight wt.
template <int FILT>
constexpr int filter_taps() { return FILT == 1 ? 4 : FILT == 2 ? 8 : 1; }

constexpr uint64_t kFilterTag = 0x66696C74ull;  // "filt"

// Bilinear tap k (dx = k & 1, dy = k >> 1) of (fu, fv) in mip l: texel centre and weight.
__device__ inline void bilinear_tap(const DevMat& m, float fu, float fv, int l, int k, float& u, float& v,
                                    float& wt) {
  const int W = m.mip_w[l], H = m.mip_h[l];
  const float x = fu * (float)W - 0.5f, y = fv * (float)H - 0.5f;
  const float x0 = floorf(x), y0 = floorf(y);
  const float fx = x - x0, fy = y - y0;
  const int xi = min(max((int)x0 + (k & 1), 0), W - 1), yi = min(max((int)y0 + (k >> 1), 0), H - 1);
  u = ((float)xi + 0.5f) / (float)W;
  v = ((float)yi + 0.5f) / (float)H;
  wt = ((k & 1) ? fx : 1.f - fx) * ((k >> 1) ? fy : 1.f - fy);
}

template <int FILT>
__device__ inline void filter_tap(const DevMat& m, const ntc_filter_query& fq, long long s, int k, uint64_t key,
                                  float& u, float& v, int& lod, float& wt) {
  float fu = fq.u, fv = fq.v;
  if (!(fu == fu)) fu = 0.f;  // NaN -> 0, as for point queries
  if (!(fv == fv)) fv = 0.f;
  const float lf = fminf(fmaxf(fq.lod, 0.f), (float)(m.M - 1));  // NaN -> 0
  const int l0 = (int)floorf(lf);
  if constexpr (FILT == 1) {
    lod = min((int)floorf(lf + 0.5f), m.M - 1);
    bilinear_tap(m, fu, fv, lod, k, u, v, wt);
  } else if constexpr (FILT == 2) {
    const int l1 = min(l0 + 1, m.M - 1);
    const float t = lf - (float)l0;
    lod = k < 4 ? l0 : l1;
    bilinear_tap(m, fu, fv, lod, k & 3, u, v, wt);
    wt *= k < 4 ? 1.f - t : t;
  } else {
    const uint64_t h1 = mix64(key + kGamma * (uint64_t)(2 * s + 1)), h2 = mix64(key + kGamma * (uint64_t)(2 * s + 2));
    const float r1 = (float)(uint32_t)(h1 >> 40) * 0x1p-24f, r2 = (float)(uint32_t)((h1 >> 16) & 0xFFFFFFu) * 0x1p-24f;
    const float r3 = (float)(uint32_t)(h2 >> 40) * 0x1p-24f;
    lod = min(l0 + (r3 < lf - (float)l0 ? 1 : 0), m.M - 1);
    u = fu + (r1 - 0.5f) / (float)m.mip_w[lod];
    v = fv + (r2 - 0.5f) / (float)m.mip_h[lod];
    wt = 1.f;
  }
}

// FP16 weight A-fragments of one layer (MTN M-tiles of S slots) held in registers, in
// the pack's operand order: S/8 fragments of 8 slots per M-tile and a 4-slot tail.
template <int S, int MTN>
struct RegLayer {
  static constexpr int S8 = S / 8, NF = S8 > 0 ? S8 : 1;
  static constexpr bool TAIL = S % 8 != 0;
  f16x8 a[MTN][NF];
  f16x4 t[MTN];
  __device__ inline void load(const _Float16* __restrict__ w, int lane) {
#pragma unroll
    for (int mo = 0; mo < MTN; ++mo) {
#pragma unroll
      for (int k = 0; k < S8; ++k) a[mo][k] = *reinterpret_cast<const f16x8*>(w + mo * S * 64 + k * 512 + lane * 8);
      if constexpr (TAIL) t[mo] = *reinterpret_cast<const f16x4*>(w + mo * S * 64 + S8 * 512 + lane * 4);
    }
  }
  // acc += A(mo) * B over the S slots of b (as mma_slots, including its separate tail)
  __device__ inline f32x4 mma(f32x4 acc, int mo, const _Float16 (&b)[S]) const {
#pragma unroll
    for (int k = 0; k < S8; ++k) {
      f16x8 bv;
#pragma unroll
      for (int j = 0; j < 8; ++j) bv[j] = b[8 * k + j];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(a[mo][k], bv, acc, 0, 0, 0);
    }
    if constexpr (TAIL) {
      f16x4 bv;
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = b[8 * S8 + j];
      const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
      acc += __builtin_amdgcn_mfma_f32_16x16x16f16(t[mo], bv, zero, 0, 0, 0);
    }
    return acc;
  }
};

// PACKED: latents come as bit-packed codes (ntc_decode); otherwise as FP32 values
// in the canonical latent layout (ntc_forward, the differentiation path).
// bias: b1 (HD), b2 (HD), b3 (C) at the three given addresses.
// bi, nb: this block's index among the nb blocks that share the n queries.
// FILT (packed codes only): 0 point queries (ntc_query), else the filter above over n
// outputs of ntc_filter_query records; fkey: the stochastic filter's counter key.
template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED, int ACT, int FILT = 0>
__device__ __forceinline__ void decode_body(const DevMat& m, const PeTable& pe, const void* __restrict__ src,
                                            const T* __restrict__ wpack, const float* __restrict__ bias1,
                                            const float* __restrict__ bias2, const float* __restrict__ bias3,
                                            const ntc_query* __restrict__ q, long long n, const TexelRect& rect,
                                            void* __restrict__ out, int out_f16, int bi, int nb,
                                            uint64_t fkey = 0) {
  static_assert(FILT == 0 || PACKED, "filtered decode reads packed codes");
  constexpr int TAPS = filter_taps<FILT>();
  const uint32_t* __restrict__ packed = reinterpret_cast<const uint32_t*>(src);
  const float* __restrict__ lat = reinterpret_cast<const float*>(src);
  using IS = InSlots<C0, C1>;
  using DL = DecodeLayout<T, C0, C1, HD, B0, B1, PACKED>;
  constexpr PackGeom pg = DL::pg;
  constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT, WB = DL::WB;
  extern __shared__ __align__(16) char smem[];
  T* w_lds = reinterpret_cast<T*>(smem);
  float* pe_lds = reinterpret_cast<float*>(smem + WB);
  float* b_lds = pe_lds + 48;  // b1 (HD), b2 (HD), b3 (C, zero-padded to 16)
  LevelBytes* lb = reinterpret_cast<LevelBytes*>(b_lds + 2 * HD + 16);
  fill_level_bytes(m, lb, threadIdx.x, blockDim.x);

  for (int i = threadIdx.x; i < WB / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(smem)[i] = reinterpret_cast<const uint4*>(wpack)[i];
  for (int i = threadIdx.x; i < 48; i += blockDim.x) pe_lds[i] = pe.v[i / 6][i % 6];
  for (int i = threadIdx.x; i < 2 * HD + 16; i += blockDim.x)
    b_lds[i] = i < HD ? bias1[i] : i < 2 * HD ? bias2[i - HD] : i < 2 * HD + C ? bias3[i - 2 * HD] : 0.f;
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const long long tiles = (n * TAPS + 15) / 16, stride = (long long)nb * 4;

  // three layers on one tile's assembled inputs, then the store (filters: the weighted
  // taps of an output are summed across its TAPS lanes first)
  auto mlp_store = [&](T (&xs)[S1], long long tile, float wt) {
    const long long s = tile * (16 / TAPS) + r / TAPS;
    f32x4 acc[MT];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + 16 * mo + 4 * g);
      acc[mo] = mma_slots<S1>(acc[mo], w_lds + pg.L1 + mo * S1 * 64, xs, lane);
    }
    T h[SH];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + HD + 16 * mo + 4 * g);
      acc[mo] = mma_slots<SH>(acc[mo], w_lds + pg.L2 + mo * SH * 64, h, lane);
    }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
    // layer 3 (no activation): lane group g holds channels 4g .. 4g+3
    f32x4 y = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
    y = mma_slots<SH>(y, w_lds + pg.L3, h, lane);
    if constexpr (TAPS > 1) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        float t = y[i] * wt;
#pragma unroll
        for (int o = 1; o < TAPS; o <<= 1) t += __shfl_xor(t, o);
        y[i] = t;
      }
      if (r % TAPS != 0) return;
    }
    store_out<C>(out, out_f16, s, n, g, y);
  };
  // LOD input (section 4.4): mip l / (M - 1) in group 0's slot after the encoding
  const float lod_norm = m.lod_in && m.M > 1 ? 1.f / (float)(m.M - 1) : 0.f;
  auto pe_slots = [&](T (&xs)[S1], int ix, int iy, int l) {
    float pv[3];
    pe_values(pe_lds, ix, iy, g, pv);
#pragma unroll
    for (int k = 0; k < 3; ++k) xs[pg.T_lat + k] = (T)pv[k];
    xs[pg.T_lat + 3] = (T)(g == 0 ? (float)l * lod_norm : 0.f);
#pragma unroll
    for (int t = pg.T_used; t < S1; ++t) xs[t] = (T)0.f;
  };
  // query record of this lane's texel of a tile (zeros past the end)
  auto load_query = [&](long long tile, float& u, float& v, int& lod, float& wt) {
    u = v = 0.f;
    lod = 0;
    wt = 1.f;
    if constexpr (FILT == 0) {
      const long long s = tile * 16 + r;
      if (tile < tiles && s < n) {
        if (rect.w > 0) {
          rect_query(rect, s, u, v, lod);
        } else {
          u = q[s].u;
          v = q[s].v;
          lod = q[s].lod;
        }
      }
    } else {
      const long long s = tile * (16 / TAPS) + r / TAPS;
      if (tile < tiles && s < n)
        filter_tap<FILT>(m, reinterpret_cast<const ntc_filter_query*>(q)[s], s, r % TAPS, fkey, u, v, lod, wt);
    }
  };

  if constexpr (PACKED && FILT == 0 && DL::paired) {
    // Point decode, one texel per lane: a wavefront takes 64 consecutive texels (four
    // 16-texel tiles) at a time.  Each lane locates its texel once and gathers its code
    // words (the next group's while the current group runs through the matrix cores),
    // then leaves the G0 windows and the G1 pairs of all four lane groups in the
    // wavefront's slab; lane (g, r) of tile k reads back texel 16k + r's group-g words.
    using TC = TexelCodes<C0, C1, B0, B1>;
    constexpr int NW0 = DL::NW0, NP = DL::NP, GW = DL::GW, SW = DL::SW;
    constexpr int G0S = paired_g0_slots(C0, B0);
    uint32_t* slab = reinterpret_cast<uint32_t*>(lb + kMaxLevels) + wave * 64 * SW;
    const long long groups = (n + 63) / 64;
    auto load_texel = [&](long long grp, float& u, float& v, int& lod) {
      u = v = 0.f;
      lod = 0;
      const long long s = grp * 64 + lane;
      if (grp < groups && s < n) {
        if (rect.w > 0) {
          rect_query(rect, s, u, v, lod);
        } else {
          u = q[s].u;
          v = q[s].v;
          lod = q[s].lod;
        }
      }
    };
    // the three layers' weights in registers for the whole kernel (the slab's stores
    // would otherwise keep the compiler from hoisting their LDS loads out of the loop);
    // measured faster than layer 1 only (3 wavefronts per SIMD either way) and than
    // weights read from LDS per tile (5 wavefronts per SIMD, 22 KiB of LDS reads a tile)
    RegLayer<S1, MT> r1;
    RegLayer<SH, MT> r2;
    RegLayer<SH, 1> r3;
    r1.load(w_lds + pg.L1, lane);
    r2.load(w_lds + pg.L2, lane);
    r3.load(w_lds + pg.L3, lane);
    auto mlp_store_reg = [&](T (&xs)[S1], long long tile) {
      const long long s = tile * 16 + r;
      f32x4 acc[MT];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + 16 * mo + 4 * g);
        acc[mo] = r1.mma(acc[mo], mo, xs);
      }
      T h[SH];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + HD + 16 * mo + 4 * g);
        acc[mo] = r2.mma(acc[mo], mo, h);
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
      f32x4 y = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
      y = r3.mma(y, 0, h);
      store_out<C>(out, out_f16, s, n, g, y);
    };
    long long grp = (long long)bi * 4 + wave;
    if (grp >= groups) return;
    float u, v;
    int lod;
    load_texel(grp, u, v, lod);
    TC cur;
    cur.fetch(m, lb, packed, u, v, lod);
    load_texel(grp + stride, u, v, lod);
    for (; grp < groups; grp += stride) {
      {
        uint32_t* my = slab + lane * SW;
#pragma unroll
        for (int gg = 0; gg < 4; ++gg) {
          f16x2 pr[NP];
          g1_pairs_words<DL::NW1, B1>(cur.g1, cur.fx, cur.fy, gg, pr);
#pragma unroll
          for (int w = 0; w < NW0; ++w) my[gg * GW + w] = cur.g0[gg][w];
#pragma unroll
          for (int p = 0; p < NP; ++p) my[gg * GW + NW0 + p] = __builtin_bit_cast(uint32_t, pr[p]);
        }
        my[4 * GW] = (uint32_t)(cur.ix & 7) | ((uint32_t)(cur.iy & 7) << 3) | ((uint32_t)cur.l << 6);
      }
      // LDS operations of a wavefront complete in order: the reads below see the writes
      // above; the barrier keeps the compiler from moving memory operations across it
      __builtin_amdgcn_wave_barrier();
      TC nxt;
      if (grp + stride < groups) nxt.fetch(m, lb, packed, u, v, lod);
      if (grp + 2 * stride < groups) load_texel(grp + 2 * stride, u, v, lod);
      // the inputs of tile k: lane (g, r) reads texel 16k + r's group-g words
      auto assemble_tile = [&](int k, T (&xs)[S1]) {
        const uint32_t* rd = slab + (16 * k + r) * SW;
        uint32_t w0[NW0];
#pragma unroll
        for (int w = 0; w < NW0; ++w) w0[w] = rd[g * GW + w];
        paired_g0<NW0, B0>(w0, xs);
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const f16x2 pv = __builtin_bit_cast(f16x2, rd[g * GW + NW0 + p]);
          xs[G0S + 2 * p] = pv[0];
          xs[G0S + 2 * p + 1] = pv[1];
        }
        const uint32_t meta = rd[4 * GW];
        pe_slots(xs, (int)(meta & 7u), (int)((meta >> 3) & 7u), (int)(meta >> 6));
      };
      {
#pragma unroll 1
        for (int k = 0; k < 4; ++k) {
          const long long tile = grp * 4 + k;
          if (tile * 16 >= n) break;  // wavefront-uniform
          T xs[S1];
          assemble_tile(k, xs);
          mlp_store_reg(xs, tile);
        }
      }
      cur = nxt;
      __builtin_amdgcn_wave_barrier();  // this group's slab reads precede the next group's writes
    }
  } else if constexpr (PACKED) {
    // Software pipeline over the wave's tiles: queries two tiles ahead, latent words
    // one tile ahead, so both gathers are in flight while the matrix cores run.
    using Raw = CodeWindow<C0, C1, B0, B1>;
    auto assemble = [&](const Raw& R, T (&xs)[S1]) {
      if constexpr (DL::paired) {
        paired_inputs(R, g, xs);
      } else {
#pragma unroll
        for (int t = 0; t < C0; ++t) xs[t] = (T)dequant<B0>(code_at<B0>(R.g0, t));
        // G1: bilinear over 4 taps, channels g, g+4, ...
        float acc[IS::n1max];
#pragma unroll
        for (int i = 0; i < IS::n1max; ++i) acc[i] = 0.f;
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
          for (int i = 0; i < IS::n1max; ++i) {
            const int ch = min(g + 4 * i, C1 - 1);
            acc[i] += R.w[k] * dequant<B1>(code_at_dyn<B1>(R.g1[k], ch));
          }
#pragma unroll
        for (int i = 0; i < IS::n1max; ++i) xs[C0 + i] = (g + 4 * i < C1) ? (T)acc[i] : (T)0.f;
      }
      pe_slots(xs, R.ix, R.iy, R.l);
    };

    long long tile = (long long)bi * 4 + wave;
    if (tile >= tiles) return;
    float u, v, wt;
    int lod;
    load_query(tile, u, v, lod, wt);
    Raw cur;
    cur.fetch(m, lb, packed, u, v, lod, g);
    float cwt = wt;
    load_query(tile + stride, u, v, lod, wt);
    for (; tile < tiles; tile += stride) {
      Raw nxt;
      float nwt = wt;
      if (tile + stride < tiles) nxt.fetch(m, lb, packed, u, v, lod, g);
      if (tile + 2 * stride < tiles) load_query(tile + 2 * stride, u, v, lod, wt);
      T xs[S1];
      assemble(cur, xs);
      mlp_store(xs, tile, cwt);
      cur = nxt;
      cwt = nwt;
    }
  } else {
    for (long long tile = (long long)bi * 4 + wave; tile < tiles; tile += stride) {
      float u, v, wt;
      int lod;
      load_query(tile, u, v, lod, wt);
      const Footprint f = locate(m, u, v, lod, g);
      T xs[S1];
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
      pe_slots(xs, f.ix, f.iy, f.l);
      mlp_store(xs, tile, wt);
    }
  }
}

template <typename T, int C0, int C1, int C, int HD, int B0, int B1, bool PACKED, int ACT>
__global__ __launch_bounds__(256) void decode_kernel(DevMat m, PeTable pe, const void* __restrict__ src,
                                                     const T* __restrict__ wpack, const float* __restrict__ bias1,
                                                     const float* __restrict__ bias2,
                                                     const float* __restrict__ bias3,
                                                     const ntc_query* __restrict__ q, long long n,
                                                     TexelRect rect, void* __restrict__ out, int out_f16) {
  decode_body<T, C0, C1, C, HD, B0, B1, PACKED, ACT>(m, pe, src, wpack, bias1, bias2, bias3, q, n, rect, out, out_f16,
                                                     blockIdx.x, gridDim.x);
}

template <typename T, int C0, int C1, int C, int HD, int B0, int B1, int ACT, int FILT>
__global__ __launch_bounds__(256) void decode_filtered_kernel(DevMat m, PeTable pe, const void* __restrict__ src,
                                                              const T* __restrict__ wpack,
                                                              const ntc_filter_query* __restrict__ fq, long long n,
                                                              uint64_t key, void* __restrict__ out, int out_f16) {
  constexpr int WB = DecodeLayout<T, C0, C1, HD, B0, B1, true>::WB;
  const float* b1 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wpack) + WB);
  decode_body<T, C0, C1, C, HD, B0, B1, true, ACT, FILT>(m, pe, src, wpack, b1, b1 + HD, b1 + 2 * HD,
                                                         reinterpret_cast<const ntc_query*>(fq), n, TexelRect{}, out,
                                                         out_f16, blockIdx.x, gridDim.x, key);
}

// Segment of a grouped launch holding block b: the last one whose first block is <= b.
__device__ inline int group_segment(const GroupArgs& ga) {
  int s = 0;
  while (s + 1 < ga.count && (int)blockIdx.x >= ga.seg[s + 1].block0) ++s;
  return s;
}

// Grouped decode: every block belongs to one material's segment of the launch and
// decodes that material's queries with its blocks; weights (biases appended) come
// from the material's decode pack.
template <typename T, int C0, int C1, int C, int HD, int B0, int B1, int ACT>
__global__ __launch_bounds__(256) void decode_grouped_kernel(const char* __restrict__ table, PeTable pe,
                                                             GroupArgs ga, const ntc_query* __restrict__ q,
                                                             char* __restrict__ out, int out_f16) {
  constexpr int WB = DecodeLayout<T, C0, C1, HD, B0, B1, true>::WB;
  if (*reinterpret_cast<const unsigned long long*>(table) != ga.hash) return;
  const GroupEntry* __restrict__ tab = reinterpret_cast<const GroupEntry*>(table + kGroupHeaderBytes);
  const int s = group_segment(ga);
  const GroupSeg sg = ga.seg[s];
  const GroupEntry& e = tab[sg.mat];
  const T* wp = as_global(reinterpret_cast<const T*>(e.wpack));
  const float* b1 = reinterpret_cast<const float*>(reinterpret_cast<const char*>(wp) + WB);
  const int nb = (s + 1 < ga.count ? ga.seg[s + 1].block0 : ga.blocks) - sg.block0;
  decode_body<T, C0, C1, C, HD, B0, B1, true, ACT>(e.m, pe, as_global(e.packed), wp, b1,
                                                   b1 + HD, b1 + 2 * HD, q + sg.q0, sg.n, TexelRect{},
                                                   out + sg.o0 * (out_f16 ? 2 : 4), out_f16,
                                                   (int)blockIdx.x - sg.block0, nb);
}

// Mixed-material decode (Appendix A): the queries of a tile may name different
// materials of one shape.  Each lane gathers its own material's codes (geometry and
// packed latents per lane, per-material level offsets in LDS); then the wave loops
// over the tile's distinct materials, broadcasting one per iteration and running the
// three layers with that material's weights (read straight from its pack, which L1
// and L2 keep), and stores the texels of that material.  FP16 packs (paired layout).
template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
__global__ __launch_bounds__(256) void decode_mixed_kernel(const char* __restrict__ table, PeTable pe,
                                                           unsigned long long hash, int nmat,
                                                           const ntc_mixed_query* __restrict__ q, long long n,
                                                           void* __restrict__ out, int out_f16) {
  using T = _Float16;
  using DL = DecodeLayout<T, C0, C1, HD, B0, B1, true>;
  static_assert(DL::paired, "mixed decode reads the paired layout");
  constexpr PackGeom pg = DL::pg;
  constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT, WB = DL::WB;
  using Raw = CodeWindow<C0, C1, B0, B1>;
  if (*reinterpret_cast<const unsigned long long*>(table) != hash) return;
  const GroupEntry* __restrict__ tab = reinterpret_cast<const GroupEntry*>(table + kGroupHeaderBytes);
  extern __shared__ __align__(16) char smem[];
  float* pe_lds = reinterpret_cast<float*>(smem);
  LevelBytes* lb = reinterpret_cast<LevelBytes*>(pe_lds + 48);
  for (int i = threadIdx.x; i < 48; i += blockDim.x) pe_lds[i] = pe.v[i / 6][i % 6];
  for (int i = threadIdx.x; i < nmat * kMaxLevels; i += blockDim.x) {
    const DevMat& dm = tab[i / kMaxLevels].m;
    const int j = i % kMaxLevels;
    LevelBytes b;
    b.g0 = (uint32_t)dm.g0_pk[j];
    b.g1 = (uint32_t)dm.g1_pk[j];
    b.g0_last = (uint32_t)(dm.g0_pk_end[j] * 4);
    b.g1_last = (uint32_t)(dm.g1_pk_end[j] * 4);
    lb[i] = b;
  }
  __syncthreads();

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const long long tiles = (n + 15) / 16, stride = (long long)gridDim.x * 4;
  for (long long tile = (long long)blockIdx.x * 4 + wave; tile < tiles; tile += stride) {
    const long long s = tile * 16 + r;
    const bool valid = s < n;
    float u = 0.f, v = 0.f;
    int lod = 0, mt = 0;
    if (valid) {
      const ntc_mixed_query qq = q[s];
      u = qq.u;
      v = qq.v;
      lod = qq.lod;
      mt = min(max(qq.material, 0), nmat - 1);
    }
    const GroupEntry& e = tab[mt];
    Raw R;
    R.fetch(e.m, lb + mt * kMaxLevels, as_global(reinterpret_cast<const uint32_t*>(e.packed)), u, v, lod, g);
    T xs[S1];
    paired_inputs(R, g, xs);
    {
      float pv[3];
      pe_values(pe_lds, R.ix, R.iy, g, pv);
#pragma unroll
      for (int k = 0; k < 3; ++k) xs[pg.T_lat + k] = (T)pv[k];
      const float lod_norm = e.m.lod_in && e.m.M > 1 ? 1.f / (float)(e.m.M - 1) : 0.f;
      xs[pg.T_lat + 3] = (T)(g == 0 ? (float)R.l * lod_norm : 0.f);
#pragma unroll
      for (int t = pg.T_used; t < S1; ++t) xs[t] = (T)0.f;
    }
    // the tile's distinct materials, one network evaluation each
    unsigned long long pending = __ballot(valid);
    while (pending) {
      const int cur = __builtin_amdgcn_readfirstlane(__shfl(mt, (int)__builtin_ctzll(pending)));
      const T* __restrict__ w = as_global(reinterpret_cast<const T*>(tab[cur].wpack));
      const float* __restrict__ bias = reinterpret_cast<const float*>(reinterpret_cast<const char*>(w) + WB);
      f32x4 acc[MT];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(bias + 16 * mo + 4 * g);
        acc[mo] = mma_slots<S1>(acc[mo], w + pg.L1 + mo * S1 * 64, xs, lane);
      }
      T h[SH];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(bias + HD + 16 * mo + 4 * g);
        acc[mo] = mma_slots<SH>(acc[mo], w + pg.L2 + mo * SH * 64, h, lane);
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) act4<ACT>(acc[mo], h + 4 * mo);
      f32x4 y = {0.f, 0.f, 0.f, 0.f};
      if (4 * g < C) y = *reinterpret_cast<const f32x4*>(bias + 2 * HD + 4 * g);
      y = mma_slots<SH>(y, w + pg.L3, h, lane);
      const bool mine = valid && mt == cur;
      if (mine) store_out<C>(out, out_f16, s, n, g, y);
      pending &= ~__ballot(mine);
    }
  }
}

// ------------------------------------------------------------------ FP8-e4m3 decode
// Same pipeline as the FP16 decoder; operands are e4m3 bytes, four slots per word.
// G0 codes go through a byte lookup (v_perm) straight to e4m3 patterns of their exact
// dequantized values; G1 values are the paired FP16 bilinear values rounded to e4m3;
// layer outputs are s_l * acc + b_l in FP32, the activation, then e4m3 again.
template <int B>
__device__ inline uint32_t codes_to_e4m3(uint32_t codes) {  // one code (< 2^B) per byte
  constexpr uint32_t L0 = e4m3_code_lut(B, 0), L1 = e4m3_code_lut(B, 1);
  if constexpr (B <= 3) {
    return __builtin_amdgcn_perm(L1, L0, codes);
  } else {
    constexpr uint32_t L2 = e4m3_code_lut(B, 2), L3 = e4m3_code_lut(B, 3);
    const uint32_t sel = codes & 0x07070707u;
    const uint32_t lo = __builtin_amdgcn_perm(L1, L0, sel), hi = __builtin_amdgcn_perm(L3, L2, sel);
    const uint32_t mask = ((codes >> 3) & 0x01010101u) * 0xFFu;
    return (hi & mask) | (lo & ~mask);
  }
}

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
__device__ __forceinline__ void decode_fp8_body(const DevMat& m, const PeTable& pe, const uint32_t* __restrict__ packed,
                                                const uint8_t* __restrict__ wpack, const float* __restrict__ scales,
                                                const float* __restrict__ bias, const ntc_query* __restrict__ q,
                                                long long n, const TexelRect& rect, void* __restrict__ out,
                                                int out_f16, int bi, int nb) {
  constexpr PackGeom pg = pack_geom_fp8(C0, C1, B0, B1, HD);
  constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT;
  constexpr int WB = ((int)pg.fwd_end + 15) / 16 * 16;
  using Raw = CodeWindow<C0, C1, B0, B1>;
  constexpr int NP = Raw::NW1 * (4 / B1);  // G1 pairs per lane group
  extern __shared__ __align__(16) char smem[];
  const uint8_t* w_lds = reinterpret_cast<const uint8_t*>(smem);
  float* pe_lds = reinterpret_cast<float*>(smem + WB);
  float* b_lds = pe_lds + 48;
  LevelBytes* lb = reinterpret_cast<LevelBytes*>(b_lds + 2 * HD + 16);
  fill_level_bytes(m, lb, threadIdx.x, blockDim.x);

  for (int i = threadIdx.x; i < WB / 16; i += blockDim.x)
    reinterpret_cast<uint4*>(smem)[i] = reinterpret_cast<const uint4*>(wpack)[i];
  for (int i = threadIdx.x; i < 48; i += blockDim.x) pe_lds[i] = pe.v[i / 6][i % 6];
  for (int i = threadIdx.x; i < 2 * HD + 16; i += blockDim.x) b_lds[i] = i < 2 * HD + C ? bias[i] : 0.f;
  __syncthreads();
  const float sc1 = scales[0], sc2 = scales[1], sc3 = scales[2];
  const float lod_norm = m.lod_in && m.M > 1 ? 1.f / (float)(m.M - 1) : 0.f;

  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, g = lane >> 4, r = lane & 15;
  const long long stride = (long long)nb * 4;

  // A operand of MFMA kk of M-tile mo of a layer pack with S slots
  auto a_op = [&](long long base, int S, int mo, int kk) -> long {
    return *reinterpret_cast<const long*>(w_lds + base + (long long)mo * S * 64 + kk * 512 + lane * 8);
  };
  // hidden layer: act(s * acc + b) of fragment mo as 4 e4m3 bytes (slots 4mo .. 4mo+3)
  auto hidden_word = [&](f32x4 acc, float s, const float* b, int mo) -> uint32_t {
    const f32x4 bb = *reinterpret_cast<const f32x4*>(b + 16 * mo + 4 * g);
    float h[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) {  // activation, saturated to the e4m3 range (the conversion alone gives NaN)
      const float z = __builtin_fmaf(acc[i], s, bb[i]);
      h[i] = ACT == 0 ? __builtin_amdgcn_fmed3f(z, 0.f, 448.f) : __builtin_amdgcn_fmed3f(act_fn<ACT>(z), -448.f, 448.f);
    }
    return cvt_e4m3x2(h[2], h[3], cvt_e4m3x2(h[0], h[1], 0u, false), true);
  };

  // As the FP16 point decode: a wavefront takes 64 texels at a time, each lane locates
  // and gathers one texel, and the code words go through the wavefront's slab (same
  // layout as FP16's: G0 windows, G1 pairs of every lane group, PE / LOD word); the
  // weight operands stay in registers (8 bytes per lane and MFMA).
  using DL = DecodeLayout<_Float16, C0, C1, HD, B0, B1, true>;
  static_assert(DL::paired, "the FP8 layout extends the paired one");
  using TC = TexelCodes<C0, C1, B0, B1>;
  constexpr int NW0 = DL::NW0, GW = DL::GW, SW = DL::SW;
  uint32_t* slab = reinterpret_cast<uint32_t*>(lb + kMaxLevels) + wave * 64 * SW;
  long w1r[MT][S1 / 8], w2r[MT][SH / 8], w3r[SH / 8];
#pragma unroll
  for (int mo = 0; mo < MT; ++mo) {
#pragma unroll
    for (int kk = 0; kk < S1 / 8; ++kk) w1r[mo][kk] = a_op(pg.L1, S1, mo, kk);
#pragma unroll
    for (int kk = 0; kk < SH / 8; ++kk) w2r[mo][kk] = a_op(pg.L2, SH, mo, kk);
  }
#pragma unroll
  for (int kk = 0; kk < SH / 8; ++kk) w3r[kk] = a_op(pg.L3, SH, 0, kk);
  const long long groups = (n + 63) / 64;
  auto load_texel = [&](long long grp, float& u, float& v, int& lod) {
    u = v = 0.f;
    lod = 0;
    const long long s = grp * 64 + lane;
    if (grp < groups && s < n) {
      if (rect.w > 0) {
        rect_query(rect, s, u, v, lod);
      } else {
        u = q[s].u;
        v = q[s].v;
        lod = q[s].lod;
      }
    }
  };
  long long grp = (long long)bi * 4 + wave;
  if (grp >= groups) return;
  float u, v;
  int lod;
  load_texel(grp, u, v, lod);
  TC cur;
  cur.fetch(m, lb, packed, u, v, lod);
  load_texel(grp + stride, u, v, lod);
  for (; grp < groups; grp += stride) {
    {
      uint32_t* my = slab + lane * SW;
#pragma unroll
      for (int gg = 0; gg < 4; ++gg) {
        f16x2 pr[NP];
        g1_pairs_words<Raw::NW1, B1>(cur.g1, cur.fx, cur.fy, gg, pr);
#pragma unroll
        for (int w = 0; w < NW0; ++w) my[gg * GW + w] = cur.g0[gg][w];
#pragma unroll
        for (int p = 0; p < NP; ++p) my[gg * GW + NW0 + p] = __builtin_bit_cast(uint32_t, pr[p]);
      }
      my[4 * GW] = (uint32_t)(cur.ix & 7) | ((uint32_t)(cur.iy & 7) << 3) | ((uint32_t)cur.l << 6);
    }
    __builtin_amdgcn_wave_barrier();  // LDS operations of a wavefront complete in order
    TC nxt;
    if (grp + stride < groups) nxt.fetch(m, lb, packed, u, v, lod);
    if (grp + 2 * stride < groups) load_texel(grp + 2 * stride, u, v, lod);
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
      const long long tile = grp * 4 + k;
      if (tile * 16 >= n) break;  // wavefront-uniform
      const uint32_t* rd = slab + (16 * k + r) * SW + g * GW;
      const uint32_t meta = slab[(16 * k + r) * SW + 4 * GW];
      // ---- inputs: S1/4 words of e4m3 bytes
      uint32_t xw[S1 / 4];
#pragma unroll
      for (int i = 0; i < S1 / 4; ++i) xw[i] = 0u;
      constexpr uint32_t BM = ((1u << B0) - 1u) * 0x01010101u;
#pragma unroll
      for (int d = 0; d < NW0; ++d) {
        const uint32_t w0 = rd[d];
#pragma unroll
        for (int kb = 0; kb < 8 / B0; ++kb) xw[(8 / B0) * d + kb] = codes_to_e4m3<B0>((w0 >> (B0 * kb)) & BM);
      }
      {
#pragma unroll
        for (int p = 0; p < NP; ++p) {
          const f16x2 pv2 = __builtin_bit_cast(f16x2, rd[NW0 + p]);
          const int t = C0 + 2 * p;
          xw[t / 4] = cvt_e4m3x2((float)pv2[0], (float)pv2[1], xw[t / 4], (t % 4) != 0);
        }
        float pv[3];
        pe_values(pe_lds, (int)(meta & 7u), (int)((meta >> 3) & 7u), g, pv);
        constexpr int t0 = pg.T_lat;  // even
        const float lodv = g == 0 ? (float)(meta >> 6) * lod_norm : 0.f;  // LOD input (section 4.4)
        xw[t0 / 4] = cvt_e4m3x2(pv[0], pv[1], xw[t0 / 4], (t0 % 4) != 0);
        xw[(t0 + 2) / 4] = cvt_e4m3x2(pv[2], lodv, xw[(t0 + 2) / 4], ((t0 + 2) % 4) != 0);
      }
      // ---- layer 1
      uint32_t hw[SH / 4];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < S1 / 8; ++kk) {
          const long b = (long)((uint64_t)xw[2 * kk] | (uint64_t)xw[2 * kk + 1] << 32);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(w1r[mo][kk], b, acc, 0, 0, 0);
        }
        hw[mo] = hidden_word(acc, sc1, b_lds, mo);
      }
      // ---- layer 2
      uint32_t hw2[SH / 4];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int kk = 0; kk < SH / 8; ++kk) {
          const long b = (long)((uint64_t)hw[2 * kk] | (uint64_t)hw[2 * kk + 1] << 32);
          acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(w2r[mo][kk], b, acc, 0, 0, 0);
        }
        hw2[mo] = hidden_word(acc, sc2, b_lds + HD, mo);
      }
      // ---- layer 3 (no activation)
      f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int kk = 0; kk < SH / 8; ++kk) {
        const long b = (long)((uint64_t)hw2[2 * kk] | (uint64_t)hw2[2 * kk + 1] << 32);
        acc = __builtin_amdgcn_mfma_f32_16x16x32_fp8_fp8(w3r[kk], b, acc, 0, 0, 0);
      }
      const f32x4 b3 = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
      f32x4 y;
#pragma unroll
      for (int i = 0; i < 4; ++i) y[i] = __builtin_fmaf(acc[i], sc3, b3[i]);
      store_out<C>(out, out_f16, tile * 16 + r, n, g, y);
    }
    cur = nxt;
    __builtin_amdgcn_wave_barrier();  // this group's slab reads precede the next group's writes
  }
}

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
__global__ __launch_bounds__(256) void decode_fp8_kernel(DevMat m, PeTable pe, const uint32_t* __restrict__ packed,
                                                         const uint8_t* __restrict__ wpack,
                                                         const float* __restrict__ scales,
                                                         const float* __restrict__ bias,
                                                         const ntc_query* __restrict__ q, long long n,
                                                         TexelRect rect, void* __restrict__ out, int out_f16) {
  decode_fp8_body<C0, C1, C, HD, B0, B1, ACT>(m, pe, packed, wpack, scales, bias, q, n, rect, out, out_f16, blockIdx.x,
                                              gridDim.x);
}

// Grouped FP8 decode (see decode_grouped_kernel); the pack holds weights, scales, biases.
template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
__global__ __launch_bounds__(256) void decode_fp8_grouped_kernel(const char* __restrict__ table, PeTable pe,
                                                                 GroupArgs ga, const ntc_query* __restrict__ q,
                                                                 char* __restrict__ out, int out_f16) {
  constexpr PackGeom pg = pack_geom_fp8(C0, C1, B0, B1, HD);
  constexpr int WB = ((int)pg.fwd_end + 15) / 16 * 16;
  if (*reinterpret_cast<const unsigned long long*>(table) != ga.hash) return;
  const GroupEntry* __restrict__ tab = reinterpret_cast<const GroupEntry*>(table + kGroupHeaderBytes);
  const int s = group_segment(ga);
  const GroupSeg sg = ga.seg[s];
  const GroupEntry& e = tab[sg.mat];
  const uint8_t* wp = as_global(reinterpret_cast<const uint8_t*>(e.wpack));
  const float* scales = reinterpret_cast<const float*>(wp + WB);
  const int nb = (s + 1 < ga.count ? ga.seg[s + 1].block0 : ga.blocks) - sg.block0;
  decode_fp8_body<C0, C1, C, HD, B0, B1, ACT>(e.m, pe, as_global(reinterpret_cast<const uint32_t*>(e.packed)), wp,
                                              scales, scales + 4,
                                              q + sg.q0, sg.n, TexelRect{}, out + sg.o0 * (out_f16 ? 2 : 4), out_f16,
                                              (int)blockIdx.x - sg.block0, nb);
}

}  // namespace ntc
