// Device-side building blocks shared by the decode and training kernels (gfx950).
//
// Matrix-core convention used throughout (verified lane layouts of gfx950 MFMA):
//   v_mfma_f32_16x16x{4f32,16f16,32_f16}: lane l = 16*g + r (g = l/16, r = l%16)
//   A operand: A[r][KW*g + j], B operand: B[KW*g + j][r], D: D[4*g + i][r], i = 0..3,
//   with KW = 1, 4, 8 values per lane respectively.
// Layers are evaluated as Z^T (features x texels) = W^T (features x inputs) * X^T:
// the 16 texels of a tile sit on r, so each lane group g carries a quarter of one
// texel's features ("slots").  A layer's D fragment (rows 16m + 4g + i) becomes
// the next layer's B fragment without any data movement: slot t of group g holds
// feature phi(g, t) = 16*(t/4) + 4*g + t%4, and the weight rows are permuted to
// match when the weights are packed.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ntc {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x4 __attribute__((ext_vector_type(4)));
typedef _Float16 f16x8 __attribute__((ext_vector_type(8)));
typedef _Float16 f16x2 __attribute__((ext_vector_type(2)));
typedef short s16x2 __attribute__((ext_vector_type(2)));

constexpr int kMaxLevels = 8;
constexpr int kMaxMips = 16;

// Geometry as the kernels see it (filled on the host from ntc_material).
struct DevMat {
  int W, H, C, M, C0, C1, B0, B1, shift, Hd, act, pe, lod_in, J, K;
  int mip_w[kMaxMips], mip_h[kMaxMips], level_of_mip[kMaxMips];
  int g0_w[kMaxLevels], g0_h[kMaxLevels], g1_w[kMaxLevels], g1_h[kMaxLevels];
  long long g0_off[kMaxLevels], g1_off[kMaxLevels];
  long long g0_pk[kMaxLevels], g1_pk[kMaxLevels];
  long long g0_pk_end[kMaxLevels], g1_pk_end[kMaxLevels];
  long long mip_off[kMaxMips];
  long long latent_count;
};

// A pointer read from device memory (a table entry) as a global-memory pointer, so the
// compiler emits global rather than flat accesses through it (flat loads also count
// against the LDS counter and serialise with LDS traffic).
template <typename T>
__device__ inline T* as_global(T* p) {
  return (T*)(__attribute__((address_space(1))) T*)p;
}

// One material of a grouped launch: its geometry, bit-packed latents and decode pack.
struct GroupEntry {
  DevMat m;
  const void* packed;
  const void* wpack;
};
// A material's share of a grouped launch: blocks [block0, next segment's block0),
// queries q0 .. q0 + n - 1, outputs from element o0.
constexpr int kGroupSegs = 32;
struct GroupSeg {
  int mat, block0;
  long long q0, n, o0;
};
// A grouped launch: `hash` must equal the table's (the table was built for the
// materials the launch was planned for), otherwise its blocks do nothing.
struct GroupArgs {
  unsigned long long hash;
  int count, blocks;
  GroupSeg seg[kGroupSegs];
};
// Device table of a grouped decode: a header (hash of the materials) then the entries.
constexpr int kGroupHeaderBytes = 256;
constexpr int kMixedMax = 64;  // materials of one mixed-material decode

// Coherent decode source: the texels of rectangle [x0, x0+w) x [y0, y0+h) of mip lod,
// row-major (w == 0: queries come from a query array instead).  inv_w, inv_h = 1 / mip
// size, so (x + 1/2) * inv_w is the exact texel centre.
struct TexelRect {
  int lod, x0, y0, w, h;
  float inv_w, inv_h;
};
__device__ inline void rect_query(const TexelRect& r, long long s, float& u, float& v, int& lod) {
  const int i = (int)s, yy = i / r.w, xx = i - yy * r.w;
  u = ((float)(r.x0 + xx) + 0.5f) * r.inv_w;
  v = ((float)(r.y0 + yy) + 0.5f) * r.inv_h;
  lod = r.lod;
}

// Positional-encoding table: pe[m][q] for texel position m = i mod 8 inside the
// 8-texel tile and value q = (sin, cos) x (1, 2, 4 cycles per tile) (section 4.3.2).
struct PeTable {
  float v[8][6];
};

// ------------------------------------------------------------------ slot maps
__host__ __device__ constexpr int hid_feature(int g, int t) { return 16 * (t / 4) + 4 * g + (t % 4); }

// Input slots of a lane group g for latent widths C0, C1 (same positions in
// every group, so slot indices are compile-time constants):
//   t <  C0                 : G0 neighbour g, channel t
//   C0 <= t < T_lat         : G1 channel g + 4 (t - C0) (padding if >= C1)
//   T_lat <= t < T_lat + 3  : positional-encoding values 3g .. 3g+2
//   t = T_lat + 3           : the LOD input in group 0 (section 4.4; zero without it)
//   beyond                  : zero padding
template <int C0, int C1>
struct InSlots {
  static constexpr int n1max = (C1 + 3) / 4;
  static constexpr int T_lat = C0 + n1max;
  static constexpr int T_used = T_lat + 4;
  static constexpr int K_LOD = 4 * C0 + C1 + 12;  // canonical row of the LOD input
  // canonical input feature of slot (g, t); -1 for padding
  static constexpr int psi(int g, int t) {
    return t < C0 ? g * C0 + t
         : t < T_lat ? (g + 4 * (t - C0) < C1 ? 4 * C0 + g + 4 * (t - C0) : -1)
         : t < T_lat + 3 ? 4 * C0 + C1 + 3 * g + (t - T_lat)
         : t == T_lat + 3 && g == 0 ? K_LOD
         : -1;
  }
};

// Sizes of the operand packs of one material (elements of the compute type).
struct PackGeom {
  int S1, SH, MT, ML, T_lat, T_used;
  long long L1, L2, L3, B3, B2, B1;  // element offsets
  long long fwd_end, train_end;      // end of forward packs, end of all packs
};
__host__ __device__ constexpr PackGeom pack_geom(int c0, int c1, int hd, bool f16) {
  PackGeom p{};
  p.T_lat = c0 + (c1 + 3) / 4;
  p.T_used = p.T_lat + 4;  // 3 positional-encoding slots and the LOD slot
  p.S1 = f16 ? (p.T_used + 3) / 4 * 4 : p.T_used;
  p.SH = hd / 4;
  p.MT = hd / 16;
  p.ML = (p.T_lat + 3) / 4;
  p.L1 = 0;
  p.L2 = p.L1 + (long long)p.MT * p.S1 * 64;
  p.L3 = p.L2 + (long long)p.MT * p.SH * 64;
  p.B3 = p.L3 + (long long)p.SH * 64;
  p.fwd_end = p.B3;
  p.B2 = p.B3 + (long long)p.MT * 4 * 64;
  p.B1 = p.B2 + (long long)p.MT * p.SH * 64;
  p.train_end = p.B1 + (long long)p.ML * p.SH * 64;
  return p;
}

// Paired input layout of the FP16 decoder reading bit-packed codes: two channels per
// 32-bit register, taken straight from the packed words (channel c and c + 16/B of
// the same dword share a register), when B <= 4.  A G0 cell's window is read as whole
// dwords; the codes past its last channel (the next cell's bits) meet zero weights.
//   G0: window dword d, pair p = d*(16/B0) + c (c < 16/B0) -> slots 2p, 2p+1 hold
//       channels d*32/B0 + c and d*32/B0 + c + 16/B0 (padding if >= C0);
//       G0S = ceil(C0 B0 / 32) * 32/B0 slots.
//   G1: lane group g, dword d, k < 4/B1: pair q = d*(4/B1) + k -> slots G0S + 2q, +1
//       hold channels ch = d*32/B1 + g + 4k and ch + 16/B1 (padding if >= C1).
//   PE: the next 3 slots; LOD input: the one after, in group 0.
__host__ __device__ constexpr bool paired_layout(int c0, int c1, int b0, int b1, bool f16) {
  return f16 && b0 <= 4 && b1 <= 4 && c0 >= 1 && c1 >= 1;
}
__host__ __device__ constexpr int paired_g0_slots(int c0, int b0) { return (c0 * b0 + 31) / 32 * (32 / b0); }
__host__ __device__ constexpr int paired_g1_slots(int c1, int b1) { return 2 * ((c1 * b1 + 31) / 32) * (4 / b1); }
__host__ __device__ constexpr PackGeom pack_geom_decode(int c0, int c1, int b0, int b1, int hd, bool f16) {
  PackGeom p = pack_geom(c0, c1, hd, f16);
  if (paired_layout(c0, c1, b0, b1, f16)) {
    p.T_lat = paired_g0_slots(c0, b0) + paired_g1_slots(c1, b1);
    p.T_used = p.T_lat + 4;
    p.S1 = (p.T_used + 3) / 4 * 4;
    p.ML = (p.T_lat + 3) / 4;
    p.L1 = 0;
    p.L2 = p.L1 + (long long)p.MT * p.S1 * 64;
    p.L3 = p.L2 + (long long)p.MT * p.SH * 64;
    p.B3 = p.L3 + (long long)p.SH * 64;
    p.fwd_end = p.B3;
    p.B2 = p.B1 = p.train_end = p.B3;  // decode packs have no backward part
  }
  return p;
}
__host__ __device__ inline void in_slot_of_paired(int k, int c0, int c1, int b0, int b1, int& g, int& t) {
  if (k < 4 * c0) {
    const int c = k % c0, per = 32 / b0, half = 16 / b0, d = c / per, cc = c % per;
    g = k / c0;
    t = cc < half ? 2 * (d * half + cc) : 2 * (d * half + cc - half) + 1;
  } else if (k < 4 * c0 + c1) {
    const int ch = k - 4 * c0, per = 32 / b1, half = 16 / b1, d = ch / per, cc = ch % per;
    g = ch % 4;
    const bool lo = cc < half;
    const int kk = ((lo ? cc : cc - half) - g) / 4;
    t = paired_g0_slots(c0, b0) + 2 * (d * (4 / b1) + kk) + (lo ? 0 : 1);
  } else {
    const int p = k - 4 * c0 - c1;  // 12: the LOD input
    g = p < 12 ? p / 3 : 0;
    t = paired_g0_slots(c0, b0) + paired_g1_slots(c1, b1) + (p < 12 ? p % 3 : 3);
  }
}

// FP8-e4m3 decode layout (16x16x32 fp8 matrix cores: 8 slots of a lane group per
// instruction, one byte each).  The paired layout's eligibility with G0 cells of
// whole dwords (so G0S = C0).  G0 codes are spread into bytes four at a time: for dword d and k < 8/B0, the word
// (w >> B0*k) & byte-mask holds in byte b the code of channel d*32/B0 + b*8/B0 + k,
// which goes to slot d*32/B0 + 4k + b.  G1 pairs and the PE follow the paired layout;
// slots are padded to a multiple of 8.  Element offsets are bytes.
__host__ __device__ constexpr bool fp8_layout(int c0, int c1, int b0, int b1, int hd) {
  return paired_layout(c0, c1, b0, b1, true) && (c0 * b0) % 32 == 0 && hd % 32 == 0;
}
__host__ __device__ constexpr PackGeom pack_geom_fp8(int c0, int c1, int b0, int b1, int hd) {
  PackGeom p{};
  p.T_lat = c0 + paired_g1_slots(c1, b1);
  p.T_used = p.T_lat + 4;
  p.S1 = (p.T_used + 7) / 8 * 8;
  p.SH = hd / 4;
  p.MT = hd / 16;
  p.ML = (p.T_lat + 3) / 4;
  p.L1 = 0;
  p.L2 = p.L1 + (long long)p.MT * p.S1 * 64;
  p.L3 = p.L2 + (long long)p.MT * p.SH * 64;
  p.B3 = p.L3 + (long long)p.SH * 64;
  p.fwd_end = p.B2 = p.B1 = p.train_end = p.B3;
  return p;
}
__host__ __device__ inline void in_slot_of_fp8(int k, int c0, int c1, int b0, int b1, int& g, int& t) {
  if (k < 4 * c0) {
    const int c = k % c0, per = 32 / b0, d = c / per, cc = c % per, b = cc / (8 / b0), kk = cc % (8 / b0);
    g = k / c0;
    t = per * d + 4 * kk + b;
  } else {
    in_slot_of_paired(k, c0, c1, b0, b1, g, t);
  }
}
// e4m3 bit pattern of a value that the format holds exactly (dequantized codes)
__host__ __device__ constexpr uint32_t e4m3_exact_bits(float v) {
  uint32_t s = v < 0 ? 0x80u : 0u;
  float a = v < 0 ? -v : v;
  if (a == 0.f) return s;
  int e = 0;
  while (a >= 2.f) { a *= 0.5f; ++e; }
  while (a < 1.f) { a *= 2.f; --e; }
  if (e < -6) {  // subnormal: m * 2^-9
    float m = a;
    for (int i = e; i < -9; ++i) m *= 0.5f;
    for (int i = -9; i < e; ++i) m *= 2.f;
    return s | (uint32_t)m;
  }
  return s | (uint32_t)(e + 7) << 3 | (uint32_t)((a - 1.f) * 8.f);
}
// Four e4m3 patterns of dequantized codes 4i .. 4i+3 of a B-bit grid, packed in a word.
__host__ __device__ constexpr uint32_t e4m3_code_lut(int B, int i) {
  const int N = 1 << B;
  uint32_t w = 0;
  for (int b = 0; b < 4; ++b) {
    const int k = 4 * i + b;
    if (k < N) w |= e4m3_exact_bits((float)(k - (N / 2 - 1)) / (float)N) << (8 * b);
  }
  return w;
}

// Runtime inverse slot maps (used where canonical weights are scattered into packs).
__host__ __device__ inline void in_slot_of(int k, int c0, int c1, int& g, int& t) {
  const int tl = c0 + (c1 + 3) / 4;
  if (k < 4 * c0) { g = k / c0; t = k % c0; }
  else if (k < 4 * c0 + c1) { const int ch = k - 4 * c0; g = ch % 4; t = c0 + ch / 4; }
  else { const int p = k - 4 * c0 - c1; g = p < 12 ? p / 3 : 0; t = tl + (p < 12 ? p % 3 : 3); }  // 12: LOD
}
__host__ __device__ inline void hid_slot_of(int h, int& g, int& t) { g = (h / 4) % 4; t = 4 * (h / 16) + h % 4; }

// ------------------------------------------------------------------ operand packs
// A pack holds, for every M-tile mo and every slot t of the K dimension, the 64
// lane values of the A operand.  Values of one lane that feed one MFMA are
// contiguous: FP32 -> 1 value per MFMA (16x16x4); FP16 -> groups of 8 slots
// (16x16x32) and a trailing group of 4 (16x16x16).
template <typename T>
__host__ __device__ inline int pack_index(int S, int mo, int t, int lane);

template <>
__host__ __device__ inline int pack_index<float>(int S, int mo, int t, int lane) {
  return (mo * S + t) * 64 + lane;
}
template <>
__host__ __device__ inline int pack_index<uint8_t>(int S, int mo, int t, int lane) {
  return mo * S * 64 + (t / 8) * 512 + lane * 8 + (t % 8);  // S is a multiple of 8
}
template <>
__host__ __device__ inline int pack_index<_Float16>(int S, int mo, int t, int lane) {
  const int s8 = S / 8 * 8;
  const int base = mo * S * 64;
  if (t < s8) return base + (t / 8) * 512 + lane * 8 + (t % 8);
  return base + s8 * 64 + lane * 4 + (t - s8);
}

// acc += A(tile) * B over S slots; `a` points at the tile's pack (mo already applied).
template <int S>
__device__ inline f32x4 mma_slots(f32x4 acc, const float* __restrict__ a, const float (&b)[S], int lane) {
#pragma unroll
  for (int t = 0; t < S; ++t) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a[t * 64 + lane], b[t], acc, 0, 0, 0);
  return acc;
}
template <int S>
__device__ inline f32x4 mma_slots(f32x4 acc, const _Float16* __restrict__ a, const _Float16 (&b)[S], int lane) {
  static_assert(S % 4 == 0, "fp16 slot counts are multiples of 4");
  constexpr int S8 = S / 8 * 8;
#pragma unroll
  for (int t = 0; t < S8; t += 8) {
    const f16x8 av = *reinterpret_cast<const f16x8*>(a + t * 64 + lane * 8);
    f16x8 bv;
#pragma unroll
    for (int j = 0; j < 8; ++j) bv[j] = b[t + j];
    acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
  }
  if constexpr (S8 < S) {
    // The 16x16x16 tail gets its own zero accumulator and is added on the VALU:
    // chaining a 16x16x32 and a 16x16x16 MFMA back-to-back through the
    // accumulator operand returns wrong sums on gfx950 with ROCm 7.2 (the
    // compiler inserts no wait states between the two shapes).
    const f16x4 av = *reinterpret_cast<const f16x4*>(a + S8 * 64 + lane * 4);
    f16x4 bv;
#pragma unroll
    for (int j = 0; j < 4; ++j) bv[j] = b[S8 + j];
    const f32x4 zero = {0.f, 0.f, 0.f, 0.f};
    const f32x4 tail = __builtin_amdgcn_mfma_f32_16x16x16f16(av, bv, zero, 0, 0, 0);
    acc += tail;
  }
  return acc;
}

// ------------------------------------------------------------------ activations (section 4.4)
// ACT: 0 ReLU, 1 hardGELU; a compile-time choice so that the per-element code is
// straight-line selects
template <int ACT>
__device__ inline float act_fn(float z) {
  if constexpr (ACT == 0) {
    // max(z, 0) on the bit pattern: one integer op, no NaN canonicalisation
    return __builtin_bit_cast(float, max(__builtin_bit_cast(int, z), 0));
  } else {
    const float p = z * (z + 1.5f) * (1.f / 3.f);
    return z < -1.5f ? 0.f : (z > 1.5f ? z : p);
  }
}
// FP32 -> e4m3 (round to nearest even) of two values into the low or high half of `old`.
__device__ inline uint32_t cvt_e4m3x2(float a, float b, uint32_t old, bool hi) {
  return hi ? (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, (int)old, true)
            : (uint32_t)__builtin_amdgcn_cvt_pk_fp8_f32(a, b, (int)old, false);
}

// a(z) of one accumulator fragment, rounded to the operand type T; ReLU in FP16
// rounds first (rounding commutes with max(., 0)) and clamps two values per op
template <int ACT, typename T>
__device__ inline void act4(const f32x4& a, T* h) {
  if constexpr (ACT == 0 && sizeof(T) == 2) {
    const s16x2 zero = {0, 0};
    const f16x2 p0 = __builtin_convertvector(a.xy, f16x2), p1 = __builtin_convertvector(a.zw, f16x2);
    const f16x2 q0 = __builtin_bit_cast(f16x2, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p0), zero));
    const f16x2 q1 = __builtin_bit_cast(f16x2, __builtin_elementwise_max(__builtin_bit_cast(s16x2, p1), zero));
    h[0] = q0[0];
    h[1] = q0[1];
    h[2] = q1[0];
    h[3] = q1[1];
  } else {
#pragma unroll
    for (int i = 0; i < 4; ++i) h[i] = (T)act_fn<ACT>(a[i]);
  }
}
template <int ACT>
__device__ inline float act_grad(float z) {
  if constexpr (ACT == 0) {
    return z > 0.f ? 1.f : 0.f;
  } else {
    const float p = (2.f * z + 1.5f) * (1.f / 3.f);
    return z < -1.5f ? 0.f : (z > 1.5f ? 1.f : p);
  }
}

// a'(z) given z and the stored activation h = a(z) in the operand type: ReLU takes
// its decision from h (h > 0 exactly when z > 0, up to underflow of the rounding)
template <int ACT, typename T>
__device__ inline float dact(float z, T h) {
  if constexpr (ACT == 0) return (float)h > 0.f ? 1.f : 0.f;
  else return act_grad<ACT>(z);
}

// ------------------------------------------------------------------ sampling (section 4.3)
__device__ inline int snap_texel(float u, int size) {
  float p = u * (float)size;
  p = (p == p) ? p : 0.f;  // NaN -> 0
  p = fminf(fmaxf(p, 0.f), (float)(size - 1));
  return (int)floorf(p);
}

// Everything one lane needs to fetch its share of a texel's inputs.
struct Footprint {
  int l, j, ix, iy;
  int g0_cell;          // G0 cell index (within the level's grid) of this lane group's neighbour
  int g0x, g0y;         // its coordinates
  int ax, ay, bx, by;   // clamped G0 footprint columns (x0, x0+1) and rows (y0, y0+1)
  int g1_cell[4];       // G1 tap cells, order (x,y), (x+1,y), (x,y+1), (x+1,y+1)
  int g1x[2], g1y[2];   // clamped G1 tap coordinates (x, x+1), (y, y+1)
  float g1_w[4];        // bilinear weights of the taps
  float fx, fy;         // fractional G1 position (g1_w are the products of fx, fy, 1-fx, 1-fy)
};

__device__ inline Footprint locate(const DevMat& m, float u, float v, int lod, int g) {
  Footprint f;
  const int l = min(max(lod, 0), m.M - 1);
  const int Wl = max(1, m.W >> l), Hl = max(1, m.H >> l);
  const int j = min(max((l - m.shift) >> 1, 0), m.J - 1);
  const int w0 = m.W >> (m.shift + 2 * j), h0 = m.H >> (m.shift + 2 * j);
  const int w1 = w0 >> 1, h1 = h0 >> 1;
  f.l = l;
  f.j = j;
  f.ix = snap_texel(u, Wl);
  f.iy = snap_texel(v, Hl);
  // texel centre in grid units: all sizes are powers of two, so the scale is an
  // exponent shift and exact
  const float cx = (float)f.ix + 0.5f, cy = (float)f.iy + 0.5f;
  const int ex = __builtin_ctz(w0) - __builtin_ctz(Wl), ey = __builtin_ctz(h0) - __builtin_ctz(Hl);
  {
    const float gx = __builtin_ldexpf(cx, ex) - 0.5f;
    const float gy = __builtin_ldexpf(cy, ey) - 0.5f;
    const int x0 = (int)floorf(gx), y0 = (int)floorf(gy);
    f.ax = min(max(x0, 0), w0 - 1);
    f.ay = min(max(y0, 0), h0 - 1);
    f.bx = min(max(x0 + 1, 0), w0 - 1);
    f.by = min(max(y0 + 1, 0), h0 - 1);
    f.g0x = min(max(x0 + (g & 1), 0), w0 - 1);
    f.g0y = min(max(y0 + (g >> 1), 0), h0 - 1);
    f.g0_cell = f.g0y * w0 + f.g0x;
  }
  {
    const float gx = __builtin_ldexpf(cx, ex - 1) - 0.5f;  // G1 has half the G0 resolution
    const float gy = __builtin_ldexpf(cy, ey - 1) - 0.5f;
    const float fx0 = floorf(gx), fy0 = floorf(gy);
    const float fx = gx - fx0, fy = gy - fy0;
    const int x0 = (int)fx0, y0 = (int)fy0;
    f.g1x[0] = min(max(x0, 0), w1 - 1);
    f.g1x[1] = min(max(x0 + 1, 0), w1 - 1);
    f.g1y[0] = min(max(y0, 0), h1 - 1);
    f.g1y[1] = min(max(y0 + 1, 0), h1 - 1);
    f.g1_cell[0] = f.g1y[0] * w1 + f.g1x[0];
    f.g1_cell[1] = f.g1y[0] * w1 + f.g1x[1];
    f.g1_cell[2] = f.g1y[1] * w1 + f.g1x[0];
    f.g1_cell[3] = f.g1y[1] * w1 + f.g1x[1];
    f.fx = fx;
    f.fy = fy;
    f.g1_w[0] = (1.f - fx) * (1.f - fy);
    f.g1_w[1] = fx * (1.f - fy);
    f.g1_w[2] = (1.f - fx) * fy;
    f.g1_w[3] = fx * fy;
  }
  return f;
}

// ------------------------------------------------------------------ spatial tiles of the latent grids
// Level j's G0 grid is cut into T x T cell tiles (T = min(Tmax, grid side)); the G1
// grid into the matching (T/2) x (T/2) tiles.  A tile owns the latents of its cells.
// Samples are counting-sorted into bins: one bin per tile (sb = 1) or, on levels
// with few cells, one bin per (tile, anchor cell) (sb = T), which orders a tile's
// samples by anchor cell.  A tile's bins are consecutive.
struct TileGeom {
  int T[kMaxLevels], ntx[kMaxLevels], nty[kMaxLevels], sb[kMaxLevels];
  int tile_base[kMaxLevels + 1];  // first tile of each level
  int bin_base[kMaxLevels + 1];   // first sort bin of each level
  int region[kMaxLevels];
  int ntiles, nbins, region_max;
  int chunk;                       // samples per work item
};

__host__ __device__ inline int sort_bin(const TileGeom& tg, int j, int tx, int ty, int ax, int ay) {
  const int sb = tg.sb[j], T = tg.T[j];
  const int tile = ty * tg.ntx[j] + tx;
  if (sb == 1) return tg.bin_base[j] + tile;
  int sx = ax - tx * T, sy = ay - ty * T;
  sx = sx < 0 ? 0 : (sx > T - 1 ? T - 1 : sx);
  sy = sy < 0 ? 0 : (sy > T - 1 ? T - 1 : sy);
  return tg.bin_base[j] + tile * T * T + sy * T + sx;
}

// Tiles whose latents a sample's footprint touches: columns [tx0, tx1], rows [ty0, ty1]
// (each range spans at most two tiles), and the primary tile holding the clamped anchor.
struct SampleBins {
  int j, tx0, tx1, ty0, ty1, ptx, pty;
};
__device__ inline SampleBins sample_bins(const Footprint& f, const TileGeom& tg) {
  SampleBins b;
  b.j = f.j;
  // tile sides are powers of two (>= 2): shifts instead of divisions
  const int ts = __builtin_ctz(tg.T[f.j]), t1s = ts - 1;
  b.tx0 = min(f.ax >> ts, f.g1x[0] >> t1s);
  b.tx1 = max(f.bx >> ts, f.g1x[1] >> t1s);
  b.ty0 = min(f.ay >> ts, f.g1y[0] >> t1s);
  b.ty1 = max(f.by >> ts, f.g1y[1] >> t1s);
  b.ptx = f.ax >> ts;
  b.pty = f.ay >> ts;
  return b;
}

// Sum over the 16 lanes of a row (lane group), by rotations within the row (DPP).
__device__ inline float row_sum16(float v) {
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x121, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x122, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x124, 0xf, 0xf, false));
  v += __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x128, 0xf, 0xf, false));
  return v;
}

// Inclusive prefix sum over the 64 lanes of a wavefront (DPP): shifts within each row
// of 16 lanes (zeros shifted in), then the last lane of each row added to the rows after it.
__device__ inline uint32_t wave_incl_sum(uint32_t x) {
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, true);  // row_shr:1
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, true);  // row_shr:2
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, true);  // row_shr:4
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, true);  // row_shr:8
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);  // row_bcast:15 into rows 1, 3
  x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);  // row_bcast:31 into rows 2, 3
  return x;
}

// Inclusive prefix maximum of non-negative values over the 64 lanes of a wavefront (DPP,
// as wave_incl_sum).
__device__ inline int wave_incl_max(int x) {
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x111, 0xf, 0xf, true));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x112, 0xf, 0xf, true));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x114, 0xf, 0xf, true));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x118, 0xf, 0xf, true));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x142, 0xa, 0xf, false));
  x = max(x, __builtin_amdgcn_update_dpp(0, x, 0x143, 0xc, 0xf, false));
  return x;
}

// Integer sum over the 16 lanes of a row (lane group), by rotations within the row (DPP).
__device__ inline int row_sum16i(int v) {
  v += __builtin_amdgcn_update_dpp(0, v, 0x121, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x122, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x124, 0xf, 0xf, false);
  v += __builtin_amdgcn_update_dpp(0, v, 0x128, 0xf, 0xf, false);
  return v;
}
// The same for 64-bit integers: both halves rotated, then a 64-bit add.
template <int CTRL>
__device__ inline long long dpp_row64(long long v) {
  const unsigned lo = (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xf, 0xf, false);
  const unsigned hi = (unsigned)__builtin_amdgcn_update_dpp(0, (int)(v >> 32), CTRL, 0xf, 0xf, false);
  return (long long)(((unsigned long long)hi << 32) | lo);
}
__device__ inline long long row_sum16i(long long v) {
  v += dpp_row64<0x121>(v);
  v += dpp_row64<0x122>(v);
  v += dpp_row64<0x124>(v);
  v += dpp_row64<0x128>(v);
  return v;
}

// The three positional-encoding values of lane group g (slots 3g..3g+2 of the 12).
__device__ inline void pe_values(const float* pe_lds, int ix, int iy, int g, float out[3]) {
  const int mpos = (g >> 1) ? (iy & 7) : (ix & 7);
  const int q0 = 3 * (g & 1);
#pragma unroll
  for (int s = 0; s < 3; ++s) out[s] = pe_lds[mpos * 6 + q0 + s];
}

// ------------------------------------------------------------------ bit-packed codes (section 4.2)
// Window of NW+1 dwords covering `nbits` bits starting at absolute bit `bit0` of a
// packed grid, realigned so that result bit 0 is `bit0`.  Dword reads are clamped to
// the grid's last dword so they never leave the grid.
template <int NW, bool ALIGNED>
__device__ inline void load_bits(const uint32_t* __restrict__ base, long long bit0, long long last_dword,
                                 uint32_t (&out)[NW]) {
  const long long d0 = bit0 >> 5;
  if constexpr (ALIGNED) {  // bit0 is a multiple of 32 and the window ends inside the grid
#pragma unroll
    for (int k = 0; k < NW; ++k) out[k] = base[d0 + k];
  } else {
    const int s = (int)(bit0 & 31);
    uint32_t w[NW + 1];
#pragma unroll
    for (int k = 0; k <= NW; ++k) w[k] = base[min(d0 + k, last_dword)];
#pragma unroll
    for (int k = 0; k < NW; ++k) out[k] = __builtin_amdgcn_alignbit(w[k + 1], w[k], s);
  }
}

template <int B, int NW>
__device__ inline int code_at(const uint32_t (&win)[NW], int c) {
  constexpr uint32_t mask = (1u << B) - 1u;
  const int p = c * B;
  return (int)((win[p >> 5] >> (p & 31)) & mask);
}

// Same with a run-time channel index (selects the window word without dynamic indexing).
template <int B, int NW>
__device__ inline int code_at_dyn(const uint32_t (&win)[NW], int c) {
  constexpr uint32_t mask = (1u << B) - 1u;
  const int p = c * B;
  const int k = p >> 5;
  uint32_t w = win[0];
#pragma unroll
  for (int i = 1; i < NW; ++i) w = (k == i) ? win[i] : w;
  return (int)((w >> (p & 31)) & mask);
}

template <int B>
__device__ inline float dequant(int code) {
  constexpr int N = 1 << B;
  return (float)(code - (N / 2 - 1)) * (1.f / (float)N);
}

// ------------------------------------------------------------------ counter noise (section 4.2)
// SplitMix64 output function (Steele, Lea, Flood 2014).
__host__ __device__ inline uint64_t mix64(uint64_t z) {
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
constexpr uint64_t kGamma = 0x9E3779B97F4A7C15ull;
__host__ __device__ inline uint64_t noise_key(uint64_t seed, int step) {
  return mix64(seed + kGamma * (uint64_t)(step + 1));
}
// U[-Q/2, Q/2) with Q = 2^-bits, 24-bit resolution; exact in FP32.
__device__ inline float noise_at(uint64_t key, long long i, int bits) {
  const uint64_t r = mix64(key + kGamma * (uint64_t)(i + 1));
  const int r24 = (int)(r >> 40);
  return (float)(r24 - (1 << 23)) * ldexpf(1.f, -24 - bits);
}

// ------------------------------------------------------------------ weight scatter into packs
// Canonical FP32 parameter p (layout W1[K][Hd], b1, W2[Hd][Hd], b2, W3[Hd][C], b3)
// is written to its place in the forward packs and, when `bwd`, in the backward
// packs (weights only; biases are read from the canonical buffer).
template <typename T>
__device__ inline void scatter_param(T* __restrict__ pack, const PackGeom& pg, int c0, int c1, int C, int Hd,
                                     long long p, float value, bool bwd, int b0 = 0, int b1 = 0,
                                     bool paired = false, int lod_in = 0) {
  const long long K = 4 * c0 + c1 + 12 + lod_in;
  const long long nW1 = K * Hd, nW2 = (long long)Hd * Hd, nW3 = (long long)Hd * C;
  const T v = (T)value;
  if (p < nW1) {
    const int k = (int)(p / Hd), h = (int)(p % Hd);
    int g, t;
    if (paired) in_slot_of_paired(k, c0, c1, b0, b1, g, t);
    else in_slot_of(k, c0, c1, g, t);
    pack[pg.L1 + pack_index<T>(pg.S1, h / 16, t, 16 * g + h % 16)] = v;
    if (bwd && t < pg.T_lat) {
      int g2, t2;
      hid_slot_of(h, g2, t2);
      pack[pg.B1 + pack_index<T>(pg.SH, t / 4, t2, 16 * g2 + 4 * g + t % 4)] = v;
    }
    return;
  }
  p -= nW1 + Hd;
  if (p >= 0 && p < nW2) {
    const int h1 = (int)(p / Hd), h2 = (int)(p % Hd);
    int g, t;
    hid_slot_of(h1, g, t);
    pack[pg.L2 + pack_index<T>(pg.SH, h2 / 16, t, 16 * g + h2 % 16)] = v;
    if (bwd) {
      int g2, t2;
      hid_slot_of(h2, g2, t2);
      pack[pg.B2 + pack_index<T>(pg.SH, h1 / 16, t2, 16 * g2 + h1 % 16)] = v;
    }
    return;
  }
  p -= nW2 + Hd;
  if (p >= 0 && p < nW3) {
    const int h = (int)(p / C), c = (int)(p % C);
    int g, t;
    hid_slot_of(h, g, t);
    pack[pg.L3 + pack_index<T>(pg.SH, 0, t, 16 * g + c)] = v;
    if (bwd) pack[pg.B3 + pack_index<T>(4, h / 16, c % 4, 16 * (c / 4) + h % 16)] = v;
  }
}

}  // namespace ntc
