// Fixed-rate latent quantization and its inverse (section 4.2), bit-exact.
//
// Every grid is an LSB-first bitstream of B-bit codes with B in {1, 2, 4, 8}, so a
// code never straddles a 32-bit word: one thread builds one output word from
// 32/B consecutive latents (coalesced float reads, coalesced word writes).
#include <algorithm>

#include "ntc_internal.h"

namespace ntc {

struct GridTab {
  int n;
  int bits[2 * kMaxLevels];
  long long lat_off[2 * kMaxLevels];  // floats
  long long count[2 * kMaxLevels];    // values in the grid
  long long w_off[2 * kMaxLevels];    // first 32-bit word in the packed buffer
  long long w_end[2 * kMaxLevels + 1];
};

static GridTab grid_tab(const ntc_material& m) {
  GridTab t{};
  t.n = 2 * m.num_levels;
  for (int j = 0; j < m.num_levels; ++j) {
    const int a = 2 * j, b = 2 * j + 1;
    t.bits[a] = m.b0;
    t.bits[b] = m.b1;
    t.lat_off[a] = m.g0_offset[j];
    t.lat_off[b] = m.g1_offset[j];
    t.count[a] = (long long)m.g0_w[j] * m.g0_h[j] * m.c0;
    t.count[b] = (long long)m.g1_w[j] * m.g1_h[j] * m.c1;
    t.w_off[a] = m.g0_packed[j] / 4;
    t.w_off[b] = m.g1_packed[j] / 4;
  }
  for (int k = 0; k < t.n; ++k) t.w_end[k] = (k + 1 < t.n) ? t.w_off[k + 1] : m.packed_bytes / 4;
  return t;
}

__device__ inline int find_grid(const GridTab& t, long long w) {
  int k = 0;
  while (k + 1 < t.n && w >= t.w_off[k + 1]) ++k;
  return k;
}

// code = clamp(rint(x N), -N/2 + 1, N/2) + N/2 - 1; x N is exact; non-finite -> code of 0.
__device__ inline uint32_t quant_code(float x, int bits) {
  const int N = 1 << bits;
  if (!isfinite(x)) x = 0.f;
  float k = rintf(x * (float)N);
  k = fminf(fmaxf(k, (float)(-N / 2 + 1)), (float)(N / 2));
  return (uint32_t)((int)k + N / 2 - 1);
}

__global__ void quantize_kernel(GridTab t, const float* __restrict__ lat, uint32_t* __restrict__ out, long long words) {
  for (long long w = blockIdx.x * (long long)blockDim.x + threadIdx.x; w < words; w += (long long)gridDim.x * blockDim.x) {
    const int k = find_grid(t, w);
    const int bits = t.bits[k];
    const int per = 32 / bits;
    const long long e0 = (w - t.w_off[k]) * per;
    uint32_t word = 0;
    for (int e = 0; e < per; ++e) {
      const long long idx = e0 + e;
      if (idx < t.count[k]) word |= quant_code(lat[t.lat_off[k] + idx], bits) << (e * bits);
    }
    out[w] = word;
  }
}

__global__ void dequantize_kernel(GridTab t, const uint32_t* __restrict__ in, float* __restrict__ lat, long long total) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < total; i += (long long)gridDim.x * blockDim.x) {
    int k = 0;
    while (k + 1 < t.n && i >= t.lat_off[k + 1]) ++k;
    const int bits = t.bits[k];
    const int N = 1 << bits;
    const long long e = i - t.lat_off[k];
    const long long bit = e * bits;
    const uint32_t code = (in[t.w_off[k] + (bit >> 5)] >> (bit & 31)) & ((1u << bits) - 1u);
    lat[i] = (float)((int)code - (N / 2 - 1)) / (float)N;
  }
}

static int blocks_for(long long work, int threads) {
  long long b = (work + threads - 1) / threads;
  const long long cap = (long long)device_cus() * 16;
  if (b > cap) b = cap;
  return (int)(b < 1 ? 1 : b);
}

hipError_t launch_quantize(const ntc_material& m, const float* lat, uint8_t* packed, hipStream_t s) {
  const GridTab t = grid_tab(m);
  const long long words = m.packed_bytes / 4;
  hipLaunchKernelGGL(quantize_kernel, dim3(blocks_for(words, 256)), dim3(256), 0, s, t, lat, (uint32_t*)packed, words);
  return hipGetLastError();
}

hipError_t launch_dequantize(const ntc_material& m, const uint8_t* packed, float* lat, hipStream_t s) {
  const GridTab t = grid_tab(m);
  hipLaunchKernelGGL(dequantize_kernel, dim3(blocks_for(m.latent_count, 256)), dim3(256), 0, s, t,
                     (const uint32_t*)packed, lat, (long long)m.latent_count);
  return hipGetLastError();
}

}  // namespace ntc
