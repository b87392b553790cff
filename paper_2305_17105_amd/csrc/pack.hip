// Canonical FP32 MLP -> matrix-core operand packs (FP32 or FP16).
#include <algorithm>

#include "ntc_internal.h"

namespace ntc {

template <typename T>
__global__ void zero_kernel(T* __restrict__ p, long long n) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n; i += (long long)gridDim.x * blockDim.x)
    p[i] = (T)0.f;
}

template <typename T>
__global__ void pack_kernel(PackGeom pg, int c0, int c1, int C, int Hd, long long P, const float* __restrict__ mlp,
                            T* __restrict__ pack, float* __restrict__ bias_out, int bwd, int b0, int b1, int paired,
                            int lod_in) {
  const long long K = 4 * c0 + c1 + 12 + lod_in;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const float v = mlp[p];
    scatter_param<T>(pack, pg, c0, c1, C, Hd, p, v, bwd != 0, b0, b1, paired != 0, lod_in);
    if (bias_out) {
      const long long b1 = K * Hd, b2 = b1 + Hd + (long long)Hd * Hd, b3 = b2 + Hd + (long long)Hd * C;
      if (p >= b1 && p < b1 + Hd) bias_out[p - b1] = v;
      else if (p >= b2 && p < b2 + Hd) bias_out[Hd + (p - b2)] = v;
      else if (p >= b3 && p < b3 + C) bias_out[2 * Hd + (p - b3)] = v;
    }
  }
}

template <typename T>
static hipError_t pack_t(const ntc_material& m, const float* mlp, bool bwd, void* packed, hipStream_t s) {
  // decode packs follow the decoder's input layout; training packs the training one
  const bool paired = !bwd && paired_layout(m.c0, m.c1, m.b0, m.b1, sizeof(T) == 2);
  const PackGeom pg = bwd ? pack_geom(m.c0, m.c1, m.hidden, sizeof(T) == 2)
                          : pack_geom_decode(m.c0, m.c1, m.b0, m.b1, m.hidden, sizeof(T) == 2);
  const long long n = bwd ? pg.train_end : pg.fwd_end;
  T* w = (T*)packed;
  float* bias = nullptr;
  if (!bwd) {
    const size_t wbytes = ((size_t)pg.fwd_end * sizeof(T) + 15) / 16 * 16;
    bias = (float*)((char*)packed + wbytes);
  }
  const int zb = (int)std::min<long long>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel<T>, dim3(zb), dim3(256), 0, s, w, n);
  const long long P = m.mlp_params;
  const int pb = (int)std::min<long long>((P + 255) / 256, 1024);
  hipLaunchKernelGGL(pack_kernel<T>, dim3(pb), dim3(256), 0, s, pg, (int)m.c0, (int)m.c1, (int)m.channels,
                     (int)m.hidden, P, mlp, w, bias, bwd ? 1 : 0, (int)m.b0, (int)m.b1, paired ? 1 : 0,
                     (int)m.lod_input);
  return hipGetLastError();
}

hipError_t launch_pack_mlp(const ntc_material& m, const float* mlp, bool f16, bool with_backward, void* packed,
                           hipStream_t s) {
  return f16 ? pack_t<_Float16>(m, mlp, with_backward, packed, s) : pack_t<float>(m, mlp, with_backward, packed, s);
}

// ------------------------------------------------------------------ FP8-e4m3 decode pack
// Layout: e4m3 weights (fwd_end bytes, 16-byte padded) | scales s1 s2 s3 (+1 pad float)
// | b1 (Hd) b2 (Hd) b3 (C) FP32.  s_l = max|W_l| / 448 (1 for an all-zero layer); the
// stored weight is the e4m3 rounding of W / s_l.
__global__ void fp8_scale_kernel(const float* __restrict__ mlp, int K, int Hd, int C, float* __restrict__ scales) {
  __shared__ float red[256];
  const int l = blockIdx.x;
  const long long off = l == 0 ? 0 : l == 1 ? (long long)K * Hd + Hd : (long long)K * Hd + Hd + (long long)Hd * Hd + Hd;
  const long long cnt = l == 0 ? (long long)K * Hd : l == 1 ? (long long)Hd * Hd : (long long)Hd * C;
  float mx = 0.f;
  for (long long i = threadIdx.x; i < cnt; i += 256) mx = fmaxf(mx, fabsf(mlp[off + i]));
  red[threadIdx.x] = mx;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) scales[l] = red[0] > 0.f ? red[0] / 448.f : 1.f;
  if (threadIdx.x == 0 && l == 0) scales[3] = 0.f;
}

__global__ void pack_fp8_kernel(PackGeom pg, int c0, int c1, int C, int Hd, int b0, int b1, long long P, int K,
                                const float* __restrict__ mlp, uint8_t* __restrict__ pack,
                                const float* __restrict__ scales, float* __restrict__ bias_out) {
  const long long nW1 = K * Hd, nW2 = (long long)Hd * Hd, nW3 = (long long)Hd * C;
  const float s1 = scales[0], s2 = scales[1], s3 = scales[2];
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const float v = mlp[p];
    long long q = p;
    if (q < nW1) {
      const int k = (int)(q / Hd), h = (int)(q % Hd);
      int g, t;
      in_slot_of_fp8(k, c0, c1, b0, b1, g, t);
      pack[pg.L1 + pack_index<uint8_t>(pg.S1, h / 16, t, 16 * g + h % 16)] = (uint8_t)cvt_e4m3x2(v / s1, 0.f, 0, false);
      continue;
    }
    q -= nW1;
    if (q < Hd) { bias_out[q] = v; continue; }
    q -= Hd;
    if (q < nW2) {
      const int h1 = (int)(q / Hd), h2 = (int)(q % Hd);
      int g, t;
      hid_slot_of(h1, g, t);
      pack[pg.L2 + pack_index<uint8_t>(pg.SH, h2 / 16, t, 16 * g + h2 % 16)] = (uint8_t)cvt_e4m3x2(v / s2, 0.f, 0, false);
      continue;
    }
    q -= nW2;
    if (q < Hd) { bias_out[Hd + q] = v; continue; }
    q -= Hd;
    if (q < nW3) {
      const int h = (int)(q / C), c = (int)(q % C);
      int g, t;
      hid_slot_of(h, g, t);
      pack[pg.L3 + pack_index<uint8_t>(pg.SH, 0, t, 16 * g + c)] = (uint8_t)cvt_e4m3x2(v / s3, 0.f, 0, false);
      continue;
    }
    q -= nW3;
    bias_out[2 * Hd + q] = v;
  }
}

size_t fp8_pack_weight_bytes(const ntc_material& m) {
  const PackGeom pg = pack_geom_fp8(m.c0, m.c1, m.b0, m.b1, m.hidden);
  return ((size_t)pg.fwd_end + 15) / 16 * 16;
}

hipError_t launch_pack_mlp_fp8(const ntc_material& m, const float* mlp, void* packed, hipStream_t s) {
  const PackGeom pg = pack_geom_fp8(m.c0, m.c1, m.b0, m.b1, m.hidden);
  const size_t wb = fp8_pack_weight_bytes(m);
  uint8_t* w = (uint8_t*)packed;
  float* scales = (float*)((char*)packed + wb);
  float* bias = scales + 4;
  const int zb = (int)std::min<long long>(((long long)wb + 255) / 256, 1024);
  hipLaunchKernelGGL(zero_kernel<uint8_t>, dim3(zb), dim3(256), 0, s, w, (long long)wb);
  hipLaunchKernelGGL(fp8_scale_kernel, dim3(3), dim3(256), 0, s, mlp, (int)m.input_width, (int)m.hidden,
                     (int)m.channels, scales);
  const long long P = m.mlp_params;
  const int pb = (int)std::min<long long>((P + 255) / 256, 1024);
  hipLaunchKernelGGL(pack_fp8_kernel, dim3(pb), dim3(256), 0, s, pg, (int)m.c0, (int)m.c1, (int)m.channels,
                     (int)m.hidden, (int)m.b0, (int)m.b1, P, (int)m.input_width, mlp, w, (const float*)scales, bias);
  return hipGetLastError();
}

}  // namespace ntc
