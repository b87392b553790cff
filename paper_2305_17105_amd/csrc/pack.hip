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
                            T* __restrict__ pack, float* __restrict__ bias_out, int bwd, int b0, int b1, int paired) {
  const long long K = 4 * c0 + c1 + 12;
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    const float v = mlp[p];
    scatter_param<T>(pack, pg, c0, c1, C, Hd, p, v, bwd != 0, b0, b1, paired != 0);
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
                     (int)m.hidden, P, mlp, w, bias, bwd ? 1 : 0, (int)m.b0, (int)m.b1, paired ? 1 : 0);
  return hipGetLastError();
}

hipError_t launch_pack_mlp(const ntc_material& m, const float* mlp, bool f16, bool with_backward, void* packed,
                           hipStream_t s) {
  return f16 ? pack_t<_Float16>(m, mlp, with_backward, packed, s) : pack_t<float>(m, mlp, with_backward, packed, s);
}

}  // namespace ntc
