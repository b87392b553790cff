// Training batches of the paper's optimiser (section 5.1): crops of texels from one
// level of detail per batch, the level drawn from an exponential distribution
// (LOD = floor(-log4 X)) or, for a fraction of the batches, uniformly.
#include "ntc_internal.h"

namespace ntc {

constexpr uint64_t kCropTag = 0x63726F70ull;

__device__ inline uint64_t crop_rand(uint64_t key, int i) { return mix64(key + kGamma * (uint64_t)(i + 1)); }

__global__ void crop_kernel(DevMat m, uint64_t key, int crops, int side, double fraction, ntc_query* __restrict__ out,
                            long long n) {
  // the batch's level of detail, recomputed by every thread from the same counters
  const double X = 1.0 - (double)(crop_rand(key, 0) >> 11) * 0x1p-53;
  int lod = 0;
  if ((double)(crop_rand(key, 1) >> 11) * 0x1p-53 < fraction) {
    lod = (int)(crop_rand(key, 2) % (uint64_t)m.M);
  } else {
    double p = 0.25;  // largest k with X <= 4^-k: exact comparisons with powers of four
    while (lod + 1 < m.M && X <= p) {
      ++lod;
      p *= 0.25;
    }
  }
  const int wl = m.mip_w[lod], hl = m.mip_h[lod];
  const float iw = 1.f / (float)wl, ih = 1.f / (float)hl;  // powers of two: exact
  const long long per = (long long)side * side;
  for (long long s = blockIdx.x * (long long)blockDim.x + threadIdx.x; s < n; s += (long long)gridDim.x * blockDim.x) {
    const int c = (int)(s / per);
    const int rem = (int)(s - (long long)c * per), jy = rem / side, ix = rem - jy * side;
    const int x0 = wl >= side ? (int)(crop_rand(key, 3 + 2 * c) % (uint64_t)(wl - side + 1)) : 0;
    const int y0 = hl >= side ? (int)(crop_rand(key, 4 + 2 * c) % (uint64_t)(hl - side + 1)) : 0;
    const int x = (x0 + ix) % wl, y = (y0 + jy) % hl;
    ntc_query q;
    q.u = ((float)x + 0.5f) * iw;
    q.v = ((float)y + 0.5f) * ih;
    q.lod = lod;
    out[s] = q;
  }
}

hipError_t launch_crop_queries(const ntc_material& mm, uint64_t seed, int step, int crops, int side, double fraction,
                               ntc_query* out, hipStream_t s) {
  const uint64_t key = mix64(mix64(seed ^ kCropTag) + kGamma * (uint64_t)(step + 1));
  const long long n = (long long)crops * side * side;
  long long grid = (n + 255) / 256;
  const long long cap = (long long)device_cus() * 8;
  if (grid > cap) grid = cap;
  hipLaunchKernelGGL(crop_kernel, dim3((unsigned)grid), dim3(256), 0, s, dev_mat(mm), key, crops, side, fraction, out, n);
  return hipGetLastError();
}

}  // namespace ntc
