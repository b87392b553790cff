// Training step of the autodecoder (sections 4.2, 4.5, 5.1) as three kernels:
//
//  1. train_fused_kernel: per 16-texel tile and wavefront, gather latents + PE,
//     MLP forward on matrix cores, L2 loss and dY, backward through the three
//     layers (transposed-weight packs, activations kept in registers), scatter of
//     the latent gradients with float atomics.  Weight gradients need the texel
//     dimension as the reduction axis, so each block of 4 wavefronts stages its 64
//     texels' activations and deltas through LDS (transpose) and accumulates
//     dW += A^T dZ on the matrix cores into registers that persist over all tiles
//     the block processes; each wavefront owns a disjoint set of dW tiles.  The
//     block writes one partial gradient vector at the end (no atomics on weights).
//  2. reduce_kernel: sums the per-block partials in a fixed order (deterministic),
//     flags non-finite gradients, finalises the loss.
//  3. adam_kernel: dense bias-corrected Adam on every parameter, clamp of the
//     latents to the quantization range, zeroing of the latent gradient, the next
//     step's noisy forward latents, the refreshed weight packs and, for FP16, the
//     dynamic loss scale.
#include <algorithm>

#include "ntc_internal.h"

namespace ntc {

struct TrainArgs {
  const float* lat_fwd;
  const void* wpack;
  const float* mlp;
  const ntc_query* q;
  long long n;
  const float* targets;
  const float* dout;
  float* lat_grad;
  float* part_dw;
  float* part_loss;
  const float* loss_scale;
  int scale_slot;
  int32_t* overflow_flag;
  int scatter;
  float inv_nc;
};

template <typename T>
constexpr int lds_row_stride() { return sizeof(T) == 4 ? 68 : 72; }

// dW tile += A rows [rowA, rowA+16) x B rows [rowB, rowB+16) summed over the 64
// texel columns of the block tile.  Lane group g covers texels 16g .. 16g+15.
template <typename T>
__device__ inline f32x4 dw_tile(f32x4 acc, const T* buf, int rowA, int rowB, int g, int r) {
  constexpr int RS = lds_row_stride<T>();
  const T* a = buf + (rowA + r) * RS + 16 * g;
  const T* b = buf + (rowB + r) * RS + 16 * g;
  if constexpr (sizeof(T) == 4) {
    f32x4 av[4], bv[4];
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      av[k] = reinterpret_cast<const f32x4*>(a)[k];
      bv[k] = reinterpret_cast<const f32x4*>(b)[k];
    }
#pragma unroll
    for (int k = 0; k < 16; ++k)
      acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[k / 4][k % 4], bv[k / 4][k % 4], acc, 0, 0, 0);
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const f16x8 av = reinterpret_cast<const f16x8*>(a)[k];
      const f16x8 bv = reinterpret_cast<const f16x8*>(b)[k];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
    }
  }
  return acc;
}

constexpr int cmax(int x, int y) { return x > y ? x : y; }

template <typename T, int C0, int C1, int C, int HD>
struct TrainCfg {
  using IS = InSlots<C0, C1>;
  static constexpr PackGeom pg = pack_geom(C0, C1, HD, sizeof(T) == 2);
  static constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT, ML = pg.ML;
  static constexpr int MT1 = (S1 + 3) / 4;        // dW1 M-tiles (X slot rows 4t+g)
  static constexpr int RX = 16 * MT1;              // X rows in the transpose buffer
  static constexpr int RS = lds_row_stride<T>();
  static constexpr int TR = cmax(cmax(RX + HD, 2 * HD), HD + 16);  // rows of the transpose buffer
  static constexpr int NT2 = (MT * MT + 3) / 4;    // dW2 tiles per wavefront
  static constexpr int NT1 = (MT1 * MT + 3) / 4;   // dW1 tiles per wavefront
  static constexpr long long K = 4 * C0 + C1 + 12;
  static constexpr long long P = K * HD + HD + (long long)HD * HD + HD + (long long)HD * C + C;
  static constexpr long long W1o = 0, b1o = K * HD, W2o = b1o + HD, b2o = W2o + (long long)HD * HD;
  static constexpr long long W3o = b2o + HD, b3o = W3o + (long long)HD * C;
  static constexpr int WB = ((int)pg.train_end * (int)sizeof(T) + 15) / 16 * 16;
  static constexpr int OFF_PE = WB;
  static constexpr int OFF_BIAS = OFF_PE + 48 * 4;
  static constexpr int OFF_TAB = OFF_BIAS + (2 * HD + 16) * 4;    // g0_off[8], g1_off[8], mip_off[16]
  static constexpr int OFF_RED = OFF_TAB + 32 * 8;
  static constexpr int OFF_BUF = (OFF_RED + 16 + 15) / 16 * 16;
  static constexpr int LDS = OFF_BUF + TR * RS * (int)sizeof(T);
};

template <typename T, int C0, int C1, int C, int HD, bool EXT_DY>
__global__ __launch_bounds__(256) void train_fused_kernel(DevMat m, PeTable pe, TrainArgs a) {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  using IS = typename Cfg::IS;
  constexpr PackGeom pg = Cfg::pg;
  constexpr int S1 = Cfg::S1, SH = Cfg::SH, MT = Cfg::MT, ML = Cfg::ML, MT1 = Cfg::MT1, RX = Cfg::RX;
  constexpr int RS = Cfg::RS;
  extern __shared__ __align__(16) char smem[];
  T* w_lds = reinterpret_cast<T*>(smem);
  float* pe_lds = reinterpret_cast<float*>(smem + Cfg::OFF_PE);
  float* b_lds = reinterpret_cast<float*>(smem + Cfg::OFF_BIAS);
  long long* tab = reinterpret_cast<long long*>(smem + Cfg::OFF_TAB);
  float* red = reinterpret_cast<float*>(smem + Cfg::OFF_RED);
  T* buf = reinterpret_cast<T*>(smem + Cfg::OFF_BUF);

  const int tid = threadIdx.x;
  for (int i = tid; i < Cfg::WB / 16; i += 256)
    reinterpret_cast<uint4*>(smem)[i] = reinterpret_cast<const uint4*>(a.wpack)[i];
  for (int i = tid; i < 48; i += 256) pe_lds[i] = pe.v[i / 6][i % 6];
  for (int i = tid; i < 2 * HD + 16; i += 256) {
    float v = 0.f;
    if (i < HD) v = a.mlp[Cfg::b1o + i];
    else if (i < 2 * HD) v = a.mlp[Cfg::b2o + i - HD];
    else if (i < 2 * HD + C) v = a.mlp[Cfg::b3o + i - 2 * HD];
    b_lds[i] = v;
  }
  if (tid < 8) { tab[tid] = m.g0_off[tid]; tab[8 + tid] = m.g1_off[tid]; }
  if (tid < 16) tab[16 + tid] = m.mip_off[tid];
  if (blockIdx.x == 0 && tid == 0 && !EXT_DY) *a.overflow_flag = 0;
  __syncthreads();

  const float scale = a.loss_scale ? a.loss_scale[a.scale_slot] : 1.f;
  const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;
  const int act = m.act;

  f32x4 acc3 = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc2[Cfg::NT2], acc1[Cfg::NT1];
#pragma unroll
  for (int k = 0; k < Cfg::NT2; ++k) acc2[k] = acc3;
#pragma unroll
  for (int k = 0; k < Cfg::NT1; ++k) acc1[k] = acc3;
  float db1 = 0.f, db2 = 0.f, db3 = 0.f, loss = 0.f;

  const long long tiles = (a.n + 63) / 64;
  for (long long tile = blockIdx.x; tile < tiles; tile += gridDim.x) {
    const long long s = tile * 64 + wave * 16 + r;
    const bool valid = s < a.n;
    float u = 0.f, v = 0.f;
    int lod = 0;
    if (valid) {
      u = a.q[s].u;
      v = a.q[s].v;
      lod = a.q[s].lod;
    }
    const Footprint f = locate(m, u, v, lod, g);
    const long long g0base = tab[f.j] + (long long)f.g0_cell * C0;
    const long long g1base = tab[8 + f.j];

    // ---------------- gather (forward latents already hold this step's noise)
    T xs[S1];
#pragma unroll
    for (int t = 0; t < C0; ++t) xs[t] = (T)a.lat_fwd[g0base + t];
#pragma unroll
    for (int i = 0; i < IS::n1max; ++i) {
      const int ch = g + 4 * i;
      float acc = 0.f;
      if (ch < C1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) acc += f.g1_w[k] * a.lat_fwd[g1base + (long long)f.g1_cell[k] * C1 + ch];
      }
      xs[C0 + i] = (T)acc;
    }
    {
      float pv[3];
      pe_values(pe_lds, f.ix, f.iy, g, pv);
#pragma unroll
      for (int k = 0; k < 3; ++k) xs[IS::T_lat + k] = (T)pv[k];
#pragma unroll
      for (int t = IS::T_used; t < S1; ++t) xs[t] = (T)0.f;
    }
    if (!valid) {
#pragma unroll
      for (int t = 0; t < S1; ++t) xs[t] = (T)0.f;
    }

    // ---------------- forward
    float z1[SH], z2[SH];
    T hs[SH];
    f32x4 acc[MT];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + 16 * mo + 4 * g);
      acc[mo] = mma_slots<S1>(acc[mo], w_lds + pg.L1 + mo * S1 * 64, xs, lane);
    }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z1[4 * mo + i] = acc[mo][i];
        hs[4 * mo + i] = (T)act_fn(acc[mo][i], act);
      }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + HD + 16 * mo + 4 * g);
      acc[mo] = mma_slots<SH>(acc[mo], w_lds + pg.L2 + mo * SH * 64, hs, lane);
    }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        z2[4 * mo + i] = acc[mo][i];
        hs[4 * mo + i] = (T)act_fn(acc[mo][i], act);
      }
    f32x4 y = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
    y = mma_slots<SH>(y, w_lds + pg.L3, hs, lane);

    // ---------------- loss and output gradient (lane group g: channels 4g..4g+3)
    T dyT[4];
    float dyv[4];
    {
      const int l = f.l;
      const long long tb = tab[16 + l] + ((long long)f.iy * m.mip_w[l] + f.ix) * C;
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int c = 4 * g + i;
        float d = 0.f;
        if (valid && c < C) {
          if constexpr (EXT_DY) {
            d = a.dout[s * C + c] * scale;
          } else {
            const float e = y[i] - a.targets[tb + c];
            loss += e * e;
            d = 2.f * e * a.inv_nc * scale;
          }
        }
        dyv[i] = d;
        dyT[i] = (T)d;
      }
    }

    // ---------------- backward through the layers
    float dz2[SH], dz1[SH];
    T dT[SH];
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
      d = mma_slots<4>(d, w_lds + pg.B3 + mo * 4 * 64, dyT, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        dz2[4 * mo + i] = d[i] * act_grad(z2[4 * mo + i], act);
        dT[4 * mo + i] = (T)dz2[4 * mo + i];
      }
    }
#pragma unroll
    for (int mo = 0; mo < MT; ++mo) {
      f32x4 d = {0.f, 0.f, 0.f, 0.f};
      d = mma_slots<SH>(d, w_lds + pg.B2 + mo * SH * 64, dT, lane);
#pragma unroll
      for (int i = 0; i < 4; ++i) dz1[4 * mo + i] = d[i] * act_grad(z1[4 * mo + i], act);
    }
    T dz1T[SH];
#pragma unroll
    for (int t = 0; t < SH; ++t) dz1T[t] = (T)dz1[t];

    if (a.scatter) {  // wavefront-uniform: the matrix-core ops run for every lane
      float dx[4 * ML];
#pragma unroll
      for (int mo = 0; mo < ML; ++mo) {
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        d = mma_slots<SH>(d, w_lds + pg.B1 + mo * SH * 64, dz1T, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) dx[4 * mo + i] = d[i];
      }
      if (valid) {
        float* gl = a.lat_grad;
#pragma unroll
        for (int t = 0; t < C0; ++t) unsafeAtomicAdd(gl + g0base + t, dx[t]);
#pragma unroll
        for (int i = 0; i < IS::n1max; ++i) {
          const int ch = g + 4 * i;
          if (ch < C1) {
#pragma unroll
            for (int k = 0; k < 4; ++k)
              if (f.g1_w[k] != 0.f)
                unsafeAtomicAdd(gl + g1base + (long long)f.g1_cell[k] * C1 + ch, f.g1_w[k] * dx[C0 + i]);
          }
        }
      }
    }

    // ---------------- weight gradients through LDS (texels become the K axis)
    const int col = wave * 16 + r;
    // layer 3: H2 rows [0, HD), dY rows [HD, HD + 16)
#pragma unroll
    for (int t = 0; t < SH; ++t) buf[hid_feature(g, t) * RS + col] = valid ? (T)act_fn(z2[t], act) : (T)0.f;
#pragma unroll
    for (int i = 0; i < 4; ++i) buf[(HD + 4 * g + i) * RS + col] = dyT[i];
    __syncthreads();
    if (wave < MT) acc3 = dw_tile<T>(acc3, buf, 16 * wave, HD, g, r);
    if (tid < 16) {
      float sum = 0.f;
#pragma unroll 8
      for (int c = 0; c < 64; ++c) sum += (float)buf[(HD + tid) * RS + c];
      db3 += sum;
    }
    __syncthreads();
    // layer 2: H1 rows [0, HD), dZ2 rows [HD, 2 HD)
#pragma unroll
    for (int t = 0; t < SH; ++t) {
      buf[hid_feature(g, t) * RS + col] = valid ? (T)act_fn(z1[t], act) : (T)0.f;
      buf[(HD + hid_feature(g, t)) * RS + col] = dT[t];
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Cfg::NT2; ++k) {
      const int id = wave + 4 * k;
      if (id < MT * MT) acc2[k] = dw_tile<T>(acc2[k], buf, 16 * (id / MT), HD + 16 * (id % MT), g, r);
    }
    if (tid < HD) {
      float sum = 0.f;
#pragma unroll 8
      for (int c = 0; c < 64; ++c) sum += (float)buf[(HD + tid) * RS + c];
      db2 += sum;
    }
    __syncthreads();
    // layer 1: X slot rows 4t+g in [0, RX), dZ1 rows [RX, RX + HD)
#pragma unroll
    for (int t = 0; t < 4 * MT1; ++t) buf[(4 * t + g) * RS + col] = t < S1 ? xs[t] : (T)0.f;
#pragma unroll
    for (int t = 0; t < SH; ++t) buf[(RX + hid_feature(g, t)) * RS + col] = dz1T[t];
    __syncthreads();
#pragma unroll
    for (int k = 0; k < Cfg::NT1; ++k) {
      const int id = wave + 4 * k;
      if (id < MT1 * MT) acc1[k] = dw_tile<T>(acc1[k], buf, 16 * (id / MT), RX + 16 * (id % MT), g, r);
    }
    if (tid < HD) {
      float sum = 0.f;
#pragma unroll 8
      for (int c = 0; c < 64; ++c) sum += (float)buf[(RX + tid) * RS + c];
      db1 += sum;
    }
    __syncthreads();
  }

  // ---------------- per-block partial gradient (canonical layout) and loss
  float* part = a.part_dw + (long long)blockIdx.x * Cfg::P;
  if (wave < MT) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * wave + 4 * g + i;
      if (r < C) part[Cfg::W3o + (long long)h * C + r] = acc3[i];
    }
  }
#pragma unroll
  for (int k = 0; k < Cfg::NT2; ++k) {
    const int id = wave + 4 * k;
    if (id < MT * MT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int h1 = 16 * (id / MT) + 4 * g + i, h2 = 16 * (id % MT) + r;
        part[Cfg::W2o + (long long)h1 * HD + h2] = acc2[k][i];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < Cfg::NT1; ++k) {
    const int id = wave + 4 * k;
    if (id < MT1 * MT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = 4 * (id / MT) + g;  // slot row 4t + gi, gi = i
        const int kin = t < S1 ? IS::psi(i, t) : -1;
        const int h = 16 * (id % MT) + r;
        if (kin >= 0) part[Cfg::W1o + (long long)kin * HD + h] = acc1[k][i];
      }
    }
  }
  if (tid < HD) {
    part[Cfg::b1o + tid] = db1;
    part[Cfg::b2o + tid] = db2;
  }
  if (tid < C) part[Cfg::b3o + tid] = db3;
  // loss: wavefront then block reduction
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if (lane == 0) red[wave] = loss;
  __syncthreads();
  if (tid == 0) a.part_loss[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ void reduce_kernel(int grid, long long P, const float* __restrict__ part, const float* __restrict__ part_loss,
                              float* __restrict__ grad, float* __restrict__ loss_out, float norm, int32_t* flag) {
  for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < P; p += (long long)gridDim.x * blockDim.x) {
    float s = 0.f;
    for (int b = 0; b < grid; ++b) s += part[(long long)b * P + p];
    grad[p] = s;
    if (flag && !isfinite(s)) atomicOr(flag, 1);
  }
  if (blockIdx.x == 0 && loss_out) {
    __shared__ float red[256];
    float s = 0.f;
    for (int b = threadIdx.x; b < grid; b += blockDim.x) s += part_loss[b];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
      if ((int)threadIdx.x < w) red[threadIdx.x] += red[threadIdx.x + w];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss_out = red[0] * norm;
  }
}

// Bits of the grid holding latent i (grids are contiguous in canonical order).
__device__ inline int latent_bits(const DevMat& m, long long i) {
  int bits = m.B0;
#pragma unroll 1
  for (int j = 0; j < m.J; ++j) {
    if (i >= m.g0_off[j]) bits = m.B0;
    if (i >= m.g1_off[j]) bits = m.B1;
  }
  return bits;
}

struct AdamArgs {
  AdamLaunch a;
  PackGeom pg;
  long long P;
  int mlp_blocks;
};

template <typename T>
__global__ __launch_bounds__(256) void adam_kernel(DevMat m, AdamArgs args) {
  const AdamLaunch& a = args.a;
  const int ovf = a.scale_state[1];
  const float scale = a.loss_scale ? a.loss_scale[a.step & 1] : 1.f;
  const float inv_s = 1.f / scale;
  const float b1 = a.beta1, b2 = a.beta2, eps = a.eps;
  const float ib1 = 1.f / a.bc1, ib2 = 1.f / a.bc2;
  if ((int)blockIdx.x < args.mlp_blocks) {
    const long long p = blockIdx.x * 256ll + threadIdx.x;
    if (p < args.P && !ovf) {
      const float gr = a.mlp_grad[p] * inv_s;
      const float mm = b1 * a.mlp_m[p] + (1.f - b1) * gr;
      const float vv = b2 * a.mlp_v[p] + (1.f - b2) * gr * gr;
      const float w = a.mlp[p] - a.lr_mlp * (mm * ib1) / (sqrtf(vv * ib2) + eps);
      a.mlp_m[p] = mm;
      a.mlp_v[p] = vv;
      a.mlp[p] = w;
      scatter_param<T>((T*)a.wpack, args.pg, m.C0, m.C1, m.C, m.Hd, p, w, true);
    }
    if (blockIdx.x == 0 && threadIdx.x == 0 && a.loss_scale) {
      float sn = scale;
      int good = a.scale_state[0];
      if (ovf) {
        sn = scale * 0.5f;
        good = 0;
      } else if (++good >= a.growth) {
        sn = scale * 2.f;
        good = 0;
      }
      a.loss_scale[(a.step + 1) & 1] = sn;
      a.scale_state[0] = good;
    }
    return;
  }
  if (a.freeze) return;
  const long long base = ((long long)blockIdx.x - args.mlp_blocks) * 256 + threadIdx.x;
  const long long stride = ((long long)gridDim.x - args.mlp_blocks) * 256;
  for (long long i = base; i < m.latent_count; i += stride) {
    const int bits = latent_bits(m, i);
    float p = a.latents[i];
    if (!ovf) {
      const float gr = a.lat_grad[i] * inv_s;
      const float mm = b1 * a.lat_m[i] + (1.f - b1) * gr;
      const float vv = b2 * a.lat_v[i] + (1.f - b2) * gr * gr;
      p = p - a.lr_lat * (mm * ib1) / (sqrtf(vv * ib2) + eps);
      const float lo = -0.5f + ldexpf(1.f, -bits - 1);  // -(N-1)/(2N)
      p = fminf(fmaxf(p, lo), 0.5f);
      a.lat_m[i] = mm;
      a.lat_v[i] = vv;
      a.latents[i] = p;
    }
    a.lat_grad[i] = 0.f;
    a.latents_fwd[i] = a.noise ? p + noise_at(a.next_key, i, bits) : p;
  }
}

__global__ void prepare_kernel(DevMat m, const float* __restrict__ lat, float* __restrict__ fwd, float* __restrict__ grad,
                               uint64_t key, int noise) {
  for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m.latent_count;
       i += (long long)gridDim.x * blockDim.x) {
    const float p = lat[i];
    fwd[i] = noise ? p + noise_at(key, i, latent_bits(m, i)) : p;
    grad[i] = 0.f;
  }
}

// ------------------------------------------------------------------ launchers
template <typename T, int C0, int C1, int C, int HD, bool EXT>
static int fused_per_cu() {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  int per_cu = 0;
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, train_fused_kernel<T, C0, C1, C, HD, EXT>, 256, Cfg::LDS) !=
          hipSuccess ||
      per_cu < 1)
    per_cu = 1;
  return per_cu;
}

template <typename T, int C0, int C1, int C, int HD>
static int grid_t(long long n) {
  const long long tiles = (n + 63) / 64;
  const long long cap = (long long)device_cus() * fused_per_cu<T, C0, C1, C, HD, false>();
  return (int)std::max<long long>(1, std::min(tiles, cap));
}

template <typename T, int C0, int C1, int C, int HD>
static hipError_t fused_t(const ntc_material& mm, const TrainLaunch& l, hipStream_t s) {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  TrainArgs a;
  a.lat_fwd = l.lat_fwd;
  a.wpack = l.wpack;
  a.mlp = l.mlp;
  a.q = l.q;
  a.n = l.n;
  a.targets = l.targets;
  a.dout = nullptr;
  a.lat_grad = l.lat_grad;
  a.part_dw = l.part_dw;
  a.part_loss = l.part_loss;
  a.loss_scale = l.loss_scale;
  a.scale_slot = l.scale_slot;
  a.overflow_flag = l.overflow_flag;
  a.scatter = l.scatter_latents ? 1 : 0;
  a.inv_nc = (float)(1.0 / ((double)l.n * C));
  hipLaunchKernelGGL((train_fused_kernel<T, C0, C1, C, HD, false>), dim3(l.grid), dim3(256), Cfg::LDS, s, dev_mat(mm),
                     pe_table(), a);
  return hipGetLastError();
}

#define NTC_TRAIN_SHAPES(X)                                                            \
  X(8, 8, 8, 64) X(10, 10, 10, 64) X(12, 12, 12, 64) X(16, 16, 16, 64) X(8, 8, 8, 32) \
  X(10, 10, 10, 32) X(12, 12, 12, 32) X(16, 16, 16, 32)

bool train_shape_supported(int c0, int c1, int c, int hd) {
#define NTC_X(a, b, cc, h) \
  if (c0 == a && c1 == b && c == cc && hd == h) return true;
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  return false;
}

int train_grid(const ntc_material& m, bool f16, long long n) {
#define NTC_X(a, b, cc, h)                                                    \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h)            \
    return f16 ? grid_t<_Float16, a, b, cc, h>(n) : grid_t<float, a, b, cc, h>(n);
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  return 1;
}

hipError_t launch_train_fused(const ntc_material& m, bool f16, const TrainLaunch& a, hipStream_t s) {
#define NTC_X(a_, b, cc, h)                                                              \
  if (m.c0 == a_ && m.c1 == b && m.channels == cc && m.hidden == h)                      \
    return f16 ? fused_t<_Float16, a_, b, cc, h>(m, a, s) : fused_t<float, a_, b, cc, h>(m, a, s);
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

hipError_t launch_reduce(const ntc_material& m, int grid, const float* part_dw, const float* part_loss, float* grad,
                         float* loss_out, float loss_norm, int32_t* overflow_flag, hipStream_t s) {
  const long long P = m.mlp_params;
  const int blocks = (int)std::max<long long>(1, std::min<long long>((P + 255) / 256, 4096));
  hipLaunchKernelGGL(reduce_kernel, dim3(blocks), dim3(256), 0, s, grid, P, part_dw, part_loss, grad, loss_out,
                     loss_norm, overflow_flag);
  return hipGetLastError();
}

hipError_t launch_adam(const ntc_material& m, const AdamLaunch& a, hipStream_t s) {
  AdamArgs args;
  args.a = a;
  args.pg = pack_geom(m.c0, m.c1, m.hidden, a.f16 != 0);
  args.P = m.mlp_params;
  args.mlp_blocks = (int)((args.P + 255) / 256);
  long long lat_blocks = a.freeze ? 0 : (m.latent_count + 255) / 256;
  const long long cap = (long long)device_cus() * 8;
  if (lat_blocks > cap) lat_blocks = cap;
  const int grid = args.mlp_blocks + (int)lat_blocks;
  if (a.f16)
    hipLaunchKernelGGL(adam_kernel<_Float16>, dim3(grid), dim3(256), 0, s, dev_mat(m), args);
  else
    hipLaunchKernelGGL(adam_kernel<float>, dim3(grid), dim3(256), 0, s, dev_mat(m), args);
  return hipGetLastError();
}

hipError_t launch_prepare(const ntc_material& m, const float* latents, float* latents_fwd, float* lat_grad, uint64_t key,
                          int noise, hipStream_t s) {
  long long blocks = (m.latent_count + 255) / 256;
  const long long cap = (long long)device_cus() * 8;
  if (blocks > cap) blocks = cap;
  if (blocks < 1) blocks = 1;
  hipLaunchKernelGGL(prepare_kernel, dim3((unsigned)blocks), dim3(256), 0, s, dev_mat(m), latents, latents_fwd,
                     lat_grad, key, noise);
  return hipGetLastError();
}

}  // namespace ntc
