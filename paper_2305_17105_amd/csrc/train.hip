// Training step of the autodecoder (sections 4.2, 4.5, 5.1).
//
// Latent gradients are not scattered with global atomics (hot-set float atomics
// serialise on small grids and even spread ones run at ~20 G/s on this GPU).
// Instead every feature level is cut into spatial tiles that own their latents:
//
//  1. bin_count / bin_scan / bin_scatter: each sample is listed under every tile
//     whose latents its footprint (2x2 G0 cells, 4 G1 taps) touches (at most 4),
//     a counting sort with per-block LDS histograms.  A tile's list is cut into
//     work items of at most `chunk` samples (a plan parameter).
//  2. train_fused_kernel: a persistent block takes work items; for each step of
//     16 texels per wavefront it gathers latents + PE, runs the MLP forward on matrix cores, the
//     L2 loss and dY, the backward through the three layers (transposed-weight
//     packs, activations in registers), accumulates the gradients of the latents
//     the tile owns in LDS (LDS atomics), and adds dW += A^T dZ through an LDS
//     transpose into per-wavefront register accumulators.  Loss and weight
//     gradients count a sample only in its primary tile (the one holding its
//     footprint anchor); secondary copies only feed the owned latents.  At the end
//     of a work item the tile's gradient is written densely with plain stores
//     (single-item tiles) or as a partial (tiles split over several items).
//  3. lat_partial_reduce: sums the partials of split tiles in a fixed order.
//  4. dw_reduce: per-block weight-gradient partials summed in a fixed order,
//     non-finite check, loss.
//  5. adam_kernel: dense bias-corrected Adam, clamp to the quantization range, next
//     step's noisy forward latents, refreshed weight packs, FP16 loss scale.
#include <algorithm>
#include <cstring>
#include <mutex>
#include <type_traits>
#include <vector>

#include "ntc_internal.h"

namespace ntc {

constexpr int kChunkDefault = 256;  // samples per work item unless tuned (tiles of at most 16 x 16)
constexpr int kBinBlockSamples = 1024;
constexpr int kBinThreads = 1024;  // threads of a binning block (one sample each)
constexpr int kMaxBins = 24576;   // LDS histogram capacity of the binning kernels (96 KiB)
constexpr int kSortedCells = 4096; // levels with at most this many G0 cells are sorted by anchor cell

struct TrainArgs {
  const float* lat_fwd;
  const void* wpack;
  const float* mlp;
  const ntc_query* q;
  long long n;
  const float* targets;
  float* lat_grad;
  float* part_lat;
  const int4* list;        // binned samples: (u bits, v bits, lod, sample index)
  const int* tile_start;   // first list position of each tile's samples
  const int* tile_total;   // number of list entries of each tile
  const int* item_base;    // first work item of each tile (ntiles + 1)
  const int* item_tile;    // tile of each work item
  const int* nitems;
  float* part_dw;
  float* part_loss;
  const float* loss_scale;
  int scale_slot;
  const int* step_dev;
  int32_t* overflow_flag;
  int binned;
  int region_max;
  float inv_nc;
  const float* dout;   // external output gradient (differentiation path) or nullptr
  float dout_scale;    // multiplies dout before the backward (FP16 range)
  float out_scale;     // multiplies the latent gradient written out
  const float* dscale; // device (dout_scale, out_scale) replacing the two above, or nullptr
  const unsigned long long* table_hash;  // grouped step: its table's hash, else nullptr
  unsigned long long hash;               // the hash the grouped step was planned with
  TileGeom tg;
};

// LDS row stride (elements) of the staging buffer for NCOL texel columns: the padding
// shifts consecutive rows by 4 banks
template <typename T, int NCOL>
constexpr int lds_row_stride() { return sizeof(T) == 4 ? NCOL + 4 : NCOL + 8; }

// dW tile += A rows [rowA, rowA+16) x B rows [rowB, rowB+16) summed over the NCOL
// texel columns of the block step.  Lane group g covers texels g*NCOL/4 .. (g+1)*NCOL/4 - 1.
template <typename T, int NCOL>
__device__ inline f32x4 dw_tile(f32x4 acc, const T* buf, int rowA, int rowB, int g, int r) {
  constexpr int RS = lds_row_stride<T, NCOL>(), GC = NCOL / 4;
  const T* a = buf + (rowA + r) * RS + GC * g;
  const T* b = buf + (rowB + r) * RS + GC * g;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < GC / 4; ++k) {
      const f32x4 av = reinterpret_cast<const f32x4*>(a)[k];
      const f32x4 bv = reinterpret_cast<const f32x4*>(b)[k];
#pragma unroll
      for (int e = 0; e < 4; ++e) acc = __builtin_amdgcn_mfma_f32_16x16x4f32(av[e], bv[e], acc, 0, 0, 0);
    }
  } else {
#pragma unroll
    for (int k = 0; k < GC / 8; ++k) {
      const f16x8 av = reinterpret_cast<const f16x8*>(a)[k];
      const f16x8 bv = reinterpret_cast<const f16x8*>(b)[k];
      acc = __builtin_amdgcn_mfma_f32_16x16x32_f16(av, bv, acc, 0, 0, 0);
    }
  }
  return acc;
}

constexpr int cmax(int x, int y) { return x > y ? x : y; }

// Sum of columns 16q .. 16q+15 of LDS row `row`.
template <typename T, int NCOL>
__device__ inline float row_part_sum(const T* buf, int row, int q) {
  constexpr int RS = lds_row_stride<T, NCOL>();
  const T* p = buf + row * RS + 16 * q;
  float s = 0.f;
  if constexpr (sizeof(T) == 4) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const f32x4 v = reinterpret_cast<const f32x4*>(p)[k];
      s += (v[0] + v[1]) + (v[2] + v[3]);
    }
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k) {
      const f16x8 v = reinterpret_cast<const f16x8*>(p)[k];
#pragma unroll
      for (int e = 0; e < 8; ++e) s += (float)v[e];
    }
  }
  return s;
}

template <typename T, int C0, int C1, int C, int HD>
struct TrainCfg {
  using IS = InSlots<C0, C1>;
  static constexpr PackGeom pg = pack_geom(C0, C1, HD, sizeof(T) == 2);
  static constexpr int S1 = pg.S1, SH = pg.SH, MT = pg.MT, ML = pg.ML;
  static constexpr int MT1 = (S1 + 3) / 4;         // dW1 M-tiles (X slot rows 4t+g)
  static constexpr int RX = 16 * MT1;               // X rows in the transpose buffer
  // Wavefronts per block (16 samples each per step) and blocks per CU.  FP16: one
  // block of 8 (2 per SIMD) with three-phase staging and 16 x 16 tiles; measured
  // faster than two blocks of 4 once the latent accumulators are FP64 (which two
  // blocks cannot fit next to a 16 x 16 tile).  FP32: one block of 4 (its packs and
  // staging are twice the size).
  static constexpr int NW = sizeof(T) == 2 ? 8 : 4;
  static constexpr int BPC = 1;
  static constexpr int NTHR = 64 * NW, NCOL = 16 * NW;
  static constexpr int RS = lds_row_stride<T, NCOL>();
  // one-phase weight-gradient staging: rows X | H1 | H2 | dZ1 | dZ2 | dY
  static constexpr int RH1 = RX, RH2 = RX + HD, RDZ1 = RX + 2 * HD, RDZ2 = RX + 3 * HD, RDY = RX + 4 * HD;
  static constexpr int TR1 = RX + 4 * HD + 16;
  static constexpr int TR3 = cmax(cmax(RX + HD, 2 * HD), HD + 16);  // three-phase staging
  // three-phase staging with the layer-1 phase in two halves of the X slot rows (MB row
  // blocks each): FP16 only, where that alone makes room for 32 x 32 tiles
  static constexpr int MB = (MT1 + 1) / 2;
  static constexpr int TR3S = cmax(cmax(16 * MB + HD, 2 * HD), HD + 16);
  static constexpr int NT2 = (MT * MT + NW - 1) / NW;     // dW2 tiles per wavefront
  static constexpr int NT1 = (MT1 * MT + NW - 1) / NW;    // dW1 tiles per wavefront
  static constexpr int WB = ((int)pg.train_end * (int)sizeof(T) + 15) / 16 * 16;
  static constexpr int OFF_PE = WB;
  static constexpr int OFF_BIAS = OFF_PE + 48 * 4;
  static constexpr int OFF_TAB = OFF_BIAS + (2 * HD + 16) * 4;  // g0_off[8], g1_off[8], mip_off[16]
  static constexpr int OFF_RED = OFF_TAB + 32 * 8;
  static constexpr int OFF_FLAG = OFF_RED + 4 * NW;  // two ints: the lost flags of alternate items
  static constexpr int OFF_BUF = (OFF_FLAG + 8 + 15) / 16 * 16;
  static constexpr int region(int t) { return t * t * C0 + (t / 2) * (t / 2) * C1; }
  static constexpr int kLdsCap = 160 * 1024 / BPC;
  static constexpr int buf_bytes(int rows) { return (rows * RS * (int)sizeof(T) + 15) / 16 * 16; }
  // One-phase staging only when it fits next to the accumulators: FP16, a 32 x 32 tile of
  // 4-byte fixed-point sums when three-phase staging would leave room for one, else (and
  // FP32) a 16 x 16 tile of 8-byte sums.  Fast accumulators and large tiles matter more
  // than fewer barriers.
  static constexpr bool ONE_PHASE =
      sizeof(T) == 2 && OFF_BUF + buf_bytes(TR3) + region(32) * 4 <= kLdsCap
          ? OFF_BUF + buf_bytes(TR1) + region(32) * 4 <= kLdsCap
          : OFF_BUF + buf_bytes(TR1) + region(16) * 8 <= kLdsCap;
  static constexpr bool SPLIT1 = sizeof(T) == 2 && !ONE_PHASE && OFF_BUF + buf_bytes(TR3) + region(32) * 4 > kLdsCap &&
                                 OFF_BUF + buf_bytes(TR3S) + region(32) * 4 <= kLdsCap;
  // two-phase staging (layers 3 and 2 together, then layer 1): FP16, where it still
  // leaves room for 32 x 32 tiles
  static constexpr int TR2 = cmax(3 * HD + 16, RX + HD);
  static constexpr bool TWO_PHASE = sizeof(T) == 2 && !ONE_PHASE && !SPLIT1 &&
                                    OFF_BUF + buf_bytes(TR2) + region(32) * 4 <= kLdsCap;
  static constexpr int TR = ONE_PHASE ? TR1 : TWO_PHASE ? TR2 : SPLIT1 ? TR3S : TR3;
  static constexpr int OFF_REG = OFF_BUF + buf_bytes(TR);
  // Owned-latent accumulators: fixed point, so a work item's sums do not depend on the
  // order of its adds (integer LDS adds also run 3x faster than FP64 ones and 25x faster
  // than FP32 ones on this GPU).  FP16 kernels: 32-bit (at 4 bytes a latent a 32 x 32 tile
  // fits); FP32 kernels: 64-bit with a finer quantum where a 16 x 16 tile of them fits,
  // else 32-bit (8 x 8 tiles leave sparse level-0 tiles with a few samples per work item:
  // 2.4x slower on the 16-channel hidden-64 shape).  A work item with a contribution
  // beyond the fixed-point range is summed again in FP32.
  static constexpr bool WIDE_FITS = OFF_REG + region(16) * 8 <= kLdsCap;
  using AccI = typename std::conditional<sizeof(T) == 2 || !WIDE_FITS, int, long long>::type;
  static constexpr int RB = (int)sizeof(AccI);
  // largest tile side whose owned-latent gradient fits next to the rest
  static constexpr int TMAX = OFF_REG + region(32) * RB <= kLdsCap ? 32 : OFF_REG + region(16) * RB <= kLdsCap ? 16 : 8;
  static constexpr int LDS = OFF_REG + region(TMAX) * RB;
};

// One block's share of a material's work items: items [item0, item1) with stride
// `istride`, its weight-gradient partial written to row `row` of a.part_dw (and its
// loss to a.part_loss[row]).  q: the material's queries (samples in query order when
// !binned); scale_slot: the loss-scale slot when the step index is not on the device;
// zero_flag: this block clears the overflow flag.  item1 < 0: all of a.nitems.  step_dev:
// the device step index (its parity picks the loss-scale slot), or nullptr.
template <typename T, int C0, int C1, int C, int HD, int ACT>
__device__ __forceinline__ void fused_body(const DevMat& m, const PeTable& pe, const TrainArgs& a,
                                           const ntc_query* __restrict__ qs, int binned, int scale_slot,
                                           const int* step_dev, int item0, int item1, int istride, int row,
                                           bool zero_flag) {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  using IS = typename Cfg::IS;
  constexpr PackGeom pg = Cfg::pg;
  constexpr int S1 = Cfg::S1, SH = Cfg::SH, MT = Cfg::MT, ML = Cfg::ML, MT1 = Cfg::MT1, RX = Cfg::RX;
  constexpr int RS = Cfg::RS, NW = Cfg::NW, NTHR = Cfg::NTHR, NCOL = Cfg::NCOL;
  extern __shared__ __align__(16) char smem[];
  T* w_lds = reinterpret_cast<T*>(smem);
  float* pe_lds = reinterpret_cast<float*>(smem + Cfg::OFF_PE);
  float* b_lds = reinterpret_cast<float*>(smem + Cfg::OFF_BIAS);
  long long* tab = reinterpret_cast<long long*>(smem + Cfg::OFF_TAB);
  float* red = reinterpret_cast<float*>(smem + Cfg::OFF_RED);
  int* lost_flag = reinterpret_cast<int*>(smem + Cfg::OFF_FLAG);
  T* buf = reinterpret_cast<T*>(smem + Cfg::OFF_BUF);
  using AccI = typename Cfg::AccI;
  constexpr bool WIDE = sizeof(AccI) == 8;
  AccI* ireg = reinterpret_cast<AccI*>(smem + Cfg::OFF_REG);    // fixed-point sums
  float* freg = reinterpret_cast<float*>(smem + Cfg::OFF_REG);  // FP32 sums of a summed-again item
  bool lost = false;  // a contribution of this item left the fixed-point range
  const int tid = threadIdx.x;
  for (int i = tid; i < Cfg::WB / 16; i += NTHR)
    reinterpret_cast<uint4*>(smem)[i] = reinterpret_cast<const uint4*>(a.wpack)[i];
  for (int i = tid; i < 48; i += NTHR) pe_lds[i] = pe.v[i / 6][i % 6];
  // canonical parameter offsets (the input width K includes the optional LOD input)
  const long long b1o = (long long)m.K * HD, W2o = b1o + HD, b2o = W2o + (long long)HD * HD, W3o = b2o + HD;
  const long long b3o = W3o + (long long)HD * C, Pn = b3o + C;
  const float lod_norm = m.lod_in && m.M > 1 ? 1.f / (float)(m.M - 1) : 0.f;
  for (int i = tid; i < 2 * HD + 16; i += NTHR) {
    float v = 0.f;
    if (i < HD) v = a.mlp[b1o + i];
    else if (i < 2 * HD) v = a.mlp[b2o + i - HD];
    else if (i < 2 * HD + C) v = a.mlp[b3o + i - 2 * HD];
    b_lds[i] = v;
  }
  if (tid < 8) {
    tab[tid] = m.g0_off[tid];
    tab[8 + tid] = m.g1_off[tid];
  }
  if (tid < 16) tab[16 + tid] = m.mip_off[tid];
  if (zero_flag && tid == 0) *a.overflow_flag = 0;
  if (tid < 2) lost_flag[tid] = 0;
  // the owned-latent accumulators start at zero; every work item's write-out clears what
  // it read, so they are zero again at the next item whatever its tile size
  for (int k = tid; k < Cfg::region(Cfg::TMAX) * (int)sizeof(AccI) / 16; k += NTHR)
    reinterpret_cast<int4*>(ireg)[k] = int4{0, 0, 0, 0};
  __syncthreads();

  const int slot = step_dev ? (*step_dev & 1) : scale_slot;
  const float scale = a.loss_scale ? a.loss_scale[slot] : 1.f;
  const float dout_scale = a.dscale ? a.dscale[0] : a.dout_scale;
  const float out_scale = a.dscale ? a.dscale[1] : a.out_scale;
  const int lane = tid & 63, wave = tid >> 6, g = lane >> 4, r = lane & 15;

  f32x4 acc3 = {0.f, 0.f, 0.f, 0.f};
  f32x4 acc2[Cfg::NT2], acc1[Cfg::NT1];
#pragma unroll
  for (int k = 0; k < Cfg::NT2; ++k) acc2[k] = acc3;
#pragma unroll
  for (int k = 0; k < Cfg::NT1; ++k) acc1[k] = acc3;
  float db1 = 0.f, db2 = 0.f, db3 = 0.f, loss = 0.f;

  const int chunk_n = a.tg.chunk;
  // The quantum of the fixed-point sums is 2^-16 (FP16 kernels) or 2^-32 (FP32 kernels)
  // of the natural unit U of the output delta (2 x loss scale / (samples x channels) for
  // the loss; 1 for a caller's delta, which comes scaled to O(1)), rounded to a power of
  // two, so the range covers the same multiples of U whatever the batch and the loss
  // scale (FP16: 16 U and more at 512 samples per work item, a rounding error of at most
  // 2^-17 U per contribution).  A latent takes at most 4 adds per sample of a work item
  // (a footprint's taps may coincide at the border), so adds of at most qlim units
  // cannot overflow.
  constexpr int kQBits = WIDE ? 32 : 16;
  float fixq = 0x1p24f;
  {
    const float U = a.dout ? 1.f : 2.f * a.inv_nc * scale;
    int ex = 0;
    if (U > 0.f && U < 0x1p90f) frexpf(U, &ex);
    fixq = ldexpf(1.f, kQBits - max(-80, min(80, ex)));
  }
  const float fixinv = 1.f / fixq;  // exact: a power of two
  const float qlim = WIDE ? fminf(0x1p62f / (float)(4 * chunk_n), 0x1p50f)
                          : fminf((float)(0x7fffffff / (4 * chunk_n)), 0x1p22f);
  const float xlim = qlim * fixinv;  // the largest contribution kept in fixed point (exact)
  // First pass: a contribution x clamped to the range and rounded to the nearest quantum
  // (adding 1.5 * 2^23, or 1.5 * 2^52 in FP64, leaves the integer in the low mantissa
  // bits); a clamped or non-finite x marks the item for the FP32 pass.  Every
  // contribution is rounded on its own, so the integer sums do not depend on how samples
  // are grouped or ordered.
  auto quant = [&](float x) -> AccI {
    const float xc = __builtin_amdgcn_fmed3f(x, -xlim, xlim);
    lost |= x != xc;
    if constexpr (WIDE) {
      return (AccI)(__double_as_longlong(fma((double)xc, (double)fixq, 0x1.8p52)) - 0x4338000000000000ll);
    } else {
      return __float_as_int(fmaf(xc, fixq, 0x1.8p23f)) - 0x4B400000;
    }
  };
  auto add_fixed = [&](int k, AccI v) {
    if constexpr (WIDE) atomicAdd(reinterpret_cast<unsigned long long*>(ireg + k), (unsigned long long)v);
    else atomicAdd(ireg + k, v);
  };
  const int nitems = item1 >= 0 ? item1 : binned ? *a.nitems : (int)((a.n + chunk_n - 1) / chunk_n);
  int par = 0;  // parity of this block's work items: which lost flag is theirs
  for (int item = item0; item < nitems; item += istride, par ^= 1) {
    // ---------------- work item -> (tile, sample range)
    int j = 0, tx = 0, ty = 0, T_ = 2, cnt;
    long long start;
    bool single = true;
    bool sorted = false;
    if (binned) {
      const int tile = a.item_tile[item];
      const int chunk = item - a.item_base[tile];
      single = (a.item_base[tile + 1] - a.item_base[tile]) == 1;
      start = (long long)a.tile_start[tile] + (long long)chunk * chunk_n;
      cnt = min(chunk_n, a.tile_total[tile] - chunk * chunk_n);
      while (j + 1 < m.J && tile >= a.tg.tile_base[j + 1]) ++j;
      const int t = tile - a.tg.tile_base[j];
      tx = t % a.tg.ntx[j];
      ty = t / a.tg.ntx[j];
      T_ = a.tg.T[j];
      sorted = a.tg.sb[j] > 1;
    } else {
      start = (long long)item * chunk_n;
      cnt = (int)min((long long)chunk_n, a.n - start);
    }
    const int T1 = T_ >> 1;
    const int ts = __builtin_ctz(T_), t1s = ts - 1;  // tile sides are powers of two >= 2
    const int R0 = T_ * T_ * C0;
    const int RG = R0 + T1 * T1 * C1;
    // the list entry (query + sample index) of one NCOL-sample step; the next step's
    // entry is loaded before this step's gathers, so it arrives with them
    auto load_entry = [&](int t0, float& u, float& v, int& lod, long long& s) {
      const int pos = t0 + wave * 16 + r;
      u = v = 0.f;
      lod = 0;
      s = 0;
      if (pos < cnt) {
        if (binned) {
          const int4 e = a.list[start + pos];
          u = __int_as_float(e.x);
          v = __int_as_float(e.y);
          lod = e.z;
          s = e.w;
        } else {
          s = start + pos;
          u = qs[s].u;
          v = qs[s].v;
          lod = qs[s].lod;
        }
      }
    };
    // FIXED: pass 1 (refine) sums the item's latent gradients again in FP32 when a
    // contribution left the fixed-point range in pass 0; it skips loss and weights
    bool refined = false;
    for (int pass = 0; pass < 2; ++pass) {
    const bool refine = pass == 1;
    refined = refine;
    if (refine) {  // block-uniform: the FP32 pass starts from zeros (pass 0 found them so)
      for (int k = tid; k < RG; k += NTHR) ireg[k] = (AccI)0;
      __syncthreads();
    }
    float nu, nv;
    int nlod;
    long long ns;
    load_entry(0, nu, nv, nlod, ns);
    for (int t0 = 0; t0 < cnt; t0 += NCOL) {
      const bool valid = t0 + wave * 16 + r < cnt;
      const float u = nu, v = nv;
      const int lod = nlod;
      const long long s = ns;
      if (t0 + NCOL < cnt) load_entry(t0 + NCOL, nu, nv, nlod, ns);
      const Footprint f = locate(m, u, v, lod, g);
      const bool primary = valid && (!binned || ((f.ax >> ts) == tx && (f.ay >> ts) == ty));
      const long long g0base = tab[f.j] + (long long)f.g0_cell * C0;
      const long long g1base = tab[8 + f.j];

      // targets of channels 4g .. 4g + 3, loaded with the gathers so that both arrive
      // while the forward waits for the latents
      float tgt[4] = {0.f, 0.f, 0.f, 0.f};
      if (!a.dout) {
        const long long tb = tab[16 + f.l] + ((long long)f.iy * max(1, m.W >> f.l) + f.ix) * C;  // mip width from m.W (no per-lane argument load)
#pragma unroll
        for (int i = 0; i < 4; ++i)
          if (4 * g + i < C) tgt[i] = a.targets[tb + 4 * g + i];
      }
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
        xs[IS::T_lat + 3] = (T)(g == 0 ? (float)f.l * lod_norm : 0.f);  // LOD input (section 4.4)
#pragma unroll
        for (int t = IS::T_used; t < S1; ++t) xs[t] = (T)0.f;
      }
      if (!valid) {
#pragma unroll
        for (int t = 0; t < S1; ++t) xs[t] = (T)0.f;
      }

      // ---------------- forward
      // h1, h2: activations in the operand type; the pre-activations z are kept only
      // where the activation's derivative needs them (ReLU reads its decision off h)
      float z1[SH], z2[SH];
      T h1[SH], h2[SH];
      f32x4 acc[MT];
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + 16 * mo + 4 * g);
        acc[mo] = mma_slots<S1>(acc[mo], w_lds + pg.L1 + mo * S1 * 64, xs, lane);
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z1[4 * mo + i] = acc[mo][i];
        act4<ACT>(acc[mo], h1 + 4 * mo);
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        acc[mo] = *reinterpret_cast<const f32x4*>(b_lds + HD + 16 * mo + 4 * g);
        acc[mo] = mma_slots<SH>(acc[mo], w_lds + pg.L2 + mo * SH * 64, h1, lane);
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
#pragma unroll
        for (int i = 0; i < 4; ++i) z2[4 * mo + i] = acc[mo][i];
        act4<ACT>(acc[mo], h2 + 4 * mo);
      }
      f32x4 y = *reinterpret_cast<const f32x4*>(b_lds + 2 * HD + 4 * g);
      y = mma_slots<SH>(y, w_lds + pg.L3, h2, lane);

      // ---------------- loss and output gradient (lane group g: channels 4g..4g+3)
      T dyT[4];
      {
#pragma unroll
        for (int i = 0; i < 4; ++i) {
          const int c = 4 * g + i;
          float d = 0.f;
          if (valid && c < C) {
            if (a.dout) {
              d = a.dout[s * C + c] * dout_scale;
            } else {
              const float e = y[i] - tgt[i];
              if (primary && !refine) loss += e * e;
              d = 2.f * e * a.inv_nc * scale;
            }
          }
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
          dz2[4 * mo + i] = d[i] * dact<ACT>(z2[4 * mo + i], h2[4 * mo + i]);
          dT[4 * mo + i] = (T)dz2[4 * mo + i];
        }
      }
#pragma unroll
      for (int mo = 0; mo < MT; ++mo) {
        f32x4 d = {0.f, 0.f, 0.f, 0.f};
        d = mma_slots<SH>(d, w_lds + pg.B2 + mo * SH * 64, dT, lane);
#pragma unroll
        for (int i = 0; i < 4; ++i) dz1[4 * mo + i] = d[i] * dact<ACT>(z1[4 * mo + i], h1[4 * mo + i]);
      }
      T dz1T[SH];
#pragma unroll
      for (int t = 0; t < SH; ++t) dz1T[t] = (T)dz1[t];

      if (binned) {  // block-uniform: the matrix-core ops run for every lane
        float dx[4 * ML];
#pragma unroll
        for (int mo = 0; mo < ML; ++mo) {
          f32x4 d = {0.f, 0.f, 0.f, 0.f};
          d = mma_slots<SH>(d, w_lds + pg.B1 + mo * SH * 64, dz1T, lane);
#pragma unroll
          for (int i = 0; i < 4; ++i) dx[4 * mo + i] = d[i];
        }
        // Gradients of the latents this tile owns, accumulated in LDS.  On levels whose
        // samples are sorted by anchor cell, a row (16 samples of one lane group) that
        // targets a single cell is summed across lanes first (one atomic per channel).
        // The fixed-point pass decides once per footprint cell which lanes add (the row
        // leader its row sum, or every owning lane its own value); every channel's add
        // then runs under that one condition.
        const int rr = lane & 15;
        const bool own0 = valid && (f.g0x >> ts) == tx && (f.g0y >> ts) == ty;
        const int key0 = own0 ? ((f.g0y - ty * T_) * T_ + (f.g0x - tx * T_)) : -1;
        const int dst0 = (key0 < 0 ? 0 : key0) * C0;
        if (!refine) {  // block-uniform
          if (sorted) {
            const int rk = __shfl(key0, lane & ~15);
            const unsigned long long bal = __ballot(key0 == rk || !valid);
            const bool uni = ((bal >> (lane & ~15)) & 0xFFFFull) == 0xFFFFull;
            const bool add = uni ? (rr == 0 && rk >= 0) : own0;
#pragma unroll
            for (int t = 0; t < C0; ++t) {
              const AccI qv = own0 ? quant(dx[t]) : (AccI)0;
              const AccI sq = row_sum16i(qv);
              if (add) add_fixed(dst0 + t, uni ? sq : qv);
            }
          } else if (own0) {
#pragma unroll
            for (int t = 0; t < C0; ++t) add_fixed(dst0 + t, quant(dx[t]));
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int x1 = f.g1x[k & 1], y1 = f.g1y[k >> 1];
            const bool own1 = valid && (x1 >> t1s) == tx && (y1 >> t1s) == ty && f.g1_w[k] != 0.f;
            const int key1 = own1 ? ((y1 - ty * T1) * T1 + (x1 - tx * T1)) : -1;
            const int dst1 = R0 + (key1 < 0 ? 0 : key1) * C1;
            if (sorted) {
              const int rk = __shfl(key1, lane & ~15);
              const unsigned long long bal = __ballot(key1 == rk || !valid);
              const bool uni = ((bal >> (lane & ~15)) & 0xFFFFull) == 0xFFFFull;
              const bool add = uni ? (rr == 0 && rk >= 0) : own1;
#pragma unroll
              for (int i = 0; i < IS::n1max; ++i) {
                const AccI qv = own1 ? quant(f.g1_w[k] * dx[C0 + i]) : (AccI)0;
                const AccI sq = row_sum16i(qv);
                if (add && (4 * i + 3 < C1 || g + 4 * i < C1)) add_fixed(dst1 + g + 4 * i, uni ? sq : qv);
              }
            } else if (own1) {
#pragma unroll
              for (int i = 0; i < IS::n1max; ++i)
                if (4 * i + 3 < C1 || g + 4 * i < C1) add_fixed(dst1 + g + 4 * i, quant(f.g1_w[k] * dx[C0 + i]));
            }
          }
        } else {
          // the FP32 pass of an item whose contributions left the fixed-point range
          if (sorted) {
            const int rk = __shfl(key0, lane & ~15);
            const unsigned long long bal = __ballot(key0 == rk || !valid);
            const bool uni = ((bal >> (lane & ~15)) & 0xFFFFull) == 0xFFFFull;
#pragma unroll
            for (int t = 0; t < C0; ++t) {
              const float sv = row_sum16(own0 ? dx[t] : 0.f);
              if (uni) {
                if (rr == 0 && rk >= 0) atomicAdd(freg + dst0 + t, sv);
              } else if (own0) {
                atomicAdd(freg + dst0 + t, dx[t]);
              }
            }
          } else if (own0) {
#pragma unroll
            for (int t = 0; t < C0; ++t) atomicAdd(freg + dst0 + t, dx[t]);
          }
#pragma unroll
          for (int k = 0; k < 4; ++k) {
            const int x1 = f.g1x[k & 1], y1 = f.g1y[k >> 1];
            const bool own1 = valid && (x1 >> t1s) == tx && (y1 >> t1s) == ty && f.g1_w[k] != 0.f;
            const int key1 = own1 ? ((y1 - ty * T1) * T1 + (x1 - tx * T1)) : -1;
            const int dst1 = R0 + (key1 < 0 ? 0 : key1) * C1;
            if (sorted) {
              const int rk = __shfl(key1, lane & ~15);
              const unsigned long long bal = __ballot(key1 == rk || !valid);
              const bool uni = ((bal >> (lane & ~15)) & 0xFFFFull) == 0xFFFFull;
#pragma unroll
              for (int i = 0; i < IS::n1max; ++i) {
                const int ch = g + 4 * i;
                const float v1 = own1 ? f.g1_w[k] * dx[C0 + i] : 0.f;
                const float sv = row_sum16(v1);
                if (ch < C1) {
                  if (uni) {
                    if (rr == 0 && rk >= 0) atomicAdd(freg + dst1 + ch, sv);
                  } else if (own1) {
                    atomicAdd(freg + dst1 + ch, v1);
                  }
                }
              }
            } else if (own1) {
#pragma unroll
              for (int i = 0; i < IS::n1max; ++i) {
                const int ch = g + 4 * i;
                if (ch < C1) atomicAdd(freg + dst1 + ch, f.g1_w[k] * dx[C0 + i]);
              }
            }
          }
        }
      }

      if (refine) continue;  // block-uniform
      // a lost contribution anywhere in the item: published by the last step's staging
      // barriers (every staging mode has at least one after its stores)
      if (binned && lost && t0 + NCOL >= cnt) lost_flag[par] = 1;
      // ---------------- weight gradients through LDS (texels become the K axis);
      // only a sample's primary copy contributes.  Column wave*16 + r holds texel r of
      // wave `wave`.  Bias gradients are row sums of the deltas: thread (row = tid / PARTS,
      // part = tid % PARTS) adds the 16 columns of its part of the row.
      const int col = wave * 16 + r;
      const T zero = (T)0.f;
      constexpr int PARTS = NCOL / 16;
      const int brow = tid / PARTS, bq = tid % PARTS;
      if constexpr (Cfg::ONE_PHASE) {
        // all operands at once: X | H1 | H2 | dZ1 | dZ2 | dY
#pragma unroll
        for (int t = 0; t < 4 * MT1; ++t) buf[(4 * t + g) * RS + col] = (t < S1 && primary) ? xs[t] : zero;
#pragma unroll
        for (int t = 0; t < SH; ++t) {
          const int h = hid_feature(g, t);
          buf[(Cfg::RH1 + h) * RS + col] = primary ? h1[t] : zero;
          buf[(Cfg::RH2 + h) * RS + col] = primary ? h2[t] : zero;
          buf[(Cfg::RDZ1 + h) * RS + col] = primary ? dz1T[t] : zero;
          buf[(Cfg::RDZ2 + h) * RS + col] = primary ? dT[t] : zero;
        }
#pragma unroll
        for (int i = 0; i < 4; ++i) buf[(Cfg::RDY + 4 * g + i) * RS + col] = primary ? dyT[i] : zero;
        __syncthreads();
        if (wave < MT) acc3 = dw_tile<T, NCOL>(acc3, buf, Cfg::RH2 + 16 * wave, Cfg::RDY, g, r);
#pragma unroll
        for (int k = 0; k < Cfg::NT2; ++k) {
          const int id = wave + NW * k;
          if (id < MT * MT) acc2[k] = dw_tile<T, NCOL>(acc2[k], buf, Cfg::RH1 + 16 * (id / MT), Cfg::RDZ2 + 16 * (id % MT), g, r);
        }
#pragma unroll
        for (int k = 0; k < Cfg::NT1; ++k) {
          const int id = wave + NW * k;
          if (id < MT1 * MT) acc1[k] = dw_tile<T, NCOL>(acc1[k], buf, 16 * (id / MT), Cfg::RDZ1 + 16 * (id % MT), g, r);
        }
        if (brow < HD) {
          db1 += row_part_sum<T, NCOL>(buf, Cfg::RDZ1 + brow, bq);
          db2 += row_part_sum<T, NCOL>(buf, Cfg::RDZ2 + brow, bq);
        }
        if (brow < 16) db3 += row_part_sum<T, NCOL>(buf, Cfg::RDY + brow, bq);
        __syncthreads();
      } else {
        if constexpr (Cfg::TWO_PHASE) {
          // layers 3 and 2 together: H2 rows [0, HD), dY rows [HD, HD + 16), H1 rows
          // [HD + 16, 2 HD + 16), dZ2 rows [2 HD + 16, 3 HD + 16)
          constexpr int RH1 = HD + 16, RZ2 = 2 * HD + 16;
#pragma unroll
          for (int t = 0; t < SH; ++t) {
            const int h = hid_feature(g, t);
            buf[h * RS + col] = primary ? h2[t] : zero;
            buf[(RH1 + h) * RS + col] = primary ? h1[t] : zero;
            buf[(RZ2 + h) * RS + col] = primary ? dT[t] : zero;
          }
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[(HD + 4 * g + i) * RS + col] = primary ? dyT[i] : zero;
          __syncthreads();
          if (wave < MT) acc3 = dw_tile<T, NCOL>(acc3, buf, 16 * wave, HD, g, r);
#pragma unroll
          for (int k = 0; k < Cfg::NT2; ++k) {
            const int id = wave + NW * k;
            if (id < MT * MT) acc2[k] = dw_tile<T, NCOL>(acc2[k], buf, RH1 + 16 * (id / MT), RZ2 + 16 * (id % MT), g, r);
          }
          if (brow < 16) db3 += row_part_sum<T, NCOL>(buf, HD + brow, bq);
          if (brow < HD) db2 += row_part_sum<T, NCOL>(buf, RZ2 + brow, bq);
          __syncthreads();
        } else {
          // layer 3: H2 rows [0, HD), dY rows [HD, HD + 16)
#pragma unroll
          for (int t = 0; t < SH; ++t) buf[hid_feature(g, t) * RS + col] = primary ? h2[t] : zero;
#pragma unroll
          for (int i = 0; i < 4; ++i) buf[(HD + 4 * g + i) * RS + col] = primary ? dyT[i] : zero;
          __syncthreads();
          if (wave < MT) acc3 = dw_tile<T, NCOL>(acc3, buf, 16 * wave, HD, g, r);
          if (brow < 16) db3 += row_part_sum<T, NCOL>(buf, HD + brow, bq);
          __syncthreads();
          // layer 2: H1 rows [0, HD), dZ2 rows [HD, 2 HD)
#pragma unroll
          for (int t = 0; t < SH; ++t) {
            buf[hid_feature(g, t) * RS + col] = primary ? h1[t] : zero;
            buf[(HD + hid_feature(g, t)) * RS + col] = primary ? dT[t] : zero;
          }
          __syncthreads();
#pragma unroll
          for (int k = 0; k < Cfg::NT2; ++k) {
            const int id = wave + NW * k;
            if (id < MT * MT) acc2[k] = dw_tile<T, NCOL>(acc2[k], buf, 16 * (id / MT), HD + 16 * (id % MT), g, r);
          }
          if (brow < HD) db2 += row_part_sum<T, NCOL>(buf, HD + brow, bq);
          __syncthreads();
        }
        if constexpr (!Cfg::SPLIT1) {
          // layer 1: X slot rows 4t+g in [0, RX), dZ1 rows [RX, RX + HD)
#pragma unroll
          for (int t = 0; t < 4 * MT1; ++t) buf[(4 * t + g) * RS + col] = (t < S1 && primary) ? xs[t] : zero;
#pragma unroll
          for (int t = 0; t < SH; ++t) buf[(RX + hid_feature(g, t)) * RS + col] = primary ? dz1T[t] : zero;
          __syncthreads();
#pragma unroll
          for (int k = 0; k < Cfg::NT1; ++k) {
            const int id = wave + NW * k;
            if (id < MT1 * MT) acc1[k] = dw_tile<T, NCOL>(acc1[k], buf, 16 * (id / MT), RX + 16 * (id % MT), g, r);
          }
          if (brow < HD) db1 += row_part_sum<T, NCOL>(buf, RX + brow, bq);
          __syncthreads();
        } else {
          // layer 1 in two halves: X slot rows of row blocks [MB h, MB h + MB) at local rows
          // [0, 16 MB), dZ1 rows [16 MB, 16 MB + HD) (written once, kept for both halves)
          constexpr int MB = Cfg::MB, RZ = 16 * MB;
#pragma unroll
          for (int h = 0; h < 2; ++h) {
#pragma unroll
            for (int t = 4 * MB * h; t < 4 * MB * (h + 1) && t < 4 * MT1; ++t)
              buf[(4 * (t - 4 * MB * h) + g) * RS + col] = (t < S1 && primary) ? xs[t] : zero;
            if (h == 0) {
#pragma unroll
              for (int t = 0; t < SH; ++t) buf[(RZ + hid_feature(g, t)) * RS + col] = primary ? dz1T[t] : zero;
            }
            __syncthreads();
#pragma unroll
            for (int k = 0; k < Cfg::NT1; ++k) {
              const int id = wave + NW * k, rb = id / MT;
              if (id < MT1 * MT && rb / MB == h)  // wave-uniform
                acc1[k] = dw_tile<T, NCOL>(acc1[k], buf, 16 * (rb - MB * h), RZ + 16 * (id % MT), g, r);
            }
            if (h == 0 && brow < HD) db1 += row_part_sum<T, NCOL>(buf, RZ + brow, bq);
            __syncthreads();
          }
        }
      }
    }

    if (binned && !refine) {
      const bool again = lost_flag[par] != 0;  // read after the last staging barrier
      // the next item's flag: its last reads were before this item's barriers, its next
      // writes come after this item's write-out barrier
      if (tid == 0) lost_flag[par ^ 1] = 0;
      if (again) {  // block-uniform
        lost = false;
        continue;
      }
    }
    // the refine pass has no staging barriers: its adds must land before the write-out
    if (refine) __syncthreads();
    break;
    }

    // ---------------- the tile's latent gradient: dense plain stores (or a partial)
    if (binned) {
      const int w0 = m.W >> (m.shift + 2 * j), w1 = w0 >> 1;
      float* dst = single ? a.lat_grad : a.part_lat + (long long)item * a.region_max;
      const float osc = single ? out_scale : 1.f;
      // latent k of the region as a float (fixed-point sums, or the FP32 sums of a
      // summed-again item)
      auto reg_value = [&](int k) -> float {
        if constexpr (WIDE) return refined ? freg[k] : (float)((double)ireg[k] * (double)fixinv);
        else return refined ? freg[k] : (float)ireg[k] * fixinv;
      };
      // rows of L region latents (a row of cells of the tile, all channels) go to
      // consecutive latents: row y of the block at region offset k0 + y L lands at
      // gbase + y gstride; 16-byte loads and stores where the rows and offsets allow
      auto copy_rows = [&](int k0, int L, int rows, long long gbase, long long gstride) {
        if (L % 4 == 0 && ((gbase | gstride) & 3) == 0) {
          const int q4 = L >> 2, n4 = rows * q4;
          for (int i = tid; i < n4; i += NTHR) {
            const int y = i / q4, o = (i - y * q4) * 4, k = k0 + y * L + o;  // k: a multiple of 4
            f32x4 val;
            if (refined) {
              val = *reinterpret_cast<const f32x4*>(freg + k);
              *reinterpret_cast<int4*>(freg + k) = int4{0, 0, 0, 0};
            } else if constexpr (WIDE) {
              const longlong2 lo = *reinterpret_cast<const longlong2*>(ireg + k);
              const longlong2 hi = *reinterpret_cast<const longlong2*>(ireg + k + 2);
              *reinterpret_cast<longlong2*>(ireg + k) = longlong2{0, 0};
              *reinterpret_cast<longlong2*>(ireg + k + 2) = longlong2{0, 0};
              const double fi = (double)fixinv;
              val = f32x4{(float)((double)lo.x * fi), (float)((double)lo.y * fi), (float)((double)hi.x * fi),
                          (float)((double)hi.y * fi)};
            } else {
              const int4 iv = *reinterpret_cast<const int4*>(ireg + k);
              *reinterpret_cast<int4*>(ireg + k) = int4{0, 0, 0, 0};
              val = f32x4{(float)iv.x * fixinv, (float)iv.y * fixinv, (float)iv.z * fixinv, (float)iv.w * fixinv};
            }
            *reinterpret_cast<f32x4*>(dst + gbase + y * gstride + o) = val * osc;
          }
        } else {
          for (int i = tid; i < rows * L; i += NTHR) {
            const int y = i / L, o = i - y * L, k = k0 + y * L + o;
            dst[gbase + y * gstride + o] = reg_value(k) * osc;
            if (refined) freg[k] = 0.f;  // the bytes this thread read
            else ireg[k] = (AccI)0;
          }
        }
      };
      if (single) {
        copy_rows(0, T_ * C0, T_, tab[j] + ((long long)ty * T_ * w0 + (long long)tx * T_) * C0, (long long)w0 * C0);
        copy_rows(R0, T1 * C1, T1, tab[8 + j] + ((long long)ty * T1 * w1 + (long long)tx * T1) * C1,
                  (long long)w1 * C1);
      } else {
        copy_rows(0, RG, 1, 0, 0);  // the region as it is
      }
      __syncthreads();
    }
  }

  // ---------------- per-block partial weight gradient (canonical layout) and loss
  float* part = a.part_dw + (long long)row * Pn;
  if (wave < MT) {
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int h = 16 * wave + 4 * g + i;
      if (r < C) part[W3o + (long long)h * C + r] = acc3[i];
    }
  }
#pragma unroll
  for (int k = 0; k < Cfg::NT2; ++k) {
    const int id = wave + NW * k;
    if (id < MT * MT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int h1 = 16 * (id / MT) + 4 * g + i, h2 = 16 * (id % MT) + r;
        part[W2o + (long long)h1 * HD + h2] = acc2[k][i];
      }
    }
  }
#pragma unroll
  for (int k = 0; k < Cfg::NT1; ++k) {
    const int id = wave + NW * k;
    if (id < MT1 * MT) {
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int t = 4 * (id / MT) + g;  // slot row 4t + gi with gi = i
        int kin = t < S1 ? IS::psi(i, t) : -1;
        if (kin == IS::K_LOD && !m.lod_in) kin = -1;  // the LOD slot holds zeros without that input
        const int h = 16 * (id % MT) + r;
        if (kin >= 0) part[(long long)kin * HD + h] = acc1[k][i];
      }
    }
  }
  // bias gradients: the PARTS part sums of each row are in consecutive lanes
  constexpr int PARTS = NCOL / 16;
#pragma unroll
  for (int o = 1; o < PARTS; o <<= 1) {
    db1 += __shfl_xor(db1, o);
    db2 += __shfl_xor(db2, o);
    db3 += __shfl_xor(db3, o);
  }
  if (tid % PARTS == 0) {
    const int row = tid / PARTS;
    if (row < HD) {
      part[b1o + row] = db1;
      part[b2o + row] = db2;
    }
    if (row < C) part[b3o + row] = db3;
  }
  for (int off = 32; off > 0; off >>= 1) loss += __shfl_xor(loss, off);
  if (lane == 0) red[wave] = loss;
  __syncthreads();
  if (tid == 0) {
    float l = 0.f;
    for (int w = 0; w < NW; ++w) l += red[w];
    a.part_loss[row] = l;
  }
}

template <typename T, int C0, int C1, int C, int HD, int ACT>
__global__ __launch_bounds__((TrainCfg<T, C0, C1, C, HD>::NTHR),
                             (TrainCfg<T, C0, C1, C, HD>::NW * TrainCfg<T, C0, C1, C, HD>::BPC / 4)) void
train_fused_kernel(DevMat m, PeTable pe, TrainArgs a) {
  if (a.table_hash && *a.table_hash != a.hash) return;  // grouped step against another table
  fused_body<T, C0, C1, C, HD, ACT>(m, pe, a, a.q, a.binned, a.scale_slot, a.step_dev, blockIdx.x, -1, gridDim.x,
                                    blockIdx.x, blockIdx.x == 0);
}

// ------------------------------------------------------------------ binning (counting sort)
struct BinArgs {
  const ntc_query* q;
  long long n;
  int per_block;
  int nbb;
  int* counts;         // [nbins][nbb]
  const int* offsets;  // [nbins][nbb], relative to the bin base
  const int* base;     // [nbins + 1]
  const int* total;    // scatter: the bin totals, scanned by every block (or nullptr: base)
  int4* list;
};

// Exclusive scan over the 1024 threads of a block (wavefront scans by shuffles, then
// the 16 wavefront totals); `total` receives the sum.  sh: 33 ints of LDS.
__device__ inline int block_exclusive_scan(int v, int* sh, int& total) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  int incl = v;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  if (lane == 63) sh[w] = incl;
  __syncthreads();
  if (w == 0) {
    const int t = lane < 16 ? sh[lane] : 0;
    int ti = t;
#pragma unroll
    for (int d = 1; d < 16; d <<= 1) {
      const int o = __shfl_up(ti, d, 64);
      if (lane >= d) ti += o;
    }
    if (lane < 16) sh[16 + lane] = ti - t;
    if (lane == 15) sh[32] = ti;
  }
  __syncthreads();
  const int r = sh[16 + w] + incl - v;
  total = sh[32];
  __syncthreads();  // sh is reused by the next scan
  return r;
}

// Exclusive scan of the bin totals by a block of 1024 threads: s_base[b] (and base[b] when
// base is given) = the list position of bin b's first entry, s_base[nb] = the list length.
__device__ __forceinline__ void bin_base_scan(int nb, const int* __restrict__ total, int* __restrict__ base,
                                              int* s_base, int* s_scan) {
  const int tid = threadIdx.x;
  const int per = (nb + 1023) / 1024;
  const int b0 = min(nb, tid * per), b1 = min(nb, b0 + per);
  int st = 0;
  for (int b = b0; b < b1; ++b) st += total[b];
  int all;
  int pt = block_exclusive_scan(st, s_scan, all);
  for (int b = b0; b < b1; ++b) {  // the totals again (cached): no register array per thread
    s_base[b] = pt;
    if (base) base[b] = pt;
    pt += total[b];
  }
  if (tid == 0) {
    s_base[nb] = all;
    if (base) base[nb] = all;
  }
}

// Bins of one sample: the sort bins of the tiles its footprint touches (at most 4,
// all different), -1 in the unused entries.
__device__ inline void sample_bin_list(const DevMat& m, const TileGeom& tg, const ntc_query& qq, int (&bk)[4]) {
  const Footprint f = locate(m, qq.u, qq.v, qq.lod, 0);
  const SampleBins sb = sample_bins(f, tg);
  const bool two_x = sb.tx1 > sb.tx0, two_y = sb.ty1 > sb.ty0;  // each range spans at most two tiles
  bk[0] = sort_bin(tg, sb.j, sb.tx0, sb.ty0, f.ax, f.ay);
  bk[1] = two_x ? sort_bin(tg, sb.j, sb.tx1, sb.ty0, f.ax, f.ay) : -1;
  bk[2] = two_y ? sort_bin(tg, sb.j, sb.tx0, sb.ty1, f.ax, f.ay) : -1;
  bk[3] = two_x && two_y ? sort_bin(tg, sb.j, sb.tx1, sb.ty1, f.ax, f.ay) : -1;
}

// bi: the binning block (of a.nbb) this block is; q: the material's queries.
// Counting pass (!SCATTER): per-block bin histograms.  Scatter pass: list positions in a
// fixed order, so a bin lists its samples by increasing sample index whatever the
// timing of the run (a stable sort of each round's entries by bin, below).
template <bool SCATTER>
__device__ __forceinline__ void bin_body(const DevMat& m, const TileGeom& tg, const BinArgs& a,
                                         const ntc_query* __restrict__ q, int bi) {
  extern __shared__ int hist[];  // nbins + 1 ints
  const int nb = tg.nbins;
  if constexpr (SCATTER) {
    // running list position of each bin in this block: the bin's base plus the entries of
    // earlier blocks; hist[nb] = the list length
    if (a.total) {  // block-uniform: the bases from the totals, in this block
      __shared__ int s_scan[1024];
      bin_base_scan(nb, a.total, nullptr, hist, s_scan);
      __syncthreads();
      for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] += a.offsets[(long long)b * a.nbb + bi];
    } else {
      for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = a.base[b] + a.offsets[(long long)b * a.nbb + bi];
      if (threadIdx.x == 0) hist[nb] = a.base[nb];
    }
  } else {
    for (int b = threadIdx.x; b < nb; b += blockDim.x) hist[b] = 0;
  }
  __syncthreads();
  const long long s0 = (long long)bi * a.per_block;
  const long long s1 = min(a.n, s0 + a.per_block);
  if constexpr (!SCATTER) {
    constexpr int U = 4;  // queries loaded together per thread and round
    for (long long s = s0 + threadIdx.x; s < s1; s += U * blockDim.x) {
      ntc_query qq[U];
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const long long sk = s + (long long)k * blockDim.x;
        if (sk < s1) qq[k] = q[sk];
      }
#pragma unroll
      for (int k = 0; k < U; ++k) {
        const long long sk = s + (long long)k * blockDim.x;
        if (sk >= s1) break;
        int bk[4];
        sample_bin_list(m, tg, qq[k], bk);
#pragma unroll
        for (int e = 0; e < 4; ++e)
          if (bk[e] >= 0) atomicAdd(&hist[bk[e]], 1);
      }
    }
    __syncthreads();
    for (int b = threadIdx.x; b < nb; b += blockDim.x) a.counts[(long long)b * a.nbb + bi] = hist[b];
  } else {
    // Scatter, one round of 1024 samples at a time.  The round's entries (bin, 4 t + e)
    // for thread t's e-th bin are sorted by bin with a stable LSD radix sort in LDS (the
    // ids start in sample order and a sample has at most one entry per bin), so each bin's
    // run lists its samples in increasing order; an entry's list position is the bin's
    // running position in this block (hist) plus its rank in the run.
    static_assert(kBinThreads == 1024, "the scatter sorts 4 entries of each of 1024 threads");
    constexpr int kE = 4 * kBinThreads;
    // 4-bit digits: as many passes as the bin indices need; the largest key of that many
    // digits marks unused entries (sorted last)
    const int passes = nb < 16 ? 1 : nb < 256 ? 2 : nb < 4096 ? 3 : 4;
    const int kInvalid = (1 << (4 * passes)) - 1;
    __shared__ __align__(16) int sbuf[2][kE];
    __shared__ float qu[kBinThreads], qv[kBinThreads];
    __shared__ int ql[kBinThreads];
    __shared__ uint32_t wsum[16][8], wpre[16][8], wtot[8];
    __shared__ int wmax[16];
    const int t = threadIdx.x, lane = t & 63, wave = t >> 6;
    const int list_len = hist[nb];
    for (long long r0 = s0; r0 < s1; r0 += kBinThreads) {
      const long long sk = r0 + t;
      int v[4];
      {
        int bk[4] = {-1, -1, -1, -1};
        if (sk < s1) {
          const ntc_query qq = q[sk];
          qu[t] = qq.u;
          qv[t] = qq.v;
          ql[t] = qq.lod;
          sample_bin_list(m, tg, qq, bk);
        }
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = ((bk[e] >= 0 ? bk[e] : kInvalid) << 12) | (4 * t + e);
      }
      // stable counting passes over the 4-bit digits of the bin
      for (int pass = 0; pass < passes; ++pass) {
        const int sh = 12 + 4 * pass;
        int d[4], lr[4];
        unsigned long long cl = 0;  // this thread's digit counts, 4 bits each
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          d[e] = (v[e] >> sh) & 15;
          lr[e] = (int)((cl >> (4 * d[e])) & 15ull);
          cl += 1ull << (4 * d[e]);
        }
        // counts of digits 2i (low half) and 2i + 1 (high half) in register i; 16-bit
        // fields hold block sums (at most 4096) without carries
        uint32_t c[8], inc[8];
#pragma unroll
        for (int i = 0; i < 8; ++i) {
          c[i] = (uint32_t)((cl >> (8 * i)) & 15ull) | ((uint32_t)((cl >> (8 * i + 4)) & 15ull) << 16);
          inc[i] = wave_incl_sum(c[i]);
        }
        if (lane == 63)
#pragma unroll
          for (int i = 0; i < 8; ++i) wsum[wave][i] = inc[i];
        __syncthreads();
        if (t < 8) {  // prefix over the wavefronts, register t
          uint32_t run = 0;
          for (int w = 0; w < 16; ++w) {
            wpre[w][t] = run;
            run += wsum[w][t];
          }
          wtot[t] = run;
        }
        __syncthreads();
        // comb[i]: first position of digits 2i, 2i + 1 (all smaller digits of the block)
        // plus the entries of those digits in earlier threads
        uint32_t comb[8];
        {
          uint32_t run = 0;
#pragma unroll
          for (int i = 0; i < 8; ++i) {
            const uint32_t tot = wtot[i], lo = tot & 0xFFFFu;
            comb[i] = (run | ((run + lo) << 16)) + wpre[wave][i] + inc[i] - c[i];
            run += lo + (tot >> 16);
          }
        }
        int* out = sbuf[pass & 1];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int i = d[e] >> 1;
          const uint32_t a01 = (i & 1) ? comb[1] : comb[0], a23 = (i & 1) ? comb[3] : comb[2];
          const uint32_t a45 = (i & 1) ? comb[5] : comb[4], a67 = (i & 1) ? comb[7] : comb[6];
          const uint32_t a03 = (i & 2) ? a23 : a01, a47 = (i & 2) ? a67 : a45;
          const uint32_t f = (i & 4) ? a47 : a03;
          out[((d[e] & 1) ? (int)(f >> 16) : (int)(f & 0xFFFFu)) + lr[e]] = v[e];
        }
        __syncthreads();
        const int4 r = reinterpret_cast<const int4*>(out)[t];
        v[0] = r.x;
        v[1] = r.y;
        v[2] = r.z;
        v[3] = r.w;
      }
      // sorted: position p = 4 t + e.  Runs of equal bins: a run starts where the bin
      // changes; its start is the running maximum of the start positions.
      const int* srt = sbuf[(passes - 1) & 1];
      const int prev = t > 0 ? srt[4 * t - 1] >> 12 : -1;
      const int next = t < kBinThreads - 1 ? srt[4 * t + 4] >> 12 : -1;
      int key[4], st[4];
      int run = 0;
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        key[e] = v[e] >> 12;
        const int before = e == 0 ? prev : key[e - 1];
        if (key[e] != before) run = 4 * t + e;
        st[e] = run;
      }
      // the start of the run open at the end of the previous thread: the largest run start
      // at or before it (threads without a run start of their own hold 0)
      const int incm = wave_incl_max(run);
      if (lane == 63) wmax[wave] = incm;
      __syncthreads();
      int carry = 0;
      for (int w = 0; w < wave; ++w) carry = max(carry, wmax[w]);
      {
        const int x = __shfl_up(incm, 1, 64);
        if (lane >= 1) carry = max(carry, x);
      }
      int lpos[4];
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int start = max(st[e], carry);  // st[e] >= carry once this thread starts a run
        lpos[e] = key[e] != kInvalid ? hist[key[e]] + (4 * t + e - start) : -1;
      }
      __syncthreads();  // every position read hist before the runs advance it
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int after = e == 3 ? next : key[e + 1];
        if (key[e] != kInvalid && key[e] != after) {
          const int start = max(st[e], carry);
          hist[key[e]] += 4 * t + e - start + 1;  // the run's last entry advances its bin
        }
        if (lpos[e] >= 0 && lpos[e] < list_len) {
          const int id = (v[e] & 4095) >> 2;
          a.list[lpos[e]] = make_int4(__float_as_int(qu[id]), __float_as_int(qv[id]), ql[id], (int)(r0 + id));
        }
      }
      __syncthreads();  // hist, the sort buffers and the queries are reused by the next round
    }
  }
}

template <bool SCATTER>
__global__ __launch_bounds__(kBinThreads) void bin_kernel(DevMat m, TileGeom tg, BinArgs a) {
  bin_body<SCATTER>(m, tg, a, a.q, blockIdx.x);
}

// Per-bin column scan over the binning blocks: one wavefront per bin, each lane
// holds 4 consecutive blocks (nbb <= 256).  Writes the per-block offsets and the
// bin total.
__device__ __forceinline__ void bin_scan1_body(int nbins, int nbb, const int* __restrict__ counts,
                                               int* __restrict__ offsets, int* __restrict__ total, int bi) {
  const int lane = threadIdx.x & 63;
  const int b = bi * 4 + (threadIdx.x >> 6);
  if (b >= nbins) return;
  int v[4];
  int sum = 0;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = lane * 4 + e;
    v[e] = k < nbb ? counts[(long long)b * nbb + k] : 0;
    sum += v[e];
  }
  int incl = sum;
#pragma unroll
  for (int d = 1; d < 64; d <<= 1) {
    const int o = __shfl_up(incl, d, 64);
    if (lane >= d) incl += o;
  }
  int run = incl - sum;
#pragma unroll
  for (int e = 0; e < 4; ++e) {
    const int k = lane * 4 + e;
    if (k < nbb) offsets[(long long)b * nbb + k] = run;
    run += v[e];
  }
  if (lane == 63) total[b] = incl;
}

__global__ __launch_bounds__(256) void bin_scan1_kernel(int nbins, int nbb, const int* __restrict__ counts,
                                                        int* __restrict__ offsets, int* __restrict__ total) {
  bin_scan1_body(nbins, nbb, counts, offsets, total, blockIdx.x);
}

// One block of 1024 threads: exclusive scan over the sort bins of their totals (list
// positions), then per tile its start, total and work items (at most tg.chunk samples
// per item, at least one), the exclusive scan of the items over the tiles, and the tile
// of every item.
__device__ __forceinline__ void bin_scan2_body(const TileGeom& tg, const int* __restrict__ total,
                                               int* __restrict__ base, int* __restrict__ tile_start,
                                               int* __restrict__ tile_total, int* __restrict__ item_base,
                                               int* __restrict__ item_tile, int* __restrict__ nitems, int* s_base,
                                               int* s_scan) {
  const int tid = threadIdx.x;
  const int nb = tg.nbins, nt = tg.ntiles;
  bin_base_scan(nb, total, base, s_base, s_scan);
  __syncthreads();
  {
    const int per = (nt + 1023) / 1024;
    const int t0 = min(nt, tid * per), t1 = min(nt, t0 + per);
    auto tile_items = [&](int tot) { return max(1, (tot + tg.chunk - 1) / tg.chunk); };
    int items = 0;
    for (int t = t0; t < t1; ++t) {
      int j = 0;
      while (j + 1 < kMaxLevels && t >= tg.tile_base[j + 1]) ++j;
      const int first = tg.bin_base[j] + (t - tg.tile_base[j]) * tg.sb[j] * tg.sb[j];
      const int st = s_base[first];
      const int tot = s_base[first + tg.sb[j] * tg.sb[j]] - st;
      tile_start[t] = st;
      tile_total[t] = tot;
      items += tile_items(tot);
    }
    int all;
    int pi = block_exclusive_scan(items, s_scan, all);  // every s_base read above precedes its barriers
    for (int t = t0; t < t1; ++t) {  // this thread's own totals, read back: no register array
      item_base[t] = pi;
      s_base[t] = pi;  // first item of each tile, for the item -> tile search
      pi += tile_items(tile_total[t]);
    }
    if (tid == 0) {
      item_base[nt] = all;
      *nitems = all;
    }
    __syncthreads();
    // tile of every item: the last tile whose first item is at or before it
    for (int i = tid; i < all; i += 1024) {
      int lo = 0, hi = nt - 1;
      while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (s_base[mid] <= i) lo = mid;
        else hi = mid - 1;
      }
      item_tile[i] = lo;
    }
  }
}

// The scatter pass with the tile tables beside it: blocks 0 .. nbb-1 scatter (each scans
// the bin totals itself), block nbb writes the per-tile starts, totals and work items
// (the one-block scan), so neither waits for the other.
struct TileTables {
  int* base;
  int* tile_start;
  int* tile_total;
  int* item_base;
  int* item_tile;
  int* nitems;
};
__global__ __launch_bounds__(kBinThreads, 8) void bin_scatter_kernel(DevMat m, TileGeom tg, BinArgs a, TileTables o) {
  if ((int)blockIdx.x == a.nbb) {
    extern __shared__ int s_base[];  // nbins + 1 ints
    __shared__ int s_scan[1024];
    bin_scan2_body(tg, a.total, o.base, o.tile_start, o.tile_total, o.item_base, o.item_tile, o.nitems, s_base,
                   s_scan);
    return;
  }
  bin_body<true>(m, tg, a, a.q, blockIdx.x);
}

// Latent gradients of tiles split over several work items: partials summed in a fixed order.
// tile: the latent tile; bx, gx: this block's share of the tile's region (of gx).
__device__ __forceinline__ void lat_partial_body(const DevMat& m, const TileGeom& tg, const int* __restrict__ item_base,
                                                 const float* __restrict__ part, int region_max,
                                                 float* __restrict__ lat_grad, float out_scale, int tile, int bx,
                                                 int gx) {
  const int it0 = item_base[tile], items = item_base[tile + 1] - it0;
  if (items <= 1) return;
  int j = 0;
  while (j + 1 < m.J && tile >= tg.tile_base[j + 1]) ++j;
  const int t = tile - tg.tile_base[j], tx = t % tg.ntx[j], ty = t / tg.ntx[j];
  const int T = tg.T[j], T1 = T >> 1;
  const int C0 = m.C0, C1 = m.C1;
  const int R0 = T * T * C0, RG = R0 + T1 * T1 * C1;
  const int w0 = m.W >> (m.shift + 2 * j), w1 = w0 >> 1;
  auto store = [&](int k, float s) {
    long long gi;
    if (k < R0) {
      const int c = k % C0, cell = k / C0, cx = cell % T, cy = cell / T;
      gi = m.g0_off[j] + ((long long)(ty * T + cy) * w0 + tx * T + cx) * C0 + c;
    } else {
      const int k1 = k - R0, c = k1 % C1, cell = k1 / C1, cx = cell % T1, cy = cell / T1;
      gi = m.g1_off[j] + ((long long)(ty * T1 + cy) * w1 + tx * T1 + cx) * C1 + c;
    }
    lat_grad[gi] = s * out_scale;
  };
  // Item i of an element goes to running sum i & 3, in increasing i (a fixed order,
  // whatever the grid); absent items and elements read as zero.  Sixteen loads in flight
  // per round: sixteen items of one element when the grid has a thread per element,
  // else four items of four elements (tiles of two or three items are the common case).
  const int step = gx * blockDim.x;
  const float* src = part + (long long)it0 * region_max;
  if (RG <= step) {
    const int k = bx * blockDim.x + threadIdx.x;
    if (k >= RG) return;
    float acc[4] = {0.f, 0.f, 0.f, 0.f};
    for (int i = 0; i < items; i += 16) {
      float v[16];
#pragma unroll
      for (int e = 0; e < 16; ++e) v[e] = i + e < items ? src[(long long)(i + e) * region_max + k] : 0.f;
#pragma unroll
      for (int e = 0; e < 16; ++e) acc[e & 3] += v[e];
    }
    store(k, (acc[0] + acc[1]) + (acc[2] + acc[3]));
    return;
  }
  for (int k0 = bx * blockDim.x + threadIdx.x; k0 < RG; k0 += 4 * step) {
    float acc[4][4] = {};
    for (int i = 0; i < items; i += 4) {
      float v[4][4];
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) {
          const int k = k0 + q * step;
          v[q][e] = (k < RG && i + e < items) ? src[(long long)(i + e) * region_max + k] : 0.f;
        }
#pragma unroll
      for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < 4; ++e) acc[q][e] += v[q][e];
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q * step < RG) store(k0 + q * step, (acc[q][0] + acc[q][1]) + (acc[q][2] + acc[q][3]));
  }
}

// Block (bx, y) of a gx x G grid takes region share bx of the split tiles among y, y + G,
// y + 2G, ...: each lane reads one candidate's item count, a ballot lists the split ones,
// and the block walks that list, so blocks are not launched per tile (most tiles are
// single items).
__device__ __forceinline__ void lat_partial_tiles(const DevMat& m, const TileGeom& tg,
                                                  const int* __restrict__ item_base, const float* __restrict__ part,
                                                  int region_max, float* __restrict__ lat_grad, float osc, int bx,
                                                  int gx, int y, int G) {
  const int lane = threadIdx.x & 63;
  for (int b0 = y; b0 < tg.ntiles; b0 += 64 * G) {
    const int t = b0 + lane * G;
    const bool split = t < tg.ntiles && item_base[t + 1] - item_base[t] > 1;
    unsigned long long mask = __ballot(split);  // the same in every wavefront
    while (mask) {
      const int i = __builtin_ctzll(mask);
      mask &= mask - 1;
      lat_partial_body(m, tg, item_base, part, region_max, lat_grad, osc, b0 + i * G, bx, gx);
    }
  }
}

// Region shares of a split-tile reduction (at least one, at most 64) and tile strides.
__host__ __device__ inline int lat_partial_gx(int region_max) {
  const int g = (region_max + 255) / 256;
  return g < 1 ? 1 : (g > 64 ? 64 : g);
}
__host__ __device__ inline int lat_partial_ty(int ntiles) { return ntiles < 64 ? (ntiles < 1 ? 1 : ntiles) : 64; }

// dscale: device (dout scale, output scale) overriding out_scale, or nullptr
__global__ __launch_bounds__(256) void lat_partial_reduce(DevMat m, TileGeom tg, const int* __restrict__ item_base,
                                   const float* __restrict__ part, int region_max, float* __restrict__ lat_grad,
                                   float out_scale, const float* __restrict__ dscale) {
  lat_partial_tiles(m, tg, item_base, part, region_max, lat_grad, dscale ? dscale[1] : out_scale, blockIdx.x,
                    gridDim.x, blockIdx.y, gridDim.y);
}

// ------------------------------------------------------------------ weight-gradient reduction
// The fused kernel's G per-block partial rows summed in a fixed order: block bx takes
// parameters [64 bx, 64 bx + 64), each of its kDwWaves wavefronts a contiguous share of
// the rows, and the shares are added in order; non-finite sums raise the flag.  Block 0
// also sums the per-block losses.
constexpr int kDwWaves = 16;
__device__ __forceinline__ void dw_reduce_body(int G, long long P, const float* __restrict__ part,
                                               float* __restrict__ grad, const float* __restrict__ part_loss,
                                               float* __restrict__ loss_out, float norm, int32_t* flag,
                                               float out_scale, int bx) {
  __shared__ float red[kDwWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const long long p = (long long)bx * 64 + lane;
  const int per = (G + kDwWaves - 1) / kDwWaves, b0 = w * per, b1 = min(G, b0 + per);
  float s = 0.f;
  if (p < P) {
#pragma unroll 8
    for (int b = b0; b < b1; ++b) s += part[(long long)b * P + p];
  }
  red[w][lane] = s;
  __syncthreads();
  if (w == 0 && p < P) {
    float t = 0.f;
#pragma unroll
    for (int k = 0; k < kDwWaves; ++k) t += red[k][lane];
    grad[p] = t * out_scale;
    if (flag && !isfinite(t)) atomicOr(flag, 1);
  }
  if (bx == 0 && loss_out) {
    __syncthreads();
    float* lr = &red[0][0];
    float l = 0.f;
    for (int b = threadIdx.x; b < G; b += blockDim.x) l += part_loss[b];
    lr[threadIdx.x] = l;
    __syncthreads();
    for (int k = kDwWaves * 32; k > 0; k >>= 1) {
      if ((int)threadIdx.x < k) lr[threadIdx.x] += lr[threadIdx.x + k];
      __syncthreads();
    }
    if (threadIdx.x == 0) *loss_out = lr[0] * norm;
  }
}

__global__ __launch_bounds__(64 * kDwWaves) void dw_reduce(int G, long long P, const float* __restrict__ part,
                                                 float* __restrict__ grad, const float* __restrict__ part_loss,
                                                 float* __restrict__ loss_out, float norm, int32_t* flag,
                                                 float out_scale, const float* __restrict__ dscale) {
  dw_reduce_body(G, P, part, grad, part_loss, loss_out, norm, flag, dscale ? dscale[1] : out_scale, blockIdx.x);
}

// ------------------------------------------------------------------ output-gradient scale
// The differentiation path multiplies the caller's dL/dy by a power of two that brings
// max |dL/dy| near 1/4 (FP16 range) and divides the gradients by it again.  Picked on the
// device, so the backward needs no host synchronisation: per-block maxima, then one
// block reduces them and writes (scale, 1 / scale).  Zero or non-finite maxima give 1.
constexpr int kScaleBlocks = 1024;
__global__ __launch_bounds__(256) void dout_amax_kernel(const float* __restrict__ d, long long count,
                                                       float* __restrict__ part) {
  __shared__ float red[4];
  float v = 0.f;
  for (long long i = blockIdx.x * 256ll + threadIdx.x; i < count; i += (long long)gridDim.x * 256)
    v = fmaxf(v, fabsf(d[i]));  // fmaxf drops NaN: a NaN-only input yields 0 (scale 1)
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
}

__global__ __launch_bounds__(256) void dout_scale_kernel(const float* __restrict__ part, int blocks,
                                                        float* __restrict__ scale) {
  __shared__ float red[4];
  float v = 0.f;
  for (int i = threadIdx.x; i < blocks; i += 256) v = fmaxf(v, part[i]);
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    const float amax = fmaxf(fmaxf(red[0], red[1]), fmaxf(red[2], red[3]));
    float sc = 1.f;
    if (amax > 0.f && amax <= 3.0e38f) {
      // 2^round(log2(0.25 / amax)) = 2^round(-2 - a - log2 g) with amax = g 2^a, g in
      // [1/2, 1): -log2 g lies in (0, 1] and rounds to 1 exactly when g < 1/sqrt(2)
      int a = 0;
      const float g = frexpf(amax, &a);
      const int k = -2 - a + (g < 0.70710678f ? 1 : 0);
      sc = ldexpf(1.f, max(-120, min(120, k)));
    }
    scale[0] = sc;
    scale[1] = 1.f / sc;
  }
}

hipError_t launch_dout_scale(const float* dout, long long count, float* work, hipStream_t s) {
  const long long want = (count + 255) / 256;
  const int blocks = (int)std::max<long long>(1, std::min<long long>(kScaleBlocks, want));
  hipLaunchKernelGGL(dout_amax_kernel, dim3(blocks), dim3(256), 0, s, dout, count, work + 2);
  hipLaunchKernelGGL(dout_scale_kernel, dim3(1), dim3(256), 0, s, work + 2, blocks, work);
  return hipGetLastError();
}

// ------------------------------------------------------------------ optimiser
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

// The same lookup with the grid starts held in registers (read once per thread): a
// loop over latents need not reload the descriptor, which may live in global memory.
struct LatentBits {
  long long g1[kMaxLevels], g0[kMaxLevels];
  int b0, b1, J;
  __device__ explicit LatentBits(const DevMat& m) : b0(m.B0), b1(m.B1), J(m.J) {
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) {
      g0[j] = m.g0_off[j];
      g1[j] = m.g1_off[j];
    }
  }
  __device__ int operator()(long long i) const {
    if (b0 == b1) return b0;
    int bits = b0;
#pragma unroll
    for (int j = 0; j < kMaxLevels; ++j) {
      if (j < J && i >= g0[j]) bits = b0;
      if (j < J && i >= g1[j]) bits = b1;
    }
    return bits;
  }
};

struct AdamArgs {
  AdamLaunch a;
  PackGeom pg;
  long long P;
  int mlp_blocks;
};

// bx, gx: this block among the gx blocks of the material's update (the first
// args.mlp_blocks take the network parameters, the rest stride over the latents).
template <typename T>
__device__ __forceinline__ void adam_body(const DevMat& m, const AdamArgs& args, int bx, int gx) {
  const AdamLaunch& a = args.a;
  const int ovf = a.scale_state[1];
  // step-dependent values: from the host, or derived from the device step index
  int step = a.step;
  float bc1 = a.bc1, bc2 = a.bc2, lr_lat = a.lr_lat, lr_mlp = a.lr_mlp;
  uint64_t next_key = a.next_key;
  if (a.step_dev) {
    step = *a.step_dev;
    const double t = (double)step + 1.0;
    bc1 = (float)(1.0 - exp(t * log((double)a.beta1)));
    bc2 = (float)(1.0 - exp(t * log((double)a.beta2)));
    next_key = noise_key(a.seed, step + 1);
  }
  if (a.lr_dev) {
    lr_lat = a.lr_dev[0];
    lr_mlp = a.lr_dev[1];
  }
  const float scale = a.loss_scale ? a.loss_scale[step & 1] : 1.f;
  const float inv_s = 1.f / scale;
  const float b1 = a.beta1, b2 = a.beta2, eps = a.eps;
  const float ib1 = 1.f / bc1, ib2 = 1.f / bc2;
  if (bx < args.mlp_blocks) {
    const long long p = bx * 256ll + threadIdx.x;
    if (p < args.P && !ovf) {
      const float gr = a.mlp_grad[p] * inv_s;
      const float mm = b1 * a.mlp_m[p] + (1.f - b1) * gr;
      const float vv = b2 * a.mlp_v[p] + (1.f - b2) * gr * gr;
      const float w = a.mlp[p] - lr_mlp * (mm * ib1) / (sqrtf(vv * ib2) + eps);
      a.mlp_m[p] = mm;
      a.mlp_v[p] = vv;
      a.mlp[p] = w;
      scatter_param<T>((T*)a.wpack, args.pg, m.C0, m.C1, m.C, m.Hd, p, w, true, 0, 0, false, m.lod_in);
    }
    if (bx == 0 && threadIdx.x == 0 && a.loss_scale) {
      float sn = scale;
      int good = a.scale_state[0];
      if (ovf) {
        sn = scale * 0.5f;
        good = 0;
      } else if (++good >= a.growth) {
        sn = scale * 2.f;
        good = 0;
      }
      a.loss_scale[(step + 1) & 1] = sn;
      a.scale_state[0] = good;
    }
    return;
  }
  if (a.freeze) return;
  const LatentBits lbits(m);
  const long long L = m.latent_count;
  // one latent: update in place (unless the step is skipped) and its forward value
  auto one = [&](long long i, float& p, float gr, float& mm, float& vv) -> float {
    const int bits = lbits(i);
    if (!ovf) {
      gr *= inv_s;
      mm = b1 * mm + (1.f - b1) * gr;
      vv = b2 * vv + (1.f - b2) * gr * gr;
      p = p - lr_lat * (mm * ib1) / (sqrtf(vv * ib2) + eps);
      const float lo = -0.5f + ldexpf(1.f, -bits - 1);  // -(N-1)/(2N)
      p = fminf(fmaxf(p, lo), 0.5f);
    }
    return a.noise ? p + noise_at(next_key, i, bits) : p;
  };
  // four consecutive latents per thread and iteration (16-byte accesses), the next
  // iteration's loads issued before this one's arithmetic and stores; then the tail
  const long long base = ((long long)bx - args.mlp_blocks) * 256 + threadIdx.x;
  const long long stride = ((long long)gx - args.mlp_blocks) * 256;
  const long long nv = L / 4;
  f32x4 np, ngr, nmm, nvv;
  if (base < nv) {
    np = reinterpret_cast<const f32x4*>(a.latents)[base];
    ngr = reinterpret_cast<const f32x4*>(a.lat_grad)[base];
    nmm = reinterpret_cast<const f32x4*>(a.lat_m)[base];
    nvv = reinterpret_cast<const f32x4*>(a.lat_v)[base];
  }
  for (long long v4 = base; v4 < nv; v4 += stride) {
    const long long i = 4 * v4;
    f32x4 p = np, gr = ngr, mm = nmm, vv = nvv;
    if (v4 + stride < nv) {
      np = reinterpret_cast<const f32x4*>(a.latents)[v4 + stride];
      ngr = reinterpret_cast<const f32x4*>(a.lat_grad)[v4 + stride];
      nmm = reinterpret_cast<const f32x4*>(a.lat_m)[v4 + stride];
      nvv = reinterpret_cast<const f32x4*>(a.lat_v)[v4 + stride];
    }
    f32x4 fw;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      float pk = p[k], mk = mm[k], vk = vv[k];
      fw[k] = one(i + k, pk, gr[k], mk, vk);
      p[k] = pk;
      mm[k] = mk;
      vv[k] = vk;
    }
    if (!ovf) {
      reinterpret_cast<f32x4*>(a.lat_m)[v4] = mm;
      reinterpret_cast<f32x4*>(a.lat_v)[v4] = vv;
      reinterpret_cast<f32x4*>(a.latents)[v4] = p;
    }
    reinterpret_cast<f32x4*>(a.latents_fwd)[v4] = fw;
  }
  for (long long i = 4 * nv + base; i < L; i += stride) {
    float p = a.latents[i], mm = a.lat_m[i], vv = a.lat_v[i];
    const float fw = one(i, p, a.lat_grad[i], mm, vv);
    if (!ovf) {
      a.lat_m[i] = mm;
      a.lat_v[i] = vv;
      a.latents[i] = p;
    }
    a.latents_fwd[i] = fw;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void adam_kernel(DevMat m, AdamArgs args) {
  adam_body<T>(m, args, blockIdx.x, gridDim.x);
}

// Device-step mode: the step index advances once the update has read it.
__global__ void step_advance_kernel(int* step) {
  if (blockIdx.x == 0 && threadIdx.x == 0) *step += 1;
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

// ------------------------------------------------------------------ grouped step
// A training step of many materials where each stage (binning, scans, partial
// reduction, weight-gradient reduction, Adam) is one launch for the whole group: a
// block finds its material's segment, then runs the single-material body on that
// material's entry of a device table.
struct TrainEntry {
  DevMat m;
  TileGeom tg;
  TrainArgs fa;       // the fused pass (queries, step slot and binning come with each launch)
  PeTable pe;
  BinArgs bin;        // q is unused: the launch's queries + q0
  AdamArgs adam;      // pointers; step-dependent scalars come with each launch
  long long q0, P;
  int nbins, ntiles, region_max, fused_grid;
  float loss_norm;
  int* offsets;
  int* total;
  int* base;
  int* tstart;
  int* ttotal;
  int* ibase;
  int* itile;
  int* nitems;
  const float* part_lat;
  float* lat_grad;
  const float* part_dw;
  float* grad;
  const float* part_loss;
  float* loss_out;
  int32_t* overflow;
};

constexpr int kTrainGroup = 64;  // materials per grouped launch
struct TrainSegs {
  unsigned long long hash;
  int count, first;             // materials first .. first + count - 1 of the table
  int block0[kTrainGroup + 1];  // first block of each material; block0[count] = all blocks
};

// The material of this block (the last segment starting at or before it) and the
// block's index within it.
__device__ inline const TrainEntry* group_member(const char* table, const TrainSegs& sg, int& bi, int& nb) {
  if (*reinterpret_cast<const unsigned long long*>(table) != sg.hash) return nullptr;
  const int b = blockIdx.x;
  int lo = 0, hi = sg.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg.block0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  bi = b - sg.block0[lo];
  nb = sg.block0[lo + 1] - sg.block0[lo];
  return reinterpret_cast<const TrainEntry*>(table + kGroupHeaderBytes) + sg.first + lo;
}

// The fused pass of the members of one kernel shape (at most kTrainGroup, any table
// entries): member i takes blocks [block0[i], block0[i + 1]), as many as its own launch
// would have, and each block runs the single-material body with the same share of the
// member's work items, so the sums equal the member's own launch bit for bit.
struct FusedSegs {
  unsigned long long hash;
  int count;
  int mat[kTrainGroup];         // table entries of the members
  int block0[kTrainGroup + 1];  // first block of each member; block0[count] = all blocks
};

template <typename T, int C0, int C1, int C, int HD, int ACT>
__global__ __launch_bounds__((TrainCfg<T, C0, C1, C, HD>::NTHR),
                             (TrainCfg<T, C0, C1, C, HD>::NW * TrainCfg<T, C0, C1, C, HD>::BPC / 4)) void
train_fused_grouped(const char* __restrict__ table, FusedSegs sg, const ntc_query* __restrict__ q, int scale_slot,
                    const int* __restrict__ step_dev, int binned) {
  if (*reinterpret_cast<const unsigned long long*>(table) != sg.hash) return;
  const int b = blockIdx.x;
  int lo = 0, hi = sg.count - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sg.block0[mid] <= b) lo = mid;
    else hi = mid - 1;
  }
  const int bi = b - sg.block0[lo], nb = sg.block0[lo + 1] - sg.block0[lo];
  // through the constant address space: the entry's loads are invariant, so the compiler
  // reloads fields rather than keeping them live (as it does with kernel arguments)
  using CEntry = const __attribute__((address_space(4))) TrainEntry;
  const TrainEntry& e = *(const TrainEntry*)((CEntry*)(table + kGroupHeaderBytes) + sg.mat[lo]);
  fused_body<T, C0, C1, C, HD, ACT>(e.m, e.pe, e.fa, q + e.q0, binned, scale_slot, step_dev, bi, -1, nb, bi, bi == 0);
}

template <bool SCATTER>
__global__ __launch_bounds__(kBinThreads, 8) void bin_grouped(const char* __restrict__ table, TrainSegs sg,
                                                   const ntc_query* __restrict__ q) {
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (e) bin_body<SCATTER>(e->m, e->tg, e->bin, q + e->q0, bi);
}

__global__ __launch_bounds__(256) void bin_scan1_grouped(const char* __restrict__ table, TrainSegs sg) {
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (e) bin_scan1_body(e->nbins, e->bin.nbb, e->bin.counts, e->offsets, e->total, bi);
}

__global__ __launch_bounds__(1024) void bin_scan2_grouped(const char* __restrict__ table, TrainSegs sg) {
  __shared__ int s_base[kMaxBins + 1];
  __shared__ int s_scan[1024];
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (e) bin_scan2_body(e->tg, e->total, e->base, e->tstart, e->ttotal, e->ibase, e->itile, e->nitems, s_base, s_scan);
}

// one block per tile of each member (a grid of gx x 64 per member, as for one material,
// would reach hundreds of thousands of blocks on a many-material step)
__global__ __launch_bounds__(256) void lat_partial_grouped(const char* __restrict__ table, TrainSegs sg) {
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (e) lat_partial_body(e->m, e->tg, e->ibase, e->part_lat, e->region_max, e->lat_grad, 1.f, bi, 0, 1);
}

__global__ __launch_bounds__(64 * kDwWaves) void dw_reduce_grouped(const char* __restrict__ table, TrainSegs sg) {
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (e)
    dw_reduce_body(e->fused_grid, e->P, e->part_dw, e->grad, e->part_loss, e->loss_out, e->loss_norm, e->overflow,
                   1.f, bi);
}

// Step-dependent Adam scalars shared by the group (from the hyper-parameters).
struct AdamHot {
  float lr_lat, lr_mlp, beta1, beta2, eps, bc1, bc2;
  uint64_t next_key, seed;
  int step, noise, freeze, growth;
  int* step_dev;
  const float* lr_dev;
};

template <typename T>
__global__ __launch_bounds__(256) void adam_grouped(const char* __restrict__ table, TrainSegs sg, AdamHot h) {
  int bi, nb;
  const TrainEntry* e = group_member(table, sg, bi, nb);
  if (!e) return;
  AdamArgs args = e->adam;
  AdamLaunch& a = args.a;
  a.lr_lat = h.lr_lat;
  a.lr_mlp = h.lr_mlp;
  a.beta1 = h.beta1;
  a.beta2 = h.beta2;
  a.eps = h.eps;
  a.bc1 = h.bc1;
  a.bc2 = h.bc2;
  a.next_key = h.next_key;
  a.seed = h.seed;
  a.step = h.step;
  a.noise = h.noise;
  a.freeze = h.freeze;
  a.growth = h.growth;
  a.step_dev = h.step_dev;
  a.lr_dev = h.lr_dev;
  adam_body<T>(e->m, args, bi, nb);
}

// ------------------------------------------------------------------ host side
template <typename T, int C0, int C1, int C, int HD, int ACT>
static int fused_per_cu() {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  static const int per_cu = blocks_per_cu(train_fused_kernel<T, C0, C1, C, HD, ACT>, Cfg::NTHR, Cfg::LDS);
  return per_cu;
}

template <typename T, int C0, int C1, int C, int HD>
static void shape_info(int act, int& tmax, int& per_cu) {
  tmax = TrainCfg<T, C0, C1, C, HD>::TMAX;
  per_cu = act ? fused_per_cu<T, C0, C1, C, HD, 1>() : fused_per_cu<T, C0, C1, C, HD, 0>();
}

// Kernel arguments of a material's fused pass from its plan and buffers.
static TrainArgs make_train_args(const ntc_material& mm, const TrainPlan& p, const TrainLaunch& l) {
  char* ws = (char*)l.workspace;
  TrainArgs a;
  a.lat_fwd = l.lat_fwd;
  a.wpack = l.wpack;
  a.mlp = l.mlp;
  a.q = l.q;
  a.n = l.n;
  a.targets = l.targets;
  a.lat_grad = l.lat_grad;
  a.part_lat = (float*)(ws + p.off_part_lat);
  a.list = (const int4*)(ws + p.off_list);
  a.tile_start = (const int*)(ws + p.off_tstart);
  a.tile_total = (const int*)(ws + p.off_ttotal);
  a.item_base = (const int*)(ws + p.off_ibase);
  a.item_tile = (const int*)(ws + p.off_itile);
  a.nitems = (const int*)(ws + p.off_misc);
  a.part_dw = (float*)(ws + p.off_part_dw);
  a.part_loss = (float*)(ws + p.off_part_loss);
  a.loss_scale = l.loss_scale;
  a.scale_slot = l.scale_slot;
  a.step_dev = l.step_dev;
  a.overflow_flag = l.overflow_flag;
  a.binned = l.scatter_latents ? 1 : 0;
  a.region_max = p.region_max;
  a.inv_nc = (float)(1.0 / ((double)l.n * mm.channels));
  a.dout = l.dout;
  a.dout_scale = l.dout_scale;
  a.out_scale = l.out_scale;
  a.dscale = l.dscale;
  a.table_hash = l.table_hash;
  a.hash = l.hash;
  a.tg = p.tg;
  return a;
}

template <typename T, int C0, int C1, int C, int HD, int ACT>
static hipError_t fused_t(const ntc_material& mm, const TrainPlan& p, const TrainLaunch& l, hipStream_t s) {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  const TrainArgs a = make_train_args(mm, p, l);
  const int slot = timing_before(TK_TRAIN_FUSED, s);
  hipLaunchKernelGGL((train_fused_kernel<T, C0, C1, C, HD, ACT>), dim3(p.grid), dim3(Cfg::NTHR), Cfg::LDS, s, dev_mat(mm),
                     pe_table(mm), a);
  timing_after(TK_TRAIN_FUSED, s, slot);
  return hipGetLastError();
}

// (c0, c1, channels, hidden): the configurations' shapes and Table 3's four profiles on a
// 9-channel texture set
#define NTC_TRAIN_SHAPES(X)                                                            \
  X(8, 8, 8, 64) X(10, 10, 10, 64) X(12, 12, 12, 64) X(16, 16, 16, 64) X(8, 8, 8, 32) \
  X(10, 10, 10, 32) X(12, 12, 12, 32) X(16, 16, 16, 32)                              \
  X(8, 12, 9, 64) X(12, 20, 9, 64) X(12, 10, 9, 64) X(16, 12, 9, 64)

bool train_shape_supported(int c0, int c1, int c, int hd) {
#define NTC_X(a, b, cc, h) \
  if (c0 == a && c1 == b && c == cc && hd == h) return true;
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  return false;
}

static size_t align256(size_t b) { return (b + 255) / 256 * 256; }

// ------------------------------------------------------------------ tuning table
// Work-item size and tile side per (shape, precision, activation), chosen by
// ntc_train_autotune; plans without an entry use the defaults.
namespace {
struct TuneKey {
  int c0, c1, c, hd, f16, act;
  bool operator==(const TuneKey& o) const {
    return c0 == o.c0 && c1 == o.c1 && c == o.c && hd == o.hd && f16 == o.f16 && act == o.act;
  }
};
struct TuneTable {
  std::mutex mu;
  std::vector<std::pair<TuneKey, TrainTune>> rows;
};
TuneTable& tune_table() {
  static TuneTable t;
  return t;
}
TuneKey tune_key(const ntc_material& m, bool f16) {
  return TuneKey{m.c0, m.c1, m.channels, m.hidden, f16 ? 1 : 0, m.activation};
}
}  // namespace

void set_train_tune(const ntc_material& m, bool f16, const TrainTune& t) {
  TuneTable& tb = tune_table();
  std::lock_guard<std::mutex> lock(tb.mu);
  const TuneKey k = tune_key(m, f16);
  for (auto& r : tb.rows)
    if (r.first == k) {
      r.second = t;
      return;
    }
  tb.rows.push_back({k, t});
}

void clear_train_tune(const ntc_material& m, bool f16) {
  TuneTable& tb = tune_table();
  std::lock_guard<std::mutex> lock(tb.mu);
  const TuneKey k = tune_key(m, f16);
  for (size_t i = 0; i < tb.rows.size(); ++i)
    if (tb.rows[i].first == k) {
      tb.rows.erase(tb.rows.begin() + (long)i);
      return;
    }
}

TrainTune get_train_tune(const ntc_material& m, bool f16) {
  TuneTable& tb = tune_table();
  std::lock_guard<std::mutex> lock(tb.mu);
  const TuneKey k = tune_key(m, f16);
  for (auto& r : tb.rows)
    if (r.first == k) return r.second;
  return TrainTune{0, 0};  // untuned: the plan's defaults
}

const TrainTune* train_tune_candidates(int* count) {
  static const TrainTune c[] = {{256, 8}, {512, 8}, {256, 16}, {512, 16}, {1024, 16}, {512, 32}, {1024, 32}};
  *count = (int)(sizeof c / sizeof c[0]);
  return c;
}

TrainPlan train_plan(const ntc_material& m, bool f16, long long n, const TrainTune* tune) {
  TrainPlan p{};
  const TrainTune tn = tune ? *tune : get_train_tune(m, f16);
  int tmax = 8, per_cu = 1;
#define NTC_X(a_, b, cc, h)                                                                          \
  if (m.c0 == a_ && m.c1 == b && m.channels == cc && m.hidden == h) {                                \
    if (f16) shape_info<_Float16, a_, b, cc, h>(m.activation, tmax, per_cu);                         \
    else shape_info<float, a_, b, cc, h>(m.activation, tmax, per_cu);                                \
  }
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  if (tn.tile > 0) tmax = std::min(tmax, tn.tile);  // tile sides at most the kernel's capacity
  // untuned: 512 samples per work item with 32 x 32 tiles (a level-0 tile of the 2048^2
  // benchmark material then takes a single item), 256 with smaller tiles
  const int chunk = tn.chunk > 0 ? tn.chunk : tmax >= 32 ? 2 * kChunkDefault : kChunkDefault;
  TileGeom& tg = p.tg;
  std::memset(&tg, 0, sizeof tg);
  tg.chunk = chunk;
  p.tune = TrainTune{chunk, tmax};
  int nb = 0, nt = 0, rmax = 0;
  for (int j = 0; j < m.num_levels; ++j) {
    const int T = std::min(tmax, std::min(m.g0_w[j], m.g0_h[j]));
    tg.T[j] = T;
    tg.ntx[j] = m.g0_w[j] / T;
    tg.nty[j] = m.g0_h[j] / T;
    const int tiles = tg.ntx[j] * tg.nty[j];
    // levels with few cells (many samples per cell) are sorted by anchor cell
    tg.sb[j] = (tiles * T * T <= kSortedCells) ? T : 1;
    tg.tile_base[j] = nt;
    tg.bin_base[j] = nb;
    tg.region[j] = T * T * m.c0 + (T / 2) * (T / 2) * m.c1;
    rmax = std::max(rmax, tg.region[j]);
    nt += tiles;
    nb += tiles * tg.sb[j] * tg.sb[j];
  }
  for (int j = m.num_levels; j <= kMaxLevels; ++j) {
    tg.tile_base[j] = nt;
    tg.bin_base[j] = nb;
  }
  tg.ntiles = nt;
  tg.nbins = nb;
  tg.region_max = rmax;
  p.region_max = rmax;
  p.nbins = nb;
  p.ntiles = nt;
  p.nbb = (int)std::max<long long>(1, std::min<long long>(256, (n + kBinBlockSamples - 1) / kBinBlockSamples));
  p.per_bin_block = (int)((n + p.nbb - 1) / p.nbb);
  p.max_items = nt + (4 * n + chunk - 1) / chunk;
  const long long work_items = std::max<long long>(p.max_items, (n + chunk - 1) / chunk);
  p.grid = (int)std::max<long long>(1, std::min<long long>(work_items, (long long)device_cus() * per_cu));
  const size_t P = (size_t)m.mlp_params;
  size_t o = 0;
  auto take = [&](size_t bytes) {
    const size_t r = o;
    o += align256(bytes);
    return r;
  };
  p.off_counts = take((size_t)p.nbb * nb * 4);
  p.off_offsets = take((size_t)p.nbb * nb * 4);
  p.off_total = take((size_t)nb * 4);
  p.off_base = take((size_t)(nb + 1) * 4);
  p.off_tstart = take((size_t)nt * 4);
  p.off_ttotal = take((size_t)nt * 4);
  p.off_ibase = take((size_t)(nt + 1) * 4);
  p.off_itile = take((size_t)p.max_items * 4);
  p.off_misc = take(64);
  p.off_list = take((size_t)4 * n * 16);
  p.off_part_lat = take((size_t)p.max_items * rmax * 4);
  p.off_part_dw = take((size_t)p.grid * P * 4);
  p.off_part_loss = take((size_t)p.grid * 4);
  p.off_grad = take(P * 4);
  p.off_dscale = take((size_t)(2 + kScaleBlocks) * 4);
  p.total = o;
  p.supported_bins = nb <= kMaxBins;
  return p;
}

static hipError_t launch_train_fused(const ntc_material& m, bool f16, const TrainPlan& p, const TrainLaunch& l,
                                     hipStream_t s) {
  hipError_t e = hipErrorInvalidValue;
#define NTC_X(a_, b_, cc, h)                                                                     \
  if (m.c0 == a_ && m.c1 == b_ && m.channels == cc && m.hidden == h)                             \
    e = f16 ? (m.activation ? fused_t<_Float16, a_, b_, cc, h, 1>(m, p, l, s)                  \
                            : fused_t<_Float16, a_, b_, cc, h, 0>(m, p, l, s))                   \
            : (m.activation ? fused_t<float, a_, b_, cc, h, 1>(m, p, l, s)                       \
                            : fused_t<float, a_, b_, cc, h, 0>(m, p, l, s));
  NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
  return e;
}

hipError_t launch_train_gradients(const ntc_material& m, bool f16, const TrainPlan& p, const TrainLaunch& l,
                                  hipStream_t s) {
  char* ws = (char*)l.workspace;
  const DevMat dm = dev_mat(m);
  if (l.scatter_latents) {
    BinArgs b;
    b.q = l.q;
    b.n = l.n;
    b.per_block = p.per_bin_block;
    b.nbb = p.nbb;
    b.counts = (int*)(ws + p.off_counts);
    b.offsets = (const int*)(ws + p.off_offsets);
    b.base = (const int*)(ws + p.off_base);
    b.list = (int4*)(ws + p.off_list);
    b.total = nullptr;
    const size_t lds = (size_t)(p.nbins + 1) * 4;
    hipLaunchKernelGGL(bin_kernel<false>, dim3(p.nbb), dim3(kBinThreads), lds, s, dm, p.tg, b);
    hipLaunchKernelGGL(bin_scan1_kernel, dim3((p.nbins + 3) / 4), dim3(256), 0, s, p.nbins, p.nbb,
                       (const int*)(ws + p.off_counts), (int*)(ws + p.off_offsets), (int*)(ws + p.off_total));
    b.total = (const int*)(ws + p.off_total);
    TileTables o;
    o.base = (int*)(ws + p.off_base);
    o.tile_start = (int*)(ws + p.off_tstart);
    o.tile_total = (int*)(ws + p.off_ttotal);
    o.item_base = (int*)(ws + p.off_ibase);
    o.item_tile = (int*)(ws + p.off_itile);
    o.nitems = (int*)(ws + p.off_misc);
    hipLaunchKernelGGL(bin_scatter_kernel, dim3(p.nbb + 1), dim3(kBinThreads), lds, s, dm, p.tg, b, o);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  e = launch_train_fused(m, f16, p, l, s);
  if (e != hipSuccess) return e;
  if (l.scatter_latents) {
    hipLaunchKernelGGL(lat_partial_reduce, dim3(lat_partial_gx(p.region_max), lat_partial_ty(p.ntiles)), dim3(256), 0,
                       s, dm, p.tg,
                       (const int*)(ws + p.off_ibase), (const float*)(ws + p.off_part_lat), p.region_max, l.lat_grad,
                       l.out_scale, l.dscale);
  }
  return hipGetLastError();
}

hipError_t launch_train_reduce(const ntc_material& m, const TrainPlan& p, void* workspace, float* loss_out,
                               float loss_norm, int32_t* overflow_flag, hipStream_t s, float* grad_out,
                               float out_scale, const float* dscale) {
  char* ws = (char*)workspace;
  const long long P = m.mlp_params;
  hipLaunchKernelGGL(dw_reduce, dim3((unsigned)((P + 63) / 64)), dim3(64 * kDwWaves), 0, s, p.grid, P,
                     (const float*)(ws + p.off_part_dw), grad_out ? grad_out : (float*)(ws + p.off_grad),
                     (const float*)(ws + p.off_part_loss), loss_out, loss_norm, overflow_flag, out_scale, dscale);
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
  if (a.step_dev && a.advance) hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, s, a.step_dev);
  return hipGetLastError();
}

hipError_t launch_step_advance(int* step_dev, hipStream_t s) {
  hipLaunchKernelGGL(step_advance_kernel, dim3(1), dim3(64), 0, s, step_dev);
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


// ------------------------------------------------------------------ grouped step (host)
// Per-material launch geometry of a grouped step, derived identically by the table
// set-up and by every step.
struct GroupMember {
  TrainPlan p;
  long long q0, n;
  int lat_blocks;  // Adam blocks over the latents (a share of the device's, by latent count)
};

static std::vector<GroupMember> plan_group(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16) {
  std::vector<GroupMember> g(nmat);
  long long lat_total = 0;
  for (int i = 0; i < nmat; ++i) lat_total += mats[i].latent_count;
  const long long cap = (long long)device_cus() * 8;
  for (int i = 0; i < nmat; ++i) {
    GroupMember& x = g[i];
    x.q0 = offsets[i];
    x.n = offsets[i + 1] - offsets[i];
    x.p = train_plan(mats[i], f16, x.n);
    const long long L = mats[i].latent_count;
    long long b = lat_total > 0 ? (cap * L + lat_total - 1) / lat_total : 1;
    b = std::max(1LL, std::min(b, (L + 255) / 256));
    x.lat_blocks = (int)b;
  }
  return g;
}

size_t train_table_bytes(int nmat) { return (size_t)kGroupHeaderBytes + (size_t)nmat * sizeof(TrainEntry); }

// FNV-1a over everything a table encodes that a step can see: the materials, their
// plans and sample groups, the precision and the buffers of every member.
unsigned long long train_group_hash(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16,
                                    const TrainLaunch* fused, const AdamLaunch* adam) {
  unsigned long long h = 1469598103934665603ULL;
  auto mix = [&](const void* p, size_t bytes) {
    const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ULL;
  };
  mix(&nmat, sizeof nmat);
  const int fl = f16 ? 1 : 0;
  mix(&fl, sizeof fl);
  const std::vector<GroupMember> g = plan_group(mats, nmat, offsets, f16);
  for (int i = 0; i < nmat; ++i) {
    const DevMat d = dev_mat(mats[i]);
    mix(&d, sizeof d);
    mix(&g[i].p.tg, sizeof g[i].p.tg);
    mix(&g[i].p.grid, sizeof g[i].p.grid);
    mix(&g[i].q0, sizeof g[i].q0);
    mix(&g[i].n, sizeof g[i].n);
    const void* ptrs[] = {fused[i].lat_fwd, fused[i].wpack, fused[i].mlp, fused[i].targets, fused[i].lat_grad,
                          fused[i].workspace, fused[i].loss_scale, fused[i].overflow_flag, adam[i].latents,
                          adam[i].lat_m, adam[i].lat_v, adam[i].mlp_m, adam[i].mlp_v, adam[i].scale_state};
    mix(ptrs, sizeof ptrs);
  }
  return h;
}

void fill_train_table(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16, const TrainLaunch* fused,
                      const AdamLaunch* adam, unsigned long long hash, void* host_table) {
  char* t = reinterpret_cast<char*>(host_table);
  std::memset(t, 0, train_table_bytes(nmat));
  std::memcpy(t, &hash, sizeof hash);
  const std::vector<GroupMember> g = plan_group(mats, nmat, offsets, f16);
  TrainEntry* ent = reinterpret_cast<TrainEntry*>(t + kGroupHeaderBytes);
  for (int i = 0; i < nmat; ++i) {
    const ntc_material& m = mats[i];
    const TrainPlan& p = g[i].p;
    TrainEntry& e = ent[i];
    char* ws = (char*)fused[i].workspace;
    e.m = dev_mat(m);
    e.tg = p.tg;
    e.fa = make_train_args(m, p, fused[i]);
    e.fa.q = nullptr;
    e.fa.table_hash = nullptr;
    e.pe = pe_table(m);
    e.bin.q = nullptr;
    e.bin.n = g[i].n;
    e.bin.per_block = p.per_bin_block;
    e.bin.nbb = p.nbb;
    e.bin.counts = (int*)(ws + p.off_counts);
    e.bin.offsets = (const int*)(ws + p.off_offsets);
    e.bin.base = (const int*)(ws + p.off_base);
    e.bin.list = (int4*)(ws + p.off_list);
    e.bin.total = nullptr;  // the grouped step scans the bases in its own launch
    e.adam.a = adam[i];
    e.adam.a.mlp_grad = (const float*)(ws + p.off_grad);
    e.adam.pg = pack_geom(m.c0, m.c1, m.hidden, f16);
    e.adam.P = m.mlp_params;
    e.adam.mlp_blocks = (int)((m.mlp_params + 255) / 256);
    e.q0 = g[i].q0;
    e.P = m.mlp_params;
    e.nbins = p.nbins;
    e.ntiles = p.ntiles;
    e.region_max = p.region_max;
    e.fused_grid = p.grid;
    e.loss_norm = 1.0f / (float)((double)g[i].n * m.channels);
    e.offsets = (int*)(ws + p.off_offsets);
    e.total = (int*)(ws + p.off_total);
    e.base = (int*)(ws + p.off_base);
    e.tstart = (int*)(ws + p.off_tstart);
    e.ttotal = (int*)(ws + p.off_ttotal);
    e.ibase = (int*)(ws + p.off_ibase);
    e.itile = (int*)(ws + p.off_itile);
    e.nitems = (int*)(ws + p.off_misc);
    e.part_lat = (const float*)(ws + p.off_part_lat);
    e.lat_grad = fused[i].lat_grad;
    e.part_dw = (const float*)(ws + p.off_part_dw);
    e.grad = (float*)(ws + p.off_grad);
    e.part_loss = (const float*)(ws + p.off_part_loss);
    e.loss_out = adam[i].loss_out;
    e.overflow = fused[i].overflow_flag;
  }
}

// One grouped launch per stage (and per kTrainGroup materials); blocks(i) gives the
// blocks of material i.
template <typename Blocks, typename Launch>
static hipError_t group_launch(int nmat, unsigned long long hash, Blocks&& blocks, Launch&& launch) {
  for (int f = 0; f < nmat; f += kTrainGroup) {
    TrainSegs sg{};
    sg.hash = hash;
    sg.first = f;
    sg.count = std::min(kTrainGroup, nmat - f);
    int total = 0;
    for (int i = 0; i < sg.count; ++i) {
      sg.block0[i] = total;
      total += blocks(f + i);
    }
    sg.block0[sg.count] = total;
    if (total == 0) continue;
    launch(sg, total);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T, int C0, int C1, int C, int HD, int ACT>
static void fused_grouped_t(const char* tab, const FusedSegs& sg, int blocks, const ntc_query* q, int scale_slot,
                            const int* step_dev, int binned, hipStream_t s) {
  using Cfg = TrainCfg<T, C0, C1, C, HD>;
  const int slot = timing_before(TK_TRAIN_FUSED, s);
  hipLaunchKernelGGL((train_fused_grouped<T, C0, C1, C, HD, ACT>), dim3(blocks), dim3(Cfg::NTHR), Cfg::LDS, s, tab,
                     sg, q, scale_slot, step_dev, binned);
  timing_after(TK_TRAIN_FUSED, s, slot);
}

// One fused launch per kernel shape (c0, c1, channels, hidden, activation) and per
// kTrainGroup members of it.
static hipError_t launch_fused_grouped(const ntc_material* mats, int nmat, bool f16, const char* tab,
                                       unsigned long long hash, const std::vector<GroupMember>& g, const ntc_query* q,
                                       int scale_slot, const int* step_dev, int binned, hipStream_t s) {
  std::vector<bool> done(nmat, false);
  for (int i0 = 0; i0 < nmat; ++i0) {
    if (done[i0]) continue;
    const ntc_material& k = mats[i0];
    std::vector<int> members;
    for (int i = i0; i < nmat; ++i)
      if (!done[i] && mats[i].c0 == k.c0 && mats[i].c1 == k.c1 && mats[i].channels == k.channels &&
          mats[i].hidden == k.hidden && mats[i].activation == k.activation) {
        members.push_back(i);
        done[i] = true;
      }
    for (size_t f = 0; f < members.size(); f += kTrainGroup) {
      FusedSegs sg{};
      sg.hash = hash;
      sg.count = (int)std::min<size_t>(kTrainGroup, members.size() - f);
      int total = 0;
      for (int i = 0; i < sg.count; ++i) {
        sg.mat[i] = members[f + i];
        sg.block0[i] = total;
        total += g[members[f + i]].p.grid;
      }
      sg.block0[sg.count] = total;
      bool found = false;
#define NTC_X(a_, b_, cc, h)                                                                                \
  if (k.c0 == a_ && k.c1 == b_ && k.channels == cc && k.hidden == h) {                                    \
    found = true;                                                                                         \
    if (f16) {                                                                                            \
      if (k.activation) fused_grouped_t<_Float16, a_, b_, cc, h, 1>(tab, sg, total, q, scale_slot, step_dev, binned, s); \
      else fused_grouped_t<_Float16, a_, b_, cc, h, 0>(tab, sg, total, q, scale_slot, step_dev, binned, s);  \
    } else {                                                                                              \
      if (k.activation) fused_grouped_t<float, a_, b_, cc, h, 1>(tab, sg, total, q, scale_slot, step_dev, binned, s); \
      else fused_grouped_t<float, a_, b_, cc, h, 0>(tab, sg, total, q, scale_slot, step_dev, binned, s);     \
    }                                                                                                     \
  }
      NTC_TRAIN_SHAPES(NTC_X)
#undef NTC_X
      if (!found) return hipErrorInvalidValue;
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
  }
  return hipSuccess;
}

hipError_t launch_train_grouped(const ntc_material* mats, int nmat, const int64_t* offsets, bool f16,
                                const void* table, unsigned long long hash, const ntc_query* q, bool scatter,
                                const TrainLaunch* fused, const AdamLaunch& hot, hipStream_t s) {
  const char* tab = reinterpret_cast<const char*>(table);
  const std::vector<GroupMember> g = plan_group(mats, nmat, offsets, f16);
  int max_bins = 0;
  for (int i = 0; i < nmat; ++i) max_bins = std::max(max_bins, g[i].p.nbins);
  hipError_t e = hipSuccess;
  auto run = [&](auto blocks, auto launch) {
    if (e == hipSuccess) e = group_launch(nmat, hash, blocks, launch);
  };
  if (scatter) {
    const size_t lds = (size_t)(max_bins + 1) * 4;
    run([&](int i) { return g[i].p.nbb; },
        [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(bin_grouped<false>, dim3(n), dim3(kBinThreads), lds, s, tab, sg, q); });
    run([&](int i) { return (g[i].p.nbins + 3) / 4; },
        [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(bin_scan1_grouped, dim3(n), dim3(256), 0, s, tab, sg); });
    run([&](int) { return 1; },
        [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(bin_scan2_grouped, dim3(n), dim3(1024), 0, s, tab, sg); });
    run([&](int i) { return g[i].p.nbb; },
        [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(bin_grouped<true>, dim3(n), dim3(kBinThreads), lds, s, tab, sg, q); });
  }
  if (e == hipSuccess)
    e = launch_fused_grouped(mats, nmat, f16, tab, hash, g, q, fused[0].scale_slot, fused[0].step_dev,
                             scatter ? 1 : 0, s);
  if (scatter)
    run([&](int i) { return g[i].p.ntiles; },
        [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(lat_partial_grouped, dim3(n), dim3(256), 0, s, tab, sg); });
  run([&](int i) { return (int)((mats[i].mlp_params + 63) / 64); },
      [&](const TrainSegs& sg, int n) { hipLaunchKernelGGL(dw_reduce_grouped, dim3(n), dim3(64 * kDwWaves), 0, s, tab, sg); });
  AdamHot h;
  h.lr_lat = hot.lr_lat;
  h.lr_mlp = hot.lr_mlp;
  h.beta1 = hot.beta1;
  h.beta2 = hot.beta2;
  h.eps = hot.eps;
  h.bc1 = hot.bc1;
  h.bc2 = hot.bc2;
  h.next_key = hot.next_key;
  h.seed = hot.seed;
  h.step = hot.step;
  h.noise = hot.noise;
  h.freeze = hot.freeze;
  h.growth = hot.growth;
  h.step_dev = hot.step_dev;
  h.lr_dev = hot.lr_dev;
  run([&](int i) { return (int)((mats[i].mlp_params + 255) / 256) + g[i].lat_blocks; },
      [&](const TrainSegs& sg, int n) {
        if (f16) hipLaunchKernelGGL(adam_grouped<_Float16>, dim3(n), dim3(256), 0, s, tab, sg, h);
        else hipLaunchKernelGGL(adam_grouped<float>, dim3(n), dim3(256), 0, s, tab, sg, h);
      });
  if (e == hipSuccess && hot.step_dev) e = launch_step_advance(hot.step_dev, s);
  return e;
}

}  // namespace ntc
