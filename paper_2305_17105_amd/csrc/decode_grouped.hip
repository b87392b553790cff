// Grouped decode of many materials (the per-material networks of section 6, decoded
// together): one launch per kernel shape covers the query groups of every material
// of that shape.  Blocks are shared out over the materials in proportion to their
// queries; each block takes its material's geometry and pointers from a device table
// and decodes a strided share of that material's tiles with the material's weights
// staged in LDS, exactly as the single-material kernel does.
#include <algorithm>
#include <cstring>
#include <vector>

#include "decode_impl.h"

namespace ntc {

namespace {

struct GroupItem {
  int mat;
  long long q0, n, o0;
};

// Splits the items of one shape into launches of at most kGroupSegs segments and
// gives each material blocks in proportion to its tiles (at least one, at most one
// per four tiles), about `cap` blocks per launch in all.
template <typename Launch>
hipError_t launch_segments(const std::vector<GroupItem>& items, long long cap, unsigned long long hash,
                           Launch&& launch) {
  for (size_t i0 = 0; i0 < items.size(); i0 += kGroupSegs) {
    const size_t i1 = std::min(items.size(), i0 + (size_t)kGroupSegs);
    long long tiles = 0;
    for (size_t i = i0; i < i1; ++i) tiles += (items[i].n + 15) / 16;
    GroupArgs ga{};
    ga.hash = hash;
    int blocks = 0;
    for (size_t i = i0; i < i1; ++i) {
      const long long t = (items[i].n + 15) / 16;
      long long b = (cap * t + tiles - 1) / tiles;
      b = std::max(1LL, std::min(b, (t + 3) / 4));
      GroupSeg& sg = ga.seg[ga.count++];
      sg.mat = items[i].mat;
      sg.block0 = blocks;
      sg.q0 = items[i].q0;
      sg.n = items[i].n;
      sg.o0 = items[i].o0;
      blocks += (int)b;
    }
    ga.blocks = blocks;
    launch(ga);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}


template <typename T, int C0, int C1, int C, int HD, int B0, int B1, int ACT>
hipError_t grouped_t(const ntc_material* mats, const char* tab, unsigned long long hash,
                     const std::vector<GroupItem>& items,
                     const ntc_query* q, char* out, bool out_f16, hipStream_t s) {
  using DL = DecodeLayout<T, C0, C1, HD, B0, B1, true>;
  constexpr int WB = DL::WB;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4 + kMaxLevels * sizeof(LevelBytes) + DL::SLAB;
  auto kern = decode_grouped_kernel<T, C0, C1, C, HD, B0, B1, ACT>;
  static const int per_cu = blocks_per_cu(kern, 256, lds);
  const PeTable pe = pe_table(mats[items[0].mat]);
  return launch_segments(items, (long long)device_cus() * per_cu, hash, [&](const GroupArgs& ga) {
    hipLaunchKernelGGL(kern, dim3((unsigned)ga.blocks), dim3(256), lds, s, tab, pe, ga, q, out, out_f16 ? 1 : 0);
  });
}

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
hipError_t grouped_fp8_t(const ntc_material* mats, const char* tab, unsigned long long hash,
                         const std::vector<GroupItem>& items,
                         const ntc_query* q, char* out, bool out_f16, hipStream_t s) {
  constexpr PackGeom pg = pack_geom_fp8(C0, C1, B0, B1, HD);
  constexpr int WB = ((int)pg.fwd_end + 15) / 16 * 16;
  const size_t lds = WB + (48 + 2 * HD + 16) * 4 + kMaxLevels * sizeof(LevelBytes) +
                     DecodeLayout<_Float16, C0, C1, HD, B0, B1, true>::SLAB;
  auto kern = decode_fp8_grouped_kernel<C0, C1, C, HD, B0, B1, ACT>;
  static const int per_cu = blocks_per_cu(kern, 256, lds);
  const PeTable pe = pe_table(mats[items[0].mat]);
  return launch_segments(items, (long long)device_cus() * per_cu, hash, [&](const GroupArgs& ga) {
    hipLaunchKernelGGL(kern, dim3((unsigned)ga.blocks), dim3(256), lds, s, tab, pe, ga, q, out, out_f16 ? 1 : 0);
  });
}

template <int C0, int C1, int C, int HD, int B0, int B1, int ACT>
hipError_t mixed_t(const char* tab, unsigned long long hash, int nmat, const PeTable& pe, const ntc_mixed_query* q,
                   long long n, void* out, bool out_f16, hipStream_t s) {
  const size_t lds = 48 * 4 + (size_t)nmat * kMaxLevels * sizeof(LevelBytes);
  auto kern = decode_mixed_kernel<C0, C1, C, HD, B0, B1, ACT>;
  static const int per_cu = blocks_per_cu(kern, 256, 48 * 4 + (size_t)kMixedMax * kMaxLevels * sizeof(LevelBytes));
  const long long tiles = (n + 15) / 16;
  const long long grid = std::min((tiles + 3) / 4, (long long)device_cus() * per_cu);
  hipLaunchKernelGGL(kern, dim3((unsigned)grid), dim3(256), lds, s, tab, pe, hash, nmat, q, n, out, out_f16 ? 1 : 0);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_decode_mixed(const ntc_material* mats, int nmat, const void* table, const ntc_mixed_query* q,
                               long long n, void* out, bool out_f16, hipStream_t s) {
  const char* tab = reinterpret_cast<const char*>(table);
  const unsigned long long hash = group_hash(mats, nmat);
  const ntc_material& m = mats[0];
  const PeTable pe = pe_table(m);
#define NTC_X(a, b, cc, h, x0, x1)                                                                          \
  if (m.c0 == a && m.c1 == b && m.channels == cc && m.hidden == h && m.b0 == x0 && m.b1 == x1)            \
    return m.activation ? mixed_t<a, b, cc, h, x0, x1, 1>(tab, hash, nmat, pe, q, n, out, out_f16, s)     \
                        : mixed_t<a, b, cc, h, x0, x1, 0>(tab, hash, nmat, pe, q, n, out, out_f16, s);
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return hipErrorInvalidValue;
}

// FNV-1a over the kernel views of the materials: what a table was built for.
unsigned long long group_hash(const ntc_material* mats, int nmat) {
  unsigned long long h = 1469598103934665603ULL;
  auto mix = [&](const void* p, size_t bytes) {
    const unsigned char* c = reinterpret_cast<const unsigned char*>(p);
    for (size_t i = 0; i < bytes; ++i) h = (h ^ c[i]) * 1099511628211ULL;
  };
  mix(&nmat, sizeof nmat);
  for (int i = 0; i < nmat; ++i) {
    const DevMat d = dev_mat(mats[i]);
    mix(&d, sizeof d);
  }
  return h;
}

void fill_group_entry(const ntc_material& m, const void* packed, const void* wpack, GroupEntry& e) {
  std::memset(&e, 0, sizeof e);
  e.m = dev_mat(m);
  e.packed = packed;
  e.wpack = wpack;
}

hipError_t launch_decode_grouped(const ntc_material* mats, int nmat, const void* table, int precision,
                                 const ntc_query* q, const int64_t* offsets, void* out, bool out_f16,
                                 hipStream_t s) {
  const char* tab = reinterpret_cast<const char*>(table);
  const unsigned long long hash = group_hash(mats, nmat);
  std::vector<long long> o0(nmat);
  long long o = 0;
  for (int i = 0; i < nmat; ++i) {
    o0[i] = o;
    o += (offsets[i + 1] - offsets[i]) * mats[i].channels;
  }
  std::vector<bool> done(nmat, false);
  std::vector<GroupItem> items;
  // the materials of one launch (shape, activation, positional encoding), in batch order
  auto collect = [&](int c0, int c1, int c, int hd, int b0, int b1, int act, int pe) {
    items.clear();
    for (int i = 0; i < nmat; ++i) {
      const ntc_material& m = mats[i];
      if (done[i] || m.c0 != c0 || m.c1 != c1 || m.channels != c || m.hidden != hd || m.b0 != b0 || m.b1 != b1 ||
          m.activation != act || m.posenc != pe)
        continue;
      done[i] = true;
      const long long n = offsets[i + 1] - offsets[i];
      if (n > 0) items.push_back(GroupItem{i, (long long)offsets[i], n, o0[i]});
    }
    return !items.empty();
  };
  char* ob = reinterpret_cast<char*>(out);
  hipError_t e = hipSuccess;
#define NTC_X(a, b, cc, h, x0, x1)                                                                              \
  for (int cls = 0; cls < 4 && e == hipSuccess; ++cls) {                                                       \
    const int act = cls & 1;                                                                                    \
    if (!collect(a, b, cc, h, x0, x1, act, cls >> 1)) continue;                                                 \
    if (precision == NTC_FP8_E4M3) {                                                                            \
      if constexpr (fp8_layout(a, b, x0, x1, h))                                                                \
        e = act ? grouped_fp8_t<a, b, cc, h, x0, x1, 1>(mats, tab, hash, items, q, ob, out_f16, s)                          \
                : grouped_fp8_t<a, b, cc, h, x0, x1, 0>(mats, tab, hash, items, q, ob, out_f16, s);                         \
      else                                                                                                      \
        e = hipErrorInvalidValue;                                                                               \
    } else if (precision == NTC_F16) {                                                                          \
      e = act ? grouped_t<_Float16, a, b, cc, h, x0, x1, 1>(mats, tab, hash, items, q, ob, out_f16, s)                      \
              : grouped_t<_Float16, a, b, cc, h, x0, x1, 0>(mats, tab, hash, items, q, ob, out_f16, s);                     \
    } else {                                                                                                    \
      e = act ? grouped_t<float, a, b, cc, h, x0, x1, 1>(mats, tab, hash, items, q, ob, out_f16, s)                         \
              : grouped_t<float, a, b, cc, h, x0, x1, 0>(mats, tab, hash, items, q, ob, out_f16, s);                        \
    }                                                                                                           \
  }
  NTC_DECODE_SHAPES(NTC_X)
#undef NTC_X
  return e;
}

}  // namespace ntc
