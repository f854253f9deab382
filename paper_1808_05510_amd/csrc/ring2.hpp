// Rows of the squared graph Laplacian L^2 in the two forms the kernels read
// (host code, no device calls; shared by the library and a host-side test).
// L = K I - N, where N is the self-padded ELL neighbour table of width K
// (nbr[k * n + i], an absent neighbour pointing to i itself): row i of L has
// the diagonal K - #self slots and -1 per present neighbour, and row i of
// L^2 is the sum over the entries (m, a) of row i of L of a times row m.
#pragma once

#include <algorithm>
#include <cstdint>
#include <vector>

namespace cr {

// Ring-2 window form (the fused operator sweep writing L w and L^2 w
// together): per tile of W2_TILE consecutive voxels, the voxels that its rows
// of L^2 read, as at most W2_NI intervals of total length at most W2_MAX; per
// voxel, W2_NE packed entries (window position in bits 0-15, the L^2
// coefficient in bits 16-23 and the L coefficient in bits 24-31, both signed
// 8-bit): entries 0..6 are the voxel and its present neighbours (the support
// of its row of L, padded with the voxel and zero coefficients), entries
// 7..24 the rest of its row of L^2 (padded the same way).  Stencil widths
// K <= 6.
constexpr int W2_TILE = 64, W2_NI = 12, W2_MAX = 1024, W2_GAP = 32, W2_NE = 25, W2_NL = 7;
constexpr int W2_TAB = 2 + 2 * W2_NI;  // count, total, starts, LDS prefixes
// The two-barrier PCG's form: r2idx[e * n + i] (e < R2_NX) the voxels of row
// i of L^2 outside the support of row i of L (padded with i); r2cf[e * n + i]
// the L^2 coefficients, e = 0 the diagonal, 1 + k the neighbour in slot k of
// the ELL table (0 for a self-padded slot), R2_C0 + e that of r2idx entry e.
constexpr int R2_NX = W2_NE - W2_NL, R2_C0 = W2_NL, R2_NC = W2_NE;

struct Ring2Host {
  bool rows = false;     // every row of L^2 fits W2_NE entries, 8-bit coefficients
  bool windows = false;  // and every tile's window fits W2_NI intervals, W2_MAX voxels
  std::vector<int32_t> r2idx;   // R2_NX * n (filled when asked for and rows)
  std::vector<int8_t> r2cf;     // R2_NC * n
  std::vector<int32_t> w2tab;   // ceil(n / W2_TILE) * W2_TAB (filled when windows)
  std::vector<uint32_t> w2ent;  // W2_NE * n
};

inline Ring2Host ring2_tables(int64_t n, int K, const int32_t* nbr, bool want_r2) {
  Ring2Host h;
  if (K > W2_NL - 1 || n <= 0) return h;
  // row i of L as (column, coefficient), the diagonal first
  auto lrow = [&](int64_t i, int32_t* col, int* cf) {
    int m = 1, self = 0;
    col[0] = (int32_t)i;
    for (int k = 0; k < K; ++k) {
      const int32_t j = nbr[(size_t)k * n + i];
      if (j == (int32_t)i) {
        ++self;
      } else {
        col[m] = j;
        cf[m] = -1;
        ++m;
      }
    }
    cf[0] = K - self;
    return m;
  };
  // every voxel's entries as (voxel, c2, c1): 0..W2_NL-1 the support of its
  // row of L (with c1), padded with the voxel itself; the rest of its row of
  // L^2 after them, padded the same way
  std::vector<int32_t> ecol((size_t)W2_NE * n);
  std::vector<int8_t> ec2((size_t)W2_NE * n), ec1((size_t)W2_NE * n);
  int32_t scol[W2_NE];
  int sc2[W2_NE], sc1[W2_NE];
  int32_t ci[W2_NL], cm[W2_NL];
  int fi[W2_NL], fm[W2_NL];
  for (int64_t i = 0; i < n; ++i) {
    const int mi = lrow(i, ci, fi);
    int ne = W2_NL;
    for (int a = 0; a < W2_NL; ++a) {
      scol[a] = a < mi ? ci[a] : (int32_t)i;
      sc1[a] = a < mi ? fi[a] : 0;
      sc2[a] = 0;
    }
    for (int a = 0; a < mi; ++a) {
      const int mm = lrow(ci[a], cm, fm);
      for (int b = 0; b < mm; ++b) {
        const int32_t j = cm[b];
        int q = -1;
        for (int e = 0; e < ne && q < 0; ++e)
          if (scol[e] == j && (e < mi || e >= W2_NL)) q = e;
        if (q < 0) {
          if (ne == W2_NE) return h;  // row of L^2 too wide: no tables
          q = ne++;
          scol[q] = j;
          sc1[q] = 0;
          sc2[q] = 0;
        }
        sc2[q] += fi[a] * fm[b];
      }
    }
    for (int e = ne; e < W2_NE; ++e) {
      scol[e] = (int32_t)i;
      sc1[e] = 0;
      sc2[e] = 0;
    }
    for (int e = 0; e < W2_NE; ++e) {
      if (sc2[e] < -128 || sc2[e] > 127) return h;
      ecol[(size_t)i * W2_NE + e] = scol[e];
      ec2[(size_t)i * W2_NE + e] = (int8_t)sc2[e];
      ec1[(size_t)i * W2_NE + e] = (int8_t)sc1[e];
    }
  }
  h.rows = true;
  if (want_r2) {
    h.r2idx.assign((size_t)R2_NX * n, 0);
    h.r2cf.assign((size_t)R2_NC * n, 0);
    for (int64_t i = 0; i < n; ++i) {
      const size_t o = (size_t)i * W2_NE;
      h.r2cf[(size_t)i] = ec2[o];
      for (int k = 0; k < K; ++k) {
        const int32_t j = nbr[(size_t)k * n + i];
        int8_t c = 0;
        if (j != (int32_t)i)
          for (int e = 1; e < W2_NL; ++e)
            if (ecol[o + e] == j && ec1[o + e] != 0) c = ec2[o + e];
        h.r2cf[(size_t)(1 + k) * n + i] = c;
      }
      for (int e = 0; e < R2_NX; ++e) {
        h.r2idx[(size_t)e * n + i] = ecol[o + W2_NL + e];
        h.r2cf[(size_t)(R2_C0 + e) * n + i] = ec2[o + W2_NL + e];
      }
    }
  }
  // window tables of the fused operator sweep
  auto pack = [](int pos, int c2, int c1) {
    return (uint32_t)pos | ((uint32_t)(uint8_t)(int8_t)c2 << 16) |
           ((uint32_t)(uint8_t)(int8_t)c1 << 24);
  };
  const int64_t nt2 = (n + W2_TILE - 1) / W2_TILE;
  std::vector<uint32_t> ent((size_t)W2_NE * n);
  std::vector<int32_t> tab((size_t)nt2 * W2_TAB, 0);
  std::vector<int32_t> idx;
  for (int64_t t = 0; t < nt2; ++t) {
    const int64_t t0 = t * W2_TILE, t1 = std::min(n, t0 + W2_TILE);
    idx.assign(ecol.begin() + (size_t)t0 * W2_NE, ecol.begin() + (size_t)t1 * W2_NE);
    std::sort(idx.begin(), idx.end());
    idx.erase(std::unique(idx.begin(), idx.end()), idx.end());
    int32_t* it = tab.data() + t * W2_TAB;
    int nint = 0, tot = 0;
    size_t a = 0;
    while (a < idx.size()) {
      size_t b = a;
      while (b + 1 < idx.size() && idx[b + 1] - idx[b] <= W2_GAP) ++b;
      if (nint == W2_NI) return h;
      it[2 + nint] = idx[a];
      it[2 + W2_NI + nint] = tot;
      tot += idx[b] - idx[a] + 1;
      ++nint;
      a = b + 1;
    }
    if (tot > W2_MAX) return h;
    it[0] = nint;
    it[1] = tot;
    auto pos = [&](int32_t j) {
      int q = 0;
      while (q + 1 < nint && it[2 + q + 1] <= j) ++q;
      return it[2 + W2_NI + q] + (j - it[2 + q]);
    };
    for (int64_t i = t0; i < t1; ++i) {
      const size_t o = (size_t)i * W2_NE;
      for (int e = 0; e < W2_NE; ++e)
        ent[(size_t)e * n + i] = pack(pos(ecol[o + e]), ec2[o + e], ec1[o + e]);
    }
  }
  h.windows = true;
  h.w2tab.swap(tab);
  h.w2ent.swap(ent);
  return h;
}

}  // namespace cr
