// Host-only helpers of libtmhip that need no GPU: the LDS block-matvec work
// planner, the azimuthal-order blocks of a dense T and the Wigner 3j symbol
// of the translation coefficients.  Plain
// C++17 (no HIP), so that a CPU build under the address and undefined-
// behaviour sanitizers can exercise them (tests/host_sanitize.cpp).
#pragma once
#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <vector>

namespace tmh {

// ---------------------------------------------------------------- m-blocks
// Blocks of the coefficient index by azimuthal order m, for the boundary
// order n = p lmax(lmax+2) + l(l+1) - 1 + m (p = 0, 1; l = 1..lmax;
// |m| <= l): block b = m + lmax holds the 2(lmax - max(1,|m|) + 1) indices
// with that m in increasing n.  A dense T that is zero between different m
// (a scatterer symmetric about the z axis) is kept as these square blocks,
// `per_site` complex numbers per scatterer.  Sized for lmax <= 6.
constexpr int MB_LM_MAX = 96, MB_BLK_MAX = 13;
struct MbMaps {
  int blk_of[MB_LM_MAX];  // n -> block
  int q_of[MB_LM_MAX];    // n -> row within its block
  int mem[MB_LM_MAX];     // block members, block after block
  int first[MB_BLK_MAX], nm[MB_BLK_MAX], off[MB_BLK_MAX];
  int nblk, per_site;
};

inline void host_mblock_maps(int lmax, MbMaps& mb) {
  mb = MbMaps{};
  const int half = lmax * (lmax + 2), L = 2 * half;
  mb.nblk = 2 * lmax + 1;
  int k = 0, off = 0;
  for (int b = 0; b < mb.nblk; ++b) {
    mb.first[b] = k;
    for (int n = 0; n < L; ++n) {
      const int r = n % half;  // l(l+1) - 1 + m
      int l = 1;
      while ((l + 1) * (l + 1) - 1 <= r) ++l;
      const int m = r - (l * (l + 1) - 1);
      if (m + lmax != b) continue;
      mb.blk_of[n] = b;
      mb.q_of[n] = k - mb.first[b];
      mb.mem[k++] = n;
    }
    mb.nm[b] = k - mb.first[b];
    mb.off[b] = off;
    off += mb.nm[b] * mb.nm[b];
  }
  mb.per_site = off;
}

// Work item of the LDS-staged block matvec: a target tile of a (sub)lattice
// and a range [b0, b1) of its displacement blocks.
struct LdsItem {
  int tile, b0, b1, sub;
};

// ---------------------------------------------------------------- planner
// Work of every displacement block of one tile (MFMA units plus the window
// copy), mirroring the kernel's per-wave clipping: the planner cuts each
// tile's block list into equal-work items.  TW = columns per wave.
inline double tile_block_work(int nx, int ny, int X0, int Y0, bool wide, int TW, int BX, int BY,
                              int win_cost, std::vector<double>& wb) {
  const int GX = TW / 4;
  // displacements relative to each wave's first row and column (as in the
  // kernel): wave w applies (x + wxo, y + wyo) at relative (x, y)
  const int dxlo = X0 - (nx - 1), dxhi = std::min(X0 + TW - 1, nx - 1);
  const int dylo = Y0 - (ny - 1), dyhi = std::min(Y0 + 3, ny - 1);
  const int nbx = (dxhi - dxlo + BX) / BX, nby = (dyhi - dylo + BY) / BY;
  wb.assign((size_t)nbx * nby, 0.0);
  int gyw[4], gxw[4];
  for (int wv = 0; wv < 4; ++wv) {
    gyw[wv] = Y0 + (wide ? 0 : 4 * wv);
    gxw[wv] = X0 + (wide ? TW * wv : 0);
  }
  double total = 0.0;
  for (int b = 0; b < nbx * nby; ++b) {
    const int bx0 = dxlo + (b % nbx) * BX, by0 = dylo + (b / nbx) * BY;
    double w = win_cost;
    for (int wv = 0; wv < 4; ++wv) {
      const int gy0 = gyw[wv], gx = gxw[wv];
      if (gy0 >= ny || gx >= nx) continue;
      const int wxo = gx - X0, wyo = gy0 - Y0;
      const int yb = std::max(by0, dylo);
      const int ye = std::min(by0 + BY - 1, std::min(Y0 + 3, ny - 1 - wyo));
      const int xb = std::max(bx0, dxlo);
      const int xe = std::min(bx0 + BX - 1, std::min(X0 + TW - 1, nx - 1 - wxo));
      if (yb > ye || xb > xe) continue;
      double row = 0.0;
      for (int dx = xb; dx <= xe; ++dx) {
        int groups = 0;
        for (int q = 0; q < GX; ++q) {
          const int gx0 = gx + 4 * q, ad = dx + wxo;  // actual displacement column
          if (gx0 < nx && gx0 + 3 - ad >= 0 && gx0 - ad < nx) ++groups;
        }
        row += 12.0 * groups + 4.0;
      }
      w += row * (ye - yb + 1);
    }
    wb[b] = w;
    total += w;
  }
  return total;
}

// Regular tiles only (the batched solver's subregions).
inline double lds_block_work(int nx, int ny, int TW, int BX, int BY, int win_cost,
                      std::vector<std::vector<double>>& wb) {
  const int tiles_x = (nx + TW - 1) / TW, tiles_y = (ny + 15) / 16;
  wb.assign((size_t)tiles_x * tiles_y, {});
  double total = 0.0;
  for (int t = 0; t < tiles_x * tiles_y; ++t)
    total += tile_block_work(nx, ny, (t % tiles_x) * TW, (t / tiles_x) * 16, false, TW, BX, BY,
                             win_cost, wb[t]);
  return total;
}

// Tiling of one lattice: regular tiles over rows [0, y_wide), wide tiles (4
// rows) over the remaining ny - y_wide < 16 rows.
struct LdsTiling {
  int TW, tiles_x, n_reg, y_wide, tiles_xw, n_wide;
};
inline LdsTiling lds_tiling(int nx, int ny, int TW) {
  LdsTiling tl;
  tl.TW = TW;
  tl.tiles_x = (nx + TW - 1) / TW;
  tl.y_wide = 16 * (ny / 16);
  tl.n_reg = tl.tiles_x * (tl.y_wide / 16);
  tl.tiles_xw = (nx + 4 * TW - 1) / (4 * TW);
  tl.n_wide = ny > tl.y_wide ? tl.tiles_xw * ((ny - tl.y_wide + 3) / 4) : 0;
  return tl;
}

// Cut every tile's blocks into items of about `per` work; appends to items
// and ibeg (ibeg gets one entry per tile, the caller closes the list).
inline void lds_split(const std::vector<std::vector<double>>& wb, double per, int sub,
               std::vector<LdsItem>& items, std::vector<int>& ibeg) {
  for (int t = 0; t < (int)wb.size(); ++t) {
    ibeg.push_back((int)items.size());
    const int nb = (int)wb[t].size();
    double wt = 0.0;
    for (double v : wb[t]) wt += v;
    int nch = std::max(1, std::min(nb, (int)std::llround(wt / per)));
    double acc = 0.0;
    int start = 0, k = 1;
    for (int b = 0; b < nb; ++b) {
      acc += wb[t][b];
      if (k < nch && acc >= k * wt / nch && b < nb - 1) {
        items.push_back(LdsItem{t, start, b + 1, sub});
        start = b + 1;
        ++k;
      }
    }
    items.push_back(LdsItem{t, start, nb, sub});
  }
}

// Items of one lattice: regular tiles first, then wide tiles (tile indices
// continue), so the two launches take contiguous item ranges.
inline void lds_plan(int nx, int ny, const LdsTiling& tl, int BX, int BY, int WBX, int WBY,
                     int win_cost, int target, std::vector<LdsItem>& items, std::vector<int>& ibeg) {
  std::vector<std::vector<double>> wb((size_t)tl.n_reg + tl.n_wide);
  double total = 0.0;
  for (int t = 0; t < tl.n_reg; ++t)
    total += tile_block_work(nx, ny, (t % tl.tiles_x) * tl.TW, (t / tl.tiles_x) * 16, false, tl.TW,
                             BX, BY, win_cost, wb[t]);
  for (int t = 0; t < tl.n_wide; ++t)
    total += tile_block_work(nx, ny, (t % tl.tiles_xw) * 4 * tl.TW, tl.y_wide + (t / tl.tiles_xw) * 4,
                             true, tl.TW, WBX, WBY, win_cost, wb[(size_t)tl.n_reg + t]);
  items.clear();
  ibeg.clear();
  lds_split(wb, total / std::max(1, target), 0, items, ibeg);
  ibeg.push_back((int)items.size());
}

// ---------------------------------------------------------------- Wigner 3j
inline long double lfact(int n) {
  long double r = 1.0L;
  for (int i = 2; i <= n; ++i) r *= (long double)i;
  return r;
}

// Wigner 3j symbol by the Racah formula (all factorials exact in long double
// for the orders used here, j <= 12).
inline double wigner3j(int j1, int j2, int j3, int m1, int m2, int m3) {
  if (m1 + m2 + m3 != 0) return 0.0;
  if (j3 < std::abs(j1 - j2) || j3 > j1 + j2) return 0.0;
  if (std::abs(m1) > j1 || std::abs(m2) > j2 || std::abs(m3) > j3) return 0.0;
  long double tri = lfact(j1 + j2 - j3) * lfact(j1 - j2 + j3) * lfact(-j1 + j2 + j3) /
                    lfact(j1 + j2 + j3 + 1);
  long double pre = std::sqrt(tri * lfact(j1 + m1) * lfact(j1 - m1) * lfact(j2 + m2) *
                              lfact(j2 - m2) * lfact(j3 + m3) * lfact(j3 - m3));
  int kmin = std::max(0, std::max(j2 - j3 - m1, j1 - j3 + m2));
  int kmax = std::min(j1 + j2 - j3, std::min(j1 - m1, j2 + m2));
  long double s = 0.0L;
  for (int k = kmin; k <= kmax; ++k) {
    long double den = lfact(k) * lfact(j1 + j2 - j3 - k) * lfact(j1 - m1 - k) *
                      lfact(j2 + m2 - k) * lfact(j3 - j2 + m1 + k) * lfact(j3 - j1 - m2 + k);
    s += ((k & 1) ? -1.0L : 1.0L) / den;
  }
  int e = j1 - j2 - m3;
  long double sign = ((e % 2) + 2) % 2 ? -1.0L : 1.0L;
  return (double)(sign * pre * s);
}

}  // namespace tmh
