// CPU driver for the host-only code of libtmhip (tm_host.h), built by
// tests/test_host_sanitize.py with the address and undefined-behaviour
// sanitizers: the LDS block-matvec planner and the Wigner 3j symbol.
//
// Planner checks, for lattices of many shapes and both kernel shapes:
//  * the item list of every work target covers each tile's displacement
//    blocks exactly once, in order, and ibeg indexes it;
//  * a replay of the kernel's iteration (tiles, waves with their rows taken
//    relative to the wave, blocks, per-wave clipping, column-group mask)
//    touches every (target, source) pair of the lattice exactly once;
//  * the planner's work per block equals the replay's MFMA count per block.
// m-block checks (lmax 1..6): the blocks partition the coefficient index,
// every member has the block's m, sizes 2(lmax - max(1,|m|) + 1), members in
// increasing order, offsets and rows consistent, 872 entries per scatterer
// at lmax 6.
// 3j checks: closed forms, selection rules and the orthogonality sum.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <vector>

#include "tm_host.h"

using namespace tmh;

static int failures = 0;
#define CHECK(cond, ...)                   \
  do {                                     \
    if (!(cond)) {                         \
      std::printf("FAIL %s:%d ", __FILE__, __LINE__); \
      std::printf(__VA_ARGS__);            \
      std::printf("\n");                   \
      ++failures;                          \
    }                                      \
  } while (0)

// number of blocks of a tile, as the kernel and planner define the grid
// (displacements relative to each wave: TW columns, 4 rows)
static int tile_blocks(int nx, int ny, int X0, int Y0, int TW, int BX, int BY) {
  const int dxlo = X0 - (nx - 1), dxhi = std::min(X0 + TW - 1, nx - 1);
  const int dylo = Y0 - (ny - 1), dyhi = std::min(Y0 + 3, ny - 1);
  return ((dxhi - dxlo + BX) / BX) * ((dyhi - dylo + BY) / BY);
}

// Replay of one (tile, block) of the kernel for one class: every pair
// (target, source) a valid column group touches gets +1 in cover; returns
// the MFMA units (12 per valid group and step) plus 4 per step, the
// planner's cost model.
static double replay_block(int nx, int ny, int X0, int Y0, bool wide, int TW, int BX, int BY, int b,
                           std::vector<int>* cover) {
  const int GX = TW / 4;
  const int dxlo = X0 - (nx - 1), dxhi = std::min(X0 + TW - 1, nx - 1);
  const int dylo = Y0 - (ny - 1);
  const int nbx = (dxhi - dxlo + BX) / BX;
  const int bx0 = dxlo + (b % nbx) * BX, by0 = dylo + (b / nbx) * BY;
  double work = 0.0;
  for (int w = 0; w < 4; ++w) {
    const int wxo = wide ? TW * w : 0, wyo = wide ? 0 : 4 * w;
    const int gy0 = Y0 + wyo, gxw = X0 + wxo;
    if (gy0 >= ny || gxw >= nx) continue;
    const int wdyhi = std::min(Y0 + 3, ny - 1 - wyo);
    const int wdxhi = std::min(X0 + TW - 1, nx - 1 - wxo);
    const int dyb = std::max(by0, dylo), dye = std::min(by0 + BY - 1, wdyhi);
    const int dxb = std::max(bx0, dxlo), dxe = std::min(bx0 + BX - 1, std::min(dxhi, wdxhi));
    for (int y = dyb; y <= dye; ++y)
      for (int x = dxb; x <= dxe; ++x) {
        work += 4.0;
        for (int g = 0; g < GX; ++g) {
          const int gx0 = gxw + 4 * g, ax = x + wxo;  // actual displacement column
          if (!(gx0 < nx && gx0 + 3 - ax >= 0 && gx0 - ax < nx)) continue;
          work += 12.0;
          if (!cover) continue;
          for (int ly = 0; ly < 4; ++ly)
            for (int lx = 0; lx < 4; ++lx) {
              const int tx = gx0 + lx, ty = gy0 + ly;
              const int sx = tx - (x + wxo), sy = ty - (y + wyo);
              if (tx >= nx || ty >= ny || sx < 0 || sx >= nx || sy < 0 || sy >= ny) continue;
              (*cover)[((size_t)ty * nx + tx) * nx * ny + (size_t)sy * nx + sx] += 1;
            }
        }
      }
  }
  return work;
}

static void check_lattice(int nx, int ny, int TW, int BX, int BY, int WBX, int WBY) {
  const LdsTiling tl = lds_tiling(nx, ny, TW);
  const int ntile = tl.n_reg + tl.n_wide;
  const bool pairs = (long long)nx * ny <= 1600;
  std::vector<int> cover(pairs ? (size_t)nx * ny * nx * ny : 0, 0);
  double replay_total = 0.0;
  for (int target : {1, 7, 300, 4096, 100000}) {
    std::vector<LdsItem> items;
    std::vector<int> ibeg;
    lds_plan(nx, ny, tl, BX, BY, WBX, WBY, 64, target, items, ibeg);
    CHECK((int)ibeg.size() == ntile + 1, "ibeg size %zu for %d tiles (%dx%d)", ibeg.size(), ntile, nx, ny);
    if ((int)ibeg.size() != ntile + 1) return;
    CHECK(ibeg[0] == 0 && ibeg[ntile] == (int)items.size(), "ibeg ends (%dx%d)", nx, ny);
    for (int t = 0; t < ntile; ++t) {
      const bool wide = t >= tl.n_reg;
      const int tt = wide ? t - tl.n_reg : t;
      const int X0 = wide ? (tt % tl.tiles_xw) * 4 * TW : (tt % tl.tiles_x) * TW;
      const int Y0 = wide ? tl.y_wide + (tt / tl.tiles_xw) * 4 : (tt / tl.tiles_x) * 16;
      const int bx = wide ? WBX : BX, by = wide ? WBY : BY;
      const int nb = tile_blocks(nx, ny, X0, Y0, TW, bx, by);
      CHECK(ibeg[t] < ibeg[t + 1], "tile %d has no item (%dx%d)", t, nx, ny);
      int next = 0;
      for (int i = ibeg[t]; i < ibeg[t + 1]; ++i) {
        CHECK(items[i].tile == t && items[i].b0 == next && items[i].b1 > items[i].b0,
              "item %d of tile %d: [%d, %d) after %d (%dx%d)", i, t, items[i].b0, items[i].b1, next, nx, ny);
        next = items[i].b1;
      }
      CHECK(next == nb, "tile %d covers %d of %d blocks (%dx%d)", t, next, nb, nx, ny);
      if (target == 1) {
        std::vector<double> wb;
        tile_block_work(nx, ny, X0, Y0, wide, TW, bx, by, 64, wb);
        CHECK((int)wb.size() == nb, "work list size %zu vs %d blocks", wb.size(), nb);
        for (int b = 0; b < nb && b < (int)wb.size(); ++b) {
          const double r = replay_block(nx, ny, X0, Y0, wide, TW, bx, by, b, pairs ? &cover : nullptr);
          CHECK(std::fabs(wb[b] - 64.0 - r) < 1e-9, "block %d of tile %d: planner %g, replay %g (%dx%d)", b,
                t, wb[b] - 64.0, r, nx, ny);
          replay_total += r;
        }
      }
    }
  }
  if (pairs) {
    size_t bad = 0;
    for (size_t i = 0; i < cover.size(); ++i) bad += cover[i] != 1;
    CHECK(bad == 0, "%zu of %zu (target, source) pairs not covered exactly once (%dx%d, TW %d)", bad,
          cover.size(), nx, ny, TW);
  }
  CHECK(replay_total > 0.0, "no work (%dx%d)", nx, ny);
}

static void check_subregions() {
  // the batched solver's regular-tile work lists: every tile row present,
  // partial last rows included
  const int shapes[][2] = {{1, 1}, {12, 9}, {20, 16}, {17, 33}, {40, 30}};
  std::vector<LdsItem> items;
  std::vector<int> ibeg;
  for (int k = 0; k < 5; ++k) {
    const int nx = shapes[k][0], ny = shapes[k][1];
    std::vector<std::vector<double>> wb;
    const double tot = lds_block_work(nx, ny, 16, 16, 8, 64, wb);
    CHECK((int)wb.size() == ((nx + 15) / 16) * ((ny + 15) / 16), "subregion tiles %dx%d", nx, ny);
    CHECK(tot > 0.0, "subregion work %dx%d", nx, ny);
    lds_split(wb, tot / 50.0, k, items, ibeg);
  }
  CHECK(!items.empty() && items.back().sub == 4, "subregion item list");
}

static void check_3j() {
  const double s3 = std::sqrt(3.0);
  CHECK(std::fabs(wigner3j(1, 1, 0, 0, 0, 0) + 1.0 / s3) < 1e-15, "(1 1 0; 0 0 0)");
  CHECK(std::fabs(wigner3j(1, 1, 2, 0, 0, 0) - std::sqrt(2.0 / 15.0)) < 1e-15, "(1 1 2; 0 0 0)");
  CHECK(std::fabs(wigner3j(2, 2, 0, 0, 0, 0) - 1.0 / std::sqrt(5.0)) < 1e-15, "(2 2 0; 0 0 0)");
  CHECK(std::fabs(wigner3j(1, 1, 1, 1, -1, 0) - 1.0 / std::sqrt(6.0)) < 1e-15, "(1 1 1; 1 -1 0)");
  for (int j = 0; j <= 12; ++j)
    for (int m = -j; m <= j; ++m)
      CHECK(std::fabs(wigner3j(j, j, 0, m, -m, 0) - (((j - m) & 1) ? -1.0 : 1.0) / std::sqrt(2.0 * j + 1)) < 1e-14,
            "(j j 0; m -m 0) j=%d m=%d", j, m);
  CHECK(wigner3j(1, 1, 3, 0, 0, 0) == 0.0 && wigner3j(2, 1, 1, 1, 1, 0) == 0.0 && wigner3j(2, 2, 1, 0, 0, 0) == 0.0,
        "selection rules");
  // orthogonality: (2 j3 + 1) sum_{m1, m2} 3j(j3) 3j(j3') = delta
  for (int j1 = 1; j1 <= 6; ++j1)
    for (int j2 = 1; j2 <= 6; ++j2)
      for (int j3 = std::abs(j1 - j2); j3 <= j1 + j2; ++j3)
        for (int j4 = std::abs(j1 - j2); j4 <= j1 + j2; ++j4)
          for (int m3 = -std::min(j3, j4); m3 <= std::min(j3, j4); ++m3) {
            double s = 0.0;
            for (int m1 = -j1; m1 <= j1; ++m1) {
              const int m2 = -m3 - m1;
              if (std::abs(m2) > j2) continue;
              s += wigner3j(j1, j2, j3, m1, m2, m3) * wigner3j(j1, j2, j4, m1, m2, m3);
            }
            s *= 2.0 * j3 + 1.0;
            CHECK(std::fabs(s - (j3 == j4 ? 1.0 : 0.0)) < 1e-12, "orthogonality j=(%d %d %d %d) m3=%d: %g", j1,
                  j2, j3, j4, m3, s);
          }
}

static void check_mblocks() {
  for (int lmax = 1; lmax <= 6; ++lmax) {
    MbMaps mb;
    host_mblock_maps(lmax, mb);
    const int L = 2 * lmax * (lmax + 2);
    std::vector<int> seen(L, 0);
    int off = 0;
    CHECK(mb.nblk == 2 * lmax + 1, "lmax %d nblk %d", lmax, mb.nblk);
    for (int b = 0; b < mb.nblk; ++b) {
      const int m = b - lmax, am = m < 0 ? -m : m;
      const int want = 2 * (lmax - (am > 1 ? am : 1) + 1);
      CHECK(mb.nm[b] == want, "lmax %d m %d size %d want %d", lmax, m, mb.nm[b], want);
      CHECK(mb.off[b] == off, "lmax %d m %d offset", lmax, m);
      off += mb.nm[b] * mb.nm[b];
      for (int q = 0; q < mb.nm[b]; ++q) {
        const int n = mb.mem[mb.first[b] + q];
        CHECK(n >= 0 && n < L, "lmax %d member out of range", lmax);
        if (n < 0 || n >= L) continue;
        ++seen[n];
        // m of n from the (p, l, m) enumeration: p-major, then l, then m = -l..l
        int idx = 0, mn = 99;
        for (int p = 0; p < 2; ++p)
          for (int l = 1; l <= lmax; ++l)
            for (int mm = -l; mm <= l; ++mm, ++idx)
              if (idx == n) mn = mm;
        CHECK(mn == m, "lmax %d n %d has m %d, block m %d", lmax, n, mn, m);
        CHECK(mb.blk_of[n] == b && mb.q_of[n] == q, "lmax %d n %d block/row", lmax, n);
        if (q > 0) CHECK(mb.mem[mb.first[b] + q - 1] < n, "lmax %d block %d not increasing", lmax, b);
      }
    }
    CHECK(mb.per_site == off, "lmax %d per_site", lmax);
    for (int n = 0; n < L; ++n) CHECK(seen[n] == 1, "lmax %d n %d seen %d times", lmax, n, seen[n]);
    if (lmax == 6) CHECK(mb.per_site == 872, "per_site %d at lmax 6", mb.per_site);
  }
}

int main() {
  const int shapes[][2] = {{1, 1}, {3, 2}, {16, 16}, {17, 5}, {5, 17}, {33, 47}, {31, 20}, {64, 20}, {100, 100}};
  for (auto& sh : shapes) {
    check_lattice(sh[0], sh[1], 16, 16, 8, 16, 8);  // complex64 kernel
    check_lattice(sh[0], sh[1], 8, 8, 16, 8, 16);   // FP64 kernel
    check_lattice(sh[0], sh[1], 16, 8, 8, 16, 4);   // other block shapes
  }
  check_subregions();
  check_mblocks();
  check_3j();
  std::printf("%s (%d failures)\n", failures ? "FAILED" : "ok", failures);
  return failures ? 1 : 0;
}
