// Block matvec with the source vectors staged in LDS.
//
// Same product as tm_matvec.hip (z_t = sum_{s != t} M(t - s) x_s over the
// lattice, one S x S complex block per displacement and z-mirror class,
// App. I.C / App. I.D), reorganised like a 2-D convolution: a workgroup owns
// a target tile of (4*GX) x 16 sites and walks its displacement range in
// blocks of BX x BY displacements.  For each block the (4*GX + BX - 1) x
// (16 + BY - 1) window of source sites is copied once from HBM/L2 into LDS
// (zeros outside the lattice), and every displacement of the block then reads
// its B operands from LDS: no per-lane bounds tests, no re-fetch through the
// vector-memory path.  The A operand (the translation block) streams from the
// table in global memory; both operands of the next displacement are fetched
// while the current one's MFMAs run.
//
// Slot groups: S = 16 NG slots per class.  A workgroup computes one group gg of
// 16 target slots and loops over the NG source groups hh inside each
// displacement block (a window per (block, hh)); its accumulators add every
// hh, so its partial sums are final for (item, rhs, class, gg).  NG = 1 for
// lmax <= 3.
//
// K ordering: the 16 input slots of a group are consumed as four MFMA K-steps; lane group
// kq = lane/16 at step s supplies slot sigma(kq, s).  FP32: sigma = 2kq+s for
// s < 2 and 8+2kq+s-2 otherwise, so each lane reads two 16-byte chunks (two
// complex64 slots each); FP64: sigma = 4s+kq, four 16-byte chunks (one
// complex128 each).  A and B use the same sigma, so the product is unchanged.
//
// LDS layout: window site (wx, wy) holds its 16 slots as 16-byte chunks;
// logical chunk h is stored at physical chunk h ^ g(wx, wy), with g chosen so
// that the 16 sites of a 4x4 group land in distinct bank groups
// (conflict-free 128-bit reads for every lane group).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "tm_internal.h"

namespace tmh {

typedef float lf32x4 __attribute__((ext_vector_type(4)));
typedef double lf64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct LdsT;
template <>
struct LdsT<float> {
  using acc_t = lf32x4;
  static constexpr int CH = 8;  // 16-byte chunks per site (16 complex64)
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int kq, int v) { return 4 * kq + v; }
  // window sites are 128 B: bank half = site parity (window width odd) and
  // g distinguishes the 8 sites of equal parity in a 4x4 patch
  __device__ static inline int swz(int h, int wx, int wy) {
    return h ^ (((wx >> 1) & 1) | ((wy & 3) << 1));
  }
};
template <>
struct LdsT<double> {
  using acc_t = lf64x4;
  static constexpr int CH = 16;  // 16 complex128
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int kq, int v) { return 4 * v + kq; }
  __device__ static inline int swz(int h, int wx, int wy) { return h ^ ((wx & 3) | ((wy & 3) << 2)); }
};

struct LdsArgs {
  const void* table;  // [D][2][S][S]
  const void* x;      // [R][2][N][S] (or packed per subregion)
  void* partial;      // [item][R*2*NG][tile sites][16]
  const LdsItem* items;
  int nx, ny, tnx, tny;
  int tiles_x, R;
  long long n_sites;
  // batched subregions (null for one lattice): per-subregion lattice and the
  // offset of its [R][2][N_k][16] block in the packed vector; a system
  // (subregion, rhs) whose flag is 0 is skipped; a nonzero *done skips all
  const SubParams* subs;
  const int* active;
  const int* done;
  // wide-tile launch: rows at and beyond y_base are tiled 4 rows high; item
  // tile indices start at tile_base; partial slots at item_base
  int y_base, tile_base, item_base;
  int S, NG;  // slots per class and its groups of 16
};

// A operand of one displacement (a 16 x 16 sub-block, rows S apart): 4 (re,
// im) pairs in sigma order.
__device__ inline void load_a(const c64* __restrict__ blk, int S, int jt, int kq, float* ar, float* ai) {
  const float4 p = *reinterpret_cast<const float4*>(blk + jt * S + 2 * kq);
  const float4 q = *reinterpret_cast<const float4*>(blk + jt * S + 8 + 2 * kq);
  ar[0] = p.x; ai[0] = p.y; ar[1] = p.z; ai[1] = p.w;
  ar[2] = q.x; ai[2] = q.y; ar[3] = q.z; ai[3] = q.w;
}
__device__ inline void load_a(const c128* __restrict__ blk, int S, int jt, int kq, double* ar, double* ai) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 p = *reinterpret_cast<const double2*>(blk + jt * S + 4 * s + kq);
    ar[s] = p.x;
    ai[s] = p.y;
  }
}

// B operand of one source site from LDS (chunk base of the site given).
__device__ inline void read_b(const float4* __restrict__ win, int base, int wx, int wy, int kq,
                              float* br, float* bi) {
  const float4 p = win[base + LdsT<float>::swz(kq, wx, wy)];
  const float4 q = win[base + LdsT<float>::swz(4 + kq, wx, wy)];
  br[0] = p.x; bi[0] = p.y; br[1] = p.z; bi[1] = p.w;
  br[2] = q.x; bi[2] = q.y; br[3] = q.z; bi[3] = q.w;
}
__device__ inline void read_b(const float4* __restrict__ win, int base, int wx, int wy, int kq,
                              double* br, double* bi) {
  const double2* w2 = reinterpret_cast<const double2*>(win);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 p = w2[base + LdsT<double>::swz(4 * s + kq, wx, wy)];
    br[s] = p.x;
    bi[s] = p.y;
  }
}

// Tile geometry.  Regular: a (4 GX) x 16 tile, wave w owns rows 4w..4w+3 and
// all GX column groups.  Wide (for the last rows of a lattice whose height
// is not a multiple of 16): a (16 GX) x 4 tile, wave w owns columns
// 4 GX w .. 4 GX w + 4 GX - 1 of the same 4 rows, so all four waves work.
template <typename T, int GX, int BX, int BY, bool WIDE = false>
struct LdsCfg {
  static constexpr int TW = 4 * GX;                // columns per wave
  static constexpr int TWT = WIDE ? 4 * TW : TW;   // tile width in sites
  static constexpr int THT = WIDE ? 4 : 16;        // tile height in sites
  // every wave reads the same 4 x TW source sites per displacement (wave w
  // of a regular tile takes its displacements shifted by 4w rows, of a wide
  // tile by TW w columns), so a window is (TW - 1 + BX) x (4 - 1 + BY) for
  // both tile shapes
  static constexpr int WX = TW - 1 + BX, WY = 4 - 1 + BY;
  static constexpr int CH = LdsT<T>::CH;
  // FP32 regular tiles use a padded layout instead of the XOR swizzle, so
  // that the address of a lane's B operand is affine in the displacement (one
  // add per step): a site takes SS = 9 chunks (8 of data) and a window row RP
  // chunks with RP = 4 (mod 16).  The reads of a 4x4 patch then cost some
  // LDS bank conflicts (about 4 cycles per read on gfx950); a conflict-free
  // padding (10 chunks per site) needs 8x6 displacement blocks to fit two
  // workgroups per CU and measured slower, the extra windows costing more
  // than the conflicts.
  static constexpr bool PAD = std::is_same<T, float>::value;
  static constexpr int SS = PAD ? CH + 1 : CH;
  static constexpr int RP = PAD ? ((WX * SS + 11) / 16) * 16 + 4 : WX * CH;
  static constexpr int CHUNKS = WY * RP;
  static constexpr size_t BYTES = (size_t)CHUNKS * 16;
};

// Complex products by three real MFMA products (T1 = Mr Xr, T2 = Mi Xi,
// T3 = (Mr + Mi)(Xr + Xi); Yr = T1 - T2, Yi = T3 - T1 - T2).
template <typename T, int GX, int BX, int BY, int PF, bool WIDE>
__global__ __launch_bounds__(256, 2) void block_matvec_lds_kernel(LdsArgs a) {
  using L = LdsT<T>;
  using Cfg = LdsCfg<T, GX, BX, BY, WIDE>;
  using acc_t = typename L::acc_t;
  using C = cplx<T>;
  constexpr int TW = Cfg::TW, TWT = Cfg::TWT, THT = Cfg::THT, WX = Cfg::WX, WY = Cfg::WY,
                CH = Cfg::CH;
  __shared__ float4 win[Cfg::CHUNKS];
  const int lane = threadIdx.x & 63;
  // wave-uniform by construction; readfirstlane lets the compiler keep the
  // per-wave bounds below in scalar registers
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int jt = lane & 15;
  const int kq = lane >> 4;
  const int lx = jt & 3, ly = jt >> 2;
  if (a.done && *a.done) return;
  const int item = a.item_base + blockIdx.x;
  const LdsItem it = a.items[item];
  const int rc = blockIdx.y;  // ((r * 2 + c) * NG + gg)
  const int NG = a.NG, S = a.S;
  const int gg = rc % NG;
  const int r = (rc / NG) >> 1, c = (rc / NG) & 1;
  int nx = a.nx, ny = a.ny, tiles_x = a.tiles_x;
  size_t N = (size_t)a.n_sites, voff = 0;
  if (a.subs) {
    const SubParams sp = a.subs[it.sub];
    if (a.active && !a.active[it.sub * a.R + r]) return;
    nx = sp.nx;
    ny = sp.ny;
    tiles_x = sp.tiles_x;
    N = (size_t)sp.nx * sp.ny;
    voff = (size_t)sp.vec_off;
  }
  const int tl = it.tile - a.tile_base;
  const int X0 = (tl % tiles_x) * TWT;
  const int Y0 = a.y_base + (tl / tiles_x) * THT;
  const int wxo = WIDE ? TW * wave : 0;  // this wave's column and row offsets in the tile
  const int wyo = WIDE ? 0 : 4 * wave;
  const int gy0 = Y0 + wyo;
  const int gxw = X0 + wxo;
  const int ty = gy0 + ly;
  const C* __restrict__ xin0 =
      reinterpret_cast<const C*>(a.x) + voff + ((size_t)r * NCLASS + c) * N * S;
  const C* __restrict__ tab = reinterpret_cast<const C*>(a.table);
  const int wxt = 2 * a.tnx - 1;
  // The tile's displacement range and its block grid.  Displacements are
  // counted relative to each wave: at relative (x, y), the wave whose sites
  // start at (gxw, gy0) applies the displacement (x + wxo, y + wyo), so that
  // all waves read source columns X0 - x .. X0 + TW - 1 - x and rows
  // Y0 - y .. Y0 + 3 - y of one shared window and have the same number of
  // steps (waves cut by the lattice edge excepted).
  const int dxlo = X0 - (nx - 1), dxhi = min(X0 + TW - 1, nx - 1);
  const int dylo = Y0 - (ny - 1), dyhi = min(Y0 + 3, ny - 1);
  const int nbx = (dxhi - dxlo + BX) / BX;
  // this wave's valid displacements (its rows and columns must reach a
  // source), relative
  const int wdylo = dylo, wdyhi = min(Y0 + 3, ny - 1 - wyo);
  const int wdxlo = dxlo, wdxhi = min(X0 + TW - 1, nx - 1 - wxo);
  const bool wave_live = gy0 < ny && gxw < nx;
  // padded layout: chunk of this lane's B operand (group 0, K-chunk kq) at the
  // block's first displacement (bx0, by0)
  const int lane_b0 = (ly + BY - 1) * Cfg::RP + (lx + BX - 1) * Cfg::SS + kq;

  acc_t t1[GX], t2[GX], t3[GX];
#pragma unroll
  for (int g = 0; g < GX; ++g) {
    t1[g] = acc_t{0, 0, 0, 0};
    t2[g] = acc_t{0, 0, 0, 0};
    t3[g] = acc_t{0, 0, 0, 0};
  }

  for (int bh = it.b0 * NG; bh < it.b1 * NG; ++bh) {
    const int b = bh / NG, hh = bh % NG;
    const C* __restrict__ xin = xin0 + SLOTS * hh;
    const int boff = (SLOTS * gg) * S + SLOTS * hh;  // sub-block (gg, hh) of a table block
    const int bx0 = dxlo + (b % nbx) * BX;
    const int by0 = dylo + (b / nbx) * BY;
    // window origin: source site of target (X0, Y0) at displacement (bx0+BX-1, by0+BY-1)
    const int wx0 = X0 - (bx0 + BX - 1), wy0 = Y0 - (by0 + BY - 1);
    const int dyb = max(by0, max(dylo, wdylo)), dye = min(by0 + BY - 1, min(dyhi, wdyhi));
    const int dxb = max(bx0, max(dxlo, wdxlo)), dxe = min(bx0 + BX - 1, min(dxhi, wdxhi));
    const bool has_work = wave_live && dyb <= dye && dxb <= dxe;  // wave-uniform
    const int ndx = dxe - dxb + 1;
    const int nq = (dye - dyb + 1) * ndx;
    // Operand pipeline, unrolled by U = PF + 1 so that every stage owns its
    // registers (no copies between stages, and each wait covers exactly the
    // load that stage consumes): the translation block of step q is fetched
    // PF steps ahead (table rows mostly miss L2, so the latency is that of
    // MALL/HBM) into set q % U, the B operands of all groups one step ahead
    // from LDS into set q % U.  Positions advance row-major over the block's
    // valid [dxb, dxe] x [dyb, dye].
    constexpr int U = PF + 1;
    T ar[U][4], ai[U][4];
    T br[U][GX][4], bi[U][GX][4];
    // (selects, not branches: positions are wave-uniform scalars)
    auto advance = [&](int& x, int& y) {
      const int wrap = x == dxe;
      x = wrap ? dxb : x + 1;
      y += wrap;
    };
    auto table_block = [&](int x, int y) {
      return tab + (((size_t)(y + wyo + a.tny - 1) * wxt + (x + wxo + a.tnx - 1)) * NCLASS + c) * (size_t)(S * S) +
             boff;
    };
    auto read_all_b = [&](int x, int y, T (*r_)[4], T (*i_)[4]) {
      if constexpr (Cfg::PAD) {
        // chunk of (group 0, K-chunk kq): lane part minus a wave-uniform part
        const int off = lane_b0 - ((x - bx0) * Cfg::SS + (y - by0) * Cfg::RP);
#pragma unroll
        for (int g = 0; g < GX; ++g) {
          const float4 p = win[off + 4 * Cfg::SS * g];
          const float4 q = win[off + 4 * Cfg::SS * g + 4];
          r_[g][0] = p.x; i_[g][0] = p.y; r_[g][1] = p.z; i_[g][1] = p.w;
          r_[g][2] = q.x; i_[g][2] = q.y; r_[g][3] = q.z; i_[g][3] = q.w;
        }
      } else {
        const int wy = ly - (y - by0) + BY - 1;
#pragma unroll
        for (int g = 0; g < GX; ++g) {
          const int wx = 4 * g + lx - (x - bx0) + BX - 1;
          read_b(win, (wy * WX + wx) * CH, wx, wy, kq, r_[g], i_[g]);
        }
      }
    };
    // The fetch positions stop at the block's last displacement, so fetches
    // past the end re-read valid data: every fetch is unconditional and the
    // compiler waits for exactly the operands a step consumes.
    auto advance_fetch = [&](int& x, int& y) {
      const int wrap = x == dxe, stop = wrap & (y == dye);
      x = stop ? x : (wrap ? dxb : x + 1);
      y += wrap & !stop;
    };
    int adx = dxb, ady = dyb, bdx = dxb, bdy = dyb, cdx = dxb, cdy = dyb;
    // the first translation blocks are fetched before the window fill, so
    // that their latency overlaps the fill's
    if (has_work) {
#pragma unroll
      for (int p = 0; p < PF; ++p) {
        load_a(table_block(adx, ady), S, jt, kq, ar[p], ai[p]);
        advance_fetch(adx, ady);
      }
    }
    __syncthreads();  // every wave is done with the previous window
    // window fill in batches of FB chunks per thread: all loads of a batch
    // are in flight together, then all its LDS stores.  Thread t fills chunk
    // h = t % CH of sites t / CH, t / CH + 256 / CH, ... (256 % CH == 0).
    {
      constexpr int SST = 256 / CH, DWX = SST % WX, DWY = SST / WX;
      constexpr int PER = (WX * WY * CH + 255) / 256, FB = (PER + 1) / 2;
      const int h = threadIdx.x % CH;
      int wx = (threadIdx.x / CH) % WX, wy = (threadIdx.x / CH) / WX;
#pragma unroll 1
      for (int q0 = 0; q0 < PER; q0 += FB) {
        float4 v[FB];
        int dst[FB];
#pragma unroll
        for (int j = 0; j < FB; ++j) {
          const int gx = wx0 + wx, gy = wy0 + wy;
          const int chunk = Cfg::PAD ? wy * Cfg::RP + wx * Cfg::SS + h : (wy * WX + wx) * CH + L::swz(h, wx, wy);
          dst[j] = (q0 + j < PER && wy < WY) ? chunk : -1;
          // sources outside the lattice read the (valid) first chunk and are
          // replaced by zeros: no branch around the load
          const bool in = dst[j] >= 0 && (unsigned)gx < (unsigned)nx && (unsigned)gy < (unsigned)ny;
          const size_t site_off = in ? (size_t)gy * nx + gx : 0;
          const float4 t = *reinterpret_cast<const float4*>(xin + site_off * S + h * (SLOTS / CH));
          v[j] = in ? t : make_float4(0.f, 0.f, 0.f, 0.f);
          wx += DWX;
          wy += DWY;
          if (wx >= WX) {
            wx -= WX;
            ++wy;
          }
        }
#pragma unroll
        for (int j = 0; j < FB; ++j)
          if (dst[j] >= 0) win[dst[j]] = v[j];
      }
    }
    __syncthreads();
    if (!has_work) continue;
    read_all_b(bdx, bdy, br[0], bi[0]);
    advance_fetch(bdx, bdy);
    // step q of the block, with q % U == K known at compile time
    auto step = [&](auto kc, int q) {
      constexpr int K = decltype(kc)::value;
      load_a(table_block(adx, ady), S, jt, kq, ar[(K + PF) % U], ai[(K + PF) % U]);
      advance_fetch(adx, ady);
      read_all_b(bdx, bdy, br[(K + 1) % U], bi[(K + 1) % U]);
      advance_fetch(bdx, bdy);
      T ms[4];
#pragma unroll
      for (int s = 0; s < 4; ++s) ms[s] = ar[K][s] + ai[K][s];
      auto group = [&](int g) {
        T xs[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) xs[s] = br[K][g][s] + bi[K][g][s];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          t1[g] = L::mma(ar[K][s], br[K][g][s], t1[g]);
          t2[g] = L::mma(ai[K][s], bi[K][g][s], t2[g]);
          t3[g] = L::mma(ms[s], xs[s], t3[g]);
        }
      };
      // group g of the wave has sources at this displacement iff its columns
      // are in the lattice and gx0 - nx < cdx <= gx0 + 3: a wave-uniform bit
      // mask, kept in a scalar register
      // (sign bits of the three differences, integer ops only)
      int gmask = 0;
#pragma unroll
      for (int g = 0; g < GX; ++g) {
        // target columns gx0..gx0+3; the actual displacement is cdx + wxo
        const int gx0 = gxw + 4 * g, gxr = X0 + 4 * g;
        gmask |= (((cdx - gxr - 4) & (gxr - cdx - nx) & (gx0 - nx)) >> 31) & (1 << g);
      }
#pragma unroll
      for (int g = 0; g < GX; ++g)
        if (gmask & (1 << g)) group(g);
      advance(cdx, cdy);
    };
    using I0 = std::integral_constant<int, 0>;
    using I1 = std::integral_constant<int, 1>;
    using I2 = std::integral_constant<int, 2>;
    using I3 = std::integral_constant<int, 3>;
    int q = 0;
    for (; q + U <= nq; q += U) {
      step(I0{}, q);
      step(I1{}, q + 1);
      if constexpr (U > 2) step(I2{}, q + 2);
      if constexpr (U > 3) step(I3{}, q + 3);
    }
    // tail: fewer than U steps, same register sets
    if (q < nq) step(I0{}, q);
    if constexpr (U > 2) {
      if (q + 1 < nq) step(I1{}, q + 1);
    }
    if constexpr (U > 3) {
      if (q + 2 < nq) step(I2{}, q + 2);
    }
  }
  // this item's partial sums for every valid target of the tile
  C* out = reinterpret_cast<C*>(a.partial) + ((size_t)item * (2 * a.R * NG) + rc) * (TWT * THT * SLOTS);
  if (ty < ny) {
#pragma unroll
    for (int g = 0; g < GX; ++g) {
      const int tx = gxw + 4 * g + lx;
      if (tx >= nx) continue;
      C* o = out + (size_t)((ty - Y0) * TWT + (tx - X0)) * SLOTS;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T yr = t1[g][v] - t2[g][v];
        const T yi = t3[g][v] - t1[g][v] - t2[g][v];
        o[L::out_row(kq, v)] = C{yr, yi};
      }
    }
  }
}

// y = x - t * z (Forward) etc., z = sum of the partials of the items covering
// the site's tile, added in item order.
template <typename T>
__global__ void lds_combine_kernel(const cplx<T>* __restrict__ partial, const int* __restrict__ ibeg,
                                   int R, int nx, LdsTiling tl, long long N,
                                   const c128* __restrict__ x, const c128* __restrict__ t,
                                   c128* __restrict__ y, long long vec, long long total, int mode,
                                   int S, int NG, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int sl = (int)(idx % S);
  const long long site = (idx / S) % N;
  // partial-sum row: ((r * 2 + c) * NG + slot group), slot within the group
  const int rc = (int)(idx / (S * N)) * NG + sl / SLOTS;
  const int slot = sl % SLOTS;
  const int sx = (int)(site % nx), sy = (int)(site / nx);
  const int TW = tl.TW;
  int tile, ls;
  if (sy < tl.y_wide) {
    tile = (sy >> 4) * tl.tiles_x + sx / TW;
    ls = (sy & 15) * TW + (sx % TW);
  } else {
    const int wy = sy - tl.y_wide;
    tile = tl.n_reg + (wy >> 2) * tl.tiles_xw + sx / (4 * TW);
    ls = (wy & 3) * (4 * TW) + (sx % (4 * TW));
  }
  // the tile's items in a fixed order, eight loads in flight and two
  // accumulator pairs (deterministic)
  const size_t stride = (size_t)(2 * R * NG) * (TW * 16) * SLOTS;
  const cplx<T>* pp = partial + ((size_t)rc * (TW * 16) + ls) * SLOTS + slot;
  const int i1 = ibeg[tile + 1];
  double sr0 = 0.0, si0 = 0.0, sr1 = 0.0, si1 = 0.0;
  int i = ibeg[tile];
  for (; i + 8 <= i1; i += 8) {
    cplx<T> v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) v[u] = pp[(size_t)(i + u) * stride];
#pragma unroll
    for (int u = 0; u < 8; u += 2) {
      sr0 += (double)v[u].re;
      si0 += (double)v[u].im;
      sr1 += (double)v[u + 1].re;
      si1 += (double)v[u + 1].im;
    }
  }
  for (; i < i1; ++i) {
    const cplx<T> v = pp[(size_t)i * stride];
    sr0 += (double)v.re;
    si0 += (double)v.im;
  }
  const double sr = sr0 + sr1, si = si0 + si1;
  c128 o;
  if (mode == (int)Op::Forward) {
    const c128 tv = t[idx % vec];
    const c128 xv = x[idx];
    o.re = xv.re - (tv.re * sr - tv.im * si);
    o.im = xv.im - (tv.re * si + tv.im * sr);
  } else if (mode == (int)Op::Adjoint) {
    const c128 xv = x[idx];
    o.re = xv.re - sr;
    o.im = xv.im - si;
  } else {
    o.re = sr;
    o.im = si;
  }
  y[idx] = o;
}

// Configurations: FP32 16x16 tiles (and 64x4 wide tiles) with 16x8
// displacement blocks in the padded layout (51 KB of LDS: three workgroups
// per CU at prefetch depth 1); FP64 8x16 tiles (and 32x4 wide tiles) with
// 8x16 blocks (73 KB: two per CU).
#ifndef TM_LDS_F32_BX
#define TM_LDS_F32_BX 16
#define TM_LDS_F32_BY 8
#endif
#ifndef TM_LDS_F32_GX
#define TM_LDS_F32_GX 4
#endif
template <typename T>
struct LdsChoice;
template <>
struct LdsChoice<float> {
  static constexpr int GX = TM_LDS_F32_GX, BX = TM_LDS_F32_BX, BY = TM_LDS_F32_BY, WBX = BX, WBY = BY;
};
template <>
struct LdsChoice<double> {
  static constexpr int GX = 2, BX = 8, BY = 16, WBX = BX, WBY = BY;
};
static_assert(LdsCfg<float, LdsChoice<float>::GX, LdsChoice<float>::BX, LdsChoice<float>::BY,
                     false>::BYTES <= 80 * 1024,
              "two FP32 workgroups per CU");
static_assert(LdsCfg<double, 2, 8, 16, false>::BYTES <= 80 * 1024, "two FP64 workgroups per CU");

template <typename T, int PF, bool WIDE>
static void lds_launch_pf(hipStream_t st, int nitems, int R, const LdsArgs& a) {
  using Ch = LdsChoice<T>;
  constexpr int BX = WIDE ? Ch::WBX : Ch::BX, BY = WIDE ? Ch::WBY : Ch::BY;
  hipLaunchKernelGGL((block_matvec_lds_kernel<T, Ch::GX, BX, BY, PF, WIDE>),
                     dim3(nitems, 2 * R * a.NG), dim3(256), 0, st, a);
}
// FP64 stages are twice as wide: depth 3 does not fit two waves' registers,
// so FP64 runs depth 2 for variant 10
template <typename T, bool WIDE = false>
static void lds_launch_any(hipStream_t st, int pf, int nitems, int R, const LdsArgs& a) {
  if (nitems <= 0) return;
  if (pf <= 1) {
    lds_launch_pf<T, 1, WIDE>(st, nitems, R, a);
  } else if constexpr (std::is_same<T, double>::value) {
    lds_launch_pf<T, 2, WIDE>(st, nitems, R, a);
  } else {
    if (pf == 2) lds_launch_pf<T, 2, WIDE>(st, nitems, R, a);
    else lds_launch_pf<T, 3, WIDE>(st, nitems, R, a);
  }
}

template <typename T>
int lds_apply(tm_ctx* c, int which, int R, const void* table, const void* xin, const c128* x,
              c128* y, int op, int items_target, hipEvent_t e0, hipEvent_t e1, int pf) {
  using Ch = LdsChoice<T>;
  using Cfg = LdsCfg<T, Ch::GX, Ch::BX, Ch::BY>;
  const Geometry& g = c->g;
  const int TW = Cfg::TW;
  const LdsTiling tl = lds_tiling(g.nx, g.ny, TW);
  const long long vec = g.vec_len(), total = vec * R;
  int rc;
  if (c->plan_kind[which] != 2 || c->plan_R[which] != R || c->plan_target[which] != items_target) {
    std::vector<LdsItem> items;
    std::vector<int> ibeg;
    lds_plan(g.nx, g.ny, tl, Ch::BX, Ch::BY, Ch::WBX, Ch::WBY, 64, items_target, items, ibeg);
    c->plan_nreg[which] = ibeg[tl.n_reg];
    if ((rc = ensure(c, c->plan_items[which], items.size() * sizeof(LdsItem))) != TM_OK) return rc;
    if ((rc = ensure(c, c->plan_ibeg[which], ibeg.size() * sizeof(int))) != TM_OK) return rc;
    // launches of the previous plan may still read it, on the context stream
    // or the side stream joined into it (the upload is not ordered with a
    // non-blocking stream)
    TM_HIP(c, hipStreamSynchronize(c->stream));
    TM_HIP(c, hipMemcpy(c->plan_items[which].p, items.data(), items.size() * sizeof(LdsItem),
                        hipMemcpyHostToDevice));
    TM_HIP(c, hipMemcpy(c->plan_ibeg[which].p, ibeg.data(), ibeg.size() * sizeof(int),
                        hipMemcpyHostToDevice));
    c->plan_kind[which] = 2;
    c->plan_R[which] = R;
    c->plan_target[which] = items_target;
    c->plan_nitems[which] = (int)items.size();
  }
  const int nitems = c->plan_nitems[which];
  if ((rc = ensure(c, c->partial,
                   (size_t)nitems * 2 * R * g.NG * TW * 16 * SLOTS * sizeof(cplx<T>))) != TM_OK)
    return rc;
  LdsArgs a;
  a.table = table;
  a.x = xin;
  a.partial = c->partial.p;
  a.items = (const LdsItem*)c->plan_items[which].p;
  a.nx = g.nx;
  a.ny = g.ny;
  a.tnx = g.tnx;
  a.tny = g.tny;
  a.tiles_x = tl.tiles_x;
  a.R = R;
  a.n_sites = g.n;
  a.subs = nullptr;
  a.active = nullptr;
  a.done = c->mv_stop;  // a stopped GMRES cycle skips its remaining matvecs
  a.y_base = 0;
  a.tile_base = 0;
  a.item_base = 0;
  a.S = g.S;
  a.NG = g.NG;
  const int nreg = c->plan_nreg[which];
  // the last ny mod 16 rows: wide tiles, launched on the side stream so that
  // their work groups fill the CUs the regular launch leaves idle at its tail
  // (the two write disjoint partial-sum slots; the combine waits for both)
  LdsArgs aw = a;
  aw.tiles_x = tl.tiles_xw;
  aw.y_base = tl.y_wide;
  aw.tile_base = tl.n_reg;
  aw.item_base = nreg;
  const bool wide = nitems > nreg;
  if (wide && !c->ev_join) {  // created once; each handle is kept only once created
    if (!c->side) {
      hipStream_t s = nullptr;
      TM_HIP(c, hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
      c->side = s;
    }
    if (!c->ev_fork) {
      hipEvent_t e = nullptr;
      TM_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
      c->ev_fork = e;
    }
    hipEvent_t e = nullptr;
    TM_HIP(c, hipEventCreateWithFlags(&e, hipEventDisableTiming));
    c->ev_join = e;
  }
  if (e0) TM_HIP(c, hipEventRecord(e0, c->stream));
  if (wide) {
    TM_HIP(c, hipEventRecord(c->ev_fork, c->stream));
    TM_HIP(c, hipStreamWaitEvent(c->side, c->ev_fork, 0));
    lds_launch_any<T, true>(c->side, pf, nitems - nreg, R, aw);
    TM_HIP(c, hipEventRecord(c->ev_join, c->side));
  }
  lds_launch_any<T, false>(c->stream, pf, nreg, R, a);
  if (wide) TM_HIP(c, hipStreamWaitEvent(c->stream, c->ev_join, 0));
  if (e1) TM_HIP(c, hipEventRecord(e1, c->stream));
  if (y) {
    const int nb = (int)((total + 255) / 256);
    hipLaunchKernelGGL(lds_combine_kernel<T>, dim3(nb), dim3(256), 0, c->stream,
                       (const cplx<T>*)c->partial.p, (const int*)c->plan_ibeg[which].p, R, g.nx, tl,
                       (long long)g.n, x, (const c128*)c->t64.p, y, vec, total, op, g.S, g.NG,
                       c->mv_stop);
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

// Uniform work split computed on the device (no host planner, no upload):
// every tile of the lattice gets `ipt` items that cut its displacement-block
// list into equal-count ranges (empty ranges allowed); ibeg[t] = t * ipt.
template <typename T>
__global__ void lds_uniform_plan_kernel(LdsItem* __restrict__ items, int* __restrict__ ibeg, int nx,
                                        int ny, LdsTiling tl, int ipt) {
  using Ch = LdsChoice<T>;
  const int ntile = tl.n_reg + tl.n_wide;
  const int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx <= ntile) {
    ibeg[idx] = idx * ipt;
  }
  if (idx >= ntile * ipt) return;
  const int t = idx / ipt, k = idx % ipt;
  int X0, Y0, BX, BY;
  if (t < tl.n_reg) {
    X0 = (t % tl.tiles_x) * tl.TW;
    Y0 = (t / tl.tiles_x) * 16;
    BX = Ch::BX;
    BY = Ch::BY;
  } else {
    const int w = t - tl.n_reg;
    X0 = (w % tl.tiles_xw) * 4 * tl.TW;
    Y0 = tl.y_wide + (w / tl.tiles_xw) * 4;
    BX = Ch::WBX;
    BY = Ch::WBY;
  }
  const int dxlo = X0 - (nx - 1), dxhi = min(X0 + tl.TW - 1, nx - 1);  // relative per wave
  const int dylo = Y0 - (ny - 1), dyhi = min(Y0 + 3, ny - 1);
  const int nb = ((dxhi - dxlo + BX) / BX) * ((dyhi - dylo + BY) / BY);
  const int chunk = (nb + ipt - 1) / ipt;
  const int b0 = min(nb, k * chunk), b1 = min(nb, b0 + chunk);
  items[idx] = LdsItem{t, b0, b1, 0};
}

// Bytes of the uniform-split matvec's buffers inside a caller-provided
// region: items, ibeg, partial sums (each 256-byte aligned).
static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
template <typename T>
size_t lds_fixed_bytes(const Geometry& g, int R, int ipt) {
  using Ch = LdsChoice<T>;
  const LdsTiling tl = lds_tiling(g.nx, g.ny, 4 * Ch::GX);
  const size_t ntile = (size_t)tl.n_reg + tl.n_wide;
  const size_t nitems = ntile * ipt;
  return align256(nitems * sizeof(LdsItem)) + align256((ntile + 1) * sizeof(int)) +
         align256(nitems * 2 * R * (size_t)g.NG * tl.TW * 16 * SLOTS * sizeof(cplx<T>));
}
// Items per tile of the default work split (about 16k workgroups).
template <typename T>
int lds_fixed_default_ipt(const Geometry& g, int R) {
  using Ch = LdsChoice<T>;
  const LdsTiling tl = lds_tiling(g.nx, g.ny, 4 * Ch::GX);
  const int ntile = tl.n_reg + tl.n_wide;
  const int target = std::max(1, (16384 + 2 * R - 1) / (2 * R));
  return std::max(1, (target + ntile - 1) / ntile);
}

// The block matvec and its combine with every buffer inside `buf` (laid out
// as lds_fixed_bytes says), the work split made on the device: enqueues only
// kernels on the context stream (regular and wide tiles one after the other),
// allocates nothing and never synchronises.
template <typename T>
int lds_apply_fixed(tm_ctx* c, int R, const void* table, const void* xin, const c128* x, c128* y,
                    int op, int pf, int ipt, void* buf) {
  using Ch = LdsChoice<T>;
  const Geometry& g = c->g;
  const LdsTiling tl = lds_tiling(g.nx, g.ny, 4 * Ch::GX);
  const int ntile = tl.n_reg + tl.n_wide;
  const int nitems = ntile * ipt;
  char* p = static_cast<char*>(buf);
  LdsItem* items = reinterpret_cast<LdsItem*>(p);
  p += align256((size_t)nitems * sizeof(LdsItem));
  int* ibeg = reinterpret_cast<int*>(p);
  p += align256((size_t)(ntile + 1) * sizeof(int));
  void* partial = p;
  const int nth = std::max(nitems, ntile + 1);
  hipLaunchKernelGGL(lds_uniform_plan_kernel<T>, dim3((nth + 255) / 256), dim3(256), 0, c->stream,
                     items, ibeg, g.nx, g.ny, tl, ipt);
  LdsArgs a;
  a.table = table;
  a.x = xin;
  a.partial = partial;
  a.items = items;
  a.nx = g.nx;
  a.ny = g.ny;
  a.tnx = g.tnx;
  a.tny = g.tny;
  a.tiles_x = tl.tiles_x;
  a.R = R;
  a.n_sites = g.n;
  a.subs = nullptr;
  a.active = nullptr;
  a.done = nullptr;
  a.y_base = 0;
  a.tile_base = 0;
  a.item_base = 0;
  a.S = g.S;
  a.NG = g.NG;
  const int nreg = tl.n_reg * ipt;
  lds_launch_any<T, false>(c->stream, pf, nreg, R, a);
  if (nitems > nreg) {
    LdsArgs aw = a;
    aw.tiles_x = tl.tiles_xw;
    aw.y_base = tl.y_wide;
    aw.tile_base = tl.n_reg;
    aw.item_base = nreg;
    lds_launch_any<T, true>(c->stream, pf, nitems - nreg, R, aw);
  }
  const long long vec = g.vec_len(), total = vec * R;
  hipLaunchKernelGGL(lds_combine_kernel<T>, dim3((int)((total + 255) / 256)), dim3(256), 0, c->stream,
                     (const cplx<T>*)partial, (const int*)ibeg, R, g.nx, tl, (long long)g.n, x,
                     (const c128*)c->t64.p, y, vec, total, op, g.S, g.NG, (const int*)nullptr);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}
template size_t lds_fixed_bytes<float>(const Geometry&, int, int);
template size_t lds_fixed_bytes<double>(const Geometry&, int, int);
template int lds_fixed_default_ipt<float>(const Geometry&, int);
template int lds_fixed_default_ipt<double>(const Geometry&, int);
template int lds_apply_fixed<float>(tm_ctx*, int, const void*, const void*, const c128*, c128*, int,
                                    int, int, void*);
template int lds_apply_fixed<double>(tm_ctx*, int, const void*, const void*, const c128*, c128*, int,
                                     int, int, void*);

template <typename T>
void lds_geometry(int& TW, int& BX, int& BY) {
  TW = 4 * LdsChoice<T>::GX;
  BX = LdsChoice<T>::BX;
  BY = LdsChoice<T>::BY;
}
template void lds_geometry<float>(int&, int&, int&);
template void lds_geometry<double>(int&, int&, int&);

// Launch the LDS kernel over a batched item list with table prefetch depth
// pf (no allocation, no host synchronisation: safe under stream capture).
template <typename T>
int lds_launch(tm_ctx* c, const void* table, const void* xin, void* partial, const LdsItem* items,
               int nitems, int R, const SubParams* subs, const int* active, const int* done, int pf) {
  LdsArgs a;
  a.table = table;
  a.x = xin;
  a.partial = partial;
  a.items = items;
  a.nx = c->g.nx;
  a.ny = c->g.ny;
  a.tnx = c->g.tnx;
  a.tny = c->g.tny;
  a.tiles_x = 0;
  a.R = R;
  a.n_sites = 0;
  a.subs = subs;
  a.active = active;
  a.done = done;
  a.y_base = 0;
  a.tile_base = 0;
  a.item_base = 0;
  a.S = c->g.S;
  a.NG = c->g.NG;
  lds_launch_any<T>(c->stream, pf, nitems, R, a);
  return TM_OK;
}
template int lds_launch<float>(tm_ctx*, const void*, const void*, void*, const LdsItem*, int, int,
                               const SubParams*, const int*, const int*, int);
template int lds_launch<double>(tm_ctx*, const void*, const void*, void*, const LdsItem*, int, int,
                                const SubParams*, const int*, const int*, int);

template int lds_apply<float>(tm_ctx*, int, int, const void*, const void*, const c128*, c128*, int,
                              int, hipEvent_t, hipEvent_t, int);
template int lds_apply<double>(tm_ctx*, int, int, const void*, const void*, const c128*, c128*, int,
                               int, hipEvent_t, hipEvent_t, int);

}  // namespace tmh
