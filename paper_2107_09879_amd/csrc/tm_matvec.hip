// Block matvec of the multiple-scattering operator on matrix cores.
//
// The operator (App. I.C, eq. "final_linear_eqs" with the block-diagonal
// preconditioner; App. I.D applies it matrix-free inside GMRES) needs
//   z_t = sum_{s != t} M(t - s) x_s,     M(dx, dy) = xi(k pitch (dx, dy, 0))^T,
// for every target site t of the lattice.  For a fixed displacement the same
// 16x16 complex block (per z-mirror class) multiplies many source vectors, so
// the product is a dense contraction: the kernel holds a tile of targets in
// MFMA accumulators and streams displacements through it.
//
// Mapping (v_mfma_{f32,f64}_16x16x4): D[i][j] += sum_k A[i][k] B[k][j] with
//   i = output slot, j = one of 16 targets (a 4x4 patch of lattice sites),
//   k = input slot; the 16 slots are consumed as four K-steps s, lane l
//   supplying slot 4*(l/16) + s, so each lane reads 4 consecutive complex
//   slots of one block row (A) and of one source vector (B) -- contiguous
//   32/64-byte loads -- and writes the 4 output slots its accumulator holds.
// Complex arithmetic uses three real products per complex product (see the
// kernel), 12 MFMAs per 16 targets per displacement.
//
// Work decomposition: a workgroup owns a 16x16-site target tile (4 waves, each
// a row of four 4x4 groups) and a contiguous range of dy chosen by the host
// planner so that all workgroups carry similar work; it loops over every dx
// that can reach the tile.  Groups whose shifted source patch lies wholly
// outside the lattice skip their MFMAs (a wave-uniform test).  Each work item
// writes its own partial sum; a second kernel adds the partials in a fixed
// order (deterministic, no atomics) and forms y = x - t * z (or the variants).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "tm_internal.h"

namespace tmh {

typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef double f64x4 __attribute__((ext_vector_type(4)));

template <typename T>
struct Mfma;
// Output layout of the 16x16 result: accumulator element v of lane l holds
// row out_row(l/16, v), column l%16.  The FP32 instruction keeps four
// consecutive rows per lane group; the FP64 one interleaves them (row
// 4*v + l/16), as measured on gfx950.
template <>
struct Mfma<float> {
  using acc_t = f32x4;
  __device__ static inline acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int kq, int v) { return 4 * kq + v; }
};
template <>
struct Mfma<double> {
  using acc_t = f64x4;
  __device__ static inline acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  __device__ static inline int out_row(int kq, int v) { return 4 * v + kq; }
};

__device__ inline void load4(const c64* __restrict__ p, float* re, float* im) {
  const float4 a = *reinterpret_cast<const float4*>(p);
  const float4 b = *reinterpret_cast<const float4*>(p + 2);
  re[0] = a.x; im[0] = a.y; re[1] = a.z; im[1] = a.w;
  re[2] = b.x; im[2] = b.y; re[3] = b.z; im[3] = b.w;
}
__device__ inline void load4(const c128* __restrict__ p, double* re, double* im) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double2 a = *reinterpret_cast<const double2*>(p + s);
    re[s] = a.x;
    im[s] = a.y;
  }
}

// One work item = one 16x16-site target tile and a contiguous range of dy
// (chosen on the host so that all items carry about the same MFMA work).
struct MvItem {
  int tile, dylo, dyhi, pad;
};

struct MvArgs {
  const void* table;      // [D][2][16][16]
  const void* x;          // [R][2][N][16]
  void* partial;          // [item][R*2][256 tile sites][16]
  const MvItem* items;
  int nx, ny, tnx, tny;
  int tiles_x, R;
  long long n_sites;
};

template <typename T>
__device__ inline void load_operands(const cplx<T>* __restrict__ tab,
                                     const cplx<T>* __restrict__ xin, int dx, int dy, int c,
                                     int jt, int kq, int wx, int tnx, int tny, int nx, int ny,
                                     const int* tx, int ty, T* ar, T* ai, T (*br)[4],
                                     T (*bi)[4]) {
  const cplx<T>* blk = tab + (((size_t)(dy + tny - 1) * wx + (dx + tnx - 1)) * NCLASS + c) *
                                 (SLOTS * SLOTS) + jt * SLOTS + 4 * kq;
  load4(blk, ar, ai);
  const int sy = ty - dy;
  const bool row_ok = (ty < ny) && (sy >= 0) && (sy < ny);
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    const int sx = tx[g] - dx;
    if (row_ok && tx[g] < nx && sx >= 0 && sx < nx) {
      load4(xin + ((size_t)sy * nx + sx) * SLOTS + 4 * kq, br[g], bi[g]);
    } else {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        br[g][s] = 0;
        bi[g][s] = 0;
      }
    }
  }
}

// Kernel variants (all compute the same product; the autotuner picks one):
//   GAUSS    complex products from three real MFMA products,
//              T1 += Mr Xr, T2 += Mi Xi, T3 += (Mr + Mi)(Xr + Xi),
//              Yr = T1 - T2, Yi = T3 - T1 - T2   (12 MFMAs per group and
//            displacement), else from four (Yr += Mr Xr - Mi Xi,
//            Yi += Mr Xi + Mi Xr; 16 MFMAs);
//   PREFETCH operands of the next displacement are loaded while the current
//            one's MFMAs run (two register sets), else loaded just before use;
//   OCC      minimum waves per SIMD the register allocation must allow.
template <typename T, bool GAUSS, bool PREFETCH, int OCC>
__global__ __launch_bounds__(256, OCC) void block_matvec_kernel(MvArgs a) {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using C = cplx<T>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int jt = lane & 15;  // target within the 4x4 group
  const int kq = lane >> 4;  // slot quad
  const MvItem it = a.items[blockIdx.x];
  const int rc = blockIdx.y;
  const int r = rc >> 1, c = rc & 1;
  const int X0 = (it.tile % a.tiles_x) * 16;
  const int Y0 = (it.tile / a.tiles_x) * 16;
  const int nx = a.nx, ny = a.ny;
  const int gy0 = Y0 + 4 * wave;
  const int ty = gy0 + (jt >> 2);
  const int lx = jt & 3;
  int tx[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) tx[g] = X0 + 4 * g + lx;
  const int wx = 2 * a.tnx - 1;
  const size_t N = (size_t)a.n_sites;
  const C* __restrict__ xin = reinterpret_cast<const C*>(a.x) + ((size_t)r * NCLASS + c) * N * SLOTS;
  const C* __restrict__ tab = reinterpret_cast<const C*>(a.table);

  acc_t t1[4], t2[4], t3[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    t1[g] = acc_t{0, 0, 0, 0};
    t2[g] = acc_t{0, 0, 0, 0};
    t3[g] = acc_t{0, 0, 0, 0};
  }
  // displacements this wave visits: dy within the item and reaching a source
  // row, dx over the tile's reach
  const int dxlo = X0 - (nx - 1), dxhi = min(X0 + 15, nx - 1);
  const int ndx = dxhi - dxlo + 1;
  const int dyb = max(it.dylo, gy0 - (ny - 1));
  const int dye = min(it.dyhi, min(gy0 + 3, ny - 1));
  const int nq = (gy0 < ny && dye >= dyb) ? (dye - dyb + 1) * ndx : 0;

  T ar[4], ai[4], br[4][4], bi[4][4];
  T nar[4], nai[4], nbr[4][4], nbi[4][4];
  if (PREFETCH && nq > 0)
    load_operands<T>(tab, xin, dxlo, dyb, c, jt, kq, wx, a.tnx, a.tny, nx, ny, tx, ty, ar, ai, br,
                     bi);
  int dx = dxlo, dy = dyb;
  for (int q = 0; q < nq; ++q) {
    int ndxv = dx + 1, ndyv = dy;
    if (ndxv > dxhi) {
      ndxv = dxlo;
      ++ndyv;
    }
    const bool more = (q + 1 < nq);
    if (PREFETCH) {
      if (more)
        load_operands<T>(tab, xin, ndxv, ndyv, c, jt, kq, wx, a.tnx, a.tny, nx, ny, tx, ty, nar,
                         nai, nbr, nbi);
    } else {
      load_operands<T>(tab, xin, dx, dy, c, jt, kq, wx, a.tnx, a.tny, nx, ny, tx, ty, ar, ai, br,
                       bi);
    }
    T ms[4];
#pragma unroll
    for (int s = 0; s < 4; ++s) ms[s] = GAUSS ? ar[s] + ai[s] : -ai[s];
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int gx0 = X0 + 4 * g;
      if (gx0 >= nx || gx0 + 3 - dx < 0 || gx0 - dx >= nx) continue;  // wave-uniform
      if (GAUSS) {
        T xs[4];
#pragma unroll
        for (int s = 0; s < 4; ++s) xs[s] = br[g][s] + bi[g][s];
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          t1[g] = M::mma(ar[s], br[g][s], t1[g]);
          t2[g] = M::mma(ai[s], bi[g][s], t2[g]);
          t3[g] = M::mma(ms[s], xs[s], t3[g]);
        }
      } else {
#pragma unroll
        for (int s = 0; s < 4; ++s) {
          t1[g] = M::mma(ar[s], br[g][s], t1[g]);
          t2[g] = M::mma(ar[s], bi[g][s], t2[g]);
          t1[g] = M::mma(ms[s], bi[g][s], t1[g]);
          t2[g] = M::mma(ai[s], br[g][s], t2[g]);
        }
      }
    }
    if (PREFETCH && more) {
#pragma unroll
      for (int s = 0; s < 4; ++s) {
        ar[s] = nar[s];
        ai[s] = nai[s];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          br[g][s] = nbr[g][s];
          bi[g][s] = nbi[g][s];
        }
      }
    }
    dx = ndxv;
    dy = ndyv;
  }
  // this item's partial sums for every valid target of the tile (zeros included)
  C* out = reinterpret_cast<C*>(a.partial) +
           ((size_t)blockIdx.x * (2 * a.R) + rc) * (256 * SLOTS);
  if (ty < ny) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      if (tx[g] >= nx) continue;
      C* o = out + (size_t)((ty - Y0) * 16 + (tx[g] - X0)) * SLOTS;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T yr = GAUSS ? t1[g][v] - t2[g][v] : t1[g][v];
        const T yi = GAUSS ? t3[g][v] - t1[g][v] - t2[g][v] : t2[g][v];
        o[M::out_row(kq, v)] = C{yr, yi};
      }
    }
  }
}

template <typename T>
int lds_apply(tm_ctx* c, int which, int R, const void* table, const void* xin, const c128* x,
              c128* y, int op, int items_target, hipEvent_t e0, hipEvent_t e1, int pf);
constexpr int LDS_VARIANT = 8;  // 8, 9, 10: LDS-staged with A prefetched 1, 2, 3 displacements ahead
constexpr int N_VARIANTS = 11;

using MvKernel = void (*)(MvArgs);
template <typename T>
static MvKernel mv_kernel(int variant) {
  switch (variant & 7) {
    case 0: return block_matvec_kernel<T, false, false, 2>;
    case 1: return block_matvec_kernel<T, true, false, 2>;
    case 2: return block_matvec_kernel<T, false, true, 2>;
    case 3: return block_matvec_kernel<T, true, true, 2>;
    case 4: return block_matvec_kernel<T, false, false, 4>;
    case 5: return block_matvec_kernel<T, true, false, 4>;
    case 6: return block_matvec_kernel<T, false, true, 4>;
    default: return block_matvec_kernel<T, true, true, 4>;
  }
}

// y = x - t * z (Forward), y = z (Coupling, CouplingT), y = x - z (Adjoint),
// z = sum of the partials of the items covering the site's tile, added in
// item order (deterministic).
template <typename T>
__global__ void combine_kernel(const cplx<T>* __restrict__ partial, const int* __restrict__ ibeg,
                               int R, int nx, int tiles_x, long long N,
                               const c128* __restrict__ x, const c128* __restrict__ t,
                               c128* __restrict__ y, long long vec, long long total, int mode) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  const int slot = (int)(idx % SLOTS);
  const long long site = (idx / SLOTS) % N;
  const int rc = (int)(idx / (SLOTS * N));  // r*2 + c
  const int sx = (int)(site % nx), sy = (int)(site / nx);
  const int tile = (sy >> 4) * tiles_x + (sx >> 4);
  const int ls = ((sy & 15) << 4) + (sx & 15);
  double sr = 0.0, si = 0.0;
  for (int i = ibeg[tile]; i < ibeg[tile + 1]; ++i) {
    const cplx<T> v = partial[(((size_t)i * (2 * R) + rc) * 256 + ls) * SLOTS + slot];
    sr += (double)v.re;
    si += (double)v.im;
  }
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

// out = (T)(t * x) or (T)x, for the block-kernel input
template <typename T>
__global__ void prep_kernel(const c128* __restrict__ x, const c128* __restrict__ t,
                            cplx<T>* __restrict__ out, long long vec, long long total) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  c128 v = x[idx];
  if (t) {
    const c128 tv = t[idx % vec];
    v = c128{tv.re * v.re - tv.im * v.im, tv.re * v.im + tv.im * v.re};
  }
  out[idx] = cplx<T>{(T)v.re, (T)v.im};
}

template <typename T>
void launch_prep(hipStream_t st, const c128* x, const c128* t, void* out, long long vec,
                 long long total) {
  hipLaunchKernelGGL(prep_kernel<T>, dim3((int)((total + 255) / 256)), dim3(256), 0, st, x, t,
                     (cplx<T>*)out, vec, total);
}
template void launch_prep<float>(hipStream_t, const c128*, const c128*, void*, long long, long long);
template void launch_prep<double>(hipStream_t, const c128*, const c128*, void*, long long, long long);

double matvec_flops(const Geometry& g) {
  // 2 classes x (L/2)^2 complex multiply-adds x 8 real flops per ordered pair
  const double N = (double)g.n;
  return 4.0 * (double)g.L * (double)g.L * N * (N - 1.0);
}

// Host work planner.  The MFMA work of a tile at a given dy is the number of
// (4x4 group, dx) pairs whose shifted source patch meets the lattice, summed
// over the wave rows that reach a source row; each tile's dy range is cut into
// chunks of about equal work so that every workgroup of the launch carries a
// similar load (no tail wave of stragglers).
static void make_plan(const Geometry& g, int target_items, std::vector<MvItem>& items,
                      std::vector<int>& ibeg) {
  const int nx = g.nx, ny = g.ny;
  const int tiles_x = (nx + 15) / 16, tiles_y = (ny + 15) / 16;
  const int tiles = tiles_x * tiles_y;
  std::vector<std::vector<double>> prof(tiles);
  std::vector<int> dylo(tiles), dyhi(tiles);
  double total = 0.0;
  for (int t = 0; t < tiles; ++t) {
    const int X0 = (t % tiles_x) * 16, Y0 = (t / tiles_x) * 16;
    const int xhi = std::min(X0 + 15, nx - 1), dxlo = X0 - (nx - 1);
    const int ndx = xhi - dxlo + 1;
    double sumcx = 0.0;
    for (int q = 0; q < 4; ++q) {
      const int gx0 = X0 + 4 * q;
      if (gx0 < nx) sumcx += std::min(gx0 + 3, xhi) - (gx0 - nx + 1) + 1;
    }
    dylo[t] = Y0 - (ny - 1);
    dyhi[t] = std::min(Y0 + 15, ny - 1);
    prof[t].assign(dyhi[t] - dylo[t] + 1, 0.0);
    for (int dy = dylo[t]; dy <= dyhi[t]; ++dy) {
      double w = 0.0;
      for (int wv = 0; wv < 4; ++wv) {
        const int gy0 = Y0 + 4 * wv;
        if (gy0 >= ny) continue;
        if (dy < gy0 - (ny - 1) || dy > std::min(gy0 + 3, ny - 1)) continue;
        w += 12.0 * sumcx + 4.0 * ndx;  // MFMAs + per-displacement overhead
      }
      prof[t][dy - dylo[t]] = w;
      total += w;
    }
  }
  const double per = total / std::max(1, target_items);
  items.clear();
  ibeg.assign(tiles + 1, 0);
  for (int t = 0; t < tiles; ++t) {
    ibeg[t] = (int)items.size();
    const int ndy = dyhi[t] - dylo[t] + 1;
    double wt = 0.0;
    for (double v : prof[t]) wt += v;
    int nch = (int)std::llround(wt / per);
    nch = std::max(1, std::min(nch, ndy));
    double acc = 0.0;
    int start = dylo[t];
    int k = 1;
    for (int dy = dylo[t]; dy <= dyhi[t]; ++dy) {
      acc += prof[t][dy - dylo[t]];
      if (k < nch && acc >= k * wt / nch && dy < dyhi[t]) {
        items.push_back(MvItem{t, start, dy, 0});
        start = dy + 1;
        ++k;
      }
    }
    items.push_back(MvItem{t, start, dyhi[t], 0});
  }
  ibeg[tiles] = (int)items.size();
}

static int default_items(int R) { return std::max(1, (16384 + 2 * R - 1) / (2 * R)); }

static int ensure_plan(tm_ctx* c, int R, int which) {
  const int target = c->mv_items[which] > 0 ? c->mv_items[which] : default_items(R);
  if (c->plan_kind[which] == 1 && c->plan_R[which] == R && c->plan_target[which] == target)
    return TM_OK;
  std::vector<MvItem> items;
  std::vector<int> ibeg;
  make_plan(c->g, target, items, ibeg);
  int rc;
  if ((rc = ensure(c, c->plan_items[which], items.size() * sizeof(MvItem))) != TM_OK) return rc;
  if ((rc = ensure(c, c->plan_ibeg[which], ibeg.size() * sizeof(int))) != TM_OK) return rc;
  // launches of the previous plan may still read it (the upload is not
  // ordered with a non-blocking context stream)
  TM_HIP(c, hipStreamSynchronize(c->stream));
  TM_HIP(c, hipMemcpy(c->plan_items[which].p, items.data(), items.size() * sizeof(MvItem),
                      hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy(c->plan_ibeg[which].p, ibeg.data(), ibeg.size() * sizeof(int),
                      hipMemcpyHostToDevice));
  c->plan_kind[which] = 1;
  c->plan_R[which] = R;
  c->plan_target[which] = target;
  c->plan_nitems[which] = (int)items.size();
  return TM_OK;
}

template <typename T>
static int apply_impl(tm_ctx* c, Op op, int R, const c128* x, c128* y) {
  const Geometry& g = c->g;
  const long long vec = g.vec_len();
  const long long total = vec * R;
  const bool transposed = (op == Op::Adjoint || op == Op::CouplingT);
  int rc;
  if (!g.lattice) {  // off-lattice: blocks formed on the fly, no tables
    const void* xin = x;
    if (!std::is_same<T, double>::value || op == Op::Adjoint) {
      if ((rc = ensure(c, c->xlow, (size_t)total * sizeof(cplx<T>))) != TM_OK) return rc;
      launch_prep<T>(c->stream, x, op == Op::Adjoint ? (const c128*)c->t64.p : nullptr, c->xlow.p, vec,
                     total);
      xin = c->xlow.p;
    }
    return offlattice_apply<T>(c, op, R, xin, x, y);
  }
  if (transposed && !c->have_tabT) {
    if ((rc = build_transposed_tables(c)) != TM_OK) return rc;
  }
  const int which = std::is_same<T, double>::value ? 0 : 1;
  const void* table = std::is_same<T, double>::value
                          ? (transposed ? c->tabT64.p : c->tab64.p)
                          : (transposed ? c->tabT32.p : c->tab32.p);
  // block-kernel input
  const cplx<T>* xin;
  const bool need_t_in = (op == Op::Adjoint);
  if (std::is_same<T, double>::value && !need_t_in) {
    xin = reinterpret_cast<const cplx<T>*>(x);
  } else {
    if ((rc = ensure(c, c->xlow, (size_t)total * sizeof(cplx<T>))) != TM_OK) return rc;
    const int nb = (int)((total + 255) / 256);
    hipLaunchKernelGGL(prep_kernel<T>, dim3(nb), dim3(256), 0, c->stream, x,
                       need_t_in ? (const c128*)c->t64.p : nullptr, (cplx<T>*)c->xlow.p, vec,
                       total);
    xin = (const cplx<T>*)c->xlow.p;
  }
  // the direct kernels (variants 0..7) are written for one 16-slot group
  // per class (lmax <= 3); larger lmax runs the LDS-staged kernel at the
  // default prefetch depth
  const int variant = (g.NG == 1 || c->mv_variant[which] >= LDS_VARIANT)
                          ? c->mv_variant[which]
                          : (std::is_same<T, double>::value ? LDS_VARIANT + 1 : LDS_VARIANT + 2);
  if (variant >= LDS_VARIANT) {
    hipEvent_t e0 = nullptr, e1 = nullptr;
    if (c->prof) {
      TM_HIP(c, hipEventCreate(&e0));
      TM_HIP(c, hipEventCreate(&e1));
    }
    const int tgt = c->mv_items[which] > 0 ? c->mv_items[which] : default_items(R);
    rc = lds_apply<T>(c, which, R, table, xin, x, y, (int)op, tgt, e0, e1,
                      variant - LDS_VARIANT + 1);
    if (c->prof && rc == TM_OK) {
      c->prof_pending[which].push_back({e0, e1});
      c->prof_acc[which].flops = matvec_flops(g) * R;
    }
    return rc;
  }
  if ((rc = ensure_plan(c, R, which)) != TM_OK) return rc;
  const int tiles_x = (g.nx + 15) / 16;
  const int nitems = c->plan_nitems[which];
  if ((rc = ensure(c, c->partial, (size_t)nitems * 2 * R * 256 * SLOTS * sizeof(cplx<T>))) != TM_OK)
    return rc;
  MvArgs a;
  a.table = table;
  a.x = xin;
  a.partial = c->partial.p;
  a.items = (const MvItem*)c->plan_items[which].p;
  a.nx = g.nx;
  a.ny = g.ny;
  a.tnx = g.tnx;
  a.tny = g.tny;
  a.tiles_x = tiles_x;
  a.R = R;
  a.n_sites = g.n;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->prof) {
    TM_HIP(c, hipEventCreate(&e0));
    TM_HIP(c, hipEventCreate(&e1));
    TM_HIP(c, hipEventRecord(e0, c->stream));
  }
  hipLaunchKernelGGL(mv_kernel<T>(c->mv_variant[which]), dim3(nitems, 2 * R), dim3(256), 0,
                     c->stream, a);
  if (c->prof) {
    TM_HIP(c, hipEventRecord(e1, c->stream));
    c->prof_pending[which].push_back({e0, e1});
    c->prof_acc[which].flops = matvec_flops(g) * R;
  }
  const int nb = (int)((total + 255) / 256);
  hipLaunchKernelGGL(combine_kernel<T>, dim3(nb), dim3(256), 0, c->stream,
                     (const cplx<T>*)c->partial.p, (const int*)c->plan_ibeg[which].p, R, g.nx, tiles_x,
                     (long long)g.n, x, (const c128*)c->t64.p, y, vec, total, (int)op);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

// Autotuner: time every kernel variant with a few work-item counts on the
// current geometry for R right-hand sides; keep the fastest per precision.
template <typename T>
static int autotune_impl(tm_ctx* c, int R, double* best_ms) {
  const Geometry& g = c->g;
  const int which = std::is_same<T, double>::value ? 0 : 1;
  const long long total = g.vec_len() * R;
  int rc;
  if ((rc = ensure(c, c->xlow, (size_t)total * sizeof(cplx<T>))) != TM_OK) return rc;
  TM_HIP(c, hipMemsetAsync(c->xlow.p, 0, (size_t)total * sizeof(cplx<T>), c->stream));
  // workgroup counts (items x 2R); smaller equal-work items keep every CU
  // busy to the end of the launch, at the price of more partial sums
  const int wg_targets[] = {4096, 8192, 16384, 32768, 65536};
  hipEvent_t e0, e1;
  TM_HIP(c, hipEventCreate(&e0));
  TM_HIP(c, hipEventCreate(&e1));
  double best = 1e300;
  int bv = c->mv_variant[which], bi = c->mv_items[which];
  // only the LDS-staged variants: the direct kernels (0..7) never won at any
  // measured size and cost up to tens of milliseconds per timed launch; FP64
  // runs variant 10 as 9
  const int vlast = std::is_same<T, double>::value ? LDS_VARIANT + 1 : N_VARIANTS - 1;
  for (int v = LDS_VARIANT; v <= vlast; ++v) {
    for (int wt : wg_targets) {
      c->mv_variant[which] = v;
      c->mv_items[which] = std::max(1, wt / (2 * R));
      double tmin = 1e300;
      for (int rep = 0; rep < 4; ++rep) {
        rc = lds_apply<T>(c, which, R, std::is_same<T, double>::value ? c->tab64.p : c->tab32.p,
                          c->xlow.p, nullptr, nullptr, 0, c->mv_items[which], e0, e1,
                          v - LDS_VARIANT + 1);
        if (rc != TM_OK) return rc;
        TM_HIP(c, hipEventSynchronize(e1));
        float ms = 0.f;
        TM_HIP(c, hipEventElapsedTime(&ms, e0, e1));
        if (rep > 0) tmin = std::min(tmin, (double)ms);
      }
      if (tmin < best) {
        best = tmin;
        bv = v;
        bi = c->mv_items[which];
      }
    }
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  c->mv_variant[which] = bv;
  c->mv_items[which] = bi;
  if (best_ms) *best_ms = best;
  return TM_OK;
}

int autotune(tm_ctx* c, int R, int prec, double* best_ms) {
  if (prec == TM_PREC_MIXED) return autotune_impl<float>(c, R, best_ms);
  return autotune_impl<double>(c, R, best_ms);
}

static int apply_raw(tm_ctx* c, Op op, int prec, int R, const c128* x, c128* y) {
  if (prec == TM_PREC_MIXED) return apply_impl<float>(c, op, R, x, y);
  return apply_impl<double>(c, op, R, x, y);
}

int apply_op(tm_ctx* c, Op op, int prec, int R, const c128* x, c128* y) {
  if (!c->t_dense || (op != Op::Forward && op != Op::Adjoint)) return apply_raw(c, op, prec, R, x, y);
  // dense T: the coupling product, then the (cheap, FP64) per-scatterer block
  const long long total = (long long)R * c->g.vec_len();
  int rc;
  if ((rc = ensure(c, c->ttmp, (size_t)2 * total * sizeof(c128))) != TM_OK) return rc;
  c128* tmp = (c128*)c->ttmp.p;
  if (op == Op::Forward) {  // y = x - T (A x)
    if ((rc = apply_raw(c, Op::Coupling, prec, R, x, tmp)) != TM_OK) return rc;
    return launch_tdense(c, R, 1, x, tmp, y);
  }
  // y = x - A^T (T^T x)
  c128* tmp2 = tmp + total;
  if ((rc = launch_tdense(c, R, 2, nullptr, x, tmp)) != TM_OK) return rc;
  if ((rc = apply_raw(c, Op::CouplingT, prec, R, tmp, tmp2)) != TM_OK) return rc;
  k_sub(c->stream, y, x, tmp2, total);
  return TM_OK;
}

}  // namespace tmh
