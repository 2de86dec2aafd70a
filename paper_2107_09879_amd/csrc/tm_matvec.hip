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
// Complex arithmetic uses four real products: Yr += Mr Xr - Mi Xi,
// Yi += Mr Xi + Mi Xr (16 MFMAs per 16 targets per displacement).
//
// Work decomposition: a workgroup owns a 16x16-site target tile (4 waves, each
// a row of four 4x4 groups) and a contiguous range of dy; it loops over every
// dx that can reach the tile.  Groups whose shifted source patch lies wholly
// outside the lattice skip their MFMAs (a wave-uniform test).  Each dy-range
// writes its own partial sum; a second kernel adds the partials in a fixed
// order (deterministic, no atomics) and forms y = x - t * z (or the variants).
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

struct MvArgs {
  const void* table;  // [D][2][16][16]
  const void* x;      // [R][2][N][16]
  void* partial;      // [P][R][2][N][16]
  int nx, ny, tnx, tny;
  int tiles_x, dy_per_chunk, R;
  long long n_sites;
};

template <typename T>
__global__ __launch_bounds__(256) void block_matvec_kernel(MvArgs a) {
  using M = Mfma<T>;
  using acc_t = typename M::acc_t;
  using C = cplx<T>;
  const int lane = threadIdx.x & 63;
  const int wave = threadIdx.x >> 6;
  const int jt = lane & 15;  // target within the 4x4 group
  const int kq = lane >> 4;  // slot quad
  const int tile = blockIdx.x;
  const int chunk = blockIdx.y;
  const int r = blockIdx.z >> 1;
  const int c = blockIdx.z & 1;
  const int X0 = (tile % a.tiles_x) * 16;
  const int Y0 = (tile / a.tiles_x) * 16;
  const int nx = a.nx, ny = a.ny;
  const int gy0 = Y0 + 4 * wave;  // first row of this wave's groups
  const int ty = gy0 + (jt >> 2);
  const int lx = jt & 3;
  const int xhi = min(X0 + 15, nx - 1);
  const int yhi = min(Y0 + 15, ny - 1);
  const int dxlo = X0 - (nx - 1), dxhi = xhi;
  const int dylo = Y0 - (ny - 1) + chunk * a.dy_per_chunk;
  const int dyhi = min(yhi, dylo + a.dy_per_chunk - 1);
  const int wx = 2 * a.tnx - 1;
  const size_t N = (size_t)a.n_sites;
  const C* __restrict__ xin = reinterpret_cast<const C*>(a.x) + ((size_t)r * NCLASS + c) * N * SLOTS;
  const C* __restrict__ tab = reinterpret_cast<const C*>(a.table);

  acc_t accr[4], acci[4];
#pragma unroll
  for (int g = 0; g < 4; ++g) {
    accr[g] = acc_t{0, 0, 0, 0};
    acci[g] = acc_t{0, 0, 0, 0};
  }

  const int wave_rows_hi = min(gy0 + 3, ny - 1);
  if (gy0 < ny) {
    for (int dy = dylo; dy <= dyhi; ++dy) {
      // source rows of this wave's targets must meet the lattice
      if (wave_rows_hi - dy < 0 || gy0 - dy >= ny) continue;
      const int sy = ty - dy;
      const bool row_ok = (ty < ny) && (sy >= 0) && (sy < ny);
      const C* trow = tab + ((size_t)(dy + a.tny - 1) * wx) * (NCLASS * SLOTS * SLOTS);
      for (int dx = dxlo; dx <= dxhi; ++dx) {
        const C* blk = trow + ((size_t)(dx + a.tnx - 1) * NCLASS + c) * (SLOTS * SLOTS) +
                       jt * SLOTS + 4 * kq;
        T ar[4], ai[4], nai[4];
        load4(blk, ar, ai);
#pragma unroll
        for (int s = 0; s < 4; ++s) nai[s] = -ai[s];
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const int gx0 = X0 + 4 * g;
          if (gx0 >= nx || gx0 + 3 - dx < 0 || gx0 - dx >= nx) continue;  // wave-uniform
          const int tx = gx0 + lx;
          const int sx = tx - dx;
          T br[4] = {0, 0, 0, 0}, bi[4] = {0, 0, 0, 0};
          if (row_ok && tx < nx && sx >= 0 && sx < nx)
            load4(xin + ((size_t)sy * nx + sx) * SLOTS + 4 * kq, br, bi);
#pragma unroll
          for (int s = 0; s < 4; ++s) {
            accr[g] = M::mma(ar[s], br[s], accr[g]);
            accr[g] = M::mma(nai[s], bi[s], accr[g]);
            acci[g] = M::mma(ar[s], bi[s], acci[g]);
            acci[g] = M::mma(ai[s], br[s], acci[g]);
          }
        }
      }
    }
  }
  // write this dy-range's partial sums (every valid target, zeros included)
  C* out = reinterpret_cast<C*>(a.partial) +
           (((size_t)chunk * a.R + r) * NCLASS + c) * N * SLOTS;
  if (ty < ny) {
#pragma unroll
    for (int g = 0; g < 4; ++g) {
      const int tx = X0 + 4 * g + lx;
      if (tx >= nx) continue;
      C* o = out + ((size_t)ty * nx + tx) * SLOTS;
#pragma unroll
      for (int v = 0; v < 4; ++v) o[M::out_row(kq, v)] = C{accr[g][v], acci[g][v]};
    }
  }
}

// y = x - t * sum (Forward), y = sum (Coupling, CouplingT), y = x - sum (Adjoint)
template <typename T>
__global__ void combine_kernel(const cplx<T>* __restrict__ partial, int P, long long chunk_stride,
                               const c128* __restrict__ x, const c128* __restrict__ t,
                               c128* __restrict__ y, long long vec, long long total, int mode) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= total) return;
  double sr = 0.0, si = 0.0;
  for (int p = 0; p < P; ++p) {
    const cplx<T> v = partial[(size_t)p * chunk_stride + idx];
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

double matvec_flops(const Geometry& g) {
  // 2 classes x (L/2)^2 complex multiply-adds x 8 real flops per ordered pair
  const double N = (double)g.n;
  return 4.0 * (double)g.L * (double)g.L * N * (N - 1.0);
}

static int choose_chunks(const tm_ctx* c, int tiles, int R, int dy_range) {
  if (c->chunks_override > 0) return std::min(c->chunks_override, dy_range);
  const long long target = 2048;  // workgroups in flight for 256 CUs
  long long per = (long long)tiles * NCLASS * R;
  int P = (int)((target + per - 1) / per);
  if (P < 1) P = 1;
  if (P > dy_range) P = dy_range;
  return P;
}

template <typename T>
static int apply_impl(tm_ctx* c, Op op, int R, const c128* x, c128* y) {
  const Geometry& g = c->g;
  const long long vec = g.vec_len();
  const long long total = vec * R;
  const bool transposed = (op == Op::Adjoint || op == Op::CouplingT);
  int rc;
  if (transposed && !c->have_tabT) {
    if ((rc = build_transposed_tables(c)) != TM_OK) return rc;
  }
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
  const int tiles_x = (g.nx + 15) / 16, tiles_y = (g.ny + 15) / 16;
  const int tiles = tiles_x * tiles_y;
  const int dy_range = g.ny + 15;
  const int P = choose_chunks(c, tiles, R, dy_range);
  const int dy_per_chunk = (dy_range + P - 1) / P;
  if ((rc = ensure(c, c->partial, (size_t)P * total * sizeof(cplx<T>))) != TM_OK) return rc;
  MvArgs a;
  a.table = table;
  a.x = xin;
  a.partial = c->partial.p;
  a.nx = g.nx;
  a.ny = g.ny;
  a.tnx = g.tnx;
  a.tny = g.tny;
  a.tiles_x = tiles_x;
  a.dy_per_chunk = dy_per_chunk;
  a.R = R;
  a.n_sites = g.n;
  const int which = std::is_same<T, double>::value ? 0 : 1;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (c->prof) {
    TM_HIP(c, hipEventCreate(&e0));
    TM_HIP(c, hipEventCreate(&e1));
    TM_HIP(c, hipEventRecord(e0, c->stream));
  }
  hipLaunchKernelGGL(block_matvec_kernel<T>, dim3(tiles, P, NCLASS * R), dim3(256), 0, c->stream,
                     a);
  if (c->prof) {
    TM_HIP(c, hipEventRecord(e1, c->stream));
    c->prof_pending[which].push_back({e0, e1});
    c->prof_acc[which].flops = matvec_flops(g) * R;
  }
  const int nb = (int)((total + 255) / 256);
  hipLaunchKernelGGL(combine_kernel<T>, dim3(nb), dim3(256), 0, c->stream,
                     (const cplx<T>*)c->partial.p, P, total, x, (const c128*)c->t64.p, y, vec,
                     total, (int)op);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int apply_op(tm_ctx* c, Op op, int prec, int R, const c128* x, c128* y) {
  if (prec == TM_PREC_MIXED) return apply_impl<float>(c, op, R, x, y);
  return apply_impl<double>(c, op, R, x, y);
}

}  // namespace tmh
