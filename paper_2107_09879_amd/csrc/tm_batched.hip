// Batched solve of many subregions of one lattice, each with several
// right-hand sides, advancing all (subregion, rhs) systems together.
//
// The paper distributes a large metasurface as independent subregion solves
// (a group of sources plus a padding region, solved alone; the fields are
// summed afterwards; App. II and the main text's distribution strategy).  On
// one GPU those solves become one batch: every Arnoldi step issues ONE
// block-matvec launch whose work items span all subregions and right-hand
// sides (the LDS-staged kernel with per-item subregion parameters), then
// segmented FP64 Gram-Schmidt, norm and scaling kernels over the packed
// vector, and a device-side Givens update per system.  A restart cycle (m
// Arnoldi steps) is captured once into a hipGraph and replayed; kernels read a
// device flag and return immediately once every system of the cycle has met
// its target, so a converged batch costs only empty launches.  Systems that
// converge earlier are masked out of the matvec and the Krylov kernels.
//
// Packed layout: subregion k holds [R][2][N_k][16] complex at vec_off_k; the
// system (k, r) is the contiguous segment [2][N_k][16] at vec_off_k +
// r*32*N_k.  Subregion sites are indexed ly*nx_k + lx, full-lattice site
// (oy+ly)*nx + (ox+lx); T comes from the full lattice.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "tm_internal.h"

namespace tmh {

// from tm_matvec_lds.hip (the planner, lds_block_work and lds_split, is in
// tm_host.h)
template <typename T>
int lds_launch(tm_ctx* c, const void* table, const void* xin, void* partial, const LdsItem* items,
               int nitems, int R, const SubParams* subs, const int* active, const int* done, int pf);
template <typename T>
void lds_geometry(int& TW, int& BX, int& BY);

constexpr int BT = 256;        // threads per block
constexpr int SEG = 4096;      // elements per segmented-reduction block

struct SegBlock {
  int sys, pad;
  long long lo, hi;
};

__device__ inline int find_sub(const SubParams* __restrict__ sp, int S, long long e, int R) {
  // largest k with vec_off_k <= e (vec_off increasing)
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (sp[mid].vec_off <= e) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

__device__ inline double bwarp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}
__device__ inline double bblock_sum(double v, double* sh) {
  v = bwarp_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// b = t * a0 gathered from the full lattice into the packed layout
__global__ void b_gather_rhs(const tm_c128* __restrict__ a0, const c128* __restrict__ t,
                             const SubParams* __restrict__ sp, int S, int R, int nxf, long long Nf,
                             SlotMaps m, long long total, c128* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = find_sub(sp, S, e, R);
  const SubParams p = sp[k];
  const long long Nk = (long long)p.nx * p.ny;
  long long q = e - p.vec_off;
  const int slot = (int)(q % m.S);
  q /= m.S;
  const long long site = q % Nk;
  q /= Nk;
  const int cls = (int)(q % NCLASS);
  const int r = (int)(q / NCLASS);
  const long long fs = (long long)(p.oy + site / p.nx) * nxf + (p.ox + site % p.nx);
  const int n = m.n_of[cls][slot];
  c128 v{0.0, 0.0};
  if (n >= 0) {
    const tm_c128 a = a0[((long long)r * Nf + fs) * m.L + n];
    const c128 tv = t[((long long)cls * Nf + fs) * m.S + slot];
    v = c128{tv.re * a.re - tv.im * a.im, tv.re * a.im + tv.im * a.re};
  }
  out[e] = v;
}

// b = t * a0 from caller-given subregion coefficients: a0 boundary
// [S][R][N_k][L] (concatenated, the output layout) -> packed slot layout
__global__ void b_gather_packed_rhs(const tm_c128* __restrict__ a0, const long long* __restrict__ out_off,
                                    const c128* __restrict__ t, const SubParams* __restrict__ sp,
                                    int S, int R, int nxf, long long Nf, SlotMaps m, long long total,
                                    c128* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = find_sub(sp, S, e, R);
  const SubParams p = sp[k];
  const long long Nk = (long long)p.nx * p.ny;
  long long q = e - p.vec_off;
  const int slot = (int)(q % m.S);
  q /= m.S;
  const long long site = q % Nk;
  q /= Nk;
  const int cls = (int)(q % NCLASS);
  const int r = (int)(q / NCLASS);
  const long long fs = (long long)(p.oy + site / p.nx) * nxf + (p.ox + site % p.nx);
  const int n = m.n_of[cls][slot];
  c128 v{0.0, 0.0};
  if (n >= 0) {
    const tm_c128 a = a0[out_off[k] + ((long long)r * Nk + site) * m.L + n];
    const c128 tv = t[((long long)cls * Nf + fs) * m.S + slot];
    v = c128{tv.re * a.re - tv.im * a.im, tv.re * a.im + tv.im * a.re};
  }
  out[e] = v;
}

// packed slot layout -> boundary [S][R][N_k][L] (concatenated, same order)
__global__ void b_unpack(const c128* __restrict__ in, const SubParams* __restrict__ sp,
                         const long long* __restrict__ out_off, int S, int R, SlotMaps m,
                         long long total, tm_c128* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  int lo = 0, hi = S - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (out_off[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const SubParams p = sp[lo];
  const long long Nk = (long long)p.nx * p.ny;
  long long q = e - out_off[lo];
  const int n = (int)(q % m.L);
  q /= m.L;
  const long long site = q % Nk;
  const int r = (int)(q / Nk);
  const c128 v = in[p.vec_off + (((long long)r * NCLASS + m.cls_of[n]) * Nk + site) * m.S + m.slot_of[n]];
  out[e] = tm_c128{v.re, v.im};
}

template <typename T>
__global__ void b_prep(const c128* __restrict__ x, cplx<T>* __restrict__ out, long long total,
                       const int* __restrict__ done) {
  if (done && *done) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const c128 v = x[e];
  out[e] = cplx<T>{(T)v.re, (T)v.im};
}

// y = x - t * (sum of partials) for the packed vector
template <typename T>
__global__ void b_combine(const cplx<T>* __restrict__ partial, const int* __restrict__ ibeg,
                          const SubParams* __restrict__ sp, int S, int R, int TW, int nxf, long long Nf,
                          const c128* __restrict__ x, const c128* __restrict__ t,
                          c128* __restrict__ y, long long total, const int* __restrict__ active,
                          const int* __restrict__ done, int SL, int NG) {
  if (done && *done) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int k = find_sub(sp, S, e, R);
  const SubParams p = sp[k];
  const long long Nk = (long long)p.nx * p.ny;
  long long q = e - p.vec_off;
  const int sl = (int)(q % SL);
  q /= SL;
  const long long site = q % Nk;
  q /= Nk;
  const int cls = (int)(q % NCLASS);
  const int r = (int)(q / NCLASS);
  if (active && !active[k * R + r]) return;
  const int slot = sl % SLOTS;
  const int sx = (int)(site % p.nx), sy = (int)(site / p.nx);
  const int tile = p.pad0 + (sy >> 4) * p.tiles_x + sx / TW;
  const int ls = (sy & 15) * TW + (sx % TW);
  // partial-sum row ((r * 2 + c) * NG + slot group)
  const int rc = (r * NCLASS + cls) * NG + sl / SLOTS;
  // the tile's items in a fixed order, eight loads in flight (deterministic)
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
  const long long fs = (long long)(p.oy + sy) * nxf + (p.ox + sx);
  const c128 tv = t[((long long)cls * Nf + fs) * SL + sl];
  const c128 xv = x[e];
  y[e] = c128{xv.re - (tv.re * sr - tv.im * si), xv.im - (tv.re * si + tv.im * sr)};
}

// partial[blk][k] = sum over the block's segment of conj(V_k) w, the
// vectors taken BKC at a time (one LDS reduction per chunk)
constexpr int BKC = 8;
__global__ __launch_bounds__(BT) void b_multidot(const c128* __restrict__ V, long long stride,
                                                 int nvec, const c128* __restrict__ w,
                                                 const SegBlock* __restrict__ blocks,
                                                 c128* __restrict__ partial, int ldp,
                                                 const int* __restrict__ active,
                                                 const int* __restrict__ done) {
  __shared__ double sh[BT / 64][2 * BKC];
  if (done && *done) return;
  const SegBlock bk = blocks[blockIdx.x];
  if (active && !active[bk.sys]) return;
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  for (int k0 = 0; k0 < nvec; k0 += BKC) {
    double sr[BKC], si[BKC];
#pragma unroll
    for (int i = 0; i < BKC; ++i) sr[i] = si[i] = 0.0;
    const int nk = min(BKC, nvec - k0);
    for (long long e = bk.lo + threadIdx.x; e < bk.hi; e += BT) {
      const c128 b = w[e];
#pragma unroll
      for (int i = 0; i < BKC; ++i) {
        if (i < nk) {
          const c128 a = V[(size_t)(k0 + i) * stride + e];
          sr[i] += a.re * b.re + a.im * b.im;
          si[i] += a.re * b.im - a.im * b.re;
        }
      }
    }
#pragma unroll
    for (int i = 0; i < BKC; ++i) {
      const double r = bwarp_sum(sr[i]), m = bwarp_sum(si[i]);
      if (ln == 0) {
        sh[wv][2 * i] = r;
        sh[wv][2 * i + 1] = m;
      }
    }
    __syncthreads();
    if (threadIdx.x < 2 * nk) {
      double s = 0.0;
      for (int q = 0; q < BT / 64; ++q) s += sh[q][threadIdx.x];
      reinterpret_cast<double*>(partial + (size_t)blockIdx.x * ldp + k0)[threadIdx.x] = s;
    }
    __syncthreads();
  }
}

// out[sys][k] = sum of the system's block partials (fixed order)
__global__ __launch_bounds__(BT) void b_reduce(const c128* __restrict__ partial, int ldp,
                                               const int* __restrict__ sys_blk, int nvec,
                                               c128* __restrict__ out, int ldo,
                                               const int* __restrict__ active,
                                               const int* __restrict__ done) {
  __shared__ double sh[BT / 64];
  if (done && *done) return;
  const int s = blockIdx.x;
  if (active && !active[s]) return;
  for (int k = 0; k < nvec; ++k) {
    double sr = 0.0, si = 0.0;
    for (int b = sys_blk[s] + threadIdx.x; b < sys_blk[s + 1]; b += BT) {
      const c128 v = partial[(size_t)b * ldp + k];
      sr += v.re;
      si += v.im;
    }
    sr = bblock_sum(sr, sh);
    si = bblock_sum(si, sh);
    if (threadIdx.x == 0) out[(size_t)s * ldo + k] = c128{sr, si};
  }
}

// w += sign * sum_k V_k h[sys][k]
__global__ __launch_bounds__(BT) void b_update(c128* __restrict__ w, const c128* __restrict__ V,
                                               long long stride, int nvec,
                                               const c128* __restrict__ h, int ldh, double sign,
                                               const SegBlock* __restrict__ blocks,
                                               const int* __restrict__ active,
                                               const int* __restrict__ done) {
  if (done && *done) return;
  const SegBlock bk = blocks[blockIdx.x];
  if (active && !active[bk.sys]) return;
  const c128* hs = h + (size_t)bk.sys * ldh;
  for (long long e = bk.lo + threadIdx.x; e < bk.hi; e += BT) {
    double sr = 0.0, si = 0.0;
    for (int k = 0; k < nvec; ++k) {
      const c128 v = V[(size_t)k * stride + e];
      const c128 c = hs[k];
      sr += v.re * c.re - v.im * c.im;
      si += v.re * c.im + v.im * c.re;
    }
    c128 o = w[e];
    o.re += sign * sr;
    o.im += sign * si;
    w[e] = o;
  }
}

__global__ __launch_bounds__(BT) void b_norm2(const c128* __restrict__ w,
                                              const SegBlock* __restrict__ blocks,
                                              double* __restrict__ partial,
                                              const int* __restrict__ active,
                                              const int* __restrict__ done) {
  __shared__ double sh[BT / 64];
  if (done && *done) return;
  const SegBlock bk = blocks[blockIdx.x];
  if (active && !active[bk.sys]) return;
  double s = 0.0;
  for (long long e = bk.lo + threadIdx.x; e < bk.hi; e += BT) {
    const c128 a = w[e];
    s += a.re * a.re + a.im * a.im;
  }
  s = bblock_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(BT) void b_norm_reduce(const double* __restrict__ partial,
                                                    const int* __restrict__ sys_blk,
                                                    double* __restrict__ out,
                                                    const int* __restrict__ active,
                                                    const int* __restrict__ done) {
  __shared__ double sh[BT / 64];
  if (done && *done) return;
  const int s = blockIdx.x;
  if (active && !active[s]) return;
  double v = 0.0;
  for (int b = sys_blk[s] + threadIdx.x; b < sys_blk[s + 1]; b += BT) v += partial[b];
  v = bblock_sum(v, sh);
  if (threadIdx.x == 0) out[s] = sqrt(v);
}

// y = x / d[sys] (0 where d is 0)
__global__ __launch_bounds__(BT) void b_scale(c128* __restrict__ y, const c128* __restrict__ x,
                                              const double* __restrict__ d,
                                              const SegBlock* __restrict__ blocks,
                                              const int* __restrict__ active,
                                              const int* __restrict__ done) {
  if (done && *done) return;
  const SegBlock bk = blocks[blockIdx.x];
  if (active && !active[bk.sys]) return;
  const double dv = d[bk.sys];
  const double f = dv > 0.0 ? 1.0 / dv : 0.0;
  for (long long e = bk.lo + threadIdx.x; e < bk.hi; e += BT) {
    const c128 v = x[e];
    y[e] = c128{f * v.re, f * v.im};
  }
}

// y = a - b
__global__ void b_sub(c128* __restrict__ y, const c128* __restrict__ a, const c128* __restrict__ b,
                      long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  y[e] = c128{a[e].re - b[e].re, a[e].im - b[e].im};
}

__global__ void b_fill(c128* __restrict__ y, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < total) y[e] = c128{0.0, 0.0};
}

// Givens state per system: H columns (rotated, [sys][m+1][m]), rotations,
// g, jend; one workgroup handles all systems.
struct zc {
  double re, im;
};
__device__ inline zc zmul(zc a, zc b) { return zc{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline zc zconj(zc a) { return zc{a.re, -a.im}; }
__device__ inline zc zadd(zc a, zc b) { return zc{a.re + b.re, a.im + b.im}; }
__device__ inline zc zsub(zc a, zc b) { return zc{a.re - b.re, a.im - b.im}; }
__device__ inline zc zneg(zc a) { return zc{-a.re, -a.im}; }
__device__ inline zc zscale(zc a, double f) { return zc{a.re * f, a.im * f}; }
__device__ inline double zabs2(zc a) { return a.re * a.re + a.im * a.im; }
__device__ inline zc zdiv(zc a, zc b) {
  const double d = zabs2(b);
  return zc{(a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d};
}
__device__ inline zc ld(c128 v) { return zc{v.re, v.im}; }
__device__ inline c128 stc(zc v) { return c128{v.re, v.im}; }

struct GivensState {
  c128 *H, *cs, *sn, *g, *d1, *d2;
  double *hn, *target;
  int *jend, *active, *done;
  int m, nsys, ldd;
};

__global__ __launch_bounds__(BT) void b_cycle_init(GivensState st, const double* __restrict__ beta,
                                                   const int* __restrict__ live) {
  __shared__ int any;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  for (int s = threadIdx.x; s < st.nsys; s += BT) {
    for (int i = 0; i <= st.m; ++i) st.g[(size_t)s * (st.m + 1) + i] = c128{0.0, 0.0};
    st.g[(size_t)s * (st.m + 1)] = c128{beta[s], 0.0};
    st.jend[s] = 0;
    const int a = live[s] && beta[s] > 0.0;
    st.active[s] = a;
    if (a) any = 1;  // benign race: every writer stores 1
  }
  __syncthreads();
  if (threadIdx.x == 0) st.done[0] = any ? 0 : 1;
}

__global__ __launch_bounds__(BT) void b_givens(GivensState st, int j) {
  __shared__ int any;
  if (st.done[0]) return;
  if (threadIdx.x == 0) any = 0;
  __syncthreads();
  const int m = st.m;
  for (int s = threadIdx.x; s < st.nsys; s += BT) {
    if (!st.active[s]) continue;
    c128* Hs = st.H + (size_t)s * (m + 1) * m;
    c128* cs = st.cs + (size_t)s * m;
    c128* sn = st.sn + (size_t)s * m;
    c128* g = st.g + (size_t)s * (m + 1);
    for (int i = 0; i <= j; ++i) {
      const c128 a = st.d1[(size_t)s * st.ldd + i], b = st.d2[(size_t)s * st.ldd + i];
      Hs[(size_t)i * m + j] = c128{a.re + b.re, a.im + b.im};
    }
    const double hn = st.hn[s];
    // previous rotations on column j (row j+1 entry is hn, real)
    for (int i = 0; i < j; ++i) {
      const zc hi = ld(Hs[(size_t)i * m + j]), hi1 = ld(Hs[(size_t)(i + 1) * m + j]);
      const zc c = ld(cs[i]), sv = ld(sn[i]);
      const zc t = zadd(zmul(zconj(c), hi), zmul(zconj(sv), hi1));
      Hs[(size_t)(i + 1) * m + j] = stc(zadd(zneg(zmul(sv, hi)), zmul(c, hi1)));
      Hs[(size_t)i * m + j] = stc(t);
    }
    const zc hjj = ld(Hs[(size_t)j * m + j]);
    const double den = sqrt(zabs2(hjj) + hn * hn);
    zc c{1.0, 0.0}, sv{0.0, 0.0};
    if (den > 0.0) {
      c = zscale(hjj, 1.0 / den);
      sv = zc{hn / den, 0.0};
    }
    cs[j] = stc(c);
    sn[j] = stc(sv);
    Hs[(size_t)j * m + j] = c128{den, 0.0};
    const zc gj = ld(g[j]);
    const zc gj1 = zneg(zmul(sv, gj));
    g[j + 1] = stc(gj1);
    g[j] = stc(zmul(zconj(c), gj));
    st.jend[s] = j + 1;
    const double est = sqrt(zabs2(gj1));
    if (est <= st.target[s] || hn == 0.0 || j + 1 == m) st.active[s] = 0;
    else any = 1;
  }
  __syncthreads();
  if (threadIdx.x == 0 && !any) st.done[0] = 1;
}

// y[sys] = R^{-1} g over the first jend columns (zero-padded to m)
__global__ void b_backsub(GivensState st, c128* __restrict__ y, const int* __restrict__ live) {
  const int s = blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= st.nsys) return;
  const int m = st.m;
  c128* ys = y + (size_t)s * m;
  for (int i = 0; i < m; ++i) ys[i] = c128{0.0, 0.0};
  if (!live[s]) return;
  const int je = st.jend[s];
  const c128* Hs = st.H + (size_t)s * (m + 1) * m;
  const c128* g = st.g + (size_t)s * (m + 1);
  for (int i = je - 1; i >= 0; --i) {
    zc acc = ld(g[i]);
    for (int q = i + 1; q < je; ++q) acc = zsub(acc, zmul(ld(Hs[(size_t)i * m + q]), ld(ys[q])));
    const zc d = ld(Hs[(size_t)i * m + i]);
    ys[i] = stc(zabs2(d) > 0.0 ? zdiv(acc, d) : zc{0.0, 0.0});
  }
}

// y = a - b on the segments of live systems
__global__ __launch_bounds__(BT) void b_sub_seg(c128* __restrict__ y, const c128* __restrict__ a,
                                                const c128* __restrict__ b,
                                                const SegBlock* __restrict__ blocks,
                                                const int* __restrict__ active) {
  const SegBlock bk = blocks[blockIdx.x];
  if (active && !active[bk.sys]) return;
  for (long long e = bk.lo + threadIdx.x; e < bk.hi; e += BT)
    y[e] = c128{a[e].re - b[e].re, a[e].im - b[e].im};
}

// ------------------------------------------------------------------ driver
struct Batch {
  int S = 0, R = 0, nsys = 0, m = 0, TW = 0;
  long long total = 0;
  std::vector<SubParams> subs;
  std::vector<long long> out_off;
  // device
  DevBuf d_sp[2], d_out_off, d_items[2], d_ibeg[2], d_blocks, d_sysblk;
  const SubParams* sp_cur = nullptr;  // subregion table of the precision in use
  std::vector<SubParams> sp_host[2];  // host copies per precision slot (0 FP64, 1 c64)
  int nitems[2] = {0, 0};
  int pf[2] = {1, 1};        // table prefetch depth of the LDS kernel per slot
  int items_tgt[2] = {0, 0};  // work items per (rhs, class) the plan was cut for
  int nblocks = 0;
  DevBuf b, x, r, w, V, xlow, partial, dots1, dots2, dpart, npart, hn, beta, bnorm, target, y;
  DevBuf H, cs, sn, g, jend, active, live, done;
  hipGraphExec_t graph[2] = {nullptr, nullptr};
  // graphs are captured and replayed on a private stream (the context stream
  // may be the legacy null stream, which cannot be captured), ordered with
  // the context stream by events
  hipStream_t side = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr;
  DevBuf a0full;
  hipStream_t ctx_stream = nullptr;
  // everything the batch allocated is freed here, on every exit path, after
  // the work queued on its streams has finished
  ~Batch() {
    if (ctx_stream) hipStreamSynchronize(ctx_stream);
    if (side) hipStreamSynchronize(side);
    for (int w = 0; w < 2; ++w)
      if (graph[w]) hipGraphExecDestroy(graph[w]);
    if (side) hipStreamDestroy(side);
    if (ev_in) hipEventDestroy(ev_in);
    if (ev_out) hipEventDestroy(ev_out);
    for (DevBuf* q : {&d_sp[0], &d_sp[1], &d_out_off, &d_items[0], &d_items[1], &d_ibeg[0], &d_ibeg[1],
                      &d_blocks, &d_sysblk, &b, &x, &r, &w, &V, &xlow, &partial, &dots1, &dots2, &dpart,
                      &npart, &hn, &beta, &bnorm, &target, &y, &H, &cs, &sn, &g, &jend, &active, &live,
                      &done, &a0full})
      release(*q);
  }
};

static int ensure_b(tm_ctx* c, DevBuf& b, size_t bytes) { return ensure(c, b, bytes); }

// Equal-work items over all subregions for precision slot w, about `target`
// items per (rhs, class) pair; the partial-sum buffer is grown to fit.
template <typename T>
static int plan_precision(tm_ctx* c, Batch& B, int w, int target) {
  int TW, BX, BY;
  lds_geometry<T>(TW, BX, BY);
  const std::vector<SubParams>& sp = B.sp_host[w];
  std::vector<std::vector<std::vector<double>>> wbs(B.S);
  double total = 0.0;
  for (int k = 0; k < B.S; ++k) total += lds_block_work(sp[k].nx, sp[k].ny, TW, BX, BY, 64, wbs[k]);
  std::vector<LdsItem> items;
  std::vector<int> ibeg;
  for (int k = 0; k < B.S; ++k) lds_split(wbs[k], total / target, k, items, ibeg);
  ibeg.push_back((int)items.size());
  int rc;
  if ((rc = ensure_b(c, B.d_items[w], items.size() * sizeof(LdsItem))) != TM_OK) return rc;
  if ((rc = ensure_b(c, B.d_ibeg[w], ibeg.size() * sizeof(int))) != TM_OK) return rc;
  TM_HIP(c, hipMemcpy(B.d_items[w].p, items.data(), items.size() * sizeof(LdsItem), hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy(B.d_ibeg[w].p, ibeg.data(), ibeg.size() * sizeof(int), hipMemcpyHostToDevice));
  B.nitems[w] = (int)items.size();
  B.items_tgt[w] = target;
  const size_t pbytes = (size_t)B.nitems[w] * 2 * B.R * c->g.NG * TW * 16 * SLOTS * sizeof(cplx<T>);
  return ensure_b(c, B.partial, pbytes);
}

static inline unsigned nbk(long long n) { return (unsigned)((n + BT - 1) / BT); }

// One application of the forward operator on the packed vector (precision
// slot w: 0 = FP64, 1 = complex64); `act` masks systems.
template <typename T>
static int b_apply(tm_ctx* c, Batch& B, const c128* xin, c128* yout, const int* act, const int* done) {
  const int w = std::is_same<T, double>::value ? 0 : 1;
  const void* src = xin;
  if (!std::is_same<T, double>::value) {
    hipLaunchKernelGGL(b_prep<T>, dim3(nbk(B.total)), dim3(BT), 0, c->stream, xin,
                       (cplx<T>*)B.xlow.p, B.total, done);
    src = B.xlow.p;
  }
  int rc = lds_launch<T>(c, w ? c->tab32.p : c->tab64.p, src, B.partial.p,
                         (const LdsItem*)B.d_items[w].p, B.nitems[w], B.R,
                         B.sp_cur, act, done, B.pf[w]);
  if (rc != TM_OK) return rc;
  hipLaunchKernelGGL(b_combine<T>, dim3(nbk(B.total)), dim3(BT), 0, c->stream,
                     (const cplx<T>*)B.partial.p, (const int*)B.d_ibeg[w].p,
                     B.sp_cur, B.S, B.R, B.TW, c->g.nx, (long long)c->g.n, xin,
                     (const c128*)c->t64.p, yout, B.total, act, done, c->g.S, c->g.NG);
  return TM_OK;
}

static GivensState gstate(Batch& B) {
  GivensState s;
  s.H = (c128*)B.H.p;
  s.cs = (c128*)B.cs.p;
  s.sn = (c128*)B.sn.p;
  s.g = (c128*)B.g.p;
  s.d1 = (c128*)B.dots1.p;
  s.d2 = (c128*)B.dots2.p;
  s.hn = (double*)B.hn.p;
  s.target = (double*)B.target.p;
  s.jend = (int*)B.jend.p;
  s.active = (int*)B.active.p;
  s.done = (int*)B.done.p;
  s.m = B.m;
  s.nsys = B.nsys;
  s.ldd = B.m + 1;
  return s;
}

// Arnoldi step j of every active system (enqueued; graph-capturable).
template <typename T>
static int b_step(tm_ctx* c, Batch& B, int j) {
  const long long L = B.total;
  c128* V = (c128*)B.V.p;
  const int* act = (const int*)B.active.p;
  const int* done = (const int*)B.done.p;
  const SegBlock* blk = (const SegBlock*)B.d_blocks.p;
  const int* sb = (const int*)B.d_sysblk.p;
  int rc = b_apply<T>(c, B, V + (size_t)j * L, (c128*)B.w.p, act, done);
  if (rc != TM_OK) return rc;
  const int ldp = B.m + 1;
  for (int pass = 0; pass < 2; ++pass) {
    c128* d = pass ? (c128*)B.dots2.p : (c128*)B.dots1.p;
    hipLaunchKernelGGL(b_multidot, dim3(B.nblocks), dim3(BT), 0, c->stream, V, L, j + 1,
                       (const c128*)B.w.p, blk, (c128*)B.dpart.p, ldp, act, done);
    hipLaunchKernelGGL(b_reduce, dim3(B.nsys), dim3(BT), 0, c->stream, (const c128*)B.dpart.p, ldp,
                       sb, j + 1, d, B.m + 1, act, done);
    hipLaunchKernelGGL(b_update, dim3(B.nblocks), dim3(BT), 0, c->stream, (c128*)B.w.p, V, L, j + 1,
                       (const c128*)d, B.m + 1, -1.0, blk, act, done);
  }
  hipLaunchKernelGGL(b_norm2, dim3(B.nblocks), dim3(BT), 0, c->stream, (const c128*)B.w.p, blk,
                     (double*)B.npart.p, act, done);
  hipLaunchKernelGGL(b_norm_reduce, dim3(B.nsys), dim3(BT), 0, c->stream, (const double*)B.npart.p,
                     sb, (double*)B.hn.p, act, done);
  hipLaunchKernelGGL(b_scale, dim3(B.nblocks), dim3(BT), 0, c->stream, V + (size_t)(j + 1) * L,
                     (const c128*)B.w.p, (const double*)B.hn.p, blk, act, done);
  hipLaunchKernelGGL(b_givens, dim3(1), dim3(BT), 0, c->stream, gstate(B), j);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

// per-system norms of a packed vector to host
static int b_norms(tm_ctx* c, Batch& B, const c128* v, const int* act, std::vector<double>& out) {
  const SegBlock* blk = (const SegBlock*)B.d_blocks.p;
  hipLaunchKernelGGL(b_norm2, dim3(B.nblocks), dim3(BT), 0, c->stream, v, blk, (double*)B.npart.p,
                     act, (const int*)nullptr);
  hipLaunchKernelGGL(b_norm_reduce, dim3(B.nsys), dim3(BT), 0, c->stream, (const double*)B.npart.p,
                     (const int*)B.d_sysblk.p, (double*)B.beta.p, act, (const int*)nullptr);
  out.assign(B.nsys, 0.0);
  TM_HIP(c, hipMemcpyAsync(out.data(), B.beta.p, B.nsys * sizeof(double), hipMemcpyDeviceToHost,
                           c->stream));
  TM_HIP(c, hipStreamSynchronize(c->stream));
  return TM_OK;
}

// Batched autotuner: one batched matvec with every system active per
// candidate (table prefetch depth x work split), the first launch of each
// untimed, the fastest kept.  Input and output are scratch vectors (the
// zeroed basis and w): timing does not depend on the values.
template <typename T>
static int b_autotune(tm_ctx* c, Batch& B) {
  const int w = std::is_same<T, double>::value ? 0 : 1;
  std::vector<int> ones(B.nsys, 1);
  TM_HIP(c, hipMemcpy(B.live.p, ones.data(), B.nsys * sizeof(int), hipMemcpyHostToDevice));
  hipEvent_t e0, e1;
  TM_HIP(c, hipEventCreate(&e0));
  if (hipEventCreate(&e1) != hipSuccess) {
    hipEventDestroy(e0);
    return set_err(c, TM_ERR_HIP, "event creation for the batched autotuner failed");
  }
  const int pfmax = w ? 3 : 2;
  const int wg_targets[] = {16384, 32768, 65536};
  float best = 1e30f;
  int best_pf = B.pf[w], best_tgt = B.items_tgt[w];
  int rc = TM_OK;
  bool timing_failed = false;
  for (int wg : wg_targets) {
    const int tgt = std::max(1, wg / (2 * B.R));
    if ((rc = plan_precision<T>(c, B, w, tgt)) != TM_OK) break;
    for (int pf = 1; pf <= pfmax && rc == TM_OK && !timing_failed; ++pf) {
      B.pf[w] = pf;
      float ms = 0.f;
      for (int rep = 0; rep < 2 && rc == TM_OK && !timing_failed; ++rep) {
        timing_failed = hipEventRecord(e0, c->stream) != hipSuccess;
        if (!timing_failed)
          rc = b_apply<T>(c, B, (const c128*)B.V.p, (c128*)B.w.p, (const int*)B.live.p, nullptr);
        if (rc == TM_OK && !timing_failed)
          timing_failed = hipEventRecord(e1, c->stream) != hipSuccess ||
                          hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess;
      }
      if (rc == TM_OK && !timing_failed && ms < best) {
        best = ms;
        best_pf = pf;
        best_tgt = tgt;
      }
    }
    if (timing_failed) break;
  }
  hipEventDestroy(e0);
  hipEventDestroy(e1);
  if (rc != TM_OK) return rc;
  if (timing_failed) return set_err(c, TM_ERR_HIP, "timing in the batched autotuner failed");
  B.pf[w] = best_pf;
  return plan_precision<T>(c, B, w, best_tgt);
}

template <typename T>
static int run_cycle(tm_ctx* c, Batch& B, bool use_graph, bool& graphed) {
  const int w = std::is_same<T, double>::value ? 0 : 1;
  graphed = false;
  if (use_graph && !B.side) {
    if (hipStreamCreateWithFlags(&B.side, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&B.ev_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&B.ev_out, hipEventDisableTiming) != hipSuccess)
      return set_err(c, TM_ERR_HIP, "stream/event creation for the batch graph failed");
  }
  if (use_graph) {
    if (!B.graph[w]) {
      // record the cycle's launches on the private stream: b_step enqueues on
      // c->stream, so point it there for the capture only
      hipGraph_t gph = nullptr;
      const hipStream_t ctx_stream = c->stream;
      c->stream = B.side;
      if (hipStreamBeginCapture(B.side, hipStreamCaptureModeThreadLocal) == hipSuccess) {
        int rc = TM_OK;
        for (int j = 0; j < B.m && rc == TM_OK; ++j) rc = b_step<T>(c, B, j);
        const hipError_t e = hipStreamEndCapture(B.side, &gph);
        if (rc == TM_OK && e == hipSuccess && gph) {
          if (hipGraphInstantiateWithFlags(&B.graph[w], gph, 0) != hipSuccess) B.graph[w] = nullptr;
        }
        if (gph) hipGraphDestroy(gph);
      }
      c->stream = ctx_stream;
      (void)hipGetLastError();
    }
    if (B.graph[w]) {
      TM_HIP(c, hipEventRecord(B.ev_in, c->stream));
      TM_HIP(c, hipStreamWaitEvent(B.side, B.ev_in, 0));
      TM_HIP(c, hipGraphLaunch(B.graph[w], B.side));
      TM_HIP(c, hipEventRecord(B.ev_out, B.side));
      TM_HIP(c, hipStreamWaitEvent(c->stream, B.ev_out, 0));
      graphed = true;
      return TM_OK;
    }
  }
  // eager: same launches, with a host check of the device flag between steps
  int* hdone = (int*)c->host_pinned;
  for (int j = 0; j < B.m; ++j) {
    int rc = b_step<T>(c, B, j);
    if (rc != TM_OK) return rc;
    TM_HIP(c, hipMemcpyAsync(hdone, B.done.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
    TM_HIP(c, hipStreamSynchronize(c->stream));
    if (*hdone) break;
  }
  return TM_OK;
}

static int batched_impl(tm_ctx* c, int S, const tm_subregion* subs, int R, const double* khat,
                        const tm_c128* pol, const tm_c128* a0_packed, tm_c128* s_out,
                        const tm_solve_opts& o, tm_solve_info* info, int use_graph) {
  const Geometry& g = c->g;
  Batch B;
  B.ctx_stream = c->stream;
  B.S = S;
  B.R = R;
  B.nsys = S * R;
  B.m = o.restart;
  int TW, BX, BY;
  lds_geometry<float>(TW, BX, BY);
  int TW64, BX64, BY64;
  lds_geometry<double>(TW64, BX64, BY64);
  long long off = 0, ooff = 0;
  int tile_base[2] = {0, 0};
  for (int k = 0; k < S; ++k) {
    const tm_subregion& q = subs[k];
    SubParams p{};
    p.nx = q.side_x;
    p.ny = q.side_y;
    p.ox = q.origin_x;
    p.oy = q.origin_y;
    p.vec_off = off;
    B.subs.push_back(p);
    B.out_off.push_back(ooff);
    off += (long long)R * NCLASS * p.nx * p.ny * g.S;
    ooff += (long long)R * p.nx * p.ny * g.L;
  }
  B.total = off;
  // tile bases differ per precision (tile width); keep both by uploading per apply
  int rc;
  // segmented blocks per system
  std::vector<SegBlock> blocks;
  std::vector<int> sysblk;
  for (int k = 0; k < S; ++k) {
    const long long len = (long long)NCLASS * B.subs[k].nx * B.subs[k].ny * g.S;
    for (int r = 0; r < R; ++r) {
      sysblk.push_back((int)blocks.size());
      const long long lo = B.subs[k].vec_off + (long long)r * len;
      for (long long e = lo; e < lo + len; e += SEG)
        blocks.push_back(SegBlock{k * R + r, 0, e, std::min(lo + len, e + SEG)});
    }
  }
  sysblk.push_back((int)blocks.size());
  B.nblocks = (int)blocks.size();
  const size_t cb = sizeof(c128);
  const long long Lt = B.total;
  const int m = B.m, ns = B.nsys;
  struct {
    DevBuf* b;
    size_t bytes;
  } allocs[] = {
      {&B.d_blocks, blocks.size() * sizeof(SegBlock)}, {&B.d_sysblk, sysblk.size() * sizeof(int)},
      {&B.d_out_off, (size_t)S * sizeof(long long)}, {&B.d_sp[0], (size_t)S * sizeof(SubParams)},
      {&B.d_sp[1], (size_t)S * sizeof(SubParams)},
      {&B.b, Lt * cb}, {&B.x, Lt * cb}, {&B.r, Lt * cb}, {&B.w, Lt * cb},
      {&B.V, (size_t)(m + 1) * Lt * cb}, {&B.xlow, Lt * sizeof(c64)},
      {&B.dots1, (size_t)ns * (m + 1) * cb}, {&B.dots2, (size_t)ns * (m + 1) * cb},
      {&B.dpart, (size_t)B.nblocks * (m + 1) * cb}, {&B.npart, (size_t)B.nblocks * sizeof(double)},
      {&B.hn, ns * sizeof(double)}, {&B.beta, ns * sizeof(double)}, {&B.bnorm, ns * sizeof(double)},
      {&B.target, ns * sizeof(double)}, {&B.y, (size_t)ns * m * cb},
      {&B.H, (size_t)ns * (m + 1) * m * cb}, {&B.cs, (size_t)ns * m * cb}, {&B.sn, (size_t)ns * m * cb},
      {&B.g, (size_t)ns * (m + 1) * cb}, {&B.jend, ns * sizeof(int)}, {&B.active, ns * sizeof(int)},
      {&B.live, ns * sizeof(int)}, {&B.done, sizeof(int) * 4},
  };
  for (auto& a : allocs)
    if ((rc = ensure_b(c, *a.b, a.bytes)) != TM_OK) return rc;
  TM_HIP(c, hipMemcpy(B.d_blocks.p, blocks.data(), blocks.size() * sizeof(SegBlock), hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy(B.d_sysblk.p, sysblk.data(), sysblk.size() * sizeof(int), hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy(B.d_out_off.p, B.out_off.data(), S * sizeof(long long), hipMemcpyHostToDevice));
  // plans for both precisions (tile widths differ): subregion params carry
  // the tile width and tile base of the precision in use, so keep two copies
  std::vector<SubParams> sp32 = B.subs, sp64 = B.subs;
  for (int k = 0; k < S; ++k) {
    sp32[k].tiles_x = (sp32[k].nx + TW - 1) / TW;
    sp32[k].pad0 = tile_base[1];
    tile_base[1] += sp32[k].tiles_x * ((sp32[k].ny + 15) / 16);
    sp64[k].tiles_x = (sp64[k].nx + TW64 - 1) / TW64;
    sp64[k].pad0 = tile_base[0];
    tile_base[0] += sp64[k].tiles_x * ((sp64[k].ny + 15) / 16);
  }
  TM_HIP(c, hipMemcpy(B.d_sp[1].p, sp32.data(), S * sizeof(SubParams), hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy(B.d_sp[0].p, sp64.data(), S * sizeof(SubParams), hipMemcpyHostToDevice));
  B.subs = sp32;
  B.sp_host[1] = sp32;
  B.sp_host[0] = sp64;
  // default launch configuration: many small equal-work items (the LDS kernel
  // runs best near one displacement block per workgroup, about 32k
  // workgroups per launch) and the context's prefetch depth
  for (int w = 0; w < 2; ++w) B.pf[w] = std::max(1, c->mv_variant[w] - 7);
  const int tgt0 = std::max(1, 32768 / (2 * R));
  if ((rc = plan_precision<float>(c, B, 1, tgt0)) != TM_OK) return rc;
  if ((rc = plan_precision<double>(c, B, 0, tgt0)) != TM_OK) return rc;
  if ((rc = ensure_pinned(c, 4096)) != TM_OK) return rc;
  auto use_sp = [&](int w) {
    B.sp_cur = (const SubParams*)B.d_sp[w].p;
    B.TW = w ? TW : TW64;
  };

  // right-hand side: plane waves on the full lattice, gathered and times T,
  // or the caller's per-subregion coefficients times T
  DevBuf& a0full = B.a0full;
  use_sp(1);
  if (a0_packed) {
    hipLaunchKernelGGL(b_gather_packed_rhs, dim3(nbk(Lt)), dim3(BT), 0, c->stream, a0_packed,
                       (const long long*)B.d_out_off.p, (const c128*)c->t64.p, B.sp_cur, S, R, g.nx,
                       (long long)g.n, c->maps, Lt, (c128*)B.b.p);
  } else {
    if ((rc = ensure_b(c, a0full, (size_t)R * g.n * g.L * cb)) != TM_OK) return rc;
    if ((rc = launch_plane_wave(c, R, khat, pol, (tm_c128*)a0full.p)) != TM_OK) return rc;
    hipLaunchKernelGGL(b_gather_rhs, dim3(nbk(Lt)), dim3(BT), 0, c->stream, (const tm_c128*)a0full.p,
                       (const c128*)c->t64.p, B.sp_cur, S, R, g.nx, (long long)g.n,
                       c->maps, Lt, (c128*)B.b.p);
  }
  std::vector<double> bn, beta;
  if ((rc = b_norms(c, B, (const c128*)B.b.p, nullptr, bn)) != TM_OK) return rc;
  release(a0full);
  hipLaunchKernelGGL(b_fill, dim3(nbk(Lt)), dim3(BT), 0, c->stream, (c128*)B.x.p, Lt);
  // basis vectors past a system's last Arnoldi step are multiplied by zero
  // coefficients in x += V y: they must hold finite values, so clear them once
  hipLaunchKernelGGL(b_fill, dim3(nbk((long long)(m + 1) * Lt)), dim3(BT), 0, c->stream, (c128*)B.V.p,
                     (long long)(m + 1) * Lt);
  TM_HIP(c, hipMemcpyAsync(B.r.p, B.b.p, Lt * cb, hipMemcpyDeviceToDevice, c->stream));
  // the Arnoldi precision's launch configuration, timed on this batch
  if (c->batch_autotune) {
    if (o.precision == TM_PREC_MIXED) {
      use_sp(1);
      rc = b_autotune<float>(c, B);
    } else {
      use_sp(0);
      rc = b_autotune<double>(c, B);
    }
    if (rc != TM_OK) return rc;
  }
  for (int w = 0; w < 2; ++w) {
    c->batch_pf[w] = (w == 0) ? std::min(B.pf[w], 2) : std::min(B.pf[w], 3);
    c->batch_items[w] = B.items_tgt[w];
  }
  // a system whose right-hand side or residual turns non-finite leaves the
  // batch with status TM_ERR_NAN; the others go on
  std::vector<int> live(ns, 1), iters(ns, 0), cycles(ns, 0), mv64(ns, 0), mvlo(ns, 0), bad(ns, 0);
  std::vector<double> relres(ns, 0.0);
  for (int s = 0; s < ns; ++s) {
    bad[s] = !std::isfinite(bn[s]);
    live[s] = !bad[s] && bn[s] > 0.0;
    relres[s] = live[s] ? 1.0 : (bad[s] ? NAN : 0.0);
  }
  const int prec = o.precision;
  bool any_graph = false;
  for (;;) {
    // residual norms of the systems still iterating; a converged system keeps
    // its last residual and leaves the batch (flags are uploaded only after
    // the stream has drained: earlier kernels read them)
    TM_HIP(c, hipStreamSynchronize(c->stream));
    TM_HIP(c, hipMemcpy(B.live.p, live.data(), ns * sizeof(int), hipMemcpyHostToDevice));
    if ((rc = b_norms(c, B, (const c128*)B.r.p, (const int*)B.live.p, beta)) != TM_OK) return rc;
    int nlive = 0;
    for (int s = 0; s < ns; ++s) {
      if (!live[s]) continue;
      relres[s] = beta[s] / bn[s];
      if (!std::isfinite(relres[s])) bad[s] = 1;
      if (bad[s] || relres[s] <= o.tol || iters[s] >= o.max_iter) live[s] = 0;
      nlive += live[s];
    }
    if (!nlive) break;
    if (c->progress) {
      double worst = 0.0;
      int cyc = 0, itmax = 0;
      for (int s = 0; s < ns; ++s) {
        itmax = std::max(itmax, iters[s]);
        cyc = std::max(cyc, cycles[s]);
        if (live[s]) worst = std::max(worst, relres[s]);
      }
      c->progress(c->progress_user, cyc, itmax, nlive, worst);
    }
    std::vector<double> tgt(ns, 0.0);
    for (int s = 0; s < ns; ++s) {
      if (!live[s]) continue;
      tgt[s] = (prec == TM_PREC_MIXED) ? std::max(o.tol * bn[s], o.inner_tol * beta[s]) : o.tol * bn[s];
      cycles[s]++;
    }
    TM_HIP(c, hipMemcpy(B.target.p, tgt.data(), ns * sizeof(double), hipMemcpyHostToDevice));
    TM_HIP(c, hipMemcpy(B.live.p, live.data(), ns * sizeof(int), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(b_cycle_init, dim3(1), dim3(BT), 0, c->stream, gstate(B),
                       (const double*)B.beta.p, (const int*)B.live.p);
    hipLaunchKernelGGL(b_scale, dim3(B.nblocks), dim3(BT), 0, c->stream, (c128*)B.V.p,
                       (const c128*)B.r.p, (const double*)B.beta.p, (const SegBlock*)B.d_blocks.p,
                       (const int*)B.live.p, (const int*)nullptr);
    bool graphed = false;
    if (prec == TM_PREC_MIXED) {
      use_sp(1);
      rc = run_cycle<float>(c, B, use_graph != 0, graphed);
    } else {
      use_sp(0);
      rc = run_cycle<double>(c, B, use_graph != 0, graphed);
    }
    if (rc != TM_OK) return rc;
    any_graph |= graphed;
    std::vector<int> je(ns);
    TM_HIP(c, hipMemcpyAsync(je.data(), B.jend.p, ns * sizeof(int), hipMemcpyDeviceToHost, c->stream));
    TM_HIP(c, hipStreamSynchronize(c->stream));
    int jmax = 0;
    for (int s = 0; s < ns; ++s) {
      if (!live[s]) continue;
      iters[s] += je[s];
      (prec == TM_PREC_MIXED ? mvlo : mv64)[s] += je[s];
      jmax = std::max(jmax, je[s]);
    }
    hipLaunchKernelGGL(b_backsub, dim3(nbk(ns)), dim3(BT), 0, c->stream, gstate(B), (c128*)B.y.p,
                       (const int*)B.live.p);
    if (jmax > 0)
      hipLaunchKernelGGL(b_update, dim3(B.nblocks), dim3(BT), 0, c->stream, (c128*)B.x.p,
                         (const c128*)B.V.p, Lt, jmax, (const c128*)B.y.p, m, 1.0,
                         (const SegBlock*)B.d_blocks.p, (const int*)B.live.p, (const int*)nullptr);
    // true residual in FP64 for the live systems
    use_sp(0);
    if ((rc = b_apply<double>(c, B, (const c128*)B.x.p, (c128*)B.w.p, (const int*)B.live.p,
                              (const int*)nullptr)) != TM_OK)
      return rc;
    for (int s = 0; s < ns; ++s)
      if (live[s]) mv64[s]++;
    hipLaunchKernelGGL(b_sub_seg, dim3(B.nblocks), dim3(BT), 0, c->stream, (c128*)B.r.p,
                       (const c128*)B.b.p, (const c128*)B.w.p, (const SegBlock*)B.d_blocks.p,
                       (const int*)B.live.p);
  }
  // output
  use_sp(1);
  hipLaunchKernelGGL(b_unpack, dim3(nbk(ooff)), dim3(BT), 0, c->stream, (const c128*)B.x.p,
                     B.sp_cur, (const long long*)B.d_out_off.p, S, R, c->maps,
                     ooff, s_out);
  TM_HIP(c, hipStreamSynchronize(c->stream));
  bool all_ok = true;
  for (int s = 0; s < ns; ++s) {
    info[s].status = bad[s] ? TM_ERR_NAN : (relres[s] <= o.tol ? TM_OK : TM_NOT_CONVERGED);
    info[s].iters = iters[s];
    info[s].cycles = cycles[s];
    info[s].matvecs_fp64 = mv64[s];
    info[s].matvecs_lowp = mvlo[s];
    info[s].rel_residual = relres[s];
    if (info[s].status != TM_OK) all_ok = false;
  }
  c->last_batch_graphed = any_graph ? 1 : 0;
  return all_ok ? TM_OK : TM_NOT_CONVERGED;
}

}  // namespace tmh

extern "C" int tm_set_batch_autotune(tm_ctx* c, int on) {
  if (!c) return TM_ERR_INVALID_ARG;
  c->batch_autotune = on ? 1 : 0;
  return TM_OK;
}

extern "C" int tm_get_batch_config(const tm_ctx* c, int precision, int* prefetch, int* items) {
  if (!c || !prefetch || !items || (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED))
    return TM_ERR_INVALID_ARG;
  const int w = precision == TM_PREC_MIXED ? 1 : 0;
  *prefetch = c->batch_pf[w];
  *items = c->batch_items[w];
  return TM_OK;
}

static int batched_entry(tm_ctx* c, int n_sub, const tm_subregion* subs, int n_rhs,
                         const double* khat, const tm_c128* pol, const tm_c128* a0_packed,
                         tm_c128* s_out, const tm_solve_opts* o, tm_solve_info* info, int use_graph) {
  if (!c) return TM_ERR_INVALID_ARG;
  hipSetDevice(c->device);
  if (!c->have_geom || !c->have_t) return tmh::set_err(c, TM_ERR_STATE, "geometry and T must be set");
  if (c->t_dense)
    return tmh::set_err(c, TM_ERR_STATE, "the batched solver takes diagonal T (spheres or tm_set_tmatrix_diag)");
  if (!c->g.lattice) return tmh::set_err(c, TM_ERR_NOT_LATTICE, "subregions need a lattice geometry");
  if (n_sub < 1 || n_rhs < 1 || n_rhs > 8 || !subs || (!a0_packed && (!khat || !pol)) || !s_out || !o ||
      !info)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if (!(o->tol > 0.0) || o->restart < 1 || o->restart > 200 || o->max_iter < 1 ||
      (o->precision != TM_PREC_FP64 && o->precision != TM_PREC_MIXED) ||
      (o->precision == TM_PREC_MIXED && !(o->inner_tol > 0.0 && o->inner_tol < 1.0)) || o->use_x0)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "invalid solver options (x0 not supported in batch)");
  int rc;
  if (!a0_packed && (rc = tmh::validate_incidence(c, n_rhs, khat, pol)) != TM_OK) return rc;
  for (int k = 0; k < n_sub; ++k) {
    const tm_subregion& q = subs[k];
    if (q.side_x < 1 || q.side_y < 1 || q.origin_x < 0 || q.origin_y < 0 ||
        q.origin_x + q.side_x > c->g.nx || q.origin_y + q.side_y > c->g.ny)
      return tmh::set_err(c, TM_ERR_INVALID_ARG, "subregion " + std::to_string(k) + " outside the lattice");
  }
  return tmh::batched_impl(c, n_sub, subs, n_rhs, khat, pol, a0_packed, s_out, *o, info, use_graph);
}

extern "C" int tm_solve_batched(tm_ctx* c, int n_sub, const tm_subregion* subs, int n_rhs,
                                const double* khat, const tm_c128* pol, tm_c128* s_out,
                                const tm_solve_opts* o, tm_solve_info* info, int use_graph) {
  if (!khat || !pol) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  return batched_entry(c, n_sub, subs, n_rhs, khat, pol, nullptr, s_out, o, info, use_graph);
}

extern "C" int tm_solve_batched_a0(tm_ctx* c, int n_sub, const tm_subregion* subs, int n_rhs,
                                   const tm_c128* a0, tm_c128* s_out, const tm_solve_opts* o,
                                   tm_solve_info* info, int use_graph) {
  if (!a0) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  return batched_entry(c, n_sub, subs, n_rhs, nullptr, nullptr, a0, s_out, o, info, use_graph);
}

extern "C" int tm_batch_graph_used(const tm_ctx* c) { return c ? c->last_batch_graphed : 0; }
