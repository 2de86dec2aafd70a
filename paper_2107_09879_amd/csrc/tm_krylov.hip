// Krylov-subspace vector kernels for GMRES (App. I.D: the non-matvec GMRES
// operations) and conversions between the boundary layout [rhs][site][n] and
// the internal class/slot layout.  All FP64; reductions are two-stage with a
// fixed assignment of elements to blocks and a fixed combine order, so every
// result is reproducible run to run.
#include "tm_internal.h"

namespace tmh {

constexpr int KB = 256;  // threads per block for vector kernels

int krylov_blocks(long long len) {
  long long b = (len + KB - 1) / KB;
  if (b > 2048) b = 2048;
  if (b < 1) b = 1;
  return (int)b;
}

__device__ inline double warp_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// block-wide sum of a double, result valid in thread 0
__device__ inline double block_sum(double v, double* sh) {
  v = warp_sum(v);
  const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
  if (l == 0) sh[w] = v;
  __syncthreads();
  double r = 0.0;
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) r += sh[i];
  __syncthreads();
  return r;
}

// partial[seg][k] = sum over segment seg of conj(V_k) w (a tall-skinny V^H w,
// bound by reading V once).  Grid (segments, chunks of KC vectors): a block
// streams its whole segment for its KC vectors, each thread keeping KC
// complex sums, and reduces the 2*KC sums once at the end.  Few enough
// segments that every thread walks many elements keeps the loads in flight
// instead of spending the block in reductions.
constexpr int KC = 8;
__global__ __launch_bounds__(KB) void multidot_kernel(const c128* __restrict__ V, long long stride,
                                                      int nvec, const c128* __restrict__ w,
                                                      long long len, c128* __restrict__ partial,
                                                      const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64][2 * KC];
  const long long per = (len + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = min(len, lo + per);
  const int wv = threadIdx.x >> 6, ln = threadIdx.x & 63;
  const int k0 = blockIdx.y * KC;
  const int nk = min(KC, nvec - k0);
  const c128* Vk = V + (size_t)k0 * stride;
  double sr[KC], si[KC];
#pragma unroll
  for (int i = 0; i < KC; ++i) sr[i] = si[i] = 0.0;
  if (nk == KC) {
#pragma unroll 2
    for (long long e = lo + threadIdx.x; e < hi; e += KB) {
      const c128 b = w[e];
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        const c128 a = Vk[(size_t)i * stride + e];
        sr[i] += a.re * b.re + a.im * b.im;
        si[i] += a.re * b.im - a.im * b.re;
      }
    }
  } else {
    for (long long e = lo + threadIdx.x; e < hi; e += KB) {
      const c128 b = w[e];
#pragma unroll
      for (int i = 0; i < KC; ++i) {
        if (i < nk) {
          const c128 a = Vk[(size_t)i * stride + e];
          sr[i] += a.re * b.re + a.im * b.im;
          si[i] += a.re * b.im - a.im * b.re;
        }
      }
    }
  }
#pragma unroll
  for (int i = 0; i < KC; ++i) {
    const double r = warp_sum(sr[i]), m = warp_sum(si[i]);
    if (ln == 0) {
      sh[wv][2 * i] = r;
      sh[wv][2 * i + 1] = m;
    }
  }
  __syncthreads();
  if (threadIdx.x < 2 * nk) {
    double s = 0.0;
    for (int q = 0; q < KB / 64; ++q) s += sh[q][threadIdx.x];
    double* out = reinterpret_cast<double*>(partial + (size_t)blockIdx.x * nvec + k0);
    out[threadIdx.x] = s;
  }
}

// Segments of a multidot over nvec vectors: about 2048 blocks in all, at
// most nblk segments (the rows of the partial-sum buffer).  Depends only on
// (len, nvec, nblk), so the reduction order is fixed for a given step.
int multidot_segments(long long len, int nvec, int nblk) {
  const int nch = (nvec + KC - 1) / KC;
  long long seg = (2048 + nch - 1) / nch;
  const long long by_len = (len + 4 * KB - 1) / (4 * KB);  // >= 4 elements per thread
  if (seg > by_len) seg = by_len;
  if (seg > nblk) seg = nblk;
  if (seg < 1) seg = 1;
  return (int)seg;
}

// out[k] = sum_blk partial[blk][k] (+ add[k]); one block per k
__global__ __launch_bounds__(KB) void reduce_dots_kernel(const c128* __restrict__ partial,
                                                         int nblk, int nvec, c128* __restrict__ out,
                                                         const c128* __restrict__ add,
                                                         const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64];
  const int k = blockIdx.x;
  double sr = 0.0, si = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) {
    const c128 v = partial[(size_t)b * nvec + k];
    sr += v.re;
    si += v.im;
  }
  sr = block_sum(sr, sh);
  si = block_sum(si, sh);
  if (threadIdx.x == 0) {
    if (add) {
      sr += add[k].re;
      si += add[k].im;
    }
    out[k] = c128{sr, si};
  }
}

// w += sign * sum_k V_k h_k (the loop over k unrolled so that several
// vectors' loads are in flight per thread)
__global__ void update_kernel(c128* __restrict__ w, const c128* __restrict__ V, long long stride,
                              int nvec, const c128* __restrict__ h, long long len, double sign,
                              const int* __restrict__ stop) {
  if (stop && *stop) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  double sr = 0.0, si = 0.0;
#pragma unroll 8
  for (int k = 0; k < nvec; ++k) {
    const c128 v = V[(size_t)k * stride + e];
    const c128 c = h[k];
    sr += v.re * c.re - v.im * c.im;
    si += v.re * c.im + v.im * c.re;
  }
  c128 o = w[e];
  o.re += sign * sr;
  o.im += sign * si;
  w[e] = o;
}

__global__ __launch_bounds__(KB) void norm2_partial_kernel(const c128* __restrict__ w, long long len,
                                                           double* __restrict__ partial,
                                                           const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64];
  const long long per = (len + gridDim.x - 1) / gridDim.x;
  const long long lo = (long long)blockIdx.x * per;
  const long long hi = min(len, lo + per);
  double s = 0.0;
  for (long long e = lo + threadIdx.x; e < hi; e += blockDim.x) {
    const c128 a = w[e];
    s += a.re * a.re + a.im * a.im;
  }
  s = block_sum(s, sh);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ __launch_bounds__(KB) void reduce_norm_kernel(const double* __restrict__ partial, int nblk,
                                                         double* __restrict__ out,
                                                         const int* __restrict__ stop) {
  if (stop && *stop) return;
  __shared__ double sh[KB / 64];
  double s = 0.0;
  for (int b = threadIdx.x; b < nblk; b += blockDim.x) s += partial[b];
  s = block_sum(s, sh);
  if (threadIdx.x == 0) out[0] = sqrt(s);
}

__global__ void scale_kernel(c128* __restrict__ y, const c128* __restrict__ x, double a,
                             long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const c128 v = x[e];
  y[e] = c128{a * v.re, a * v.im};
}

__global__ void sub_kernel(c128* __restrict__ out, const c128* __restrict__ a,
                           const c128* __restrict__ b, long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  out[e] = c128{a[e].re - b[e].re, a[e].im - b[e].im};
}

__global__ void add_kernel(c128* __restrict__ out, const c128* __restrict__ a,
                           const c128* __restrict__ b, long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  out[e] = c128{a[e].re + b[e].re, a[e].im + b[e].im};
}

__global__ void copy_kernel(c128* __restrict__ out, const c128* __restrict__ in, long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  out[e] = in[e];
}

__global__ void mul_t_kernel(c128* __restrict__ out, const c128* __restrict__ t,
                             const c128* __restrict__ x, long long vec, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const c128 a = t[e % vec], b = x[e];
  out[e] = c128{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re};
}

// boundary [R][N][L] -> slot [R][2][N][S]
__global__ void pack_kernel(const tm_c128* __restrict__ in, c128* __restrict__ out, SlotMaps m,
                            long long N, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int slot = (int)(e % m.S);
  const long long site = (e / m.S) % N;
  const int cls = (int)((e / (m.S * N)) % NCLASS);
  const long long r = e / (m.S * N * NCLASS);
  const int n = m.n_of[cls][slot];
  c128 v{0.0, 0.0};
  if (n >= 0) {
    const tm_c128 a = in[(r * N + site) * m.L + n];
    v = c128{a.re, a.im};
  }
  out[e] = v;
}

// slot [R][2][N][S] -> boundary [R][N][L]
__global__ void unpack_kernel(const c128* __restrict__ in, tm_c128* __restrict__ out, SlotMaps m,
                              long long N, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int n = (int)(e % m.L);
  const long long site = (e / m.L) % N;
  const long long r = e / (m.L * N);
  const c128 v = in[((r * NCLASS + m.cls_of[n]) * N + site) * m.S + m.slot_of[n]];
  out[e] = tm_c128{v.re, v.im};
}

static inline unsigned nb_of(long long n) { return (unsigned)((n + KB - 1) / KB); }

void pack_slots(hipStream_t st, const Geometry& g, const SlotMaps& m, int R, const tm_c128* in,
                c128* out) {
  const long long total = g.vec_len() * R;
  hipLaunchKernelGGL(pack_kernel, dim3(nb_of(total)), dim3(KB), 0, st, in, out, m,
                     (long long)g.n, total);
}
void unpack_slots(hipStream_t st, const Geometry& g, const SlotMaps& m, int R, const c128* in,
                  tm_c128* out) {
  const long long total = (long long)R * g.n * g.L;
  hipLaunchKernelGGL(unpack_kernel, dim3(nb_of(total)), dim3(KB), 0, st, in, out, m,
                     (long long)g.n, total);
}
int k_multidot(hipStream_t st, const c128* V, long long stride, int nvec, const c128* w,
               long long len, c128* partial, int nblk, const int* stop) {
  const int nseg = multidot_segments(len, nvec, nblk);
  hipLaunchKernelGGL(multidot_kernel, dim3(nseg, (nvec + KC - 1) / KC), dim3(KB), 0, st, V, stride,
                     nvec, w, len, partial, stop);
  return nseg;
}
void k_reduce_dots(hipStream_t st, const c128* partial, int nblk, int nvec, c128* out,
                   const c128* add, const int* stop) {
  hipLaunchKernelGGL(reduce_dots_kernel, dim3(nvec), dim3(KB), 0, st, partial, nblk, nvec, out,
                     add, stop);
}
void k_update(hipStream_t st, c128* w, const c128* V, long long stride, int nvec, const c128* h,
              long long len, double sign, const int* stop) {
  hipLaunchKernelGGL(update_kernel, dim3(nb_of(len)), dim3(KB), 0, st, w, V, stride, nvec, h, len,
                     sign, stop);
}
void k_norm2_partial(hipStream_t st, const c128* w, long long len, double* partial, int nblk,
                     const int* stop) {
  hipLaunchKernelGGL(norm2_partial_kernel, dim3(nblk), dim3(KB), 0, st, w, len, partial, stop);
}
void k_reduce_norm(hipStream_t st, const double* partial, int nblk, double* out, const int* stop) {
  hipLaunchKernelGGL(reduce_norm_kernel, dim3(1), dim3(KB), 0, st, partial, nblk, out, stop);
}
void k_scale(hipStream_t st, c128* y, const c128* x, double a, long long len) {
  hipLaunchKernelGGL(scale_kernel, dim3(nb_of(len)), dim3(KB), 0, st, y, x, a, len);
}
void k_axpy_dev(hipStream_t st, c128* y, const c128* x, const c128* V, long long stride, int nvec,
                const c128* coef, long long len) {
  (void)x;
  hipLaunchKernelGGL(update_kernel, dim3(nb_of(len)), dim3(KB), 0, st, y, V, stride, nvec, coef,
                     len, 1.0, (const int*)nullptr);
}
void k_sub(hipStream_t st, c128* out, const c128* a, const c128* b, long long len) {
  hipLaunchKernelGGL(sub_kernel, dim3(nb_of(len)), dim3(KB), 0, st, out, a, b, len);
}
void k_add(hipStream_t st, c128* out, const c128* a, const c128* b, long long len) {
  hipLaunchKernelGGL(add_kernel, dim3(nb_of(len)), dim3(KB), 0, st, out, a, b, len);
}
void k_copy(hipStream_t st, c128* out, const c128* in, long long len) {
  hipLaunchKernelGGL(copy_kernel, dim3(nb_of(len)), dim3(KB), 0, st, out, in, len);
}
void k_mul_t(hipStream_t st, c128* out, const c128* t, const c128* x, long long len_per_rhs,
             int R) {
  const long long total = len_per_rhs * R;
  hipLaunchKernelGGL(mul_t_kernel, dim3(nb_of(total)), dim3(KB), 0, st, out, t, x, len_per_rhs,
                     total);
}

// ---------------------------------------------------------------- GMRES
// One restarted cycle's Hessenberg reduction on the device (one thread: the
// work per step is O(j) complex operations).  The rotations follow the host
// form they replace: G_i = [[conj(c), conj(s)], [-s, c]] with
// c = H(j,j)/d, s = H(j+1,j)/d, d = sqrt(|H(j,j)|^2 + |H(j+1,j)|^2).
struct GmView {
  GmFlags* f;
  c128 *H, *cs, *sn, *g, *y;
};
__host__ __device__ inline size_t gm_off_H() { return 64; }
__host__ __device__ inline GmView gm_view(void* state, int m) {
  char* b = static_cast<char*>(state);
  GmView v;
  v.f = reinterpret_cast<GmFlags*>(b);
  v.H = reinterpret_cast<c128*>(b + gm_off_H());
  v.cs = v.H + (size_t)(m + 1) * m;
  v.sn = v.cs + m;
  v.g = v.sn + m;
  v.y = v.g + (m + 1);
  return v;
}
size_t gm_state_bytes(int m) {
  return gm_off_H() + ((size_t)(m + 1) * m + 2 * (size_t)m + (m + 1) + m) * sizeof(c128);
}
const c128* gm_y(const void* state, int m) { return gm_view(const_cast<void*>(state), m).y; }

__device__ inline double cabs(c128 a) { return hypot(a.re, a.im); }
__device__ inline c128 cmul(c128 a, c128 b) { return c128{a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ inline c128 cconj(c128 a) { return c128{a.re, -a.im}; }
__device__ inline c128 cadd(c128 a, c128 b) { return c128{a.re + b.re, a.im + b.im}; }
__device__ inline c128 csubc(c128 a, c128 b) { return c128{a.re - b.re, a.im - b.im}; }
__device__ inline c128 cdiv(c128 a, c128 b) {
  // Smith's algorithm (scaled by the larger component of b)
  if (fabs(b.re) >= fabs(b.im)) {
    const double r = b.im / b.re, d = b.re + b.im * r;
    return c128{(a.re + a.im * r) / d, (a.im - a.re * r) / d};
  }
  const double r = b.re / b.im, d = b.re * r + b.im;
  return c128{(a.re * r + a.im) / d, (a.im * r - a.re) / d};
}

__global__ void gm_cycle_init_kernel(void* state, int m, const double* __restrict__ beta) {
  GmView v = gm_view(state, m);
  for (int i = threadIdx.x; i <= m; i += blockDim.x) v.g[i] = c128{i == 0 ? beta[0] : 0.0, 0.0};
  if (threadIdx.x == 0) {
    v.f->stop = 0;
    v.f->jend = 0;
    v.f->nonfinite = 0;
    v.f->inv_hn = 0.0;
    v.f->est = beta[0];
  }
}

__global__ void gm_givens_kernel(void* state, int m, int j, const c128* __restrict__ h1,
                                 const c128* __restrict__ h2, const double* __restrict__ hn,
                                 double target) {
  if (threadIdx.x != 0) return;
  GmView v = gm_view(state, m);
  if (v.f->stop) return;
  auto Hij = [&](int i, int k) -> c128& { return v.H[(size_t)i * m + k]; };
  const double h = hn[0];
  for (int i = 0; i <= j; ++i) Hij(i, j) = cadd(h1[i], h2[i]);
  Hij(j + 1, j) = c128{h, 0.0};
  if (!isfinite(h)) {
    v.f->nonfinite = 1;
    v.f->stop = 1;
    return;
  }
  for (int i = 0; i < j; ++i) {
    const c128 a = Hij(i, j), b = Hij(i + 1, j);
    const c128 t = cadd(cmul(cconj(v.cs[i]), a), cmul(cconj(v.sn[i]), b));
    Hij(i + 1, j) = csubc(cmul(v.cs[i], b), cmul(v.sn[i], a));
    Hij(i, j) = t;
  }
  const double den = hypot(cabs(Hij(j, j)), cabs(Hij(j + 1, j)));
  if (den == 0.0) {
    v.cs[j] = c128{1.0, 0.0};
    v.sn[j] = c128{0.0, 0.0};
  } else {
    v.cs[j] = c128{Hij(j, j).re / den, Hij(j, j).im / den};
    v.sn[j] = c128{Hij(j + 1, j).re / den, Hij(j + 1, j).im / den};
  }
  Hij(j, j) = c128{den, 0.0};
  Hij(j + 1, j) = c128{0.0, 0.0};
  const c128 gj = v.g[j];
  v.g[j + 1] = c128{-(v.sn[j].re * gj.re - v.sn[j].im * gj.im), -(v.sn[j].re * gj.im + v.sn[j].im * gj.re)};
  v.g[j] = cmul(cconj(v.cs[j]), gj);
  v.f->jend = j + 1;
  v.f->est = cabs(v.g[j + 1]);
  v.f->inv_hn = h > 0.0 ? 1.0 / h : 0.0;
  if (!isfinite(v.f->est)) v.f->nonfinite = 1;
  if (v.f->est <= target || h == 0.0 || v.f->nonfinite) v.f->stop = 1;
}

// v = w / H(j+1, j) unless the cycle has stopped
__global__ void gm_scale_next_kernel(c128* __restrict__ vnext, const c128* __restrict__ w,
                                     const GmFlags* __restrict__ f, long long len) {
  if (f->stop) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  const double a = f->inv_hn;
  const c128 x = w[e];
  vnext[e] = c128{a * x.re, a * x.im};
}

// y = H(0:jend, 0:jend)^-1 g(0:jend), zeros past jend
__global__ void gm_backsub_kernel(void* state, int m) {
  if (threadIdx.x != 0) return;
  GmView v = gm_view(state, m);
  const int jend = v.f->jend;
  for (int i = m - 1; i >= jend; --i) v.y[i] = c128{0.0, 0.0};
  for (int i = jend - 1; i >= 0; --i) {
    c128 s = v.g[i];
    for (int q = i + 1; q < jend; ++q) s = csubc(s, cmul(v.H[(size_t)i * m + q], v.y[q]));
    const c128 d = v.H[(size_t)i * m + i];
    v.y[i] = (d.re != 0.0 || d.im != 0.0) ? cdiv(s, d) : c128{0.0, 0.0};
  }
}

// x += sum_{k < jend} V_k y_k (jend from the device flags: basis vectors of
// the steps after the stop were never formed)
__global__ void gm_update_x_kernel(c128* __restrict__ x, const c128* __restrict__ V, long long stride,
                                   const void* __restrict__ state, int m, long long len) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= len) return;
  GmView v = gm_view(const_cast<void*>(state), m);
  const int nvec = v.f->jend;
  double sr = 0.0, si = 0.0;
  for (int k = 0; k < nvec; ++k) {
    const c128 a = V[(size_t)k * stride + e];
    const c128 c = v.y[k];
    sr += a.re * c.re - a.im * c.im;
    si += a.re * c.im + a.im * c.re;
  }
  c128 o = x[e];
  o.re += sr;
  o.im += si;
  x[e] = o;
}

void k_gm_update_x(hipStream_t st, c128* x, const c128* V, long long len, const void* state, int m) {
  hipLaunchKernelGGL(gm_update_x_kernel, dim3(nb_of(len)), dim3(KB), 0, st, x, V, len, state, m, len);
}

void k_gm_cycle_init(hipStream_t st, void* state, int m, const double* beta) {
  hipLaunchKernelGGL(gm_cycle_init_kernel, dim3(1), dim3(KB), 0, st, state, m, beta);
}
void k_gm_givens(hipStream_t st, void* state, int m, int j, const c128* h1, const c128* h2,
                 const double* hn, double target) {
  hipLaunchKernelGGL(gm_givens_kernel, dim3(1), dim3(64), 0, st, state, m, j, h1, h2, hn, target);
}
void k_gm_scale_next(hipStream_t st, c128* v, const c128* w, const void* state, long long len) {
  hipLaunchKernelGGL(gm_scale_next_kernel, dim3(nb_of(len)), dim3(KB), 0, st, v, w,
                     (const GmFlags*)state, len);
}
void k_gm_backsub(hipStream_t st, void* state, int m) {
  hipLaunchKernelGGL(gm_backsub_kernel, dim3(1), dim3(64), 0, st, state, m);
}

}  // namespace tmh
