// Block matvec for scatterers at arbitrary positions in the z = 0 plane: the
// translation blocks are formed on the fly per (target, source) pair instead
// of being read from a per-displacement table (the paper's own GPU matvec
// computes matrix elements on the fly, App. I.D).  For a pair with
// d = x_t - x_s (r = |d|, azimuth phi) and every entry (i, j) of a z-mirror
// class block,
//   M_ij(d) = e^{i dm_ij phi} sum_q C_ijq h_q(k r)
// (App. I.C, eq. "tran_coeff", the Legendre factor at theta = pi/2 folded into
// C), and z_t = sum_{s != t} M(x_t - x_s) x_s.  The transposed operator uses
// (A^T)_ts = M(x_s - x_t)^T.
//
// One thread per target; the workgroups of a launch split the sources into
// chunks (blockIdx.z) whose partial sums a combine kernel adds in chunk order
// (deterministic).  Sources of a chunk are staged through LDS in groups; the
// coefficient loop is uniform across the wave, so its constants are scalar
// loads.  Arithmetic in T (FP64, or FP32 for the mixed path with k r reduced
// modulo 2 pi in FP64 before the FP32 sine and cosine).
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "tm_internal.h"

namespace tmh {

constexpr int OL_THREADS = 256;
constexpr int OL_GROUP = 64;  // sources staged per LDS pass

// h_q(kr), q = 0..Q-1 (Q >= 3 a template argument), by upward recurrence from
// h_0 and h_1, with k r reduced modulo 2 pi in FP64 before the sine and cosine
template <typename T, int Q>
__device__ inline void ol_hankel_fixed(double kr, T* hr, T* hi) {
  const double twopi = 6.283185307179586476925286766559;
  const double red = kr - twopi * rint(kr / twopi);
  T s, c;
  if (sizeof(T) == 4) {
    float sf, cf;
    sincosf((float)red, &sf, &cf);
    s = (T)sf;
    c = (T)cf;
  } else {
    double sd, cd;
    sincos(red, &sd, &cd);
    s = (T)sd;
    c = (T)cd;
  }
  const T x = (T)kr, ix = (T)1 / x;
  hr[0] = s * ix;
  hi[0] = -c * ix;
  hr[1] = -(c * x - s) * ix * ix;
  hi[1] = -(s * x + c) * ix * ix;
#pragma unroll
  for (int q = 1; q < Q - 1; ++q) {
    const T f = (T)(2 * q + 1) * ix;
    hr[q + 1] = f * hr[q] - hr[q - 1];
    hi[q + 1] = f * hi[q] - hi[q - 1];
  }
}

// partial[chunk][r][c][t][S] = sum over the chunk's sources of M x_s (or M^T).
// The same product for lmax <= 3 with every loop over coefficients unrolled
// (lmax a template argument): the Hankel values, phases, the source vector
// and the output accumulators sit in registers at fixed places and the
// constants (in T: the complex64 kernel reads an FP32 copy) are scalar loads
// at fixed offsets.  The phase of an entry is split as
//   e^{i (m_j - m_i) phi} = e^{i d_j phi} e^{-i d_i phi},  d_j = m_j - m_0
// (d_j = dm[c][0][j]): the source vector is rotated once per (pair, j) and
// the sum over j once per (pair, i), instead of once per entry.  For the
// transposed operator (entry (j, i), displacement source - target) the two
// rotations change sign; the operator is a template argument, so that the
// constants of every entry sit at fixed offsets from one base.
// a * b + c in one rounding (the sums below are written as chains of these,
// which the compiler does not form on its own from a*b - c*d + e)
template <typename T>
__device__ inline T ol_fma(T a, T b, T c) {
  if constexpr (sizeof(T) == 4)
    return __builtin_fmaf(a, b, c);
  else
    return __builtin_fma(a, b, c);
}

template <typename T, int Q>
__device__ inline void ol_rot(const T* er, const T* ei, int d, T& pr, T& pi) {
  const int ad = d < 0 ? -d : d;
  pr = er[0];
  pi = ei[0];
#pragma unroll
  for (int u = 1; u < Q; ++u)
    if (u == ad) {
      pr = er[u];
      pi = ei[u];
    }
  if (d < 0) pi = -pi;
}

template <typename T, int LMAX, bool TR>
__global__ __launch_bounds__(OL_THREADS) void offlattice_small_kernel(
    const double* __restrict__ xy, const cplx<T>* __restrict__ x, const T* __restrict__ coef,
    const int* __restrict__ dm, int N, double k, int chunk, cplx<T>* __restrict__ partial,
    const int* __restrict__ stop) {
  constexpr int Q = 2 * LMAX + 1;           // Hankel orders and phase powers
  constexpr int NH = LMAX * (LMAX + 2);     // members of a class
  constexpr int S = 16 * ((NH + 15) / 16);  // slots of a class
  if (stop && *stop) return;  // a stopped GMRES cycle
  extern __shared__ double ol_lds[];
  double* sxy = ol_lds;                                            // [OL_GROUP][2]
  cplx<T>* sx = reinterpret_cast<cplx<T>*>(ol_lds + 2 * OL_GROUP);  // [OL_GROUP][S]
  const int t = blockIdx.x * OL_THREADS + threadIdx.x;
  const int rc = blockIdx.y;  // r * 2 + c
  const int c = rc & 1;
  const int s0 = blockIdx.z * chunk, s1 = min(N, s0 + chunk);
  const bool live = t < N;
  const double xt = live ? xy[2 * t] : 0.0, yt = live ? xy[2 * t + 1] : 0.0;
  const cplx<T>* xin = x + (size_t)rc * N * S;
  const T* cf = coef + (size_t)c * S * S * Q * 2;
  const int* dmc = dm + (size_t)c * S * S;
  const int sg = TR ? -1 : 1;
  int d[NH];
#pragma unroll
  for (int j = 0; j < NH; ++j) d[j] = sg * dmc[j];  // +-(m_j - m_0)
  T yr[NH], yi[NH];
#pragma unroll
  for (int i = 0; i < NH; ++i) yr[i] = yi[i] = (T)0;
  for (int g0 = s0; g0 < s1; g0 += OL_GROUP) {
    const int ng = min(OL_GROUP, s1 - g0);
    __syncthreads();
    for (int q = threadIdx.x; q < ng * S; q += OL_THREADS) {
      const int ss = q / S, j = q % S;
      sx[q] = xin[(size_t)(g0 + ss) * S + j];
    }
    for (int q = threadIdx.x; q < 2 * ng; q += OL_THREADS) sxy[q] = xy[2 * g0 + q];
    __syncthreads();
    if (!live) continue;
    for (int ss = 0; ss < ng; ++ss) {
      const int s = g0 + ss;
      if (s == t) continue;
      // displacement of the block: target - source (source - target for A^T)
      const double dx = TR ? sxy[2 * ss] - xt : xt - sxy[2 * ss];
      const double dy = TR ? sxy[2 * ss + 1] - yt : yt - sxy[2 * ss + 1];
      const double r = sqrt(dx * dx + dy * dy);
      T hr[Q], hi[Q];
      ol_hankel_fixed<T, Q>(k * r, hr, hi);
      const T cph = (T)(dx / r), sph = (T)(dy / r);
      T er[Q], ei[Q];
      er[0] = (T)1;
      ei[0] = (T)0;
#pragma unroll
      for (int mu = 1; mu < Q; ++mu) {
        er[mu] = er[mu - 1] * cph - ei[mu - 1] * sph;
        ei[mu] = er[mu - 1] * sph + ei[mu - 1] * cph;
      }
      // source vector rotated by e^{i d_j phi}
      const cplx<T>* xs = sx + (size_t)ss * S;
      T vr[NH], vi[NH];
#pragma unroll
      for (int j = 0; j < NH; ++j) {
        T pr, pi;
        ol_rot<T, Q>(er, ei, d[j], pr, pi);
        const cplx<T> v = xs[j];
        vr[j] = ol_fma(pr, v.re, -pi * v.im);
        vi[j] = ol_fma(pr, v.im, pi * v.re);
      }
#pragma unroll
      for (int i = 0; i < NH; ++i) {
        T ar = (T)0, ai = (T)0;
#pragma unroll
        for (int j = 0; j < NH; ++j) {
          const T* ce = cf + (size_t)(TR ? j * S + i : i * S + j) * Q * 2;
          T sr = (T)0, si = (T)0;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const T cr = ce[2 * q], ci = ce[2 * q + 1];
            sr = ol_fma(-ci, hi[q], ol_fma(cr, hr[q], sr));
            si = ol_fma(ci, hr[q], ol_fma(cr, hi[q], si));
          }
          ar = ol_fma(-si, vi[j], ol_fma(sr, vr[j], ar));
          ai = ol_fma(si, vr[j], ol_fma(sr, vi[j], ai));
        }
        T pr, pi;
        ol_rot<T, Q>(er, ei, -d[i], pr, pi);
        yr[i] = ol_fma(-pi, ai, ol_fma(pr, ar, yr[i]));
        yi[i] = ol_fma(pi, ar, ol_fma(pr, ai, yi[i]));
      }
    }
  }
  if (!live) return;
  cplx<T>* out = partial + (((size_t)blockIdx.z * gridDim.y + rc) * N + t) * S;
#pragma unroll
  for (int i = 0; i < NH; ++i) out[i] = cplx<T>{yr[i], yi[i]};
#pragma unroll
  for (int i = NH; i < S; ++i) out[i] = cplx<T>{(T)0, (T)0};
}

// The product for lmax 4..6: loops over entries at run time (unrolled, classes
// of up to 48 members would not fit the register file), the sum over q
// unrolled with the Hankel values in registers, FP32 constants for the
// complex64 kernel, and (complex64) the phases e^{i mu phi} of the current
// pair in an LDS table [mu][thread] read once per entry.  LDS per workgroup
// stays under 64 KB: at lmax 6, 25 KB of staged sources and 27 KB of phases
// (FP32), 50 KB of staged sources (FP64).
template <typename T, int LMAX, bool TR>
__global__ __launch_bounds__(OL_THREADS) void offlattice_mid_kernel(
    const double* __restrict__ xy, const cplx<T>* __restrict__ x, const T* __restrict__ coef,
    const int* __restrict__ dm, int N, double k, int chunk, cplx<T>* __restrict__ partial,
    const int* __restrict__ stop) {
  constexpr int Q = 2 * LMAX + 1;
  constexpr int NH = LMAX * (LMAX + 2);
  constexpr int S = 16 * ((NH + 15) / 16);
  // the FP32 kernel reads each entry's phase from an LDS table; the FP64 one
  // (whose table would not fit beside the staged sources) selects it in registers
  constexpr bool PHT = sizeof(T) == 4;
  if (stop && *stop) return;  // a stopped GMRES cycle
  extern __shared__ double ol_lds[];
  double* sxy = ol_lds;                                             // [OL_GROUP][2]
  cplx<T>* sx = reinterpret_cast<cplx<T>*>(ol_lds + 2 * OL_GROUP);  // [OL_GROUP][S]
  cplx<T>* sph = sx + (size_t)OL_GROUP * S;                          // [Q][OL_THREADS] (PHT)
  const int t = blockIdx.x * OL_THREADS + threadIdx.x;
  const int rc = blockIdx.y;  // r * 2 + c
  const int c = rc & 1;
  const int s0 = blockIdx.z * chunk, s1 = min(N, s0 + chunk);
  const bool live = t < N;
  const double xt = live ? xy[2 * t] : 0.0, yt = live ? xy[2 * t + 1] : 0.0;
  const cplx<T>* xin = x + (size_t)rc * N * S;
  const T* cf = coef + (size_t)c * S * S * Q * 2;
  const int* dmc = dm + (size_t)c * S * S;
  cplx<T>* myph = sph + threadIdx.x;
  T yr[NH], yi[NH];
#pragma unroll
  for (int i = 0; i < NH; ++i) yr[i] = yi[i] = (T)0;
  for (int g0 = s0; g0 < s1; g0 += OL_GROUP) {
    const int ng = min(OL_GROUP, s1 - g0);
    __syncthreads();
    for (int q = threadIdx.x; q < ng * S; q += OL_THREADS) {
      const int ss = q / S, j = q % S;
      sx[q] = xin[(size_t)(g0 + ss) * S + j];
    }
    for (int q = threadIdx.x; q < 2 * ng; q += OL_THREADS) sxy[q] = xy[2 * g0 + q];
    __syncthreads();
    if (!live) continue;
    for (int ss = 0; ss < ng; ++ss) {
      const int s = g0 + ss;
      if (s == t) continue;
      const double dx = TR ? sxy[2 * ss] - xt : xt - sxy[2 * ss];
      const double dy = TR ? sxy[2 * ss + 1] - yt : yt - sxy[2 * ss + 1];
      const double r = sqrt(dx * dx + dy * dy);
      T hr[Q], hi[Q];
      ol_hankel_fixed<T, Q>(k * r, hr, hi);
      const T cph = (T)(dx / r), sphi = (T)(dy / r);
      T er[Q], ei[Q];
      er[0] = (T)1;
      ei[0] = (T)0;
#pragma unroll
      for (int mu = 1; mu < Q; ++mu) {
        er[mu] = er[mu - 1] * cph - ei[mu - 1] * sphi;
        ei[mu] = er[mu - 1] * sphi + ei[mu - 1] * cph;
      }
      if constexpr (PHT) {
#pragma unroll
        for (int mu = 0; mu < Q; ++mu) myph[(size_t)mu * OL_THREADS] = cplx<T>{er[mu], ei[mu]};
      }
      const cplx<T>* xs = sx + (size_t)ss * S;
      for (int i = 0; i < NH; ++i) {
        T ar = (T)0, ai = (T)0;
        for (int j = 0; j < NH; ++j) {
          const int e = TR ? j * S + i : i * S + j;
          const T* ce = cf + (size_t)e * Q * 2;
          T sr = (T)0, si = (T)0;
#pragma unroll
          for (int q = 0; q < Q; ++q) {
            const T cr = ce[2 * q], ci = ce[2 * q + 1];
            sr = ol_fma(-ci, hi[q], ol_fma(cr, hr[q], sr));
            si = ol_fma(ci, hr[q], ol_fma(cr, hi[q], si));
          }
          const int mu = dmc[e];
          T qr, qi;
          if constexpr (PHT) {
            const cplx<T> ph = myph[(size_t)(mu < 0 ? -mu : mu) * OL_THREADS];
            qr = ph.re;
            qi = mu < 0 ? -ph.im : ph.im;
          } else {
            ol_rot<T, Q>(er, ei, mu, qr, qi);
          }
          const T mr = ol_fma(-si, qi, sr * qr), mi = ol_fma(si, qr, sr * qi);
          const cplx<T> v = xs[j];
          ar = ol_fma(-mi, v.im, ol_fma(mr, v.re, ar));
          ai = ol_fma(mi, v.re, ol_fma(mr, v.im, ai));
        }
        yr[i] += ar;
        yi[i] += ai;
      }
    }
  }
  if (!live) return;
  cplx<T>* out = partial + (((size_t)blockIdx.z * gridDim.y + rc) * N + t) * S;
#pragma unroll
  for (int i = 0; i < NH; ++i) out[i] = cplx<T>{yr[i], yi[i]};
#pragma unroll
  for (int i = NH; i < S; ++i) out[i] = cplx<T>{(T)0, (T)0};
}

// y = x - t * z (Forward), x - z (Adjoint, z from t x), or z, z = sum of the
// chunks' partials in chunk order.
template <typename T>
__global__ void offlattice_combine_kernel(const cplx<T>* __restrict__ partial, int nchunk,
                                          long long total, const c128* __restrict__ x,
                                          const c128* __restrict__ t, long long vec,
                                          c128* __restrict__ y, int mode, const int* __restrict__ stop) {
  if (stop && *stop) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  double sr = 0.0, si = 0.0;
  for (int q = 0; q < nchunk; ++q) {
    const cplx<T> v = partial[(size_t)q * total + e];
    sr += (double)v.re;
    si += (double)v.im;
  }
  c128 o;
  if (mode == (int)Op::Forward) {
    const c128 tv = t[e % vec], xv = x[e];
    o = c128{xv.re - (tv.re * sr - tv.im * si), xv.im - (tv.re * si + tv.im * sr)};
  } else if (mode == (int)Op::Adjoint) {
    const c128 xv = x[e];
    o = c128{xv.re - sr, xv.im - si};
  } else {
    o = c128{sr, si};
  }
  y[e] = o;
}

template <typename T>
int offlattice_apply(tm_ctx* c, Op op, int R, const void* xin, const c128* x, c128* y) {
  const Geometry& g = c->g;
  const int N = g.n, S = g.S;
  const long long total = g.vec_len() * R;
  // enough workgroups to fill the chip: target blocks x (rhs, class) x chunks
  const int tb = (N + OL_THREADS - 1) / OL_THREADS;
  int nchunk = std::max(1, std::min((N + OL_GROUP - 1) / OL_GROUP, 2048 / std::max(1, tb * 2 * R)));
  const int chunk = (N + nchunk - 1) / nchunk;
  nchunk = (N + chunk - 1) / chunk;
  int rc;
  if ((rc = ensure(c, c->partial, (size_t)nchunk * total * sizeof(cplx<T>))) != TM_OK) return rc;
  // constants buffer: coef (FP64), dm, coef (FP32)
  const size_t ne = (size_t)NCLASS * S * S;
  const size_t cb = ne * (2 * g.lmax + 1) * 2 * sizeof(double), db = ne * sizeof(int);
  const T* coefT = std::is_same<T, float>::value ? (const T*)((const char*)c->olc.p + cb + db)
                                                 : (const T*)c->olc.p;
  const int* dm = (const int*)((const char*)c->olc.p + cb);
  const size_t lds = 2 * OL_GROUP * sizeof(double) + (size_t)OL_GROUP * S * sizeof(cplx<T>);
  const bool tr = (op == Op::Adjoint || op == Op::CouplingT);
  const dim3 grid(tb, 2 * R, nchunk);
#define OL_SMALL2(LM, TRV)                                                                        \
  hipLaunchKernelGGL((offlattice_small_kernel<T, LM, TRV>), grid, dim3(OL_THREADS), lds, c->stream, \
                     (const double*)c->xy.p, (const cplx<T>*)xin, coefT, dm, N, g.k, chunk,          \
                     (cplx<T>*)c->partial.p, c->mv_stop)
#define OL_SMALL(LM)          \
  {                           \
    if (tr)                   \
      OL_SMALL2(LM, true);    \
    else                      \
      OL_SMALL2(LM, false);   \
  }
  // the mid kernel adds a phase table [Q][OL_THREADS] behind the staged sources
  const size_t lds_mid =
      lds + (std::is_same<T, float>::value ? (size_t)(2 * g.lmax + 1) * OL_THREADS * sizeof(cplx<T>) : 0);
#define OL_MID2(LM, TRV)                                                                           \
  hipLaunchKernelGGL((offlattice_mid_kernel<T, LM, TRV>), grid, dim3(OL_THREADS), lds_mid,         \
                     c->stream, (const double*)c->xy.p, (const cplx<T>*)xin, coefT, dm, N, g.k,     \
                     chunk, (cplx<T>*)c->partial.p, c->mv_stop)
#define OL_MID(LM)            \
  {                           \
    if (tr)                   \
      OL_MID2(LM, true);      \
    else                      \
      OL_MID2(LM, false);     \
  }
  // FP64 takes the run-time-loop kernel at every lmax: unrolled, it needs 256
  // VGPRs at lmax 3 (one wave per SIMD)
  constexpr bool fp64 = std::is_same<T, double>::value;
  switch (g.lmax) {
    case 1:
      if constexpr (fp64) OL_MID(1) else OL_SMALL(1);
      break;
    case 2:
      if constexpr (fp64) OL_MID(2) else OL_SMALL(2);
      break;
    case 3:
      if constexpr (fp64) OL_MID(3) else OL_SMALL(3);
      break;
    case 4: OL_MID(4); break;
    case 5: OL_MID(5); break;
    case 6: OL_MID(6); break;
    default:
      return set_err(c, TM_ERR_INVALID_ARG, "lmax outside 1..6");
  }
#undef OL_MID
#undef OL_MID2
#undef OL_SMALL
#undef OL_SMALL2
  hipLaunchKernelGGL(offlattice_combine_kernel<T>, dim3((unsigned)((total + 255) / 256)), dim3(256), 0,
                     c->stream, (const cplx<T>*)c->partial.p, nchunk, total, x, (const c128*)c->t64.p,
                     g.vec_len(), y, (int)op, c->mv_stop);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}
template int offlattice_apply<float>(tm_ctx*, Op, int, const void*, const c128*, c128*);
template int offlattice_apply<double>(tm_ctx*, Op, int, const void*, const c128*, c128*);

}  // namespace tmh
