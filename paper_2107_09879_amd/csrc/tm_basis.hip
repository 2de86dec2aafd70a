// Per-scatterer and readout kernels built on the spherical-wave basis:
//   * Mie T-matrix diagonal of a sphere and its radius derivative
//     (the sphere case of App. I.B's T-matrix; Lorenz-Mie coefficients with
//     Riccati-Bessel functions, t_{l,p=0} = -b_l, t_{l,p=1} = -a_l);
//   * plane-wave incident coefficients (App. II, eqs. "integrand_p_0" and
//     "integrand_p_1": the second printed forms, with the scatterer-centre
//     phase e^{i k khat.x_i});
//   * scattered near field E_sca(x) = sum_i s_i^T Phi(k(x - x_i)) (App. I.C,
//     eq. "sca_fld_concise") and its far-field amplitude;
//   * point-detector vector and radius-gradient contraction (App. IV).
// Basis (App. I.A): Phi_lm0 = z_l [i pi theta_hat - tau phi_hat] e^{im phi} / sqrt(2l(l+1)),
// Phi_lm1 = [l(l+1) z_l/rho Pbar r_hat + (rho z_l)'/rho (tau theta_hat + i pi phi_hat)]
// e^{im phi} / sqrt(2l(l+1)), Pbar normalised without Condon-Shortley phase,
// pi = m Pbar / sin(theta), tau = d Pbar / d theta.
#include <cmath>
#include <vector>

#include "tm_internal.h"

namespace tmh {

template <typename T>
struct cx {
  T re, im;
  __device__ cx() : re(0), im(0) {}
  __device__ cx(T r, T i) : re(r), im(i) {}
};
template <typename T>
__device__ inline cx<T> operator+(cx<T> a, cx<T> b) { return cx<T>(a.re + b.re, a.im + b.im); }
template <typename T>
__device__ inline cx<T> operator-(cx<T> a, cx<T> b) { return cx<T>(a.re - b.re, a.im - b.im); }
template <typename T>
__device__ inline cx<T> operator*(cx<T> a, cx<T> b) {
  return cx<T>(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re);
}
template <typename T>
__device__ inline cx<T> operator*(T a, cx<T> b) { return cx<T>(a * b.re, a * b.im); }
template <typename T>
__device__ inline cx<T> operator/(cx<T> a, cx<T> b) {
  const T d = b.re * b.re + b.im * b.im;
  return cx<T>((a.re * b.re + a.im * b.im) / d, (a.im * b.re - a.re * b.im) / d);
}
template <typename T>
__device__ inline cx<T> mul_i(cx<T> a) { return cx<T>(-a.im, a.re); }
// i^e
template <typename T>
__device__ inline cx<T> ipow(int e) {
  switch (((e % 4) + 4) % 4) {
    case 0: return cx<T>(1, 0);
    case 1: return cx<T>(0, 1);
    case 2: return cx<T>(-1, 0);
    default: return cx<T>(0, -1);
  }
}

__device__ inline void sincos_t(float x, float* s, float* c) { sincosf(x, s, c); }
__device__ inline void sincos_t(double x, double* s, double* c) { sincos(x, s, c); }

__device__ inline void plm_of_n(int n, int lmax, int& p, int& l, int& m) {
  const int half = lmax * (lmax + 2);
  p = n / half;
  const int r = n - p * half;
  l = 1;
  while ((l + 1) * (l + 1) - 1 <= r) ++l;
  m = r - (l * (l + 1) - 1);
}
__device__ inline int n_of_plm(int p, int l, int m, int lmax) {
  return p * lmax * (lmax + 2) + l * (l + 1) - 1 + m;
}

// Normalised Legendre data at one (l, |m|): Pbar, U = Pbar/sin(theta) (|m| >= 1,
// regular at the poles), tau = dPbar/dtheta.  Recurrences on
// u_l^m = P_l^m / sin(theta): u_m^m = (2m-1)!! sin^{m-1}, (l-m) u_l^m =
// cos (2l-1) u_{l-1}^m - (l+m-1) u_{l-2}^m, dP_l^m/dtheta = l cos u_l^m -
// (l+m) u_{l-1}^m; for m = 0, tau = -P_l^1 = -sin u_l^1.
template <typename T>
__device__ inline void legendre_one(int l, int am, T ct, T st, T& P, T& U, T& tau) {
  T nrm = (T)(2 * l + 1) / (T)2;
  for (int q = l - am + 1; q <= l + am; ++q) nrm /= (T)q;
  nrm = sqrt(nrm);
  if (am == 0) {
    T p0 = 1, p1 = ct;
    T Pl = (l == 0) ? p0 : p1;
    for (int q = 2; q <= l; ++q) {
      const T p2 = ((T)(2 * q - 1) * ct * p1 - (T)(q - 1) * p0) / (T)q;
      p0 = p1;
      p1 = p2;
      Pl = p2;
    }
    T u0 = 0, u1 = 1, ul = (l >= 1) ? (T)1 : (T)0;
    for (int q = 2; q <= l; ++q) {
      const T u2 = ((T)(2 * q - 1) * ct * u1 - (T)q * u0) / (T)(q - 1);
      u0 = u1;
      u1 = u2;
      ul = u2;
    }
    P = nrm * Pl;
    U = 0;
    tau = -nrm * st * ul;
    return;
  }
  T um = 1;
  for (int q = 1; q <= 2 * am - 1; q += 2) um *= (T)q;
  for (int q = 0; q < am - 1; ++q) um *= st;
  T uprev = 0, ucur = um;
  for (int q = am + 1; q <= l; ++q) {
    const T un = ((T)(2 * q - 1) * ct * ucur - (T)(q + am - 1) * uprev) / (T)(q - am);
    uprev = ucur;
    ucur = un;
  }
  P = nrm * st * ucur;
  U = nrm * ucur;
  tau = nrm * ((T)l * ct * ucur - (T)(l + am) * uprev);
}

// ---------------------------------------------------------------- Mie
// j_l(z) by its power series z^l/(2l+1)!! sum_k (-z^2/2)^k / (k! prod (2l+2i+1))
// (accurate for the small size parameters of subwavelength spheres, |z| <= 12).
__device__ inline cx<double> sph_j_series(int l, cx<double> z) {
  const cx<double> mz2h = (-0.5) * (z * z);
  cx<double> term(1.0, 0.0), sum(1.0, 0.0);
  for (int k = 1; k < 120; ++k) {
    term = (1.0 / ((double)k * (double)(2 * l + 2 * k + 1))) * (term * mz2h);
    sum = sum + term;
    if (fabs(term.re) + fabs(term.im) < 1e-18 * (fabs(sum.re) + fabs(sum.im))) break;
  }
  cx<double> zl(1.0, 0.0);
  double df = 1.0;
  for (int q = 0; q < l; ++q) zl = zl * z;
  for (int q = 1; q <= 2 * l + 1; q += 2) df *= (double)q;
  return (1.0 / df) * (zl * sum);
}

// Sphere T entries for l = 1..lmax: t[p][l] (p = 0: -b_l, p = 1: -a_l) and
// their radius derivatives dt[p][l] = k d t / dx, x = k r, m = relative index.
__device__ void mie_t_of_l(double x, double k, cx<double> m, int lmax, cx<double> (*t)[LMAX_SUPPORTED + 1],
                           cx<double> (*dt)[LMAX_SUPPORTED + 1]) {
  const cx<double> X(x, 0.0);
  const cx<double> Y = m * X;
  cx<double> jx[LMAX_SUPPORTED + 1], hx[LMAX_SUPPORTED + 1], jy[LMAX_SUPPORTED + 1];
  double sx, cxs;
  sincos(x, &sx, &cxs);
  double y0 = -cxs / x, y1 = -cxs / (x * x) - sx / x;
  for (int l = 0; l <= lmax; ++l) {
    jx[l] = sph_j_series(l, X);
    jy[l] = sph_j_series(l, Y);
    double yl;
    if (l == 0) yl = y0;
    else if (l == 1) yl = y1;
    else {
      yl = (double)(2 * l - 1) / x * y1 - y0;
      y0 = y1;
      y1 = yl;
    }
    hx[l] = cx<double>(jx[l].re, yl);
  }
  for (int l = 1; l <= lmax; ++l) {
    const double ll = (double)(l * (l + 1));
    const cx<double> px = X * jx[l];
    const cx<double> pdx = X * jx[l - 1] - (double)l * jx[l];
    const cx<double> xx = X * hx[l];
    const cx<double> xdx = X * hx[l - 1] - (double)l * hx[l];
    const cx<double> py = Y * jy[l];
    const cx<double> pdy = Y * jy[l - 1] - (double)l * jy[l];
    const double fx = ll / (x * x) - 1.0;
    const cx<double> fy = cx<double>(ll, 0.0) / (Y * Y) - cx<double>(1.0, 0.0);
    const cx<double> pddx = fx * px, xddx = fx * xx, pddy = fy * py;
    const cx<double> na = m * py * pdx - px * pdy;
    const cx<double> da = m * py * xdx - xx * pdy;
    const cx<double> nb = py * pdx - m * px * pdy;
    const cx<double> db = py * xdx - m * xx * pdy;
    const cx<double> m2 = m * m;
    const cx<double> na_x = m2 * pdy * pdx + m * py * pddx - pdx * pdy - m * px * pddy;
    const cx<double> da_x = m2 * pdy * xdx + m * py * xddx - xdx * pdy - m * xx * pddy;
    const cx<double> nb_x = m * pdy * pdx + py * pddx - m * pdx * pdy - m2 * px * pddy;
    const cx<double> db_x = m * pdy * xdx + py * xddx - m * xdx * pdy - m2 * xx * pddy;
    const cx<double> a = na / da, b = nb / db;
    const cx<double> dadx = (na_x * da - na * da_x) / (da * da);
    const cx<double> dbdx = (nb_x * db - nb * db_x) / (db * db);
    t[0][l] = cx<double>(-b.re, -b.im);
    t[1][l] = cx<double>(-a.re, -a.im);
    dt[0][l] = (-k) * dbdx;
    dt[1][l] = (-k) * dadx;
  }
}

__global__ void mie_kernel(const double* __restrict__ radii, int N, double k, double nre,
                           double nim, int lmax, SlotMaps mp, c128* __restrict__ t64,
                           c64* __restrict__ t32, c128* __restrict__ dt64) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= N) return;
  cx<double> t[2][LMAX_SUPPORTED + 1], dt[2][LMAX_SUPPORTED + 1];
  mie_t_of_l(k * radii[i], k, cx<double>(nre, nim), lmax, t, dt);
  for (int l = 1; l <= lmax; ++l)
    for (int mm = -l; mm <= l; ++mm)
      for (int p = 0; p < 2; ++p) {
        const int n = n_of_plm(p, l, mm, lmax);
        const size_t o = ((size_t)mp.cls_of[n] * N + i) * mp.S + mp.slot_of[n];
        t64[o] = c128{t[p][l].re, t[p][l].im};
        t32[o] = c64{(float)t[p][l].re, (float)t[p][l].im};
        dt64[o] = c128{dt[p][l].re, dt[p][l].im};
      }
}

// one sphere: out[0 .. 2 lmax) = t[p][l], out[2 lmax .. 4 lmax) = dt[p][l],
// index p * lmax + (l - 1)
__global__ void mie_one_kernel(double radius, double k, double nre, double nim, int lmax,
                               tm_c128* __restrict__ out) {
  if (threadIdx.x != 0) return;
  cx<double> t[2][LMAX_SUPPORTED + 1], dt[2][LMAX_SUPPORTED + 1];
  mie_t_of_l(k * radius, k, cx<double>(nre, nim), lmax, t, dt);
  for (int p = 0; p < 2; ++p)
    for (int l = 1; l <= lmax; ++l) {
      out[p * lmax + l - 1] = tm_c128{t[p][l].re, t[p][l].im};
      out[2 * lmax + p * lmax + l - 1] = tm_c128{dt[p][l].re, dt[p][l].im};
    }
}

// t (boundary [N][L]) -> slot layouts
__global__ void set_t_kernel(const tm_c128* __restrict__ t, int N, SlotMaps mp,
                             c128* __restrict__ t64, c64* __restrict__ t32) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)N * mp.L) return;
  const int n = (int)(e % mp.L);
  const long long i = e / mp.L;
  const size_t o = ((size_t)mp.cls_of[n] * N + i) * mp.S + mp.slot_of[n];
  const tm_c128 v = t[e];
  t64[o] = c128{v.re, v.im};
  t32[o] = c64{(float)v.re, (float)v.im};
}

// Dense per-scatterer T (boundary order, T[i][n][n']) applied to slot-layout
// vectors [R][class][site][S].  One thread per output element; pads give 0
// (modes 0, 2) or x (mode 1, where x's pads are 0).
__global__ void tdense_kernel(const tm_c128* __restrict__ T, SlotMaps mp, long long N, int mode,
                              const c128* __restrict__ x, const c128* __restrict__ z,
                              c128* __restrict__ y, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int slot = (int)(e % mp.S);
  const long long site = (e / mp.S) % N;
  const long long rc = e / (mp.S * N);
  const long long r = rc / NCLASS;
  const int c = (int)(rc % NCLASS);
  const int n = mp.n_of[c][slot];
  const int L = mp.L;
  double ar = 0.0, ai = 0.0;
  if (n >= 0) {
    const tm_c128* Ti = T + (size_t)site * L * L;
    for (int n2 = 0; n2 < L; ++n2) {
      const c128 zv = z[((size_t)(r * NCLASS + mp.cls_of[n2]) * N + site) * mp.S + mp.slot_of[n2]];
      const tm_c128 tv = mode == 2 ? Ti[(size_t)n2 * L + n] : Ti[(size_t)n * L + n2];
      ar += tv.re * zv.re - tv.im * zv.im;
      ai += tv.re * zv.im + tv.im * zv.re;
    }
  }
  if (mode == 1) {
    const c128 xv = x[e];
    y[e] = c128{xv.re - ar, xv.im - ai};
  } else {
    y[e] = c128{ar, ai};
  }
}

// Structure test of a dense T: *flag |= 1 if some entry couples two different
// azimuthal orders (m(n) != m(n')) and is not exactly zero (NaN counts).
__global__ void tdense_mcheck_kernel(const tm_c128* __restrict__ T, MbMaps mb, int L,
                                     long long total, int* __restrict__ flag) {
  int hit = 0;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (long long)gridDim.x * blockDim.x) {
    const int n2 = (int)(e % L);
    const int n = (int)((e / L) % L);
    if (mb.blk_of[n] != mb.blk_of[n2]) {
      const tm_c128 v = T[e];
      if (!(v.re == 0.0) || !(v.im == 0.0)) hit = 1;
    }
  }
  if (__any(hit) && (threadIdx.x & 63) == 0) atomicOr(flag, 1);
}

// Tm[i][off_b + q nm_b + t] = T[i][mem_b[q]][mem_b[t]] for every m-block b
__global__ void tdense_mpack_kernel(const tm_c128* __restrict__ T, MbMaps mb, int L, long long N,
                                    c128* __restrict__ Tm) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= N * mb.per_site) return;
  const long long i = e / mb.per_site;
  const int r = (int)(e % mb.per_site);
  int b = 0;
  while (b + 1 < mb.nblk && mb.off[b + 1] <= r) ++b;
  const int nm = mb.nm[b];
  const int q = (r - mb.off[b]) / nm, t = (r - mb.off[b]) % nm;
  const tm_c128 v = T[((size_t)i * L + mb.mem[mb.first[b] + q]) * L + mb.mem[mb.first[b] + t]];
  Tm[e] = c128{v.re, v.im};
}

// The dense-T apply of tdense_kernel for a T kept as m-blocks: the same
// thread mapping and the same nonzero terms in the same order (members of a
// block in increasing n), reading nm_b instead of L entries per output.
__global__ void tdense_mb_kernel(const c128* __restrict__ Tm, MbMaps mb, SlotMaps mp, long long N,
                                 int mode, const c128* __restrict__ x, const c128* __restrict__ z,
                                 c128* __restrict__ y, long long total) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= total) return;
  const int slot = (int)(e % mp.S);
  const long long site = (e / mp.S) % N;
  const long long rc = e / (mp.S * N);
  const long long r = rc / NCLASS;
  const int c = (int)(rc % NCLASS);
  const int n = mp.n_of[c][slot];
  double ar = 0.0, ai = 0.0;
  if (n >= 0) {
    const int b = mb.blk_of[n], q = mb.q_of[n], nm = mb.nm[b], f = mb.first[b];
    const c128* Tb = Tm + (size_t)site * mb.per_site + mb.off[b];
    for (int t = 0; t < nm; ++t) {
      const int n2 = mb.mem[f + t];
      const c128 zv = z[((size_t)(r * NCLASS + mp.cls_of[n2]) * N + site) * mp.S + mp.slot_of[n2]];
      const c128 tv = mode == 2 ? Tb[t * nm + q] : Tb[q * nm + t];
      ar += tv.re * zv.re - tv.im * zv.im;
      ai += tv.re * zv.im + tv.im * zv.re;
    }
  }
  if (mode == 1) {
    const c128 xv = x[e];
    y[e] = c128{xv.re - ar, xv.im - ai};
  } else {
    y[e] = c128{ar, ai};
  }
}

// ---------------------------------------------------------------- plane wave
struct PwArgs {
  double khat[3 * 8];
  double pol[6 * 8];  // re, im interleaved per component
};

__global__ void plane_wave_kernel(PwArgs pw, int R, int N, int L, int lmax, SitePos sp, double k,
                                  tm_c128* __restrict__ a0) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)R * N * L) return;
  const int n = (int)(e % L);
  const long long i = (e / L) % N;
  const int r = (int)(e / ((long long)L * N));
  const double* kh = pw.khat + 3 * r;
  const double* po = pw.pol + 6 * r;
  const double sb = sqrt(kh[0] * kh[0] + kh[1] * kh[1]);
  const double cb = kh[2];
  const double al = (sb > 0.0) ? atan2(kh[1], kh[0]) : 0.0;
  double sa, ca;
  sincos(al, &sa, &ca);
  const double bh[3] = {cb * ca, cb * sa, -sb};
  const double ah[3] = {-sa, ca, 0.0};
  cx<double> bA, aA;
  for (int q = 0; q < 3; ++q) {
    const cx<double> pq(po[2 * q], po[2 * q + 1]);
    bA = bA + bh[q] * pq;
    aA = aA + ah[q] * pq;
  }
  int p, l, m;
  plm_of_n(n, lmax, p, l, m);
  double P, U, tau;
  legendre_one<double>(l, m < 0 ? -m : m, cb, sb, P, U, tau);
  const double pi = (double)m * U;
  double sm, cm;
  sincos(-(double)m * al, &sm, &cm);
  const cx<double> pre = (-4.0 / sqrt(2.0 * l * (l + 1))) * cx<double>(cm, sm);
  cx<double> v;
  if (p == 0)
    v = pre * ipow<double>(l) * (mul_i(pi * bA) + tau * aA);
  else
    v = pre * ipow<double>(l + 1) * (tau * bA - mul_i(pi * aA));
  double xi, yi;
  sp.at(i, xi, yi);
  double sph, cph;
  sincos(k * (kh[0] * xi + kh[1] * yi), &sph, &cph);
  v = cx<double>(cph, sph) * v;
  a0[e] = tm_c128{v.re, v.im};
}

// ---------------------------------------------------------------- readout
// Hankel functions h_0..h_lmax at x with e^{ix} given as (c, s).
template <typename T>
__device__ inline void hankel_set(T x, T c, T s, int lmax, cx<T>* h) {
  const T ix = (T)1 / x;
  h[0] = cx<T>(s * ix, -c * ix);
  h[1] = cx<T>(-(c * x - s) * ix * ix, -(s * x + c) * ix * ix);
  for (int q = 1; q < lmax; ++q) {
    const T f = (T)(2 * q + 1) * ix;
    h[q + 1] = cx<T>(f * h[q].re - h[q - 1].re, f * h[q].im - h[q - 1].im);
  }
}

constexpr int NF_MAXR = 4;

// Phase and distance of one (point, sphere) pair for the near field: kr in
// FP64 (|kr| reaches 1e3..1e4 across a metasurface), its reduction modulo 2 pi,
// and 1/r in the basis precision.  The FP32 basis takes 1/sqrt(r^2) from the
// hardware reciprocal square root, refines r = r^2 / sqrt(r^2) by one FP64
// Newton step (relative error ~1e-14), and evaluates the sine and cosine of
// the reduced phase on the hardware units, whose argument is in revolutions.
template <typename T>
struct NfPhase;

template <>
struct NfPhase<float> {
  static __device__ inline void eval(double r2, double k, float& sn, float& cs, float& x, float& irr) {
    const float y = __builtin_amdgcn_rsqf((float)r2);
    const double r0 = r2 * (double)y;
    const double rr = fma(0.5 * (double)y, fma(-r0, r0, r2), r0);
    const double t = (k * rr) * 0.15915494309189533576888376337251;  // revolutions
    const float fr = (float)(t - rint(t));
    sn = __builtin_amdgcn_sinf(fr);
    cs = __builtin_amdgcn_cosf(fr);
    x = (float)(k * rr);
    irr = y;
  }
  static __device__ inline float rsqrt_pos(float v) { return __builtin_amdgcn_rsqf(v); }
  static __device__ inline float rcp(float v) { return __builtin_amdgcn_rcpf(v); }
};

template <>
struct NfPhase<double> {
  static __device__ inline void eval(double r2, double k, double& sn, double& cs, double& x, double& irr) {
    const double rr = sqrt(r2);
    const double kr = k * rr;
    const double twopi = 6.283185307179586476925286766559;
    const double red = kr - twopi * rint(kr * 0.15915494309189533576888376337251);
    sincos(red, &sn, &cs);
    x = kr;
    irr = 1.0 / rr;
  }
  static __device__ inline double rsqrt_pos(double v) { return 1.0 / sqrt(v); }
  static __device__ inline double rcp(double v) { return 1.0 / v; }
};

// Near field with compile-time lmax and RHS count (all basis values in
// registers).  Each workgroup stages the coefficients of CH spheres at a time
// in LDS (every thread reads the same entries: broadcast) and each thread
// accumulates the field of one point.
//
// The +-m terms of one (l, |m|) share P, U, tau and conj(e^{i|m|phi}), so
// they are folded.  With s(+m) = a + ib, s(-m) = a' + ib' and
// e = e^{i|m|phi} = c + id,
//   sMe = s(+m) e + s(-m) e* = (c A+ - d B-) + i (c B+ + d A-),
//   dMe = s(+m) e - s(-m) e* = (c A- - d B+) + i (c B- + d A+),
// A+- = a +- a', B+- = b +- b'; the four sums are formed once per sphere when
// the coefficients are staged (likewise sNe, dNe from the N-type pair).
// Staging also multiplies in the real constants sqrt((2l+1)/2 (l-m)!/(l+m)!)
// and 1/sqrt(2l(l+1)).  The l-dependent radial factors come out of the sum
// over |m|:
//   E_r  += c_l sum_m P sNe,
//   E_th += i a_l sum_m U dMe + b_l sum_m tau sNe,
//   E_ph += -a_l sum_m tau sMe + i b_l sum_m U dNe,
// with a_l = h_l, b_l = (x h_{l-1} - l h_l)/x, c_l = l(l+1) h_l/x,
// P = sin u_l^m, U = |m| u_l^m, tau = l cos u_l^m - (l+|m|) u_{l-1}^m for
// |m| >= 1 (u = P_l^m / sin), P = P_l^0 and tau = -sin u_l^1 for m = 0.
// Staged layout per (sphere, RHS), in reals: for l = 1..LMAX at offset
// 4 (l^2 - 1): m = 0 as [M.re, M.im, N.re, N.im], then for |m| = 1..l
// [M: A+, A-, B+, B-][N: A+, A-, B+, B-].
template <typename T, int LMAX, int R>
__global__ __launch_bounds__(256) void near_field_v2(
    const tm_c128* __restrict__ s, int N, SitePos sp, double k,
    const double* __restrict__ pts, int P, tm_c128* __restrict__ E) {
  constexpr int L = 2 * LMAX * (LMAX + 2), H = LMAX * (LMAX + 2);
  constexpr int NF = 2 * L;                     // staged reals per (sphere, RHS)
  constexpr int NU = LMAX * (LMAX + 3) / 2;     // (l, |m|) units per (sphere, RHS)
  // spheres staged per LDS chunk: at most 48 KB of coefficients
  constexpr int CHN = (LMAX <= 3) ? 32 : 8;
  __shared__ __align__(16) T sh[CHN][R][NF];
  __shared__ __align__(16) double shp[CHN][2];  // centres of the staged spheres
  const int ip = blockIdx.x * blockDim.x + threadIdx.x;
  const bool live = ip < P;
  const double px = live ? pts[3 * ip] : 0.0, py = live ? pts[3 * ip + 1] : 0.0,
               pz = live ? pts[3 * ip + 2] : 1.0;
  const T invk = (T)(1.0 / k);
  cx<T> acc[R][3];
  for (int i0 = 0; i0 < N; i0 += CHN) {
    const int nch = min(CHN, N - i0);
    __syncthreads();
    if (threadIdx.x < nch) sp.at(i0 + threadIdx.x, shp[threadIdx.x][0], shp[threadIdx.x][1]);
    for (int q = threadIdx.x; q < nch * R * NU; q += blockDim.x) {
      const int u = q % NU, rr = (q / NU) % R, ii = q / (NU * R);
      int l = 1;
      while ((l + 1) * (l + 2) / 2 - 1 <= u) ++l;  // units before l: (l-1)(l+2)/2
      const int am = u - (l - 1) * (l + 2) / 2;
      double v = (2.0 * l + 1.0) / 2.0;
      for (int f = l - am + 1; f <= l + am; ++f) v /= (double)f;
      const double w = sqrt(v / (2.0 * l * (l + 1)));
      const tm_c128* si = s + ((size_t)rr * N + (i0 + ii)) * L;
      T* dst = &sh[ii][rr][4 * (l * l - 1) + (am == 0 ? 0 : 8 * am - 4)];
      const int np = l * (l + 1) - 1 + am, nm = l * (l + 1) - 1 - am;
      if (am == 0) {
        dst[0] = (T)(w * si[np].re);
        dst[1] = (T)(w * si[np].im);
        dst[2] = (T)(w * si[H + np].re);
        dst[3] = (T)(w * si[H + np].im);
      } else {
#pragma unroll
        for (int t = 0; t < 2; ++t) {
          const tm_c128 a = si[t * H + np], b = si[t * H + nm];
          dst[4 * t + 0] = (T)(w * (a.re + b.re));
          dst[4 * t + 1] = (T)(w * (a.re - b.re));
          dst[4 * t + 2] = (T)(w * (a.im + b.im));
          dst[4 * t + 3] = (T)(w * (a.im - b.im));
        }
      }
    }
    __syncthreads();
    for (int ii = 0; ii < nch; ++ii) {
      const double dx = px - shp[ii][0];
      const double dy = py - shp[ii][1];
      const double dz = pz;
      const double rho2 = dx * dx + dy * dy;
      T sn, cs, x, irr;
      NfPhase<T>::eval(rho2 + dz * dz, k, sn, cs, x, irr);
      const T ix = irr * invk;
      const T ct = (T)dz * irr;
      T cf = 1, sf = 0, st = 0;
      if (rho2 > 0.0) {
        const T ir = NfPhase<T>::rsqrt_pos((T)rho2);
        cf = (T)dx * ir;
        sf = (T)dy * ir;
        st = ((T)rho2 * ir) * irr;
      }
      // Hankel h_0..h_LMAX
      cx<T> h[LMAX + 1];
      h[0] = cx<T>(sn * ix, -cs * ix);
      if (LMAX >= 1) h[1] = cx<T>(-(cs * x - sn) * ix * ix, -(sn * x + cs) * ix * ix);
#pragma unroll
      for (int q = 1; q < LMAX; ++q) {
        const T f = (T)(2 * q + 1) * ix;
        h[q + 1] = cx<T>(f * h[q].re - h[q - 1].re, f * h[q].im - h[q - 1].im);
      }
      // u_l^m = P_l^m / sin (m >= 1), P_l^0, and u_l^1 for tau_l^0
      T u[LMAX + 2][LMAX + 1];
#pragma unroll
      for (int am = 1; am <= LMAX; ++am) {
        T um = 1;
#pragma unroll
        for (int q = 1; q <= 2 * am - 1; q += 2) um *= (T)q;
#pragma unroll
        for (int q = 0; q < am - 1; ++q) um *= st;
        u[am - 1][am] = 0;
        u[am][am] = um;
#pragma unroll
        for (int l = am + 1; l <= LMAX; ++l)
          u[l][am] = ((T)(2 * l - 1) * ct * u[l - 1][am] - (T)(l + am - 1) * (l - 2 >= am ? u[l - 2][am] : (T)0)) *
                     (T)(1.0 / (l - am));
      }
      T p0[LMAX + 1];
      p0[0] = 1;
      if (LMAX >= 1) p0[1] = ct;
#pragma unroll
      for (int l = 2; l <= LMAX; ++l)
        p0[l] = ((T)(2 * l - 1) * ct * p0[l - 1] - (T)(l - 1) * p0[l - 2]) * (T)(1.0 / l);
      cx<T> e[LMAX + 1];
      e[0] = cx<T>(1, 0);
#pragma unroll
      for (int am = 1; am <= LMAX; ++am) e[am] = e[am - 1] * cx<T>(cf, sf);
      cx<T> Er[R], Et[R], Ep[R];
#pragma unroll
      for (int l = 1; l <= LMAX; ++l) {
        const cx<T> al = h[l];
        const cx<T> bl = cx<T>((x * h[l - 1].re - (T)l * h[l].re) * ix, (x * h[l - 1].im - (T)l * h[l].im) * ix);
        const cx<T> cl = ((T)(l * (l + 1)) * ix) * h[l];
        cx<T> X[R], Y1[R], Y2[R], Z1[R], Z2[R];
#pragma unroll
        for (int am = 0; am <= l; ++am) {
          const int off = 4 * (l * l - 1) + (am == 0 ? 0 : 8 * am - 4);
          if (am == 0) {
            const T Pb = p0[l], tau = -st * u[l][1];
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const T* c = &sh[ii][r][off];
              const cx<T> sM(c[0], c[1]), sN(c[2], c[3]);
              X[r] = X[r] + Pb * sN;
              Y2[r] = Y2[r] + tau * sN;
              Z1[r] = Z1[r] + tau * sM;
            }
          } else {
            const T Pb = st * u[l][am], Ub = (T)am * u[l][am];
            const T tau = (T)l * ct * u[l][am] - (T)(l + am) * u[l - 1][am];
            const T c = e[am].re, d = e[am].im;
#pragma unroll
            for (int r = 0; r < R; ++r) {
              const T* g = &sh[ii][r][off];
              const cx<T> sMe(c * g[0] - d * g[3], c * g[2] + d * g[1]);
              const cx<T> dMe(c * g[1] - d * g[2], c * g[3] + d * g[0]);
              const cx<T> sNe(c * g[4] - d * g[7], c * g[6] + d * g[5]);
              const cx<T> dNe(c * g[5] - d * g[6], c * g[7] + d * g[4]);
              X[r] = X[r] + Pb * sNe;
              Y1[r] = Y1[r] + Ub * dMe;
              Y2[r] = Y2[r] + tau * sNe;
              Z1[r] = Z1[r] + tau * sMe;
              Z2[r] = Z2[r] + Ub * dNe;
            }
          }
        }
#pragma unroll
        for (int r = 0; r < R; ++r) {
          Er[r] = Er[r] + cl * X[r];
          Et[r] = Et[r] + mul_i(al * Y1[r]) + bl * Y2[r];
          Ep[r] = Ep[r] - al * Z1[r] + mul_i(bl * Z2[r]);
        }
      }
#pragma unroll
      for (int r = 0; r < R; ++r) {
        acc[r][0] = acc[r][0] + (st * cf) * Er[r] + (ct * cf) * Et[r] - sf * Ep[r];
        acc[r][1] = acc[r][1] + (st * sf) * Er[r] + (ct * sf) * Et[r] + cf * Ep[r];
        acc[r][2] = acc[r][2] + ct * Er[r] - st * Et[r];
      }
    }
  }
  if (!live) return;
#pragma unroll
  for (int r = 0; r < R; ++r)
#pragma unroll
    for (int q = 0; q < 3; ++q)
      E[((size_t)r * P + ip) * 3 + q] = tm_c128{(double)acc[r][q].re, (double)acc[r][q].im};
}

template <typename T, int LMAX>
static void nf_dispatch_r(int R, dim3 g, hipStream_t st, const tm_c128* s, int N, SitePos sp, double k,
                          const double* pts, int P, tm_c128* E) {
  switch (R) {
    case 1: hipLaunchKernelGGL((near_field_v2<T, LMAX, 1>), g, dim3(256), 0, st, s, N, sp, k, pts, P, E); break;
    case 2: hipLaunchKernelGGL((near_field_v2<T, LMAX, 2>), g, dim3(256), 0, st, s, N, sp, k, pts, P, E); break;
    case 3: hipLaunchKernelGGL((near_field_v2<T, LMAX, 3>), g, dim3(256), 0, st, s, N, sp, k, pts, P, E); break;
    default: hipLaunchKernelGGL((near_field_v2<T, LMAX, 4>), g, dim3(256), 0, st, s, N, sp, k, pts, P, E); break;
  }
}

template <typename T>
static void nf_dispatch(int lmax, int R, dim3 g, hipStream_t st, const tm_c128* s, int N, SitePos sp,
                        double k, const double* pts, int P, tm_c128* E) {
  switch (lmax) {
    case 1: nf_dispatch_r<T, 1>(R, g, st, s, N, sp, k, pts, P, E); break;
    case 2: nf_dispatch_r<T, 2>(R, g, st, s, N, sp, k, pts, P, E); break;
    case 3: nf_dispatch_r<T, 3>(R, g, st, s, N, sp, k, pts, P, E); break;
    case 4: nf_dispatch_r<T, 4>(R, g, st, s, N, sp, k, pts, P, E); break;
    case 5: nf_dispatch_r<T, 5>(R, g, st, s, N, sp, k, pts, P, E); break;
    default: nf_dispatch_r<T, 6>(R, g, st, s, N, sp, k, pts, P, E); break;
  }
}

// F(d) = (1/k) sum_i e^{-ik d.x_i} sum_n s_{i,n} F_n(d), with
// F_n = (-i)^{l+1} [i pi th - tau ph] e^{im phi} (p = 0), (-i)^l [tau th + i pi ph] e^{im phi}
// (p = 1), times 1/sqrt(2l(l+1)): the h_l(x) ~ (-i)^{l+1} e^{ix}/x limit.
// One workgroup per (rhs, direction): threads stride over scatterers to form
// c_n = sum_i e^{-ik d.x_i} s_{i,n}, then a fixed-order wave + LDS reduction.
constexpr int FF_THREADS = 256;
template <int LMAXT>
__global__ __launch_bounds__(FF_THREADS) void far_field_kernel(
    const tm_c128* __restrict__ s, int R, int N, int L, int lmax, SitePos sp, double k,
    const double* __restrict__ dirs, int D, tm_c128* __restrict__ F) {
  constexpr int LM = 2 * LMAXT * (LMAXT + 2);
  __shared__ double red[FF_THREADS / 64][2 * LM];
  const int e = blockIdx.x;
  const int r = e / D, id = e % D;
  const double ux = dirs[3 * id], uy = dirs[3 * id + 1], uz = dirs[3 * id + 2];
  double cr[LM], ci[LM];
#pragma unroll
  for (int n = 0; n < LM; ++n) cr[n] = ci[n] = 0.0;
  for (int i = threadIdx.x; i < N; i += FF_THREADS) {
    double xi, yi;
    sp.at(i, xi, yi);
    double sph, cph;
    sincos(-k * (ux * xi + uy * yi), &sph, &cph);
    const tm_c128* si = s + ((size_t)r * N + i) * L;
#pragma unroll
    for (int n = 0; n < LM; ++n) {
      if (n < L) {
        const tm_c128 v = si[n];
        cr[n] += cph * v.re - sph * v.im;
        ci[n] += cph * v.im + sph * v.re;
      }
    }
  }
  const int w = threadIdx.x >> 6, ln = threadIdx.x & 63;
#pragma unroll
  for (int n = 0; n < LM; ++n) {
    double a = cr[n], b = ci[n];
    for (int o = 32; o > 0; o >>= 1) {
      a += __shfl_xor(a, o, 64);
      b += __shfl_xor(b, o, 64);
    }
    if (ln == 0) {
      red[w][2 * n] = a;
      red[w][2 * n + 1] = b;
    }
  }
  __syncthreads();
  if (threadIdx.x != 0) return;
  const double rho = sqrt(ux * ux + uy * uy);
  const double ct = uz, st = rho;
  double cf = 1.0, sf = 0.0;
  if (rho > 0.0) {
    cf = ux / rho;
    sf = uy / rho;
  }
  cx<double> Ft, Fp;
  for (int n = 0; n < L; ++n) {
    double a = 0.0, b = 0.0;
    for (int q = 0; q < FF_THREADS / 64; ++q) {
      a += red[q][2 * n];
      b += red[q][2 * n + 1];
    }
    int p, l, m;
    plm_of_n(n, lmax, p, l, m);
    double Pb, U, tau;
    legendre_one<double>(l, m < 0 ? -m : m, ct, st, Pb, U, tau);
    const double pi = (double)m * U;
    double sm, cm;
    sincos((double)m * atan2(sf, cf), &sm, &cm);
    const cx<double> em(cm, sm);
    const double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
    const cx<double> c = nrm * (cx<double>(a, b) * em);
    if (p == 0) {
      const cx<double> f = ipow<double>(-(l + 1)) * c;  // (-i)^{l+1} = i^{-(l+1)}
      Ft = Ft + mul_i(pi * f);
      Fp = Fp - tau * f;
    } else {
      const cx<double> f = ipow<double>(-l) * c;
      Ft = Ft + tau * f;
      Fp = Fp + mul_i(pi * f);
    }
  }
  const double ik = 1.0 / k;
  const cx<double> Fx = ik * ((ct * cf) * Ft - sf * Fp);
  const cx<double> Fy = ik * ((ct * sf) * Ft + cf * Fp);
  const cx<double> Fz = ik * ((-st) * Ft);
  F[(size_t)e * 3 + 0] = tm_c128{Fx.re, Fx.im};
  F[(size_t)e * 3 + 1] = tm_c128{Fy.re, Fy.im};
  F[(size_t)e * 3 + 2] = tm_c128{Fz.re, Fz.im};
}

// v[i][n] = sum_c w_c Phi_n(k(xd - x_i))_c
// Cartesian components of the outgoing function Phi_n(k (dx, dy, dz)), FP64
// (the same definition as the near-field kernels: spherical components of
// M / N over sqrt(2l(l+1)), rotated to x, y, z).
__device__ void outgoing_xyz(int n, int lmax, double dx, double dy, double dz, double k,
                             cx<double>& Ex, cx<double>& Ey, cx<double>& Ez) {
  const double rho2 = dx * dx + dy * dy;
  const double rr = sqrt(rho2 + dz * dz);
  const double x = k * rr;
  double sn, cs;
  sincos(x, &sn, &cs);
  cx<double> h[LMAX_SUPPORTED + 1];
  hankel_set<double>(x, cs, sn, lmax, h);
  const double ct = dz / rr, st = sqrt(rho2) / rr;
  double cf = 1.0, sf = 0.0;
  if (rho2 > 0.0) {
    cf = dx / sqrt(rho2);
    sf = dy / sqrt(rho2);
  }
  int p, l, m;
  plm_of_n(n, lmax, p, l, m);
  double Pb, U, tau;
  legendre_one<double>(l, m < 0 ? -m : m, ct, st, Pb, U, tau);
  const double pi = (double)m * U;
  // e^{i m phi} = (cf + i sf)^m
  cx<double> em(1.0, 0.0);
  const cx<double> ef(cf, m < 0 ? -sf : sf);
  for (int q = 0; q < (m < 0 ? -m : m); ++q) em = em * ef;
  const double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
  cx<double> Er, Et, Ep;
  if (p == 0) {
    Et = mul_i(pi * h[l]);
    Ep = (-tau) * h[l];
  } else {
    const cx<double> dh = (1.0 / x) * (x * h[l - 1] - (double)l * h[l]);
    Er = ((double)(l * (l + 1)) / x * Pb) * h[l];
    Et = tau * dh;
    Ep = mul_i(pi * dh);
  }
  Er = nrm * (Er * em);
  Et = nrm * (Et * em);
  Ep = nrm * (Ep * em);
  Ex = (st * cf) * Er + (ct * cf) * Et - sf * Ep;
  Ey = (st * sf) * Er + (ct * sf) * Et + cf * Ep;
  Ez = ct * Er - st * Et;
}

__global__ void detector_kernel(double xdx, double xdy, double xdz, double wxr, double wxi,
                                double wyr, double wyi, double wzr, double wzi, int N, int L,
                                int lmax, SitePos sp, double k,
                                tm_c128* __restrict__ v) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)N * L) return;
  const int n = (int)(e % L);
  const long long i = e / L;
  cx<double> Ex, Ey, Ez;
  double sx_, sy_;
  sp.at(i, sx_, sy_);
  outgoing_xyz(n, lmax, xdx - sx_, xdy - sy_, xdz, k, Ex, Ey, Ez);
  const cx<double> o = cx<double>(wxr, wxi) * Ex + cx<double>(wyr, wyi) * Ey + cx<double>(wzr, wzi) * Ez;
  v[e] = tm_c128{o.re, o.im};
}

// Transpose of the near-field map: v[r][i][n] = sum_p sum_c w[r][p][c]
// Phi_n(k(x_p - x_i))_c.  One thread per (i, n) and right-hand side
// (blockIdx.y); points and weights stream through LDS in tiles of NFT_TILE.
constexpr int NFT_TILE = 256;
__global__ __launch_bounds__(256) void near_field_t_kernel(
    const double* __restrict__ pts, const tm_c128* __restrict__ w, int P, int N, int L, int lmax,
    SitePos sp, double k, tm_c128* __restrict__ v) {
  __shared__ double spt[NFT_TILE][3];
  __shared__ cplx<double> sw[NFT_TILE][3];
  const int r = blockIdx.y;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const bool active = e < (long long)N * L;
  const int n = active ? (int)(e % L) : 0;
  const long long i = active ? e / L : 0;
  double xi, yi;
  sp.at(i, xi, yi);
  cx<double> acc(0.0, 0.0);
  const tm_c128* wr = w + (size_t)r * P * 3;
  for (int p0 = 0; p0 < P; p0 += NFT_TILE) {
    const int np = min(NFT_TILE, P - p0);
    __syncthreads();
    for (int t = threadIdx.x; t < np; t += blockDim.x) {
      for (int c3 = 0; c3 < 3; ++c3) {
        spt[t][c3] = pts[(size_t)(p0 + t) * 3 + c3];
        const tm_c128 q = wr[(size_t)(p0 + t) * 3 + c3];
        sw[t][c3] = cplx<double>{q.re, q.im};
      }
    }
    __syncthreads();
    if (active) {
      for (int t = 0; t < np; ++t) {
        cx<double> Ex, Ey, Ez;
        outgoing_xyz(n, lmax, spt[t][0] - xi, spt[t][1] - yi, spt[t][2], k, Ex, Ey, Ez);
        acc = acc + cx<double>(sw[t][0].re, sw[t][0].im) * Ex + cx<double>(sw[t][1].re, sw[t][1].im) * Ey +
              cx<double>(sw[t][2].re, sw[t][2].im) * Ez;
      }
    }
  }
  if (active) v[(size_t)r * N * L + e] = tm_c128{acc.re, acc.im};
}

// grad[r][i] = 2 Re sum_slots mu * dt * aexc   (slot layout inputs)
__global__ void grad_kernel(const c128* __restrict__ mu, const c128* __restrict__ dt,
                            const c128* __restrict__ aexc, int R, int N, int S, double* __restrict__ g) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)R * N) return;
  const int r = (int)(e / N);
  const long long i = e % N;
  double acc = 0.0;
  for (int c = 0; c < NCLASS; ++c) {
    for (int sl = 0; sl < S; ++sl) {
      const size_t o = ((size_t)c * N + i) * S + sl;
      const size_t ov = (size_t)r * NCLASS * N * S + o;
      const c128 a = mu[ov], d = dt[o], b = aexc[ov];
      const double pr = a.re * d.re - a.im * d.im, pi = a.re * d.im + a.im * d.re;
      acc += pr * b.re - pi * b.im;
    }
  }
  g[e] = 2.0 * acc;
}

static inline unsigned nblk(long long n, int t = 256) { return (unsigned)((n + t - 1) / t); }

// ---------------------------------------------------------------- position gradient
// Coupling and incident terms of dO/dx_i, dO/dy_i (slot layout inputs):
//   g_a = 2 Re[ lam_i . (D_a s)_i - s_i . (D_a^T lam)_i + i k khat_a lam_i . a0_i ],
// lam = T^T mu, D_a the derivative blocks of the coupling operator.  One
// thread per (rhs, scatterer); grad [R][N][2].
struct GposArgs {
  double kk[2 * 16];  // k khat_x, k khat_y per right-hand side of the chunk
  int use_inc;
};
__global__ void gpos_contract_kernel(const c128* __restrict__ lam, const c128* __restrict__ s,
                                     const c128* __restrict__ a0, const c128* __restrict__ dxs,
                                     const c128* __restrict__ dys, const c128* __restrict__ dxtl,
                                     const c128* __restrict__ dytl, int R, int N, int S, GposArgs ga,
                                     double* __restrict__ grad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)R * N) return;
  const int r = (int)(e / N);
  const long long i = e % N;
  double gxr = 0.0, gyr = 0.0, ir = 0.0, ii = 0.0;
  for (int c = 0; c < NCLASS; ++c) {
    for (int sl = 0; sl < S; ++sl) {
      const size_t o = (((size_t)r * NCLASS + c) * N + i) * S + sl;
      const c128 l = lam[o], x = s[o];
      const c128 p = dxs[o], q = dys[o], u = dxtl[o], v = dytl[o];
      // Re(l p) - Re(x u)
      gxr += (l.re * p.re - l.im * p.im) - (x.re * u.re - x.im * u.im);
      gyr += (l.re * q.re - l.im * q.im) - (x.re * v.re - x.im * v.im);
      if (ga.use_inc) {
        const c128 b = a0[o];
        ir += l.re * b.re - l.im * b.im;
        ii += l.re * b.im + l.im * b.re;
      }
    }
  }
  // Re(i kk (ir + i ii)) = -kk ii
  grad[e * 2 + 0] = 2.0 * (gxr - ga.kk[2 * r] * ii);
  grad[e * 2 + 1] = 2.0 * (gyr - ga.kk[2 * r + 1] * ii);
}

// Detector term: grad[r][i][a] += 2 Re[ sum_u s_iu d/dx_i,a (sum_c w_c Phi_u(k(xd - x_i))_c) ]
// for a = x, y.  By the addition theorem about x_d, Phi_u(k(xd - x_i)) =
// sum_v xi_uv(k(xd - x_i)) R Phi_v(0); only the three N-type l' = 1 regular
// waves are nonzero at their centre, so the derivative is
// -sum_v grad xi_uv(d) W_v with W_v = w . R Phi_v(0) and
// grad xi_uv = e^{i mu phi} sum_q C_uvq [k h_q' Pbar rhat + h_q tau thhat / r
//                                         + i mu h_q (Pbar/sin) phhat / r].
struct DgradArgs {
  double W[16 * 3 * 2];  // W_v per right-hand side of the chunk (re, im)
};
__global__ void gpos_detector_kernel(const tm_c128* __restrict__ s, const c128* __restrict__ coef,
                                     const int* __restrict__ dm, int R, int N, int L, int lmax,
                                     SitePos sp, double k,
                                     double xdx, double xdy, double xdz, DgradArgs wa,
                                     double* __restrict__ grad) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)R * N) return;
  const int r = (int)(e / N);
  const long long i = e % N;
  double sx_, sy_;
  sp.at(i, sx_, sy_);
  const double dx = xdx - sx_;
  const double dy = xdy - sy_;
  const double dz = xdz;
  const double rho2 = dx * dx + dy * dy;
  const double rr = sqrt(rho2 + dz * dz);
  const double x = k * rr;
  double sn, cs;
  sincos(x, &sn, &cs);
  cx<double> h[LMAX_SUPPORTED + 3];
  hankel_set<double>(x, cs, sn, lmax + 2, h);
  const double ct = dz / rr, st = sqrt(rho2) / rr;
  double cf = 1.0, sf = 0.0;
  if (rho2 > 0.0) {
    cf = dx / sqrt(rho2);
    sf = dy / sqrt(rho2);
  }
  const double rh[2] = {st * cf, st * sf}, th[2] = {ct * cf, ct * sf}, ph[2] = {-sf, cf};
  const int Q = lmax + 2;
  cx<double> acc[2];
  const tm_c128* si = s + ((size_t)r * N + i) * L;
  for (int u = 0; u < L; ++u) {
    const cx<double> su(si[u].re, si[u].im);
    for (int v = 0; v < 3; ++v) {
      const cx<double> W(wa.W[(r * 3 + v) * 2], wa.W[(r * 3 + v) * 2 + 1]);
      const int mu = dm[u * 3 + v], am = mu < 0 ? -mu : mu;
      cx<double> gr, gt, gp;
      for (int q = am; q < Q; ++q) {
        const c128 cq = coef[((size_t)u * 3 + v) * Q + q];
        if (cq.re == 0.0 && cq.im == 0.0) continue;
        const cx<double> C(cq.re, cq.im);
        double P, U, tau;
        legendre_one<double>(q, am, ct, st, P, U, tau);
        const cx<double> hq = h[q];
        const cx<double> hp = (q == 0) ? cx<double>(-h[1].re, -h[1].im)
                                       : h[q - 1] - ((double)(q + 1) / x) * hq;
        gr = gr + (k * P) * (C * hp);
        gt = gt + (tau / rr) * (C * hq);
        gp = gp + ((double)mu * U / rr) * mul_i(C * hq);
      }
      double sm, cm;
      sincos((double)mu * atan2(sf, cf), &sm, &cm);
      const cx<double> em(cm, sm);
      for (int a = 0; a < 2; ++a) {
        const cx<double> G = em * (rh[a] * gr + th[a] * gt + ph[a] * gp);
        acc[a] = acc[a] - su * (G * W);
      }
    }
  }
  grad[e * 2 + 0] += 2.0 * acc[0].re;
  grad[e * 2 + 1] += 2.0 * acc[1].re;
}

int launch_gpos_contract(tm_ctx* c, int R, const c128* lam, const c128* s, const c128* a0,
                         const c128* dxs, const c128* dys, const c128* dxtl, const c128* dytl,
                         const double* khat, double* grad) {
  const Geometry& g = c->g;
  const long long vec = g.vec_len();
  for (int r0 = 0; r0 < R; r0 += 16) {
    const int nr = std::min(16, R - r0);
    GposArgs ga{};
    ga.use_inc = khat ? 1 : 0;
    for (int r = 0; r < nr && khat; ++r) {
      ga.kk[2 * r] = g.k * khat[3 * (r0 + r)];
      ga.kk[2 * r + 1] = g.k * khat[3 * (r0 + r) + 1];
    }
    const size_t off = (size_t)r0 * vec;
    hipLaunchKernelGGL(gpos_contract_kernel, dim3(nblk((long long)nr * g.n)), dim3(256), 0,
                       c->stream, lam + off, s + off, a0 ? a0 + off : nullptr, dxs + off, dys + off,
                       dxtl + off, dytl + off, nr, g.n, g.S, ga, grad + (size_t)r0 * g.n * 2);
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_gpos_detector(tm_ctx* c, int R, const tm_c128* s, const c128* coef, const int* dm,
                         const double* xd, const tm_c128* w, double* grad) {
  const Geometry& g = c->g;
  // w . R Phi_v(0) for the N-type l' = 1 regular waves at their centre:
  // R Phi_{1,-1}(0) = (1/3) sqrt(3/4) (1, -i, 0), R Phi_{1,0}(0) = (1/3) sqrt(3/2) (0, 0, 1),
  // R Phi_{1,+1}(0) = (1/3) sqrt(3/4) (1, i, 0)  (j_1(r)/r -> 1/3, (r j_1)'/r -> 2/3)
  const double a = sqrt(0.75) / 3.0, b = sqrt(1.5) / 3.0;
  for (int r0 = 0; r0 < R; r0 += 16) {
    const int nr = std::min(16, R - r0);
    DgradArgs wa{};
    for (int r = 0; r < nr; ++r) {
      const tm_c128* wr = w + 3 * (r0 + r);
      // (1, -i, 0) . w = wx - i wy ; (1, i, 0) . w = wx + i wy
      wa.W[(r * 3 + 0) * 2] = a * (wr[0].re + wr[1].im);
      wa.W[(r * 3 + 0) * 2 + 1] = a * (wr[0].im - wr[1].re);
      wa.W[(r * 3 + 1) * 2] = b * wr[2].re;
      wa.W[(r * 3 + 1) * 2 + 1] = b * wr[2].im;
      wa.W[(r * 3 + 2) * 2] = a * (wr[0].re - wr[1].im);
      wa.W[(r * 3 + 2) * 2 + 1] = a * (wr[0].im + wr[1].re);
    }
    hipLaunchKernelGGL(gpos_detector_kernel, dim3(nblk((long long)nr * g.n)), dim3(256), 0,
                       c->stream, s + (size_t)r0 * g.n * g.L, coef, dm, nr, g.n, g.L, g.lmax,
                       site_pos(c), g.k, xd[0], xd[1], xd[2], wa,
                       grad + (size_t)r0 * g.n * 2);
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}



// ---------------------------------------------------------------- null-field T-matrix
// T-matrix of a body of revolution about z by the null-field method (App.
// I.B): for each m the matrices of surface integrals
//   O_ab = 2 pi sum_nodes w [ R Phi_{l'mp'}(k_s x) x Phi_{l,-m,1-p}(k_b x)
//                             + (k_s/k_b) R Phi_{l'm,1-p'}(k_s x) x Phi_{l,-m,p}(k_b x) ] . n
// (outgoing test waves) and R_ab (the same with regular test waves), a = (l, p),
// b = (l', p'), and T_m = -R O^{-1}.  The two terms add and the regular-test
// matrix multiplies the inverse, the forms that reproduce the Lorenz-Mie T on
// a sphere in this basis.  One workgroup per (scatterer, m); the surface is a
// cylinder of radius a_i and height h centred on the scatterer (bottom cap,
// side, top cap, nq Gauss-Legendre nodes each).
constexpr int EB_NB = 2 * LMAX_SUPPORTED;       // largest m block (l = 1..lmax, two types)
constexpr int EB_CHUNK = 32;                    // surface nodes staged per pass

// j_l(z), l = 0..lmax+1 at complex z by the power series (|z| <= 12)
__device__ inline void sph_j_all(int lmax, cx<double> z, cx<double>* j) {
  for (int l = 0; l <= lmax; ++l) j[l] = sph_j_series(l, z);
}

// Spherical components (r, theta, phi) of Phi_lmp without e^{imphi}, from the
// radial pair (z_l, (x z_l)'/x at x) and the Legendre data (Pbar, m Pbar/sin, tau).
__device__ inline void vswf_rtp(int l, int p, cx<double> zl, cx<double> dz, cx<double> x, double P,
                                double pim, double tau, cx<double>* v) {
  const double nrm = 1.0 / sqrt(2.0 * l * (l + 1));
  if (p == 0) {
    v[0] = cx<double>(0.0, 0.0);
    v[1] = nrm * mul_i(pim * zl);
    v[2] = (-nrm * tau) * zl;
  } else {
    v[0] = (nrm * l * (l + 1) * P) * (zl / x);
    v[1] = (nrm * tau) * dz;
    v[2] = mul_i((nrm * pim) * dz);
  }
}

__device__ inline cx<double> cross_dot_n(const cx<double>* a, const cx<double>* b, double nr, double nt) {
  // (a x b) . n with n = (nr, nt, 0) in (r, theta, phi)
  const cx<double> cr = a[1] * b[2] - a[2] * b[1];
  const cx<double> ct = a[2] * b[0] - a[0] * b[2];
  return nr * cr + nt * ct;
}

struct EbNode {
  double r, th, nr, nt, w;
};

__global__ __launch_bounds__(256) void ebcm_cylinder_kernel(const double* __restrict__ radii, double height,
                                                            double k, double nre, double nim, int lmax,
                                                            int nq, const double* __restrict__ gl,
                                                            tm_c128* __restrict__ T) {
  const int i = blockIdx.x;
  const int m = (int)blockIdx.y - lmax;
  const int am = m < 0 ? -m : m;
  const int l0 = am > 1 ? am : 1;
  const int nl = lmax - l0 + 1, nb = 2 * nl;
  const int L = 2 * lmax * (lmax + 2);
  const double a = radii[i];
  const cx<double> nrel(nre, nim);
  const cx<double> ks = k * nrel;
  __shared__ EbNode nodes[EB_CHUNK];
  // per node: test waves (outgoing and regular at k_b) and internal waves (regular at k_s),
  // each for l = l0..lmax and both types, in (r, theta, phi) components
  __shared__ cplx<double> wout[EB_CHUNK][EB_NB][3], wreg[EB_CHUNK][EB_NB][3], wint[EB_CHUNK][EB_NB][3];
  __shared__ cplx<double> Pm[EB_NB][EB_NB], Qm[EB_NB][EB_NB];
  const int tid = threadIdx.x;
  const int ea = tid / EB_NB, eb = tid % EB_NB;  // entry (a, b) of this thread
  const bool own = tid < EB_NB * EB_NB && ea < nb && eb < nb;
  cx<double> accO, accR;
  const int total = 3 * nq;
  for (int n0 = 0; n0 < total; n0 += EB_CHUNK) {
    const int cnt = min(EB_CHUNK, total - n0);
    __syncthreads();
    if (tid < cnt) {
      // node n0 + tid on the generating curve: segment, Gauss-Legendre point
      const int q = n0 + tid, seg = q / nq, g = q % nq;
      const double u = 0.5 * (gl[2 * g] + 1.0), wg = gl[2 * g + 1];
      double rho, z, ncr, ncz, wl;
      if (seg == 0) {        // bottom cap, normal -z
        rho = a * u; z = -0.5 * height; ncr = 0.0; ncz = -1.0; wl = 0.5 * a * wg;
      } else if (seg == 1) { // side, normal rho_hat
        rho = a; z = height * (u - 0.5); ncr = 1.0; ncz = 0.0; wl = 0.5 * height * wg;
      } else {               // top cap, normal +z
        rho = a * u; z = 0.5 * height; ncr = 0.0; ncz = 1.0; wl = 0.5 * a * wg;
      }
      const double r = sqrt(rho * rho + z * z), th = atan2(rho, z);
      const double st = sin(th), ct = cos(th);
      EbNode nd;
      nd.r = r;
      nd.th = th;
      nd.nr = ncr * st + ncz * ct;
      nd.nt = ncr * ct - ncz * st;
      nd.w = wl * rho;
      nodes[tid] = nd;
      // radial functions
      const double xb = k * r;
      double sn, cs;
      sincos(xb, &sn, &cs);
      cx<double> hb[LMAX_SUPPORTED + 2], jb[LMAX_SUPPORTED + 2], js[LMAX_SUPPORTED + 2];
      hankel_set<double>(xb, cs, sn, lmax, hb);
      sph_j_all(lmax, cx<double>(xb, 0.0), jb);
      const cx<double> xs = r * ks;
      sph_j_all(lmax, xs, js);
      for (int li = 0; li < nl; ++li) {
        const int l = l0 + li;
        double P, U, tau;
        legendre_one<double>(l, am, ct, st, P, U, tau);
        const double pim = (double)m * U;  // the internal waves carry +m
        const cx<double> X(xb, 0.0);
        const cx<double> dhb = hb[l - 1] - ((double)l / xb) * hb[l];
        const cx<double> djb = jb[l - 1] - ((double)l / xb) * jb[l];
        const cx<double> djs = js[l - 1] - ((double)l) * (js[l] / xs);
        for (int p = 0; p < 2; ++p) {
          cx<double> v[3];
          // test waves carry -m: pi changes sign, Pbar and tau do not
          vswf_rtp(l, p, hb[l], dhb, X, P, -pim, tau, v);
          for (int c = 0; c < 3; ++c) wout[tid][2 * li + p][c] = cplx<double>{v[c].re, v[c].im};
          vswf_rtp(l, p, jb[l], djb, X, P, -pim, tau, v);
          for (int c = 0; c < 3; ++c) wreg[tid][2 * li + p][c] = cplx<double>{v[c].re, v[c].im};
          vswf_rtp(l, p, js[l], djs, xs, P, pim, tau, v);
          for (int c = 0; c < 3; ++c) wint[tid][2 * li + p][c] = cplx<double>{v[c].re, v[c].im};
        }
      }
    }
    __syncthreads();
    if (own) {
      // row a = (l, p) -> test index 2 li + p; column b = (l', p') -> internal
      const int la = ea >> 1, pa = ea & 1, lb = eb >> 1, pb = eb & 1;
      const cx<double> ratio = ks / cx<double>(k, 0.0);
      for (int q = 0; q < cnt; ++q) {
        const EbNode nd = nodes[q];
        cx<double> ip[3], iq[3], o1[3], o0[3], r1[3], r0[3];
        for (int c = 0; c < 3; ++c) {
          ip[c] = cx<double>(wint[q][2 * lb + pb][c].re, wint[q][2 * lb + pb][c].im);
          iq[c] = cx<double>(wint[q][2 * lb + 1 - pb][c].re, wint[q][2 * lb + 1 - pb][c].im);
          o1[c] = cx<double>(wout[q][2 * la + 1 - pa][c].re, wout[q][2 * la + 1 - pa][c].im);
          o0[c] = cx<double>(wout[q][2 * la + pa][c].re, wout[q][2 * la + pa][c].im);
          r1[c] = cx<double>(wreg[q][2 * la + 1 - pa][c].re, wreg[q][2 * la + 1 - pa][c].im);
          r0[c] = cx<double>(wreg[q][2 * la + pa][c].re, wreg[q][2 * la + pa][c].im);
        }
        const cx<double> fo = cross_dot_n(ip, o1, nd.nr, nd.nt) + ratio * cross_dot_n(iq, o0, nd.nr, nd.nt);
        const cx<double> fr = cross_dot_n(ip, r1, nd.nr, nd.nt) + ratio * cross_dot_n(iq, r0, nd.nr, nd.nt);
        accO = accO + nd.w * fo;
        accR = accR + nd.w * fr;
      }
    }
  }
  if (own) {
    const double tp = 6.283185307179586476925286766559;
    Pm[ea][eb] = cplx<double>{tp * accO.re, tp * accO.im};
    Qm[ea][eb] = cplx<double>{tp * accR.re, tp * accR.im};
  }
  __syncthreads();
  if (tid == 0) {
    // T_m O = -R  <=>  O^T T_m^T = -R^T: Gaussian elimination with partial
    // pivoting on O^T (columns of the unknown: the rows of T_m)
    cx<double> A[EB_NB][EB_NB], B[EB_NB][EB_NB];
    for (int r_ = 0; r_ < nb; ++r_)
      for (int c_ = 0; c_ < nb; ++c_) {
        A[r_][c_] = cx<double>(Pm[c_][r_].re, Pm[c_][r_].im);   // O^T
        B[r_][c_] = cx<double>(-Qm[c_][r_].re, -Qm[c_][r_].im); // -R^T
      }
    for (int c_ = 0; c_ < nb; ++c_) {
      int piv = c_;
      double best = -1.0;
      for (int r_ = c_; r_ < nb; ++r_) {
        const double v = A[r_][c_].re * A[r_][c_].re + A[r_][c_].im * A[r_][c_].im;
        if (v > best) {
          best = v;
          piv = r_;
        }
      }
      if (piv != c_)
        for (int q = 0; q < nb; ++q) {
          const cx<double> t1 = A[c_][q];
          A[c_][q] = A[piv][q];
          A[piv][q] = t1;
          const cx<double> t2 = B[c_][q];
          B[c_][q] = B[piv][q];
          B[piv][q] = t2;
        }
      const cx<double> inv = cx<double>(1.0, 0.0) / A[c_][c_];
      for (int r_ = c_ + 1; r_ < nb; ++r_) {
        const cx<double> f = A[r_][c_] * inv;
        for (int q = c_; q < nb; ++q) A[r_][q] = A[r_][q] - f * A[c_][q];
        for (int q = 0; q < nb; ++q) B[r_][q] = B[r_][q] - f * B[c_][q];
      }
    }
    for (int r_ = nb - 1; r_ >= 0; --r_) {
      const cx<double> inv = cx<double>(1.0, 0.0) / A[r_][r_];
      for (int q = 0; q < nb; ++q) {
        cx<double> acc = B[r_][q];
        for (int c_ = r_ + 1; c_ < nb; ++c_) acc = acc - A[r_][c_] * B[c_][q];
        B[r_][q] = acc * inv;
      }
    }
    // B = T_m^T: T_m[a][b] = B[b][a]; scatter into the boundary order
    tm_c128* Ti = T + (size_t)i * L * L;
    const int half = lmax * (lmax + 2);
    for (int a_ = 0; a_ < nb; ++a_)
      for (int b_ = 0; b_ < nb; ++b_) {
        const int la = l0 + (a_ >> 1), pa = a_ & 1, lb = l0 + (b_ >> 1), pb = b_ & 1;
        const int na = pa * half + la * (la + 1) - 1 + m, nbi = pb * half + lb * (lb + 1) - 1 + m;
        Ti[(size_t)na * L + nbi] = tm_c128{B[b_][a_].re, B[b_][a_].im};
      }
  }
}

__global__ void fill_c128_kernel(tm_c128* __restrict__ p, long long n) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = tm_c128{0.0, 0.0};
}

// Gauss-Legendre nodes and weights on [-1, 1] as (x, w) pairs.
static void gauss_legendre(int n, std::vector<double>& out) {
  out.assign((size_t)2 * n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = cos(pi * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      pp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    out[2 * i] = z;
    out[2 * i + 1] = 2.0 / ((1.0 - z * z) * pp * pp);
  }
}

// Dense T of N cylinders (radii device [N]) into T device [N][L][L].
int launch_ebcm_cylinders(tm_ctx* c, hipStream_t st, int N, const double* radii, double height, double k,
                          double nre, double nim, int lmax, int nq, tm_c128* T) {
  std::vector<double> gl;
  gauss_legendre(nq, gl);
  double* dgl = nullptr;
  if (hipMalloc((void**)&dgl, gl.size() * sizeof(double)) != hipSuccess) {
    (void)hipGetLastError();
    return c ? set_err(c, TM_ERR_OOM, "device allocation failed") : TM_ERR_OOM;
  }
  const int L = 2 * lmax * (lmax + 2);
  int rc = TM_OK;
  if (hipMemcpyAsync(dgl, gl.data(), gl.size() * sizeof(double), hipMemcpyHostToDevice, st) != hipSuccess)
    rc = TM_ERR_HIP;
  if (rc == TM_OK) {
    const long long tot = (long long)N * L * L;
    hipLaunchKernelGGL(fill_c128_kernel, dim3(nblk(tot)), dim3(256), 0, st, T, tot);
    hipLaunchKernelGGL(ebcm_cylinder_kernel, dim3(N, 2 * lmax + 1), dim3(256), 0, st, radii, height, k,
                       nre, nim, lmax, nq, dgl, T);
    if (hipGetLastError() != hipSuccess) rc = TM_ERR_HIP;
  }
  // the host nodes are read by the asynchronous copy; the buffer goes after the launch
  if (hipStreamSynchronize(st) != hipSuccess) rc = TM_ERR_HIP;
  hipFree(dgl);
  if (rc != TM_OK && c) set_err(c, rc, "null-field T-matrix launch failed");
  return rc;
}

// ---------------------------------------------------------------- jinc sources
// Expansion coefficients of a jinc source (App. II, "Implementing jinc source
// in the vector spherical harmonic basis") about every scatterer: the source
// field is the disk of plane waves
//   E(x) = (1/2pi) int int A(b, a) e^{i k(b, a).(x - x0)} sin b cos b da db,
// and its coefficients about x_i integrate the plane-wave coefficients of App.
// II over the disk with the field phase e^{i k.(x_i - x0)}.  The azimuthal
// integral is taken in closed form,
//   Gamma_m(xi, eta, rho) = (i^{m-1} e^{-i m xi}/2) [e^{i(xi-eta)} J_{m-1}(rho)
//                                                   - e^{-i(xi-eta)} J_{m+1}(rho)],
// with (rho_t, phi0, z_c) the cylindrical coordinates of x_i - x0 and
// rho = k rho_t sin b; the polar integral is Gauss-Legendre on [0, pi/2].
// One thread per (source, scatterer, coefficient), as the paper assigns them.

// J_n(x) for |n| <= 8 and x >= 0: power series below x = 8 (at most three
// digits of cancellation), else upward recurrence from J_0, J_1 (stable
// while n < x); J_{-n} = (-1)^n J_n.
__device__ inline double bessel_jn(int n, double x) {
  const int an = n < 0 ? -n : n;
  const double sg = (n < 0 && (an & 1)) ? -1.0 : 1.0;
  double v;
  if (x < 8.0) {
    const double h = 0.5 * x, h2 = -h * h;
    double term = 1.0;
    for (int q = 1; q <= an; ++q) term *= h / (double)q;  // (x/2)^n / n!
    double sum = term;
    for (int kk = 1; kk < 60; ++kk) {
      term *= h2 / ((double)kk * (double)(kk + an));
      sum += term;
      if (fabs(term) < 1e-17 * fabs(sum)) break;
    }
    v = sum;
  } else {
    double jm = j0(x), jc = j1(x);
    if (an == 0) {
      v = jm;
    } else {
      for (int q = 1; q < an; ++q) {
        const double jn = (2.0 * q / x) * jc - jm;
        jm = jc;
        jc = jn;
      }
      v = jc;
    }
  }
  return sg * v;
}

// Gamma_m(xi, eta, rho) from J_{m-1}(rho), J_{m+1}(rho)
__device__ inline cx<double> gamma_m(int m, double xi, double eta, double jm1, double jp1) {
  double s1, c1, s2, c2;
  sincos(-(double)m * xi, &s1, &c1);
  sincos(xi - eta, &s2, &c2);
  const cx<double> pre = ipow<double>(m - 1) * cx<double>(0.5 * c1, 0.5 * s1);
  const cx<double> br(c2 * jm1 - c2 * jp1, s2 * jm1 + s2 * jp1);  // e^{i d} J- - e^{-i d} J+
  return pre * br;
}

// nodes: [nb][3] = (sin b, cos b, weight) of Gauss-Legendre on [0, pi/2]
__device__ cx<double> jinc_coeff(int n, int lmax, double dx, double dy, double dz, double k,
                                 cx<double> Ax, cx<double> Ay, const double* __restrict__ nodes,
                                 int nb) {
  int p, l, m;
  plm_of_n(n, lmax, p, l, m);
  const int am = m < 0 ? -m : m;
  const double rho_t = sqrt(dx * dx + dy * dy);
  const double phi0 = rho_t > 0.0 ? atan2(dy, dx) : 0.0;
  const double nrm = -4.0 / sqrt(2.0 * l * (l + 1));
  const cx<double> il = ipow<double>(p == 0 ? l : l + 1);
  cx<double> acc;
  for (int q = 0; q < nb; ++q) {
    const double sb = nodes[3 * q], cb = nodes[3 * q + 1], w = nodes[3 * q + 2];
    double P, U, tau;
    legendre_one<double>(l, am, cb, sb, P, U, tau);
    const double pi = (double)m * U;  // m Pbar / sin b
    const double rho = k * rho_t * sb;
    const double jm1 = bessel_jn(m - 1, rho), jp1 = bessel_jn(m + 1, rho);
    const cx<double> g0 = gamma_m(m, phi0, 0.0, jm1, jp1);
    const cx<double> g1 = gamma_m(m, phi0, 0.5 * 3.14159265358979323846, jm1, jp1);
    cx<double> c0, c1;
    if (p == 0) {
      c0 = mul_i(pi * Ax) + (tau * cb) * Ay;
      c1 = mul_i(pi * Ay) - (tau * cb) * Ax;
    } else {
      c0 = tau * Ax - mul_i((pi * cb) * Ay);
      c1 = tau * Ay + mul_i((pi * cb) * Ax);
    }
    double sz, cz;
    sincos(k * dz * cb, &sz, &cz);
    acc = acc + (w * nrm * sb) * (cx<double>(cz, sz) * (c0 * g0 + c1 * g1));
  }
  return il * acc;
}

struct JincSrc {
  double x0, y0, z0;
  double axr, axi, ayr, ayi;
};

// a0[r][i][n] = coefficients of source r about scatterer i (one lattice)
__global__ void jinc_rhs_kernel(const JincSrc* __restrict__ src, int R, int N, int L, int lmax,
                                SitePos sp, double k,
                                const double* __restrict__ nodes, int nb, tm_c128* __restrict__ a0) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long long)R * N * L) return;
  const int n = (int)(e % L);
  const long long i = (e / L) % N;
  const int r = (int)(e / ((long long)L * N));
  const JincSrc s = src[r];
  double xi, yi;
  sp.at(i, xi, yi);
  const cx<double> v = jinc_coeff(n, lmax, xi - s.x0, yi - s.y0, -s.z0, k, cx<double>(s.axr, s.axi),
                                  cx<double>(s.ayr, s.ayi), nodes, nb);
  a0[e] = tm_c128{v.re, v.im};
}

// Packed subregion layout [S][R][N_k][L] (concatenated): system (k, r) gets
// the sum over its group of sources src[grp[k R + r] .. grp[k R + r + 1]).
__global__ void jinc_rhs_packed_kernel(const JincSrc* __restrict__ src, const int* __restrict__ grp,
                                       const SubParams* __restrict__ sp,
                                       const long long* __restrict__ out_off, int S, int R, int L,
                                       int lmax, double x0, double y0, double pitch, double k,
                                       const double* __restrict__ nodes, int nb, long long total,
                                       tm_c128* __restrict__ a0) {
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
  const int n = (int)(q % L);
  q /= L;
  const long long site = q % Nk;
  const int r = (int)(q / Nk);
  const double xi = x0 + pitch * (double)(p.ox + site % p.nx);
  const double yi = y0 + pitch * (double)(p.oy + site / p.nx);
  cx<double> acc;
  for (int j = grp[lo * R + r]; j < grp[lo * R + r + 1]; ++j) {
    const JincSrc s = src[j];
    acc = acc + jinc_coeff(n, lmax, xi - s.x0, yi - s.y0, -s.z0, k, cx<double>(s.axr, s.axi),
                           cx<double>(s.ayr, s.ayi), nodes, nb);
  }
  a0[e] = tm_c128{acc.re, acc.im};
}

// Gauss-Legendre nodes on [0, pi/2] (Newton on P_n from the Chebyshev-like
// first guesses) as (sin b, cos b, weight) triples.
static void beta_nodes(int n, std::vector<double>& out) {
  out.assign((size_t)3 * n, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = cos(pi * (i + 0.75) / (n + 0.5)), pp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int j = 2; j <= n; ++j) {
        const double p2 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p0) / j;
        p0 = p1;
        p1 = p2;
      }
      if (n == 1) {
        p1 = z;
        p0 = 1.0;
      }
      pp = n * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / pp;
      z -= dz;
      if (fabs(dz) < 1e-16) break;
    }
    const double w = 2.0 / ((1.0 - z * z) * pp * pp);
    const double b = 0.25 * pi * (z + 1.0);
    out[3 * i] = sin(b);
    out[3 * i + 1] = cos(b);
    out[3 * i + 2] = 0.25 * pi * w;
  }
}

// Polar nodes for sources up to a distance rmax from the scatterers: the
// integrand oscillates like e^{i k z cos b} J(k rho sin b), k rmax radians over
// the interval.
int jinc_beta_count(double k, double rmax) { return 40 + (int)ceil(k * rmax); }

static int upload_jinc(tm_ctx* c, int nsrc, const tm_jinc* src, int nb, DevBuf& buf,
                       JincSrc** dsrc, double** dnodes, size_t extra, void** dextra) {
  std::vector<JincSrc> hs((size_t)nsrc);
  for (int j = 0; j < nsrc; ++j)
    hs[j] = JincSrc{src[j].x0, src[j].y0, src[j].z0, src[j].ax.re, src[j].ax.im, src[j].ay.re,
                    src[j].ay.im};
  std::vector<double> nodes;
  beta_nodes(nb, nodes);
  const size_t sb = ((hs.size() * sizeof(JincSrc)) + 255) & ~(size_t)255;
  const size_t nbb = ((nodes.size() * sizeof(double)) + 255) & ~(size_t)255;
  int rc;
  if ((rc = ensure(c, buf, sb + nbb + extra)) != TM_OK) return rc;
  *dsrc = (JincSrc*)buf.p;
  *dnodes = (double*)((char*)buf.p + sb);
  if (dextra) *dextra = (char*)buf.p + sb + nbb;
  TM_HIP(c, hipMemcpyAsync(*dsrc, hs.data(), hs.size() * sizeof(JincSrc), hipMemcpyHostToDevice,
                           c->stream));
  TM_HIP(c, hipMemcpyAsync(*dnodes, nodes.data(), nodes.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  // the host vectors die with this call: wait for the copies
  TM_HIP(c, hipStreamSynchronize(c->stream));
  return TM_OK;
}

int launch_jinc_rhs(tm_ctx* c, int R, const tm_jinc* src, int nb, tm_c128* a0) {
  const Geometry& g = c->g;
  JincSrc* dsrc;
  double* dnodes;
  int rc;
  if ((rc = upload_jinc(c, R, src, nb, c->jinc_buf, &dsrc, &dnodes, 0, nullptr)) != TM_OK) return rc;
  const long long total = (long long)R * g.n * g.L;
  hipLaunchKernelGGL(jinc_rhs_kernel, dim3(nblk(total)), dim3(256), 0, c->stream, dsrc, R, g.n, g.L,
                     g.lmax, site_pos(c), g.k, dnodes, nb, a0);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_jinc_rhs_packed(tm_ctx* c, int S, const tm_subregion* subs, int R, int nsrc,
                           const tm_jinc* src, const int* grp, int nb, tm_c128* a0) {
  const Geometry& g = c->g;
  std::vector<SubParams> sp((size_t)S);
  std::vector<long long> off((size_t)S);
  long long tot = 0;
  for (int k = 0; k < S; ++k) {
    sp[k] = SubParams{subs[k].side_x, subs[k].side_y, 0, subs[k].origin_x, subs[k].origin_y, 0, 0};
    off[k] = tot;
    tot += (long long)R * subs[k].side_x * subs[k].side_y * g.L;
  }
  const size_t b_sp = ((sp.size() * sizeof(SubParams)) + 255) & ~(size_t)255;
  const size_t b_off = ((off.size() * sizeof(long long)) + 255) & ~(size_t)255;
  const size_t b_grp = (size_t)(S * R + 1) * sizeof(int);
  JincSrc* dsrc;
  double* dnodes;
  void* dx;
  int rc;
  if ((rc = upload_jinc(c, nsrc, src, nb, c->jinc_buf, &dsrc, &dnodes, b_sp + b_off + b_grp, &dx)) !=
      TM_OK)
    return rc;
  SubParams* dsp = (SubParams*)dx;
  long long* doff = (long long*)((char*)dx + b_sp);
  int* dgrp = (int*)((char*)dx + b_sp + b_off);
  TM_HIP(c, hipMemcpyAsync(dsp, sp.data(), sp.size() * sizeof(SubParams), hipMemcpyHostToDevice, c->stream));
  TM_HIP(c, hipMemcpyAsync(doff, off.data(), off.size() * sizeof(long long), hipMemcpyHostToDevice, c->stream));
  TM_HIP(c, hipMemcpyAsync(dgrp, grp, b_grp, hipMemcpyHostToDevice, c->stream));
  hipLaunchKernelGGL(jinc_rhs_packed_kernel, dim3(nblk(tot)), dim3(256), 0, c->stream, dsrc, dgrp, dsp,
                     doff, S, R, g.L, g.lmax, g.x0, g.y0, g.pitch, g.k, dnodes, nb, tot, a0);
  TM_HIP(c, hipGetLastError());
  // the host arrays above are read by the asynchronous copies
  TM_HIP(c, hipStreamSynchronize(c->stream));
  return TM_OK;
}

int launch_mie(tm_ctx* c, const double* radii, double n_re, double n_im) {
  const Geometry& g = c->g;
  hipLaunchKernelGGL(mie_kernel, dim3(nblk(g.n, 64)), dim3(64), 0, c->stream, radii, g.n, g.k,
                     n_re, n_im, g.lmax, c->maps, (c128*)c->t64.p, (c64*)c->t32.p,
                     (c128*)c->dt64.p);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_tdense(tm_ctx* c, int R, int mode, const c128* x, const c128* z, c128* y) {
  const Geometry& g = c->g;
  const long long total = (long long)R * g.vec_len();
  if (c->t_mblock)
    hipLaunchKernelGGL(tdense_mb_kernel, dim3(nblk(total)), dim3(256), 0, c->stream,
                       (const c128*)c->tmb.p, c->mbmaps, c->maps, (long long)g.n, mode, x, z, y,
                       total);
  else
    hipLaunchKernelGGL(tdense_kernel, dim3(nblk(total)), dim3(256), 0, c->stream,
                       (const tm_c128*)c->tden.p, c->maps, (long long)g.n, mode, x, z, y, total);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int tdense_prepare(tm_ctx* c) {
  const Geometry& g = c->g;
  const MbMaps& mb = c->mbmaps;
  c->t_mblock = false;
  int rc;
  if ((rc = ensure(c, c->tmflag, sizeof(int))) != TM_OK) return rc;
  TM_HIP(c, hipMemsetAsync(c->tmflag.p, 0, sizeof(int), c->stream));
  const long long total = (long long)g.n * g.L * g.L;
  const long long nb = std::min<long long>(nblk(total), 8192);
  hipLaunchKernelGGL(tdense_mcheck_kernel, dim3((unsigned)nb), dim3(256), 0, c->stream,
                     (const tm_c128*)c->tden.p, mb, g.L, total, (int*)c->tmflag.p);
  TM_HIP(c, hipGetLastError());
  int flag = 1;
  TM_HIP(c, hipMemcpyAsync(&flag, c->tmflag.p, sizeof(int), hipMemcpyDeviceToHost, c->stream));
  TM_HIP(c, hipStreamSynchronize(c->stream));
  if (flag) return TM_OK;  // couples different m: the general apply
  const long long packed = (long long)g.n * mb.per_site;
  if ((rc = ensure(c, c->tmb, (size_t)packed * sizeof(c128))) != TM_OK) return rc;
  hipLaunchKernelGGL(tdense_mpack_kernel, dim3(nblk(packed)), dim3(256), 0, c->stream,
                     (const tm_c128*)c->tden.p, mb, g.L, (long long)g.n, (c128*)c->tmb.p);
  TM_HIP(c, hipGetLastError());
  c->t_mblock = true;
  return TM_OK;
}

int launch_mie_one(hipStream_t st, double radius, double k, double nre, double nim, int lmax,
                   tm_c128* out) {
  hipLaunchKernelGGL(mie_one_kernel, dim3(1), dim3(64), 0, st, radius, k, nre, nim, lmax, out);
  return hipGetLastError() == hipSuccess ? TM_OK : TM_ERR_HIP;
}

int launch_set_tdiag(tm_ctx* c, const tm_c128* t) {
  const Geometry& g = c->g;
  hipLaunchKernelGGL(set_t_kernel, dim3(nblk((long long)g.n * g.L)), dim3(256), 0, c->stream, t,
                     g.n, c->maps, (c128*)c->t64.p, (c64*)c->t32.p);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_get_tdiag(tm_ctx* c, tm_c128* t, tm_c128* dt) {
  unpack_slots(c->stream, c->g, c->maps, 1, (const c128*)c->t64.p, t);
  if (dt) unpack_slots(c->stream, c->g, c->maps, 1, (const c128*)c->dt64.p, dt);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_plane_wave(tm_ctx* c, int R, const double* khat, const tm_c128* pol, tm_c128* a0) {
  const Geometry& g = c->g;
  for (int r0 = 0; r0 < R; r0 += 8) {
    const int nr = std::min(8, R - r0);
    PwArgs pw{};
    for (int r = 0; r < nr; ++r) {
      for (int q = 0; q < 3; ++q) {
        pw.khat[3 * r + q] = khat[3 * (r0 + r) + q];
        pw.pol[6 * r + 2 * q] = pol[3 * (r0 + r) + q].re;
        pw.pol[6 * r + 2 * q + 1] = pol[3 * (r0 + r) + q].im;
      }
    }
    const long long total = (long long)nr * g.n * g.L;
    hipLaunchKernelGGL(plane_wave_kernel, dim3(nblk(total)), dim3(256), 0, c->stream, pw, nr, g.n,
                       g.L, g.lmax, site_pos(c), g.k,
                       a0 + (size_t)r0 * g.n * g.L);
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_near_field(tm_ctx* c, int R, const tm_c128* s, int P, const double* pts, tm_c128* E,
                      int precision) {
  const Geometry& g = c->g;
  for (int r0 = 0; r0 < R; r0 += NF_MAXR) {
    const int nr = std::min(NF_MAXR, R - r0);
    const tm_c128* sr = s + (size_t)r0 * g.n * g.L;
    tm_c128* Er = E + (size_t)r0 * P * 3;
    if (precision == TM_PREC_MIXED)
      nf_dispatch<float>(g.lmax, nr, dim3(nblk(P)), c->stream, sr, g.n, site_pos(c),
                         g.k, pts, P, Er);
    else
      nf_dispatch<double>(g.lmax, nr, dim3(nblk(P)), c->stream, sr, g.n, site_pos(c), g.k, pts,
                          P, Er);
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_far_field(tm_ctx* c, int R, const tm_c128* s, int D, const double* dirs, tm_c128* F) {
  const Geometry& g = c->g;
#define FF_LAUNCH(LM)                                                                              \
  hipLaunchKernelGGL(far_field_kernel<LM>, dim3((unsigned)((long long)R * D)), dim3(FF_THREADS), 0, \
                     c->stream, s, R, g.n, g.L, g.lmax, site_pos(c), g.k, dirs, D, F)
  // per-thread coefficient sums sized for the geometry's lmax
  switch (g.lmax) {
    case 1: FF_LAUNCH(1); break;
    case 2: FF_LAUNCH(2); break;
    case 3: FF_LAUNCH(3); break;
    case 4: FF_LAUNCH(4); break;
    case 5: FF_LAUNCH(5); break;
    default: FF_LAUNCH(6); break;
  }
#undef FF_LAUNCH
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_detector(tm_ctx* c, const double* xd, const tm_c128* w, tm_c128* v) {
  const Geometry& g = c->g;
  hipLaunchKernelGGL(detector_kernel, dim3(nblk((long long)g.n * g.L)), dim3(256), 0, c->stream,
                     xd[0], xd[1], xd[2], w[0].re, w[0].im, w[1].re, w[1].im, w[2].re, w[2].im,
                     g.n, g.L, g.lmax, site_pos(c), g.k, v);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_near_field_t(tm_ctx* c, int R, int P, const double* pts, const tm_c128* w, tm_c128* v) {
  const Geometry& g = c->g;
  hipLaunchKernelGGL(near_field_t_kernel, dim3(nblk((long long)g.n * g.L), R), dim3(256), 0,
                     c->stream, pts, w, P, g.n, g.L, g.lmax, site_pos(c), g.k, v);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int launch_grad(tm_ctx* c, int R, const c128* mu_slot, const c128* aexc_slot, double* grad) {
  const Geometry& g = c->g;
  hipLaunchKernelGGL(grad_kernel, dim3(nblk((long long)R * g.n)), dim3(256), 0, c->stream, mu_slot,
                     (const c128*)c->dt64.p, aexc_slot, R, g.n, g.S, grad);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

}  // namespace tmh
