// Translation-table build: one block of translation coefficients per lattice
// displacement (App. I.C, addition theorem and eq. "tran_coeff").
//
// For a source scatterer at x_s and a target at x_t = x_s + pitch*(dx, dy, 0),
// the field the source radiates, sum_u s_u Phi_u(k(x - x_s)), re-expands about
// x_t as sum_v a_v R Phi_v(k(x - x_t)) with a_v = sum_u xi_uv(k(x_t - x_s)) s_u,
// i.e. the matvec block is M(dx,dy) = xi^T.  With u = (l, m, p), v = (l', m', p'):
//   xi_uv(d) = e^{i(m-m') phi_d} sum_q C_uvq h_q(k|d|),
//   C_uvq = (p == p' ? a5 : b5)(l, m | l', m' | q) * Pbar_q^{|m-m'|}(cos theta_d = 0),
// where a5/b5 are the Wigner-3j expressions of eq. "tran_coeff" read as:
// (l, m) the source indices, q the Legendre/Hankel order (printed as p),
// second 3j of b5 with lower row (l l' q-1), normalisation root
// sqrt((2l+1)(2l'+1)/(2 l(l+1) l'(l'+1))).  The constants C are computed on
// the host once per geometry (exact factorials); the per-displacement work --
// Hankel functions, phases, sums, rounding to complex64 -- runs on the GPU.
//
// Table layout: [disp][class][S target slots][S source slots], with
// disp = (dy + tny - 1) * (2 tnx - 1) + (dx + tnx - 1); the dx = dy = 0 block
// is zero so the matvec needs no special case for the excluded self term.
// The transposed table holds the blocks of A^T: (A^T)_ts = xi(x_s - x_t) =
// S xi(x_t - x_s) S with S = diag((-1)^(l+p)), so MT(dx,dy)[i][j] =
// sigma_i sigma_j M(dx,dy)[j][i].
#include <cmath>

#include <algorithm>

#include "tm_internal.h"

namespace tmh {

// i^e as (re, im)
static void ipow(int e, double& re, double& im) {
  switch (((e % 4) + 4) % 4) {
    case 0: re = 1; im = 0; break;
    case 1: re = 0; im = 1; break;
    case 2: re = -1; im = 0; break;
    default: re = 0; im = -1; break;
  }
}

static long double dfact(int n) {  // double factorial, (-1)!! = 0!! = 1
  long double r = 1.0L;
  for (int i = n; i > 1; i -= 2) r *= (long double)i;
  return r;
}

// Normalised associated Legendre function at x = 0, no Condon-Shortley phase:
// P_q^mu(0) = (-1)^((q-mu)/2) (q+mu-1)!!/(q-mu)!! for q+mu even, else 0.
static double pbar_at_zero(int q, int mu) {
  if (mu > q || ((q + mu) & 1)) return 0.0;
  long double p = dfact(q + mu - 1) / dfact(q - mu);
  if (((q - mu) / 2) & 1) p = -p;
  long double nrm = std::sqrt((2.0L * q + 1.0L) / 2.0L * lfact(q - mu) / lfact(q + mu));
  return (double)(nrm * p);
}

static void plm_of(int n, int lmax, int& p, int& l, int& m) {
  int half = lmax * (lmax + 2);
  p = n / half;
  int r = n % half;  // = l(l+1) - 1 + m
  l = 1;
  while ((l + 1) * (l + 2) - 1 - (l + 1) <= r) ++l;  // first index of l+1 is (l+1)^2-1
  m = r - (l * (l + 1) - 1);
}

void host_slot_maps(int lmax, Geometry& g, SlotMaps& mp) {
  g.L = 2 * lmax * (lmax + 2);
  g.S = slots_for_lmax(lmax);
  g.NG = g.S / SLOTS;
  g.cls_of.assign(g.L, 0);
  g.slot_of.assign(g.L, 0);
  for (int c = 0; c < NCLASS; ++c) g.n_of[c].assign(g.S, -1);
  int cnt[NCLASS] = {0, 0};
  for (int n = 0; n < g.L; ++n) {
    int p, l, m;
    plm_of(n, lmax, p, l, m);
    int c = (((l + m + p) % 2) + 2) % 2;
    g.cls_of[n] = c;
    g.slot_of[n] = cnt[c];
    g.n_of[c][cnt[c]] = n;
    cnt[c]++;
  }
  mp = SlotMaps{};
  mp.L = g.L;
  mp.lmax = lmax;
  mp.S = g.S;
  for (int n = 0; n < g.L; ++n) {
    mp.cls_of[n] = g.cls_of[n];
    mp.slot_of[n] = g.slot_of[n];
  }
  for (int c = 0; c < NCLASS; ++c)
    for (int s = 0; s < SMAX; ++s) mp.n_of[c][s] = s < g.S ? g.n_of[c][s] : -1;
}

// Host constants: coef[c][i][j][q] (i target slot, j source slot) and
// dm[c][i][j] = m_src - m_tgt, sig[c][i] = (-1)^(l+p).
static void host_table_constants(const Geometry& g, int Q, std::vector<double>& coef,
                                 std::vector<int>& dm, std::vector<int>& sig) {
  const int S = g.S;
  coef.assign((size_t)NCLASS * S * S * Q * 2, 0.0);
  dm.assign((size_t)NCLASS * S * S, 0);
  sig.assign((size_t)NCLASS * S, 0);
  for (int c = 0; c < NCLASS; ++c) {
    for (int i = 0; i < S; ++i) {
      int nv = g.n_of[c][i];
      if (nv >= 0) {
        int pp, lp, mp;
        plm_of(nv, g.lmax, pp, lp, mp);
        sig[c * S + i] = ((lp + pp) & 1) ? -1 : 1;
      }
      for (int j = 0; j < S; ++j) {
        int nu = g.n_of[c][j];
        if (nu < 0 || nv < 0) continue;
        int p, l, m, pp, lp, mp;
        plm_of(nu, g.lmax, p, l, m);
        plm_of(nv, g.lmax, pp, lp, mp);
        dm[(c * S + i) * S + j] = m - mp;
        double root = std::sqrt((2.0 * l + 1) * (2.0 * lp + 1) /
                                (2.0 * l * (l + 1) * lp * (lp + 1)));
        double sgn = ((std::abs(m - mp)) & 1) ? -1.0 : 1.0;  // (-1)^(m-m')
        for (int q = std::abs(l - lp); q <= l + lp; ++q) {
          double w1 = wigner3j(l, lp, q, m, -mp, mp - m);
          double val;
          if (p == pp) {
            double wa = wigner3j(l, lp, q, 0, 0, 0);
            val = (l * (l + 1) + lp * (lp + 1) - q * (q + 1)) * std::sqrt(2.0 * q + 1) * w1 * wa;
          } else {
            if (q < 1) continue;
            double wb = wigner3j(l, lp, q - 1, 0, 0, 0);
            double arg = (double)(l + lp + 1 + q) * (l + lp + 1 - q) * (q + l - lp) * (q - l + lp) *
                         (2 * q + 1);
            if (arg <= 0) continue;
            val = std::sqrt(arg) * w1 * wb;
          }
          val *= root * sgn * pbar_at_zero(q, std::abs(m - mp));
          double re, im;
          ipow(std::abs(m - mp) - std::abs(m) - std::abs(mp) + lp - l + q, re, im);
          size_t o = ((((size_t)c * S + i) * S + j) * Q + q) * 2;
          coef[o] = re * val;
          coef[o + 1] = im * val;
        }
      }
    }
  }
}

// Coefficients of xi_uv for source truncation lmax and the three N-type l' = 1
// targets v = (p' = 1, l' = 1, m' = -1, 0, 1) at a general displacement (no
// Legendre factor folded in): coef[(u * 3 + v) * (lmax + 2) + q] for
// q = 0..lmax+1, dm[u * 3 + v] = m_u - m'.  Used by the detector term of the
// position gradient, whose displacement x_d - x_i leaves the lattice plane.
void detector_grad_constants(int lmax, std::vector<c128>& coef, std::vector<int>& dm) {
  const int L = 2 * lmax * (lmax + 2), Q = lmax + 2;
  coef.assign((size_t)L * 3 * Q, c128{0.0, 0.0});
  dm.assign((size_t)L * 3, 0);
  for (int u = 0; u < L; ++u) {
    int p, l, m;
    plm_of(u, lmax, p, l, m);
    for (int v = 0; v < 3; ++v) {
      const int pp = 1, lp = 1, mp = v - 1;
      dm[u * 3 + v] = m - mp;
      const double root = std::sqrt((2.0 * l + 1) * (2.0 * lp + 1) / (2.0 * l * (l + 1) * lp * (lp + 1)));
      const double sgn = ((std::abs(m - mp)) & 1) ? -1.0 : 1.0;
      for (int q = std::abs(l - lp); q <= l + lp; ++q) {
        const double w1 = wigner3j(l, lp, q, m, -mp, mp - m);
        double val;
        if (p == pp) {
          const double wa = wigner3j(l, lp, q, 0, 0, 0);
          val = (l * (l + 1) + lp * (lp + 1) - q * (q + 1)) * std::sqrt(2.0 * q + 1) * w1 * wa;
        } else {
          if (q < 1) continue;
          const double wb = wigner3j(l, lp, q - 1, 0, 0, 0);
          const double arg =
              (double)(l + lp + 1 + q) * (l + lp + 1 - q) * (q + l - lp) * (q - l + lp) * (2 * q + 1);
          if (arg <= 0) continue;
          val = std::sqrt(arg) * w1 * wb;
        }
        val *= root * sgn;
        double re, im;
        ipow(std::abs(m - mp) - std::abs(m) - std::abs(mp) + lp - l + q, re, im);
        coef[((size_t)u * 3 + v) * Q + q] = c128{re * val, im * val};
      }
    }
  }
}

// Spherical Hankel functions h_0..h_qmax of the first kind by upward
// recurrence h_{q+1} = (2q+1)/x h_q - h_{q-1} from h_0 = -i e^{ix}/x,
// h_1 = -e^{ix}(x + i)/x^2 (stable for h: the growing y_q dominates).
__device__ inline void hankel_up(double x, int qmax, double* hr, double* hi) {
  double s, c;
  sincos(x, &s, &c);
  double ix = 1.0 / x;
  hr[0] = s * ix;   // -i (c + i s)/x = (s - i c)/x
  hi[0] = -c * ix;
  // -(c + i s)(x + i)/x^2 = -(c x - s + i(s x + c))/x^2
  hr[1] = -(c * x - s) * ix * ix;
  hi[1] = -(s * x + c) * ix * ix;
  for (int q = 1; q < qmax; ++q) {
    double f = (2 * q + 1) * ix;
    hr[q + 1] = f * hr[q] - hr[q - 1];
    hi[q + 1] = f * hi[q] - hi[q - 1];
  }
}

// Per displacement d: h_q(k|d|) for q <= qmax (rad[d][q]) and e^{i mu phi}
// for |mu| <= qmax (ang[d][mu + qmax]), the transcendental part of every
// entry of the block, computed once per displacement.
__global__ void table_radial_kernel(int tnx, int tny, double pitch, double k, int qmax,
                                    long long D, c128* __restrict__ rad, c128* __restrict__ ang) {
  const long long d = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (d >= D) return;
  const int wx = 2 * tnx - 1;
  const int dx = (int)(d % wx) - (tnx - 1);
  const int dy = (int)(d / wx) - (tny - 1);
  c128* rd = rad + d * (qmax + 1);
  c128* ad = ang + d * (2 * qmax + 1);
  double hr[QMAX + 1] = {0}, hi[QMAX + 1] = {0};
  double phi = 0.0;
  if (dx != 0 || dy != 0) {
    const double X = pitch * dx, Y = pitch * dy;
    phi = atan2(Y, X);
    hankel_up(k * sqrt(X * X + Y * Y), qmax, hr, hi);
  }
  for (int q = 0; q <= qmax; ++q) rd[q] = c128{hr[q], hi[q]};
  for (int mu = -qmax; mu <= qmax; ++mu) {
    double s, c;
    sincos((double)mu * phi, &s, &c);
    ad[mu + qmax] = c128{c, s};
  }
}

// Thread = one (class, target slot, source slot) entry of every block
// (blockIdx.y picks a range of 512 entries); the workgroups stride over the
// displacements and the entry's coefficients stay in registers:
// entry(d) = e^{i dm phi(d)} sum_q coef_q h_q(k|d|), q <= QM = 2 lmax.
constexpr int TB_UNROLL = 4;
template <int QM>
__global__ __launch_bounds__(512) void build_table_kernel(
    const double* __restrict__ coef, const int* __restrict__ dm, const int* __restrict__ sig,
    const c128* __restrict__ rad, const c128* __restrict__ ang, c128* __restrict__ tab64,
    c64* __restrict__ tab32, int tnx, int tny, long long D, int S, int transpose) {
  const int ent = blockIdx.y * 512 + threadIdx.x;
  if (ent >= NCLASS * S * S) return;
  const int c = ent / (S * S);
  const int i = (ent / S) % S;
  const int j = ent % S;
  // transposed table: MT[i][j] = sig_i sig_j M[j][i]
  const int ii = transpose ? j : i, jj = transpose ? i : j;
  constexpr int Q = QM + 1;
  const double* cf = coef + ((((size_t)c * S + ii) * S + jj) * Q) * 2;
  double ar[Q], ai[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    ar[q] = cf[2 * q];
    ai[q] = cf[2 * q + 1];
  }
  const int mu = dm[(c * S + ii) * S + jj] + QM;
  const double sg = transpose ? (double)(sig[c * S + i] * sig[c * S + j]) : 1.0;
  const int wx = 2 * tnx - 1;
  const long long center = (long long)(tny - 1) * wx + (tnx - 1);  // d of (0, 0)
  const size_t blk = (size_t)NCLASS * S * S;
  for (long long d0 = blockIdx.x; d0 < D; d0 += (long long)gridDim.x * TB_UNROLL) {
#pragma unroll
    for (int u = 0; u < TB_UNROLL; ++u) {
      const long long d = d0 + (long long)u * gridDim.x;
      if (d >= D) break;
      const c128* rd = rad + d * Q;
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        const c128 h = rd[q];
        sr += ar[q] * h.re - ai[q] * h.im;
        si += ar[q] * h.im + ai[q] * h.re;
      }
      const c128 e = ang[d * (2 * QM + 1) + mu];
      double re = sg * (sr * e.re - si * e.im), im = sg * (sr * e.im + si * e.re);
      if (d == center) re = im = 0.0;
      const size_t out = (size_t)d * blk + (size_t)ent;
      tab64[out] = c128{re, im};
      tab32[out] = c64{(float)re, (float)im};
    }
  }
}

// Derivative blocks for the position gradient: D_a(d) = d xi(k d)^T / d d_a
// for the in-plane directions a = x, y (physical units, 1/length).  In the
// plane theta = pi/2, so the theta_hat term of the gradient has no x, y
// component and the z-mirror class structure of the blocks is kept:
//   D_a[i][j](d) = k e^{i dm phi} sum_q coef_q [ h_q'(kd) rhat_a + i dm h_q(kd)/(kd) phihat_a ],
// rhat = (cos phi, sin phi), phihat = (-sin phi, cos phi), h_q' = h_{q-1} - (q+1)/x h_q.
// The transposed variant holds the blocks of the transposed operator:
// xi(-d) = S xi(d) S gives d xi(-d)/dd = -S (d xi(d)/dd) S, so
// DT_a[i][j] = -sig_i sig_j D_a[j][i].
template <int QM>
__global__ __launch_bounds__(512) void build_dtable_kernel(
    const double* __restrict__ coef, const int* __restrict__ dm, const int* __restrict__ sig,
    c128* __restrict__ tab, int tnx, int tny, long long D, int S, double pitch, double k, int axis,
    int transpose) {
  const int ent = blockIdx.y * 512 + threadIdx.x;
  if (ent >= NCLASS * S * S) return;
  const int c = ent / (S * S);
  const int i = (ent / S) % S;
  const int j = ent % S;
  const int ii = transpose ? j : i, jj = transpose ? i : j;
  constexpr int Q = QM + 1;
  const double* cf = coef + ((((size_t)c * S + ii) * S + jj) * Q) * 2;
  double ar[Q], ai[Q];
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    ar[q] = cf[2 * q];
    ai[q] = cf[2 * q + 1];
  }
  const int mu = dm[(c * S + ii) * S + jj];
  const double sg = transpose ? -(double)(sig[c * S + i] * sig[c * S + j]) : 1.0;
  const int wx = 2 * tnx - 1;
  const size_t blk = (size_t)NCLASS * S * S;
  for (long long d = blockIdx.x; d < D; d += gridDim.x) {
    const int dx = (int)(d % wx) - (tnx - 1);
    const int dy = (int)(d / wx) - (tny - 1);
    double re = 0.0, im = 0.0;
    if (dx != 0 || dy != 0) {
      const double X = pitch * dx, Y = pitch * dy;
      const double rr = sqrt(X * X + Y * Y);
      const double cph = X / rr, sph = Y / rr;
      const double x = k * rr;
      double hr[Q + 1], hi[Q + 1];
      hankel_up(x, QM + 1, hr, hi);
      const double ra = axis == 0 ? cph : sph;    // rhat_a
      const double pa = axis == 0 ? -sph : cph;   // phihat_a
      double sr = 0.0, si = 0.0;
#pragma unroll
      for (int q = 0; q < Q; ++q) {
        // h_q' (x)
        double dr, di;
        if (q == 0) {
          dr = -hr[1];
          di = -hi[1];
        } else {
          dr = hr[q - 1] - (q + 1) / x * hr[q];
          di = hi[q - 1] - (q + 1) / x * hi[q];
        }
        // f_q = h_q' ra + i mu h_q / x pa
        const double fr = dr * ra - mu * hi[q] / x * pa;
        const double fi = di * ra + mu * hr[q] / x * pa;
        sr += ar[q] * fr - ai[q] * fi;
        si += ar[q] * fi + ai[q] * fr;
      }
      double s_, c_;
      sincos((double)mu * atan2(Y, X), &s_, &c_);
      re = sg * k * (sr * c_ - si * s_);
      im = sg * k * (sr * s_ + si * c_);
    }
    tab[(size_t)d * blk + (size_t)ent] = c128{re, im};
  }
}

// The four FP64 derivative tables (x, y; forward and transposed).
int build_derivative_tables(tm_ctx* c) {
  const Geometry& g = c->g;
  std::vector<double> coef;
  std::vector<int> dm, sig;
  const int qmax = 2 * g.lmax;
  host_table_constants(g, qmax + 1, coef, dm, sig);
  const long long D = g.n_disp();
  const size_t blk = (size_t)NCLASS * g.S * g.S;
  int rc;
  for (int t = 0; t < 4; ++t)
    if ((rc = ensure(c, c->dtab[t], (size_t)D * blk * sizeof(c128))) != TM_OK) return rc;
  double* dcoef = nullptr;
  int *ddm = nullptr, *dsig = nullptr;
  TM_HIP(c, hipMalloc((void**)&dcoef, coef.size() * sizeof(double)));
  TM_HIP(c, hipMalloc((void**)&ddm, dm.size() * sizeof(int)));
  TM_HIP(c, hipMalloc((void**)&dsig, sig.size() * sizeof(int)));
  TM_HIP(c, hipMemcpyAsync(dcoef, coef.data(), coef.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  TM_HIP(c, hipMemcpyAsync(ddm, dm.data(), dm.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  TM_HIP(c, hipMemcpyAsync(dsig, sig.data(), sig.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  const unsigned nchunk = (unsigned)((blk + 511) / 512);
  const unsigned nwg = (unsigned)std::min<long long>(D, std::max(1u, 4096u / nchunk));
  const dim3 grid(nwg, nchunk);
  for (int t = 0; t < 4; ++t) {
    const int axis = t & 1, transpose = t >> 1;
#define DT_LAUNCH(QM)                                                                        \
  hipLaunchKernelGGL(build_dtable_kernel<QM>, grid, dim3(512), 0, c->stream, dcoef, ddm, dsig, \
                     (c128*)c->dtab[t].p, g.tnx, g.tny, D, g.S, g.pitch, g.k, axis, transpose)
    switch (qmax) {
      case 2: DT_LAUNCH(2); break;
      case 4: DT_LAUNCH(4); break;
      case 6: DT_LAUNCH(6); break;
      case 8: DT_LAUNCH(8); break;
      case 10: DT_LAUNCH(10); break;
      default: DT_LAUNCH(12); break;
    }
#undef DT_LAUNCH
  }
  TM_HIP(c, hipGetLastError());
  TM_HIP(c, hipStreamSynchronize(c->stream));
  TM_HIP(c, hipFree(dcoef));
  TM_HIP(c, hipFree(ddm));
  TM_HIP(c, hipFree(dsig));
  c->have_dtab = true;
  return TM_OK;
}

static int build_impl(tm_ctx* c, DevBuf& t64, DevBuf& t32, int transpose) {
  const Geometry& g = c->g;
  std::vector<double> coef;
  std::vector<int> dm, sig;
  const int qmax = 2 * g.lmax;
  host_table_constants(g, qmax + 1, coef, dm, sig);
  const long long D = g.n_disp();
  const size_t blk = (size_t)NCLASS * g.S * g.S;
  int rc;
  if ((rc = ensure(c, t64, (size_t)D * blk * sizeof(c128))) != TM_OK) return rc;
  if ((rc = ensure(c, t32, (size_t)D * blk * sizeof(c64))) != TM_OK) return rc;
  double* dcoef = nullptr;
  int *ddm = nullptr, *dsig = nullptr;
  c128 *rad = nullptr, *ang = nullptr;
  TM_HIP(c, hipMalloc((void**)&dcoef, coef.size() * sizeof(double)));
  TM_HIP(c, hipMalloc((void**)&ddm, dm.size() * sizeof(int)));
  TM_HIP(c, hipMalloc((void**)&dsig, sig.size() * sizeof(int)));
  TM_HIP(c, hipMalloc((void**)&rad, (size_t)D * (qmax + 1) * sizeof(c128)));
  TM_HIP(c, hipMalloc((void**)&ang, (size_t)D * (2 * qmax + 1) * sizeof(c128)));
  TM_HIP(c, hipMemcpyAsync(dcoef, coef.data(), coef.size() * sizeof(double),
                           hipMemcpyHostToDevice, c->stream));
  TM_HIP(c, hipMemcpyAsync(ddm, dm.data(), dm.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  TM_HIP(c, hipMemcpyAsync(dsig, sig.data(), sig.size() * sizeof(int), hipMemcpyHostToDevice,
                           c->stream));
  hipLaunchKernelGGL(table_radial_kernel, dim3((unsigned)((D + 255) / 256)), dim3(256), 0, c->stream,
                     g.tnx, g.tny, g.pitch, g.k, qmax, D, rad, ang);
  const unsigned nchunk = (unsigned)((blk + 511) / 512);
  const unsigned nwg = (unsigned)std::min<long long>(D, std::max(1u, 4096u / nchunk));
  const dim3 grid(nwg, nchunk);
  // the kernel's coefficient registers are sized by the Legendre/Hankel order
#define TB_LAUNCH(QM)                                                                           \
  hipLaunchKernelGGL(build_table_kernel<QM>, grid, dim3(512), 0, c->stream, dcoef, ddm, dsig,   \
                     (const c128*)rad, (const c128*)ang, (c128*)t64.p, (c64*)t32.p, g.tnx, g.tny, \
                     D, g.S, transpose)
  switch (qmax) {
    case 2: TB_LAUNCH(2); break;
    case 4: TB_LAUNCH(4); break;
    case 6: TB_LAUNCH(6); break;
    case 8: TB_LAUNCH(8); break;
    case 10: TB_LAUNCH(10); break;
    default: TB_LAUNCH(12); break;
  }
#undef TB_LAUNCH
  TM_HIP(c, hipGetLastError());
  // the host vectors above are read by the async copies; wait before they go
  TM_HIP(c, hipStreamSynchronize(c->stream));
  TM_HIP(c, hipFree(dcoef));
  TM_HIP(c, hipFree(ddm));
  TM_HIP(c, hipFree(dsig));
  TM_HIP(c, hipFree(rad));
  TM_HIP(c, hipFree(ang));
  return TM_OK;
}

int build_tables(tm_ctx* c) { return build_impl(c, c->tab64, c->tab32, 0); }

// Off-lattice geometries: no displacement tables; the on-the-fly matvec reads
// the per-entry constants coef [2][S][S][Q] (complex, Pbar_q(0) folded in: every
// scatterer lies in z = 0), dm [2][S][S] and coef again in FP32 from one
// device buffer.
int build_offlattice_constants(tm_ctx* c) {
  const Geometry& g = c->g;
  std::vector<double> coef;
  std::vector<int> dm, sig;
  const int Q = 2 * g.lmax + 1;
  host_table_constants(g, Q, coef, dm, sig);
  // followed by an FP32 copy of coef for the complex64 kernel (no conversion per use)
  std::vector<float> coef32(coef.begin(), coef.end());
  const size_t cb = coef.size() * sizeof(double), db = dm.size() * sizeof(int);
  const size_t fb = coef32.size() * sizeof(float);
  int rc;
  if ((rc = ensure(c, c->olc, cb + db + fb)) != TM_OK) return rc;
  TM_HIP(c, hipMemcpy(c->olc.p, coef.data(), cb, hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy((char*)c->olc.p + cb, dm.data(), db, hipMemcpyHostToDevice));
  TM_HIP(c, hipMemcpy((char*)c->olc.p + cb + db, coef32.data(), fb, hipMemcpyHostToDevice));
  return TM_OK;
}

int build_transposed_tables(tm_ctx* c) {
  int rc = build_impl(c, c->tabT64, c->tabT32, 1);
  if (rc == TM_OK) c->have_tabT = true;
  return rc;
}

}  // namespace tmh
