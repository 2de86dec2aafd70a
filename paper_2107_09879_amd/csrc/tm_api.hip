// C ABI of libtmhip: context, set-up, restarted GMRES drivers, readout and
// sensitivities.  The host enqueues whole GMRES cycles; every vector
// operation, reduction, matvec, Givens rotation and the least-squares solve
// is a HIP kernel on the context stream.  Per cycle the host reads back one
// record (the true residual norm, the number of Arnoldi steps taken, a
// non-finite flag): the steps of a cycle after its convergence test fired
// on the device return at once.
//
// Solver (App. I.D: matrix-free matvecs inside GMRES; the preconditioned
// system of App. I.C):
//   restarted GMRES(m), x0 = 0 unless given, classical Gram-Schmidt with one
//   re-orthogonalisation pass (CGS2) in FP64, complex Givens rotations, stop
//   when the FP64 true residual ||b - B s||/||b|| <= tol.
// Mixed precision (iterative refinement): each cycle starts from the FP64
// true residual r = b - B s, runs Arnoldi with the complex64/FP32-accumulate
// operator (basis, Hessenberg and rotations in FP64) until the estimated
// residual falls by inner_tol or the cycle ends, then updates s in FP64.
#include <algorithm>
#include <cmath>
#include <complex>
#include <cstring>

#include "tm_internal.h"

using tmh::c128;
using tmh::Op;

namespace tmh {

int set_err(tm_ctx* c, int code, const std::string& msg) {
  if (c) c->err = msg;
  return code;
}

int ensure(tm_ctx* c, DevBuf& b, size_t bytes) {
  if (b.bytes >= bytes && b.p) return TM_OK;
  if (b.p) {
    hipStreamSynchronize(c->stream);
    hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
  }
  if (bytes == 0) return TM_OK;
  hipError_t e = hipMalloc(&b.p, bytes);
  if (e != hipSuccess) {
    b.p = nullptr;
    (void)hipGetLastError();
    return set_err(c, TM_ERR_OOM, "device allocation of " + std::to_string(bytes) + " bytes failed");
  }
  b.bytes = bytes;
  return TM_OK;
}

void release(DevBuf& b) {
  if (b.p) hipFree(b.p);
  b.p = nullptr;
  b.bytes = 0;
}

int ensure_pinned(tm_ctx* c, size_t bytes) {
  if (c->host_pinned_bytes >= bytes) return TM_OK;
  if (c->host_pinned) hipHostFree(c->host_pinned);
  c->host_pinned = nullptr;
  c->host_pinned_bytes = 0;
  if (hipHostMalloc(&c->host_pinned, bytes, hipHostMallocDefault) != hipSuccess) {
    (void)hipGetLastError();
    return set_err(c, TM_ERR_OOM, "pinned host allocation failed");
  }
  c->host_pinned_bytes = bytes;
  return TM_OK;
}

// Plane-wave incidences: khat unit vectors, pol finite and transverse.
int validate_incidence(tm_ctx* c, int R, const double* khat, const tm_c128* pol) {
  for (int r = 0; r < R; ++r) {
    const double* kh = khat + 3 * r;
    const double nk = std::sqrt(kh[0] * kh[0] + kh[1] * kh[1] + kh[2] * kh[2]);
    if (!std::isfinite(nk) || std::fabs(nk - 1.0) > 1e-9)
      return set_err(c, TM_ERR_INVALID_ARG, "khat must be a unit vector");
    double dr = 0, di = 0;
    for (int q = 0; q < 3; ++q) {
      if (!std::isfinite(pol[3 * r + q].re) || !std::isfinite(pol[3 * r + q].im))
        return set_err(c, TM_ERR_NAN, "non-finite polarisation");
      dr += kh[q] * pol[3 * r + q].re;
      di += kh[q] * pol[3 * r + q].im;
    }
    if (std::hypot(dr, di) > 1e-9)
      return set_err(c, TM_ERR_INVALID_ARG, "polarisation must be transverse to khat");
  }
  return TM_OK;
}

// ---------------------------------------------------------------- GMRES
struct Gm {
  tm_ctx* c;
  Op op;
  long long len;
  int nblk;
  c128 *V, *w, *r, *dots, *dots2, *dp;
  double *np, *nout;
};

static double dev_norm(Gm& G, const c128* v) {
  k_norm2_partial(G.c->stream, v, G.len, G.np, G.nblk);
  k_reduce_norm(G.c->stream, G.np, G.nblk, G.nout);
  double h = 0.0;
  hipMemcpyAsync(G.c->host_pinned, G.nout, sizeof(double), hipMemcpyDeviceToHost, G.c->stream);
  hipStreamSynchronize(G.c->stream);
  std::memcpy(&h, G.c->host_pinned, sizeof(double));
  return h;
}

// x (slot, one RHS) solves B x = b with B the operator `op`.
static int gmres(tm_ctx* c, Op op, const c128* b, c128* x, const tm_solve_opts& o, bool use_x0,
                 tm_solve_info& info) {
  const Geometry& g = c->g;
  const long long len = g.vec_len();
  const int m = o.restart;
  int rc;
  // workspace: basis (m+1) vectors, w, r
  if ((rc = ensure(c, c->basis, (size_t)(m + 1) * len * sizeof(c128))) != TM_OK) return rc;
  if ((rc = ensure(c, c->work_c, (size_t)2 * len * sizeof(c128))) != TM_OK) return rc;
  const int nblk = krylov_blocks(len);
  if ((rc = ensure(c, c->dotpart, (size_t)nblk * (m + 2) * sizeof(c128))) != TM_OK) return rc;
  if ((rc = ensure(c, c->dots, (size_t)(2 * (m + 2) + 4) * sizeof(c128))) != TM_OK) return rc;
  if ((rc = ensure(c, c->scal, (size_t)(nblk + 8) * sizeof(double))) != TM_OK) return rc;
  if ((rc = ensure_pinned(c, (size_t)(2 * m + 6) * sizeof(c128))) != TM_OK) return rc;
  Gm G;
  G.c = c;
  G.op = op;
  G.len = len;
  G.nblk = nblk;
  G.V = (c128*)c->basis.p;
  G.w = (c128*)c->work_c.p;
  G.r = G.w + len;
  G.dp = (c128*)c->dotpart.p;
  G.dots = (c128*)c->dots.p;
  G.dots2 = G.dots + (m + 2);
  G.np = (double*)c->scal.p;
  G.nout = G.np + nblk;
  hipStream_t st = c->stream;

  info = tm_solve_info{};
  const double bnorm = dev_norm(G, b);
  if (!std::isfinite(bnorm)) return set_err(c, TM_ERR_NAN, "right-hand side is not finite");
  if (bnorm == 0.0) {
    TM_HIP(c, hipMemsetAsync(x, 0, len * sizeof(c128), st));
    info.status = TM_OK;
    return TM_OK;
  }
  if (use_x0) {
    if ((rc = apply_op(c, op, TM_PREC_FP64, 1, x, G.r)) != TM_OK) return rc;
    info.matvecs_fp64++;
    k_sub(st, G.r, b, G.r, len);
  } else {
    TM_HIP(c, hipMemsetAsync(x, 0, len * sizeof(c128), st));
    k_copy(st, G.r, b, len);
  }
  if ((rc = ensure(c, c->gm_dev, gm_state_bytes(m))) != TM_OK) return rc;
  void* gs = c->gm_dev.p;
  const int* stop = &static_cast<const GmFlags*>(gs)->stop;
  // the matvecs of apply_op skip their work once the cycle has stopped;
  // cleared on every way out of this function
  struct StopGuard {
    tm_ctx* c;
    ~StopGuard() { c->mv_stop = nullptr; }
  } guard{c};
  const int which_prof = (o.precision == TM_PREC_MIXED) ? 1 : 0;
  int it = 0;
  double relres = 0.0;
  const int prec = o.precision;
  double beta = dev_norm(G, G.r);
  for (;;) {
    relres = beta / bnorm;
    if (!std::isfinite(beta)) return set_err(c, TM_ERR_NAN, "residual became non-finite");
    if (relres <= o.tol || it >= o.max_iter) break;
    if (c->progress) c->progress(c->progress_user, info.cycles, it, 1, relres);
    info.cycles++;
    k_scale(st, G.V, G.r, 1.0 / beta, len);
    k_gm_cycle_init(st, gs, m, G.nout);  // G.nout holds beta
    const double target =
        (prec == TM_PREC_MIXED) ? std::max(o.tol * bnorm, o.inner_tol * beta) : o.tol * bnorm;
    const int jmax = std::min(m, o.max_iter - it);
    c->mv_stop = stop;
    int launched = 0;
    for (int j = 0; j < jmax; ++j) {
      ++launched;
      c128* vj = G.V + (size_t)j * len;
      if ((rc = apply_op(c, op, prec, 1, vj, G.w)) != TM_OK) return rc;
      // CGS2: h1 = V^H w, w -= V h1, h2 = V^H w, w -= V h2, H(:,j) = h1 + h2
      int nseg = k_multidot(st, G.V, len, j + 1, G.w, len, G.dp, nblk, stop);
      k_reduce_dots(st, G.dp, nseg, j + 1, G.dots, nullptr, stop);
      k_update(st, G.w, G.V, len, j + 1, G.dots, len, -1.0, stop);
      nseg = k_multidot(st, G.V, len, j + 1, G.w, len, G.dp, nblk, stop);
      k_reduce_dots(st, G.dp, nseg, j + 1, G.dots2, nullptr, stop);
      k_update(st, G.w, G.V, len, j + 1, G.dots2, len, -1.0, stop);
      k_norm2_partial(st, G.w, len, G.np, nblk, stop);
      k_reduce_norm(st, G.np, nblk, G.nout, stop);
      k_gm_givens(st, gs, m, j, G.dots, G.dots2, G.nout, target);
      k_gm_scale_next(st, G.V + (size_t)(j + 1) * len, G.w, gs, len);
      // with a progress callback, a long cycle also reports every 50 steps
      // (one readback of the flags there; a cycle already stopped ends here)
      if (c->progress && (j + 1) % 50 == 0 && j + 1 < jmax) {
        TM_HIP(c, hipMemcpyAsync(c->host_pinned, gs, sizeof(GmFlags), hipMemcpyDeviceToHost, st));
        TM_HIP(c, hipStreamSynchronize(st));
        GmFlags fl;
        std::memcpy(&fl, c->host_pinned, sizeof(GmFlags));
        if (fl.stop) break;
        c->progress(c->progress_user, info.cycles - 1, it + fl.jend, 1, fl.est / bnorm);
      }
    }
    c->mv_stop = nullptr;
    const size_t prof_mark = c->prof ? c->prof_pending[which_prof].size() : 0;
    // y = H^-1 g on the device, x += V y (y is zero past the steps taken)
    k_gm_backsub(st, gs, m);
    k_gm_update_x(st, x, G.V, len, gs, m);
    // true residual in FP64
    if ((rc = apply_op(c, op, TM_PREC_FP64, 1, x, G.r)) != TM_OK) return rc;
    info.matvecs_fp64++;
    k_sub(st, G.r, b, G.r, len);
    // the cycle's one readback: residual norm and the flags
    k_norm2_partial(st, G.r, len, G.np, nblk);
    k_reduce_norm(st, G.np, nblk, G.nout);
    TM_HIP(c, hipMemcpyAsync(c->host_pinned, G.nout, sizeof(double), hipMemcpyDeviceToHost, st));
    TM_HIP(c, hipMemcpyAsync((char*)c->host_pinned + 16, gs, sizeof(GmFlags), hipMemcpyDeviceToHost, st));
    TM_HIP(c, hipStreamSynchronize(st));
    GmFlags fl;
    std::memcpy(&beta, c->host_pinned, sizeof(double));
    std::memcpy(&fl, (const char*)c->host_pinned + 16, sizeof(GmFlags));
    if (fl.nonfinite) return set_err(c, TM_ERR_NAN, "Arnoldi produced a non-finite value");
    it += fl.jend;
    if (prec == TM_PREC_MIXED) info.matvecs_lowp += fl.jend;
    else info.matvecs_fp64 += fl.jend;
    // matvecs launched after the convergence test fired did no work: their
    // profile records (the last ones of the Arnoldi loop) are dropped
    if (c->prof && fl.jend < launched) {
      auto& pend = c->prof_pending[which_prof];
      const size_t drop = (size_t)(launched - fl.jend);
      const size_t mark = prof_mark;
      if (mark >= drop && mark <= pend.size()) {
        for (size_t k = mark - drop; k < mark; ++k) {
          hipEventDestroy(pend[k].first);
          hipEventDestroy(pend[k].second);
        }
        pend.erase(pend.begin() + (mark - drop), pend.begin() + mark);
      }
    }
  }
  info.iters = it;
  info.rel_residual = relres;
  info.status = (relres <= o.tol) ? TM_OK : TM_NOT_CONVERGED;
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

}  // namespace tmh

// ============================================================== C ABI
extern "C" {

int tm_abi_version(void) { return TMHIP_ABI_VERSION; }

int tm_coeff_count(int lmax) {
  if (lmax < 1 || lmax > tmh::LMAX_SUPPORTED) return 0;
  return 2 * lmax * (lmax + 2);
}

const char* tm_status_string(int s) {
  switch (s) {
    case TM_OK: return "ok";
    case TM_NOT_CONVERGED: return "not converged";
    case TM_ERR_INVALID_ARG: return "invalid argument";
    case TM_ERR_OVERLAP: return "enclosing spheres overlap";
    case TM_ERR_NOT_LATTICE: return "positions are not a z=0 rectangular lattice";
    case TM_ERR_OOM: return "out of device memory";
    case TM_ERR_HIP: return "HIP runtime error";
    case TM_ERR_NAN: return "non-finite input";
    case TM_ERR_STATE: return "call out of order";
    default: return "unknown status";
  }
}

const char* tm_last_error(const tm_ctx* c) { return c ? c->err.c_str() : "null context"; }

void tm_default_opts(tm_solve_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->restart = 50;
  o->max_iter = 2000;
  o->precision = TM_PREC_FP64;
  o->inner_tol = 1e-4;
  o->use_x0 = 0;
}

int tm_create(tm_ctx** out, int device, void* stream) {
  if (!out) return TM_ERR_INVALID_ARG;
  *out = nullptr;
  int ndev = 0;
  if (hipGetDeviceCount(&ndev) != hipSuccess || device < 0 || device >= ndev) {
    (void)hipGetLastError();
    return TM_ERR_INVALID_ARG;
  }
  if (hipSetDevice(device) != hipSuccess) return TM_ERR_HIP;
  tm_ctx* c = new (std::nothrow) tm_ctx();
  if (!c) return TM_ERR_OOM;
  c->device = device;
  c->stream = (hipStream_t)stream;
  const int rc = tmh::noalloc_init(c);
  if (rc != TM_OK) {
    delete c;
    return rc;
  }
  *out = c;
  return TM_OK;
}

void tm_destroy(tm_ctx* c) {
  if (!c) return;
  hipSetDevice(c->device);
  hipStreamSynchronize(c->stream);
  for (tmh::DevBuf* b : {&c->dtab[0], &c->dtab[1], &c->dtab[2], &c->dtab[3], &c->gpos, &c->jinc_buf,
                        &c->gm_dev, &c->tmb, &c->tmflag})
    tmh::release(*b);
  for (tmh::DevBuf* b : {&c->tab64, &c->tab32, &c->tabT64, &c->tabT32, &c->t64, &c->t32, &c->dt64,
                        &c->tden, &c->ttmp, &c->partial, &c->xlow, &c->work_a, &c->work_b, &c->work_c, &c->basis,
                        &c->dots, &c->dotpart, &c->scal, &c->plan_items[0], &c->plan_items[1],
                        &c->plan_ibeg[0], &c->plan_ibeg[1]})
    tmh::release(*b);
  if (c->host_pinned) hipHostFree(c->host_pinned);
  if (c->side) {
    hipStreamSynchronize(c->side);
    hipStreamDestroy(c->side);
  }
  if (c->ev_fork) hipEventDestroy(c->ev_fork);
  if (c->ev_join) hipEventDestroy(c->ev_join);
  for (int w = 0; w < 2; ++w)
    for (auto& pr : c->prof_pending[w]) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
  delete c;
}

#define CHECK_CTX(c)                  \
  do {                                \
    if (!(c)) return TM_ERR_INVALID_ARG; \
    hipSetDevice((c)->device);        \
  } while (0)

// Lattice detection: row-major nx x ny grid of equal pitch in z = 0.
static bool detect_lattice(int n, const double* pos, int& nx, int& ny, double& pitch) {
  const double x0 = pos[0], y0 = pos[1];
  nx = 1;
  while (nx < n && pos[3 * nx + 1] == y0) ++nx;
  if (n % nx != 0) return false;
  ny = n / nx;
  pitch = 1.0;
  if (nx > 1) pitch = pos[3] - pos[0];
  else if (ny > 1) pitch = pos[3 * nx + 1] - pos[1];
  if (!(pitch > 0.0)) return false;
  const double tolp = 1e-9 * pitch;
  for (int i = 0; i < n; ++i) {
    const int ix = i % nx, iy = i / nx;
    if (std::fabs(pos[3 * i] - (x0 + ix * pitch)) > tolp ||
        std::fabs(pos[3 * i + 1] - (y0 + iy * pitch)) > tolp || std::fabs(pos[3 * i + 2]) > tolp)
      return false;
  }
  return true;
}

int tm_set_geometry(tm_ctx* c, int n, const double* pos, double k, int lmax) {
  CHECK_CTX(c);
  if (n < 1 || !pos) return tmh::set_err(c, TM_ERR_INVALID_ARG, "need n >= 1 positions");
  if (lmax < 1 || lmax > tmh::LMAX_SUPPORTED)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "lmax must be in [1, 6]");
  if (!(k > 0.0) || !std::isfinite(k)) return tmh::set_err(c, TM_ERR_INVALID_ARG, "k must be > 0");
  for (int i = 0; i < 3 * n; ++i)
    if (!std::isfinite(pos[i])) return tmh::set_err(c, TM_ERR_NAN, "non-finite position");
  int nx = 0, ny = 0;
  double pitch = 0.0;
  const bool lattice = detect_lattice(n, pos, nx, ny, pitch);
  if (!lattice) {
    // arbitrary centres in the plane z = 0 (the z-mirror class split holds)
    double scale = 0.0;
    for (int i = 0; i < n; ++i) scale = std::max(scale, std::hypot(pos[3 * i], pos[3 * i + 1]));
    const double tolz = 1e-9 * std::max(scale, 1.0 / k);
    for (int i = 0; i < n; ++i)
      if (std::fabs(pos[3 * i + 2]) > tolz)
        return tmh::set_err(c, TM_ERR_NOT_LATTICE,
                            "scatterer " + std::to_string(i) + " is off the z = 0 plane");
  }
  tmh::Geometry& g = c->g;
  g = tmh::Geometry{};
  g.n = n;
  g.lattice = lattice;
  g.nx = lattice ? nx : n;
  g.ny = lattice ? ny : 1;
  g.lmax = lmax;
  g.pitch = lattice ? pitch : 0.0;
  g.k = k;
  g.x0 = pos[0];
  g.y0 = pos[1];
  g.tnx = g.nx;
  g.tny = g.ny;
  tmh::host_slot_maps(lmax, g, c->maps);
  tmh::host_mblock_maps(lmax, c->mbmaps);
  c->have_geom = c->have_t = c->have_dt = c->have_tabT = c->have_dtab = c->t_dense = false;
  c->t_mblock = false;
  c->plan_R[0] = c->plan_R[1] = -1;
  int rc;
  if (lattice) {
    if ((rc = tmh::build_tables(c)) != TM_OK) return rc;
    c->host_xy.clear();
  } else {
    // no displacement tables: release a previous lattice's
    for (tmh::DevBuf* b : {&c->tab64, &c->tab32, &c->tabT64, &c->tabT32})
      if (b->p) {
        TM_HIP(c, hipStreamSynchronize(c->stream));
        tmh::release(*b);
      }
    c->host_xy.assign((size_t)2 * n, 0.0);
    for (int i = 0; i < n; ++i) {
      c->host_xy[2 * i] = pos[3 * i];
      c->host_xy[2 * i + 1] = pos[3 * i + 1];
    }
    // coincident centres leave a block undefined
    std::vector<std::pair<double, double>> sorted(n);
    for (int i = 0; i < n; ++i) sorted[i] = {pos[3 * i], pos[3 * i + 1]};
    std::sort(sorted.begin(), sorted.end());
    for (int i = 1; i < n; ++i)
      if (sorted[i] == sorted[i - 1]) return tmh::set_err(c, TM_ERR_OVERLAP, "two scatterers share a centre");
    if ((rc = tmh::ensure(c, c->xy, (size_t)2 * n * sizeof(double))) != TM_OK) return rc;
    TM_HIP(c, hipMemcpy(c->xy.p, c->host_xy.data(), (size_t)2 * n * sizeof(double), hipMemcpyHostToDevice));
    if ((rc = tmh::build_offlattice_constants(c)) != TM_OK) return rc;
  }
  const size_t vb = (size_t)g.vec_len();
  if ((rc = tmh::ensure(c, c->t64, vb * sizeof(c128))) != TM_OK) return rc;
  if ((rc = tmh::ensure(c, c->t32, vb * sizeof(tmh::c64))) != TM_OK) return rc;
  if ((rc = tmh::ensure(c, c->dt64, vb * sizeof(c128))) != TM_OK) return rc;
  TM_HIP(c, hipMemsetAsync(c->t64.p, 0, vb * sizeof(c128), c->stream));
  TM_HIP(c, hipMemsetAsync(c->t32.p, 0, vb * sizeof(tmh::c64), c->stream));
  TM_HIP(c, hipMemsetAsync(c->dt64.p, 0, vb * sizeof(c128), c->stream));
  c->have_geom = true;
  return TM_OK;
}

int tm_get_lattice(const tm_ctx* c, int* nx, int* ny, double* pitch) {
  if (!c || !c->have_geom) return TM_ERR_STATE;
  if (nx) *nx = c->g.nx;
  if (ny) *ny = c->g.ny;
  if (pitch) *pitch = c->g.pitch;
  return TM_OK;
}

int tm_mie(int lmax, double k, double radius, double n_re, double n_im, tm_c128* t_out,
           tm_c128* dtdr_out) {
  if (lmax < 1 || lmax > tmh::LMAX_SUPPORTED || !t_out) return TM_ERR_INVALID_ARG;
  if (!std::isfinite(k) || !std::isfinite(radius) || !std::isfinite(n_re) || !std::isfinite(n_im))
    return TM_ERR_NAN;
  const double nabs = std::hypot(n_re, n_im);
  if (!(k > 0.0) || !(radius > 0.0) || n_im < 0.0 || k * radius * std::max(1.0, nabs) > 12.0)
    return TM_ERR_INVALID_ARG;
  tm_c128* d = nullptr;
  const size_t bytes = (size_t)4 * lmax * sizeof(tm_c128);
  if (hipMalloc((void**)&d, bytes) != hipSuccess) return TM_ERR_OOM;
  int rc = tmh::launch_mie_one(nullptr, radius, k, n_re, n_im, lmax, d);
  tm_c128 h[4 * tmh::LMAX_SUPPORTED];
  if (rc == TM_OK && hipMemcpy(h, d, bytes, hipMemcpyDeviceToHost) != hipSuccess) rc = TM_ERR_HIP;
  if (hipFree(d) != hipSuccess && rc == TM_OK) rc = TM_ERR_HIP;
  if (rc != TM_OK) return rc;
  for (int q = 0; q < 2 * lmax; ++q) {
    t_out[q] = h[q];
    if (dtdr_out) dtdr_out[q] = h[2 * lmax + q];
  }
  return TM_OK;
}

namespace {
// Enclosing spheres of radii `re` must not intersect (App. I.C): on a
// lattice every pair closer than twice the largest radius is visited by
// displacement; off a lattice, by a cell grid of that size.
int check_enclosing(tm_ctx* c, const std::vector<double>& re, const char* what) {
  const tmh::Geometry& g = c->g;
  double rmax = 0.0;
  for (double v : re) rmax = std::max(rmax, v);
  auto fail = [&](int i, int j) {
    return tmh::set_err(c, TM_ERR_OVERLAP, std::string(what) + " " + std::to_string(i) + " and " +
                                              std::to_string(j) + " overlap");
  };
  if (g.lattice) {
    const int reach = (int)std::floor(2.0 * rmax / g.pitch);
    for (int dy = 0; dy <= reach; ++dy)
      for (int dx = (dy == 0 ? 1 : -reach); dx <= reach; ++dx) {
        const double dist = g.pitch * std::hypot((double)dx, (double)dy);
        if (dist > 2.0 * rmax) continue;
        for (int iy = 0; iy + dy < g.ny; ++iy)
          for (int ix = std::max(0, -dx); ix < g.nx && ix + dx < g.nx; ++ix) {
            const int i = iy * g.nx + ix, j = (iy + dy) * g.nx + ix + dx;
            if (re[i] + re[j] >= dist) return fail(i, j);
          }
      }
    return TM_OK;
  }
  const std::vector<double>& xy = c->host_xy;
  const double cell = std::max(2.0 * rmax, 1e-300);
  double xmin = xy[0], ymin = xy[1];
  for (int i = 0; i < g.n; ++i) {
    xmin = std::min(xmin, xy[2 * i]);
    ymin = std::min(ymin, xy[2 * i + 1]);
  }
  std::vector<std::pair<long long, int>> key(g.n);
  auto cx_of = [&](int i) { return (long long)std::floor((xy[2 * i] - xmin) / cell); };
  auto cy_of = [&](int i) { return (long long)std::floor((xy[2 * i + 1] - ymin) / cell); };
  const long long W = 1 << 30;
  for (int i = 0; i < g.n; ++i) key[i] = {cy_of(i) * W + cx_of(i), i};
  std::sort(key.begin(), key.end());
  for (int a = 0; a < g.n; ++a) {
    const int i = key[a].second;
    const long long cxi = cx_of(i), cyi = cy_of(i);
    for (long long dyc = -1; dyc <= 1; ++dyc)
      for (long long dxc = -1; dxc <= 1; ++dxc) {
        const long long kk = (cyi + dyc) * W + (cxi + dxc);
        auto it = std::lower_bound(key.begin(), key.end(), std::make_pair(kk, -1));
        for (; it != key.end() && it->first == kk; ++it) {
          const int j = it->second;
          if (j <= i) continue;
          const double d = std::hypot(xy[2 * i] - xy[2 * j], xy[2 * i + 1] - xy[2 * j + 1]);
          if (re[i] + re[j] >= d) return fail(std::min(i, j), std::max(i, j));
        }
      }
  }
  return TM_OK;
}
}  // namespace

int tm_set_spheres(tm_ctx* c, const double* radii, double n_re, double n_im) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!radii) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null radii");
  if (!std::isfinite(n_re) || !std::isfinite(n_im) || n_im < 0.0)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "invalid refractive index");
  const tmh::Geometry& g = c->g;
  std::vector<double> r(g.n);
  TM_HIP(c, hipMemcpyAsync(r.data(), radii, g.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TM_HIP(c, hipStreamSynchronize(c->stream));
  const double nabs = std::hypot(n_re, n_im);
  for (int i = 0; i < g.n; ++i) {
    if (!std::isfinite(r[i])) return tmh::set_err(c, TM_ERR_NAN, "non-finite radius");
    if (!(r[i] > 0.0)) return tmh::set_err(c, TM_ERR_INVALID_ARG, "radius must be > 0");
    if (g.k * r[i] * std::max(1.0, nabs) > 12.0)
      return tmh::set_err(c, TM_ERR_INVALID_ARG, "k r |n| > 12 is outside the supported range");
  }
  // non-intersecting spheres (App. I.C), diagonal and farther neighbours included
  int rc = check_enclosing(c, r, "spheres");
  if (rc != TM_OK) return rc;
  rc = tmh::launch_mie(c, radii, n_re, n_im);
  if (rc != TM_OK) return rc;
  c->have_t = c->have_dt = true;
  c->t_dense = c->t_mblock = false;
  return TM_OK;
}

int tm_set_cylinders(tm_ctx* c, const double* radii, double height, double n_re, double n_im,
                     int n_quad) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!radii) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null radii");
  if (!std::isfinite(n_re) || !std::isfinite(n_im) || n_im < 0.0 || !(height > 0.0) ||
      !std::isfinite(height) || n_quad < 0 || n_quad > 1024 || (n_quad > 0 && n_quad < 4))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "invalid cylinder parameters");
  const tmh::Geometry& g = c->g;
  std::vector<double> r(g.n), re(g.n);
  TM_HIP(c, hipMemcpyAsync(r.data(), radii, g.n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
  TM_HIP(c, hipStreamSynchronize(c->stream));
  const double nabs = std::hypot(n_re, n_im);
  for (int i = 0; i < g.n; ++i) {
    if (!std::isfinite(r[i])) return tmh::set_err(c, TM_ERR_NAN, "non-finite radius");
    if (!(r[i] > 0.0)) return tmh::set_err(c, TM_ERR_INVALID_ARG, "radius must be > 0");
    re[i] = std::hypot(r[i], 0.5 * height);
    if (g.k * re[i] * std::max(1.0, nabs) > 12.0)
      return tmh::set_err(c, TM_ERR_INVALID_ARG, "k r_enclosing |n| > 12 is outside the supported range");
  }
  int rc;
  if ((rc = check_enclosing(c, re, "the enclosing spheres of cylinders")) != TM_OK) return rc;
  const size_t bytes = (size_t)g.n * g.L * g.L * sizeof(tm_c128);
  if ((rc = tmh::ensure(c, c->tden, bytes)) != TM_OK) return rc;
  if ((rc = tmh::launch_ebcm_cylinders(c, c->stream, g.n, radii, height, g.k, n_re, n_im, g.lmax,
                                       n_quad > 0 ? n_quad : 96, (tm_c128*)c->tden.p)) != TM_OK)
    return rc;
  c->have_t = true;
  c->have_dt = false;
  c->t_dense = true;
  return tmh::tdense_prepare(c);
}

int tm_ebcm_cylinder(int lmax, double k, double radius, double height, double n_re, double n_im,
                     int n_quad, tm_c128* T_out) {
  if (lmax < 1 || lmax > tmh::LMAX_SUPPORTED || !T_out || n_quad < 0 || n_quad > 1024 ||
      (n_quad > 0 && n_quad < 4))
    return TM_ERR_INVALID_ARG;
  if (!std::isfinite(k) || !std::isfinite(radius) || !std::isfinite(height) || !std::isfinite(n_re) ||
      !std::isfinite(n_im))
    return TM_ERR_NAN;
  if (!(k > 0.0) || !(radius > 0.0) || !(height > 0.0) || n_im < 0.0 ||
      k * std::hypot(radius, 0.5 * height) * std::max(1.0, std::hypot(n_re, n_im)) > 12.0)
    return TM_ERR_INVALID_ARG;
  const int L = 2 * lmax * (lmax + 2);
  double* dr = nullptr;
  tm_c128* dT = nullptr;
  if (hipMalloc((void**)&dr, sizeof(double)) != hipSuccess ||
      hipMalloc((void**)&dT, (size_t)L * L * sizeof(tm_c128)) != hipSuccess) {
    (void)hipGetLastError();
    if (dr) hipFree(dr);
    return TM_ERR_OOM;
  }
  int rc = TM_OK;
  if (hipMemcpy(dr, &radius, sizeof(double), hipMemcpyHostToDevice) != hipSuccess) rc = TM_ERR_HIP;
  if (rc == TM_OK)
    rc = tmh::launch_ebcm_cylinders(nullptr, nullptr, 1, dr, height, k, n_re, n_im, lmax,
                                    n_quad > 0 ? n_quad : 96, dT);
  if (rc == TM_OK &&
      hipMemcpy(T_out, dT, (size_t)L * L * sizeof(tm_c128), hipMemcpyDeviceToHost) != hipSuccess)
    rc = TM_ERR_HIP;
  hipFree(dr);
  hipFree(dT);
  return rc;
}

int tm_set_tmatrix_diag(tm_ctx* c, const tm_c128* t) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!t) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null T");
  int rc = tmh::launch_set_tdiag(c, t);
  if (rc != TM_OK) return rc;
  TM_HIP(c, hipMemsetAsync(c->dt64.p, 0, c->dt64.bytes, c->stream));
  c->have_t = true;
  c->have_dt = false;
  c->t_dense = c->t_mblock = false;
  return TM_OK;
}

int tm_set_tmatrix_dense(tm_ctx* c, const tm_c128* T) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!T) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null T");
  const tmh::Geometry& g = c->g;
  const size_t bytes = (size_t)g.n * g.L * g.L * sizeof(tm_c128);
  int rc;
  if ((rc = tmh::ensure(c, c->tden, bytes)) != TM_OK) return rc;
  TM_HIP(c, hipMemcpyAsync(c->tden.p, T, bytes, hipMemcpyDeviceToDevice, c->stream));
  c->have_t = true;
  c->have_dt = false;
  c->t_dense = true;
  return tmh::tdense_prepare(c);
}

int tm_get_tmatrix_diag(tm_ctx* c, tm_c128* t, tm_c128* dtdr) {
  CHECK_CTX(c);
  if (!c->have_t) return tmh::set_err(c, TM_ERR_STATE, "T not set");
  if (c->t_dense) return tmh::set_err(c, TM_ERR_STATE, "T was set dense; it has no diagonal form");
  if (!t) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null output");
  return tmh::launch_get_tdiag(c, t, c->have_dt ? dtdr : nullptr);
}

int tm_plane_wave_rhs(tm_ctx* c, int R, const double* khat, const tm_c128* pol, tm_c128* a0) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (R < 1 || !khat || !pol || !a0) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  int rc;
  if ((rc = tmh::validate_incidence(c, R, khat, pol)) != TM_OK) return rc;
  return tmh::launch_plane_wave(c, R, khat, pol, a0);
}

static int validate_opts(tm_ctx* c, const tm_solve_opts* o) {
  if (!o) return tmh::set_err(c, TM_ERR_INVALID_ARG, "null options");
  if (!(o->tol > 0.0) || o->restart < 1 || o->restart > 1000 || o->max_iter < 1 ||
      (o->precision != TM_PREC_FP64 && o->precision != TM_PREC_MIXED) ||
      (o->precision == TM_PREC_MIXED && !(o->inner_tol > 0.0 && o->inner_tol < 1.0)))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "invalid solver options");
  return TM_OK;
}

static int solve_common(tm_ctx* c, Op op, int R, const tm_c128* rhs, tm_c128* out,
                        const tm_solve_opts* o, tm_solve_info* info) {
  CHECK_CTX(c);
  if (!c->have_geom || !c->have_t) return tmh::set_err(c, TM_ERR_STATE, "geometry and T must be set");
  if (R < 1 || !rhs || !out || !info) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  int rc;
  if ((rc = validate_opts(c, o)) != TM_OK) return rc;
  const tmh::Geometry& g = c->g;
  const long long len = g.vec_len();
  if ((rc = tmh::ensure(c, c->work_a, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
  if ((rc = tmh::ensure(c, c->work_b, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
  c128* bsl = (c128*)c->work_a.p;
  c128* xsl = (c128*)c->work_b.p;
  tmh::pack_slots(c->stream, g, c->maps, R, rhs, bsl);
  if (op == Op::Forward) {  // b = T a0
    if (c->t_dense) {
      if ((rc = tmh::ensure(c, c->ttmp, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
      if ((rc = tmh::launch_tdense(c, R, 0, nullptr, bsl, (c128*)c->ttmp.p)) != TM_OK) return rc;
      tmh::k_copy(c->stream, bsl, (const c128*)c->ttmp.p, (long long)R * len);
    } else {
      tmh::k_mul_t(c->stream, bsl, (const c128*)c->t64.p, bsl, len, R);
    }
  }
  if (o->use_x0) tmh::pack_slots(c->stream, g, c->maps, R, out, xsl);
  bool all_ok = true;
  for (int r = 0; r < R; ++r) {
    rc = tmh::gmres(c, op, bsl + (size_t)r * len, xsl + (size_t)r * len, *o, o->use_x0 != 0, info[r]);
    if (rc != TM_OK) return rc;
    if (info[r].status != TM_OK) all_ok = false;
  }
  tmh::unpack_slots(c->stream, g, c->maps, R, xsl, out);
  TM_HIP(c, hipStreamSynchronize(c->stream));
  return all_ok ? TM_OK : TM_NOT_CONVERGED;
}

int tm_solve(tm_ctx* c, int R, const tm_c128* a0, tm_c128* s, const tm_solve_opts* o,
             tm_solve_info* info) {
  return solve_common(c, Op::Forward, R, a0, s, o, info);
}

int tm_adjoint_solve(tm_ctx* c, int R, const tm_c128* v, tm_c128* mu, const tm_solve_opts* o,
                     tm_solve_info* info) {
  return solve_common(c, Op::Adjoint, R, v, mu, o, info);
}

int tm_apply_operator(tm_ctx* c, int R, const tm_c128* x, tm_c128* y, int precision, int op) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if ((op == TM_OP_FORWARD || op == TM_OP_ADJOINT) && !c->have_t)
    return tmh::set_err(c, TM_ERR_STATE, "T not set");
  if (R < 1 || !x || !y || x == y || op < 0 || op > 3 ||
      (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  const tmh::Geometry& g = c->g;
  const long long len = g.vec_len();
  int rc;
  if ((rc = tmh::ensure(c, c->work_a, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
  if ((rc = tmh::ensure(c, c->work_b, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
  tmh::pack_slots(c->stream, g, c->maps, R, x, (c128*)c->work_a.p);
  if ((rc = tmh::apply_op(c, (Op)op, precision, R, (const c128*)c->work_a.p, (c128*)c->work_b.p)) !=
      TM_OK)
    return rc;
  tmh::unpack_slots(c->stream, g, c->maps, R, (const c128*)c->work_b.p, y);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

namespace {
int check_jinc(tm_ctx* c, int n, const tm_jinc* src) {
  for (int j = 0; j < n; ++j) {
    const tm_jinc& q = src[j];
    const double v[7] = {q.x0, q.y0, q.z0, q.ax.re, q.ax.im, q.ay.re, q.ay.im};
    for (double x : v)
      if (!std::isfinite(x)) return tmh::set_err(c, TM_ERR_NAN, "non-finite jinc source " + std::to_string(j));
  }
  return TM_OK;
}
// polar nodes for the largest source-to-scatterer distance of a lattice box
int jinc_nodes(const tmh::Geometry& g, int n, const tm_jinc* src, int ox, int oy, int sx, int sy) {
  double rmax = 0.0;
  for (int j = 0; j < n; ++j) {
    const double xs[2] = {g.x0 + g.pitch * ox, g.x0 + g.pitch * (ox + sx - 1)};
    const double ys[2] = {g.y0 + g.pitch * oy, g.y0 + g.pitch * (oy + sy - 1)};
    for (double x : xs)
      for (double y : ys)
        rmax = std::max(rmax, std::sqrt((x - src[j].x0) * (x - src[j].x0) +
                                        (y - src[j].y0) * (y - src[j].y0) + src[j].z0 * src[j].z0));
  }
  return tmh::jinc_beta_count(g.k, rmax);
}
}  // namespace

int tm_jinc_rhs(tm_ctx* c, int R, const tm_jinc* src, int n_beta, tm_c128* a0) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (R < 1 || !src || !a0 || n_beta < 0 || n_beta > 100000)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  int rc;
  if ((rc = check_jinc(c, R, src)) != TM_OK) return rc;
  const tmh::Geometry& g = c->g;
  int nb = n_beta;
  if (nb == 0 && g.lattice) {
    nb = jinc_nodes(g, R, src, 0, 0, g.nx, g.ny);
  } else if (nb == 0) {
    double rmax = 0.0;
    for (int j = 0; j < R; ++j)
      for (int i = 0; i < g.n; ++i)
        rmax = std::max(rmax, std::sqrt(std::pow(c->host_xy[2 * i] - src[j].x0, 2) +
                                        std::pow(c->host_xy[2 * i + 1] - src[j].y0, 2) +
                                        src[j].z0 * src[j].z0));
    nb = tmh::jinc_beta_count(g.k, rmax);
  }
  return tmh::launch_jinc_rhs(c, R, src, nb, a0);
}

int tm_jinc_rhs_batched(tm_ctx* c, int n_sub, const tm_subregion* subs, int R, int n_src,
                        const tm_jinc* src, const int* groups, int n_beta, tm_c128* a0) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!c->g.lattice) return tmh::set_err(c, TM_ERR_NOT_LATTICE, "subregions need a lattice geometry");
  if (n_sub < 1 || R < 1 || n_src < 0 || !subs || !groups || !a0 || (n_src > 0 && !src) || n_beta < 0 ||
      n_beta > 100000)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  const tmh::Geometry& g = c->g;
  if (groups[0] != 0 || groups[n_sub * R] != n_src)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "groups must run from 0 to n_src");
  for (int q = 0; q < n_sub * R; ++q)
    if (groups[q + 1] < groups[q]) return tmh::set_err(c, TM_ERR_INVALID_ARG, "groups must not decrease");
  for (int k = 0; k < n_sub; ++k) {
    const tm_subregion& q = subs[k];
    if (q.side_x < 1 || q.side_y < 1 || q.origin_x < 0 || q.origin_y < 0 ||
        q.origin_x + q.side_x > g.nx || q.origin_y + q.side_y > g.ny)
      return tmh::set_err(c, TM_ERR_INVALID_ARG, "subregion " + std::to_string(k) + " outside the lattice");
  }
  int rc;
  if ((rc = check_jinc(c, n_src, src)) != TM_OK) return rc;
  int nb = n_beta;
  if (nb == 0) {
    nb = 1;
    for (int k = 0; k < n_sub; ++k)
      for (int r = 0; r < R; ++r) {
        const int j0 = groups[k * R + r], j1 = groups[k * R + r + 1];
        if (j1 > j0)
          nb = std::max(nb, jinc_nodes(g, j1 - j0, src + j0, subs[k].origin_x, subs[k].origin_y,
                                       subs[k].side_x, subs[k].side_y));
      }
  }
  return tmh::launch_jinc_rhs_packed(c, n_sub, subs, R, n_src, src, groups, nb, a0);
}

int tm_grad_position(tm_ctx* c, int R, const tm_c128* mu, const tm_c128* s, const tm_c128* a0,
                     const double* khat, const double* xd, const tm_c128* w, double* grad) {
  CHECK_CTX(c);
  if (!c->have_geom || !c->have_t) return tmh::set_err(c, TM_ERR_STATE, "geometry and T must be set");
  if (!c->g.lattice)
    return tmh::set_err(c, TM_ERR_NOT_LATTICE, "position gradients use the lattice's derivative tables");
  if (R < 1 || !mu || !s || !grad || (khat && !a0) || (!xd) != (!w))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if (khat)
    for (int q = 0; q < 3 * R; ++q)
      if (!std::isfinite(khat[q])) return tmh::set_err(c, TM_ERR_NAN, "non-finite khat");
  if (xd) {
    for (int q = 0; q < 3; ++q)
      if (!std::isfinite(xd[q])) return tmh::set_err(c, TM_ERR_NAN, "non-finite detector point");
    for (int q = 0; q < 3 * R; ++q)
      if (!std::isfinite(w[q].re) || !std::isfinite(w[q].im))
        return tmh::set_err(c, TM_ERR_NAN, "non-finite detector weight");
  }
  const tmh::Geometry& g = c->g;
  int rc;
  if (!c->have_dtab && (rc = tmh::build_derivative_tables(c)) != TM_OK) return rc;
  const long long vec = g.vec_len(), tot = (long long)R * vec;
  std::vector<c128> dcoef;
  std::vector<int> ddm;
  tmh::detector_grad_constants(g.lmax, dcoef, ddm);
  const size_t vb = (size_t)tot * sizeof(c128);
  const size_t cb = dcoef.size() * sizeof(c128), db = ddm.size() * sizeof(int);
  if ((rc = tmh::ensure(c, c->gpos, 7 * vb + cb + db)) != TM_OK) return rc;
  c128* base = (c128*)c->gpos.p;
  c128 *lam = base, *ss = base + tot, *aa = base + 2 * tot, *dxs = base + 3 * tot,
       *dys = base + 4 * tot, *dxtl = base + 5 * tot, *dytl = base + 6 * tot;
  c128* coef = base + 7 * tot;
  int* dm = (int*)(coef + dcoef.size());
  // lambda = T^T mu (the paper's adjoint unknown), in slot layout
  tmh::pack_slots(c->stream, g, c->maps, R, mu, aa);
  if (c->t_dense) {
    if ((rc = tmh::launch_tdense(c, R, 2, nullptr, aa, lam)) != TM_OK) return rc;
  } else {
    tmh::k_mul_t(c->stream, lam, (const c128*)c->t64.p, aa, vec, R);
  }
  tmh::pack_slots(c->stream, g, c->maps, R, s, ss);
  if (khat) tmh::pack_slots(c->stream, g, c->maps, R, a0, aa);
  // the four derivative products (FP64 block matvec on the derivative tables)
  const int tgt = c->mv_items[0] > 0 ? c->mv_items[0] : std::max(1, (16384 + 2 * R - 1) / (2 * R));
  const void* src[4] = {ss, ss, lam, lam};
  c128* dst[4] = {dxs, dys, dxtl, dytl};
  for (int t = 0; t < 4; ++t)
    if ((rc = tmh::lds_apply<double>(c, 0, R, c->dtab[t].p, src[t], nullptr, dst[t], TM_OP_COUPLING,
                                     tgt, nullptr, nullptr, 2)) != TM_OK)
      return rc;
  if ((rc = tmh::launch_gpos_contract(c, R, lam, ss, khat ? aa : nullptr, dxs, dys, dxtl, dytl, khat,
                                      grad)) != TM_OK)
    return rc;
  if (xd) {
    TM_HIP(c, hipMemcpyAsync(coef, dcoef.data(), cb, hipMemcpyHostToDevice, c->stream));
    TM_HIP(c, hipMemcpyAsync(dm, ddm.data(), db, hipMemcpyHostToDevice, c->stream));
    if ((rc = tmh::launch_gpos_detector(c, R, s, coef, dm, xd, w, grad)) != TM_OK) return rc;
    // the host constants are read by the asynchronous copies
    TM_HIP(c, hipStreamSynchronize(c->stream));
  }
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

int tm_near_field(tm_ctx* c, int R, const tm_c128* s, int P, const double* pts, tm_c128* E,
                  int precision) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (R < 1 || P < 0 || !s || (P > 0 && (!pts || !E)) ||
      (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if (P == 0) return TM_OK;
  return tmh::launch_near_field(c, R, s, P, pts, E, precision);
}

int tm_far_field(tm_ctx* c, int R, const tm_c128* s, int D, const double* dirs, tm_c128* F) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (R < 1 || D < 0 || !s || (D > 0 && (!dirs || !F)))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if (D == 0) return TM_OK;
  return tmh::launch_far_field(c, R, s, D, dirs, F);
}

int tm_detector_vector(tm_ctx* c, const double* xd, const tm_c128* w, tm_c128* v) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!xd || !w || !v) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  for (int q = 0; q < 3; ++q)
    if (!std::isfinite(xd[q]) || !std::isfinite(w[q].re) || !std::isfinite(w[q].im))
      return tmh::set_err(c, TM_ERR_NAN, "non-finite detector input");
  return tmh::launch_detector(c, xd, w, v);
}

int tm_near_field_adjoint(tm_ctx* c, int R, int P, const double* pts, const tm_c128* w,
                          tm_c128* v) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (R < 1 || R > 65535 || P < 0 || !v || (P > 0 && (!pts || !w)))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  return tmh::launch_near_field_t(c, R, P, pts, w, v);
}

int tm_grad_radius(tm_ctx* c, int R, const tm_c128* mu, const tm_c128* s, const tm_c128* a0,
                   double* grad) {
  CHECK_CTX(c);
  if (!c->have_dt) return tmh::set_err(c, TM_ERR_STATE, "dT/dr unavailable (spheres not set)");
  if (R < 1 || !mu || !s || !a0 || !grad) return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  const tmh::Geometry& g = c->g;
  const long long len = g.vec_len();
  int rc;
  if ((rc = tmh::ensure(c, c->work_a, (size_t)2 * R * len * sizeof(c128))) != TM_OK) return rc;
  if ((rc = tmh::ensure(c, c->work_b, (size_t)R * len * sizeof(c128))) != TM_OK) return rc;
  c128* s_sl = (c128*)c->work_a.p;
  c128* a_sl = s_sl + (size_t)R * len;
  c128* as_sl = (c128*)c->work_b.p;
  // exciting field a_exc = a0 + A s
  tmh::pack_slots(c->stream, g, c->maps, R, s, s_sl);
  if ((rc = tmh::apply_op(c, Op::Coupling, TM_PREC_FP64, R, s_sl, as_sl)) != TM_OK) return rc;
  tmh::pack_slots(c->stream, g, c->maps, R, a0, a_sl);
  tmh::k_add(c->stream, a_sl, a_sl, as_sl, (long long)R * len);
  tmh::pack_slots(c->stream, g, c->maps, R, mu, s_sl);
  return tmh::launch_grad(c, R, s_sl, a_sl, grad);
}

int tm_set_matvec_config(tm_ctx* c, int precision, int variant, int items) {
  CHECK_CTX(c);
  if ((precision != TM_PREC_FP64 && precision != TM_PREC_MIXED) || variant < 0 || variant > 10 ||
      items < 0)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad matvec configuration");
  const int w = precision == TM_PREC_MIXED ? 1 : 0;
  c->mv_variant[w] = variant;
  c->mv_items[w] = items;
  return TM_OK;
}

int tm_get_matvec_config(tm_ctx* c, int precision, int* variant, int* items) {
  CHECK_CTX(c);
  if (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED)
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad precision");
  const int w = precision == TM_PREC_MIXED ? 1 : 0;
  if (variant) *variant = c->mv_variant[w];
  if (items) *items = c->mv_items[w];
  return TM_OK;
}

int tm_autotune(tm_ctx* c, int n_rhs, int precision, double* best_ms) {
  CHECK_CTX(c);
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (n_rhs < 1 || (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if (!c->g.lattice) return tmh::set_err(c, TM_ERR_NOT_LATTICE, "the tuned kernels are the lattice's");
  return tmh::autotune(c, n_rhs, precision, best_ms);
}

int tm_set_progress(tm_ctx* c, tm_progress_fn fn, void* user) {
  CHECK_CTX(c);
  c->progress = fn;
  c->progress_user = user;
  return TM_OK;
}

int tm_profile_enable(tm_ctx* c, int enable) {
  CHECK_CTX(c);
  c->prof = enable != 0;
  return TM_OK;
}

int tm_profile_reset(tm_ctx* c) {
  CHECK_CTX(c);
  hipStreamSynchronize(c->stream);
  for (int w = 0; w < 2; ++w) {
    for (auto& pr : c->prof_pending[w]) {
      hipEventDestroy(pr.first);
      hipEventDestroy(pr.second);
    }
    c->prof_pending[w].clear();
    c->prof_acc[w] = tmh::ProfAcc{};
  }
  return TM_OK;
}

int tm_profile_query(tm_ctx* c, int which, double* total_ms, long long* launches,
                     double* flops_per_launch) {
  CHECK_CTX(c);
  if (which < 0 || which > 1) return tmh::set_err(c, TM_ERR_INVALID_ARG, "which must be 0 or 1");
  TM_HIP(c, hipStreamSynchronize(c->stream));
  for (auto& pr : c->prof_pending[which]) {
    float ms = 0.f;
    TM_HIP(c, hipEventElapsedTime(&ms, pr.first, pr.second));
    c->prof_acc[which].ms += ms;
    c->prof_acc[which].launches++;
    hipEventDestroy(pr.first);
    hipEventDestroy(pr.second);
  }
  c->prof_pending[which].clear();
  if (total_ms) *total_ms = c->prof_acc[which].ms;
  if (launches) *launches = c->prof_acc[which].launches;
  if (flops_per_launch) *flops_per_launch = c->prof_acc[which].flops;
  return TM_OK;
}

}  // extern "C"
