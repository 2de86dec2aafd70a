// Internal declarations of libtmhip (not part of the C ABI).
//
// Internal vector layout ("slot layout"): the in-plane lattice makes every
// translation block split into two classes c = (l + m + p) mod 2 (z-mirror
// symmetry of App. I.C's alpha/beta: P_q^|mu|(0) vanishes unless q + |mu| is
// even, alpha needs l+l'+q even and beta odd).  Each class holds L/2
// coefficients (8, 15, 24, 35, 48 for lmax 2..6), padded to S = 16, 32 or 48
// slots (whole groups of 16, the MFMA tile edge), so a per-scatterer vector
// is stored as
//   [rhs][class 0..1][site 0..N-1][slot 0..S-1]   complex
// and a translation block per displacement as [class][S][S].  Pad slots are
// zero in every table, T and vector, and stay zero under every operation.
#pragma once
#include <hip/hip_runtime.h>
#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "../../include/tmhip.h"
#include "tm_host.h"

namespace tmh {

constexpr int SLOTS = 16;          // slots per group (the MFMA tile edge)
constexpr int NCLASS = 2;
constexpr int LMAX_SUPPORTED = 6;
constexpr int SMAX = 48;           // slots per class at lmax 6 (48 members)
constexpr int LM_MAX = 2 * LMAX_SUPPORTED * (LMAX_SUPPORTED + 2);  // 96 coefficients
constexpr int QMAX = 2 * LMAX_SUPPORTED;
// slots per class for lmax: L/2 = lmax(lmax+2) rounded up to a multiple of 16
inline int slots_for_lmax(int lmax) { return SLOTS * ((lmax * (lmax + 2) + SLOTS - 1) / SLOTS); }

template <typename T>
struct cplx {
  T re, im;
};
using c64 = cplx<float>;
using c128 = cplx<double>;

struct Geometry {
  int n = 0, nx = 0, ny = 0, lmax = 0, L = 0;
  bool lattice = true;  // false: arbitrary positions in z = 0 (no displacement tables)
  int S = SLOTS, NG = 1;                      // slots per class, groups of 16 per class
  double pitch = 0.0, k = 0.0, x0 = 0.0, y0 = 0.0;
  // slot map: for boundary index n -> class, slot; and per class the list
  std::vector<int> cls_of, slot_of;           // [L]
  std::vector<int> n_of[NCLASS];              // [class][slot] -> n or -1
  int tnx = 0, tny = 0;                       // table half extents (= nx, ny)
  long long n_disp() const { return (long long)(2 * tnx - 1) * (2 * tny - 1); }
  long long vec_len() const { return (long long)NCLASS * n * S; }  // complex per RHS
};

// Device-side argument bundle for coefficient maps.
struct SlotMaps {
  int cls_of[LM_MAX];
  int slot_of[LM_MAX];
  int n_of[NCLASS][SMAX];
  int L, lmax, S;
};

static_assert(MB_LM_MAX == LM_MAX && MB_BLK_MAX == 2 * LMAX_SUPPORTED + 1,
              "m-block maps sized for the supported lmax");

// Scatterer centres in the z = 0 plane as kernels see them: on a lattice
// they follow from the site index, otherwise from a device array [N][2].
struct SitePos {
  const double* xy;  // device [N][2] (x, y), or null on a lattice
  int nx;
  double x0, y0, pitch;
  __device__ inline void at(long long i, double& x, double& y) const {
    if (xy) {
      x = xy[2 * i];
      y = xy[2 * i + 1];
    } else {
      x = x0 + pitch * (double)(i % nx);
      y = y0 + pitch * (double)(i / nx);
    }
  }
};

// One subregion of a batched solve: its lattice, the offset of its
// [R][2][N_k][S] block in the packed vector, and its origin in the full
// lattice (for T and positions).
struct SubParams {
  int nx, ny, tiles_x, ox;
  int oy, pad0;
  long long vec_off;
};


// Workspace buffer that grows on demand.
struct DevBuf {
  void* p = nullptr;
  size_t bytes = 0;
};

struct ProfAcc {
  double ms = 0.0;
  long long launches = 0;
  double flops = 0.0;
};

}  // namespace tmh

struct tm_ctx {
  int device = 0;
  hipStream_t stream = nullptr;
  // second stream (default priority) for the wide-tile launch of the block
  // matvec, forked from and joined back into `stream` by the two events
  hipStream_t side = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;
  std::string err;
  tm_progress_fn progress = nullptr;  // optional per-cycle callback
  void* progress_user = nullptr;
  tmh::Geometry g;
  tmh::SlotMaps maps{};
  bool have_geom = false, have_t = false, have_dt = false;
  bool t_dense = false;  // T given as dense per-scatterer blocks (tden), not diagonal
  bool t_mblock = false;  // ... and zero between different m: applied from tmb
  // translation tables [D][2][S][S]
  tmh::DevBuf tab64, tab32, tabT64, tabT32;
  bool have_tabT = false;
  // FP64 derivative tables of the position gradient: d/dx, d/dy, and the
  // transposed operator's d/dx, d/dy (built on first use)
  tmh::DevBuf dtab[4];
  bool have_dtab = false;
  tmh::DevBuf gpos;  // position-gradient workspace (slot-layout vectors)
  tmh::DevBuf jinc_buf;  // jinc sources, polar nodes and subregion tables
  tmh::DevBuf xy;        // scatterer centres [N][2] (off-lattice geometries)
  tmh::DevBuf olc;       // off-lattice translation constants (coef, dm)
  std::vector<double> host_xy;  // the same on the host (off-lattice)
  // T and dT/dr in slot layout [2][N][S]
  tmh::DevBuf t64, t32, dt64;
  tmh::DevBuf tden, ttmp;  // dense T [N][L][L] (boundary order); its scratch vector
  tmh::DevBuf tmb, tmflag;  // dense T as m-blocks [N][per_site]; structure flag
  tmh::MbMaps mbmaps{};
  // workspaces
  tmh::DevBuf partial, xlow, work_a, work_b, work_c, basis, dots, dotpart, scal;
  // single-system GMRES state on the device (flags, Hessenberg, rotations)
  tmh::DevBuf gm_dev;
  // while set, the block-matvec kernels of apply_op return at once when the
  // pointed-to flag is nonzero (the GMRES cycle has stopped)
  const int* mv_stop = nullptr;
  // host staging (pinned)
  void* host_pinned = nullptr;
  size_t host_pinned_bytes = 0;
  // profiling
  bool prof = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  tmh::ProfAcc prof_acc[2];
  std::vector<std::pair<hipEvent_t, hipEvent_t>> prof_pending[2];
  // matvec launch configuration per precision slot (0 = FP64, 1 = complex64):
  // kernel variant, target work items per (rhs, class), and the cached plan
  // default: the LDS-staged kernels (FP64 prefetch depth 2, complex64 depth 3)
  int mv_variant[2] = {9, 8};
  int mv_items[2] = {0, 0};
  tmh::DevBuf plan_items[2], plan_ibeg[2];
  // the cached plan of a precision slot is reused only for the same kernel
  // family (1 = direct, 2 = LDS-staged), R and work-item target
  int plan_kind[2] = {0, 0};
  int plan_R[2] = {-1, -1}, plan_target[2] = {0, 0}, plan_nitems[2] = {0, 0};
  int plan_nreg[2] = {0, 0};  // LDS plan: items of regular tiles (wide-tile items follow)
  int last_batch_graphed = 0;
  // batched solves: time the candidate launch configurations before solving
  // (1) or use the fixed default (0); the configuration of the last batched
  // solve per precision slot (table prefetch depth, items per (rhs, class))
  int batch_autotune = 0;
  int batch_pf[2] = {0, 0}, batch_items[2] = {0, 0};
};

namespace tmh {

inline SitePos site_pos(const tm_ctx* c) {
  return SitePos{c->g.lattice ? nullptr : (const double*)c->xy.p, c->g.nx, c->g.x0, c->g.y0, c->g.pitch};
}

// ---- error helpers -------------------------------------------------------
int set_err(tm_ctx* c, int code, const std::string& msg);
#define TM_HIP(ctx, call)                                                       \
  do {                                                                          \
    hipError_t e_ = (call);                                                     \
    if (e_ != hipSuccess)                                                       \
      return ::tmh::set_err((ctx), TM_ERR_HIP,                                   \
                           std::string(#call ": ") + hipGetErrorString(e_));    \
  } while (0)

int ensure(tm_ctx* c, DevBuf& b, size_t bytes);
int validate_incidence(tm_ctx* c, int R, const double* khat, const tm_c128* pol);
int ensure_pinned(tm_ctx* c, size_t bytes);
void release(DevBuf& b);

// ---- launchers implemented in the .hip files ------------------------------
// tables (tm_table.hip)
int build_tables(tm_ctx* c);            // forward tables, FP64 + c64
int build_transposed_tables(tm_ctx* c); // A^T tables
int build_derivative_tables(tm_ctx* c); // position-gradient tables (FP64)
int build_offlattice_constants(tm_ctx* c);  // per-entry constants of the on-the-fly matvec
// on-the-fly block matvec for off-lattice geometries (tm_offlattice.hip)
enum class Op;
template <typename T>
int offlattice_apply(tm_ctx* c, Op op, int R, const void* xin, const c128* x, c128* y);
void detector_grad_constants(int lmax, std::vector<c128>& coef, std::vector<int>& dm);
void host_slot_maps(int lmax, Geometry& g, SlotMaps& m);

// basis kernels (tm_basis.hip)
int launch_mie(tm_ctx* c, const double* radii, double n_re, double n_im);
int launch_set_tdiag(tm_ctx* c, const tm_c128* t);
int launch_get_tdiag(tm_ctx* c, tm_c128* t, tm_c128* dt);
int launch_plane_wave(tm_ctx* c, int R, const double* khat, const tm_c128* pol, tm_c128* a0);
int launch_near_field(tm_ctx* c, int R, const tm_c128* s, int P, const double* pts, tm_c128* E,
                      int precision);
int launch_far_field(tm_ctx* c, int R, const tm_c128* s, int D, const double* dirs, tm_c128* F);
int launch_detector(tm_ctx* c, const double* xd, const tm_c128* w, tm_c128* v);
// dense T on slot-layout vectors: mode 0 y = T z, 1 y = x - T z, 2 y = T^T z
int launch_tdense(tm_ctx* c, int R, int mode, const c128* x, const c128* z, c128* y);
// after tden is filled: if T is zero between different m, pack its m-blocks
// into tmb and set t_mblock (the apply then reads only the blocks)
int tdense_prepare(tm_ctx* c);
int launch_mie_one(hipStream_t st, double radius, double k, double nre, double nim, int lmax,
                   tm_c128* out);
int launch_near_field_t(tm_ctx* c, int R, int P, const double* pts, const tm_c128* w, tm_c128* v);
int launch_grad(tm_ctx* c, int R, const c128* mu_slot, const c128* aexc_slot, double* grad);
// position gradient (slot-layout inputs; khat host [R][3] or null)
int launch_gpos_contract(tm_ctx* c, int R, const c128* lam, const c128* s, const c128* a0,
                         const c128* dxs, const c128* dys, const c128* dxtl, const c128* dytl,
                         const double* khat, double* grad);
// detector term of the position gradient (boundary-layout s; xd, w host)
int launch_gpos_detector(tm_ctx* c, int R, const tm_c128* s, const c128* coef, const int* dm,
                         const double* xd, const tm_c128* w, double* grad);

// null-field T-matrices of cylinders (tm_basis.hip): T device [N][L][L];
// c may be null (then no error message is recorded)
int launch_ebcm_cylinders(tm_ctx* c, hipStream_t st, int N, const double* radii, double height, double k,
                          double nre, double nim, int lmax, int nq, tm_c128* T);
// jinc sources (tm_basis.hip): one lattice [R][N][L], or packed subregions
// with one source group per (subregion, rhs)
int jinc_beta_count(double k, double rmax);
int launch_jinc_rhs(tm_ctx* c, int R, const tm_jinc* src, int nb, tm_c128* a0);
int launch_jinc_rhs_packed(tm_ctx* c, int S, const tm_subregion* subs, int R, int nsrc,
                           const tm_jinc* src, const int* grp, int nb, tm_c128* a0);

// layout conversions (tm_krylov.hip)
void pack_slots(hipStream_t st, const Geometry& g, const SlotMaps& m, int R, const tm_c128* in,
                c128* out);
void unpack_slots(hipStream_t st, const Geometry& g, const SlotMaps& m, int R, const c128* in,
                  tm_c128* out);

// matvec (tm_matvec.hip)
enum class Op { Forward = 0, Coupling = 1, Adjoint = 2, CouplingT = 3 };
// x, y in slot layout FP64, R right-hand sides contiguous (stride vec_len).
int apply_op(tm_ctx* c, Op op, int prec, int R, const c128* x, c128* y);
double matvec_flops(const Geometry& g);
int autotune(tm_ctx* c, int R, int prec, double* best_ms);

// block-kernel input: out = (T)(t * x) (t non-null) or (T)x
template <typename T>
void launch_prep(hipStream_t st, const c128* x, const c128* t, void* out, long long vec,
                 long long total);
// LDS-staged matvec with a device-made uniform work split (ipt items per
// tile) and every buffer inside `buf` (tm_matvec_lds.hip); no allocation,
// no host synchronisation
template <typename T>
int lds_apply(tm_ctx* c, int which, int R, const void* table, const void* xin, const c128* x,
              c128* y, int op, int items_target, hipEvent_t e0, hipEvent_t e1, int pf);
template <typename T>
size_t lds_fixed_bytes(const Geometry& g, int R, int ipt);
template <typename T>
int lds_fixed_default_ipt(const Geometry& g, int R);
template <typename T>
int lds_apply_fixed(tm_ctx* c, int R, const void* table, const void* xin, const c128* x, c128* y,
                    int op, int pf, int ipt, void* buf);
// per-device address of the allocation-free entry point's scratch array,
// looked up once per device by tm_create (tm_noalloc.hip)
int noalloc_init(tm_ctx* c);

// Krylov kernels (tm_krylov.hip).  `stop` (nullable, device): the kernel
// returns at once when *stop is nonzero.  k_multidot returns the number of
// partial-sum rows it wrote (at most nblk), to be passed to k_reduce_dots.
int k_multidot(hipStream_t st, const c128* V, long long stride, int nvec, const c128* w,
                long long len, c128* partial, int nblk, const int* stop = nullptr);
void k_reduce_dots(hipStream_t st, const c128* partial, int nblk, int nvec, c128* out,
                   const c128* add, const int* stop = nullptr);
void k_update(hipStream_t st, c128* w, const c128* V, long long stride, int nvec,
              const c128* h, long long len, double sign, const int* stop = nullptr);
void k_norm2_partial(hipStream_t st, const c128* w, long long len, double* partial, int nblk,
                     const int* stop = nullptr);
void k_reduce_norm(hipStream_t st, const double* partial, int nblk, double* out,
                   const int* stop = nullptr);
// Device-side Givens of one restarted GMRES cycle.  Layout of the state
// buffer: GmFlags, then H [(m+1) x m], cs [m], sn [m], g [m+1], y [m]
// (complex).  One Arnoldi step: column j of H from the two CGS passes' dots
// and the new vector's norm, the previous rotations applied, a new rotation,
// the residual estimate |g[j+1]|; `stop` is raised when the estimate reaches
// `target`, on a zero (lucky breakdown) or non-finite norm.
struct GmFlags {
  int stop, jend, nonfinite, pad;
  double inv_hn, est;
};
size_t gm_state_bytes(int m);
void k_gm_cycle_init(hipStream_t st, void* state, int m, const double* beta);
void k_gm_givens(hipStream_t st, void* state, int m, int j, const c128* h1, const c128* h2,
                 const double* hn, double target);
void k_gm_scale_next(hipStream_t st, c128* v, const c128* w, const void* state, long long len);
void k_gm_backsub(hipStream_t st, void* state, int m);
void k_gm_update_x(hipStream_t st, c128* x, const c128* V, long long len, const void* state, int m);
const c128* gm_y(const void* state, int m);
void k_scale(hipStream_t st, c128* y, const c128* x, double a, long long len);
void k_axpy_dev(hipStream_t st, c128* y, const c128* x, const c128* V, long long stride,
                int nvec, const c128* coef, long long len);
void k_sub(hipStream_t st, c128* out, const c128* a, const c128* b, long long len);
void k_add(hipStream_t st, c128* out, const c128* a, const c128* b, long long len);
void k_copy(hipStream_t st, c128* out, const c128* in, long long len);
void k_mul_t(hipStream_t st, c128* out, const c128* t, const c128* x, long long len_per_rhs,
             int R);
int krylov_blocks(long long len);

}  // namespace tmh
