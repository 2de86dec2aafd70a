// Allocation-free operator application (for callers that cannot allocate:
// code under HIP graph capture, tight serving loops).
//
// Every buffer the call needs beyond the caller's x and y and the context's
// tables (the packed input and output, the low-precision copy of the input,
// the work split and the partial sums of the block matvec) lives in one
// file-scope device array, `scratch`, of TM_NOALLOC_SCRATCH_BYTES.  Each GPU
// holds its own copy of the array for the life of the process; its device
// address is looked up once per device (tm_create) with hipGetSymbolAddress
// and only that address is handed to kernels.  Calls on one GPU share the
// array: calls that overlap in time on one GPU (two streams, two threads)
// race.  Nothing in the array needs to start at zero: every word a call
// reads was written earlier in the same call.
#include <algorithm>
#include <mutex>

#include "tm_internal.h"

namespace tmh {

static __device__ __align__(256) unsigned char scratch[TM_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_mu;
void* g_scratch[kMaxDevices] = {};  // device address of `scratch`, per device

size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }
}  // namespace

int noalloc_init(tm_ctx* c) {
  if (c->device < 0 || c->device >= kMaxDevices)
    return set_err(c, TM_ERR_INVALID_ARG, "device index beyond the scratch table");
  std::lock_guard<std::mutex> lk(g_mu);
  if (g_scratch[c->device]) return TM_OK;
  // the calling thread has c->device current (tm_create set it)
  void* p = nullptr;
  const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p) {
    (void)hipGetLastError();
    return set_err(c, TM_ERR_HIP,
                   std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
  }
  g_scratch[c->device] = p;
  return TM_OK;
}

static void* scratch_of(int device) {
  std::lock_guard<std::mutex> lk(g_mu);
  return (device >= 0 && device < kMaxDevices) ? g_scratch[device] : nullptr;
}

// Largest items-per-tile (at most the default split's) whose buffers fit
// `avail` bytes; 0 if not even one item per tile fits.
template <typename T>
static int fit_ipt(const Geometry& g, int R, size_t avail) {
  int hi = lds_fixed_default_ipt<T>(g, R);
  if (lds_fixed_bytes<T>(g, R, 1) > avail) return 0;
  int lo = 1;  // fits
  while (lo < hi) {
    const int mid = lo + (hi - lo + 1) / 2;
    if (lds_fixed_bytes<T>(g, R, mid) <= avail) lo = mid;
    else hi = mid - 1;
  }
  return lo;
}

template <typename T>
static int apply_noalloc(tm_ctx* c, int R, const tm_c128* x, tm_c128* y, int op, char* base) {
  const Geometry& g = c->g;
  const long long vec = g.vec_len(), total = vec * R;
  const bool transposed = (op == TM_OP_ADJOINT || op == TM_OP_COUPLING_T);
  const bool need_prep = !std::is_same<T, double>::value || op == TM_OP_ADJOINT;
  const size_t vbytes = align256((size_t)total * sizeof(c128));
  const size_t lbytes = need_prep ? align256((size_t)total * sizeof(cplx<T>)) : 0;
  const size_t fixed = 2 * vbytes + lbytes;
  if (fixed >= (size_t)TM_NOALLOC_SCRATCH_BYTES)
    return set_err(c, TM_ERR_INVALID_ARG,
                   "problem too large for the allocation-free scratch (" +
                       std::to_string(fixed) + " bytes of vectors, limit " +
                       std::to_string((size_t)TM_NOALLOC_SCRATCH_BYTES) + ")");
  const int ipt = fit_ipt<T>(g, R, (size_t)TM_NOALLOC_SCRATCH_BYTES - fixed);
  if (ipt < 1)
    return set_err(c, TM_ERR_INVALID_ARG,
                   "problem too large for the allocation-free scratch (limit " +
                       std::to_string((size_t)TM_NOALLOC_SCRATCH_BYTES) + " bytes)");
  c128* xa = reinterpret_cast<c128*>(base);
  c128* yb = reinterpret_cast<c128*>(base + vbytes);
  void* xl = need_prep ? (void*)(base + 2 * vbytes) : nullptr;
  void* rest = base + fixed;
  pack_slots(c->stream, g, c->maps, R, x, xa);
  const void* xin = xa;
  if (need_prep) {
    launch_prep<T>(c->stream, xa, op == TM_OP_ADJOINT ? (const c128*)c->t64.p : nullptr, xl, vec,
                   total);
    xin = xl;
  }
  const int which = std::is_same<T, double>::value ? 0 : 1;
  const void* table = std::is_same<T, double>::value
                          ? (transposed ? c->tabT64.p : c->tab64.p)
                          : (transposed ? c->tabT32.p : c->tab32.p);
  // the context's LDS prefetch depth (variants 8..10), else the default
  int pf = c->mv_variant[which] >= 8 ? c->mv_variant[which] - 7 : (which == 0 ? 2 : 1);
  int rc = lds_apply_fixed<T>(c, R, table, xin, xa, yb, op, pf, ipt, rest);
  if (rc != TM_OK) return rc;
  unpack_slots(c->stream, g, c->maps, R, yb, y);
  TM_HIP(c, hipGetLastError());
  return TM_OK;
}

}  // namespace tmh

extern "C" int tm_apply_operator_noalloc(tm_ctx* c, int R, const tm_c128* x, tm_c128* y,
                                         int precision, int op) {
  if (!c) return TM_ERR_INVALID_ARG;
  if (!c->have_geom) return tmh::set_err(c, TM_ERR_STATE, "set geometry first");
  if (!c->g.lattice) return tmh::set_err(c, TM_ERR_NOT_LATTICE, "the allocation-free operator needs a lattice");
  if (R < 1 || !x || !y || x == y || op < 0 || op > 3 ||
      (precision != TM_PREC_FP64 && precision != TM_PREC_MIXED))
    return tmh::set_err(c, TM_ERR_INVALID_ARG, "bad arguments");
  if ((op == TM_OP_FORWARD || op == TM_OP_ADJOINT) && !c->have_t)
    return tmh::set_err(c, TM_ERR_STATE, "T not set");
  if (c->t_dense && (op == TM_OP_FORWARD || op == TM_OP_ADJOINT))
    return tmh::set_err(c, TM_ERR_STATE,
                        "the allocation-free operator takes diagonal T-matrices only");
  if ((op == TM_OP_ADJOINT || op == TM_OP_COUPLING_T) && !c->have_tabT)
    return tmh::set_err(c, TM_ERR_STATE,
                        "transposed tables not built yet (one tm_apply_operator call with a "
                        "transposed op, or tm_adjoint_solve, builds them)");
  char* base = static_cast<char*>(tmh::scratch_of(c->device));
  if (!base) return tmh::set_err(c, TM_ERR_STATE, "scratch address not set up for this device");
  if (precision == TM_PREC_MIXED) return tmh::apply_noalloc<float>(c, R, x, y, op, base);
  return tmh::apply_noalloc<double>(c, R, x, y, op, base);
}
