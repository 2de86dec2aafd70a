"""Python binding of libtmhip (ctypes; argument marshalling only).

Every method forwards to the C entry point of the same name in
include/tmhip.h; all computation happens in the library's HIP kernels.  Device
arrays are torch tensors on the context's GPU (complex128 / float64,
contiguous); host arrays are numpy arrays.  torch is imported before the
library is loaded so that the library binds to the HIP runtime torch already
uses (one runtime per process); loading fails loudly if the library is
missing or a second HIP runtime would be mapped.
"""
import ctypes
import os

import numpy as np
import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libtmhip.so")

TM_OK = 0
TM_NOT_CONVERGED = 1
TM_PREC_FP64 = 0
TM_PREC_MIXED = 1
OPS = {"forward": 0, "coupling": 1, "adjoint": 2, "coupling_t": 3}
PRECISIONS = {"fp64": TM_PREC_FP64, "mixed": TM_PREC_MIXED, TM_PREC_FP64: 0, TM_PREC_MIXED: 1}


class TmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"tmhip status {code}: {msg}")
        self.code = code


class SolveOpts(ctypes.Structure):
    _fields_ = [("tol", ctypes.c_double), ("restart", ctypes.c_int), ("max_iter", ctypes.c_int),
                ("precision", ctypes.c_int), ("inner_tol", ctypes.c_double), ("use_x0", ctypes.c_int)]


class SolveInfo(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int), ("iters", ctypes.c_int), ("cycles", ctypes.c_int),
                ("matvecs_fp64", ctypes.c_int), ("matvecs_lowp", ctypes.c_int),
                ("rel_residual", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class Jinc(ctypes.Structure):
    _fields_ = [("x0", ctypes.c_double), ("y0", ctypes.c_double), ("z0", ctypes.c_double),
                ("axr", ctypes.c_double), ("axi", ctypes.c_double), ("ayr", ctypes.c_double),
                ("ayi", ctypes.c_double)]


def _jinc_array(sources):
    """[(x0, y0, z0, ax, ay)] -> a ctypes array of tm_jinc."""
    arr = (Jinc * max(1, len(sources)))()
    for j, (x0, y0, z0, ax, ay) in enumerate(sources):
        ax, ay = complex(ax), complex(ay)
        arr[j] = Jinc(float(x0), float(y0), float(z0), ax.real, ax.imag, ay.real, ay.imag)
    return arr


class Subregion(ctypes.Structure):
    _fields_ = [("origin_x", ctypes.c_int), ("origin_y", ctypes.c_int), ("side_x", ctypes.c_int),
                ("side_y", ctypes.c_int)]


_lib = None

# void (*)(void* user, int cycles, int iters, int n_live, double max_rel_residual)
PROGRESS_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                               ctypes.c_double)


def _hip_runtimes_mapped():
    paths = set()
    with open("/proc/self/maps") as f:
        for line in f:
            if "libamdhip64" in line:
                paths.add(os.path.realpath(line.split()[-1]))
    return paths


def load():
    """Load libtmhip.so (once).  Raises if it is missing or not loadable."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2107_09879_amd.build")
    lib = ctypes.CDLL(LIB_PATH, mode=ctypes.RTLD_GLOBAL)
    runtimes = _hip_runtimes_mapped()
    if len(runtimes) > 1:
        raise ImportError(f"two HIP runtimes mapped in one process: {sorted(runtimes)}")
    P, I, D, L = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_longlong
    sig = {
        "tm_create": (I, [ctypes.POINTER(P), I, P]),
        "tm_destroy": (None, [P]),
        "tm_status_string": (ctypes.c_char_p, [I]),
        "tm_last_error": (ctypes.c_char_p, [P]),
        "tm_coeff_count": (I, [I]),
        "tm_abi_version": (I, []),
        "tm_set_geometry": (I, [P, I, P, D, I]),
        "tm_get_lattice": (I, [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(D)]),
        "tm_set_spheres": (I, [P, P, D, D]),
        "tm_set_tmatrix_diag": (I, [P, P]),
        "tm_set_tmatrix_dense": (I, [P, P]),
        "tm_get_tmatrix_diag": (I, [P, P, P]),
        "tm_plane_wave_rhs": (I, [P, I, P, P, P]),
        "tm_default_opts": (None, [ctypes.POINTER(SolveOpts)]),
        "tm_solve": (I, [P, I, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
        "tm_adjoint_solve": (I, [P, I, P, P, ctypes.POINTER(SolveOpts), ctypes.POINTER(SolveInfo)]),
        "tm_apply_operator": (I, [P, I, P, P, I, I]),
        "tm_apply_operator_noalloc": (I, [P, I, P, P, I, I]),
        "tm_grad_position": (I, [P, I, P, P, P, P, P, P, P]),
        "tm_jinc_rhs": (I, [P, I, P, I, P]),
        "tm_set_cylinders": (I, [P, P, D, D, D, I]),
        "tm_ebcm_cylinder": (I, [I, D, D, D, D, D, I, P]),
        "tm_jinc_rhs_batched": (I, [P, I, P, I, I, P, P, I, P]),
        "tm_solve_batched_a0": (I, [P, I, P, I, P, P, P, P, I]),
        "tm_near_field": (I, [P, I, P, I, P, P, I]),
        "tm_near_field_adjoint": (I, [P, I, I, P, P, P]),
        "tm_mie": (I, [I, D, D, D, D, P, P]),
        "tm_far_field": (I, [P, I, P, I, P, P]),
        "tm_detector_vector": (I, [P, P, P, P]),
        "tm_grad_radius": (I, [P, I, P, P, P, P]),
        "tm_solve_batched": (I, [P, I, P, I, P, P, P, ctypes.POINTER(SolveOpts),
                                 ctypes.POINTER(SolveInfo), I]),
        "tm_batch_graph_used": (I, [P]),
        "tm_set_batch_autotune": (I, [P, I]),
        "tm_get_batch_config": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "tm_set_matvec_config": (I, [P, I, I, I]),
        "tm_get_matvec_config": (I, [P, I, ctypes.POINTER(I), ctypes.POINTER(I)]),
        "tm_autotune": (I, [P, I, I, ctypes.POINTER(D)]),
        "tm_set_progress": (I, [P, PROGRESS_FN, P]),
        "tm_profile_enable": (I, [P, I]),
        "tm_profile_query": (I, [P, I, ctypes.POINTER(D), ctypes.POINTER(L), ctypes.POINTER(D)]),
        "tm_profile_reset": (I, [P]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def ebcm_cylinder(lmax, k, radius, height, n_rel, n_quad=0):
    """T [L, L] (host) of one cylinder from tm_ebcm_cylinder."""
    lib = load()
    L = 2 * lmax * (lmax + 2)
    T = np.zeros((L, L), dtype=np.complex128)
    n = complex(n_rel)
    rc = lib.tm_ebcm_cylinder(int(lmax), float(k), float(radius), float(height), n.real, n.imag,
                              int(n_quad), T.ctypes.data_as(ctypes.c_void_p))
    if rc != TM_OK:
        raise TmError(rc, "tm_ebcm_cylinder failed")
    return T


def mie(lmax, k, radius, n_rel):
    """(t [2][lmax], dt/dr [2][lmax]) of one sphere from tm_mie (host arrays;
    p = 0 rows hold -b_l, p = 1 rows -a_l)."""
    lib = load()
    n = complex(n_rel)
    t = np.zeros((2, lmax), dtype=np.complex128)
    d = np.zeros((2, lmax), dtype=np.complex128)
    rc = lib.tm_mie(int(lmax), float(k), float(radius), n.real, n.imag,
                    t.ctypes.data_as(ctypes.c_void_p), d.ctypes.data_as(ctypes.c_void_p))
    if rc != TM_OK:
        raise TmError(rc, lib.tm_status_string(rc).decode())
    return t, d


def _ptr(t):
    return ctypes.c_void_p(t.data_ptr())


def _shape(t, dtype, name, tail=None, lead_max=None):
    """Type, dtype and shape of an array bound for the device.

    tail: the trailing dimensions the library assumes (None entries match any
    size); lead_max: the largest number of leading dimensions allowed (a
    missing leading rhs dimension means one right-hand side)."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if tail is not None:
        tail = tuple(tail)
        shp = tuple(t.shape)
        nlead = len(shp) - len(tail)
        ok = 0 <= nlead <= (lead_max if lead_max is not None else 0)
        ok = ok and all(w is None or w == v for w, v in zip(tail, shp[nlead:]))
        if not ok:
            want = ("[R, " if lead_max else "[") + ", ".join("*" if w is None else str(w) for w in tail) + "]"
            raise ValueError(f"{name} must have shape {want}, got {list(shp)}")
    return t


def _place(t, name, device=None):
    """The array on the context's device, contiguous, conjugation resolved."""
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA/HIP torch tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the context on {device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    # the library reads raw memory: materialise lazy conjugate / negative views
    if t.is_conj():
        t = t.resolve_conj()
    if t.is_neg():
        t = t.resolve_neg()
    return t


def _dev(t, dtype, name, device=None, tail=None, lead_max=None):
    return _place(_shape(t, dtype, name, tail, lead_max), name, device)


def _devs(device, *specs):
    """Several arrays: every shape is checked before any device check, so a
    mis-shaped argument raises ValueError whatever the others hold.
    specs: (tensor, dtype, name, tail, lead_max)."""
    ts = [_shape(t, dt, nm, tl, lm) for t, dt, nm, tl, lm in specs]
    return [_place(t, sp[2], device) for t, sp in zip(ts, specs)]


def _host(a, dtype, name, shape):
    """A contiguous host copy of `a` with the given shape (None = any size)."""
    a = np.ascontiguousarray(a, dtype=dtype)
    if a.ndim != len(shape) or any(w is not None and w != v for w, v in zip(shape, a.shape)):
        want = "[" + ", ".join("*" if w is None else str(w) for w in shape) + "]"
        raise ValueError(f"{name} must have shape {want}, got {list(a.shape)}")
    return a


def _incidence(khat, pol):
    kh = _host(np.atleast_2d(khat), np.float64, "khat", (None, 3))
    po = _host(np.atleast_2d(pol), np.complex128, "pol", (kh.shape[0], 3))
    return kh, po


def _nrhs(t, tail_dims):
    return t.shape[0] if t.dim() > tail_dims else 1


class Context:
    """One tm_ctx on a device, enqueuing on torch's current stream."""

    def __init__(self, device=0, stream=None):
        self.lib = load()
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = ctypes.c_void_p()
        self._check(self.lib.tm_create(ctypes.byref(h), device, ctypes.c_void_p(stream.cuda_stream)))
        self.h = h
        self.n = 0
        self.lmax = 0
        self.L = 0

    def _check(self, rc, allow=(TM_OK,)):
        if rc not in allow:
            msg = ""
            if getattr(self, "h", None):
                msg = self.lib.tm_last_error(self.h).decode()
            raise TmError(rc, f"{self.lib.tm_status_string(rc).decode()}: {msg}")
        return rc

    def close(self):
        if getattr(self, "h", None):
            self.lib.tm_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    # ---- set-up
    def set_geometry(self, positions, k, lmax):
        pos = _host(positions, np.float64, "positions", (None, 3))
        self._check(self.lib.tm_set_geometry(self.h, len(pos), pos.ctypes.data_as(ctypes.c_void_p),
                                             float(k), int(lmax)))
        self.n, self.lmax, self.L = len(pos), int(lmax), self.lib.tm_coeff_count(int(lmax))
        self.k = float(k)

    def get_lattice(self):
        nx, ny, p = ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        self._check(self.lib.tm_get_lattice(self.h, ctypes.byref(nx), ctypes.byref(ny), ctypes.byref(p)))
        return nx.value, ny.value, p.value

    def set_spheres(self, radii, n_rel):
        r = _dev(radii, torch.float64, "radii", self.device, (self.n,))
        n_rel = complex(n_rel)
        self._check(self.lib.tm_set_spheres(self.h, _ptr(r), n_rel.real, n_rel.imag))

    def set_cylinders(self, radii, height, n_rel, n_quad=0):
        """tm_set_cylinders: null-field T-matrices of cylinders (radii device [N])."""
        (radii,) = _devs(self.device, (radii, torch.float64, "radii", (self.n,), None))
        n = complex(n_rel)
        self._check(self.lib.tm_set_cylinders(self.h, _ptr(radii), float(height), n.real, n.imag,
                                              int(n_quad)))

    def set_tmatrix_diag(self, t):
        t = _dev(t, torch.complex128, "t", self.device, (self.n, self.L))
        self._check(self.lib.tm_set_tmatrix_diag(self.h, _ptr(t)))

    def set_tmatrix_dense(self, T):
        """T [N, L, L] complex128 on the device (row-major per scatterer)."""
        T = _dev(T, torch.complex128, "T", self.device, (self.n, self.L, self.L))
        self._check(self.lib.tm_set_tmatrix_dense(self.h, _ptr(T)))

    def get_tmatrix_diag(self):
        t = torch.empty(self.n, self.L, dtype=torch.complex128, device=self.device)
        dt = torch.empty_like(t)
        self._check(self.lib.tm_get_tmatrix_diag(self.h, _ptr(t), _ptr(dt)))
        return t, dt

    def plane_wave_rhs(self, khat, pol):
        kh, po = _incidence(khat, pol)
        R = kh.shape[0]
        a0 = torch.empty(R, self.n, self.L, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_plane_wave_rhs(self.h, R, kh.ctypes.data_as(ctypes.c_void_p),
                                               po.ctypes.data_as(ctypes.c_void_p), _ptr(a0)))
        return a0

    # ---- solve
    @staticmethod
    def make_opts(tol=1e-8, restart=50, max_iter=2000, precision="fp64", inner_tol=1e-4, use_x0=False):
        o = SolveOpts()
        load().tm_default_opts(ctypes.byref(o))
        o.tol, o.restart, o.max_iter = tol, restart, max_iter
        o.precision = PRECISIONS[precision]
        o.inner_tol, o.use_x0 = inner_tol, int(bool(use_x0))
        return o

    def _solve(self, fname, rhs, x0, **kw):
        _shape(rhs, torch.complex128, "rhs", (self.n, self.L), 1)
        if x0 is not None:
            _shape(x0, torch.complex128, "x0", (self.n, self.L), 1)
            if x0.shape != rhs.shape:
                raise ValueError(f"x0 must have the shape of the right-hand side {list(rhs.shape)}")
            x0 = _place(x0, "x0", self.device)
        rhs = _place(rhs, "rhs", self.device)
        R = _nrhs(rhs, 2)
        fn = getattr(self.lib, fname)
        out = x0.clone() if x0 is not None else torch.zeros_like(rhs)
        o = self.make_opts(use_x0=x0 is not None, **kw)
        infos = (SolveInfo * R)()
        self._check(fn(self.h, R, _ptr(rhs), _ptr(out), ctypes.byref(o), infos),
                    allow=(TM_OK, TM_NOT_CONVERGED))
        return out, [i.as_dict() for i in infos]

    def solve(self, a0, x0=None, **kw):
        return self._solve("tm_solve", a0, x0, **kw)

    def adjoint_solve(self, v, x0=None, **kw):
        return self._solve("tm_adjoint_solve", v, x0, **kw)

    def solve_batched(self, subs, khat, pol, use_graph=True, **kw):
        """subs: [(origin_x, origin_y, side_x, side_y)]; returns ([s_k [R, N_k, L]], infos [S][R])."""
        S = len(subs)
        arr = (Subregion * S)(*[Subregion(*map(int, q)) for q in subs])
        kh, po = _incidence(khat, pol)
        R = kh.shape[0]
        sizes = [R * q[2] * q[3] * self.L for q in subs]
        out = torch.empty(sum(sizes), dtype=torch.complex128, device=self.device)
        o = self.make_opts(**kw)
        infos = (SolveInfo * (S * R))()
        self._check(self.lib.tm_solve_batched(self.h, S, arr, R, kh.ctypes.data_as(ctypes.c_void_p),
                                              po.ctypes.data_as(ctypes.c_void_p), _ptr(out),
                                              ctypes.byref(o), infos, int(bool(use_graph))),
                    allow=(TM_OK, TM_NOT_CONVERGED))
        res, off = [], 0
        for q, n in zip(subs, sizes):
            res.append(out[off:off + n].view(R, q[2] * q[3], self.L))
            off += n
        info = [[infos[k * R + r].as_dict() for r in range(R)] for k in range(S)]
        return res, info

    def jinc_rhs(self, sources, n_beta=0):
        """tm_jinc_rhs: [R, N, L] incident coefficients of jinc sources
        [(x0, y0, z0, ax, ay)] (App. II)."""
        R = len(sources)
        if R < 1:
            raise ValueError("need at least one source")
        a0 = torch.empty(R, self.n, self.L, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_jinc_rhs(self.h, R, _jinc_array(sources), int(n_beta), _ptr(a0)))
        return a0

    def jinc_rhs_batched(self, subs, groups, n_beta=0):
        """tm_jinc_rhs_batched: groups[k][r] is the list of jinc sources
        exciting system (subregion k, rhs r); returns the packed coefficients
        (flat, the layout tm_solve_batched_a0 takes)."""
        S = len(subs)
        R = len(groups[0])
        if len(groups) != S or any(len(g) != R for g in groups):
            raise ValueError("groups must be [n_sub][n_rhs] lists of sources")
        flat, off = [], [0]
        for k in range(S):
            for r in range(R):
                flat.extend(groups[k][r])
                off.append(len(flat))
        arr = (Subregion * S)(*[Subregion(*map(int, q)) for q in subs])
        grp = np.ascontiguousarray(off, dtype=np.int32)
        n = sum(R * q[2] * q[3] * self.L for q in subs)
        a0 = torch.empty(n, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_jinc_rhs_batched(self.h, S, arr, R, len(flat), _jinc_array(flat),
                                                 grp.ctypes.data_as(ctypes.c_void_p), int(n_beta),
                                                 _ptr(a0)))
        return a0

    def solve_batched_a0(self, subs, a0, n_rhs, use_graph=True, **kw):
        """tm_solve_batched_a0: a0 flat packed [sum_k R N_k L]; returns
        ([s_k [R, N_k, L]], infos [S][R])."""
        S = len(subs)
        R = int(n_rhs)
        sizes = [R * q[2] * q[3] * self.L for q in subs]
        (a0,) = _devs(self.device, (a0, torch.complex128, "a0", (sum(sizes),), None))
        arr = (Subregion * S)(*[Subregion(*map(int, q)) for q in subs])
        out = torch.empty(sum(sizes), dtype=torch.complex128, device=self.device)
        o = self.make_opts(**kw)
        infos = (SolveInfo * (S * R))()
        self._check(self.lib.tm_solve_batched_a0(self.h, S, arr, R, _ptr(a0), _ptr(out), ctypes.byref(o),
                                                 infos, int(bool(use_graph))),
                    allow=(TM_OK, TM_NOT_CONVERGED))
        res, off = [], 0
        for q, n in zip(subs, sizes):
            res.append(out[off:off + n].view(R, q[2] * q[3], self.L))
            off += n
        info = [[infos[k * R + r].as_dict() for r in range(R)] for k in range(S)]
        return res, info

    def batch_graph_used(self):
        return bool(self.lib.tm_batch_graph_used(self.h))

    def set_batch_autotune(self, on=True):
        self._check(self.lib.tm_set_batch_autotune(self.h, int(bool(on))))

    def batch_config(self, precision):
        """(table prefetch depth, items per (rhs, class)) of the last batched solve."""
        pf, it = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tm_get_batch_config(self.h, PRECISIONS[precision], ctypes.byref(pf),
                                                 ctypes.byref(it)))
        return pf.value, it.value

    def apply_operator(self, x, op="forward", precision="fp64"):
        x = _dev(x, torch.complex128, "x", self.device, (self.n, self.L), 1)
        R = _nrhs(x, 2)
        y = torch.empty_like(x)
        self._check(self.lib.tm_apply_operator(self.h, R, _ptr(x), _ptr(y), PRECISIONS[precision],
                                               OPS[op]))
        return y

    def apply_operator_noalloc(self, x, out, op="forward", precision="fp64"):
        """tm_apply_operator_noalloc: writes into the caller's `out` (same
        shape as x); the library allocates nothing for the call."""
        x = _dev(x, torch.complex128, "x", self.device, (self.n, self.L), 1)
        out = _dev(out, torch.complex128, "out", self.device, (self.n, self.L), 1)
        if out.shape != x.shape:
            raise ValueError(f"out has shape {tuple(out.shape)}, x {tuple(x.shape)}")
        R = _nrhs(x, 2)
        self._check(self.lib.tm_apply_operator_noalloc(self.h, R, _ptr(x), _ptr(out),
                                                       PRECISIONS[precision], OPS[op]))
        return out

    # ---- readout
    def near_field(self, s, pts, precision="fp64"):
        s, pts = _devs(self.device, (s, torch.complex128, "s", (self.n, self.L), 1),
                       (pts, torch.float64, "pts", (None, 3), None))
        R = _nrhs(s, 2)
        E = torch.empty(R, pts.shape[0], 3, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_near_field(self.h, R, _ptr(s), pts.shape[0], _ptr(pts), _ptr(E),
                                           PRECISIONS[precision]))
        return E

    def near_field_adjoint(self, pts, w):
        """v = transpose of the near-field map applied to w [R, P, 3]."""
        _shape(pts, torch.float64, "pts", (None, 3))
        pts, w = _devs(self.device, (pts, torch.float64, "pts", (None, 3), None),
                       (w, torch.complex128, "w", (pts.shape[0], 3), 1))
        R = _nrhs(w, 2)
        v = torch.empty(R, self.n, self.L, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_near_field_adjoint(self.h, R, pts.shape[0], _ptr(pts), _ptr(w), _ptr(v)))
        return v

    def far_field(self, s, dirs):
        s, dirs = _devs(self.device, (s, torch.complex128, "s", (self.n, self.L), 1),
                        (dirs, torch.float64, "dirs", (None, 3), None))
        R = _nrhs(s, 2)
        F = torch.empty(R, dirs.shape[0], 3, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_far_field(self.h, R, _ptr(s), dirs.shape[0], _ptr(dirs), _ptr(F)))
        return F

    # ---- sensitivities
    def detector_vector(self, xd, w):
        xd = _host(xd, np.float64, "xd", (3,))
        w = _host(w, np.complex128, "w", (3,))
        v = torch.empty(self.n, self.L, dtype=torch.complex128, device=self.device)
        self._check(self.lib.tm_detector_vector(self.h, xd.ctypes.data_as(ctypes.c_void_p),
                                                w.ctypes.data_as(ctypes.c_void_p), _ptr(v)))
        return v

    def grad_radius(self, mu, s, a0):
        spec = [(t, torch.complex128, nm, (self.n, self.L), 1) for t, nm in ((mu, "mu"), (s, "s"), (a0, "a0"))]
        for t, *rest in spec:
            _shape(t, *rest)
        R = _nrhs(mu, 2)
        if _nrhs(s, 2) != R or _nrhs(a0, 2) != R:
            raise ValueError("mu, s and a0 must hold the same number of right-hand sides")
        mu, s, a0 = _devs(self.device, *spec)
        g = torch.empty(R, self.n, dtype=torch.float64, device=self.device)
        self._check(self.lib.tm_grad_radius(self.h, R, _ptr(mu), _ptr(s), _ptr(a0), _ptr(g)))
        return g

    # ---- matvec configuration / autotuner
    def grad_position(self, mu, s, a0=None, khat=None, xd=None, w=None):
        """tm_grad_position: [R, N, 2] in-plane position gradient.  khat (host
        [R, 3]) adds the plane-wave incident term (a0 required); xd (host [3])
        with w (host [R, 3]) adds the point-detector term."""
        mu, s = _devs(self.device, (mu, torch.complex128, "mu", (self.n, self.L), 1),
                      (s, torch.complex128, "s", (self.n, self.L), 1))
        R = _nrhs(mu, 2)
        if _nrhs(s, 2) != R:
            raise ValueError("mu and s must have the same number of right-hand sides")
        kh = a0p = None
        if khat is not None:
            if a0 is None:
                raise ValueError("khat needs a0")
            (a0,) = _devs(self.device, (a0, torch.complex128, "a0", (self.n, self.L), 1))
            if _nrhs(a0, 2) != R:
                raise ValueError("a0 must have the same number of right-hand sides as mu")
            kh = _host(np.atleast_2d(khat), np.float64, "khat", (R, 3))
            a0p = _ptr(a0)
        xdp = wp = None
        if (xd is None) != (w is None):
            raise ValueError("xd and w go together")
        if xd is not None:
            xdh = _host(xd, np.float64, "xd", (3,))
            wh = _host(np.atleast_2d(w), np.complex128, "w", (R, 3))
            xdp, wp = xdh.ctypes.data_as(ctypes.c_void_p), wh.ctypes.data_as(ctypes.c_void_p)
        g = torch.empty(R, self.n, 2, dtype=torch.float64, device=self.device)
        self._check(self.lib.tm_grad_position(
            self.h, R, _ptr(mu), _ptr(s), a0p, None if kh is None else kh.ctypes.data_as(ctypes.c_void_p),
            xdp, wp, _ptr(g)))
        return g

    def set_matvec_config(self, precision, variant, items=0):
        self._check(self.lib.tm_set_matvec_config(self.h, PRECISIONS[precision], int(variant), int(items)))

    def get_matvec_config(self, precision):
        v, i = ctypes.c_int(), ctypes.c_int()
        self._check(self.lib.tm_get_matvec_config(self.h, PRECISIONS[precision], ctypes.byref(v),
                                                  ctypes.byref(i)))
        return v.value, i.value

    def autotune(self, n_rhs=1, precision="mixed"):
        ms = ctypes.c_double()
        self._check(self.lib.tm_autotune(self.h, int(n_rhs), PRECISIONS[precision], ctypes.byref(ms)))
        return ms.value, self.get_matvec_config(precision)

    # ---- progress
    def set_progress(self, fn):
        """fn(cycles, iters, n_live, max_rel_residual) after every restart
        cycle of the solvers, or None to remove it."""
        if fn is None:
            self._progress = None
            self._check(self.lib.tm_set_progress(self.h, PROGRESS_FN(), None))
            return
        self._progress = PROGRESS_FN(lambda _u, c, i, n, r: fn(c, i, n, r))
        self._check(self.lib.tm_set_progress(self.h, self._progress, None))

    # ---- profiling
    def profile_enable(self, on=True):
        self._check(self.lib.tm_profile_enable(self.h, int(bool(on))))

    def profile_reset(self):
        self._check(self.lib.tm_profile_reset(self.h))

    def profile_query(self, which):
        ms, n, fl = ctypes.c_double(), ctypes.c_longlong(), ctypes.c_double()
        self._check(self.lib.tm_profile_query(self.h, int(which), ctypes.byref(ms), ctypes.byref(n),
                                              ctypes.byref(fl)))
        return ms.value, n.value, fl.value
