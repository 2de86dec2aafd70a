"""Seeded synthetic inputs for the T-matrix workloads.

This module is shared by the oracle's tests and the HIP path's tests, smoke
check and benchmark.  It only builds inputs (positions, radii, incidence
directions and polarisations, subregion boxes, detector and field points) and
holds none of the method's arithmetic.

Common settings: wavelength 1 in the (vacuum) host, k = 2 pi, dielectric
spheres of relative index 2.0, square lattice in the z = 0 plane with pitch
0.6 wavelengths; site (ix, iy) sits at (ix*pitch, iy*pitch, 0) and has index
iy*nx + ix.  Radii come from numpy.random.default_rng(seed) in index order.

The paper's scatterers are silicon cylinders taken from external libraries
(App. III); those libraries are not available, so these spheres stand in for
them, with lattice sizes matching the paper's per-GPU subregion scale.  The
"cyl6" workload puts silicon cylinders of the paper's dimensions on its
lattice instead (T-matrices from the null-field method, lmax 6).
"""
import numpy as np

WAVELENGTH = 1.0
K = 2.0 * np.pi / WAVELENGTH
PITCH = 0.6
N_REL = 2.0


# the paper's meta-atoms in wavelength units: silicon cylinders (n = 3.48) of
# height 940 nm on a 1070 nm square lattice at 1550 nm
CYL_N_REL = 3.48
CYL_HEIGHT = 0.94 / 1.55
CYL_PITCH = 1.07 / 1.55


def lattice_positions(nx, ny=None, pitch=PITCH):
    ny = nx if ny is None else ny
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny))
    pos = np.zeros((nx * ny, 3))
    pos[:, 0] = ix.ravel() * pitch
    pos[:, 1] = iy.ravel() * pitch
    return pos


def uniform_radii(n, lo, hi, seed):
    return np.random.default_rng(seed).uniform(lo, hi, n)


def lens_radii(nx, ny=None, pitch=PITCH, focal=100.0, lo=0.12, hi=0.28):
    """Radii mapped linearly from a hyperbolic focusing phase (wrapped to [0, 2 pi))."""
    ny = nx if ny is None else ny
    pos = lattice_positions(nx, ny, pitch)
    c = np.array([(nx - 1) / 2.0 * pitch, (ny - 1) / 2.0 * pitch])
    rho = np.hypot(pos[:, 0] - c[0], pos[:, 1] - c[1])
    phase = K * (focal - np.sqrt(rho * rho + focal * focal))
    wrapped = np.mod(phase, 2.0 * np.pi)
    return lo + (hi - lo) * wrapped / (2.0 * np.pi)


def incidence(name):
    """(khat, polarisation) for the named plane-wave right-hand side."""
    a = np.deg2rad(10.0)
    table = {
        "x": ([0.0, 0.0, 1.0], [1.0, 0.0, 0.0]),
        "y": ([0.0, 0.0, 1.0], [0.0, 1.0, 0.0]),
        # 10 degrees in the x-z plane: p (in-plane) and s (y) polarisation
        "p10": ([np.sin(a), 0.0, np.cos(a)], [np.cos(a), 0.0, -np.sin(a)]),
        "s10": ([np.sin(a), 0.0, np.cos(a)], [0.0, 1.0, 0.0]),
    }
    kh, po = table[name]
    return np.array(kh, dtype=float), np.array(po, dtype=complex)


def incidences(names):
    kh, po = zip(*(incidence(n) for n in names))
    return np.array(kh), np.array(po)


def subregions(seed=3, count=48, full=300, lo=20, hi=80, buffer=10):
    """Overlapping square boxes (origin_x, origin_y, side) inside a full x full
    layout; side = core + 2 * buffer with core uniform in [lo, hi]."""
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        s = int(rng.integers(lo, hi + 1)) + 2 * buffer
        ox, oy = (int(v) for v in rng.integers(0, full - s + 1, 2))
        out.append((ox, oy, s))
    return out


def near_field_plane(n_side, extent, z):
    """n_side x n_side points on [0, extent]^2 at height z, row-major in y."""
    g = np.linspace(0.0, extent, n_side)
    X, Y = np.meshgrid(g, g)
    return np.stack([X.ravel(), Y.ravel(), np.full(X.size, z)], 1)


CONFIGS = {
    "c1": dict(name="8x8 lattice, lmax 2 (1024 unknowns)", nx=8, lmax=2, seed=1,
               radii=(0.15, 0.25), rhs=["x"]),
    "c2": dict(name="100x100 lattice, lmax 3 (3e5 unknowns)", nx=100, lmax=3, seed=2,
               radii=(0.15, 0.25), rhs=["x"], tol=1e-8, restart=50),
    "c3": dict(name="48 subregions of a 300x300 lens layout, lmax 3, 4 RHS", nx=300, lmax=3,
               seed=3, lens=True, rhs=["x", "y", "p10", "s10"], tol=1e-8, restart=50),
    "c4": dict(name="150x150 lattice adjoint, lmax 3", nx=150, lmax=3, seed=4,
               radii=(0.12, 0.28), rhs=["x"], detector=(74.5 * PITCH, 74.5 * PITCH, 50.0)),
    "c5": dict(name="300x300 lens tile, lmax 3, 2 RHS", nx=300, lmax=3, lens=True,
               rhs=["x", "y"], tol=1e-8, restart=50, plane=(1000, 299 * PITCH, 5.0)),
    "offl": dict(name="100x100 jittered lattice (off-lattice blocks), lmax 3 (3e5 unknowns)", nx=100,
                 lmax=3, seed=2, radii=(0.15, 0.25), rhs=["x"], tol=1e-8, restart=50,
                 jitter=(0.035, 8)),
    "cyl6": dict(name="100x100 silicon-cylinder lattice, lmax 6 (9.6e5 unknowns)", nx=100, lmax=6,
                 seed=6, radii=(0.05, 0.16), pitch=CYL_PITCH, cylinders=(CYL_HEIGHT, CYL_N_REL),
                 rhs=["x"], tol=1e-8, restart=200),
}


def config_inputs(key):
    """(positions [N,3], radii [N], khat [R,3], pol [R,3], cfg) for a config."""
    cfg = CONFIGS[key]
    n = cfg["nx"]
    pos = lattice_positions(n, n, cfg.get("pitch", PITCH))
    if cfg.get("jitter"):
        # every site moved in-plane by up to amp in x and in y (seeded), so that no
        # two sites share a displacement and the per-displacement table does not apply
        amp, jseed = cfg["jitter"]
        pos[:, :2] += np.random.default_rng(jseed).uniform(-amp, amp, (n * n, 2))
    if cfg.get("lens"):
        radii = lens_radii(n, n)
    else:
        radii = uniform_radii(n * n, cfg["radii"][0], cfg["radii"][1], cfg["seed"])
    kh, po = incidences(cfg["rhs"])
    return pos, radii, kh, po, cfg
