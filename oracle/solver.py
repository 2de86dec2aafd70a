"""Multiple-scattering system, solve, readout and adjoint (oracle, FP64).

Test infrastructure only.

System (App. I.C, eq. "final_linear_eqs" with the block-diagonal
preconditioner M = diag(T_i)): the exciting field of scatterer j is
  a_j = a0_j + sum_{i != j} xi(k(x_j - x_i))^T s_i,     s_j = T_j a_j,
so with A_ji = xi(k(x_j - x_i))^T (reading: the off-diagonal blocks of the
Maxwell operator are -xi^T, as in the per-scatterer equation that precedes the
matrix display) the preconditioned system is
  B s = b,   B = I - T A,   b = T a0.
The oracle assembles B densely and solves it with LAPACK (numpy.linalg.solve,
partial-pivoting LU); for sizes where B does not fit in memory it applies A
block by block with its own restarted GMRES.

Readout (eq. "sca_fld_concise"): E_sca(x) = sum_i s_i^T Phi(k(x - x_i)); the far
field F(d) = lim_r r e^{-ikr} E_sca(r d) = (1/k) sum_i e^{-ik d.x_i} s_i^T F(d).

Adjoint (App. IV): for O = f(z) with z linear in s, dO/dp_i = 2 Re[f'(z) dz/dp_i],
dz/dp_i = -v^T Omega^{-1} (dOmega/dp_i) s.  In preconditioned form
B ds = dT_i a_exc with a_exc = a0 + A s, so with B^T mu = w (w = f'(z)-weighted
detector vector) dO/dr_i = 2 Re[mu_i^T (dt_i * a_exc_i)].  This equals the
paper's expression with its adjoint unknown = T mu.
"""
import numpy as np

from .translation import Translation
from .vswf import n_coeffs, vswf, vswf_farfield


# ----------------------------------------------------------------------------
# dense assembly
# ----------------------------------------------------------------------------
def coupling_dense(positions, k, lmax):
    """A with A[j, :, i, :] = xi(k(x_j - x_i))^T, shape [N*L, N*L]."""
    pos = np.asarray(positions, dtype=float)
    N = len(pos)
    L = n_coeffs(lmax)
    tr = Translation(k, lmax)
    jj, ii = np.nonzero(~np.eye(N, dtype=bool))
    A = np.zeros((N, L, N, L), dtype=complex)
    chunk = 4096
    for c0 in range(0, len(jj), chunk):
        j = jj[c0:c0 + chunk]
        i = ii[c0:c0 + chunk]
        X = tr.blocks(pos[j] - pos[i])  # [P, u, v]
        A[j, :, i, :] = np.transpose(X, (0, 2, 1))
    return A.reshape(N * L, N * L)


def tmatrix_dense(t):
    """Block-diagonal T from a [N, L] diagonal or [N, L, L] dense array."""
    t = np.asarray(t)
    N, L = t.shape[0], t.shape[1]
    T = np.zeros((N * L, N * L), dtype=complex)
    for i in range(N):
        T[i * L:(i + 1) * L, i * L:(i + 1) * L] = np.diag(t[i]) if t.ndim == 2 else t[i]
    return T


def system_dense(positions, k, lmax, t):
    A = coupling_dense(positions, k, lmax)
    T = tmatrix_dense(t)
    return np.eye(A.shape[0]) - T @ A, A, T


def solve_dense(positions, k, lmax, t, a0):
    """Scattered coefficients s [R, N, L] for incident coefficients a0 [R, N, L]."""
    a0 = np.asarray(a0, dtype=complex)
    single = a0.ndim == 2
    if single:
        a0 = a0[None]
    R, N, L = a0.shape
    B, A, T = system_dense(positions, k, lmax, t)
    rhs = T @ a0.reshape(R, N * L).T
    s = np.linalg.solve(B, rhs).T.reshape(R, N, L)
    return s[0] if single else s


# ----------------------------------------------------------------------------
# matrix-free coupling for large lattices (blocks from the per-pair routine,
# cached per displacement only to save time)
# ----------------------------------------------------------------------------
class LatticeCoupling:
    """A applied block by block for sites x_(ix,iy) = origin + pitch*(ix, iy, 0)."""

    def __init__(self, nx, ny, pitch, k, lmax):
        self.nx, self.ny, self.pitch, self.k, self.lmax = nx, ny, pitch, k, lmax
        self.L = n_coeffs(lmax)
        tr = Translation(k, lmax)
        dx, dy = np.meshgrid(np.arange(-(nx - 1), nx), np.arange(-(ny - 1), ny))
        dx, dy = dx.ravel(), dy.ravel()
        keep = (dx != 0) | (dy != 0)
        self.dxy = np.stack([dx[keep], dy[keep]], 1)
        d = np.zeros((len(self.dxy), 3))
        d[:, 0] = pitch * self.dxy[:, 0]
        d[:, 1] = pitch * self.dxy[:, 1]
        self.blk = np.empty((len(d), self.L, self.L), dtype=complex)
        for c0 in range(0, len(d), 2048):
            self.blk[c0:c0 + 2048] = tr.blocks(d[c0:c0 + 2048])

    def apply(self, x, transpose=False):
        """(A x) for x [N, L] (site index iy*nx+ix); A^T x when transpose.

        A_ts = xi(x_t - x_s)^T, so (A x)_t = sum_s x_s @ xi(x_t - x_s) in
        row-vector form; (A^T)_ts = A_st^T = xi(x_s - x_t), so
        (A^T x)_t = sum_s x_s @ xi(x_s - x_t)^T.
        """
        nx, ny, L = self.nx, self.ny, self.L
        X = np.asarray(x, dtype=complex).reshape(ny, nx, L)
        Y = np.zeros_like(X)
        for (ddx, ddy), blk in zip(self.dxy, self.blk):
            if not transpose:
                # displacement = x_t - x_s, i.e. s = t - (ddx, ddy)
                tx0, tx1 = max(0, ddx), min(nx, nx + ddx)
                ty0, ty1 = max(0, ddy), min(ny, ny + ddy)
                Y[ty0:ty1, tx0:tx1] += X[ty0 - ddy:ty1 - ddy, tx0 - ddx:tx1 - ddx] @ blk
            else:
                # displacement = x_s - x_t, i.e. s = t + (ddx, ddy)
                tx0, tx1 = max(0, -ddx), min(nx, nx - ddx)
                ty0, ty1 = max(0, -ddy), min(ny, ny - ddy)
                Y[ty0:ty1, tx0:tx1] += X[ty0 + ddy:ty1 + ddy, tx0 + ddx:tx1 + ddx] @ blk.T
        return Y.reshape(nx * ny, L)


def rows_A(positions, k, lmax, x, rows, transpose=False):
    """Selected rows of A x (or A^T x) for arbitrary positions, one by one."""
    pos = np.asarray(positions, dtype=float)
    x = np.asarray(x, dtype=complex)
    tr = Translation(k, lmax)
    out = []
    for j in rows:
        others = np.array([i for i in range(len(pos)) if i != j])
        acc = np.zeros(x.shape[1], dtype=complex)
        for c0 in range(0, len(others), 4096):
            i = others[c0:c0 + 4096]
            if not transpose:
                X = tr.blocks(pos[j] - pos[i])  # xi(x_j - x_i): [P, u, v]
                acc += np.einsum('puv,pu->v', X, x[i])
            else:
                X = tr.blocks(pos[i] - pos[j])  # (A^T)_{ji} = A_{ij}^T = xi(x_i - x_j)
                acc += np.einsum('puv,pv->u', X, x[i])
        out.append(acc)
    return np.array(out)


# ----------------------------------------------------------------------------
# restarted GMRES (own code; modified Gram-Schmidt, Givens rotations)
# ----------------------------------------------------------------------------
def gmres(matvec, b, tol=1e-12, restart=50, maxiter=5000, x0=None):
    """Solve M x = b to relative (true) residual tol; returns (x, iters, relres)."""
    b = np.asarray(b, dtype=complex).ravel()
    nb = np.linalg.norm(b)
    x = np.zeros_like(b) if x0 is None else np.asarray(x0, dtype=complex).ravel().copy()
    if nb == 0.0:
        return x, 0, 0.0
    it = 0
    r = b - matvec(x) if x0 is not None else b.copy()
    while True:
        beta = np.linalg.norm(r)
        if beta / nb <= tol or it >= maxiter:
            return x, it, beta / nb
        V = np.zeros((restart + 1, len(b)), dtype=complex)
        H = np.zeros((restart + 1, restart), dtype=complex)
        cs = np.zeros(restart, dtype=complex)
        sn = np.zeros(restart, dtype=complex)
        g = np.zeros(restart + 1, dtype=complex)
        g[0] = beta
        V[0] = r / beta
        j_end = 0
        for j in range(restart):
            w = matvec(V[j])
            for i in range(j + 1):
                H[i, j] = np.vdot(V[i], w)
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] != 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                tmp = cs[i].conjugate() * H[i, j] + sn[i].conjugate() * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = tmp
            den = np.hypot(abs(H[j, j]), abs(H[j + 1, j]))
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j].conjugate() * g[j]
            it += 1
            j_end = j + 1
            if abs(g[j + 1]) / nb <= tol or it >= maxiter:
                break
        y = np.linalg.solve(np.triu(H[:j_end, :j_end]), g[:j_end])
        x = x + V[:j_end].T @ y
        r = b - matvec(x)


# ----------------------------------------------------------------------------
# readout
# ----------------------------------------------------------------------------
def near_field(s, positions, k, lmax, pts):
    """E_sca at points pts [P, 3] for coefficients s [N, L] -> [P, 3]."""
    pos = np.asarray(positions, dtype=float)
    pts = np.asarray(pts, dtype=float)
    E = np.zeros((len(pts), 3), dtype=complex)
    for c0 in range(0, len(pos), 256):
        d = pts[:, None, :] - pos[None, c0:c0 + 256, :]
        Phi = vswf(lmax, k, d, regular=False)  # [P, n, L, 3]
        E += np.einsum('nl,pnlc->pc', s[c0:c0 + 256], Phi)
    return E


def far_field(s, positions, k, lmax, dirs):
    """F(d) = lim r e^{-ikr} E_sca(r d) for unit directions dirs [D, 3] -> [D, 3]."""
    pos = np.asarray(positions, dtype=float)
    dirs = np.asarray(dirs, dtype=float)
    Fn = vswf_farfield(lmax, dirs)  # [D, L, 3]
    ph = np.exp(-1j * k * dirs @ pos.T)  # [D, N]
    c = ph @ np.asarray(s, dtype=complex)  # [D, L]
    return np.einsum('dl,dlc->dc', c, Fn) / k


def extinction(s, positions, k, lmax, khat, pol):
    """C_ext = (4 pi / k) Im[pol^* . F(khat)] for unit-amplitude incidence."""
    F = far_field(s, positions, k, lmax, np.asarray(khat, dtype=float)[None])[0]
    return 4.0 * np.pi / k * np.imag(np.vdot(pol, F))


def scattering(s, positions, k, lmax, n_theta=96, n_phi=192):
    """C_sca = closed-surface integral of |F|^2 (Gauss-Legendre x trapezoid)."""
    xg, wg = np.polynomial.legendre.leggauss(n_theta)
    phis = np.arange(n_phi) * 2.0 * np.pi / n_phi
    th = np.arccos(xg)
    T, P = np.meshgrid(th, phis, indexing='ij')
    dirs = np.stack([np.sin(T) * np.cos(P), np.sin(T) * np.sin(P), np.cos(T)], -1).reshape(-1, 3)
    F = far_field(s, positions, k, lmax, dirs)
    w = (wg[:, None] * np.full(n_phi, 2.0 * np.pi / n_phi)[None, :]).ravel()
    return float(np.sum(w * np.sum(np.abs(F) ** 2, axis=1)))


# ----------------------------------------------------------------------------
# adjoint (App. IV) for a point detector and O = sum_c |E_inc,c + E_sca,c|^2
# ----------------------------------------------------------------------------
def detector_vectors(positions, k, lmax, xd):
    """v[c, i, n] = Phi_n(k(xd - x_i))_c, so E_sca,c(xd) = sum v[c] * s."""
    pos = np.asarray(positions, dtype=float)
    Phi = vswf(lmax, k, np.asarray(xd, dtype=float)[None, :] - pos, regular=False)  # [N, L, 3]
    return np.transpose(Phi, (2, 0, 1))


def objective_and_gradient_dense(positions, k, lmax, radii, mrel, khat, pol, xd):
    """O and dO/dr_i for the total field intensity at xd (dense LU throughout)."""
    from .mie import mie_tmatrix_diag_many
    from .vswf import plane_wave_coeffs

    pos = np.asarray(positions, dtype=float)
    N = len(pos)
    L = n_coeffs(lmax)
    t, dt = mie_tmatrix_diag_many(lmax, k, radii, mrel)
    a0 = plane_wave_coeffs(lmax, k, khat, pol, pos)
    B, A, T = system_dense(pos, k, lmax, t)
    s = np.linalg.solve(B, (t * a0).ravel())
    v = detector_vectors(pos, k, lmax, xd).reshape(3, N * L)
    Einc = np.asarray(pol, dtype=complex) * np.exp(1j * k * np.dot(khat, xd))
    Etot = Einc + v @ s
    O = float(np.sum(np.abs(Etot) ** 2))
    w = np.conj(Etot) @ v  # f'(z) weights folded in: dO = 2 Re[w^T ds]
    mu = np.linalg.solve(B.T, w)
    a_exc = a0.ravel() + A @ s
    g = 2.0 * np.real((mu * dt.ravel() * a_exc).reshape(N, L).sum(1))
    return O, g, s.reshape(N, L), mu.reshape(N, L)
