"""The T-matrix solve and its field readout as differentiable torch functions.

TMatrixSolve maps radii to scattered-field coefficients s: the forward pass
builds the Mie T-matrices and the incident coefficients and solves the
multiple-scattering system (I - T A) s = T a_inc with the library's GMRES;
the backward pass is the adjoint method of App. IV.  For a real loss L whose
gradient with respect to s arrives as G = dL/dRe(s) + i dL/dIm(s) (torch's
convention for complex tensors), one solve with the transposed operator,
(I - A^T T) mu = conj(G), gives

    dL/dr_i = Re sum_{n in sphere i} mu_n (dt_n/dr_i) (a_inc + A s)_n,

at the cost of one forward solve whatever the number of radii.  The
library's radius-gradient kernel returns twice this real part (the factor an
intensity objective carries), so the backward halves it.

NearField maps s to the scattered field at points (eq. "sca_fld_concise");
it is linear in s, E = V s, so its backward is grad_s = V^H grad_E, computed
as conj(V^T conj(grad_E)) by the library's transposed near-field kernel.

Every step (Mie, right-hand side, forward and adjoint solves, readout, its
transpose, the gradient contraction) runs in the library's HIP kernels; this
module moves tensors between torch's autograd and the C entry points.
"""
import torch

from . import tmhip


def _check(info, what):
    bad = [d for d in info if d["status"] != tmhip.TM_OK]
    if bad:
        raise RuntimeError(f"{what} did not converge: {bad[0]}")


class TMatrixSolve(torch.autograd.Function):
    """s(radii) for a fixed lattice, incidence and relative refractive index.

    forward(radii [N] float64 on the context's GPU, ctx, n_rel, khat [R][3],
    pol [R][3], opts dict) -> s [R, N, L] complex128.  `opts` takes the
    keywords of Context.make_opts (tol, restart, max_iter, precision,
    inner_tol); the adjoint solve uses the same options.  Raises if a solve
    does not reach its tolerance.
    """

    @staticmethod
    def forward(fctx, radii, ctx, n_rel, khat, pol, opts):
        radii = radii.detach().contiguous()
        ctx.set_spheres(radii, n_rel)
        a0 = ctx.plane_wave_rhs(khat, pol)
        s, info = ctx.solve(a0, **opts)
        _check(info, "forward solve")
        fctx.ctx, fctx.n_rel, fctx.opts = ctx, n_rel, dict(opts)
        fctx.save_for_backward(radii, s, a0)
        return s

    @staticmethod
    def backward(fctx, grad_s):
        radii, s, a0 = fctx.saved_tensors
        ctx = fctx.ctx
        # T and dT/dr of the saved radii: the context may have been given
        # other spheres since the forward pass
        ctx.set_spheres(radii, fctx.n_rel)
        # conj_physical: a lazily conjugated view would hand the library
        # the unconjugated memory
        w = grad_s.to(torch.complex128).conj_physical().contiguous()
        mu, info = ctx.adjoint_solve(w, **fctx.opts)
        _check(info, "adjoint solve")
        g = 0.5 * ctx.grad_radius(mu, s, a0).sum(0)
        return g, None, None, None, None, None


class NearField(torch.autograd.Function):
    """E_sca [R, P, 3] at pts [P][3] (float64, device) from s [R, N, L]."""

    @staticmethod
    def forward(fctx, s, ctx, pts, precision):
        fctx.ctx, fctx.pts = ctx, pts
        return ctx.near_field(s.detach().contiguous(), pts, precision)

    @staticmethod
    def backward(fctx, grad_e):
        w = grad_e.to(torch.complex128).conj_physical().contiguous()
        return fctx.ctx.near_field_adjoint(fctx.pts, w).conj_physical(), None, None, None


def scattered_coefficients(ctx, radii, n_rel, khat, pol, **opts):
    """Differentiable s(radii); see TMatrixSolve."""
    return TMatrixSolve.apply(radii, ctx, n_rel, khat, pol, opts)


def near_field(ctx, s, pts, precision="fp64"):
    """Differentiable E_sca(pts) from s; see NearField."""
    return NearField.apply(s, ctx, pts, precision)


def tmatrix_solve(ctx, radii, n_rel, khat, pol, pts=None, precision="fp64", **opts):
    """radii -> s, or radii -> E_sca at pts when pts is given, differentiable
    with respect to the radii through the adjoint solve."""
    s = scattered_coefficients(ctx, radii, n_rel, khat, pol, precision=precision, **opts)
    return s if pts is None else near_field(ctx, s, pts, precision)
