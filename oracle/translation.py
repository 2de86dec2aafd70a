"""Translation coefficients of the vector addition theorem (oracle, FP64).

Test infrastructure only.

App. I.C ("Simulating collective scattering") gives the addition theorem
  Phi_u(k(x - x_s)) = sum_v xi_uv(k d) R Phi_v(k(x - x_t)),  |x - x_t| < |d|,
with xi = delta_pp' alpha + (1 - delta_pp') beta and, eq. "tran_coeff",
  alpha_{lm;l'm'}(d) = e^{i(m-m')phi_d} sum_q a5(l,m|l',m'|q) h_q(k|d|) Pbar_q^|m-m'|(cos theta_d)
  beta_{lm;l'm'}(d)  = e^{i(m-m')phi_d} sum_q b5(l,m|l',m'|q) h_q(k|d|) Pbar_q^|m-m'|(cos theta_d)
  a5 = i^{|m-m'|-|m|-|m'|+l'-l+q} (-1)^{m-m'} [l(l+1)+l'(l'+1)-q(q+1)] sqrt(2q+1)
       * sqrt((2l+1)(2l'+1) / (2 l(l+1) l'(l'+1))) * 3j(l l' q; m -m' m'-m) 3j(l l' q; 0 0 0)
  b5 = (same phase) sqrt((l+l'+1+q)(l+l'+1-q)(q+l-l')(q-l+l')(2q+1))
       * (same root) * 3j(l l' q; m -m' m'-m) 3j(l l' q-1; 0 0 0)
Readings (each fixed by the pointwise addition-theorem pin in the tests):
  * the regular functions R Phi appear on the right-hand side (the display
    prints Phi on both sides);
  * (l, m, p) indexes the outgoing (source) wave, (l', m', p') the regular one;
  * d = x_t - x_s, the expansion centre minus the source centre -- the sign
    that the coupled equations of App. I.C use, xi(k_b(x_j - x_i)) for the
    wave of scatterer i re-expanded about scatterer j;
  * the summation index printed as p is the Legendre/Hankel order q;
  * b5's second 3j has lower row (l l' q-1) (the print repeats alpha's);
  * the normalisation root carries l'(l'+1) (the print shows l'+1).
"""
import numpy as np

from .special import pbar, sph_h1, wigner3j
from .vswf import index_list


def ab5(l, m, lp, mp, q):
    """(a5, b5) of eq. "tran_coeff" under the readings above."""
    phase = (1j) ** (abs(m - mp) - abs(m) - abs(mp) + lp - l + q) * (-1) ** (m - mp)
    root = np.sqrt((2 * l + 1) * (2 * lp + 1) / (2.0 * l * (l + 1) * lp * (lp + 1)))
    w1 = wigner3j(l, lp, q, m, -mp, mp - m)
    wa = wigner3j(l, lp, q, 0, 0, 0)
    wb = wigner3j(l, lp, q - 1, 0, 0, 0) if q >= 1 else 0.0
    fa = (l * (l + 1) + lp * (lp + 1) - q * (q + 1)) * np.sqrt(2 * q + 1)
    arg = (l + lp + 1 + q) * (l + lp + 1 - q) * (q + l - lp) * (q - l + lp) * (2 * q + 1)
    fb = np.sqrt(arg) if arg > 0 else 0.0
    return phase * root * fa * w1 * wa, phase * root * fb * w1 * wb


class Translation:
    """xi(k d) blocks for source truncation lmax_s and target truncation lmax_t."""

    def __init__(self, k, lmax_s, lmax_t=None):
        self.k = float(k)
        self.lmax_s = lmax_s
        self.lmax_t = lmax_s if lmax_t is None else lmax_t
        S = index_list(self.lmax_s)
        T = index_list(self.lmax_t)
        self.qmax = self.lmax_s + self.lmax_t
        # coef[u, v, q] and |m_u - m_v|, m_u - m_v
        self.coef = np.zeros((len(S), len(T), self.qmax + 1), dtype=complex)
        self.dm = np.zeros((len(S), len(T)), dtype=int)
        for a, (p, l, m) in enumerate(S):
            for b, (pp, lp, mp) in enumerate(T):
                self.dm[a, b] = m - mp
                for q in range(abs(l - lp), l + lp + 1):
                    A5, B5 = ab5(l, m, lp, mp, q)
                    self.coef[a, b, q] = A5 if p == pp else B5

    def blocks(self, d):
        """xi(k d) for displacement vectors d [P, 3] -> [P, Ls, Lt]."""
        d = np.atleast_2d(np.asarray(d, dtype=float))
        r = np.linalg.norm(d, axis=1)
        ct = np.clip(d[:, 2] / r, -1.0, 1.0)
        phi = np.arctan2(d[:, 1], d[:, 0])
        h = np.stack([sph_h1(q, self.k * r) for q in range(self.qmax + 1)], 1)  # [P, Q]
        mu_max = self.qmax
        Pq = np.zeros((len(r), self.qmax + 1, mu_max + 1))
        for q in range(self.qmax + 1):
            for mu in range(q + 1):
                Pq[:, q, mu] = pbar(q, mu, ct)
        adm = np.abs(self.dm)
        # radial-angular factor: sum_q coef[u,v,q] h_q Pbar_q^{|dm|}
        hp = h[:, :, None] * Pq  # [P, Q, MU]
        hp_uv = hp[:, :, adm]  # [P, Q, Ls, Lt]
        s = np.einsum('uvq,pquv->puv', self.coef, hp_uv)
        return s * np.exp(1j * self.dm[None, :, :] * phi[:, None, None])

    def block(self, d):
        return self.blocks(np.asarray(d, dtype=float)[None, :])[0]
