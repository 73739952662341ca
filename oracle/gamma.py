"""Second-order SCC-DFTB charge kernel gamma_AB(R) (oracle).

Elstner et al., Phys. Rev. B 58, 7260 (1998): the Coulomb interaction of two
exponential charge densities with decay tau = 16 U / 5,
  gamma_AB(R) = 1/R - S(tau_A, tau_B, R)
  equal tau:   S = e^{-tau R} (1/R + 11 tau/16 + 3 tau^2 R/16 + tau^3 R^2/48)
  unequal tau: S = e^{-ta R} K(ta, tb, R) + e^{-tb R} K(tb, ta, R),
               K(a, b, R) = b^4 a / (2 (a^2-b^2)^2) - (b^6 - 3 a^2 b^4) / ((a^2-b^2)^3 R)
and gamma_AA = U_A on site.  The paper uses this kernel through DFTB-SCC
(Computational details); it does not restate it.

Evaluation.  The unequal-tau form is a removable singularity at ta = tb: its
two terms grow like 1 / (ta - tb)^3 and cancel, so in FP64 it loses about
three digits per decade of x = |ta - tb| / (ta + tb) (x = 1e-5 gives
percent-level errors).  Here
  x = 0 or x < 1e-9        the equal-tau form at tau = (ta + tb)/2 (its error
                           is O(x^2) relative, below 1e-17);
  1e-9 <= x < 0.15         the unequal-tau form evaluated in 50-digit decimal
                           arithmetic (the cancellation costs at most 27 of
                           the 50 digits), rounded to FP64;
  x >= 0.15                the unequal-tau form in FP64 (error below 2e-15 of
                           1/R there).
The same three branches give the radial derivative.

Pinned by: R -> 0 limits (U for equal tau, the closed form
0.5 (ta tb/(ta+tb) + ta^2 tb^2/(ta+tb)^3) for unequal), gamma -> 1/R at large R,
symmetry in (A, B), central finite differences of the derivative, and gamma
and d gamma / dR at finite R against a quadrature of the Coulomb integral of
the two normalised exponential densities in Fourier space (equal, unequal and
near-equal exponents; continuity across the branch switches).
"""
import decimal
import math

import numpy as np

X_EQUAL = 1e-9
X_DECIMAL = 0.15
_DEC = decimal.Context(prec=50)


def tau_of(u):
    return 16.0 * u / 5.0


def _equal(t, r):
    e = math.exp(-t * r)
    poly = 1.0 / r + 11.0 * t / 16.0 + 3.0 * t * t * r / 16.0 + t ** 3 * r * r / 48.0
    dpoly = -1.0 / (r * r) + 3.0 * t * t / 16.0 + t ** 3 * r / 24.0
    s = e * poly
    return s, -t * s + e * dpoly


def _unequal(ta, tb, r, one, exp):
    s = 0 * one
    ds = 0 * one
    for a, b in ((ta, tb), (tb, ta)):
        d2 = a * a - b * b
        k1 = b ** 4 * a / (2 * d2 * d2)
        k2 = (b ** 6 - 3 * a * a * b ** 4) / (d2 ** 3)
        e = exp(-a * r)
        val = e * (k1 - k2 / r)
        s += val
        ds += -a * val + e * (k2 / (r * r))
    return s, ds


def gamma_r(ua, ub, r):
    """(gamma, d gamma / dR) for two distinct sites at distance r > 0."""
    ta, tb = tau_of(ua), tau_of(ub)
    x = abs(ta - tb) / (ta + tb)
    if x < X_EQUAL:
        s, ds = _equal(0.5 * (ta + tb), r)
    elif x < X_DECIMAL:
        D = decimal.Decimal
        with decimal.localcontext(_DEC):
            s, ds = _unequal(D(ta), D(tb), D(r), D(1), lambda z: z.exp())
            g = 1 / D(r) - s
            dg = -1 / (D(r) * D(r)) - ds
        return float(g), float(dg)
    else:
        s, ds = _unequal(ta, tb, r, 1.0, math.exp)
    return 1.0 / r - s, -1.0 / (r * r) - ds


def gamma_matrix(params, species, pos, deriv=False):
    """gamma (Na x Na); with deriv also dgamma/dR (Na x Na) as radial derivative."""
    U = params["hubbard_u"]
    na = len(species)
    G = np.zeros((na, na))
    dG = np.zeros((na, na))
    for a in range(na):
        G[a, a] = U[species[a]]
        for b in range(a + 1, na):
            r = float(np.linalg.norm(pos[b] - pos[a]))
            g, dg = gamma_r(U[species[a]], U[species[b]], r)
            G[a, b] = G[b, a] = g
            dG[a, b] = dG[b, a] = dg
    return (G, dG) if deriv else G
