"""Second-order SCC-DFTB charge kernel gamma_AB(R) (oracle).

Elstner et al., Phys. Rev. B 58, 7260 (1998): the Coulomb interaction of two
exponential charge densities with decay tau = 16 U / 5,
  gamma_AB(R) = 1/R - S(tau_A, tau_B, R)
  equal tau:   S = e^{-tau R} (1/R + 11 tau/16 + 3 tau^2 R/16 + tau^3 R^2/48)
  unequal tau: S = e^{-ta R} K(ta, tb, R) + e^{-tb R} K(tb, ta, R),
               K(a, b, R) = b^4 a / (2 (a^2-b^2)^2) - (b^6 - 3 a^2 b^4) / ((a^2-b^2)^3 R)
and gamma_AA = U_A on site.  The paper uses this kernel through DFTB-SCC
(Computational details); it does not restate it.

Pinned by: R -> 0 limits (U for equal tau, the closed form
0.5 (ta tb/(ta+tb) + ta^2 tb^2/(ta+tb)^3) for unequal), gamma -> 1/R at large R,
symmetry in (A, B) and central finite differences of the derivative.
"""
import math

import numpy as np


def tau_of(u):
    return 16.0 * u / 5.0


def gamma_r(ua, ub, r):
    """(gamma, d gamma / dR) for two distinct sites at distance r > 0."""
    ta, tb = tau_of(ua), tau_of(ub)
    if abs(ta - tb) < 1e-10 * max(ta, tb):
        t = 0.5 * (ta + tb)
        e = math.exp(-t * r)
        poly = 1.0 / r + 11.0 * t / 16.0 + 3.0 * t * t * r / 16.0 + t ** 3 * r * r / 48.0
        dpoly = -1.0 / (r * r) + 3.0 * t * t / 16.0 + t ** 3 * r / 24.0
        s = e * poly
        ds = -t * s + e * dpoly
    else:
        def kpart(a, b):
            d2 = a * a - b * b
            k1 = b ** 4 * a / (2.0 * d2 * d2)
            k2 = (b ** 6 - 3.0 * a * a * b ** 4) / (d2 ** 3)
            e = math.exp(-a * r)
            val = e * (k1 - k2 / r)
            dval = -a * val + e * (k2 / (r * r))
            return val, dval
        v1, d1 = kpart(ta, tb)
        v2, d2_ = kpart(tb, ta)
        s, ds = v1 + v2, d1 + d2_
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
