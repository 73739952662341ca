"""Born charges Z_A = d mu / d R_A (oracle).

The nuclear force of the paper carries the dipole derivative d mu_n / d r_{n,j}
(Theory: the forces F^m; Results: the Born charges are its bottleneck and are
obtained by finite differences of the SCC dipole).  Two forms:

  Mulliken replacement (Results, the cheap substitute):   Z_A = Q_A I_3
  Exact by central finite differences of the converged SCC dipole:
      Z_A[a][b] = (mu_a(R + h e_{A b}) - mu_a(R - h e_{A b})) / (2 h)

Layout: Z[A][a][b] = d mu_a / d R_{A b}.  Displaced SCCs are warm-started from
the undisplaced charges.

  Exact by forward finite differences (the paper's own scheme, Computational
  details), against the undisplaced dipole mu(R):
      Z_A[a][b] = (mu_a(R + h e_{A b}) - mu_a(R)) / h
  3 N_a displaced SCCs per unit; first-order in h.

  Exact by the Maxwell relation (the force on an atom responds to a uniform
  field exactly as the dipole responds to that atom's displacement):
      Z_A[a][b] = d F_{A b} / d field_a
               = (F_{A b}(+e e_a) - F_{A b}(-e e_a)) / (2 e)
  six field-perturbed SCC evaluations per unit instead of 6 N_a displaced ones.

Pinned by: acoustic sum rule sum_A Z_A = 0 for a neutral unit, the rotational
sum rule sum_A Z_A (theta x R_A) = theta x mu, the C2v pattern of a symmetric
monomer in its own frame, and agreement of the two independent exact routes
(tests/test_oracle_born_cavity_md.py).
"""
import numpy as np

from .scc import scc_unit


def born_mulliken(charges):
    charges = np.asarray(charges, dtype=np.float64)
    return charges[:, None, None] * np.eye(3)[None, :, :]


def born_field(params, species, pos, e=1.0e-4, tol=1e-12, max_iter=200, dq_center=None):
    """Returns (Z (Na,3,3), worst SCC status over the 6 field-perturbed runs)."""
    pos = np.asarray(pos, dtype=np.float64)
    na = len(species)
    Z = np.zeros((na, 3, 3))
    worst = 0
    for a in range(3):
        fs = []
        for sgn in (1.0, -1.0):
            fld = np.zeros(3)
            fld[a] = sgn * e
            r = scc_unit(params, species, pos, tol=tol, max_iter=max_iter, dq_start=dq_center, field=fld)
            worst |= r["status"]
            fs.append(r["forces"])
        Z[:, a, :] = (fs[0] - fs[1]) / (2.0 * e)
    return Z, worst


def born_fd_forward(params, species, pos, mu_center, h=1.0e-3, tol=1e-12, max_iter=200, dq_center=None):
    """Forward differences against the undisplaced dipole mu_center (3,).
    Returns (Z (Na,3,3), worst SCC status over the 3 Na displaced runs)."""
    pos = np.asarray(pos, dtype=np.float64)
    mu0 = np.asarray(mu_center, dtype=np.float64)
    na = len(species)
    Z = np.zeros((na, 3, 3))
    worst = 0
    for a in range(na):
        for b in range(3):
            x = pos.copy()
            x[a, b] += h
            r = scc_unit(params, species, x, tol=tol, max_iter=max_iter, dq_start=dq_center, want_forces=False)
            worst |= r["status"]
            Z[a, :, b] = (r["dipole"] - mu0) / h
    return Z, worst


def born_fd(params, species, pos, h=1.0e-3, tol=1e-12, max_iter=200, dq_center=None):
    """Returns (Z (Na,3,3), worst SCC status over the 6 Na displaced runs)."""
    pos = np.asarray(pos, dtype=np.float64)
    na = len(species)
    Z = np.zeros((na, 3, 3))
    worst = 0
    for a in range(na):
        for b in range(3):
            mus = []
            for sgn in (1.0, -1.0):
                x = pos.copy()
                x[a, b] += sgn * h
                r = scc_unit(params, species, x, tol=tol, max_iter=max_iter, dq_start=dq_center,
                             want_forces=False)
                worst |= r["status"]
                mus.append(r["dipole"])
            Z[a, :, b] = (mus[0] - mus[1]) / (2.0 * h)
    return Z, worst
