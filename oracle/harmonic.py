"""Harmonic matter backend (oracle), used only to pin the cavity integrator.

Each unit is one particle of mass m in V = 1/2 m Omega^2 |r - r0|^2 with a
linear dipole mu = d (r - r0), so Z = d I.  Coupled to the cavity this is a
set of linear oscillators whose exact frequencies are the square roots of the
mass-weighted Hessian of the cavity Hamiltonian; with one mode, one cell,
phi = 1 and dt -> 0 the bright pair splits linearly in lambda (Results: Rabi
splitting proportional to the coupling, as in a Jaynes-Cummings model).
"""
import numpy as np


class HarmonicBackend:
    def __init__(self, masses, omega0, dip, r0):
        self.m = np.asarray(masses, dtype=np.float64)
        self.w0 = np.asarray(omega0, dtype=np.float64)
        self.d = np.asarray(dip, dtype=np.float64)
        self.r0 = np.asarray(r0, dtype=np.float64)

    def evaluate(self, r):
        x = r - self.r0
        k = self.m * self.w0 ** 2
        U = len(self.m)
        return {"energy": 0.5 * k * (x ** 2).sum(1), "forces": -k[:, None] * x,
                "mu": self.d[:, None] * x, "Z": self.d[:, None, None] * np.eye(3)[None],
                "charges": self.d.copy(), "status": np.zeros(U, dtype=np.int32)}


def polariton_hessian(masses, omega0, dip, phi, omega, lam, pol_axis=2):
    """Mass-weighted Hessian over (x_n along the polarisation, q_m):
    d2/dx dx' = Omega^2 delta + sum_m lam^2 phi_mn phi_mn' dt_n dt_n',
    d2/dq dx  = omega_m lam_m phi_mn dt_n,  d2/dq2 = omega_m^2, dt_n = d_n/sqrt(m_n)."""
    m = np.asarray(masses)
    dt_ = np.asarray(dip) / np.sqrt(m)
    U, M = len(m), len(omega)
    Hs = np.zeros((U + M, U + M))
    A = (lam[:, None] * phi) * dt_[None, :]          # (M, U)
    Hs[:U, :U] = np.diag(np.asarray(omega0) ** 2) + A.T @ A
    Hs[U:, :U] = (omega[:, None]) * A
    Hs[:U, U:] = Hs[U:, :U].T
    Hs[U:, U:] = np.diag(omega ** 2)
    return Hs
