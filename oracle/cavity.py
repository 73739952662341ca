"""Multimode Fabry-Perot cavity in mode space (oracle).

The paper's light-matter Hamiltonian in the dipole gauge beyond the
long-wavelength limit (Theory, Eq. hlm_bigin with mode function
f_k(R_n) = g0 / sqrt(omega_k) e^{i k R_n}) is, for classical photons and real
standing-wave modes (the +-k plane-wave pairs recombined), the Pauli-Fierz form

  H = H_M + sum_m [ p_m^2/2 + 1/2 omega_m^2 (q_m + (lambda_m/omega_m) F_m)^2 ],
  F_m = sum_n phi_m(X_n) (e . mu_n),   phi_m(X) = sin(k_m X + theta_m).

With one mode, one cell and phi = 1 this is the paper's single-box Hamiltonian
(Eq. hlm4) with eta = lambda omega.  Derived quantities:

  field felt by cell n:   E_n = sum_m lambda_m omega_m phi_m(X_n) (q_m + lambda_m F_m / omega_m)
  nuclear coupling force: -E_n (e . Z_{n,j})         (Eq. dpj, last two terms)
  photon coupling force:  -lambda_m omega_m F_m       (Eq. dpj, the -eta mu_n term)
  free photon motion:     exact rotation of (q, p) by omega dt (Step 3, Eq. qknk)

Pinned by: closed-form free-mode motion, the single-box special case, and the
normal modes of a harmonic polariton (tests/test_oracle_cavity.py).
"""
import numpy as np


def mode_functions(k, theta, unit_x):
    """phi (M, U)."""
    return np.sin(np.outer(k, unit_x) + np.asarray(theta)[:, None])


def dipole_sums(phi, mu_pol):
    return phi @ mu_pol


def fields(phi, omega, lam, q, F):
    g = lam * omega * (q + lam * F / omega)
    return phi.T @ g


def photon_coupling_force(omega, lam, F):
    return -lam * omega * F


def rotate(q, p, omega, dt):
    c, s = np.cos(omega * dt), np.sin(omega * dt)
    return q * c + p * s / omega, p * c - omega * q * s


def photon_energy(q, p, omega, lam, F):
    x = q + lam * F / omega
    return float(0.5 * (p @ p) + 0.5 * ((omega * x) @ (omega * x)))
