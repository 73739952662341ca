"""Second-order SCC-DFTB evaluation of one unit (oracle).

The paper computes the matter potential V_n, its gradient and the cell dipole
mu_n on the fly with second-order SCC-DFTB (Theory: the -grad V_n term of the
nuclear force; Computational details).  Its formulas are the standard ones
(Elstner et al. 1998), written out here for a closed-shell unit at zero
electronic temperature:

  Delta q_A = q_A - q0_A,  q_A = sum_{mu in A} (P S)_{mu mu}          (Mulliken)
  V_A = sum_C gamma_AC Delta q_C
  H_{mu nu} = H0_{mu nu} + 1/2 S_{mu nu} (V_{A(mu)} + V_{B(nu)})
  H C = S C eps,  lowest n_occ = N_el/2 orbitals doubly occupied (aufbau)
  P = 2 C_occ C_occ^T,  W = 2 C_occ diag(eps_occ) C_occ^T
  E = sum P o H0 + 1/2 Dq^T gamma Dq + sum_{A<B} A_AB exp(-alpha_AB R_AB)
  F_A = -sum P dH0/dR_A + sum [W - 1/2 P (V_A + V_B)] o dS/dR_A
        - Dq_A sum_C dgamma_AC/dR_A Dq_C - dE_rep/dR_A
  Q_A = -Delta q_A,  mu = sum_A Q_A R_A.

Self-consistency is reached with Johnson's modified Broyden mixing (Phys. Rev.
B 38, 12807 (1988)); converged when max_A |Dq_out - Dq_in| < tol.  After
convergence every reported quantity (charges, dipole, energy, the V of the
force) uses Dq_out, the Mulliken charges of the final density; W uses the final
eigenvalues.

Pinned by: eigen residuals and S-orthonormality, Tr(PS) = N_el, PSP = 2P,
charge neutrality, mixer/start independence of the fixed point, the non-SCC
limit, forces = -central finite differences of E, translational and rotational
sum rules (tests/test_oracle_scc.py).
"""
import math

import numpy as np
from scipy.linalg import solve_triangular

from .gamma import gamma_matrix
from .sk import build_h0_s, orbital_offsets, pair_blocks

ST_NOT_CONVERGED = 1
ST_NOT_PD = 2
ST_DEGENERATE = 4
ST_NAN = 8

GAP_MIN = 1.0e-6


class Broyden:
    """Johnson's modified Broyden mixer on the charge vector.

    u_n = alpha dF_n + dx_n (dF, dx normalised by |F_n - F_{n-1}|),
    x_{m+1} = x_m + alpha F_m - sum_n gamma_n u_n,
    gamma = c (w0^2 I + a)^{-1},  a_kn = dF_k . dF_n,  c_k = dF_k . F_m,
    unit weights, a sliding window of at most max_hist pairs."""

    def __init__(self, alpha=0.2, w0=0.01, max_hist=20):
        self.alpha, self.w0, self.max_hist = alpha, w0, max_hist
        self.x_prev = None
        self.f_prev = None
        self.dfs, self.us = [], []

    def next(self, x_in, x_out):
        f = x_out - x_in
        if self.x_prev is not None:
            df = f - self.f_prev
            nrm = math.sqrt(float(df @ df))
            if nrm > 1e-300:
                df = df / nrm
                self.dfs.append(df)
                self.us.append(self.alpha * df + (x_in - self.x_prev) / nrm)
                if len(self.dfs) > self.max_hist:
                    self.dfs.pop(0)
                    self.us.pop(0)
        self.x_prev, self.f_prev = x_in.copy(), f.copy()
        x_new = x_in + self.alpha * f
        if self.dfs:
            DF = np.array(self.dfs)
            UU = np.array(self.us)
            a = DF @ DF.T
            beta = np.linalg.inv(self.w0 ** 2 * np.eye(len(DF)) + a)
            c = DF @ f
            x_new = x_new - (c @ beta) @ UU
        return x_new


class Linear:
    def __init__(self, alpha=0.2):
        self.alpha = alpha

    def next(self, x_in, x_out):
        return x_in + self.alpha * (x_out - x_in)


def unit_electrons(params, species):
    return float(sum(params["q0"][s] for s in species))


def mulliken_atoms(params, species, P, S):
    off = orbital_offsets(params, species)
    q_orb = (P * S).sum(axis=1)
    return np.array([q_orb[off[a]:off[a + 1]].sum() for a in range(len(species))])


def repulsion(params, species, pos, deriv=False):
    na = len(species)
    e = 0.0
    grad = np.zeros((na, 3))
    for a in range(na):
        for b in range(a + 1, na):
            t = int(species[a]) + int(species[b])
            A, al = params["rep_a"][t], params["rep_alpha"][t]
            d = pos[b] - pos[a]
            r = float(np.linalg.norm(d))
            v = A * math.exp(-al * r)
            e += v
            g = -al * v * d / r
            grad[b] += g
            grad[a] -= g
    return (e, grad) if deriv else e


def energy_forces(params, species, pos, P, W, dq, H0, field=None):
    """Total energy and forces F = -dE/dR from a converged density.  With a
    uniform field, E gains sum_A Dq_A (field . R_A) (the energy -mu . field of
    the Mulliken dipole), V_A gains field . R_A and F_A gains -Dq_A field."""
    G, dG = gamma_matrix(params, species, pos, deriv=True)
    V = G @ dq
    vext = np.zeros(len(species)) if field is None else pos @ np.asarray(field, dtype=np.float64)
    V = V + vext
    off = orbital_offsets(params, species)
    e_band = float((P * H0).sum())
    e_coul = 0.5 * float(dq @ G @ dq)
    e_rep, grad = repulsion(params, species, pos, deriv=True)
    e_field = float(dq @ vext)
    if field is not None:
        grad = grad + dq[:, None] * np.asarray(field, dtype=np.float64)[None, :]
    na = len(species)
    for a in range(na):
        for b in range(a + 1, na):
            d = pos[b] - pos[a]
            r = float(np.linalg.norm(d))
            _, _, dH, dS = pair_blocks(params, species[a], species[b], d, deriv=True)
            Pb = P[off[a]:off[a + 1], off[b]:off[b + 1]]
            Wb = W[off[a]:off[a + 1], off[b]:off[b + 1]]
            g = 2.0 * (np.einsum("gij,ij->g", dH, Pb)
                       - np.einsum("gij,ij->g", dS, Wb - 0.5 * Pb * (V[a] + V[b])))
            g = g + dq[a] * dq[b] * dG[a, b] * d / r
            grad[b] += g
            grad[a] -= g
    return e_band + e_coul + e_rep + e_field, -grad, {"band": e_band, "coulomb": e_coul, "repulsion": e_rep,
                                                       "field": e_field}


def scc_unit(params, species, pos, tol=1e-12, max_iter=200, mixer="broyden", dq_start=None,
             gamma_scale=1.0, want_forces=True, mix_alpha=0.2, field=None):
    """SCC-DFTB of one unit, optionally in a uniform external field (3,).
    Returns a dict with energy, forces (Na,3), dq (Na,), charges Q = -dq,
    dipole (3,), P, W, eps, S, H0, n_iter, status."""
    species = np.asarray(species)
    pos = np.asarray(pos, dtype=np.float64)
    status = 0
    if not np.all(np.isfinite(pos)):
        return {"status": ST_NAN}
    H0, S = build_h0_s(params, species, pos)
    G = gamma_matrix(params, species, pos) * gamma_scale
    off = orbital_offsets(params, species)
    orb_atom = np.repeat(np.arange(len(species)), np.diff(off))
    q0 = np.array([params["q0"][s] for s in species])
    n_el = q0.sum()
    n_occ = int(round(n_el)) // 2
    try:
        L = np.linalg.cholesky(S)
    except np.linalg.LinAlgError:
        return {"status": ST_NOT_PD}
    mix = Broyden(alpha=mix_alpha) if mixer == "broyden" else Linear(alpha=mix_alpha)
    dq_in = np.zeros(len(species)) if dq_start is None else np.array(dq_start, dtype=np.float64)
    vext = np.zeros(len(species)) if field is None else pos @ np.asarray(field, dtype=np.float64)
    converged = False
    for it in range(1, max_iter + 1):
        V = G @ dq_in + vext
        Vo = V[orb_atom]
        H = H0 + 0.5 * S * (Vo[:, None] + Vo[None, :])
        Hp = solve_triangular(L, solve_triangular(L, H, lower=True).T, lower=True).T
        Hp = 0.5 * (Hp + Hp.T)
        eps, Y = np.linalg.eigh(Hp)
        C = solve_triangular(L.T, Y, lower=False)
        Cocc = C[:, :n_occ]
        P = 2.0 * Cocc @ Cocc.T
        dq_out = mulliken_atoms(params, species, P, S) - q0
        if np.max(np.abs(dq_out - dq_in)) < tol:
            converged = True
            break
        dq_in = mix.next(dq_in, dq_out)
    if not converged:
        status |= ST_NOT_CONVERGED
    if n_occ < len(eps) and eps[n_occ] - eps[n_occ - 1] < GAP_MIN:
        status |= ST_DEGENERATE
    W = 2.0 * (Cocc * eps[:n_occ]) @ Cocc.T
    out = {
        "dq": dq_out, "charges": -dq_out, "dipole": (-dq_out) @ pos,
        "P": P, "W": W, "eps": eps, "C": C, "S": S, "H0": H0, "H": H, "n_iter": it,
        "status": status, "n_occ": n_occ,
    }
    if want_forces:
        e, f, parts = energy_forces(params, species, pos, P, W, dq_out, H0, field=field)
        if gamma_scale != 1.0:
            # energy of the scaled model (used only by the non-SCC limit pin)
            e = parts["band"] + 0.5 * gamma_scale * float(dq_out @ gamma_matrix(params, species, pos) @ dq_out) \
                + parts["repulsion"]
        out.update({"energy": e, "forces": f, "energy_parts": parts})
    return out


def eval_units(params, species, pos, unit_off, tol=1e-12, max_iter=200, want_forces=True, dq_start=None):
    """Loop of scc_unit over units given in CSR form (unit_off[U+1]).
    Returns energy (U,), forces (Na_tot,3), charges (Na_tot,), dipole (U,3),
    status (U,), n_iter (U,)."""
    U = len(unit_off) - 1
    na = unit_off[-1]
    energy = np.zeros(U)
    forces = np.zeros((na, 3))
    charges = np.zeros(na)
    dipole = np.zeros((U, 3))
    status = np.zeros(U, dtype=np.int32)
    n_iter = np.zeros(U, dtype=np.int32)
    for u in range(U):
        a0, a1 = unit_off[u], unit_off[u + 1]
        r = scc_unit(params, species[a0:a1], pos[a0:a1], tol=tol, max_iter=max_iter, want_forces=want_forces,
                     dq_start=None if dq_start is None else dq_start[a0:a1])
        status[u] = r["status"]
        if "dq" not in r:
            continue
        charges[a0:a1] = r["charges"]
        dipole[u] = r["dipole"]
        n_iter[u] = r["n_iter"]
        if want_forces:
            energy[u] = r["energy"]
            forces[a0:a1] = r["forces"]
    return {"energy": energy, "forces": forces, "charges": charges, "dipole": dipole,
            "status": status, "n_iter": n_iter}
