"""Cavity molecular-dynamics step (oracle).

The paper integrates classical nuclei and photons with a velocity-Verlet-like
scheme (Theory, Step 1 Eq. pj1 and Step 3 Eq. qknk): half-kick the photon
momenta with the light-matter coupling force only, velocity-Verlet the nuclei
(the second nuclear half-kick uses the new positions but the OLD photon
coordinates), half-kick the photon momenta again at the new positions, then
propagate the free photons exactly.  In mode space (no real-space transform is
needed when the photon state is kept per mode) one step of length dt is

  1. p_m   -= dt/2 lambda_m omega_m F_m(t)
  2. p_nj  += dt/2 [ -dV/dr(t) - E_n(t) (e . Z_nj(t)) ]
  3. r     += dt p / m
  4. matter evaluation at r(t+dt): -dV/dr, mu, Z
  5. F_m(t+dt);  E_n' with q_m(t)
  6. p_nj  += dt/2 [ -dV/dr(t+dt) - E_n' (e . Z_nj(t+dt)) ]
  7. p_m   -= dt/2 lambda_m omega_m F_m(t+dt)
  8. (q_m, p_m) <- exact rotation by omega_m dt
  9. E_n(t+dt) with the rotated q for the next step.

Photon start (Step 0 reading): q_m = -lambda_m F_m / omega_m, p_m = 0, the
minimum of the photon energy at frozen matter.  A thermal start draws (q_m, p_m)
from the classical Boltzmann distribution of that photon energy at temperature
T instead: p_m = sqrt(kT) xi_m, q_m = -lambda_m F_m / omega_m + sqrt(kT) xi'_m / omega_m,
with the standard normal draws xi passed in (no random numbers are drawn here).

Pinned by: the free-mode closed form (lambda = 0), the normal-mode frequencies
of a harmonic polariton, bounded energy error that shrinks with dt on the
exact-Born path (tests/test_oracle_cavity.py, tests/test_oracle_md.py).
"""
import numpy as np

from . import cavity as cav
from .born import born_fd, born_fd_forward, born_field, born_mulliken
from .scc import scc_unit
from .surrogate import predict_unit
from cavgen.constants import KB


class DFTBBackend:
    """SCC-DFTB matter for every unit; Born charges by the Mulliken replacement
    or by finite differences (born="fd": central, of the dipole in the atom
    displacements; born="fd_forward": forward, against the undisplaced dipole;
    born="field": central, of the forces in a uniform field, step h in atomic
    units of field).  With born_every = k > 1 the exact Born charges are
    recomputed on every k-th evaluation only (the first included) and reused in
    between (the paper refreshes them every 3 steps, Theory, Step 1).

    born="surrogate": the learned ensemble's prediction (surrogate.predict_unit
    with the Mulliken charges of the same SCC), and, for a unit whose largest
    per-atom, per-component ensemble standard deviation exceeds
    surrogate["threshold"], the exact route surrogate["fallback"] ("field" or
    "fd") with step h instead.  surrogate = {"nets", "norms", "threshold",
    "fallback", "emulate_bf16"} in the form predict_unit takes."""

    def __init__(self, params, species, unit_off, born="mulliken", tol=1e-12, h=1e-3, max_iter=200, born_every=1,
                 surrogate=None):
        self.params, self.species, self.unit_off = params, np.asarray(species), np.asarray(unit_off)
        self.born, self.tol, self.h, self.max_iter = born, tol, h, max_iter
        self.n_units = len(unit_off) - 1
        self.born_every = int(born_every)
        self.calls = 0
        self.Z_last = None
        self.surrogate = surrogate
        self.fallback_units = []

    def evaluate(self, r):
        U = self.n_units
        na = self.unit_off[-1]
        out = {"energy": np.zeros(U), "forces": np.zeros((na, 3)), "mu": np.zeros((U, 3)),
               "Z": np.zeros((na, 3, 3)), "charges": np.zeros(na), "status": np.zeros(U, dtype=np.int32)}
        for u in range(U):
            a0, a1 = self.unit_off[u], self.unit_off[u + 1]
            sp = self.species[a0:a1]
            res = scc_unit(self.params, sp, r[a0:a1], tol=self.tol, max_iter=self.max_iter)
            out["status"][u] = res["status"]
            out["energy"][u] = res["energy"]
            out["forces"][a0:a1] = res["forces"]
            out["mu"][u] = res["dipole"]
            out["charges"][a0:a1] = res["charges"]
            refresh = self.calls % self.born_every == 0
            born = self.born
            if born == "surrogate":
                sg = self.surrogate
                Z, sd = predict_unit(sp, r[a0:a1], sg["nets"], sg["norms"], res["charges"],
                                     emulate_bf16=sg.get("emulate_bf16", False))
                if float(sd.max()) > sg["threshold"]:
                    born = sg["fallback"]
                    self.fallback_units.append((self.calls, u))
            if born == "surrogate":
                pass
            elif self.born in ("fd", "fd_forward", "field") and not refresh:
                Z = self.Z_last[a0:a1]
            elif born == "fd":
                Z, st = born_fd(self.params, sp, r[a0:a1], h=self.h, tol=self.tol, max_iter=self.max_iter,
                                dq_center=res["dq"])
                out["status"][u] |= st
            elif born == "fd_forward":
                Z, st = born_fd_forward(self.params, sp, r[a0:a1], res["dipole"], h=self.h, tol=self.tol,
                                        max_iter=self.max_iter, dq_center=res["dq"])
                out["status"][u] |= st
            elif born == "field":
                Z, st = born_field(self.params, sp, r[a0:a1], e=self.h, tol=self.tol, max_iter=self.max_iter,
                                   dq_center=res["dq"])
                out["status"][u] |= st
            else:
                Z = born_mulliken(res["charges"])
            out["Z"][a0:a1] = Z
        if self.born in ("fd", "fd_forward", "field") and self.calls % self.born_every == 0:
            self.Z_last = out["Z"].copy()
        self.calls += 1
        return out


class Cavity:
    def __init__(self, omega, k, theta, lam, unit_x, pol):
        self.omega = np.asarray(omega, dtype=np.float64)
        self.lam = np.asarray(lam, dtype=np.float64)
        self.pol = np.asarray(pol, dtype=np.float64)
        self.phi = cav.mode_functions(np.asarray(k), np.asarray(theta), np.asarray(unit_x))


def _zpol(Z, pol):
    # (e . Z_j)_b = sum_a e_a Z_j[a][b]
    return np.einsum("a,jab->jb", pol, Z)


def init_state(backend, cavity, r, p, masses, atom_unit, photons="relaxed", kT=0.0, xi=None):
    """photons: "relaxed" (minimum of the photon energy at frozen matter),
    "zero" (q = p = 0) or "thermal" (Boltzmann at kT about the relaxed start;
    xi holds 2M standard normal draws: xi[:M] for q, xi[M:] for p)."""
    ev = backend.evaluate(r)
    F = cav.dipole_sums(cavity.phi, ev["mu"] @ cavity.pol)
    pm = np.zeros_like(cavity.omega)
    if photons in ("relaxed", "thermal"):
        q = -cavity.lam * F / cavity.omega
    else:
        q = np.zeros_like(cavity.omega)
    if photons == "thermal":
        M = len(cavity.omega)
        xi = np.asarray(xi, dtype=np.float64)
        q = q + np.sqrt(kT) * xi[:M] / cavity.omega
        pm = np.sqrt(kT) * xi[M:2 * M]
    E = cav.fields(cavity.phi, cavity.omega, cavity.lam, q, F)
    return {"r": np.array(r, dtype=np.float64), "p": np.array(p, dtype=np.float64), "q": q, "pm": pm,
            "ev": ev, "F": F, "E": E, "masses": np.asarray(masses, dtype=np.float64),
            "atom_unit": np.asarray(atom_unit)}


def step(st, backend, cavity, dt):
    lwo = cavity.lam * cavity.omega
    au, m = st["atom_unit"], st["masses"]
    pm = st["pm"] - 0.5 * dt * lwo * st["F"]
    fn = st["ev"]["forces"] - st["E"][au][:, None] * _zpol(st["ev"]["Z"], cavity.pol)
    p = st["p"] + 0.5 * dt * fn
    r = st["r"] + dt * p / m[:, None]
    ev = backend.evaluate(r)
    F1 = cav.dipole_sums(cavity.phi, ev["mu"] @ cavity.pol)
    E1 = cav.fields(cavity.phi, cavity.omega, cavity.lam, st["q"], F1)
    fn1 = ev["forces"] - E1[au][:, None] * _zpol(ev["Z"], cavity.pol)
    p = p + 0.5 * dt * fn1
    pm = pm - 0.5 * dt * lwo * F1
    q, pm = cav.rotate(st["q"], pm, cavity.omega, dt)
    E = cav.fields(cavity.phi, cavity.omega, cavity.lam, q, F1)
    st.update({"r": r, "p": p, "q": q, "pm": pm, "ev": ev, "F": F1, "E": E})
    return st


def observables(st, cavity, unit_off=None):
    m = st["masses"]
    ke = float((st["p"] ** 2 / (2.0 * m[:, None])).sum())
    v = float(st["ev"]["energy"].sum())
    eph = cav.photon_energy(st["q"], st["pm"], cavity.omega, cavity.lam, st["F"])
    out = {"kinetic": ke, "potential": v, "photon": eph, "total": ke + v + eph}
    if unit_off is not None:
        U = len(unit_off) - 1
        temps = np.zeros(U)
        for u in range(U):
            a0, a1 = unit_off[u], unit_off[u + 1]
            pu = st["p"][a0:a1]
            mu_ = m[a0:a1]
            pcm = pu.sum(0)
            prel = pu - mu_[:, None] * pcm / mu_.sum()
            ke_u = float((prel ** 2 / (2.0 * mu_[:, None])).sum())
            dof = 3 * (a1 - a0) - 3
            temps[u] = 2.0 * ke_u / (dof * KB) if dof > 0 else 0.0
        out["temperature"] = float(temps.mean())
    return out
