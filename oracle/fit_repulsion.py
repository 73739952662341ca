"""Choose the synthetic parameter seed and fit the pair-repulsion prefactors.

Run once (python -m oracle.fit_repulsion); it writes cavgen/repulsion_<seed>.json.
Uses only the oracle and the seeded parameter draws.

Seed rule.  The workload gives only ranges for the exponential Slater-Koster
tables.  Many draws leave the isolated water with a HOMO-LUMO gap of a few mHa,
where zero-temperature aufbau SCC sloshes charge between molecules.  The seed
is therefore the one, among 3277..3676, whose monomer (0.96 A, 104.5 deg) SCC
gap is at least 0.09 Ha, whose fitted prefactors are both positive, and whose
smallest gap over the first 8 clusters of the 8-water workload is the largest.

Repulsion.  E_rep = sum_{A<B} A_AB exp(-alpha r), alpha = 2.0 /bohr.  A_OH and
A_HH solve the 2x2 linear system that zeroes the radial and the in-plane
tangential force on H1 of the monomer at its template geometry (symmetric
stretch and bend balance); A_OO = A_OH.
"""
import json
import math
import sys

import numpy as np

from cavgen import params as CP
from cavgen.systems import make_system, monomer_template
from oracle.scc import scc_unit

SEED_LO, SEED_HI = 3277, 3677
MONOMER_GAP_MIN = 0.09


def fit_prefactors(p, alpha=2.0):
    tmpl = monomer_template()
    sp = np.array([0, 1, 1])
    r = scc_unit(p, sp, tmpl, tol=1e-12, max_iter=200)
    if r["status"]:
        return None
    n = r["n_occ"]
    gap = r["eps"][n] - r["eps"][n - 1]
    F = r["forces"]
    u1 = tmpl[1] - tmpl[0]
    r1 = np.linalg.norm(u1)
    u1 = u1 / r1
    t1 = np.cross(np.array([0.0, 0.0, 1.0]), u1)
    d21 = tmpl[1] - tmpl[2]
    rhh = np.linalg.norm(d21)
    u21 = d21 / rhh
    f_oh = alpha * math.exp(-alpha * r1) * u1
    f_hh = alpha * math.exp(-alpha * rhh) * u21
    M = np.array([[f_oh @ u1, f_hh @ u1], [f_oh @ t1, f_hh @ t1]])
    b = -np.array([F[1] @ u1, F[1] @ t1])
    A = np.linalg.solve(M, b)
    return gap, float(A[0]), float(A[1])


def main():
    sysd = make_system(2, n_units=8)
    uo = sysd["unit_off"]
    best = None
    for seed in range(SEED_LO, SEED_HI):
        p = CP.make_params(seed, with_repulsion=False)
        fit = fit_prefactors(p)
        if fit is None:
            continue
        gap, a_oh, a_hh = fit
        if gap < MONOMER_GAP_MIN or a_oh <= 0 or a_hh <= 0:
            continue
        gaps = []
        for u in range(8):
            a0, a1 = uo[u], uo[u + 1]
            r = scc_unit(p, sysd["species"][a0:a1], sysd["pos"][a0:a1], tol=1e-10, max_iter=150,
                         want_forces=False)
            if r["status"]:
                gaps = None
                break
            n = r["n_occ"]
            gaps.append(r["eps"][n] - r["eps"][n - 1])
        if gaps is None:
            continue
        print(f"seed {seed}: monomer gap {gap:.4f}  min cluster gap {min(gaps):.4f}", flush=True)
        if best is None or min(gaps) > best[1]:
            best = (seed, min(gaps), a_oh, a_hh, gap)
    seed, cgap, a_oh, a_hh, gap = best
    out = {"seed": seed, "alpha": 2.0, "A_OH": a_oh, "A_HH": a_hh, "A_OO": a_oh,
           "monomer_gap": gap, "min_cluster_gap": cgap}
    path = CP.repulsion_file(seed)
    with open(path, "w") as f:
        json.dump(out, f, indent=2)
    print("wrote", path, out)
    return 0


if __name__ == "__main__":
    sys.exit(main())
