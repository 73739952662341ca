"""Slater-Koster two-centre blocks of H0 and S, and their derivatives (oracle).

Follows the standard Slater-Koster direction-cosine rules (Slater and Koster,
Phys. Rev. 94, 1498 (1954), Table I) that second-order SCC-DFTB uses for its
non-SCC Hamiltonian (paper: Computational details, DFTB-SCC).  The radial
functions are the synthetic tables of the workload: H_t(r) = a exp(-b r),
S_t(r) = c exp(-d r).

Orbital order per atom: O -> s, px, py, pz ; H -> s.
For a pair (A, B) the direction cosines are u = (R_B - R_A)/|R_B - R_A| and
  <s_A|s_B>     = V_ss
  <s_A|p_B,b>   = u_b V_sp          (table of s on A, p on B)
  <p_A,a|s_B>   = -u_a V_sp'        (table of s on B, p on A)
  <p_A,a|p_B,b> = u_a u_b (V_pps - V_ppp) + delta_ab V_ppp
Derivatives are taken with respect to d = R_B - R_A, i.e. d/dR_B = -d/dR_A.

Pinned by: symmetric H0/S; a diatomic along z returns the raw table values;
rotation invariance of the spectrum (tests/test_oracle_sk.py); central finite
differences of every block element.
"""
import math

import numpy as np

# table indices (see cavgen.params)
OO_SS, OO_SP, OO_PPS, OO_PPP, OH_SS, OH_SP, HH_SS = range(7)


def radial(sk, t, r):
    """(H, S, dH/dr, dS/dr) of table t at distance r."""
    a, b, c, d = sk[t]
    h = a * math.exp(-b * r)
    s = c * math.exp(-d * r)
    return h, s, -b * h, -d * s


def _labels(sp):
    # (l, cartesian index) per orbital
    return [(0, -1), (1, 0), (1, 1), (1, 2)] if sp == 0 else [(0, -1)]


def pair_blocks(params, spA, spB, dvec, deriv=False):
    """H0 and S blocks <mu_A|.|nu_B> (nA x nB); with deriv, also their
    derivatives with respect to d = R_B - R_A as arrays (3, nA, nB)."""
    sk = params["sk"]
    d = np.asarray(dvec, dtype=np.float64)
    r = math.sqrt(float(d @ d))
    u = d / r
    LA, LB = _labels(spA), _labels(spB)
    nA, nB = len(LA), len(LB)
    H = np.zeros((nA, nB))
    S = np.zeros((nA, nB))
    dH = np.zeros((3, nA, nB))
    dS = np.zeros((3, nA, nB))

    # which table each (l_A, l_B) combination uses
    if spA == 0 and spB == 0:
        t_ss, t_sp_AB, t_sp_BA, t_pps, t_ppp = OO_SS, OO_SP, OO_SP, OO_PPS, OO_PPP
    elif spA == 0 and spB == 1:
        t_ss, t_sp_AB, t_sp_BA, t_pps, t_ppp = OH_SS, None, OH_SP, None, None
    elif spA == 1 and spB == 0:
        t_ss, t_sp_AB, t_sp_BA, t_pps, t_ppp = OH_SS, OH_SP, None, None, None
    else:
        t_ss, t_sp_AB, t_sp_BA, t_pps, t_ppp = HH_SS, None, None, None, None

    def du(a, g):  # d u_a / d d_g
        return ((1.0 if a == g else 0.0) - u[a] * u[g]) / r

    for i, (la, a) in enumerate(LA):
        for j, (lb, b) in enumerate(LB):
            if la == 0 and lb == 0:
                h, s, hp, spr = radial(sk, t_ss, r)
                H[i, j], S[i, j] = h, s
                for g in range(3):
                    dH[g, i, j] = hp * u[g]
                    dS[g, i, j] = spr * u[g]
            elif la == 0 and lb == 1:
                h, s, hp, spr = radial(sk, t_sp_AB, r)
                H[i, j], S[i, j] = u[b] * h, u[b] * s
                for g in range(3):
                    dH[g, i, j] = du(b, g) * h + u[b] * hp * u[g]
                    dS[g, i, j] = du(b, g) * s + u[b] * spr * u[g]
            elif la == 1 and lb == 0:
                h, s, hp, spr = radial(sk, t_sp_BA, r)
                H[i, j], S[i, j] = -u[a] * h, -u[a] * s
                for g in range(3):
                    dH[g, i, j] = -(du(a, g) * h + u[a] * hp * u[g])
                    dS[g, i, j] = -(du(a, g) * s + u[a] * spr * u[g])
            else:
                hs, ss_, hsp, ssp = radial(sk, t_pps, r)
                hp_, sp_, hpp, spp = radial(sk, t_ppp, r)
                dl = 1.0 if a == b else 0.0
                H[i, j] = u[a] * u[b] * (hs - hp_) + dl * hp_
                S[i, j] = u[a] * u[b] * (ss_ - sp_) + dl * sp_
                for g in range(3):
                    duu = du(a, g) * u[b] + u[a] * du(b, g)
                    dH[g, i, j] = duu * (hs - hp_) + u[a] * u[b] * (hsp - hpp) * u[g] + dl * hpp * u[g]
                    dS[g, i, j] = duu * (ss_ - sp_) + u[a] * u[b] * (ssp - spp) * u[g] + dl * spp * u[g]
    if deriv:
        return H, S, dH, dS
    return H, S


def orbital_offsets(params, species):
    n_orb = params["n_orb"]
    off = np.zeros(len(species) + 1, dtype=np.int64)
    for a, s in enumerate(species):
        off[a + 1] = off[a] + n_orb[s]
    return off


def build_h0_s(params, species, pos):
    """Assemble the unit's H0 and S (n x n) over all intra-unit atom pairs (no
    cutoff; units do not interact electronically, Theory: non-interacting cells)."""
    off = orbital_offsets(params, species)
    n = int(off[-1])
    H0 = np.zeros((n, n))
    S = np.eye(n)
    onsite = params["onsite"]
    for a, sa in enumerate(species):
        o = off[a]
        H0[o, o] = onsite[sa, 0]
        if sa == 0:
            for k in range(1, 4):
                H0[o + k, o + k] = onsite[sa, 1]
    na = len(species)
    for a in range(na):
        for b in range(a + 1, na):
            Hb, Sb = pair_blocks(params, species[a], species[b], pos[b] - pos[a])
            H0[off[a]:off[a + 1], off[b]:off[b + 1]] = Hb
            S[off[a]:off[a + 1], off[b]:off[b + 1]] = Sb
            H0[off[b]:off[b + 1], off[a]:off[a + 1]] = Hb.T
            S[off[b]:off[b + 1], off[a]:off[a + 1]] = Sb.T
    return H0, S
