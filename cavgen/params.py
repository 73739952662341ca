"""Seeded synthetic SCC-DFTB parameter set (the paper's own Slater-Koster set is
not given; the workload replaces it by exponential radial tables).

Everything here is input data. Table layout (shared by every consumer):

  index  pair   integral                      orbitals
  0      O-O    ss sigma
  1      O-O    sp sigma   (s on one O, p on the other)
  2      O-O    pp sigma
  3      O-O    pp pi
  4      O-H    ss sigma   (s_H, s_O)
  5      O-H    sp sigma   (s_H, p_O)
  6      H-H    ss sigma

Each table t carries four numbers (a, b, c, d): the hopping radial function is
a*exp(-b*r) (hartree) and the overlap radial function is c*exp(-d*r).

Draw order (numpy default_rng(seed)): for t = 0..6 in the order above, one
uniform draw each of a in [-0.5, -0.1], b in [0.8, 1.6], c in [0.2, 0.6],
d in [0.8, 1.6], in that order.  Pair repulsion is A*exp(-alpha*r) with
alpha = 2.0 /bohr for every pair type; the prefactors A_OH and A_HH are read
from the data file repulsion_<seed>.json (A_OO = A_OH), written once by a
script that places the isolated monomer's equilibrium at 0.96 A / 104.5 deg.
"""
import json
import os

import numpy as np

from . import constants as K

N_TABLES = 7
TABLE_NAMES = ("OO_ss", "OO_sp", "OO_pps", "OO_ppp", "OH_ss", "OH_sp", "HH_ss")
PARAM_SEED = 3366
REP_ALPHA = 2.0

ONSITE = ((-0.87, -0.33), (-0.24, 0.0))   # [species][l]: O {s, p}, H {s, -}
HUBBARD_U = (0.50, 0.42)                  # O, H (hartree)
Q0 = (6.0, 1.0)                           # neutral valence populations
N_ORB = (4, 1)                            # O: s px py pz ; H: s


def draw_sk_tables(seed=PARAM_SEED):
    rng = np.random.default_rng(seed)
    sk = np.zeros((N_TABLES, 4))
    for t in range(N_TABLES):
        sk[t, 0] = rng.uniform(-0.5, -0.1)
        sk[t, 1] = rng.uniform(0.8, 1.6)
        sk[t, 2] = rng.uniform(0.2, 0.6)
        sk[t, 3] = rng.uniform(0.8, 1.6)
    return sk


def repulsion_file(seed=PARAM_SEED):
    return os.path.join(os.path.dirname(__file__), f"repulsion_{seed}.json")


def make_params(seed=PARAM_SEED, with_repulsion=True):
    """Return the parameter dictionary used by every consumer.

    Keys: sk (7,4), onsite (2,2), hubbard_u (2,), q0 (2,), n_orb (2,),
    rep_a (3,) for pair types OO, OH, HH, rep_alpha (3,), mass (2,) in m_e.
    """
    p = {
        "seed": seed,
        "sk": draw_sk_tables(seed),
        "onsite": np.array(ONSITE, dtype=np.float64),
        "hubbard_u": np.array(HUBBARD_U, dtype=np.float64),
        "q0": np.array(Q0, dtype=np.float64),
        "n_orb": np.array(N_ORB, dtype=np.int64),
        "rep_alpha": np.full(3, REP_ALPHA),
        "rep_a": np.zeros(3),
        "mass": np.array(K.MASS_AMU) * K.AMU,
    }
    if with_repulsion:
        path = repulsion_file(seed)
        with open(path) as f:
            rep = json.load(f)
        p["rep_a"] = np.array([rep["A_OH"], rep["A_OH"], rep["A_HH"]], dtype=np.float64)
        p["rep_alpha"] = np.full(3, float(rep["alpha"]))
    return p
