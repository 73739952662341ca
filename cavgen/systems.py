"""Seeded synthetic systems: water-cluster units, Maxwell-Boltzmann velocities and
the Fabry-Perot mode comb for the five workloads of the cavity-DFTB hot path.

Stand-in for the paper's data: the paper propagates periodic liquid-water cells
(Computational details) that need its unnamed parameter set; here every unit is
an isolated water cluster generated from a seed, spaced along a 1-D cavity axis.

Draw order for a workload (numpy default_rng(100 + workload index)):
  1. waters per unit for all units (only for the mixed-size workloads 4 and 5);
  2. then per unit, in unit order: its cluster geometry (per molecule: site
     jitter (3), random rotation (4 normal draws -> quaternion), atom jitter
     (9); the whole cluster is redrawn while any intermolecular atom pair is
     closer than 1.5 A) followed by its velocities (3 per atom).
So the first k units of a workload are the same whatever the unit count.
"""
import math
from dataclasses import dataclass, field

import numpy as np

from . import constants as K

OH_BOND = 0.96 * K.ANGSTROM
HOH_ANGLE = math.radians(104.5)
LATTICE = 3.1 * K.ANGSTROM
SITE_JITTER = 0.1 * K.ANGSTROM
ATOM_JITTER = 0.02 * K.ANGSTROM
MIN_PAIR = 1.5 * K.ANGSTROM
CAVITY_LENGTH = 50.0 * K.MICRON
WN_LO, WN_HI = 1500.0, 4000.0     # cm^-1


@dataclass
class Workload:
    index: int
    name: str
    n_units: int
    waters: str            # "1", "8", "loguniform32", "uniform8"
    n_modes: int
    scc_tol: float
    born: str              # "mulliken", "fd", "surrogate"
    n_steps: int
    dt_fs: float = 0.25
    coupling: float = 0.005
    temperature: float = 300.0
    fd_h: float = 1.0e-3
    extra: dict = field(default_factory=dict)


WORKLOADS = {
    1: Workload(1, "8 x H2O monomer, Mulliken", 8, "1", 16, 1e-12, "mulliken", 100),
    2: Workload(2, "4096 x 8-water cluster, Mulliken", 4096, "8", 256, 1e-8, "mulliken", 1000),
    3: Workload(3, "1024 x 8-water cluster, exact Born (central FD)", 1024, "8", 256, 1e-12, "fd", 200),
    4: Workload(4, "16384 x 1-32-water clusters (log-uniform), Mulliken", 16384, "loguniform32", 1024, 1e-8,
                "mulliken", 500),
    5: Workload(5, "65536 x 1-8-water clusters, surrogate Born", 65536, "uniform8", 2048, 1e-8, "surrogate", 2000),
}


def monomer_template():
    """O at the origin, both H in the xy plane, bisector along +x."""
    h = HOH_ANGLE / 2.0
    return np.array([
        [0.0, 0.0, 0.0],
        [OH_BOND * math.cos(h), OH_BOND * math.sin(h), 0.0],
        [OH_BOND * math.cos(h), -OH_BOND * math.sin(h), 0.0],
    ])


def _rotation(rng):
    q = rng.normal(size=4)
    q /= np.linalg.norm(q)
    w, x, y, z = q
    return np.array([
        [1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
        [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
        [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)],
    ])


def _sites(w):
    s = int(math.ceil(round(w ** (1.0 / 3.0), 12)))
    while s ** 3 < w:
        s += 1
    out = []
    for i in range(s):
        for j in range(s):
            for k in range(s):
                out.append((i, j, k))
    return np.array(out[:w], dtype=np.float64) * LATTICE


def make_cluster(rng, w):
    """Positions (3w, 3) in bohr and species (3w,) for a w-water cluster."""
    tmpl = monomer_template()
    sites = _sites(w)
    while True:
        pos = np.empty((3 * w, 3))
        for i in range(w):
            site = sites[i] + rng.normal(0.0, SITE_JITTER, size=3)
            rot = _rotation(rng)
            jit = rng.normal(0.0, ATOM_JITTER, size=(3, 3))
            pos[3 * i:3 * i + 3] = tmpl @ rot.T + site + jit
        if w == 1:
            break
        d = np.linalg.norm(pos[:, None, :] - pos[None, :, :], axis=-1)
        mol = np.arange(3 * w) // 3
        inter = mol[:, None] != mol[None, :]
        if d[inter].min() >= MIN_PAIR:
            break
    species = np.tile(np.array([0, 1, 1], dtype=np.int8), w)
    return pos, species


def maxwell_boltzmann(rng, masses, temperature):
    v = rng.normal(size=(len(masses), 3)) * np.sqrt(K.KB * temperature / masses)[:, None]
    vcm = (masses[:, None] * v).sum(0) / masses.sum()
    return v - vcm


def waters_per_unit(wl, rng):
    if wl.waters == "1":
        return np.ones(wl.n_units, dtype=np.int64)
    if wl.waters == "8":
        return np.full(wl.n_units, 8, dtype=np.int64)
    if wl.waters == "loguniform32":
        u = rng.uniform(0.0, math.log(33.0), size=wl.n_units)
        return np.clip(np.floor(np.exp(u)).astype(np.int64), 1, 32)
    if wl.waters == "uniform8":
        return rng.integers(1, 9, size=wl.n_units).astype(np.int64)
    raise ValueError(wl.waters)


def mode_comb(n_modes, coupling=0.005):
    """omega_m = 1500 + m*2500/(M-1) cm^-1 (endpoints included), k_m = omega_m/c,
    phase 0, the same coupling for every mode."""
    if n_modes == 1:
        wn = np.array([WN_LO])
    else:
        wn = WN_LO + np.arange(n_modes) * (WN_HI - WN_LO) / (n_modes - 1)
    omega = wn / K.HARTREE_CM
    k = omega / K.C_AU
    theta = np.zeros(n_modes)
    lam = np.full(n_modes, coupling)
    return omega, k, theta, lam


def make_system(index, n_units=None, masses_me=None):
    """Generate workload `index` (1..5), optionally only its first n_units units.

    Returns a dict of numpy arrays: species (n_atoms,) int8, pos (n_atoms,3),
    vel (n_atoms,3), unit_off (n_units+1,) int32, unit_x (n_units,),
    omega/k/theta/lam (n_modes,), pol (3,), plus the Workload record."""
    wl = WORKLOADS[index]
    rng = np.random.default_rng(100 + index)
    nw = waters_per_unit(wl, rng)
    n_use = wl.n_units if n_units is None else int(n_units)
    masses_me = np.array(K.MASS_AMU) * K.AMU if masses_me is None else masses_me
    pos_l, sp_l, vel_l = [], [], []
    off = [0]
    for u in range(n_use):
        pos, sp = make_cluster(rng, int(nw[u]))
        vel = maxwell_boltzmann(rng, masses_me[sp], wl.temperature)
        pos_l.append(pos)
        sp_l.append(sp)
        vel_l.append(vel)
        off.append(off[-1] + len(sp))
    omega, k, theta, lam = mode_comb(wl.n_modes, wl.coupling)
    unit_x = (np.arange(wl.n_units)[:n_use] + 0.5) * CAVITY_LENGTH / wl.n_units
    return {
        "workload": wl,
        "species": np.concatenate(sp_l).astype(np.int8),
        "pos": np.concatenate(pos_l),
        "vel": np.concatenate(vel_l),
        "unit_off": np.array(off, dtype=np.int32),
        "unit_x": unit_x,
        "omega": omega, "k": k, "theta": theta, "lam": lam,
        "pol": np.array([0.0, 0.0, 1.0]),
        "dt": wl.dt_fs * K.FS,
    }
