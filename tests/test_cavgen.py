"""Seeded input generator: determinism, geometry and the printed-coupling fixture."""
import os

import numpy as np
import pytest

from cavgen import make_params, make_system, monomer_template, mode_comb
from cavgen import constants as K
from oracle.harmonic import polariton_hessian

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_deterministic_and_prefix_stable():
    a = make_system(4, n_units=12)
    b = make_system(4, n_units=12)
    for k in ("pos", "vel", "species", "unit_off"):
        assert np.array_equal(a[k], b[k])
    c = make_system(4, n_units=5)
    assert np.array_equal(c["pos"], a["pos"][:c["unit_off"][-1]])
    p1, p2 = make_params(), make_params()
    assert np.array_equal(p1["sk"], p2["sk"])


def test_geometry_and_velocities():
    t = monomer_template()
    assert np.linalg.norm(t[1] - t[0]) == pytest.approx(0.96 * K.ANGSTROM)
    v1, v2 = t[1] - t[0], t[2] - t[0]
    ang = np.degrees(np.arccos(v1 @ v2 / np.linalg.norm(v1) / np.linalg.norm(v2)))
    assert ang == pytest.approx(104.5)
    s = make_system(2, n_units=3)
    m = np.array(K.MASS_AMU)[s["species"]] * K.AMU
    for u in range(3):
        a0, a1 = s["unit_off"][u], s["unit_off"][u + 1]
        pos = s["pos"][a0:a1]
        mol = np.arange(a1 - a0) // 3
        d = np.linalg.norm(pos[:, None] - pos[None], axis=-1)
        assert d[mol[:, None] != mol[None]].min() >= 1.5 * K.ANGSTROM
        assert np.max(np.abs((m[a0:a1, None] * s["vel"][a0:a1]).sum(0))) < 1e-12
    w, k, th, lam = mode_comb(16)
    assert w[0] * K.HARTREE_CM == pytest.approx(1500) and w[-1] * K.HARTREE_CM == pytest.approx(4000)


def test_printed_rabi_splittings_are_linear_in_eta():
    rows = np.loadtxt(os.path.join(GOLDEN, "rabi_splitting_linear.txt"))
    eta_mult, split_ev = rows[:, 0], rows[:, 1]
    # the paper's numbers are linear through the origin ...
    assert np.allclose(split_ev / eta_mult, split_ev[0], rtol=1e-12)
    # ... and so is the harmonic polariton of the cavity model at resonance
    w0 = 0.19 / 27.211386
    m = np.array([1.0])
    sim = []
    for e in eta_mult:
        lam = e * 1e-4 / w0          # eta = lambda omega0 (single-box case)
        f = np.sqrt(np.linalg.eigvalsh(polariton_hessian(m, [w0], [1.0], np.ones((1, 1)), np.array([w0]),
                                                        np.array([lam]))))
        sim.append(f[1] - f[0])
    sim = np.array(sim)
    assert np.allclose(sim / sim[0], split_ev / split_ev[0], rtol=1e-3)
