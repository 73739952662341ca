"""Pins of the oracle's SCC-DFTB unit evaluation (CPU only)."""
import numpy as np
import pytest
from scipy.linalg import eigh as gen_eigh

from cavgen import make_system, monomer_template
from oracle.scc import scc_unit


@pytest.fixture(scope="module")
def cluster():
    s = make_system(2, n_units=1)
    return s["species"], s["pos"]


@pytest.fixture(scope="module")
def conv(params, cluster):
    return scc_unit(params, *cluster, tol=1e-12)


def test_eigen_residual_and_orthonormality(conv):
    H, S, C, eps = conv["H"], conv["S"], conv["C"], conv["eps"]
    assert conv["status"] == 0
    assert np.max(np.abs(H @ C - S @ C * eps)) <= 1e-12 * np.max(np.abs(H))
    assert np.max(np.abs(C.T @ S @ C - np.eye(len(eps)))) < 1e-12
    assert np.all(np.diff(eps) >= 0)


def test_density_trace_idempotency_neutrality(conv, cluster):
    P, S = conv["P"], conv["S"]
    n_el = 8.0 * 8
    assert np.trace(P @ S) == pytest.approx(n_el, abs=1e-11)
    assert np.max(np.abs(P @ S @ P - 2.0 * P)) < 1e-12
    assert abs(conv["dq"].sum()) < 1e-11
    assert np.array_equal(conv["P"], conv["P"].T) or np.max(np.abs(P - P.T)) < 1e-15


def test_fixed_point_independent_of_mixer_and_start(params, cluster, conv):
    lin = scc_unit(params, *cluster, tol=1e-12, mixer="linear", mix_alpha=0.1, max_iter=2000)
    rng = np.random.default_rng(5)
    start = rng.normal(scale=0.2, size=len(cluster[0]))
    start -= start.mean()
    other = scc_unit(params, *cluster, tol=1e-12, dq_start=start)
    assert lin["status"] == 0 and other["status"] == 0
    assert np.max(np.abs(lin["dq"] - conv["dq"])) < 1e-11
    assert np.max(np.abs(other["dq"] - conv["dq"])) < 1e-11
    assert lin["energy"] == pytest.approx(conv["energy"], abs=1e-11)


def test_non_scc_limit_is_one_generalised_diagonalisation(params, cluster):
    r = scc_unit(params, *cluster, tol=1e-13, gamma_scale=0.0)
    H0, S = r["H0"], r["S"]
    w, C = gen_eigh(H0, S)          # library special case: the plain tight-binding problem
    nocc = r["n_occ"]
    P = 2.0 * C[:, :nocc] @ C[:, :nocc].T
    assert np.max(np.abs(P - r["P"])) < 1e-12
    assert np.max(np.abs(w - r["eps"])) < 1e-12


def test_monomer_equilibrium_and_sum_rules(params, conv, cluster):
    m = scc_unit(params, np.array([0, 1, 1]), monomer_template(), tol=1e-13)
    assert np.max(np.abs(m["forces"])) < 1e-10         # repulsion fitted at the template geometry
    F = conv["forces"]
    pos = cluster[1]
    assert np.max(np.abs(F.sum(0))) < 1e-11            # translation
    assert np.max(np.abs(np.cross(pos, F).sum(0))) < 1e-10   # rotation (isolated unit, no field)


@pytest.mark.slow
def test_forces_are_minus_energy_gradient(params):
    s = make_system(2, n_units=1)
    sp, pos = s["species"][:9], s["pos"][:9]     # three molecules of the cluster
    r0 = scc_unit(params, sp, pos, tol=1e-13)
    h = 1e-4
    rng = np.random.default_rng(3)
    for (a, g) in [(0, 0), (1, 2), (4, 1), (8, 0), (6, 2)]:
        e = np.zeros_like(pos)
        e[a, g] = h
        ep = scc_unit(params, sp, pos + e, tol=1e-13, dq_start=r0["dq"])["energy"]
        em = scc_unit(params, sp, pos - e, tol=1e-13, dq_start=r0["dq"])["energy"]
        fd = -(ep - em) / (2 * h)
        assert r0["forces"][a, g] == pytest.approx(fd, rel=1e-6, abs=1e-9)
    del rng


def test_energy_invariant_under_rigid_motion(params, cluster, conv):
    q, _ = np.linalg.qr(np.random.default_rng(2).normal(size=(3, 3)))
    pos2 = cluster[1] @ q.T + 1.7
    r2 = scc_unit(params, cluster[0], pos2, tol=1e-12)
    assert r2["energy"] == pytest.approx(conv["energy"], abs=1e-11)
    assert np.max(np.abs(r2["dq"] - conv["dq"])) < 1e-11
    assert np.max(np.abs(r2["forces"] - conv["forces"] @ q.T)) < 1e-10
    assert np.max(np.abs(r2["dipole"] - conv["dipole"] @ q.T)) < 1e-10


def test_nan_position_flagged(params):
    pos = monomer_template().copy()
    pos[1, 0] = np.nan
    assert scc_unit(params, np.array([0, 1, 1]), pos)["status"] & 8
