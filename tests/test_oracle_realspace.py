"""Pins of the real-space / reciprocal-space photon propagation oracle."""
import numpy as np
import pytest

from oracle import realspace as rs
from oracle.harmonic import HarmonicBackend

AMU = 1822.888486


def test_round_trip_is_identity_both_ways():
    rng = np.random.default_rng(0)
    for N in (1, 2, 7, 16):
        w0 = 0.0075
        wk = rs.dispersion(N, w0, 137.036, 5e4)
        q, p = rng.normal(size=N), rng.normal(size=N) * w0
        q2, p2 = rs.to_realspace(*rs.to_kspace(q, p, w0, wk), w0, wk)
        assert np.allclose(q2, q, rtol=0, atol=1e-13) and np.allclose(p2, p, rtol=0, atol=1e-13 * w0)
        qk, pk = rng.normal(size=N), rng.normal(size=N) * w0
        qk2, pk2 = rs.to_kspace(*rs.to_realspace(qk, pk, w0, wk), w0, wk)
        assert np.allclose(qk2, qk, rtol=0, atol=1e-13) and np.allclose(pk2, pk, rtol=0, atol=1e-13 * w0)


def test_dispersion_grid_is_symmetric_and_starts_at_omega0():
    wk = rs.dispersion(8, 0.0075, 137.036, 5e4)
    assert wk[0] == 0.0075
    k = rs.k_grid(8, 5e4)
    assert np.allclose(k[1:4], -k[7:4:-1]) and k[4] > 0      # j = 1..3 and -3..-1, then j = N/2
    assert np.allclose(wk[1:4], wk[7:4:-1])


def test_parseval_for_flat_dispersion():
    rng = np.random.default_rng(1)
    N, w0 = 9, 0.008
    q, p = rng.normal(size=N), rng.normal(size=N) * w0
    qk, pk = rs.to_kspace(q, p, w0, np.full(N, w0))
    assert 0.5 * np.sum(pk ** 2 + w0 ** 2 * qk ** 2) == pytest.approx(0.5 * np.sum(p ** 2 + w0 ** 2 * q ** 2), rel=1e-13)


def _one_cell_map(be, cav, dt):
    T = np.zeros((4, 4))
    for j in range(4):
        v = np.zeros(4)
        v[j] = 1.0
        r = np.zeros((1, 3))
        pp = np.zeros((1, 3))
        r[0, 2], pp[0, 2] = v[0], v[1]
        st = {"r": r, "p": pp, "q": v[2:3].copy(), "pn": v[3:4].copy(), "ev": be.evaluate(r),
              "masses": be.m.copy(), "atom_unit": np.arange(1)}
        rs.step(st, be, cav, dt)
        T[:, j] = [st["r"][0, 2], st["p"][0, 2], st["q"][0], st["pn"][0]]
    return T


def test_single_cell_harmonic_polariton_frequencies():
    # one cell, harmonic matter (mu = d x): the scheme is a linear map whose
    # frequencies approach those of H = p^2/2m + m W^2 x^2/2 + p_q^2/2 + w0^2 (q + eta d x / w0^2)^2 / 2,
    # mass-weighted Hessian [[W^2 + eta^2 d^2 / (m w0^2), eta d / sqrt m], [eta d / sqrt m, w0^2]]
    m = np.array([16.0 * AMU])
    W, w0, d, eta = 0.0075, 0.0078, 0.6, 0.004
    be = HarmonicBackend(m, np.array([W]), np.array([d]), np.zeros((1, 3)))
    cav = rs.RealSpaceCavity(eta, w0, np.array([w0]), np.array([0.0, 0.0, 1.0]))
    H = np.array([[W ** 2 + eta ** 2 * d ** 2 / (m[0] * w0 ** 2), eta * d / np.sqrt(m[0])],
                  [eta * d / np.sqrt(m[0]), w0 ** 2]])
    exact = np.sort(np.sqrt(np.linalg.eigvalsh(H)))
    errs = []
    for dt in (20.0, 10.0, 5.0):
        mu = np.linalg.eigvals(_one_cell_map(be, cav, dt))
        assert np.max(np.abs(np.abs(mu) - 1.0)) < 1e-10
        num = np.sort(np.abs(np.angle(mu)))[::2] / dt
        err = np.max(np.abs(num - exact) / exact)
        assert err < (exact.max() * dt) ** 2
        errs.append(err)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0


class _NoMatter:
    def __init__(self, n):
        self.n = n

    def evaluate(self, r):
        return {"energy": np.zeros(self.n), "forces": np.zeros_like(r), "mu": np.zeros((self.n, 3)),
                "Z": np.zeros((self.n, 3, 3))}


def test_free_photons_rotate_with_their_dispersion():
    rng = np.random.default_rng(2)
    N, w0, dt = 12, 0.0075, 10.0
    wk = rs.dispersion(N, w0, 137.036, 2e4)
    cav = rs.RealSpaceCavity(0.0, w0, wk, np.array([0.0, 0.0, 1.0]))
    q0, p0 = rng.normal(size=N), rng.normal(size=N) * w0
    qk0, pk0 = rs.to_kspace(q0, p0, w0, wk)
    st = {"r": np.zeros((N, 3)), "p": np.zeros((N, 3)), "q": q0.copy(), "pn": p0.copy(),
          "ev": _NoMatter(N).evaluate(np.zeros((N, 3))), "masses": np.ones(N), "atom_unit": np.arange(N)}
    for _ in range(50):
        rs.step(st, _NoMatter(N), cav, dt)
    t = 50 * dt
    assert np.allclose(st["qk"], qk0 * np.cos(wk * t) + pk0 / wk * np.sin(wk * t), rtol=0, atol=1e-11)
    assert np.allclose(st["pk"], pk0 * np.cos(wk * t) - wk * qk0 * np.sin(wk * t), rtol=0, atol=1e-11 * w0)


def _uniform_map(be, cav, N, dt):
    """One-step map over (x, p_x, q, p_q) of a state that is the same in all N
    cells; such a state stays uniform, i.e. only k = 0 is excited."""
    T = np.zeros((4, 4))
    for j in range(4):
        v = np.zeros(4)
        v[j] = 1.0
        r = np.zeros((N, 3))
        pp = np.zeros((N, 3))
        r[:, 2], pp[:, 2] = v[0], v[1]
        st = {"r": r, "p": pp, "q": np.full(N, v[2]), "pn": np.full(N, v[3]), "ev": be.evaluate(r),
              "masses": be.m.copy(), "atom_unit": np.arange(N)}
        rs.step(st, be, cav, dt)
        assert np.allclose(st["r"][:, 2], st["r"][0, 2], rtol=1e-12, atol=1e-15)
        T[:, j] = [st["r"][0, 2], st["p"][0, 2], st["q"][0], st["pn"][0]]
    return T


def test_k0_rabi_splitting_of_harmonic_cells_is_linear_in_eta():
    # N cells with resonant harmonic matter and a dispersive cavity: the k = 0
    # polariton pair has the frequencies of the one-cell 2 x 2 Hessian, and
    # their splitting grows linearly with eta (Results: splittings at eta_0,
    # 2 eta_0, 3 eta_0 in the ratio 1 : 2 : 3, as for a Jaynes-Cummings model)
    N, W, d, dt = 8, 0.0075, 0.6, 5.0
    m = np.full(N, 16.0 * AMU)
    be = HarmonicBackend(m, np.full(N, W), np.full(N, d), np.zeros((N, 3)))
    wk = rs.dispersion(N, W, 137.036, 2e4)
    splits = []
    for eta in (4e-4, 8e-4, 1.2e-3):
        cav = rs.RealSpaceCavity(eta, W, wk, np.array([0.0, 0.0, 1.0]))
        mu = np.linalg.eigvals(_uniform_map(be, cav, N, dt))
        num = np.sort(np.abs(np.angle(mu)))[::2] / dt
        g = eta * d / np.sqrt(m[0])
        H = np.array([[W ** 2 + eta ** 2 * d ** 2 / (m[0] * W ** 2), g], [g, W ** 2]])
        exact = np.sort(np.sqrt(np.linalg.eigvalsh(H)))
        assert np.max(np.abs(num - exact) / exact) < (exact.max() * dt) ** 2
        splits.append(num[1] - num[0])
        # to first order in the coupling the splitting is g / W
        assert splits[-1] == pytest.approx(g / W, rel=0.05)
    assert splits[1] / splits[0] == pytest.approx(2.0, rel=5e-3)
    assert splits[2] / splits[0] == pytest.approx(3.0, rel=5e-3)


def test_thermal_start_has_kT_over_two_per_quadratic_term():
    rng = np.random.default_rng(7)
    kT = 300.0 * 3.166811563e-6
    for N, flat in ((4096, True), (4096, False), (1000, False)):
        w0 = 0.0075
        wk = np.full(N, w0) if flat else rs.dispersion(N, w0, 137.036, 2e4)
        xi = rng.normal(size=2 * N)
        dq, dp = rs.thermal_offset(kT, xi, w0, wk)
        qk, pk = rs.to_kspace(dq, dp, w0, wk)
        kin, pot = 0.5 * pk ** 2, 0.5 * wk ** 2 * qk ** 2
        tol = 5.0 * kT / 2 * np.sqrt(2.0 / N)  # five standard errors of a mean of kT/2 chi^2_1
        assert abs(kin.mean() - kT / 2) < tol and abs(pot.mean() - kT / 2) < tol
        assert abs(np.mean(qk * pk * wk)) < 5.0 * kT / np.sqrt(N)  # q and p uncorrelated
        if flat:  # Parseval: the same equipartition per cell in real space
            assert abs(np.mean(0.5 * dp ** 2) - kT / 2) < tol
            assert abs(np.mean(0.5 * w0 ** 2 * dq ** 2) - kT / 2) < tol
    # the thermal start adds the fluctuation to the relaxed start
    be = HarmonicBackend(np.full(4, 16.0 * AMU), np.full(4, 0.0075), np.full(4, 0.6), np.zeros((4, 3)))
    r = rng.normal(size=(4, 3)) * 0.1
    cav = rs.RealSpaceCavity(1e-3, 0.0075, rs.dispersion(4, 0.0075, 137.036, 2e4), np.array([0.0, 0.0, 1.0]))
    xi = rng.normal(size=8)
    st0 = rs.init_state(be, cav, r, np.zeros((4, 3)), be.m, np.arange(4))
    st1 = rs.init_state(be, cav, r, np.zeros((4, 3)), be.m, np.arange(4), kT=kT, xi=xi)
    dq, dp = rs.thermal_offset(kT, xi, cav.omega0, cav.omega_k)
    assert np.allclose(st1["q"] - st0["q"], dq, rtol=0, atol=1e-15) and np.allclose(st1["pn"], dp, rtol=0, atol=1e-18)
