"""Pins of the oracle's Slater-Koster assembly and gamma kernel (CPU only).

Each check is fixed by something other than the oracle itself: the textbook
diatomic special case, rotation/permutation invariance, finite differences and
the closed-form limits of the Elstner kernel."""
import math

import numpy as np
import pytest
from scipy.linalg import eigh as gen_eigh

from cavgen import make_system
from oracle.gamma import gamma_r, gamma_matrix, tau_of
from oracle.sk import build_h0_s, pair_blocks


def _table(params, t, r):
    a, b, c, d = params["sk"][t]
    return a * math.exp(-b * r), c * math.exp(-d * r)


@pytest.mark.parametrize("r", [1.3, 2.7, 5.9])
def test_diatomic_along_z_gives_table_values(params, r):
    # O-O along +z: <s|s>=ss, <s|pz>=sp, <pz|s>=-sp, <pz|pz>=pp sigma, <px|px>=pp pi
    H, S = pair_blocks(params, 0, 0, np.array([0.0, 0.0, r]))
    for M, k in ((H, 0), (S, 1)):
        ss = _table(params, 0, r)[k]
        sp = _table(params, 1, r)[k]
        pps = _table(params, 2, r)[k]
        ppp = _table(params, 3, r)[k]
        assert M[0, 0] == pytest.approx(ss, rel=1e-14)
        assert M[0, 3] == pytest.approx(sp, rel=1e-14)
        assert M[3, 0] == pytest.approx(-sp, rel=1e-14)
        assert M[3, 3] == pytest.approx(pps, rel=1e-14)
        assert M[1, 1] == pytest.approx(ppp, rel=1e-14)
        assert M[2, 2] == pytest.approx(ppp, rel=1e-14)
        assert M[0, 1] == 0 and M[1, 2] == 0 and M[1, 3] == 0
    # H above O: <s_H|pz_O> with direction H->O = -z
    H, S = pair_blocks(params, 1, 0, np.array([0.0, 0.0, -r]))
    assert H[0, 0] == pytest.approx(_table(params, 4, r)[0], rel=1e-14)
    assert H[0, 3] == pytest.approx(-_table(params, 5, r)[0], rel=1e-14)
    Hb, _ = pair_blocks(params, 0, 1, np.array([0.0, 0.0, r]))
    assert np.allclose(Hb, H.T, rtol=1e-14, atol=0)
    Hh, Sh = pair_blocks(params, 1, 1, np.array([0.0, r, 0.0]))
    assert Hh[0, 0] == pytest.approx(_table(params, 6, r)[0], rel=1e-14)


def _rot(seed):
    rng = np.random.default_rng(seed)
    q, _ = np.linalg.qr(rng.normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_h0_s_symmetric_and_invariant(params):
    s = make_system(2, n_units=1)
    sp, pos = s["species"], s["pos"]
    H0, S = build_h0_s(params, sp, pos)
    assert np.array_equal(H0, H0.T) and np.array_equal(S, S.T)
    assert np.all(np.diag(S) == 1.0)
    ev = gen_eigh(H0, S, eigvals_only=True)
    # rigid rotation + translation
    R = _rot(7)
    pos2 = pos @ R.T + np.array([3.0, -1.0, 0.5])
    ev2 = gen_eigh(*build_h0_s(params, sp, pos2), eigvals_only=True)
    assert np.max(np.abs(ev - ev2)) < 1e-12
    # permutation of the molecules (atom order) must not change the spectrum
    perm = np.concatenate([np.arange(3 * i, 3 * i + 3) for i in (5, 2, 7, 0, 1, 6, 3, 4)])
    ev3 = gen_eigh(*build_h0_s(params, sp[perm], pos[perm]), eigvals_only=True)
    assert np.max(np.abs(ev - ev3)) < 1e-12
    # swapping O/H order inside a pair: block(B,A) = block(A,B)^T
    d = pos[4] - pos[0]
    Hab, Sab = pair_blocks(params, sp[0], sp[4], d)
    Hba, Sba = pair_blocks(params, sp[4], sp[0], -d)
    assert np.allclose(Hab, Hba.T, rtol=0, atol=1e-16) and np.allclose(Sab, Sba.T, rtol=0, atol=1e-16)


@pytest.mark.parametrize("pair", [(0, 0), (0, 1), (1, 0), (1, 1)])
def test_sk_derivatives_central_fd(params, pair):
    rng = np.random.default_rng(11)
    d = rng.normal(size=3)
    d *= 2.4 / np.linalg.norm(d)
    _, _, dH, dS = pair_blocks(params, pair[0], pair[1], d, deriv=True)
    h = 1e-5
    for g in range(3):
        e = np.zeros(3)
        e[g] = h
        Hp, Sp = pair_blocks(params, pair[0], pair[1], d + e)
        Hm, Sm = pair_blocks(params, pair[0], pair[1], d - e)
        assert np.allclose((Hp - Hm) / (2 * h), dH[g], rtol=1e-7, atol=1e-10)
        assert np.allclose((Sp - Sm) / (2 * h), dS[g], rtol=1e-7, atol=1e-10)


def test_gamma_limits(params):
    uO, uH = params["hubbard_u"]
    # equal exponents: gamma(R->0) -> U
    for u in (uO, uH):
        g, _ = gamma_r(u, u, 1e-4)
        assert g == pytest.approx(u, abs=1e-6)
    # unequal exponents: closed form of the R->0 limit of two Slater densities
    ta, tb = tau_of(uO), tau_of(uH)
    g0 = 0.5 * (ta * tb / (ta + tb) + ta ** 2 * tb ** 2 / (ta + tb) ** 3)
    assert g0 == pytest.approx(0.4558, abs=1e-4)
    g, _ = gamma_r(uO, uH, 2e-3)
    assert g == pytest.approx(g0, abs=1e-5)
    # point charges at large R, symmetry in (A, B), monotone decrease
    for (a, b) in ((uO, uO), (uO, uH), (uH, uH)):
        g, _ = gamma_r(a, b, 20.0)
        assert abs(g - 1 / 20.0) < 1e-9
        assert gamma_r(a, b, 3.1)[0] == gamma_r(b, a, 3.1)[0] or \
            abs(gamma_r(a, b, 3.1)[0] - gamma_r(b, a, 3.1)[0]) < 1e-15
        vals = [gamma_r(a, b, r)[0] for r in np.linspace(0.5, 12, 30)]
        assert np.all(np.diff(vals) < 0)
        assert all(0 < v < 1 / r for v, r in zip(vals, np.linspace(0.5, 12, 30)))


@pytest.mark.parametrize("pair", [(0.5, 0.5), (0.5, 0.42), (0.42, 0.42)])
def test_gamma_derivative_fd(pair):
    for r in (1.1, 1.8, 2.9, 5.7):
        _, dg = gamma_r(pair[0], pair[1], r)
        h = 1e-5
        fd = (gamma_r(pair[0], pair[1], r + h)[0] - gamma_r(pair[0], pair[1], r - h)[0]) / (2 * h)
        assert dg == pytest.approx(fd, rel=1e-7, abs=1e-11)


def test_gamma_matrix_onsite(params):
    s = make_system(1, n_units=1)
    G = gamma_matrix(params, s["species"], s["pos"])
    assert G[0, 0] == 0.5 and G[1, 1] == 0.42 and np.array_equal(G, G.T)


def _gamma_fourier(ua, ub, r):
    """Coulomb integral of two normalised exponential densities
    rho(x) = tau^3 e^{-tau |x|} / (8 pi) by quadrature in Fourier space:
    rho^(k) = (1 + k^2/tau^2)^-2 and
      gamma(R)    = (2/pi) int_0^inf rho_a^ rho_b^ sin(kR)/(kR) dk,
      dgamma/dR   = (2/pi) int_0^inf rho_a^ rho_b^ [cos(kR)/R - sin(kR)/(k R^2)] dk,
    Gauss-Legendre (40 nodes) on panels no wider than 0.5 and pi/R, up to
    k = 200 (the integrand falls as k^-9; the tail is below 1e-17)."""
    ta, tb = tau_of(ua), tau_of(ub)
    w = min(0.5, math.pi / r)
    edges = np.arange(0.0, 200.0 + w, w)
    x, wt = np.polynomial.legendre.leggauss(40)
    half = 0.5 * np.diff(edges)
    k = (0.5 * (edges[1:] + edges[:-1]))[:, None] + half[:, None] * x[None, :]
    wk = half[:, None] * wt[None, :]
    f = (1.0 + k * k / (ta * ta)) ** -2 * (1.0 + k * k / (tb * tb)) ** -2
    kr = k * r
    g = 2.0 / math.pi * np.sum(wk * f * np.sin(kr) / kr)
    dg = 2.0 / math.pi * np.sum(wk * f * (np.cos(kr) / r - np.sin(kr) / (kr * r)))
    return g, dg


@pytest.mark.parametrize("pair", [(0.5, 0.5), (0.5, 0.42), (0.42, 0.42), (0.5, 0.5 * (1 + 1e-6)),
                                  (0.5, 0.5 * (1 + 2e-7)), (0.5, 0.5 * (1 + 1e-3)), (0.3, 0.9)])
@pytest.mark.parametrize("r", [0.3, 1.0, 2.0, 4.0])
def test_gamma_against_fourier_quadrature(pair, r):
    # fixes the whole curve at finite R, not only its limits: a wrong term of
    # either closed form, or cancellation at near-equal exponents, fails here
    g, dg = gamma_r(pair[0], pair[1], r)
    gq, dgq = _gamma_fourier(pair[0], pair[1], r)
    assert abs(g - gq) <= 2e-13 and abs(dg - dgq) <= 2e-13, (g, gq, dg, dgq)


@pytest.mark.parametrize("x_switch", [1e-9, 0.15])
@pytest.mark.parametrize("r", [0.7, 1.9, 3.6])
def test_gamma_continuous_across_branch_switches(x_switch, r):
    # exponents ta = t (1 + x), tb = t (1 - x) just below and just above each
    # switch of the evaluation (x -+ 1e-12 x): the jump between the two sides
    # equals the change along the curve (slope from a wide central difference
    # on one side) to rounding
    t = 1.4

    def g_at(x):
        return gamma_r(t * (1 + x) * 5 / 16, t * (1 - x) * 5 / 16, r)

    lo, hi = g_at(x_switch * (1 - 1e-12)), g_at(x_switch * (1 + 1e-12))
    dx = 2e-12 * x_switch
    for c in (0, 1):
        slope = (g_at(x_switch * 1.02)[c] - g_at(x_switch * 1.01)[c]) / (0.01 * x_switch)
        assert abs(hi[c] - lo[c] - slope * dx) <= 1e-14, (c, hi[c] - lo[c], slope * dx)
    gq, dgq = _gamma_fourier(t * (1 + x_switch) * 5 / 16, t * (1 - x_switch) * 5 / 16, r)
    assert abs(hi[0] - gq) <= 2e-13 and abs(hi[1] - dgq) <= 2e-13
