"""Pins of the oracle's Born charges, cavity model and MD integrator (CPU only)."""
import numpy as np
import pytest

from cavgen import make_system, monomer_template, mode_comb
from cavgen.constants import FS, AMU
from oracle import cavity as cav
from oracle import md
from oracle.born import born_fd, born_field, born_mulliken
from oracle.harmonic import HarmonicBackend, polariton_hessian
from oracle.scc import scc_unit


@pytest.fixture(scope="module")
def monomer_born(params):
    pos = monomer_template()
    sp = np.array([0, 1, 1])
    c = scc_unit(params, sp, pos, tol=1e-12)
    Z, st = born_fd(params, sp, pos, h=1e-3, tol=1e-12, dq_center=c["dq"])
    return pos, c, Z, st


def test_born_mulliken_is_charge_times_identity():
    q = np.array([-0.4, 0.2, 0.2])
    Z = born_mulliken(q)
    assert np.array_equal(Z[1], 0.2 * np.eye(3))


def test_born_fd_sum_rules(monomer_born):
    pos, c, Z, st = monomer_born
    assert st == 0
    # acoustic sum rule: rigid translation leaves the dipole of a neutral unit unchanged
    assert np.max(np.abs(Z.sum(0))) < 1e-5
    # rotational sum rule: sum_A Z_A (theta x R_A) = theta x mu
    mu = c["dipole"]
    for th in np.eye(3):
        lhs = sum(Z[a] @ np.cross(th, pos[a]) for a in range(3))
        assert np.max(np.abs(lhs - np.cross(th, mu))) < 1e-5
    # C2v monomer in its own frame (bisector x, plane xy): Z_O is diagonal
    ZO = Z[0]
    off = ZO - np.diag(np.diag(ZO))
    assert np.max(np.abs(off)) < 1e-8
    # H1 and H2 are mirror images under y -> -y
    Mr = np.diag([1.0, -1.0, 1.0])
    assert np.max(np.abs(Mr @ Z[1] @ Mr - Z[2])) < 1e-8


def test_field_energy_and_force_consistency(params):
    # the field term is the energy -mu . field of the Mulliken dipole: dE/dfield = -mu,
    # and the forces stay the exact negative gradient in a field
    s = make_system(1, n_units=1)
    sp, pos = s["species"], s["pos"]
    f = np.array([2e-3, -1e-3, 3e-3])
    r0 = scc_unit(params, sp, pos, tol=1e-13, field=f)
    h = 1e-5
    for a in range(3):
        e = np.zeros(3)
        e[a] = h
        ep = scc_unit(params, sp, pos, tol=1e-13, field=f + e)["energy"]
        em = scc_unit(params, sp, pos, tol=1e-13, field=f - e)["energy"]
        assert -(ep - em) / (2 * h) == pytest.approx(r0["dipole"][a], rel=1e-6, abs=1e-10)
    for (at, g) in [(0, 2), (1, 0)]:
        d = np.zeros_like(pos)
        d[at, g] = 1e-4
        ep = scc_unit(params, sp, pos + d, tol=1e-13, field=f)["energy"]
        em = scc_unit(params, sp, pos - d, tol=1e-13, field=f)["energy"]
        assert r0["forces"][at, g] == pytest.approx(-(ep - em) / 2e-4, rel=1e-6, abs=1e-9)


def test_maxwell_relation_born_equals_displacement_born(params, monomer_born):
    # two independent exact routes: dF/dfield and dmu/dR
    pos, c, Z, st = monomer_born
    Zf, stf = born_field(params, np.array([0, 1, 1]), pos, e=1e-4, tol=1e-13, dq_center=c["dq"])
    assert stf == 0
    assert np.max(np.abs(Zf - Z)) < 2e-6
    s = make_system(2, n_units=1)
    sp, p3 = s["species"][:9], s["pos"][:9]
    c3 = scc_unit(params, sp, p3, tol=1e-13)
    Zd, _ = born_fd(params, sp, p3, h=1e-3, tol=1e-13, dq_center=c3["dq"])
    Zm, _ = born_field(params, sp, p3, e=1e-4, tol=1e-13, dq_center=c3["dq"])
    assert np.max(np.abs(Zm - Zd)) < 5e-6


def _free_state(q0, p0, omega):
    return {"r": np.zeros((1, 3)), "p": np.zeros((1, 3)), "q": q0.copy(), "pm": p0.copy(),
            "masses": np.ones(1), "atom_unit": np.zeros(1, dtype=int)}


def test_free_mode_closed_form():
    omega, k, theta, lam = mode_comb(4, coupling=0.0)
    cavity = md.Cavity(omega, k, theta, lam, np.array([1000.0]), np.array([0.0, 0.0, 1.0]))
    be = HarmonicBackend(np.array([1.0]), np.array([0.01]), np.array([0.0]), np.zeros((1, 3)))
    st = md.init_state(be, cavity, np.zeros((1, 3)), np.zeros((1, 3)), np.ones(1), np.zeros(1, dtype=int),
                       photons="zero")
    q0 = np.array([0.3, -0.2, 0.1, 0.05])
    p0 = np.array([0.001, 0.002, -0.003, 0.0])
    st["q"], st["pm"] = q0.copy(), p0.copy()
    dt = 0.25 * FS
    n = 10000
    for _ in range(n):
        md.step(st, be, cavity, dt)
    t = n * dt
    q_ref = q0 * np.cos(omega * t) + p0 / omega * np.sin(omega * t)
    p_ref = p0 * np.cos(omega * t) - omega * q0 * np.sin(omega * t)
    assert np.max(np.abs(st["q"] - q_ref)) < 1e-12 * 1e3
    assert np.max(np.abs(st["pm"] - p_ref)) < 1e-12 * 1e3 * np.max(omega)


def test_single_box_special_case_matches_paper_hamiltonian():
    # one mode, one cell, phi = 1: Pauli-Fierz photon energy equals
    # omega0 a^dag a + eta q mu + eta^2 mu^2 / (2 omega0^2) with eta = lambda omega0
    rng = np.random.default_rng(0)
    for _ in range(5):
        w, lam, q, p, mu = rng.uniform(0.005, 0.02), rng.uniform(0, 0.1), rng.normal(), rng.normal(), rng.normal()
        eta = lam * w
        paper = 0.5 * (p * p + w * w * q * q) + eta * q * mu + eta ** 2 * mu ** 2 / (2 * w * w)
        ours = cav.photon_energy(np.array([q]), np.array([p]), np.array([w]), np.array([lam]), np.array([mu]))
        assert ours == pytest.approx(paper, rel=1e-13)


def _one_step_map(be, cavity, dt, n_units):
    """Matrix of the (linear) one-step map over (z_n, p_zn, q_m, p_m)."""
    M = len(cavity.omega)
    dim = 2 * n_units + 2 * M
    T = np.zeros((dim, dim))
    for j in range(dim):
        v = np.zeros(dim)
        v[j] = 1.0
        r = np.zeros((n_units, 3))
        p = np.zeros((n_units, 3))
        r[:, 2], p[:, 2] = v[:n_units], v[n_units:2 * n_units]
        ev = be.evaluate(r)
        F = cav.dipole_sums(cavity.phi, ev["mu"] @ cavity.pol)
        q, pm = v[2 * n_units:2 * n_units + M], v[2 * n_units + M:]
        st = {"r": r, "p": p, "q": q.copy(), "pm": pm.copy(), "ev": ev, "F": F,
              "E": cav.fields(cavity.phi, cavity.omega, cavity.lam, q, F),
              "masses": be.m.copy(), "atom_unit": np.arange(n_units)}
        md.step(st, be, cavity, dt)
        T[:, j] = np.concatenate([st["r"][:, 2], st["p"][:, 2], st["q"], st["pm"]])
    return T


@pytest.mark.parametrize("n_units,n_modes", [(1, 1), (3, 2)])
def test_harmonic_polariton_normal_modes(n_units, n_modes):
    rng = np.random.default_rng(n_units)
    m = np.full(n_units, 16.0 * AMU)
    w0 = np.full(n_units, 0.0075)               # ~1650 cm^-1
    dip = rng.uniform(0.3, 0.8, size=n_units)
    omega = 0.0075 + 0.0005 * np.arange(n_modes)
    lam = np.full(n_modes, 0.05)
    X = rng.uniform(0, 5e5, size=n_units)
    k = omega / 137.036
    cavity = md.Cavity(omega, k, np.zeros(n_modes), lam, X, np.array([0.0, 0.0, 1.0]))
    be = HarmonicBackend(m, w0, dip, np.zeros((n_units, 3)))
    exact = np.sort(np.sqrt(np.linalg.eigvalsh(polariton_hessian(m, w0, dip, cavity.phi, omega, lam))))
    errs = []
    for dt in (20.0, 10.0, 5.0):
        T = _one_step_map(be, cavity, dt, n_units)
        mu = np.linalg.eigvals(T)
        assert np.max(np.abs(np.abs(mu) - 1.0)) < 1e-10          # symplectic-like: no growth or decay
        num = np.sort(np.abs(np.angle(mu)))[::2] / dt
        err = np.max(np.abs(num - exact) / exact)
        assert err < (exact.max() * dt) ** 2
        errs.append(err)
    assert errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0   # second order in dt


def test_rabi_splitting_linear_in_coupling():
    m = np.array([16.0 * AMU])
    w0 = np.array([0.0075])
    dip = np.array([0.5])
    split = []
    for lam in (0.01, 0.02, 0.04):
        H = polariton_hessian(m, w0, dip, np.ones((1, 1)), np.array([0.0075]), np.array([lam]))
        f = np.sqrt(np.linalg.eigvalsh(H))
        split.append(f[1] - f[0])
    assert split[1] / split[0] == pytest.approx(2.0, rel=1e-2)
    assert split[2] / split[1] == pytest.approx(2.0, rel=1e-2)
    # resonant splitting ~ lambda * d / sqrt(m) for weak coupling
    assert split[0] == pytest.approx(0.01 * 0.5 / np.sqrt(m[0]), rel=2e-2)


@pytest.mark.slow
def test_exact_born_nve_energy_bounded_and_shrinks_with_dt(params):
    s = make_system(1, n_units=1)
    sp, unit_off = s["species"], np.array([0, 3])
    masses = params["mass"][sp]
    omega = np.array([0.0075, 0.017])
    cavity = md.Cavity(omega, omega / 137.036, np.zeros(2), np.full(2, 0.05), np.array([2.0e5]),
                       np.array([0.0, 0.0, 1.0]))
    be = md.DFTBBackend(params, sp, unit_off, born="fd", tol=1e-12)
    maxdev = []
    for dt_fs, n in ((0.5, 60), (0.25, 120)):
        st = md.init_state(be, cavity, s["pos"], s["vel"] * masses[:, None], masses, np.zeros(3, dtype=int))
        e0 = md.observables(st, cavity)["total"]
        devs = []
        for _ in range(n):
            md.step(st, be, cavity, dt_fs * FS)
            devs.append(md.observables(st, cavity)["total"] - e0)
        maxdev.append(np.max(np.abs(devs)))
        ke = md.observables(st, cavity)["kinetic"]
        assert np.max(np.abs(devs)) < 1e-2 * max(ke, 1e-3)
    assert maxdev[0] / maxdev[1] > 1.6      # first-order splitting: error at least halves


def test_forward_fd_born_is_first_order(params, monomer_born):
    # against the independent field route, the forward-difference error halves with h
    from oracle.born import born_fd_forward
    pos, c, Z, st = monomer_born
    sp = np.array([0, 1, 1])
    Zf, _ = born_field(params, sp, pos, e=1e-4, tol=1e-13, dq_center=c["dq"])
    errs = []
    for h in (4e-3, 2e-3, 1e-3):
        Zw, stw = born_fd_forward(params, sp, pos, c["dipole"], h=h, tol=1e-13, dq_center=c["dq"])
        assert stw == 0
        errs.append(np.max(np.abs(Zw - Zf)))
    assert 1.7 < errs[0] / errs[1] < 2.3 and 1.7 < errs[1] / errs[2] < 2.3
    # forward and backward (h -> -h) differences average to the central one
    Zp, _ = born_fd_forward(params, sp, pos, c["dipole"], h=1e-3, tol=1e-13, dq_center=c["dq"])
    Zm, _ = born_fd_forward(params, sp, pos, c["dipole"], h=-1e-3, tol=1e-13, dq_center=c["dq"])
    assert np.max(np.abs(0.5 * (Zp + Zm) - Z)) < 1e-8


def test_born_refresh_interval_reuses_the_tensors(params):
    s = make_system(1, n_units=2)
    be = md.DFTBBackend(params, s["species"], s["unit_off"], born="fd_forward", born_every=3)
    r = s["pos"].copy()
    Zs = []
    for k in range(4):
        Zs.append(be.evaluate(r + 0.01 * k)["Z"])
    assert np.array_equal(Zs[1], Zs[0]) and np.array_equal(Zs[2], Zs[0])
    assert not np.array_equal(Zs[3], Zs[0])
    ref = md.DFTBBackend(params, s["species"], s["unit_off"], born="fd_forward")
    assert np.array_equal(ref.evaluate(r + 0.03)["Z"], Zs[3])


def test_thermal_photon_start_is_boltzmann_about_the_relaxed_start():
    # p_m ~ N(0, kT), q_m ~ N(-lambda F / omega, kT / omega^2): the photon energy at
    # frozen matter (whose minimum is the relaxed start) has kT/2 per quadratic term
    rng = np.random.default_rng(11)
    n_units, M = 6, 4096
    kT = 300.0 * 3.166811563e-6
    m = np.full(n_units, 16.0 * AMU)
    be = HarmonicBackend(m, np.full(n_units, 0.0075), rng.uniform(0.3, 0.8, n_units), np.zeros((n_units, 3)))
    omega, k, theta, lam = mode_comb(M)
    cavity = md.Cavity(omega, k, theta, lam, rng.uniform(0, 5e5, n_units), np.array([0.0, 0.0, 1.0]))
    r = rng.normal(size=(n_units, 3)) * 0.05
    xi = rng.normal(size=2 * M)
    st0 = md.init_state(be, cavity, r, np.zeros((n_units, 3)), m, np.arange(n_units))
    st = md.init_state(be, cavity, r, np.zeros((n_units, 3)), m, np.arange(n_units), photons="thermal", kT=kT, xi=xi)
    assert cav.photon_energy(st0["q"], st0["pm"], omega, cavity.lam, st0["F"]) == pytest.approx(0.0, abs=1e-20)
    kin = 0.5 * st["pm"] ** 2
    pot = 0.5 * (omega * (st["q"] + cavity.lam * st["F"] / omega)) ** 2
    tol = 5.0 * kT / 2 * np.sqrt(2.0 / M)
    assert abs(kin.mean() - kT / 2) < tol and abs(pot.mean() - kT / 2) < tol
    total = cav.photon_energy(st["q"], st["pm"], omega, cavity.lam, st["F"])
    assert total == pytest.approx(kin.sum() + pot.sum(), rel=1e-12)
    # kT = 0 is the relaxed start
    st_cold = md.init_state(be, cavity, r, np.zeros((n_units, 3)), m, np.arange(n_units), photons="thermal", kT=0.0,
                            xi=xi)
    assert np.array_equal(st_cold["q"], st0["q"]) and not np.any(st_cold["pm"])


def test_unit_temperature_matches_equipartition():
    # Momenta drawn here from the Maxwell-Boltzmann distribution at 300 K
    # (p ~ N(0, m kT) per component, no centre-of-mass correction) for units of
    # 1, 2 and 5 atoms-of-water sizes.  With the centre-of-mass motion removed
    # a unit keeps 3 N - 3 quadratic momentum terms, so equipartition gives
    # <2 KE_rel / ((3N - 3) k_B)> = T exactly.  Counting 3N terms, or keeping the
    # centre-of-mass motion, biases the mean by a factor (3N-3)/3N or 3N/(3N-3)
    # (x0.67 / x1.5 for a monomer); the statistical error here is 0.3 %.
    from cavgen.constants import KB, MASS_AMU
    rng = np.random.default_rng(2024)
    T = 300.0
    for waters, n_units in ((1, 20000), (2, 10000), (5, 4000)):
        sp = np.tile([0, 1, 1], waters)
        na = len(sp)
        unit_off = np.arange(n_units + 1) * na
        m_unit = np.array(MASS_AMU)[sp] * AMU
        m = np.tile(m_unit, n_units)
        p = rng.normal(size=(n_units * na, 3)) * np.sqrt(m * KB * T)[:, None]
        st = {"p": p, "masses": m, "q": np.zeros(1), "pm": np.zeros(1), "F": np.zeros(1),
              "ev": {"energy": np.zeros(n_units)}}
        cavity = md.Cavity(np.ones(1), np.zeros(1), np.zeros(1), np.zeros(1), np.zeros(n_units),
                           np.array([0.0, 0.0, 1.0]))
        got = md.observables(st, cavity, unit_off)["temperature"]
        dof = 3 * na - 3
        sigma = T * np.sqrt(2.0 / (dof * n_units))
        assert abs(got - T) < 4.0 * sigma, (waters, got, sigma)
        assert abs(got - T * dof / (3 * na)) > 10 * sigma and abs(got - T * 3 * na / dof) > 10 * sigma
