"""Pins of the spectrum post-processing (host code, no GPU): the autocorrelation
against its definition written out, a sampled cosine against its own frequency,
and a harmonic polariton run through the oracle integrator against the exact
frequencies of that (linear) discrete-time map, which are where the sampled
trajectory's spectral lines lie.
"""
import numpy as np
import pytest

from oracle import cavity as cav
from oracle import md
from oracle.harmonic import HarmonicBackend
from paper_2512_03277_amd import spectra

AMU = 1822.888486
DT = 10.3353  # 0.25 fs


def test_autocorrelation_is_the_origin_average():
    rng = np.random.default_rng(1)
    x = rng.normal(size=(37, 3))
    L = 11
    dx = x - x.mean(0)
    ref = np.array([np.mean([np.mean([dx[t0 + t, k] * dx[t0, k] for t0 in range(37 - t)]) for k in range(3)])
                    for t in range(L + 1)])
    assert np.allclose(spectra.autocorrelation(x, L), ref, rtol=1e-13, atol=1e-15)


def test_cosine_line_sits_at_its_frequency():
    nu0 = 1650.0
    w0 = nu0 / spectra.HARTREE_CM
    t = np.arange(8000) * DT
    x = np.cos(w0 * t + 0.3)[:, None]
    f, I = spectra.spectrum(spectra.autocorrelation(x), DT, omega_squared=False)
    assert spectra.peak(f, I, 1000, 3000) == pytest.approx(nu0, abs=0.05)
    # the omega^2 prefactor moves the maximum up by about 2 sigma^2 / nu of the line
    f, I = spectra.spectrum(spectra.autocorrelation(x), DT)
    p = spectra.peak(f, I, 1000, 3000)
    assert 0.0 < p - nu0 < 2.0


def test_two_lines_are_resolved():
    t = np.arange(8000) * DT
    nus = (1600.0, 3700.0)
    x = sum(np.cos(nu / spectra.HARTREE_CM * t) for nu in nus)
    f, I = spectra.spectrum(spectra.autocorrelation(x), DT, omega_squared=False)
    assert spectra.peak(f, I, 1000, 2500) == pytest.approx(nus[0], abs=0.1)
    assert spectra.peak(f, I, 2500, 4500) == pytest.approx(nus[1], abs=0.1)
    assert spectra.resolution_cm(2000, DT) == pytest.approx(66.7, abs=0.1)


def _map_frequencies(be, cavity, dt):
    """Angles of the eigenvalues of the one-step map over (z, p_z, q, p_q) / dt."""
    T = np.zeros((4, 4))
    for j in range(4):
        v = np.zeros(4)
        v[j] = 1.0
        r = np.zeros((1, 3))
        p = np.zeros((1, 3))
        r[0, 2], p[0, 2] = v[0], v[1]
        ev = be.evaluate(r)
        F = cav.dipole_sums(cavity.phi, ev["mu"] @ cavity.pol)
        st = {"r": r, "p": p, "q": v[2:3].copy(), "pm": v[3:4].copy(), "ev": ev, "F": F,
              "E": cav.fields(cavity.phi, cavity.omega, cavity.lam, v[2:3], F),
              "masses": be.m.copy(), "atom_unit": np.arange(1)}
        md.step(st, be, cavity, dt)
        T[:, j] = [st["r"][0, 2], st["p"][0, 2], st["q"][0], st["pm"][0]]
    ang = np.sort(np.abs(np.angle(np.linalg.eigvals(T))))[::2]
    return ang / dt * spectra.HARTREE_CM


def test_harmonic_polariton_lines_from_an_oracle_trajectory():
    # one oscillator at 1650 cm^-1 coupled to one resonant mode: the upper and
    # lower polariton lines appear in both the dipole and the photon spectra
    w = 1650.0 / spectra.HARTREE_CM
    m = np.array([16.0 * AMU])
    be = HarmonicBackend(m, np.array([w]), np.array([0.5]), np.zeros((1, 3)))
    cavity = md.Cavity(np.array([w]), np.array([w / 137.036]), np.array([np.pi / 2]), np.array([0.4]),
                       np.array([0.0]), np.array([0.0, 0.0, 1.0]))
    lines = _map_frequencies(be, cavity, DT)
    assert lines[1] - lines[0] > 200.0  # well above the resolution of the run below
    r = np.zeros((1, 3))
    r[0, 2] = 0.05
    st = md.init_state(be, cavity, r, np.zeros((1, 3)), m, np.arange(1), photons="zero")
    z, q = [], []
    for _ in range(6000):
        md.step(st, be, cavity, DT)
        z.append(st["ev"]["mu"][0, 2])
        q.append(st["q"][0])
    for series in (np.array(z), np.array(q)):
        f, I = spectra.spectrum(spectra.autocorrelation(series), DT)
        mid = 0.5 * (lines[0] + lines[1])
        assert spectra.peak(f, I, 500.0, mid) == pytest.approx(lines[0], abs=2.0)
        assert spectra.peak(f, I, mid, 4000.0) == pytest.approx(lines[1], abs=2.0)
    rep = spectra.peak_report(np.array(z)[:, None], np.array(z)[:, None], DT, 500.0, 4000.0)
    assert rep["shift_cm"] == 0.0 and rep["centroid_shift_cm"] == 0.0


def test_per_series_spectra_and_top_peaks():
    t = np.arange(6000) * DT
    nus = (1500.0, 2200.0)
    x = np.stack([np.cos(nus[0] / spectra.HARTREE_CM * t) + 0.5 * np.cos(nus[1] / spectra.HARTREE_CM * t),
                  np.cos(nus[1] / spectra.HARTREE_CM * t)], axis=1)
    f, I = spectra.spectrum_per_series(x, DT, omega_squared=False)
    assert I.shape == (2, len(f))
    p0 = spectra.top_peaks(f, I[0], 1000.0, 3000.0, count=2)
    assert p0 == pytest.approx(list(nus), abs=0.2)
    assert spectra.top_peaks(f, I[1], 1000.0, 3000.0, count=1) == pytest.approx([nus[1]], abs=0.2)

    # a single line: its window side lobes are not reported as lines
    assert len(spectra.top_peaks(f, I[1], 1000.0, 3000.0, count=3)) == 1


def test_near_normal_average_resolves_the_polariton_pair_of_an_oracle_run():
    # harmonic cells in the oracle's real-space scheme, all displaced at random so
    # that every k is excited: the photon spectrum averaged over the modes near
    # normal incidence has its two lines at the k = 0 polariton frequencies
    from oracle import realspace as rs
    N, W, d, eta, dt = 32, 0.0075, 0.6, 0.002, DT
    m = np.full(N, 16.0 * AMU)
    be = HarmonicBackend(m, np.full(N, W), np.full(N, d), np.zeros((N, 3)))
    wk = rs.dispersion(N, W, 137.036, 1.0e6)
    cav = rs.RealSpaceCavity(eta, W, wk, np.array([0.0, 0.0, 1.0]))
    rng = np.random.default_rng(9)
    r = np.zeros((N, 3))
    r[:, 2] = rng.normal(size=N) * 0.05
    st = rs.init_state(be, cav, r, np.zeros((N, 3)), m, np.arange(N))
    qk = []
    for _ in range(6000):
        rs.step(st, be, cav, dt)
        qk.append(st["qk"].copy())
    qk = np.array(qk)
    near = np.nonzero((wk - W) * spectra.HARTREE_CM <= 10.0)[0]
    assert len(near) >= 5
    f, I = spectra.averaged_spectrum(qk, dt, near)
    g = eta * d / np.sqrt(m[0])
    H = np.array([[W ** 2 + eta ** 2 * d ** 2 / (m[0] * W ** 2), g], [g, W ** 2]])
    exact = np.sqrt(np.linalg.eigvalsh(H)) * spectra.HARTREE_CM
    lines = spectra.top_peaks(f, I, W * spectra.HARTREE_CM - 700.0, W * spectra.HARTREE_CM + 700.0, count=2)
    assert len(lines) == 2
    res = spectra.resolution_cm(6000, dt)
    assert np.allclose(lines, exact, atol=0.15 * res)
    with pytest.raises(ValueError):
        spectra.averaged_spectrum(qk, dt, [])


def test_centroid_of_a_line_and_of_two_lines():
    t = np.arange(8000) * DT
    nu0 = 1650.0
    f, I = spectra.spectrum(spectra.autocorrelation(np.cos(nu0 / spectra.HARTREE_CM * t)), DT, omega_squared=False)
    # a symmetric line centred in a symmetric window: the centroid is its centre
    assert spectra.centroid(f, I, nu0 - 300.0, nu0 + 300.0) == pytest.approx(nu0, abs=1.0)
    # two equal lines: the centroid lies midway, where neither maximum is
    x = np.cos(1600.0 / spectra.HARTREE_CM * t) + np.cos(1700.0 / spectra.HARTREE_CM * t)
    f, I = spectra.spectrum(spectra.autocorrelation(x), DT, omega_squared=False)
    assert spectra.centroid(f, I, 1350.0, 1950.0) == pytest.approx(1650.0, abs=1.0)
    with pytest.raises(ValueError):
        spectra.centroid(f, I, -2.0, -1.0)


def test_combine_spectra_averages_starts_with_fixed_band():
    # two starts of the same two-path record: each start's autocorrelations are
    # saved as the bench does, combined on the host, and the line is found at its
    # frequency with zero shift between identical paths; the band centroid is
    # taken over the fixed band, the same for both paths
    import importlib.util
    import os
    spec = importlib.util.spec_from_file_location(
        "bench_for_spectra", os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "bench.py"))
    bench = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(bench)
    t = np.arange(4000) * DT
    nu = 1650.0
    w = nu / spectra.HARTREE_CM
    per = []
    rng = np.random.default_rng(3)
    for start in (0, 1):
        x = np.cos(w * t[:, None] + rng.uniform(0, 2 * np.pi, size=(1, 6)))
        q = np.cos(1.3 * w * t[:, None] + rng.uniform(0, 2 * np.pi, size=(1, 4)))
        C, Cq = spectra.autocorrelation(x), spectra.autocorrelation(q)
        per.append({"start": start, "units_in_ir_average": 6, "C_ir_surrogate": C, "C_ir_exact": C,
                    "C_pol_surrogate": Cq, "C_pol_exact": Cq, "md_steps_per_s_surrogate": 1.0,
                    "md_steps_per_s_exact": 1.0, "bad_units_surrogate": 0, "bad_units_exact": 0,
                    "steps": len(t), "dt": DT, "units": 6})
    rep = bench.combine_spectra(per)
    assert rep["ir_peak_exact_cm"] == pytest.approx(nu, abs=2.0)
    assert rep["polariton_peak_exact_cm"] == pytest.approx(1.3 * nu, abs=3.0)
    assert rep["ir_shift_cm"] == 0.0 and rep["ir_centroid_shift_cm"] == 0.0 and rep["ir_band_cm"] == [1000.0, 4500.0]
    assert rep["ir_shift_single_starts_cm"] == [0.0, 0.0] and rep["starts"] == [0, 1]
    assert rep["ir_overlap"] == pytest.approx(1.0) and rep["polariton_overlap"] == pytest.approx(1.0)
    assert len(rep["ir_lines_exact_cm"]) >= 1 and rep["ir_lines_exact_cm"][0] == pytest.approx(nu, abs=2.0)


def test_overlap_of_spectra():
    t = np.arange(4000) * DT
    f, Ia = spectra.spectrum(spectra.autocorrelation(np.cos(1600.0 / spectra.HARTREE_CM * t)), DT,
                             omega_squared=False)
    _, Ib = spectra.spectrum(spectra.autocorrelation(np.cos(1900.0 / spectra.HARTREE_CM * t)), DT,
                             omega_squared=False)
    # the same shape at any scale overlaps fully; separated lines hardly at all
    assert spectra.overlap(f, Ia, 3.0 * Ia, 1000.0, 2500.0) == pytest.approx(1.0)
    assert spectra.overlap(f, Ia, Ib, 1000.0, 2500.0) < 0.05
    # a line against itself plus a second, equal line: 1 / sqrt(2) to within the side lobes
    assert spectra.overlap(f, Ia, Ia + Ib, 1000.0, 2500.0) == pytest.approx(2 ** -0.5, abs=0.03)
    with pytest.raises(ValueError):
        spectra.overlap(f, Ia, Ib, -2.0, -1.0)


def test_matched_line_follows_the_same_line_across_runs():
    # run b has one line; run a the same line 3 cm^-1 higher plus a stronger second
    # line: the largest values differ by the line spacing, the matched line by 3
    t = np.arange(8000) * DT
    w = 1.0 / spectra.HARTREE_CM
    xb = np.cos(1400.0 * w * t)
    xa = np.cos(1403.0 * w * t) + 1.3 * np.cos(1700.0 * w * t)
    r = spectra.report_from_acf(spectra.autocorrelation(xa), spectra.autocorrelation(xb), DT, 1000.0, 2500.0, len(t))
    assert r["shift_cm"] == pytest.approx(300.0, abs=5.0)
    assert r["matched_line_shift_cm"] == pytest.approx(3.0, abs=1.0)
