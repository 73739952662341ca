"""GPU parity of the real-space / reciprocal-space photon propagation against
the oracle (oracle/realspace.py): full MD steps with SCC-DFTB matter for a
power-of-two cell count (FFT stages) and for another count (direct sums), and
free photons at 1024 cells rotating exactly with their dispersion.
"""
import numpy as np
import pytest

from cavgen import make_params, make_system
from oracle import md as omd
from oracle import realspace as ors

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2512_03277_amd as cd  # noqa: E402

DEV = torch.device("cuda:0")
ETA, W0, C, A = 0.01, 0.0075, 137.036, 1.0e4


@pytest.fixture(scope="module")
def params():
    return make_params()


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


def _subsystem(s, units):
    off = s["unit_off"]
    idx = np.concatenate([np.arange(off[u], off[u + 1]) for u in units])
    out = dict(s)
    out.update({"species": s["species"][idx], "pos": s["pos"][idx], "vel": s["vel"][idx],
                "unit_off": np.concatenate([[0], np.cumsum([off[u + 1] - off[u] for u in units])]).astype(np.int32),
                "unit_x": s["unit_x"][list(units)]})
    return out


@pytest.mark.parametrize("units", [list(range(8)), [0, 2, 3, 5, 7]])
def test_realspace_md_steps_match_the_oracle(params, units):
    s = _subsystem(make_system(1), units)
    n, steps = len(units), 3
    masses = params["mass"][s["species"]]
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-12, 300, 0.2)
    ctx.set_realspace_cavity(ETA, W0, C, A)
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qn = torch.zeros(n, dtype=torch.float64, device=DEV)
    pn = torch.zeros_like(qn)
    rec = torch.zeros(steps, n, dtype=torch.float64, device=DEV)
    obs = torch.zeros(steps, cd.N_OBS, dtype=torch.float64, device=DEV)
    ctx.init_photons_realspace(r, qn, pn)
    ctx.step_realspace(r, p, qn, pn, steps, s["dt"], cd.BORN_MULLIKEN, 0.0, obs, rec)
    assert ctx.sync() == 0
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="mulliken", tol=1e-12)
    cav = ors.RealSpaceCavity(ETA, W0, ors.dispersion(n, W0, C, A), s["pol"])
    atom_unit = np.repeat(np.arange(n), np.diff(s["unit_off"]))
    st = ors.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    qk_ref = []
    for _ in range(steps):
        ors.step(st, be, cav, s["dt"])
        qk_ref.append(st["qk"].copy())
    assert _rel(r.cpu().numpy(), st["r"]) <= 1e-9 and _rel(p.cpu().numpy(), st["p"]) <= 1e-8
    assert _rel(qn.cpu().numpy(), st["q"]) <= 1e-8 and _rel(pn.cpu().numpy(), st["pn"]) <= 1e-8
    assert _rel(rec.cpu().numpy(), np.array(qk_ref)) <= 1e-8
    o = obs.cpu().numpy()[-1]
    mu = st["ev"]["mu"] @ np.asarray(s["pol"])
    assert o[2] == pytest.approx(ors.photon_energy(st["q"], st["pn"], mu, cav), rel=1e-8, abs=1e-12)
    ctx.close()


@pytest.mark.parametrize("n", [1024, 3000])
def test_free_photons_rotate_with_their_dispersion_at_scale(params, n):
    # 1024 cells: radix-2 transform stages; 3000 cells: direct sums
    s = make_system(5, n_units=n)
    steps = 40
    masses = params["mass"][s["species"]]
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-10, 200, 0.2)
    ctx.set_realspace_cavity(0.0, W0, C, A)  # eta = 0: matter and photons decouple
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qn = torch.zeros(n, dtype=torch.float64, device=DEV)
    pn = torch.zeros_like(qn)
    ctx.init_photons_realspace(r, qn, pn)
    rng = np.random.default_rng(4)
    q0, p0 = rng.normal(size=n), rng.normal(size=n) * W0
    qn.copy_(_t(q0))
    pn.copy_(_t(p0))
    rec = torch.zeros(steps, n, dtype=torch.float64, device=DEV)
    ctx.step_realspace(r, p, qn, pn, steps, s["dt"], cd.BORN_MULLIKEN, 0.0, None, rec)
    ctx.sync()
    wk = ors.dispersion(n, W0, C, A)
    qk0, pk0 = ors.to_kspace(q0, p0, W0, wk)
    t = steps * s["dt"]
    ref = qk0 * np.cos(wk * t) + pk0 / wk * np.sin(wk * t)
    assert np.max(np.abs(rec.cpu().numpy()[-1] - ref)) <= 1e-11 * np.max(np.abs(ref))
    ctx.close()


def test_realspace_cavity_rejects_large_non_power_of_two(params):
    s = make_system(5, n_units=4100)
    ctx = cd.context_from_system(params, s)
    with pytest.raises(RuntimeError):
        ctx.set_realspace_cavity(ETA, W0, C, A)
    ctx.close()


@pytest.mark.parametrize("units", [list(range(8)), [0, 2, 3, 5, 7]])
def test_thermal_realspace_start_and_steps_match_the_oracle(params, units):
    s = _subsystem(make_system(1), units)
    n, steps = len(units), 2
    kT = 300.0 * 3.166811563e-6
    masses = params["mass"][s["species"]]
    xi = np.random.default_rng(5).normal(size=2 * n)
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-12, 300, 0.2)
    ctx.set_realspace_cavity(ETA, W0, C, A)
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qn = torch.zeros(n, dtype=torch.float64, device=DEV)
    pn = torch.zeros_like(qn)
    ctx.init_photons_realspace_thermal(r, qn, pn, kT, _t(xi))
    assert ctx.sync() == 0
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="mulliken", tol=1e-12)
    cav = ors.RealSpaceCavity(ETA, W0, ors.dispersion(n, W0, C, A), s["pol"])
    atom_unit = np.repeat(np.arange(n), np.diff(s["unit_off"]))
    st = ors.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit, kT=kT, xi=xi)
    assert _rel(qn.cpu().numpy(), st["q"]) <= 1e-10 and _rel(pn.cpu().numpy(), st["pn"]) <= 1e-10
    ctx.step_realspace(r, p, qn, pn, steps, s["dt"], cd.BORN_MULLIKEN, 0.0, None, None)
    assert ctx.sync() == 0
    for _ in range(steps):
        ors.step(st, be, cav, s["dt"])
    assert _rel(r.cpu().numpy(), st["r"]) <= 1e-9 and _rel(p.cpu().numpy(), st["p"]) <= 1e-8
    assert _rel(qn.cpu().numpy(), st["q"]) <= 1e-8 and _rel(pn.cpu().numpy(), st["pn"]) <= 1e-8
    with pytest.raises(RuntimeError):
        ctx.init_photons_realspace_thermal(r, qn, pn, -1.0, _t(xi))
    ctx.close()


def test_thermal_mode_start_matches_the_oracle(params):
    s = make_system(1)
    masses = params["mass"][s["species"]]
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-12, 300, 0.2)
    M = ctx.n_modes
    kT = 300.0 * 3.166811563e-6
    xi = np.random.default_rng(6).normal(size=2 * M)
    r = _t(s["pos"])
    qm = torch.zeros(M, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    ctx.init_photons_thermal(r, qm, pm, kT, _t(xi))
    assert ctx.sync() == 0
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="mulliken", tol=1e-12)
    cavity = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cavity, s["pos"], s["vel"] * masses[:, None], masses, atom_unit, photons="thermal",
                        kT=kT, xi=xi)
    assert _rel(qm.cpu().numpy(), st["q"]) <= 1e-10 and _rel(pm.cpu().numpy(), st["pm"]) <= 1e-12
    with pytest.raises(RuntimeError):
        ctx.init_photons_thermal(r, qm, pm, float("nan"), _t(xi))
    ctx.close()


def _rs_run(params, s, eta, steps):
    n = len(s["unit_off"]) - 1
    masses = params["mass"][s["species"]]
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-12, 300, 0.2)
    ctx.set_realspace_cavity(eta, W0, C, A)
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qn = torch.zeros(n, dtype=torch.float64, device=DEV)
    pn = torch.zeros_like(qn)
    rec = torch.zeros(steps, n, dtype=torch.float64, device=DEV)
    ctx.init_photons_realspace(r, qn, pn)
    ctx.step_realspace(r, p, qn, pn, steps, s["dt"], cd.BORN_MULLIKEN, 0.0, None, rec)
    assert ctx.sync() == 0
    out = (p.cpu().numpy(), rec.cpu().numpy())
    ctx.close()
    return out


def test_realspace_eta_sweep_matches_the_oracle_and_responds_linearly(params):
    # the coupling sweep of the Rabi-splitting study on the GPU: at each eta the
    # device scheme equals the oracle's (whose k = 0 polariton pair splits
    # linearly in eta on harmonic cells, tests/test_oracle_realspace.py), and the
    # photon response the matter drives is linear in eta: after a few steps from
    # the relaxed photon start, q_k(eta) / eta is the same at eta, 2 eta and 4 eta
    # up to a correction of relative size 4e-5 here; the response is odd in eta
    # (eta -> -eta, q -> -q), so that correction is of order eta^2 and grows
    # fourfold per doubling (3.99 in the oracle)
    s = _subsystem(make_system(1), list(range(8)))
    n, steps = 8, 4
    masses = params["mass"][s["species"]]
    recs = {}
    for eta in (2.5e-3, 5e-3, 1e-2):
        p_g, rec = _rs_run(params, s, eta, steps)
        be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="mulliken", tol=1e-12)
        cav = ors.RealSpaceCavity(eta, W0, ors.dispersion(n, W0, C, A), s["pol"])
        atom_unit = np.repeat(np.arange(n), np.diff(s["unit_off"]))
        st = ors.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
        qk = []
        for _ in range(steps):
            ors.step(st, be, cav, s["dt"])
            qk.append(st["qk"].copy())
        assert _rel(p_g, st["p"]) <= 1e-8 and _rel(rec, np.array(qk)) <= 1e-8
        recs[eta] = rec
    r1, r2, r4 = recs[2.5e-3] / 2.5e-3, recs[5e-3] / 5e-3, recs[1e-2] / 1e-2
    d12, d24 = np.max(np.abs(r2 - r1)), np.max(np.abs(r4 - r2))
    assert d12 <= 1e-3 * np.max(np.abs(r1))                 # linear to 0.1 %
    assert d24 == pytest.approx(4.0 * d12, rel=0.1)         # the deviation is of order eta^2
