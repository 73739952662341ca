"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Bars (parity mode, SCC tol 1e-12): energies rel 1e-12, forces max-abs
<= 1e-9 x max|F|, Mulliken charges abs 1e-10 e, dipoles 1e-10 x sum_A |R_A|
(the charge bar carried through mu = sum Q R), finite-
difference Born charges abs 1e-8 e, cavity sums rel 1e-12, one MD step rel 1e-9.
"""
import numpy as np
import pytest

from cavgen import make_params, make_system, mode_comb
from cavgen.systems import CAVITY_LENGTH
from oracle import cavity as ocav
from oracle import md as omd
from oracle.born import born_fd, born_fd_forward, born_field
from oracle.scc import eval_units, scc_unit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2512_03277_amd as cd  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def subsystem(s, units):
    """CSR system made of the listed units of s (same cavity)."""
    off = s["unit_off"]
    idx = np.concatenate([np.arange(off[u], off[u + 1]) for u in units])
    new_off = np.concatenate([[0], np.cumsum([off[u + 1] - off[u] for u in units])]).astype(np.int32)
    out = dict(s)
    out.update({"species": s["species"][idx], "pos": s["pos"][idx], "vel": s["vel"][idx], "unit_off": new_off,
                "unit_x": s["unit_x"][list(units)]})
    return out


def gpu_eval(ctx, pos):
    U, NA = ctx.n_units, ctx.n_atoms
    out = {"energy": torch.zeros(U, dtype=torch.float64, device=DEV),
           "forces": torch.zeros(NA, 3, dtype=torch.float64, device=DEV),
           "charges": torch.zeros(NA, dtype=torch.float64, device=DEV),
           "dipole": torch.zeros(U, 3, dtype=torch.float64, device=DEV),
           "status": torch.zeros(U, dtype=torch.int32, device=DEV)}
    ctx.eval_units(_t(pos), out["energy"], out["forces"], out["charges"], out["dipole"], out["status"])
    ctx.sync()
    return {k: v.cpu().numpy() for k, v in out.items()}


def assert_parity(g, r, frel=1e-9, qabs=1e-10, erel=1e-12, pos=None, unit_off=None):
    """The dipole bar follows from the charge bar: |d mu_n| <= qabs * sum_A |R_A|."""
    assert np.all(g["status"] == 0), g["status"]
    assert np.max(np.abs(g["energy"] - r["energy"])) <= erel * np.max(np.abs(r["energy"]))
    assert np.max(np.abs(g["forces"] - r["forces"])) <= frel * np.max(np.abs(r["forces"]))
    assert np.max(np.abs(g["charges"] - r["charges"])) <= qabs
    if pos is not None:
        rn = np.linalg.norm(pos, axis=1)
        bound = np.array([rn[unit_off[u]:unit_off[u + 1]].sum() for u in range(len(unit_off) - 1)]) * qabs
        assert np.all(np.abs(g["dipole"] - r["dipole"]).max(axis=1) <= bound)


@pytest.fixture(scope="module")
def params():
    return make_params()


def make_ctx(params, s, tol=1e-12, max_iter=300):
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(tol, max_iter, 0.2)
    return ctx


def test_monomers_parity(params):
    s = make_system(1)
    g = gpu_eval(make_ctx(params, s), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])


def test_eight_water_clusters_parity(params):
    s = make_system(2, n_units=12)
    g = gpu_eval(make_ctx(params, s), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])


def test_mixed_sizes_parity(params):
    # 1..8 waters: orbital buckets 8, 16, 32 and 48 in one call, ragged sizes
    s = make_system(5, n_units=20)
    g = gpu_eval(make_ctx(params, s), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])


def test_log_uniform_sizes_up_to_64_orbitals(params):
    full = make_system(4, n_units=60)
    nw = np.diff(full["unit_off"]) // 3
    units = [u for u in range(60) if nw[u] * 6 <= 64][:14]
    assert any(nw[u] * 6 > 48 for u in units)
    s = subsystem(full, units)
    g = gpu_eval(make_ctx(params, s), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])


def test_large_units_global_scratch_buckets(params):
    # 11..32 waters (66..192 orbitals): the buckets whose working matrices live in global scratch,
    # next to small units of the same workload, in one call
    full = make_system(4, n_units=60)
    nw = np.diff(full["unit_off"]) // 3
    big = [u for u in range(60) if nw[u] >= 11]
    units = [big[0], 2, big[-3], big[-1], 5]           # include the largest sizes present
    assert max(nw[u] for u in units) >= 29
    s = subsystem(full, units)
    g = gpu_eval(make_ctx(params, s), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])


def test_warm_start_reaches_the_same_fixed_point(params):
    s = make_system(2, n_units=6)
    ctx = make_ctx(params, s)
    gpu_eval(ctx, s["pos"])
    rng = np.random.default_rng(0)
    pos2 = s["pos"] + rng.normal(scale=0.01, size=s["pos"].shape)
    warm = gpu_eval(ctx, pos2)                 # starts from the stored basis and charges
    ctx.reset_warm_start()
    cold = gpu_eval(ctx, pos2)
    assert np.max(np.abs(warm["charges"] - cold["charges"])) < 1e-10
    assert np.max(np.abs(warm["forces"] - cold["forces"])) < 1e-9 * np.max(np.abs(cold["forces"]))
    r = eval_units(params, s["species"], pos2, s["unit_off"], tol=1e-12)
    assert_parity(warm, r, pos=pos2, unit_off=s["unit_off"])


def test_full_size_eight_water_workload_sampled(params):
    # 4096 units of 8 waters, the benchmarked shape; compare sampled units
    s = make_system(2)
    ctx = make_ctx(params, s, tol=1e-12)
    g = gpu_eval(ctx, s["pos"])
    assert np.all(g["status"] == 0)
    off = s["unit_off"]
    for u in (0, 1371, 2048, 4095):
        a0, a1 = off[u], off[u + 1]
        r = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
        assert abs(g["energy"][u] - r["energy"]) <= 1e-12 * abs(r["energy"])
        assert np.max(np.abs(g["forces"][a0:a1] - r["forces"])) <= 1e-9 * np.max(np.abs(r["forces"]))
        assert np.max(np.abs(g["charges"][a0:a1] - r["charges"])) <= 1e-10
    # property at any size: every unit neutral, forces sum to zero
    q = g["charges"].reshape(4096, 24)
    assert np.max(np.abs(q.sum(1))) < 1e-10
    F = g["forces"].reshape(4096, 24, 3)
    assert np.max(np.abs(F.sum(1))) < 1e-10


def test_full_size_fd_born_workload_sampled(params):
    # 1024 units of 8 waters with central-difference Born charges (147,456
    # displaced SCCs, +h then -h launches), the roofline shape; sampled units
    # against the oracle's central differences, the acoustic sum at any size
    s = make_system(3)
    ctx = make_ctx(params, s, tol=1e-12)
    born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FD, 1e-3, born, st)
    ctx.sync()
    Z = born.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    off = s["unit_off"]
    for u in (0, 1023):
        a0, a1 = off[u], off[u + 1]
        c = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
        Zr, _ = born_fd(params, s["species"][a0:a1], s["pos"][a0:a1], h=1e-3, tol=1e-12, dq_center=c["dq"])
        assert np.max(np.abs(Z[a0:a1] - Zr)) <= 1e-8
    assert np.max(np.abs(Z.reshape(1024, 24, 3, 3).sum(1))) < 1e-5


def test_throughput_tolerance_matches_oracle_within_scc_error(params):
    # the benchmark runs SCC to 1e-8; results stay within the SCC error of the exact fixed point
    s = make_system(2, n_units=8)
    g = gpu_eval(make_ctx(params, s, tol=1e-8), s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, frel=1e-5, qabs=1e-7, erel=1e-9, pos=s["pos"], unit_off=s["unit_off"])


def test_deterministic_bitwise(params):
    s = make_system(5, n_units=16)
    a = gpu_eval(make_ctx(params, s), s["pos"])
    b = gpu_eval(make_ctx(params, s), s["pos"])
    for k in a:
        assert np.array_equal(a[k], b[k]), k


def test_schedule_does_not_change_results(params):
    # job queue (largest units first) vs fixed stride, and fewer workgroups per CU:
    # every job computes the same numbers wherever it runs
    full = make_system(4, n_units=60)
    s = subsystem(full, list(range(0, 60, 3)))
    outs = []
    for queue, cap in ((True, 0), (False, 0), (True, 1)):
        ctx = make_ctx(params, s, tol=1e-10)
        ctx.set_schedule(queue, cap)
        outs.append(gpu_eval(ctx, s["pos"]))
        born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
        ctx.born_charges(_t(s["pos"]), cd.BORN_FIELD, 1e-4, born)
        ctx.sync()
        outs[-1]["born"] = born.cpu().numpy()
    for o in outs[1:]:
        for k in outs[0]:
            assert np.array_equal(outs[0][k], o[k]), k


def test_born_fd_parity_and_sum_rule(params):
    s = subsystem(make_system(5, n_units=6), [0, 1, 5])
    ctx = make_ctx(params, s)
    born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FD, 1e-3, born, st)
    ctx.sync()
    Z = born.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    off = s["unit_off"]
    for u in range(ctx.n_units):
        a0, a1 = off[u], off[u + 1]
        c = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
        Zr, _ = born_fd(params, s["species"][a0:a1], s["pos"][a0:a1], h=1e-3, tol=1e-12, dq_center=c["dq"])
        assert np.max(np.abs(Z[a0:a1] - Zr)) <= 1e-8
        assert np.max(np.abs(Z[a0:a1].sum(0))) < 1e-5


def test_born_field_parity(params):
    # Maxwell-relation route against the oracle's field route, and against the
    # displacement route within the two finite-difference errors
    s = subsystem(make_system(5, n_units=6), [0, 1, 5])
    ctx = make_ctx(params, s)
    born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
    born_d = torch.zeros_like(born)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FIELD, 1e-4, born, st)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FD, 1e-3, born_d)
    ctx.sync()
    Z, Zd = born.cpu().numpy(), born_d.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    off = s["unit_off"]
    for u in range(ctx.n_units):
        a0, a1 = off[u], off[u + 1]
        c = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
        Zr, stf = born_field(params, s["species"][a0:a1], s["pos"][a0:a1], e=1e-4, tol=1e-12, dq_center=c["dq"])
        assert stf == 0
        # force bar 1e-9 x max|F| over a field step of 2e-4 a.u.
        assert np.max(np.abs(Z[a0:a1] - Zr)) <= 1e-7
    assert np.max(np.abs(Z - Zd)) <= 1e-5


def test_born_field_across_orbital_buckets(params):
    # units of several orbital buckets in one call: every atom's tensor is written
    s = subsystem(make_system(4, n_units=64), list(range(0, 64, 9)))
    ctx = make_ctx(params, s)
    born = torch.full((ctx.n_atoms, 3, 3), float("nan"), dtype=torch.float64, device=DEV)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FIELD, 1e-4, born, st)
    ctx.sync()
    Z = born.cpu().numpy()
    good = st.cpu().numpy() == 0
    off = s["unit_off"]
    for u in np.nonzero(good)[0]:
        a0, a1 = off[u], off[u + 1]
        assert np.all(np.isfinite(Z[a0:a1]))
        assert np.max(np.abs(Z[a0:a1].sum(0))) < 1e-5        # acoustic sum rule of the exact tensor
    u = int(np.nonzero(good)[0][-1])
    a0, a1 = off[u], off[u + 1]
    c = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
    Zr, _ = born_field(params, s["species"][a0:a1], s["pos"][a0:a1], e=1e-4, tol=1e-12, dq_center=c["dq"])
    assert np.max(np.abs(Z[a0:a1] - Zr)) <= 1e-7


def test_born_mulliken_is_charge_identity(params):
    s = make_system(1)
    ctx = make_ctx(params, s)
    born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_MULLIKEN, 0.0, born)
    ctx.sync()
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    Z = born.cpu().numpy()
    assert np.max(np.abs(Z - r["charges"][:, None, None] * np.eye(3))) <= 1e-10


@pytest.mark.parametrize("U,M", [(4096, 256), (4093, 2047), (3, 5)])
def test_cavity_forces_parity(params, U, M):
    # cavity sums at the benchmarked shape (4096 cells, 256 modes) and ragged ones
    s = {"unit_x": (np.arange(U) + 0.5) * CAVITY_LENGTH / U, "pol": np.array([0.0, 0.0, 1.0])}
    s["omega"], s["k"], s["theta"], s["lam"] = mode_comb(M)
    rng = np.random.default_rng(4)
    off = np.arange(U + 1, dtype=np.int32) * 3
    sp = np.tile(np.array([0, 1, 1], dtype=np.int8), U)
    ctx = cd.Context(params, sp, off, s["unit_x"], s["omega"], s["k"], s["theta"], s["lam"], s["pol"])
    mu = rng.normal(size=U)
    q = rng.normal(scale=10.0, size=M)
    F = torch.zeros(M, dtype=torch.float64, device=DEV)
    E = torch.zeros(U, dtype=torch.float64, device=DEV)
    fq = torch.zeros(M, dtype=torch.float64, device=DEV)
    ctx.cavity_forces(_t(mu), _t(q), F, E, fq)
    ctx.sync()
    phi = ocav.mode_functions(s["k"], s["theta"], s["unit_x"])
    Fr = ocav.dipole_sums(phi, mu)
    Er = ocav.fields(phi, s["omega"], s["lam"], q, Fr)
    fqr = ocav.photon_coupling_force(s["omega"], s["lam"], Fr)
    scaleF = np.abs(phi) @ np.abs(mu)
    assert np.all(np.abs(F.cpu().numpy() - Fr) <= 1e-12 * scaleF)
    g = s["lam"] * s["omega"] * (q + s["lam"] * Fr / s["omega"])
    scaleE = np.abs(phi).T @ np.abs(g)
    assert np.all(np.abs(E.cpu().numpy() - Er) <= 1e-12 * scaleE + 1e-15)
    assert np.all(np.abs(fq.cpu().numpy() - fqr) <= 1e-12 * np.abs(s["lam"] * s["omega"]) * scaleF)


def _oracle_md(params, s, born, n_steps):
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born=born, tol=1e-12)
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    masses = params["mass"][s["species"]]
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    for _ in range(n_steps):
        omd.step(st, be, cav, s["dt"])
    return st, cav


def _gpu_md(params, s, born_mode, n_steps):
    ctx = make_ctx(params, s)
    masses = params["mass"][s["species"]]
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    obs = torch.zeros(n_steps, cd.N_OBS, dtype=torch.float64, device=DEV)
    ctx.init_photons(r, qm, pm)
    ctx.step(r, p, qm, pm, n_steps, s["dt"], born_mode, 1e-3, obs)
    assert ctx.sync() == 0
    return r.cpu().numpy(), p.cpu().numpy(), qm.cpu().numpy(), pm.cpu().numpy(), obs.cpu().numpy()


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("n_steps,tol", [(1, 1e-9), (10, 1e-7)])
def test_md_steps_mulliken_parity(params, n_steps, tol):
    s = make_system(1)
    r, p, qm, pm, obs = _gpu_md(params, s, cd.BORN_MULLIKEN, n_steps)
    st, cav = _oracle_md(params, s, "mulliken", n_steps)
    assert _rel(r, st["r"]) <= tol and _rel(p, st["p"]) <= tol
    assert _rel(qm, st["q"]) <= tol and _rel(pm, st["pm"]) <= tol
    o = omd.observables(st, cav, s["unit_off"])
    assert abs(obs[-1, 3] - o["total"]) <= tol * abs(o["total"])
    assert abs(obs[-1, 0] - o["kinetic"]) <= tol * o["kinetic"]
    assert abs(obs[-1, 4] - o["temperature"]) <= tol * o["temperature"]


def test_md_step_exact_born_parity(params):
    s = subsystem(make_system(1), [0, 3])
    r, p, qm, pm, obs = _gpu_md(params, s, cd.BORN_FD, 2)
    st, _ = _oracle_md(params, s, "fd", 2)
    assert _rel(r, st["r"]) <= 1e-9 and _rel(p, st["p"]) <= 1e-8
    assert _rel(qm, st["q"]) <= 1e-8 and _rel(pm, st["pm"]) <= 1e-8


@pytest.mark.parametrize("route", ["fd", "field"])
def test_md_steps_exact_born_second_order_starts(params, route):
    # five steps: from the second Born evaluation on, every +h / +field SCC starts
    # from its charge response at the previous evaluation and every -h / -field
    # SCC from the reflected + charges; the trajectory still follows the
    # oracle's within the exact-Born bars
    s = subsystem(make_system(1), [0, 3, 5])
    mode, h = (cd.BORN_FD, 1e-3) if route == "fd" else (cd.BORN_FIELD, 1e-4)
    n = 5
    ctx = make_ctx(params, s)
    masses = params["mass"][s["species"]]
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    ctx.step(r, p, qm, pm, n, s["dt"], mode, h)
    assert ctx.sync() == 0
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born=route, tol=1e-12, h=h)
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    for _ in range(n):
        omd.step(st, be, cav, s["dt"])
    rn, pn, qn, pmn = (x.cpu().numpy() for x in (r, p, qm, pm))
    assert _rel(rn, st["r"]) <= 1e-9 and _rel(pn, st["p"]) <= 1e-8
    assert _rel(qn, st["q"]) <= 1e-8 and _rel(pmn, st["pm"]) <= 1e-8
    ctx.close()


def test_born_fd_forward_parity(params):
    # the paper's forward differences against the undisplaced dipole
    s = subsystem(make_system(5, n_units=6), [0, 1, 5])
    ctx = make_ctx(params, s)
    born = torch.zeros(ctx.n_atoms, 3, 3, dtype=torch.float64, device=DEV)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=DEV)
    ctx.born_charges(_t(s["pos"]), cd.BORN_FD_FORWARD, 1e-3, born, st)
    ctx.sync()
    Z = born.cpu().numpy()
    assert np.all(st.cpu().numpy() == 0)
    off = s["unit_off"]
    for u in range(ctx.n_units):
        a0, a1 = off[u], off[u + 1]
        c = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12)
        Zr, _ = born_fd_forward(params, s["species"][a0:a1], s["pos"][a0:a1], c["dipole"], h=1e-3, tol=1e-12,
                                dq_center=c["dq"])
        # SCC tolerance 1e-12 on both dipoles, divided by h
        assert np.max(np.abs(Z[a0:a1] - Zr)) <= 5e-8


def test_md_steps_forward_born_refresh_every_three(params):
    s = subsystem(make_system(1), [0, 3])
    masses = params["mass"][s["species"]]
    out = {}
    for every in (3, 1):
        ctx = make_ctx(params, s)
        ctx.set_born_interval(every)
        r = _t(s["pos"])
        p = _t(s["vel"] * masses[:, None])
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
        pm = torch.zeros_like(qm)
        ctx.init_photons(r, qm, pm)
        ctx.step(r, p, qm, pm, 4, s["dt"], cd.BORN_FD_FORWARD, 1e-3)
        assert ctx.sync() == 0
        out[every] = [x.cpu().numpy() for x in (r, p, qm, pm)]
        ctx.close()
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="fd_forward", tol=1e-12, h=1e-3, born_every=3)
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    for _ in range(4):
        omd.step(st, be, cav, s["dt"])
    r, p, qm, pm = out[3]
    assert _rel(r, st["r"]) <= 1e-9 and _rel(p, st["p"]) <= 1e-8
    assert _rel(qm, st["q"]) <= 1e-8 and _rel(pm, st["pm"]) <= 1e-8
    assert not np.array_equal(out[1][1], out[3][1])  # the stale tensors change the momenta


def test_md_step_field_born_parity(params):
    s = subsystem(make_system(1), [0, 3])
    ctx = make_ctx(params, s)
    masses = params["mass"][s["species"]]
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    ctx.step(r, p, qm, pm, 2, s["dt"], cd.BORN_FIELD, 1e-4)
    assert ctx.sync() == 0
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born="field", tol=1e-12, h=1e-4)
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    for _ in range(2):
        omd.step(st, be, cav, s["dt"])
    assert _rel(r.cpu().numpy(), st["r"]) <= 1e-9 and _rel(p.cpu().numpy(), st["p"]) <= 1e-8
    assert _rel(qm.cpu().numpy(), st["q"]) <= 1e-8 and _rel(pm.cpu().numpy(), st["pm"]) <= 1e-8


def test_status_flags(params):
    s = make_system(1)
    ctx = make_ctx(params, s, max_iter=2)
    g = gpu_eval(ctx, s["pos"])
    assert np.all(g["status"] & 1)                # not converged in 2 iterations
    ctx = make_ctx(params, s)
    pos = s["pos"].copy()
    pos[4, 1] = np.nan
    g = gpu_eval(ctx, pos)
    assert g["status"][1] & 8 and np.all(g["status"][[0, 2, 3, 4, 5, 6, 7]] == 0)
    # no valid density: zero charges, dipole, energy and forces for that unit only
    assert np.all(g["dipole"][1] == 0.0) and g["energy"][1] == 0.0
    assert np.all(g["charges"][3:6] == 0.0) and np.all(g["forces"][3:6] == 0.0)
    ok = np.r_[0:3, 6:len(pos)]
    assert np.all(np.isfinite(g["forces"][ok])) and np.all(np.isfinite(g["dipole"][[0, 2, 3, 4, 5, 6, 7]]))


def test_failed_unit_does_not_poison_the_cavity(params):
    # a unit with a non-finite position drops out of the mode sums: every other
    # unit keeps finite, unchanged-in-kind dynamics and the totals stay finite
    s = make_system(5, n_units=8)
    masses = params["mass"][s["species"]]
    out = {}
    for tag in ("clean", "nan"):
        ctx = make_ctx(params, s, tol=1e-10)
        pos = s["pos"].copy()
        if tag == "nan":
            pos[s["unit_off"][2], 0] = np.nan
        r = _t(pos)
        p = _t(s["vel"] * masses[:, None])
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
        pm = torch.zeros_like(qm)
        obs = torch.zeros(3, cd.N_OBS, dtype=torch.float64, device=DEV)
        ctx.init_photons(r, qm, pm)
        ctx.step(r, p, qm, pm, 3, s["dt"], cd.BORN_MULLIKEN, 0.0, obs)
        ctx.sync()
        out[tag] = (r.cpu().numpy(), qm.cpu().numpy(), obs.cpu().numpy())
        ctx.close()
    a0, a1 = s["unit_off"][2], s["unit_off"][3]
    keep = np.r_[0:a0, a1:len(s["pos"])]
    r_nan, q_nan, o_nan = out["nan"]
    assert np.all(np.isfinite(r_nan[keep])) and np.all(np.isfinite(q_nan)) and np.all(np.isfinite(o_nan))
    assert np.all(o_nan[:, 5] == 1)  # exactly the one unit is flagged
    # the other units feel only the missing unit's (tiny) cavity contribution
    assert np.max(np.abs(r_nan[keep] - out["clean"][0][keep])) < 1e-6


def test_autotune_launch_table_keeps_results(params, tmp_path):
    # per-bucket search, written as a launch table, read back by the library;
    # the tuned context reaches the oracle's fixed point, and entries that keep
    # the default eigensolver leave every bit of the results unchanged
    from paper_2512_03277_amd import autotune
    s = subsystem(make_system(4, n_units=24), list(range(0, 24, 2)))
    entries, timings, base, final = autotune.tune(params, s, steps=1, warmup=1)
    assert base > 0 and final > 0 and len(timings) > len(entries)
    path = tmp_path / "table.json"
    path.write_text(autotune.table_json(entries, timings, 4, "mulliken", base, final))
    ref = gpu_eval(make_ctx(params, s), s["pos"])
    ctx = make_ctx(params, s)
    assert ctx.load_launch_table(str(path)) == len(entries)
    present = set()
    for e in entries:
        n_units, wg_max, wg_cur = ctx.bucket_info(e["bucket"])
        assert n_units > 0 and 1 <= e["wg_per_cu"] <= wg_max and wg_cur == e["wg_per_cu"]
        present.add(e["bucket"])
    assert present == {b for b in cd.binding.BUCKETS if ctx.bucket_info(b)[0] > 0}
    g = gpu_eval(ctx, s["pos"])
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert_parity(g, r, pos=s["pos"], unit_off=s["unit_off"])
    if all(e["eig_mode"] == cd.EIG_AUTO for e in entries):
        for k in g:
            assert np.array_equal(g[k], ref[k]), k
    else:
        assert np.max(np.abs(g["charges"] - ref["charges"])) <= 1e-10
    # another architecture's entries are skipped; an entry without "arch" is an error
    other = tmp_path / "other.json"
    other.write_text('{"entries": [{"arch": "gfx942", "bucket": 48, "wg_per_cu": 1}]}')
    assert ctx.load_launch_table(str(other)) == 0
    bad = tmp_path / "bad.json"
    bad.write_text('{"entries": [{"bucket": 48, "wg_per_cu": 1}]}')
    with pytest.raises(cd.CavdftbError):
        ctx.load_launch_table(str(bad))
    with pytest.raises(cd.CavdftbError):
        ctx.set_bucket_schedule(40, 1)
    ctx.close()


def test_read_work_arrays_match_the_evaluation(params):
    # the context's work arrays after init_photons / a step are those of an
    # evaluation at the same positions; the field is the cavity gather's
    s = make_system(5, n_units=8)
    ctx = make_ctx(params, s, tol=1e-12)
    masses = params["mass"][s["species"]]
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    ctx.step(r, p, qm, pm, 2, s["dt"], cd.BORN_MULLIKEN, 0.0, None)
    U, NA = ctx.n_units, ctx.n_atoms
    w = {k: torch.zeros(n, dtype=torch.float64, device=DEV) for k, n in
         (("mu_pol", U), ("dipole", 3 * U), ("energy", U), ("charges", NA), ("forces", 3 * NA), ("field", U))}
    for k, which in (("mu_pol", cd.WORK_MU_POL), ("dipole", cd.WORK_DIPOLE), ("energy", cd.WORK_ENERGY),
                     ("charges", cd.WORK_CHARGES), ("forces", cd.WORK_FORCES), ("field", cd.WORK_FIELD)):
        ctx.read_work(which, w[k])
    ctx.sync()
    ref = make_ctx(params, s, tol=1e-12)
    g = gpu_eval(ref, r.cpu().numpy())
    wk = {k: v.cpu().numpy() for k, v in w.items()}
    assert np.max(np.abs(wk["energy"] - g["energy"])) <= 1e-10 * np.max(np.abs(g["energy"]))
    assert np.max(np.abs(wk["forces"].reshape(-1, 3) - g["forces"])) <= 1e-8 * np.max(np.abs(g["forces"]))
    assert np.max(np.abs(wk["charges"] - g["charges"])) <= 1e-10
    assert np.max(np.abs(wk["dipole"].reshape(-1, 3) - g["dipole"])) <= 1e-8
    assert np.allclose(wk["mu_pol"], wk["dipole"].reshape(-1, 3) @ np.asarray(s["pol"]), rtol=0, atol=1e-14)
    field = torch.zeros(U, dtype=torch.float64, device=DEV)
    ctx.cavity_forces(w["mu_pol"], qm, field=field)
    ctx.sync()
    assert torch.equal(field, w["field"])
    with pytest.raises(RuntimeError):
        ctx.read_work(17, w["energy"])
    ref.close()
    ctx.close()


def test_observables_over_many_workgroups_match_their_definition(params):
    # 1024 units and 2048 modes: the step observables are reduced over several
    # workgroups of partial sums, then totalled in one; compared with the oracle's
    # definition evaluated on the state and work arrays the device returns
    s = make_system(5, n_units=1024)
    masses = params["mass"][s["species"]]
    ctx = cd.context_from_system(params, s)
    ctx.set_scc(1e-8, 200)
    U, M = ctx.n_units, ctx.n_modes
    assert U == 1024 and M == 2048
    r = _t(s["pos"])
    p = _t(s["vel"] * masses[:, None])
    qm = torch.zeros(M, dtype=torch.float64, device=DEV)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    obs = torch.zeros(2, cd.N_OBS, dtype=torch.float64, device=DEV)
    ctx.step(r, p, qm, pm, 2, s["dt"], cd.BORN_MULLIKEN, 0.0, obs)
    n_bad = ctx.sync()
    energy = torch.empty(U, dtype=torch.float64, device=DEV)
    mu = torch.empty(U, dtype=torch.float64, device=DEV)
    ctx.read_work(cd.WORK_ENERGY, energy)
    ctx.read_work(cd.WORK_MU_POL, mu)
    ctx.sync()
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    mu_h = mu.cpu().numpy()
    st = {"p": p.cpu().numpy(), "masses": masses, "ev": {"energy": energy.cpu().numpy()},
          "q": qm.cpu().numpy(), "pm": pm.cpu().numpy(), "F": ocav.dipole_sums(cav.phi, mu_h)}
    o = omd.observables(st, cav, s["unit_off"])
    row = obs.cpu().numpy()[-1]
    assert row[0] == pytest.approx(o["kinetic"], rel=1e-12)
    assert row[1] == pytest.approx(o["potential"], rel=1e-12)
    assert row[2] == pytest.approx(o["photon"], rel=1e-10)
    assert row[3] == pytest.approx(o["total"], rel=1e-12)
    assert row[4] == pytest.approx(o["temperature"], rel=1e-12)
    assert row[5] == n_bad
    assert abs(row[7] - mu_h.sum()) <= 1e-12 * np.abs(mu_h).sum()
    ctx.close()
