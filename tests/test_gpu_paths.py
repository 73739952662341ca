"""GPU parity of the paths the single-unit tests leave out, through the C ABI
against the FP64 oracle:

* gamma at near-equal Hubbard U (the series branch of the kernel, the
  extended-precision branch of the oracle) and at the workload's U;
* MD trajectories of 8-water clusters (48-orbital bucket: warm MO basis,
  quadratic charge extrapolation from the fourth step, cost-ordered job queue,
  graph replay) and of a mixed 1-8-water set, Mulliken and central-difference
  Born routes;
* the surrogate route inside MD steps, with some units falling back to the
  exact field route, against the oracle's surrogate route;
* the status bits for an overlap that is not positive definite and for a
  degenerate Fermi level;
* sampled units of the uneven 16,384-unit workload at its full shape, with the
  one unit whose SCC does not converge flagged.

Bars as in test_gpu_parity: energies rel 1e-12, forces 1e-9 max|F|, charges
1e-10 e; MD states rel 1e-9 after 1 step, 1e-7 after 10 (Mulliken), 1e-8
after 2 (exact Born).
"""
import numpy as np
import pytest

from cavgen import make_params, make_system
from oracle import md as omd
from oracle import surrogate as osg
from oracle.scc import eval_units, scc_unit

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2512_03277_amd as cd  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


@pytest.fixture(scope="module")
def params():
    return make_params()


def subsystem(s, units):
    off = s["unit_off"]
    idx = np.concatenate([np.arange(off[u], off[u + 1]) for u in units])
    out = dict(s)
    out.update({"species": s["species"][idx], "pos": s["pos"][idx], "vel": s["vel"][idx],
                "unit_off": np.concatenate([[0], np.cumsum([off[u + 1] - off[u] for u in units])]).astype(np.int32),
                "unit_x": s["unit_x"][list(units)]})
    return out


def with_extra_unit(s, species, pos):
    """s plus one more unit (placed at the end of the cavity axis)."""
    out = dict(s)
    n = len(species)
    out["species"] = np.concatenate([s["species"], np.asarray(species, dtype=s["species"].dtype)])
    out["pos"] = np.vstack([s["pos"], np.asarray(pos, dtype=np.float64)])
    out["vel"] = np.vstack([s["vel"], np.zeros((n, 3))])
    out["unit_off"] = np.concatenate([s["unit_off"], [s["unit_off"][-1] + n]]).astype(np.int32)
    out["unit_x"] = np.concatenate([s["unit_x"], [s["unit_x"][-1] * 1.01]])
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


def unit_parity(g, r, u, a0, a1):
    assert abs(g["energy"][u] - r["energy"]) <= 1e-12 * abs(r["energy"])
    assert np.max(np.abs(g["forces"][a0:a1] - r["forces"])) <= 1e-9 * np.max(np.abs(r["forces"]))
    assert np.max(np.abs(g["charges"][a0:a1] - r["charges"])) <= 1e-10


def make_ctx(params, s, tol=1e-12, max_iter=300, stream=None):
    ctx = cd.context_from_system(params, s, stream=stream)
    ctx.set_scc(tol, max_iter, 0.2)
    return ctx


# ---------------------------------------------------------------- gamma branches
@pytest.mark.parametrize("u_h", [0.5 * (1 + 1e-6), 0.5 * (1 + 3e-2), 0.42])
def test_hubbard_u_branches_parity(params, u_h):
    # O-H pairs at relative exponent differences 5e-7 and 1.5e-2 (the kernel's
    # series about equal exponents, the oracle's 50-digit closed form) and at the
    # workload's U (x = 0.087, also the series); 8-water clusters and monomers
    p = dict(params)
    p["hubbard_u"] = np.array([params["hubbard_u"][0], u_h])
    s = subsystem(make_system(5, n_units=12), list(range(12)))
    g = gpu_eval(make_ctx(p, s), s["pos"])
    r = eval_units(p, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert np.all(g["status"] == 0) and np.all(r["status"] == 0)
    off = s["unit_off"]
    for u in range(len(off) - 1):
        a0, a1 = off[u], off[u + 1]
        unit_parity(g, {"energy": r["energy"][u], "forces": r["forces"][a0:a1], "charges": r["charges"][a0:a1]},
                    u, a0, a1)


# ---------------------------------------------------------------- MD trajectories
def _oracle_md(params, s, born, n_steps, h=1e-3, surrogate=None):
    be = omd.DFTBBackend(params, s["species"], s["unit_off"], born=born, tol=1e-12, h=h, surrogate=surrogate)
    cav = omd.Cavity(s["omega"], s["k"], s["theta"], s["lam"], s["unit_x"], s["pol"])
    masses = params["mass"][s["species"]]
    atom_unit = np.repeat(np.arange(len(s["unit_off"]) - 1), np.diff(s["unit_off"]))
    st = omd.init_state(be, cav, s["pos"], s["vel"] * masses[:, None], masses, atom_unit)
    for _ in range(n_steps):
        omd.step(st, be, cav, s["dt"])
    return st, cav, be


def _gpu_md(params, s, born_mode, n_steps, h=1e-3, graph=True, setup=None):
    """n_steps MD steps in one call on a context with its own stream and graph
    replay on (the launches of a step are replayed from the fourth MD step)."""
    stream = torch.cuda.Stream()
    masses = params["mass"][s["species"]]
    with torch.cuda.stream(stream):
        ctx = make_ctx(params, s, stream=stream)
        if setup is not None:
            setup(ctx)
        ctx.set_graph(graph)
        r = _t(s["pos"])
        p = _t(s["vel"] * masses[:, None])
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
        pm = torch.zeros_like(qm)
        obs = torch.zeros(n_steps, cd.N_OBS, dtype=torch.float64, device=DEV)
        ctx.init_photons(r, qm, pm)
        ctx.step(r, p, qm, pm, n_steps, s["dt"], born_mode, h, obs)
        n_bad = ctx.sync()
        counters = ctx.read_counters()
        out = [x.cpu().numpy() for x in (r, p, qm, pm, obs)]
        ctx.close()
    assert n_bad == 0
    return out, counters


def _rel(a, b):
    return np.max(np.abs(a - b)) / np.max(np.abs(b))


@pytest.mark.parametrize("which", ["8water", "mixed"])
def test_md_ten_steps_mulliken_parity(params, which):
    if which == "8water":
        s = make_system(2, n_units=3)                 # 48-orbital bucket only
    else:
        s = subsystem(make_system(5, n_units=12), [0, 1, 2, 3, 5, 7])  # 1-8 waters, several buckets
    (r, p, qm, pm, obs), cnt = _gpu_md(params, s, cd.BORN_MULLIKEN, 10)
    assert cnt["graph_replays"] >= 6                  # steps 4..10 replayed
    st, cav, _ = _oracle_md(params, s, "mulliken", 10)
    tol = 1e-7
    assert _rel(r, st["r"]) <= tol and _rel(p, st["p"]) <= tol
    assert _rel(qm, st["q"]) <= tol and _rel(pm, st["pm"]) <= tol
    o = omd.observables(st, cav, s["unit_off"])
    assert abs(obs[-1, 3] - o["total"]) <= tol * abs(o["total"])
    assert abs(obs[-1, 0] - o["kinetic"]) <= tol * o["kinetic"]
    assert abs(obs[-1, 4] - o["temperature"]) <= tol * o["temperature"]


def test_md_two_steps_central_fd_eight_water_parity(params):
    # the photon variables follow the unit dipoles, whose bar is the charge bar
    # carried through mu = sum Q R: 1e-10 e x sum_A |R_A| (about 2e-8 a.u. for 24
    # atoms) on |mu| of order 0.5 a.u., so q_m and p_m get 1e-7 relative
    s = make_system(2, n_units=2)
    (r, p, qm, pm, _), _ = _gpu_md(params, s, cd.BORN_FD, 2, graph=False)
    st, _, _ = _oracle_md(params, s, "fd", 2)
    assert _rel(r, st["r"]) <= 1e-9 and _rel(p, st["p"]) <= 1e-8
    assert _rel(qm, st["q"]) <= 1e-7 and _rel(pm, st["pm"]) <= 1e-7


def _ensemble(seed):
    rng = np.random.default_rng(seed)
    P = np.stack([np.stack([osg.init_params(rng) for _ in range(4)]) for _ in range(2)]).astype(np.float32)
    N = np.stack([np.concatenate([rng.uniform(0, 1, osg.N_IN), rng.uniform(0.5, 2, osg.N_IN), rng.normal(0, 0.2, 9),
                                  rng.uniform(0.05, 0.2, 9)]) for _ in range(2)]).astype(np.float32)
    nets = [[P[sp, m].astype(np.float64) for m in range(4)] for sp in (0, 1)]
    Nh = N.astype(np.float64)
    norms = [osg.unpack_norm(Nh[sp]) for sp in (0, 1)]
    return nets, norms, _t(P, torch.float32), _t(N, torch.float32)


def test_md_surrogate_route_parity(params):
    # The surrogate's Born tensors enter MD through the cavity force -E_n e.Z.
    # With lambda raised 20x that force is a few 1e-3 hartree/bohr, so the
    # route matters: the Mulliken route moves the momenta by far more than the
    # bar.  Units whose ensemble spread exceeds the threshold take the exact
    # field route on both sides; the threshold sits in the widest gap of the
    # oracle's per-unit spreads so BF16/FP32 rounding cannot move a unit across.
    s = dict(subsystem(make_system(5, n_units=12), list(range(8))))
    s["lam"] = s["lam"] * 20.0
    nets, norms, P, N = _ensemble(7)
    q = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12, want_forces=False)["charges"]
    off = s["unit_off"]
    spread = np.array([osg.predict_unit(s["species"][off[u]:off[u + 1]], s["pos"][off[u]:off[u + 1]], nets, norms,
                                        q[off[u]:off[u + 1]], emulate_bf16=True)[1].max() for u in range(8)])
    srt = np.sort(spread)
    gaps = srt[2:-1] / srt[1:-2]                       # keep at least two units on each side
    i = int(np.argmax(gaps)) + 1
    thr = float(np.sqrt(srt[i] * srt[i + 1]))
    assert gaps.max() > 1.05
    sg = {"nets": nets, "norms": norms, "threshold": thr, "fallback": "field", "emulate_bf16": True}
    steps, h = 2, 1e-4

    def setup(ctx):
        ctx.set_surrogate(P.view(-1), N.view(-1), thr)
        ctx.set_fallback(cd.BORN_FIELD)

    (r, p, qm, pm, _), cnt = _gpu_md(params, s, cd.BORN_SURROGATE, steps, h=h, graph=False, setup=setup)
    st, cav, be = _oracle_md(params, s, "surrogate", steps, h=h, surrogate=sg)
    assert cnt["surrogate_fallback_units"] == len(be.fallback_units) > 0
    # bar: the network outputs agree within 1e-3 of max|Z| (BF16 operands, FP32
    # vs FP64 accumulation); each of the 2 n_steps half-kicks moves p by at most
    # dt/2 max|E| 1e-3 max|Z|; positions follow through dt/m
    Emax = np.max(np.abs(st["E"]))
    zmax = np.max(np.abs(st["ev"]["Z"]))
    bar_p = steps * s["dt"] * Emax * 1e-3 * zmax * 2.0 + 1e-8 * np.max(np.abs(st["p"]))
    assert np.max(np.abs(p - st["p"])) <= bar_p
    m = params["mass"][s["species"]][:, None]
    assert np.max(np.abs(r - st["r"])) <= steps * s["dt"] * bar_p / m.min() + 1e-9 * np.max(np.abs(st["r"]))
    assert _rel(qm, st["q"]) <= 1e-6 and _rel(pm, st["pm"]) <= 1e-6
    # the same steps on the Mulliken route move the momenta by much more than the bar
    stm, _, _ = _oracle_md(params, s, "mulliken", steps)
    assert np.max(np.abs(stm["p"] - st["p"])) > 20 * bar_p


# ---------------------------------------------------------------- status bits
def test_not_positive_definite_overlap_flagged(params):
    # five oxygen atoms 0.01 bohr apart on a line: with these tables the
    # overlap matrix has a negative eigenvalue (about -0.07); the unit reports
    # zero outputs and bit 2, the other units are untouched
    base = make_system(1)
    pos = np.zeros((5, 3))
    pos[:, 2] = np.arange(5) * 0.01
    pos += base["pos"][0]
    s = with_extra_unit(base, [0] * 5, pos)
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert r["status"][-1] == 2
    g = gpu_eval(make_ctx(params, s), s["pos"])
    assert g["status"][-1] == 2 and np.all(g["status"][:-1] == 0)
    a0 = s["unit_off"][-2]
    assert g["energy"][-1] == 0.0 and np.all(g["forces"][a0:] == 0.0) and np.all(g["charges"][a0:] == 0.0)
    assert np.all(g["dipole"][-1] == 0.0)
    for u in range(len(s["unit_off"]) - 2):
        b0, b1 = s["unit_off"][u], s["unit_off"][u + 1]
        unit_parity(g, {"energy": r["energy"][u], "forces": r["forces"][b0:b1], "charges": r["charges"][b0:b1]},
                    u, b0, b1)


def test_degenerate_fermi_level_flagged(params):
    # a lone oxygen atom: 6 electrons in s + three degenerate p levels, so the
    # HOMO and LUMO are both p (gap 0) and bit 4 is set on both sides; charges,
    # energy and (zero) forces are unique and still compared
    base = make_system(1)
    s = with_extra_unit(base, [0], base["pos"][:1] + 5.0)
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    assert r["status"][-1] == 4
    g = gpu_eval(make_ctx(params, s), s["pos"])
    assert g["status"][-1] == 4 and np.all(g["status"][:-1] == 0)
    a0 = s["unit_off"][-2]
    assert abs(g["energy"][-1] - r["energy"][-1]) <= 1e-12 * abs(r["energy"][-1])
    assert abs(g["charges"][a0]) <= 1e-12 and np.all(g["forces"][a0:] == 0.0)


# ---------------------------------------------------------------- uneven workload, full shape
def test_uneven_workload_full_shape_sampled(params):
    # 16,384 units of 1-32 waters (6-192 orbitals, unsorted): sampled units of
    # every bucket against the oracle, neutrality and zero net force at any size,
    # and the 27-water unit 11611, whose SCC does not converge on this model
    # (the oracle does not converge it either), flagged with bit 1
    s = make_system(4)
    U = len(s["unit_off"]) - 1
    assert U == 16384
    ctx = make_ctx(params, s, tol=1e-12, max_iter=150)
    g = gpu_eval(ctx, s["pos"])
    off = s["unit_off"]
    nw = np.diff(off) // 3
    assert g["status"][11611] & 1
    r_bad = scc_unit(params, s["species"][off[11611]:off[11612]], s["pos"][off[11611]:off[11612]], tol=1e-12,
                     max_iter=150, want_forces=False)
    assert r_bad["status"] & 1
    ok = g["status"] == 0
    picks = [0, int(np.argmax(nw)), int(np.argmin(nw))]
    for lo, hi in ((2, 4), (9, 11), (15, 21)):
        cand = np.nonzero((nw >= lo) & (nw <= hi) & ok)[0]
        picks.append(int(cand[len(cand) // 2]))
    for u in picks:
        assert ok[u], u
        a0, a1 = off[u], off[u + 1]
        r = scc_unit(params, s["species"][a0:a1], s["pos"][a0:a1], tol=1e-12, max_iter=300)
        assert r["status"] == 0
        unit_parity(g, r, u, a0, a1)
    # neutrality and zero net force: the sum of N_a charges each within the
    # 1e-10 e bar, the sum of N_a forces each within 1e-9 max|F|
    na = np.diff(off)
    q = np.add.reduceat(g["charges"], off[:-1])
    F = np.abs(np.add.reduceat(g["forces"], off[:-1], axis=0)).max(1)
    fmax = np.maximum.reduceat(np.abs(g["forces"]).max(1), off[:-1])
    assert np.all(np.abs(q[ok]) <= 1e-10 * na[ok]), np.max(np.abs(q[ok]) / na[ok])
    assert np.all(F[ok] <= 1e-9 * na[ok] * fmax[ok])
    ctx.close()


# ---------------------------------------------------------------- large-unit eigensolver
def _large_units(n_per_bucket=2):
    full = make_system(4, n_units=300)
    nw = np.diff(full["unit_off"]) // 3
    units = []
    for lo, hi in ((11, 16), (17, 21), (22, 32)):       # orbital buckets 96, 128, 192
        cand = [u for u in range(300) if lo <= nw[u] <= hi]
        units += cand[:n_per_bucket]
    units.append(int(np.argmax(nw)))
    return subsystem(full, units), nw[units]


def test_tridiagonal_solver_forced_parity(params):
    # every SCC iteration of the 96/128/192-orbital units diagonalised by
    # Householder tridiagonalisation + bisection + twisted-factorisation vectors
    # + blocked back-transform; parity with the oracle at tol 1e-12
    s, nw = _large_units()
    assert nw.max() >= 29 and nw.min() <= 16
    ctx = make_ctx(params, s)
    ctx.set_eigensolver(cd.EIG_FULL)
    ctx.reset_counters()
    g = gpu_eval(ctx, s["pos"])
    cnt = ctx.read_counters()
    assert cnt["tridiagonal_solves"] >= cnt["scc_iterations"] > 0
    assert cnt["tridiagonal_fallbacks"] == 0
    r = eval_units(params, s["species"], s["pos"], s["unit_off"], tol=1e-12)
    off = s["unit_off"]
    for u in range(len(off) - 1):
        a0, a1 = off[u], off[u + 1]
        assert g["status"][u] == 0, (u, g["status"][u])
        unit_parity(g, {"energy": r["energy"][u], "forces": r["forces"][a0:a1], "charges": r["charges"][a0:a1]},
                    u, a0, a1)
    ctx.close()


def test_eigensolver_modes_agree(params):
    # the default schedule (cold tridiagonal solve, then occupied-virtual steps),
    # tridiagonal solves every iteration and Jacobi for every full solve reach the
    # same fixed point; a warm MD-like second evaluation too
    s, _ = _large_units(1)
    rng = np.random.default_rng(3)
    pos2 = s["pos"] + rng.normal(scale=0.01, size=s["pos"].shape)
    outs = {}
    for mode in (cd.EIG_AUTO, cd.EIG_FULL, cd.EIG_JACOBI):
        ctx = make_ctx(params, s)
        ctx.set_eigensolver(mode)
        outs[mode] = (gpu_eval(ctx, s["pos"]), gpu_eval(ctx, pos2), ctx.read_counters())
        ctx.close()
    assert outs[cd.EIG_AUTO][2]["tridiagonal_solves"] > 0
    assert outs[cd.EIG_JACOBI][2]["tridiagonal_solves"] == 0
    for mode in (cd.EIG_FULL, cd.EIG_JACOBI):
        for k in (0, 1):
            a, b = outs[cd.EIG_AUTO][k], outs[mode][k]
            assert np.all(a["status"] == 0) and np.all(b["status"] == 0)
            assert np.max(np.abs(a["charges"] - b["charges"])) <= 1e-10
            assert np.max(np.abs(a["energy"] - b["energy"])) <= 1e-12 * np.max(np.abs(a["energy"]))
            assert np.max(np.abs(a["forces"] - b["forces"])) <= 1e-9 * np.max(np.abs(a["forces"]))


def test_bucket_streams_leave_results_unchanged(params):
    # the bucket launches of an evaluation on 1 stream or spread over 4: the
    # buckets hold disjoint units, so every result bit is the same, for MD steps
    # (eager and graph-replayed) and for a plain evaluation
    s = subsystem(make_system(4, n_units=120), list(range(0, 120, 5)))
    ctx = make_ctx(params, s)
    assert sum(ctx.bucket_info(b)[0] > 0 for b in cd.binding.BUCKETS) >= 4
    with pytest.raises(cd.CavdftbError):
        ctx.set_bucket_streams(0)
    with pytest.raises(cd.CavdftbError):
        ctx.set_bucket_streams(5)
    ctx.close()
    runs = {}
    for n in (1, 4):
        for graph in (False, True):
            runs[n, graph] = _gpu_md(params, s, cd.BORN_MULLIKEN, 6, graph=graph,
                                     setup=lambda c, n=n: c.set_bucket_streams(n))[0]
    for key, out in runs.items():
        for name, a, b in zip(("r", "p", "qm", "pm", "obs"), runs[1, False], out):
            assert np.array_equal(a, b), (key, name)
    evals = []
    for n in (1, 4):
        ctx = make_ctx(params, s)
        ctx.set_bucket_streams(n)
        evals.append(gpu_eval(ctx, s["pos"]))
        ctx.close()
    for k in evals[0]:
        assert np.array_equal(evals[0][k], evals[1][k]), k


def test_failed_unit_gets_the_short_stagnation_window(params):
    # the 27-water unit of the uneven workload whose SCC does not converge, with a
    # unit that does: cold evaluations twice at the same geometry.  The first
    # stops after the full stagnation window, the second (the unit failed last
    # time) after the short one; both flag it, and the converging unit's results
    # are bitwise the same in both
    full = make_system(4)
    nw = np.diff(full["unit_off"]) // 3
    bad = 11611
    assert nw[bad] == 27
    s = subsystem(full, [bad, 0])
    ctx = make_ctx(params, s, tol=1e-8, max_iter=100)
    ctx.set_warm_start(False)
    g1 = gpu_eval(ctx, s["pos"])
    it1 = ctx.read_counters()["scc_iterations"]
    ctx.reset_counters()
    g2 = gpu_eval(ctx, s["pos"])
    it2 = ctx.read_counters()["scc_iterations"]
    assert g1["status"][0] & cd.binding.ST_NOT_CONVERGED and g2["status"][0] & cd.binding.ST_NOT_CONVERGED
    assert g1["status"][1] == 0 and g2["status"][1] == 0
    a0 = s["unit_off"][1]
    assert g1["energy"][1] == g2["energy"][1] and np.array_equal(g1["charges"][a0:], g2["charges"][a0:])
    assert it2 <= it1 - 10, (it1, it2)
    ctx.close()
