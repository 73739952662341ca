"""MD steps replayed from a captured hipGraph (cavdftb_set_graph) against the
same steps issued eagerly: every call's state and observables bitwise, for the
Mulliken, field, displacement and surrogate (with device-side fallback
compaction) routes, with the program's own eager work and synchronisations
between the replays.
"""
import numpy as np
import pytest

from cavgen import make_params, make_system
from oracle import surrogate as osg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

import paper_2512_03277_amd as cd  # noqa: E402

DEV = torch.device("cuda:0")
CALLS, STEPS = 3, 4


@pytest.fixture(scope="module")
def params():
    return make_params()


def _t(a, dtype=torch.float64):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _subsystem(s, units):
    off = s["unit_off"]
    idx = np.concatenate([np.arange(off[u], off[u + 1]) for u in units])
    out = dict(s)
    out.update({"species": s["species"][idx], "pos": s["pos"][idx], "vel": s["vel"][idx],
                "unit_off": np.concatenate([[0], np.cumsum([off[u + 1] - off[u] for u in units])]).astype(np.int32),
                "unit_x": s["unit_x"][list(units)]})
    return out


def _ensemble(seed=3):
    rng = np.random.default_rng(seed)
    P = np.stack([np.stack([osg.init_params(rng) for _ in range(4)]) for _ in range(2)]).astype(np.float32)
    N = np.stack([np.concatenate([rng.uniform(0, 1, osg.N_IN), rng.uniform(0.5, 2, osg.N_IN), rng.normal(0, 0.2, 9),
                                  rng.uniform(0.05, 0.2, 9)]) for _ in range(2)]).astype(np.float32)
    return _t(P, torch.float32), _t(N, torch.float32)


def _run(params, s, mode, h, graph, stream, surrogate=None):
    """CALLS calls of STEPS MD steps; the state and obs after every call."""
    masses = params["mass"][s["species"]]
    with torch.cuda.stream(stream):
        ctx = cd.context_from_system(params, s, stream=stream)
        ctx.set_scc(1e-10, 200, 0.2)
        if surrogate is not None:
            ctx.set_surrogate(surrogate[0].view(-1), surrogate[1].view(-1), 0.3)
            ctx.set_fallback(cd.BORN_FIELD)
        ctx.set_graph(graph)
        r = _t(s["pos"])
        p = _t(s["vel"] * masses[:, None])
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
        pm = torch.zeros_like(qm)
        obs = torch.zeros(STEPS, cd.N_OBS, dtype=torch.float64, device=DEV)
        ctx.init_photons(r, qm, pm)
        out = []
        for _ in range(CALLS):
            ctx.step(r, p, qm, pm, STEPS, s["dt"], mode, h, obs)
            ctx.sync()
            out.append([x.cpu().numpy().copy() for x in (r, p, qm, pm, obs)])
            # eager work of the program between replays
            junk = (r * 2.0 + 1.0).square().sum()
            torch.cuda.synchronize()
            assert torch.isfinite(junk)
        cnt = ctx.read_counters()
    return ctx, out, cnt


@pytest.mark.parametrize("route", ["mulliken", "field", "fd", "surrogate"])
def test_graph_replays_match_eager_steps(params, route):
    s = _subsystem(make_system(4, n_units=40), list(range(0, 40, 4)))  # several orbital buckets
    if route == "surrogate":
        s = make_system(5, n_units=12)
    mode = {"mulliken": cd.BORN_MULLIKEN, "field": cd.BORN_FIELD, "fd": cd.BORN_FD,
            "surrogate": cd.BORN_SURROGATE}[route]
    h = 1e-4 if route in ("field", "surrogate") else 1e-3
    sg = _ensemble() if route == "surrogate" else None
    stream = torch.cuda.Stream()  # default priority; the null stream cannot be captured
    _, eager, ce = _run(params, s, mode, h, False, stream, sg)
    ctx, graph, cg = _run(params, s, mode, h, True, stream, sg)
    for c in range(CALLS):
        for name, a, b in zip(("r", "p", "qm", "pm", "obs"), eager[c], graph[c]):
            assert np.array_equal(a, b), (route, c, name)
    # the first call's first two steps run eagerly (charge extrapolation not yet at
    # full depth), every later step replays the one captured graph
    assert ce["graph_replays"] == 0 and ce["graph_captures"] == 0
    assert cg["graph_captures"] == 1
    assert cg["graph_replays"] == CALLS * STEPS - 2
    assert cg["scc_launches"] == ce["scc_launches"]
    ctx.close()


def test_graph_recaptures_after_a_setting_change(params):
    s = _subsystem(make_system(4, n_units=40), list(range(0, 40, 8)))
    stream = torch.cuda.Stream()
    masses = params["mass"][s["species"]]
    with torch.cuda.stream(stream):
        ctx = cd.context_from_system(params, s, stream=stream)
        ctx.set_scc(1e-10, 200, 0.2)
        ctx.set_graph(True)
        r = _t(s["pos"])
        p = _t(s["vel"] * masses[:, None])
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=DEV)
        pm = torch.zeros_like(qm)
        ctx.init_photons(r, qm, pm)
        ctx.step(r, p, qm, pm, 5, s["dt"], cd.BORN_MULLIKEN, 0.0, None)
        ctx.sync()
        assert ctx.read_counters()["graph_captures"] == 1
        ctx.set_scc(1e-10, 150, 0.2)  # same solver, new setting: the graph is stale
        ctx.step(r, p, qm, pm, 2, s["dt"], cd.BORN_MULLIKEN, 0.0, None)
        ctx.sync()
        c = ctx.read_counters()
        assert c["graph_captures"] == 2 and c["graph_replays"] == 5
        ctx.set_graph(False)
        ctx.step(r, p, qm, pm, 1, s["dt"], cd.BORN_MULLIKEN, 0.0, None)
        ctx.sync()
        assert ctx.read_counters()["graph_replays"] == 5
        assert torch.isfinite(r).all()
        ctx.close()


def test_graph_needs_a_capturable_stream(params):
    s = make_system(1)
    ctx = cd.context_from_system(params, s)  # null stream
    with pytest.raises(RuntimeError):
        ctx.set_graph(True)
    ctx.set_graph(False)
    ctx.close()
