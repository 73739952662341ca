"""The allocation-free backward pass (cavdftb_sg_backward_noalloc) against the
entry point it is a variant of (cavdftb_sg_backward with a caller's work
buffer): the same kernels and the same fixed-order tile reduction, so the
gradients must agree bit for bit, on two calls in a row (the second with a
smaller batch, so the array holds the first call's partial sums when it
starts), and sizes beyond the array's limit are rejected."""
import numpy as np
import pytest

from oracle import surrogate as osg

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():  # pragma: no cover
    pytest.skip("no GPU", allow_module_level=True)

from paper_2512_03277_amd import binding as B  # noqa: E402

DEV = torch.device("cuda:0")


def _t(a, dtype=torch.float32):
    return torch.tensor(np.ascontiguousarray(a), dtype=dtype, device=DEV)


def _case(rng, n):
    th = osg.init_params(rng)
    w = _t(th)
    x = _t(rng.normal(size=(n, osg.N_IN)))
    y = torch.empty(n, 9, dtype=torch.float32, device=DEV)
    act = torch.empty(n, 256, dtype=torch.float32, device=DEV)
    B.sg_forward(w, x, n, y, act)
    dy = _t(rng.normal(size=(n, 9)) * 0.1)
    return w, x, act, dy


def test_noalloc_backward_equals_the_work_buffer_variant():
    rng = np.random.default_rng(5)
    for n in (B.SG_NOALLOC_MAX_ROWS, 1000, 150):      # full array, then smaller batches over stale contents
        w, x, act, dy = _case(rng, n)
        ref = torch.empty(osg.N_PARAM, dtype=torch.float32, device=DEV)
        work = torch.empty((n + 63) // 64, osg.N_PARAM, dtype=torch.float32, device=DEV)
        B.sg_backward(w, x, act, dy, n, ref, work)
        got = torch.full((osg.N_PARAM,), float("nan"), dtype=torch.float32, device=DEV)
        B.sg_backward_noalloc(w, x, act, dy, n, got)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), n
        assert torch.isfinite(got).all()


def test_noalloc_backward_matches_the_oracle_gradient():
    # the BF16-emulating oracle backward pass, to the bar of the surrogate tests
    rng = np.random.default_rng(6)
    n = 200
    th = osg.init_params(rng)
    x = rng.normal(size=(n, osg.N_IN))
    dy = rng.normal(size=(n, 9)) * 0.1
    _, cache = osg.forward(th, x, emulate_bf16=True)
    g_ref = osg.unpack(osg.backward(th, cache, dy, emulate_bf16=True))
    w, xt = _t(th), _t(x)
    y = torch.empty(n, 9, dtype=torch.float32, device=DEV)
    act = torch.empty(n, 256, dtype=torch.float32, device=DEV)
    B.sg_forward(w, xt, n, y, act)
    grad = torch.empty(osg.N_PARAM, dtype=torch.float32, device=DEV)
    B.sg_backward_noalloc(w, xt, act, _t(dy), n, grad)
    torch.cuda.synchronize()
    gg = osg.unpack(grad.cpu().numpy().astype(np.float64))
    for name in g_ref:
        assert np.max(np.abs(gg[name] - g_ref[name])) <= 1e-3 * np.max(np.abs(g_ref[name])), name


def test_noalloc_backward_rejects_oversized_batches():
    rng = np.random.default_rng(7)
    w, x, act, dy = _case(rng, 64)
    grad = torch.empty(osg.N_PARAM, dtype=torch.float32, device=DEV)
    with pytest.raises(B.CavdftbError):
        B.sg_backward_noalloc(w, x, act, dy, B.SG_NOALLOC_MAX_ROWS + 1, grad)
    with pytest.raises(B.CavdftbError):
        B.sg_backward_noalloc(w, x, act, dy, 0, grad)
