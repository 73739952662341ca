"""Pins of the surrogate oracle (CPU only)."""
import numpy as np
import pytest

from cavgen import make_system
from oracle import surrogate as sg


@pytest.fixture(scope="module")
def cluster():
    s = make_system(2, n_units=1)
    return s["species"], s["pos"]


def _rot(seed):
    q, _ = np.linalg.qr(np.random.default_rng(seed).normal(size=(3, 3)))
    if np.linalg.det(q) < 0:
        q[:, 0] *= -1
    return q


def test_descriptors_invariant_and_cut_off(cluster):
    sp, pos = cluster
    G = sg.descriptors(sp, pos)
    Q = _rot(1)
    assert np.allclose(sg.descriptors(sp, pos @ Q.T + 2.0), G, rtol=0, atol=1e-13)
    perm = np.concatenate([np.arange(3 * i, 3 * i + 3) for i in (7, 3, 0, 5, 1, 2, 6, 4)])
    assert np.allclose(sg.descriptors(sp[perm], pos[perm]), G[perm], rtol=0, atol=1e-13)
    # a pair beyond the cutoff contributes nothing; the cutoff function and its slope vanish at Rc
    far = np.array([[0.0, 0.0, 0.0], [sg.RC + 1e-9, 0.0, 0.0]])
    assert np.all(sg.descriptors(np.array([0, 1]), far) == 0.0)
    h = 1e-6
    assert sg.cutoff(np.array([sg.RC - h]))[0] < 1e-11
    # one neighbour: the Gaussian comb sums to ~ fc(R) sqrt(2 pi) sigma / spacing in the grid interior
    r = 3.0 * sg.ANG
    two = np.array([[0.0, 0.0, 0.0], [r, 0.0, 0.0]])
    g = sg.descriptors(np.array([0, 1]), two)[0]
    assert g[:16].sum() == 0.0
    assert g[16:].sum() == pytest.approx(sg.cutoff(np.array([r]))[0] * np.sqrt(2 * np.pi), rel=1e-3)


def test_frames_orthonormal_right_handed_and_covariant(cluster):
    sp, pos = cluster
    R = sg.local_frames(sp, pos)
    for Ra in R:
        assert np.allclose(Ra.T @ Ra, np.eye(3), atol=1e-13)
        assert np.linalg.det(Ra) == pytest.approx(1.0, abs=1e-13)
    Q = _rot(2)
    R2 = sg.local_frames(sp, pos @ Q.T - 1.0)
    assert np.allclose(R2, np.einsum("ij,njk->nik", Q, R), atol=1e-12)


def test_backward_matches_central_differences():
    rng = np.random.default_rng(0)
    th = sg.init_params(rng)
    x = rng.normal(size=(7, sg.N_IN))
    t = rng.normal(size=(7, sg.N_OUT))
    y, cache = sg.forward(th, x)
    _, dy = sg.mse_and_grad(y, t)
    g = sg.backward(th, cache, dy)
    h = 1e-6
    for k in rng.choice(sg.N_PARAM, size=40, replace=False).tolist() + [sg.N_PARAM - 1, 0]:
        e = np.zeros_like(th)
        e[k] = h
        lp = sg.mse_and_grad(sg.forward(th + e, x)[0], t)[0]
        lm = sg.mse_and_grad(sg.forward(th - e, x)[0], t)[0]
        assert g[k] == pytest.approx((lp - lm) / (2 * h), rel=1e-6, abs=1e-10)


def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    v = np.concatenate([rng.normal(size=2000) * 10.0 ** rng.integers(-6, 6, size=2000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -2.5, 0.0]]).astype(np.float32)
    ref = torch.tensor(v).to(torch.bfloat16).to(torch.float32).numpy()
    assert np.array_equal(sg.bf16(v).astype(np.float32), ref)


def test_prediction_equivariant_with_exact_sum_rule(cluster):
    sp, pos = cluster
    rng = np.random.default_rng(4)
    nets = [[sg.init_params(rng) for _ in range(4)] for _ in range(2)]
    norms = [{"x_mean": np.zeros(32), "x_std": np.ones(32), "y_mean": np.zeros(9), "y_scale": np.full(9, 0.3)}
             for _ in range(2)]
    q = np.where(np.asarray(sp) == 0, -0.5, 0.25)
    Z, std = sg.predict_unit(sp, pos, nets, norms, q)
    assert np.max(np.abs(Z.sum(0))) < 1e-13
    Q = _rot(5)
    Z2, std2 = sg.predict_unit(sp, pos @ Q.T + 0.7, nets, norms, q)
    assert np.allclose(Z2, np.einsum("ij,njk,lk->nil", Q, Z, Q), atol=1e-12)
    assert np.all(std >= 0)
    Zb, _ = sg.predict_unit(sp, pos, nets, norms, q, emulate_bf16=True)
    assert np.max(np.abs(Zb - Z)) < 0.05 * np.max(np.abs(Z))   # BF16 operands: small, non-zero change
    assert np.max(np.abs(Zb - Z)) > 0.0


def test_first_adam_step_moves_by_lr_times_sign():
    th = np.array([1.0, -2.0, 3.0])
    g = np.array([0.5, -4.0, 1e-3])
    new, m, v = sg.adam_step(th, g, np.zeros(3), np.zeros(3), 1, lr=0.01)
    assert np.allclose(new - th, -0.01 * np.sign(g), rtol=1e-4)


def test_local_frame_round_trip(cluster):
    sp, pos = cluster
    R = sg.local_frames(sp, pos)
    Z = np.random.default_rng(6).normal(size=(len(sp), 3, 3))
    zl = sg.to_local(Z, R)
    assert np.allclose(np.einsum("nij,njk,nlk->nil", R, zl, R), Z, atol=1e-13)
    q = np.arange(len(sp)) * 0.01
    zq = sg.to_local(Z, R, q)
    assert np.allclose(zq + q[:, None, None] * np.eye(3), zl, atol=1e-14)
