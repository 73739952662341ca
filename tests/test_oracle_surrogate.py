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
    G2 = sg.descriptors(np.array([0, 1]), two)
    g = G2[0]
    fc = sg.cutoff(np.array([r]))[0]
    assert g[:16].sum() == 0.0
    assert g[16:32].sum() == pytest.approx(fc * np.sqrt(2 * np.pi), rel=1e-3)
    # direction moments of that neighbour: the O (one H: lab frame) sees it along +x,
    # the H (frame e1 = O -> H = +x) sees the O along -x; the 8-Gaussian comb sums
    # to ~ fc sqrt(2 pi) as well, and the other components vanish
    vo = g[32:].reshape(2, 8, 3)
    assert np.all(vo[0] == 0.0) and np.all(vo[1][:, 1:] == 0.0)
    assert vo[1][:, 0].sum() == pytest.approx(fc * np.sqrt(2 * np.pi), rel=2e-2)
    vh = G2[1][32:].reshape(2, 8, 3)
    assert np.all(vh[1] == 0.0)
    assert vh[0][:, 0].sum() == pytest.approx(-fc * np.sqrt(2 * np.pi), rel=2e-2)
    assert np.allclose(vh[0][:, 1:], 0.0, atol=1e-15)


def test_direction_moments_mirror_across_the_molecular_plane():
    # a water in the xy plane (bisector +x, normal along z) and one more O above or
    # below that plane at mirror positions: only the component along the normal
    # (e2) changes sign; the radial comb and the in-plane components do not
    a = sg.ANG
    th = np.deg2rad(52.0)
    wat = np.array([[0.0, 0.0, 0.0], [0.96 * a * np.cos(th), 0.96 * a * np.sin(th), 0.0],
                    [0.96 * a * np.cos(th), -0.96 * a * np.sin(th), 0.0]])
    sp = np.array([0, 1, 1, 0])
    up = np.vstack([wat, [[2.9 * a, 0.8 * a, 1.1 * a]]])
    dn = np.vstack([wat, [[2.9 * a, 0.8 * a, -1.1 * a]]])
    Gu, Gd = sg.descriptors(sp, up)[0], sg.descriptors(sp, dn)[0]
    R = sg.local_frames(sp, up)[0]
    assert np.allclose(R[:, 0], [1.0, 0.0, 0.0], atol=1e-14) and abs(abs(R[2, 1]) - 1.0) < 1e-14
    assert np.array_equal(Gu[:32], Gd[:32])
    mu, md = Gu[32:].reshape(2, 8, 3), Gd[32:].reshape(2, 8, 3)
    assert np.allclose(mu[:, :, [0, 2]], md[:, :, [0, 2]], atol=1e-15)
    assert np.allclose(mu[:, :, 1], -md[:, :, 1], atol=1e-15)
    assert np.abs(mu[0, :, 1]).max() > 1e-3  # the O neighbour's normal component is there


def test_frames_of_fragments():
    # an O with one H and a lone H take the lab frame; an H whose O has no second
    # H keeps e1 = O -> H and an e2 normal to it
    a = sg.ANG
    sp = np.array([0, 1, 1])
    pos = np.array([[0.0, 0.0, 0.0], [0.6 * a, 0.7 * a, 0.2 * a], [9.0 * a, 0.0, 0.0]])
    R = sg.local_frames(sp[:2], pos[:2])
    assert np.array_equal(R[0], np.eye(3))
    e1 = pos[1] / np.linalg.norm(pos[1])
    Rh = R[1]
    assert np.allclose(Rh[:, 0], e1, atol=1e-15)
    assert np.allclose(Rh.T @ Rh, np.eye(3), atol=1e-14) and np.linalg.det(Rh) == pytest.approx(1.0, abs=1e-14)
    Rl = sg.local_frames(np.array([1, 1]), pos[1:])
    assert np.array_equal(Rl[0], np.eye(3)) and np.array_equal(Rl[1], np.eye(3))


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
    norms = [{"x_mean": np.zeros(sg.N_IN), "x_std": np.ones(sg.N_IN), "y_mean": np.zeros(9), "y_scale": np.full(9, 0.3)}
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
