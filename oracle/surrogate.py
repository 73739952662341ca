"""Learned Born-charge surrogate (oracle, FP64 with a BF16-emulation mode).

The exact Born charges are the method's bottleneck (Results: the dipole
derivatives are evaluated numerically and dominate the cost; Conclusion).  The
surrogate replaces them by a small ensemble of per-species neural networks on
rotation-invariant descriptors, with exact finite differences as the
fallback where the ensemble disagrees.  Concrete form (the paper gives none;
each choice below is a reading, not the paper's):

  local frame  O: e1 = bisector of the two nearest H, e2 = normal of their
               plane; H: e1 = direction nearest O -> H, e2 = normal of the plane
               of that O and its two nearest H; e3 = e1 x e2.  R = [e1 e2 e3].
               Fragments that lack those atoms take the lab frame (local_frames).
  descriptors  radial comb, columns s*16 + k:
                 sum_{B != A, species B = s, R_AB < Rc} g_k(R_AB) fc(R_AB),
                 g_k(r) = exp(-(r - r_k)^2 / (2 sigma^2)), fc(r) = (cos(pi r / Rc) + 1) / 2,
                 16 centres r_k uniform on [0.5, 6] A, sigma = their spacing, Rc = 6 A;
               direction moments in the atom's own frame, columns 32 + s*24 + 3k + i:
                 sum_B g'_k(R_AB) fc(R_AB) (e_i . u_AB), u_AB the unit vector A -> B,
                 on 8 centres uniform on [0.5, 6] A (sigma' their spacing).
               80 inputs per atom.  The moments see where the neighbouring
               molecules sit relative to the atom's own molecule (hydrogen-bond
               geometry), which the radial comb cannot.
  network      per central species, per member: 80 -> 128 SiLU -> 128 SiLU -> 9,
               on standardised inputs x = (G - mu_x) / sd_x; the 9 outputs y
               give dZ_loc = (y * y_scale + y_mean) reshaped 3 x 3 (row-major),
               the correction to the paper's Mulliken replacement Q_A I in the
               atom's frame (the charge-flux part the replacement misses).
  prediction   Z = Q_A I + R dZ_loc R^T per member, with the exact Mulliken
               charge Q_A of the SCC; ensemble mean and per-component standard
               deviation; then per unit Z_A -= (1/N_a) sum_B Z_B (acoustic sum
               rule).  A unit whose largest standard deviation exceeds the
               threshold is recomputed by exact finite differences.
  training     mean squared error on the standardised local-frame targets,
               Adam with FP32 master weights, BF16 operands at every matrix
               product (round to nearest even), FP32 accumulation.

Pinned by: descriptor invariances (rigid motions, permutations), cutoff
smoothness, the radial comb sum and the moments of one neighbour, orthonormal
right-handed frames that rotate with the molecule, backward pass against
central finite differences, equivariance Z(QR) = Q Z(R) Q^T and an exact
acoustic sum rule, BF16 rounding against torch's bfloat16 conversion, and the
first Adam step (tests/test_oracle_surrogate.py).
"""
import math

import numpy as np

ANG = 1.8897261246
N_RAD = 16
RC = 6.0 * ANG
CENTRES = np.linspace(0.5, 6.0, N_RAD) * ANG
SIGMA = CENTRES[1] - CENTRES[0]
N_VEC = 8  # Gaussians of the direction moments
CENTRES_V = np.linspace(0.5, 6.0, N_VEC) * ANG
SIGMA_V = CENTRES_V[1] - CENTRES_V[0]
N_IN, N_HID, N_OUT = 2 * N_RAD + 2 * 3 * N_VEC, 128, 9
# flat parameter layout of one network
SHAPES = (("W1", (N_IN, N_HID)), ("b1", (N_HID,)), ("W2", (N_HID, N_HID)), ("b2", (N_HID,)),
          ("W3", (N_HID, N_OUT)), ("b3", (N_OUT,)))
N_PARAM = sum(int(np.prod(s)) for _, s in SHAPES)


def unpack(theta):
    out, o = {}, 0
    for name, shp in SHAPES:
        k = int(np.prod(shp))
        out[name] = np.asarray(theta[o:o + k]).reshape(shp)
        o += k
    return out


def pack(d):
    return np.concatenate([np.asarray(d[name], dtype=np.float64).ravel() for name, _ in SHAPES])


def unpack_norm(v):
    """The normalisation of one species from its flat layout
    [x_mean (N_IN) | x_std (N_IN) | y_mean (9) | y_scale (9)]."""
    v = np.asarray(v, dtype=np.float64)
    return {"x_mean": v[:N_IN], "x_std": v[N_IN:2 * N_IN], "y_mean": v[2 * N_IN:2 * N_IN + N_OUT],
            "y_scale": v[2 * N_IN + N_OUT:2 * N_IN + 2 * N_OUT]}


def init_params(rng):
    """He-style uniform initialisation of one network."""
    d = {}
    for name, shp in SHAPES:
        if name.startswith("W"):
            lim = math.sqrt(6.0 / shp[0]) * (0.5 if name == "W3" else 1.0)
            d[name] = rng.uniform(-lim, lim, size=shp)
        else:
            d[name] = np.zeros(shp)
    return pack(d)


# ---------------------------------------------------------------- BF16
def bf16(x):
    """Round float64 values to bfloat16 precision (round to nearest, ties to
    even, via the float32 bit pattern) and return them as float64."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    u = (u + 0x7FFF + lsb) & 0xFFFF0000
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


# ---------------------------------------------------------------- descriptors and frames
def cutoff(r):
    return np.where(r < RC, 0.5 * (np.cos(np.pi * r / RC) + 1.0), 0.0)


def descriptors(species, pos, frames=None):
    """G (Na, N_IN): the radial comb of each neighbour species (columns
    s*16 + k) and the frame-resolved first moments (columns 32 + s*24 + 3k + i)
    of the neighbours' directions, sum_B g_k(R_AB) fc(R_AB) (e_i(A) . u_AB),
    u_AB = (R_B - R_A) / R_AB, on an 8-Gaussian comb.  frames: local_frames of
    the unit (computed when not given)."""
    species = np.asarray(species)
    pos = np.asarray(pos, dtype=np.float64)
    na = len(species)
    R = local_frames(species, pos) if frames is None else np.asarray(frames)
    G = np.zeros((na, N_IN))
    for a in range(na):
        for b in range(na):
            if a == b:
                continue
            d = pos[b] - pos[a]
            r = float(np.linalg.norm(d))
            if r >= RC:
                continue
            fc = 0.5 * (math.cos(math.pi * r / RC) + 1.0)
            g = np.exp(-(r - CENTRES) ** 2 / (2.0 * SIGMA ** 2)) * fc
            G[a, species[b] * N_RAD:(species[b] + 1) * N_RAD] += g
            ga = np.exp(-(r - CENTRES_V) ** 2 / (2.0 * SIGMA_V ** 2)) * fc
            u = R[a].T @ (d / r)  # direction in the atom's frame
            o = 2 * N_RAD + species[b] * 3 * N_VEC
            G[a, o:o + 3 * N_VEC] += np.outer(ga, u).ravel()
    return G


def _unit(v):
    return v / np.linalg.norm(v)


def _nearest(pos, a, cand):
    d = [(float(np.linalg.norm(pos[c] - pos[a])), c) for c in cand if c != a]
    d.sort()
    return [c for _, c in d]


def _complete(e1):
    """A unit e2 normal to e1: the lab y axis (z when y is within 0.9 of e1)
    with its e1 part removed."""
    t = np.array([0.0, 1.0, 0.0]) if abs(e1[1]) <= 0.9 else np.array([0.0, 0.0, 1.0])
    return _unit(t - (t @ e1) * e1)


def local_frames(species, pos):
    """R (Na, 3, 3) with columns e1, e2, e3 in lab coordinates.  Fragments
    without the atoms a frame needs (an O with fewer than two H, an H without
    an O) take the lab frame; an H whose O has no second H takes e2 from
    _complete(e1)."""
    species = np.asarray(species)
    pos = np.asarray(pos, dtype=np.float64)
    na = len(species)
    Hs = [i for i in range(na) if species[i] == 1]
    Os = [i for i in range(na) if species[i] == 0]
    R = np.zeros((na, 3, 3))
    for a in range(na):
        e1, e2 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 1.0, 0.0])
        if species[a] == 0:
            near = _nearest(pos, a, Hs)
            if len(near) >= 2:
                h1, h2 = near[:2]
                u1, u2 = _unit(pos[h1] - pos[a]), _unit(pos[h2] - pos[a])
                e1 = _unit(u1 + u2)
                e2 = _unit(np.cross(u1, u2))
        elif Os:
            o = _nearest(pos, a, Os)[0]
            e1 = _unit(pos[a] - pos[o])
            others = [h for h in _nearest(pos, o, Hs) if h != a]
            if others:
                e2 = _unit(np.cross(pos[a] - pos[o], pos[others[0]] - pos[o]))
                e2 = _unit(e2 - (e2 @ e1) * e1)
            else:
                e2 = _complete(e1)
        e3 = np.cross(e1, e2)
        R[a] = np.stack([e1, e2, e3], axis=1)
    return R


# ---------------------------------------------------------------- network
def silu(z):
    return z / (1.0 + np.exp(-z))


def dsilu(z):
    s = 1.0 / (1.0 + np.exp(-z))
    return s * (1.0 + z * (1.0 - s))


def forward(theta, x, emulate_bf16=False):
    """x (n, N_IN) standardised inputs -> y (n, 9); returns (y, cache)."""
    p = unpack(theta)
    q = bf16 if emulate_bf16 else (lambda v: v)
    z1 = q(x) @ q(p["W1"]) + p["b1"]
    h1 = silu(z1)
    z2 = q(h1) @ q(p["W2"]) + p["b2"]
    h2 = silu(z2)
    y = q(h2) @ q(p["W3"]) + p["b3"]
    return y, {"x": x, "z1": z1, "h1": h1, "z2": z2, "h2": h2}


def backward(theta, cache, dy, emulate_bf16=False):
    """Gradient of sum(dy * y) with respect to the flat parameters."""
    p = unpack(theta)
    q = bf16 if emulate_bf16 else (lambda v: v)
    g = {}
    g["W3"] = q(cache["h2"]).T @ q(dy)
    g["b3"] = dy.sum(0)
    dh2 = q(dy) @ q(p["W3"]).T
    dz2 = dh2 * dsilu(cache["z2"])
    g["W2"] = q(cache["h1"]).T @ q(dz2)
    g["b2"] = dz2.sum(0)
    dh1 = q(dz2) @ q(p["W2"]).T
    dz1 = dh1 * dsilu(cache["z1"])
    g["W1"] = q(cache["x"]).T @ q(dz1)
    g["b1"] = dz1.sum(0)
    return pack(g)


def mse_and_grad(y, t):
    d = y - t
    n = d.size
    return float((d * d).sum() / n), 2.0 * d / n


def adam_step(theta, grad, m, v, t, lr=1e-3, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (Kingma & Ba 2015) with bias correction; t starts at 1."""
    m = b1 * m + (1.0 - b1) * grad
    v = b2 * v + (1.0 - b2) * grad * grad
    mh = m / (1.0 - b1 ** t)
    vh = v / (1.0 - b2 ** t)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v


# ---------------------------------------------------------------- prediction
def predict_unit(species, pos, nets, norms, charges, emulate_bf16=False):
    """nets[s] = list of flat parameter vectors (members) for species s;
    norms[s] = dict(x_mean, x_std, y_mean, y_scale); charges = Mulliken Q_A.
    Returns the ensemble mean Born tensors after the acoustic-sum projection
    (Na,3,3) and the per-atom per-component ensemble standard deviation."""
    species = np.asarray(species)
    R = local_frames(species, pos)
    G = descriptors(species, pos, R)
    na = len(species)
    members = len(nets[0])
    Zm = np.zeros((members, na, 3, 3))
    for s in (0, 1):
        idx = np.nonzero(species == s)[0]
        if len(idx) == 0:
            continue
        nm = norms[s]
        x = (G[idx] - nm["x_mean"]) / nm["x_std"]
        for mb in range(members):
            y, _ = forward(nets[s][mb], x, emulate_bf16)
            zl = (y * nm["y_scale"] + nm["y_mean"]).reshape(-1, 3, 3)
            Zm[mb, idx] = np.einsum("nij,njk,nlk->nil", R[idx], zl, R[idx])
    Zm = Zm + np.asarray(charges)[None, :, None, None] * np.eye(3)[None, None]
    mean = Zm.mean(0)
    std = Zm.std(0)
    mean = mean - mean.mean(0, keepdims=True)
    return mean, std


def to_local(Z, R, charges=None):
    """Training targets in the atom's frame: R^T Z R - Q I (the correction to the
    Mulliken replacement), or R^T Z R without charges."""
    zl = np.einsum("nji,njk,nkl->nil", R, Z, R)
    if charges is not None:
        zl = zl - np.asarray(charges)[:, None, None] * np.eye(3)[None]
    return zl
