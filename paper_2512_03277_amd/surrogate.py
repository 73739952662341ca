"""Training and evaluation driver of the learned Born-charge surrogate.

The exact Born charges (central finite differences of the SCC dipole) are the
method's bottleneck (Results; Conclusion).  This module builds their learned
replacement on the GPU with the library's own kernels:

  1. geometries from Mulliken-path cavity MD of 8-water clusters, plus
     sub-clusters of 1..7 waters cut from them (the surrogate is used on
     units of 1..8 waters);
  2. exact Born labels (cavdftb_born_charges: the force response to a uniform
     field, six SCCs per unit; or central differences of the dipole);
  3. descriptors, local frames and local-frame targets (sg_features,
     sg_to_local), standardisation statistics (sg_moments, sg_prep);
  4. per species and ensemble member: bootstrap resample, minibatch Adam on the
     mean squared error (sg_gather, sg_forward, sg_mse, sg_backward, sg_adam),
     FP32 master weights, BF16 operands.

The host only draws random numbers (initial weights, bootstrap and shuffle
indices) and sequences the calls; every arithmetic step is a kernel.
"""
import math
import time

import numpy as np

from . import binding as B


def _torch():
    import torch
    return torch


# ---------------------------------------------------------------- data
def md_snapshots(params, system, n_snap, stride, warm=10, dt=None, tol=1e-8, log=None):
    """Positions (device tensor [n_snap, n_atoms, 3]) every `stride` steps of
    Mulliken-path cavity MD after `warm` steps."""
    torch = _torch()
    dev = torch.device("cuda:0")
    ctx = B.context_from_system(params, system)
    ctx.set_scc(tol, 200, 0.5)
    masses = params["mass"][system["species"]]
    r = torch.tensor(system["pos"], device=dev)
    p = torch.tensor(system["vel"] * masses[:, None], device=dev)
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=dev)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    dt = system["dt"] if dt is None else dt
    ctx.step(r, p, qm, pm, warm, dt)
    out = torch.empty(n_snap, ctx.n_atoms, 3, dtype=torch.float64, device=dev)
    t0 = time.time()
    for k in range(n_snap):
        ctx.step(r, p, qm, pm, stride, dt)
        out[k].copy_(r)
        if log and (k % 16 == 15 or k == n_snap - 1):
            ctx.sync()
            log(f"  snapshot {k + 1}/{n_snap} ({time.time() - t0:.1f} s)")
    ctx.sync()
    ctx.close()
    return out


def sub_clusters(system, pos, rng):
    """Cut, from every 8-water unit of `system` at positions `pos` (host), a
    cluster of its first w molecules, w uniform on 1..7.  Returns a system dict
    (same cavity) of the cut units."""
    off = system["unit_off"]
    U = len(off) - 1
    w = rng.integers(1, 8, size=U)
    idx = np.concatenate([np.arange(off[u], off[u] + 3 * w[u]) for u in range(U)])
    new_off = np.concatenate([[0], np.cumsum(3 * w)]).astype(np.int32)
    out = dict(system)
    out.update({"species": system["species"][idx], "pos": pos[idx], "vel": system["vel"][idx],
                "unit_off": new_off})
    return out


def exact_born(params, system, pos_list, route="field", tol=1e-10, log=None):
    """Exact Born charges (route "field": force response to a uniform field of
    1e-4 a.u.; "fd": central differences of the dipole, h = 1e-3 bohr) and
    Mulliken charges for each position set (device tensors [n_atoms, 3]);
    returns (born [n_snap, n_atoms, 9], charges [n_snap, n_atoms], good
    [n_snap, n_atoms] (bool: the atom's unit evaluated with status 0), bad-unit
    count)."""
    mode, h = (B.BORN_FIELD, 1e-4) if route == "field" else (B.BORN_FD, 1e-3)
    torch = _torch()
    dev = torch.device("cuda:0")
    ctx = B.context_from_system(params, system)
    ctx.set_scc(tol, 300, 0.5)
    out = torch.empty(len(pos_list), ctx.n_atoms, 9, dtype=torch.float64, device=dev)
    q = torch.empty(len(pos_list), ctx.n_atoms, dtype=torch.float64, device=dev)
    st = torch.zeros(ctx.n_units, dtype=torch.int32, device=dev)
    st2 = torch.zeros_like(st)
    counts = torch.tensor(np.diff(system["unit_off"]).astype(np.int64), device=dev)
    good = torch.empty(len(pos_list), ctx.n_atoms, dtype=torch.bool, device=dev)
    bad = 0
    for k, pos in enumerate(pos_list):
        ctx.eval_units(pos.contiguous(), charges=q[k], unit_status=st)
        ctx.born_charges(pos.contiguous(), mode, h, out[k], st2)
        ok = (st == 0) & (st2 == 0)
        good[k] = torch.repeat_interleave(ok, counts)
        bad += int((~ok).sum())
        if log and (k % 16 == 15 or k == len(pos_list) - 1):
            log(f"  labels {k + 1}/{len(pos_list)}")
    ctx.sync()
    ctx.close()
    return out, q, good, bad


def features_and_targets(params, system, pos_list, born, charges, good=None):
    """Per species: descriptor rows (FP64 [N_s, SG_N_IN]) and local-frame targets,
    the correction R^T Z R - Q I to the Mulliken replacement (FP64 [N_s, 9]),
    over all snapshots; atoms of units without a clean evaluation (good False)
    are left out."""
    torch = _torch()
    dev = torch.device("cuda:0")
    ctx = B.context_from_system(params, system)
    NA = ctx.n_atoms
    sp = torch.tensor(system["species"], device=dev)
    feats = [[], []]
    targs = [[], []]
    feat = torch.empty(NA, B.SG_N_IN, dtype=torch.float64, device=dev)
    frames = torch.empty(NA, 9, dtype=torch.float64, device=dev)
    zl = torch.empty(NA, 9, dtype=torch.float64, device=dev)
    for k, pos in enumerate(pos_list):
        ctx.sg_features(pos.contiguous(), feat, frames)
        B.sg_to_local(frames, born[k].contiguous(), charges[k].contiguous(), None, NA, zl)
        for s in (0, 1):
            m = sp == s
            if good is not None:
                m = m & good[k]
            feats[s].append(feat[m].clone())
            targs[s].append(zl[m].clone())
    ctx.sync()
    ctx.close()
    return [torch.cat(feats[s]) for s in (0, 1)], [torch.cat(targs[s]) for s in (0, 1)]


# ---------------------------------------------------------------- training
def init_params(rng):
    """Uniform +-sqrt(6/fan_in) weights (half width for the output layer), zero biases."""
    parts = []
    for fan_in, fan_out, scale in ((B.SG_N_IN, 128, 1.0), (128, 128, 1.0), (128, B.SG_N_OUT, 0.5)):
        lim = scale * math.sqrt(6.0 / fan_in)
        parts.append(rng.uniform(-lim, lim, size=fan_in * fan_out))
        parts.append(np.zeros(fan_out))
    return np.concatenate(parts).astype(np.float32)


def norm_from_data(feat, targ):
    """[x_mean 32 | x_std 32 | y_mean 9 | y_scale 9] from the data (kernel moments)."""
    torch = _torch()
    dev = feat.device
    out = torch.empty(B.SG_N_NORM, dtype=torch.float32, device=dev)
    B.sg_moments(feat.contiguous(), None, feat.shape[0], B.SG_N_IN, out[:2 * B.SG_N_IN])
    B.sg_moments(targ.contiguous(), None, targ.shape[0], B.SG_N_OUT, out[2 * B.SG_N_IN:])
    return out


def train_network(feat, targ, norm, rng, epochs=40, batch=512, lr=2e-3, lr_final=1e-4, bootstrap=True,
                  log=None):
    """Train one network on standardised data; returns (params, last epoch loss)."""
    torch = _torch()
    dev = feat.device
    N = feat.shape[0]
    x_all = torch.empty(N, B.SG_N_IN, dtype=torch.float32, device=dev)
    t_all = torch.empty(N, B.SG_N_OUT, dtype=torch.float32, device=dev)
    B.sg_prep(feat.contiguous(), None, N, B.SG_N_IN, norm[:2 * B.SG_N_IN], x_all)
    B.sg_prep(targ.contiguous(), None, N, B.SG_N_OUT, norm[2 * B.SG_N_IN:], t_all)
    w = torch.tensor(init_params(rng), device=dev)
    m = torch.zeros_like(w)
    v = torch.zeros_like(w)
    grad = torch.empty_like(w)
    xb = torch.empty(batch, B.SG_N_IN, dtype=torch.float32, device=dev)
    tb = torch.empty(batch, B.SG_N_OUT, dtype=torch.float32, device=dev)
    yb = torch.empty(batch, B.SG_N_OUT, dtype=torch.float32, device=dev)
    dyb = torch.empty_like(yb)
    act = torch.empty(batch, 2 * 128, dtype=torch.float32, device=dev)
    work = torch.empty((batch + 63) // 64, B.SG_N_PARAM, dtype=torch.float32, device=dev)
    lwork = torch.empty((batch * B.SG_N_OUT + 255) // 256, dtype=torch.float32, device=dev)
    loss = torch.zeros(1, dtype=torch.float32, device=dev)
    sample = rng.integers(0, N, size=N) if bootstrap else np.arange(N)
    nb = N // batch
    step = 0
    last = None
    for ep in range(epochs):
        perm = torch.tensor(sample[rng.permutation(N)].astype(np.int32), device=dev)  # one upload per epoch
        lr_ep = lr * (lr_final / lr) ** (ep / max(epochs - 1, 1))
        tot = torch.zeros(1, dtype=torch.float32, device=dev)
        for b in range(nb):
            idx = perm[b * batch:(b + 1) * batch]
            B.sg_gather(x_all, idx, batch, B.SG_N_IN, xb)
            B.sg_gather(t_all, idx, batch, B.SG_N_OUT, tb)
            B.sg_forward(w, xb, batch, yb, act)
            B.sg_mse(yb, tb, batch * B.SG_N_OUT, dyb, loss, lwork)
            B.sg_backward(w, xb, act, dyb, batch, grad, work)
            step += 1
            B.sg_adam(w, grad, m, v, w.numel(), lr_ep, 0.9, 0.999, 1e-8, step)
            tot += loss
        last = float(tot) / max(nb, 1)
        if log:
            log(f"    epoch {ep:3d} lr {lr_ep:.2e} loss {last:.5f}")
    return w, last


def train_ensemble(feats, targs, seed=0, epochs=40, batch=512, lr=2e-3, log=None):
    """params [2][members][N_PARAM] and norm [2][N_NORM] (FP32 device tensors)."""
    torch = _torch()
    dev = feats[0].device
    params = torch.empty(2, B.SG_MEMBERS, B.SG_N_PARAM, dtype=torch.float32, device=dev)
    norms = torch.empty(2, B.SG_N_NORM, dtype=torch.float32, device=dev)
    losses = {}
    for s in (0, 1):
        norms[s] = norm_from_data(feats[s], targs[s])
        for mb in range(B.SG_MEMBERS):
            rng = np.random.default_rng(seed * 1000 + s * 10 + mb)
            t0 = time.time()
            w, last = train_network(feats[s], targs[s], norms[s], rng, epochs=epochs, batch=batch, lr=lr, log=log)
            params[s, mb] = w
            losses[(s, mb)] = last
            if log:
                log(f"  species {s} member {mb}: final loss {last:.5f} ({time.time() - t0:.1f} s)")
    return params, norms, losses


# ---------------------------------------------------------------- evaluation
def evaluate(params_sg, norm_sg, params, system, pos_list, born_exact, h=1e-3, thr=1e9, good=None):
    """RMSE (elementary charges, over atoms x 9 components) of the surrogate
    (fallback disabled unless thr is finite) and of the Mulliken replacement
    Z = Q I against the exact Born charges, over the atoms marked good.
    Returns a dict."""
    torch = _torch()
    dev = torch.device("cuda:0")
    ctx = B.context_from_system(params, system)
    ctx.set_scc(1e-10, 300, 0.5)
    ctx.set_surrogate(params_sg.contiguous().view(-1), norm_sg.contiguous().view(-1), thr)
    NA = ctx.n_atoms
    zs = torch.empty(NA, 9, dtype=torch.float64, device=dev)
    zm = torch.empty(NA, 9, dtype=torch.float64, device=dev)
    std = torch.empty(NA, dtype=torch.float64, device=dev)
    se_s = se_m = 0.0
    cnt = 0
    max_std = []
    for k, pos in enumerate(pos_list):
        ctx.born_charges(pos.contiguous(), B.BORN_SURROGATE, h, zs, None, std)
        ctx.born_charges(pos.contiguous(), B.BORN_MULLIKEN, h, zm)
        ex = born_exact[k]
        w = good[k][:, None].to(ex.dtype) if good is not None else torch.ones_like(ex[:, :1])
        se_s += float((((zs - ex) ** 2) * w).sum())
        se_m += float((((zm - ex) ** 2) * w).sum())
        cnt += int(w.sum()) * ex.shape[1]
        max_std.append(float(std.max()))
    cnt_fallback = ctx.read_counters()["surrogate_fallback_units"]
    ctx.close()
    return {"rmse_surrogate": math.sqrt(se_s / cnt), "rmse_mulliken": math.sqrt(se_m / cnt),
            "max_ensemble_std": max(max_std), "fallback_units": cnt_fallback}


def build_training_set(params, n_units=1024, n_train=16, n_val=4, stride=10, n_sub=4, seed=0, log=None,
                       route="field", workload=3):
    """Geometries, exact labels and features for training and validation (time
    blocks: the validation snapshots come after the training ones)."""
    from cavgen import make_system
    rng = np.random.default_rng(seed)
    s = make_system(workload, n_units=n_units)  # 8-water clusters (workloads 2 and 3)
    t0 = time.time()
    snaps = md_snapshots(params, s, n_train + n_val, stride, log=log)
    if log:
        log(f"sampled {n_train + n_val} snapshots of {n_units} units in {time.time() - t0:.1f} s")
    t0 = time.time()
    born, charges, good, bad = exact_born(params, s, list(snaps), route=route, log=log)
    if log:
        log(f"exact Born labels: {len(snaps)} x {n_units} units in {time.time() - t0:.1f} s ({bad} bad units)")
    sub_pos, sub_sys = [], []
    host = snaps.cpu().numpy()
    for k in range(min(n_sub, n_train)):
        ss = sub_clusters(s, host[k], rng)
        sub_sys.append(ss)
        sub_pos.append(ss["pos"])
    fe_t, ta_t = features_and_targets(params, s, list(snaps[:n_train]), born[:n_train], charges[:n_train],
                                      good[:n_train])
    torch = _torch()
    for ss in sub_sys:
        p = [torch.tensor(ss["pos"], device=snaps.device)]
        bz, qz, gz, _ = exact_born(params, ss, p, route=route)
        f2, t2 = features_and_targets(params, ss, p, bz, qz, gz)
        for sp in (0, 1):
            fe_t[sp] = torch.cat([fe_t[sp], f2[sp]])
            ta_t[sp] = torch.cat([ta_t[sp], t2[sp]])
    return {"system": s, "train": (fe_t, ta_t), "val_pos": list(snaps[n_train:]), "val_born": born[n_train:],
            "val_good": good[n_train:], "sub_systems": sub_sys}


def main(argv=None):
    import argparse
    import os
    ap = argparse.ArgumentParser(description="train the Born-charge surrogate ensemble on the GPU")
    ap.add_argument("--units", type=int, default=1024)
    ap.add_argument("--workload", type=int, default=3, choices=[2, 3], help="source of the 8-water clusters")
    ap.add_argument("--train-snapshots", type=int, default=16)
    ap.add_argument("--val-snapshots", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=40)
    ap.add_argument("--stride", type=int, default=10, help="MD steps between training snapshots")
    ap.add_argument("--batch", type=int, default=512)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--sub", type=int, default=4, help="snapshots also cut into 1..7-water sub-clusters")
    ap.add_argument("--route", choices=["field", "fd"], default="field", help="exact route of the labels")
    ap.add_argument("--dump", default=None, help="also save a sample of the training rows (npz) for inspection")
    ap.add_argument("--no-train", action="store_true")
    ap.add_argument("--out", default=os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                                                  "surrogate_ensemble.npz"))
    args = ap.parse_args(argv)
    from cavgen import make_params
    params = make_params()

    def log(msg):
        print(msg, flush=True)
    data = build_training_set(params, n_units=args.units, n_train=args.train_snapshots, n_val=args.val_snapshots,
                              stride=args.stride, n_sub=args.sub, log=log, route=args.route, workload=args.workload)
    fe, ta = data["train"]
    n_sub_geo = sum(len(ss["unit_off"]) - 1 for ss in data["sub_systems"])
    log(f"training geometries: {args.train_snapshots * args.units} clusters + {n_sub_geo} sub-clusters; "
        f"atoms: O {fe[0].shape[0]}, H {fe[1].shape[0]}")
    if args.dump:
        rng = np.random.default_rng(1)
        out = {}
        for sp in (0, 1):
            pick = rng.choice(fe[sp].shape[0], size=min(20000, fe[sp].shape[0]), replace=False)
            out[f"feat{sp}"] = fe[sp][pick].cpu().numpy()
            out[f"targ{sp}"] = ta[sp][pick].cpu().numpy()
        np.savez(args.dump, **out)
        log(f"wrote {args.dump}")
    if args.no_train:
        return 0
    t0 = time.time()
    psg, nsg, losses = train_ensemble(fe, ta, epochs=args.epochs, batch=args.batch, lr=args.lr, log=log)
    log(f"training took {time.time() - t0:.1f} s")
    ev = evaluate(psg, nsg, params, data["system"], data["val_pos"], data["val_born"], good=data["val_good"])
    log(f"held-out: {ev}")
    os.makedirs(os.path.dirname(args.out), exist_ok=True)
    n_sub_geo = sum(len(ss["unit_off"]) - 1 for ss in data["sub_systems"])
    n_train_geo = args.train_snapshots * args.units + n_sub_geo
    np.savez(args.out, params=psg.cpu().numpy(), norm=nsg.cpu().numpy(),
             rmse_surrogate=ev["rmse_surrogate"], rmse_mulliken=ev["rmse_mulliken"],
             rmse_heldout_surrogate=ev["rmse_surrogate"], rmse_heldout_mulliken=ev["rmse_mulliken"],
             heldout_geometries=args.val_snapshots * args.units, train_geometries=n_train_geo,
             train_atoms_o=fe[0].shape[0], train_atoms_h=fe[1].shape[0], stride_steps=args.stride,
             epochs=args.epochs)
    log(f"wrote {args.out}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
