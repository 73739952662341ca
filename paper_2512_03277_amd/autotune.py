"""Per-bucket launch schedules chosen by measurement, stored as a launch table.

Units are grouped into orbital buckets (8 ... 192 orbitals); each bucket is one
SCC-kernel launch per evaluation.  Per bucket the cost depends on settings that
do not change the physics:

  wg_per_cu   resident workgroups per CU (1 .. the maximum its LDS, registers
              and scratch allow): more workgroups hide latency, fewer leave
              each more cache;
  job_queue   device job queue over the units ordered by their last cost
              (longest first), or a fixed stride over the list;
  eig_mode    for buckets above 64 orbitals, the full diagonalisation by the
              tridiagonal solver (CAVDFTB_EIG_AUTO) or by cyclic Jacobi
              (CAVDFTB_EIG_JACOBI).

The workgroup count and job order leave every result bit unchanged; the
eigensolver changes results within the SCC tolerance.

`tune` searches one bucket at a time, largest estimated cost first, the other
buckets at their current best (coordinate search).  The timed work is the SCC
evaluation of an MD step (with its Born route): warm-started evaluations that
alternate between two geometries one MD step apart, taken after a few MD
steps of the workload, so every candidate does the same work (a running
trajectory of these synthetic clusters heats, and its step time drifts by
large factors).  Each candidate is timed right after the incumbent and
replaces it only when faster by more than `min_gain`, so timing noise does
not pick settings.
`table_json` writes the result as a launch table (one flat object per bucket with "arch" and
"bucket"), which the library reads with cavdftb_load_launch_table.
"""
import itertools
import json
import time

from . import binding as B


def _candidates(bucket, wg_max):
    wgs = list(range(1, wg_max + 1))
    eigs = (B.EIG_AUTO, B.EIG_JACOBI) if bucket > 64 else (B.EIG_AUTO,)
    return [{"wg_per_cu": w, "job_queue": q, "eig_mode": e} for w, q, e in itertools.product(wgs, (1, 0), eigs)]


def apply(ctx, table_entries):
    for e in table_entries:
        ctx.set_bucket_schedule(e["bucket"], e["wg_per_cu"], e["eig_mode"], e["job_queue"])


def tune(params, system, born_mode=B.BORN_MULLIKEN, h=1e-3, steps=4, warmup=3, tol=None, max_iter=100,
         mix_alpha=0.6, min_gain=0.01, log=None):
    """Returns (entries, timings, ms per step at the defaults, ms per step with
    the entries), the last two timed back to back at the end of the search.
    entries: one dict per bucket present in the layout."""
    import torch
    dev = torch.device("cuda:0")
    masses = params["mass"][system["species"]]
    tol = system["workload"].scc_tol if tol is None else tol
    ctx = B.context_from_system(params, system)
    ctx.set_scc(tol, max_iter, mix_alpha)
    r = torch.tensor(system["pos"], device=dev)
    p = torch.tensor(system["vel"] * masses[:, None], device=dev)
    qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=dev)
    pm = torch.zeros_like(qm)
    ctx.init_photons(r, qm, pm)
    ctx.step(r, p, qm, pm, warmup, system["dt"], born_mode, h, None)
    ctx.sync()
    # two nearby geometries an MD step apart; evaluations alternate between them,
    # each warm-started from the other's stored basis and charges, which is the
    # SCC work of an MD step without the drift of a running trajectory
    pos_a = r.clone()
    pos_b = (r + system["dt"] * p / torch.tensor(masses, device=dev)[:, None]).contiguous()
    U, NA = ctx.n_units, ctx.n_atoms
    ustat = torch.zeros(U, dtype=torch.int32, device=dev)
    en = torch.zeros(U, dtype=torch.float64, device=dev)
    fo = torch.zeros(NA, 3, dtype=torch.float64, device=dev)
    born = torch.zeros(NA, 9, dtype=torch.float64, device=dev)

    def evaluate(pos):
        if born_mode == B.BORN_MULLIKEN:
            ctx.eval_units(pos, en, fo, None, None, ustat)
        else:
            ctx.born_charges(pos, born_mode, h, born, ustat)

    def measure():
        evaluate(pos_a)  # untimed: the first evaluation after a setting change
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(steps):
            evaluate(pos_b if i % 2 == 0 else pos_a)
        ctx.sync()
        torch.cuda.synchronize()
        return 1e3 * (time.perf_counter() - t0) / steps

    present = []
    for b in B.BUCKETS:
        n_units, wg_max, wg_cur = ctx.bucket_info(b)
        if n_units > 0:
            present.append((n_units * (b / 48.0) ** 3, b, wg_max, wg_cur))
    present.sort(reverse=True)
    current = {b: {"wg_per_cu": wg_cur, "job_queue": 1, "eig_mode": B.EIG_AUTO} for _, b, _, wg_cur in present}

    def put(b, st):
        ctx.set_bucket_schedule(b, st["wg_per_cu"], st["eig_mode"], st["job_queue"])

    for b, st in current.items():
        put(b, st)
    start = measure()
    timings = [{"tried_bucket": None, "setting": None, "ms_per_eval": start}]
    if log:
        log(f"  defaults {start:.3f} ms/eval")
    # paired comparison: the incumbent is timed right before each candidate
    for _, b, wg_max, _ in present:
        for cand in _candidates(b, wg_max):
            if cand == current[b]:
                continue
            put(b, current[b])
            ms_inc = measure()
            put(b, cand)
            ms = measure()
            timings.append({"tried_bucket": b, "setting": cand, "ms_per_eval": ms, "incumbent_ms_per_eval": ms_inc})
            if log:
                log(f"  bucket {b}: {json.dumps(cand)} {ms:.3f} ms/eval (incumbent {ms_inc:.3f})")
            if ms < ms_inc * (1.0 - min_gain):
                current[b] = cand
        put(b, current[b])
    # final paired comparison: every bucket at its default, then the table
    defaults = {b: {"wg_per_cu": wg_cur, "job_queue": 1, "eig_mode": B.EIG_AUTO} for _, b, _, wg_cur in present}
    for b, st in defaults.items():
        put(b, st)
    baseline = measure()
    for b, st in current.items():
        put(b, st)
    final = measure()
    ctx.close()
    entries = [dict({"arch": "gfx950", "bucket": b}, **current[b]) for b in sorted(current)]
    return entries, timings, baseline, final


def table_json(entries, timings, workload, born, baseline_ms, tuned_ms):
    """The launch table as JSON text: "entries" are the objects the library
    applies; the timing records name their bucket "tried_bucket" so that they
    are not read as entries."""
    return json.dumps({"arch": "gfx950", "tuned_on": {"workload": workload, "born": born},
                       "baseline_ms_per_eval": baseline_ms, "tuned_ms_per_eval": tuned_ms,
                       "entries": entries, "timings": timings}, indent=1)


def main(argv=None):
    import argparse
    import os
    ap = argparse.ArgumentParser(description="choose per-bucket SCC launch schedules for a workload by timing")
    ap.add_argument("--workload", type=int, default=4)
    ap.add_argument("--units", type=int, default=None)
    ap.add_argument("--born", choices=["mulliken", "fd", "field"], default=None)
    ap.add_argument("--steps", type=int, default=4, help="timed evaluations per candidate")
    ap.add_argument("--out", default=None, help="launch table to write (default: the package's data directory)")
    args = ap.parse_args(argv)
    from cavgen import make_params, make_system
    params = make_params()
    s = make_system(args.workload, n_units=args.units)
    born = args.born or s["workload"].born
    mode, h = {"mulliken": (B.BORN_MULLIKEN, 0.0), "fd": (B.BORN_FD, 1e-3), "field": (B.BORN_FIELD, 1e-4),
               "surrogate": (B.BORN_MULLIKEN, 0.0)}[born]

    def log(msg):
        print(msg, flush=True)
    entries, timings, base, final = tune(params, s, mode, h, steps=args.steps, log=log)
    log(f"tuned: {base:.3f} -> {final:.3f} ms/eval")
    out = args.out or os.path.join(os.path.dirname(os.path.abspath(__file__)), "data",
                                   f"launch_table_gfx950_w{args.workload}.json")
    with open(out, "w") as f:
        f.write(table_json(entries, timings, args.workload, born, base, final))
    log(f"wrote {out}")
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
