"""Launch and solver settings chosen by measurement.

For one batch layout the SCC kernel's cost depends on a few settings that do
not change its results beyond the SCC tolerance:

  job_queue       device job queue over units ordered largest first, or a fixed
                  stride over the job list (cavdftb_set_schedule);
  max_wg_per_cu   resident workgroups per CU (1 or the occupancy maximum);
  jacobi_factor   stop of the full-Jacobi iterations relative to the charge
                  residual (cavdftb_set_tuning).

`tune` times a few warm MD steps of the real workload for every combination on
the GPU and returns the fastest; `apply` sets a result on a context.  The
choice is per workload (size mix, Born route), so the result is meant to be
stored next to the workload's run configuration.
"""
import itertools
import json
import time

from . import binding as B

CANDIDATES = {
    "job_queue": (True, False),
    "max_wg_per_cu": (0, 1),
    "jacobi_factor": (1e-4, 1e-3, 1e-2),
}


def apply(ctx, setting):
    ctx.set_schedule(setting["job_queue"], setting["max_wg_per_cu"])
    ctx.set_tuning(setting["jacobi_factor"], True)


def tune(params, system, born_mode=B.BORN_MULLIKEN, h=1e-3, steps=4, warmup=2, tol=None, log=None):
    """Returns (best setting, list of (setting, ms per MD step)).  Every candidate
    starts from the same state: a fresh context primed by `warmup` steps."""
    import torch
    dev = torch.device("cuda:0")
    masses = params["mass"][system["species"]]
    tol = system["workload"].scc_tol if tol is None else tol
    results = []
    keys = list(CANDIDATES)
    for values in itertools.product(*(CANDIDATES[k] for k in keys)):
        setting = dict(zip(keys, values))
        ctx = B.context_from_system(params, system)
        ctx.set_scc(tol, 200, 0.6)
        apply(ctx, setting)
        r = torch.tensor(system["pos"], device=dev)
        p = torch.tensor(system["vel"] * masses[:, None], device=dev)
        qm = torch.zeros(ctx.n_modes, dtype=torch.float64, device=dev)
        pm = torch.zeros_like(qm)
        ctx.init_photons(r, qm, pm)
        ctx.step(r, p, qm, pm, warmup, system["dt"], born_mode, h, None)
        ctx.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        ctx.step(r, p, qm, pm, steps, system["dt"], born_mode, h, None)
        ctx.sync()
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
        ctx.close()
        results.append((setting, ms))
        if log:
            log(f"  {json.dumps(setting)}: {ms:.3f} ms/step")
    best = min(results, key=lambda x: x[1])[0]
    return best, results


def main(argv=None):
    import argparse
    ap = argparse.ArgumentParser(description="choose SCC launch / solver settings for a workload by timing")
    ap.add_argument("--workload", type=int, default=2)
    ap.add_argument("--units", type=int, default=None)
    ap.add_argument("--born", choices=["mulliken", "fd", "field"], default=None)
    ap.add_argument("--steps", type=int, default=4)
    ap.add_argument("--out", default=None, help="write the best setting and all timings (JSON)")
    args = ap.parse_args(argv)
    from cavgen import make_params, make_system
    params = make_params()
    s = make_system(args.workload, n_units=args.units)
    born = args.born or s["workload"].born
    mode, h = {"mulliken": (B.BORN_MULLIKEN, 0.0), "fd": (B.BORN_FD, 1e-3), "field": (B.BORN_FIELD, 1e-4)}[born]

    def log(msg):
        print(msg, flush=True)
    best, res = tune(params, s, mode, h, steps=args.steps, log=log)
    log(f"best: {json.dumps(best)}")
    if args.out:
        with open(args.out, "w") as f:
            json.dump({"workload": args.workload, "born": born, "best": best,
                       "timings": [{"setting": st, "ms_per_step": ms} for st, ms in res]}, f, indent=1)
    return 0


if __name__ == "__main__":
    raise SystemExit(main())
