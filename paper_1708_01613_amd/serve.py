"""Drivers for the batched-ensemble and served-stream workloads.

Both compare the library's batched forms with a sequential baseline that runs
each lattice alone, one after the other, with per-step launches of the
single-lattice kernels (flb_step):

* ensemble(members, steps): every member advances `steps` steps.  Batched:
  one flb_batch (autotuned tiles, steps replayed from captured HIP graphs).
* served(trace): jobs arrive at the trace's Poisson times.  Server mode
  submits each job at its arrival time and pumps the job server (admission
  by device footprint, continuous batching, FIFO or shortest-remaining-work
  scheduling); sequential mode runs the jobs first-come first-served, one at
  a time.  Completion latency is measured
  from arrival to the round that finished the job.

Aggregate MLUPS = sum over jobs of cells x steps / makespan.
"""
import time

import numpy as np

from . import foamlbm


def _cells(p):
    return p["nx"] * p["ny"] * p.get("nz", 1)


def ensemble(members, steps, mode="batched", autotune=True, log=None):
    import torch

    total = sum(_cells(p) for p, _ in members) * steps
    if mode in ("batched", "persistent"):
        b = foamlbm.Batch([p for p, _ in members])
        if mode == "persistent":
            b.set_persistent(True)
        for k, (_, nuc) in enumerate(members):
            b.members[k].set_nuclei(nuc)
        b.synchronize()
        tuned_ms = b.autotune(reps=3) if autotune else None
        tuning = b.tuning()
        b.step(1)  # first capture and table build outside the timed region
        b.synchronize()
        t0 = time.perf_counter()
        b.step(steps)
        b.synchronize()
        dt = time.perf_counter() - t0
        total = sum(_cells(p) for p, _ in members) * steps
        out = dict(mode=mode, seconds=dt, MLUPS=total / dt / 1e6, tuning=tuning, autotune_ms=tuned_ms)
        b.close()
        return out
    sims = []
    for p, nuc in members:
        s = foamlbm.Sim(**p)
        s.set_nuclei(nuc)
        s.step(1)
        sims.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in sims:
        s.step(steps)
        s.stream.synchronize()
    dt = time.perf_counter() - t0
    for s in sims:
        s.close()
    return dict(mode=mode, seconds=dt, MLUPS=total / dt / 1e6)


def offered_mlups(trace, rate):
    """Lattice updates per second the trace asks for, in millions."""
    return rate * float(np.mean([_cells(j["params"]) * j["steps"] for j in trace])) / 1e6


def served(trace, mode="server", pool_bytes=64 << 30, chunk_steps=100, graph_steps=20, policy=None, max_cells=None,
           log=None):
    """Run a job trace (list of dicts with arrival, params, nuclei, steps)."""
    import torch

    n = len(trace)
    order = sorted(range(n), key=lambda k: trace[k]["arrival"])
    latency = np.zeros(n)
    work = sum(_cells(j["params"]) * j["steps"] for j in trace)
    if mode == "server":
        srv = foamlbm.Server(pool_bytes=pool_bytes, chunk_steps=chunk_steps, graph_steps=graph_steps, policy=policy,
                             max_cells=max_cells)
        ids = {}
        nxt = 0
        pending = set()
        t0 = time.perf_counter()
        while nxt < n or pending:
            now = time.perf_counter() - t0
            while nxt < n and trace[order[nxt]]["arrival"] <= now:
                k = order[nxt]
                j = trace[k]
                ids[k] = srv.submit(j["steps"], j["nuclei"], **j["params"])
                pending.add(k)
                nxt += 1
            if not pending:
                time.sleep(max(0.0, trace[order[nxt]]["arrival"] - (time.perf_counter() - t0)))
                continue
            srv.pump()
            now = time.perf_counter() - t0
            for k in list(pending):
                st, _ = srv.state(ids[k])
                if st in (foamlbm.FLB_JOB_DONE, foamlbm.FLB_JOB_FAILED):
                    if st == foamlbm.FLB_JOB_FAILED:
                        raise RuntimeError(f"job {k} failed")
                    latency[k] = now - trace[k]["arrival"]
                    pending.discard(k)
                    srv.release(ids[k])
            if log and nxt % 32 == 0:
                log(f"served t={now:.1f}s submitted={nxt} pending={len(pending)}")
        makespan = time.perf_counter() - t0
        srv.close()
    else:
        t0 = time.perf_counter()
        for k in order:
            j = trace[k]
            wait = j["arrival"] - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(wait)
            s = foamlbm.Sim(**j["params"])
            s.set_nuclei(j["nuclei"])
            s.step(j["steps"])
            _ = s.density()  # the result, as the server hands it back
            latency[k] = time.perf_counter() - t0 - j["arrival"]
            s.close()
            torch.cuda.empty_cache()
        makespan = time.perf_counter() - t0
    return dict(mode=mode, jobs=n, makespan_s=makespan, MLUPS=work / makespan / 1e6,
                p50_s=float(np.percentile(latency, 50)), p99_s=float(np.percentile(latency, 99)),
                mean_s=float(latency.mean()))


def main(argv=None):
    """Command line: one batched-ensemble or served-stream measurement, one
    JSON line (used for the profiles of these workloads)."""
    import argparse
    import json

    from . import inputs

    ap = argparse.ArgumentParser(prog="python -m paper_1708_01613_amd.serve")
    sub = ap.add_subparsers(dest="cmd", required=True)
    e = sub.add_parser("ensemble")
    e.add_argument("--steps", type=int, default=1000)
    e.add_argument("--mode", choices=("batched", "persistent", "sequential"), default="batched")
    s = sub.add_parser("served")
    s.add_argument("--jobs", type=int, default=48)
    s.add_argument("--steps", type=int, default=1000)
    s.add_argument("--d3-fraction", type=float, default=0.5)
    s.add_argument("--policy", choices=("fifo", "shortest", "sequential"), default="fifo")
    s.add_argument("--max-cells", type=int, default=None)
    a = ap.parse_args(argv)
    if a.cmd == "ensemble":
        members, _ = inputs.config_ensemble()
        r = ensemble(members, a.steps, mode=a.mode)
    else:
        trace = inputs.arrival_trace(n_requests=a.jobs, d3_fraction=a.d3_fraction)
        for j in trace:
            j["steps"] = a.steps
        if a.policy == "sequential":
            r = served(trace, mode="sequential")
        else:
            pol = foamlbm.FLB_SERVE_FIFO if a.policy == "fifo" else foamlbm.FLB_SERVE_SHORTEST
            r = served(trace, mode="server", policy=pol, max_cells=a.max_cells)
    print(json.dumps(r), flush=True)


if __name__ == "__main__":
    main()
