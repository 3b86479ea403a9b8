#!/usr/bin/env python3
"""Benchmark of the fused Shan-Chen foam step on one MI355X.

Workload: D3Q19 256^3, FP32 populations, tau 1, G -5.5, 2000 seeded nuclei
(radii U[3, 8]), film barrier and rupture test on (maps rebuilt every 10
steps), inputs resident in HBM.  A "step" is one time step of the whole hot
path: fused step kernel (pull, moments, psi, force with barrier, velocity
shift, BGK, store, FP64 partials, rupture test) plus its share of the map
refreshes.  The lattice is first advanced past the step at which the rupture
test starts (untimed), so every timed step runs the whole path.  Prints one
JSON line.

  python bench.py [--steps K] [--warmup W] [--gpus 1]
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E peak
# algorithmic bytes per lattice update: read Q*s + write Q*s + 1 flag byte
# (the kernel reads a 4-byte barrier mask instead of the flag byte: 156 B)
DESIGN_BYTES = 156
BYTES_PER_UPDATE = {("d3q19", "f32"): 153, ("d3q19", "f16s"): 77, ("d3q19", "f64"): 305,
                    ("d2q9", "f32"): 73, ("d2q9", "f16s"): 37, ("d2q9", "f64"): 145,
                    # two lattices, two passes: 2 x 19 x 4 B read twice and written once,
                    # 4 arrays x 4 B written, 2 x 4 B read, a 4 B mask
                    ("d3q19_two_lattice", "f32"): 2 * 76 * 2 + 2 * 76 + 16 + 8 + 4}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(steps=10):
    """The FP64 oracle on the host cores over a bounded sample of the same
    workload: the same 256^3 lattice and nuclei, film on, the first `steps`
    steps (including the map refresh at step 0) on all cores; then one more
    step (not a refresh step) on one thread.  Returns the report and the
    oracle, whose state after `steps` steps the per-field errors use."""
    from oracle import OracleSim
    from paper_1708_01613_amd import inputs

    params, nuc, _ = inputs.config_foam3d("f32")
    n = params["nx"]
    kw = {k: params[k] for k in ("lattice", "nx", "ny", "nz", "tau", "G", "rho0", "rho_liquid", "rho_gas",
                                 "noise_amp", "seed", "film_on")}
    s = OracleSim(**kw, k_own=10, zone_width=6, rupture_warmup=200)
    s.set_nuclei(nuc)
    t0 = time.perf_counter()
    s.step(steps)
    dt = time.perf_counter() - t0
    threads = s.threads()
    rho, u = s.density(), s.velocity()
    rep = {"value": round(n ** 3 * steps / dt / 1e6, 3), "unit": "MLUPS", "cores": threads, "kind": "oracle",
           "sample": f"D3Q19 {n}^3 FP64 oracle, the same {len(nuc)} nuclei, film on, first {steps} steps "
                     f"incl. one map refresh, {dt:.1f} s on {threads} OpenMP threads"}
    if steps % 10:
        return rep, (rho, u)
    # one thread, one step that is not a refresh step (step steps + 1)
    s.step(1)
    s.set_threads(1)
    t0 = time.perf_counter()
    s.step(1)
    d1 = time.perf_counter() - t0
    s.set_threads(threads)
    rep["single_thread"] = {"value": round(n ** 3 / d1 / 1e6, 3), "unit": "MLUPS", "cores": 1,
                            "sample": f"one step without a map refresh (step {steps + 1}), {d1:.1f} s"}
    del s
    return rep, (rho, u)


def spinodals(G):
    """Gas and liquid spinodal densities of p0 = rho/3 + (G/6) psi^2 with
    psi = 1 - exp(-rho): dp0/drho = 0 at exp(-rho) = (1 -+ sqrt(1 + 4/G)) / 2."""
    import math

    y = math.sqrt(1.0 + 4.0 / G)
    return -math.log((1.0 + y) / 2.0), -math.log((1.0 - y) / 2.0)


def field_errors(sim_rho, sim_u, o_rho, o_u, G):
    """Density (max relative) and velocity (max absolute over the largest
    oracle speed) errors against the FP64 oracle, per phase: gas below the
    gas spinodal, liquid above the liquid spinodal, interface between."""
    import numpy as np

    rg, rl = spinodals(G)
    umax = float(np.abs(o_u).max())
    phases = {"gas": o_rho < rg, "interface": (o_rho >= rg) & (o_rho <= rl), "liquid": o_rho > rl}
    out = {}
    for name, sel in phases.items():
        if not sel.any():
            continue
        out[name] = {"cells": int(sel.sum()),
                     "density_max_rel": float(np.max(np.abs(sim_rho[sel] - o_rho[sel]) / o_rho[sel])),
                     "velocity_max_abs_over_umax": float(np.max(np.abs(sim_u[:, sel] - o_u[:, sel])) / umax)}
    return out


# rocprofv3 FETCH_SIZE / WRITE_SIZE summary of the step kernel on this
# workload; its traffic is reported only while the kernel sources are the
# ones it was measured on
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_step_d3q19_256_f32_traffic.md")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1708_01613_amd", "csrc", f) for f in ("step.hpp", "lattice.hpp")]


def kernel_source_hash():
    import hashlib

    h = hashlib.sha256()
    for p in KERNEL_SOURCES:
        with open(p, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


class _Skipped(Exception):
    pass


def measured_traffic():
    try:
        text = open(TRAFFIC_PROFILE).read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if ":" in line and line.strip().startswith("- "):
            k, v = line.strip()[2:].split(":", 1)
            vals[k.strip()] = v.strip().strip("`")
    if vals.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def _rounded(r):
    return {k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}


def batched_and_served(args):
    """The batched-ensemble and served-stream workloads: 64 uneven D2Q9
    lattices (one batch vs one lattice at a time), and Poisson streams of
    mixed D2Q9/D3Q19 jobs in two mixes (the job server with FIFO and with
    shortest-remaining-work scheduling vs first-come first-served one job at
    a time)."""
    import torch

    from paper_1708_01613_amd import foamlbm, inputs, serve

    out = {}
    members, _ = inputs.config_ensemble()
    cells = sum(p["nx"] * p["ny"] for p, _ in members)
    seq_steps = min(args.ensemble_steps, 2000)
    # the persistent launch (one cooperative launch per stretch between
    # refreshes, grid barriers between the phases of a step) against the
    # graph replay of per-step launches
    for mode, steps in (("batched", args.ensemble_steps), ("persistent", seq_steps), ("sequential", seq_steps)):
        r = serve.ensemble(members, steps, mode=mode)
        log(f"ensemble {mode}: {r['MLUPS']:.0f} MLUPS over {steps} steps")
        out[f"ensemble_{mode}"] = dict(_rounded(r), steps=steps)
        torch.cuda.empty_cache()
    out["ensemble"] = {"lattices": len(members), "cells": cells, "steps": args.ensemble_steps,
                       "speedup": round(out["ensemble_batched"]["MLUPS"] / out["ensemble_sequential"]["MLUPS"], 2),
                       "graph_over_persistent": round(out["ensemble_batched"]["MLUPS"] /
                                                      out["ensemble_persistent"]["MLUPS"], 2)}
    rate = 20.0
    for tag, d3 in (("mix50", 0.5), ("mix10", 0.1)):
        trace = inputs.arrival_trace(n_requests=args.serve_jobs, rate=rate, d3_fraction=d3)
        for j in trace:
            j["steps"] = args.serve_steps
        res = {"jobs": len(trace), "d3_fraction": d3, "rate_per_s": rate, "steps_per_job": args.serve_steps,
               "offered_MLUPS": round(serve.offered_mlups(trace, rate), 1)}
        for name, mode, policy in (("fifo", "server", foamlbm.FLB_SERVE_FIFO),
                                   ("shortest", "server", foamlbm.FLB_SERVE_SHORTEST),
                                   ("sequential", "sequential", None)):
            r = serve.served(trace, mode=mode, policy=policy)
            log(f"served {tag} {name}: {r['MLUPS']:.0f} MLUPS p50 {r['p50_s']:.3f}s p99 {r['p99_s']:.3f}s")
            res[name] = _rounded(r)
            torch.cuda.empty_cache()
        out[f"served_{tag}"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--n", type=int, default=256, help="cube side (the workload is 256)")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline and the per-field errors")
    ap.add_argument("--tile", type=int, default=-1, help="fixed tile variant (default: autotune)")
    ap.add_argument("--lz", type=int, default=0)
    ap.add_argument("--xcd", type=int, default=-1)
    ap.add_argument("--no-forms", action="store_true", help="skip the batched, served and 2-D foam measurements")
    ap.add_argument("--ensemble-steps", type=int, default=10000)
    ap.add_argument("--serve-jobs", type=int, default=48)
    ap.add_argument("--serve-steps", type=int, default=5000)
    ap.add_argument("--foam2d-steps", type=int, default=20000)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py measures one GPU; --gpus {args.gpus} is not supported: the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1708_01613_amd import foamlbm, inputs

    torch.cuda.set_device(0)
    params, nuc, _ = inputs.config_foam3d("f32", n=args.n)
    params.update(k_own=10, zone_width=6, rupture_warmup=200)
    log(f"creating {params['nx']}^3 D3Q19 f32 lattice, {len(nuc)} nuclei")
    sim = foamlbm.Sim(**params)
    sim.set_nuclei(nuc)
    if args.tile >= 0:
        sim.set_tuning(args.tile, args.lz, args.xcd)
    else:
        tuned = sim.autotune(reps=3)
        log(f"autotuned step kernel {tuned:.4f} ms")
    N = params["nx"] * params["ny"] * params["nz"]
    tun = sim.tuning()
    log(f"tuning {tun}")

    # untimed set-up: past the step at which the rupture test starts (its
    # first evaluation unites a burst of pairs), so that every warmup and
    # timed step runs the rupture test and the mask pruning as well
    setup = params["rupture_warmup"] + 1
    sim.step(setup)
    sim.step(args.warmup)
    torch.cuda.synchronize()
    r0 = sim.stats()["n_ruptures"]
    log(f"set-up {setup} + warmup {args.warmup} steps done")
    t0 = time.perf_counter()
    sim.step(args.steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    wall = t1 - t0
    mlups = N * args.steps / wall / 1e6
    st = sim.stats()
    log(f"timed {args.steps} steps: {wall * 1e3 / args.steps:.3f} ms/step, {mlups:.0f} MLUPS, "
        f"{st['n_ruptures'] - r0} ruptures in the window")

    # the same number of steps again with every phase bracketed by HIP events
    # on the library's stream: the share of each kernel group in a step
    ph_total, ph = sim.time_phases(args.steps)
    shares = {k: {"ms_per_step": round(v / args.steps, 4), "share": round(v / ph_total, 4)} for k, v in ph.items()}
    log("phases " + ", ".join(f"{k} {v['ms_per_step']:.4f} ms" for k, v in shares.items()))

    # dominant kernel alone: every step-kernel launch bracketed by HIP events
    # on the library's stream (maps frozen, so no refresh runs in between)
    nk = max(20, min(200, args.steps))
    _, ksum = sim.time_steps(nk, refresh=False, kernel=True)
    kms = ksum / nk
    bpu = BYTES_PER_UPDATE[("d3q19", "f32")]
    achieved = bpu * N / (kms * 1e-3) / 1e9
    log(f"step kernel {kms:.4f} ms, {achieved:.0f} GB/s algorithmic")
    del sim
    torch.cuda.empty_cache()
    copy = foamlbm.copy_bandwidth(1 << 30, reps=10)
    log(f"device copy ceiling (16-byte accesses) {copy:.0f} GB/s")
    # FP16-shifted storage variant of the same workload (kernel time only)
    variants = {}
    try:
        p16 = dict(params, storage="f16s")
        s16 = foamlbm.Sim(**p16)
        s16.set_nuclei(nuc)
        if args.tile < 0:
            s16.autotune(reps=3)
        s16.step(10)
        ms16 = s16.time_steps(nk, refresh=False, kernel=True)[1] / nk
        t16 = s16.tuning()
        variants["d3q19_f16s_kernel"] = {"ms": round(ms16, 4), "MLUPS": round(N / (ms16 * 1e-3) / 1e6, 1),
                                         "GBs_algorithmic": round(77 * N / (ms16 * 1e-3) / 1e9, 1),
                                         "kernel": (f"k_step<D3Q19K,SF16S,{t16['tile_x']},{t16['tile_m']}>"
                                                    if t16["tile_x"] else "k_psi+k_collide<D3Q19K,SF16S>")}
        del s16
        torch.cuda.empty_cache()
    except Exception as exc:  # a variant failing must not hide the main line
        variants["d3q19_f16s_kernel"] = {"error": str(exc)}
    # the two-lattice model (melt and gas lattices, Sec. 2.1.5) on the same
    # lattice and nuclei: the whole path and its step kernels (k_psi_tl +
    # k_collide_tl: both lattices read twice and written once, the four
    # density / pseudopotential arrays written and two of them read, the mask)
    try:
        ptl = dict(params, model=1, G_mg=0.3, tau_g=1.0, rho_g_bubble=0.4, rho_g_liquid=0.05)
        stl = foamlbm.Sim(**ptl)
        stl.set_nuclei(nuc)
        stl.step(setup)
        torch.cuda.synchronize()
        ntl = max(20, min(100, args.steps))
        t0 = time.perf_counter()
        stl.step(ntl)
        torch.cuda.synchronize()
        wtl = time.perf_counter() - t0
        mstl = stl.time_steps(nk, refresh=False, kernel=True)[1] / nk
        btl = BYTES_PER_UPDATE[("d3q19_two_lattice", "f32")]
        variants["d3q19_two_lattice"] = {
            "steps": ntl, "MLUPS": round(N * ntl / wtl / 1e6, 1), "ms_per_step": round(wtl * 1e3 / ntl, 4),
            "kernel_ms": round(mstl, 4), "bytes_per_update": btl,
            "GBs_algorithmic": round(btl * N / (mstl * 1e-3) / 1e9, 1),
            "frac": round(btl * N / (mstl * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "kernel": "k_psi_tl+k_collide_tl<D3Q19K,SF32>", "n_bubbles": stl.stats()["n_bubbles"]}
        log(f"two-lattice d3q19 256^3: {variants['d3q19_two_lattice']['MLUPS']:.0f} MLUPS whole path, "
            f"step kernels {mstl:.4f} ms")
        del stl
        torch.cuda.empty_cache()
    except Exception as exc:
        variants["d3q19_two_lattice"] = {"error": str(exc)}
    # the validation case of Sec. 5 in lattice units: two growing bubbles in a
    # container open for the liquid (two lattices, gas release at the nuclei,
    # open planes across y), stepped until the rupture criterion fires
    try:
        if args.no_forms:
            raise _Skipped()
        nx2, ny2, R2, gap2 = 128, 96, 10.0, 16.0
        c2 = (nx2 - 1) / 2
        pc = dict(lattice=0, storage="f32", nx=nx2, ny=ny2, nz=1, tau=1.0, G=-5.0, rho0=1.0, rho_liquid=2.0,
                  rho_gas=0.15, noise_amp=0.0, model=1, G_mg=0.3, tau_g=1.0, rho_g_bubble=0.4, rho_g_liquid=0.05,
                  growth_on=1, gas_A=1.0, gas_dndt=0.1, open_z=1, rho_res=2.0, film_on=1, rupture_warmup=20,
                  k_own=5, zone_width=6)
        sc = foamlbm.Sim(**pc)
        sc.set_nuclei([[c2 - R2 - gap2 / 2 - 0.5, ny2 / 2, 0, R2], [c2 + R2 + gap2 / 2 + 0.5, ny2 / 2, 0, R2]])
        m0 = sc.stats()["mass"]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        done, first = 0, None
        while done < 1500 and first is None:
            sc.step(50)
            done += 50
            ev = sc.rupture_events()
            if len(ev):
                first = int(min(e[0] for e in ev))
        torch.cuda.synchronize()
        wc = time.perf_counter() - t0
        kc = sc.time_steps(100, refresh=False, kernel=True)[1] / 100
        n2c = nx2 * ny2
        variants["d2q9_container_growth"] = {
            "cells": n2c, "steps": done, "first_rupture_step": first, "MLUPS": round(n2c * done / wc / 1e6, 1),
            "kernel_ms": round(kc, 4), "mass_change": round(sc.stats()["mass"] - m0, 3),
            "kernel": "k_psi_tl+k_collide_tl<D2Q9K,SF32>, open planes, gas release"}
        log(f"d2q9 container growth: first rupture at step {first}, {variants['d2q9_container_growth']['MLUPS']:.0f} MLUPS")
        del sc
    except _Skipped:
        pass
    except Exception as exc:
        variants["d2q9_container_growth"] = {"error": str(exc)}
    # the 2-D foam-growth workload: D2Q9 1024^2 FP32, film on, bubble labels,
    # the size histogram and the overlap with the previous labels read back
    # every 500 steps over its full horizon (whole path, then the step kernel
    # alone), always with its own autotuned tile
    try:
        if args.no_forms:
            raise _Skipped()
        p2, nuc2, _ = inputs.config_foam2d()
        n2 = p2["nx"] * p2["ny"]
        s2 = foamlbm.Sim(**p2)
        s2.set_nuclei(nuc2)
        s2.autotune(reps=3)
        torch.cuda.synchronize()
        steps2, every = args.foam2d_steps, 500
        prev, _ = s2.labels()
        merges = 0
        t0 = time.perf_counter()
        for _ in range(steps2 // every):
            s2.step(every)
            lab2, nb2 = s2.labels()
            s2.histogram(64, 1.0)
            # coalescence tracking: current bubbles overlapping two or more
            # bubbles of the previous snapshot
            pairs, _ = s2.match_labels(prev)
            if len(pairs):
                merges += int((np.bincount(pairs[:, 1]) >= 2).sum())
            prev = lab2
        torch.cuda.synchronize()
        w2 = time.perf_counter() - t0
        ms2 = s2.time_steps(nk, refresh=False, kernel=True)[1] / nk
        t2 = s2.tuning()
        st2 = s2.stats()
        variants["d2q9_1024_foam"] = {
            "steps": steps2, "labels_every": every, "MLUPS": round(n2 * steps2 / w2 / 1e6, 1),
            "n_bubbles": nb2, "coalescences": merges, "n_ruptures": st2["n_ruptures"], "kernel_ms": round(ms2, 4),
            "kernel_GBs_algorithmic": round(BYTES_PER_UPDATE[("d2q9", "f32")] * n2 / (ms2 * 1e-3) / 1e9, 1),
            "kernel": (f"k_step<D2Q9K,SF32,{t2['tile_x']},{t2['tile_m']}>" if t2["tile_x"]
                       else "k_psi+k_collide<D2Q9K,SF32>"),
            # variant index: 0-2 marches 64/128/256 wide, 3-4 flat tiles of 8/16 rows
            "tile": t2["tile"]}
        log(f"d2q9 1024^2 foam: {variants['d2q9_1024_foam']['MLUPS']:.0f} MLUPS over {steps2} steps, "
            f"step kernel {ms2:.4f} ms")
        del s2
        torch.cuda.empty_cache()
    except _Skipped:
        pass
    except Exception as exc:
        variants["d2q9_1024_foam"] = {"error": str(exc)}

    forms = None if args.no_forms else batched_and_served(args)
    cpu, errors = None, None
    if not args.no_cpu:
        cpu, (o_rho, o_u) = cpu_baseline()
        log(f"cpu oracle {cpu['value']} MLUPS on {cpu['cores']} threads; "
            f"one thread {cpu.get('single_thread', {}).get('value')} MLUPS")
        # per-field errors of the two storage forms against the oracle after
        # the same 10 steps from the same initial state
        errors = {"steps": 10, "phases": "gas: rho below the gas spinodal; liquid: above the liquid spinodal; "
                                         "interface: between (spinodals of p0 at G)"}
        for stor in ("f32", "f16s"):
            g = foamlbm.Sim(**dict(params, storage=stor))
            g.set_nuclei(nuc)
            g.step(10)
            errors[stor] = field_errors(g.density(), g.velocity(), o_rho, o_u, params["G"])
            del g
            torch.cuda.empty_cache()
        log("per-field errors " + json.dumps(errors))
    line = {
        "metric": "MLUPS & %HBM peak (D3Q19 256^3 FP32); batched MLUPS + p50/p99 latency",
        "value": round(mlups, 1),
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(wall * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"D3Q19 {params['nx']}^3 FP32 foam, {len(nuc)} uniform nuclei r~U[3,8], G=-5.5, "
                               "tau=1, film barrier + rupture on, maps every 10 steps from the current density",
                   "cells": N, "tuning": tun, "setup_steps": setup,
                   "timed_steps_from": setup + args.warmup},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(),
                     "kernel": (f"k_step<D3Q19K,SF32,{tun['tile_x']},{tun['tile_m']}>" if tun["tile_x"]
                                else "k_psi+k_collide<D3Q19K,SF32>"), "kernel_ms": round(kms, 4),
                     "bytes_per_update": bpu, "design_bytes_per_update": DESIGN_BYTES,
                     "copy_ceiling_GBs": round(copy, 1), "frac_of_copy": round(achieved / copy, 4)},
        "cpu_baseline": cpu,
        "phases": shares,
        "field_errors": errors,
        "variants": variants,
        "batched_and_served": forms,
        "checks": {"mass": st["mass"], "n_bubbles": st["n_bubbles"], "n_ruptures": st["n_ruptures"],
                   "ruptures_in_window": st["n_ruptures"] - r0, "step": st["step"]},
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
