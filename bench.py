"""Benchmark: Wavelet Monte Carlo dynamics sweeps on one MI355X.

Workload: semi-dilute periodic solution, 256 chains x 128 beads (32,768 beads), FENE + WCA,
box L = 84 (c/c* ~ 1), wavelet levels lambda = 1 .. L/4 in octave bands plus plane waves,
A0 = 0.5, synthetic self-avoiding random-walk start, 200 equilibration sweeps.

A step is one sweep. Before the timed sweeps every run tunes its launches from its equilibrated
state (wmc_tune, which restores that state; `--tune 0` keeps the plan's launches) and reports the
choices in `tuning`. Prints one JSON line:
  value         bead-updates/s of the timed sweeps (beads displaced per Metropolis test,
                wavelet and plane wave, accepted or not, summed; inputs resident in HBM)
  tau_per_wall_s  physical time (units of tau) advanced per wall-clock second
  accepted_bead_updates_per_s  beads displaced by accepted moves per second
  roofline      the dominant kernel class, timed with HIP events on the library's stream, beside
                the bandwidth of a plain 1 GiB device copy measured in the same run
  cpu_baseline  the FP64 oracle on the host, on a bounded sample of sweeps of the same state
  mixed         the same system in mixed precision (FP32 LDS tiles: offsets, displacements,
                distances and energy terms; FP64 positions; FP64 recheck near the threshold),
                from the FP64 run's final state
  batched       mixed precision on many systems at once: 8 independent copies of the solution,
                and the 32,768 beads as 8 smaller solutions of the same chains and concentration;
                ratio_vs_fp64 compares with the single-system FP64 value
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0

# HBM bytes per launch (FP64 pass, planned launches) from rocprofv3 FETCH_SIZE / WRITE_SIZE passes,
# scaled by a plain copy of known size (profiles/traffic_sweep_semidilute32k.md; levels 3 and 4 share
# one cell-group kernel, whose average is given for both); valid only for the device source they
# were measured on, otherwise the bench reports null
TRAFFIC_SOURCE_SHA16 = "81d604046c9f7362"
TRAFFIC_BYTES_PER_LAUNCH = {"level0": 42.86e6, "level1": 17.40e6, "level2": 16.88e6, "level3": 6.02e6, "level4": 6.02e6, "plane_waves": 28.94e6, "grid": 9.59e6}


def measured_traffic(cls: str):
    import hashlib

    src = os.path.join(ROOT, "paper_1611_09160_amd", "csrc", "wmc_device.hip")
    with open(src, "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    return TRAFFIC_BYTES_PER_LAUNCH.get(cls) if sha == TRAFFIC_SOURCE_SHA16 else None


def algorithmic_bytes_per_sweep(cls: str, N: int, n_fine: int, pw_attempts_per_sweep: float) -> float:
    """Bytes one sweep's launches of a kernel class must move at minimum.

    level passes: every bead's position is read and written once per level, plus 16 B of its
      sorted neighbour-grid entries (index and cell start, read by the halo gather and the pair
      search): N (24 + 24 + 16) = 64 B per bead.
    grid: per build read positions, write the reference copy and the cell of every bead, count,
      scan, scatter and sort: N (24 + 24 + 4 + 4 + 8 + 8) + 12 n_fine (6 builds per sweep here,
      one per level and one before the plane waves; the caller passes the build count).
    plane waves: per test read positions, write and re-read trial positions, read the
      neighbour grid and write accepted positions: N (24 + 24 + 24 + 8 + 24).
    """
    if cls.startswith("level"):
        return N * (24 + 24 + 16)
    if cls == "grid":
        return N * (24 + 24 + 4 + 4 + 8 + 8) + 12.0 * n_fine
    if cls == "plane_waves":
        return N * (24 + 24 + 24 + 8 + 24) * pw_attempts_per_sweep
    return 0.0


def run_gpu(cfg, precision: str, equilibrate: int, warmup: int, steps: int, start=None, tune: int = 0):
    import numpy as np
    import torch

    from paper_1611_09160_amd import wmc

    g = wmc.WMC(dict(cfg["params"], precision=precision), cfg["sys_offset"], cfg["chain_offset"],
                cfg["pos"] if start is None else start)
    if start is None:
        g.sweep(equilibrate)
    # launch tuning from the equilibrated state (the tuner restores that state), outside the timing
    tuned = g.tune(tune) if tune > 0 else None
    g.sweep(warmup)
    torch.cuda.synchronize()
    o0 = g.observables()
    tau0 = g.tau().sum()
    g.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.sweep(steps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kt = g.kernel_times()
    o1 = g.observables()
    tau1 = g.tau().sum()
    beads = int(o1["bead_updates"].sum() - o0["bead_updates"].sum() + o1["pw_bead_updates"] - o0["pw_bead_updates"])
    acc_beads = int(o1["accepted_bead_updates"] - o0["accepted_bead_updates"])
    res = dict(
        seconds=dt, steps=steps, bead_updates=beads, bead_updates_per_s=beads / dt, ms_per_step=1000.0 * dt / steps,
        accepted_bead_updates_per_s=acc_beads / dt,
        tau_per_wall_s=(tau1 - tau0) / dt, sweeps_per_s=steps / dt,
        acceptance=[round(float(a) / max(1, b), 4) for a, b in
                    zip(o1["accepts"] - o0["accepts"], o1["attempts"] - o0["attempts"]) if b > 0],
        pw_attempts=int(o1["pw_attempts"] - o0["pw_attempts"]), overflows=int(o1["overflows"]),
        violations=int(o1["violations"]), wait_timeouts=int(o1["wait_timeouts"]), rechecks=int(o1["rechecks"] - o0["rechecks"]), kernel_ms=kt,
        tuning=None if tuned is None else {
            "levels": [(f"tile:{lv['pass']}/{lv['variant']}" + (f"/{lv['width']}" if lv["width"] else "")
                        if "tile" in lv["cells"] else "") + (" " if lv["cells"] == "tile+global" else "") +
                       (("global:" + ("groups" if lv["groups"] == "on" else "cells") + f"/{lv['variant']}")
                        if "global" in lv["cells"] else "") for lv in tuned["levels"]],
            "plane_wave_groups": tuned["plane_wave_groups"], "trial_sweeps": tuned["trial_sweeps"]},
    )
    return g, res


def run_batched(cfg, precision: str, equilibrate: int, warmup: int, steps: int, tune: int = 0) -> dict:
    """Many independent systems advanced together (one launch per level and colour serves all)."""
    g, r = run_gpu(cfg, precision, equilibrate, warmup, steps, tune=tune)
    nsys = len(cfg["sys_offset"]) - 1
    out = dict(value=round(r["bead_updates_per_s"], 1), unit="bead-updates/s", ms_per_step=round(r["ms_per_step"], 3),
               accepted_bead_updates_per_s=round(r["accepted_bead_updates_per_s"], 1), systems=nsys, beads=int(cfg["sys_offset"][-1]), precision=precision,
               tau_per_wall_s_per_system=round(r["tau_per_wall_s"] / nsys, 4),
               tau_per_wall_s_total=round(r["tau_per_wall_s"], 4), overflows=r["overflows"], tuning=r["tuning"],
               kernel_ms={k: [round(v[0], 3), v[1]] for k, v in r["kernel_ms"].items()})
    g.close()
    return out


def run_oracle(cfg, start, sweep0: int, budget_s: float):
    from oracle import oracle as O

    o = O.Oracle(cfg["params"], cfg["sys_offset"], cfg["chain_offset"], start)
    o.set_sweep(sweep0)
    t0 = time.perf_counter()
    n = 0
    while True:
        o.sweep(1)
        n += 1
        if time.perf_counter() - t0 > budget_s or n >= 50:
            break
    dt = time.perf_counter() - t0
    ob = o.observables()
    beads = int(ob["bead_updates"].sum() + ob["pw_bead_updates"])
    return dict(value=beads / dt, unit="bead-updates/s", cores=1, kind="oracle",
                sample=f"{n} sweeps of the equilibrated workload state, single-threaded FP64 C (gcc -O3)",
                seconds=round(dt, 2), tau_per_wall_s=float(o.tau().sum()) / dt)


def other_workloads(warmup: int, steps: int) -> dict:
    """Throughput of the paper's other two workload shapes (FP64): the 1024-bead dilute chain in
    L = 128 with plane waves, and the 64-bead ideal chain in an infinite system (pure wavelets, and
    with the infinite-system plane waves)."""
    from paper_1611_09160_amd import workloads as W

    out = {}
    cases = (("dilute_chain_1024", W.config(2), {}, 50),
             ("ideal_chain_64", W.config(1), {}, 200),
             ("ideal_chain_64_w+F", W.config(1), dict(plane_waves=1), 200))
    for name, cfg, over, equil in cases:
        cfg = dict(cfg, params=dict(cfg["params"], **over))
        g, r = run_gpu(cfg, "fp64", equil, warmup, steps)
        g.close()
        out[name] = dict(value=round(r["bead_updates_per_s"], 1), unit="bead-updates/s",
                         tau_per_wall_s=round(r["tau_per_wall_s"], 4), ms_per_step=round(r["ms_per_step"], 3),
                         beads=int(cfg["sys_offset"][-1]), workload=cfg["name"] + (" + plane waves" if over else ""))
    return out


def copy_bandwidth_gbs(mib: int = 1024, reps: int = 10) -> float:
    """HBM bandwidth of a plain device-to-device copy (bytes read + written per second), the
    measured counterpart of the vendor peak"""
    import torch

    a = torch.ones(mib * (1 << 20) // 8, dtype=torch.float64, device="cuda")
    b = torch.empty_like(a)
    b.copy_(a)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    torch.cuda.synchronize()
    return 2.0 * a.numel() * 8 * reps / (e0.elapsed_time(e1) / 1000.0) / 1e9


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=40)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--equilibrate", type=int, default=200)
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-batched", action="store_true")
    ap.add_argument("--no-others", action="store_true", help="skip the dilute and ideal-chain lines")
    ap.add_argument("--batch-equilibrate", type=int, default=100)
    ap.add_argument("--tune", type=int, default=6, metavar="K",
                    help="launch tuning before the timed sweeps, K trial sweeps per choice (0: the plan's launches)")
    ap.add_argument("--copy-check", type=int, default=0, metavar="MB",
                    help="only copy a buffer of MB megabytes 4 times (reference for HBM byte counters)")
    args = ap.parse_args()
    if args.copy_check:
        import torch

        a = torch.ones(args.copy_check * (1 << 20) // 8, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        for _ in range(4):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps(dict(copy_check_bytes=a.numel() * 8, copies=4)))
        return 0
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); multi-GPU sharding is not built.",
              file=sys.stderr)
        return 2
    import numpy as np

    from paper_1611_09160_amd import wmc

    # libwmc's code object is registered before torch initialises the device (in this order a
    # process run under rocprofv3 writes the profiler's results at exit)
    wmc.lib()
    import torch

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1611_09160_amd import workloads as W

    cfg = W.config(3)
    N = int(cfg["sys_offset"][-1])
    g64, r64 = run_gpu(cfg, "fp64", args.equilibrate, args.warmup, args.steps, tune=args.tune)
    start = g64.positions()
    sweep0 = args.equilibrate + args.warmup + args.steps
    gm, rmix = run_gpu(cfg, "mixed", 0, args.warmup, args.steps, start=start, tune=args.tune)
    # roofline of the dominant kernel class of the FP64 run (a level's LDS-tile cells run as one
    # launch per sweep; its global-list cells, if any, as one launch per colour)
    kt = r64["kernel_ms"]
    n_fine = 55 ** 3
    steps = r64["steps"]
    dom = max(kt, key=lambda k: kt[k][0])
    ms, launches = kt[dom]
    per_sweep = algorithmic_bytes_per_sweep(dom, N, n_fine, r64["pw_attempts"] / steps)
    if dom == "grid":
        per_sweep *= launches / steps
    alg = per_sweep * steps / launches
    avg_s = ms / 1000.0 / launches
    achieved = alg / avg_s / 1e9
    traffic = measured_traffic(dom)
    roof = dict(bound="hbm", kernel=dom, achieved=round(achieved, 3), peak=HBM_PEAK_GBS, unit="GB/s",
                frac=achieved / HBM_PEAK_GBS, traffic=traffic, traffic_unit="bytes per launch",
                measured_copy_gbs=round(copy_bandwidth_gbs(), 1),
                avg_launch_us=round(avg_s * 1e6, 2),
                launches=launches, algorithmic_bytes_per_launch=int(alg),
                share_of_step=round(ms / (r64["seconds"] * 1000.0), 3))
    # every context is closed explicitly before the process ends (none is left to a finaliser)
    g64.close()
    gm.close()
    batched = None
    if not args.no_batched:
        copies = run_batched(W.replicas(3, 8), "mixed", args.batch_equilibrate, args.warmup, args.steps, args.tune)
        split = run_batched(W.batch_semidilute(8, 32), "mixed", args.batch_equilibrate, args.warmup, args.steps,
                            args.tune)
        ref = r64["bead_updates_per_s"]
        copies["ratio_vs_fp64"] = round(copies["value"] / ref, 3)
        split["ratio_vs_fp64"] = round(split["value"] / ref, 3)
        copies["workload"] = "8 independent copies of the 32,768-bead solution (each its own start)"
        split["workload"] = "the 32,768 beads as 8 solutions of 32 x 128 beads, L = 42, same concentration"
        batched = dict(copies=copies, split_32k=split)
    others = None if args.no_others else other_workloads(args.warmup, args.steps)
    cpu = None
    if not args.no_cpu:
        cpu = run_oracle(cfg, start, sweep0, args.cpu_budget)
    line = dict(
        metric="bead-updates/s + physical time/wall-s at 32k beads; mixed vs FP64 same GPU",
        value=round(r64["bead_updates_per_s"], 1), unit="bead-updates/s", n_gpus=1, steps=args.steps,
        warmup=args.warmup, ms_per_step=round(r64["ms_per_step"], 3), higher_is_better=True, scaling="weak",
        vs_baseline=None, dtype="f64", data="synthetic",
        config=dict(workload="semi-dilute periodic solution 256 chains x 128 beads (32768), FENE k=30 R0=1.5 + WCA, "
                             "L=84 (c/c*~1), lambda 1..21 octave levels + plane waves, A0=0.5, plain FP64 GPU path",
                    n_beads=N, box_L=84.0, equilibration_sweeps=args.equilibrate),
        tau_per_wall_s=round(r64["tau_per_wall_s"], 4), sweeps_per_s=round(r64["sweeps_per_s"], 2),
        accepted_bead_updates_per_s=round(r64["accepted_bead_updates_per_s"], 1),
        acceptance_per_level=r64["acceptance"], roofline=roof, cpu_baseline=cpu,
        tuning=r64["tuning"],
        mixed=dict(value=round(rmix["bead_updates_per_s"], 1), ms_per_step=round(rmix["ms_per_step"], 3),
                   tuning=rmix["tuning"],
                   tau_per_wall_s=round(rmix["tau_per_wall_s"], 4), rechecks=rmix["rechecks"],
                   accepted_bead_updates_per_s=round(rmix["accepted_bead_updates_per_s"], 1),
                   ratio_vs_fp64=round(rmix["bead_updates_per_s"] / r64["bead_updates_per_s"], 3)),
        batched=batched, other_workloads=others,
        kernel_ms_fp64={k: [round(v[0], 3), v[1]] for k, v in kt.items()},
        kernel_ms_mixed={k: [round(v[0], 3), v[1]] for k, v in rmix["kernel_ms"].items()},
        checks=dict(overflows=r64["overflows"] + rmix["overflows"], violations=r64["violations"],
                    wait_timeouts=r64["wait_timeouts"] + rmix["wait_timeouts"]),
    )
    print(json.dumps(line))
    bad = {k: v for k, v in line["checks"].items() if v}
    if bad:
        print(f"bench.py: the run is invalid: {bad} (every count must be 0)", file=sys.stderr)
        return 3
    return 0


if __name__ == "__main__":
    rc = main() or 0
    sys.stdout.flush()
    sys.stderr.flush()
    # Every context is closed. Outside a profiler the process ends without exit-time destructors;
    # under rocprofv3 it takes the normal exit, in which the profiler writes its results (the
    # process can then fault inside exit() after they are written, once libwmc's code object is
    # loaded; a copy-only run exits cleanly).
    if not any(k.startswith("ROCPROF") for k in os.environ):
        os._exit(rc)
    if rc:
        sys.exit(rc)
