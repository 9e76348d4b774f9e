#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (the force microbenchmark configuration): a Plummer sphere of
N = 65,536 equal masses (seed 2002), softening 1e-4, Henon units.  One
timed step runs the whole block-step hot path five times, once for each
active-set size N_act in {1, 64, 1024, 8192, 65,536} (random subsets,
seed 2003): the times and steps are reset so that exactly that subset is
due (positions and derivatives carry on), then
schedule -> predict all N sources -> evaluate a, da, d2a, phi of the active
particles -> split-source reduction -> corrector + interpolation + new block
step.  The last block has every particle active, which synchronizes the
system; the step ends with the FP64 energy / angular momentum sums of the
synchronized state.

value = force interactions (N * N_act summed over the five blocks) per
second of wall time over the timed steps, inputs resident in HBM.

Also reported: the same for the all-FP64 path and the FP32-pair mode and
the speedups; the energy error of the three on the 1024-body Plummer run to
t = 1 (eta = 0.45); the
per-phase GPU time; the roofline of the dominant kernel (the evaluation
kernel at N_act = N, timed with HIP events on its stream); and the CPU
oracle timed on a bounded sample of the same step.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G interactions/s (acc+jerk+snap), mixed vs FP64 at equal ΔE/E; % VALU peak"
N_ACTS = (1, 64, 1024, 8192, 65536)
# algorithmic flops per pair (FMA = 2, rsqrt = 4; the count of the method's
# difference, distance, rsqrt, alpha/beta, A/J/S and accumulation terms)
FLOPS_PER_PAIR = 83
PAPER_FLOPS_PER_PAIR = 97      # the paper's convention (Table 2)
# MI355X: 256 CUs x 4 SIMD x 16 lanes x 2.4 GHz; FMA = 2 flops.  Packed FP32
# is switched off for every kernel of the library, so the attainable FP32 vector rate equals
# the FP64 vector rate.
PEAK_FP32_NONPACKED = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.6 TFLOP/s
PEAK_FP32_DATASHEET = 157.3                          # counts packed FP32
PEAK_FP64 = 78.6
# HBM bytes per launch of the dominant kernel (mixed evaluation, N_act = N =
# 65,536, LPI 1, 4 waves, split 16) from rocprofv3 FETCH_SIZE and WRITE_SIZE
# passes over `bench.py --profile-pass`, each scaled by what the counter
# reads for a 1 GiB device copy (FETCH x 2.0, WRITE x 1.0): 29.71 MB read +
# 83.89 MB written (profiles/force_mixed_plummer65536_counters.txt).  Must be
# re-measured (or set to None) whenever that kernel changes.
TRAFFIC = 113.6e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=65536)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for rocprofv3 counter passes: a plain copy of a known "
                         "size (counter calibration), then the mixed steps only")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


class Workload:
    """The N-body state and the five prepared active-set schedules."""

    def __init__(self, n, precision, autotune):
        import numpy as np
        import torch

        import ics
        from paper_1207_2367_amd import System
        self.n = n
        m, x, v = ics.plummer(n, 2002)
        self.sys = System(m, x, v, 1e-4, precision=precision)
        if autotune:
            self.sys.autotune(150.0)
        self.t0 = torch.zeros(n, dtype=torch.float64, device="cuda")
        self.dts = []
        self.sizes = [min(k, n) for k in N_ACTS]
        rng = np.random.default_rng(2003)
        for na in self.sizes:
            dt = np.full(n, 2.0 ** -4)
            dt[rng.choice(n, na, replace=False)] = 2.0 ** -10
            self.dts.append(torch.as_tensor(dt, device="cuda"))
        self.n_act_of = {id(d): na for d, na in zip(self.dts, self.sizes)}
        self.pairs_per_step = float(sum(n * na for na in self.sizes))

    def step(self):
        # only t and dt are reset before each block (two device copies): the
        # particles with the short step are then exactly the prepared subset;
        # positions and derivatives carry on from the previous blocks (the
        # sphere moves by ~1e-3 time units per step)
        s = self.sys
        for dt in self.dts:
            s.set_state(t=self.t0, dt=dt)
            na, tb = s.block_step(1.0 / 16)
            assert na == self.n_act_of[id(dt)]
        return s.energy()

    def run(self, steps, warmup, profile=False):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        if profile:
            self.sys.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        prof = self.sys.profile(False) if profile else None
        return t1 - t0, prof


def energy_error(precision):
    """Delta E / E of the 1024-body Plummer sphere integrated to t = 1."""
    import ics
    from paper_1207_2367_amd import NBodyError, System
    m, x, v = ics.plummer(1024, 1001)
    s = System(m, x, v, 1e-4, precision=precision)
    e0 = sum(s.energy()[:2])
    try:
        st = s.step(1.0)
    except NBodyError as e:
        return None, str(e)
    e1 = sum(s.energy()[:2])
    return (e1 - e0) / e0, st["block_steps"]


def cpu_baseline(n, seconds):
    """The oracle timed on this host's cores on a bounded sample of the same
    step: one block step (schedule, predict all N, evaluate the sampled
    active set, correct it) with a sampled active set sized for ~seconds."""
    import numpy as np

    import ics
    import oracle
    m, x, v = ics.plummer(n, 2002)
    a = ics.plummer_mean_acc(x)
    cores = int(os.environ.get("OMP_NUM_THREADS", 0)) or len(os.sched_getaffinity(0))

    def one(n_act):
        it = oracle.Integrator(m, x, v, 1e-4)
        dt = np.full(n, 2.0 ** -4)
        dt[np.random.default_rng(2003).choice(n, n_act, replace=False)] = 2.0 ** -10
        it.set_state(a=a, t=np.zeros(n), dt=dt)
        t0 = time.perf_counter()
        err, na, tb = it.block_step(1.0 / 16)
        return time.perf_counter() - t0, na

    dt_cal, _ = one(1024)
    rate = 1024 * n / max(dt_cal, 1e-6)
    n_act = int(min(n, max(64, seconds * rate / n)))
    # repeat the step until about `seconds` of work have been timed
    el, pairs, reps = 0.0, 0.0, 0
    while el < 0.8 * seconds or reps == 0:
        e, na = one(n_act)
        el += e
        pairs += float(na) * n
        reps += 1
    cpu_model = ""
    try:
        with open("/proc/cpuinfo") as f:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        pass
    return {"value": round(pairs / el / 1e9, 4), "unit": "G interactions/s", "cores": cores,
            "kind": "oracle", "cpu": cpu_model,
            "sample": f"{reps} block step(s) of the N={n} Plummer sphere, each with a random active "
                      f"set of {na} particles (predict all N, evaluate {na} x {n} pairs, correct): "
                      f"{el:.1f} s in total, FP64 C oracle, OpenMP over active particles"}


def summarize_profile(d):
    """Text summary of rocprofv3 CSV output in directory d: kernel-trace
    durations grouped by (kernel, grid size) and, when present, counter
    values per dispatch of the evaluation kernels and of the calibration
    copy.  Printed to stdout (the source of the files in profiles/)."""
    import csv
    import glob
    import statistics
    out = []
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        groups = {}
        for r in rows:
            name = r["Kernel_Name"]
            grid = int(r.get("Grid_Size_X", r.get("Grid_Size", 0)) or 0)
            key = (name, r.get("Grid_Size_X", ""), r.get("Grid_Size_Y", ""), r.get("Workgroup_Size_X", ""))
            dur = (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6
            groups.setdefault(key, []).append(dur)
        tot = sum(sum(v) for v in groups.values())
        out.append(f"# {os.path.basename(f)}: {len(rows)} dispatches, {tot:.3f} ms total")
        out.append("calls  total_ms   avg_ms  median_ms     min_ms     max_ms   share  grid_x x grid_y (wg)  kernel")
        for key, v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:25]:
            short = key[0].replace("(anonymous namespace)::", "").split("(")[0][:90]
            out.append(f"{len(v):5d} {sum(v):9.3f} {statistics.mean(v):9.5f} {statistics.median(v):9.5f} "
                       f"{min(v):9.5f} {max(v):9.5f} {100 * sum(v) / tot:6.2f}%  {key[1]} x {key[2]} "
                       f"({key[3]})  {short}")
        # the dominant kernel of the bench: the shape of the last mixed-mode
        # evaluation longer than 1 ms (the full active set of the last timed
        # step; later mixed launches are the small energy-error runs); its
        # dispatches in launch order (autotune repetitions, warm-up, steps)
        mixed = sorted((r for r in rows if "force_kernel<0," in r["Kernel_Name"]),
                       key=lambda r: int(r["Start_Timestamp"]))
        mixed_long = [r for r in mixed
                      if int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) > 1_000_000]
        if mixed_long:
            r = mixed_long[-1]
            shape = (r["Kernel_Name"], r["Grid_Size_X"], r["Grid_Size_Y"])
            seq = [r for r in mixed if (r["Kernel_Name"], r["Grid_Size_X"], r["Grid_Size_Y"]) == shape]
            seq.sort(key=lambda r: int(r["Start_Timestamp"]))
            durs = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e6 for r in seq]
            kname = shape[0].replace("(anonymous namespace)::", "").split("(")[0]
            out.append(f"# dominant kernel {kname} grid {shape[1]} x {shape[2]}: "
                       f"{len(durs)} dispatches in launch order (ms): "
                       + " ".join(f"{x:.4f}" for x in durs))
    for f in sorted(glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)):
        rows = sorted(csv.DictReader(open(f)), key=lambda r: -float(r["TotalDurationNs"]))
        out.append(f"\n# --stats ({os.path.basename(f)}), top 12 by total time: name, calls, "
                   "total ms, avg ms")
        for r in rows[:12]:
            short = r["Name"].replace("(anonymous namespace)::", "").split("(")[0][:60]
            out.append(f"{short:60s} {int(r['Calls']):7d} {float(r['TotalDurationNs']) / 1e6:10.3f} "
                       f"{float(r['AverageNs']) / 1e6:10.5f}")
    for f in sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)):
        rows = list(csv.DictReader(open(f)))
        per = {}
        for r in rows:
            name = r["Kernel_Name"]
            if not ("force_kernel" in name or "copy" in name.lower() or "reduce_split" in name):
                continue
            key = (int(r["Dispatch_Id"]),
                   name.replace("(anonymous namespace)::", "").split("(")[0][:70], r["Grid_Size"])
            per.setdefault(key, {})
            per[key][r["Counter_Name"]] = per[key].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
        # listed: the dispatches of the dominant kernel's shape (the last
        # mixed-mode evaluation longer than 1 ms) and the largest copy (the
        # 1 GiB calibration copy of the profile pass)
        dur = {}
        for r in rows:
            dur[int(r["Dispatch_Id"])] = (r["Kernel_Name"], int(r["Grid_Size"]),
                                          int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        copies = [k_ for k_ in per if "copy" in k_[1].lower()]
        mixed = [k_ for k_ in per if "force_kernel<0," in k_[1] and dur[k_[0]][2] > 1_000_000]
        listed = []
        if mixed:
            dom = max(mixed, key=lambda k_: k_[0])
            listed = [k_ for k_ in mixed if k_[1:] == dom[1:]]
        if copies:
            listed.append(max(copies, key=lambda k_: int(k_[2])))
        out.append(f"# {os.path.basename(f)}")
        for key in sorted(listed):
            vals = " ".join(f"{k}={v:.6g}" for k, v in sorted(per[key].items()))
            out.append(f"dispatch {key[0]:5d} grid {key[2]:>9} {dur[key[0]][2] / 1e6:8.3f} ms  "
                       f"{key[1]}  {vals}")
        # calibration: the 1 GiB copy against the bytes it moves; then the
        # dominant kernel (the last mixed-mode evaluation longer than 1 ms)
        # scaled by it
        if copies and mixed:
            cp = max(copies, key=lambda k_: int(k_[2]))
            dom = max(mixed, key=lambda k_: k_[0])
            for cname in ("FETCH_SIZE", "WRITE_SIZE"):
                if cname in per[cp] and cname in per[dom]:
                    fac = (1 << 30) / (per[cp][cname] * 1024.0)
                    byt = per[dom][cname] * 1024.0 * fac
                    out.append(f"# {cname}: 1 GiB copy (dispatch {cp[0]}) counts {per[cp][cname]:.6g} KiB "
                               f"-> factor {fac:.4f}; dominant kernel dispatch {dom[0]} ({dom[1]}, grid "
                               f"{dom[2]}, {dur[dom[0]][2] / 1e6:.3f} ms) {per[dom][cname]:.6g} KiB "
                               f"-> {byt / 1e6:.2f} MB per launch")
    print("\n".join(out))


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-profile":
        summarize_profile(sys.argv[2])
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path has "
              "no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1207_2367_amd import PREC_FP32PAIR, PREC_FP64, PREC_MIXED
    from paper_1207_2367_amd import nbody
    if not os.path.exists(nbody.lib_path()):
        import __graft_entry__
        __graft_entry__.build()

    if args.profile_pass:
        # calibration for the HBM counters: copy 1 GiB that is not cache
        # resident (a second buffer is written in between), then the steps
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        b = torch.empty_like(a).fill_(2.0)
        c = torch.empty_like(a).fill_(3.0)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b, c
        wl = Workload(args.n, PREC_MIXED, not args.no_autotune)
        wl.run(args.steps, args.warmup)
        torch.cuda.synchronize()
        log("profile pass done")
        return

    log(f"mixed: N={args.n}, warmup {args.warmup}, steps {args.steps}")
    wl = Workload(args.n, PREC_MIXED, not args.no_autotune)
    launches = {na: wl.sys.get_launch(na) for na in wl.sizes}
    el, prof = wl.run(args.steps, args.warmup, profile=True)
    value = wl.pairs_per_step * args.steps / el / 1e9
    na_log, pr_log, ms_log = wl.sys.force_log()
    log(f"mixed: {el / args.steps * 1e3:.3f} ms/step, {value:.2f} G interactions/s")

    # dominant kernel: the evaluation at N_act = N
    import numpy as np
    sel = na_log == args.n
    avg_ms = float(ms_log[sel].mean())
    pairs = float(args.n) * args.n
    achieved = FLOPS_PER_PAIR * pairs / (avg_ms * 1e-3) / 1e12
    per_nact = {}
    for na in wl.sizes:
        s = na_log == na
        t = float(ms_log[s].mean())
        per_nact[str(na)] = {"kernel_ms": round(t, 5),
                             "G_interactions_per_s": round(na * args.n / (t * 1e-3) / 1e9, 3),
                             "launch": {"lanes_per_i": launches[na][0], "waves": launches[na][1],
                                        "split": launches[na][2]}}
    phases = {k: round(v[0] / args.steps, 4) for k, v in prof.items() if k != "pairs"}

    ks = args.fp64_steps or max(2, args.steps // 2)
    other = {}
    for name, prec in (("fp64", PREC_FP64), ("fp32pair", PREC_FP32PAIR)):
        log(f"{name} path")
        wd = Workload(args.n, prec, not args.no_autotune)
        eld, _ = wd.run(ks, 1, profile=True)
        na_d, _, ms_d = wd.sys.force_log()
        other[name] = (wd.pairs_per_step * ks / eld / 1e9, float(ms_d[na_d == args.n].mean()))
        del wd
    value_f64, avg_ms_d = other["fp64"]
    value_p32, avg_ms_p = other["fp32pair"]

    log("energy error, 1024-body Plummer to t = 1")
    de_mixed, steps_m = energy_error(PREC_MIXED)
    de_f64, steps_d = energy_error(PREC_FP64)
    de_p32, steps_p = energy_error(PREC_FP32PAIR)

    cpu = None
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        cpu = cpu_baseline(args.n, args.cpu_seconds)

    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"Plummer N={args.n} (seed 2002), eps=1e-4, Henon units; one step = "
                        "block steps with N_act in {1, 64, 1024, 8192, 65536} (schedule, "
                        "predict, evaluate, reduce, correct, new steps) + FP64 energy of the "
                        "synchronized state",
            "n": args.n, "n_act": list(wl.sizes), "precision": "mixed",
        },
        "roofline": {
            "bound": "alu", "achieved": round(achieved, 3), "peak": round(PEAK_FP32_NONPACKED, 2),
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32_NONPACKED, 4),
            "traffic": TRAFFIC,
            "traffic_unit": "bytes per launch (FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "kernel": "evaluation (force) kernel, N_act = N",
            "kernel_avg_ms": round(avg_ms, 5), "flops_per_pair": FLOPS_PER_PAIR,
            "peak_basis": "FP32 vector without packed math: 256 CU x 64 lanes x 2 flop x 2.4 GHz "
                          "(packed FP32 is disabled in the library)",
            "frac_vs_fp32_datasheet_157.3": round(achieved / PEAK_FP32_DATASHEET, 4),
        },
        "fp64_path": {
            "value": round(value_f64, 3), "unit": "G interactions/s",
            "kernel_ms_at_N": round(avg_ms_d, 5),
            "kernel_tflops": round(FLOPS_PER_PAIR * pairs / (avg_ms_d * 1e-3) / 1e12, 3),
            "frac_fp64_peak": round(FLOPS_PER_PAIR * pairs / (avg_ms_d * 1e-3) / 1e12 / PEAK_FP64, 4),
        },
        "fp32pair_path": {
            "value": round(value_p32, 3), "unit": "G interactions/s",
            "kernel_ms_at_N": round(avg_ms_p, 5),
            "kernel_tflops": round(FLOPS_PER_PAIR * pairs / (avg_ms_p * 1e-3) / 1e12, 3),
        },
        "speedup_mixed_vs_fp64": round(value / value_f64, 3),
        "kernel_speedup_mixed_vs_fp64": round(avg_ms_d / avg_ms, 3),
        "kernel_speedup_fp32pair_vs_fp64": round(avg_ms_d / avg_ms_p, 3),
        "dE_over_E_plummer1024_t1": {"mixed": de_mixed, "fp64": de_f64, "fp32pair": de_p32,
                                     "block_steps": [steps_m, steps_d, steps_p]},
        "paper_equiv_gflops": round(value * PAPER_FLOPS_PER_PAIR, 1),
        "per_n_act": per_nact,
        "phase_ms_per_step": phases,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
