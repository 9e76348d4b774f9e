#!/usr/bin/env python3
"""Benchmark of the hot path on one MI355X.

Workload (the largest single-GPU configuration): a Plummer sphere of
N = 8,388,608 equal masses (seed 5005), softening 1e-4, Henon units, with
N_act = 65,536 active particles (seed 5006).  One timed step is one block
time step of the whole system in which exactly those particles are due:
schedule (sweep of all N) -> predict all N sources to the block time ->
evaluate a, da, d2a of the active particles against all N sources (mixed
precision) -> split-source reduction -> corrector + interpolation of the
higher derivatives + new block steps.  Before each step the times and
steps of all particles are reset (two device copies, inside the timed
region) so that the same particles are due again; positions and
derivatives carry on.

Preparation (not timed): the state starts from the generator (positions,
velocities, the smooth Plummer acceleration as every source's
acceleration); one evaluation of the active set against all sources then
gives those particles consistent a, da, d2a (the start-up passes of a full
initialization are two N^2 FP64 evaluations, minutes at this size).  That
first evaluation is also checked against the oracle on sampled particles.

value = N * N_act * steps / wall time of the timed steps (inputs resident in
HBM), in G interactions/s.

Also reported: the same step in the FP64 and FP32-pair modes and the
speedups; the FP64 energy / angular-momentum pass (once, on the synchronized
prepared state, N^2/2 pairs); the energy error of the three modes on the
65,536-body sphere integrated to t = 1/8 ("at equal Delta E / E"); the
65,536-body force-microbenchmark sizes N_act = 1 ... 65,536 (kernel times
and per-particle errors against the oracle); the roofline of the dominant
kernel (the mixed evaluation of the timed steps, HIP events on its stream);
and the CPU oracle timed on a bounded sample of the same block step, on all
host cores and on one.
"""
from __future__ import annotations

import argparse
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "G interactions/s (acc+jerk+snap), mixed vs FP64 at equal ΔE/E; % VALU peak"
EPS = 1e-4
N_BIG, NACT_BIG, SEED_BIG, SEED_SUB = 1 << 23, 65536, 5005, 5006
N_MICRO, SEED_MICRO, SEED_MICRO_SUB = 65536, 2002, 2003
MICRO_NACTS = (1, 64, 1024, 8192, 65536)
MICRO_WARM, MICRO_REPS = 3, 15   # untimed and timed calls per size (median reported)
DT_ACTIVE, DT_REST = 2.0 ** -10, 1.0 / 16
# algorithmic flops per pair (FMA = 2, rsqrt = 4; the count of the method's
# difference, distance, rsqrt, alpha/beta, A/J/S and accumulation terms)
FLOPS_PER_PAIR = 83
PAPER_FLOPS_PER_PAIR = 97      # the paper's convention (Table 2)
# MI355X published vector peaks (TFLOP/s).  Packed FP32 (which the FP32
# figure counts) is switched off for every kernel of the library, so an FP32
# kernel can reach at most half of it: 256 CU x 64 lanes x 2 x 2.4 GHz.
PEAK_FP32 = 157.3
PEAK_FP32_NONPACKED = 256 * 64 * 2 * 2.4e9 / 1e12   # 78.6
PEAK_FP64 = 78.6
# HBM bytes of the dominant kernel per launch come from the committed
# rocprofv3 FETCH_SIZE / WRITE_SIZE summary of this kernel (copy-calibrated)
COUNTERS_FILE = os.path.join(ROOT, "profiles", "force_mixed_plummer8m_counters.txt")


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=N_BIG)
    ap.add_argument("--n-act", type=int, default=NACT_BIG)
    ap.add_argument("--fp64-steps", type=int, default=None)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the timed steps (no energy pass, micro sizes, energy error)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--profile-pass", action="store_true",
                    help="short run for rocprofv3 counter passes: a plain copy of a known "
                         "size (counter calibration), then the mixed steps only")
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def err_stats(got, ref):
    """Per-particle relative error ||got_i - ref_i|| / ||ref_i||: max, p99,
    median and the fraction within 1e-6."""
    import numpy as np
    got, ref = np.asarray(got, dtype=np.float64), np.asarray(ref, dtype=np.float64)
    if got.ndim == 1:
        e = np.abs(got - ref) / np.abs(ref)
    else:
        e = np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)),
            "median": float(np.median(e)), "frac_le_1e-6": float((e <= 1e-6).mean())}


class BigStep:
    """The 8M-body system with one active set due at every block step."""

    def __init__(self, gen, precision, check=None):
        import numpy as np
        import torch

        from paper_1207_2367_amd import System
        m, x, v, a, sub = gen
        n = self.n = m.shape[0]
        self.n_act = sub.shape[0]
        dev = "cuda"
        self.sys = s = System(m, x, v, EPS, precision=precision, skip_startup=True)
        a_dev = torch.as_tensor(a, device=dev)
        s.set_state(a=a_dev)
        sub_dev = torch.as_tensor(sub, device=dev).to(torch.int32)
        got = s.force(sub_dev)
        torch.cuda.synchronize()
        self.errors = None
        if check is not None:
            pos, ref = check
            self.errors = {q: err_stats(g[pos].cpu().numpy(), r)
                           for q, g, r in zip(("acc", "jrk", "snp", "pot"), got, ref)}
        # consistent derivatives for the active particles, the smooth model
        # for the others; all at t = 0
        A = a_dev.clone()
        A[sub_dev.long()] = got[0]
        JK = torch.zeros_like(A)
        JK[sub_dev.long()] = got[1]
        SN = torch.zeros_like(A)
        SN[sub_dev.long()] = got[2]
        self.t0 = torch.zeros(n, dtype=torch.float64, device=dev)
        self.dt = torch.full((n,), DT_REST, dtype=torch.float64, device=dev)
        self.dt[sub_dev.long()] = DT_ACTIVE
        s.set_state(a=A, jk=JK, sn=SN, t=self.t0, dt=self.dt)
        torch.cuda.synchronize()
        del A, JK, SN, got, a_dev

    def step(self):
        s = self.sys
        s.set_state(t=self.t0, dt=self.dt)
        na, _ = s.block_step(DT_REST)
        assert na == self.n_act, (na, self.n_act)

    def run(self, steps, warmup):
        import torch
        for _ in range(warmup):
            self.step()
        torch.cuda.synchronize()
        self.sys.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            self.step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        prof = self.sys.profile(False)
        na, _, ms = self.sys.force_log()
        kms = float(ms[na == self.n_act].mean())
        phases = {k: round(v[0] / steps, 4) for k, v in prof.items() if k != "pairs"}
        return el, kms, phases

    def close(self):
        self.sys.close()


def micro_sizes(precisions):
    """The 65,536-body force microbenchmark: for N_act = 1 ... 65,536 the
    evaluation's time (nbody_force after the autotuner; the median of
    MICRO_REPS event-timed calls after MICRO_WARM untimed ones) and the
    per-particle errors of up to 512 active particles against the oracle."""
    import numpy as np
    import torch

    import ics
    import oracle
    from paper_1207_2367_amd import System
    n = N_MICRO
    m, x, v = ics.plummer(n, SEED_MICRO)
    a = ics.plummer_mean_acc(x)
    out = {}
    # the oracle first: the GPU's clock drops while it idles, and the small
    # sizes are timed right after a few warm-up calls
    subsets = {}
    refs = {}
    for na in MICRO_NACTS:
        idx = ics.active_subset(n, na, SEED_MICRO_SUB)
        pos = np.arange(na) if na <= 512 else np.sort(
            np.random.default_rng(na).choice(na, 512, replace=False))
        subsets[na] = (idx, pos)
        refs[na] = oracle.force(m, x, v, a, EPS, idx[pos])
    for name, prec in precisions:
        s = System(m, x, v, EPS, precision=prec, skip_startup=True)
        s.set_state(a=a)
        s.autotune(150.0)
        res = {}
        for na in MICRO_NACTS:
            idx, pos = subsets[na]
            idx_dev = torch.as_tensor(idx, device="cuda").to(torch.int32)
            got = s.force(idx_dev)
            for _ in range(MICRO_WARM):
                s.force(idx_dev)
            s.profile(True)
            for _ in range(MICRO_REPS):
                s.force(idx_dev)
            torch.cuda.synchronize()
            s.profile(False)
            lna, _, lms = s.force_log()
            t = float(np.median(lms[lna == na]))
            lp = s.get_launch(na)
            res[str(na)] = {"kernel_ms": round(t, 5),
                            "G_interactions_per_s": round(na * n / (t * 1e-3) / 1e9, 3),
                            "launch": {"lanes_per_i": lp[0], "waves": lp[1], "split": lp[2],
                                       "i_per_lane": lp[3]},
                            "errors": {q: err_stats(g.cpu().numpy()[pos], r) for q, g, r in
                                       zip(("acc", "jrk", "snp", "pot"), got, refs[na])}}
        s.close()
        out[name] = res
    return out


def energy_error(precision, n=N_MICRO, t_end=0.125):
    """Delta E / E of the 65,536-body Plummer sphere (seed 2002, full FP64
    start-up) integrated to t = 1/8 with block steps (eta 0.45)."""
    import ics
    from paper_1207_2367_amd import NBodyError, System
    m, x, v = ics.plummer(n, SEED_MICRO)
    s = System(m, x, v, EPS, precision=precision)
    try:
        e0 = sum(s.energy()[:2])
        st = s.step(t_end)
        e1 = sum(s.energy()[:2])
        return {"dE_over_E": (e1 - e0) / e0, "block_steps": st["block_steps"],
                "interactions": st["interactions"]}
    except NBodyError as e:
        return {"error": str(e)}
    finally:
        s.close()


def read_traffic():
    """HBM bytes per launch of the dominant kernel from the committed
    counter summary: (bytes, kernel, grid) or None."""
    try:
        text = open(COUNTERS_FILE).read()
    except OSError:
        return None
    tot, kern = 0.0, None
    for name in ("FETCH_SIZE", "WRITE_SIZE"):
        mm = re.search(r"# %s: .*dominant kernel dispatch \d+ \((.+?), grid (\d+), "
                       r"[\d.]+ ms\) [\d.e+]+ KiB -> ([\d.]+) MB per launch" % name, text)
        if not mm:
            return None
        kern = (mm.group(1), int(mm.group(2)))
        tot += float(mm.group(3)) * 1e6
    return tot, kern


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            return next((ln.split(":", 1)[1].strip() for ln in f if ln.startswith("model name")), "")
    except OSError:
        return ""


def cpu_baseline(gen, seconds):
    """The oracle timed on this host's cores on a bounded sample of the
    same block step (predict all N, evaluate a sampled active set against
    all N sources, correct it), on all cores and on one core."""
    import ctypes

    import numpy as np

    import oracle
    m, x, v, a, sub = gen
    n = m.shape[0]
    it = oracle.Integrator(m, x, v, EPS)
    gomp = ctypes.CDLL("libgomp.so.1")
    all_cores = len(os.sched_getaffinity(0))

    def one(n_act):
        dt = np.full(n, DT_REST)
        dt[sub[:n_act]] = DT_ACTIVE
        it.set_state(a=a, jk=0.0, sn=0.0, cr=0.0, t=np.zeros(n), dt=dt)
        t0 = time.perf_counter()
        it.block_step(DT_REST)
        return time.perf_counter() - t0

    res = {}
    for label, cores in (("all", all_cores), ("one", 1)):
        gomp.omp_set_num_threads(int(cores))
        cal = one(16)                      # predict all N + 16 x N pairs
        per_pair = max(cal - 0.0, 1e-9) / (16.0 * n)
        na = int(min(sub.shape[0], max(16, seconds / per_pair / n)))
        el, pairs, reps = 0.0, 0.0, 0
        while el < 0.8 * seconds or reps == 0:
            el += one(na)
            pairs += float(na) * n
            reps += 1
        res[label] = {"value": round(pairs / el / 1e9, 4), "cores": cores, "n_act": na,
                      "reps": reps, "seconds": round(el, 2)}
    gomp.omp_set_num_threads(all_cores)
    return {"value": res["all"]["value"], "unit": "G interactions/s", "cores": all_cores,
            "kind": "oracle", "cpu": cpu_model(), "nproc": os.cpu_count(),
            "one_core": res["one"],
            "sample": f"block steps of the N={n} Plummer sphere (seed {SEED_BIG}) in which a "
                      f"sampled subset of the benchmark's active set is due (predict all N, "
                      f"evaluate the subset against all N sources, correct): "
                      f"{res['all']['reps']} x {res['all']['n_act']} active on {all_cores} "
                      f"cores ({res['all']['seconds']} s), {res['one']['reps']} x "
                      f"{res['one']['n_act']} active on one core ({res['one']['seconds']} s); "
                      "FP64 C oracle, OpenMP over active particles"}


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
        # the dominant kernel of the bench: the mixed-mode evaluation shape
        # with the largest total time; its dispatches in launch order
        mixed = sorted((r for r in rows if "force_kernel<0," in r["Kernel_Name"]),
                       key=lambda r: int(r["Start_Timestamp"]))
        by_shape = {}
        for r in mixed:
            shape = (r["Kernel_Name"], r["Grid_Size_X"], r["Grid_Size_Y"])
            by_shape[shape] = by_shape.get(shape, 0) + int(r["End_Timestamp"]) - int(r["Start_Timestamp"])
        if by_shape:
            shape = max(by_shape, key=by_shape.get)
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


def make_inputs(n, n_act):
    import ics
    m, x, v = ics.plummer(n, SEED_BIG)
    a = ics.plummer_mean_acc(x)
    sub = ics.active_subset(n, n_act, SEED_SUB)
    return m, x, v, a, sub


def main():
    if len(sys.argv) == 3 and sys.argv[1] == "--summarize-profile":
        summarize_profile(sys.argv[2])
        return
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); the hot path has "
              "no multi-GPU mode", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    log(f"inputs: Plummer N={args.n}, {args.n_act} active")
    t_in = time.perf_counter()
    gen = make_inputs(args.n, args.n_act)
    log(f"inputs ready in {time.perf_counter() - t_in:.1f} s")

    # the oracle first, before anything touches the GPU: the CPU baseline and
    # the reference values of sampled active particles (for the check of the
    # first evaluation of each mode)
    import oracle
    m, x, v, a, sub = gen
    cpu = None
    check = None
    if not args.profile_pass:
        if not args.no_cpu_baseline:
            log("cpu baseline (oracle)")
            cpu = cpu_baseline(gen, args.cpu_seconds)
            log(f"cpu baseline: {cpu['value']} G/s on {cpu['cores']} cores, "
                f"{cpu['one_core']['value']} G/s on one")
        pos = np.sort(np.random.default_rng(9).choice(sub.shape[0], min(256, sub.shape[0]),
                                                      replace=False))
        t_o = time.perf_counter()
        check = (pos, oracle.force(m, x, v, a, EPS, sub[pos]))
        log(f"oracle reference of {pos.size} sampled particles in {time.perf_counter() - t_o:.1f} s")

    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    from paper_1207_2367_amd import PREC_FP32PAIR, PREC_FP64, PREC_MIXED
    from paper_1207_2367_amd import nbody
    if not os.path.exists(nbody.lib_path()):
        raise RuntimeError("libnbody.so is not built (python __graft_entry__.py build)")

    if args.profile_pass:
        # calibration for the HBM counters: copy 1 GiB that is not cache
        # resident (a second buffer is written in between), then the steps
        ca = torch.empty(1 << 28, dtype=torch.float32, device="cuda").fill_(1.0)
        cb = torch.empty_like(ca).fill_(2.0)
        cc = torch.empty_like(ca).fill_(3.0)
        cb.copy_(ca)
        torch.cuda.synchronize()
        del ca, cb, cc
        wl = BigStep(gen, PREC_MIXED)
        wl.run(args.steps, args.warmup)
        wl.close()
        torch.cuda.synchronize()
        log("profile pass done")
        return

    log(f"mixed: warmup {args.warmup}, steps {args.steps}")
    wl = BigStep(gen, PREC_MIXED, check)
    el, avg_ms, phases = wl.run(args.steps, args.warmup)
    pairs = float(args.n) * args.n_act
    value = pairs * args.steps / el / 1e9
    log(f"mixed: {el / args.steps * 1e3:.2f} ms/step, {value:.2f} G interactions/s, "
        f"kernel {avg_ms:.3f} ms")
    errors_mixed = wl.errors
    launch = wl.sys.get_launch(args.n_act)
    energy = None
    if not args.no_extras:
        # a8: the FP64 energy / angular momentum of the whole system, once, on
        # the synchronized prepared state (N^2 / 2 pairs)
        wl.sys.set_state(t=wl.t0, dt=wl.dt)
        torch.cuda.synchronize()
        t_e = time.perf_counter()
        ek, ep, L = wl.sys.energy()
        energy = {"ms": round((time.perf_counter() - t_e) * 1e3, 2), "ekin": ek, "epot": ep,
                  "L": L, "pairs": float(args.n) * (args.n - 1) / 2}
        log(f"energy pass: {energy['ms']:.1f} ms")
    wl.close()
    del wl

    ks = args.fp64_steps or max(2, args.steps // 2)
    other = {}
    for name, prec in (("fp64", PREC_FP64), ("fp32pair", PREC_FP32PAIR)):
        log(f"{name}: warmup 1, steps {ks}")
        wd = BigStep(gen, prec, check)
        eld, kmd, phd = wd.run(ks, 1)
        other[name] = {"value": round(pairs * ks / eld / 1e9, 3), "unit": "G interactions/s",
                       "ms_per_step": round(eld / ks * 1e3, 3), "kernel_ms": round(kmd, 4),
                       "kernel_tflops": round(FLOPS_PER_PAIR * pairs / (kmd * 1e-3) / 1e12, 3),
                       "errors": wd.errors, "phase_ms_per_step": phd}
        wd.close()
        del wd
    del gen

    micro = dE = None
    if not args.no_extras:
        log("force microbenchmark sizes (65,536 bodies)")
        micro = micro_sizes((("mixed", PREC_MIXED), ("fp64", PREC_FP64)))
        log("energy error, 65,536-body Plummer to t = 1/8")
        dE = {name: energy_error(prec) for name, prec in
              (("mixed", PREC_MIXED), ("fp64", PREC_FP64), ("fp32pair", PREC_FP32PAIR))}

    achieved = FLOPS_PER_PAIR * pairs / (avg_ms * 1e-3) / 1e12
    tr = read_traffic()
    # the kernel as rocprofv3 names it: force_kernel<precision, lanes per
    # particle, waves, eps == 0, potential, particles per lane group>, and
    # its grid in work-items (x: N_act * lanes / particles per group; y: split)
    kname = f"force_kernel<0, {launch[0]}, {launch[1]}, false, false, {max(1, launch[3])}>"
    grid_x = args.n_act * launch[0] // max(1, launch[3])
    traffic = None
    traffic_note = "no counter summary of this kernel"
    if tr is not None:
        if tr[1][0] == "void nb::" + kname and tr[1][1] == grid_x * launch[2]:
            traffic = round(tr[0])
            traffic_note = ("FETCH_SIZE + WRITE_SIZE per launch of this kernel, each scaled by "
                            "what the counter reads for a 1 GiB copy; "
                            + os.path.relpath(COUNTERS_FILE, ROOT))
        else:
            traffic_note = "the counter summary is of another kernel shape"
    f64 = other["fp64"]
    line = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "G interactions/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(el / args.steps * 1e3, 3),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {
            "workload": f"Plummer N={args.n} (seed {SEED_BIG}), eps=1e-4, Henon units, "
                        f"{args.n_act} active (seed {SEED_SUB}); one step = one block step "
                        "(schedule all N, predict all N, evaluate the active set against all "
                        "N sources, split reduction, correct + interpolate + new steps)",
            "n": args.n, "n_act": args.n_act, "precision": "mixed",
            "launch": {"lanes_per_i": launch[0], "waves": launch[1], "split": launch[2],
                       "i_per_lane": launch[3]},
        },
        "roofline": {
            "bound": "alu", "achieved": round(achieved, 3), "peak": PEAK_FP32,
            "unit": "TFLOP/s", "frac": round(achieved / PEAK_FP32, 4),
            "traffic": traffic, "traffic_note": traffic_note,
            "algorithmic_bytes": args.n * 68 + args.n_act * (4 + 68 + 80),
            "kernel": kname + f" grid {grid_x} x {launch[2]}",
            "kernel_avg_ms": round(avg_ms, 4), "flops_per_pair": FLOPS_PER_PAIR,
            "peak_basis": "MI355X FP32 vector 157.3 TFLOP/s (counts packed FP32)",
            "nonpacked_ceiling": {"peak": round(PEAK_FP32_NONPACKED, 2),
                                  "frac": round(achieved / PEAK_FP32_NONPACKED, 4),
                                  "note": "packed FP32 is switched off in the library, so "
                                          "0.5 of 157.3 is this kernel's ceiling"},
        },
        "errors_vs_oracle": {"sampled_active": 0 if check is None else int(check[0].size),
                             "mixed": errors_mixed, "fp64": f64["errors"],
                             "fp32pair": other["fp32pair"]["errors"]},
        "fp64_path": {k: f64[k] for k in ("value", "unit", "ms_per_step", "kernel_ms",
                                          "kernel_tflops")}
                     | {"frac_fp64_peak": round(f64["kernel_tflops"] / PEAK_FP64, 4)},
        "fp32pair_path": {k: other["fp32pair"][k] for k in ("value", "unit", "ms_per_step",
                                                              "kernel_ms", "kernel_tflops")}
                         | {"frac_fp32_peak": round(other["fp32pair"]["kernel_tflops"] / PEAK_FP32, 4),
                            "note": "every pair term in FP32: misses 1e-6 per particle for the "
                                    "jerk of some particles (errors_vs_oracle.fp32pair)"},
        "speedup_mixed_vs_fp64": round(value / f64["value"], 3),
        "kernel_speedup_mixed_vs_fp64": round(f64["kernel_ms"] / avg_ms, 3),
        "kernel_speedup_fp32pair_vs_fp64": round(f64["kernel_ms"] / other["fp32pair"]["kernel_ms"], 3),
        "dE_over_E_plummer65536_t0.125": dE,
        "energy_pass_8m": energy,
        "micro_plummer65536": micro,
        "paper_equiv_gflops": round(value * PAPER_FLOPS_PER_PAIR, 1),
        "paper_context": "about 4.1 G interactions/s per NVIDIA Tesla M2070 (400 GFLOPS at 97 "
                         "flops per interaction, 8M-body Plummer run)",
        "phase_ms_per_step": phases,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
