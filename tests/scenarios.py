"""Runs of the five workload configurations of the hot path on one GPU with
their checks against the FP64 oracle, each printing one JSON line (the
measured numbers quoted in the design notes; bench.py is the timed
benchmark).  Test infrastructure: not collected by pytest, run by hand:

    python tests/scenarios.py plummer1k      # 1024-body sphere to t = 1
    python tests/scenarios.py force64k       # force microbenchmark errors
    python tests/scenarios.py plummer1m      # 1M bodies to t = 0.125
    python tests/scenarios.py king256        # 256 King clusters to t = 1
    python tests/scenarios.py plummer8m      # 8M sources x 65,536 active
    python tests/scenarios.py bfactor16k     # split-source on/off vs N_act
    python tests/scenarios.py etascan        # energy error against eta
    python tests/scenarios.py etascan:32768:mixed   # one size, one path
    python tests/scenarios.py blocks32k      # where a small-block run spends its time
    python tests/scenarios.py plummer_to64:2097152   # 8M configuration's steps, 2M bodies
"""
from __future__ import annotations

import json
import math
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

GROUPS = [(1, 20, "A"), (21, 100, "B"), (101, 1000, "C"), (1001, 10000, "D"),
          (10001, 100000, "E"), (100001, 1 << 40, "F")]


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


def _rel_rows(g, r):
    g, r = np.asarray(g), np.asarray(r)
    if g.ndim == 1:
        return np.abs(g - r) / np.abs(r)
    return np.linalg.norm(g - r, axis=1) / np.linalg.norm(r, axis=1)


def _err_stats(e):
    return {"max": float(e.max()), "p99": float(np.percentile(e, 99)),
            "median": float(np.median(e)), "frac_le_1e-6": float((e <= 1e-6).mean())}


def _run(system, t_end, profile=True, pieces=1, t_start=0.0):
    """Advance from t_start to t_end in `pieces` equal calls (each a multiple
    of dt_max when both are), printing progress after each; returns summed
    stats."""
    if profile:
        system.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = None
    for k in range(1, pieces + 1):
        s = system.step(t_start + (t_end - t_start) * k / pieces)
        if st is None:
            st = s
        else:
            for key in ("block_steps", "active_total", "interactions"):
                st[key] += s[key]
            st["hist"] = [a + b for a, b in zip(st["hist"], s["hist"])]
        _log(f"  t = {t_start + (t_end - t_start) * k / pieces:.4f}: {st['block_steps']} block steps, "
             f"{time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = system.profile(False) if profile else None
    return st, wall, prof


def plummer1k():
    """1024-body Plummer sphere, eps 1e-4, eta 0.45, dt_max 1/16, to t = 1:
    oracle, GPU FP64 and GPU mixed."""
    import ics
    import oracle
    from paper_1207_2367_amd import PREC_FP32PAIR, PREC_FP64, PREC_MIXED, System
    m, x, v = ics.plummer(1024, 1001)
    it = oracle.Integrator(m, x, v, 1e-4)
    it.init(1.0)
    e0 = sum(it.energy()[:2])
    L0 = np.linalg.norm(it.energy()[2])
    t0 = time.perf_counter()
    it.run(1.0 / 16)
    x16 = it.x.copy()
    err, steps, pairs, hist = it.run(1.0)
    t_or = time.perf_counter() - t0
    res = {"config": "plummer1k", "oracle": {
        "dE_over_E": (sum(it.energy()[:2]) - e0) / e0,
        "dL_over_L": (np.linalg.norm(it.energy()[2]) - L0) / L0,
        "wall_s": t_or, "cores": len(os.sched_getaffinity(0))}}
    for name, prec in (("gpu_fp64", PREC_FP64), ("gpu_mixed", PREC_MIXED),
                       ("gpu_fp32pair", PREC_FP32PAIR)):
        s = System(m, x, v, 1e-4, precision=prec)
        g0 = sum(s.energy()[:2])
        gL0 = np.linalg.norm(s.energy()[2])
        st16, _, _ = _run(s, 1.0 / 16, profile=False)
        dx16 = float(np.abs(s.get_state()["x"].cpu().numpy() - x16).max())
        st, wall, _ = _run(s, 1.0, profile=False, t_start=1.0 / 16)
        ek, ep, L = s.energy()
        res[name] = {"dE_over_E": (ek + ep - g0) / g0,
                     "dL_over_L": (np.linalg.norm(L) - gL0) / gL0,
                     "block_steps": st16["block_steps"] + st["block_steps"],
                     "max_dx_vs_oracle_t1_16": dx16, "wall_s_1_16_to_1": wall,
                     "interactions": st16["interactions"] + st["interactions"]}
    # the whole run 0 -> 1 (mixed) with the device-resident block-step loop
    # (automatic for this size) and with every block on the host-sized path
    for name, lim in (("loop", -1), ("host_path", 0)):
        s = System(m, x, v, 1e-4, precision=PREC_MIXED)
        s.set_step_loop(lim)
        st, wall, _ = _run(s, 1.0, profile=False)
        res[f"gpu_mixed_{name}_0_to_1"] = {"wall_s": wall, "block_steps": st["block_steps"],
                                            "us_per_block_step": wall / st["block_steps"] * 1e6}
    return res


def force64k():
    """Force microbenchmark: N = 65,536 (seed 2002), active subsets of
    sizes 1 .. 65,536 (seed 2003), per-particle errors of both paths against
    the oracle (all particles for N_act <= 8192, 1024 sampled otherwise)."""
    import ics
    import oracle
    from paper_1207_2367_amd import PREC_FP32PAIR, PREC_FP64, PREC_MIXED, System
    n = 65536
    m, x, v = ics.plummer(n, 2002)
    a = ics.plummer_mean_acc(x)
    rng = np.random.default_rng(2003)
    res = {"config": "force64k", "n": n, "cases": []}
    systems = {}
    for name, prec in (("mixed", PREC_MIXED), ("fp64", PREC_FP64), ("fp32pair", PREC_FP32PAIR)):
        s = System(m, x, v, 1e-4, precision=prec)
        s.set_state(x=x, v=v, a=a, t=np.zeros(n), dt=np.full(n, 1.0 / 16))
        systems[name] = s
    for na in (1, 64, 1024, 8192, 65536):
        idx = np.sort(rng.choice(n, na, replace=False))
        chk = np.arange(na) if na <= 8192 else np.sort(np.random.default_rng(7).choice(na, 1024, replace=False))
        ref = oracle.force(m, x, v, a, 1e-4, idx[chk])
        case = {"n_act": na}
        for name, s in systems.items():
            got = [q.cpu().numpy() for q in s.force(idx)]
            case[name] = {q: _err_stats(_rel_rows(g[chk], r))
                          for q, g, r in zip(("acc", "jrk", "snp", "pot"), got, ref)}
        res["cases"].append(case)
        _log(f"force64k n_act {na} done")
    return res


def _hist_groups(hist):
    """Per-block N_act log2 histogram -> the paper's Fig. 7 groups (approx.,
    by the bin's lower edge)."""
    out = {g: 0 for _, _, g in GROUPS}
    for b, c in enumerate(hist):
        lo = 1 << b
        for a, z, g in GROUPS:
            if a <= lo <= z:
                out[g] += c
    return out


def _sampled_force_check(m, x, v, smp, prec):
    """Evaluation of the sampled particles against the oracle on inputs that
    both take from the generators: positions and velocities of the initial
    conditions and the smooth Plummer model's acceleration as the sources'
    acceleration (a context that skips the start-up passes)."""
    import ics
    import oracle
    from paper_1207_2367_amd import System
    a = ics.plummer_mean_acc(x)
    s = System(m, x, v, 1e-4, precision=prec, skip_startup=True)
    s.set_state(a=a)
    got = [q.cpu().numpy() for q in s.force(smp)]
    ref = oracle.force(m, x, v, a, 1e-4, smp)
    s.close()
    return got, ref


def _by_log2(na_log, pr_log, ms_log):
    """Evaluation launches grouped by floor(log2 N_act): count, pairs, time,
    rate (the efficiency of the batched launches by block size)."""
    out = {}
    for na, pr, ms in zip(na_log, pr_log, ms_log):
        if na <= 0:
            continue
        b = int(math.log2(na))
        o = out.setdefault(b, [0, 0.0, 0.0])
        o[0] += 1
        o[1] += float(pr)
        o[2] += float(ms)
    return {f"2^{b}": {"launches": o[0], "pairs": o[1], "ms": o[2],
                       "G_per_s": o[1] / (o[2] * 1e-3) / 1e9 if o[2] > 0 else None}
            for b, o in sorted(out.items())}


def plummer1m(t_end=0.125, n=1 << 20):
    """1M-body Plummer sphere (seed 3003), eps 1e-4, eta 0.45, to t = 0.125:
    mixed and FP64 paths, energy error, block N_act histogram, throughput,
    per-phase time; sampled forces checked against the oracle on the initial
    conditions."""
    import ics
    import oracle
    from paper_1207_2367_amd import PREC_FP64, PREC_MIXED, System
    m, x, v = ics.plummer(n, 3003)
    res = {"config": "plummer1m", "n": n, "t_end": t_end}
    smp = ics.active_subset(n, 256, 31)
    got, ref = _sampled_force_check(m, x, v, smp, PREC_MIXED)
    res["force_check_t0"] = {q: _err_stats(_rel_rows(g, r)) for q, g, r in
                             zip(("acc", "jrk", "snp", "pot"), got, ref)}
    for name, prec in (("mixed", PREC_MIXED), ("fp64", PREC_FP64)):
        t0 = time.perf_counter()
        s = System(m, x, v, 1e-4, precision=prec)
        torch.cuda.synchronize()
        t_init = time.perf_counter() - t0
        e0 = sum(s.energy()[:2])
        st, wall, prof = _run(s, t_end, pieces=16)
        na_log, pr_log, ms_log = s.force_log()
        e1 = sum(s.energy()[:2])
        # share of the evaluation time by the paper's Fig. 7 groups of N_act
        gt = {g: 0.0 for _, _, g in GROUPS}
        for na_, ms_ in zip(na_log, ms_log):
            for lo, hi, g in GROUPS:
                if lo <= na_ <= hi:
                    gt[g] += float(ms_)
        tot = sum(gt.values()) or 1.0
        res[name] = {"dE_over_E": (e1 - e0) / e0, "block_steps": st["block_steps"],
                     "force_time_share_by_group": {g: gt[g] / tot for g in gt},
                     "interactions": st["interactions"], "wall_s": wall, "init_s": t_init,
                     "G_interactions_per_s": st["interactions"] / wall / 1e9,
                     "phase_ms": {k: v[0] for k, v in prof.items() if k != "pairs"},
                     "n_act_log2_hist": st["hist"][:24],
                     "groups": _hist_groups(st["hist"])}
        _log(f"plummer1m {name}: {json.dumps(res[name])[:300]}")
        s.close()
        del s
        torch.cuda.empty_cache()
    return res


def bh64k(n=65536, t_end=0.125):
    """The 65,536-body Plummer sphere of the benchmark alone and around a
    central black hole of 1 % and 5 % of the mass (paper Sect. 5.5: such an
    object makes the blocks with few particles carry more of the run time):
    block steps, N_act groups of the paper's Fig. 7 and their share of the
    evaluation time, per-phase time and throughput to t = 1/8 (mixed); the
    hole's and 255 sampled stars' forces against the oracle at t = 0."""
    import ics
    from paper_1207_2367_amd import PREC_MIXED, System
    n = int(n)
    res = {"config": "bh64k", "n_stars": n, "t_end": t_end}
    for m_bh in (0.0, 0.01, 0.05):
        name = f"m_bh={m_bh}"
        m, x, v = ics.plummer_bh(n, 2002, m_bh) if m_bh > 0 else ics.plummer(n, 2002)
        if m_bh == 0.01:
            smp = np.concatenate([[0], ics.active_subset(m.size - 1, 255, 41) + 1])
            got, ref = _sampled_force_check(m, x, v, smp, PREC_MIXED)
            res["force_check_t0"] = {q: _err_stats(_rel_rows(g, r)) for q, g, r in
                                     zip(("acc", "jrk", "snp", "pot"), got, ref)}
            res["force_check_t0_hole"] = {q: float(_rel_rows(g[:1], r[:1])[0]) for q, g, r in
                                          zip(("acc", "jrk", "snp", "pot"), got, ref)}
        s = System(m, x, v, 1e-4, precision=PREC_MIXED)
        e0 = sum(s.energy()[:2])
        st, wall, _ = _run(s, t_end, profile=False, pieces=4)
        e1 = sum(s.energy()[:2])
        # the same run with the event timing of every phase and the per-launch log
        s = System(m, x, v, 1e-4, precision=PREC_MIXED)
        st2, wall2, prof = _run(s, t_end, pieces=4)
        na_log, pr_log, ms_log = s.force_log()
        gt = {g: 0.0 for _, _, g in GROUPS}
        for na_, ms_ in zip(na_log, ms_log):
            for lo, hi, g in GROUPS:
                if lo <= na_ <= hi:
                    gt[g] += float(ms_)
        tot = sum(gt.values()) or 1.0
        res[name] = {"dE_over_E": (e1 - e0) / e0, "block_steps": st["block_steps"],
                     "interactions": st["interactions"], "wall_s": wall,
                     "us_per_block_step": wall / st["block_steps"] * 1e6,
                     "G_interactions_per_s": st["interactions"] / wall / 1e9,
                     "groups": _hist_groups(st["hist"]),
                     "force_time_share_by_group": {g: gt[g] / tot for g in gt},
                     "profiled_wall_s": wall2,
                     "phase_ms": {k: q[0] for k, q in prof.items() if k != "pairs"}}
        _log(f"bh64k {name}: {json.dumps(res[name])[:300]}")
        s.close()
        del s
        torch.cuda.empty_cache()
    return res


def ensemble(t_end=0.25):
    """The 256-cluster King ensemble of king256 on the GPU alone (autotune,
    then block steps to t_end; no oracle runs): a short workload to trace."""
    import ics
    from paper_1207_2367_amd import PREC_MIXED, System
    m, x, v, off = ics.king_ensemble()
    s = System(m, x, v, 1e-4, precision=PREC_MIXED, offsets=off)
    s.autotune(100.0)
    st, wall, _ = _run(s, float(t_end), profile=False, pieces=4)
    return {"config": "ensemble", "n_total": int(m.size), "t_end": float(t_end),
            "block_steps": st["block_steps"], "interactions": st["interactions"],
            "wall_s": wall, "us_per_block_step": wall / st["block_steps"] * 1e6}


def king256(t_end=1.0):
    """256 King W0 = 6 clusters (Kroupa-like masses), all advanced together in
    one context to t = 1; 12 clusters also integrated by the oracle."""
    import ics
    import oracle
    from paper_1207_2367_amd import PREC_MIXED, System
    m, x, v, off = ics.king_ensemble()
    n = m.size
    sizes = np.diff(off)
    res = {"config": "king256", "n_total": int(n), "clusters": int(sizes.size)}
    t0 = time.perf_counter()
    s = System(m, x, v, 1e-4, precision=PREC_MIXED, offsets=off)
    s.autotune(100.0)
    torch.cuda.synchronize()
    res["init_s"] = time.perf_counter() - t0
    # per-cluster energies through separate contexts would cost N_c^2 each;
    # the ensemble energy of the whole context is one call
    e0 = sum(s.energy()[:2])
    st, wall, _ = _run(s, t_end, profile=False, pieces=16)
    e1 = sum(s.energy()[:2])
    # the phase breakdown from the same ensemble's next time unit with the
    # event timing on (which adds host work of its own)
    st2, wall2, prof = _run(s, 2 * t_end, pieces=16, t_start=t_end)
    na_log, pr_log, ms_log = s.force_log()
    res["mixed"] = {"dE_over_E_total": (e1 - e0) / e0, "block_steps": st["block_steps"],
                    "interactions": st["interactions"], "wall_s": wall,
                    "G_interactions_per_s": st["interactions"] / wall / 1e9,
                    "profiled_run": {"t": [t_end, 2 * t_end], "block_steps": st2["block_steps"],
                                     "interactions": st2["interactions"], "wall_s": wall2},
                    "phase_ms": {k: v[0] for k, v in prof.items() if k != "pairs"},
                    "evaluation_by_log2_n_act": _by_log2(na_log, pr_log, ms_log)}
    # oracle on the 8 smallest + 4 seeded-random clusters, and the GPU on
    # the same clusters alone
    pick = list(np.argsort(sizes)[:8]) + list(np.random.default_rng(4200).choice(sizes.size, 4, replace=False))
    per = []
    for c in pick:
        sl = slice(off[c], off[c + 1])
        it = oracle.Integrator(m[sl], x[sl], v[sl], 1e-4)
        it.init(t_end)
        o0 = sum(it.energy()[:2])
        for k in range(1, 17):   # in pieces, so that a long run keeps printing
            it.run(t_end * k / 16)
            if sizes[c] > 4000:
                _log(f"  king256 oracle cluster {c} (n = {sizes[c]}): t = {t_end * k / 16}")
        o1 = sum(it.energy()[:2])
        g = System(m[sl], x[sl], v[sl], 1e-4, precision=PREC_MIXED)
        g0 = sum(g.energy()[:2])
        g.step(t_end)
        g1 = sum(g.energy()[:2])
        per.append({"cluster": int(c), "n": int(sizes[c]), "oracle_dE_over_E": (o1 - o0) / o0,
                    "gpu_mixed_dE_over_E": (g1 - g0) / g0})
        _log(f"  king256 cluster {per[-1]}")
    res["per_cluster"] = per
    return res


def plummer8m(n=1 << 23, n_act=65536):
    """8M sources x 65,536 active (seed 5005 / 5006): the mixed evaluation
    alone (the state is the smooth-model start, no start-up passes), timed,
    with 1024 sampled particles checked against the oracle."""
    import ics
    import oracle
    from paper_1207_2367_amd import PREC_MIXED, System, nbody
    m, x, v = ics.plummer(n, 5005)
    a = ics.plummer_mean_acc(x)
    cfg = nbody.default_config(precision=PREC_MIXED)
    res = {"config": "plummer8m", "n": n, "n_act": n_act,
           "workspace_GB": nbody.workspace_bytes(n, cfg) / 1e9}
    # the start-up passes (two FP64 N^2 evaluations) would take minutes at
    # this size and are not part of this measurement: skip them and set the
    # state directly
    s = System(m, x, v, 1e-4, precision=PREC_MIXED, skip_startup=True)
    s.set_state(x=x, v=v, a=a, t=np.zeros(n), dt=np.full(n, 1.0 / 16))
    idx = ics.active_subset(n, n_act, 5006)
    s.autotune(200.0)
    s.force(idx)
    torch.cuda.synchronize()
    s.profile(True)
    reps = 3
    t0 = time.perf_counter()
    for _ in range(reps):
        got = s.force(idx)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / reps
    prof = s.profile(False)
    kms = prof["force"][0] / prof["force"][1]
    res["kernel_ms"] = kms
    res["wall_ms"] = wall * 1e3
    res["G_interactions_per_s_kernel"] = n * n_act / (kms * 1e-3) / 1e9
    res["tflops_83"] = 83 * n * n_act / (kms * 1e-3) / 1e12
    chk = np.sort(np.random.default_rng(9).choice(n_act, 1024, replace=False))
    ref = oracle.force(m, x, v, a, 1e-4, idx[chk])
    res["errors"] = {q: _err_stats(_rel_rows(g.cpu().numpy()[chk], r))
                     for q, g, r in zip(("acc", "jrk", "snp", "pot"), got, ref)}
    return res


def bfactor16k(n=16384):
    """Speed of the evaluation against active-set size for 16,384 sources
    (the paper's Fig. 8 setting, 1M bodies over 64 GPUs): the split-source
    factor and lanes per particle switched off (one lane per particle, one
    split, 4 waves) against the autotuned shapes."""
    import ics
    from paper_1207_2367_amd import PREC_MIXED, System
    m, x, v = ics.plummer(n, 2002)
    s = System(m, x, v, 1e-4, precision=PREC_MIXED)
    s.autotune(100.0)
    rows = []
    for b in range(0, 15):
        na = 1 << b
        idx = ics.active_subset(n, na, 100 + b)
        r = {"n_act": na}
        for name, shape in (("bfactor_off", (1, 4, 1)), ("autotuned", (0, 0, 0))):
            s.set_launch(*shape)
            r[name + "_launch"] = s.get_launch(na)
            s.force(idx)
            s.profile(True)
            for _ in range(20):
                s.force(idx)
            prof = s.profile(False)
            ms = prof["force"][0] / prof["force"][1] + (prof["reduce"][0] / 20 if prof["reduce"][1] else 0.0)
            r[name + "_ms"] = ms
            r[name + "_G_per_s"] = na * n / (ms * 1e-3) / 1e9
        r["gain"] = r["bfactor_off_ms"] / r["autotuned_ms"]
        rows.append(r)
    return {"config": "bfactor16k", "n": n, "rows": rows}


def etascan(n=None, precs="mixed,fp64", etas=(0.2, 0.3, 0.45, 0.6, 0.8, 1.0), t_end=10.0):
    """Energy and angular-momentum error against eta (the paper's Fig. 1
    experiment): Plummer spheres of 2^15 and 2^16 bodies (or n), 10 time
    units, the paper's average of the relative errors at t = 1 .. 10, the
    mixed and the FP64 paths (or the comma-separated list precs), at the
    given eta values (or a comma-separated list)."""
    import ics
    from paper_1207_2367_amd import PREC_FP64, PREC_MIXED, NBodyError, System
    ns = (1 << 15, 1 << 16) if n is None else (int(n),)
    if isinstance(etas, str):
        etas = tuple(float(e) for e in etas.split(","))
    modes = [(p, {"mixed": PREC_MIXED, "fp64": PREC_FP64}[p]) for p in precs.split(",")]
    rows = []
    for n in ns:
        m, x, v = ics.plummer(n, 7000 + n % 997)
        for eta in etas:
            for name, prec in modes:
                s = System(m, x, v, 1e-4, precision=prec, eta=eta)
                ek, ep, L = s.energy()
                e0, l0 = ek + ep, np.linalg.norm(L)
                de, dl, steps, inter, t0 = [], [], 0, 0.0, time.perf_counter()
                try:
                    for t in range(1, int(t_end) + 1):
                        st = s.step(float(t))
                        steps += st["block_steps"]
                        inter += st["interactions"]
                        ek, ep, L = s.energy()
                        de.append(abs((ek + ep - e0) / e0))
                        dl.append(abs((np.linalg.norm(L) - l0) / l0))
                        _log(f"  n {n} eta {eta} {name}: t = {t}, {steps} block steps, "
                             f"dE/E {de[-1]:.3e}, {time.perf_counter() - t0:.1f} s")
                    err = None
                except NBodyError as e:
                    err = str(e)
                rows.append({"n": n, "eta": eta, "precision": name,
                             "dE_avg": float(np.mean(de)) if de else None,
                             "dL_avg": float(np.mean(dl)) if dl else None,
                             "block_steps": steps, "interactions": inter,
                             "wall_s": time.perf_counter() - t0, "error": err})
                _log(f"etascan {rows[-1]}")
    return {"config": "etascan", "rows": rows}


def blocks32k(n=32768, t_end=1.0):
    """Where the time of a small-block integration goes: a 32,768-body
    Plummer sphere (seed 7000 + n % 997, eta 0.45) to t = 1 (schedule from
    per-level counts, then from the sweep), then with the phase profile; per
    block step: wall time, GPU time by phase, evaluation efficiency by
    N_act."""
    import ics
    from paper_1207_2367_amd import PREC_MIXED, System
    n = int(n)
    m, x, v = ics.plummer(n, 7000 + n % 997)
    s = System(m, x, v, 1e-4, precision=PREC_MIXED)
    st0, wall0, _ = _run(s, float(t_end), profile=False, pieces=4)
    # the same with the schedule from a sweep of every particle per block
    # step instead of the per-level counts
    s = System(m, x, v, 1e-4, precision=PREC_MIXED)
    s.set_schedule(1)
    st1, wall1, _ = _run(s, float(t_end), profile=False, pieces=4)
    # the same run again with the event timing of every phase (which adds
    # host work of its own)
    s = System(m, x, v, 1e-4, precision=PREC_MIXED)
    st, wall, prof = _run(s, float(t_end), pieces=4)
    na_log, pr_log, ms_log = s.force_log()
    steps = st["block_steps"]
    phase_ms = {k: v[0] for k, v in prof.items() if k != "pairs"}
    # and with autotuned launch shapes instead of the rule
    s = System(m, x, v, 1e-4, precision=PREC_MIXED)
    s.autotune(50.0)
    st2, wall2, _ = _run(s, float(t_end), profile=False, pieces=4)
    return {"config": "blocks32k", "n": n, "block_steps": steps, "wall_s": wall0,
            "wall_s_sweep_schedule": wall1, "block_steps_sweep_schedule": st1["block_steps"],
            "us_per_block_step_sweep_schedule": wall1 / st1["block_steps"] * 1e6,
            "wall_s_autotuned": wall2, "block_steps_autotuned": st2["block_steps"],
            "wall_s_profiled": wall, "interactions": st["interactions"],
            "us_per_block_step": wall0 / st0["block_steps"] * 1e6,
            "gpu_us_per_block_step_by_phase": {k: v / steps * 1e3 for k, v in phase_ms.items()},
            "launches_by_phase": {k: v[1] for k, v in prof.items() if k != "pairs"},
            "evaluation_by_log2_n_act": _by_log2(na_log, pr_log, ms_log)}


def plummer_to64(n=1 << 21, t_end=1.0 / 64):
    """The 8M-body configuration's integration at a size that fits one run
    (seed 5005, eps 1e-4, eta 0.45): one FP64 start-up, its state copied
    into a mixed context, then both paths to t = 1/64 (the target caps the
    last steps); energy error, block-level N_act histogram (log2 bins and
    the paper's Fig. 7 groups), interactions and rates."""
    import ics
    from paper_1207_2367_amd import PREC_FP64, PREC_MIXED, System
    n = int(n)
    t_end = float(t_end)
    m, x, v = ics.plummer(n, 5005)
    res = {"config": "plummer_to64", "n": n, "t_end": t_end}
    t0 = time.perf_counter()
    f = System(m, x, v, 1e-4, precision=PREC_FP64)
    torch.cuda.synchronize()
    res["startup_s"] = time.perf_counter() - t0
    _log(f"  start-up of {n} bodies: {res['startup_s']:.1f} s")
    st0 = f.get_state()
    g = System(m, x, v, 1e-4, precision=PREC_MIXED, skip_startup=True)
    g.set_state(**st0)
    e0 = sum(f.energy()[:2])
    for name, s in (("mixed", g), ("fp64", f)):
        st, wall, _ = _run(s, t_end, profile=False, pieces=4)
        e1 = sum(s.energy()[:2])
        res[name] = {"dE_over_E": (e1 - e0) / e0, "block_steps": st["block_steps"],
                     "interactions": st["interactions"], "wall_s": wall,
                     "G_interactions_per_s": st["interactions"] / wall / 1e9,
                     "hist_log2": st["hist"], "groups": _hist_groups(st["hist"])}
        _log(f"  {name}: {res[name]['block_steps']} block steps, dE/E {res[name]['dE_over_E']:.3e}")
        s.close()
    return res


RUNS = {"plummer1k": plummer1k, "force64k": force64k, "plummer1m": plummer1m,
        "king256": king256, "plummer8m": plummer8m, "bfactor16k": bfactor16k,
        "etascan": etascan, "blocks32k": blocks32k, "bh64k": bh64k, "ensemble": ensemble,
        "plummer_to64": plummer_to64}


def _default(o):
    if isinstance(o, (np.integer,)):
        return int(o)
    if isinstance(o, (np.floating,)):
        return float(o)
    return str(o)


def _close_systems():
    """Release every GPU system the run left alive (so that no library call
    runs from a destructor while the interpreter shuts down)."""
    import gc

    from paper_1207_2367_amd import System
    gc.collect()
    for o in gc.get_objects():
        if type(o) is System:   # (isinstance would touch deprecated torch objects)
            o.close()
    torch.cuda.synchronize()


if __name__ == "__main__":
    # each argument: NAME or NAME:ARG[:ARG...] (positional arguments of the run)
    for spec in sys.argv[1:]:
        name, *args = spec.split(":")
        _log(f"scenario {spec}")
        out = RUNS[name](*args)
        _close_systems()
        print(json.dumps(out, default=_default), flush=True)
