"""The persistent ensemble path (every block step of every cluster in one
launch; groups of workgroups integrate clusters independently, paper Sect. 3
block steps per cluster) against the host-sized path (one batched launch
sequence per block step) and the oracle.  In FP64 both paths and the oracle
take the same block steps: identical counts, N_act histogram, interactions,
times and steps of every particle; positions and velocities agree to the
rounding of the split sums as amplified by close pairs (1e-9)."""
import numpy as np
import pytest

import ics
import oracle
from gpu_helpers import cpu, log_case

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _pair(m, x, v, off, prec):
    from paper_1207_2367_amd import System
    loop = System(m, x, v, EPS, precision=prec, offsets=off)
    host = System(m, x, v, EPS, precision=prec, offsets=off)
    host.set_step_loop(0)
    return loop, host


@pytest.mark.parametrize("sizes", [[400, 256, 900, 1, 2100, 37],
                                   [8192] + [300] * 30,
                                   [3000, 2500, 12, 700, 5, 4096, 1500, 64]],
                         ids=["mixed-sizes", "one-dominant", "several-groups"])
def test_ensemble_loop_matches_host_path_fp64(sizes):
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    log_case(test="ensemble_vs_host", n=m.size, clusters=len(sizes))
    loop, host = _pair(m, x, v, off, 1)
    for t in (1.0 / 32, 1.0 / 8):
        a = loop.step(t)
        b = host.step(t)
        assert a["block_steps"] == b["block_steps"], (t, a["block_steps"], b["block_steps"])
        assert a["active_total"] == b["active_total"]
        assert a["interactions"] == b["interactions"]
        assert a["hist"] == b["hist"]
    ga = {k: cpu(q) for k, q in loop.get_state().items()}
    gb = {k: cpu(q) for k, q in host.get_state().items()}
    assert np.array_equal(ga["t"], gb["t"]) and np.array_equal(ga["dt"], gb["dt"])
    # the two paths sum the split partials of different launch shapes: the
    # states differ by rounding, amplified in the clusters' tight pairs
    for k in ("x", "v"):
        assert np.abs(ga[k] - gb[k]).max() <= 1e-9 * max(1.0, np.abs(gb[k]).max()), k
    ea, eb = loop.energy(), host.energy()
    assert abs(ea[0] + ea[1] - eb[0] - eb[1]) <= 1e-11 * abs(eb[0] + eb[1])
    loop.close()
    host.close()


def test_ensemble_loop_matches_oracle_fp64():
    """Four clusters (one of a single body) to t = 1/8 on the ensemble path
    against the oracle: the same block steps, interactions and histogram,
    positions to 1e-10."""
    from paper_1207_2367_amd import System
    sizes = [300, 1, 520, 128]
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    it = oracle.Integrator(m, x, v, EPS, offsets=off)
    assert it.init(0.125) == 0
    err, steps, pairs, hist = it.run(0.125)
    assert err == 0
    s = System(m, x, v, EPS, precision=1, offsets=off)
    st = s.step(0.125)
    assert st["block_steps"] == steps and st["interactions"] == pairs
    assert list(st["hist"]) == list(hist[:40])
    g = {k: cpu(q) for k, q in s.get_state().items()}
    assert np.abs(g["x"] - it.x).max() < 1e-10
    s.close()


@pytest.mark.parametrize("prec", [0, 2], ids=["mixed", "fp32pair"])
def test_ensemble_loop_mixed_modes(prec):
    """Mixed and FP32-pair evaluation on the ensemble path.  Mixed: the
    energy error of the ensemble to t = 1/4 is that of the host path (the
    two differ only in the rounding of the split sums).  FP32 pair terms
    make the step criterion noisy (the acceleration's FP32 rounding enters
    the fifth-derivative estimate), so the two paths' different roundings
    choose different steps: there both must only conserve energy to 1e-6."""
    sizes = [600, 1500, 300, 2000, 256]
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    loop, host = _pair(m, x, v, off, prec)
    e0 = sum(host.energy()[:2])
    a = loop.step(0.25)
    b = host.step(0.25)
    ea = (sum(loop.energy()[:2]) - e0) / abs(e0)
    eb = (sum(host.energy()[:2]) - e0) / abs(e0)
    log_case(test="ensemble_modes", prec=prec, dE_loop=ea, dE_host=eb,
             steps=(a["block_steps"], b["block_steps"]))
    assert abs(ea) < 1e-6 and abs(eb) < 1e-6
    if prec == 0:
        assert abs(ea - eb) <= 0.5 * max(abs(ea), abs(eb)) + 1e-12
        assert abs(a["interactions"] - b["interactions"]) <= 0.02 * b["interactions"]
    loop.close()
    host.close()


def test_ensemble_loop_deterministic_and_resumes():
    """Two runs give identical bits; a run split at t = 1/16 equals one to
    t = 1/8 (every cluster is synchronized at 1/16)."""
    from paper_1207_2367_amd import System
    sizes = [700, 900, 33, 2048]
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    runs = []
    for split in (False, True):
        s = System(m, x, v, EPS, precision=0, offsets=off)
        if split:
            s.step(1.0 / 16)
        s.step(1.0 / 8)
        runs.append({k: cpu(q).copy() for k, q in s.get_state().items()})
        s.close()
    s = System(m, x, v, EPS, precision=0, offsets=off)
    s.step(1.0 / 8)
    again = {k: cpu(q) for k, q in s.get_state().items()}
    for k in runs[0]:
        assert np.array_equal(runs[0][k], again[k]), k
        assert np.array_equal(runs[0][k], runs[1][k]), k
    s.close()
