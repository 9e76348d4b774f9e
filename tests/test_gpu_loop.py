"""The device-resident block-step loop of nbody_step (block steps of one
system inside one cooperative launch, three grid barriers per step) against
the host-sized path and the FP64 oracle, through the C ABI.

The loop evaluates with its own launch shape (64 lanes per active particle,
its own split of the sources), so its sums differ from the host path's in
rounding only.  In FP64 that leaves the block structure unchanged: the same
block steps, N_act histogram and interaction count, and states equal to
roundoff.  In the mixed mode the FP32 jerk and snap terms differ at their
rounding level, which can move a new step across a power of two (either
neighbour is correct), so there the runs are compared by their statistics
and by the distance between the trajectories.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_helpers import cpu, log_case

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _system(m, x, v, prec, loop, **kw):
    from paper_1207_2367_amd import System
    s = System(m, x, v, EPS, precision=prec, **kw)
    s.set_step_loop(loop)
    return s


def _state(s):
    return {k: cpu(q) for k, q in s.get_state().items()}


@pytest.mark.parametrize("prec", [1, 0, 2], ids=["fp64", "mixed", "fp32pair"])
def test_loop_matches_host_path(prec):
    """A 4096-body sphere to t = 1/16: host path only, the loop on every
    block (automatic limit), and the loop with a limit of 8 active particles,
    which hands every larger block to the host path and resumes after it."""
    n = 4096
    m, x, v = ics.plummer(n, 4242)
    ref = _system(m, x, v, prec, 0)
    st_ref = ref.step(1.0 / 16)
    g_ref = _state(ref)
    for lim in (-1, 8):
        log_case(test="loop_vs_host", prec=prec, limit=lim)
        s = _system(m, x, v, prec, lim)
        st = s.step(1.0 / 16)
        g = _state(s)
        dx = np.abs(g["x"] - g_ref["x"]).max()
        print(f"prec {prec} limit {lim}: steps {st['block_steps']} vs {st_ref['block_steps']}, "
              f"max |dx| {dx:.2e}")
        assert np.all(g["t"] == 1.0 / 16)
        if prec == 1:
            assert st["block_steps"] == st_ref["block_steps"]
            assert st["active_total"] == st_ref["active_total"]
            assert st["interactions"] == st_ref["interactions"]
            assert st["hist"] == st_ref["hist"]
            assert dx < 1e-12
            assert np.abs(g["v"] - g_ref["v"]).max() < 1e-11
        else:
            assert abs(st["block_steps"] - st_ref["block_steps"]) <= 0.02 * st_ref["block_steps"]
            assert dx < 1e-6


def test_loop_energy_and_oracle_blocks():
    """The 1024-body sphere (all of its blocks run inside the loop) to
    t = 1/4 in FP64: the same number of block steps and interactions as the
    oracle, positions equal to roundoff-driven drift, and the same energy
    error."""
    n = 1024
    m, x, v = ics.plummer(n, 1001)
    it = oracle.Integrator(m, x, v, EPS)
    it.init(0.25)
    e0 = sum(it.energy()[:2])
    err, steps, pairs, hist = it.run(0.25)
    assert err == 0
    de_o = (sum(it.energy()[:2]) - e0) / e0
    s = _system(m, x, v, 1, -1)
    g0 = sum(s.energy()[:2])
    st = s.step(0.25)
    de_g = (sum(s.energy()[:2]) - g0) / g0
    g = _state(s)
    dx = np.abs(g["x"] - it.x).max()
    print(f"steps oracle {steps} gpu {st['block_steps']}; dE/E {de_o:.4e} {de_g:.4e}; max|dx| {dx:.2e}")
    assert st["block_steps"] == steps
    assert st["interactions"] == pairs
    assert dx < 1e-9
    assert abs(de_g - de_o) <= 1e-3 * abs(de_o) + 1e-14


@pytest.mark.parametrize("loop", [0, -1], ids=["host", "loop"])
def test_black_hole_blocks_match_oracle(loop):
    """4096 Plummer stars around a central black hole of 5 % of the mass
    (a heavy particle and stiffer central dynamics) to t = 1/16 in FP64, on
    the host-sized path and through the device loop: the oracle's block
    steps and interaction count, positions and velocities to roundoff-level
    drift, the same energy error."""
    m, x, v = ics.plummer_bh(4096, 1001, 0.05)
    it = oracle.Integrator(m, x, v, EPS)
    it.init(1.0 / 16)
    e0 = sum(it.energy()[:2])
    err, steps, pairs, hist = it.run(1.0 / 16)
    assert err == 0
    de_o = (sum(it.energy()[:2]) - e0) / e0
    log_case(test="black_hole", loop=loop, n=m.size)
    s = _system(m, x, v, 1, loop)
    g0 = sum(s.energy()[:2])
    st = s.step(1.0 / 16)
    de_g = (sum(s.energy()[:2]) - g0) / g0
    g = _state(s)
    dx = np.abs(g["x"] - it.x).max()
    dv = np.abs(g["v"] - it.v).max()
    print(f"loop {loop}: steps oracle {steps} gpu {st['block_steps']}; max|dx| {dx:.2e} "
          f"max|dv| {dv:.2e}; dE/E {de_o:.4e} {de_g:.4e}")
    assert st["block_steps"] == steps and st["interactions"] == pairs
    assert dx < 1e-10 and dv < 1e-9
    assert abs(de_g - de_o) <= 1e-3 * abs(de_o) + 1e-14


@pytest.mark.parametrize("loop", [0, -1], ids=["host", "loop"])
def test_loop_reports_dtmin(loop):
    """A pair plunging towards each other without softening: the start-up
    passes succeed, then within the first steps the criterion asks for less
    than dt_min = 2^-16 (as the oracle finds): NBODY_EDTMIN from the device
    loop as from the host path."""
    from paper_1207_2367_amd import NBodyError, System
    m = np.array([0.4, 0.4, 0.2])
    xx = np.array([[0.0, 0, 0], [0.01, 0, 0], [1.0, 0, 0]])
    vv = np.array([[0.0, 0, 0], [-3.0, 0.05, 0], [0.0, 0, 0]])
    it = oracle.Integrator(m, xx, vv, 0.0, dt_min=2.0 ** -16)
    assert it.init(1.0) == 0
    assert it.run(2.0 ** -6)[0] == oracle.EDTMIN
    s = System(m, xx, vv, 0.0, precision=1, dt_min=2.0 ** -16)
    s.set_step_loop(loop)
    with pytest.raises(NBodyError) as e:
        s.step(2.0 ** -6)
    assert e.value.code == -4


def test_loop_deterministic_and_resumes():
    """Mixed mode through the loop: identical bits on a second run, and
    0 -> 1/8 equals 0 -> 1/16 -> 1/8 (the loop stops at the first target and
    a new launch picks up)."""
    n = 2048
    m, x, v = ics.plummer(n, 77)
    a = _system(m, x, v, 0, -1)
    a.step(0.125)
    b = _system(m, x, v, 0, -1)
    b.step(0.0625)
    b.step(0.125)
    c = _system(m, x, v, 0, -1)
    c.step(0.125)
    sa, sb, sc = _state(a), _state(b), _state(c)
    for k in sa:
        assert np.array_equal(sa[k], sc[k]), k
        assert np.array_equal(sa[k], sb[k]), k


def test_profiling_counts_and_results():
    """Event timing of the phases (paper Table 1 sections) over a run: one
    schedule and one predictor launch per block step plus the final empty
    schedule, one evaluation and one corrector per block step, the logged
    evaluations' pairs summing to the run's interactions, and the same bits
    as the same run without profiling on the host-sized path (profiling
    keeps the device loop off)."""
    n = 2048
    m, x, v = ics.plummer(n, 99)
    a = _system(m, x, v, 0, 0)
    st_a = a.step(1.0 / 16)
    b = _system(m, x, v, 0, -1)
    b.profile(True)
    st_b = b.step(1.0 / 16)
    prof = b.profile(False)
    na, pr, ms = b.force_log()
    steps = st_b["block_steps"]
    print({k: v for k, v in prof.items()}, steps)
    assert steps == st_a["block_steps"] and st_b["interactions"] == st_a["interactions"]
    assert prof["schedule"][1] == steps + 1 and prof["predict"][1] == steps + 1
    assert prof["force"][1] == steps and prof["correct"][1] == steps
    assert prof["energy"][1] == 0
    assert na.size == steps and int(na.sum()) == st_b["active_total"]
    assert abs(pr.sum() - st_b["interactions"]) <= 1e-9 * st_b["interactions"]
    assert abs(prof["pairs"] - st_b["interactions"]) <= 1e-9 * st_b["interactions"]
    assert np.all(ms > 0) and all(prof[k][0] > 0 for k in ("schedule", "predict", "force", "correct"))
    sa, sb = _state(a), _state(b)
    for k in sa:
        assert np.array_equal(sa[k], sb[k]), k
