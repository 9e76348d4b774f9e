"""The schedule of nbody_step from per-level counts (one system on the
host-sized path: the next block time is the earliest next multiple of an
occupied level's step, its particles those of the levels whose step divides
it) against the sweep of every particle's next time and the FP64 oracle,
through the C ABI.

The two schedules pick the same block times and the same particles; only
the order of the active list differs (chunks fill it in order of completion
instead of index order), and no particle's evaluation or correction depends
on its slot, so every precision gives bit-identical states.
"""
import numpy as np
import pytest

import ics
import oracle
from gpu_helpers import cpu, log_case

pytestmark = pytest.mark.gpu

EPS = 1e-4


def _system(m, x, v, prec, mode, loop=0, **kw):
    from paper_1207_2367_amd import System
    s = System(m, x, v, EPS, precision=prec, **kw)
    s.set_step_loop(loop)
    s.set_schedule(mode)
    return s


def _state(s):
    return {k: cpu(q) for k, q in s.get_state().items()}


def _run(s, targets):
    tot = {"block_steps": 0, "active_total": 0, "interactions": 0.0, "hist": [0] * 40}
    for t in targets:
        st = s.step(t)
        for k in ("block_steps", "active_total", "interactions"):
            tot[k] += st[k]
        tot["hist"] = [a + b for a, b in zip(tot["hist"], st["hist"])]
    return tot


def _same(st, st_ref, g, g_ref):
    for k in ("block_steps", "active_total", "interactions", "hist"):
        assert st[k] == st_ref[k], k
    for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt"):
        assert np.array_equal(g[k], g_ref[k]), k


@pytest.mark.parametrize("prec", [1, 0, 2], ids=["fp64", "mixed", "fp32pair"])
def test_levels_match_sweep(prec):
    """A 4096-body sphere to t = 1/16 in three calls on the host-sized path:
    block steps, histogram, interactions and every state array identical
    with either schedule."""
    n = 4096
    m, x, v = ics.plummer(n, 4242)
    targets = (1.0 / 64, 1.0 / 32, 1.0 / 16)
    ref = _system(m, x, v, prec, 1)
    st_ref = _run(ref, targets)
    log_case(test="levels_vs_sweep", prec=prec, n=n)
    s = _system(m, x, v, prec, 0)
    st = _run(s, targets)
    print(f"steps {st['block_steps']} (sweep {st_ref['block_steps']})", flush=True)
    _same(st, st_ref, _state(s), _state(ref))
    s.close()
    ref.close()


def test_levels_automatic_on_larger_system():
    """A 65,536-body sphere (the device loop is off at this size, so the
    automatic mode schedules from levels) to t = 1/32 in the mixed mode:
    identical to the sweep, blocks of every size up to all particles."""
    n = 65536
    m, x, v = ics.plummer(n, 777)
    ref = _system(m, x, v, 0, 1, loop=-1)
    st_ref = _run(ref, (1.0 / 32,))
    log_case(test="levels_auto", n=n)
    s = _system(m, x, v, 0, 0, loop=-1)
    st = _run(s, (1.0 / 32,))
    print("hist", st["hist"][:18], flush=True)
    _same(st, st_ref, _state(s), _state(ref))
    s.close()
    ref.close()


def test_levels_oracle_blocks_and_energy():
    """The 1024-body sphere to t = 1/4 in FP64 on the host-sized path with
    the schedule from levels: the oracle's block steps, interactions and
    histogram, positions equal to roundoff-driven drift, the same energy
    error."""
    n = 1024
    m, x, v = ics.plummer(n, 1001)
    it = oracle.Integrator(m, x, v, EPS)
    it.init(0.25)
    e0 = sum(it.energy()[:2])
    err, steps, pairs, hist = it.run(0.25)
    assert err == 0
    de_o = (sum(it.energy()[:2]) - e0) / e0
    log_case(test="levels_oracle", n=n)
    s = _system(m, x, v, 1, 0)
    g0 = sum(s.energy()[:2])
    st = s.step(0.25)
    de_g = (sum(s.energy()[:2]) - g0) / g0
    g = _state(s)
    dx = np.abs(g["x"] - it.x).max()
    print(f"steps oracle {steps} gpu {st['block_steps']}; dE/E {de_o:.4e} {de_g:.4e}; "
          f"max|dx| {dx:.2e}")
    assert st["block_steps"] == steps
    assert st["interactions"] == pairs
    assert list(st["hist"]) == list(hist[:len(st["hist"])])
    assert dx < 1e-9
    assert abs(de_g - de_o) <= 1e-3 * abs(de_o) + 1e-14
    s.close()


def test_levels_black_hole_matches_oracle():
    """4096 Plummer stars around a central black hole of 5 % of the mass to
    t = 1/16 in FP64 with the schedule from levels: the oracle's block steps
    and interaction count, positions and velocities to roundoff drift."""
    m, x, v = ics.plummer_bh(4096, 1001, 0.05)
    it = oracle.Integrator(m, x, v, EPS)
    it.init(1.0 / 16)
    err, steps, pairs, hist = it.run(1.0 / 16)
    assert err == 0
    log_case(test="levels_black_hole", n=m.size)
    s = _system(m, x, v, 1, 0)
    st = s.step(1.0 / 16)
    g = _state(s)
    dx = np.abs(g["x"] - it.x).max()
    dv = np.abs(g["v"] - it.v).max()
    print(f"steps oracle {steps} gpu {st['block_steps']}; max|dx| {dx:.2e} max|dv| {dv:.2e}")
    assert st["block_steps"] == steps and st["interactions"] == pairs
    assert dx < 1e-10 and dv < 1e-9
    s.close()


def test_levels_decline_state_off_the_grid():
    """A state in which one particle's step is not a power of two, or one
    particle's time is not a multiple of its step (set with nbody_set_state):
    the schedule from levels declines and the sweep takes every block, so
    both modes end alike -- here with NBODY_EDTMIN, since such a particle can
    never land on the target by halving its step, as the sweep alone gives
    -- with identical states."""
    from paper_1207_2367_amd import NBodyError
    n = 2048
    m, x, v = ics.plummer(n, 99)
    for what in ("dt", "t"):
        runs = []
        for mode in (0, 1):
            s = _system(m, x, v, 1, mode)
            g = _state(s)
            t, dt = g["t"].copy(), g["dt"].copy()
            if what == "dt":
                dt[5] = 3.0 * dt[5] / 4.0
            else:
                t[7] = dt[7] / 2.0
            s.set_state(t=t, dt=dt)
            log_case(test="levels_decline", what=what, mode=mode)
            try:
                st, code = _run(s, (1.0 / 32,)), 0
            except NBodyError as e:
                st, code = None, e.code
            runs.append((code, st, _state(s)))
            s.close()
        print(what, "codes", runs[0][0], runs[1][0], flush=True)
        assert runs[0][0] == runs[1][0]
        if runs[0][1] is not None:
            for k in ("block_steps", "active_total", "interactions", "hist"):
                assert runs[0][1][k] == runs[1][1][k], k
        for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt"):
            assert np.array_equal(runs[0][2][k], runs[1][2][k]), k
