"""Edge cases of the hot path through the C ABI, against the FP64 oracle or
closed forms: a one-particle system and one-particle clusters (no sources:
zero force, zero potential, the largest step, free motion), coincident
distinct particles under softening (zero mutual force, -m/eps potential,
paper Sect. 2), and the largest workload's source count (2^23 sources) on
sampled active particles."""
import numpy as np
import pytest
import torch

import ics
import oracle
from gpu_helpers import (FORCE_TOL, check_force, cpu, force, gpu_system, term_sums, log_case,
                         plummer_inputs)

pytestmark = pytest.mark.gpu

EPS = 1e-4
DMAX = 1.0 / 16
PRECS = [0, 1, 2]
IDS = ["mixed", "fp64", "fp32pair"]


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_single_particle(prec):
    """One body: every derivative and the potential are exactly zero, the
    step is the largest allowed, and the motion is free."""
    from paper_1207_2367_amd import System
    m = np.array([0.5])
    x = np.array([[0.1, -0.2, 0.3]])
    v = np.array([[0.01, 0.02, -0.03]])
    log_case(test="single_particle", prec=prec)
    s = System(m, x, v, EPS, precision=prec)
    st = s.get_state()
    for q in ("a", "jk", "sn", "cr"):
        assert not cpu(st[q]).any(), q
    assert cpu(st["dt"])[0] == DMAX
    ga, gj, gs, gp = (cpu(q) for q in force(s, [0]))
    assert not ga.any() and not gj.any() and not gs.any() and gp[0] == 0.0
    res = s.step(0.25)
    assert res["block_steps"] == 4
    st = s.get_state()
    assert np.abs(cpu(st["x"]) - (x + 0.25 * v)).max() <= 4e-16
    assert np.array_equal(cpu(st["v"]), v)
    ek, ep, L = s.energy()
    assert ep == 0.0 and abs(ek - 0.5 * 0.5 * (v * v).sum()) <= 1e-17


@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_one_particle_clusters(prec):
    """Clusters of one body among ordinary ones: the singletons move freely
    with the largest step; the rest integrates as the oracle does."""
    from paper_1207_2367_amd import System
    sizes = [1, 300, 1, 120]
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    rng = np.random.default_rng(11)
    for c in (0, 2):
        x[off[c]] = rng.normal(size=3)
        v[off[c]] = 0.1 * rng.normal(size=3)
    log_case(test="one_particle_clusters", prec=prec, sizes=sizes)
    it = oracle.Integrator(m, x, v, EPS, offsets=off)
    assert it.init(0.125) == 0
    assert it.run(0.125)[0] == 0
    s = System(m, x, v, EPS, precision=prec, offsets=off)
    s.step(0.125)
    st = s.get_state()
    gx, gt = cpu(st["x"]), cpu(st["t"])
    assert np.array_equal(gt, it.t)
    for c in (0, 2):
        i = off[c]
        assert np.abs(gx[i] - (x[i] + 0.125 * v[i])).max() <= 1e-15
        assert cpu(st["dt"])[i] == DMAX
    tol = 1e-9 if prec == 1 else 1e-6
    assert np.abs(gx - it.x).max() < tol


def test_force_empty_and_oversized_lists():
    """An empty active list does nothing (empty outputs, NBODY_OK); a count
    above n is rejected before any device work."""
    import ctypes as C

    from paper_1207_2367_amd import nbody
    m, x, v, a = plummer_inputs(300, 5)
    s = gpu_system(m, x, v, a, EPS, 0)
    got = s.force(np.zeros(0, dtype=np.int64))
    assert all(q.shape[0] == 0 for q in got)
    dummy = C.c_void_p(256)
    assert nbody.load().nbody_force(s.ctx, 301, dummy, dummy, dummy, dummy, None) == nbody.EINVAL
    assert nbody.load().nbody_force(s.ctx, -1, dummy, dummy, dummy, dummy, None) == nbody.EINVAL
    # the context still works
    ref = oracle.force(m, x, v, a, EPS, np.array([3, 7]))
    got = cpu(force(s, np.array([3, 7]))[0])
    assert np.abs(got - ref[0]).max() < 1e-12 * np.abs(ref[0]).max()


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_coincident_particles(prec):
    """Two distinct bodies at the same place (softened): no mutual force,
    a mutual potential of -m/eps each; a third body far away."""
    m = np.array([0.3, 0.2, 0.5])
    x = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [1.1, -0.4, 0.2]])
    v = np.array([[0.0, 0.1, 0.0], [0.05, -0.1, 0.02], [0.0, 0.0, 0.1]])
    a = ics.random_vectors(3, 5, 0.3)
    log_case(test="coincident", prec=prec)
    idx = [0, 1, 2]
    ref = oracle.force(m, x, v, a, EPS, idx)
    # the mutual potential dominates: -m_j / eps
    assert abs(ref[3][0] - (-0.2 / EPS - 0.5 / np.linalg.norm(x[2] - x[0]))) < 1e-12 * 0.2 / EPS
    s = gpu_system(m, x, v, a, EPS, prec)
    check_force(FORCE_TOL[prec], force(s, idx), ref, term_sums(m, x, v, a, EPS, idx))


@pytest.fixture(scope="module")
def big():
    n = 1 << 23
    m, x, v, a = plummer_inputs(n, 5005)
    idx = ics.active_subset(n, 12, 5006)
    return m, x, v, a, idx, oracle.force(m, x, v, a, EPS, idx), term_sums(m, x, v, a, EPS, idx)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_8m_sources_sampled(big, prec):
    """2^23 sources (the largest workload's system), 12 sampled active
    particles against the oracle, in the heuristic and a split-heavy launch
    shape."""
    from paper_1207_2367_amd import System
    m, x, v, a, idx, ref, S = big
    n = m.shape[0]
    log_case(test="8m_sources", prec=prec, n=n, n_act=len(idx))
    s = System(m, x, v, EPS, precision=prec, skip_startup=True)
    s.set_state(x=x, v=v, a=a, t=np.zeros(n), dt=np.full(n, DMAX))
    for shape in ((0, 0, 0), (64, 4, 1024)):
        s.set_launch(*shape)
        check_force(FORCE_TOL[prec], force(s, idx), ref, S)
    del s
    torch.cuda.empty_cache()


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_bench_active_set_8m_sampled(big, prec):
    """The benchmark's evaluation: 65,536 active particles (seed 5006)
    against the 2^23 sources, in the launch shape the library picks for it
    (its rule splits such long source ranges past the usual lane cap), 16 of
    the active particles against the oracle one by one."""
    from paper_1207_2367_amd import System
    m, x, v, a = big[:4]
    n = m.shape[0]
    idx = ics.active_subset(n, 65536, 5006)
    pos = np.sort(np.random.default_rng(7).choice(idx.size, 16, replace=False))
    ref = oracle.force(m, x, v, a, EPS, idx[pos])
    S = term_sums(m, x, v, a, EPS, idx[pos])
    s = System(m, x, v, EPS, precision=prec, skip_startup=True)
    s.set_state(x=x, v=v, a=a, t=np.zeros(n), dt=np.full(n, DMAX))
    shape = s.get_launch(idx.size)
    log_case(test="bench_active_8m", prec=prec, n=n, n_act=idx.size, launch=shape)
    assert shape[2] > 16   # past the 2^19-lane cap: every split keeps >= 2^17 sources
    got = [cpu(q) for q in force(s, idx)]
    check_force(FORCE_TOL[prec], [g[pos] for g in got], ref, S)
    s.close()
    del s
    torch.cuda.empty_cache()
