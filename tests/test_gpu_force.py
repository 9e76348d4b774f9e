"""GPU parity of the evaluation step (paper Sect. 3, item 2, softened as in
Sect. 2) through the C ABI: the mixed-precision and the FP64 kernels against
the FP64 oracle, element by element, on seeded Plummer inputs.

Tolerance (per particle i and quantity Q, with S_i(Q) = sum_j |Q_ij| the sum
of the magnitudes of the pair terms and kappa_i(Q) = S_i(Q) / |sum_j Q_ij|
the condition number of the sum):

    every output finite, and ||Q_gpu - Q_oracle|| <= k(Q) * S_i(Q)

i.e. relative error <= k kappa_i, written so that a zero reference (a
one-body cluster) or a non-finite output cannot slip through.  A pair term
evaluated in FP32 (unit roundoff u = 2^-24 = 6e-8) carries about a dozen
roundings (difference, r^2, rsqrt, r^-3, alpha, beta, products), i.e. at
most ~16 u = 1e-6 relative; a sum of such terms is off by at most that
times S_i.  The snap pair term has one more cancelling level
(-6 alpha J - 3 beta A): 2e-6.  Terms computed in FP64 (the mixed mode's
acceleration, jerk and potential: 1/r from an FP32 seed and one Newton
step, ~1e-14) get 1e-11; the FP64 mode 1e-12 (1e-11 snap).  Where a plain
per-particle bound is stated (FORCE_TOL's second entry: 1e-6 for the mixed
mode's a, da and potential) it is asserted as well on every row with a
non-zero reference.  The tests print the plain max / p99 errors and the
fraction within 1e-6.
"""
import numpy as np
import pytest
import torch

import ics
import oracle
from gpu_helpers import (FORCE_TOL, check_force, cpu, force, gpu_system, term_sums, log_case,
                         plummer_inputs)

pytestmark = pytest.mark.gpu

TOL = FORCE_TOL
PRECS = [0, 1, 2]
IDS = ["mixed", "fp64", "fp32pair"]
EPS = 1e-4


def _check(prec, got, ref, S):
    return check_force(TOL[prec], got, ref, S)


@pytest.fixture(scope="module")
def inputs():
    n = 5000 + 77     # several tiles of every size and a ragged tail
    return plummer_inputs(n, 2002)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
@pytest.mark.parametrize("n_act", [1, 7, 64, 333, 5077])
def test_force_parity(inputs, prec, n_act):
    m, x, v, a = inputs
    n = m.shape[0]
    log_case(test="force_parity", prec=prec, n=n, n_act=n_act)
    idx = ics.active_subset(n, n_act, 7 + n_act)
    ref = oracle.force(m, x, v, a, EPS, idx)
    s = gpu_system(m, x, v, a, EPS, prec)
    got = force(s, idx)
    torch.cuda.synchronize()
    _check(prec, got, ref, term_sums(m, x, v, a, EPS, idx))


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_every_launch_shape(inputs, prec):
    """Each lanes-per-particle / waves / split-source / particles-per-lane
    shape gives the same result to the tolerance (fixed-order reductions);
    150 active particles leave the last i-block of every shape ragged."""
    m, x, v, a = inputs
    n = m.shape[0]
    idx = ics.active_subset(n, 150, 5)
    ref = oracle.force(m, x, v, a, EPS, idx)
    S = term_sums(m, x, v, a, EPS, idx)
    s = gpu_system(m, x, v, a, EPS, prec)
    for lpi in (1, 2, 4, 8, 16, 32, 64):
        for waves in (1, 2, 4):
            for split in (1, 3, 16):
                for ipt in ((1, 2) if lpi <= 4 else (1,)):
                    log_case(test="launch_shape", prec=prec, lpi=lpi, waves=waves, split=split,
                             ipt=ipt)
                    s.set_launch(lpi, waves, split, ipt)
                    got = force(s, idx)
                    torch.cuda.synchronize()
                    _check(prec, got, ref, S)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_deterministic(inputs, prec):
    m, x, v, a = inputs
    idx = ics.active_subset(m.shape[0], 1000, 3)
    s = gpu_system(m, x, v, a, EPS, prec)
    r1 = [cpu(q).copy() for q in force(s, idx)]
    r2 = [cpu(q).copy() for q in force(s, idx)]
    for p, q in zip(r1, r2):
        assert np.array_equal(p, q)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_unsoftened_kepler(prec):
    """eps = 0 (masked self pair): circular binary closed forms plus a few
    far particles of negligible mass."""
    m1, m2, R = 0.25, 0.75, 0.8
    M = m1 + m2
    w = np.sqrt(M / R ** 3)
    u = np.array([np.cos(0.7), np.sin(0.7), 0.0])
    ut = np.array([-np.sin(0.7), np.cos(0.7), 0.0])
    x = np.array([-(m2 / M) * R * u, (m1 / M) * R * u])
    v = np.array([-(m2 / M) * R * w * ut, (m1 / M) * R * w * ut])
    a = -w * w * x
    log_case(test="kepler_eps0", prec=prec)
    s = gpu_system(np.array([m1, m2]), x, v, a, 0.0, prec)
    ga, gj, gs, gp = (cpu(q) for q in force(s, [0, 1]))
    tol = {0: 1e-6, 1: 1e-13, 2: 1e-6}[prec]
    assert np.abs(ga + w ** 2 * x).max() < tol * w ** 2 * R
    assert np.abs(gj + w ** 2 * v).max() < tol * w ** 3 * R
    assert np.abs(gs - w ** 4 * x).max() < 4 * tol * w ** 4 * R
    np.testing.assert_allclose(gp, [-m2 / R, -m1 / R], rtol=tol)


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_clusters(prec):
    """Independent clusters: each particle only feels its own cluster."""
    sizes = [300, 77, 1200, 256, 640]
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    a = ics.random_vectors(m.size, 4, 0.5)
    idx = np.sort(np.concatenate([ics.active_subset(sizes[c], max(1, sizes[c] // 5), c) + off[c]
                                  for c in range(len(sizes))]))
    log_case(test="clusters", prec=prec, n=m.size, n_act=idx.size)
    ref = [np.zeros((idx.size, 3)) for _ in range(3)] + [np.zeros(idx.size)]
    S = np.zeros((idx.size, 4))
    for c in range(len(sizes)):
        sel = (idx >= off[c]) & (idx < off[c + 1])
        r = oracle.force(m, x, v, a, EPS, idx[sel], (off[c], off[c + 1]))
        S[sel] = term_sums(m, x, v, a, EPS, idx[sel], (off[c], off[c + 1]))
        for q in range(4):
            ref[q][sel] = r[q]
    s = gpu_system(m, x, v, a, EPS, prec, offsets=off)
    for shape in ((0, 0, 0), (1, 4, 1), (8, 1, 4), (64, 1, 2)):
        s.set_launch(*shape)
        _check(prec, force(s, idx), ref, S)


@pytest.mark.parametrize("n_clusters", [1500, 9000])
def test_force_many_clusters(n_clusters):
    """1500 clusters of 1-12 bodies (more clusters than the 1024 lanes of
    the block-table scan) and 9000 (more than the block table keeps in LDS,
    so the search runs in global memory), a third of them without active
    particles: each active particle feels only its own cluster, in a split
    and an unsplit shape."""
    rng = np.random.default_rng(n_clusters)
    sizes = rng.integers(1, 13, n_clusters)
    off = np.concatenate([[0], np.cumsum(sizes)])
    m, x, v, a = plummer_inputs(int(off[-1]), n_clusters + 1)
    keep = rng.random(sizes.size) < 2 / 3
    idx = np.sort(np.concatenate([np.arange(off[c], off[c + 1])[rng.random(sizes[c]) < 0.5]
                                  for c in range(sizes.size) if keep[c]]))
    log_case(test="many_clusters", n=m.size, clusters=sizes.size, n_act=idx.size)
    ref = [np.zeros((idx.size, 3)) for _ in range(3)] + [np.zeros(idx.size)]
    S = np.zeros((idx.size, 4))
    cl = np.searchsorted(off, idx, side="right") - 1
    for c in np.unique(cl):
        sel = cl == c
        r = oracle.force(m, x, v, a, EPS, idx[sel], (off[c], off[c + 1]))
        S[sel] = term_sums(m, x, v, a, EPS, idx[sel], (off[c], off[c + 1]))
        for q in range(4):
            ref[q][sel] = r[q]
    s = gpu_system(m, x, v, a, EPS, 0, offsets=off)
    for shape in ((0, 0, 0), (1, 4, 1), (16, 1, 2)):
        s.set_launch(*shape)
        _check(0, force(s, idx), ref, S)


def test_force_validate_rejects_bad_index():
    from paper_1207_2367_amd import NBodyError
    m, x, v, a = plummer_inputs(512, 1)
    s = gpu_system(m, x, v, a, EPS, 0, validate=True)
    s.force([1, 5, 9])
    for bad in ([3, 2], [0, 512], [-1, 4], [4, 4]):
        with pytest.raises(NBodyError) as e:
            s.force(bad)
        assert e.value.code == -1


@pytest.mark.parametrize("prec", PRECS, ids=IDS)
def test_force_full_size_sampled(prec):
    """The N = 65,536 Plummer sphere with every particle active, in the
    launch shapes the benchmark times (the autotuner's choice after the same
    150 ms search, and (1, 4, 16), its usual result) and the heuristic one:
    256 sampled particles against the oracle, one by one, and the third law
    over the whole system."""
    n = 65536
    m, x, v, a = plummer_inputs(n, 2002)
    s = gpu_system(m, x, v, a, EPS, prec)
    idx = np.arange(n)
    sample = ics.active_subset(n, 256, 99)
    ref = oracle.force(m, x, v, a, EPS, sample)
    S = term_sums(m, x, v, a, EPS, sample)
    mm = m[:, None]
    for shape in ((0, 0, 0), (1, 4, 16), "tuned"):
        if shape == "tuned":
            s.set_launch(0, 0, 0)
            s.autotune(150.0)
        else:
            s.set_launch(*shape)
        log_case(test="full_size", prec=prec, n=n, launch=s.get_launch(n))
        got = [cpu(q) for q in force(s, idx)]
        _check(prec, [g[sample] for g in got], ref, S)
        # third law: sum_i m_i a_i = sum_i m_i da_i = 0 (FP64 sums in the
        # mixed and FP64 modes)
        for q in (0, 1):
            scale = np.abs(mm * got[q]).sum()
            assert np.abs((mm * got[q]).sum(0)).max() < (1e-6 if prec == 2 else 1e-13) * scale


@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_force_active_sets_65536(prec):
    """The force microbenchmark's system (Plummer N = 65,536, seed 2002)
    with its active-set sizes N_act = 1, 64, 1024, 8192, 65,536 (seeded
    random subsets, automatic launch shapes): up to 512 active particles
    per set against the oracle one by one.  The mixed mode must meet the
    plain per-particle bound 1e-6 on a, da and the potential (and its
    snap the k S_i bound); the printed lines give the plain max / p99 of
    every quantity."""
    n = 65536
    m, x, v, a = plummer_inputs(n, 2002)
    s = gpu_system(m, x, v, a, EPS, prec)
    for n_act in (1, 64, 1024, 8192, 65536):
        idx = ics.active_subset(n, n_act, 2003)
        pos = np.arange(n_act) if n_act <= 512 else np.sort(
            np.random.default_rng(n_act).choice(n_act, 512, replace=False))
        smp = idx[pos]
        log_case(test="active_sets_65536", prec=prec, n_act=n_act, launch=s.get_launch(n_act))
        ref = oracle.force(m, x, v, a, EPS, smp)
        got = [cpu(q)[pos] for q in force(s, idx)]
        _check(prec, got, ref, term_sums(m, x, v, a, EPS, smp))
