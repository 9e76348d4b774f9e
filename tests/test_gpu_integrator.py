"""GPU parity of the block-time-step machinery through the C ABI against the
FP64 oracle: initialization, predictor (paper Sect. 3 item 1), scheduler
(Table 1 section 1), corrector + interpolation + step criterion (item 3,
Eqs. indtstp/As), whole block steps and whole runs, energy bookkeeping
(Sect. 5.1), determinism, checkpoint/resume and error paths.

Element-wise parts (predictor, corrector, energy) are FP64 on both sides and
must agree to a few units of roundoff.  Integer parts (active sets, block
times) must be identical.  A new block step is a power of two taken from a
floating-point criterion, so where the oracle's criterion lies within the
evaluation's relative error of a power of two either neighbour is correct;
every other step must match exactly.
"""
import math

import numpy as np
import pytest
import torch

import ics
import oracle
from gpu_helpers import abs_err_rows, cpu, log_case, norm_rows, plummer_inputs, term_sums

pytestmark = pytest.mark.gpu

EPS = 1e-4
DMIN, DMAX = 2.0 ** -25, 1.0 / 16


def _system(m, x, v, prec, **kw):
    from paper_1207_2367_amd import System
    return System(m, x, v, EPS, precision=prec, **kw)


def _near_pow2(crit, rel):
    """True where crit lies within relative distance rel of a power of two."""
    crit = np.asarray(crit, dtype=np.float64)
    lo = 2.0 ** np.floor(np.log2(crit))
    return (np.abs(crit / lo - 1) < rel) | (np.abs(crit / (2 * lo) - 1) < rel)


def _random_state(n, seed):
    """Synthetic block-consistent state: dt a power of two, t a multiple."""
    rng = np.random.default_rng(seed)
    m, x, v = ics.plummer(n, seed)
    a, jk, sn, cr = (ics.random_vectors(n, seed + k, s) for k, s in ((1, 1.0), (2, 3.0), (3, 10.0), (4, 30.0)))
    dt = 2.0 ** -rng.integers(4, 12, n).astype(float)
    t = dt * rng.integers(0, 6, n)
    return m, x, v, a, jk, sn, cr, t, dt


# ----------------------------------------------------------------- init
@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_init_parity(prec):
    n = 3000
    m, x, v = ics.plummer(n, 77)
    log_case(test="init", prec=prec, n=n)
    it = oracle.Integrator(m, x, v, EPS)
    assert it.init(math.inf) == 0
    s = _system(m, x, v, prec)
    g = {k: cpu(q) for k, q in s.get_state().items()}
    S = term_sums(m, x, v, it.a, EPS, np.arange(n))
    # the start-up evaluation is FP64 in both precisions: |error| <= 1e-12
    # times the sum of term magnitudes; the crackle (whose sum has one more
    # level of terms) 4e-12 of the snap's condition number, relative
    for key, q in (("a", 0), ("jk", 1), ("sn", 2)):
        e = abs_err_rows(g[key], getattr(it, key))
        assert np.all(e <= 1e-12 * S[:, q]), (key, np.nanmax(e))
    e = abs_err_rows(g["cr"], it.cr) / norm_rows(it.cr)
    assert np.all(e <= 4e-12 * S[:, 2] / norm_rows(it.sn)), np.nanmax(e)
    assert np.array_equal(g["x"], it.x) and np.array_equal(g["v"], it.v)
    assert np.all(g["t"] == 0)
    nrm = lambda q: np.linalg.norm(q, axis=1)
    crit = 0.1 * np.sqrt(nrm(it.a) * nrm(it.sn) + nrm(it.jk) ** 2) / np.sqrt(nrm(it.jk) * nrm(it.cr) + nrm(it.sn) ** 2)
    diff = g["dt"] != it.dt
    assert np.all(_near_pow2(crit[diff], 1e-11)), np.nonzero(diff)[0][:5]
    print(f"init: {diff.sum()} borderline first-step mismatches of {n}")


# ------------------------------------------------------------ predictor
def test_predict_parity():
    n = 4099
    m, x, v, a, jk, sn, cr, t, dt = _random_state(n, 5)
    s = _system(m, x, v, 1)
    s.set_state(x=x, v=v, a=a, jk=jk, sn=sn, cr=cr, t=t, dt=dt)
    T = 0.4375
    ref = oracle.predict(x, v, a, jk, sn, cr, t, T)
    got = [cpu(q) for q in s.predict(T)]
    for gq, rq in zip(got, ref):
        scale = np.abs(rq).max()
        assert np.abs(gq - rq).max() <= 4e-16 * 64 * scale


# ------------------------------------------------------------ scheduler
@pytest.mark.parametrize("clusters", [0, 4, 1300], ids=["one", "four", "many"])
def test_schedule_parity(clusters):
    """Active set and block time against the oracle's schedule, per cluster;
    1300 clusters give more schedule chunks than the scan's 1024 lanes."""
    n = 9001
    m, x, v, a, jk, sn, cr, t, dt = _random_state(n, 9)
    off = None
    if clusters == 4:
        off = [0, 2500, 2501, 7000, n]
    elif clusters:
        cuts = np.sort(np.random.default_rng(1300).choice(np.arange(1, n), clusters - 1, replace=False))
        off = [0] + [int(q) for q in cuts] + [n]
    s = _system(m, x, v, 0, offsets=off)
    s.set_state(t=t, dt=dt)
    for T in (1.0, 0.0625, 2.0 ** -9):
        idx, tn = s.schedule(T)
        idx = cpu(idx)
        ref_idx, ref_t = [], math.inf
        for c0, c1 in (zip(off[:-1], off[1:]) if off else [(0, n)]):
            ri, rt = oracle.schedule(t[c0:c1], dt[c0:c1])
            if rt <= T:
                ref_idx.append(ri + c0)
                ref_t = min(ref_t, rt)
        ref_idx = np.concatenate(ref_idx) if ref_idx else np.zeros(0, dtype=np.int64)
        log_case(test="schedule", clusters=clusters, T=T, n_act=len(ref_idx))
        assert np.array_equal(idx, ref_idx)
        assert tn == ref_t


# ------------------------------------------------------------ corrector
def test_correct_parity():
    n = 3001
    m, x, v, a, jk, sn, cr, t, dt = _random_state(n, 21)
    rng = np.random.default_rng(4)
    idx = np.sort(rng.choice(n, 1200, replace=False))
    # new derivatives close to the Taylor values, as after a real step
    a1 = a[idx] + dt[idx, None] * jk[idx] + ics.random_vectors(idx.size, 8, 1e-3)
    j1 = jk[idx] + dt[idx, None] * sn[idx] + ics.random_vectors(idx.size, 9, 1e-3)
    s1 = sn[idx] + dt[idx, None] * cr[idx] + ics.random_vectors(idx.size, 10, 1e-3)
    T = 1.0
    it = oracle.Integrator(m, x, v, EPS)
    it.set_state(x=x, v=v, a=a, jk=jk, sn=sn, cr=cr, t=t, dt=dt)
    # the oracle's correct takes one block time per call: one call per particle
    for k, i in enumerate(idx):
        e = it.correct([i], t[i] + dt[i], T, a1[k:k + 1], j1[k:k + 1], s1[k:k + 1])
        assert e in (0, oracle.EDTMIN)
    s = _system(m, x, v, 1)
    s.set_state(x=x, v=v, a=a, jk=jk, sn=sn, cr=cr, t=t, dt=dt)
    try:
        s.correct(idx, T, a1, j1, s1)
    except Exception as ex:      # a random state may ask for a step below dt_min
        assert getattr(ex, "code", None) == -4
    g = {k: cpu(q) for k, q in s.get_state().items()}
    for key in ("x", "v", "a", "jk", "sn"):
        np.testing.assert_allclose(g[key], getattr(it, key), rtol=1e-13, atol=1e-13 * np.abs(getattr(it, key)).max())
    # crackle comes from divided differences: relative to |a| / h^3
    sc = np.abs(a1).max() / dt[idx].min() ** 3
    assert np.abs(g["cr"] - it.cr).max() <= 1e-11 * sc
    assert np.array_equal(g["t"], it.t)
    diff = np.nonzero(g["dt"] != it.dt)[0]
    assert diff.size <= 3, diff       # only criterion values on a power-of-two boundary


# ------------------------------------------------------- block steps
@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_block_steps_match_oracle(prec):
    """From the same state, GPU and oracle select the same blocks at the same
    times for the first block steps, and the states stay close."""
    n = 1024
    m, x, v = ics.plummer(n, 1001)
    it = oracle.Integrator(m, x, v, EPS)
    assert it.init(1.0) == 0
    s = _system(m, x, v, prec)
    s.set_state(**{k: getattr(it, k) for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt")})
    log_case(test="block_steps", prec=prec)
    first_diff = None
    for step in range(40):
        err, na, tb = it.block_step(1.0)
        gna, gtb = s.block_step(1.0)
        assert err == 0
        if (gna, gtb) != (na, tb):
            first_diff = step
            break
    g = {k: cpu(q) for k, q in s.get_state().items()}
    print(f"first differing block: {first_diff}; max |dx| {np.abs(g['x'] - it.x).max():.2e}, "
          f"dt mismatches {(g['dt'] != it.dt).sum()}")
    if prec == 1:
        # FP64: identical blocks throughout, states equal to roundoff
        assert first_diff is None
        assert np.array_equal(g["t"], it.t)
        assert np.abs(g["x"] - it.x).max() < 1e-13 and np.abs(g["v"] - it.v).max() < 1e-12
    else:
        # mixed: the first block is fixed by the shared state; afterwards a
        # new step whose criterion sits near a power of two may take the
        # other level (both are correct), and the runs part ways
        assert first_diff is None or first_diff >= 1
        if first_diff is None:
            assert np.array_equal(g["t"], it.t)
            assert np.abs(g["x"] - it.x).max() < 1e-9


@pytest.mark.parametrize("split", [64, 256])
def test_block_steps_many_splits_match_oracle(split):
    """The split sums of the corrector with several lanes per sum (4 lanes
    from 33 splits on, 8 from 129): a pinned launch shape with 64 or 256
    source splits (only the splits that hold sources count, so some lanes
    sum none) keeps the FP64 block steps of the 1024-body sphere equal to
    the oracle's, with states equal to roundoff."""
    n = 1024
    m, x, v = ics.plummer(n, 1001)
    it = oracle.Integrator(m, x, v, EPS)
    assert it.init(1.0) == 0
    s = _system(m, x, v, 1)
    s.set_state(**{k: getattr(it, k) for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt")})
    s.set_launch(lanes_per_i=64, waves=4, split=split)
    log_case(test="block_steps_many_splits", split=split)
    for step in range(40):
        err, na, tb = it.block_step(1.0)
        gna, gtb = s.block_step(1.0)
        assert err == 0
        assert (gna, gtb) == (na, tb), step
    g = {k: cpu(q) for k, q in s.get_state().items()}
    dx = np.abs(g["x"] - it.x).max()
    print(f"split {split}: max |dx| {dx:.2e}")
    assert np.array_equal(g["t"], it.t) and np.array_equal(g["dt"], it.dt)
    assert dx < 1e-13 and np.abs(g["v"] - it.v).max() < 1e-12


def test_plummer_1024_to_t1_energy():
    """The 1024-body Plummer sphere, eps = 1e-4, eta = 0.45, dt_max = 1/16,
    to t = 1: oracle, GPU FP64 and GPU mixed.  Same block structure as the
    oracle at first, close trajectories at t = 1/16, and energy errors of the
    same size (the mixed path within 2x of the FP64 path, plus a floor set by
    the FP32 force error)."""
    n = 1024
    m, x, v = ics.plummer(n, 1001)
    it = oracle.Integrator(m, x, v, EPS)
    it.init(1.0)
    e0 = sum(it.energy()[:2])
    it.run(1.0 / 16)
    x16 = it.x.copy()
    err, steps, pairs, hist = it.run(1.0)
    de_o = (sum(it.energy()[:2]) - e0) / e0
    res = {}
    for prec in (1, 0):
        s = _system(m, x, v, prec)
        g0 = sum(s.energy()[:2])
        assert abs(g0 - e0) < 1e-13 * abs(e0)
        st16 = s.step(1.0 / 16)
        gx16 = cpu(s.get_state()["x"])
        st = s.step(1.0)
        g1 = sum(s.energy()[:2])
        res[prec] = ((g1 - g0) / g0, np.abs(gx16 - x16).max(), st16["block_steps"] + st["block_steps"])
    print(f"dE/E oracle {de_o:.3e} gpu-fp64 {res[1][0]:.3e} gpu-mixed {res[0][0]:.3e}; "
          f"max|dx| at 1/16 fp64 {res[1][1]:.2e} mixed {res[0][1]:.2e}; steps {steps} {res[1][2]} {res[0][2]}")
    assert res[1][1] < 1e-9 and res[0][1] < 1e-6
    assert abs(res[1][0]) < 3 * abs(de_o) + 1e-12
    # "equal energy error": the mixed path within 2x of the FP64 path
    assert abs(res[0][0]) <= 2 * abs(res[1][0])
    # the all-FP32 pair mode also integrates this sphere
    s = _system(m, x, v, 2)
    g0 = sum(s.energy()[:2])
    s.step(1.0)
    de32 = (sum(s.energy()[:2]) - g0) / g0
    print(f"dE/E fp32pair {de32:.3e}")
    assert abs(de32) < 1e-7


@pytest.mark.parametrize("sizes", [[700, 300, 1500, 256], [5077], [4096], [3000, 1, 2100, 2]],
                         ids=["king4", "odd5077", "even4096", "split_clusters"])
def test_energy_parity_and_clusters(sizes):
    """Energy and angular momentum (Sect. 5.1) against the oracle: odd and
    even cluster sizes (the two window rules of the energy pass), clusters
    of one and two bodies, and sizes that split the pass over workgroups."""
    m, x, v, off = ics.king_ensemble(len(sizes), sizes=sizes)
    log_case(test="energy", sizes=sizes)
    for prec in (0, 1):
        s = _system(m, x, v, prec, offsets=off)
        ek, ep, L = s.energy()
        rk, rp, rL = oracle.energy(m, x, v, EPS, off)
        assert abs(ek - rk) < 1e-14 * abs(rk)
        assert abs(ep - rp) < 1e-12 * abs(rp)
        assert np.abs(np.array(L) - rL).max() < 1e-14 * np.abs(rL).max() + 1e-16


def test_clusters_block_steps_match_oracle():
    m, x, v, off = ics.king_ensemble(3, sizes=[400, 256, 900])
    it = oracle.Integrator(m, x, v, EPS, offsets=off)
    assert it.init(0.125) == 0
    s = _system(m, x, v, 1, offsets=off)
    s.set_state(**{k: getattr(it, k) for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt")})
    for step in range(25):
        err, na, tb = it.block_step(0.125)
        gna, gtb = s.block_step(0.125)
        assert err == 0 and (gna, gtb) == (na, tb), (step, na, gna, tb, gtb)
    g = {k: cpu(q) for k, q in s.get_state().items()}
    assert np.abs(g["x"] - it.x).max() < 1e-12


@pytest.mark.parametrize("prec", [0, 1], ids=["mixed", "fp64"])
def test_deterministic_and_resume(prec):
    """Two identical runs give identical bits; running 0 -> T equals running
    0 -> T/2, checkpointing, restoring into a new system and running on."""
    n = 2048
    m, x, v = ics.plummer(n, 31)
    a = _system(m, x, v, prec)
    # T/2 and T are multiples of dt_max, so the target cap never acts
    a.step(0.125)
    sa = {k: cpu(q) for k, q in a.get_state().items()}
    b = _system(m, x, v, prec)
    b.step(0.0625)
    ck = {k: q.clone() for k, q in b.get_state().items()}
    c = _system(m, x, v, prec)
    c.set_state(**ck)
    c.step(0.125)
    sc = {k: cpu(q) for k, q in c.get_state().items()}
    a2 = _system(m, x, v, prec)
    a2.step(0.125)
    s2 = {k: cpu(q) for k, q in a2.get_state().items()}
    for k in sa:
        assert np.array_equal(sa[k], s2[k]), k
        assert np.array_equal(sa[k], sc[k]), k


def test_error_paths():
    from paper_1207_2367_amd import NBodyError
    m, x, v = ics.plummer(256, 3)
    bad = x.copy()
    bad[7, 1] = np.nan
    with pytest.raises(NBodyError) as e:
        _system(m, bad, v, 0)
    assert e.value.code == -3
    s = _system(m, x, v, 0)
    with pytest.raises(NBodyError) as e:
        s.step(1e-9)             # not on the dt_min grid
    assert e.value.code == -1
    s.step(2.0 ** -6)
    with pytest.raises(NBodyError) as e:
        s.step(2.0 ** -7)        # behind the particles
    assert e.value.code == -1
    # a close unsoftened pair with a large minimum step: the criterion asks
    # for less than dt_min
    from paper_1207_2367_amd import System
    xx = np.array([[0.0, 0, 0], [1e-4, 0, 0], [1.0, 0, 0]])
    vv = np.array([[0.0, 0, 0], [0.0, 1.0, 0], [0.0, 0, 0]])
    with pytest.raises(NBodyError) as e:
        System(np.array([0.4, 0.4, 0.2]), xx, vv, 0.0, dt_min=2.0 ** -10)
    assert e.value.code == -4


def test_energy_requires_common_time():
    """The energy sums of Sect. 5.1 are defined at a common time: with the
    particles of a cluster at different times nbody_energy returns ESTATE
    (and computes nothing); clusters may each sit at their own time."""
    from paper_1207_2367_amd import NBodyError
    m, x, v = ics.plummer(512, 5)
    s = _system(m, x, v, 1)
    e0 = s.energy()
    t = np.zeros(512)
    t[100:] = 1.0 / 16
    s.set_state(t=t)
    with pytest.raises(NBodyError) as e:
        s.energy()
    assert e.value.code == -5
    s.set_state(t=np.full(512, 1.0 / 16))
    assert s.energy()[:2] == e0[:2]          # same positions and velocities
    sizes = [200, 312]
    mc, xc, vc, off = ics.king_ensemble(2, sizes=sizes)
    sc = _system(mc, xc, vc, 1, offsets=off)
    tc = np.zeros(512)
    tc[off[1]:] = 1.0 / 16                   # each cluster at one time
    sc.set_state(t=tc)
    sc.energy()
    tc[off[1] + 5] = 0.0
    sc.set_state(t=tc)
    with pytest.raises(NBodyError) as e:
        sc.energy()
    assert e.value.code == -5


def test_correct_rejects_bad_index_lists():
    """nbody_correct with a list index outside [0, n) skips it and returns
    EINVAL (the other particles are corrected); with validate on, a list out
    of range or not ascending is refused before any change."""
    from paper_1207_2367_amd import NBodyError
    n = 600
    m, x, v, a, jk, sn, cr, t, dt = _random_state(n, 23)
    t[:] = 0.0
    dt[:] = 1.0 / 16
    a1, j1, s1 = a[:2] + 1e-3, jk[:2], sn[:2]
    s = _system(m, x, v, 1)
    s.set_state(x=x, v=v, a=a, jk=jk, sn=sn, cr=cr, t=t, dt=dt)
    with pytest.raises(NBodyError) as e:
        s.correct([3, n + 7], 1.0 / 16, a1, j1, s1)
    assert e.value.code == -1
    g = s.get_state()
    assert cpu(g["t"])[3] == 1.0 / 16 and (cpu(g["t"])[4:] == 0).all()
    sv = _system(m, x, v, 1, validate=True)
    sv.set_state(x=x, v=v, a=a, jk=jk, sn=sn, cr=cr, t=t, dt=dt)
    for bad in ([5, 3], [3, n], [-1, 3], [4, 4]):
        with pytest.raises(NBodyError) as e:
            sv.correct(bad, 1.0 / 16, a1, j1, s1)
        assert e.value.code == -1
    assert (cpu(sv.get_state()["t"]) == 0).all()
