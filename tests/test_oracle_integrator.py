"""Pins of the oracle's predictor, corrector, derivative interpolation,
time-step criterion, block rules, scheduler and whole integration (paper
Sect. 3 items 1 and 3, Eqs. indtstp/As, Sect. 5.1) against polynomial
exactness, closed forms, invariants and the convergence order of the
scheme on the Kepler problem."""
import math

import numpy as np
import numpy.polynomial.polynomial as P
import pytest

import ics
import oracle


def _poly_traj(deg, seed, scale=1.0):
    """Random polynomial trajectory r(t) (3 components), coefficient arrays."""
    rng = np.random.default_rng(seed)
    return [rng.normal(0, scale, deg + 1) for _ in range(3)]


def _deriv(cs, k, t):
    return np.array([P.polyval(t, P.polyder(c, k)) if k else P.polyval(t, c) for c in cs])


# ------------------------------------------------------------ predictor
def test_predictor_exact_for_quintic_trajectories():
    """Given the exact derivatives at t_i, the Taylor predictor reproduces
    position, velocity and acceleration of a quintic r(t) at any later T."""
    n = 6
    trajs = [_poly_traj(5, 100 + k) for k in range(n)]
    t = np.array([0.0, 0.125, 0.25, 0.5, 0.0625, 0.375])
    T = 0.75
    st = [np.array([_deriv(trajs[k], d, t[k]) for k in range(n)]) for d in range(6)]
    xp, vp, ap = oracle.predict(*st, t, T)
    for k in range(n):
        np.testing.assert_allclose(xp[k], _deriv(trajs[k], 0, T), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(vp[k], _deriv(trajs[k], 1, T), rtol=1e-13, atol=1e-13)
        np.testing.assert_allclose(ap[k], _deriv(trajs[k], 2, T), rtol=1e-13, atol=1e-13)


def test_predictor_identity_at_own_time():
    m, x, v = ics.plummer(50, 3)
    rnd = [ics.random_vectors(50, s) for s in range(4)]
    t = np.full(50, 0.25)
    xp, vp, ap = oracle.predict(x, v, *rnd, t, 0.25)
    assert np.array_equal(xp, x) and np.array_equal(vp, v) and np.array_equal(ap, rnd[0])


# ------------------------------------------------------- interpolation
def test_interpolation_recovers_quintic_derivatives():
    """For a quintic a(t) the derivatives of the end-point interpolant are
    the exact 3rd, 4th and 5th derivatives at the end of the step."""
    for seed in range(5):
        cs = _poly_traj(5, seed)   # a(t) itself
        t0, h = 0.3, 2.0 ** -(seed + 2)
        a0, j0, s0 = (_deriv(cs, k, t0) for k in range(3))
        a1, j1, s1 = (_deriv(cs, k, t0 + h) for k in range(3))
        crk, pop, a5 = oracle.interpolate(h, a0, j0, s0, a1, j1, s1)
        ex = [_deriv(cs, k, t0 + h) for k in (3, 4, 5)]
        # the end-point differences D0, D1, D2 cancel to O(h^3), O(h^2), O(h)
        # of |a|, so the k-th derivative carries ~ eps_mach |a| / h^(k)
        sa = np.abs(a0).max() + np.abs(a1).max()
        u = 2.0 ** -52
        assert np.abs(crk - ex[0]).max() < 200 * u * sa / h ** 3
        assert np.abs(pop - ex[1]).max() < 2000 * u * sa / h ** 4
        assert np.abs(a5 - ex[2]).max() < 5000 * u * sa / h ** 5


def test_interpolation_error_order_for_degree_six():
    """For a(t) = t^6 the fifth-derivative estimate is off by O(h) and the
    crackle by O(h^3): halving h halves and divides by 8 the errors."""
    def err(h):
        t0 = 0.0
        cs = [np.array([0, 0, 0, 0, 0, 0, 1.0])] * 3
        a0, j0, s0 = (_deriv(cs, k, t0) for k in range(3))
        a1, j1, s1 = (_deriv(cs, k, t0 + h) for k in range(3))
        crk, pop, a5 = oracle.interpolate(h, a0, j0, s0, a1, j1, s1)
        return abs(a5[0] - 720 * h), abs(crk[0] - 120 * h ** 3)
    e1, e2 = err(0.1), err(0.05)
    assert 1.9 < e1[0] / e2[0] < 2.1
    assert 7.5 < e1[1] / e2[1] < 8.5


# ------------------------------------------------------------ corrector
def _corrector_case(deg, h, seed):
    cs = _poly_traj(deg, seed)
    t0 = 0.25
    st = oracle.Integrator(np.ones(1), _deriv(cs, 0, t0)[None], _deriv(cs, 1, t0)[None], 0.0,
                           dt_min=2.0 ** -40, dt_max=1.0)
    st.set_state(a=_deriv(cs, 2, t0)[None], jk=_deriv(cs, 3, t0)[None],
                 sn=_deriv(cs, 4, t0)[None], t=[t0], dt=[h])
    a1, j1, s1 = (_deriv(cs, k, t0 + h)[None] for k in (2, 3, 4))
    err = st.correct([0], t0 + h, 10.0, a1, j1, s1)
    return cs, t0, st, err


def test_corrector_exact_for_degree_six_trajectories():
    """The Hermite corrector integrates a quartic acceleration exactly: for a
    degree-6 r(t) both the corrected velocity and position are exact."""
    for seed in range(4):
        h = 2.0 ** -3
        cs, t0, st, err = _corrector_case(6, h, seed)
        assert err == oracle.OK
        np.testing.assert_allclose(st.v[0], _deriv(cs, 1, t0 + h), rtol=1e-14, atol=1e-14)
        np.testing.assert_allclose(st.x[0], _deriv(cs, 0, t0 + h), rtol=1e-14, atol=1e-14)
        assert st.t[0] == t0 + h


def test_corrector_velocity_exact_for_quintic_acceleration():
    """For a degree-7 r(t) (quintic a) the velocity is still exact; the
    position is not, and its error scales as h^7."""
    for seed in range(3):
        h = 2.0 ** -3
        cs, t0, st, _ = _corrector_case(7, h, seed)
        np.testing.assert_allclose(st.v[0], _deriv(cs, 1, t0 + h), rtol=1e-14, atol=1e-14)
    errs = []
    for h in (2.0 ** -2, 2.0 ** -3):
        cs, t0, st, _ = _corrector_case(7, h, 7)
        errs.append(np.abs(st.x[0] - _deriv(cs, 0, t0 + h)).max())
    assert errs[1] > 0 and 100 < errs[0] / errs[1] < 160   # 2^7 = 128


# ------------------------------------------------------- step criterion
def test_dt_criterion_circular_orbit_closed_form():
    """On a circular orbit |a^(k)| = w^k |a|, so A(1) = sqrt(2) w |a|,
    A(4) = sqrt(2) w^4 |a| and the criterion gives eta / w."""
    w, R, eta = 1.7, 0.6, 0.45
    th = 0.3
    # successive derivatives of x(t) = R (cos wt, sin wt, 0)
    d = [R * w ** k * np.array([math.cos(th + k * math.pi / 2), math.sin(th + k * math.pi / 2), 0.0])
         for k in range(8)]
    dt = oracle.dt_criterion(d[2], d[3], d[4], d[5], d[6], d[7], eta)
    assert abs(dt - eta / w) < 1e-14


def test_dt_criterion_hand_values():
    e = np.array([1.0, 0.0, 0.0])
    z = np.zeros(3)
    # A1 = sqrt(1*1 + 0) = 1, A4 = sqrt(8*1 + 0) = sqrt 8 -> eta * 8^(-1/6)
    assert abs(oracle.dt_criterion(e, z, e, 8 * e, z, e, 0.5) - 0.5 * 8 ** (-1 / 6)) < 1e-15
    # A1 = sqrt(0 + 4) = 2, A4 = sqrt(0 + 1/4) = 1/2 -> eta * 4^(1/3)
    assert abs(oracle.dt_criterion(e, 2 * e, z, z, 0.5 * e, z, 0.3) - 0.3 * 4 ** (1 / 3)) < 1e-15
    assert oracle.dt_criterion(e, e, e, z, z, z, 0.3) == math.inf


# --------------------------------------------------------- block rules
DMIN, DMAX = 2.0 ** -25, 1.0 / 16


def test_block_rules_hand_cases():
    bd = oracle.block_dt
    assert bd(0.3, 0.0, 0.0, 1.0, DMIN, DMAX) == (0, DMAX)          # clamp high
    assert bd(0.01, 0.0, 0.0, 1.0, DMIN, DMAX) == (0, 2.0 ** -7)    # round down
    assert bd(2.0 ** -7, 0.0, 0.0, 1.0, DMIN, DMAX) == (0, 2.0 ** -7)  # exact power
    # growth: at most doubling and only at even multiples of the old step
    assert bd(1.0, 2.0 ** -8, 2.0 ** -6, 1.0, DMIN, DMAX) == (0, 2.0 ** -7)
    assert bd(1.0, 2.0 ** -8, 3 * 2.0 ** -8, 1.0, DMIN, DMAX) == (0, 2.0 ** -8)
    # shrink always allowed
    assert bd(1e-4, 2.0 ** -4, 2.0 ** -4, 1.0, DMIN, DMAX) == (0, 2.0 ** -14)
    # target cap
    assert bd(1.0, 2.0 ** -4, 0.0, 1.0 / 64, DMIN, DMAX) == (0, 1.0 / 64)
    assert bd(1.0, 2.0 ** -6, 1.0 / 64, 1.0 / 64 + 2.0 ** -9, DMIN, DMAX) == (0, 2.0 ** -9)
    # below the minimum step -> error
    assert bd(1e-9, 2.0 ** -4, 0.0, 1.0, DMIN, DMAX)[0] == oracle.EDTMIN
    assert bd(float("nan"), 2.0 ** -4, 0.0, 1.0, DMIN, DMAX)[0] == oracle.ENONFINITE


def test_block_rule_invariants_random():
    rng = np.random.default_rng(0)
    for _ in range(3000):
        lo = int(rng.integers(3, 20))
        dt_old = 2.0 ** -lo
        t_new = dt_old * int(rng.integers(1, 64))
        crit = 10 ** rng.uniform(-7, 0)
        t_target = t_new + 2.0 ** -int(rng.integers(0, 25)) * int(rng.integers(1, 4))
        err, dt = oracle.block_dt(crit, dt_old, t_new, t_target, DMIN, DMAX)
        if err:
            continue
        e = math.frexp(dt)
        assert e[0] == 0.5                       # power of two
        assert DMIN <= dt <= DMAX
        assert dt <= 2 * dt_old
        assert dt <= crit or dt == DMIN
        assert math.fmod(t_new, dt) == 0.0       # commensurate
        assert t_new + dt <= t_target


def test_schedule_matches_brute_force():
    rng = np.random.default_rng(3)
    n = 2000
    dt = 2.0 ** -rng.integers(2, 12, n).astype(float)
    t = dt * rng.integers(0, 8, n)
    idx, tn = oracle.schedule(t, dt)
    assert tn == (t + dt).min()
    assert np.array_equal(idx, np.nonzero(t + dt == tn)[0])


# ---------------------------------------------------------- integration
def _kepler_state(e, a_sm=None):
    """Two bodies, pericentre start, period 1 (a^3 = M / (4 pi^2))."""
    m = np.array([0.4, 0.6])
    M = m.sum()
    a_sm = (M / (4 * math.pi ** 2)) ** (1 / 3)
    rp = a_sm * (1 - e)
    vp = math.sqrt(M * (1 + e) / rp)
    rel_x, rel_v = np.array([rp, 0, 0]), np.array([0, vp, 0])
    x = np.array([-(m[1] / M) * rel_x, (m[0] / M) * rel_x])
    v = np.array([-(m[1] / M) * rel_v, (m[0] / M) * rel_v])
    return m, x, v


def test_kepler_sixth_order_convergence():
    """Shared fixed steps (dt_min = dt_max = h) over one Kepler period of an
    e = 0.5 orbit: the position error against the exact periodic solution
    falls as h^6."""
    errs = []
    hs = [2.0 ** -k for k in (7, 8, 9)]
    for h in hs:
        m, x0, v0 = _kepler_state(0.5)
        # a large eta keeps the criterion above h, so every step is h
        it = oracle.Integrator(m, x0, v0, 0.0, eta=2.0, eta_init=1.0, dt_min=h, dt_max=h)
        assert it.init(1.0) == 0
        err, steps, _, _ = it.run(1.0)
        assert err == 0 and steps == round(1 / h)
        errs.append(np.abs(it.x - x0).max())
    s1 = math.log2(errs[0] / errs[1])
    s2 = math.log2(errs[1] / errs[2])
    assert 5.5 < s1 < 6.6 and 5.5 < s2 < 6.6, (errs, s1, s2)


def test_block_steps_plummer_conserve_energy_and_momentum():
    """Block-step run of a small Plummer sphere: the block invariants hold
    after every step; energy, momentum and angular momentum are conserved to
    the scheme's accuracy."""
    m, x, v = ics.plummer(256, 17)
    it = oracle.Integrator(m, x, v, 1e-4, eta=0.45)
    T = 0.125
    assert it.init(T) == 0
    e0 = sum(it.energy()[:2])
    p0 = (m[:, None] * it.v).sum(0)
    L0 = it.energy()[2]
    last = 0.0
    nsteps = 0
    while (it.t < T).any():
        err, na, tb = it.block_step(T)
        assert err == 0 and na > 0
        assert tb >= last
        last = tb
        nsteps += 1
        assert np.all(np.fmod(it.t, it.dt) == 0)
        assert np.all((it.dt >= DMIN) & (it.dt <= DMAX))
        assert np.all((it.t + it.dt <= T) | (it.t == T))
    assert np.all(it.t == T)
    e1 = sum(it.energy()[:2])
    assert abs((e1 - e0) / e0) < 1e-8, (e1 - e0) / e0
    # individual steps apply the two halves of a pair interaction at
    # different times, so momentum and L drift at the integration-error level
    assert np.abs((m[:, None] * it.v).sum(0) - p0).max() < 1e-8
    assert np.abs(it.energy()[2] - L0).max() < 1e-8
    assert nsteps > 8


def test_clusters_are_independent():
    """Two clusters integrated together give exactly what each gives alone."""
    m1, x1, v1 = ics.plummer(64, 1)
    m2, x2, v2 = ics.plummer(96, 2)
    off = [0, 64, 160]
    both = oracle.Integrator(np.concatenate([m1, m2]), np.concatenate([x1, x2]),
                             np.concatenate([v1, v2]), 1e-4, offsets=off)
    assert both.init(0.0625) == 0
    assert both.run(0.0625)[0] == 0
    for (m, x, v), sl in (((m1, x1, v1), slice(0, 64)), ((m2, x2, v2), slice(64, 160))):
        one = oracle.Integrator(m, x, v, 1e-4)
        assert one.init(0.0625) == 0
        assert one.run(0.0625)[0] == 0
        assert np.array_equal(one.x, both.x[sl]) and np.array_equal(one.v, both.v[sl])
        assert np.array_equal(one.dt, both.dt[sl])


def test_run_counters_hand_case():
    """orc_run's block-step count, interaction count (N_c times N_act per
    cluster and step) and log2 N_act histogram against a hand count.  Two
    clusters (5 and 3 bodies) whose criterion, with eta = 1000, is far above
    dt_max = 2^-10 = d, so every particle takes the largest step that the
    block rules allow.  Cluster 0 starts with step d and keeps it (blocks of
    5 at d, 2d, 3d, 4d).  In cluster 1 two bodies start with d/4 and one
    with d; a step may only double where the new time is a multiple of
    twice the old step, so its blocks are d/4 (2 active), d/2 (2), then d,
    2d, 3d, 4d (3 each).  Every block step takes one block of each cluster
    still short of the target 4d: 6 block steps, 4 * 5 * 5 + 2 * 3 * 2 +
    4 * 3 * 3 = 148 interactions, blocks of 5 in bin 2 (4) and of 2 and 3
    in bin 1 (6); the block times of the whole system (min over the
    clusters) are d/4, d/2, d, 2d, 3d, 4d with 7, 7, 8, 8, 3, 3 active.
    A second run to 4.5 d must first halve every step (the target cap):
    one block step of all 8 bodies, 25 + 9 interactions."""
    d = 2.0 ** -10
    m0, x0, v0 = ics.plummer(5, 31)
    m1, x1, v1 = ics.plummer(3, 32)
    m = np.concatenate([m0 / 2, m1 / 2])
    x = np.concatenate([x0, x1 + 10.0])
    v = np.concatenate([v0, v1])
    off = [0, 5, 8]

    def fresh():
        it = oracle.Integrator(m, x, v, 1e-4, eta=1000.0, dt_max=d, offsets=off)
        assert it.init(4 * d) == oracle.OK
        it.set_state(dt=np.array([d] * 5 + [d / 4, d, d / 4]), t=np.zeros(8))
        return it

    it = fresh()
    err, steps, pairs, hist = it.run(4 * d)
    assert err == oracle.OK
    assert np.all(it.t == 4 * d) and np.all(it.dt == d)
    assert steps == 6
    assert pairs == 4 * 25 + 2 * 6 + 4 * 9 == 148
    want = np.zeros(64, dtype=np.int64)
    want[2], want[1] = 4, 6
    assert np.array_equal(hist, want)
    err, steps, pairs, hist = it.run(4.5 * d)
    assert err == oracle.OK and np.all(it.t == 4.5 * d) and np.all(it.dt == d / 2)
    assert (steps, pairs) == (1, 34)
    want = np.zeros(64, dtype=np.int64)
    want[2], want[1] = 1, 1
    assert np.array_equal(hist, want)

    it = fresh()
    seq = [it.block_step(4 * d) for _ in range(6)]
    assert [s[0] for s in seq] == [oracle.OK] * 6
    assert [s[1] for s in seq] == [7, 7, 8, 8, 3, 3]
    assert [s[2] for s in seq] == [d / 4, d / 2, d, 2 * d, 3 * d, 4 * d]
    assert it.block_step(4 * d)[1] == 0
