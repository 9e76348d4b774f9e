"""Pins of the oracle's direct-summation evaluation (paper Sect. 3, item 2,
with the softened potential of Sect. 2) against facts that do not come from
the oracle itself: Kepler kinematics, derivatives of the softened potential
taken numerically in high precision, Newton's third law, symmetry
invariances and closed-form potentials."""
import math

import mpmath as mp
import numpy as np
import pytest

import ics
import oracle


def _rel(a, b):
    return np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b)


# --------------------------------------------------------------- Kepler
def _kepler_orbit(m1, m2, a_sm, e, t):
    """Exact two-body relative orbit at time t (pericentre at t = 0) by
    Kepler's equation solved to 50 digits.  Returns body 1's position."""
    M = m1 + m2
    n = mp.sqrt(M / a_sm ** 3)
    Mean = n * t
    E = mp.findroot(lambda E: E - e * mp.sin(E) - Mean, Mean)
    xr = a_sm * (mp.cos(E) - e)
    yr = a_sm * mp.sqrt(1 - e * e) * mp.sin(E)
    # body 1 sits at -(m2/M) r_rel in the centre-of-mass frame
    return [-(m2 / M) * xr, -(m2 / M) * yr, mp.mpf(0)]


def _kepler_derivs(m1, m2, a_sm, e, t0, k):
    return [mp.diff(lambda t: _kepler_orbit(m1, m2, a_sm, e, t)[d], t0, k) for d in range(2)] + [0]


@pytest.mark.parametrize("e,phase", [(0.0, 0.3), (0.5, 0.1), (0.5, 1.7), (0.9, 0.05)])
def test_kepler_two_body_derivatives(e, phase):
    """With eps = 0, a, da, d2a of body 1 are the 2nd, 3rd and 4th time
    derivatives of its Kepler orbit (derived from Kepler's equation, not
    from the force law)."""
    mp.mp.dps = 40
    m1, m2, a_sm = mp.mpf("0.3"), mp.mpf("0.7"), mp.mpf("1.3")
    M = m1 + m2
    t0 = mp.mpf(phase)
    d = [[float(q) for q in _kepler_derivs(m1, m2, a_sm, e, t0, k)] for k in range(5)]
    # body 2 = -(m1/m2) * body 1 in the COM frame
    s = -float(m1 / m2)
    pos = np.array([d[0], [s * q for q in d[0]]])
    vel = np.array([d[1], [s * q for q in d[1]]])
    acc = np.array([d[2], [s * q for q in d[2]]])
    mass = np.array([float(m1), float(m2)])
    a, j, sn, pot = oracle.force(mass, pos, vel, acc, 0.0)
    assert _rel(a[0], d[2]) < 1e-13
    assert _rel(j[0], d[3]) < 1e-12
    assert _rel(sn[0], d[4]) < 1e-11
    r = np.linalg.norm(pos[1] - pos[0])
    assert abs(pot[0] + float(m2) / r) < 1e-14 * float(m2) / r


def test_circular_binary_closed_form():
    """Uniform circular motion: a = -w^2 x, da = -w^2 v, d2a = w^4 x with
    w^2 = M / R^3 (Kepler's third law); potential -m2 / R."""
    m1, m2, R = 0.25, 0.75, 0.8
    M = m1 + m2
    w = math.sqrt(M / R ** 3)
    th = 0.7
    u = np.array([math.cos(th), math.sin(th), 0.0])
    ut = np.array([-math.sin(th), math.cos(th), 0.0])
    x1, x2 = -(m2 / M) * R * u, (m1 / M) * R * u
    v1, v2 = -(m2 / M) * R * w * ut, (m1 / M) * R * w * ut
    pos, vel = np.array([x1, x2]), np.array([v1, v2])
    acc = -w * w * pos
    a, j, s, pot = oracle.force(np.array([m1, m2]), pos, vel, acc, 0.0)
    np.testing.assert_allclose(a, -w ** 2 * pos, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(j, -w ** 2 * vel, rtol=1e-14, atol=1e-15)
    np.testing.assert_allclose(s, w ** 4 * pos, rtol=1e-13, atol=1e-14)
    np.testing.assert_allclose(pot, [-m2 / R, -m1 / R], rtol=1e-15)


# ------------------------------------------------- softened derivatives
def test_softened_terms_are_time_derivatives_of_the_potential_gradient():
    """With eps > 0, the acceleration is minus the gradient of the softened
    potential (paper Eq. softpot), and the jerk and snap are its first and
    second time derivatives along trajectories r_k(t) = x_k + v_k t + a_k t^2/2.
    All derivatives are taken numerically by mpmath at 40 digits from the
    potential alone."""
    mp.mp.dps = 40
    rng = np.random.default_rng(11)
    n = 5
    x = rng.normal(0, 0.3, (n, 3))
    v = rng.normal(0, 0.5, (n, 3))
    a = rng.normal(0, 0.8, (n, 3))
    m = rng.uniform(0.1, 1.0, n)
    eps = 0.05
    acc, jrk, snp, pot = oracle.force(m, x, v, a, eps)
    X = [[mp.mpf(q) for q in row] for row in x]
    V = [[mp.mpf(q) for q in row] for row in v]
    A = [[mp.mpf(q) for q in row] for row in a]
    for i in (0, 3):
        def phi(dx, dy, dz, t):
            tot = mp.mpf(0)
            ri = [X[i][d] + V[i][d] * t + A[i][d] * t * t / 2 + (dx, dy, dz)[d] for d in range(3)]
            for j in range(n):
                if j == i:
                    continue
                rj = [X[j][d] + V[j][d] * t + A[j][d] * t * t / 2 for d in range(3)]
                s2 = sum((rj[d] - ri[d]) ** 2 for d in range(3)) + mp.mpf(eps) ** 2
                tot -= mp.mpf(m[j]) / mp.sqrt(s2)
            return tot
        assert abs(float(phi(0, 0, 0, 0)) - pot[i]) < 1e-14 * abs(pot[i])
        for d in range(3):
            order = [0, 0, 0, 0]
            order[d] = 1
            for k, got in enumerate((acc, jrk, snp)):
                order[3] = k
                ref = -mp.diff(phi, (0, 0, 0, 0), tuple(order))
                assert abs(got[i, d] - float(ref)) < 1e-12 * (1 + abs(float(ref))), (i, d, k)


def test_crackle_is_third_time_derivative_of_the_potential_gradient():
    """The start-up evaluation's crackle (and its a, da, d2a) equal minus the
    gradient of the softened potential and its first three time derivatives
    along cubic trajectories r_k(t) = x + v t + a t^2/2 + j t^3/6, taken
    numerically by mpmath from the potential alone."""
    mp.mp.dps = 40
    rng = np.random.default_rng(23)
    n = 4
    x = rng.normal(0, 0.3, (n, 3))
    v = rng.normal(0, 0.5, (n, 3))
    a = rng.normal(0, 0.8, (n, 3))
    jk = rng.normal(0, 1.5, (n, 3))
    m = rng.uniform(0.1, 1.0, n)
    eps = 0.05
    acc, jrk, snp, crk = oracle.force4(m, x, v, a, jk, eps)
    ref3 = oracle.force(m, x, v, a, eps)
    for got, ref in zip((acc, jrk, snp), ref3[:3]):
        np.testing.assert_allclose(got, ref, rtol=1e-13, atol=1e-13)
    X, V, A, Jk = ([[mp.mpf(q) for q in row] for row in arr] for arr in (x, v, a, jk))
    for i in (1, 2):
        def phi(dx, dy, dz, t):
            tot = mp.mpf(0)
            def traj(k, d):
                return X[k][d] + V[k][d] * t + A[k][d] * t ** 2 / 2 + Jk[k][d] * t ** 3 / 6
            ri = [traj(i, d) + (dx, dy, dz)[d] for d in range(3)]
            for j in range(n):
                if j == i:
                    continue
                s2 = sum((traj(j, d) - ri[d]) ** 2 for d in range(3)) + mp.mpf(eps) ** 2
                tot -= mp.mpf(m[j]) / mp.sqrt(s2)
            return tot
        for d in range(3):
            order = [0, 0, 0, 3]
            order[d] = 1
            ref = -mp.diff(phi, (0, 0, 0, 0), tuple(order))
            assert abs(crk[i, d] - float(ref)) < 1e-11 * (1 + abs(float(ref))), (i, d)


def test_circular_binary_crackle_and_first_step():
    """Circular binary: crackle = w^4 v (kinematics), and the start-up step
    criterion with p = 4 gives eta_init A(1)/A(2) = eta_init / w, rounded
    down to a power of two."""
    m1, m2, R = 0.3, 0.7, 0.5
    M = m1 + m2
    w = math.sqrt(M / R ** 3)
    u, ut = np.array([1.0, 0, 0]), np.array([0, 1.0, 0])
    x = np.array([-(m2 / M) * R * u, (m1 / M) * R * u])
    v = np.array([-(m2 / M) * R * w * ut, (m1 / M) * R * w * ut])
    acc, jrk, snp, crk = oracle.force4(np.array([m1, m2]), x, v, -w * w * x, -w * w * v, 0.0)
    np.testing.assert_allclose(crk, w ** 4 * v, rtol=1e-13, atol=1e-13 * w ** 4 * R)
    it = oracle.Integrator(np.array([m1, m2]), x, v, 0.0, eta_init=0.2, dt_min=2.0 ** -30, dt_max=1.0)
    assert it.init(math.inf) == 0
    np.testing.assert_allclose(it.cr, w ** 4 * v, rtol=1e-12, atol=1e-12 * w ** 4 * R)
    want = 2.0 ** math.floor(math.log2(0.2 / w))
    assert np.all(it.dt == want)


# ---------------------------------------------------------- invariants
def _plummer_inputs(n, seed):
    m, x, v = ics.plummer(n, seed)
    return m, x, v, ics.plummer_mean_acc(x)


def _pair_scale(m, x, v, a, eps):
    """sum_i m_i sum_j |pair term| bounds, by brute force in numpy, for the
    tolerance of the third-law sums."""
    r = x[None, :, :] - x[:, None, :]
    s2 = (r * r).sum(-1) + eps * eps
    np.fill_diagonal(s2, np.inf)
    w = m[None, :] / s2 ** 1.5
    sa = (m[:, None] * w * np.sqrt((r * r).sum(-1))).sum()
    dv = np.linalg.norm(v[None] - v[:, None], axis=-1)
    da = np.linalg.norm(a[None] - a[:, None], axis=-1)
    sj = (m[:, None] * w * (dv + 3 * np.sqrt((r * r).sum(-1)) * dv / np.sqrt(s2))).sum()
    ss = (m[:, None] * w * (da + 10 * dv * dv / np.sqrt(s2) + 10 * np.sqrt((r * r).sum(-1)) * da / np.sqrt(s2))).sum()
    return sa, sj, ss


def test_newtons_third_law():
    """With every particle active the mass-weighted sums of a, da, d2a vanish
    (each pair term is antisymmetric after weighting by mass)."""
    m, x, v, a = _plummer_inputs(600, 5)
    m = m * np.random.default_rng(1).uniform(0.5, 1.5, m.size)
    eps = 1e-4
    acc, jrk, snp, _ = oracle.force(m, x, v, a, eps)
    sa, sj, ss = _pair_scale(m, x, v, a, eps)
    assert np.abs((m[:, None] * acc).sum(0)).max() < 1e-14 * sa
    assert np.abs((m[:, None] * jrk).sum(0)).max() < 1e-14 * sj
    assert np.abs((m[:, None] * snp).sum(0)).max() < 1e-14 * ss


def test_translation_galilean_and_rotation_invariance():
    m, x, v, a = _plummer_inputs(300, 6)
    eps = 1e-4
    idx = ics.active_subset(300, 40, 9)
    ref = oracle.force(m, x, v, a, eps, idx)
    # shifted origin, moving frame, uniformly accelerated frame
    sh = oracle.force(m, x + [0.25, -0.5, 0.125], v + [0.3, 0.1, -0.2], a + [1.0, -2.0, 0.5], eps, idx)
    for q, r in zip(sh, ref):
        np.testing.assert_allclose(q, r, rtol=1e-9, atol=1e-9 * np.abs(r).max())
    # rotation: vectors rotate, potential unchanged
    th = 0.9
    Rz = np.array([[math.cos(th), -math.sin(th), 0], [math.sin(th), math.cos(th), 0], [0, 0, 1]])
    Rx = np.array([[1, 0, 0], [0, math.cos(0.4), -math.sin(0.4)], [0, math.sin(0.4), math.cos(0.4)]])
    Q = Rz @ Rx
    ro = oracle.force(m, x @ Q.T, v @ Q.T, a @ Q.T, eps, idx)
    for q, r in zip(ro[:3], ref[:3]):
        np.testing.assert_allclose(q, r @ Q.T, rtol=1e-9, atol=1e-10 * np.abs(r).max())
    np.testing.assert_allclose(ro[3], ref[3], rtol=1e-12)
    # linearity in the source masses
    k2 = oracle.force(2.5 * m, x, v, a, eps, idx)
    for q, r in zip(k2, ref):
        np.testing.assert_allclose(q, 2.5 * r, rtol=1e-13, atol=1e-14 * np.abs(r).max())


def test_ring_potential_closed_form():
    """A particle at the centre of a ring of K equal masses feels no force and
    the potential -K m / sqrt(R^2 + eps^2)."""
    K, R, mm, eps = 12, 0.7, 0.05, 0.01
    th = 2 * np.pi * np.arange(K) / K
    x = np.concatenate([[[0, 0, 0]], np.stack([R * np.cos(th), R * np.sin(th), 0 * th], 1)])
    m = np.concatenate([[1.0], np.full(K, mm)])
    z = np.zeros_like(x)
    acc, jrk, snp, pot = oracle.force(m, x, z, z, eps, [0])
    assert abs(pot[0] + K * mm / math.sqrt(R * R + eps * eps)) < 1e-15
    assert np.abs(acc).max() < 1e-15


def test_self_term_excluded_by_index():
    """eps > 0: a distinct particle at the same position adds -m/eps to the
    potential and nothing to a, da, d2a; the particle itself adds nothing.
    eps = 0 with all particles apart stays finite."""
    eps = 1e-3
    x = np.array([[0.1, 0.2, 0.3], [0.1, 0.2, 0.3], [1.0, 0.0, 0.0]])
    v = np.array([[0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [0.0, 1.0, 0.0]])
    m = np.array([0.5, 0.25, 0.25])
    acc, jrk, snp, pot = oracle.force(m, x, v, np.zeros_like(x), eps, [0])
    d = x[2] - x[0]
    s = math.sqrt(d @ d + eps * eps)
    assert abs(pot[0] - (-0.25 / eps - 0.25 / s)) < 1e-12
    np.testing.assert_allclose(acc[0], 0.25 * d / s ** 3, rtol=1e-14)
    m0, x0, v0, a0 = _plummer_inputs(64, 3)
    out = oracle.force(m0, x0, v0, a0, 0.0)
    assert all(np.isfinite(q).all() for q in out)


def test_potential_two_ways():
    """The pairwise potential energy equals half the mass-weighted sum of the
    per-particle potentials that the evaluation returns."""
    m, x, v, a = _plummer_inputs(700, 8)
    eps = 1e-4
    _, _, _, pot = oracle.force(m, x, v, a, eps)
    ek, ep, _ = oracle.energy(m, x, v, eps)
    assert abs(0.5 * (m * pot).sum() - ep) < 1e-13 * abs(ep)
    assert abs(ek - 0.5 * (m * (v * v).sum(1)).sum()) < 1e-15


def test_source_range_restricts_sum():
    """Splitting the sources into two ranges and adding gives the full sum
    (the split-source decomposition of paper Sect. 3)."""
    m, x, v, a = _plummer_inputs(400, 12)
    idx = ics.active_subset(400, 30, 2)
    full = oracle.force(m, x, v, a, 1e-4, idx)
    lo = oracle.force(m, x, v, a, 1e-4, idx, (0, 170))
    hi = oracle.force(m, x, v, a, 1e-4, idx, (170, 400))
    for f, p, q in zip(full, lo, hi):
        np.testing.assert_allclose(p + q, f, rtol=1e-12, atol=1e-13 * np.abs(f).max())
