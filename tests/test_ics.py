"""Checks of the seeded input generators (they are inputs, not parity
subjects): Plummer and King models in Henon units, the Kroupa-like mass
spectrum, the ensemble sizes and active subsets."""
import math

import numpy as np
from scipy import stats

import ics
import oracle


def test_plummer_henon_units_and_profile():
    m, x, v = ics.plummer(4096, 1001)
    assert abs(m.sum() - 1) < 1e-14
    assert np.abs((m[:, None] * x).sum(0)).max() < 1e-14
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-14
    ek, ep, _ = oracle.energy(m, x, v, 1e-4)
    assert abs(ek + ep + 0.25) < 0.02          # E = -1/4 up to O(N^-1/2) scatter
    assert abs(ek / -ep - 0.5) < 0.03          # virial equilibrium
    r = np.linalg.norm(x, axis=1)
    b = ics.PLUMMER_B
    cdf = lambda rr: rr ** 3 / (rr * rr + b * b) ** 1.5 / 0.999
    assert stats.kstest(r, cdf).pvalue > 1e-3


def test_plummer_is_seeded():
    a = ics.plummer(100, 5)
    b = ics.plummer(100, 5)
    c = ics.plummer(100, 6)
    assert all(np.array_equal(p, q) for p, q in zip(a, b))
    assert not np.array_equal(a[1], c[1])


def test_plummer_black_hole():
    """Particle 0 is the hole (mass m_bh, at the centre of mass, at rest in
    that frame); the stars are the star-only model's, with the remaining
    mass, shifted with it."""
    n, mbh = 2048, 0.01
    m, x, v = ics.plummer_bh(n, 7, mbh)
    ms, xs, vs = ics.plummer(n, 7)
    assert m.shape == (n + 1,) and x.shape == (n + 1, 3)
    assert m[0] == mbh and abs(m.sum() - 1) < 1e-14
    assert np.allclose(m[1:], ms * (1 - mbh), rtol=0, atol=1e-18)
    assert np.abs((m[:, None] * x).sum(0)).max() < 1e-15
    assert np.abs((m[:, None] * v).sum(0)).max() < 1e-15
    # the hole sits where the stars' centre of mass was, i.e. at the origin
    # up to the shift the frame change applies to everything alike
    shift = x[1:] - xs
    assert np.abs(shift - shift[0]).max() < 1e-15
    assert np.abs(x[0] - shift[0]).max() < 1e-15
    assert np.abs(v[1:] - vs - (v[1:] - vs)[0]).max() < 1e-15


def test_king_w0_6_concentration_and_units():
    r, W, M = ics.king_profile(6.0)
    # tidal concentration log10(r_t / r_0) of the W0 = 6 King model ~ 1.25
    assert abs(math.log10(r[-1]) - 1.25) < 0.02
    m, x, v = ics.king(4096, 6.0, 7)
    ek, ep, _ = oracle.energy(m, x, v, 1e-4)
    assert abs(ek + ep + 0.25) < 0.02
    assert abs(ek / -ep - 0.5) < 0.04


def test_kroupa_like_spectrum():
    m = ics.kroupa_like(200000, 3)
    assert abs(m.sum() - 1) < 1e-12
    mu = m / m.min() * 0.1            # back to physical masses (m_min ~ 0.1)
    assert mu.max() <= 10.0 * 1.01
    # slope of each leg from the log-log histogram
    for lo, hi, slope in ((0.12, 0.45, -1.3), (0.6, 8.0, -2.3)):
        edges = np.geomspace(lo, hi, 12)
        h, _ = np.histogram(mu, edges)
        c = np.sqrt(edges[1:] * edges[:-1])
        dens = h / np.diff(edges)
        fit = np.polyfit(np.log(c), np.log(dens), 1)[0]
        assert abs(fit - slope) < 0.15, (lo, hi, fit)


def test_ensemble_sizes_and_offsets():
    s = ics.ensemble_sizes()
    assert s.size == 256 and s.min() >= 256 and s.max() <= 16384
    assert 0.8e6 < s.sum() < 1.3e6
    m, x, v, off = ics.king_ensemble(4, sizes=[300, 500, 256, 1000])
    assert list(off) == [0, 300, 800, 1056, 2056]
    for c in range(4):
        assert abs(m[off[c]:off[c + 1]].sum() - 1) < 1e-12


def test_active_subset():
    idx = ics.active_subset(65536, 1024, 2003)
    assert idx.size == 1024 and np.all(np.diff(idx) > 0) and idx.min() >= 0 and idx.max() < 65536
