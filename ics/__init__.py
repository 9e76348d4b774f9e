"""Seeded synthetic inputs for the N-body hot path.

This module holds input generators only: initial conditions (Plummer sphere,
King W0 model, Kroupa-like mass spectrum), active subsets and smooth
synthetic derivative fields.  It contains none of the integration method's
arithmetic (no pairwise forces, no predictor, corrector, step criterion or
energy sums), so that the oracle and the GPU library can both be fed from it
without sharing any of the computation under test.

Units are Henon units: G = M = 1, E = -1/4.  The paper's Plummer runs use
b = M = G = 1 (Sect. 5); a Plummer sphere in Henon units has scale length
b = 3 pi / 16, and the energies below are those of the continuous models, so
a finite sample carries the usual O(N^-1/2) scatter about E = -1/4.
"""
from __future__ import annotations

import math

import numpy as np
from scipy.integrate import solve_ivp
from scipy.special import erf

PLUMMER_B = 3.0 * math.pi / 16.0   # Plummer scale length in Henon units


def _isotropic(rng, n):
    z = rng.uniform(-1.0, 1.0, n)
    ph = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(1.0 - z * z)
    return np.stack([s * np.cos(ph), s * np.sin(ph), z], axis=1)


def _com_frame(m, x, v):
    M = m.sum()
    x -= (m[:, None] * x).sum(0) / M
    v -= (m[:, None] * v).sum(0) / M
    return x, v


def plummer(n: int, seed: int, *, mfrac_max: float = 0.999):
    """Equal-mass Plummer sphere (density of paper Sect. 5) in Henon units.

    Radii follow the inverse cumulative mass M(r) = r^3 / (r^2 + b^2)^(3/2)
    (mass fractions above ``mfrac_max`` are redrawn); speeds are drawn by
    rejection from g(q) = q^2 (1 - q^2)^(7/2), v = q v_esc(r), as in
    Aarseth, Henon & Wielen (1974).  Returns (mass[n], pos[n,3], vel[n,3]).
    """
    rng = np.random.default_rng(seed)
    b = PLUMMER_B
    X = rng.uniform(0.0, 1.0, n)
    while True:
        bad = X > mfrac_max
        if not bad.any():
            break
        X[bad] = rng.uniform(0.0, 1.0, int(bad.sum()))
    r = b / np.sqrt(X ** (-2.0 / 3.0) - 1.0)
    x = r[:, None] * _isotropic(rng, n)
    q = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        qq = rng.uniform(0.0, 1.0, todo.size)
        yy = rng.uniform(0.0, 0.1, todo.size)
        ok = yy < qq * qq * (1.0 - qq * qq) ** 3.5
        q[todo[ok]] = qq[ok]
        todo = todo[~ok]
    vesc = np.sqrt(2.0) * (r * r + b * b) ** -0.25
    v = (q * vesc)[:, None] * _isotropic(rng, n)
    m = np.full(n, 1.0 / n)
    x, v = _com_frame(m, x, v)
    return m, x, v


def plummer_bh(n: int, seed: int, m_bh: float = 0.01):
    """A Plummer sphere of ``n`` stars (as ``plummer``) with a central
    massive black hole: particle 0 is the hole, of mass ``m_bh`` at rest at
    the centre, and the stars share the mass 1 - m_bh (their positions and
    velocities are those of the star-only model, so the system starts close
    to, not exactly in, equilibrium).  The paper notes that such an object
    makes the blocks with few particles carry much more of the run time
    (Sect. 5.5); the hole's mass and placement are this generator's choice.
    Returns (mass[n+1], pos[n+1,3], vel[n+1,3]) in the centre-of-mass frame."""
    ms, xs, vs = plummer(n, seed)
    m = np.concatenate([[m_bh], ms * (1.0 - m_bh)])
    x = np.concatenate([np.zeros((1, 3)), xs])
    v = np.concatenate([np.zeros((1, 3)), vs])
    x, v = _com_frame(m, x, v)
    return m, x, v


def plummer_mean_acc(pos):
    """Acceleration of the smooth Plummer model at ``pos`` (Henon units),
    -r / (r^2 + b^2)^(3/2).  Used only as a realistic synthetic source
    acceleration field for kernel-level tests."""
    r2 = (pos * pos).sum(1)
    return -pos / ((r2 + PLUMMER_B ** 2) ** 1.5)[:, None]


# ---------------------------------------------------------------- King W0
def _king_rho(W):
    W = np.maximum(W, 0.0)
    return np.exp(W) * erf(np.sqrt(W)) - np.sqrt(4.0 * W / math.pi) * (1.0 + 2.0 * W / 3.0)


def king_profile(W0: float, npts: int = 4000):
    """Solve King's (1966) dimensionless Poisson equation
    W'' + 2 W' / r = -9 rho(W) / rho(W0), W(0) = W0, W'(0) = 0 out to the
    tidal radius W = 0, in units of the King radius and of sigma (G = 1).
    Returns (r, W, Menc) on a grid, with Menc the enclosed mass."""
    rho0 = _king_rho(np.array(W0))

    def rhs(r, y):
        W, dW = y
        return [dW, -9.0 * _king_rho(np.array(W)) / rho0 - 2.0 * dW / r]

    def hit(r, y):
        return y[0]
    hit.terminal, hit.direction = True, -1
    r0 = 1e-6
    # series start: W = W0 - (3/2) r^2
    sol = solve_ivp(rhs, (r0, 1e4), [W0 - 1.5 * r0 * r0, -3.0 * r0], events=hit,
                    rtol=1e-12, atol=1e-14, dense_output=True, max_step=0.01)
    rt = sol.t_events[0][0]
    r = np.concatenate([[0.0], np.geomspace(r0, rt, npts)])
    Y = sol.sol(np.clip(r, r0, rt))
    W = np.clip(Y[0], 0.0, None)
    W[0] = W0
    # r^2 W' = -9 int rho/rho0 r^2 dr  and  M(r) = 4 pi rho0_phys int ... ;
    # with rho0_phys = 9 / (4 pi) (King radius, sigma = G = 1): M(r) = -r^2 W'
    Menc = np.clip(-(r ** 2) * np.concatenate([[0.0], Y[1][1:]]), 0.0, None)
    Menc[-1] = -(rt ** 2) * sol.sol(rt)[1]
    Menc = np.maximum.accumulate(Menc)
    return r, W, Menc


def king(n: int, W0: float, seed: int, masses=None):
    """King (1966) model with central potential W0, sampled in Henon units.

    Radii come from the inverse enclosed-mass profile; speeds from
    f(v) ~ v^2 (exp(W - v^2/2) - 1), v < sqrt(2 W), by rejection.  The model
    is then scaled to M = 1 and potential energy -1/2 of the continuous
    model (W = -G int M(r) dM / r), i.e. E = -1/4 by the virial theorem.
    ``masses`` (optional, summing to 1) are assigned independently of phase
    space.  Returns (mass[n], pos[n,3], vel[n,3])."""
    rng = np.random.default_rng(seed)
    r, W, Menc = king_profile(W0)
    Mtot = Menc[-1]
    # potential energy of the continuous model, W = -int M(r)/r dM
    dM = np.diff(Menc)
    rm = 0.5 * (r[1:] + r[:-1])
    Mm = 0.5 * (Menc[1:] + Menc[:-1])
    Wpot = -np.sum(np.where(rm > 0, Mm / np.maximum(rm, 1e-300), 0.0) * dM)
    u = rng.uniform(0.0, 1.0, n) * Mtot
    rr = np.interp(u, Menc, r)
    Wr = np.interp(rr, r, W)
    x = rr[:, None] * _isotropic(rng, n)
    v = np.empty(n)
    todo = np.arange(n)
    while todo.size:
        w = Wr[todo]
        vmax = np.sqrt(2.0 * w)
        vv = rng.uniform(0.0, 1.0, todo.size) * vmax
        g = vv * vv * (np.exp(w - 0.5 * vv * vv) - 1.0)
        # bound of g on [0, vmax]: at most vmax^2 (e^w - 1)
        gmax = vmax * vmax * (np.exp(w) - 1.0) + 1e-300
        ok = rng.uniform(0.0, 1.0, todo.size) * gmax < g
        v[todo[ok]] = vv[ok]
        todo = todo[~ok]
    vel = v[:, None] * _isotropic(rng, n)
    # scale to Henon units: M = 1, W = -1/2
    L = -(Mtot ** 2) / (2.0 * Wpot)        # length unit in King radii
    V = math.sqrt(Mtot / L)                # velocity unit (G = 1)
    x /= L
    vel /= V
    m = np.full(n, 1.0 / n) if masses is None else np.asarray(masses, dtype=np.float64)
    x, vel = _com_frame(m, x, vel)
    return m, x, vel


def kroupa_like(n: int, seed: int, mlo=0.1, mbr=0.5, mhi=10.0, a1=1.3, a2=2.3):
    """Broken power law dN/dm ~ m^-a1 on [mlo, mbr), ~ m^-a2 on [mbr, mhi],
    continuous at mbr, drawn by inverse CDF and normalised to total mass 1."""
    rng = np.random.default_rng(seed)
    k2 = mbr ** (a2 - a1)                   # continuity factor for the upper leg

    def seg(lo, hi, a):
        return (hi ** (1 - a) - lo ** (1 - a)) / (1 - a)
    w1 = seg(mlo, mbr, a1)
    w2 = k2 * seg(mbr, mhi, a2)
    u = rng.uniform(0.0, 1.0, n) * (w1 + w2)
    m = np.empty(n)
    lo = u < w1
    m[lo] = (mlo ** (1 - a1) + (1 - a1) * u[lo]) ** (1.0 / (1 - a1))
    uu = (u[~lo] - w1) / k2
    m[~lo] = (mbr ** (1 - a2) + (1 - a2) * uu) ** (1.0 / (1 - a2))
    return m / m.sum()


def ensemble_sizes(k: int = 256, seed: int = 4004, nmin: int = 256, nmax: int = 16384):
    """Cluster sizes N_k = round(exp(U(ln nmin, ln nmax)))."""
    rng = np.random.default_rng(seed)
    return np.rint(np.exp(rng.uniform(math.log(nmin), math.log(nmax), k))).astype(np.int64)


def king_ensemble(k: int = 256, W0: float = 6.0, seed: int = 4004, sizes=None):
    """``k`` independent King W0 clusters with Kroupa-like masses, each in its
    own Henon units, concatenated.  Returns (mass, pos, vel, offsets[k+1])."""
    sizes = ensemble_sizes(k, seed) if sizes is None else np.asarray(sizes, dtype=np.int64)
    ms, xs, vs = [], [], []
    for c, nc in enumerate(sizes):
        mm = kroupa_like(int(nc), 4100 + c)
        m, x, v = king(int(nc), W0, 4100 + c + 100000, masses=mm)
        ms.append(m)
        xs.append(x)
        vs.append(v)
    off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
    return np.concatenate(ms), np.concatenate(xs), np.concatenate(vs), off


def active_subset(n: int, n_act: int, seed: int):
    """``n_act`` distinct indices of [0, n), ascending."""
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n, n_act, replace=False)).astype(np.int64)


def random_vectors(n: int, seed: int, scale=1.0):
    """Gaussian 3-vectors, used as synthetic derivative fields."""
    return np.random.default_rng(seed).normal(0.0, scale, (n, 3))
