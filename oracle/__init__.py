"""Plain FP64 CPU oracle for the Hermite-6 block-step direct N-body method
of arXiv:1207.2367 (Capuzzo-Dolcetta, Spera & Punzo).

TEST INFRASTRUCTURE ONLY: the tests, the smoke check and the CPU-baseline
leg of the benchmark are the only code allowed to import this package.  The
GPU library never calls it and shares no code with it.

The arithmetic lives in ``nbody_oracle.c`` (plain C, binary64, no FMA
contraction, no fast-math); this module compiles it with gcc and wraps it
with ctypes and numpy.  Every function names the passage of the paper it
follows; the readings taken where the paper is silent are listed in the C
source.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "nbody_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
CFLAGS = ["-O2", "-fopenmp", "-ffp-contract=off", "-fno-fast-math", "-std=c11",
          "-shared", "-fPIC"]

OK, EINVAL, ENONFINITE, EDTMIN = 0, -1, -3, -4

_lib = None


def build() -> str:
    """Compile the oracle with gcc (always recompiles)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    # the mutation test points this at deliberately broken builds of the oracle
    alt = os.environ.get("NBODY_ORACLE_LIB")
    if alt:
        lib = C.CDLL(alt)
    else:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = C.CDLL(_LIB)
    d, i64, vp = C.c_double, C.c_int64, C.c_void_p
    lib.orc_force.argtypes = [i64, vp, vp, vp, vp, d, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.orc_force.restype = None
    lib.orc_force4.argtypes = [i64, vp, vp, vp, vp, vp, d, i64, i64, i64, vp, vp, vp, vp, vp]
    lib.orc_force4.restype = None
    lib.orc_predict.argtypes = [i64, vp, vp, vp, vp, vp, vp, vp, d, vp, vp, vp]
    lib.orc_predict.restype = None
    lib.orc_interpolate.argtypes = [d, vp, vp, vp, vp, vp, vp, vp, vp, vp]
    lib.orc_interpolate.restype = None
    lib.orc_dt_criterion.argtypes = [vp, vp, vp, vp, vp, vp, d]
    lib.orc_dt_criterion.restype = d
    lib.orc_block_dt.argtypes = [d, d, d, d, d, d, C.POINTER(d)]
    lib.orc_block_dt.restype = C.c_int
    lib.orc_schedule.argtypes = [i64, vp, vp, vp, C.POINTER(i64), C.POINTER(d)]
    lib.orc_schedule.restype = None
    lib.orc_correct.argtypes = [C.POINTER(_State), i64, vp, d, d, vp, vp, vp]
    lib.orc_correct.restype = C.c_int
    lib.orc_init.argtypes = [C.POINTER(_State), i64, vp, d]
    lib.orc_init.restype = C.c_int
    lib.orc_block_step.argtypes = [C.POINTER(_State), i64, vp, d, C.POINTER(i64), C.POINTER(d)]
    lib.orc_block_step.restype = C.c_int
    lib.orc_run.argtypes = [C.POINTER(_State), i64, vp, d, C.POINTER(i64), C.POINTER(d), vp]
    lib.orc_run.restype = C.c_int
    lib.orc_energy.argtypes = [i64, vp, vp, vp, d, i64, vp, vp, vp, vp]
    lib.orc_energy.restype = None
    _lib = lib
    return lib


class _State(C.Structure):
    _fields_ = [("n", C.c_int64)] + [
        (k, C.c_void_p) for k in ("m", "x", "v", "a", "jk", "sn", "cr", "t", "dt")
    ] + [(k, C.c_double) for k in ("eps", "eta", "eta_init", "dt_min", "dt_max")]


def _f64(a, shape=None):
    a = np.ascontiguousarray(a, dtype=np.float64)
    if shape is not None:
        a = a.reshape(shape)
    return a


def _i64(a):
    return np.ascontiguousarray(a, dtype=np.int64)


def _p(a):
    return a.ctypes.data_as(C.c_void_p)


# --------------------------------------------------------------------------
# single operations
# --------------------------------------------------------------------------
def force(mass, pos, vel, acc, eps, idx=None, j_range=None):
    """Direct-summation a, da, d2a and potential of the particles ``idx``
    against the sources in ``j_range`` (default all), paper Sect. 3 item 2
    with the softened potential of Sect. 2.  Returns (acc, jrk, snp, pot)
    with shapes [n_act, 3] x 3 and [n_act]."""
    lib = _load()
    m = _f64(mass)
    n = m.shape[0]
    x, v, a = _f64(pos, (n, 3)), _f64(vel, (n, 3)), _f64(acc, (n, 3))
    idx = _i64(np.arange(n) if idx is None else idx)
    j0, j1 = (0, n) if j_range is None else j_range
    na = idx.shape[0]
    out = [np.zeros((na, 3)) for _ in range(3)] + [np.zeros(na)]
    lib.orc_force(n, _p(m), _p(x), _p(v), _p(a), float(eps), int(j0), int(j1), na,
                  _p(idx), *[_p(o) for o in out])
    return tuple(out)


def force4(mass, pos, vel, acc, jrk, eps, idx=None, j_range=None):
    """a, da, d2a and the crackle of the particles ``idx`` (the evaluation
    of paper Sect. 3 item 2 extended by one derivative, used at the start).
    Returns (acc, jrk, snp, crk), each [n_act, 3]."""
    lib = _load()
    m = _f64(mass)
    n = m.shape[0]
    x, v, a, j = (_f64(q, (n, 3)) for q in (pos, vel, acc, jrk))
    idx = _i64(np.arange(n) if idx is None else idx)
    j0, j1 = (0, n) if j_range is None else j_range
    na = idx.shape[0]
    out = [np.zeros((na, 3)) for _ in range(4)]
    lib.orc_force4(n, _p(m), _p(x), _p(v), _p(a), _p(j), float(eps), int(j0), int(j1), na,
                   _p(idx), *[_p(o) for o in out])
    return tuple(out)


def predict(pos, vel, acc, jrk, snp, crk, t, T):
    """Taylor predictor of paper Sect. 3 item 1 for every particle, with
    h = T - t_i.  Returns (pos, vel, acc) at T."""
    lib = _load()
    t = _f64(t)
    n = t.shape[0]
    ins = [_f64(q, (n, 3)) for q in (pos, vel, acc, jrk, snp, crk)]
    outs = [np.empty((n, 3)) for _ in range(3)]
    lib.orc_predict(n, *[_p(q) for q in ins], _p(t), float(T), *[_p(o) for o in outs])
    return tuple(outs)


def interpolate(h, a0, j0, s0, a1, j1, s1):
    """Crackle, pop and 5th derivative at the end of a step from the quintic
    through (a, da, d2a) at both ends.  Returns three 3-vectors."""
    lib = _load()
    ins = [_f64(q, (3,)) for q in (a0, j0, s0, a1, j1, s1)]
    outs = [np.empty(3) for _ in range(3)]
    lib.orc_interpolate(float(h), *[_p(q) for q in ins], *[_p(o) for o in outs])
    return tuple(outs)


def dt_criterion(a, jk, sn, cr, pp, a5, eta):
    """Generalized Aarseth criterion, Eqs. (indtstp), (As) with p = 6."""
    lib = _load()
    ins = [_f64(q, (3,)) for q in (a, jk, sn, cr, pp, a5)]
    return lib.orc_dt_criterion(*[_p(q) for q in ins], float(eta))


def block_dt(dt_crit, dt_old, t_new, t_target, dt_min, dt_max):
    """Power-of-two block step rules.  Returns (err, dt)."""
    lib = _load()
    out = C.c_double(0.0)
    err = lib.orc_block_dt(float(dt_crit), float(dt_old), float(t_new),
                           float(t_target), float(dt_min), float(dt_max), C.byref(out))
    return err, out.value


def schedule(t, dt):
    """Next block time and its active set (ascending indices)."""
    lib = _load()
    t, dt = _f64(t), _f64(dt)
    n = t.shape[0]
    idx = np.empty(n, dtype=np.int64)
    na, tn = C.c_int64(0), C.c_double(0.0)
    lib.orc_schedule(n, _p(t), _p(dt), _p(idx), C.byref(na), C.byref(tn))
    return idx[: na.value].copy(), tn.value


def energy(mass, pos, vel, eps, offsets=None):
    """(E_kin, E_pot, L[3]) with the softened potential energy."""
    lib = _load()
    m = _f64(mass)
    n = m.shape[0]
    off = _i64([0, n] if offsets is None else offsets)
    ek, ep, L = np.zeros(1), np.zeros(1), np.zeros(3)
    lib.orc_energy(n, _p(m), _p(_f64(pos, (n, 3))), _p(_f64(vel, (n, 3))), float(eps),
                   off.shape[0] - 1, _p(off), _p(ek), _p(ep), _p(L))
    return float(ek[0]), float(ep[0]), L


# --------------------------------------------------------------------------
# integrator
# --------------------------------------------------------------------------
class Integrator:
    """Whole block-step Hermite-6 integration of one system or of several
    independent clusters (``offsets``), paper Sect. 3 and Table 1."""

    def __init__(self, mass, pos, vel, eps, eta=0.45, eta_init=0.1,
                 dt_min=2.0 ** -25, dt_max=1.0 / 16, offsets=None):
        self.m = _f64(mass).copy()
        n = self.n = self.m.shape[0]
        self.x = _f64(pos, (n, 3)).copy()
        self.v = _f64(vel, (n, 3)).copy()
        self.a, self.jk, self.sn, self.cr = (np.zeros((n, 3)) for _ in range(4))
        self.t, self.dt = np.zeros(n), np.zeros(n)
        self.off = _i64([0, n] if offsets is None else offsets)
        self.params = (float(eps), float(eta), float(eta_init), float(dt_min), float(dt_max))
        self._st = _State(n, *[_p(q) for q in (self.m, self.x, self.v, self.a, self.jk,
                                               self.sn, self.cr, self.t, self.dt)],
                          *self.params)

    @property
    def nc(self):
        return self.off.shape[0] - 1

    def init(self, t_target):
        return _load().orc_init(C.byref(self._st), self.nc, _p(self.off), float(t_target))

    def correct(self, idx, t_new, t_target, acc1, jrk1, snp1):
        idx = _i64(idx)
        na = idx.shape[0]
        ins = [_f64(q, (na, 3)) for q in (acc1, jrk1, snp1)]
        return _load().orc_correct(C.byref(self._st), na, _p(idx), float(t_new),
                                   float(t_target), *[_p(q) for q in ins])

    def block_step(self, t_target):
        na, tb = C.c_int64(0), C.c_double(0.0)
        err = _load().orc_block_step(C.byref(self._st), self.nc, _p(self.off),
                                     float(t_target), C.byref(na), C.byref(tb))
        return err, na.value, tb.value

    def run(self, t_target):
        """Returns (err, block_steps, interactions, log2 N_act histogram[64])."""
        steps, pairs = C.c_int64(0), C.c_double(0.0)
        hist = np.zeros(64, dtype=np.int64)
        err = _load().orc_run(C.byref(self._st), self.nc, _p(self.off), float(t_target),
                              C.byref(steps), C.byref(pairs), _p(hist))
        return err, steps.value, pairs.value, hist

    def energy(self):
        return energy(self.m, self.x, self.v, self.params[0], self.off)

    def state(self):
        return {k: getattr(self, k).copy() for k in ("x", "v", "a", "jk", "sn", "cr", "t", "dt")}

    def set_state(self, **kw):
        for k, val in kw.items():
            getattr(self, k)[...] = val
