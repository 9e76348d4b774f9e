"""ctypes binding of the C ABI in include/nbody.h.

Argument marshalling only: every step of the method runs in the library's
HIP kernels.  torch supplies device memory (inputs, outputs and the
workspace) and the stream.  The library must have been built
(``python -m paper_1207_2367_amd.build``); there is no fallback.
"""
from __future__ import annotations

import contextlib
import ctypes as C
import os
import sys

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libnbody.so")

OK, EINVAL, EDEVICE, ENONFINITE, EDTMIN, ESTATE = 0, -1, -2, -3, -4, -5
PREC_MIXED, PREC_FP64, PREC_FP32PAIR = 0, 1, 2

_lib = None


class NBodyError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"nbody error {code}: {msg}")
        self.code = code


class Config(C.Structure):
    _fields_ = [
        ("eta", C.c_double), ("eta_init", C.c_double), ("dt_min", C.c_double),
        ("dt_max", C.c_double), ("precision", C.c_int32), ("n_clusters", C.c_int32),
        ("cluster_offsets", C.POINTER(C.c_int64)), ("stream", C.c_void_p),
        ("validate", C.c_int32), ("skip_startup", C.c_int32),
    ]


class StepStats(C.Structure):
    _fields_ = [("block_steps", C.c_int64), ("active_total", C.c_int64),
                ("interactions", C.c_double), ("hist", C.c_int64 * 40)]


NPHASE = 6
PHASES = ("schedule", "predict", "force", "reduce", "correct", "energy")


class ProfileTimes(C.Structure):
    _fields_ = [("ms", C.c_double * NPHASE), ("launches", C.c_int64 * NPHASE),
                ("pairs", C.c_double)]


class Launch(C.Structure):
    _fields_ = [("lanes_per_i", C.c_int32), ("waves", C.c_int32), ("split", C.c_int32),
                ("i_per_lane", C.c_int32)]


EXPORTS = [
    "nbody_default_config", "nbody_workspace_bytes", "nbody_init", "nbody_free",
    "nbody_force", "nbody_predict", "nbody_schedule", "nbody_correct", "nbody_block_step",
    "nbody_step", "nbody_get_state", "nbody_set_state", "nbody_energy", "nbody_autotune",
    "nbody_set_launch", "nbody_get_launch", "nbody_set_step_loop", "nbody_set_schedule",
    "nbody_strerror",
    "nbody_last_error",
    "nbody_profile", "nbody_profile_force_log", "nbody_force_noalloc",
    "nbody_get_tuning", "nbody_set_tuning",
]


def lib_path() -> str:
    return _LIB_PATH


def load():
    """Load libnbody.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise RuntimeError(f"{_LIB_PATH} is missing: build it with "
                           "`python -m paper_1207_2367_amd.build`")
    lib = C.CDLL(_LIB_PATH)
    vp, i64, d, i32 = C.c_void_p, C.c_int64, C.c_double, C.c_int32
    P = C.POINTER
    sig = {
        "nbody_default_config": (None, [P(Config)]),
        "nbody_workspace_bytes": (C.c_size_t, [i64, P(Config)]),
        "nbody_init": (C.c_int, [P(vp), i64, vp, vp, vp, d, P(Config), vp, C.c_size_t]),
        "nbody_free": (None, [vp]),
        "nbody_force": (C.c_int, [vp, i64, vp, vp, vp, vp, vp]),
        "nbody_predict": (C.c_int, [vp, d, vp, vp, vp]),
        "nbody_schedule": (C.c_int, [vp, d, vp, P(i64), P(d)]),
        "nbody_correct": (C.c_int, [vp, i64, vp, d, vp, vp, vp]),
        "nbody_block_step": (C.c_int, [vp, d, P(i64), P(d)]),
        "nbody_step": (C.c_int, [vp, d, P(StepStats)]),
        "nbody_get_state": (C.c_int, [vp] + [vp] * 8),
        "nbody_set_state": (C.c_int, [vp] + [vp] * 8),
        "nbody_energy": (C.c_int, [vp, P(d), P(d), P(d)]),
        "nbody_autotune": (C.c_int, [vp, d]),
        "nbody_set_launch": (C.c_int, [vp, P(Launch)]),
        "nbody_get_tuning": (C.c_int, [vp, P(Launch), i32]),
        "nbody_set_tuning": (C.c_int, [vp, P(Launch), i32]),
        "nbody_get_launch": (C.c_int, [vp, i64, P(Launch)]),
        "nbody_set_step_loop": (C.c_int, [vp, i64]),
        "nbody_set_schedule": (C.c_int, [vp, C.c_int]),
        "nbody_profile": (C.c_int, [vp, C.c_int, P(ProfileTimes)]),
        "nbody_profile_force_log": (i64, [vp, i64, vp, vp, vp]),
        "nbody_strerror": (C.c_char_p, [C.c_int]),
        "nbody_last_error": (C.c_char_p, [vp]),
        "nbody_force_noalloc": (C.c_int, [i64, vp, vp, vp, vp, d, i32, i64, vp, vp, vp, vp, vp,
                                          vp]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def default_config(**kw) -> Config:
    cfg = Config()
    load().nbody_default_config(C.byref(cfg))
    for k, v in kw.items():
        setattr(cfg, k, v)
    return cfg


def workspace_bytes(n: int, cfg: Config) -> int:
    return int(load().nbody_workspace_bytes(int(n), C.byref(cfg)))


def _ptr(t):
    return None if t is None else C.c_void_p(t.data_ptr())


def _dev_f64(t, shape, device):
    t = torch.as_tensor(t, dtype=torch.float64, device=device).contiguous()
    if tuple(t.shape) != tuple(shape):
        t = t.reshape(shape).contiguous()
    return t


def _dev_i32(t, device):
    return torch.as_tensor(t, device=device).to(torch.int32).contiguous()


def force_noalloc(mass, pos, vel, acc, eps, idx, precision=PREC_MIXED, out=None, pot=True,
                  device="cuda"):
    """nbody_force_noalloc: a, da, d2a (and the potential) of particles
    ``idx`` against the given arrays, with no context or workspace.  Inputs
    are taken as device FP64 tensors (copied there if they are not); the
    call is queued on the current stream."""
    dev = torch.device(device)
    m = _dev_f64(mass, (-1,), dev)
    n = m.shape[0]
    x, v, a = (_dev_f64(q, (n, 3), dev) for q in (pos, vel, acc))
    idx = _dev_i32(idx, dev)
    na = idx.shape[0]
    if out is None:
        out = [torch.empty((na, 3), dtype=torch.float64, device=dev) for _ in range(3)]
        out.append(torch.empty(na, dtype=torch.float64, device=dev) if pot else None)
    stream = torch.cuda.current_stream(dev)
    rc = load().nbody_force_noalloc(n, _ptr(m), _ptr(x), _ptr(v), _ptr(a), float(eps),
                                    int(precision), na, _ptr(idx), *[_ptr(o) for o in out],
                                    C.c_void_p(stream.cuda_stream))
    if rc != OK:
        raise NBodyError(rc, load().nbody_strerror(rc).decode())
    # the inputs may be temporaries of this call: keep them until the
    # queued work is done
    for t in (m, x, v, a, idx):
        t.record_stream(stream)
    return tuple(out)


class System:
    """One N-body system (or ensemble of clusters) resident on the GPU."""

    def __init__(self, mass, pos, vel, eps, *, eta=0.45, eta_init=0.1,
                 dt_min=2.0 ** -25, dt_max=1.0 / 16, precision=PREC_MIXED,
                 offsets=None, validate=False, skip_startup=False, device="cuda"):
        lib = load()
        self.device = torch.device(device)
        mass = _dev_f64(mass, (-1,), self.device)
        n = self.n = mass.shape[0]
        pos = _dev_f64(pos, (n, 3), self.device)
        vel = _dev_f64(vel, (n, 3), self.device)
        self._offsets = None
        cfg = default_config(eta=eta, eta_init=eta_init, dt_min=dt_min, dt_max=dt_max,
                             precision=precision, validate=1 if validate else 0,
                             skip_startup=1 if skip_startup else 0)
        if offsets is not None and len(offsets) > 2:
            self._offsets = (C.c_int64 * len(offsets))(*[int(o) for o in offsets])
            cfg.n_clusters = len(offsets) - 1
            cfg.cluster_offsets = C.cast(self._offsets, C.POINTER(C.c_int64))
        self.stream = torch.cuda.current_stream(self.device)
        cfg.stream = C.c_void_p(self.stream.cuda_stream)
        self.cfg = cfg
        self.eps = float(eps)
        ws = workspace_bytes(n, cfg)
        if ws == 0:
            raise NBodyError(EINVAL, "invalid configuration")
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        ctx = C.c_void_p()
        rc = lib.nbody_init(C.byref(ctx), n, _ptr(mass), _ptr(pos), _ptr(vel), self.eps,
                            C.byref(cfg), _ptr(self.workspace), ws)
        if rc != OK:
            raise NBodyError(rc, lib.nbody_strerror(rc).decode())
        self.ctx = ctx

    # ------------------------------------------------------------ helpers
    @contextlib.contextmanager
    def _on_ctx_stream(self):
        """Run a call on the context's stream: it first waits for the work
        the caller queued on the current stream (inputs), temporaries are
        allocated on it, and the current stream then waits for it (outputs)."""
        cur = torch.cuda.current_stream(self.device)
        if cur == self.stream:
            yield
            return
        self.stream.wait_stream(cur)
        with torch.cuda.stream(self.stream):
            yield
        cur.wait_stream(self.stream)

    def _check(self, rc):
        if rc != OK:
            msg = load().nbody_last_error(self.ctx).decode()
            raise NBodyError(rc, msg or load().nbody_strerror(rc).decode())

    def close(self):
        if getattr(self, "ctx", None):
            load().nbody_free(self.ctx)
            self.ctx = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # no HIP calls while the interpreter shuts down (the runtime's own
        # teardown may already be under way, and module globals may already
        # be cleared): close() systems explicitly
        if _finalizing():
            return
        try:
            self.close()
        except Exception:
            pass

    # ----------------------------------------------------------- the ABI
    def force(self, idx, out=None, pot=True):
        """a, da, d2a, potential of particles ``idx`` (ascending) from the
        stored state of all sources of their cluster."""
        with self._on_ctx_stream():
            idx = _dev_i32(idx, self.device)
            na = idx.shape[0]
            if out is None:
                out = [torch.empty((na, 3), dtype=torch.float64, device=self.device)
                       for _ in range(3)]
                out.append(torch.empty(na, dtype=torch.float64, device=self.device) if pot else None)
            rc = load().nbody_force(self.ctx, na, _ptr(idx), *[_ptr(o) for o in out])
            self._check(rc)
        return tuple(out)

    def predict(self, t):
        with self._on_ctx_stream():
            outs = [torch.empty((self.n, 3), dtype=torch.float64, device=self.device)
                    for _ in range(3)]
            self._check(load().nbody_predict(self.ctx, float(t), *[_ptr(o) for o in outs]))
        return tuple(outs)

    def schedule(self, t_target):
        with self._on_ctx_stream():
            idx = torch.empty(self.n, dtype=torch.int32, device=self.device)
            na, tn = C.c_int64(0), C.c_double(0.0)
            self._check(load().nbody_schedule(self.ctx, float(t_target), _ptr(idx), C.byref(na),
                                              C.byref(tn)))
        return idx[: na.value], tn.value

    def correct(self, idx, t_target, acc, jrk, snp):
        with self._on_ctx_stream():
            idx = _dev_i32(idx, self.device)
            na = idx.shape[0]
            ins = [_dev_f64(q, (na, 3), self.device) for q in (acc, jrk, snp)]
            self._check(load().nbody_correct(self.ctx, na, _ptr(idx), float(t_target),
                                             *[_ptr(q) for q in ins]))

    def block_step(self, t_target):
        na, tb = C.c_int64(0), C.c_double(0.0)
        self._check(load().nbody_block_step(self.ctx, float(t_target), C.byref(na), C.byref(tb)))
        return na.value, tb.value

    def step(self, t_target):
        st = StepStats()
        self._check(load().nbody_step(self.ctx, float(t_target), C.byref(st)))
        return {"block_steps": st.block_steps, "active_total": st.active_total,
                "interactions": st.interactions, "hist": list(st.hist)}

    def get_state(self):
        n = self.n
        with self._on_ctx_stream():
            vec = [torch.empty((n, 3), dtype=torch.float64, device=self.device) for _ in range(6)]
            sc = [torch.empty(n, dtype=torch.float64, device=self.device) for _ in range(2)]
            self._check(load().nbody_get_state(self.ctx, *[_ptr(q) for q in vec + sc]))
        keys = ("x", "v", "a", "jk", "sn", "cr", "t", "dt")
        return dict(zip(keys, vec + sc))

    def set_state(self, x=None, v=None, a=None, jk=None, sn=None, cr=None, t=None, dt=None):
        n = self.n
        with self._on_ctx_stream():
            vec = [None if q is None else _dev_f64(q, (n, 3), self.device)
                   for q in (x, v, a, jk, sn, cr)]
            sc = [None if q is None else _dev_f64(q, (n,), self.device) for q in (t, dt)]
            self._check(load().nbody_set_state(self.ctx, *[_ptr(q) for q in vec + sc]))
            # the copies are queued on the context's stream; temporaries made
            # here belong to that stream, so the caching allocator reuses them
            # only after the copies
            for q in vec + sc:
                if q is not None:
                    q.record_stream(self.stream)

    def energy(self):
        ek, ep, L = C.c_double(0), C.c_double(0), (C.c_double * 3)()
        self._check(load().nbody_energy(self.ctx, C.byref(ek), C.byref(ep), L))
        return ek.value, ep.value, [L[0], L[1], L[2]]

    def autotune(self, max_ms=200.0, cache=None):
        """Measure launch shapes (nbody_autotune).  With ``cache`` (a JSON
        file path) a table stored there for the same system shape,
        precision and device is loaded instead of measuring, and a new
        measurement is stored."""
        import json
        key = {"n": self.n, "clusters": None if self._offsets is None else list(self._offsets),
               "precision": int(self.cfg.precision),
               "device": torch.cuda.get_device_name(self.device)}
        if cache is not None and os.path.exists(cache):
            with open(cache) as f:
                data = json.load(f)
            if data.get("key") == key:
                self.set_tuning(data["table"])
                return
        self._check(load().nbody_autotune(self.ctx, float(max_ms)))
        if cache is not None:
            tmp = cache + ".tmp"
            with open(tmp, "w") as f:
                json.dump({"key": key, "table": self.get_tuning()}, f)
            os.replace(tmp, cache)

    def get_tuning(self):
        """The autotuner's table: [(lanes_per_i, waves, split, i_per_lane)]
        per power of two of N_act (zeros: no tuned shape)."""
        tab = (Launch * 40)()
        cnt = load().nbody_get_tuning(self.ctx, tab, 40)
        if cnt < 0:
            self._check(int(cnt))
        return [(e.lanes_per_i, e.waves, e.split, e.i_per_lane) for e in tab[:cnt]]

    def set_tuning(self, table):
        tab = (Launch * max(1, len(table)))(*[Launch(*map(int, e)) for e in table])
        self._check(load().nbody_set_tuning(self.ctx, tab, len(table)))

    def set_launch(self, lanes_per_i=0, waves=0, split=0, i_per_lane=0):
        sh = Launch(int(lanes_per_i), int(waves), int(split), int(i_per_lane))
        self._check(load().nbody_set_launch(self.ctx, C.byref(sh)))

    def set_step_loop(self, max_active=-1):
        """Device-resident block steps of step(): automatic limit (< 0),
        off (0) or at most max_active active particles per block."""
        self._check(load().nbody_set_step_loop(self.ctx, int(max_active)))

    def set_schedule(self, mode=0):
        """How step() finds the next block: 0 from per-level counts where the
        state allows it (the default), 1 by a sweep of all particles."""
        self._check(load().nbody_set_schedule(self.ctx, int(mode)))

    def profile(self, enable):
        """Start (enable=True, clears) or stop event timing of the phases;
        returns the totals so far as {phase: (ms, launches)} plus pairs."""
        pt = ProfileTimes()
        self._check(load().nbody_profile(self.ctx, 1 if enable else 0, C.byref(pt)))
        out = {ph: (pt.ms[k], pt.launches[k]) for k, ph in enumerate(PHASES)}
        out["pairs"] = pt.pairs
        return out

    def force_log(self):
        """Per-launch force-kernel records: (n_act, pairs, ms) arrays."""
        import numpy as np
        lib = load()
        n = lib.nbody_profile_force_log(self.ctx, 0, None, None, None)
        if n < 0:
            self._check(int(n))
        na = np.zeros(n, dtype=np.int64)
        pr = np.zeros(n)
        ms = np.zeros(n)
        lib.nbody_profile_force_log(self.ctx, n, na.ctypes.data_as(C.c_void_p),
                                    pr.ctypes.data_as(C.c_void_p), ms.ctypes.data_as(C.c_void_p))
        return na, pr, ms

    def get_launch(self, n_act):
        sh = Launch()
        self._check(load().nbody_get_launch(self.ctx, int(n_act), C.byref(sh)))
        return sh.lanes_per_i, sh.waves, sh.split, sh.i_per_lane
