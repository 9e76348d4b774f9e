"""Host-side checks of the C ABI that need no GPU: the library loads, it
exports every function that include/nbody.h declares, and argument
validation that happens before any device work returns the documented
codes."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nbody.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(nbody_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    from paper_1207_2367_amd import nbody
    return nbody.load()


def test_exports_every_declared_symbol(lib):
    names = _declared()
    assert len(names) >= 17
    for name in names:
        assert hasattr(lib, name), name
    from paper_1207_2367_amd import nbody
    assert sorted(nbody.EXPORTS) == names


def test_default_config_and_workspace_size(lib):
    from paper_1207_2367_amd import nbody
    cfg = nbody.default_config()
    assert cfg.eta == 0.45 and cfg.eta_init == 0.1
    assert cfg.dt_min == 2.0 ** -25 and cfg.dt_max == 1.0 / 16
    assert cfg.precision == nbody.PREC_MIXED and cfg.n_clusters == 1
    ws = nbody.workspace_bytes(65536, cfg)
    # the state alone is 176 bytes per particle; the total stays modest
    assert 176 * 65536 < ws < 4096 * 65536
    assert ws % 256 == 0
    f64 = nbody.default_config(precision=nbody.PREC_FP64)
    assert nbody.workspace_bytes(65536, f64) > ws   # 80-byte source records


@pytest.mark.parametrize("field,value", [
    ("eta", 0.0), ("eta", -1.0), ("eta_init", 0.0), ("dt_min", 3e-8), ("dt_max", 0.1),
    ("dt_min", 0.25), ("precision", 7),
])
def test_workspace_rejects_bad_config(lib, field, value):
    from paper_1207_2367_amd import nbody
    cfg = nbody.default_config(**{field: value})
    assert nbody.workspace_bytes(1024, cfg) == 0


def test_cluster_offsets_validated(lib):
    from paper_1207_2367_amd import nbody
    good = (C.c_int64 * 3)(0, 10, 30)
    cfg = nbody.default_config(n_clusters=2, cluster_offsets=C.cast(good, C.POINTER(C.c_int64)))
    assert nbody.workspace_bytes(30, cfg) > 0
    assert nbody.workspace_bytes(31, cfg) == 0               # offsets must end at n
    bad = (C.c_int64 * 3)(0, 10, 10)
    cfg.cluster_offsets = C.cast(bad, C.POINTER(C.c_int64))
    assert nbody.workspace_bytes(10, cfg) == 0               # empty cluster


def test_init_rejects_bad_arguments_before_device_work(lib):
    from paper_1207_2367_amd import nbody
    cfg = nbody.default_config()
    ctx = C.c_void_p()
    dummy = C.c_void_p(256)
    # n <= 0, NULL pointers, negative or non-finite softening, small workspace
    assert lib.nbody_init(C.byref(ctx), 0, dummy, dummy, dummy, 1e-4, C.byref(cfg), dummy, 1 << 30) == nbody.EINVAL
    assert lib.nbody_init(C.byref(ctx), 16, None, dummy, dummy, 1e-4, C.byref(cfg), dummy, 1 << 30) == nbody.EINVAL
    assert lib.nbody_init(C.byref(ctx), 16, dummy, dummy, dummy, -1.0, C.byref(cfg), dummy, 1 << 30) == nbody.EINVAL
    assert lib.nbody_init(C.byref(ctx), 16, dummy, dummy, dummy, float("nan"), C.byref(cfg), dummy, 1 << 30) == nbody.EINVAL
    assert lib.nbody_init(C.byref(ctx), 16, dummy, dummy, dummy, 1e-4, C.byref(cfg), dummy, 64) == nbody.EINVAL
    assert lib.nbody_init(C.byref(ctx), 16, dummy, dummy, dummy, 1e-4, C.byref(cfg), C.c_void_p(257), 1 << 30) == nbody.EINVAL
    assert ctx.value is None


def test_strerror(lib):
    for code in (0, -1, -2, -3, -4, -5, -99):
        assert isinstance(lib.nbody_strerror(code), bytes)
    assert lib.nbody_last_error(None) == b"null context"


def test_null_context_calls_are_rejected(lib):
    from paper_1207_2367_amd import nbody
    assert lib.nbody_set_step_loop(None, -1) == nbody.EINVAL
    assert lib.nbody_set_schedule(None, 0) == nbody.EINVAL
    assert lib.nbody_set_launch(None, None) == nbody.EINVAL
    assert lib.nbody_step(None, 1.0, None) == nbody.EINVAL
    assert lib.nbody_autotune(None, 10.0) == nbody.EINVAL
    assert lib.nbody_get_tuning(None, None, 0) == nbody.EINVAL
    assert lib.nbody_set_tuning(None, None, 0) == nbody.EINVAL


def test_noalloc_arguments_rejected_before_device_work(lib):
    """nbody_force_noalloc checks sizes against its fixed scratch (and its
    other arguments) on the host, before any device call."""
    from paper_1207_2367_amd import nbody
    d = C.c_void_p(256)
    args = (d, d, d, d)
    outs = (d, d, d, None, None)
    # 1,310,720 sources do not fit the 64 MiB scratch in any precision (56 B
    # per source at the least)
    for prec in (0, 1, 2):
        assert lib.nbody_force_noalloc(5 << 18, *args, 1e-4, prec, 1, d, *outs) == nbody.EINVAL
    # FP64 records (80 B) plus one split of partials (80 B per active
    # particle): 450,000 sources all active exceed 64 MiB
    assert lib.nbody_force_noalloc(450000, *args, 1e-4, 1, 450000, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *args, -1.0, 0, 1, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *args, float("inf"), 0, 1, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *args, 1e-4, 7, 1, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *args, 1e-4, 0, 5, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(0, *args, 1e-4, 0, 0, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, None, d, d, d, 1e-4, 0, 1, d, *outs) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *args, 1e-4, 0, 0, d, *outs) == nbody.OK
