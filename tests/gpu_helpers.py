"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import ics


def rel_err_rows(got, ref):
    """Per-particle relative error ||got_i - ref_i|| / ||ref_i|| (rows); rows
    with a zero reference give inf (or nan), never a silent pass."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    with np.errstate(divide="ignore", invalid="ignore"):
        if got.ndim == 1:
            return np.abs(got - ref) / np.abs(ref)
        return np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)


def abs_err_rows(got, ref):
    """Per-particle absolute error ||got_i - ref_i|| (nan if got_i is not
    finite, so that no comparison with it can pass)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    d = got - ref
    e = np.abs(d) if d.ndim == 1 else np.linalg.norm(d, axis=1)
    fin = np.isfinite(got) if got.ndim == 1 else np.isfinite(got).all(axis=1)
    return np.where(fin, e, np.nan)


def norm_rows(q):
    q = np.asarray(q, dtype=np.float64)
    return np.abs(q) if q.ndim == 1 else np.linalg.norm(q, axis=1)


def term_sums(m, x, v, a, eps, idx, j_range=None):
    """S_i(Q) = sum_j |Q_ij| for Q = a, da, d2a, potential and each listed
    particle, where |Q_ij| adds the magnitudes of the sub-terms a pair term
    is built from (m v / r^3 and 3 alpha A for the jerk; m a / r^3, 6 alpha J
    and 3 beta A for the snap).  An evaluation whose sub-terms carry relative
    error e is off by at most e S_i(Q) in absolute terms, i.e. by e kappa_i
    relative to the sum, kappa_i = S_i / |sum_j Q_ij| being its condition
    number.  FP64 pair terms (torch on the CPU, multithreaded): a test-side
    diagnostic that scales the tolerance.  The potential's entry includes
    m_i / eps when i is among the sources, because the kernels sum over
    every source including j = i and then remove that self term."""
    j0, j1 = (0, m.shape[0]) if j_range is None else j_range
    xs, vs, as_, ms = (torch.from_numpy(np.ascontiguousarray(q[j0:j1], dtype=np.float64))
                       for q in (x, v, a, m))
    ar = torch.arange(j0, j1)
    out = np.zeros((len(idx), 4))
    for k, i in enumerate(idx):
        r = xs - torch.from_numpy(np.asarray(x[i], dtype=np.float64))
        w = vs - torch.from_numpy(np.asarray(v[i], dtype=np.float64))
        q = as_ - torch.from_numpy(np.asarray(a[i], dtype=np.float64))
        s2 = (r * r).sum(1) + eps * eps
        keep = ar != i
        rinv = torch.where(keep, torch.where(s2 > 0, s2, torch.ones_like(s2)).rsqrt(),
                           torch.zeros_like(s2))
        mr3 = ms * rinv ** 3
        r2i = rinv * rinv
        al = (r * w).sum(1) * r2i
        be = ((w * w).sum(1) + (r * q).sum(1)) * r2i + al * al
        A = mr3[:, None] * r
        J = mr3[:, None] * w - 3 * al[:, None] * A
        nA = A.norm(dim=1)
        out[k, 0] = float(nA.sum())
        out[k, 1] = float((mr3 * w.norm(dim=1) + 3 * al.abs() * nA).sum())
        out[k, 2] = float((mr3 * q.norm(dim=1) + 6 * al.abs() * J.norm(dim=1)
                           + 3 * be.abs() * nA).sum())
        out[k, 3] = float((ms * rinv).sum()) + (m[i] / eps if eps > 0 and j0 <= i < j1 else 0.0)
    return out


# Tolerances per precision mode for (a, da, d2a, potential): (k, plain).
# Every row must be finite with |got - ref| <= k S_i(Q) (S from term_sums);
# where plain is set, also |got - ref| <= plain |ref| on rows whose reference
# is not zero.  The reasoning is in the docstring of test_gpu_force.py.
FORCE_TOL = {
    0: ((1e-11, 1e-6), (1e-11, 1e-6), (2e-6, None), (1e-11, 1e-6)),     # mixed
    1: ((1e-12, 1e-11), (1e-12, 1e-11), (1e-11, 1e-10), (1e-12, 1e-11)),  # FP64
    2: ((1e-6, None), (1e-6, None), (2e-6, None), (1e-6, None)),        # FP32 pairs
}
NAMES = ("a", "da", "d2a", "pot")


def check_force(tol, got, ref, S):
    """Assert the per-particle bounds of ``tol`` (a FORCE_TOL entry) for
    (a, da, d2a, phi): no non-finite value, |got - ref| <= k S_i, and the
    plain relative bound where one is set.  Prints the plain max / p99
    relative errors, the fraction within 1e-6 and the largest condition
    number.  Returns the plain max relative error per quantity."""
    gots = [cpu(q) for q in got]
    worst = []
    lines = []
    for q, (g, r) in enumerate(zip(gots, ref)):
        r = np.asarray(r, dtype=np.float64)
        assert g.shape == r.shape, (NAMES[q], g.shape, r.shape)
        k, plain = tol[q]
        e = abs_err_rows(g, r)
        nr = norm_rows(r)
        nz = nr > 0
        rel = np.where(nz, e / np.where(nz, nr, 1.0), np.where(e == 0, 0.0, np.inf))
        rel = np.where(np.isnan(e), np.nan, rel)
        kap = np.where(nz, S[:, q] / np.where(nz, nr, 1.0), np.inf)
        worst.append(float(np.nanmax(rel)) if np.isfinite(rel).any() else float("nan"))
        fin = rel[np.isfinite(rel)]
        lines.append(f"{NAMES[q]}: max {worst[-1]:.2e} p99 "
                     f"{np.percentile(fin, 99) if fin.size else float('nan'):.1e} "
                     f"<=1e-6 {(rel <= 1e-6).mean():.4f} kappa<= "
                     f"{np.max(kap[np.isfinite(kap)], initial=1.0):.1f}")
        bad = np.nonzero(~np.isfinite(e))[0]
        assert bad.size == 0, (NAMES[q], "non-finite output rows", bad[:5])
        bad = np.nonzero(~(e <= k * S[:, q]))[0]
        assert bad.size == 0, (NAMES[q], "above k*S", bad[:5], e[bad[:5]], S[bad[:5], q])
        if plain is not None:
            bad = np.nonzero(nz & ~(e <= plain * nr))[0]
            assert bad.size == 0, (NAMES[q], "above plain", bad[:5], rel[bad[:5]])
    print(" | ".join(lines), flush=True)
    return worst


def cpu(t):
    if hasattr(t, "detach"):
        return t.detach().cpu().numpy()
    return np.asarray(t)


def plummer_inputs(n, seed):
    """Plummer positions and velocities and the smooth-model acceleration as
    the sources' acceleration (kernel-level input for the snap term)."""
    m, x, v = ics.plummer(n, seed)
    return m, x, v, ics.plummer_mean_acc(x)


def gpu_system(m, x, v, a, eps, precision, **kw):
    """A GPU system whose stored state is exactly (x, v, a) at t = 0."""
    from paper_1207_2367_amd import System
    s = System(m, x, v, eps, precision=precision, **kw)
    n = m.shape[0]
    s.set_state(x=x, v=v, a=a, t=np.zeros(n), dt=np.full(n, 1.0 / 16))
    return s


def force(system, idx):
    """nbody_force into NaN-filled outputs (so an output the kernel fails to
    write cannot pass on stale memory)."""
    na = len(idx)
    out = [torch.full((na, 3), float("nan"), dtype=torch.float64, device="cuda") for _ in range(3)]
    out.append(torch.full((na,), float("nan"), dtype=torch.float64, device="cuda"))
    return system.force(idx, out=out)


def log_case(**kw):
    print("CASE " + " ".join(f"{k}={v}" for k, v in kw.items()), flush=True)


def sync():
    torch.cuda.synchronize()
