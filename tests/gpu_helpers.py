"""Shared helpers of the GPU parity tests (not collected by pytest)."""
import numpy as np
import torch

import ics


def rel_err_rows(got, ref):
    """Per-particle relative error ||got_i - ref_i|| / ||ref_i|| (rows)."""
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    if got.ndim == 1:
        return np.abs(got - ref) / np.abs(ref)
    return np.linalg.norm(got - ref, axis=1) / np.linalg.norm(ref, axis=1)


def kappa(m, x, v, a, eps, idx, j_range=None):
    """Condition number of each evaluated sum, kappa_i(Q) = sum_j |Q_ij| /
    |sum_j Q_ij| for Q = a, da, d2a, potential, where |Q_ij| adds the
    magnitudes of the sub-terms a pair term is built from (m v / r^3 and
    3 alpha A for the jerk; m a / r^3, 6 alpha J and 3 beta A for the snap).
    FP64 pair terms (torch on the CPU, multithreaded): a test-side
    diagnostic that scales the tolerance (an evaluation whose sub-terms carry
    relative error e has a sum error <= e kappa)."""
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
        S = mr3[:, None] * q - 6 * al[:, None] * J - 3 * be[:, None] * A
        nA = A.norm(dim=1)
        # magnitudes of the sub-terms each pair term is built from
        nJ = mr3 * w.norm(dim=1) + 3 * al.abs() * nA
        nS = mr3 * q.norm(dim=1) + 6 * al.abs() * J.norm(dim=1) + 3 * be.abs() * nA
        for c, (T, nT) in enumerate(((A, nA), (J, nJ), (S, nS))):
            out[k, c] = float(nT.sum()) / max(float(T.sum(0).norm()), 1e-300)
        # the kernels sum the potential over every source including j = i and
        # then remove the self term -m_i / eps, whose size sets the rounding
        phi = abs(float((ms * rinv).sum()))
        out[k, 3] = 1.0 + (m[i] / eps / phi if eps > 0 and j0 <= i < j1 else 0.0)
    return out


# precision -> tolerance factors for (a, da, d2a, potential); the reasoning
# is in the docstring of test_gpu_force.py
FORCE_TOL = {0: (1e-11, 1e-6, 2e-6, 1e-11), 1: (1e-12, 1e-12, 1e-11, 1e-12),
             2: (1e-6, 1e-6, 2e-6, 1e-6)}


def check_force(tol, got, ref, kap):
    """Per-particle relative errors of (a, da, d2a, phi) within tol * kappa;
    prints the plain max / p99 errors and the fraction within 1e-6."""
    ga, gj, gs, gp = (cpu(q) for q in got)
    ra, rj, rs, rp = ref
    errs = [rel_err_rows(ga, ra), rel_err_rows(gj, rj), rel_err_rows(gs, rs),
            rel_err_rows(gp, rp)]
    worst = [float(e.max()) for e in errs]
    print("max rel err a %.2e da %.2e d2a %.2e pot %.2e" % tuple(worst), flush=True)
    print("p99 %s | within 1e-6: %s | max kappa %s" % (
        [f"{np.percentile(e, 99):.1e}" for e in errs],
        [f"{(e <= 1e-6).mean():.4f}" for e in errs],
        [f"{k:.1f}" for k in kap.max(0)]), flush=True)
    for q, e in enumerate(errs):
        bound = tol[q] * kap[:, q]
        bad = np.nonzero(e > bound)[0]
        assert bad.size == 0, (q, bad[:5], e[bad[:5]], kap[bad[:5], q])
    return worst


def cpu(t):
    return t.detach().cpu().numpy()


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
