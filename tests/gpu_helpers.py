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
    FP64 pair terms in numpy: a test-side diagnostic that scales the
    tolerance (an evaluation whose sub-terms carry relative error e has a
    sum error <= e kappa)."""
    j0, j1 = (0, m.shape[0]) if j_range is None else j_range
    out = np.zeros((len(idx), 4))
    xs, vs, as_, ms = x[j0:j1], v[j0:j1], a[j0:j1], m[j0:j1]
    for k, i in enumerate(idx):
        r, w, q = xs - x[i], vs - v[i], as_ - a[i]
        s2 = (r * r).sum(1) + eps * eps
        keep = np.arange(j0, j1) != i
        rinv = np.where(keep, 1.0 / np.sqrt(np.where(s2 > 0, s2, 1.0)), 0.0)
        mr3 = ms * rinv ** 3
        al = (r * w).sum(1) * rinv ** 2
        be = ((w * w).sum(1) + (r * q).sum(1)) * rinv ** 2 + al * al
        A = mr3[:, None] * r
        J = mr3[:, None] * w - 3 * al[:, None] * A
        S = mr3[:, None] * q - 6 * al[:, None] * J - 3 * be[:, None] * A
        nA = np.linalg.norm(A, axis=1)
        # magnitudes of the sub-terms each pair term is built from
        nJ = mr3 * np.linalg.norm(w, axis=1) + 3 * np.abs(al) * nA
        nS = (mr3 * np.linalg.norm(q, axis=1) + 6 * np.abs(al) * np.linalg.norm(J, axis=1)
              + 3 * np.abs(be) * nA)
        for c, (T, nT) in enumerate(((A, nA), (J, nJ), (S, nS))):
            out[k, c] = nT.sum() / max(np.linalg.norm(T.sum(0)), 1e-300)
        # the kernels sum the potential over every source including j = i and
        # then remove the self term -m_i / eps, whose size sets the rounding
        phi = np.abs((ms * rinv).sum())
        out[k, 3] = 1.0 + (m[i] / eps / phi if eps > 0 and j0 <= i < j1 else 0.0)
    return out


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
