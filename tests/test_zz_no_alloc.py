"""The evaluation entry point that allocates nothing (nbody_force_noalloc:
sources from caller arrays, records and split partials in the library's
fixed per-GPU scratch) against the context entry point nbody_force on the
same inputs, two calls in a row (the second smaller, so the scratch holds
the first call's contents), in every precision."""
import numpy as np
import pytest
import torch

import ics
import oracle
from gpu_helpers import FORCE_TOL, check_force, cpu, gpu_system, log_case, plummer_inputs, term_sums

pytestmark = pytest.mark.gpu

EPS = 1e-4


@pytest.mark.parametrize("prec", [0, 1, 2], ids=["mixed", "fp64", "fp32pair"])
def test_noalloc_matches_context_entry_point(prec):
    from paper_1207_2367_amd import nbody
    for n, n_act, seed in ((5077, 333, 2002), (1200, 64, 7)):
        log_case(test="noalloc", prec=prec, n=n, n_act=n_act)
        m, x, v, a = plummer_inputs(n, seed)
        idx = ics.active_subset(n, n_act, seed + 1)
        s = gpu_system(m, x, v, a, EPS, prec)
        ctx_out = [cpu(q).copy() for q in s.force(idx)]
        torch.cuda.synchronize()
        s.close()
        out = [torch.full((n_act, 3), float("nan"), dtype=torch.float64, device="cuda")
               for _ in range(3)]
        out.append(torch.full((n_act,), float("nan"), dtype=torch.float64, device="cuda"))
        got = nbody.force_noalloc(m, x, v, a, EPS, idx, precision=prec, out=out)
        torch.cuda.synchronize()
        got = [cpu(q) for q in got]
        ref = oracle.force(m, x, v, a, EPS, idx)
        S = term_sums(m, x, v, a, EPS, idx)
        # to the parity bar against the oracle, and against the context entry
        # point: both evaluate the same records with the same kernels, so the
        # sums agree to FP64 rounding (FP32 sums of the snap: its k S bound)
        check_force(FORCE_TOL[prec], got, ref, S)
        k_snap = FORCE_TOL[prec][2][0]
        for q in range(4):
            g, c = np.asarray(got[q]), np.asarray(ctx_out[q])
            assert np.isfinite(g).all()
            d = np.abs(g - c) if g.ndim == 1 else np.linalg.norm(g - c, axis=1)
            if q == 2 or prec == 2:
                bound = 2 * FORCE_TOL[prec][q][0] * S[:, q]
            else:
                bound = 1e-12 * S[:, q]
            assert (d <= bound).all(), (q, d.max())


def test_noalloc_rejects_oversized_and_bad_arguments():
    from paper_1207_2367_amd import nbody
    lib = nbody.load()
    d = torch.zeros(8, dtype=torch.float64, device="cuda")
    i = torch.zeros(1, dtype=torch.int32, device="cuda")
    p = [d.data_ptr()] * 4
    # 2^20 sources do not fit the 64 MiB scratch in the mixed (68 B per
    # source) and FP64 (80 B) modes
    for prec in (0, 1):
        assert lib.nbody_force_noalloc(1 << 20, *p, 1e-4, prec, 1, i.data_ptr(), *p[:3], None,
                                       None) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *p, -1.0, 0, 1, i.data_ptr(), *p[:3], None,
                                   None) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *p, 1e-4, 7, 1, i.data_ptr(), *p[:3], None,
                                   None) == nbody.EINVAL
    assert lib.nbody_force_noalloc(4, *p, 1e-4, 0, 5, i.data_ptr(), *p[:3], None,
                                   None) == nbody.EINVAL
