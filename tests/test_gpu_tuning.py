"""The autotuner's table through the C ABI: a table measured once and
stored (nbody_get_tuning) gives another context the same launch shapes and
bitwise the same evaluation (nbody_set_tuning); the Python cache file does
the same across contexts; invalid tables are refused."""
import numpy as np
import pytest

import ics
from gpu_helpers import cpu, force, gpu_system, log_case, plummer_inputs

pytestmark = pytest.mark.gpu

EPS = 1e-4


def test_tuning_table_round_trip(tmp_path):
    from paper_1207_2367_amd import NBodyError
    n = 4096
    m, x, v, a = plummer_inputs(n, 31)
    s1 = gpu_system(m, x, v, a, EPS, 0)
    cache = str(tmp_path / "tune.json")
    s1.autotune(40.0, cache=cache)
    table = s1.get_tuning()
    assert len(table) == 13   # sizes 1, 2, ..., 4096
    s2 = gpu_system(m, x, v, a, EPS, 0)
    s2.autotune(40.0, cache=cache)    # loaded, not measured
    assert s2.get_tuning() == table
    for na in (1, 5, 64, 700, 4096):
        log_case(test="tuning", n_act=na)
        assert s1.get_launch(na) == s2.get_launch(na)
        idx = ics.active_subset(n, na, na)
        r1 = [cpu(q).copy() for q in force(s1, idx)]
        r2 = [cpu(q).copy() for q in force(s2, idx)]
        for p, q in zip(r1, r2):
            assert np.array_equal(p, q)
    bad = list(table)
    bad[3] = (8, 4, 16, 2)       # two particles per lane group need lanes_per_i <= 4
    with pytest.raises(NBodyError):
        s2.set_tuning(bad)
    assert s2.get_tuning() == table
    s2.set_tuning([])
    assert s2.get_tuning() == []
    s1.close()
    s2.close()
