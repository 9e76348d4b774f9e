"""The GPU parity harness itself, on the CPU: check_force must fail on a
non-finite output, on a wrong value where the reference is zero (a one-body
cluster) and on an error just above its bound, and pass the oracle's own
values.  Outputs here are built on the host from oracle results; nothing
runs on a GPU."""
import numpy as np
import pytest

import ics
import oracle
from gpu_helpers import FORCE_TOL, check_force, term_sums

EPS = 1e-4


@pytest.fixture(scope="module")
def case():
    # two clusters: a 300-body sphere and a one-body cluster (zero force,
    # zero potential once the self term is removed)
    m, x, v = ics.plummer(301, 11)
    a = ics.plummer_mean_acc(x)
    idx = np.array([0, 5, 17, 120, 299, 300])
    ref = [np.zeros((idx.size, 3)) for _ in range(3)] + [np.zeros(idx.size)]
    S = np.zeros((idx.size, 4))
    for sel, (j0, j1) in ((idx < 300, (0, 300)), (idx == 300, (300, 301))):
        r = oracle.force(m, x, v, a, EPS, idx[sel], (j0, j1))
        S[sel] = term_sums(m, x, v, a, EPS, idx[sel], (j0, j1))
        for q in range(4):
            ref[q][sel] = r[q]
    return ref, S


def _copy(ref):
    return [q.copy() for q in ref]


def test_reference_rows_are_as_expected(case):
    ref, S = case
    assert np.all(ref[0][-1] == 0) and ref[3][-1] == 0 and np.all(S[-1, :3] == 0)
    assert S[-1, 3] > 0          # the removed self term sets the potential's scale
    assert np.all(S[:-1] > 0)


@pytest.mark.parametrize("prec", [0, 1, 2])
def test_exact_values_pass(case, prec):
    ref, S = case
    check_force(FORCE_TOL[prec], _copy(ref), ref, S)


@pytest.mark.parametrize("bad", [np.nan, np.inf, -np.inf])
@pytest.mark.parametrize("q", [0, 1, 2, 3])
@pytest.mark.parametrize("row", [1, 5])
def test_non_finite_fails(case, bad, q, row):
    ref, S = case
    got = _copy(ref)
    if q < 3:
        got[q][row, 1] = bad
    else:
        got[q][row] = bad
    with pytest.raises(AssertionError):
        check_force(FORCE_TOL[0], got, ref, S)


def test_all_nan_fails(case):
    ref, S = case
    got = [np.full_like(q, np.nan) for q in ref]
    with pytest.raises(AssertionError):
        check_force(FORCE_TOL[1], got, ref, S)


@pytest.mark.parametrize("q", [0, 1, 2, 3])
def test_wrong_value_on_zero_reference_fails(case, q):
    """The one-body cluster's reference is exactly zero (a, da, d2a) or
    zero after the self term (potential): a wrong value there fails."""
    ref, S = case
    got = _copy(ref)
    if q < 3:
        got[q][-1] = [1e-3, 0.0, 0.0]
    else:
        got[q][-1] = 1e-3
    with pytest.raises(AssertionError):
        check_force(FORCE_TOL[2], got, ref, S)


@pytest.mark.parametrize("prec", [0, 1, 2])
@pytest.mark.parametrize("q", [0, 1, 2])
def test_error_at_the_bound(case, prec, q):
    """An error of 0.9 of the row's bound passes, 1.1 of it fails."""
    ref, S = case
    k, plain = FORCE_TOL[prec][q]
    row = 2
    r = ref[q][row]
    bound = k * S[row, q]
    if plain is not None:
        bound = min(bound, plain * np.linalg.norm(r))
    u = np.array([0.6, 0.0, 0.8])
    for f, ok in ((0.9, True), (1.1, False)):
        got = _copy(ref)
        got[q][row] = r + f * bound * u
        if ok:
            check_force(FORCE_TOL[prec], got, ref, S)
        else:
            with pytest.raises(AssertionError):
                check_force(FORCE_TOL[prec], got, ref, S)


def test_shape_mismatch_fails(case):
    ref, S = case
    got = _copy(ref)
    got[0] = got[0][:-1]
    with pytest.raises(AssertionError):
        check_force(FORCE_TOL[0], got, ref, S)
