"""CPU checks of the threaded oracle runs and the comparison rules the
full-size GPU tests use (tests/oracle_runs.py): the threaded sketch equals
the oracle's single pass, the block-by-block top-K equals a full decode and
sort, and the band rule accepts the oracle's own answer, any answer that
swaps entries inside the band, and rejects a set that drops a sure entry or
holds an entry below the band."""
import numpy as np
import pytest

from oracle import cmm_oracle as O
import oracle_runs as R


def _product(n, m, seed):
    g = np.random.default_rng(seed)
    X = g.standard_normal((m, n))
    return X.T.copy(), X


def test_threaded_sketch_equals_oracle_run():
    A, B = _product(150, 40, 1)
    c_ref, tabs, _ = O.run(A, B, 512, 5, 77, subtract_diag=True)
    c, AB = R.sketch(A, B, tabs, 512, subtract_diag=True)
    np.testing.assert_allclose(c, c_ref, rtol=0, atol=1e-9 * np.abs(c_ref).max())
    R.check_sketch(c, c_ref)


def test_check_sketch_rejects_a_large_entry_error():
    A, B = _product(60, 20, 2)
    c_ref, tabs, _ = O.run(A, B, 128, 3, 5)
    bad = c_ref.copy()
    bad[1, 7] += 1e-3 * np.abs(c_ref[1]).max()
    with pytest.raises(AssertionError):
        R.check_sketch(bad, c_ref)


@pytest.mark.parametrize("rows_per_block", [1, 7, 64, 1000])
def test_blockwise_topk_equals_full_decode(rows_per_block):
    A, B = _product(90, 30, 3)
    c_ref, tabs, _ = O.run(A, B, 256, 3, 9, subtract_diag=True)
    i, j = O.candidates("upper", 90, 90)
    lin_full, val_full = O.topk(O.decode(c_ref, tabs, i, j), i * 90 + j, 25)
    bi, bj, bv = R.topk_upper(c_ref, tabs, 90, 25, rows_per_block=rows_per_block)
    assert (bi * 90 + bj).tolist() == lin_full.tolist()
    assert bv.tolist() == val_full.tolist()


def test_band_rule():
    A, B = _product(80, 30, 4)
    c_ref, tabs, _ = O.run(A, B, 128, 1, 11, subtract_diag=True)   # d = 1: many ties
    K = 10
    ri, rj, rv = R.topk_upper(c_ref, tabs, 80, K)
    tau = abs(rv[-1])
    dec = lambda i, j: O.decode(c_ref, tabs, i, j)
    delta = 1e-9 * np.abs(c_ref).max()
    R.band_check(ri, rj, rv, ri, rj, rv, tau, delta, dec)
    # a wider band accepts swapping the last entry for another one inside it
    i, j = O.candidates("upper", 80, 80)
    v = dec(i, j)
    order = np.lexsort((i * 80 + j, -np.abs(v)))
    nxt = order[K]
    wide = 2 * (tau - abs(v[nxt])) + 1e-12
    gi = np.append(ri[:-1], i[nxt]); gj = np.append(rj[:-1], j[nxt]); gv = np.append(rv[:-1], v[nxt])
    R.band_check(gi, gj, gv, ri, rj, rv, tau, max(wide, delta), dec)
    # dropping the largest entry, or returning one far below the band, fails
    far = order[-1]
    gi = np.append(ri[1:], i[far]); gj = np.append(rj[1:], j[far]); gv = np.append(rv[1:], v[far])
    with pytest.raises(AssertionError):
        R.band_check(gi, gj, gv, ri, rj, rv, tau, delta, dec)
    # a returned value off by more than half the band fails
    with pytest.raises(AssertionError):
        R.band_check(ri, rj, rv + 0.51 * max(wide, delta) + 1e-6, ri, rj, rv, tau, max(wide, delta), dec)
