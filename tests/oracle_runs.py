"""Oracle runs over products too large for a single-threaded pass.

Test infrastructure: the arithmetic is the oracle's own functions
(``oracle.cmm_oracle``); this module only splits their work over host
threads (numpy releases the interpreter lock inside them) and applies the
comparison rules the tests share.  It computes nothing of the method itself.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

from oracle import cmm_oracle as O

THREADS = max(1, min(16, os.cpu_count() or 1))


def _rep(tabs, t):
    """Hash tables of repetition t alone, in the (d, n) shape the oracle takes."""
    return tuple(x[t:t + 1] for x in tabs)


def sketch(A, B, tabs, b, subtract_diag=False):
    """(c, AB): the definition-form sketch of AB (O.bin_product on the float64
    product) for every repetition, one thread per repetition, and the
    diagonal removed with O.subtract_diagonal when asked."""
    AB = np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    d = tabs[0].shape[0]
    with ThreadPoolExecutor(min(THREADS, d)) as ex:
        rows = list(ex.map(lambda t: O.bin_product(AB, _rep(tabs, t), b)[0], range(d)))
    c = np.array(rows)
    if subtract_diag:
        c = O.subtract_diagonal(c, np.diag(AB).copy(), tabs, b)
    return c, AB


def check_sketch(c_gpu, c_ref, rel_tol=1e-5):
    """Per repetition: relative L2 error <= rel_tol and the largest entry
    error <= rel_tol * max |c_t| (both the scope's float32 budget).  Returns
    (worst rel. L2, worst max|dc| / max|c_t|)."""
    worst_l2 = worst_inf = 0.0
    for t in range(c_ref.shape[0]):
        dc = c_gpu[t] - c_ref[t]
        l2 = float(np.linalg.norm(dc) / np.linalg.norm(c_ref[t]))
        inf = float(np.abs(dc).max() / np.abs(c_ref[t]).max())
        assert l2 <= rel_tol, (t, l2)
        assert inf <= rel_tol, (t, inf)
        worst_l2, worst_inf = max(worst_l2, l2), max(worst_inf, inf)
    return worst_l2, worst_inf


def decode_band(c_gpu, c_ref):
    """Half-width of the tolerance band of a top-K comparison: twice the
    largest error of the float32 sketch the GPU decodes from, plus a float32
    rounding allowance.  The median is 1-Lipschitz in the max norm, so every
    GPU estimate is within half of this of the oracle's."""
    c32 = np.asarray(c_gpu, dtype=np.float32).astype(np.float64)
    return 2.0 * (np.abs(c32 - c_ref).max() + 1e-6 * np.abs(c_ref).max())


def topk_upper(c_ref, tabs, n, K, rows_per_block=256):
    """The oracle's top-K over i < j of an n x n product, decoded block of
    rows by block of rows so that the n(n-1)/2 estimates are never held at
    once: every block keeps its entries at or above its own K-th magnitude
    (ties included), and the kept ones are ranked by (-|C|, i n + j).
    Returns (i, j, values) of the first K and the candidate list."""
    b = c_ref.shape[1]

    def block(r0):
        r1 = min(n, r0 + rows_per_block)
        ii = np.repeat(np.arange(r0, r1), n)
        jj = np.tile(np.arange(n), r1 - r0)
        keep = ii < jj
        ii, jj = ii[keep], jj[keep]
        if ii.size == 0:
            return ii, jj, np.zeros(0)
        v = O.decode(c_ref, tabs, ii, jj)
        if v.size > K:
            kth = np.partition(np.abs(v), v.size - K)[v.size - K]
            sel = np.abs(v) >= kth
            ii, jj, v = ii[sel], jj[sel], v[sel]
        return ii, jj, v
    with ThreadPoolExecutor(THREADS) as ex:
        parts = list(ex.map(block, range(0, n, rows_per_block)))
    ii = np.concatenate([p[0] for p in parts]); jj = np.concatenate([p[1] for p in parts])
    vv = np.concatenate([p[2] for p in parts])
    lin = ii * n + jj
    sel_lin, sel_val = O.topk(vv, lin, K)
    return sel_lin // n, sel_lin % n, sel_val


def band_check(got_i, got_j, got_v, ref_i, ref_j, ref_v, tau, delta, decode_ref):
    """The rule for several correct answers near the K-th magnitude tau: every
    oracle entry above tau + delta is returned, every returned entry's oracle
    magnitude is at least tau - delta, and every returned value is within
    delta/2 of the oracle's decode of the same position (decode_ref(i, j))."""
    got = set(zip(np.asarray(got_i).tolist(), np.asarray(got_j).tolist()))
    sure = {(int(a), int(c)) for a, c, v in zip(ref_i, ref_j, ref_v) if abs(v) > tau + delta}
    assert sure <= got, sorted(sure - got)[:5]
    ref_at_got = decode_ref(np.asarray(got_i), np.asarray(got_j))
    assert np.all(np.abs(ref_at_got) >= tau - delta), float(np.abs(ref_at_got).min())
    err = float(np.abs(np.asarray(got_v, dtype=np.float64) - ref_at_got).max())
    assert err <= delta / 2 + 1e-12 * max(1.0, abs(tau)), (err, delta)
    return err
