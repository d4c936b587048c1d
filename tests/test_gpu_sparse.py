"""GPU parity of the sparse-operand sketch (Corollary 8) through the C ABI.

The sparse path stages each column of A / row of B by scattering its
entries into a zeroed row and then runs the dense path unchanged, so its
sketch is bit-identical to the dense call on the densified matrices (the
diagonal removed too: both sum the diagonal over the same k-chunks in the
same order, and the subtraction adds exact fixed-point bucket sums), and
within the float32 tolerance of the oracle.
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sps

from oracle import cmm_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(cmm):
    c = cmm.Context(0)
    yield c
    c.close()


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _csr_parts(M):
    """(ptr int64, idx int32, val float32) device arrays of a scipy CSR/CSC."""
    return (_dev(M.indptr.astype(np.int64)), _dev(M.indices.astype(np.int32)),
            _dev(M.data.astype(np.float32)))


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("dens", [0.03, 0.0005])
def test_sparse_equals_dense_and_oracle(cmm, ctx, dens):
    _say(f"case: sparse operands density {dens}")
    n1, m, n3, b, d = 700, 300, 650, 4096, 5
    A = sps.random(n1, m, density=dens, format="csc", random_state=1, dtype=np.float64)
    B = sps.random(m, n3, density=dens, format="csr", random_state=2, dtype=np.float64)
    A.data = A.data.astype(np.float32).astype(np.float64) - 0.5
    B.data = B.data.astype(np.float32).astype(np.float64) - 0.5
    sk = cmm.sketch_product_sparse(ctx, *_csr_parts(A), *_csr_parts(B), n1, m, n3, b, d, seed=33)
    Ad = A.toarray(); Bd = B.toarray()
    dense = cmm.sketch_product(ctx, _dev(Ad.T.astype(np.float32)), _dev(Bd.astype(np.float32)), b, d,
                               seed=33)
    np.testing.assert_array_equal(sk.c(), dense.c())
    c_ref, _, _ = O.run(Ad, Bd, b, d, 33)
    for t in range(d):
        if np.linalg.norm(c_ref[t]) > 0:
            assert _rel(sk.c()[t], c_ref[t]) <= 1e-5


def test_sparse_covariance_zero_diagonal(cmm, ctx):
    _say("case: sparse covariance with the diagonal removed")
    n, m, b, d = 500, 400, 2048, 3
    X = sps.random(m, n, density=0.05, format="csr", random_state=7, dtype=np.float64)
    X.data = X.data.astype(np.float32).astype(np.float64) * 2 - 1
    # A = X^T by columns k is X by rows k: both operands are the CSR of X
    parts = _csr_parts(X)
    sk = cmm.sketch_product_sparse(ctx, *parts, *parts, n, m, n, b, d, seed=8, subtract_diag=True)
    Xd = X.toarray()
    dX = _dev(Xd.astype(np.float32))
    dense = cmm.sketch_product(ctx, dX, dX.clone(), b, d, seed=8, subtract_diag=True)
    cs, cd = sk.c(), dense.c()
    np.testing.assert_array_equal(cs, cd)
    c_ref, _, _ = O.run(Xd.T, Xd, b, d, 8, subtract_diag=True)
    for t in range(d):
        assert _rel(cs[t], c_ref[t]) <= 1e-5
    oi, oj, ov = sk.topk(10, "upper")
    assert np.all(oi < oj)


def test_sparse_empty_rows_and_empty_operand(cmm, ctx):
    _say("case: sparse operands with empty columns and an all-zero operand")
    n1, m, n3, b, d = 200, 64, 150, 1024, 3
    A = sps.random(n1, m, density=0.02, format="csc", random_state=3, dtype=np.float64)
    A = A.tolil(); A[:, 10:30] = 0; A = A.tocsc(); A.eliminate_zeros()
    A.data = A.data.astype(np.float32).astype(np.float64)
    B = sps.csr_matrix((m, n3), dtype=np.float64)          # no entries at all
    sk = cmm.sketch_product_sparse(ctx, *_csr_parts(A), *_csr_parts(B), n1, m, n3, b, d, seed=4)
    assert np.abs(sk.c()).max() == 0.0
    B2 = sps.random(m, n3, density=0.05, format="csr", random_state=5, dtype=np.float64)
    B2.data = B2.data.astype(np.float32).astype(np.float64)
    sk2 = cmm.sketch_product_sparse(ctx, *_csr_parts(A), *_csr_parts(B2), n1, m, n3, b, d, seed=4)
    c_ref, _, _ = O.run(A.toarray(), B2.toarray(), b, d, 4)
    for t in range(d):
        assert _rel(sk2.c()[t], c_ref[t]) <= 1e-5


def test_sparse_invalid_input_rejected(cmm, ctx):
    _say("case: sparse index out of range / decreasing offsets")
    m, n = 8, 16
    ptr = np.array([0, 1, 1, 2, 2, 3, 3, 4, 4], np.int64)
    idx = np.array([0, 5, 15, 3], np.int32)
    val = np.ones(4, np.float32)
    good = (_dev(ptr), _dev(idx), _dev(val))
    bad_idx = (_dev(ptr), _dev(np.array([0, 5, 16, 3], np.int32)), _dev(val))
    bad_ptr = (_dev(np.array([0, 2, 1, 2, 2, 3, 3, 4, 4], np.int64)), _dev(idx), _dev(val))
    cmm.sketch_product_sparse(ctx, *good, *good, n, m, n, 64, 2, seed=1).free()
    for badp in (bad_idx, bad_ptr):
        with pytest.raises(cmm.CmmError) as e:
            cmm.sketch_product_sparse(ctx, *badp, *good, n, m, n, 64, 2, seed=1)
        assert e.value.code == cmm.CMM_EINVAL
