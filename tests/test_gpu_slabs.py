"""GPU parity of products computed in k-slabs under a workspace limit,
through the C ABI.

A product is the sum of its m outer products (eq. (1)) and the sketch is
linear, so a product split into consecutive k-slabs, each sketched with the
same hash functions and added in float64, must match the oracle to the same
float32 tolerance as the unsplit product, and the unsplit one again once the
default limit is restored (the same launches in the same order; only the
diagonal's float64 atomic adds may round in another order).
"""
import sys

import numpy as np
import pytest
import scipy.sparse as sps

from oracle import cmm_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(cmm):
    c = cmm.Context(0)
    yield c
    c.set_workspace_limit(0)
    c.close()


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _check_oracle(c, c_ref):
    for t in range(c_ref.shape[0]):
        nrm = np.linalg.norm(c_ref[t])
        assert nrm > 0
        rel = np.linalg.norm(c[t] - c_ref[t]) / nrm
        assert rel <= REL_TOL, (t, rel)


# (dtype, n, m, b, d, limit bytes): limits from a few MB (tens of slabs) down
# to one byte (one k per slab)
CASES = [
    ("f32", 600, 500, 4096, 5, 8 << 20),
    ("bf16", 300, 257, 1 << 14, 3, 24 << 20),
    ("fp8", 400, 333, 2048, 7, 6 << 20),
    ("f32", 50, 23, 256, 3, 1),
]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}_n{c[1]}_m{c[2]}_b{c[3]}_d{c[4]}_lim{c[5]}" for c in CASES])
def test_slabbed_product_matches_oracle_and_unsplit(cmm, ctx, case):
    dtype, n, m, b, d, limit = case
    _say(f"case: k-slabs {case}")
    w = W.covariance_workload("slabs", n, m, 4, 0.9, b, d, 8, dtype, 31 + n, 77 + m)
    At = _dev(w.At_store)
    B = At.clone()
    sA = _dev(w.scaleA) if w.scaleA is not None else None
    sB = sA.clone() if sA is not None else None

    def product():
        return cmm.sketch_product(ctx, At, B, b, d, seed=w.seed, dtype=dtype, scaleA=sA, scaleB=sB,
                                  subtract_diag=True)
    whole = product().c()
    ctx.set_workspace_limit(limit)
    try:
        sk = product()
        split = sk.c()
        oi, oj, ov = sk.topk(8, "upper")
    finally:
        ctx.set_workspace_limit(0)
    Aq, Bq = W.dequantised(w)
    c_ref, tabs, _ = O.run(Aq, Bq, b, d, w.seed, subtract_diag=True)
    _check_oracle(split, c_ref)
    _check_oracle(whole, c_ref)
    assert np.all(oi < oj)
    err = np.abs(split - c_ref).max()
    assert np.abs(ov - O.decode(c_ref, tabs, oi, oj)).max() <= err + 1e-6 * np.abs(c_ref).max()
    # default limit restored: the unsplit launches again (equal but for the
    # order of the diagonal's float64 atomic adds)
    again = product().c()
    assert np.abs(again - whole).max() <= 1e-12 * np.abs(whole).max()


def test_slabbed_strided_operands(cmm, ctx):
    """Operands with leading dimensions above n: a slab starts k0 * ld
    elements in."""
    _say("case: k-slabs over strided operands")
    n1, m, n3, b, d = 200, 150, 170, 2048, 3
    g = np.random.default_rng(5)
    Abig = g.standard_normal((m, n1 + 37)).astype(np.float32)
    Bbig = g.standard_normal((m, n3 + 11)).astype(np.float32)
    dA, dB = _dev(Abig), _dev(Bbig)
    At, Bv = dA[:, :n1], dB[:, :n3]
    assert At.stride(0) == n1 + 37 and Bv.stride(0) == n3 + 11
    ctx.set_workspace_limit(4 << 20)
    try:
        split = cmm.sketch_product(ctx, At, Bv, b, d, seed=9).c()
    finally:
        ctx.set_workspace_limit(0)
    c_ref, _, _ = O.run(Abig[:, :n1].astype(np.float64).T, Bbig[:, :n3].astype(np.float64), b, d, 9)
    _check_oracle(split, c_ref)


def test_slabbed_sparse_operands(cmm, ctx):
    """Sparse operands: a slab's column / row offsets start at k0."""
    _say("case: k-slabs over sparse operands")
    n1, m, n3, b, d = 400, 300, 350, 4096, 5
    A = sps.random(n1, m, density=0.02, format="csc", random_state=11, dtype=np.float64)
    Bs = sps.random(m, n3, density=0.02, format="csr", random_state=12, dtype=np.float64)
    A.data = A.data.astype(np.float32).astype(np.float64) - 0.5
    Bs.data = Bs.data.astype(np.float32).astype(np.float64) - 0.5

    def parts(M):
        return (_dev(M.indptr.astype(np.int64)), _dev(M.indices.astype(np.int32)),
                _dev(M.data.astype(np.float32)))
    pa, pb = parts(A), parts(Bs)
    ctx.set_workspace_limit(3 << 20)
    try:
        split = cmm.sketch_product_sparse(ctx, *pa, *pb, n1, m, n3, b, d, seed=13).c()
    finally:
        ctx.set_workspace_limit(0)
    c_ref, _, _ = O.run(A.toarray(), Bs.toarray(), b, d, 13)
    _check_oracle(split, c_ref)


def test_negative_limit_rejected(cmm, ctx):
    _say("case: negative workspace limit")
    with pytest.raises(cmm.CmmError) as e:
        ctx.set_workspace_limit(-1)
    assert e.value.code == cmm.CMM_EINVAL
