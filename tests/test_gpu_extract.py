"""GPU parity of the sublinear extraction (Section 4, Figure 3) through the
C ABI, against the oracle's FINDSIGNIFICANTENTRIES on the same operands and
hash functions.

* Planted sparse products AB = S (B = pinv(A) S): the GPU returns exactly
  the oracle's set, which is exactly the support of S (every decision is far
  from delta/2).
* A noisy covariance product: decisions close to delta/2 may differ between
  the float32 GPU sketches and the float64 oracle, so the GPU set must
  contain every position the oracle decodes in more than d/2 + 1
  repetitions and only positions it decodes at least d/2 - 1 times.
"""
import sys

import numpy as np
import pytest

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


def _sparse(n1, m, n3, nnz, seed):
    g = np.random.default_rng(seed)
    A = g.standard_normal((n1, m))
    S = np.zeros((n1, n3))
    pos = g.choice(n1 * n3, nnz, replace=False)
    S.flat[pos] = g.choice([-1.0, 1.0], nnz) * g.uniform(1.0, 2.0, nnz)
    B = np.linalg.pinv(A) @ S
    return A, B, np.sort(pos)


SPARSE = [
    # (n1, m, n3, nnz, b, d, dtype)
    (300, 200, 250, 40, 4096, 7, "f32"),
    (128, 160, 128, 16, 1024, 5, "f32"),
    (200, 256, 200, 25, 2048, 9, "bf16"),
]


@pytest.mark.parametrize("case", SPARSE, ids=[f"{c[0]}x{c[1]}x{c[2]}_nnz{c[3]}_b{c[4]}_d{c[5]}_{c[6]}" for c in SPARSE])
def test_extract_sparse_product_exact(cmm, ctx, case):
    n1, m, n3, nnz, b, d, dtype = case
    _say(f"case: extraction of a planted sparse product {case}")
    A, B, support = _sparse(n1, m, n3, nnz, n1 + b)
    At32 = np.ascontiguousarray(A.T).astype(np.float32)
    B32 = B.astype(np.float32)
    if dtype == "bf16":
        sa, sb = W.bf16_encode(At32), W.bf16_encode(B32)
        Aq = (sa.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64).T
        Bq = (sb.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    else:
        sa, sb = At32, B32
        Aq, Bq = At32.astype(np.float64).T, B32.astype(np.float64)
    gi, gj, total, sk = cmm.find_significant(ctx, _dev(sa), _dev(sb), b, d, 0.5, seed=71,
                                             dtype=dtype, want_sketch=True)
    tabs = O.hash_tables(O.hash_params(71, d), n1, n3, b)
    cr, cc = O.masked_sketches(Aq, Bq, tabs, b)
    kept, _ = O.find_significant(cr, cc, n1, n3, 0.5)
    np.testing.assert_array_equal(np.sort(gi * n3 + gj), kept)
    np.testing.assert_array_equal(kept, support)
    assert total == len(kept)
    # the sketch of AB handed back is the ordinary sketch product
    alone = cmm.sketch_product(ctx, _dev(sa), _dev(sb), b, d, seed=71, dtype=dtype).c()
    np.testing.assert_array_equal(sk.c(), alone)


def test_extract_sparse_with_zero_diagonal(cmm, ctx):
    """Square product with the diagonal removed (CMM_SUBTRACT_DIAG): the
    planted diagonal entries are not reported, the off-diagonal ones are."""
    _say("case: extraction with the diagonal removed")
    n, m, b, d = 150, 180, 2048, 7
    g = np.random.default_rng(12)
    A = g.standard_normal((n, m))
    S = np.zeros((n, n))
    off = [(3, 40), (77, 12), (100, 149), (5, 6), (140, 2)]
    for (i, j) in off:
        S[i, j] = 1.5
    for i in (0, 50, 99):
        S[i, i] = 2.0
    B = np.linalg.pinv(A) @ S
    At32 = np.ascontiguousarray(A.T).astype(np.float32)
    B32 = B.astype(np.float32)
    gi, gj, total = cmm.find_significant(ctx, _dev(At32), _dev(B32), b, d, 0.5, seed=9,
                                         subtract_diag=True)
    tabs = O.hash_tables(O.hash_params(9, d), n, n, b)
    cr, cc = O.masked_sketches(At32.astype(np.float64).T, B32.astype(np.float64), tabs, b,
                               subtract_diag=True)
    kept, _ = O.find_significant(cr, cc, n, n, 0.5)
    np.testing.assert_array_equal(np.sort(gi * n + gj), kept)
    np.testing.assert_array_equal(kept, sorted(i * n + j for (i, j) in off))


def test_extract_noisy_covariance_band(cmm, ctx):
    _say("case: extraction on a noisy covariance product")
    X, pairs, _ = W.covariance_observations(256, 512, 12, 0.95, 21)
    X = X.astype(np.float32)
    b, d = 4096, 7
    A, B = X.astype(np.float64).T, X.astype(np.float64)
    AB = A @ B
    np.fill_diagonal(AB, 0.0)
    delta = 6.0 * np.sqrt((AB ** 2).sum() / b)
    gi, gj, total = cmm.find_significant(ctx, _dev(X), _dev(X.copy()), b, d, delta, seed=5,
                                         subtract_diag=True)
    tabs = O.hash_tables(O.hash_params(5, d), 256, 256, b)
    cr, cc = O.masked_sketches(A, B, tabs, b, subtract_diag=True)
    kept, counts = O.find_significant(cr, cc, 256, 256, delta)
    got = set((gi * 256 + gj).tolist())
    sure = {k for k, v in counts.items() if 2 * v >= d + 2}
    maybe = {k for k, v in counts.items() if 2 * v >= d - 2}
    assert sure <= got, sorted(sure - got)[:5]
    assert got <= maybe, sorted(got - maybe)[:5]
    planted = {int(p) * 256 + int(q) for p, q in pairs} | {int(q) * 256 + int(p) for p, q in pairs}
    _say(f"  returned {len(got)} positions; oracle {len(kept)}; identical: {got == set(kept.tolist())}; "
         f"planted found {len(got & planted)} of {len(planted)}")


def test_extract_errors_and_cap(cmm, ctx):
    _say("case: extraction argument errors and the output cap")
    A, B, support = _sparse(64, 80, 64, 10, 3)
    dA = _dev(np.ascontiguousarray(A.T).astype(np.float32))
    dB = _dev(B.astype(np.float32))
    with pytest.raises(cmm.CmmError) as e:
        cmm.find_significant(ctx, dA, dB, 512, 5, 0.0)
    assert e.value.code == cmm.CMM_EINVAL
    gi, gj, total = cmm.find_significant(ctx, dA, dB, 512, 5, 0.5, seed=2, cap=4)
    assert total == 10 and len(gi) == 4
    assert set((gi * 64 + gj).tolist()) <= set(support.tolist())
