"""GPU parity of the non-zero count by doubling search (Section 5.1)
through the C ABI: the returned b is an integer decided by zero counts, and
equals the oracle's on the same float32 operands (every bucket is far from
the zero threshold in these cases); it brackets the true count."""
import sys

import numpy as np
import pytest

from oracle import cmm_oracle as O

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
    """AB = S exactly up to rounding (A of full row rank, m >= n1)."""
    g = np.random.default_rng(seed)
    A = g.standard_normal((n1, m))
    S = np.zeros((n1, n3))
    pos = g.choice(n1 * n3, nnz, replace=False)
    S.flat[pos] = g.choice([-1.0, 1.0], nnz) * g.uniform(1.0, 2.0, nnz)
    return A, np.linalg.pinv(A) @ S


CASES = [(128, 160, 128, 500, 5), (200, 256, 220, 5, 9), (100, 150, 90, 60, 7)]


@pytest.mark.parametrize("case", CASES, ids=[f"{c[0]}x{c[1]}x{c[2]}_nnz{c[3]}_d{c[4]}" for c in CASES])
def test_nnz_matches_oracle_and_brackets(cmm, ctx, case):
    n1, m, n3, nnz, d = case
    _say(f"case: nnz estimate {case}")
    A, B = _sparse(n1, m, n3, nnz, nnz + n1)
    At32 = np.ascontiguousarray(A.T).astype(np.float32)
    B32 = B.astype(np.float32)
    b, zeros = cmm.estimate_nnz(ctx, _dev(At32), _dev(B32), d, seed=11)
    bo, zo = O.estimate_nnz(At32.astype(np.float64).T, B32.astype(np.float64), d, 11)
    assert b == bo, (b, bo)
    assert np.abs(zeros - zo).max() <= 1
    assert nnz <= b <= 10 * max(nnz, 2)


def test_nnz_zero_and_dense_products(cmm, ctx):
    _say("case: nnz estimate of a zero and of a dense product")
    g = np.random.default_rng(1)
    A = g.standard_normal((40, 60)).astype(np.float32)      # stored k-major: m = 40, n1 = 60
    Z = np.zeros((40, 50), np.float32)
    b, _ = cmm.estimate_nnz(ctx, _dev(A), _dev(Z), 3, seed=3)
    assert b == 16
    Bd = g.standard_normal((40, 50)).astype(np.float32)
    b, _ = cmm.estimate_nnz(ctx, _dev(A), _dev(Bd), 5, seed=3)
    bo, _ = O.estimate_nnz(A.astype(np.float64).T, Bd.astype(np.float64), 5, 3)
    assert b == bo and 3000 <= b <= 30000
