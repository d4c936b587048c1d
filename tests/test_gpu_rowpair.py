"""GPU parity of the spectral step at every FFT row length, through the C ABI.

The spectral step of a product with R = b / C > 1 runs two kernels: the row
kernel for rows 1 .. R/2 - 1 and the pair kernel for rows 0 and R/2 (one
C-point FFT per side and k, then the real split).  Both are instantiated for
C = 2^4 .. 2^13; a stored tuning selects C, so every instantiation is run here
with R = 2 (the pair kernel alone), 4 and 16, and each sketch is compared with
the float64 oracle (rel. L2 1e-5 per repetition, the parity tolerance).
"""
import sys

import numpy as np
import pytest

from oracle import cmm_oracle as O

pytestmark = pytest.mark.gpu

REL_TOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(cmm):
    c = cmm.Context(0)
    yield c
    c.close()


CASES = [(L, R) for L in range(4, 14) for R in (2, 4, 16)]


@pytest.mark.parametrize("case", CASES, ids=[f"C2^{c[0]}_R{c[1]}" for c in CASES])
def test_row_length_and_pair(cmm, ctx, case):
    import torch
    L, R = case
    b = R << L
    n1, n3, m, d = 180, 150, 37, 3
    seed = 1000 * L + R
    _say(f"case: row length 2^{L}, R = {R}, b = {b}")
    g = np.random.default_rng(seed)
    At = g.standard_normal((m, n1)).astype(np.float32)
    B = g.standard_normal((m, n3)).astype(np.float32)
    ctx.set_tuning(n1, m, n3, b, d, "f32", (L, 16, 64))
    assert ctx.tuning(n1, m, n3, b, d, "f32")[0] == L
    sk = cmm.sketch_product(ctx, torch.from_numpy(At).cuda(), torch.from_numpy(B).cuda(), b, d, seed=seed)
    c = sk.c()
    sk.free()
    c_ref, _, _ = O.run(At.astype(np.float64).T, B.astype(np.float64), b, d, seed)
    for t in range(d):
        rel = np.linalg.norm(c[t] - c_ref[t]) / np.linalg.norm(c_ref[t])
        assert rel <= REL_TOL, (t, rel)


@pytest.mark.parametrize("L", [4, 9, 12])
def test_row_pair_with_diagonal(cmm, ctx, L):
    """The diagonal subtraction after a spectral step with the pair kernel."""
    import torch
    R = 4
    b = R << L
    n, m, d = 160, 41, 5
    seed = 77 + L
    _say(f"case: row length 2^{L}, R = {R}, diagonal subtracted")
    g = np.random.default_rng(seed)
    X = g.standard_normal((m, n)).astype(np.float32)
    ctx.set_tuning(n, m, n, b, d, "f32", (L, 32, 512))
    dX = torch.from_numpy(X).cuda()
    sk = cmm.sketch_product(ctx, dX, dX.clone(), b, d, seed=seed, subtract_diag=True)
    c = sk.c()
    sk.free()
    c_ref, _, _ = O.run(X.astype(np.float64).T, X.astype(np.float64), b, d, seed, subtract_diag=True)
    for t in range(d):
        rel = np.linalg.norm(c[t] - c_ref[t]) / np.linalg.norm(c_ref[t])
        assert rel <= REL_TOL, (t, rel)
