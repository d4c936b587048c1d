"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Tolerances
----------
* hashes, bucket indices: bit-exact.
* sketch c (float32 operands, float32 FFT, float64 cross-k sum and inverse
  FFT): per repetition ||c_gpu - c_oracle||_2 / ||c_oracle||_2 <= 1e-5.
* estimates: the median is 1-Lipschitz in the max-norm, so
  |C_gpu - C_oracle| <= max|c32_gpu - c_oracle| (+ float32 rounding).
* top-K: entries whose oracle magnitude lies outside the band
  [tau_K - delta, tau_K + delta] must agree (tau_K the K-th oracle
  magnitude, delta twice the largest estimate difference); inside the band
  any choice is valid and is only checked for being a correct estimate.
"""
import math
import sys

import numpy as np
import pytest

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
    c.close()


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


def _rel_l2(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _rand_problem(n1, m, n3, seed):
    g = np.random.default_rng(seed)
    At = g.standard_normal((m, n1)).astype(np.float32)
    B = g.standard_normal((m, n3)).astype(np.float32)
    return At, B


def _oracle_c(At, B, b, d, seed, subtract_diag=False):
    A = At.astype(np.float64).T
    Bf = B.astype(np.float64)
    c, tabs, AB = O.run(A, Bf, b, d, seed, subtract_diag=subtract_diag)
    return c, tabs, AB


# ------------------------------------------------------------------ hashing

def test_hash_tables_bit_exact(cmm, ctx):
    _say("case: hash tables n1=777 n3=513 b=4096 d=5 seed=99")
    At, B = _rand_problem(777, 33, 513, 1)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), 4096, 5, seed=99)
    pr = O.hash_params(99, 5)
    np.testing.assert_array_equal(sk.hash_params(), pr)
    h1, s1, h2, s2 = O.hash_tables(pr, 777, 513, 4096)
    for t in range(5):
        g1, gs1, g2, gs2 = sk.hashes(t)
        np.testing.assert_array_equal(g1, h1[t]); np.testing.assert_array_equal(gs1, s1[t])
        np.testing.assert_array_equal(g2, h2[t]); np.testing.assert_array_equal(gs2, s2[t])


def test_hash_explicit_params_bit_exact(cmm, ctx):
    _say("case: explicit hash parameters near the modulus")
    P = O.P61
    pr = np.array([[[P - 1, P - 1], [1, 0], [P - 2, 12345], [2**60 + 3, P - 7]]], dtype=np.uint64)
    At, B = _rand_problem(1000, 8, 999, 2)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), 1 << 20, 1, hash_params=pr)
    h1, s1, h2, s2 = O.hash_tables(pr, 1000, 999, 1 << 20)
    g1, gs1, g2, gs2 = sk.hashes(0)
    np.testing.assert_array_equal(g1, h1[0]); np.testing.assert_array_equal(gs1, s1[0])
    np.testing.assert_array_equal(g2, h2[0]); np.testing.assert_array_equal(gs2, s2[0])


# ------------------------------------------------------------------- sketch

SHAPES = [
    # (n1, m, n3, b, d): every FFT row length 2^4..2^12, single and multi-row
    (37, 19, 23, 16, 1),
    (50, 40, 70, 64, 2),
    (200, 64, 150, 256, 3),
    (300, 130, 260, 1024, 3),
    (257, 77, 311, 4096, 2),
    (500, 90, 450, 8192, 3),
    (1000, 120, 900, 1 << 14, 2),
    (700, 65, 1100, 1 << 16, 3),
    (333, 50, 444, 1 << 18, 1),
    (4000, 31, 100, 512, 5),       # many members per bucket
]


@pytest.mark.parametrize("shape", SHAPES, ids=[f"{s[0]}x{s[1]}x{s[2]}_b{s[3]}_d{s[4]}" for s in SHAPES])
def test_sketch_parity_f32(cmm, ctx, shape):
    n1, m, n3, b, d = shape
    _say(f"case: sketch f32 {shape}")
    At, B = _rand_problem(n1, m, n3, n1 + 7 * b)
    seed = 1234 + b
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=seed)
    c_gpu = sk.c()
    c_ref, _, _ = _oracle_c(At, B, b, d, seed)
    for t in range(d):
        assert _rel_l2(c_gpu[t], c_ref[t]) <= REL_TOL, (t, _rel_l2(c_gpu[t], c_ref[t]))


def test_sketch_parity_strided_operands(cmm, ctx):
    _say("case: strided lda/ldb")
    import torch
    g = np.random.default_rng(5)
    Abig = g.standard_normal((80, 301)).astype(np.float32)
    Bbig = g.standard_normal((80, 260)).astype(np.float32)
    At, B = Abig[:, :290], Bbig[:, :257]
    dA, dB = _dev(Abig), _dev(Bbig)
    sk = cmm.sketch_product(ctx, dA[:, :290], dB[:, :257], 2048, 2, seed=8, n1=290, n3=257)
    c_ref, _, _ = _oracle_c(At, B, 2048, 2, 8)
    c_gpu = sk.c()
    for t in range(2):
        assert _rel_l2(c_gpu[t], c_ref[t]) <= REL_TOL


def test_injective_tables_give_product(cmm, ctx):
    """h1(i) = i, h2(j) = n1 j, s = +1, b >= n1 n3: the sketch is AB itself
    and every estimate equals (AB)_ij (numpy float64 GEMM)."""
    _say("case: injective explicit tables")
    n1, m, n3 = 24, 40, 20
    b = 512
    At, B = _rand_problem(n1, m, n3, 9)
    h1 = np.arange(n1)[None, :]; h2 = (n1 * np.arange(n3))[None, :]
    s1 = np.ones((1, n1)); s2 = np.ones((1, n3))
    sk = cmm.sketch_product_tables(ctx, _dev(At), _dev(B), b, h1, s1, h2, s2)
    AB = At.astype(np.float64).T @ B.astype(np.float64)
    c = sk.c()[0]
    for i in range(n1):
        for j in range(n3):
            assert abs(c[i + n1 * j] - AB[i, j]) <= 1e-5 * np.abs(AB).max()
    assert np.abs(c[n1 * n3:]).max() <= 1e-5 * np.abs(AB).max()


def test_k_split_merge(cmm, ctx):
    _say("case: merge of two k-ranges")
    At, B = _rand_problem(300, 100, 280, 11)
    whole = cmm.sketch_product(ctx, _dev(At), _dev(B), 2048, 3, seed=4)
    p1 = cmm.sketch_product(ctx, _dev(At[:45]), _dev(B[:45]), 2048, 3, seed=4)
    p2 = cmm.sketch_product(ctx, _dev(At[45:]), _dev(B[45:]), 2048, 3, seed=4)
    p1.merge(p2)
    cw, cm = whole.c(), p1.c()
    for t in range(3):
        assert _rel_l2(cm[t], cw[t]) <= REL_TOL


def test_subtract_diagonal_parity(cmm, ctx):
    _say("case: covariance with diagonal subtraction")
    X, _, _ = W.covariance_observations(320, 200, 8, 0.9, 3)
    X = X.astype(np.float32)
    dX = _dev(X)
    sk = cmm.sketch_product(ctx, dX, dX, 2048, 3, seed=21, subtract_diag=True)
    c_ref, _, _ = _oracle_c(X, X, 2048, 3, 21, subtract_diag=True)
    c_gpu = sk.c()
    for t in range(3):
        assert _rel_l2(c_gpu[t], c_ref[t]) <= REL_TOL


def test_subtract_diagonal_deterministic_with_collisions(cmm, ctx):
    """3000 diagonal entries into 256 buckets: each bucket takes about a
    dozen of them per repetition.  Two runs give the same bits, the result
    matches the oracle, and subtracting the host-computed float64 diagonal
    from the plain sketch (cmm_sketch_subtract_diagonal) agrees with it."""
    import torch
    _say("case: diagonal subtraction with many collisions, determinism")
    g = np.random.default_rng(12)
    n, m, b, d = 3000, 50, 256, 4
    X = g.standard_normal((m, n)).astype(np.float32)
    dX = _dev(X)
    runs = [cmm.sketch_product(ctx, dX, dX.clone(), b, d, seed=31, subtract_diag=True) for _ in range(3)]
    cs = [r.c() for r in runs]
    for c in cs[1:]:
        np.testing.assert_array_equal(c, cs[0])
    c_ref, _, _ = _oracle_c(X, X, b, d, 31, subtract_diag=True)
    for t in range(d):
        assert _rel_l2(cs[0][t], c_ref[t]) <= REL_TOL
    plain = cmm.sketch_product(ctx, dX, dX.clone(), b, d, seed=31)
    Xd = X.astype(np.float64)
    diag = torch.from_numpy(np.einsum("ki,ki->i", Xd, Xd)).cuda()
    plain.subtract_diagonal(diag)
    cp = plain.c()
    assert np.abs(cp - cs[0]).max() <= 1e-9 * np.abs(cs[0]).max()
    again = cmm.sketch_product(ctx, dX, dX.clone(), b, d, seed=31)
    again.subtract_diagonal(diag)
    np.testing.assert_array_equal(again.c(), cp)
    for r in runs + [plain, again]:
        r.free()


# ----------------------------------------------------- decoding and top-K

def _tables_np(tabs):
    return tuple(np.asarray(x) for x in tabs)


def test_estimates_parity(cmm, ctx):
    _say("case: estimates")
    import torch
    At, B = _rand_problem(400, 150, 350, 13)
    b, d, seed = 4096, 5, 77
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=seed)
    c_ref, tabs, _ = _oracle_c(At, B, b, d, seed)
    c_gpu = sk.c()
    g = np.random.default_rng(1)
    qi = g.integers(0, 400, 5000); qj = g.integers(0, 350, 5000)
    est = sk.estimate_batch(_dev(qi), _dev(qj)).cpu().numpy().astype(np.float64)
    ref = O.decode(c_ref, tabs, qi, qj)
    bound = np.abs(c_gpu.astype(np.float32).astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max()
    assert np.abs(est - ref).max() <= bound
    for (i, j) in [(0, 0), (399, 349), (17, 123)]:
        assert abs(sk.estimate(i, j) - O.decode(c_ref, tabs, [i], [j])[0]) <= bound


def _check_topk(got_lin, got_val, vals, lin, K, delta):
    order = np.lexsort((lin, -np.abs(vals)))
    ref_lin = lin[order[:K]]
    tau = abs(vals[order[K - 1]])
    mag = dict(zip(lin.tolist(), np.abs(vals).tolist()))
    sure = {l for l in ref_lin.tolist() if mag[l] > tau + delta}
    got = set(got_lin.tolist())
    assert sure <= got, sorted(sure - got)[:5]
    for l in got:
        assert mag[l] >= tau - delta, (l, mag[l], tau)
    assert len(got) == K
    # returned order: |value| non-increasing
    assert np.all(np.diff(np.abs(got_val)) <= 1e-6 * max(1.0, abs(got_val[0])))


@pytest.mark.parametrize("mode", ["all", "upper"])
def test_topk_parity(cmm, ctx, mode):
    _say(f"case: top-K {mode}")
    X, _, _ = W.covariance_observations(600, 300, 12, 0.9, 4)
    X = X.astype(np.float32)
    dX = _dev(X)
    b, d, K = 8192, 5, 40
    sk = cmm.sketch_product(ctx, dX, dX, b, d, seed=31, subtract_diag=True)
    c_ref, tabs, _ = _oracle_c(X, X, b, d, 31, subtract_diag=True)
    oi, oj, ov = sk.topk(K, mode)
    i, j = O.candidates(mode, 600, 600)
    vals = O.decode(c_ref, tabs, i, j)
    lin = i * 600 + j
    delta = 2 * (np.abs(sk.c().astype(np.float32).astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max())
    _check_topk(oi * 600 + oj, ov, vals, lin, K, delta)
    # returned values are the estimates at the returned positions
    ref_at = O.decode(c_ref, tabs, oi, oj)
    assert np.abs(ov - ref_at).max() <= delta


TOPK_LARGE = [
    # (n1, n3, m, b, d, K, mode): at least 64 tiles of 16 rows, so the sampled
    # threshold and the fused histogram + collect pass run
    (1500, 1400, 200, 1 << 14, 5, 64, "all"),
    (1600, 1600, 150, 1 << 14, 3, 2048, "upper"),
    (1200, 1300, 100, 1024, 1, 50, "all"),      # d = 1: ~1500 equal magnitudes per bucket
    (1024, 1024, 64, 4096, 1, 1, "upper"),
    # even d, and b above the screening bitmap's width (several buckets per bit)
    (1100, 1050, 64, 1 << 17, 6, 100, "all"),
]


@pytest.mark.parametrize("case", TOPK_LARGE, ids=[f"{c[0]}x{c[1]}_b{c[3]}_d{c[4]}_K{c[5]}_{c[6]}" for c in TOPK_LARGE])
def test_topk_parity_large_domain(cmm, ctx, case):
    n1, n3, m, b, d, K, mode = case
    _say(f"case: top-K large domain {case}")
    At, B = _rand_problem(n1, m, n3, 1000 + n1 + K)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=61 + K)
    c_ref, tabs, _ = _oracle_c(At, B, b, d, 61 + K)
    oi, oj, ov = sk.topk(K, mode)
    i, j = O.candidates(mode, n1, n3)
    vals = O.decode(c_ref, tabs, i, j)
    delta = 2 * (np.abs(sk.c().astype(np.float32).astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max())
    _check_topk(oi * n3 + oj, ov, vals, i * n3 + j, K, delta)
    assert np.abs(ov - O.decode(c_ref, tabs, oi, oj)).max() <= delta
    if mode == "upper":
        assert np.all(oi < oj)
    # equal magnitudes come out in increasing linear index
    mag, lin = np.abs(ov), oi * n3 + oj
    same = mag[1:] == mag[:-1]
    assert np.all(lin[1:][same] > lin[:-1][same])


# (n1, m, n3, b, d, K): 500 rows decode every row; from 1024 rows a 1-in-16
# sample sets a threshold and rows that cannot reach it stop early (d = 5,
# 7; K = 1000 of 1024 leaves too few rows above it, so the exact pass runs)
COLUMN_CASES = [
    (500, 120, 64, 4096, 3, 6),
    (3000, 80, 40, 8192, 5, 40),
    (2048, 64, 24, 8192, 7, 300),
    (1024, 40, 8, 4096, 5, 1000),
]


@pytest.mark.parametrize("case", COLUMN_CASES, ids=[f"{c[0]}x{c[2]}_d{c[4]}_K{c[5]}" for c in COLUMN_CASES])
def test_topk_per_column_parity(cmm, ctx, case):
    n1, m, n3, b, d, K = case
    _say(f"case: top-K per column {case}")
    At, B = _rand_problem(n1, m, n3, 17 + n1)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=41)
    c_ref, tabs, _ = _oracle_c(At, B, b, d, 41)
    oi, oj, ov = sk.topk(K, "column")
    C = O.decode_all(c_ref, tabs, n1, n3)
    delta = 2 * (np.abs(sk.c().astype(np.float32).astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max())
    for jj in range(n3):
        rows = oi[jj * K:(jj + 1) * K]
        assert np.all(oj[jj * K:(jj + 1) * K] == jj)
        _check_topk(rows, ov[jj * K:(jj + 1) * K], C[:, jj], np.arange(n1), K, delta)


# --------------------------------------------------------------- precision

@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_sketch_parity_low_precision(cmm, ctx, dtype):
    """Arithmetic error: the GPU on bf16 / fp8 operands against the oracle on
    the same dequantised values, to the float32 tolerance."""
    _say(f"case: sketch {dtype}")
    import torch
    X, _, _ = W.covariance_observations(512, 256, 8, 0.8, 6)
    store, scale, deq = W._encode(X, dtype)
    dS = _dev(store)
    dsc = _dev(scale) if scale is not None else None
    sk = cmm.sketch_product(ctx, dS, dS, 4096, 3, seed=55, dtype=dtype, scaleA=dsc, scaleB=dsc,
                            subtract_diag=True, n1=512, n3=512, m=256)
    c_ref, _, _ = O.run(deq.T, deq, 4096, 3, 55, subtract_diag=True)
    c_gpu = sk.c()
    for t in range(3):
        assert _rel_l2(c_gpu[t], c_ref[t]) <= REL_TOL, (t, _rel_l2(c_gpu[t], c_ref[t]))


# ---------------------------------------------------------------- errors

def test_error_codes(cmm, ctx):
    _say("case: error codes")
    At, B = _rand_problem(64, 16, 64, 1)
    dA, dB = _dev(At), _dev(B)
    with pytest.raises(cmm.CmmError) as e:
        cmm.sketch_product(ctx, dA, dB, 1000, 1)        # b not a power of two
    assert e.value.code == cmm.CMM_EINVAL
    with pytest.raises(cmm.CmmError) as e:
        cmm.sketch_product(ctx, dA, dB, 1024, 0)        # d < 1
    assert e.value.code == cmm.CMM_EINVAL
    sk = cmm.sketch_product(ctx, dA, dB, 1024, 1)
    with pytest.raises(cmm.CmmError) as e:
        sk.estimate(64, 0)
    assert e.value.code == cmm.CMM_EINVAL
    with pytest.raises(cmm.CmmError) as e:
        sk.topk(64 * 64 + 1, "all")
    assert e.value.code == cmm.CMM_EINVAL
