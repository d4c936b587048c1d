"""GPU parity at the edges of the accepted argument ranges, through the C ABI:
degenerate sizes (1 x 1 x 1, m = 1), the most repetitions (d = 63), the
largest staged dimension (24576, one count-sketch row of LDS), many more
entries than buckets (n >> b), the smallest and largest b, and the tuning
cache loaded from CMM_TUNE_CACHE at context creation."""
import json
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


def _dev(x):
    import torch
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


EDGES = [
    # (n1, m, n3, b, d)
    (1, 1, 1, 16, 1),
    (1, 7, 300, 64, 3),
    (300, 1, 1, 1024, 2),
    (64, 9, 48, 256, 63),
    (24576, 6, 100, 1 << 15, 2),
    (5000, 3, 4000, 16, 4),
    (200, 50, 220, 1 << 20, 1),
]


@pytest.mark.parametrize("case", EDGES, ids=[f"{c[0]}x{c[1]}x{c[2]}_b{c[3]}_d{c[4]}" for c in EDGES])
def test_edge_sizes_match_oracle(cmm, ctx, case):
    n1, m, n3, b, d = case
    _say(f"case: edge sizes {case}")
    g = np.random.default_rng(n1 + 3 * n3 + b)
    At = g.standard_normal((m, n1)).astype(np.float32)
    B = g.standard_normal((m, n3)).astype(np.float32)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=n1 + d)
    c = sk.c()
    c_ref, tabs, _ = O.run(At.astype(np.float64).T, B.astype(np.float64), b, d, n1 + d)
    for t in range(d):
        nrm = np.linalg.norm(c_ref[t])
        if nrm == 0:
            assert np.abs(c[t]).max() <= 1e-6
        else:
            assert np.linalg.norm(c[t] - c_ref[t]) / nrm <= REL_TOL, (t, np.linalg.norm(c[t] - c_ref[t]) / nrm)
    # an estimate and the top-1 on every edge case
    K = 1
    oi, oj, ov = sk.topk(K, "all")
    assert 0 <= oi[0] < n1 and 0 <= oj[0] < n3
    assert abs(ov[0] - O.decode(c_ref, tabs, oi, oj)[0]) <= 2 * np.abs(c - c_ref).max() + 1e-6 * np.abs(c_ref).max()


def test_tuning_cache_from_environment(cmm, tmp_path, monkeypatch):
    """A tuning table saved by one context is loaded by a context created
    later with CMM_TUNE_CACHE naming it (read when the context is created)."""
    _say("case: tuning cache through CMM_TUNE_CACHE")
    path = str(tmp_path / "tune.json")
    c = cmm.Context(0)
    try:
        c.set_tuning(2000, 300, 1500, 1 << 15, 3, "bf16", (11, 64, 2048))
        c.save_tuning(path)
    finally:
        c.close()
    assert json.load(open(path))[0]["kmax"] == 64
    monkeypatch.setenv("CMM_TUNE_CACHE", path)
    c2 = cmm.Context(0)
    try:
        assert c2.tuning(2000, 300, 1500, 1 << 15, 3, "bf16") == (11, 64, 2048)
    finally:
        c2.close()
    monkeypatch.setenv("CMM_TUNE_CACHE", str(tmp_path / "missing.json"))
    c3 = cmm.Context(0)      # a missing cache file is not an error
    c3.close()


def _column_band_check(oi, ov, C, K, delta):
    """Per column: every row whose oracle |C| is above the K-th one by more
    than delta is returned, every returned row is within delta of it, and the
    returned values are the estimates at the returned rows."""
    n1, n3 = C.shape
    oi = oi.reshape(n3, K)
    ov = ov.reshape(n3, K)
    for j in range(n3):
        mag = np.abs(C[:, j])
        order = np.lexsort((np.arange(n1), -mag))
        tau = mag[order[K - 1]]
        sure = {int(i) for i in order[:K] if mag[i] > tau + delta}
        got = set(oi[j].tolist())
        assert len(got) == K and sure <= got, (j, sorted(sure - got)[:5])
        assert np.all(mag[oi[j]] >= tau - delta), j
        assert np.abs(ov[j] - C[oi[j], j]).max() <= delta, j


@pytest.mark.parametrize("dtype", ["f32", "bf16", "fp8"])
def test_large_hashed_dimension(cmm, ctx, dtype):
    """n1 = 40000: above the 24576 floats a count-sketch row stages in LDS,
    so A's rows are gathered from global memory (B's are staged); top-K over
    all entries and per column (the column's keys still fit in LDS)."""
    import workloads as W
    n1, m, n3, b, d, K = 40000, 6, 48, 1 << 16, 3, 4
    _say(f"case: large hashed dimension {dtype} n1={n1}")
    g = np.random.default_rng(17)
    At = g.standard_normal((m, n1))
    B = g.standard_normal((m, n3))
    sa, scA, Aq = W._encode(At, dtype)
    sb, scB, Bq = W._encode(B, dtype)
    sk = cmm.sketch_product(ctx, _dev(sa), _dev(sb), b, d, seed=5, dtype=dtype,
                            scaleA=None if scA is None else _dev(scA),
                            scaleB=None if scB is None else _dev(scB))
    c = sk.c()
    c_ref, tabs, _ = O.run(Aq.T, Bq, b, d, 5)
    for t in range(d):
        assert np.linalg.norm(c[t] - c_ref[t]) / np.linalg.norm(c_ref[t]) <= REL_TOL
    delta = 2 * (np.abs(c.astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max())
    C = O.decode_all(c_ref, tabs, n1, n3)
    oi, oj, ov = sk.topk(K, "all")
    lin = np.arange(n1 * n3)
    vals = C.reshape(-1)
    order = np.lexsort((lin, -np.abs(vals)))
    tau = abs(vals[order[K - 1]])
    got = set((oi * n3 + oj).tolist())
    assert {int(l) for l in order[:K] if abs(vals[l]) > tau + delta} <= got
    assert all(abs(vals[l]) >= tau - delta for l in got)
    ci, _, cv = sk.topk(K, "column")
    _column_band_check(ci, cv, C, K, delta)


@pytest.mark.parametrize("n1", [20000, 50000])
def test_column_topk_tall_columns(cmm, ctx, n1):
    """Per-column top-K above 16384 rows: keys in up to 159 KB of LDS
    (20000), and recomputed every round past that (50000)."""
    m, n3, b, d, K = 4, 16, 1 << 15, 3, 3
    _say(f"case: per-column top-K with n1={n1}")
    g = np.random.default_rng(n1)
    At = g.standard_normal((m, n1)).astype(np.float32)
    B = g.standard_normal((m, n3)).astype(np.float32)
    sk = cmm.sketch_product(ctx, _dev(At), _dev(B), b, d, seed=3)
    c = sk.c()
    c_ref, tabs, _ = O.run(At.astype(np.float64).T, B.astype(np.float64), b, d, 3)
    delta = 2 * (np.abs(c.astype(np.float64) - c_ref).max() + 1e-6 * np.abs(c_ref).max())
    ci, cj, cv = sk.topk(K, "column")
    assert np.array_equal(cj.reshape(n3, K), np.repeat(np.arange(n3)[:, None], K, axis=1))
    _column_band_check(ci, cv, O.decode_all(c_ref, tabs, n1, n3), K, delta)


def test_hashed_dimension_limits(cmm, ctx):
    _say("case: hashed dimension limits (dense 65535, sparse 24576)")
    At = _dev(np.zeros((2, 65536), np.float32))
    B = _dev(np.zeros((2, 8), np.float32))
    with pytest.raises(cmm.CmmError) as e:
        cmm.sketch_product(ctx, At, B, 64, 1, seed=1)
    assert e.value.code == cmm.CMM_EUNSUPPORTED
    import torch
    ptr = _dev(np.zeros(3, np.int64))
    idx = torch.zeros(0, dtype=torch.int32, device="cuda")
    val = torch.zeros(0, dtype=torch.float32, device="cuda")
    with pytest.raises(cmm.CmmError) as e:
        cmm.sketch_product_sparse(ctx, ptr, idx, val, ptr, idx, val, 30000, 2, 8, 64, 1, seed=1)
    assert e.value.code == cmm.CMM_EUNSUPPORTED
