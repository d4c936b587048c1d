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
