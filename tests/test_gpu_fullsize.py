"""GPU parity at the benchmark's full sizes, in the launch configuration
bench.py times (the size class autotuned first).

* covariance n = m = 4096, float32, b = 2^16, d = 5: the whole sketch
  against the oracle and the top-64 over i < j (tolerance band).
* DCT transform n = 8192, bf16, b = 2^17, d = 7: the whole sketch, and the
  per-column top-16 (DECOMPRESS over a column, Figure 1) of 64 random
  columns against the oracle's decode of those columns.
* covariance n = m = 16384, fp8 e4m3fn with per-column scales, b = 2^18,
  d = 9: the whole sketch (float64 AB of 2.7e8 entries, binned per
  repetition), 10^5 uniformly sampled estimates, and the top-256 over i < j
  against the oracle's top-256 decoded block by block.

Every sketch comparison asserts, per repetition, relative L2 error <= 1e-5
and largest entry error <= 1e-5 max|c_t| (the float32 budget); estimates
are within the largest error of the float32 sketch the GPU decodes from.
The batched form's 64 products are compared in test_gpu_batch.py.
"""
import sys

import numpy as np
import pytest

from oracle import cmm_oracle as O
import workloads as W
import oracle_runs as R

pytestmark = [pytest.mark.gpu, pytest.mark.timeout(900)]


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


def _product(cmm, ctx, w):
    """The product as bench.py runs it: the size class tuned first, then one
    sketch product on device copies of the stored operands."""
    ctx.autotune(w.n1, w.m, w.n3, w.b, w.d, w.dtype)
    At = _dev(w.At_store)
    B = At.clone() if w.same_operand else _dev(w.B_store)
    sA = _dev(w.scaleA) if w.scaleA is not None else None
    sB = _dev(w.scaleB) if w.scaleB is not None else None
    sk = cmm.sketch_product(ctx, At, B, w.b, w.d, seed=w.seed, dtype=w.dtype, scaleA=sA,
                            scaleB=sB, subtract_diag=w.subtract_diag, n1=w.n1, n3=w.n3, m=w.m)
    return sk


def _tables(w):
    return O.hash_tables(O.hash_params(w.seed, w.d), w.n1, w.n3, w.b)


def test_covariance_4096_f32(cmm, ctx):
    _say("case: covariance n=m=4096 f32 b=2^16 d=5 (whole sketch, top-64)")
    w = W.make_workload(2)
    sk = _product(cmm, ctx, w)
    c_gpu = sk.c()
    A, B = W.dequantised(w)
    tabs = _tables(w)
    c_ref, _ = R.sketch(A, B, tabs, w.b, subtract_diag=True)
    l2, inf = R.check_sketch(c_gpu, c_ref)
    _say(f"  rel L2 {l2:.2e}, max|dc|/max|c| {inf:.2e}")
    oi, oj, ov = sk.topk(w.K, "upper")
    delta = R.decode_band(c_gpu, c_ref)
    ri, rj, rv = R.topk_upper(c_ref, tabs, w.n1, w.K)
    R.band_check(oi, oj, ov, ri, rj, rv, abs(rv[-1]), delta,
                 lambda i, j: O.decode(c_ref, tabs, i, j))
    sk.free()


def test_transform_8192_bf16(cmm, ctx):
    _say("case: DCT transform n=8192 bf16 b=2^17 d=7 (whole sketch, top-16 of 64 columns)")
    w = W.make_workload(3)
    sk = _product(cmm, ctx, w)
    c_gpu = sk.c()
    A, B = W.dequantised(w)
    tabs = _tables(w)
    c_ref, _ = R.sketch(A, B, tabs, w.b)
    l2, inf = R.check_sketch(c_gpu, c_ref)
    _say(f"  rel L2 {l2:.2e}, max|dc|/max|c| {inf:.2e}")
    oi, oj, ov = sk.topk(w.K, "column")
    delta = R.decode_band(c_gpu, c_ref)
    g = np.random.default_rng(33)
    cols = np.sort(g.choice(w.n3, 64, replace=False))
    Ccols = O.decode(c_ref, tabs, np.arange(w.n1)[:, None], cols[None, :])   # n1 x 64
    rows_ref, vals_ref = O.topk_per_column(Ccols, w.K)
    worst = 0.0
    for q, j in enumerate(cols):
        got_r = oi[j * w.K:(j + 1) * w.K]
        got_v = ov[j * w.K:(j + 1) * w.K]
        assert np.all(oj[j * w.K:(j + 1) * w.K] == j)
        assert len(set(got_r.tolist())) == w.K
        worst = max(worst, R.band_check(
            got_r, np.full(w.K, j), got_v, rows_ref[q], np.full(w.K, j), vals_ref[q],
            abs(vals_ref[q][-1]), delta, lambda i, jj: Ccols[i, q]))
    _say(f"  per-column top-16 of 64 columns inside the band; largest value error {worst:.2e}")
    hits = sum(len(set(oi[j * w.K:(j + 1) * w.K].tolist()) & set(w.planted[j].tolist())) for j in range(w.n3))
    _say(f"  spike recall in the per-column top-16 (reported): {hits / (w.n3 * w.K):.4f}")
    sk.free()


def test_covariance_16384_fp8(cmm, ctx):
    _say("case: covariance n=m=16384 fp8 b=2^18 d=9 (whole sketch, 1e5 estimates, top-256)")
    import torch
    w = W.make_workload(4)
    sk = _product(cmm, ctx, w)
    c_gpu = sk.c()
    X = W.dequantised(w)[1]                  # m x n, what the GPU reads
    tabs = _tables(w)
    c_ref, _ = R.sketch(np.ascontiguousarray(X.T), X, tabs, w.b, subtract_diag=True)
    del X
    l2, inf = R.check_sketch(c_gpu, c_ref)
    _say(f"  rel L2 {l2:.2e}, max|dc|/max|c| {inf:.2e}")
    delta = R.decode_band(c_gpu, c_ref)
    # 10^5 uniformly sampled estimates (any i, j)
    g = np.random.default_rng(44)
    si = g.integers(0, w.n1, 100_000); sj = g.integers(0, w.n3, 100_000)
    est = sk.estimate_batch(torch.from_numpy(si).cuda(), torch.from_numpy(sj).cuda()).cpu().numpy()
    err = float(np.abs(est.astype(np.float64) - O.decode(c_ref, tabs, si, sj)).max())
    assert err <= delta / 2, (err, delta)
    _say(f"  1e5 sampled estimates: largest error {err:.3e} (bound {delta / 2:.3e})")
    oi, oj, ov = sk.topk(w.K, "upper")
    assert np.all(oi < oj)
    ri, rj, rv = R.topk_upper(c_ref, tabs, w.n1, w.K)
    R.band_check(oi, oj, ov, ri, rj, rv, abs(rv[-1]), delta,
                 lambda i, j: O.decode(c_ref, tabs, i, j))
    same = len(set(zip(oi.tolist(), oj.tolist())) & set(zip(ri.tolist(), rj.tolist())))
    _say(f"  top-256 inside the band ({same} of 256 positions identical to the oracle's)")
    got = {(int(a), int(b)) for a, b in zip(oi, oj)}
    want = {(int(min(p, q)), int(max(p, q))) for p, q in w.planted}
    _say(f"  planted-pair recall in the top-256 (reported): {len(got & want) / len(want):.4f}")
    sk.free()
