"""GPU tests of the batched form and of the tuning table.

* Every product of a batch (one HIP graph launch over products of uneven
  n1, m, n3, b, d and dtype) equals its standalone result bit for bit (the
  diagonal subtraction included); and each matches
  the oracle within the float32 sketch tolerance (rel. L2 1e-5 per
  repetition).
* Graph replays are checked one by one, with eager work (operand rescaling
  by powers of two, another library call) between them: doubling an operand
  doubles the sketch exactly (every step is linear and the fixed-point scale
  of the spectral fold follows the column maximum by a power of two).
* A product computed under any tuning of the table matches the oracle.
"""
import json
import os
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


# (n1, m, n3, b, d, dtype, subtract_diag): uneven sizes, all three dtypes,
# every FFT row regime (b below, at and above one LDS row)
MIX = [
    (300, 200, 300, 2048, 3, "f32", True),
    (777, 130, 513, 4096, 5, "f32", False),
    (1024, 257, 1024, 1 << 14, 2, "bf16", False),
    (150, 64, 190, 256, 1, "f32", False),
    (2000, 97, 1500, 1 << 16, 3, "fp8", False),
    (520, 300, 520, 8192, 4, "bf16", True),
    (64, 33, 80, 16, 2, "f32", False),
]


def _operands(n1, m, n3, dtype, seed, same):
    g = np.random.default_rng(seed)
    At = g.standard_normal((m, n1))
    B = At.copy() if same else g.standard_normal((m, n3))
    if dtype == "f32":
        return At.astype(np.float32), B.astype(np.float32), None, None
    if dtype == "bf16":
        return W.bf16_encode(At), W.bf16_encode(B), None, None
    sa = (np.abs(At).max(axis=0) / 448.0).astype(np.float32)
    sb = (np.abs(B).max(axis=0) / 448.0).astype(np.float32)
    return W.e4m3fn_encode(At / sa[None, :]), W.e4m3fn_encode(B / sb[None, :]), sa, sb


def _deq(store, dtype, scale):
    if dtype == "f32":
        return store.astype(np.float64)
    if dtype == "bf16":
        return (store.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    mag = W.e4m3fn_grid()[(store & 0x7F).astype(np.int64)]
    v = np.where((store & 0x80) != 0, -mag, mag).astype(np.float32) * scale[None, :]
    return v.astype(np.float64)


@pytest.fixture(scope="module")
def mix(cmm):
    items = []
    for q, (n1, m, n3, b, d, dt, diag) in enumerate(MIX):
        At, B, sa, sb = _operands(n1, m, n3, dt, 500 + q, diag)
        items.append(dict(n1=n1, m=m, n3=n3, b=b, d=d, dtype=dt, diag=diag, seed=900 + q,
                          At=At, B=B, sa=sa, sb=sb,
                          dAt=_dev(At), dB=_dev(B),
                          dsa=None if sa is None else _dev(sa), dsb=None if sb is None else _dev(sb)))
    return items


def _problems(cmm, items):
    return [cmm.problem(x["dAt"], x["dB"], x["b"], x["d"], seed=x["seed"], dtype=x["dtype"],
                        scaleA=x["dsa"], scaleB=x["dsb"], subtract_diag=x["diag"])
            for x in items]


def _standalone(cmm, ctx, x):
    return cmm.sketch_product(ctx, x["dAt"], x["dB"], x["b"], x["d"], seed=x["seed"],
                              dtype=x["dtype"], scaleA=x["dsa"], scaleB=x["dsb"],
                              subtract_diag=x["diag"]).c()


def _same(c_batch, c_alone, diag):
    # every step is deterministic, the diagonal subtraction included (its
    # bucket sums are exact fixed-point sums), so a batch product equals its
    # standalone run bit for bit
    return np.array_equal(c_batch, c_alone)


def test_batch_equals_standalone_and_oracle(cmm, ctx, mix):
    _say(f"case: batch of {len(MIX)} mixed products vs standalone and oracle")
    alone = [_standalone(cmm, ctx, x) for x in mix]
    bt = cmm.Batch(ctx, _problems(cmm, mix))
    bt.run()
    for q, x in enumerate(mix):
        c = bt.sketch(q).c()
        assert _same(c, alone[q], x["diag"]), (q, np.abs(c - alone[q]).max())
        A = _deq(x["At"], x["dtype"], x["sa"]).T
        B = _deq(x["B"], x["dtype"], x["sb"])
        c_ref, _, _ = O.run(A, B, x["b"], x["d"], x["seed"], subtract_diag=x["diag"])
        for t in range(x["d"]):
            assert _rel_l2(c[t], c_ref[t]) <= REL_TOL, (q, t, _rel_l2(c[t], c_ref[t]))
    bt.free()


def _upper_domain(n1, n3):
    return sum(max(0, n3 - i - 1) for i in range(n1))


@pytest.mark.parametrize("mode", ["all", "upper", "column"])
def test_batch_topk_equals_per_product(cmm, ctx, mix, mode):
    """cmm_batch_topk shares the host waits of all products; its results are
    those of cmm_topk on every product (the same kernels and thresholds),
    with a different K per product, over products that take the sampled
    fast path (n1 >= 1024) and ones that take the digit passes."""
    _say(f"case: batch top-K ({mode}) vs per-product top-K")
    bt = cmm.Batch(ctx, _problems(cmm, mix))
    bt.run()
    Ks = []
    for q, x in enumerate(mix):
        if mode == "column":
            Ks.append(min(1 + q, x["n1"]))
        else:
            dom = x["n1"] * x["n3"] if mode == "all" else _upper_domain(x["n1"], x["n3"])
            Ks.append(min(5 + 7 * q, dom))
    got = bt.topk(Ks, mode)
    assert len(got) == len(mix)
    for q in range(len(mix)):
        want = bt.sketch(q).topk(Ks[q], mode)
        for a, b in zip(got[q], want):
            assert np.array_equal(a, b), (q, mode)
    # invalid K for one product: nothing is returned, the error names it
    bad = list(Ks)
    bad[3] = 0
    with pytest.raises(cmm.CmmError) as e:
        bt.topk(bad, mode)
    assert e.value.code == cmm.CMM_EINVAL
    bad[3] = mix[3]["n1"] * mix[3]["n3"] + 1
    with pytest.raises(cmm.CmmError) as e:
        bt.topk(bad, mode)
    assert e.value.code == cmm.CMM_EINVAL
    bt.free()


def test_batch_topk_across_groups(cmm, ctx):
    """A batch of more than 256 products: the batch top-K runs in groups of
    256 and writes each product's results at its own offset."""
    import torch
    _say("case: batch top-K over 260 small products (two groups)")
    g = np.random.default_rng(4242)
    ops, probs, Ks = [], [], []
    for q in range(260):
        n1, n3, m = int(g.integers(20, 70)), int(g.integers(20, 70)), int(g.integers(5, 30))
        At = torch.from_numpy(g.standard_normal((m, n1)).astype(np.float32)).cuda()
        B = torch.from_numpy(g.standard_normal((m, n3)).astype(np.float32)).cuda()
        ops.append((At, B))
        probs.append(cmm.problem(At, B, 256, 1 + q % 3, seed=q))
        Ks.append(1 + q % 5)
    bt = cmm.Batch(ctx, probs, keep=ops)
    bt.run()
    got = bt.topk(Ks, "all")
    for q in (0, 1, 255, 256, 257, 259):
        want = bt.sketch(q).topk(Ks[q], "all")
        for a, b in zip(got[q], want):
            assert np.array_equal(a, b), q
    assert [len(x[0]) for x in got] == Ks
    bt.free()


def test_graph_replays_with_eager_work_between(cmm, ctx, mix):
    _say("case: repeated graph replays with operand rescaling between them")
    import torch
    alone = [_standalone(cmm, ctx, x) for x in mix]
    saved = [(x["dAt"].clone(), x["dB"].clone()) for x in mix]
    bt = cmm.Batch(ctx, _problems(cmm, mix))
    try:
        for r in range(4):
            # eager work between replays: rescale every f32 A operand by 2^r
            # in place (torch kernels) and run a standalone library call
            for q, x in enumerate(mix):
                if x["dtype"] == "f32":
                    x["dAt"].copy_(saved[q][0] * float(2 ** r))
            torch.cuda.synchronize()
            other = _standalone(cmm, ctx, mix[3])
            assert np.array_equal(other, alone[3] * (2.0 ** r))
            bt.run()
            for q, x in enumerate(mix):
                # A B (and its diagonal) scale with A
                want = alone[q] * (2.0 ** r if x["dtype"] == "f32" else 1.0)
                c = bt.sketch(q).c()
                assert _same(c, want, x["diag"]), (r, q, np.abs(c - want).max())
    finally:
        for q, x in enumerate(mix):
            x["dAt"].copy_(saved[q][0]); x["dB"].copy_(saved[q][1])
        torch.cuda.synchronize()
        bt.free()


def test_batch_replay_deterministic(cmm, ctx, mix):
    _say("case: identical replays give identical sketches")
    bt = cmm.Batch(ctx, _problems(cmm, mix))
    bt.run()
    first = [bt.sketch(q).c() for q in range(len(mix))]
    for _ in range(3):
        bt.run(asynchronous=True)
    import torch
    torch.cuda.synchronize()
    for q, x in enumerate(mix):
        assert _same(bt.sketch(q).c(), first[q], x["diag"])
    bt.free()


def test_one_shot_batched(cmm, ctx, mix):
    _say("case: cmm_sketch_product_batched hands owned sketches back")
    alone = [_standalone(cmm, ctx, x) for x in mix]
    sks = cmm.sketch_product_batched(ctx, _problems(cmm, mix))
    assert len(sks) == len(mix)
    for q, x in enumerate(mix):
        assert _same(sks[q].c(), alone[q], x["diag"])
    i, j, v = sks[1].topk(8, "all")
    assert len(i) == 8
    for s in sks:
        s.free()


def test_batch_errors(cmm, ctx, mix):
    _say("case: batch argument errors")
    probs = _problems(cmm, mix[:2])
    bad = _problems(cmm, mix[:2])
    bad[1].b = 1000
    with pytest.raises(cmm.CmmError) as e:
        cmm.Batch(ctx, bad)
    assert e.value.code == cmm.CMM_EINVAL and "problem 1" in str(e.value)
    bad = _problems(cmm, mix[:1])
    bad[0].flags = 2
    with pytest.raises(cmm.CmmError) as e:
        cmm.Batch(ctx, bad)
    assert e.value.code == cmm.CMM_EINVAL
    with pytest.raises(cmm.CmmError):
        cmm.cmm_batch_create(ctx.handle, [], 0)
    bt = cmm.Batch(ctx, probs)
    h = cmm.cmm_batch_sketch(bt.handle, 0)
    with pytest.raises(cmm.CmmError) as e:
        cmm.cmm_sketch_free(h)
    assert e.value.code == cmm.CMM_ESTATE
    with pytest.raises(cmm.CmmError) as e:
        cmm.cmm_batch_sketch(bt.handle, 2)
    assert e.value.code == cmm.CMM_EINVAL
    bt.free()


TUNINGS = [(10, 32, 512), (11, 64, 1024), (12, 128, 4096), (13, 16, 64), (9, 128, 1)]


@pytest.mark.parametrize("tuning", TUNINGS, ids=[f"c{t[0]}_k{t[1]}_cs{t[2]}" for t in TUNINGS])
def test_any_tuning_matches_oracle(cmm, tuning):
    _say(f"case: tuning {tuning} on 900x211x700 b=2^15 d=2")
    n1, m, n3, b, d = 900, 211, 700, 1 << 15, 2
    c = cmm.Context(0)
    try:
        c.set_tuning(n1, m, n3, b, d, "f32", tuning)
        got = c.tuning(n1, m, n3, b, d, "f32")
        assert got == (min(tuning[0], 15), tuning[1], tuning[2])
        g = np.random.default_rng(77)
        At = g.standard_normal((m, n1)).astype(np.float32)
        B = g.standard_normal((m, n3)).astype(np.float32)
        sk = cmm.sketch_product(c, _dev(At), _dev(B), b, d, seed=5)
        c_gpu = sk.c()
        sk.free()
        c_ref, _, _ = O.run(At.astype(np.float64).T, B.astype(np.float64), b, d, 5)
        for t in range(d):
            assert _rel_l2(c_gpu[t], c_ref[t]) <= REL_TOL, (t, _rel_l2(c_gpu[t], c_ref[t]))
    finally:
        c.close()


def test_autotune_and_cache_round_trip(cmm, tmp_path):
    _say("case: autotune 1000x256x1000 b=2^14 d=3 f32, save and load")
    c = cmm.Context(0)
    try:
        tu, ms = c.autotune(1000, 256, 1000, 1 << 14, 3, "f32")
        assert 4 <= tu[0] <= 13 and 1 <= tu[1] <= 128 and tu[2] >= 1 and ms > 0
        assert c.tuning(1000, 256, 1000, 1 << 14, 3, "f32") == (min(tu[0], 14), tu[1], tu[2])
        # same size class (powers-of-two ceilings) shares the entry
        assert c.tuning(900, 200, 1020, 1 << 14, 3, "f32") == (min(tu[0], 14), tu[1], tu[2])
        path = str(tmp_path / "tune.json")
        c.save_tuning(path)
        entries = json.load(open(path))
        assert len(entries) == 1 and entries[0]["log2c"] == tu[0] and entries[0]["kmax"] == tu[1]
    finally:
        c.close()
    c2 = cmm.Context(0)
    try:
        c2.load_tuning(path)
        assert c2.tuning(1000, 256, 1000, 1 << 14, 3, "f32") == (min(tu[0], 14), tu[1], tu[2])
    finally:
        c2.close()
    _say(f"  chosen (log2c, kmax, cs_blocks) = {tu}, {ms:.3f} ms")


def test_batched_covariance_workload_subset(cmm, ctx):
    """Eight products of the batched covariance workload recipe (bf16,
    d = 5, b = next power of two of 8n) at reduced n, autotuned, against the
    oracle."""
    _say("case: batched covariance recipe, 8 products, n in [128, 1024], autotuned")
    ws = W.batched_workloads(count=8, seed=77, lo=128, hi=1024)
    dev = [(_dev(w.At_store),) for w in ws]
    probs = [cmm.problem(dv[0], dv[0], w.b, w.d, seed=w.seed, dtype=w.dtype, subtract_diag=True)
             for w, dv in zip(ws, dev)]
    bt = cmm.Batch(ctx, probs, autotune=True, keep=dev)
    bt.run()
    for q, w in enumerate(ws):
        A, B = W.dequantised(w)
        c_ref, _, _ = O.run(A, B, w.b, w.d, w.seed, subtract_diag=True)
        c = bt.sketch(q).c()
        for t in range(w.d):
            assert _rel_l2(c[t], c_ref[t]) <= REL_TOL, (q, t)
    bt.free()


@pytest.mark.timeout(900)
def test_batched_workload_every_product_vs_oracle(cmm, ctx):
    """The batched benchmark workload as bench.py runs it (64 bf16 covariance
    products, n = m log-uniform in [512, 8192], b = next power of two of 8n,
    d = 5, diagonal subtracted, size classes autotuned, one graph replay):
    every product's whole sketch against the oracle (per repetition rel. L2
    and largest entry error <= 1e-5), and every product's top-(planted pairs)
    over i < j against the oracle's inside the tolerance band."""
    import oracle_runs as R
    _say("case: batched workload, 64 products, every sketch and top-K vs the oracle")
    ws = W.batched_workloads()
    dev, probs = [], []
    for w in ws:
        A = _dev(w.At_store)
        B = A.clone()
        dev.append((A, B))
        probs.append(cmm.problem(A, B, w.b, w.d, seed=w.seed, dtype=w.dtype, subtract_diag=True))
    bt = cmm.Batch(ctx, probs, autotune=True, keep=dev)
    bt.run()
    res = bt.topk([w.K for w in ws], "upper")
    worst_l2 = worst_inf = 0.0
    for q, w in enumerate(ws):
        c = bt.sketch(q).c()
        A, B = W.dequantised(w)
        tabs = O.hash_tables(O.hash_params(w.seed, w.d), w.n1, w.n3, w.b)
        c_ref, _ = R.sketch(A, B, tabs, w.b, subtract_diag=True)
        l2, inf = R.check_sketch(c, c_ref)
        worst_l2, worst_inf = max(worst_l2, l2), max(worst_inf, inf)
        oi, oj, ov = res[q]
        ri, rj, rv = R.topk_upper(c_ref, tabs, w.n1, w.K)
        R.band_check(oi, oj, ov, ri, rj, rv, abs(rv[-1]), R.decode_band(c, c_ref),
                     lambda i, j: O.decode(c_ref, tabs, i, j))
        if q % 16 == 15:
            _say(f"  {q + 1} products checked")
    _say(f"  worst rel L2 {worst_l2:.2e}, worst max|dc|/max|c| {worst_inf:.2e}")
    bt.free()
