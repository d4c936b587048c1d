"""GPU parity of the Frobenius-norm bound (Section 5.2) through the C ABI.

* sign tables (degree-3 polynomial parity): bit-exact against the oracle;
* X_t: the GPU sums in float64 from the same float32 values the oracle
  multiplies, so |X_gpu - X_oracle| <= 1e-10 * sum_k |u_t[k] v_t[k]| (the
  scale of the terms; the sum itself may cancel);
* bound = 32 * median X_t^2: within 1e-9 relative of the oracle's.
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


def _check_X(Xg, A, B, s1, s2, diag_zero=False):
    AB = A @ B
    if diag_zero:
        np.fill_diagonal(AB, 0.0)
    Xo = O.ams_sketch(AB, s1, s2)
    for t in range(len(Xo)):
        u = s1[t].astype(np.float64) @ A
        v = B @ s2[t].astype(np.float64)
        scale = float(np.sum(np.abs(u * v))) + (float(np.abs(np.diag(A @ B)).sum()) if diag_zero else 0.0)
        assert abs(Xg[t] - Xo[t]) <= 1e-10 * scale, (t, Xg[t], Xo[t], scale)
    return Xo


@pytest.mark.parametrize("shape", [(777, 513, 7), (40, 3000, 63), (1, 1, 1)])
def test_frobenius_signs_bit_exact(cmm, ctx, shape):
    n1, n3, d = shape
    _say(f"case: AMS sign tables {shape}")
    s1g, s2g = cmm.cmm_frobenius_signs(ctx.handle, n1, n3, d, 12345)
    s1o, s2o = O.ams_signs(O.ams_params(12345, d), n1, n3)
    np.testing.assert_array_equal(s1g, s1o)
    np.testing.assert_array_equal(s2g, s2o)


def test_frobenius_f32_parity(cmm, ctx):
    _say("case: Frobenius bound f32 300x200x250 d=5")
    g = np.random.default_rng(4)
    At = g.standard_normal((200, 300)).astype(np.float32)
    B = g.standard_normal((200, 250)).astype(np.float32)
    Xg, bound = cmm.frobenius_bound(ctx, _dev(At), _dev(B), 5, seed=7)
    A64, B64 = At.astype(np.float64).T, B.astype(np.float64)
    s1, s2 = O.ams_signs(O.ams_params(7, 5), 300, 250)
    Xo = _check_X(Xg, A64, B64, s1, s2)
    assert abs(bound - O.frobenius_bound(Xo)) <= 1e-9 * O.frobenius_bound(Xo)


@pytest.mark.parametrize("dtype", ["bf16", "fp8"])
def test_frobenius_low_precision_parity(cmm, ctx, dtype):
    _say(f"case: Frobenius bound {dtype} covariance with zero diagonal")
    X, _, _ = W.covariance_observations(400, 300, 8, 0.9, 6)
    if dtype == "bf16":
        store, sc = W.bf16_encode(X), None
        Xq = (store.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    else:
        sc = (np.abs(X).max(axis=0) / 448.0).astype(np.float32)
        store = W.e4m3fn_encode(X / sc[None, :])
        mag = W.e4m3fn_grid()[(store & 0x7F).astype(np.int64)]
        Xq = (np.where((store & 0x80) != 0, -mag, mag).astype(np.float32) * sc[None, :]).astype(np.float64)
    d_s = _dev(store)
    d_s2 = d_s.clone()
    dsc = None if sc is None else _dev(sc)
    Xg, bound = cmm.frobenius_bound(ctx, d_s, d_s2, 9, seed=3, dtype=dtype, scaleA=dsc, scaleB=dsc,
                                    subtract_diag=True)
    s1, s2 = O.ams_signs(O.ams_params(3, 9), 400, 400)
    Xo = _check_X(Xg, Xq.T, Xq, s1, s2, diag_zero=True)
    assert abs(bound - O.frobenius_bound(Xo)) <= 1e-9 * O.frobenius_bound(Xo)


def test_frobenius_bound_covers_the_norm(cmm, ctx):
    """The bound is above ||AB||_F^2 for a product whose norm the oracle
    knows (Section 5.2's claim, checked at one seed per size)."""
    _say("case: Frobenius bound above the true norm")
    g = np.random.default_rng(5)
    for n, m in [(256, 64), (1024, 128)]:
        At = g.standard_normal((m, n)).astype(np.float32)
        B = g.standard_normal((m, n)).astype(np.float32)
        _, bound = cmm.frobenius_bound(ctx, _dev(At), _dev(B), 9, seed=n)
        F2 = float(((At.astype(np.float64).T @ B.astype(np.float64)) ** 2).sum())
        assert bound >= F2
        assert bound <= 32 * 40 * F2


def test_frobenius_errors(cmm, ctx):
    _say("case: Frobenius bound argument errors")
    x = _dev(np.zeros((4, 4), np.float32))
    for d in (0, 64):
        with pytest.raises(cmm.CmmError) as e:
            cmm.frobenius_bound(ctx, x, x, d)
        assert e.value.code == cmm.CMM_EINVAL
    with pytest.raises(cmm.CmmError) as e:
        cmm.cmm_frobenius_bound(ctx.handle, x, 4, x, 4, 4, 4, 4, 0, None, None, 3, 1, cmm.CMM_ASYNC)
    assert e.value.code == cmm.CMM_EINVAL


@pytest.mark.timeout(300)
def test_frobenius_fullsize_covariance_4096(cmm, ctx):
    """Covariance n = m = 4096 float32 (the sketch benchmark's operands), d = 9,
    zero diagonal: X against the oracle; the estimate against ||Q~||_F."""
    _say("case: Frobenius bound covariance n=m=4096 f32 d=9")
    w = W.make_workload(2)
    dA = _dev(w.At_store)
    dB = dA.clone()
    Xg, bound = cmm.frobenius_bound(ctx, dA, dB, 9, seed=w.seed, subtract_diag=True)
    A, B = W.dequantised(w)
    s1, s2 = O.ams_signs(O.ams_params(w.seed, 9), w.n1, w.n3)
    Xo = _check_X(Xg, A, B, s1, s2, diag_zero=True)
    AB = A @ B
    np.fill_diagonal(AB, 0.0)
    F2 = float((AB ** 2).sum())
    _say(f"  32*median X^2 / ||AB~||_F^2 = {bound / F2:.2f}; median X^2 / ||AB~||_F^2 = {bound / 32 / F2:.3f}")
    assert abs(bound - O.frobenius_bound(Xo)) <= 1e-9 * O.frobenius_bound(Xo)
