"""Stream ordering through the C ABI: asynchronous products (CMM_ASYNC),
work of two contexts on two streams at once, and switching a context's
stream.  Each result must equal the synchronous single-stream result."""
import sys

import numpy as np
import pytest

from oracle import cmm_oracle as O

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _operands(seed, n1=700, m=300, n3=650):
    import torch
    g = np.random.default_rng(seed)
    At = torch.from_numpy(g.standard_normal((m, n1)).astype(np.float32)).cuda()
    B = torch.from_numpy(g.standard_normal((m, n3)).astype(np.float32)).cuda()
    return At, B


def test_async_products_follow_stream_order(cmm):
    """Products issued with CMM_ASYNC between torch operations on the same
    stream see the operands as those operations leave them."""
    import torch
    _say("case: asynchronous products in stream order")
    ctx = cmm.Context(0)
    try:
        At, B = _operands(1)
        b, d = 8192, 5
        ref = cmm.sketch_product(ctx, At, B, b, d, seed=4).c()
        sks = []
        for r in range(3):
            sks.append(cmm.sketch_product(ctx, At, B, b, d, seed=4, asynchronous=True))
            At.mul_(2.0)      # queued behind the product on the same stream
        torch.cuda.synchronize()
        for r, sk in enumerate(sks):
            # scaling A by 2^r scales the sketch by exactly 2^r
            np.testing.assert_array_equal(sk.c(), ref * (2.0 ** r))
        c_ref, _, _ = O.run(At.cpu().numpy().astype(np.float64).T / 8.0,
                            B.cpu().numpy().astype(np.float64), b, d, 4)
        for t in range(d):
            assert np.linalg.norm(ref[t] - c_ref[t]) / np.linalg.norm(c_ref[t]) <= 1e-5
    finally:
        ctx.close()


def test_two_contexts_on_two_streams(cmm):
    import torch
    _say("case: two contexts on two streams at once")
    s1, s2 = torch.cuda.Stream(), torch.cuda.Stream()
    A1, B1 = _operands(2)
    A2, B2 = _operands(3, 500, 400, 520)
    torch.cuda.synchronize()
    with torch.cuda.stream(s1):
        c1 = cmm.Context(0)
    with torch.cuda.stream(s2):
        c2 = cmm.Context(0)
    try:
        outs = []
        for _ in range(3):
            outs.append((cmm.sketch_product(c1, A1, B1, 4096, 3, seed=7, asynchronous=True),
                         cmm.sketch_product(c2, A2, B2, 16384, 5, seed=8, subtract_diag=False,
                                            asynchronous=True)))
        torch.cuda.synchronize()
        ref = cmm.Context(0)
        try:
            r1 = cmm.sketch_product(ref, A1, B1, 4096, 3, seed=7).c()
            r2 = cmm.sketch_product(ref, A2, B2, 16384, 5, seed=8).c()
        finally:
            ref.close()
        for x1, x2 in outs:
            np.testing.assert_array_equal(x1.c(), r1)
            np.testing.assert_array_equal(x2.c(), r2)
    finally:
        c1.close()
        c2.close()


def test_switching_stream(cmm):
    import torch
    _say("case: switching a context's stream")
    ctx = cmm.Context(0)
    try:
        At, B = _operands(5)
        ref = cmm.sketch_product(ctx, At, B, 2048, 3, seed=2).c()
        s = torch.cuda.Stream()
        s.wait_stream(torch.cuda.current_stream())
        ctx.set_stream(s)
        with torch.cuda.stream(s):
            sk = cmm.sketch_product(ctx, At, B, 2048, 3, seed=2, asynchronous=True)
            oi, oj, ov = sk.topk(5, "all")
        s.synchronize()
        np.testing.assert_array_equal(sk.c(), ref)
        ctx.set_stream(None)
        sk2 = cmm.sketch_product(ctx, At, B, 2048, 3, seed=2)
        oi2, oj2, ov2 = sk2.topk(5, "all")
        np.testing.assert_array_equal(oi, oi2)
        np.testing.assert_array_equal(oj, oj2)
        np.testing.assert_array_equal(ov, ov2)
    finally:
        ctx.close()
