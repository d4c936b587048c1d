"""cmm_sketch_product_noalloc through the C ABI: its output equals that of
cmm_sketch_product_ex on the same inputs, and the oracle's within the
float32 budget, on two calls in a row (the second with a smaller input that
reuses the same device scratch), and the device's free memory does not
change across the calls.  A product larger than the scratch is refused
with CMM_EUNSUPPORTED before any work."""
import sys

import numpy as np
import pytest

from oracle import cmm_oracle as O
import workloads as W

pytestmark = pytest.mark.gpu

# (n1, m, n3, b, d, dtype, subtract_diag, seed): the second is smaller
CASES = [
    (900, 300, 900, 8192, 5, "f32", True, 71),
    (300, 100, 250, 2048, 3, "bf16", False, 72),
]


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _operands(n1, m, n3, dtype, same, seed):
    g = np.random.default_rng(seed)
    At = g.standard_normal((m, n1))
    B = At.copy() if same else g.standard_normal((m, n3))
    if dtype == "f32":
        return At.astype(np.float32), B.astype(np.float32)
    return W.bf16_encode(At), W.bf16_encode(B)


def _deq(x, dtype):
    if dtype == "f32":
        return x.astype(np.float64)
    return (x.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)


def test_noalloc_matches_product_ex_and_oracle(cmm):
    import torch
    ctx = cmm.Context(0)
    items = []
    for (n1, m, n3, b, d, dt, diag, seed) in CASES:
        At, B = _operands(n1, m, n3, dt, diag, seed)
        items.append(dict(n1=n1, m=m, n3=n3, b=b, d=d, dt=dt, diag=diag, seed=seed, At=At, B=B,
                          dAt=torch.from_numpy(At).cuda(), dB=torch.from_numpy(B).cuda(),
                          out=torch.full((d, b), float("nan"), dtype=torch.float64, device="cuda")))
    # the existing entry point on every case first (it allocates)
    ref_ex = []
    for x in items:
        sk = cmm.sketch_product(ctx, x["dAt"], x["dB"], x["b"], x["d"], seed=x["seed"], dtype=x["dt"],
                                subtract_diag=x["diag"])
        ref_ex.append(sk.c())
        sk.free()
    warm = torch.zeros((items[1]["d"], items[1]["b"]), dtype=torch.float64, device="cuda")
    x = items[1]
    cmm.sketch_product_noalloc(ctx, x["dAt"], x["dB"], x["b"], x["d"], warm, seed=x["seed"], dtype=x["dt"],
                               subtract_diag=x["diag"])
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for q, x in enumerate(items):
        _say(f"case: noalloc call {q}: n1={x['n1']} m={x['m']} n3={x['n3']} b={x['b']} d={x['d']} {x['dt']}")
        cmm.sketch_product_noalloc(ctx, x["dAt"], x["dB"], x["b"], x["d"], x["out"], seed=x["seed"],
                                   dtype=x["dt"], subtract_diag=x["diag"])
    torch.cuda.synchronize()
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1)
    for q, x in enumerate(items):
        c = x["out"].cpu().numpy()
        assert np.all(np.isfinite(c))
        c_ex = ref_ex[q]
        c_ref, _, _ = O.run(_deq(x["At"], x["dt"]).T, _deq(x["B"], x["dt"]), x["b"], x["d"], x["seed"],
                            subtract_diag=x["diag"])
        for t in range(x["d"]):
            for other in (c_ex[t], c_ref[t]):
                rel = np.linalg.norm(c[t] - other) / np.linalg.norm(other)
                assert rel <= 1e-5, (q, t, rel)
        _say(f"  max |noalloc - product_ex| = {np.abs(c - c_ex).max():.3e}, "
             f"rel L2 vs oracle {max(np.linalg.norm(c[t] - c_ref[t]) / np.linalg.norm(c_ref[t]) for t in range(x['d'])):.2e}")
    ctx.close()


def test_noalloc_refuses_a_product_beyond_the_scratch(cmm):
    import torch
    ctx = cmm.Context(0)
    n, m, b, d = 4096, 4096, 1 << 16, 5          # needs about a gigabyte of workspace
    X = torch.zeros((m, n), dtype=torch.float32, device="cuda")
    out = torch.zeros((d, b), dtype=torch.float64, device="cuda")
    with pytest.raises(cmm.CmmError) as e:
        cmm.sketch_product_noalloc(ctx, X, X, b, d, out, seed=1)
    assert e.value.code == cmm.CMM_EUNSUPPORTED
    ctx.close()
