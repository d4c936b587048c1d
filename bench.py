"""Benchmark of the compressed-matrix-multiplication hot path on one MI355X.

One step = one whole pass of the path over one synthetic product: hashing,
bucket layout, count sketches of all columns of A and rows of B, fused FFT +
spectral multiply-accumulate over k, float64 inverse FFT, diagonal
correction, then decode + median + top-K.  Inputs are resident in HBM before
the timed region.

Default workload: sample covariance of n = 4096 variables from m = 4096
samples with 64 planted correlated pairs, float32, b = 2^16, d = 5, top-64
over i < j with the diagonal subtracted.  A and B are two distinct device
buffers holding the observation matrix.

Prints one JSON line (see the keys below).  ``value`` is the input GB/s of the
whole step: bytes(A) + bytes(B) as stored, divided by the step time.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBPS = 8000.0
FP32_VECTOR_PEAK_TFLOPS = 157.3
METRIC = "sketch-product input GB/s (% HBM peak), BF16 vs FP32 at equal error"


def nominal_fft_mac_flop(m: int, b: int, d: int) -> float:
    """Forward transforms of both sketches (2.5 b log2 b each, the usual
    real-FFT convention) plus the complex multiply-accumulate of b/2+1 bins,
    for every k and repetition."""
    return m * d * (2 * 2.5 * b * math.log2(b) + 8 * (b // 2 + 1))


def expected_nonempty(n: int, b: int) -> float:
    return b * (1.0 - (1.0 - 1.0 / b) ** n)


def parse():
    p = argparse.ArgumentParser()
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=20)
    p.add_argument("--warmup", type=int, default=3)
    p.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4])
    p.add_argument("--dtype", default=None, help="override the workload's dtype (f32/bf16/fp8)")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    return p.parse_args()


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(the sketch would shard over k with one all-reduce of c; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    import workloads as W

    cmm.load()
    torch.cuda.init()
    w = W.make_workload(args.workload, dtype=args.dtype)
    esz = {"f32": 4, "bf16": 2, "fp8": 1}[w.dtype]
    n1, m, n3, b, d, K = w.n1, w.m, w.n3, w.b, w.d, w.K
    At = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(w.B_store)).cuda()
    if w.same_operand:
        Bd = At.clone()   # a second buffer: B is read from its own memory
    sA = torch.from_numpy(w.scaleA).cuda() if w.scaleA is not None else None
    sB = torch.from_numpy(w.scaleB).cuda() if w.scaleB is not None else None
    input_bytes = (n1 * m + m * n3) * esz
    ctx = cmm.Context(0)

    def step():
        sk = cmm.sketch_product(ctx, At, Bd, b, d, seed=w.seed, dtype=w.dtype, scaleA=sA,
                                scaleB=sB, subtract_diag=w.subtract_diag, n1=n1, n3=n3, m=m)
        res = sk.topk(K, w.mode)
        return sk, res

    for _ in range(args.warmup):
        sk, _ = step()
        sk.free()
    torch.cuda.synchronize()

    ctx.profile(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        sk, res = step()
        sk.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    kern = {k: ctx.profile_read(k) for k in ("hash", "layout", "countsketch", "fft_mac", "ifft", "decode")}
    ctx.profile(False)

    ms = (t1 - t0) * 1e3 / args.steps
    value = input_bytes / (ms * 1e-3) / 1e9
    fft_ms, fft_n = kern["fft_mac"]
    fft_avg_ms = fft_ms / max(fft_n, 1)
    flop = nominal_fft_mac_flop(m, b, d)
    achieved_tflops = flop / (fft_avg_ms * 1e-3) / 1e12
    cs_ms, cs_n = kern["countsketch"]
    cs_avg_ms = cs_ms / max(cs_n, 1)
    nb = expected_nonempty(n1, b) + expected_nonempty(n3, b)
    cs_bytes = input_bytes + d * m * nb * 4
    cs_gbps = cs_bytes / (cs_avg_ms * 1e-3) / 1e9

    # one more product kept for the parity check against the oracle
    sk, (oi, oj, ov) = step()
    c_gpu = sk.c()

    out = {
        "metric": METRIC,
        "value": round(value, 3),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {
            "workload": (f"covariance n=m={n1} b={b} d={d} top-{K} i<j, diagonal subtracted"
                         if w.mode == "upper" else
                         f"{w.name} n1={n1} m={m} n3={n3} b={b} d={d} top-{K} {w.mode}"),
            "n1": n1, "m": m, "n3": n3, "b": b, "d": d, "K": K, "topk_mode": w.mode,
            "input_bytes": input_bytes,
        },
        "hbm_frac": round(value / HBM_PEAK_GBPS, 5),
        "input_elements_per_s": round((n1 * m + m * n3) / (ms * 1e-3), 1),
        "nominal_fft_gflops": round(flop / (ms * 1e-3) / 1e9, 1),
        "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in kern.items()},
        "roofline": {
            "kernel": "fft_mac",
            "bound": "alu",
            "achieved": round(achieved_tflops, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": None,
            "flop_per_launch": flop,
            "avg_launch_ms": round(fft_avg_ms, 4),
        },
        "countsketch": {
            "achieved": round(cs_gbps, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(cs_gbps / HBM_PEAK_GBPS, 4), "bytes_per_launch_pair": cs_bytes,
            "avg_ms": round(cs_avg_ms, 4),
        },
    }

    if not args.no_cpu:
        out["cpu_baseline"], out["parity"] = cpu_baseline(w, c_gpu, oi, oj, ov, input_bytes)
    sk.free()
    ctx.close()
    print(json.dumps(out), flush=True)


def cpu_baseline(w, c_gpu, oi, oj, ov, input_bytes):
    """The FP64 oracle on the host cores over the whole workload (exact
    float64 product, binning into the sketch for all repetitions, diagonal,
    decode of every candidate and top-K), plus the GPU-vs-oracle error."""
    import numpy as np
    import workloads as W
    from oracle import cmm_oracle as O
    try:
        from threadpoolctl import threadpool_info
        cores = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        cores = os.cpu_count() or 1
    A, B = W.dequantised(w)
    t0 = time.perf_counter()
    c_ref, tabs, AB = O.run(A, B, w.b, w.d, w.seed, subtract_diag=w.subtract_diag)
    if w.mode == "column":
        sample = "sketch of the whole product; decode + top-K of the first 256 columns"
        C = O.decode(c_ref, tabs, np.arange(w.n1)[:, None], np.arange(256)[None, :])
        O.topk_per_column(C, w.K)
    else:
        i, j = O.candidates(w.mode, w.n1, w.n3)
        vals = O.decode(c_ref, tabs, i, j)
        O.topk(vals, i * w.n3 + j, w.K)
        sample = "the whole workload once: float64 AB, binning, diagonal, decode of every candidate, top-K"
    t1 = time.perf_counter()
    secs = t1 - t0
    rel = max(float(np.linalg.norm(c_gpu[t] - c_ref[t]) / np.linalg.norm(c_ref[t])) for t in range(w.d))
    if w.mode != "column":
        ref_at = O.decode(c_ref, tabs, oi, oj)
        est_err = float(np.abs(ov - ref_at).max())
    else:
        est_err = None
    base = {"value": round(input_bytes / secs / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "sample": sample, "seconds": round(secs, 2)}
    parity = {"max_rel_l2_c": rel, "max_abs_err_topk_values": est_err, "tolerance": 1e-5}
    return base, parity


if __name__ == "__main__":
    main()
