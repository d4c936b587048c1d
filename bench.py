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

Prints one JSON line.  ``value`` is the input GB/s of the whole step:
bytes(A) + bytes(B) as stored, divided by the step time.  The same workload
is also run with its operands in the other two formats (``bf16_same_workload``
and ``fp8_same_workload`` beside the float32 default): element rate, top-K
overlap and planted recall against the headline run, and, with the oracle,
each format's arithmetic error (against the float64 oracle of the values it
multiplies) apart from its quantisation error.

The default run also measures the other single-product workloads
(``configs``: covariance 256 f32, DCT 8192 bf16 with top-16 per column,
covariance 16384 fp8 with top-256), each with its own tuning, step time,
per-kernel times, spectral roofline and count-sketch HBM rate, and compares
the count sketch with plain HBM streams of its shape (``stream_ceiling``).
``countsketch_d1`` is the count sketch of the default workload's operands with
one repetition instead of five (the same input read, a fifth of the writes).
Step times come from a region with the library's timing events off; a second
region of the same steps with the events on gives the per-kernel times.

The batched form (``batched_form``; ``--workload 5`` makes it the headline):
64 covariance products, n = m log-uniform in [512, 8192], b = next power of
two of 8n, d = 5, bf16 operands, diagonal subtracted, recorded once into one
HIP graph after autotuning every size class; one step is one graph replay
plus the top-(planted pairs) selection of every product, in one batch top-K
call whose host waits all products share.
"""
from __future__ import annotations

import argparse
import copy
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
KERNELS = ("hash", "layout", "countsketch", "fft_mac", "ifft", "decode")


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
    p.add_argument("--workload", type=int, default=2, choices=[1, 2, 3, 4, 5],
                   help="1 covariance 256 f32, 2 covariance 4096 f32 (default), 3 DCT 8192 bf16, "
                        "4 covariance 16384 fp8, 5 the batched form (64 bf16 covariance products)")
    p.add_argument("--dtype", default=None, help="override the workload's dtype (f32/bf16/fp8)")
    p.add_argument("--d", type=int, default=None, help="override the number of repetitions")
    p.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    p.add_argument("--no-compare", action="store_true", help="skip the runs of the same workload in the other operand formats")
    p.add_argument("--no-batched", action="store_true", help="skip the batched-form measurement")
    p.add_argument("--no-extract", action="store_true", help="skip the sublinear-extraction measurement")
    p.add_argument("--no-sparse", action="store_true", help="skip the sparse-operand measurement")
    p.add_argument("--no-autotune", action="store_true",
                   help="use the built-in geometry instead of tuning the size class first")
    p.add_argument("--geometry", type=str, default=None,
                   help="log2c,kmax,cs_blocks: run the headline with this geometry instead of tuning")
    p.add_argument("--no-configs", action="store_true",
                   help="skip the per-workload measurements of the other benchmark workloads")
    p.add_argument("--no-stream", action="store_true", help="skip the HBM stream-ceiling probes")
    p.add_argument("--stream-ceiling", action="store_true",
                   help="only measure plain HBM streams (read, write, copy, 1:5 read:write; ordinary "
                        "and streaming stores) and print them")
    p.add_argument("--replay-trace", type=int, default=0, metavar="N",
                   help="build the batched workload's graph, then run N graph replays 100 ms apart "
                        "(no top-K) so that a kernel trace can separate one replay's dispatches")
    p.add_argument("--tune-cache", type=str, default=None, metavar="PATH",
                   help="with --replay-trace: load the batch's size-class geometry from PATH if it exists, "
                        "else autotune and save it there (so counter runs replay the same launches)")
    p.add_argument("--copy-calibration", action="store_true",
                   help="only run a plain 1 GiB device copy (reference for HBM byte counters)")
    return p.parse_args()


def copy_calibration():
    """A plain copy kernel of known size: 2^28 float32 values (1 GiB read,
    1 GiB written), launched 3 times.  Its FETCH_SIZE / WRITE_SIZE counters
    convert the counters of the measured kernels to bytes."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": x.numel() * 4, "copy_bytes_written": y.numel() * 4,
                      "launches": 3}), flush=True)


def run_timed(ctx, w, steps, warmup):
    """Time ``steps`` whole steps (after ``warmup``) of workload ``w``.  The
    timed region runs with the library's timing events off; a second region
    of the same steps with the events on gives the per-kernel times and the
    count sketch's byte record.  Returns the last product for checks."""
    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    esz = {"f32": 4, "bf16": 2, "fp8": 1}[w.dtype]
    At = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
    Bd = torch.from_numpy(np.ascontiguousarray(w.B_store)).cuda()
    if w.same_operand:
        Bd = At.clone()   # a second buffer: B is read from its own memory
    sA = torch.from_numpy(w.scaleA).cuda() if w.scaleA is not None else None
    sB = torch.from_numpy(w.scaleB).cuda() if w.scaleB is not None else None

    def step():
        sk = cmm.sketch_product(ctx, At, Bd, w.b, w.d, seed=w.seed, dtype=w.dtype, scaleA=sA,
                                scaleB=sB, subtract_diag=w.subtract_diag, n1=w.n1, n3=w.n3, m=w.m)
        return sk, sk.topk(w.K, w.mode)

    for _ in range(warmup):
        sk, _ = step()
        sk.free()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        sk, res = step()
        sk.free()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    ctx.profile(True)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    for _ in range(steps):
        sk, res = step()
        sk.free()
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    kern = {k: ctx.profile_read(k) for k in KERNELS}
    cs_bytes = ctx.profile_bytes("countsketch")
    ctx.profile(False)
    sk, res = step()     # one more product, kept for the checks
    return {"ms": (t1 - t0) * 1e3 / steps, "ms_profiled": (t3 - t2) * 1e3 / steps, "kern": kern,
            "cs_bytes": cs_bytes, "sketch": sk, "topk": res,
            "input_bytes": (w.n1 * w.m + w.m * w.n3) * esz}


def describe(w):
    if w.mode == "upper":
        return f"{w.name}: covariance n=m={w.n1} b={w.b} d={w.d} top-{w.K} i<j, diagonal subtracted, {w.dtype}"
    return f"{w.name}: n1={w.n1} m={w.m} n3={w.n3} b={w.b} d={w.d} top-{w.K} {w.mode}, {w.dtype}"


def measure(ctx, w, steps, warmup, autotune=True, geometry=None):
    """One workload: tuning, timed steps, per-kernel times, the spectral
    kernels' roofline and the count sketch's HBM rate.  Returns
    (summary dict, run_timed result)."""
    n1, m, n3, b, d = w.n1, w.m, w.n3, w.b, w.d
    tuned = None
    if geometry:
        ctx.set_tuning(n1, m, n3, b, d, w.dtype, tuple(geometry))
    elif autotune:
        t0 = time.perf_counter()
        tu, tms = ctx.autotune(n1, m, n3, b, d, w.dtype)
        tuned = {"log2c_kmax_csblocks": list(tu), "product_ms": round(tms, 4),
                 "seconds": round(time.perf_counter() - t0, 2)}
    r = run_timed(ctx, w, steps, warmup)
    ms, kern, input_bytes = r["ms"], r["kern"], r["input_bytes"]
    value = input_bytes / (ms * 1e-3) / 1e9
    fft_ms, fft_n = kern["fft_mac"]
    fft_avg_ms = fft_ms / max(fft_n, 1)
    flop = nominal_fft_mac_flop(m, b, d)
    achieved_tflops = flop / (fft_avg_ms * 1e-3) / 1e12
    cs_ms, cs_n = kern["countsketch"]
    cs_avg_ms = cs_ms / max(cs_n, 1)
    cs_rd, cs_wr = r["cs_bytes"]
    cs_bytes = (cs_rd + cs_wr) / max(cs_n, 1)        # bytes the two launches move, padding included
    nb = expected_nonempty(n1, b) + expected_nonempty(n3, b)
    cs_bytes_nb = input_bytes + d * m * nb * 4      # expected non-empty buckets only
    geom = list(ctx.tuning(n1, m, n3, b, d, w.dtype))
    out = {
        "workload": describe(w), "dtype": w.dtype, "n1": n1, "m": m, "n3": n3, "b": b, "d": d,
        "K": w.K, "topk_mode": w.mode, "input_bytes": input_bytes, "geometry": geom,
        "autotune": tuned, "steps": steps, "warmup": warmup,
        "ms_per_step": round(ms, 4), "value": round(value, 3), "unit": "GB/s",
        "hbm_frac": round(value / HBM_PEAK_GBPS, 5),
        "input_elements_per_s": round((n1 * m + m * n3) / (ms * 1e-3), 1),
        "nominal_fft_gflops": round(flop / (ms * 1e-3) / 1e9, 1),
        "ms_per_step_with_kernel_events": round(r["ms_profiled"], 4),
        "kernel_ms_per_step": {k: round(v[0] / max(v[1], 1), 4) for k, v in kern.items()},
        "roofline": {
            "kernel": "fft_mac",
            "kernels": ["k_fft_mac", "k_fft_mac_pair"],
            "bound": "alu",
            "achieved": round(achieved_tflops, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved_tflops / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": traffic_record(w, geom),
            "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "flop_per_launch": flop,
            "avg_launch_ms": round(fft_avg_ms, 4),
        },
        "countsketch": {
            "avg_ms": round(cs_avg_ms, 4),
            "bytes_per_launch_pair": cs_bytes,
            "achieved": round(cs_bytes / (cs_avg_ms * 1e-3) / 1e9, 1), "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(cs_bytes / (cs_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "bytes_read": cs_rd / max(cs_n, 1), "bytes_written": cs_wr / max(cs_n, 1),
            "bytes_expected_nonempty_only": cs_bytes_nb,
            "frac_expected_nonempty_only": round(cs_bytes_nb / (cs_avg_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
        },
        "decode_topk_ms": round(kern["decode"][0] / max(kern["decode"][1], 1), 4),
    }
    return out, r


def run_batched(ctx, steps, warmup, with_oracle=True):
    """The batched covariance workload as one graph replay per step."""
    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    import workloads as W
    t0 = time.perf_counter()
    ws = W.batched_workloads()
    gen_s = time.perf_counter() - t0
    dev, probs = [], []
    for w in ws:
        A = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
        B = A.clone()   # a second buffer: B is read from its own memory
        dev.append((A, B))
        probs.append(cmm.problem(A, B, w.b, w.d, seed=w.seed, dtype=w.dtype, subtract_diag=True))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    bt = cmm.Batch(ctx, probs, autotune=True, keep=dev)
    create_s = time.perf_counter() - t0

    def step():
        bt.run(asynchronous=True)
        return bt.topk([w.K for w in ws], "upper")

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    ctx.profile(True)
    t0 = time.perf_counter()
    for _ in range(steps):
        res = step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    graph_ms, graph_n = ctx.profile_read("batch")
    dec_ms, _ = ctx.profile_read("decode")
    ctx.profile(False)
    ms = (t1 - t0) * 1e3 / steps
    input_bytes = sum(2 * w.n1 * w.m * 2 for w in ws)
    # the same products one after another through the standalone call
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for w, (A, B) in zip(ws, dev):
        cmm.sketch_product(ctx, A, B, w.b, w.d, seed=w.seed, dtype=w.dtype,
                           subtract_diag=True).free()
    torch.cuda.synchronize()
    alone_ms = (time.perf_counter() - t0) * 1e3
    hits = sum(len({(int(min(a, c)), int(max(a, c))) for a, c in zip(oi, oj)}
                   & {(int(min(p, q)), int(max(p, q))) for p, q in w.planted})
               for w, (oi, oj, _) in zip(ws, res))
    classes = sorted({(w.b, W.next_pow2(w.n1)) for w in ws})
    out = {
        "workload": "64 covariance products, n=m log-uniform in [512, 8192], b=next_pow2(8n), "
                    "d=5, bf16, diagonal subtracted, top-(planted pairs) i<j each",
        "value": round(input_bytes / (ms * 1e-3) / 1e9, 3), "unit": "GB/s",
        "ms_per_step": round(ms, 4), "steps": steps, "warmup": warmup,
        "graph_replay_ms": round(graph_ms / max(graph_n, 1), 4),
        "topk_ms_per_step": round(dec_ms / max(steps, 1), 4),
        "standalone_sequential_sketch_ms": round(alone_ms, 3),
        "input_bytes": input_bytes, "products": len(ws), "size_classes": len(classes),
        "tuning": batched_tuning(ctx, classes),
        "create_s": round(create_s, 2), "generate_s": round(gen_s, 2),
        "planted_recall": round(hits / sum(len(w.planted) for w in ws), 4),
    }
    out["roofline"] = batched_roofline(out, ws)
    if with_oracle:
        from oracle import cmm_oracle as O
        worst = 0.0
        for q in sorted(range(len(ws)), key=lambda q: ws[q].n1)[:3]:
            w = ws[q]
            A, Bq = W.dequantised(w)
            c_ref, _, _ = O.run(A, Bq, w.b, w.d, w.seed, subtract_diag=True)
            c = bt.sketch(q).c()
            worst = max(worst, max(float(np.linalg.norm(c[t] - c_ref[t]) / np.linalg.norm(c_ref[t]))
                                   for t in range(w.d)))
        out["max_rel_l2_c_vs_oracle_3_smallest"] = worst
    bt.free()
    return out


def run_frobenius(ctx, w, steps):
    """The Frobenius-norm bound of Section 5.2 on the same operands and d:
    sign tables, two sign-weighted row-sum passes (one read of A and of B),
    the per-repetition dot products; HIP-event time per call, input GB/s."""
    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    esz = {"f32": 4, "bf16": 2, "fp8": 1}[w.dtype]
    At = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
    Bd = At.clone() if w.same_operand else torch.from_numpy(np.ascontiguousarray(w.B_store)).cuda()
    sA = torch.from_numpy(w.scaleA).cuda() if w.scaleA is not None else None
    sB = torch.from_numpy(w.scaleB).cuda() if w.scaleB is not None else None

    def call():
        return cmm.frobenius_bound(ctx, At, Bd, w.d, seed=w.seed, dtype=w.dtype, scaleA=sA, scaleB=sB,
                                   subtract_diag=w.subtract_diag, n1=w.n1, n3=w.n3, m=w.m)
    call()
    torch.cuda.synchronize()
    ctx.profile(True)
    for _ in range(steps):
        X, bound = call()
    ms, n = ctx.profile_read("frobenius")
    ctx.profile(False)
    avg = ms / max(n, 1)
    nbytes = (w.n1 * w.m + w.m * w.n3) * esz
    return {"ms": round(avg, 4), "input_GBps": round(nbytes / (avg * 1e-3) / 1e9, 1),
            "hbm_frac": round(nbytes / (avg * 1e-3) / 1e9 / HBM_PEAK_GBPS, 4),
            "bound": bound, "median_X2": bound / 32.0, "d": w.d}


def run_sparse(ctx, w, steps):
    """Sparse operands (Corollary 8): covariance of a 1 %-dense m-by-n
    observation matrix with the same n, m, b, d, both operands its CSR rows;
    the sparse call against the dense call on the densified matrix."""
    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    import workloads as W
    ptr, idx, val = W.sparse_observations(w.n1, w.m, 0.01, 4242)
    dp, di, dv = (torch.from_numpy(ptr).cuda(), torch.from_numpy(idx).cuda(),
                  torch.from_numpy(val).cuda())
    dense = np.zeros((w.m, w.n1), np.float32)
    for k in range(w.m):
        dense[k, idx[ptr[k]:ptr[k + 1]]] = val[ptr[k]:ptr[k + 1]]
    dA = torch.from_numpy(dense).cuda()
    dB = dA.clone()

    def timed(fn):
        fn().free()
        torch.cuda.synchronize()
        ctx.profile(True)
        t0 = time.perf_counter()
        for _ in range(steps):
            fn().free()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) * 1e3 / steps
        cs = ctx.profile_read("countsketch")
        ctx.profile(False)
        return ms, cs[0] / max(cs[1], 1)
    ms_s, cs_s = timed(lambda: cmm.sketch_product_sparse(ctx, dp, di, dv, dp, di, dv, w.n1, w.m, w.n1,
                                                        w.b, w.d, seed=w.seed, subtract_diag=True))
    ms_d, cs_d = timed(lambda: cmm.sketch_product(ctx, dA, dB, w.b, w.d, seed=w.seed, subtract_diag=True))
    same = np.array_equal
    a = cmm.sketch_product_sparse(ctx, dp, di, dv, dp, di, dv, w.n1, w.m, w.n1, w.b, w.d, seed=w.seed)
    bd = cmm.sketch_product(ctx, dA, dB, w.b, w.d, seed=w.seed)
    identical = bool(same(a.c(), bd.c()))
    a.free(); bd.free()
    nnz = int(ptr[-1])
    return {"workload": f"covariance n=m={w.n1}, 1 % dense ({nnz} entries per operand), b={w.b}, d={w.d}",
            "sparse_sketch_ms": round(ms_s, 4), "dense_sketch_ms": round(ms_d, 4),
            "sparse_countsketch_ms": round(cs_s, 4), "dense_countsketch_ms": round(cs_d, 4),
            "sketch_identical_to_dense": identical}


def run_nnz(ctx, w):
    """Section 5.1 on the covariance of a 0.1 %-dense m-by-n observation
    matrix (dense operands, same n, m, d): the returned b against the true
    number of non-zeros of X^T X off the diagonal (scipy), and the time of
    the whole doubling search."""
    import numpy as np
    import scipy.sparse as sps
    import torch
    import paper_1108_1320_amd as cmm
    import workloads as W
    ptr, idx, val = W.sparse_observations(w.n1, w.m, 0.001, 4343)
    X = sps.csr_matrix((val, idx, ptr), shape=(w.m, w.n1))
    Q = (X.T @ X).tocoo()
    true_nnz = int(np.sum((Q.row != Q.col) & (Q.data != 0)))
    dX = torch.from_numpy(X.toarray().astype(np.float32)).cuda()
    dY = dX.clone()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    b, _ = cmm.estimate_nnz(ctx, dX, dY, w.d, seed=w.seed, subtract_diag=True)
    torch.cuda.synchronize()
    return {"workload": f"covariance n=m={w.n1}, 0.1 % dense, diagonal removed, d={w.d}",
            "b": int(b), "true_nnz": true_nnz, "ms": round((time.perf_counter() - t0) * 1e3, 2)}


def run_extract(ctx, w, median_x2):
    """FINDSIGNIFICANTENTRIES (Section 4) on the same operands: delta = 3 x
    the Frobenius estimate sqrt(median X^2) / sqrt(b); time of one call
    (1 + 2 * 63 sketch products: the product and one per bit of the row and
    column codes, then decode and vote), positions returned
    and the planted pairs among them."""
    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    At = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
    Bd = At.clone() if w.same_operand else torch.from_numpy(np.ascontiguousarray(w.B_store)).cuda()
    sA = torch.from_numpy(w.scaleA).cuda() if w.scaleA is not None else None
    sB = torch.from_numpy(w.scaleB).cuda() if w.scaleB is not None else None
    delta = 3.0 * float(np.sqrt(max(median_x2, 0.0) / w.b))

    def call():
        return cmm.find_significant(ctx, At, Bd, w.b, w.d, delta, seed=w.seed, dtype=w.dtype,
                                    scaleA=sA, scaleB=sB, subtract_diag=w.subtract_diag,
                                    n1=w.n1, n3=w.n3, m=w.m)
    call()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    gi, gj, total = call()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    res = {"ms": round(ms, 2), "delta": round(delta, 3), "sketch_products": 1 + 2 * 63,
           "returned": int(total)}
    if w.planted is not None and w.mode == "upper":
        got = {(int(a), int(c)) for a, c in zip(gi, gj)}
        want = {(int(min(p, q)), int(max(p, q))) for p, q in w.planted}
        res["planted_found"] = len({(min(a, c), max(a, c)) for a, c in got} & want)
        res["planted"] = len(want)
    return res


def traffic_record(w, geometry):
    """HBM bytes per spectral step (both fft_mac kernels) from the committed
    rocprofv3 counter summary (profiles/fft_mac_traffic.json), if it holds a
    record of this workload at this row length and k per block (the first two
    of log2c, kmax, cs_blocks; the count-sketch blocks do not change the
    spectral launches) and the kernel source has not changed since the
    counters were taken (else None)."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "fft_mac_traffic.json")
    src = os.path.join(ROOT, "paper_1108_1320_amd", "csrc", "k_fft_mac.hip")
    if not os.path.exists(rec_path) or w.dtype != {"covariance-256": "f32", "covariance-4096": "f32",
                                                   "dct-8192": "bf16", "covariance-16384": "fp8"}.get(w.name):
        return None
    rec = json.load(open(rec_path))
    if rec.get("fft_mac_source_sha256_16") != hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]:
        return None
    for r in rec.get("records", []):
        if r["workload"] == w.name and list(r["geometry"])[:2] == list(geometry)[:2]:
            return r["read_bytes"] + r["write_bytes"]
    return None


def planted_recall(w, oi, oj):
    """Fraction of planted correlated pairs found in the top-K (covariance)."""
    if w.planted is None or w.mode != "upper":
        return None
    got = {(int(min(a, c)), int(max(a, c))) for a, c in zip(oi, oj)}
    want = {(int(min(p, q)), int(max(p, q))) for p, q in w.planted}
    return round(len(got & want) / max(len(want), 1), 4)


def stream_ceiling(ctx, gib=1.0, reps=10):
    """What plain HBM streams reach on this GPU, for the count sketch's
    access pattern: reads only, writes only, a copy, and reads with five
    times as many bytes written in five output planes (the count sketch
    writes about 5.3 bytes per byte it reads at covariance 4096), each with
    ordinary and with streaming (non-temporal) stores."""
    nb = int(gib * (1 << 30))
    out = {}

    def rate(rd, wr, nt):
        ms = ctx.stream_probe(rd, wr, nt, reps)
        gbps = (rd + wr) / (ms * 1e-3) / 1e9
        return {"read_bytes": rd, "write_bytes": wr, "ms": round(ms, 4), "GBps": round(gbps, 1),
                "frac": round(gbps / HBM_PEAK_GBPS, 4)}
    out["read"] = rate(nb, 0, False)
    out["write"] = rate(0, nb, False)
    out["write_nt"] = rate(0, nb, True)
    out["copy"] = rate(nb, nb, False)
    out["copy_nt"] = rate(nb, nb, True)
    out["read1_write5"] = rate(nb // 5 // 16 * 16, 5 * (nb // 5 // 16 * 16), False)
    out["read1_write5_nt"] = rate(nb // 5 // 16 * 16, 5 * (nb // 5 // 16 * 16), True)
    return out


def batched_tuning(ctx, classes):
    """Geometry (log2c, kmax, cs_blocks) of each size class of the batch."""
    return {f"b={b},n<={n}": list(ctx.tuning(n, n, n, b, 5, "bf16")) for b, n in classes}


def batched_traffic_record(tuning):
    """HBM bytes of the spectral kernels over one graph replay of the batched
    form, from the committed rocprofv3 counter summary, if it was taken with
    the same per-class geometry and the current kernel source (else None)."""
    import hashlib
    rec_path = os.path.join(ROOT, "profiles", "fft_mac_traffic.json")
    src = os.path.join(ROOT, "paper_1108_1320_amd", "csrc", "k_fft_mac.hip")
    if not os.path.exists(rec_path):
        return None
    rec = json.load(open(rec_path))
    if rec.get("fft_mac_source_sha256_16") != hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]:
        return None
    for r in rec.get("batched_records", []):
        if r["tuning"] == tuning:
            return r["read_bytes"] + r["write_bytes"]
    return None


def batched_roofline(out, ws):
    """Nominal FFT + MAC flops of every product of the batch over the graph
    replay time: the replay also holds the layout, count-sketch, inverse-FFT
    and diagonal kernels, so this is a lower bound on the spectral kernels'
    own rate.  `traffic`: the spectral kernels' HBM bytes per replay."""
    flop = sum(nominal_fft_mac_flop(w.m, w.b, w.d) for w in ws)
    ms = out["graph_replay_ms"]
    tf = flop / (ms * 1e-3) / 1e12
    return {"kernel": "fft_mac (whole graph replay)", "bound": "alu", "achieved": round(tf, 3),
            "peak": FP32_VECTOR_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP32_VECTOR_PEAK_TFLOPS, 4),
            "traffic": batched_traffic_record(out.get("tuning")),
            "traffic_unit": "bytes per graph replay, spectral kernels only (rocprofv3 FETCH_SIZE + WRITE_SIZE, "
                            "copy-calibrated)",
            "flop_per_launch": flop, "avg_launch_ms": ms}


# Steps and warm-up of the other benchmark workloads in the default run,
# sized so that each is timed for well under a second.
OTHER_CONFIGS = {1: (20, 3), 3: (10, 2), 4: (5, 1)}


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(the sketch would shard over k with one all-reduce of c; not built).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    import paper_1108_1320_amd as cmm
    import workloads as W

    cmm.load()
    torch.cuda.init()
    if args.replay_trace:
        ctx = cmm.Context(0)
        ws = W.batched_workloads()
        dev, probs = [], []
        for w in ws:
            A = torch.from_numpy(np.ascontiguousarray(w.At_store)).cuda()
            B = A.clone()
            dev.append((A, B))
            probs.append(cmm.problem(A, B, w.b, w.d, seed=w.seed, dtype=w.dtype, subtract_diag=True))
        if args.tune_cache and os.path.exists(args.tune_cache):
            ctx.load_tuning(args.tune_cache)
        bt = cmm.Batch(ctx, probs, autotune=True, keep=dev)
        if args.tune_cache and not os.path.exists(args.tune_cache):
            ctx.save_tuning(args.tune_cache)
        bt.run()
        torch.cuda.synchronize()
        ms = []
        for _ in range(args.replay_trace):
            time.sleep(0.1)
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            bt.run(asynchronous=True)
            e1.record()
            torch.cuda.synchronize()
            ms.append(e0.elapsed_time(e1))
        classes = sorted({(w.b, W.next_pow2(w.n1)) for w in ws})
        print(json.dumps({"replays": args.replay_trace, "replay_ms": [round(x, 3) for x in ms],
                          "products": len(ws), "tuning": batched_tuning(ctx, classes)}), flush=True)
        bt.free()
        ctx.close()
        return
    if args.stream_ceiling:
        ctx = cmm.Context(0)
        print(json.dumps({"stream_ceiling": stream_ceiling(ctx), "peak_GBps": HBM_PEAK_GBPS}), flush=True)
        ctx.close()
        return
    if args.workload == 5:
        ctx = cmm.Context(0)
        bres = run_batched(ctx, args.steps, args.warmup, not args.no_cpu)
        ctx.close()
        print(json.dumps({
            "metric": METRIC, "value": bres["value"], "unit": "GB/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": bres["ms_per_step"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic", "config": {"workload": bres["workload"]},
            "roofline": bres["roofline"], "batched_form": bres}), flush=True)
        return
    w = W.make_workload(args.workload, dtype=args.dtype)
    if args.d is not None:
        w.d = args.d
    ctx = cmm.Context(0)
    geometry = [int(x) for x in args.geometry.split(",")] if args.geometry else None
    head, r = measure(ctx, w, args.steps, args.warmup, autotune=not args.no_autotune, geometry=geometry)
    sk, (oi, oj, ov) = r["sketch"], r["topk"]
    c_gpu = sk.c()
    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": w.dtype,
        "data": "synthetic",
        "config": {
            "workload": describe(w),
            "n1": w.n1, "m": w.m, "n3": w.n3, "b": w.b, "d": w.d, "K": w.K, "topk_mode": w.mode,
            "input_bytes": head["input_bytes"], "geometry": head["geometry"],
        },
        "roofline": head["roofline"],
    }
    for k in ("autotune", "hbm_frac", "input_elements_per_s", "nominal_fft_gflops",
              "ms_per_step_with_kernel_events", "kernel_ms_per_step", "countsketch", "decode_topk_ms"):
        out[k] = head[k]
    if args.workload == 2 and args.d is None and not args.no_configs:
        # the count sketch of the same operands with one repetition: the
        # kernel streams its input once whatever d is, so the bytes it writes
        # (and its HBM rate) fall with d
        w1 = copy.copy(w)
        w1.d = 1
        r1, rk1 = measure(ctx, w1, args.steps, args.warmup, autotune=False, geometry=head["geometry"])
        rk1["sketch"].free()
        out["countsketch_d1"] = {"d": 1, "geometry": r1["geometry"], "ms_per_step": r1["ms_per_step"],
                                 **r1["countsketch"]}
        del rk1
    if not args.no_stream:
        sc = stream_ceiling(ctx, gib=1.0, reps=10)
        out["stream_ceiling"] = sc
        best = max(sc["read1_write5"]["GBps"], sc["read1_write5_nt"]["GBps"])
        out["countsketch"]["measured_ceiling_GBps"] = best
        out["countsketch"]["frac_of_measured_ceiling"] = round(out["countsketch"]["achieved"] / best, 4)
        if "countsketch_d1" in out:
            # one repetition reads about as many bytes as it writes: a copy
            best1 = max(sc["copy"]["GBps"], sc["copy_nt"]["GBps"])
            out["countsketch_d1"]["measured_ceiling_GBps"] = best1
            out["countsketch_d1"]["measured_ceiling_stream"] = "copy"
            out["countsketch_d1"]["frac_of_measured_ceiling"] = round(out["countsketch_d1"]["achieved"] / best1, 4)
    out["frobenius_bound"] = run_frobenius(ctx, w, args.steps)
    if not args.no_sparse and args.workload == 2:
        out["sparse_form"] = run_sparse(ctx, w, args.steps)
    if not args.no_sparse and args.workload == 2:
        out["nnz_estimate"] = run_nnz(ctx, w)
    if not args.no_extract and w.mode != "column":
        out["find_significant"] = run_extract(ctx, w, out["frobenius_bound"]["median_X2"])
    c_ref = None
    if not args.no_cpu:
        out["cpu_baseline"], out["parity"], c_ref = cpu_baseline(w, c_gpu, oi, oj, ov, head["input_bytes"])
        out["parity"]["planted_recall"] = planted_recall(w, oi, oj)
        fb = out["frobenius_bound"]
        fb["bound_over_true"] = round(fb["bound"] / out["parity"]["frobenius_norm_sq"], 3)
        fb["median_X2_over_true"] = round(fb["median_X2"] / out["parity"]["frobenius_norm_sq"], 4)
    if not args.no_compare and w.mode != "column":
        # the same product in the other operand formats, each against the
        # float64 oracle of its own dequantised operands (arithmetic error)
        # and of the float32 operands (quantisation error), with top-K and
        # planted recall compared to this run's
        for dt in ("f32", "bf16", "fp8"):
            if dt != w.dtype:
                out[f"{dt}_same_workload"] = compare_format(ctx, args, w, dt, c_ref, oi, oj, head["value"])
    sk.free()
    if not args.no_configs and args.workload == 2 and args.dtype is None and args.d is None:
        # the other single-product benchmark workloads, each with its own
        # tuning, timing, kernel times and roofline
        out["configs"] = {}
        for key, (st, wu) in OTHER_CONFIGS.items():
            t0 = time.perf_counter()
            wk = W.make_workload(key)
            gen_s = time.perf_counter() - t0
            res, rk = measure(ctx, wk, st, wu, autotune=not args.no_autotune)
            oi_k, oj_k, _ = rk["topk"]
            res["planted_recall"] = (planted_recall(wk, oi_k, oj_k) if wk.mode == "upper"
                                     else spike_recall(wk, oi_k))
            res["generate_s"] = round(gen_s, 2)
            rk["sketch"].free()
            out["configs"][wk.name] = res
            del wk, rk
    if not args.no_batched:
        out["batched_form"] = run_batched(ctx, max(3, args.steps // 4), 1, not args.no_cpu)
    ctx.close()
    print(json.dumps(out), flush=True)


def spike_recall(w, oi):
    """Transform workload: fraction of the planted spike rows found in the
    per-column top-K."""
    hits = sum(len(set(oi[j * w.K:(j + 1) * w.K].tolist()) & set(w.planted[j].tolist())) for j in range(w.n3))
    return round(hits / (w.n3 * w.K), 4)


def compare_format(ctx, args, w0, dtype, c_ref0, oi0, oj0, value0):
    """The same product with its operands stored as ``dtype``: element rate
    against this run, top-K overlap, planted recall, and (when the oracle
    ran) its error split into arithmetic (GPU vs the float64 oracle of the
    values it multiplies) and quantisation (oracle of those values vs the
    oracle of the float32 operands)."""
    import numpy as np
    import workloads as W
    from oracle import cmm_oracle as O
    w = W.make_workload(args.workload, dtype=dtype)
    w.d = w0.d
    if not args.no_autotune:
        ctx.autotune(w.n1, w.m, w.n3, w.b, w.d, dtype)
    esz = {"f32": 4, "bf16": 2, "fp8": 1}
    r = run_timed(ctx, w, max(3, args.steps // 2), 1)
    v = r["input_bytes"] / (r["ms"] * 1e-3) / 1e9
    oi, oj, _ = r["topk"]
    both = set(zip(oi.tolist(), oj.tolist())) & set(zip(oi0.tolist(), oj0.tolist()))
    res = {"dtype": dtype, "value": round(v, 3), "unit": "GB/s", "ms_per_step": round(r["ms"], 4),
           "input_elements_per_s": round((w.n1 * w.m + w.m * w.n3) / (r["ms"] * 1e-3), 1),
           "element_rate_vs_this_run": round((v / esz[dtype]) / (value0 / esz[w0.dtype]), 4),
           f"topk_overlap_with_{w0.dtype}": round(len(both) / w.K, 4),
           "planted_recall": planted_recall(w, oi, oj),
           "geometry": list(ctx.tuning(w.n1, w.m, w.n3, w.b, w.d, dtype)),
           "kernel_ms_per_step": {k: round(x[0] / max(x[1], 1), 4) for k, x in r["kern"].items()}}
    if c_ref0 is not None:
        c_q = r["sketch"].c()
        Aq, Bq = W.dequantised(w)
        c_refq, _, _ = O.run(Aq, Bq, w.b, w.d, w.seed, subtract_diag=w.subtract_diag)
        if w0.dtype == "f32":
            c_ref32 = c_ref0
        else:
            w32 = W.make_workload(args.workload, dtype="f32")
            A32, B32 = W.dequantised(w32)
            c_ref32, _, _ = O.run(A32, B32, w.b, w.d, w.seed, subtract_diag=w.subtract_diag)

        def rel(x, y):
            return max(float(np.linalg.norm(x[t] - y[t]) / np.linalg.norm(y[t])) for t in range(w.d))
        res["max_rel_l2_c_arithmetic"] = rel(c_q, c_refq)
        res["max_rel_l2_c_quantisation"] = rel(c_refq, c_ref32)
        res["max_rel_l2_c_vs_f64_oracle_of_f32_operands"] = rel(c_q, c_ref32)
    r["sketch"].free()
    return res


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
    est_err = None
    if w.mode != "column":
        est_err = float(np.abs(ov - O.decode(c_ref, tabs, oi, oj)).max())
    AB0 = AB.copy()
    if w.subtract_diag:
        np.fill_diagonal(AB0, 0.0)
    fro2 = float((AB0 ** 2).sum())
    base = {"value": round(input_bytes / secs / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "sample": sample, "seconds": round(secs, 2)}
    parity = {"max_rel_l2_c": rel, "max_abs_err_topk_values": est_err, "tolerance": 1e-5,
              "frobenius_norm_sq": fro2}
    return base, parity, c_ref


if __name__ == "__main__":
    main()
