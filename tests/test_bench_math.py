"""CPU checks of the arithmetic behind the benchmark's reported figures and of
the synthetic input recipe: the nominal FLOP count of the spectral kernel,
the expected number of non-empty buckets (used for the count sketch's
algorithmic bytes), the traffic record's gating, the multi-GPU refusal and
the workload generators' shapes and structure."""
import math
import os
import subprocess
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402
import workloads as W  # noqa: E402


def test_nominal_flop_count_by_hand():
    # covariance 4096: per (rep, k) two real transforms of length 2^16
    # (2.5 b log2 b each) and 2^15 + 1 complex multiply-adds of 8 flops
    per = 2 * 2.5 * 65536 * 16 + 8 * 32769
    assert per == 5505032
    assert bench.nominal_fft_mac_flop(4096, 65536, 5) == 4096 * 5 * per == 112743055360
    # b = 16: two transforms of 2.5 * 16 * 4 flops and 9 bins of 8
    assert bench.nominal_fft_mac_flop(1, 16, 1) == 2 * 160 + 72


def test_expected_nonempty_matches_simulation():
    g = np.random.default_rng(3)
    for n, b in ((4096, 65536), (1000, 1024), (50, 16)):
        sims = [len(np.unique(g.integers(0, b, n))) for _ in range(200)]
        mean = float(np.mean(sims))
        se = float(np.std(sims)) / math.sqrt(len(sims)) + 1e-9
        assert abs(mean - bench.expected_nonempty(n, b)) <= 4 * se + 0.5, (n, b, mean)
    assert bench.expected_nonempty(0, 1024) == 0.0
    assert abs(bench.expected_nonempty(10 ** 6, 16) - 16) < 1e-9


def test_traffic_record_only_for_its_workload():
    import json
    import hashlib
    rec = os.path.join(ROOT, "profiles", "fft_mac_traffic.json")
    assert os.path.exists(rec)
    data = json.load(open(rec))
    recs = [(r["workload"], tuple(r["geometry"])) for r in data["records"]]
    assert recs
    src = os.path.join(ROOT, "paper_1108_1320_amd", "csrc", "k_fft_mac.hip")
    fresh = data["fft_mac_source_sha256_16"] == hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    from types import SimpleNamespace          # the record is keyed by name and format only
    dtype_of = {c["name"]: c["dtype"] for c in W.CONFIGS.values()}
    for name, geo in recs:
        w = SimpleNamespace(name=name, dtype=dtype_of[name])
        t = bench.traffic_record(w, geo)          # present while the source is unchanged
        assert (t > 0) if fresh else (t is None)
        assert bench.traffic_record(w, (9, 7, 5)) is None   # no record at another geometry
        other = SimpleNamespace(name=name, dtype="bf16" if dtype_of[name] != "bf16" else "f32")
        assert bench.traffic_record(other, geo) is None     # same workload, other operand format


def test_batched_traffic_record_only_for_its_tuning():
    import json
    import hashlib
    rec = os.path.join(ROOT, "profiles", "fft_mac_traffic.json")
    data = json.load(open(rec))
    src = os.path.join(ROOT, "paper_1108_1320_amd", "csrc", "k_fft_mac.hip")
    fresh = data["fft_mac_source_sha256_16"] == hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    for r in data.get("batched_records", []):
        t = bench.batched_traffic_record(r["tuning"])
        assert (t == r["read_bytes"] + r["write_bytes"] and t > 0) if fresh else (t is None)
        other = {k: [v[0] - 1] + list(v[1:]) for k, v in r["tuning"].items()}
        assert bench.batched_traffic_record(other) is None   # another geometry of some class
    assert bench.batched_traffic_record({"b=1,n<=1": [1, 1, 1]}) is None
    assert bench.batched_traffic_record(None) is None


def test_multi_gpu_request_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr


def test_covariance_recipe():
    X, pairs, rho = W.covariance_observations(300, 2000, 12, (0.5, 0.95), 7)
    assert X.shape == (2000, 300)
    assert np.allclose(X.mean(axis=0), 0.0, atol=1e-12)          # centred variables
    flat = np.asarray(pairs).reshape(-1)
    assert len(set(flat.tolist())) == flat.size                  # disjoint pairs
    C = np.corrcoef(X, rowvar=False)
    for (p, q), r in zip(pairs, np.atleast_1d(rho)):
        assert 0.5 <= r <= 0.95
        assert abs(C[p, q] - r) < 0.1                             # planted correlation
    off = C[np.triu_indices(300, 1)]
    planted = {(min(p, q), max(p, q)) for p, q in pairs}
    mask = np.array([(i, j) not in planted for i, j in zip(*np.triu_indices(300, 1))])
    assert np.abs(off[mask]).max() < 0.15                         # the rest independent


def test_dct_recipe():
    n = 64
    D = W.dct2_orthonormal(n)
    assert np.allclose(D @ D.T, np.eye(n), atol=1e-12)
    A, B, rows = W.transform_operands(n, 4, 1e-3, 11)
    P = A @ B                                                      # = S + D eps, eps of std 1e-3
    for j in range(n):
        spikes = set(np.asarray(rows)[j].tolist())
        assert len(spikes) == 4
        others = [i for i in range(n) if i not in spikes]
        assert np.abs(P[others, j]).max() < 0.01                   # only noise off the spikes
        top = set(np.argsort(-np.abs(P[:, j]))[:4].tolist())
        assert {r for r in spikes if abs(P[r, j]) > 0.02} <= top  # spikes above the noise rank first


def test_batched_recipe():
    sizes = W.batched_sizes()
    assert len(sizes) == 64
    for n, b, pairs, _, _ in sizes:
        assert 512 <= n <= 8192
        assert b == 1 << math.ceil(math.log2(8 * n))
        assert 4 <= pairs <= 128
    logs = np.log([s[0] for s in sizes])
    # log-uniform: the logs spread over the whole range, not clustered
    assert logs.min() < math.log(700) and logs.max() > math.log(6000)
