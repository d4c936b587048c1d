"""Seeded synthetic inputs for the compressed-matrix-multiplication sketch.

This module is shared by the tests, the benchmark and the checks that run the
CPU oracle.  It only *generates and encodes inputs*: it holds none of the
method's arithmetic (no hashing, no sketching, no decoding).  Every generator
takes an explicit integer seed and uses numpy's PCG64, so the same call gives
the same matrices on every machine.

Shapes follow the paper's two motivating problems (Section 1):

* covariance: m observations of n variables arranged as the n-by-m matrix
  A = X^T, product A A^T (Section 3.2).  ``X`` here is the m-by-n
  observation matrix (one row per sample); a few disjoint variable pairs are
  planted with correlation rho, as in the experiment of Figure 2.
* transform: columns of B are made sparse by an orthonormal basis (the
  JPEG-style batch transform of Section 1); A's rows are the orthonormal
  DCT-II basis vectors, B = D^T S + noise with S column-sparse.

Storage convention handed to the GPU library (the single-pass order of
Section 2.2): A is given column-major, i.e. as the m-by-n1 row-major array
At with At[k, i] = A[i, k]; B is given row-major, m-by-n3.  For a covariance
product both are the observation matrix X itself.

Low-precision encodings (input preparation only):

* bf16: round-to-nearest-even of the float32 value, stored as uint16 bits.
* fp8: OCP e4m3fn bits (uint8) with one float32 scale per stored column,
  scale = amax(column) / 448, code = RNE(x / scale), saturating at 448.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "rng", "covariance_observations", "dct2_orthonormal", "transform_operands",
    "bf16_encode", "e4m3fn_encode", "e4m3fn_grid", "Workload", "make_workload",
    "CONFIGS", "batched_sizes", "batched_workloads", "sparse_observations", "next_pow2",
]


def rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def next_pow2(x: int) -> int:
    return 1 << max(0, int(math.ceil(math.log2(x))))


# --------------------------------------------------------------------------
# generators (float64, mathematical orientation)
# --------------------------------------------------------------------------

def covariance_observations(n: int, m: int, n_pairs: int, rho, seed: int):
    """m-by-n observations X of n variables, centred per variable.

    Variables are i.i.d. N(0,1) except ``n_pairs`` disjoint random pairs
    (p, q) where X[:, q] = rho * X[:, p] + sqrt(1 - rho^2) * Z.  ``rho`` is a
    float or a (lo, hi) range sampled uniformly per pair.  Returns
    (X, pairs, rhos) with pairs as an (n_pairs, 2) int array.
    """
    g = rng(seed)
    X = g.standard_normal((m, n))
    perm = g.permutation(n)[: 2 * n_pairs].reshape(n_pairs, 2) if n_pairs else np.zeros((0, 2), np.int64)
    if isinstance(rho, tuple):
        rhos = g.uniform(rho[0], rho[1], size=n_pairs)
    else:
        rhos = np.full(n_pairs, float(rho))
    for (p, q), r in zip(perm, rhos):
        z = g.standard_normal(m)
        X[:, q] = r * X[:, p] + math.sqrt(1.0 - r * r) * z
    X -= X.mean(axis=0, keepdims=True)
    return X, perm.astype(np.int64), rhos


def dct2_orthonormal(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix D (rows are basis vectors).

    D[k, i] = sqrt(2/n) * g_k * cos(pi * (2i+1) * k / (2n)), g_0 = 1/sqrt(2).
    The angle is reduced exactly in integers before the cosine.
    """
    k = np.arange(n, dtype=np.int64)[:, None]
    i = np.arange(n, dtype=np.int64)[None, :]
    num = ((2 * i + 1) * k) % (4 * n)
    D = np.cos(np.pi * num.astype(np.float64) / (2.0 * n))
    D *= math.sqrt(2.0 / n)
    D[0, :] *= 1.0 / math.sqrt(2.0)
    return D


def transform_operands(n: int, spikes: int, noise_std: float, seed: int):
    """A = D (orthonormal DCT-II), B = D^T S + eps with ``spikes`` N(0,1)
    entries at distinct random rows of every column of S.

    Returns (A, B, S_rows) with S_rows an (n, spikes) array of the spike
    rows of each column.
    """
    g = rng(seed)
    D = dct2_orthonormal(n)
    S = np.zeros((n, n))
    rows = np.empty((n, spikes), np.int64)
    for j in range(n):
        r = g.choice(n, size=spikes, replace=False)
        rows[j] = r
        S[r, j] = g.standard_normal(spikes)
    B = D.T @ S + noise_std * g.standard_normal((n, n))
    return D, B, rows


# --------------------------------------------------------------------------
# encodings
# --------------------------------------------------------------------------

def bf16_encode(x) -> np.ndarray:
    """float -> bfloat16 bits (uint16), round to nearest even."""
    f = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = f.view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = (u + np.uint64(0x7FFF) + lsb) >> np.uint64(16)
    return r.astype(np.uint16)


def e4m3fn_grid() -> np.ndarray:
    """Non-negative finite e4m3fn values indexed by code 0..126."""
    vals = np.empty(127)
    for code in range(127):
        e, mnt = code >> 3, code & 7
        vals[code] = (mnt / 8.0) * 2.0 ** -6 if e == 0 else (1.0 + mnt / 8.0) * 2.0 ** (e - 7)
    return vals


_E4M3 = e4m3fn_grid()
# float32 value of every code 0..255 (sign bit 0x80; the two NaN codes 0x7F
# and 0xFF, which the encoder never produces, read as NaN)
_E4M3_SIGNED32 = np.array([(-1.0 if c & 0x80 else 1.0) * _E4M3[c & 0x7F] if c & 0x7F != 0x7F else np.nan
                           for c in range(256)], dtype=np.float32)


def _e4m3fn_chunk(v: np.ndarray) -> np.ndarray:
    """e4m3fn codes of a float64 chunk from its IEEE bits: for |v| >= 2^-6 the
    top 3 of the 52 mantissa bits are rounded half-to-even (a carry moves to
    the next binade); below 2^-6 the value is rounded to a multiple of 2^-9
    (subnormal codes 0..7, 8 being the smallest normal).  Saturates at 448."""
    a = np.minimum(np.abs(v), 448.0)
    bits = a.view(np.uint64)
    e = (bits >> np.uint64(52)).astype(np.int64) - 1023
    mant = bits & np.uint64((1 << 52) - 1)
    q = (mant >> np.uint64(49)).astype(np.int64)
    rem = mant & np.uint64((1 << 49) - 1)
    half = np.uint64(1 << 48)
    q += ((rem > half) | ((rem == half) & (q % 2 == 1))).astype(np.int64)
    carry = q == 8
    normal = ((e + 7 + carry) << 3) | np.where(carry, 0, q)
    code = np.where(a < 2.0 ** -6, np.rint(a * 512.0).astype(np.int64), normal)
    return (code | np.where(np.signbit(v), 0x80, 0)).astype(np.uint8)


def e4m3fn_encode(x) -> np.ndarray:
    """float -> OCP e4m3fn bits (uint8), round to nearest even, saturating;
    chunks of 2^21 values on a few threads."""
    from concurrent.futures import ThreadPoolExecutor
    x = np.asarray(x, dtype=np.float64)
    out = np.empty(x.shape, dtype=np.uint8)
    xf, of = x.reshape(-1), out.reshape(-1)
    step = 1 << 21

    def one(s0):
        of[s0:s0 + step] = _e4m3fn_chunk(xf[s0:s0 + step])
    starts = range(0, xf.size, step)
    if xf.size <= step:
        for s0 in starts:
            one(s0)
    else:
        with ThreadPoolExecutor(max_workers=8) as ex:
            list(ex.map(one, starts))
    return out


# --------------------------------------------------------------------------
# workload configurations
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """One product AB to sketch, in both orientations.

    A (n1 x m) and B (m x n3) are float64 values of exactly what the GPU reads
    (after dequantisation for bf16/fp8).  ``At_store``/``B_store`` are the
    encoded k-major arrays handed to the library; ``scaleA``/``scaleB`` are
    the per-stored-column fp8 scales (None otherwise).
    """
    name: str
    n1: int
    m: int
    n3: int
    b: int
    d: int
    K: int
    dtype: str                     # "f32" | "bf16" | "fp8"
    mode: str                      # "all" | "upper" | "column"
    seed: int                      # hash seed
    subtract_diag: bool
    At_store: np.ndarray = field(repr=False)
    B_store: np.ndarray = field(repr=False)
    scaleA: np.ndarray | None = field(default=None, repr=False)
    scaleB: np.ndarray | None = field(default=None, repr=False)
    A_ref: np.ndarray | None = field(default=None, repr=False)   # unquantised float64 A
    B_ref: np.ndarray | None = field(default=None, repr=False)
    planted: np.ndarray | None = field(default=None, repr=False)
    same_operand: bool = False     # covariance: A = X^T and B = X share storage


def _encode(mat_kmajor: np.ndarray, dtype: str):
    """Encode a k-major float64 array; returns (stored, scale, dequantised f64)."""
    if dtype == "f32":
        s = np.ascontiguousarray(mat_kmajor.astype(np.float32))
        return s, None, s.astype(np.float64)
    if dtype == "bf16":
        s = bf16_encode(mat_kmajor.astype(np.float32))
        deq = (s.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
        return s, None, deq
    if dtype == "fp8":
        amax = np.abs(mat_kmajor).max(axis=0)
        scale = np.where(amax > 0, amax / 448.0, 1.0).astype(np.float32)
        s = e4m3fn_encode(mat_kmajor / scale.astype(np.float64)[None, :])
        return s, scale, _decode_store(s, "fp8", scale)[2]
    raise ValueError(dtype)


def covariance_workload(name, n, m, n_pairs, rho, b, d, K, dtype, data_seed, hash_seed,
                        mode="upper", subtract_diag=True) -> Workload:
    X, pairs, _ = covariance_observations(n, m, n_pairs, rho, data_seed)
    store, scale, deq = _encode(X, dtype)
    return Workload(name=name, n1=n, m=m, n3=n, b=b, d=d, K=K, dtype=dtype, mode=mode,
                    seed=hash_seed, subtract_diag=subtract_diag,
                    At_store=store, B_store=store, scaleA=scale, scaleB=scale,
                    A_ref=X.T, B_ref=X, planted=pairs, same_operand=True)


def transform_workload(name, n, spikes, noise_std, b, d, K, dtype, data_seed, hash_seed) -> Workload:
    A, B, rows = transform_operands(n, spikes, noise_std, data_seed)
    sa, scA, _ = _encode(np.ascontiguousarray(A.T), dtype)
    sb, scB, _ = _encode(B, dtype)
    return Workload(name=name, n1=n, m=n, n3=n, b=b, d=d, K=K, dtype=dtype, mode="column",
                    seed=hash_seed, subtract_diag=False, At_store=sa, B_store=sb,
                    scaleA=scA, scaleB=scB, A_ref=A, B_ref=B, planted=rows)


def dequantised(w: Workload):
    """(A, B) as float64 values the GPU actually multiplies (math orientation)."""
    _, _, At = _decode_store(w.At_store, w.dtype, w.scaleA)
    if w.same_operand:
        return At.T, At
    _, _, Bq = _decode_store(w.B_store, w.dtype, w.scaleB)
    return At.T, Bq


def _decode_store(store, dtype, scale):
    if dtype == "f32":
        return store, None, store.astype(np.float64)
    if dtype == "bf16":
        return store, None, (store.astype(np.uint32) << np.uint32(16)).view(np.float32).astype(np.float64)
    val = _E4M3_SIGNED32[store] * scale.astype(np.float32)[None, :]
    return store, scale, val.astype(np.float64)


# The benchmark workloads, keyed 1 to 4 (key 5, the batched form, is built
# by ``batched_workloads``).  Data seed 1000 + key, hash seed 2000 + key.
CONFIGS = {
    1: dict(name="covariance-256", kind="cov", n=256, m=256, pairs=16, rho=0.9, b=1 << 10, d=1, K=16,
            dtype="f32"),
    2: dict(name="covariance-4096", kind="cov", n=4096, m=4096, pairs=64, rho=(0.5, 0.95), b=1 << 16, d=5,
            K=64, dtype="f32"),
    3: dict(name="dct-8192", kind="transform", n=8192, spikes=16, noise=1e-3, b=1 << 17, d=7, K=16,
            dtype="bf16"),
    4: dict(name="covariance-16384", kind="cov", n=16384, m=16384, pairs=256, rho=(0.5, 0.95), b=1 << 18,
            d=9, K=256, dtype="fp8"),
}


def make_workload(key: int, n: int | None = None, dtype: str | None = None) -> Workload:
    """Build benchmark workload ``key``; ``n`` optionally shrinks it (same
    recipe, m = n, b scaled to keep b/n) for tests that must run quickly."""
    c = dict(CONFIGS[key])
    if n is not None and n != c["n"]:
        ratio = c["b"] // c["n"]
        c["b"] = max(16, next_pow2(ratio * n))
        c["pairs"] = min(c.get("pairs", 0), n // 4)
        c["n"] = n
        c["m"] = n
    dt = dtype or c["dtype"]
    name = c["name"]
    if c["kind"] == "cov":
        return covariance_workload(name, c["n"], c.get("m", c["n"]), c["pairs"], c["rho"], c["b"], c["d"],
                                   c["K"], dt, 1000 + key, 2000 + key)
    return transform_workload(name, c["n"], c["spikes"], c["noise"], c["b"], c["d"], c["K"], dt,
                              1000 + key, 2000 + key)


def batched_sizes(count: int = 64, seed: int = 1005, lo: int = 512, hi: int = 8192):
    """n = m = round(exp U[ln lo, ln hi]) per product, b = next power of two
    of 8n, planted pairs U{4..128}; returns a list of (n, b, pairs, data_seed,
    hash_seed)."""
    g = rng(seed)
    out = []
    for p in range(count):
        n = int(round(math.exp(g.uniform(math.log(lo), math.log(hi)))))
        pairs = int(g.integers(4, 129))
        out.append((n, next_pow2(8 * n), min(pairs, n // 2), 100000 + p, 2000 + 100 * 5 + p))
    return out


def batched_workloads(count: int = 64, seed: int = 1005, lo: int = 512, hi: int = 8192, d: int = 5,
                      dtype: str = "bf16"):
    """The batched covariance workload: one covariance product per entry of
    ``batched_sizes`` (n = m, b = next power of two of 8n, 4..128 planted
    pairs with rho in [0.5, 0.95], d repetitions, operands stored in
    ``dtype``), each selecting its top-(planted pairs) over i < j."""
    out = []
    for p, (n, b, pairs, data_seed, hash_seed) in enumerate(batched_sizes(count, seed, lo, hi)):
        out.append(covariance_workload(f"batched-64.{p}", n, n, pairs, (0.5, 0.95), b, d, pairs, dtype,
                                       data_seed, hash_seed))
    return out


def sparse_observations(n: int, m: int, density: float, seed: int):
    """m-by-n sparse observation matrix in CSR form (indptr int64, indices
    int32, data float32 N(0,1)): each row holds round(density * n) distinct
    random variables.  For a covariance product both operands are these rows
    (A = X^T by columns k is X by rows k)."""
    g = rng(seed)
    per = max(1, int(round(density * n)))
    indptr = np.arange(m + 1, dtype=np.int64) * per
    indices = np.empty(m * per, dtype=np.int32)
    for k in range(m):
        indices[k * per:(k + 1) * per] = np.sort(g.choice(n, per, replace=False))
    data = g.standard_normal(m * per).astype(np.float32)
    return indptr, indices, data
