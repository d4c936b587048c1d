"""CPU oracle for the compressed matrix product sketch (Pagh, "Compressed
Matrix Multiplication").

TEST INFRASTRUCTURE.  Only the test-suite, the package's smoke check and the
benchmark's CPU-baseline leg may import or run this module.  The GPU library
never calls it, and it shares no code, tables or constants with the GPU path.

Everything here is plain and slow on purpose: float64 numpy, exact Python
integers for hashing, library primitives (matrix product, sort, bincount) used
only as single steps, no blocking or reordering beyond what the definitions
state.  Indices are 0-based (the paper's [n] = {1..n} shifted by one).

What it computes
----------------
For d repetitions t, hash functions h1_t, h2_t into {0..b-1} and s1_t, s2_t
into {-1,+1} define the splitting function h(i,j) = (h1(i)+h2(j)) mod b and
sign s(i,j) = s1(i)s2(j) (Section 2.2, decomposable hashing).  The sketch of
the product is the COUNT SKETCH of AB under (h, s):

    c_t[u] = sum over (i,j) with h(i,j) = u of s(i,j) (AB)_ij

(Section 2.2; the estimator analysed in Theorem 2).  Two independent
formulations are provided and checked against each other:

* ``sketch_from_product`` -- the definition: form AB in float64, bin it.
* ``sketch_polynomial``   -- the algorithm of Figure 1 without the FFT: for
  every outer product a_k b_k (eq. (1)) build the two count-sketch
  polynomials and multiply them modulo x^b - 1 by direct cyclic convolution
  (the wrap (p mod x^b) + (p div x^b) of the abstract).

Decoding (DECOMPRESS of Figure 1): X_t = s1_t(i) s2_t(j) c_t[h(i,j)], estimate
= median over t (middle value for odd d, mean of the two middle values for
even d).  Top-K ranks |C_ij| descending, ties by linear index i*n3+j.

Hash family (Section 2.2, polynomial hashing): g(x) = (a*x + c) mod p with
p = 2^61 - 1; h = g mod b (b a power of two), s = +1 if g is even else -1.
Parameters (a, c) per repetition t and function f (h1=0, s1=1, h2=2, s2=3)
come from the SplitMix64 counter stream (Steele, Lea, Flood 2014) of the
seed: outputs z_{8t+2f+1}, z_{8t+2f+2}; a = 1 + z mod (p-1), c = z' mod p.
The paper leaves the source of randomness open; this is the reading chosen.

Parity status of each function is stated in its docstring ("pinned by ...").
"""
from __future__ import annotations

import numpy as np

P61 = (1 << 61) - 1
_M64 = (1 << 64) - 1
_GAMMA = 0x9E3779B97F4A7C15


# ---------------------------------------------------------------------------
# randomness and hashing
# ---------------------------------------------------------------------------

def splitmix64(seed: int, count: int) -> list[int]:
    """First ``count`` outputs z_1..z_count of SplitMix64 seeded with ``seed``.

    Output k mixes the counter seed + k*gamma (mod 2^64) through two
    xor-shift-multiply rounds and a final xor-shift.  Pinned by published
    known answers in the tests.
    """
    out = []
    for k in range(1, count + 1):
        z = (seed + k * _GAMMA) & _M64
        z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
        z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
        out.append(z ^ (z >> 31))
    return out


def hash_params(seed: int, d: int) -> np.ndarray:
    """(d, 4, 2) uint64 array of (a, c) for h1, s1, h2, s2 of each repetition."""
    z = splitmix64(seed, 8 * d)
    out = np.zeros((d, 4, 2), dtype=np.uint64)
    for t in range(d):
        for f in range(4):
            za, zc = z[8 * t + 2 * f], z[8 * t + 2 * f + 1]
            out[t, f, 0] = 1 + za % (P61 - 1)
            out[t, f, 1] = zc % P61
    return out


def cw_hash(a: int, c: int, xs) -> list[int]:
    """Carter-Wegman degree-1 polynomial hash (a*x + c) mod (2^61-1), exact."""
    a, c = int(a), int(c)
    return [(a * int(x) + c) % P61 for x in xs]


def hash_tables(params: np.ndarray, n1: int, n3: int, b: int):
    """Evaluate h1, s1 on 0..n1-1 and h2, s2 on 0..n3-1 for every repetition.

    Returns int64 arrays h1 (d,n1), s1 (d,n1), h2 (d,n3), s2 (d,n3).
    """
    d = params.shape[0]
    h1 = np.zeros((d, n1), np.int64); s1 = np.zeros((d, n1), np.int64)
    h2 = np.zeros((d, n3), np.int64); s2 = np.zeros((d, n3), np.int64)
    for t in range(d):
        g = cw_hash(params[t, 0, 0], params[t, 0, 1], range(n1)); h1[t] = [v % b for v in g]
        g = cw_hash(params[t, 1, 0], params[t, 1, 1], range(n1)); s1[t] = [1 - 2 * (v % 2) for v in g]
        g = cw_hash(params[t, 2, 0], params[t, 2, 1], range(n3)); h2[t] = [v % b for v in g]
        g = cw_hash(params[t, 3, 0], params[t, 3, 1], range(n3)); s2[t] = [1 - 2 * (v % 2) for v in g]
    return h1, s1, h2, s2


# ---------------------------------------------------------------------------
# dequantisation of stored operands (float64 values the sketch is of)
# ---------------------------------------------------------------------------

def _e4m3fn_value(code: int) -> float:
    """Value of an OCP e4m3fn byte: 1 sign, 4 exponent (bias 7), 3 mantissa
    bits; exponent 0 is subnormal; S.1111.111 is NaN; no infinities."""
    sign = -1.0 if code & 0x80 else 1.0
    e, mnt = (code >> 3) & 0xF, code & 7
    if e == 15 and mnt == 7:
        return float("nan")
    if e == 0:
        return sign * mnt * 2.0 ** -9
    return sign * (8 + mnt) * 2.0 ** (e - 10)


_E4M3_TABLE = np.array([_e4m3fn_value(c) for c in range(256)])


def dequantise(stored: np.ndarray, dtype: str, scale=None) -> np.ndarray:
    """float64 values of a stored k-major operand (f32 / bf16 bits / fp8 bits
    times a per-column scale)."""
    if dtype == "f32":
        return np.asarray(stored, dtype=np.float64)
    if dtype == "bf16":
        bits = np.asarray(stored, dtype=np.uint16).astype(np.uint32) << np.uint32(16)
        return bits.view(np.float32).astype(np.float64)
    if dtype == "fp8":
        # an element's value is the float32 product of its decoded code and
        # its column scale
        v = _E4M3_TABLE[np.asarray(stored, dtype=np.uint8).astype(np.int64)].astype(np.float32)
        if scale is not None:
            v = v * np.asarray(scale, dtype=np.float32)[None, :]
        return v.astype(np.float64)
    raise ValueError(dtype)


# ---------------------------------------------------------------------------
# the sketch
# ---------------------------------------------------------------------------

def countsketch(v: np.ndarray, h: np.ndarray, s: np.ndarray, b: int) -> np.ndarray:
    """COUNT SKETCH of a weighted vector (Section 2.2): p[u] = sum_{h(i)=u}
    s(i) v_i, i.e. the coefficients of the polynomial p_v^{h,s}(x).
    Pinned by brute force in the tests."""
    p = np.zeros(b)
    np.add.at(p, h, s * v)
    return p


def cyclic_convolution(x: np.ndarray, y: np.ndarray) -> np.ndarray:
    """(x * y) mod (z^b - 1) by the direct double sum over nonzero terms:
    out[(u+w) mod b] += x[u] y[w].  No FFT."""
    b = x.shape[0]
    ux, uy = np.nonzero(x)[0], np.nonzero(y)[0]
    if ux.size == 0 or uy.size == 0:
        return np.zeros(b)
    idx = (ux[:, None] + uy[None, :]) % b
    return np.bincount(idx.ravel(), weights=np.outer(x[ux], y[uy]).ravel(), minlength=b)


def sketch_polynomial(A: np.ndarray, B: np.ndarray, tables, b: int) -> np.ndarray:
    """Figure 1's COMPRESSEDPRODUCT with the FFT product replaced by direct
    cyclic convolution: for each repetition t and each k, convolve the count
    sketches of column a_k (h1, s1) and row b_k (h2, s2) and sum over k.
    Returns c (d, b).  Pinned against ``sketch_from_product`` and, for
    injective hashes, against the plain matrix product."""
    h1, s1, h2, s2 = tables
    d = h1.shape[0]
    c = np.zeros((d, b))
    for t in range(d):
        for k in range(A.shape[1]):
            pa = countsketch(A[:, k], h1[t], s1[t], b)
            pb = countsketch(B[k, :], h2[t], s2[t], b)
            c[t] += cyclic_convolution(pa, pb)
    return c


def bin_product(AB: np.ndarray, tables, b: int, row_block: int = 1024) -> np.ndarray:
    """Bin a given n1-by-n3 matrix M by h(i,j) with sign s(i,j): the COUNT
    SKETCH definition applied to M (rows processed in blocks to bound memory)."""
    h1, s1, h2, s2 = tables
    d = h1.shape[0]
    n1 = AB.shape[0]
    c = np.zeros((d, b))
    for t in range(d):
        for r0 in range(0, n1, row_block):
            r1 = min(n1, r0 + row_block)
            idx = (h1[t, r0:r1, None] + h2[t, None, :]) % b
            w = (s1[t, r0:r1, None] * s2[t, None, :]) * AB[r0:r1]
            c[t] += np.bincount(idx.ravel(), weights=w.ravel(), minlength=b)
    return c


def sketch_from_product(A: np.ndarray, B: np.ndarray, tables, b: int) -> np.ndarray:
    """The definition: c_t[u] = sum_{h(i,j)=u} s(i,j) (AB)_ij with AB formed
    exactly in float64.  Pinned by brute-force loops on tiny inputs."""
    AB = np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    return bin_product(AB, tables, b)


def sketch_buckets(A: np.ndarray, B: np.ndarray, tables, b: int, t: int, us,
                   zero_diagonal: bool = False) -> np.ndarray:
    """Selected entries c_t[u] of the definition, one bucket at a time: the
    pairs (i, j) with (h1(i) + h2(j)) mod b = u are listed from h2's inverse,
    and each (AB)_ij is the float64 dot product of row i of A and column j of
    B.  ``zero_diagonal`` leaves out i = j (the sketch of AB with a zero
    diagonal).  For products too large to form whole."""
    h1, s1, h2, s2 = tables
    order = np.argsort(h2[t], kind="stable")
    hsorted = h2[t][order]
    out = np.empty(len(us))
    for q, u in enumerate(us):
        need = (u - h1[t]) % b                      # h2(j) needed for each i
        lo = np.searchsorted(hsorted, need, side="left")
        hi = np.searchsorted(hsorted, need, side="right")
        ii = np.repeat(np.arange(h1.shape[1]), hi - lo)
        jj = order[np.concatenate([np.arange(a, z) for a, z in zip(lo, hi)])] if len(ii) else np.zeros(0, np.int64)
        if zero_diagonal:
            keep = ii != jj
            ii, jj = ii[keep], jj[keep]
        vals = np.einsum("pk,kp->p", A[ii, :], B[:, jj]) if len(ii) else np.zeros(0)
        out[q] = float((s1[t, ii] * s2[t, jj] * vals).sum())
    return out


def subtract_diagonal(c: np.ndarray, diag: np.ndarray, tables, b: int) -> np.ndarray:
    """Sketch of AB with its diagonal zeroed (Section 3.2, Q-tilde): remove
    s1(i)s2(i)(AB)_ii from bucket h(i,i) of every repetition."""
    h1, s1, h2, s2 = tables
    out = c.copy()
    n = diag.shape[0]
    for t in range(c.shape[0]):
        idx = (h1[t, :n] + h2[t, :n]) % b
        np.add.at(out[t], idx, -(s1[t, :n] * s2[t, :n]) * diag)
    return out


# ---------------------------------------------------------------------------
# decoding, median, top-K
# ---------------------------------------------------------------------------

def median(x: np.ndarray, axis: int = 0) -> np.ndarray:
    """Median along ``axis``: middle order statistic for odd length, mean of
    the two middle ones for even length."""
    x = np.sort(x, axis=axis)
    d = x.shape[axis]
    lo = np.take(x, (d - 1) // 2, axis=axis)
    hi = np.take(x, d // 2, axis=axis)
    return lo if d % 2 else 0.5 * (lo + hi)


def decode(c: np.ndarray, tables, i, j) -> np.ndarray:
    """DECOMPRESS(i, j) of Figure 1 for arrays of index pairs: median over t
    of s1_t(i) s2_t(j) c_t[(h1_t(i) + h2_t(j)) mod b]."""
    h1, s1, h2, s2 = tables
    b = c.shape[1]
    i, j = np.broadcast_arrays(np.asarray(i, dtype=np.int64), np.asarray(j, dtype=np.int64))
    X = np.empty((c.shape[0],) + i.shape)
    for t in range(c.shape[0]):
        X[t] = s1[t, i] * s2[t, j] * c[t, (h1[t, i] + h2[t, j]) % b]
    return median(X, axis=0)


def candidates(mode: str, n1: int, n3: int):
    """Linear indices i*n3+j of the candidate domain: all entries, or i<j."""
    i, j = np.meshgrid(np.arange(n1), np.arange(n3), indexing="ij")
    if mode == "upper":
        keep = i < j
        return i[keep], j[keep]
    return i.ravel(), j.ravel()


def topk(values: np.ndarray, lin: np.ndarray, K: int):
    """First K of (values, lin) sorted by |value| descending, then lin
    ascending.  Returns (lin, values) of the selection."""
    order = np.lexsort((lin, -np.abs(values)))[:K]
    return lin[order], values[order]


def topk_per_column(C: np.ndarray, K: int):
    """For every column j of an n1-by-n3 estimate matrix, the K rows with the
    largest |C_ij| (ties by smaller i).  Returns (rows (n3,K), vals (n3,K))."""
    n1, n3 = C.shape
    rows = np.empty((n3, K), np.int64); vals = np.empty((n3, K))
    ii = np.arange(n1)
    for j in range(n3):
        o = np.lexsort((ii, -np.abs(C[:, j])))[:K]
        rows[j] = o; vals[j] = C[o, j]
    return rows, vals


def decode_all(c: np.ndarray, tables, n1: int, n3: int, row_block: int = 512) -> np.ndarray:
    """All n1*n3 estimates (only for sizes where that fits in memory)."""
    out = np.empty((n1, n3))
    jj = np.arange(n3)
    for r0 in range(0, n1, row_block):
        r1 = min(n1, r0 + row_block)
        ii = np.arange(r0, r1)
        out[r0:r1] = decode(c, tables, ii[:, None], jj[None, :])
    return out


# ---------------------------------------------------------------------------
# Frobenius-norm upper bound (Section 5.2, from the AMS sketch of Section 2.1)
# ---------------------------------------------------------------------------

# Reading (the paper leaves the source open): the sign polynomials of the
# bound use the same SplitMix64 stream as the count-sketch hashes, from output
# 1024 on (the count sketch uses at most z_1..z_504, d <= 63).
AMS_STREAM_OFFSET = 1024


def ams_params(seed: int, d: int) -> np.ndarray:
    """(d, 2, 4) uint64 coefficients (a0, a1, a2, a3) of the degree-3 sign
    polynomials of s1 (f = 0) and s2 (f = 1) of every repetition t:
    a_c = z_{1024 + 8t + 4f + c + 1} mod (2^61 - 1).  Degree-3 polynomials
    with uniform coefficients form a 4-wise independent family, as Section
    5.2 asks of s1 and s2.  Pinned by the 4-point sign statistics in the
    tests."""
    z = splitmix64(seed, AMS_STREAM_OFFSET + 8 * d)
    out = np.zeros((d, 2, 4), dtype=np.uint64)
    for t in range(d):
        for f in range(2):
            for c in range(4):
                out[t, f, c] = z[AMS_STREAM_OFFSET + 8 * t + 4 * f + c] % P61
    return out


def poly_hash(coefs, xs) -> list[int]:
    """sum_c a_c x^c mod (2^61 - 1), exact integers.  Pinned by hand values
    at the modulus edges."""
    cs = [int(a) for a in coefs]
    return [sum(a * pow(int(x), c, P61) for c, a in enumerate(cs)) % P61 for x in xs]


def ams_signs(params: np.ndarray, n1: int, n3: int):
    """s1 (d, n1) and s2 (d, n3) in {-1, +1}: +1 where the polynomial value is
    even (as for the count-sketch signs)."""
    d = params.shape[0]
    s1 = np.zeros((d, n1), np.int64); s2 = np.zeros((d, n3), np.int64)
    for t in range(d):
        s1[t] = [1 - 2 * (g % 2) for g in poly_hash(params[t, 0], range(n1))]
        s2[t] = [1 - 2 * (g % 2) for g in poly_hash(params[t, 1], range(n3))]
    return s1, s2


def ams_sketch(AB: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """X_t = sum over (i,j) of s1_t(i) s2_t(j) (AB)_ij: the AMS sketch of AB
    with the product sign s(i,j) = s1(i) s2(j) (Section 2.1), one per
    repetition.  Definition form; pinned against ``ams_sketch_outer``, a hand
    example and the moments of Section 5.2."""
    AB = np.asarray(AB, dtype=np.float64)
    return np.array([float(s1[t].astype(np.float64) @ AB @ s2[t].astype(np.float64))
                     for t in range(s1.shape[0])])


def ams_sketch_outer(A: np.ndarray, B: np.ndarray, s1: np.ndarray, s2: np.ndarray) -> np.ndarray:
    """The same sketch summed over the outer products a_k b_k of eq. (1): the
    sketch of an outer product is the product of the two vectors' sketches
    (Section 2.1), X_t = sum_k (sum_i s1(i) A_ik)(sum_j s2(j) B_kj)."""
    A = np.asarray(A, dtype=np.float64); B = np.asarray(B, dtype=np.float64)
    out = np.zeros(s1.shape[0])
    for t in range(s1.shape[0]):
        u = s1[t].astype(np.float64) @ A          # one value per k
        v = B @ s2[t].astype(np.float64)          # one value per k
        out[t] = float(np.sum(u * v))
    return out


def frobenius_bound(X: np.ndarray) -> float:
    """32 times the median over repetitions of X_t^2: X^2 is an unbiased
    estimator of ||AB||_F^2 with variance at most 8 E[X^2]^2, so by
    Chebyshev it is within a factor 32 with probability 3/4, and the median
    of d estimators times 32 is an upper bound with high probability
    (Section 5.2)."""
    return 32.0 * float(median(np.asarray(X, dtype=np.float64) ** 2, 0))


def frobenius(A: np.ndarray, B: np.ndarray, d: int, seed: int, subtract_diag: bool = False):
    """(X, bound, s1, s2) for AB (with its diagonal zeroed if asked, the Q~ of
    Section 3.2)."""
    n1, n3 = A.shape[0], B.shape[1]
    s1, s2 = ams_signs(ams_params(seed, d), n1, n3)
    AB = np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    if subtract_diag:
        AB = AB.copy()
        np.fill_diagonal(AB, 0.0)
    X = ams_sketch(AB, s1, s2)
    return X, frobenius_bound(X), s1, s2


# ---------------------------------------------------------------------------
# number of non-zeros by doubling search (Section 5.1)
# ---------------------------------------------------------------------------

# Reading: the random diagonal matrices of Section 5.1 have entries uniform in
# [1, 2): D1[i] = 1 + (z >> 11) 2^-53 with z the SplitMix64 output
# 2^40 + i + 1 of the seed, D2[j] the same from output 2^41 + j + 1 (the
# values are used in float32).  A bucket counts as zero when its magnitude is
# at most zero_rel times the largest magnitude of its repetition (the float32
# sketch is never exactly zero); b starts at 16, the smallest sketch length
# the library takes, and doubles up to 2^20.

NNZ_D1_OFFSET = 1 << 40
NNZ_D2_OFFSET = 1 << 41


def _splitmix64_at(seed: int, k: int) -> int:
    """Output k (k >= 1) of SplitMix64 seeded with ``seed``."""
    z = (seed + k * _GAMMA) & _M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & _M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & _M64
    return z ^ (z >> 31)


def nnz_weights(seed: int, n: int, offset: int) -> np.ndarray:
    """Random diagonal entries in [1, 2), rounded to float32."""
    w = [1.0 + (_splitmix64_at(seed, offset + x + 1) >> 11) * 2.0 ** -53 for x in range(n)]
    return np.array(w, dtype=np.float32)


def estimate_nnz(A: np.ndarray, B: np.ndarray, d: int, seed: int, zero_rel: float = 1e-5,
                 b_max: int = 1 << 20, subtract_diag: bool = False):
    """Doubling search of Section 5.1 on D1 A B D2: the first b (16, 32, ...)
    at which at least 4b/5 buckets of the sketch are zero for every one of
    the d hash functions; returns (b, zeros per repetition at that b), or
    (-1, zeros at b_max) if no b up to b_max qualifies."""
    n1, n3 = A.shape[0], B.shape[1]
    D1 = nnz_weights(seed, n1, NNZ_D1_OFFSET).astype(np.float64)
    D2 = nnz_weights(seed, n3, NNZ_D2_OFFSET).astype(np.float64)
    As = np.asarray(A, np.float64) * D1[:, None]
    Bs = np.asarray(B, np.float64) * D2[None, :]
    b = 16
    zeros = None
    while b <= b_max:
        c, _, _ = run(As, Bs, b, d, seed, subtract_diag=subtract_diag)
        mx = np.abs(c).max(axis=1)
        zeros = np.array([int(np.sum(np.abs(c[t]) <= zero_rel * mx[t])) for t in range(d)])
        if np.all(5 * zeros >= 4 * b):
            return b, zeros
        b *= 2
    return -1, zeros


# ---------------------------------------------------------------------------
# sublinear extraction of significant entries (Section 4, Figure 3)
# ---------------------------------------------------------------------------

# Reading: the paper's expander code is not given.  The code used is the
# binary BCH code of length 63 with designed distance 23 (Bose, Ray-Chaudhuri,
# Hocquenghem): 16 information bits, minimum distance >= 23, so every word
# within Hamming distance t = 11 of a codeword decodes to it (a fraction
# delta = 11/63 of the 63 bits).  Index x is encoded as the systematic
# codeword of the message x + 1 (message 0, the all-zero word, is kept for
# "nothing here": a bucket without a significant entry thresholds to a string
# of low weight, which decodes to message 0 or fails).  Indices need
# x + 1 < 2^16.  Decoding: syndromes S_1..S_22 in GF(2^6), Berlekamp-Massey
# for the error locator, a search over the 63 positions for its roots
# (Chien search); more than 11 errors, or a locator whose roots are not all
# distinct positions, fails.

BCH_N, BCH_K, BCH_T = 63, 16, 11
GF64_POLY = 0b1000011          # x^6 + x + 1, primitive over GF(2)


def _gf64_tables():
    exp = [0] * 126
    log = [0] * 64
    v = 1
    for i in range(63):
        exp[i] = exp[i + 63] = v
        log[v] = i
        v <<= 1
        if v & 64:
            v ^= GF64_POLY
    return exp, log


_GF_EXP, _GF_LOG = _gf64_tables()


def _gf_mul(a: int, b: int) -> int:
    return 0 if a == 0 or b == 0 else _GF_EXP[_GF_LOG[a] + _GF_LOG[b]]


def _poly2_mul(a: int, b: int) -> int:
    """Product of two GF(2) polynomials held as bit masks (bit i = x^i)."""
    out = 0
    while b:
        if b & 1:
            out ^= a
        a <<= 1
        b >>= 1
    return out


def _poly2_mod(a: int, m: int) -> int:
    dm = m.bit_length() - 1
    while a and a.bit_length() - 1 >= dm:
        a ^= m << (a.bit_length() - 1 - dm)
    return a


def _minimal_poly(i: int) -> int:
    """Minimal polynomial over GF(2) of alpha^i: the product of (x - alpha^j)
    over the cyclotomic coset {i, 2i, 4i, ...} mod 63 (coefficients come out
    in GF(2))."""
    coset, j = [], i % 63
    while j not in coset:
        coset.append(j)
        j = (2 * j) % 63
    poly = [1]                      # coefficients in GF(64), lowest degree first
    for j in coset:
        root = _GF_EXP[j]
        nxt = [0] * (len(poly) + 1)
        for d, c in enumerate(poly):
            nxt[d + 1] ^= c                      # c x^(d+1)
            nxt[d] ^= _gf_mul(c, root)           # c root x^d (minus = plus)
        poly = nxt
    assert all(c in (0, 1) for c in poly)
    return sum(c << d for d, c in enumerate(poly))


def bch_generator() -> int:
    """Generator polynomial (bit mask) of the narrow-sense BCH code of length
    63 with roots alpha^1 .. alpha^22: the product of the distinct minimal
    polynomials of those roots (degree 47)."""
    g, seen = 1, set()
    for i in range(1, 2 * BCH_T + 1):
        mp = _minimal_poly(i)
        if mp not in seen:
            seen.add(mp)
            g = _poly2_mul(g, mp)
    return g


BCH_G = bch_generator()


def bch_encode(msg: int) -> int:
    """Systematic codeword (63-bit mask): message bits at positions 47..62,
    parity = (msg x^47) mod g at positions 0..46."""
    shifted = msg << (BCH_N - BCH_K)
    return shifted | _poly2_mod(shifted, BCH_G)


def bch_decode(word: int):
    """The message of the codeword within distance 11 of ``word`` (63-bit
    mask), or None when the decoder finds no such codeword."""
    synd = []
    for j in range(1, 2 * BCH_T + 1):
        s = 0
        for p in range(BCH_N):
            if word >> p & 1:
                s ^= _GF_EXP[(j * p) % 63]
        synd.append(s)
    if not any(synd):
        return word >> (BCH_N - BCH_K)
    # Berlekamp-Massey: shortest LFSR (error locator sigma) generating S_1..S_22
    sigma, prev = [1], [1]
    L, m, bprev = 0, 1, 1
    for n_ in range(2 * BCH_T):
        disc = synd[n_]
        for i in range(1, L + 1):
            if i < len(sigma):
                disc ^= _gf_mul(sigma[i], synd[n_ - i])
        if disc == 0:
            m += 1
            continue
        coef = _gf_mul(disc, _GF_EXP[(63 - _GF_LOG[bprev]) % 63])
        nxt = sigma + [0] * max(0, len(prev) + m - len(sigma))
        for i, c in enumerate(prev):
            nxt[i + m] ^= _gf_mul(coef, c)
        if 2 * L <= n_:
            prev, L, bprev, m = sigma, n_ + 1 - L, disc, 1
        else:
            m += 1
        sigma = nxt
    if L > BCH_T:
        return None
    # Chien search: error at position p where sigma(alpha^-p) = 0
    errors = []
    for p in range(BCH_N):
        acc = 0
        for i, c in enumerate(sigma):
            if c:
                acc ^= _gf_mul(c, _GF_EXP[(-i * p) % 63])
        if acc == 0:
            errors.append(p)
    if len(errors) != L:
        return None
    for p in errors:
        word ^= 1 << p
    return word >> (BCH_N - BCH_K)


def code_length() -> int:
    """l: bits of the code of one index."""
    return BCH_N


def code_encode(x: int) -> list[int]:
    """E(x): the 63 bits (position 0 first) of the codeword of message x + 1."""
    if not 0 <= x < (1 << BCH_K) - 1:
        raise ValueError("index out of the code's range")
    w = bch_encode(x + 1)
    return [(w >> p) & 1 for p in range(BCH_N)]


def code_decode(bits):
    """x from a (corrupted) 63-bit string, or None if the decoder fails or
    finds message 0 (no index)."""
    w = 0
    for p, v in enumerate(bits):
        if int(v):
            w |= 1 << p
    msg = bch_decode(w)
    if msg is None or msg == 0:
        return None
    return msg - 1


def masked_sketches(A: np.ndarray, B: np.ndarray, tables, b: int, subtract_diag: bool = False):
    """Count sketches, with the same hash functions, of the submatrix products
    of eq. (3): (I_{E_r} A) B for the l bits r of the row code and
    A (B I_{E_r}) for the l bits of the column code.  Returns
    (c_rows (l, d, b), c_cols (l, d, b))."""
    A = np.asarray(A, dtype=np.float64); B = np.asarray(B, dtype=np.float64)
    n1, n3 = A.shape[0], B.shape[1]
    ell = code_length()
    E1 = np.array([code_encode(i) for i in range(n1)])   # (n1, l)
    E3 = np.array([code_encode(j) for j in range(n3)])   # (n3, l)
    rows, cols = [], []
    for r in range(ell):
        P = (A * E1[:, r][:, None]) @ B
        if subtract_diag:
            np.fill_diagonal(P, 0.0)
        rows.append(bin_product(P, tables, b))
    for r in range(ell):
        P = A @ (B * E3[:, r][None, :])
        if subtract_diag:
            np.fill_diagonal(P, 0.0)
        cols.append(bin_product(P, tables, b))
    return np.array(rows), np.array(cols)


def find_significant(c_rows: np.ndarray, c_cols: np.ndarray, n1: int, n3: int, delta: float):
    """FINDSIGNIFICANTENTRIES (Figure 3): for every repetition t and bucket k,
    the bit string s_r = [|p^(t,r)[k]| > delta/2] over the row-code sketches
    and then the column-code sketches is decoded into (i, j) and inserted
    into a multiset; positions inserted fewer than d/2 times are deleted.
    Returns the sorted linear indices i*n3 + j of the kept positions and the
    multiset counts."""
    ell = code_length()
    d, b = c_rows.shape[1], c_rows.shape[2]
    counts: dict[int, int] = {}
    for t in range(d):
        for k in range(b):
            s1 = [abs(c_rows[r, t, k]) > delta / 2 for r in range(ell)]
            s3 = [abs(c_cols[r, t, k]) > delta / 2 for r in range(ell)]
            if sum(s1) == 0 or sum(s3) == 0:      # message 0: nothing here
                continue
            i, j = code_decode(s1), code_decode(s3)
            if i is None or j is None or i >= n1 or j >= n3:
                continue
            key = i * n3 + j
            counts[key] = counts.get(key, 0) + 1
    kept = sorted(k for k, v in counts.items() if 2 * v >= d)
    return np.array(kept, dtype=np.int64), counts


# ---------------------------------------------------------------------------
# a whole product, as the GPU path is asked for it
# ---------------------------------------------------------------------------

def run(A: np.ndarray, B: np.ndarray, b: int, d: int, seed: int, subtract_diag: bool = False,
        params: np.ndarray | None = None, tables=None):
    """Sketch of AB (definition form) for ``d`` repetitions; returns
    (c, tables, AB)."""
    n1, n3 = A.shape[0], B.shape[1]
    if tables is None:
        params = hash_params(seed, d) if params is None else params
        tables = hash_tables(params, n1, n3, b)
    AB = np.asarray(A, dtype=np.float64) @ np.asarray(B, dtype=np.float64)
    c = bin_product(AB, tables, b)
    if subtract_diag:
        c = subtract_diagonal(c, np.diag(AB).copy(), tables, b)
    return c, tables, AB
