"""Pins of the CPU oracle against what the paper and mathematics fix.

None of these compare the oracle with itself: each checks a function against
a known answer, a closed form, a theorem of the paper, brute force, or an
independent formulation that shares no code with it.
"""
import math
import os

import numpy as np
import pytest

from oracle import cmm_oracle as O
import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


# ---------------------------------------------------------------- randomness

def test_splitmix64_known_answers():
    with open(os.path.join(GOLDEN, "splitmix64_kat.txt")) as f:
        rows = [l.split() for l in f if l.strip() and not l.startswith("#")]
    for row in rows:
        seed = int(row[0], 0)
        want = [int(x, 0) for x in row[1:]]
        assert O.splitmix64(seed, len(want)) == want


def test_hash_params_ranges():
    pr = O.hash_params(12345, 7)
    assert pr.shape == (7, 4, 2)
    a = pr[:, :, 0].astype(object); c = pr[:, :, 1].astype(object)
    assert all(1 <= int(x) < O.P61 for x in a.ravel())
    assert all(0 <= int(x) < O.P61 for x in c.ravel())
    # 8d distinct stream outputs feed 8d distinct parameters
    assert len({int(x) for x in pr.ravel()}) == 8 * 7


def test_hash_params_seed0_known_answers():
    """Repetition 0's h1 and s1 parameters for seed 0 equal the values worked
    out by hand from the published SplitMix64 outputs z1..z4 of seed 0
    (tests/golden/hash_params_seed0.txt): catches an off-by-one in the output
    index, swapped a/c, or a wrong modulus."""
    with open(os.path.join(GOLDEN, "hash_params_seed0.txt")) as f:
        rows = {r[0]: (int(r[1]), int(r[2])) for r in
                (l.split() for l in f if l.strip() and not l.startswith("#"))}
    pr = O.hash_params(0, 1)
    assert (int(pr[0, 0, 0]), int(pr[0, 0, 1])) == rows["h1"]
    assert (int(pr[0, 1, 0]), int(pr[0, 1, 1])) == rows["s1"]
    # the hash values those parameters give, worked out by hand: g(0) = c,
    # g(1) = a + c (below p here), h = g mod 1024, s from the parity of g
    a, c = rows["h1"]
    h1, s1, _, _ = O.hash_tables(pr, 2, 1, 1024)
    assert h1[0].tolist() == [c % 1024, (a + c) % 1024] == [503, 949]
    a, c = rows["s1"]
    assert s1[0].tolist() == [1 - 2 * (c % 2), 1 - 2 * ((a + c) % 2)] == [-1, -1]


def test_hash_params_counter_layout():
    """SplitMix64 is a counter generator: output k of seed s is output 1 of
    seed s + (k - 1) * gamma (mod 2^64).  Function f of repetition t reads
    outputs 8t + 2f + 1 and 8t + 2f + 2, so its parameters must equal the
    repetition-0 h1 parameters of the seed advanced by (8t + 2f) gamma; with
    the known answers above this pins every (t, f) slot."""
    gamma = 0x9E3779B97F4A7C15
    for seed in (0, 2002, 2**64 - 5):
        pr = O.hash_params(seed, 4)
        for t in range(4):
            for f in range(4):
                moved = (seed + (8 * t + 2 * f) * gamma) % 2**64
                q = O.hash_params(moved, 1)
                assert (int(pr[t, f, 0]), int(pr[t, f, 1])) == (int(q[0, 0, 0]), int(q[0, 0, 1])), (seed, t, f)


def _mersenne_mod(v: int) -> int:
    """v mod (2^61-1) by repeated folding of 61-bit digits (an independent
    route to the same residue)."""
    while v >> 61:
        v = (v & O.P61) + (v >> 61)
    return 0 if v == O.P61 else v


def test_cw_hash_known_values():
    assert O.cw_hash(3, 5, [7]) == [26]
    p = O.P61
    assert O.cw_hash(p - 1, p - 1, [2]) == [p - 3]          # 3(p-1) = 3p - 3
    assert O.cw_hash(1, 0, [p, p + 1]) == [0, 1]
    g = np.random.default_rng(0)
    for _ in range(200):
        a = int(g.integers(1, 2**61 - 1)); c = int(g.integers(0, 2**61 - 1)); x = int(g.integers(0, 2**32))
        assert O.cw_hash(a, c, [x])[0] == _mersenne_mod(a * x + c)


def test_hash_tables_definition():
    pr = O.hash_params(7, 2)
    h1, s1, h2, s2 = O.hash_tables(pr, 10, 9, 64)
    for t in range(2):
        for x in range(10):
            g = (int(pr[t, 0, 0]) * x + int(pr[t, 0, 1])) % O.P61
            assert h1[t, x] == g & 63
            gs = (int(pr[t, 1, 0]) * x + int(pr[t, 1, 1])) % O.P61
            assert s1[t, x] == (1 if gs % 2 == 0 else -1)


def test_hash_pairwise_collisions():
    """2-wise independence (Section 2.2): over random parameters a pair of
    distinct keys collides with probability ~1/b, and a sign pair agrees
    with probability ~1/2."""
    b, trials = 16, 4000
    coll = agree = 0
    for s in range(trials):
        pr = O.hash_params(10_000 + s, 1)
        h1, s1, _, _ = O.hash_tables(pr, 6, 1, b)
        coll += int(h1[0, 2] == h1[0, 5])
        agree += int(s1[0, 1] == s1[0, 4])
    p = coll / trials
    assert abs(p - 1 / b) < 4 * math.sqrt((1 / b) * (1 - 1 / b) / trials)
    q = agree / trials
    assert abs(q - 0.5) < 4 * math.sqrt(0.25 / trials)


# ------------------------------------------------------------- dequantising

def test_e4m3fn_known_values():
    # OCP 8-bit floating point spec, E4M3: max normal 448, min normal 2^-6,
    # min subnormal 2^-9, 0x7f / 0xff are NaN.
    v = O.dequantise(np.array([[0x7E, 0x08, 0x01, 0x38, 0xB8, 0x00, 0x80, 0x7F]], np.uint8), "fp8")[0]
    assert v[0] == 448.0 and v[1] == 2.0 ** -6 and v[2] == 2.0 ** -9
    assert v[3] == 1.0 and v[4] == -1.0 and v[5] == 0.0 and v[6] == 0.0
    assert math.isnan(v[7])
    # the encoder of the input generator inverts the decoder on every finite code
    codes = np.array([c for c in range(256) if (c & 0x7F) != 0x7F], np.uint8)
    vals = O.dequantise(codes[None, :], "fp8")[0]
    back = W.e4m3fn_encode(vals)
    same = (back == codes) | ((vals == 0) & ((back & 0x7F) == 0))
    assert same.all()


def test_bf16_known_values():
    v = O.dequantise(np.array([[0x3F80, 0xC000, 0x0000, 0x7F7F]], np.uint16), "bf16")[0]
    assert v[0] == 1.0 and v[1] == -2.0 and v[2] == 0.0
    assert v[3] == float(np.float32(3.3895313892515355e38))


# ------------------------------------------------------------------ sketch

def test_countsketch_bruteforce():
    g = np.random.default_rng(1)
    v = g.standard_normal(40); h = g.integers(0, 8, 40); s = g.choice([-1, 1], 40)
    p = O.countsketch(v, h, s, 8)
    for u in range(8):
        acc = 0.0
        for i in range(40):
            if h[i] == u:
                acc += s[i] * v[i]
        assert abs(p[u] - acc) < 1e-12


def test_hand_worked_example():
    A = np.array([[1.0], [2.0]]); B = np.array([[3.0, 4.0]])
    h1 = np.array([[0, 1]]); h2 = np.array([[0, 1]])
    with open(os.path.join(GOLDEN, "hand_sketch.txt")) as f:
        rows = [[int(x) for x in l.split()] for l in f if l.strip() and not l.startswith("#")]
    for s10, s11, s20, s21, c0, c1 in rows:
        tabs = (h1, np.array([[s10, s11]]), h2, np.array([[s20, s21]]))
        for fn in (O.sketch_from_product, O.sketch_polynomial):
            c = fn(A, B, tabs, 2)
            assert c[0].tolist() == [c0, c1]


def _brute_sketch(A, B, tabs, b):
    h1, s1, h2, s2 = tabs
    d = h1.shape[0]
    n1, m = A.shape; n3 = B.shape[1]
    c = [[0.0] * b for _ in range(d)]
    for t in range(d):
        for i in range(n1):
            for j in range(n3):
                ab = 0.0
                for k in range(m):
                    ab += float(A[i, k]) * float(B[k, j])
                u = (int(h1[t, i]) + int(h2[t, j])) % b
                c[t][u] += int(s1[t, i]) * int(s2[t, j]) * ab
    return np.array(c)


def test_definition_bruteforce():
    g = np.random.default_rng(2)
    A = g.standard_normal((5, 4)); B = g.standard_normal((4, 6))
    tabs = O.hash_tables(O.hash_params(99, 3), 5, 6, 8)
    np.testing.assert_allclose(O.sketch_from_product(A, B, tabs, 8), _brute_sketch(A, B, tabs, 8),
                               rtol=0, atol=1e-12)


@pytest.mark.parametrize("shape,b,d", [((13, 7, 11), 16, 3), ((32, 9, 20), 64, 2), ((20, 20, 20), 16, 1)])
def test_polynomial_equals_definition(shape, b, d):
    n1, m, n3 = shape
    g = np.random.default_rng(n1 * 100 + b)
    A = g.standard_normal((n1, m)); B = g.standard_normal((m, n3))
    tabs = O.hash_tables(O.hash_params(5 + b, d), n1, n3, b)
    c1 = O.sketch_polynomial(A, B, tabs, b)
    c2 = O.sketch_from_product(A, B, tabs, b)
    np.testing.assert_allclose(c1, c2, rtol=0, atol=1e-11 * np.abs(c2).max())


def test_injective_hashes_recover_product():
    """h1(i) = i, h2(j) = n1*j, s = +1 and b >= n1*n3 make the splitting
    function injective, so the sketch holds AB itself (c[i + n1 j] = (AB)_ij)
    and decoding returns AB.  Checked against numpy's matrix product; the
    polynomial form uses no matrix product."""
    n1, m, n3 = 6, 5, 7
    b = 64
    g = np.random.default_rng(3)
    A = g.standard_normal((n1, m)); B = g.standard_normal((m, n3))
    tabs = (np.arange(n1)[None, :], np.ones((1, n1), np.int64),
            (n1 * np.arange(n3))[None, :], np.ones((1, n3), np.int64))
    c = O.sketch_polynomial(A, B, tabs, b)
    AB = A @ B
    for i in range(n1):
        for j in range(n3):
            assert abs(c[0, i + n1 * j] - AB[i, j]) < 1e-12
    C = O.decode_all(c, tabs, n1, n3)
    np.testing.assert_allclose(C, AB, rtol=0, atol=1e-12)


def test_b1_is_ams_sketch():
    """b = 1: every pair shares the one bucket, so the sketch is the AMS
    sketch of AB, the sum over k of (s1 . a_k)(s2 . b_k) (Section 2.1)."""
    g = np.random.default_rng(4)
    A = g.standard_normal((9, 8)); B = g.standard_normal((8, 10))
    tabs = O.hash_tables(O.hash_params(17, 2), 9, 10, 1)
    for fn in (O.sketch_from_product, O.sketch_polynomial):
        c = fn(A, B, tabs, 1)
        for t in range(2):
            ams = sum(float(tabs[1][t] @ A[:, k]) * float(B[k, :] @ tabs[3][t]) for k in range(8))
            assert abs(c[t, 0] - ams) < 1e-11


def test_k_split_linearity():
    """The sketch is linear in the outer products (eq. (1)): splitting k
    into two ranges and adding the sketches gives the whole sketch."""
    g = np.random.default_rng(5)
    A = g.standard_normal((10, 12)); B = g.standard_normal((12, 9))
    tabs = O.hash_tables(O.hash_params(23, 2), 10, 9, 32)
    whole = O.sketch_polynomial(A, B, tabs, 32)
    part = O.sketch_polynomial(A[:, :5], B[:5], tabs, 32) + O.sketch_polynomial(A[:, 5:], B[5:], tabs, 32)
    np.testing.assert_allclose(whole, part, rtol=0, atol=1e-12)


def test_subtract_diagonal_matches_binning_zeroed_diagonal():
    g = np.random.default_rng(6)
    X = g.standard_normal((11, 8))
    A, B = X.T, X
    tabs = O.hash_tables(O.hash_params(31, 3), 8, 8, 16)
    c, _, AB = O.run(A, B, 16, 3, 0, subtract_diag=True, tables=tabs)
    Z = AB - np.diag(np.diag(AB))
    np.testing.assert_allclose(c, O.bin_product(Z, tabs, 16), rtol=0, atol=1e-11)


# -------------------------------------------------------------- decoding

def test_median_conventions():
    x = np.array([[3.0, 1.0], [1.0, 4.0], [2.0, 1.0]])
    assert O.median(x, 0).tolist() == [2.0, 1.0]
    y = np.array([[4.0], [1.0], [3.0], [2.0]])
    assert O.median(y, 0).tolist() == [2.5]
    g = np.random.default_rng(7)
    for d in range(1, 12):
        z = g.standard_normal((d, 50))
        np.testing.assert_array_equal(O.median(z, 0), np.median(z, axis=0))


def test_topk_order_and_ties():
    vals = np.array([1.0, -3.0, 3.0, 0.5, -3.0, 2.0])
    lin = np.array([10, 4, 7, 1, 2, 3])
    sel_lin, sel_val = O.topk(vals, lin, 4)
    assert sel_lin.tolist() == [2, 4, 7, 3]
    assert sel_val.tolist() == [-3.0, -3.0, 3.0, 2.0]


def test_candidates_hand_listing():
    """The candidate domains written out by hand: every (i, j) of a 2 x 3
    product in linear-index order, and the n(n-1)/2 pairs i < j of n = 4."""
    i, j = O.candidates("all", 2, 3)
    assert list(zip(i.tolist(), j.tolist())) == [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2)]
    i, j = O.candidates("upper", 4, 4)
    assert list(zip(i.tolist(), j.tolist())) == [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3)]
    for n in (1, 2, 5, 37):
        i, j = O.candidates("upper", n, n)
        assert len(i) == n * (n - 1) // 2
        assert np.all(i < j) and len(set(zip(i.tolist(), j.tolist()))) == len(i)
    assert len(O.candidates("all", 7, 3)[0]) == 21


def test_topk_per_column_hand_example_with_ties():
    """Per-column selection on a hand example: column 0 has a tie of |3| at
    rows 1 and 2 (smaller row first), column 1 a three-way tie of |2| at
    rows 0, 1 and 3 of which only the two smallest rows are kept."""
    C = np.array([[1.0, -2.0],
                  [-3.0, 2.0],
                  [3.0, 0.5],
                  [0.0, -2.0]])
    rows, vals = O.topk_per_column(C, 2)
    assert rows.tolist() == [[1, 2], [0, 1]]
    assert vals.tolist() == [[-3.0, 3.0], [-2.0, 2.0]]
    rows, vals = O.topk_per_column(C, 4)
    assert rows.tolist() == [[1, 2, 0, 3], [0, 1, 3, 2]]
    assert vals.tolist() == [[-3.0, 3.0, 1.0, 0.0], [-2.0, 2.0, -2.0, 0.5]]


def test_theorem2_unbiased_and_variance():
    """Theorem 2: with d = 1 the estimate is unbiased and its variance is at
    most ||AB||_F^2 / b; for a pairwise-independent splitting function it is
    close to (||AB||_F^2 - AB_ij^2) / b."""
    g = np.random.default_rng(8)
    A = g.standard_normal((6, 5)); B = g.standard_normal((5, 7))
    AB = A @ B
    b, S = 16, 3000
    i, j = 2, 3
    est = np.empty(S)
    for s in range(S):
        tabs = O.hash_tables(O.hash_params(50_000 + s, 1), 6, 7, b)
        c = O.sketch_from_product(A, B, tabs, b)
        est[s] = O.decode(c, tabs, [i], [j])[0]
    fro2 = float((AB ** 2).sum())
    se = math.sqrt(fro2 / b / S)
    assert abs(est.mean() - AB[i, j]) < 4 * se
    var = est.var(ddof=1)
    assert var <= fro2 / b * 1.15
    assert abs(var - (fro2 - AB[i, j] ** 2) / b) < 0.15 * fro2 / b


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_theorem5_sparse_product_exact(seed):
    """Theorem 5: AB with at most b/8 nonzeros and d >= 6 lg n is decoded
    exactly.  The product is sparse only through cancellation: A = Q random
    orthogonal, B = Q^T S."""
    n = 32
    g = np.random.default_rng(100 + seed)
    Q, _ = np.linalg.qr(g.standard_normal((n, n)))
    S = np.zeros((n, n))
    pos = g.choice(n * n, size=16, replace=False)
    S.flat[pos] = g.standard_normal(16) * 10
    A, B = Q, Q.T @ S
    b = 128                                   # 16 nonzeros = b/8
    d = int(math.ceil(6 * math.log2(n))) | 1  # 31
    c, tabs, AB = O.run(A, B, b, d, 900 + seed)
    C = O.decode_all(c, tabs, n, n)
    assert np.abs(C - S).max() < 1e-9 * np.abs(S).max()


def test_theorem6_tail_bound():
    """Theorem 6: with d >= 6 lg n every estimate is within
    12 sqrt(Err_F^{b/20}(AB) / b) of AB."""
    n = 32
    g = np.random.default_rng(200)
    A = g.standard_normal((n, n)); B = g.standard_normal((n, n)) * 0.05
    B += np.eye(n) * 0                        # keep B generic
    P = np.zeros((n, n)); P.flat[g.choice(n * n, 12, replace=False)] = 40.0
    AB_target = A @ B + P
    B2 = np.linalg.solve(A, AB_target)        # A @ B2 = AB_target
    b = 256
    d = int(math.ceil(6 * math.log2(n))) | 1
    c, tabs, AB = O.run(A, B2, b, d, 321)
    C = O.decode_all(c, tabs, n, n)
    mags = np.sort(np.abs(AB).ravel())[::-1]
    err_f = float((mags[b // 20:] ** 2).sum())
    bound = 12 * math.sqrt(err_f / b)
    assert np.abs(C - AB).max() < bound


def test_sketch_buckets_matches_definition():
    """One-bucket-at-a-time evaluation equals the binned definition, with and
    without the diagonal."""
    g = np.random.default_rng(9)
    A = g.standard_normal((37, 11)); B = g.standard_normal((11, 37))
    tabs = O.hash_tables(O.hash_params(41, 2), 37, 37, 32)
    full = O.sketch_from_product(A, B, tabs, 32)
    AB = A @ B
    zeroed = O.bin_product(AB - np.diag(np.diag(AB)), tabs, 32)
    us = [0, 5, 17, 31]
    for t in range(2):
        np.testing.assert_allclose(O.sketch_buckets(A, B, tabs, 32, t, us), full[t, us], atol=1e-12)
        np.testing.assert_allclose(O.sketch_buckets(A, B, tabs, 32, t, us, zero_diagonal=True),
                                   zeroed[t, us], atol=1e-12)


# --------------------------------------------------------------------------
# Frobenius-norm bound (Section 5.2; AMS sketch of Section 2.1)
# --------------------------------------------------------------------------

def test_poly_hash_hand_values():
    P = O.P61
    assert O.poly_hash([5, 0, 0, 0], [0, 1, 12345]) == [5, 5, 5]
    assert O.poly_hash([0, 1, 0, 0], [P - 1, P, P + 3]) == [P - 1, 0, 3]
    # x^3: (p-1)^3 = -1 mod p; 2^21 cubed is 2^63 = 4 * 2^61 = 4 mod p
    assert O.poly_hash([0, 0, 0, 1], [P - 1, 2, 1 << 21]) == [P - 1, 8, 4]
    assert O.poly_hash([1, 1, 1, 1], [2]) == [15]
    assert O.poly_hash([P - 1, P - 1, 0, 0], [1]) == [P - 2]


def test_ams_params_stream_and_range():
    p = O.ams_params(77, 3)
    z = O.splitmix64(77, 1024 + 24)
    assert p.shape == (3, 2, 4)
    assert int(p[2, 1, 3]) == z[1024 + 8 * 2 + 4 * 1 + 3] % O.P61
    assert all(int(v) < O.P61 for v in p.ravel())


def _signs_at(seed, xs):
    p = O.ams_params(seed, 1)
    return [1 - 2 * (g % 2) for g in O.poly_hash(p[0, 0], xs)]


@pytest.mark.parametrize("xs", [(0, 1, 2, 3), (5, 1000, 77, 1 << 20)])
def test_ams_signs_four_wise(xs):
    """Degree-3 polynomial signs are 4-wise independent (Section 5.2 needs
    it): over many seeds every pattern of the four signs is equally likely,
    and every product of two, three or four of them averages to 0."""
    S = 1600
    pats = np.zeros(16, np.int64)
    prods = {k: [] for k in [(0, 1), (1, 2), (0, 3), (0, 1, 2), (1, 2, 3), (0, 1, 2, 3)]}
    for seed in range(S):
        s = _signs_at(seed, xs)
        pats[sum((1 if s[q] < 0 else 0) << q for q in range(4))] += 1
        for k in prods:
            prods[k].append(np.prod([s[q] for q in k]))
    chi2 = float(((pats - S / 16) ** 2 / (S / 16)).sum())
    assert chi2 < 45.0, chi2          # 15 dof; P(chi2 > 45) < 1e-4
    for k, v in prods.items():
        assert abs(np.mean(v)) < 4.5 / np.sqrt(S), (k, np.mean(v))


def test_ams_sketch_definition_equals_outer_products():
    g = np.random.default_rng(3)
    A = g.standard_normal((9, 5)); B = g.standard_normal((5, 7))
    s1, s2 = O.ams_signs(O.ams_params(11, 4), 9, 7)
    np.testing.assert_allclose(O.ams_sketch(A @ B, s1, s2), O.ams_sketch_outer(A, B, s1, s2),
                               rtol=1e-12, atol=1e-12)


def test_ams_hand_example():
    rows = {}
    for line in open(os.path.join(GOLDEN, "hand_ams.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            rows[k] = [float(x) for x in v]
    A = np.array(rows["A"])[:, None]; B = np.array(rows["B"])[None, :]
    s1 = np.array([rows["s1"]], np.int64); s2 = np.array([rows["s2"]], np.int64)
    assert O.ams_sketch(A @ B, s1, s2)[0] == rows["X"][0]
    assert O.ams_sketch_outer(A, B, s1, s2)[0] == rows["X"][0]
    Z = A @ B
    np.fill_diagonal(Z, 0.0)
    assert O.ams_sketch(Z, s1, s2)[0] == rows["X_zero_diagonal"][0]


def test_ams_moments_section_5_2():
    """X^2 is unbiased for ||AB||_F^2 with variance at most 8 E[X^2]^2."""
    g = np.random.default_rng(8)
    A = g.standard_normal((12, 8)); B = g.standard_normal((8, 10))
    AB = A @ B
    F2 = float((AB ** 2).sum())
    S = 1500
    x2 = np.array([O.ams_sketch(AB, *O.ams_signs(O.ams_params(seed, 1), 12, 10))[0] ** 2
                   for seed in range(S)])
    se = x2.std() / np.sqrt(S)
    assert abs(x2.mean() - F2) < 4 * se, (x2.mean(), F2, se)
    assert x2.var() <= 8 * F2 ** 2 * 1.2


def test_frobenius_bound_holds_and_is_not_vacuous():
    """32 * median of d = 9 estimators bounds ||AB||_F^2 from above.

    Chebyshev with Var(X^2) <= 8 E[X^2]^2 controls only the upper tail
    (P(X^2 > 32 ||AB||_F^2) <= 8/31^2).  Whether 32 * median stays above
    ||AB||_F^2 depends on the lower tail P(X^2 < ||AB||_F^2 / 32), about 0.17
    per estimator for this product (near-Gaussian X gives 0.14), so the median
    of 9 falls short with probability about 1e-2: the bound may fail rarely,
    and fails for at most a few of 200 seeds."""
    g = np.random.default_rng(9)
    A = g.standard_normal((10, 6)); B = g.standard_normal((6, 11))
    F2 = float(((A @ B) ** 2).sum())
    ratios, fails, over = [], 0, 0
    for seed in range(200):
        X, bound, _, _ = O.frobenius(A, B, 9, 5000 + seed)
        fails += bound < F2
        over += int(np.sum(X ** 2 > 32 * F2))
        ratios.append(bound / F2)
    assert fails <= 8, fails                   # expected about 2
    assert over <= 0.02 * 200 * 9, over        # Chebyshev: rate <= 8/961
    assert np.median(ratios) < 64.0


# --------------------------------------------------------------------------
# sublinear extraction (Section 4, Figure 3) with the complement code
# --------------------------------------------------------------------------

def test_bch_generator_known_answer():
    """The generator polynomial of the binary primitive BCH code of length 63
    correcting 11 errors, as tabulated in octal in the coding-theory
    literature (Lin and Costello, Error Control Coding, appendix of BCH
    generator polynomials: n = 63, k = 16, t = 11): 6331141367235453."""
    assert O.BCH_G == 0o6331141367235453


def test_bch_generator_divides_x63_plus_1_and_has_the_roots():
    """g(x) divides x^63 + 1 over GF(2) (plain polynomial long division,
    independent of the field tables), has degree 63 - 16, and vanishes at
    alpha^1 .. alpha^22 (evaluated by Horner's rule in GF(2^6))."""
    g = O.BCH_G
    assert g.bit_length() - 1 == 47
    a, m = (1 << 63) | 1, g
    while a and a.bit_length() >= m.bit_length():
        a ^= m << (a.bit_length() - m.bit_length())
    assert a == 0
    # GF(2^6) by shift-and-reduce multiplication (no tables)
    def mul(x, y):
        r = 0
        while y:
            if y & 1:
                r ^= x
            y >>= 1
            x <<= 1
            if x & 64:
                x ^= 0b1000011
        return r
    def power(x, e):
        r = 1
        for _ in range(e):
            r = mul(r, x)
        return r
    alpha = 2
    for j in range(1, 23):
        aj = power(alpha, j)
        acc = 0
        for bit in range(g.bit_length() - 1, -1, -1):
            acc = mul(acc, aj) ^ ((g >> bit) & 1)
        assert acc == 0, j


def test_bch_minimum_distance_by_enumeration():
    """Every non-zero codeword has weight >= 23 (the code is linear, so the
    minimum distance is the minimum weight): all 65535 messages."""
    assert min(bin(O.bch_encode(m)).count("1") for m in range(1, 1 << 16)) >= 23
    assert O.bch_encode(5) >> 47 == 5                         # systematic


def test_bch_decodes_up_to_eleven_errors():
    """DECODE recovers the index from any string within distance
    floor(delta l) = 11 of its codeword: random messages with 0..11 random
    flips, and the worst placements (the 11 highest and the 11 lowest bit
    positions)."""
    g = np.random.default_rng(5)
    for trial in range(400):
        x = int(g.integers(0, 65534))
        e = O.code_encode(x)
        flips = g.choice(63, int(g.integers(0, 12)), replace=False) if trial % 3 else g.choice(63, 11, replace=False)
        f = list(e)
        for q in flips:
            f[q] ^= 1
        assert O.code_decode(f) == x
    for x in (0, 1, 4095, 65533):
        for block in (range(52, 63), range(0, 11)):
            f = O.code_encode(x)
            for q in block:
                f[q] ^= 1
            assert O.code_decode(f) == x


def test_bch_empty_and_beyond_capacity():
    """A string of weight <= 11 (an empty bucket, or one entry whose bits
    mostly drowned) is message 0 or nothing, never an index; strings far from
    every codeword (14 flips) are rejected rather than decoded wrongly in
    these trials."""
    assert O.code_decode([0] * 63) is None
    g = np.random.default_rng(6)
    for _ in range(100):
        w = [0] * 63
        for q in g.choice(63, int(g.integers(1, 12)), replace=False):
            w[q] = 1
        assert O.code_decode(w) is None
    wrong = 0
    for _ in range(100):
        x = int(g.integers(0, 65534))
        f = O.code_encode(x)
        for q in g.choice(63, 14, replace=False):
            f[q] ^= 1
        r = O.code_decode(f)
        wrong += r is not None and r != x
    assert wrong == 0


def _sparse_product(n1, m, n3, nnz, seed, small=0):
    """A (n1 x m, full row rank) and B = pinv(A) S, so AB = S exactly up to
    rounding: nnz entries of magnitude in [1, 2] (and `small` of 0.01)."""
    g = np.random.default_rng(seed)
    A = g.standard_normal((n1, m))
    S = np.zeros((n1, n3))
    pos = g.choice(n1 * n3, nnz + small, replace=False)
    S.flat[pos[:nnz]] = g.choice([-1.0, 1.0], nnz) * g.uniform(1.0, 2.0, nnz)
    S.flat[pos[nnz:]] = 0.01
    B = np.linalg.pinv(A) @ S
    return A, B, np.sort(pos[:nnz])


@pytest.mark.parametrize("case", [(64, 64, 64, 12, 256, 7), (40, 90, 70, 20, 512, 9),
                                  (100, 120, 30, 8, 128, 5)])
def test_find_significant_recovers_sparse_product(case):
    """Theorem 7 / Corollary 8: a product with few non-zeros (far fewer than
    b) is returned exactly: every non-zero position and nothing else."""
    n1, m, n3, nnz, b, d = case
    A, B, support = _sparse_product(n1, m, n3, nnz, n1 + n3)
    tabs = O.hash_tables(O.hash_params(17, d), n1, n3, b)
    cr, cc = O.masked_sketches(A, B, tabs, b)
    kept, _ = O.find_significant(cr, cc, n1, n3, 0.5)
    np.testing.assert_array_equal(kept, support)


def test_find_significant_omits_entries_below_delta():
    """Entries well below Delta are not reported (Theorem 7 may omit them);
    entries well above it are."""
    A, B, support = _sparse_product(60, 80, 60, 10, 3, small=25)
    tabs = O.hash_tables(O.hash_params(23, 7), 60, 60, 512)
    cr, cc = O.masked_sketches(A, B, tabs, 512)
    kept, _ = O.find_significant(cr, cc, 60, 60, 0.5)
    np.testing.assert_array_equal(kept, support)


def test_masked_sketch_definition():
    """Masked sketch r is the sketch of the product with the rows (columns)
    whose code bit r is 0 removed: it equals the whole product's sketch minus
    the sketch of the product restricted to the other rows (columns)."""
    g = np.random.default_rng(2)
    A = g.standard_normal((20, 9)); B = g.standard_normal((9, 13))
    tabs = O.hash_tables(O.hash_params(4, 3), 20, 13, 64)
    cr, cc = O.masked_sketches(A, B, tabs, 64)
    whole = O.bin_product(A @ B, tabs, 64)
    E1 = np.array([O.code_encode(i) for i in range(20)])
    E3 = np.array([O.code_encode(j) for j in range(13)])
    for r in (0, 17, 46, 62):
        rest = O.bin_product(((1 - E1[:, r])[:, None] * A) @ B, tabs, 64)
        np.testing.assert_allclose(cr[r] + rest, whole, atol=1e-12)
        rest = O.bin_product(A @ (B * (1 - E3[:, r])[None, :]), tabs, 64)
        np.testing.assert_allclose(cc[r] + rest, whole, atol=1e-12)


# --------------------------------------------------------------------------
# number of non-zeros by doubling search (Section 5.1)
# --------------------------------------------------------------------------

def test_nnz_weights_range_and_stream():
    w = O.nnz_weights(9, 50, O.NNZ_D1_OFFSET)
    assert w.dtype == np.float32 and np.all(w >= 1.0) and np.all(w <= 2.0)
    z = O.splitmix64(9, 3)
    assert O._splitmix64_at(9, 3) == z[2]          # same stream definition
    assert abs(float(O.nnz_weights(9, 1, 0)[0]) - (1.0 + (z[0] >> 11) * 2.0 ** -53)) < 1e-7


@pytest.mark.parametrize("nnz", [5, 40, 300])
def test_nnz_estimate_brackets_true_count(nnz):
    """Section 5.1: the returned b is an upper bound on the number of
    non-zeros (whp) and, since the search stops once b/5 exceeds it, at most
    ten times it (doubling).  AB = S is formed from dense A and B (B =
    pinv(A) S), so the non-zeros are the product's, not the operands'
    structure: the random diagonal scaling keeps cancellation from hiding
    or creating them."""
    A, B, support = _sparse_product(80, 100, 90, nnz, nnz)
    for seed in range(3):
        b, zeros = O.estimate_nnz(A, B, 7, seed)
        assert nnz <= b <= 10 * max(nnz, 2), (nnz, b)
        assert np.all(5 * zeros >= 4 * b)


def test_nnz_estimate_zero_product_and_dense_product():
    g = np.random.default_rng(0)
    A = g.standard_normal((30, 20)); Z = np.zeros((20, 25))
    assert O.estimate_nnz(A, Z, 3, 1)[0] == 16
    # a dense 30 x 25 product (750 non-zeros) needs b >= 750
    b, _ = O.estimate_nnz(A, g.standard_normal((20, 25)), 3, 1)
    assert 750 <= b <= 7500
