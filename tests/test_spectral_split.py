"""CPU checks of the algebra the spectral kernels rely on (numpy only, no
library call): the four-step split of a length-b DFT of a real sequence
(Section 2.2's FFT of the count-sketch polynomials), the row pair {0, R/2}
computed as one length-2C real DFT through a C-point complex FFT and the
real split, and the fold slot rule taken from the fold-entry encoding.

These pin the identities, not the kernels: the GPU parity tests compare the
kernels with the float64 oracle.
"""
import numpy as np
import pytest

CASES = [(2, 16), (4, 32), (16, 64), (16, 4096), (64, 256)]


def _sparse_real(b, nnz, rng):
    x = np.zeros(b)
    idx = rng.choice(b, nnz, replace=False)
    x[idx] = rng.standard_normal(nnz)
    return x


@pytest.mark.parametrize("R,C", CASES)
def test_four_step_rows(R, C):
    """Row f1 of the spectrum: X[f1 + R f2] = DFT_C(z)[f2] with
    z[r] = w_b^(f1 r) * sum_q x[r + C q] w_R^(f1 q)."""
    rng = np.random.default_rng(R * 1000 + C)
    b = R * C
    x = _sparse_real(b, max(1, b // 16), rng)
    X = np.fft.fft(x)
    r = np.arange(C)
    for f1 in range(R // 2 + 1):
        q = np.arange(R)
        wq = np.exp(-2j * np.pi * f1 * q / R)
        z = np.exp(-2j * np.pi * f1 * r / b) * (x.reshape(R, C) * wq[:, None]).sum(0)
        row = np.fft.fft(z)
        assert np.allclose(row, X[f1 + R * np.arange(C)], atol=1e-9 * max(1.0, np.abs(X).max()))


def _two_p(x, C):
    """2 P[f] for f < C and 2 P[C] of the length-2C real DFT P of the 2C-fold
    of x, from one C-point complex FFT of z[s] = p[2s] + i p[2s+1]."""
    p = x.reshape(-1, 2 * C).sum(0)
    z = p[0::2] + 1j * p[1::2]
    Z = np.fft.fft(z)
    f = np.arange(C)
    Zm = Z[(C - f) % C]
    ev = Z + np.conj(Zm)
    od = -1j * (Z - np.conj(Zm))
    w = np.exp(-2j * np.pi * f / (2 * C))
    return ev + w * od, 2.0 * (Z[0].real - Z[0].imag)


@pytest.mark.parametrize("R,C", CASES)
def test_row_pair_from_one_fft(R, C):
    """Rows 0 and R/2 of X_A X_B from the 2C real split, with the mirror
    mapping the pair kernel writes: row 0 position g is frequency 2g, row
    R/2 position g is 2g + 1, frequencies at or above C by conjugation."""
    rng = np.random.default_rng(7 * R + C)
    b = R * C
    xa = _sparse_real(b, max(1, b // 16), rng)
    xb = _sparse_real(b, max(1, b // 16), rng)
    pa, na = _two_p(xa, C)
    pb, nb = _two_p(xb, C)
    acc, accn = pa * pb, na * nb              # 4 P_A P_B
    row0 = np.empty(C, complex)
    rowh = np.empty(C, complex)
    for g in range(C):
        if 2 * g < C:
            row0[g] = acc[2 * g]
        elif 2 * g == C:
            row0[g] = accn
        else:
            row0[g] = np.conj(acc[2 * (C - g)])
        rowh[g] = acc[2 * g + 1] if 2 * g + 1 < C else np.conj(acc[2 * (C - 1 - g) + 1])
    XA, XB = np.fft.fft(xa), np.fft.fft(xb)
    ref0 = (XA * XB)[R * np.arange(C)]
    refh = (XA * XB)[R // 2 + R * np.arange(C)]
    scale = np.abs(XA * XB).max()
    assert np.abs(0.25 * row0 - ref0).max() <= 1e-9 * scale
    assert np.abs(0.25 * rowh - refh).max() <= 1e-9 * scale


def _swizzle(i):
    return i ^ ((i >> 4) & 15)


@pytest.mark.parametrize("R,C", CASES)
def test_pair_fold_slot_from_entry(R, C):
    """The fold entry of bucket u holds 8 * swizzle(u mod C) in bits 0..15
    and 8 * (u div (C/16)) in bits 16..31.  The pair fold's slot
    (u mod 2C) div 2 and half (u mod 2C) mod 2 follow from u mod C and bit 4
    of the weight index, the parity of u div C."""
    log2c = int(np.log2(C))
    u = np.arange(R * C, dtype=np.int64)
    entry = ((u >> (log2c - 4)) << 19) | (_swizzle(u & (C - 1)) << 3)
    rc = _swizzle((entry & 0xFFFF) >> 3)
    assert np.array_equal(rc, u % C)
    qpar = (entry >> 23) & 1
    assert np.array_equal(qpar, (u // C) & 1)
    slot = (rc >> 1) + (C // 2) * qpar
    assert np.array_equal(slot, (u % (2 * C)) >> 1)
    assert np.array_equal(rc & 1, (u % (2 * C)) & 1)
    # the swizzle is an involution, so positions and slots map both ways
    assert np.array_equal(_swizzle(_swizzle(u)), u)
