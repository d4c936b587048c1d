"""CPU check of the in-register radix-16 transforms of the spectral kernel
(paper_1108_1320_amd/csrc/cmm_dft.h, built for the host with hipcc): the
plain 16-point DFT, the form with its inputs multiplied by 15 twiddles
folded into the butterflies, and the form with one common input factor,
each against numpy's FFT of the same float32 inputs in float64.  The
float32 error budget of a 16-point transform of unit-size inputs is a few
1e-6; a dropped or misplaced twiddle gives errors of order 1."""
import os
import shutil
import subprocess

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"


@pytest.fixture(scope="module")
def dft_exe(tmp_path_factory):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    exe = str(tmp_path_factory.mktemp("dft") / "dft_check")
    src = os.path.join(ROOT, "tests", "host", "dft_check.cpp")
    inc = os.path.join(ROOT, "paper_1108_1320_amd", "csrc")
    r = subprocess.run([HIPCC, "-O2", "-x", "hip", "--offload-arch=gfx950", "-I", inc, src, "-o", exe],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stderr[-2000:]
    return exe


def test_radix16_forms_against_numpy(dft_exe):
    g = np.random.default_rng(2024)
    n = 3000
    x = (g.uniform(-1, 1, (n, 16)) + 1j * g.uniform(-1, 1, (n, 16))).astype(np.complex64)
    ang = g.uniform(0, 2 * np.pi, (n, 15))
    u = np.exp(1j * ang).astype(np.complex64)
    s = (0.5 * np.exp(1j * g.uniform(0, 2 * np.pi, n))).astype(np.complex64)
    case = np.concatenate([x.view(np.float32).reshape(n, 32), u.view(np.float32).reshape(n, 30),
                           s.view(np.float32).reshape(n, 2)], axis=1).astype(np.float32)
    r = subprocess.run([dft_exe], input=np.int32(n).tobytes() + case.tobytes(), capture_output=True, timeout=60)
    assert r.returncode == 0
    out = np.frombuffer(r.stdout, np.float32).reshape(n, 3, 32).view(np.complex64).reshape(n, 3, 16)
    x64 = x.astype(np.complex128)
    ref_plain = np.fft.fft(x64, axis=1)
    tw = np.concatenate([np.ones((n, 1)), u.astype(np.complex128)], axis=1)
    ref_tw = np.fft.fft(x64 * tw, axis=1)
    ref_sc = np.fft.fft(x64 * s.astype(np.complex128)[:, None], axis=1)
    for got, ref in ((out[:, 0], ref_plain), (out[:, 1], ref_tw), (out[:, 2], ref_sc)):
        err = np.abs(got.astype(np.complex128) - ref).max()
        assert err < 1e-5, err
