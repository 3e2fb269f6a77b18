"""The register-resident line FFT (csrc/fft_reg.hpp), compiled for the host
from the same template the kernels use: every radix path (2, 3, 4, 5 and
their mixtures) against the O(N^2) DFT in long double.  Bounds: FP64 1e-14,
FP32 1e-6 relative (one rounding per butterfly level, log N levels)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_register_fft_matches_dft(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = str(tmp_path / "fft_reg_check")
    r = subprocess.run([hipcc, "-x", "hip", "--offload-arch=gfx950", "-O1", "-std=c++17",
                        os.path.join(HERE, "native", "fft_reg_check.cpp"), "-o", exe],
                       capture_output=True, text=True, timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120).stdout
    lines = [l.split() for l in out.strip().splitlines()]
    assert len(lines) == 8
    for n, d1, d2, f1, f2 in lines:
        assert float(d1) < 1e-14 and float(d2) < 1e-14, n
        assert float(f1) < 1e-6 and float(f2) < 1e-6, n
