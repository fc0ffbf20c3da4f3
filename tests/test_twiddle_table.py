"""The FFT kernels' compile-time twiddle tables (paper_1805_02247_amd/csrc/twiddle.h), built
with the host compiler and compared with exp(-2 pi i j / n) in FP64 (numpy): every entry is
the float nearest the exact value, up to 1 ulp (and to 1e-15 absolute next to the zeros)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

CSRC = os.path.join(os.path.dirname(__file__), "..", "paper_1805_02247_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs a host C++ compiler")
def test_twiddle_tables_match_fp64(tmp_path):
    src = tmp_path / "tw.cpp"
    sizes = [16, 32, 64, 128, 256, 512]
    body = "\n".join(
        f"  {{ constexpr auto t = pmr::make_tw_table<{n}>(); for (int j = 0; j < {n}; ++j) "
        f"printf(\"{n} %d %.9e %.9e\\n\", j, t.v[j].re, t.v[j].im); }}" for n in sizes)
    src.write_text('#include <cstdio>\n#include "twiddle.h"\nint main() {\n' + body + "\n}\n")
    exe = tmp_path / "tw"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    rows = np.loadtxt(subprocess.run([str(exe)], capture_output=True, text=True, check=True)
                      .stdout.splitlines())
    for n in sizes:
        r = rows[rows[:, 0] == n]
        j = r[:, 1].astype(np.int64)
        ref = np.exp(-2j * np.pi * j / n)
        got = (r[:, 2] + 1j * r[:, 3])
        ulp = np.spacing(np.abs(ref.real).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got.real - ref.real) <= np.maximum(ulp, 1e-15)), n
        ulp = np.spacing(np.abs(ref.imag).astype(np.float32)).astype(np.float64)
        assert np.all(np.abs(got.imag - ref.imag) <= np.maximum(ulp, 1e-15)), n
