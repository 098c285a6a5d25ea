"""Register-FFT templates of the HIP kernels, compiled for the host and checked
against a direct DFT in long double (all radix-2/3/4 sizes used by the library)."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))


def test_register_fft_templates_on_host(tmp_path):
    cxx = shutil.which("g++") or shutil.which("c++")
    if cxx is None:
        pytest.skip("no host C++ compiler")
    exe = tmp_path / "fft_host_test"
    src = os.path.join(HERE, "native", "fft_host_test.cpp")
    r = subprocess.run([cxx, "-std=c++17", "-O2", "-o", str(exe), src], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    print(r.stdout)
    assert r.returncode == 0, r.stdout
    assert "FAIL" not in r.stdout
