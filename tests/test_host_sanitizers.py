"""The host FP64 wavelet design of the library (the C++ behind
os3d_wavelet_coeffs and os3d_steering_matrix, and the plans and layouts the
device kernels rely on) built with g++ under AddressSanitizer and
UndefinedBehaviorSanitizer, driven over a grid of window parameters up to the
largest L, and its coefficients compared with the oracle's (Sec. 3.2,
Eqs. 12-16).  CPU only; skipped where g++ or the sanitizer runtimes are
missing."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1505_07690_amd", "csrc")


@pytest.fixture(scope="module")
def driver_output(tmp_path_factory):
    gxx = shutil.which("g++")
    if gxx is None:
        pytest.skip("g++ not available")
    exe = str(tmp_path_factory.mktemp("host") / "design_driver")
    cmd = [gxx, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-I", CSRC, os.path.join(CSRC, "host_setup.cpp"),
           os.path.join(ROOT, "tests", "host", "design_driver.cpp"), "-o", exe]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        if "asan" in r.stderr.lower() or "ubsan" in r.stderr.lower():
            pytest.skip("sanitizer runtimes not available")
        raise AssertionError(r.stderr)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    run = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert run.returncode == 0, run.stdout[-2000:] + run.stderr[-4000:]
    assert "ERROR: AddressSanitizer" not in run.stderr and "runtime error" not in run.stderr, run.stderr[-4000:]
    return run.stdout


def test_host_design_runs_clean_under_sanitizers(driver_output):
    last = driver_output.strip().splitlines()[-1].split()
    assert last[0] == "plans" and last[3] == "0", last  # no failed plan, pairing or layout check
    assert int(last[1]) > 100


def test_sanitized_coefficients_match_oracle(driver_output):
    rows = [ln.split() for ln in driver_output.splitlines() if ln.startswith("coef ")]
    assert len(rows) == 9 * 3 * 3 * 2 * 2
    worst = 0.0
    for r in rows:
        L, s, k, coeffs, variant = int(r[1]), float(r[2]), int(r[3]), int(r[4]), int(r[5])
        a_lib = np.array([float(x) for x in r[6:]])
        p = O.WaveletParams(L=L, s_theta=s, k=k, coeffs=("lsq", "quadrature")[coeffs],
                            variant=("cake", "plate")[variant])
        c = O.sh_coeffs_A(p) if coeffs == 0 else O.sh_coeffs_A_quadrature(p)
        a_or = O.cake_coeffs(c, p.variant)
        worst = max(worst, np.max(np.abs(a_lib - a_or)) / max(1.0, np.max(np.abs(a_or))))
    assert worst < 1e-10, worst
