"""The host-only reference-element code built with AddressSanitizer and
UndefinedBehaviorSanitizer (host pass only) and run on the CPU: no memory
or undefined-behaviour error, and the tables' invariants."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_reference_tables_under_host_sanitizers(tmp_path):
    exe = str(tmp_path / "ref_asan")
    csrc = os.path.join(ROOT, "paper_1906_11082_amd", "csrc")
    # the sanitizers apply to the host pass only; nothing here runs on a GPU
    cmd = [HIPCC, "-std=c++17", "-O1", "-g", "-fno-omit-frame-pointer", "-Xarch_host", "-fsanitize=address",
           "-Xarch_host", "-fsanitize=undefined", "-I", os.path.join(ROOT, "include"), "-I", csrc,
           os.path.join(csrc, "nm_ref.cpp"), os.path.join(HERE, "host_ref_driver.cpp"), "-o", exe]
    subprocess.run(cmd, check=True, capture_output=True, timeout=600)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="halt_on_error=1")
    out = subprocess.run([exe], capture_output=True, text=True, timeout=120, env=env)
    assert out.returncode == 0, out.stderr[-2000:]
    assert "ERROR" not in out.stderr and "runtime error" not in out.stderr, out.stderr[-2000:]
    lines = out.stdout.strip().splitlines()
    assert len(lines) == 5
    for ln in lines[:4]:
        f = ln.split()
        # the mass matrices integrate 1 over the reference tetrahedron {r_i >= -1, sum r_i <= -1}: volume 8/6
        assert abs(float(f[f.index("sum") + 1]) - 8.0 / 6.0) < 1e-12
        lo, hi = float(f[-4]), float(f[-3])
        du = int(f[1])
        want = (0.5, 2.5) if du == 1 else (0.25, 4.3475)
        assert abs(lo - want[0]) < 1e-4 and abs(hi - want[1]) < 1e-4, ln
    assert lines[4].split()[1:] == ["1", "3"]
