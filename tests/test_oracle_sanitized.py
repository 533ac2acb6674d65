"""The oracle built with the address and undefined-behaviour sanitizers
(g++, host only) runs every grid entry point on small curved, periodic, copy,
1D/2D/3D grids, with the conductivity models and the atmosphere, without a
report and without a failed recovery."""
import os
import subprocess


def test_oracle_under_sanitizers(orc, tmp_path):
    exe = orc.build_sanitized(str(tmp_path))
    env = dict(os.environ, OMP_NUM_THREADS="2", ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=600, env=env)
    print(r.stdout)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.count("failed 0,") == 5
