"""The CPU oracles under AddressSanitizer and UndefinedBehaviorSanitizer.

tests/oracle_sanitize_main.c drives the LB oracle and the finite-difference
oracle through every lattice, wall kind, anisotropy and option on small,
ragged and degenerate domains (a single node, a 2 x 3 x 1 box, one-node
slabs).  Built with gcc and both sanitizers (host code only), the run must
end cleanly: no out-of-bounds access, no use after free, no leak, no
undefined arithmetic, no non-finite field.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")


def test_oracles_run_clean_under_sanitizers(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           "-I", ORACLE, "-I", HERE,
           "-o", exe, os.path.join(HERE, "oracle_sanitize_main.c"),
           os.path.join(ORACLE, "lbpf_oracle.c"), "-lm"]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "all cases clean" in r.stdout
