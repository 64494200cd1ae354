"""Host sanitizers over the oracle and the input generators.

``sanitize_main.c`` drives every routine of ``oracle/oracle.c`` and of
``graphgen/graphgen.c`` on small graphs (degenerate, random, core+tail, R-MAT
with a chain, implicit, a packed batch).  It is built here with
AddressSanitizer and UndefinedBehaviorSanitizer, every report fatal, and must
exit cleanly with all of its cross-checks passed.  Host code only (gcc); the
GPU library is not involved.
"""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_and_generators_under_asan_ubsan(tmp_path):
    exe = tmp_path / "sanitize_main"
    cmd = ["gcc", "-g", "-O1", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
           os.path.join(HERE, "sanitize_main.c"), os.path.join(ROOT, "oracle", "oracle.c"),
           os.path.join(ROOT, "graphgen", "graphgen.c"), "-lm", "-o", str(exe)]
    subprocess.check_call(cmd)
    env = dict(os.environ)
    env["ASAN_OPTIONS"] = "detect_leaks=1:abort_on_error=0:verify_asan_link_order=0"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=600, env=env)
    assert r.returncode == 0, r.stdout[-4000:] + r.stderr[-4000:]
    assert "all checks passed" in r.stdout
