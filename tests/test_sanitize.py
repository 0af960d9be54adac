"""The seeded generators and the oracle under AddressSanitizer and
UndefinedBehaviorSanitizer (host code only): tests/sanitize_driver.c runs
every generator family and every oracle entry point once on a small graph;
any memory error, leak or undefined behaviour fails the run."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_and_generators_sanitized(tmp_path):
    exe = str(tmp_path / "sanitize_driver")
    src = [os.path.join(ROOT, p) for p in ("tests/sanitize_driver.c", "oracle/oracle.c", "oracle/prune.c",
                                           "gsp_inputs/gen.c")]
    cmd = ["gcc", "-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=all", "-ffp-contract=off", "-Wall", "-Wno-unknown-pragmas", "-Werror",
           "-o", exe] + src + ["-lm"]
    b = subprocess.run(cmd, capture_output=True, text=True)
    assert b.returncode == 0, b.stderr[-4000:]
    env = dict(os.environ, ASAN_OPTIONS="halt_on_error=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.stdout[-2000:], r.stderr[-4000:])
    lines = r.stdout.splitlines()
    assert [x.split(":")[0] for x in lines] == ["sbm", "rmat", "dcsbm", "road"], r.stdout
