"""Host AddressSanitizer and UndefinedBehaviorSanitizer over the C++ oracle
(``oracle/katz_ref.cpp``) and the graph generators (``synthgraph/gen.cpp``):
a small driver (``tests/sanitize/driver.cpp``) runs every generator and every
oracle entry point on small graphs, with one and with three OpenMP threads,
built with g++ -fsanitize=address,undefined; any finding aborts the run."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_oracle_and_generators_are_sanitizer_clean():
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "driver")
        cmd = ["g++", "-O1", "-g", "-std=c++17", "-fopenmp", "-ffp-contract=off",
               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
               os.path.join(ROOT, "tests", "sanitize", "driver.cpp"), os.path.join(ROOT, "oracle", "katz_ref.cpp"),
               os.path.join(ROOT, "synthgraph", "gen.cpp"), "-o", exe]
        subprocess.run(cmd, check=True, capture_output=True, text=True)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1:verify_asan_link_order=0",
                   UBSAN_OPTIONS="print_stacktrace=1")
        out = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert out.returncode == 0, out.stdout + out.stderr
        assert "all ok" in out.stdout
