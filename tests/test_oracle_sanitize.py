"""The oracle's C sources built with AddressSanitizer and UndefinedBehaviorSanitizer
(host code only) and driven through every entry point by tests/oracle_sanitize_main.c:
an out-of-bounds access, a leak, a use after free or undefined arithmetic in the
oracle ends the run with an error."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not available")
def test_oracle_under_sanitizers(tmp_path):
    exe = str(tmp_path / "oracle_sanitize")
    srcs = [os.path.join(HERE, "oracle_sanitize_main.c"), os.path.join(ROOT, "oracle", "pirrt_oracle.c"),
            os.path.join(ROOT, "oracle", "rrg_oracle.c")]
    flags = ["-std=c11", "-O1", "-g", "-fno-omit-frame-pointer", "-ffp-contract=off", "-msse2", "-mfpmath=sse",
             "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
    r = subprocess.run(["gcc"] + flags + srcs + ["-o", exe, "-lm"], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:exitcode=3:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr, r.stderr[-4000:]
    assert "oracle sanitizer run ok" in r.stdout
