"""The CPU oracle built with the address and undefined-behaviour sanitizers
runs every entry point on small fields and on corrupted streams (bit flips,
truncations, hostile stored floats) without a report."""
import os
import shutil
import subprocess
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")


def _have_sanitizers(tmp):
    src = os.path.join(tmp, "probe.c")
    open(src, "w").write("int main(void){return 0;}\n")
    r = subprocess.run(["gcc", "-fsanitize=address,undefined,float-cast-overflow", src, "-o", os.path.join(tmp, "probe")],
                       capture_output=True)
    return r.returncode == 0


def test_oracle_under_sanitizers():
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    with tempfile.TemporaryDirectory() as tmp:
        if not _have_sanitizers(tmp):
            pytest.skip("gcc has no sanitizer runtime here")
        exe = os.path.join(tmp, "san_check")
        cmd = ["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
               "-fsanitize=address,undefined,float-cast-overflow", "-fno-sanitize-recover=all",
               "-I" + ORACLE, os.path.join(ORACLE, "cpo.c"), os.path.join(ORACLE, "san_check.c"),
               "-o", exe, "-lm"]
        subprocess.check_call(cmd)
        env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        env.pop("LD_PRELOAD", None)
        r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=600)
        assert r.returncode == 0, r.stderr[-4000:]
        assert "san_check ok" in r.stdout
