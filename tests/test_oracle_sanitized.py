"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer.

The oracle is rebuilt with -fsanitize=address,undefined (any finding
aborts) into a temporary directory and the CPU pin suite of the oracle runs
against that build in a child process (the sanitizer runtime preloaded), so
that an out-of-bounds access, an overflow of a signed index or a misaligned
load anywhere in the oracle fails the suite instead of passing silently."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


@pytest.mark.skipif(_runtime("libasan.so") is None, reason="no AddressSanitizer runtime")
def test_oracle_pins_under_asan_ubsan(tmp_path):
    lib = str(tmp_path / "liboracle_asan.so")
    oracle.build(out=lib, extra_flags=["-fsanitize=address,undefined",
                                       "-fno-sanitize-recover=all",
                                       "-fno-omit-frame-pointer"])
    env = dict(os.environ)
    env["TRIMAP_ORACLE_LIB"] = lib
    env["LD_PRELOAD"] = " ".join(x for x in (_runtime("libasan.so"), _runtime("libubsan.so"))
                                 if x)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "print_stacktrace=1:halt_on_error=1"
    tests = sorted(os.path.join(ROOT, "tests", f) for f in os.listdir(os.path.join(ROOT, "tests"))
                   if f.startswith("test_oracle_") and f != os.path.basename(__file__))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "-m", "not gpu and not slow", *tests],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "AddressSanitizer" not in tail and "runtime error" not in tail, tail
    assert " passed" in r.stdout, tail
