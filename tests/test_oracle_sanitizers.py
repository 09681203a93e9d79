"""The CPU oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a copy of the oracle built with both sanitizers runs every oracle
pin in a child process (the ASan runtime preloaded), which must finish cleanly
with no sanitizer report."""
import os
import subprocess
import sys
import tempfile

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
sys.path.insert(0, {tests!r})
import oracle, pins
orc = oracle.Oracle(oracle.load({lib!r}))
for check in pins.ALL_CHECKS:
    check(orc)
print("pins ok", len(pins.ALL_CHECKS))
"""


def test_oracle_pins_under_asan_and_ubsan():
    with tempfile.TemporaryDirectory() as tmp:
        lib = os.path.join(tmp, "liboracle_san.so")
        flags = [f for f in oracle.CFLAGS if f != "-O2"] + [
            "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
        subprocess.run(["gcc", *flags, "-o", lib, oracle._SRC], check=True)
        asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
        env = dict(os.environ, LD_PRELOAD=asan, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
                   UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
        code = CHILD.format(root=ROOT, tests=os.path.join(ROOT, "tests"), lib=lib)
        r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True, timeout=900)
        assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
        assert "pins ok" in r.stdout
        assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
