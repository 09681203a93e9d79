"""The CPU oracle under gcc's AddressSanitizer and UndefinedBehaviorSanitizer:
tests/oracle_sanitize_main.c drives every oracle entry point over ordinary,
empty, one-pixel and hostile inputs and the three vertex orders over empty,
single, degenerate and ragged clouds; any out-of-bounds access, leak, use
after free, signed overflow, bad shift or out-of-range float conversion ends
the run with a report.  A second run over a copy of the oracle with a planted
off-by-one write shows that the check has teeth."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HARNESS = os.path.join(ROOT, "tests", "oracle_sanitize_main.c")
ORACLE = os.path.join(ROOT, "oracle", "pcr_oracle.c")
# the oracle's own floating-point flags, plus the sanitizers
FLAGS = ["-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-msse2", "-mfpmath=sse",
         "-fexcess-precision=standard", "-fsanitize=address,undefined,float-cast-overflow",
         "-fno-sanitize-recover=all", "-fno-omit-frame-pointer"]


def build(tmp_path, oracle_src):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = str(tmp_path / "oracle_sanitize")
    r = subprocess.run(["gcc", *FLAGS, "-o", exe, HARNESS, oracle_src, "-lm"], capture_output=True, text=True)
    if r.returncode != 0 and "sanitize" in r.stderr:
        pytest.skip("sanitizer runtime not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr
    return exe


def run(exe):
    return subprocess.run([exe], capture_output=True, text=True, timeout=120)


def test_oracle_is_clean_under_sanitizers(tmp_path):
    r = run(build(tmp_path, ORACLE))
    assert r.returncode == 0, r.stderr[-4000:]
    assert "ok" in r.stdout


def test_sanitizer_run_catches_a_planted_overflow(tmp_path):
    src = open(ORACLE).read()
    old = ("void oracle_resolve_basic(const uint64_t *fb, uint32_t W, uint32_t H, uint32_t *out)\n{\n"
           "    for (uint64_t p = 0; p < (uint64_t)W * H; ++p)")
    assert src.count(old) == 1
    mutant = tmp_path / "oracle_mutant.c"
    mutant.write_text(src.replace(old, old.replace("p < (uint64_t)W * H", "p <= (uint64_t)W * H")))
    r = run(build(tmp_path, str(mutant)))
    assert r.returncode != 0
    assert "AddressSanitizer" in r.stderr
