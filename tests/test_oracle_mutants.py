"""Planted mistakes in copies of the oracle must each fail at least one pin.

Every mutant is a plausible slip (a dropped term, a transposed or wrong matrix
entry, a flipped sign or axis, a closed edge, a wrong shift, constant or
comparison, a broken tie-break or shuffle, fused multiply-add).  The mutants are
built from a copy of oracle/pcr_oracle.c in a temporary directory; the oracle
itself is not touched.
"""
import os
import subprocess
import tempfile

import pytest

import oracle
import pins

SRC = os.path.join(os.path.dirname(oracle.__file__), "pcr_oracle.c")

# (name, [(old, new), ...], extra compiler flags)
MUTANTS = [
    ("dropped z term in x", [("m[1] * y) + m[2] * z) + m[3]", "m[1] * y)) + m[3]")], []),
    ("depth from clip z row", [("((m[12] * x + m[13] * y) + m[14] * z) + m[15]",
                                "((m[8] * x + m[9] * y) + m[10] * z) + m[11]")], []),
    ("transposed matrix (x row)", [("((m[0] * x + m[1] * y) + m[2] * z) + m[3]",
                                    "((m[0] * x + m[4] * y) + m[8] * z) + m[12]")], []),
    ("sign of ndc x", [("(cx * rw + 1.0f) * hw", "(1.0f - cx * rw) * hw")], []),
    ("y axis flipped", [("*pid_out = py * W + px", "*pid_out = (H - 1 - py) * W + px")], []),
    ("row stride H", [("*pid_out = py * W + px", "*pid_out = py * H + px")], []),
    ("closed right edge", [("fx < (float)W", "fx <= (float)W")], []),
    ("approximate reciprocal", [("float rw = 1.0f / cw;",
                                 "float rw = _mm_cvtss_f32(_mm_rcp_ss(_mm_set_ss(cw)));")], []),
    ("fused multiply-add", [], ["-ffp-contract=fast", "-mfma"]),
    ("depth shifted by 24", [("((uint64_t)dbits << 32) | (uint64_t)pts[i].rgba",
                              "((uint64_t)dbits << 24) | (uint64_t)pts[i].rgba")], []),
    ("max instead of min", [("if (key < fb[pid])", "if (key > fb[pid] || fb[pid] == 0xFFFFFFFFFFFFFFFFull)")], []),
    ("resolve shows depth", [("(uint32_t)fb[p];", "(uint32_t)(fb[p] >> 32);")], []),
    ("epsilon 10%", [("* 1.01f", "* 1.1f")], []),
    ("strict threshold", [("if (!(u2f(dbits) <= u2f(D[pid]) * 1.01f))", "if (!(u2f(dbits) < u2f(D[pid]) * 1.01f))")],
     []),
    ("red and green swapped", [("RG[p] += (sum[p] << 32) + sum[npix + p];", "RG[p] += (sum[npix + p] << 32) + sum[p];")],
     []),
    ("count of two", [("sum[3 * npix + pid] += 1;", "sum[3 * npix + pid] += 2;")], []),
    ("green from the red half", [("RG[p] & 0xFFFFFFFFull, BA[p] >> 32", "RG[p] >> 32, BA[p] >> 32")], []),
    ("hq alpha 0", [("uint32_t colour = 0xFF000000u;", "uint32_t colour = 0u;")], []),
    ("blue from the green byte", [("sum[c * npix + pid] += (pts[i].rgba >> (8 * c)) & 0xFFu;",
                                   "sum[c * npix + pid] += (pts[i].rgba >> (8 * (c ? 1 : 0))) & 0xFFu;")], []),
    ("morton y/z swapped", [("<< (3 * i + 1);", "<< (3 * i + 9999);"), ("<< (3 * i + 2);", "<< (3 * i + 1);"),
                            ("<< (3 * i + 9999);", "<< (3 * i + 2);")], []),
    ("morton 2^21 - 1 scale", [("* 2097152.0f", "* 2097151.0f")], []),
    ("non-cubic box", [("quantize21(pts[i].y, lo[1], size)", "quantize21(pts[i].y, lo[1], sy)")], []),
    ("unstable ties", [("return x->idx < y->idx ? -1 : 1;", "return x->idx < y->idx ? 1 : -1;")], []),
    ("splitmix counter from 0", [("seed + (k + 1) * 0x9E3779B97F4A7C15ull", "seed + k * 0x9E3779B97F4A7C15ull")], []),
    ("batches not moved", [("uint64_t s = b * batch,", "uint64_t s = r * batch,")], []),
    ("last partial batch dropped", [("uint64_t nb = (n + batch - 1) / batch;", "uint64_t nb = n / batch;")], []),
    ("depth without reciprocal", [("float rw = 1.0f / w;", "float rw = w;")], []),
    ("depth offset subtracted", [("return a + t;", "return a - t;")], []),
    ("depth coefficients swapped", [("float t = b * rw;", "float t = a * rw;"), ("return a + t;", "return b + t;")],
     []),
    ("linear depth from the colour word", [("depth_value(u2f((uint32_t)(fb[p] >> 32))", "depth_value(u2f((uint32_t)fb[p])")],
     []),
    ("uncovered depth 0", [("out[p] = empty;", "out[p] = 0.0f;")], []),
    ("hq depth empty test on 0", [("D[p] == 0xFFFFFFFFu ? empty", "D[p] == 0u ? empty")], []),
    ("packed green field at 27", [("(r << 46) | (g << 28) | (b << 10) | 1u", "(r << 46) | (g << 27) | (b << 10) | 1u")],
     []),
    ("packed count of 9 bits", [("uint64_t a = P[p] & 0x3FFull;", "uint64_t a = P[p] & 0x1FFull;")], []),
    ("packed red and blue swapped", [("(r << 46) | (g << 28) | (b << 10) | 1u", "(b << 46) | (g << 28) | (r << 10) | 1u")],
     []),
    ("packed red field of 17 bits", [("((P[p] >> 46) & 0x3FFFFull)", "((P[p] >> 46) & 0x1FFFFull)")], []),
    ("packed threshold strict", [("        if (depth <= limit) {\n            uint64_t r = pts[i].rgba & 0xFFu;\n            uint64_t g = (pts[i].rgba >> 8) & 0xFFu;\n            uint64_t b = (pts[i].rgba >> 16) & 0xFFu;\n            P[pid]",
                                  "        if (depth < limit) {\n            uint64_t r = pts[i].rgba & 0xFFu;\n            uint64_t g = (pts[i].rgba >> 8) & 0xFFu;\n            uint64_t b = (pts[i].rgba >> 16) & 0xFFu;\n            P[pid]")], []),
]


def _build(tmp, name, subs, flags):
    with open(SRC) as f:
        text = f.read()
    for old, new in subs:
        assert old in text, f"mutation anchor not found for {name!r}: {old!r}"
        text = text.replace(old, new)
    src = os.path.join(tmp, "m.c")
    with open(src, "w") as f:
        f.write(text)
    out = os.path.join(tmp, "libm.so")
    cflags = [c for c in oracle.CFLAGS if not (flags and c == "-ffp-contract=off")]
    subprocess.run(["gcc", *cflags, *flags, "-o", out, src], check=True)
    return out


@pytest.mark.parametrize("name,subs,flags", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_mutant_is_caught(name, subs, flags):
    with tempfile.TemporaryDirectory() as tmp:
        orc = oracle.Oracle(oracle.load(_build(tmp, name, subs, flags)))
        failed = []
        for check in pins.ALL_CHECKS:
            try:
                check(orc)
            except (AssertionError, ValueError, IndexError, OverflowError):
                failed.append(check.__name__)
        assert failed, f"no pin catches the mutant {name!r}"
