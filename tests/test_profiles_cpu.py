"""The committed rocprofv3 summaries: each gives the commands that produced
it, and those commands run only committed files (bench.py legs that exist)."""
import glob
import os
import re

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _legs():
    src = open(os.path.join(ROOT, "bench.py")).read()
    m = re.search(r'"--leg", default="main", choices=\[([^\]]*)\]', src, re.S)
    return set(re.findall(r'"(\w+)"', m.group(1)))


def test_every_profile_names_runnable_commands():
    legs = _legs()
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md")))
    assert files, "no profile summaries committed"
    for f in files:
        text = open(f).read()
        blocks = re.findall(r"```\n(.*?)```", text, re.S)
        assert blocks, f"{f}: no command block"
        cmds = [c for b in blocks for c in b.strip().splitlines()]
        assert cmds, f
        for c in cmds:
            assert c.startswith("rocprofv3 "), (f, c)
            prog = c.split(" -- ", 1)[1]
            assert prog.startswith("python3 bench.py"), (f, c)     # run from the repository root
            leg = re.search(r"--leg (\w+)", prog)
            assert leg is None or leg.group(1) in legs, (f, c)
            assert "_work" not in c, (f, c)
        assert "| kernel |" in text, f"{f}: no kernel table"


def test_measured_traffic_matches_the_render_sources():
    """The bench line's measured traffic (FETCH_SIZE / WRITE_SIZE of the
    profiled kernels) was taken from the current render sources; the bench
    reports null traffic otherwise."""
    import bench
    sha = bench.render_sources_sha()
    assert bench.MEASURED_TRAFFIC, "no measured traffic"
    for key, rec in bench.MEASURED_TRAFFIC.items():
        assert rec["src"] == sha, key
        assert bench.traffic_for(*key) == rec["fetch_bytes"] + rec["write_bytes"]
