"""GPU tests of the measurement helpers: the visible-point count against the
oracle's projection, the atomic probe's final buffer against the same
atomics replayed on the host from the probe's documented address and value
rule, and the read probe (reads only, any record count)."""
import numpy as np
import pytest

from gpu_util import upload
from paper_2104_07526_amd import pcr, synth

pytestmark = pytest.mark.gpu

M32 = np.uint64(0xFFFFFFFF)


@pytest.mark.parametrize("case", ["sphere_720p", "terrain_oblique", "terrain_closeup", "empty"])
def test_count_visible_matches_the_oracle(orc, case):
    if case == "sphere_720p":
        pts, (m, W, H) = synth.sphere(300_000, seed=3), (synth.sphere_view(1280, 720), 1280, 720)
    elif case == "empty":
        pts, (m, W, H) = synth.sphere(0, seed=3), (synth.sphere_view(64, 48), 64, 48)
    else:
        pts = synth.terrain(400_003, seed=7)
        W, H = 1920, 1080
        m = getattr(synth, case)(W, H)
    pid, _ = orc.project_all(pts, m, W, H)
    want = int(np.count_nonzero(pid != 0xFFFFFFFF))
    got = pcr.count_visible(upload(pts), m, W, H)
    print(case, len(pts), want, flush=True)
    assert got == want


def mix32(x):
    x = x & M32
    x ^= x >> np.uint64(16)
    x = (x * np.uint64(0x7FEB352D)) & M32
    x ^= x >> np.uint64(15)
    x = (x * np.uint64(0x846CA68B)) & M32
    x ^= x >> np.uint64(16)
    return x


def expected_probe(words, pattern, workgroups, iters, seed):
    """Final buffer of the probe from all-ones, the atomics replayed on the
    host: lane gid's iteration `it` takes min(buf[idx], hl << 32 | gid)."""
    gid = np.arange(workgroups * 256, dtype=np.uint64)
    wave, lane = gid >> np.uint64(6), gid & np.uint64(63)
    buf = np.full(words, np.iinfo(np.uint64).max, np.uint64)
    W = np.uint64(words)
    for it in range(iters):
        it = np.uint64(it)
        hl = mix32(gid * np.uint64(0x9E3779B9) + it * np.uint64(0x85EBCA6B) + np.uint64(seed))
        hw = mix32(wave * np.uint64(0xC2B2AE35) + it * np.uint64(0x27D4EB2F) + np.uint64(seed))
        if pattern == pcr.PROBE_RANDOM:
            idx = (hl * W) >> np.uint64(32)
        elif pattern == pcr.PROBE_LINE:
            hg = mix32(hw ^ (((lane >> np.uint64(3)) * np.uint64(0x165667B1)) & M32))
            idx = ((hg * (W >> np.uint64(3))) >> np.uint64(32)) * np.uint64(8) + (lane & np.uint64(7))
        elif pattern == pcr.PROBE_ADDRESS:
            idx = (hw * W) >> np.uint64(32)
        else:
            idx = ((hw * (W >> np.uint64(6))) >> np.uint64(32)) * np.uint64(64) + lane
        np.minimum.at(buf, idx.astype(np.int64), (hl << np.uint64(32)) | gid)
    return buf


@pytest.mark.parametrize("pattern", [pcr.PROBE_RANDOM, pcr.PROBE_LINE, pcr.PROBE_ADDRESS, pcr.PROBE_CONTIGUOUS])
@pytest.mark.parametrize("returning", [False, True])
def test_probe_atomics_final_buffer(pattern, returning):
    import torch
    words, workgroups, iters, seed = 4096, 3, 5, 11
    buf = torch.full((words,), -1, dtype=torch.int64, device="cuda")
    sink = torch.zeros(1, dtype=torch.int64, device="cuda")
    ops = pcr.probe_atomics(buf, pattern, returning, workgroups=workgroups, iters=iters, seed=seed, sink=sink)
    assert ops == workgroups * 256 * iters
    got = buf.cpu().numpy().view(np.uint64)
    want = expected_probe(words, pattern, workgroups, iters, seed)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("n16", [1, 255, 1024, 1025, 300_001])
@pytest.mark.parametrize("per_thread", [4, 8])
def test_probe_read_only_reads(n16, per_thread):
    import torch
    buf = torch.zeros(4 * n16 + 3, dtype=torch.int32, device="cuda")   # a partial record at the end
    buf[: 4 * n16] = torch.arange(4 * n16, dtype=torch.int32, device="cuda")
    keep = buf.clone()
    sink = torch.full((1,), 7, dtype=torch.int32, device="cuda")
    nbytes = pcr.probe_read(buf, per_thread=per_thread, workgroups=37, sink=sink)
    torch.cuda.synchronize()
    assert nbytes == 16 * n16
    assert torch.equal(buf, keep)
    # record i holds 4i .. 4i+3, whose XOR is 0: every lane's fold is 0, never
    # the fixed value at which the probe stores it
    assert int(sink.item()) == 7


def test_probe_read_refuses_bad_arguments():
    import torch
    buf = torch.zeros(64, dtype=torch.int32, device="cuda")
    sink = torch.zeros(1, dtype=torch.int32, device="cuda")
    with pytest.raises(pcr.PcrError):
        pcr.probe_read(buf, per_thread=5, sink=sink)
    with pytest.raises(pcr.PcrError):
        pcr.probe_read(buf, workgroups=0, sink=sink)
