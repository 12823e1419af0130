"""Host-side parts of the benchmark's contract (CPU): the multi-GPU refusal
and the HBM-traffic figure taken from the committed counter summary."""
import json
import os
import re
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _profile_blob():
    text = open(bench.PROFILE).read()
    return json.loads(re.search(r"```json\n(.*?)\n```", text, re.S).group(1))


def test_traffic_comes_from_the_counter_summary():
    """Scaled FETCH_SIZE + WRITE_SIZE per dispatch over the launch time, for
    the lattice the summary covers; the summary's sources still hash to what
    was profiled (otherwise the figure would be dropped)."""
    blob = _profile_blob()
    nodes = blob["nodes"]
    ms = 0.25
    for st in ("f32", "f16", "bf16"):
        pd = blob["per_dispatch"][st]
        gbs, byts = bench.measured_traffic(st, ms, nodes)
        assert gbs is not None, f"{st}: profiled sources changed since the counter runs"
        want = (pd["fetch_kib"] * blob["fetch_scale"] + pd["write_kib"] * blob["write_scale"]) * 1024
        assert byts == pytest.approx(want, rel=1e-12)
        assert gbs == pytest.approx(want / (ms * 1e-3) / 1e9, rel=1e-12)
        # and about the layout's bytes per node and launch: the counters saw
        # the whole lattice (a multi-step pass re-reads its bands' halo rows)
        lo, hi = (0.9, 1.5) if pd["steps_per_launch"] >= 2 else (0.9, 1.1)
        assert lo * bench.LAYOUT_BYTES[st] < byts / nodes < hi * bench.LAYOUT_BYTES[st]


def test_traffic_dropped_for_another_lattice():
    blob = _profile_blob()
    assert bench.measured_traffic("f32", 0.25, blob["nodes"] + 1) == (None, None)


def test_valu_issue_from_the_counter_summary():
    """The vector-ALU issue fraction of a pass comes from the summary's
    instruction count over the launch time: at the profiled trace average
    it lies within the issue rate, and it is dropped for another lattice."""
    blob = _profile_blob()
    nodes = blob["nodes"]
    for st in ("f32", "f16", "bf16"):
        pd = blob["per_dispatch"][st]
        frac = bench.measured_valu_issue(st, pd["avg_ns"] * 1e-6, nodes)
        assert frac == pytest.approx(pd["valu_instr"] / (256 * 2.4e9 * pd["avg_ns"] * 1e-9),
                                     rel=1e-12)
        assert 0.0 < frac <= 1.0
    assert bench.measured_valu_issue("f32", 0.25, nodes + 1) is None
