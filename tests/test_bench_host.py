"""Host-side logic of bench.py (no GPU): the one-GPU refusal, the event filter
of the timed steps, the op -> kernel map and the traffic lookup's checksum."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

STEP_OPS = ("compress", "compress_b", "mean", "decompress", "variance", "negate", "add", "mul")


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_every_step_op_maps_to_a_kernel():
    assert set(STEP_OPS) == set(bench.KERNEL_OF)
    assert bench.KERNEL_OF["compress"] == bench.KERNEL_OF["compress_b"]


class _Event:
    made = 0

    def __init__(self, enable_timing=False):
        _Event.made += 1

    def record(self):
        pass


class _Cuda:
    Event = _Event


class _Torch:
    cuda = _Cuda


def test_timer_times_only_the_named_ops():
    _Event.made = 0
    ran = []
    tm = bench.Timer(_Torch, only={"compress", "compress_b"})
    for op in STEP_OPS:
        tm.run((0, op), lambda op=op: ran.append(op))
    assert ran == list(STEP_OPS)  # every op still runs, in order
    assert set(k[1] for k in tm.pairs) == {"compress", "compress_b"}
    assert _Event.made == 4  # one start/end pair per timed op
    full = bench.Timer(_Torch)
    for op in STEP_OPS:
        full.run((0, op), lambda: None)
    assert len(full.pairs) == len(STEP_OPS)


def test_traffic_needs_the_current_kernel_source(tmp_path, monkeypatch):
    src = os.path.join(ROOT, "paper_2408_11971_amd", "csrc", "kernels.hip")
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    f = tmp_path / "traffic.json"
    launches = [(0, 0, 0.01, "compress"), (0, 0, 0.001, "compress")]
    f.write_text(json.dumps({"kernels_hip_sha256": sha,
                             "bytes": {"rel0.01/compress": 100, "rel0.001/compress": 300}}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(f))
    assert bench.measured_traffic("k_compress<1>", launches) == 200
    assert bench.measured_traffic("k_compress<1>", [(0, 0, 0.0001, "compress")]) is None
    f.write_text(json.dumps({"kernels_hip_sha256": "0" * 64,
                             "bytes": {"rel0.01/compress": 100, "rel0.001/compress": 300}}))
    assert bench.measured_traffic("k_compress<1>", launches) is None


@pytest.mark.parametrize("name", ["grf512_ops_pmc_traffic.json"])
def test_committed_traffic_summary_is_well_formed(name):
    t = json.load(open(os.path.join(ROOT, "profiles", name)))
    assert len(t["kernels_hip_sha256"]) == 64
    for rel in ("rel0.01", "rel0.001", "rel0.0001"):
        for op in STEP_OPS:
            assert t["bytes"][f"{rel}/{op}"] > 0
