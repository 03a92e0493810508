"""The asynchronous entry points captured in a graph: compress, add, scalar
multiply, Hadamard product and mean recorded once, replayed several times
with new input data written (eagerly) between replays.  Every replay must
equal the oracle on that replay's data: the look-back generation of each
encoder launch comes from device memory, so status words a previous replay
published never pass for the current one.
"""
import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu


def test_captured_ops_replay_with_new_data():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    dev = torch.device("cuda:0")
    n, L, eb = 1_500_007, 64, 0.002
    cap = hz.compress_bound(n, L)
    x = torch.empty(n, dtype=torch.float32, device=dev)
    y = torch.empty(n, dtype=torch.float32, device=dev)
    cx = torch.empty(cap, dtype=torch.uint8, device=dev)
    cy = torch.empty(cap, dtype=torch.uint8, device=dev)
    cz = torch.empty(cap, dtype=torch.uint8, device=dev)
    cm = torch.empty(cap, dtype=torch.uint8, device=dev)
    ch = torch.empty(cap, dtype=torch.uint8, device=dev)
    res = [hz.new_result(dev) for _ in range(6)]
    ctx = hz.context(0)
    s = torch.cuda.Stream()
    datasets = []
    for k in range(4):
        a = synth.sinusoid_1d(n, seed=40 + k) * (1.0 + k)
        b = synth.sinusoid_1d(n, seed=50 + k)
        datasets.append((a.astype(np.float32), b.astype(np.float32)))

    def ops():
        hz.compress_async(x, eb, L, cx, res[0], ctx)
        hz.compress_async(y, eb, L, cy, res[1], ctx)
        hz.add_async(cx, cy, cz, res[2], ctx)
        hz.mul_async(cx, -1.75, cm, res[3], ctx)
        hz.mean_async(cx, res[4], ctx)
        hz.hadamard_async(cx, cy, ch, res[5], ctx)

    # warm up on the side stream, then capture
    x.copy_(torch.from_numpy(datasets[0][0]))
    y.copy_(torch.from_numpy(datasets[0][1]))
    torch.cuda.synchronize()
    with torch.cuda.stream(s):
        ops()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        ops()
    torch.cuda.synchronize()
    for rep, (a, b) in enumerate(datasets[1:] + datasets[:1] + datasets[2:3]):
        print(f"case graph replay {rep}", flush=True)
        x.copy_(torch.from_numpy(a))          # eager work between replays
        y.copy_(torch.from_numpy(b))
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        recs = [hz.read_result(r) for r in res]
        assert all(r["code"] == 0 for r in recs), recs
        ac, bc = ref.compress(a, eb, L), ref.compress(b, eb, L)
        assert np.array_equal(cx[:recs[0]["out_bytes"]].cpu().numpy(), ac), rep
        assert np.array_equal(cy[:recs[1]["out_bytes"]].cpu().numpy(), bc), rep
        assert np.array_equal(cz[:recs[2]["out_bytes"]].cpu().numpy(), ref.add(ac, bc)), rep
        assert np.array_equal(cm[:recs[3]["out_bytes"]].cpu().numpy(), ref.mul(ac, -1.75)), rep
        assert recs[4]["value"] == ref.mean(ac), rep
        assert np.array_equal(ch[:recs[5]["out_bytes"]].cpu().numpy(), ref.hadamard(ac, bc)), rep
        # an eager call on the same context between replays
        assert np.array_equal(hz.add(cx[:recs[0]["out_bytes"]], cy[:recs[1]["out_bytes"]]).cpu().numpy(),
                              ref.add(ac, bc))
