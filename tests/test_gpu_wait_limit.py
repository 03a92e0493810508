"""The encoders' bounded look-back wait, forced from the host.

A context's poll limit of 0 makes every encoder tile but the first give up on
its look-back at once: the launch drains normally and reports ERR_TIMEOUT.
Single-tile inputs never wait and stay exact; after the limit is restored the
same context produces the oracle's streams again (a launch that gave up leaves
no state behind that a later launch could mistake for its own).  No kernel
stalls in these tests: the condition is made by the host's limit alone.
"""
import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu

N_MULTI = 200_003   # 6251 segments of 32: several 1024-segment encoder tiles
N_SINGLE = 8_000    # 250 segments: one tile at every tile size (256, 512, 1024)
L, EB = 32, 1e-3


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def field(n, seed, dev):
    x = synth.sinusoid_1d(n, seed=seed).astype(np.float32)
    return x, torch.from_numpy(x).to(dev)


def test_limit_zero_times_out_and_recovers(dev):
    print("case wait limit 0: compress/add/sub/mul/hadamard", flush=True)
    ctx = hz.Context(0)
    try:
        a, ga = field(N_MULTI, 1, dev)
        b, gb = field(N_MULTI, 2, dev)
        ca, cb = ref.compress(a, EB, L), ref.compress(b, EB, L)
        da, db = torch.from_numpy(ca).to(dev), torch.from_numpy(cb).to(dev)
        cap = hz.compress_bound(N_MULTI, L)
        out = torch.empty(cap, dtype=torch.uint8, device=dev)
        res = hz.new_result(dev)
        ctx.set_wait_limit(0)
        calls = {
            "compress": lambda: hz.compress_async(ga, EB, L, out, res, ctx),
            "add": lambda: hz.add_async(da, db, out, res, ctx),
            "sub": lambda: hz.sub_async(da, db, out, res, ctx),
            "mul": lambda: hz.mul_async(da, 1.75, out, res, ctx),
            "hadamard": lambda: hz.hadamard_async(da, db, out, res, ctx),
        }
        for name, call in calls.items():
            call()
            r = hz.read_result(res, ctx)
            assert r["code"] == hz.ERR_TIMEOUT, (name, r)
        # one tile never waits: exact even at limit 0
        s, gs = field(N_SINGLE, 3, dev)
        hz.compress_async(gs, EB, L, out, res, ctx)
        r = hz.read_result(res, ctx)
        assert r["code"] == hz.OK, r
        assert np.array_equal(out[:r["out_bytes"]].cpu().numpy(), ref.compress(s, EB, L))
        # the default limit restores exact results on the same context
        ctx.set_wait_limit(hz.DEFAULT_WAIT_LIMIT)
        expect = {
            "compress": ca,
            "add": ref.add(ca, cb),
            "sub": ref.sub(ca, cb),
            "mul": ref.mul(ca, 1.75),
            "hadamard": ref.hadamard(ca, cb),
        }
        for name, call in calls.items():
            call()
            r = hz.read_result(res, ctx)
            assert r["code"] == hz.OK, (name, r)
            assert np.array_equal(out[:r["out_bytes"]].cpu().numpy(), expect[name]), name
    finally:
        torch.cuda.synchronize()
        ctx.close()


def test_batch_limit_zero_isolates_fields(dev):
    print("case wait limit 0: batch", flush=True)
    ctx = hz.Context(0)
    try:
        ctx.set_wait_limit(0)   # taken by the plan at creation
        sizes = [N_SINGLE, N_MULTI, 1000, 3 * 32768 + 5]
        fields, hosts = [], []
        for i, n in enumerate(sizes):
            x, gx = field(n, 10 + i, dev)
            out = torch.empty(hz.batch_out_cap(n, L), dtype=torch.uint8, device=dev)
            fields.append((gx, EB, L, out))
            hosts.append(x)
        b = hz.Batch(fields, ctx=ctx)
        b.launch()
        res = b.results()
        for (gx, _, _, out), x, r in zip(fields, hosts, res):
            one_tile = (x.size + 31) // 32 <= b.info()["threads"]
            if one_tile:
                assert r["code"] == hz.OK, r
                assert np.array_equal(out[:r["out_bytes"]].cpu().numpy(), ref.compress(x, EB, L))
            else:
                assert r["code"] == hz.ERR_TIMEOUT, r
        b.close()
        # a plan made at the default limit is exact on the same context
        ctx.set_wait_limit(hz.DEFAULT_WAIT_LIMIT)
        b = hz.Batch(fields, ctx=ctx)
        b.launch()
        for (gx, _, _, out), x, r in zip(fields, hosts, b.results()):
            assert r["code"] == hz.OK, r
            assert np.array_equal(out[:r["out_bytes"]].cpu().numpy(), ref.compress(x, EB, L))
        b.close()
    finally:
        torch.cuda.synchronize()
        ctx.close()
