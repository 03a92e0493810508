"""Batched compression (many fields in one captured persistent launch) against
the CPU oracle.

Every field's stream must be byte-identical to the oracle's stream of that
field at the block size the plan used; its mean and variance must equal the
oracle's reductions of that stream (1e-12 relative; both come from exact
integer sums).  Autotuned block sizes must follow the stated rule (smallest
stream of the field's first 2^20 elements, ties to the larger block), checked
with the oracle's stream sizes.  The captured launch is replayed with other
GPU work and synchronizations in between and every replay must reproduce the
first.  A field with a NaN or an out-of-range bin fails alone.
"""
import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu

REL = 1e-12
TUNE_SAMPLE = 1 << 20


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def close(a, b, rel=REL):
    return a == b or abs(a - b) <= rel * max(abs(a), abs(b))


def tuned_block(x, eb):
    m = x[:min(x.size, TUNE_SAMPLE)]
    best, best_bytes = 32, None
    for L in (32, 64, 128):
        b = ref.compress(m, eb, L).size
        if best_bytes is None or b <= best_bytes:
            best, best_bytes = L, b
    return best


def make_fields(seed, sizes, blocks):
    rng = np.random.default_rng(seed)
    out = []
    for i, n in enumerate(sizes):
        spec = {"index": i, "shape": (n,), "seed": int(rng.integers(0, 2**31 - 1)),
                "rel_eb": float(rng.choice([1e-2, 1e-3, 1e-4]))}
        x = synth.batch_field(spec)
        eb = synth.rel_eb(x, spec["rel_eb"])
        out.append((x, eb, blocks[i % len(blocks)]))
    return out


def run_batch(fields, dev, tune_grid=False):
    gx = [torch.from_numpy(x).to(dev) for x, _, _ in fields]
    outs = [torch.zeros(hz.batch_out_cap(x.size, L), dtype=torch.uint8, device=dev)
            for x, _, L in fields]
    b = hz.Batch([(gx[i], eb, L, outs[i]) for i, (_, eb, L) in enumerate(fields)],
                 tune_grid=tune_grid)
    return b, gx, outs


def check_against_oracle(fields, res, outs):
    for i, ((x, eb, L), r) in enumerate(zip(fields, res)):
        assert r["code"] == hz.OK, f"field {i} failed with {r['code']}"
        want_L = L if L else tuned_block(x, eb)
        assert r["block"] == want_L, f"field {i}: block {r['block']} != {want_L}"
        c = ref.compress(x, eb, want_L)
        got = outs[i][:r["out_bytes"]].cpu().numpy()
        assert r["out_bytes"] == c.size, f"field {i} (n={x.size}, L={want_L})"
        assert np.array_equal(got, c), f"field {i} stream differs (n={x.size}, L={want_L})"
        assert close(r["mean"], ref.mean(c)), f"field {i} mean"
        assert close(r["variance"], ref.variance(c)), f"field {i} variance"


SIZES = [1, 5, 31, 32, 33, 100, 1000, 8191, 8192, 8193, 20000, 3 * 8192 + 77, 65537, 150001,
         257, 4096, 70000, 12345, 2, 99999]


def test_batch_fixed_blocks_match_oracle(dev):
    print("case batch fixed blocks", flush=True)
    fields = make_fields(11, SIZES, [32, 64, 128])
    b, _, outs = run_batch(fields, dev)
    b.launch()
    res = b.results()
    check_against_oracle(fields, res, outs)
    info = b.info()
    assert info["fields"] == len(fields)
    assert info["raw_bytes"] == sum(4 * x.size for x, _, _ in fields)


def test_batch_autotuned_blocks_and_grid(dev):
    print("case batch autotune", flush=True)
    fields = make_fields(12, SIZES + [TUNE_SAMPLE + 4099], [0, 0, 32, 0, 128])
    b, _, outs = run_batch(fields, dev, tune_grid=True)
    b.launch()
    res = b.results()
    check_against_oracle(fields, res, outs)
    assert b.info()["grid"] >= 1


def test_batch_sums_of_large_bins(dev):
    """Segments whose bins reach 2^26 or more sum them one by one (the 32/64-bit
    per-segment sums would not be exact): mean and variance still equal the
    oracle's, beside fields of small bins and ragged lengths."""
    print("case batch large bins", flush=True)
    rng = np.random.default_rng(21)
    big = rng.uniform(-2.0**30, 2.0**30, 70001).astype(np.float32)
    mixed = rng.normal(0.0, 1.0, 50000).astype(np.float32)
    mixed[1000:1100] = 2.0**29  # a run of large bins inside small ones
    fields = [(big, 0.5, 32), (mixed, 0.5, 64), (big[:33333], 0.5, 128),
              (rng.normal(0.0, 1.0, 8193).astype(np.float32), 1e-3, 32)]
    b, _, outs = run_batch(fields, dev)
    b.launch()
    check_against_oracle(fields, b.results(), outs)


def test_batch_matches_single_field_ops(dev):
    print("case batch vs single ops", flush=True)
    fields = make_fields(13, [8193, 100000, 33, 77777], [32, 64, 128, 32])
    b, gx, outs = run_batch(fields, dev)
    b.launch()
    res = b.results()
    for i, (x, eb, L) in enumerate(fields):
        c = hz.compress(gx[i], eb, L)
        assert torch.equal(c, outs[i][:res[i]["out_bytes"]])
        assert hz.mean(c) == res[i]["mean"]
        assert hz.variance(c) == res[i]["variance"]


def test_batch_graph_replays_reproduce(dev):
    print("case batch replays", flush=True)
    fields = make_fields(14, SIZES[:12], [32, 64, 128, 0])
    b, gx, outs = run_batch(fields, dev)
    b.launch()
    first = b.results()
    first_streams = [o.clone() for o in outs]
    scratch = torch.randn(1 << 20, device=dev)
    for rep in range(3):
        # other GPU work between replays, including the library's own ops
        for o in outs:
            o.fill_(0xA5)
        scratch.mul_(1.0001)
        hz.compress(scratch, 0.01, 64)
        torch.cuda.synchronize()
        b.launch()
        again = b.results()
        assert again == first, f"replay {rep} results differ"
        for i, o in enumerate(outs):
            nbytes = first[i]["out_bytes"]
            assert torch.equal(o[:nbytes], first_streams[i][:nbytes]), f"replay {rep} field {i}"


def test_batch_field_errors_are_isolated(dev):
    print("case batch errors", flush=True)
    fields = make_fields(15, [5000, 9000, 300, 20000], [32, 64, 32, 128])
    bad = fields[1][0].copy()
    bad[4321] = np.nan
    fields[1] = (bad, fields[1][1], fields[1][2])
    big = np.full(3000, 1e6, dtype=np.float32)
    fields[2] = (big, 1e-6, 32)  # bins of 5e11 leave the int32 range
    b, _, outs = run_batch(fields, dev)
    b.launch()
    res = b.results()
    assert res[1]["code"] == hz.ERR_NONFINITE
    assert res[2]["code"] == hz.ERR_RANGE
    good = [0, 3]
    check_against_oracle([fields[i] for i in good], [res[i] for i in good],
                         [outs[i] for i in good])
    # a clean replay after the failures still matches
    b.launch()
    assert b.results()[0] == res[0]


def test_batch_rejects_bad_fields(dev):
    print("case batch arg errors", flush=True)
    x = torch.zeros(100, device=dev)
    out = torch.zeros(hz.batch_out_cap(100, 32), dtype=torch.uint8, device=dev)
    small = torch.zeros(64, dtype=torch.uint8, device=dev)
    with pytest.raises(hz.HoszpError) as e:
        hz.Batch([(x, 0.1, 32, out), (x, 0.1, 32, small)])
    assert e.value.code == hz.ERR_CAPACITY and "field 1" in str(e.value)
    with pytest.raises(hz.HoszpError) as e:
        hz.Batch([(x, -1.0, 32, out)])
    assert e.value.code == hz.ERR_ARG
    for bad_block in (48, 256):  # 256 is a valid stream block, but not in a batch
        with pytest.raises(hz.HoszpError) as e:
            hz.Batch([(x, 0.1, bad_block, torch.zeros(hz.batch_out_cap(100, 256), dtype=torch.uint8,
                                                        device=dev))])
        assert e.value.code == hz.ERR_ARG


def test_batch_full_size_sampled(dev):
    """The 4096-field batch (log-uniform 4 KB..64 MB, ~29 GB) as the benchmark
    runs it: every field must succeed, a seeded sample of fields up to 2M
    elements must match the oracle, and the largest fields must match the
    single-field GPU path (itself pinned to the oracle above)."""
    print("case batch full size", flush=True)
    specs = synth.batch_specs(4096, seed=7)
    _, xs = synth.batch_arena(specs, dev)
    ebs = [sp["rel_eb"] * synth.value_range(x) for sp, x in zip(specs, xs)]
    outs = [torch.empty((hz.batch_out_cap(x.numel(), 0) + 15) // 16 * 16, dtype=torch.uint8,
                        device=dev) for x in xs]
    b = hz.Batch([(xs[i], ebs[i], 0, outs[i]) for i in range(len(xs))], tune_grid=True)
    b.launch()
    res = b.results()
    assert all(r["code"] == hz.OK for r in res)
    rng = np.random.default_rng(3)
    small = [i for i, x in enumerate(xs) if x.numel() <= (1 << 21)]
    for i in rng.choice(small, size=12, replace=False):
        x = xs[i].cpu().numpy()
        c = ref.compress(x, ebs[i], res[i]["block"])
        assert res[i]["out_bytes"] == c.size, f"field {i}"
        assert np.array_equal(outs[i][:c.size].cpu().numpy(), c), f"field {i}"
        assert close(res[i]["mean"], ref.mean(c)) and close(res[i]["variance"], ref.variance(c))
    for i in sorted(range(len(xs)), key=lambda k: -xs[k].numel())[:3]:
        c = hz.compress(xs[i], ebs[i], res[i]["block"])
        assert torch.equal(c, outs[i][:res[i]["out_bytes"]]), f"field {i}"
        assert hz.mean(c) == res[i]["mean"] and hz.variance(c) == res[i]["variance"]


def fnv_signature(ns, blocks, cus):
    """The plan-shape key of the tuning cache (FNV-1a over little-endian
    64-bit words: tag, compute units, field count, then n and block of every
    field)."""
    h = 1469598103934665603
    words = [0x484F535A42415431, cus, len(ns)]
    for n, L in zip(ns, blocks):
        words += [n, L]
    for v in words:
        for k in range(8):
            h ^= (v >> (8 * k)) & 0xFF
            h = (h * 1099511628211) & 0xFFFFFFFFFFFFFFFF
    return h


@pytest.mark.parametrize("threads", [512, 1024])
def test_tuned_plan_tile_sizes_and_cache(dev, tmp_path, monkeypatch, threads):
    """Both tile sizes the autotuner chooses between give the oracle's streams;
    a tuned plan records its choice in the cache file, and a plan of the same
    shape takes the recorded choice (here forced to `threads`)."""
    print(f"case batch tile threads={threads}", flush=True)
    sizes = [1000, 33000, 70001, 5, 262144 + 77, 1 << 20, 40000]
    fields = make_fields(31, sizes, [32, 64, 128, 32, 64, 128, 32])
    cache = tmp_path / "tune.jsonl"
    monkeypatch.setenv("HOSZP_TUNE_CACHE", str(cache))
    b, gx, outs = run_batch(fields, dev, tune_grid=True)
    lines = cache.read_text().splitlines()
    assert len(lines) == 1
    rec = __import__("json").loads(lines[0])
    info = b.info()
    assert info["threads"] == rec["threads"] and info["grid"] == rec["grid"]
    b.launch()
    check_against_oracle(fields, b.results(), outs)
    b.close()
    # force the other tile size through the cache
    cus = torch.cuda.get_device_properties(dev).multi_processor_count
    key = fnv_signature([x.size for x, _, _ in fields], [L for _, _, L in fields], cus)
    assert f"{key:016x}" == rec["key"]
    with open(cache, "a") as f:
        f.write('{"key": "%016x", "threads": %d, "grid": %d, "ms": 1.0}\n' % (key, threads, cus))
    b, gx, outs = run_batch(fields, dev, tune_grid=True)
    info = b.info()
    assert info["threads"] == threads and info["grid"] == cus
    assert len(cache.read_text().splitlines()) == 2  # read, not tuned again
    for _ in range(2):
        b.launch()
        check_against_oracle(fields, b.results(), outs)
    b.close()
