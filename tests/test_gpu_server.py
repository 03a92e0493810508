"""Serving: the continuous-batching server against the same queries run alone.

A small device store (1-D sinusoid fields, a 3-D Kolmogorov field and
climate-like steps at several block sizes) is queried with a seeded mix of
mean / variance / add / negate / multiply on both paths.  Every query must give
the same code, value and output stream bytes when it runs alone (one slot, one
query at a time) as in the mix (several slots, Poisson arrivals fast enough
that queries overlap on the device).  Homomorphic results must also equal the
direct library calls and the CPU oracle (every op, including variance and
multiply); the pool budget must hold at every moment.
"""
import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
import paper_2408_11971_amd as hz  # noqa: E402

pytestmark = pytest.mark.gpu

MIX = [("mean", 0.3), ("variance", 0.3), ("add", 0.2), ("negate", 0.1), ("mul", 0.1)]


@pytest.fixture(scope="module")
def store():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    dev = torch.device("cuda:0")
    entries = []  # (stream tensor, header, group, host stream or None)

    def put(x, eb, L, group):
        c = hz.compress(torch.from_numpy(x).to(dev), eb, L).clone()
        entries.append((c, hz.header_of(c), group, x))

    a = synth.sinusoid_1d(1 << 18, seed=1)
    b = synth.sinusoid_1d(1 << 18, seed=2)
    eb = synth.rel_eb(a, 1e-3)
    put(a, eb, 32, "sin")
    put(b, eb, 32, "sin")
    g1 = synth.grf_3d(48, seed=3).ravel()
    g2 = synth.grf_3d(48, seed=4).ravel()
    egr = synth.rel_eb(g1, 1e-2)
    put(g1, egr, 32, "grf")
    put(g2, egr, 32, "grf")
    for t, step in enumerate(synth.climate_steps(3, 90, 180)):
        x = step.ravel()
        for L in (32, 64, 128):
            put(x, synth.rel_eb(x, 1e-4), L, f"clim{t}_{L}")
    return entries


def build_requests(server, store, count, seed, paths=(hz.PATH_HOMOMORPHIC,)):
    rng = np.random.default_rng(seed)
    names = [m[0] for m in MIX]
    probs = np.array([m[1] for m in MIX])
    groups = {}
    for i, e in enumerate(store):
        groups.setdefault(e[2], []).append(i)
    reqs = server.make_requests(count)
    picks = []
    for k in range(count):
        op = names[rng.choice(len(names), p=probs)]
        i = int(rng.integers(len(store)))
        j = int(rng.choice(groups[store[i][2]]))
        path = paths[int(rng.integers(len(paths)))]
        s = float(rng.uniform(-2, 2))
        c, h = store[i][0], store[i][1]
        hz.fill_request(reqs[k], op, c, store[j][0] if op == "add" else None, scalar=s,
                        path=path, tag=k, info=h)
        picks.append((op, i, j, s, path))
    return reqs, picks


def outputs(comps):
    """(code, value, out_bytes, host copy of the output stream or None)."""
    return [(int(c["code"]), float(c["value"]), int(c["out_bytes"]),
             _d2h(int(c["d_out"]), int(c["out_bytes"])) if c["d_out"] else None) for c in comps]


def _loaded_hip_runtime():
    """Path of the HIP runtime library this process already has mapped (the
    one torch and the library use), whatever its soname version."""
    with open("/proc/self/maps") as f:
        for line in f:
            path = line.split()[-1]
            if "libamdhip64.so" in path:
                return path
    raise RuntimeError("the HIP runtime is not loaded")


def _d2h(ptr, nbytes):
    """Host copy of device bytes at ptr (a stream held in the server's pool),
    through the HIP runtime the process already uses."""
    import ctypes
    hip = ctypes.CDLL(_loaded_hip_runtime())
    buf = np.empty(nbytes, dtype=np.uint8)
    torch.cuda.synchronize()
    rc = hip.hipMemcpy(ctypes.c_void_p(buf.ctypes.data), ctypes.c_void_p(ptr),
                       ctypes.c_size_t(nbytes), 2)  # hipMemcpyDeviceToHost
    assert rc == 0
    return buf


def run_alone(store, reqs):
    srv = hz.Server(slots=1, pool_bytes=256 << 20, keep_outputs=True)
    comps = []
    for k in range(reqs.size):
        srv.submit(reqs[k:k + 1])
        got = srv.drain()
        assert got.size == 1 and int(got[0]["tag"]) == k
        comps.append(got[0])
    res = outputs(comps)
    for c in comps:
        if c["d_out"]:
            srv.release(c["d_out"])
    srv.close()
    return res


@pytest.mark.parametrize("paths", [(hz.PATH_HOMOMORPHIC,), (hz.PATH_HOMOMORPHIC, hz.PATH_TRADITIONAL)])
def test_results_same_alone_and_in_the_mix(store, paths):
    print(f"case server mix paths={paths}", flush=True)
    srv = hz.Server(slots=8, pool_bytes=256 << 20, keep_outputs=True)
    reqs, picks = build_requests(srv, store, 240, seed=8 + len(paths), paths=paths)
    arrivals = np.cumsum(np.random.default_rng(5).exponential(1 / 20000.0, size=reqs.size))
    comps, start = srv.replay(reqs, arrivals)
    assert (comps["tag"] == np.arange(reqs.size)).all()
    mix = outputs(comps)
    # queries really overlapped: some query was launched before an earlier one finished
    order = np.argsort(comps["admit_s"])
    adm, done = comps["admit_s"][order], comps["done_s"][order]
    assert (adm[1:] < np.maximum.accumulate(done)[:-1]).any()
    st = srv.stats()
    assert st["completed"] == reqs.size and st["failed"] == 0
    assert st["pool_peak"] <= st["pool_bytes"]
    for c in comps:
        if c["d_out"]:
            srv.release(c["d_out"])
    srv.close()
    alone = run_alone(store, reqs)
    for k, (m, a) in enumerate(zip(mix, alone)):
        assert m[0] == a[0] == hz.OK, f"query {k} {picks[k]}: codes {m[0]} {a[0]}"
        assert m[1] == a[1], f"query {k} {picks[k]}: value {m[1]} != {a[1]}"
        assert m[2] == a[2], f"query {k} {picks[k]}: size"
        if m[3] is not None:
            assert np.array_equal(m[3], a[3]), f"query {k} {picks[k]}: stream differs"
    # every homomorphic result equals the direct call and the oracle
    for k in range(reqs.size):
        op, i, j, s, path = picks[k]
        if path != hz.PATH_HOMOMORPHIC:
            continue
        c = store[i][0]
        if op == "mean":
            assert mix[k][1] == hz.mean(c)
        elif op == "variance":
            assert mix[k][1] == hz.variance(c)
        else:
            want = {"negate": lambda: hz.negate(c), "mul": lambda: hz.mul(c, s),
                    "add": lambda: hz.add(c, store[j][0])}[op]()
            assert np.array_equal(mix[k][3], want.cpu().numpy())
        hc = store[i][0].cpu().numpy()
        if op == "mean":
            assert mix[k][1] == ref.mean(hc)
        elif op == "variance":
            want = ref.variance(hc)
            assert abs(mix[k][1] - want) <= 1e-12 * abs(want), (mix[k][1], want)
        elif op == "negate":
            assert np.array_equal(mix[k][3], ref.negate(hc))
        elif op == "mul":
            assert np.array_equal(mix[k][3], ref.mul(hc, s)), f"mul by {s!r}"
        elif op == "add":
            assert np.array_equal(mix[k][3], ref.add(hc, store[j][0].cpu().numpy()))
    assert {picks[k][0] for k in range(reqs.size)} >= {"mean", "variance", "negate", "add", "mul"}


def test_tight_pool_admits_by_budget(store):
    """A pool that holds about two decompress-then-compute queries at a time:
    everything still completes, queries wait for memory, the peak stays within
    the pool."""
    print("case server tight pool", flush=True)
    big = max(store, key=lambda e: e[1]["n"])
    need = (4 * big[1]["n"] + 255) // 256 * 256 * 2 + hz.compress_bound(big[1]["n"], big[1]["block"])
    srv = hz.Server(slots=8, pool_bytes=2 * need + 4096, keep_outputs=False)
    reqs = srv.make_requests(64)
    for k in range(64):
        hz.fill_request(reqs[k], "add", big[0], big[0], path=hz.PATH_TRADITIONAL, tag=k,
                        info=big[1])
    comps, _ = srv.replay(reqs, np.zeros(64))
    st = srv.stats()
    assert (comps["code"] == hz.OK).all() and st["completed"] == 64
    assert st["pool_peak"] <= st["pool_bytes"]
    # never more than two in flight: a third admission waits for a completion
    ev = sorted([(t, 1) for t in comps["admit_s"]] + [(t, -1) for t in comps["done_s"]])
    live = np.cumsum([d for _, d in ev])
    assert live.max() <= 2
    srv.close()


def test_request_errors(store):
    print("case server errors", flush=True)
    srv = hz.Server(slots=2, pool_bytes=1 << 20)
    c, h = store[0][0], store[0][1]
    reqs = srv.make_requests(1)
    hz.fill_request(reqs[0], "add", c, c, path=hz.PATH_TRADITIONAL, info=h)
    with pytest.raises(hz.HoszpError) as e:  # needs far more than a 1 MiB pool
        srv.submit(reqs)
    assert e.value.code == hz.ERR_CAPACITY
    reqs[0]["op"] = 9
    with pytest.raises(hz.HoszpError) as e:
        srv.submit(reqs)
    assert e.value.code == hz.ERR_ARG
    # a corrupt stream fails alone and is reported through its completion
    bad = c.clone()
    bad[0] = 0
    hz.fill_request(reqs[0], "mean", bad, info=h, tag=7)
    srv.submit(reqs)
    got = srv.drain()
    assert got.size == 1 and int(got[0]["tag"]) == 7 and int(got[0]["code"]) == hz.ERR_FORMAT
    srv.close()
