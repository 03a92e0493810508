"""Benchmark of the HoSZp hot path on one MI355X.

Workload: the 3-D 512^3 float32 Kolmogorov-spectrum random field (two seeded
fields A and B, 537 MB each) at relative error bounds 1e-2, 1e-3 and 1e-4 of
A's value range, block 32.  One step runs, for every bound, the whole hot
path on device-resident data through the C ABI (async entry points, one
stream):

    compress A, compress B, mean(A), decompress(B), variance(A), negate(B),
    add(A, B), mul(A, 3.14)

Every op of a step reads its own copy of its input streams (four copies of
each stream per bound, made once), so no op finds its input in the 256 MB
last-level cache because the op before it just read it.  One instrumented
step before the timed ones names the kernel with the largest share of a
step; the timed steps carry HIP events only around that kernel's launches
(the roofline's live durations).  The per-op table times every op alone
after a 1 GiB cache-flushing write (median of --reps), the step's ops and
the remaining Table II ops (element-wise subtraction, scalar addition,
Hadamard product, covariance, block means); the decompress-then-compute
workflow (decompress, float32 op in HBM, re-compress for
compression-as-output ops) is timed the same way for the comparison.  Then
the climate-like sweep (100 1800x3600 steps, blocks 32/64/128; each op over
the whole sweep, captured in a graph and replayed), and the CPU oracle on a
bounded sample, on one thread and on all host cores.

stdout: one JSON line.  Diagnostics go to stderr.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "homomorphic op GB/s (raw-equiv) vs decompress+op; compress/decompress GB/s"
HBM_PEAK_GBS = 8000.0
RELS = (1e-2, 1e-3, 1e-4)
BLOCK = 32
SCALAR = 3.14


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--n", type=int, default=512, help="edge of the cubic field")
    ap.add_argument("--cpu-sample", type=int, default=1 << 24,
                    help="elements of each field the oracle is timed on (0 = skip)")
    ap.add_argument("--reps", type=int, default=5, help="flushed repetitions per op")
    ap.add_argument("--trad-reps", type=int, default=3)
    ap.add_argument("--climate-steps", type=int, default=100,
                    help="climate-like 1800x3600 steps of the sweep leg (0 = skip)")
    ap.add_argument("--cpu-threads", type=int, default=16,
                    help="most host threads for the all-core oracle leg")
    ap.add_argument("--workload", choices=("grf512", "batch", "serve"), default="grf512",
                    help="grf512: the 512^3 field ops (default); batch: 4096 uneven fields "
                         "compressed with mean/variance in one captured launch; serve: Poisson "
                         "query streams over a device store of compressed fields")
    ap.add_argument("--batch-count", type=int, default=4096)
    ap.add_argument("--store-gb", type=float, default=40.0)
    ap.add_argument("--serve-seconds", type=float, default=10.0,
                    help="arrival window per offered rate")
    ap.add_argument("--leg-batch", type=int, default=1,
                    help="default workload: also run the 4096-field batch (0 = skip)")
    ap.add_argument("--leg-serve-gb", type=float, default=10.0,
                    help="default workload: store size of the short serving leg (0 = skip)")
    ap.add_argument("--leg-serve-seconds", type=float, default=2.0,
                    help="default workload: arrival window per rate of the serving leg")
    ap.add_argument("--leg-c1", type=int, default=1,
                    help="default workload: also time the 2^20-element 1-D field (0 = skip)")
    ap.add_argument("--rates", default="1000,5000,20000,50000")
    ap.add_argument("--slots", type=int, default=8)
    return ap.parse_args()


class Timer:
    """HIP events on the current stream around one enqueued op.  `only`: the
    op names (second item of a key) to time; other ops just run."""

    def __init__(self, torch, only=None):
        self.torch = torch
        self.pairs = {}
        self.only = only

    def run(self, key, fn):
        name = key[1] if isinstance(key, tuple) else key
        if self.only is not None and name not in self.only:
            fn()
            return
        s = self.torch.cuda.Event(enable_timing=True)
        e = self.torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        self.pairs.setdefault(key, []).append((s, e))

    def mean_us(self, key):
        ps = self.pairs[key]
        return 1000.0 * sum(s.elapsed_time(e) for s, e in ps) / len(ps)


FLUSH_BYTES = 1 << 30
COPIES = 4  # read-only copies of each stream per bound: every op of a step reads its own


class Flusher:
    """Writes a 1 GiB buffer, which evicts the L2 caches and the 256 MB
    last-level cache, so the op timed next reads its inputs from HBM."""

    def __init__(self, torch, dev):
        self.buf = torch.empty(FLUSH_BYTES // 4, dtype=torch.float32, device=dev)

    def __call__(self):
        self.buf.fill_(1.0)


def time_flushed(torch, flush, fn, reps):
    """Median device time (us) of fn over `reps` runs, each after a flush,
    with HIP events on the current stream around fn alone."""
    pairs = []
    for _ in range(reps):
        flush()
        s = torch.cuda.Event(enable_timing=True)
        e = torch.cuda.Event(enable_timing=True)
        s.record()
        fn()
        e.record()
        pairs.append((s, e))
    torch.cuda.synchronize()
    ts = sorted(1000.0 * s.elapsed_time(e) for s, e in pairs)
    return ts[len(ts) // 2]


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the library has no "
              "multi-GPU path", file=sys.stderr)
        sys.exit(2)
    if args.workload == "batch":
        return bench_batch(args)
    if args.workload == "serve":
        return bench_serve(args)
    import torch

    import paper_2408_11971_amd as hz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    ctx = hz.context(0)
    n3 = args.n
    N = n3 ** 3
    log(f"generating two {n3}^3 fields on the GPU")
    A = synth.grf_3d(n3, seed=3, device=dev).view(-1)
    B = synth.grf_3d(n3, seed=4, device=dev).view(-1)
    rng = synth.value_range(A)
    ebs = [rel * rng for rel in RELS]
    cap = hz.compress_bound(N, BLOCK)
    W = [{k: torch.empty(cap, dtype=torch.uint8, device=dev)
          for k in ("a", "b", "neg", "sum", "mul", "sub", "sadd", "had", "trad")} for _ in ebs]
    dec = torch.empty(N, dtype=torch.float32, device=dev)
    d2 = torch.empty(N, dtype=torch.float32, device=dev)
    t32 = torch.empty(N, dtype=torch.float32, device=dev)
    nbk = (N + BLOCK - 1) // BLOCK
    bmeans = torch.empty(nbk, dtype=torch.float64, device=dev)
    res = {name: hz.new_result(dev) for name in
           ("ca", "cb", "mean", "dec", "var", "neg", "add", "mul", "sub", "sadd", "had", "cov",
            "bm", "t0", "t1", "t2")}

    def check(name):
        r = hz.read_result(res[name], ctx)
        if r["code"] != 0:
            raise RuntimeError(f"{name} failed with code {r['code']}")
        return r

    # the streams of every bound, and COPIES read-only copies of each: the ops
    # of a step read different copies, so no op finds its input in a cache
    # because the op before it touched it (a copy is read once per step)
    R = []
    for i, eb in enumerate(ebs):
        hz.compress_async(A, eb, BLOCK, W[i]["a"], res["ca"], ctx)
        hz.compress_async(B, eb, BLOCK, W[i]["b"], res["cb"], ctx)
        ca_b, cb_b = check("ca")["out_bytes"], check("cb")["out_bytes"]
        R.append(([W[i]["a"][:ca_b].clone() for _ in range(COPIES)],
                  [W[i]["b"][:cb_b].clone() for _ in range(COPIES)]))

    def step(tm):
        for i, eb in enumerate(ebs):
            RA, RB = R[i]
            w = W[i]
            tm.run((i, "compress"), lambda: hz.compress_async(A, eb, BLOCK, w["a"], res["ca"], ctx))
            tm.run((i, "compress_b"), lambda: hz.compress_async(B, eb, BLOCK, w["b"], res["cb"], ctx))
            tm.run((i, "mean"), lambda: hz.mean_async(RA[0], res["mean"], ctx))
            tm.run((i, "decompress"), lambda: hz.decompress_async(RB[0], dec, res["dec"], ctx))
            tm.run((i, "variance"), lambda: hz.variance_async(RA[1], res["var"], ctx))
            tm.run((i, "negate"), lambda: hz.negate_async(RB[1], w["neg"], res["neg"], ctx))
            tm.run((i, "add"), lambda: hz.add_async(RA[2], RB[2], w["sum"], res["add"], ctx))
            tm.run((i, "mul"), lambda: hz.mul_async(RA[3], SCALAR, w["mul"], res["mul"], ctx))

    log("warmup")
    for _ in range(args.warmup):
        step(Timer(torch))
    torch.cuda.synchronize()
    for name in ("ca", "cb", "mean", "dec", "var", "neg", "add", "mul"):
        check(name)

    # One instrumented, untimed step names the kernel with the largest share
    # of a step; the timed steps carry HIP events only around that kernel's
    # launches (its live duration is the roofline's denominator), so event
    # packets between the other ops do not slow the steps being timed.
    probe = Timer(torch)
    step(probe)
    torch.cuda.synchronize()
    share = {}
    for (i, op), _ in probe.pairs.items():
        share[KERNEL_OF[op]] = share.get(KERNEL_OF[op], 0.0) + probe.mean_us((i, op))
    kname = max(share, key=share.get)
    timed_ops = {op for op in KERNEL_OF if KERNEL_OF[op] == kname}
    tm = Timer(torch, only=timed_ops)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step(tm)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_per_step = 1000.0 * wall / args.steps
    for name in ("ca", "cb", "mean", "dec", "var", "neg", "add", "mul"):
        check(name)

    # output sizes and block statistics of every bound
    sizes = []
    for i, eb in enumerate(ebs):
        RA, RB = R[i]
        w = W[i]
        hz.add_async(RA[2], RB[2], w["sum"], res["add"], ctx)
        hz.negate_async(RB[1], w["neg"], res["neg"], ctx)
        hz.mul_async(RA[3], SCALAR, w["mul"], res["mul"], ctx)
        hz.sub_async(RA[0], RB[0], w["sub"], res["sub"], ctx)
        hz.scalar_add_async(RB[1], SCALAR, w["sadd"], res["sadd"], ctx)
        hz.hadamard_async(RA[2], RB[2], w["had"], res["had"], ctx)
        sz = {k: check(r)["out_bytes"] for k, r in (("sum", "add"), ("neg", "neg"), ("mul", "mul"),
                                                   ("sub", "sub"), ("sadd", "sadd"), ("had", "had"))}
        sz["ca"], sz["cb"] = RA[0].numel(), RB[0].numel()
        for key, c in (("a", RA[0]), ("b", RB[0])):
            h = hz.header_of(c)
            wd = c[64:64 + h["nb"]].to(torch.int32)
            sz["nonconst_" + key] = int((wd > 0).sum().item())
            sz["payload_" + key] = h["payload_bytes"]
        sz["nb"] = nbk
        sizes.append(sz)

    # ---- plain device copy of one field: the measured HBM ceiling (read + write 4N bytes)
    tc = Timer(torch)
    for _ in range(5):
        tc.run("copy", lambda: t32.copy_(A))
    torch.cuda.synchronize()
    copy_gbps = 8 * N / tc.mean_us("copy") / 1e3

    # ---- every op alone, after a cache flush, and the decompress-then-compute
    # workflow the same way
    log("timing each op after a cache flush, homomorphic and decompress-then-compute")
    flush = Flusher(torch, dev)
    ops = {}
    raw_per_step = 0
    launches = []  # (algorithmic bytes, us, rel, op) of the dominant kernel's launches in a step
    for i, rel in enumerate(RELS):
        RA, RB = R[i]
        w = W[i]
        eb = ebs[i]
        sz = sizes[i]
        C, Cb = sz["ca"], sz["cb"]
        red_a = sz["nb"] + 4 * sz["nb"] + 4 * sz["nonconst_a"] + sz["payload_a"]
        red_b = sz["nb"] + 4 * sz["nb"] + 4 * sz["nonconst_b"] + sz["payload_b"]
        hom = {
            "compress": (4 * N, 4 * N + C,
                         lambda: hz.compress_async(A, eb, BLOCK, w["a"], res["ca"], ctx)),
            "decompress": (4 * N, Cb + 4 * N,
                           lambda: hz.decompress_async(RB[0], dec, res["dec"], ctx)),
            "mean": (4 * N, red_a, lambda: hz.mean_async(RA[0], res["mean"], ctx)),
            "variance": (4 * N, red_a, lambda: hz.variance_async(RA[1], res["var"], ctx)),
            "negate": (4 * N, 2 * Cb, lambda: hz.negate_async(RB[1], w["neg"], res["neg"], ctx)),
            "add": (8 * N, C + Cb + sz["sum"],
                    lambda: hz.add_async(RA[2], RB[2], w["sum"], res["add"], ctx)),
            "mul": (4 * N, C + sz["mul"],
                    lambda: hz.mul_async(RA[3], SCALAR, w["mul"], res["mul"], ctx)),
            "sub": (8 * N, C + Cb + sz["sub"],
                    lambda: hz.sub_async(RA[0], RB[0], w["sub"], res["sub"], ctx)),
            "scalar_add": (4 * N, 2 * Cb,
                           lambda: hz.scalar_add_async(RB[1], SCALAR, w["sadd"], res["sadd"], ctx)),
            "hadamard": (8 * N, C + Cb + sz["had"],
                         lambda: hz.hadamard_async(RA[2], RB[2], w["had"], res["had"], ctx)),
            "covariance": (8 * N, red_a + red_b,
                           lambda: hz.covariance_async(RA[3], RB[3], res["cov"], ctx)),
            "block_means": (4 * N, red_a + 8 * sz["nb"],
                            lambda: hz.block_means_async(RA[0], bmeans, res["bm"], ctx)),
        }

        def dec1(c):
            hz.decompress_async(c, dec, res["t0"], ctx)

        def dec2(a, b):
            hz.decompress_async(a, dec, res["t0"], ctx)
            hz.decompress_async(b, d2, res["t1"], ctx)

        def recompress():
            hz.compress_async(t32, eb, BLOCK, w["trad"], res["t2"], ctx)

        trad = {
            "mean": lambda: (dec1(RA[0]), hz.f32_mean_async(dec, res["t1"], ctx)),
            "variance": lambda: (dec1(RA[1]), hz.f32_variance_async(dec, res["t1"], ctx)),
            "negate": lambda: (dec1(RB[1]), hz.f32_negate_async(dec, t32, ctx), recompress()),
            "add": lambda: (dec2(RA[2], RB[2]), hz.f32_add_async(dec, d2, t32, ctx), recompress()),
            "mul": lambda: (dec1(RA[3]), hz.f32_mul_async(dec, SCALAR, t32, ctx), recompress()),
            "sub": lambda: (dec2(RA[0], RB[0]), hz.f32_sub_async(dec, d2, t32, ctx), recompress()),
            "scalar_add": lambda: (dec1(RB[1]), hz.f32_scalar_add_async(dec, SCALAR, t32, ctx),
                                   recompress()),
            "hadamard": lambda: (dec2(RA[2], RB[2]), hz.f32_hadamard_async(dec, d2, t32, ctx),
                                 recompress()),
        }
        row = {"cr": round(4 * N / C, 3),
               "const_block_pct": round(100.0 * (1 - sz["nonconst_a"] / sz["nb"]), 2)}
        for op, (raw, alg, fn) in hom.items():
            us = time_flushed(torch, flush, fn, args.reps)
            entry = {"us": round(us, 2), "gbps_raw": round(raw / us / 1e3, 1),
                     "hbm_gbps": round(alg / us / 1e3, 1),
                     "hbm_frac": round(alg / us / 1e3 / HBM_PEAK_GBS, 4)}
            if op in trad:
                t_us = time_flushed(torch, flush, trad[op], args.trad_reps)
                entry["trad_us"] = round(t_us, 2)
                entry["speedup_vs_trad"] = round(t_us / us, 2)
            row[op] = entry
            if op in KERNEL_OF:
                raw_per_step += raw
            if op in timed_ops:  # the dominant kernel: durations from the timed steps
                launches.append((alg, tm.mean_us((i, op)), rel, op))
        raw_per_step += 4 * N  # compress of B
        if "compress_b" in timed_ops:
            launches.append((4 * N + Cb, tm.mean_us((i, "compress_b")), rel, "compress_b"))
        ops[f"rel{rel:g}"] = row
    for name in ("ca", "dec", "mean", "var", "neg", "add", "mul", "sub", "sadd", "had", "cov",
                 "bm", "t0", "t1", "t2"):
        check(name)

    value = raw_per_step / (ms_per_step / 1000.0) / 1e9
    ls = launches
    alg_avg = sum(x[0] for x in ls) / len(ls)
    us_avg = sum(x[1] for x in ls) / len(ls)
    achieved = alg_avg / us_avg / 1e3
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": measured_traffic(kname, ls),
                "kernel": kname, "launches_per_step": len(ls),
                "bytes_per_launch": round(alg_avg), "us_per_launch": round(us_avg, 2),
                "events_include": PREPASS_NOTE.get(kname, "the kernel alone")}

    climate = None
    if args.climate_steps > 0:
        del dec, d2, t32, bmeans
        R.clear()
        W.clear()
        torch.cuda.empty_cache()
        climate = bench_climate(args, torch, hz, synth, ctx, dev)

    c1 = run_c1(torch, hz, synth, ctx, dev) if args.leg_c1 else None

    cpu = None
    if args.cpu_sample > 0:
        cpu = cpu_baseline(A, B, ebs, min(args.cpu_sample, N), args.cpu_threads)
    del A, B
    torch.cuda.empty_cache()
    batch = run_batch(args, 5, 2, False) if args.leg_batch and args.batch_count > 0 else None
    serve = (run_serve(args, args.leg_serve_gb, args.leg_serve_seconds, args.rates, False)
             if args.leg_serve_gb > 0 else None)

    line = {
        "metric": METRIC, "value": round(value, 1), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 bins (f64 quantization, int64/int128 sums)", "data": "synthetic",
        "config": {"workload": f"grf3d_{n3}^3_k-5/3_two_fields", "n": N, "block": BLOCK,
                   "rel_eb": list(RELS), "ops_per_step": 8 * len(RELS),
                   "raw_bytes_per_step": raw_per_step, "parallelism": "single_gpu",
                   "copy_gbps": round(copy_gbps, 1),
                   "step_reads": f"each op of a step reads its own one of {COPIES} copies of "
                                 "its input streams (a copy is read once per step)",
                   "ops_timing": f"each op alone after a {FLUSH_BYTES >> 20} MiB cache-flushing "
                                 f"write, median of {args.reps} (decompress-then-compute: "
                                 f"{args.trad_reps})"},
        "roofline": roofline,
        "cpu_baseline": cpu,
        "ops": ops,
        "climate": climate,
        "c1_1d": c1,
        "batch": batch,
        "serve": serve,
    }
    print(json.dumps(line), flush=True)


def run_c1(torch, hz, synth, ctx, dev, reps=20):
    """The 2^20-element 1-D field (sum of 8 sinusoids plus noise, seeds 1 and
    2, eb = 1e-3 of the range, block 32): each op replayed `reps` times from
    a graph.  4 MiB per field stays in the 256 MB last-level cache, so these
    rates are cache-resident, not HBM figures."""
    n = 1 << 20
    a = synth.sinusoid_1d(n, seed=1)
    b = synth.sinusoid_1d(n, seed=2)
    eb = synth.rel_eb(a, 1e-3)
    A = torch.from_numpy(a).to(dev)
    B = torch.from_numpy(b).to(dev)
    cap = hz.compress_bound(n, 32)
    ca, cb, co = (torch.empty(cap, dtype=torch.uint8, device=dev) for _ in range(3))
    dec = torch.empty(n, dtype=torch.float32, device=dev)
    res = hz.new_result(dev)
    hz.compress_async(A, eb, 32, ca, res, ctx)
    C = hz.read_result(res, ctx)["out_bytes"]
    hz.compress_async(B, eb, 32, cb, res, ctx)
    Cb = hz.read_result(res, ctx)["out_bytes"]
    sa, sb = ca[:C], cb[:Cb]
    ops = {
        "compress": (4 * n, lambda: hz.compress_async(A, eb, 32, ca, res, ctx)),
        "decompress": (4 * n, lambda: hz.decompress_async(sa, dec, res, ctx)),
        "negate": (4 * n, lambda: hz.negate_async(sa, co, res, ctx)),
        "add": (8 * n, lambda: hz.add_async(sa, sb, co, res, ctx)),
        "mean": (4 * n, lambda: hz.mean_async(sa, res, ctx)),
        "variance": (4 * n, lambda: hz.variance_async(sa, res, ctx)),
    }
    out = {"n": n, "block": 32, "rel_eb": 1e-3, "cr": round(4 * n / C, 3),
           "note": "cache-resident (4 MiB per field): not an HBM roofline row", "ops": {}}
    for op, (raw, fn) in ops.items():
        us = graph_us(torch, lambda: [fn() for _ in range(reps)], 3) / reps
        out["ops"][op] = {"us": round(us, 2), "gbps_raw": round(raw / us / 1e3, 1)}
    r = hz.read_result(res, ctx)
    if r["code"] != 0:
        raise RuntimeError(f"1-D field ops failed: {r['code']}")
    return out


def graph_us(torch, body, reps):
    """Capture body() (async library calls on the current stream) in a graph,
    replay it `reps` times and return the median replay time (us)."""
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        body()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        body()
    torch.cuda.synchronize()
    ts = []
    for _ in range(reps):
        a = torch.cuda.Event(enable_timing=True)
        b = torch.cuda.Event(enable_timing=True)
        a.record()
        g.replay()
        b.record()
        torch.cuda.synchronize()
        ts.append(1000.0 * a.elapsed_time(b))
    del g
    ts.sort()
    return ts[len(ts) // 2]


def bench_climate(args, torch, hz, synth, ctx, dev):
    """The climate-like sweep: `climate_steps` 1800x3600 float32 steps made on
    the GPU, one error bound for the whole sweep (1e-4 of its value range, so
    consecutive steps can be added), blocks 32/64/128.  Each op runs over the
    whole sweep (per-step mean/variance/negate/scalar multiply, pairwise
    add of steps t and t+1), captured in a graph and replayed (median of 3);
    decompress-then-compute the same way."""
    import numpy as np

    T = args.climate_steps
    log(f"generating {T} climate-like 1800x3600 steps on the GPU")
    X = synth.climate_steps_device(T, device=dev)
    n = X.shape[1]
    eb = 1e-4 * synth.value_range(X)
    scal = np.random.default_rng(9).uniform(-2.0, 2.0, T).tolist()
    res = [hz.new_result(dev) for _ in range(3)]
    dec = torch.empty(n, dtype=torch.float32, device=dev)
    d2 = torch.empty(n, dtype=torch.float32, device=dev)
    t32 = torch.empty(n, dtype=torch.float32, device=dev)
    out = {"steps": T, "shape": [1800, 3600], "eb": eb, "blocks": {}}
    for L in (32, 64, 128):
        log(f"climate sweep, block {L}")
        cap = hz.compress_bound(n, L)
        C = [torch.empty(cap, dtype=torch.uint8, device=dev) for _ in range(T)]
        o = torch.empty(cap, dtype=torch.uint8, device=dev)
        sizes = []
        for t in range(T):
            hz.compress_async(X[t], eb, L, C[t], res[0], ctx)
            r = hz.read_result(res[0], ctx)
            if r["code"] != 0:
                raise RuntimeError(f"climate compress failed: {r['code']}")
            sizes.append(r["out_bytes"])
        S = [C[t][:sizes[t]] for t in range(T)]
        hom = {
            "compress": (4 * n * T, lambda: [hz.compress_async(X[t], eb, L, C[t], res[0], ctx)
                                             for t in range(T)]),
            "decompress": (4 * n * T, lambda: [hz.decompress_async(S[t], dec, res[0], ctx)
                                               for t in range(T)]),
            "mean": (4 * n * T, lambda: [hz.mean_async(S[t], res[0], ctx) for t in range(T)]),
            "variance": (4 * n * T, lambda: [hz.variance_async(S[t], res[0], ctx)
                                             for t in range(T)]),
            "negate": (4 * n * T, lambda: [hz.negate_async(S[t], o, res[0], ctx) for t in range(T)]),
            "add": (8 * n * (T - 1), lambda: [hz.add_async(S[t], S[t + 1], o, res[0], ctx)
                                              for t in range(T - 1)]),
            "mul": (4 * n * T, lambda: [hz.mul_async(S[t], scal[t], o, res[0], ctx)
                                        for t in range(T)]),
        }

        def trad_unary(t, f32op):
            hz.decompress_async(S[t], dec, res[1], ctx)
            f32op(t)

        trad = {
            "mean": lambda: [trad_unary(t, lambda t: hz.f32_mean_async(dec, res[2], ctx))
                             for t in range(T)],
            "variance": lambda: [trad_unary(t, lambda t: hz.f32_variance_async(dec, res[2], ctx))
                                 for t in range(T)],
            "negate": lambda: [(trad_unary(t, lambda t: hz.f32_negate_async(dec, t32, ctx)),
                                hz.compress_async(t32, eb, L, o, res[2], ctx)) for t in range(T)],
            "add": lambda: [(hz.decompress_async(S[t], dec, res[1], ctx),
                             hz.decompress_async(S[t + 1], d2, res[1], ctx),
                             hz.f32_add_async(dec, d2, t32, ctx),
                             hz.compress_async(t32, eb, L, o, res[2], ctx)) for t in range(T - 1)],
            "mul": lambda: [(trad_unary(t, lambda t: hz.f32_mul_async(dec, scal[t], t32, ctx)),
                             hz.compress_async(t32, eb, L, o, res[2], ctx)) for t in range(T)],
        }
        row = {"cr": round(4 * n * T / sum(sizes), 3)}
        for op, (raw, body) in hom.items():
            us = graph_us(torch, body, 3)
            entry = {"us_per_sweep": round(us, 1), "gbps_raw": round(raw / us / 1e3, 1)}
            if op in trad:
                t_us = graph_us(torch, trad[op], 3)
                entry["trad_us_per_sweep"] = round(t_us, 1)
                entry["speedup_vs_trad"] = round(t_us / us, 2)
            row[op] = entry
        for r in res:
            rr = hz.read_result(r, ctx)
            if rr["code"] != 0:
                raise RuntimeError(f"climate sweep failed: {rr['code']}")
        out["blocks"][str(L)] = row
        del C, S, o
        torch.cuda.empty_cache()
    return out


def run_batch(args, steps, warmup, with_cpu):
    """4096 fields of log-uniform size 4 KB..64 MB (seed 7), per-field relative
    bound 1e-2/1e-3/1e-4 of the field's range, autotuned block size and grid;
    one step = one replay of the captured batch launch (compress every field
    and produce its mean and variance).  Returns a summary dict."""
    import numpy as np
    import torch

    import paper_2408_11971_amd as hz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    specs = synth.batch_specs(args.batch_count, seed=7)
    ns = [int(np.prod(sp["shape"])) for sp in specs]
    log(f"generating {len(specs)} fields ({4 * sum(ns) / 1e9:.2f} GB) on the GPU")
    arena, xs = synth.batch_arena(specs, dev)
    ebs = [sp["rel_eb"] * synth.value_range(x) for sp, x in zip(specs, xs)]
    caps = [(hz.batch_out_cap(n, 0) + 15) // 16 * 16 for n in ns]
    out_arena = torch.empty(sum(caps), dtype=torch.uint8, device=dev)
    outs, o = [], 0
    for c in caps:
        outs.append(out_arena[o:o + c])
        o += c
    torch.cuda.synchronize()
    log("planning (autotuning block sizes and grid)")
    t0 = time.perf_counter()
    b = hz.Batch([(xs[i], ebs[i], 0, outs[i]) for i in range(len(xs))], tune_grid=True)
    plan_s = time.perf_counter() - t0
    info = b.info()
    for _ in range(warmup):
        b.launch()
    torch.cuda.synchronize()
    res = b.results()
    bad = [i for i, r in enumerate(res) if r["code"] != 0]
    if bad:
        raise RuntimeError(f"batch fields failed: {bad[:10]}")
    tm = Timer(torch)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        tm.run("batch", b.launch)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    res = b.results()
    us = tm.mean_us("batch")
    raw = info["raw_bytes"]
    out_total = sum(r["out_bytes"] for r in res)
    alg = raw + out_total
    achieved = alg / us / 1e3
    blocks = {L: sum(1 for r in res if r["block"] == L) for L in (32, 64, 128)}
    cpu = cpu_baseline_batch(specs, xs, ebs, res) if with_cpu else None
    out = {"value": round(raw / us / 1e3, 1), "unit": "GB/s", "ms_per_batch": round(us / 1e3, 3),
           "ms_per_step_wall": round(1000.0 * wall / steps, 3),
           "workload": f"batch_{len(specs)}_fields_4KB-64MB_loguniform", "fields": len(specs),
           "raw_bytes": raw, "stream_bytes": out_total, "cr": round(raw / out_total, 3),
           "total_tiles": info["total_tiles"], "grid": info["grid"],
           "tile_threads": info.get("threads"), "blocks_chosen": blocks,
           "plan_seconds": round(plan_s, 2),
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": None, "kernel": "k_batch", "launches_per_step": 1,
                        "bytes_per_launch": alg, "us_per_launch": round(us, 2),
                        "events_include": "the kernel alone"},
           "cpu_baseline": cpu}
    b.close()
    del arena, out_arena, xs, outs
    torch.cuda.empty_cache()
    return out


def bench_batch(args):
    r = run_batch(args, args.steps, args.warmup, args.cpu_sample > 0)
    line = {
        "metric": "batched compress + mean/variance GB/s (raw)", "value": r["value"],
        "unit": "GB/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": r["ms_per_step_wall"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 bins (f64 quantization, int64/int128 sums)", "data": "synthetic",
        "config": {k: r[k] for k in ("workload", "fields", "raw_bytes", "stream_bytes", "cr",
                                     "total_tiles", "grid", "tile_threads", "blocks_chosen",
                                     "plan_seconds")},
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu_baseline"],
    }
    line["config"]["parallelism"] = "single_gpu"
    print(json.dumps(line), flush=True)


def cpu_baseline_batch(specs, xs, ebs, res, budget_s=15.0):
    """The oracle on a seeded random sample of the batch's fields (compress at
    the block the plan chose, then mean and variance), until ~budget_s."""
    import numpy as np

    from oracle import ref

    order = np.random.default_rng(8).permutation(len(specs))
    raw, nf, sec = 0, 0, 0.0
    for i in order:
        if sec > budget_s:
            break
        x = xs[i].cpu().numpy()
        t0 = time.perf_counter()
        c = ref.compress(x, ebs[i], res[i]["block"])
        ref.mean(c)
        ref.variance(c)
        sec += time.perf_counter() - t0
        raw += 4 * x.size
        nf += 1
    return {"value": round(raw / sec / 1e9, 4), "unit": "GB/s", "cores": 1, "kind": "oracle",
            "sample": f"{nf} fields drawn at random (seed 8) from the batch, "
                      f"{raw / 1e6:.0f} MB raw, compress + mean + variance ({sec:.1f} s)"}


SERVE_MIX = (("mean", 0.3), ("variance", 0.3), ("add", 0.2), ("negate", 0.1), ("mul", 0.1))


def run_serve(args, store_gb, seconds, rates_s, with_cpu):
    """A device store of ~store_gb of compressed fields (replicas of the
    512^3 fields at the three bounds and of climate-like 1800x3600 steps at
    blocks 32/64/128, half the bytes each), queried by open-loop Poisson
    streams (seed 8) at each offered rate for serve_seconds with the mix
    mean 30 %, variance 30 %, add 20 % (partner from the same field group),
    negate 10 %, multiply 10 % (scalar U(-2, 2), seed 9), once on the
    homomorphic path and once on the decompress-compute-recompress path.
    Returns a summary dict."""
    import numpy as np
    import torch

    import paper_2408_11971_amd as hz
    import synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    base = []  # (stream, header, group)
    log("building the store: 512^3 fields")
    for seed in (3, 4):
        x = synth.grf_3d(512, seed=seed, device=dev).view(-1)
        if seed == 3:
            rng3 = synth.value_range(x)
        for rel in RELS:
            c = hz.compress(x, rel * rng3, 32).clone()
            base.append((c, hz.header_of(c), f"grf_{rel:g}"))
        del x
    log("building the store: climate-like steps")
    for t, step in enumerate(synth.climate_steps(4)):
        xs = torch.from_numpy(step.ravel()).to(dev)
        eb = 1e-4 * synth.value_range(step)
        for L in (32, 64, 128):
            c = hz.compress(xs, eb, L).clone()
            base.append((c, hz.header_of(c), f"clim{t}_{L}"))
    target = store_gb * 1e9
    entries = []
    for kind in ("grf", "clim"):
        group = [b for b in base if b[2].startswith(kind)]
        per = sum(int(b[0].numel()) for b in group)
        reps = max(1, int(round(target / 2 / per)))
        for r in range(reps):
            for c, h, g in group:
                entries.append((c if r == 0 else c.clone(), h, g))
    torch.cuda.synchronize()
    store_bytes = sum(int(e[0].numel()) for e in entries)
    log(f"store: {len(entries)} streams, {store_bytes / 1e9:.1f} GB")
    ptr = np.array([e[0].data_ptr() for e in entries], dtype=np.uint64)
    nbytes = np.array([e[1]["total_bytes"] for e in entries], dtype=np.uint64)
    nel = np.array([e[1]["n"] for e in entries], dtype=np.uint64)
    blk = np.array([e[1]["block"] for e in entries], dtype=np.uint32)
    ebs = np.array([e[1]["eb"] for e in entries], dtype=np.float64)
    groups = {}
    for i, e in enumerate(entries):
        groups.setdefault(e[2], []).append(i)
    gid = [groups[e[2]] for e in entries]
    ops = [hz.OPS[m[0]] for m in SERVE_MIX]
    probs = np.array([m[1] for m in SERVE_MIX])
    rates = [float(r) for r in rates_s.split(",")]
    rng = np.random.default_rng(8)
    srng = np.random.default_rng(9)
    traces = []
    for lam in rates:
        gaps = rng.exponential(1.0 / lam, size=int(lam * seconds * 1.5) + 16)
        arr = np.cumsum(gaps)
        arr = arr[arr < seconds]
        k = arr.size
        ent = rng.integers(len(entries), size=k)
        op = np.array(ops)[rng.choice(len(ops), size=k, p=probs)]
        partner = np.array([gid[e][int(rng.integers(len(gid[e])))] for e in ent])
        scal = srng.uniform(-2.0, 2.0, size=k)
        traces.append((lam, arr, ent, op, partner, scal))
    pool = int(min(48e9, 24 * 4 * int(nel.max())))
    line_rows = {}
    qps_hom_top = None
    alg_hom_top = None
    for path, pname in ((hz.PATH_HOMOMORPHIC, "homomorphic"),
                        (hz.PATH_TRADITIONAL, "decompress_compute_recompress")):
        srv = hz.Server(slots=args.slots, pool_bytes=pool, keep_outputs=False)
        for lam, arr, ent, op, partner, scal in traces:
            reqs = srv.make_requests(arr.size)
            reqs["op"] = op
            reqs["path"] = path
            reqs["d_a"] = ptr[ent]
            reqs["a_bytes"] = nbytes[ent]
            is_add = op == hz.OP_ADD
            reqs["d_b"] = np.where(is_add, ptr[partner], 0)
            reqs["b_bytes"] = np.where(is_add, nbytes[partner], 0)
            reqs["n"] = nel[ent]
            reqs["block"] = blk[ent]
            reqs["eb"] = ebs[ent]
            reqs["scalar"] = scal
            reqs["tag"] = np.arange(arr.size)
            log(f"{pname}: offered {lam:.0f}/s, {arr.size} queries")
            comps, start = srv.replay(reqs, arr)
            if (comps["code"] != 0).any():
                raise RuntimeError(f"{pname}: {(comps['code'] != 0).sum()} queries failed")
            lat = comps["done_s"] - (start + arr)
            span = float(comps["done_s"].max() - start)
            qps = arr.size / span
            row = {"offered_qps": lam, "queries": int(arr.size), "achieved_qps": round(qps, 1),
                   "p50_ms": round(1e3 * float(np.percentile(lat, 50)), 4),
                   "p99_ms": round(1e3 * float(np.percentile(lat, 99)), 4),
                   "span_s": round(span, 3)}
            line_rows.setdefault(f"{lam:.0f}", {})[pname] = row
            if path == hz.PATH_HOMOMORPHIC and lam == rates[-1]:
                qps_hom_top = qps
                # algorithmic bytes of the run: the streams read and written
                out_b = np.where(op == hz.OP_MEAN, 0, np.where(op == hz.OP_VARIANCE, 0,
                                                             comps["out_bytes"]))
                rd = nbytes[ent] + np.where(is_add, nbytes[partner], 0)
                alg_hom_top = (float(rd.sum() + out_b.sum()), span)
        st = srv.stats()
        log(f"{pname}: pool peak {st['pool_peak'] / 1e9:.2f} GB, queue peak {st['queue_peak']}")
        srv.close()
    for lam, row in line_rows.items():
        h, t = row["homomorphic"], row["decompress_compute_recompress"]
        row["p99_speedup"] = round(t["p99_ms"] / h["p99_ms"], 2)
        row["qps_ratio"] = round(h["achieved_qps"] / t["achieved_qps"], 2)
    cpu = cpu_baseline_serve(entries, traces[0]) if with_cpu else None
    achieved = alg_hom_top[0] / alg_hom_top[1] / 1e9
    out = {"value": round(qps_hom_top, 1), "unit": "queries/s",
           "workload": f"serve_store_{store_bytes / 1e9:.0f}GB_poisson",
           "store_streams": len(entries), "store_bytes": store_bytes, "slots": args.slots,
           "pool_bytes": pool, "seconds_per_rate": seconds, "mix": dict(SERVE_MIX),
           "rates": line_rows,
           "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                        "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                        "traffic": None,
                        "kernel": "all kernels of the run at the highest rate (aggregate)",
                        "launches_per_step": None, "bytes_per_launch": None,
                        "us_per_launch": None, "events_include": "host clock over the whole run"},
           "cpu_baseline": cpu}
    del entries, base
    torch.cuda.empty_cache()
    return out


def bench_serve(args):
    r = run_serve(args, args.store_gb, args.serve_seconds, args.rates, args.cpu_sample > 0)
    line = {
        "metric": "serving queries/s at the highest offered rate (homomorphic), with p50/p99 "
                  "latency vs decompress-compute-recompress",
        "value": r["value"], "unit": "queries/s", "n_gpus": 1,
        "steps": len(r["rates"]), "warmup": 0, "ms_per_step": None, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None,
        "dtype": "int32 bins (f64 quantization, int64/int128 sums)", "data": "synthetic",
        "config": {k: r[k] for k in ("workload", "store_streams", "store_bytes", "slots",
                                     "pool_bytes", "seconds_per_rate", "mix")},
        "rates": r["rates"],
        "roofline": r["roofline"],
        "cpu_baseline": r["cpu_baseline"],
    }
    line["config"]["parallelism"] = "single_gpu"
    print(json.dumps(line), flush=True)


def cpu_baseline_serve(entries, trace, budget_s=15.0):
    """The oracle answering the first queries of the lowest-rate trace that
    hit climate-step streams (the 512^3 streams take the oracle seconds per
    query), until ~budget_s."""
    import numpy as np

    from oracle import ref

    lam, arr, ent, op, partner, scal = trace
    host = {}
    sec, done = 0.0, 0
    names = {0: "mean", 1: "variance", 2: "negate", 3: "add", 4: "mul"}
    for k in range(arr.size):
        if sec > budget_s:
            break
        e = int(ent[k])
        if entries[e][1]["n"] > 10_000_000:
            continue
        for i in (e, int(partner[k])):
            if i not in host:
                host[i] = entries[i][0].cpu().numpy()
        t0 = time.perf_counter()
        o = names[int(op[k])]
        if o == "mean":
            ref.mean(host[e])
        elif o == "variance":
            ref.variance(host[e])
        elif o == "negate":
            ref.negate(host[e])
        elif o == "add":
            ref.add(host[e], host[int(partner[k])])
        else:
            ref.mul(host[e], float(scal[k]))
        sec += time.perf_counter() - t0
        done += 1
    return {"value": round(done / sec, 2), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "sample": f"{done} queries of the {lam:.0f}/s trace on climate-step streams "
                      f"({sec:.1f} s)"}


KERNEL_OF = {"compress": "k_compress<1>", "compress_b": "k_compress<1>",
             "decompress": "k_decode<2>", "mean": "k_decode<0>",
             "variance": "k_decode<1>", "negate": "k_negate", "add": "k_add", "mul": "k_mul"}
PREPASS_NOTE = {k: "the kernel and its width pre-pass k_widths (one launch before it)"
                for k in ("k_decode<0>", "k_decode<1>", "k_decode<2>", "k_mul")}
PREPASS_NOTE["k_add"] = "the kernel and the two width pre-passes of its inputs"
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "grf512_ops_pmc_traffic.json")


def measured_traffic(kname, ls):
    """HBM bytes per launch of `kname` from the committed PMC summary, averaged
    over the same launches; None when kernels.hip changed since it was taken."""
    import hashlib
    try:
        t = json.load(open(TRAFFIC_FILE))
    except (OSError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2408_11971_amd", "csrc", "kernels.hip")
    if hashlib.sha256(open(src, "rb").read()).hexdigest() != t.get("kernels_hip_sha256"):
        return None
    vals = []
    for _, _, rel, op in ls:
        v = t["bytes"].get(f"rel{rel:g}/{op}")
        if v is None:
            return None
        vals.append(v)
    return round(sum(vals) / len(vals))


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def oracle_pass(a, b, ebs):
    """The 8 ops of a step (at every bound) by the oracle on host arrays;
    returns raw-equivalent bytes processed."""
    from oracle import ref

    for eb in ebs:
        ca = ref.compress(a, eb, BLOCK)
        cb = ref.compress(b, eb, BLOCK)
        ref.mean(ca)
        ref.decompress(cb)
        ref.variance(ca)
        ref.negate(cb)
        ref.add(ca, cb)
        ref.mul(ca, SCALAR)
    return 4 * a.size * 9 * len(ebs)


def cpu_baseline(A, B, ebs, n, threads=None):
    """The oracle (unchanged, single-threaded code) on the first n elements of
    both fields: once on one thread, then on all host cores (up to
    --cpu-threads), each thread running the same op sequence on its own
    block-aligned slice.  The oracle is C called through ctypes, which
    releases the interpreter lock, so the threads run in parallel."""
    from concurrent.futures import ThreadPoolExecutor

    a = A[:n].cpu().numpy()
    b = B[:n].cpu().numpy()
    log(f"timing the CPU oracle on {n} elements per field, 1 thread")
    t0 = time.perf_counter()
    raw = oracle_pass(a, b, ebs)
    sec1 = time.perf_counter() - t0
    avail = len(os.sched_getaffinity(0))
    p = max(1, min(threads or avail, avail))
    per = (n // p + BLOCK - 1) // BLOCK * BLOCK
    parts = [(a[k:k + per], b[k:k + per]) for k in range(0, n, per)]
    log(f"timing the CPU oracle on {len(parts)} threads")
    t0 = time.perf_counter()
    with ThreadPoolExecutor(max_workers=len(parts)) as ex:
        rawp = sum(ex.map(lambda ab: oracle_pass(ab[0], ab[1], ebs), parts))
    secp = time.perf_counter() - t0
    return {"value": round(rawp / secp / 1e9, 4), "unit": "GB/s", "cores": len(parts),
            "kind": "oracle",
            "sample": f"first {n} elements of each 512^3 field, the 8 ops of a step at all 3 "
                      f"bounds, split into {len(parts)} block-aligned slices run on one thread "
                      f"each ({secp:.1f} s)",
            "one_core": {"value": round(raw / sec1 / 1e9, 4), "cores": 1,
                         "seconds": round(sec1, 2)},
            "host": {"nproc": os.cpu_count(), "affinity": avail, "cpu_model": cpu_model()}}


if __name__ == "__main__":
    main()
