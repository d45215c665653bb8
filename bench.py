"""Benchmark of the exact GF(p) dot-product path on one MI355X.

One step = the batched dot products of the 4096-pair workload (lengths
log-uniform in [1e3, 1e6], seed 2) in its three batches: p = 65521 classical
residues with delayed reduction, p = 2^31-1 in Montgomery form (B = 2^32), and
p = 4294967291 reduced after every term.  Inputs are generated on the device
before the timed region; `value` is the whole step's algorithmic traffic
(8 bytes per term) divided by its time.

Prints ONE JSON line (see the keys below).  Extra measurements of the other
workloads (single dot, fp64/Zech, plain one-launch-per-pair) go under
"extras" and are not part of `value`.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402
import torch  # noqa: E402

METRIC = "exact GF(p) dot GB/s & Gelem/s, fgemm_modp GOPS; batched/served vs plain, p99"
HBM_PEAK_GBS = 8000.0
BATCHES = [  # (p, representation, algorithm, label)
    (65521, "zpz", "delayed", "p=65521 zpz delayed"),
    (2147483647, "mont", "delayed", "p=2^31-1 montgomery B=2^32"),
    (4294967291, "zpz", "perterm", "p=4294967291 zpz per-term"),
]
SEED = 2


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def lengths_config2():
    import synth
    return synth.log_uniform_lengths(SEED, 0, 4096, 3.0, 6.0)


class Batch:
    """Device-resident inputs of one batch: instance k is x = stream 2k,
    y = stream 2k+1 of the shared generator, each 16-byte aligned."""

    def __init__(self, fd, p, rep, algo, ns, dtype, seed=SEED):
        import synth
        self.p, self.rep, self.algo, self.ns = p, rep, algo, ns
        self.F = fd.Field(p, rep)
        esz = torch.tensor([], dtype=dtype).element_size()
        align = max(1, 16 // esz)
        pad = [(int(n) + align - 1) // align * align for n in ns]
        self.offs = np.concatenate([[0], np.cumsum(pad)])
        tot = int(self.offs[-1])
        self.X = torch.empty(tot, dtype=dtype, device="cuda")
        self.Y = torch.empty(tot, dtype=dtype, device="cuda")
        m, lo = (p, 0)
        for k, n in enumerate(ns):
            o = int(self.offs[k])
            synth.fill_device(self.X[o:o + int(n)], seed, 2 * k, m, lo)
            synth.fill_device(self.Y[o:o + int(n)], seed, 2 * k + 1, m, lo)
        xs = [self.X[int(self.offs[k]):int(self.offs[k]) + int(n)] for k, n in enumerate(ns)]
        ys = [self.Y[int(self.offs[k]):int(self.offs[k]) + int(n)] for k, n in enumerate(ns)]
        self.xs, self.ys = xs, ys
        self.desc = fd.Field.make_desc(xs, ys)
        self.out = torch.empty(len(ns), dtype=dtype, device="cuda")
        self.bytes = int(np.sum(ns)) * 2 * esz
        self.terms = int(np.sum(ns))

    def run(self):
        self.F.dot_many(self.desc, out=self.out, algo=self.algo)


def cpu_baseline(batches, max_instances=384):
    """The oracle (as it stands) on the first instances of every batch,
    regenerated on the host from the same seeds."""
    import oracle
    import synth
    terms = 0
    nbytes = 0
    elapsed = 0.0
    for b in batches:
        ns = b.ns[:max_instances]
        xs = [synth.uniform_int(SEED, 2 * k, int(n), b.p).astype(np.uint32) for k, n in enumerate(ns)]
        ys = [synth.uniform_int(SEED, 2 * k + 1, int(n), b.p).astype(np.uint32) for k, n in enumerate(ns)]
        t0 = time.perf_counter()
        res = oracle.dot_many(b.p, b.rep, xs, ys)
        elapsed += time.perf_counter() - t0
        gpu = b.out[:len(ns)].cpu().numpy()
        if res.tobytes() != gpu.tobytes():
            raise SystemExit(f"GPU and oracle disagree on batch p={b.p}")
        terms += int(np.sum(ns))
        nbytes += int(np.sum(ns)) * 8
    cores = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    return {"value": round(nbytes / elapsed / 1e9, 4), "unit": "GB/s", "cores": cores,
            "kind": "oracle", "gelem_per_s": round(terms / elapsed / 1e9, 4),
            "sample": f"first {max_instances} instances of each of the 3 batches "
                      f"({terms} terms, {nbytes / 1e9:.2f} GB), per-term __int128 reduction, "
                      f"OpenMP over instances; {elapsed:.2f} s"}


def time_events(fn, reps):
    s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    s.record()
    for _ in range(reps):
        fn()
    e.record()
    torch.cuda.synchronize()
    return s.elapsed_time(e) / 1e3 / reps


def extras_plain(fd, b, limit=4096):
    """One fdot_modp launch per pair, same stream, same kernels."""
    outs = torch.empty(len(b.ns), dtype=b.out.dtype, device="cuda")

    def plain():
        for k in range(min(limit, len(b.ns))):
            b.F.dot(b.xs[k], b.ys[k], out=outs[k:k + 1], algo=b.algo)

    plain()
    t = time_events(plain, 1)
    tb = time_events(b.run, 3)
    if outs.cpu().numpy().tobytes() != b.out.cpu().numpy().tobytes():
        raise SystemExit("plain and batched results differ")
    return {"batch": f"p={b.p} {b.rep} {b.algo}", "plain_ms": round(t * 1e3, 3),
            "batched_ms": round(tb * 1e3, 3), "speedup": round(t / tb, 2)}


def graph_time(fd, fn, reps=20):
    """Seconds per replay of a HIP graph holding the launches made by fn():
    device time including launch gaps, without host-side call overhead."""
    s = torch.cuda.Stream()
    fd.workspace_reserve(4096, stream=s)
    with torch.cuda.stream(s):
        fn()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        fn()
    g.replay()
    torch.cuda.synchronize()
    return time_events(g.replay, reps)


def extras_single(fd):
    """Single dot, p = 32749, n = 1e6: 64 dots on 64 distinct buffer pairs
    (512 MB, above the 256 MB last-level cache) replayed from one HIP graph;
    reports device time per dot, cold, and the same dot repeated (hot)."""
    import synth
    p, n, pairs = 32749, 1_000_000, 64
    F = fd.Field(p, "zpz")
    X = torch.empty((pairs, n), dtype=torch.uint32, device="cuda")
    Y = torch.empty((pairs, n), dtype=torch.uint32, device="cuda")
    for i in range(pairs):
        synth.fill_device(X[i], 1, 2 * i, p)
        synth.fill_device(Y[i], 1, 2 * i + 1, p)
    out = torch.empty(pairs, dtype=torch.uint32, device="cuda")

    def cold():
        for i in range(pairs):
            F.dot(X[i], Y[i], out=out[i:i + 1])

    def hot():
        for i in range(pairs):
            F.dot(X[0], Y[0], out=out[i:i + 1])
    tc = graph_time(fd, cold) / pairs
    th = graph_time(fd, hot) / pairs
    eager = time_events(lambda: F.dot(X[0], Y[0], out=out[:1]), 200)
    return {"workload": "single dot p=32749 n=1e6 zpz", "graph_hot_us": round(th * 1e6, 2),
            "graph_cold_us": round(tc * 1e6, 2), "cold_GBps": round(8 * n / tc / 1e9, 1),
            "cold_gelem_per_s": round(n / tc / 1e9, 2),
            "eager_call_us": round(eager * 1e6, 2)}


def extras_config3(fd):
    """1024 pairs of length 4e6: fp64 residues mod 2^26-5 and Zech codes
    mod 32749, one batched call each."""
    out = {}
    ns = np.full(1024, 4_000_000, dtype=np.int64)
    for p, rep, algo, dt, label in [(67108859, "fp64", "delayed", torch.float64, "fp64 p=2^26-5"),
                                    (32749, "zech", "zech_exp", torch.uint16, "zech p=32749 exp"),
                                    (32749, "zech", "zech_tplus1", torch.uint16,
                                     "zech p=32749 plus-one")]:
        b = Batch(fd, p, rep, algo, ns, dt, seed=3)
        b.run()
        t = time_events(b.run, 3)
        out[label] = {"GBps": round(b.bytes / t / 1e9, 1), "gelem_per_s": round(b.terms / t / 1e9, 2),
                      "ms": round(t * 1e3, 3)}
        del b
        torch.cuda.empty_cache()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--extras", choices=["all", "none"], default="all")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    import paper_cs_0404008_amd as fd
    torch.cuda.set_device(0)
    ns = lengths_config2()
    log(f"config 2: {len(ns)} pairs, {int(ns.sum())} terms per batch")
    batches = [Batch(fd, p, rep, algo, ns, torch.uint32) for p, rep, algo, _ in BATCHES]
    torch.cuda.synchronize()
    for _ in range(args.warmup):
        for b in batches:
            b.run()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in batches]
    per_batch = [0.0 for _ in batches]
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for i, b in enumerate(batches):
            ev[i][0].record()
            b.run()
            ev[i][1].record()
        torch.cuda.synchronize()
        for i in range(len(batches)):
            per_batch[i] += ev[i][0].elapsed_time(ev[i][1]) / 1e3
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    step_gpu = sum(per_batch) / args.steps
    total_bytes = sum(b.bytes for b in batches)
    total_terms = sum(b.terms for b in batches)
    value = total_bytes / step_gpu / 1e9
    dom = max(range(len(batches)), key=lambda i: per_batch[i])
    dom_t = per_batch[dom] / args.steps
    achieved = batches[dom].bytes / dom_t / 1e9
    result = {
        "metric": METRIC, "value": round(value, 2), "unit": "GB/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(step_gpu * 1e3, 4), "wall_ms_per_step": round(wall / args.steps * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u32",
        "data": "synthetic (SplitMix64, seed 2)",
        "config": {"workload": "batched exact dot, 4096 pairs, n log-uniform [1e3,1e6]",
                   "batches": [lab for _, _, _, lab in BATCHES],
                   "terms_per_batch": int(ns.sum()), "parallelism": "1 GPU"},
        "gelem_per_s": round(total_terms / step_gpu / 1e9, 3),
        "per_batch_ms": {BATCHES[i][3]: round(per_batch[i] / args.steps * 1e3, 4)
                         for i in range(len(batches))},
        "roofline": {"bound": "hbm", "kernel": f"dot_kernel batched, {BATCHES[dom][3]}",
                     "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        result["cpu_baseline"] = cpu_baseline(batches)
    if args.extras == "all":
        extras = {}
        log("extras: plain vs batched ...")
        extras["plain_vs_batched"] = extras_plain(fd, batches[0])
        del batches
        torch.cuda.empty_cache()
        log("extras: single dot ...")
        extras["single_dot"] = extras_single(fd)
        torch.cuda.empty_cache()
        log("extras: fp64 / zech ...")
        extras["config3"] = extras_config3(fd)
        result["extras"] = extras
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
