"""Autotuner for the launch parameters and accumulation schedules.

Every schedule and launch shape of the library computes the same exact
result, so tuning is a pure speed question: each candidate setting is timed
on the device (median of several timed repetitions, HIP events on the
current stream) and its output is compared bit for bit with the output of
the current setting before it may win.  The winners are written as
``key=value`` lines, the format the library reads at start-up from the file
named by the FDOT_TUNE_FILE environment variable; ``apply`` sets them in the
running process.

What is tuned:

* the single dot product: smallest chunk (``min_chunk.<rep>``) and the
  number of first-level combination words (``spread.<rep>``);
* the batched dot product of a given batch: bytes per range
  (``many.range.<rep>``), workgroups per CU (``wg_per_cu.<rep>``) and
  wavefronts per range (``many.slices.<rep>``);
* the schedule that ``algo="auto"`` picks where several apply: per-term
  reduction against division on demand and the block-overflow hybrid for
  classical residues of primes with lambda < 2 (Sec. 2.1, 3.3, 3.4), delayed
  blocks against division on demand and the hybrid for Montgomery residues
  (Sec. 3.2.1, 3.3, 3.4), value table against Zech addition for discrete
  logarithms (Sec. 2.4);
* the matrix-core tiling of ``fgemm_modp`` (``gemm.i8.tile``,
  ``gemm.f64.waves``);
* the size above which ``fgemm_modp`` switches from the FP64 matrix cores to
  int8 digit products, per digit count (``gemm.split.min_work.d<D>``), from
  square products timed on both paths (``tune_split``);
* the representation that ``fdot_choose_rep`` returns for each prime size
  (``auto.rep.b<bits>``): the Conclusion's install-time choice of the
  switching thresholds between representations, made here by timing the
  streaming dot in every representation that admits the largest prime of
  each bit length (``rep_sweep``).

Command line: ``python -m paper_cs_0404008_amd.autotune --out tune.txt``
tunes on synthetic inputs of the benchmark's shapes (``--small`` for a quick
run) and writes the file.
"""
from __future__ import annotations

import argparse
import itertools
import statistics
import sys

import numpy as np
import torch

from . import ALGOS, REPS as ALGOS_REP, Field, tune_get, tune_set

REP_KEYS = ("zpz", "mont", "fp64", "zech", "centred")


def _time(fn, reps: int = 3, inner: int = 3) -> float:
    """Median over reps of the mean device time of `inner` calls (seconds)."""
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        s, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        s.record()
        for _ in range(inner):
            fn()
        e.record()
        torch.cuda.synchronize()
        out.append(s.elapsed_time(e) / 1e3 / inner)
    return statistics.median(out)


class _Settings:
    """Temporarily applied tuning keys (restored on exit)."""

    def __init__(self, settings: dict):
        self.settings = settings
        self.saved = {}

    def __enter__(self):
        for k, v in self.settings.items():
            self.saved[k] = tune_get(k)
            tune_set(k, v)
        return self

    def __exit__(self, *exc):
        for k, v in self.saved.items():
            tune_set(k, v)


def _search(run, read, candidates, reps=3):
    """Times run() under every candidate setting; a candidate whose output
    (read()) differs from the first one's is an error.  Returns (best
    settings, table of (settings, seconds))."""
    ref = None
    table = []
    for cand in candidates:
        with _Settings(cand):
            run()
            torch.cuda.synchronize()
            got = read()
            if ref is None:
                ref = got
            elif not np.array_equal(got, ref):
                raise RuntimeError(f"setting {cand} changed the result")
            table.append((cand, _time(run, reps)))
    best = min(table, key=lambda t: t[1])[0]
    return best, table


def tune_batched(field: Field, desc: torch.Tensor, algo: str = "auto",
                 ranges=(262144, 524288, 1048576), wg_per_cu=(1, 2), slices=(1, 2),
                 reps: int = 3):
    """Launch shape of fdot_modp_many for this batch."""
    rep = field.rep
    out = torch.empty(desc.shape[0], dtype=field.dtype, device=desc.device)
    cands = [{f"many.range.{rep}": r, f"wg_per_cu.{rep}": w, f"many.slices.{rep}": s}
             for r, w, s in itertools.product(ranges, wg_per_cu, slices)]
    return _search(lambda: field.dot_many(desc, out=out, algo=algo),
                   lambda: out.cpu().numpy().copy(), cands, reps)


def tune_single(field: Field, x: torch.Tensor, y: torch.Tensor,
                min_chunk=(256, 512, 1024, 2048, 4096), spread=(1, 8, 32, 64), reps: int = 3):
    """Launch shape of one fdot_modp call (a dot short enough to be bound by
    latency and by the combination of its units rather than by HBM):
    smallest chunk in elements (``min_chunk.<rep>``) and first-level
    combination words (``spread.<rep>``)."""
    rep = field.rep
    out = torch.empty(1, dtype=field.dtype, device=x.device)
    cands = [{f"min_chunk.{rep}": m, f"spread.{rep}": s}
             for m, s in itertools.product(min_chunk, spread)]
    return _search(lambda: field.dot(x, y, out=out), lambda: out.cpu().numpy().copy(), cands,
                   reps)


def tune_schedule(field: Field, desc: torch.Tensor, reps: int = 3):
    """The schedule that algo="auto" uses for this field's representation,
    where there is a choice; returns ({key: algo code}, table) or ({}, [])."""
    rep = field.rep
    info = field.info
    if rep == "zpz" and info["lambda_u64"] < 2:
        key, algos = "auto.zpz.lambda1", ("perterm", "overflow", "hybrid")
    elif rep == "mont":
        key, algos = "auto.mont", ("delayed", "overflow", "hybrid")
    elif rep == "zech":
        key, algos = "auto.zech", ("zech_exp", "zech_tplus1")
    else:
        return {}, []
    out = torch.empty(desc.shape[0], dtype=field.dtype, device=desc.device)
    ref = None
    table = []
    for a in algos:
        field.dot_many(desc, out=out, algo=a)
        torch.cuda.synchronize()
        got = out.cpu().numpy().copy()
        if ref is None:
            ref = got
        elif not np.array_equal(got, ref):
            raise RuntimeError(f"schedule {a} changed the result")
        table.append(({key: ALGOS[a]}, _time(lambda: field.dot_many(desc, out=out, algo=a), reps)))
    return min(table, key=lambda t: t[1])[0], table


def tune_gemm(field: Field, A: torch.Tensor, B: torch.Tensor, reps: int = 3):
    """Matrix-core tiling of fgemm_modp for this representation and shape."""
    C = torch.empty((A.shape[0], B.shape[1]), dtype=field.dtype, device=A.device)
    if field.rep == "centred":
        cands = [{"gemm.i8.tile": t} for t in (8, 9, 7, 5, 6, 4, 2)]
    elif field.rep in ("fp64", "zpz", "mont"):
        cands = [{"gemm.f64.waves": w} for w in (8, 4, 16)]
    else:
        return {}, []
    return _search(lambda: field.gemm(A, B, out=C), lambda: C.cpu().numpy().copy(), cands, reps)


def tune_split(cases=((32749, "zpz", torch.uint32), (1048573, "fp64", torch.float64),
                       (67108859, "fp64", torch.float64)),
               sizes=(256, 512, 768, 1024, 1536, 2048, 3072, 4096), reps: int = 3):
    """Crossover of the FP64 matrix cores and the int8 digit products, per
    digit count D: the smallest n such that the digit products are at least
    as fast at every timed size from n up; writes n^3 as
    gemm.split.min_work.d<D>.  Both paths must give the same bits."""
    from synth import fill_device
    settings, table = {}, []
    for p, rep, dt in cases:
        F = Field(p, rep)
        h = (p - 1) // 2
        d = 1 if h <= 127 else 2 if h <= 32639 else 3 if h <= 8355711 else 4
        faster = []
        for n in sizes:
            A = torch.empty((n, n), dtype=dt, device="cuda")
            B = torch.empty((n, n), dtype=dt, device="cuda")
            fill_device(A, 12, 0, p, 0)
            fill_device(B, 12, 1, p, 0)
            C = torch.empty((n, n), dtype=dt, device="cuda")
            times = {}
            outs = {}
            for path, kv in (("fp64", {"gemm.split.disable": 1}), ("digits", {"gemm.split.min_work": 1})):
                with _Settings(kv):
                    F.gemm(A, B, out=C)
                    torch.cuda.synchronize()
                    outs[path] = C.cpu().numpy().copy()
                    times[path] = _time(lambda: F.gemm(A, B, out=C), reps)
            if not np.array_equal(outs["fp64"], outs["digits"]):
                raise RuntimeError(f"digit products changed the result at p={p} n={n}")
            faster.append(times["digits"] <= times["fp64"])
            table.append((p, rep, d, n, times["fp64"], times["digits"]))
            del A, B, C
            torch.cuda.empty_cache()
        cross = None
        for i in range(len(sizes)):
            if all(faster[i:]):
                cross = sizes[i]
                break
        if cross is not None:
            settings[f"gemm.split.min_work.d{d}"] = cross ** 3
    return settings, table


def _is_prime(n: int) -> bool:
    if n < 2:
        return False
    for q in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):
        if n % q == 0:
            return n == q
    d, r = n - 1, 0
    while d % 2 == 0:
        d, r = d // 2, r + 1
    for a in (2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37):  # deterministic below 3.3e24
        x = pow(a, d, n)
        if x in (1, n - 1):
            continue
        for _ in range(r - 1):
            x = x * x % n
            if x == n - 1:
                break
        else:
            return False
    return True


def largest_prime_below(x: int) -> int:
    q = x - 1
    while not _is_prime(q):
        q -= 1
    return q


def rep_sweep(primes, bytes_per_call: int = 1 << 30, reps: int = 3):
    """Streaming dot throughput of every representation that admits each
    prime: rows (p, rep, n, seconds per call, Gelem/s, GB/s).  Each call
    reads bytes_per_call bytes (n = bytes_per_call / (2 * element size)), so
    the operands do not stay in the last-level cache between calls."""
    from synth import fill_device
    rows = []
    for p in primes:
        for rep in REP_KEYS:
            try:
                F = Field(p, rep)
            except Exception:  # the representation does not admit p
                continue
            n = bytes_per_call // (2 * F.info["elem_bytes"])
            m, lo = (p, 0) if rep != "centred" else (p, -((p - 1) // 2))
            x = torch.empty(n, dtype=F.dtype, device="cuda")
            y = torch.empty(n, dtype=F.dtype, device="cuda")
            fill_device(x, 9, 0, m, lo)
            fill_device(y, 9, 1, m, lo)
            out = torch.empty(1, dtype=F.dtype, device="cuda")
            t = _time(lambda: F.dot(x, y, out=out), reps)
            rows.append({"p": p, "rep": rep, "n": n, "s": t, "gelem_per_s": n / t / 1e9,
                         "GBps": 2 * n * F.info["elem_bytes"] / t / 1e9})
            del x, y, out, F
            torch.cuda.empty_cache()
    return rows


def tune_representation(bits=range(8, 33), bytes_per_call: int = 1 << 30, reps: int = 3):
    """auto.rep.b<bits> for each bit length: the fastest representation
    (elements per second) for the largest prime of that length."""
    primes = [largest_prime_below(1 << b) for b in bits]
    rows = rep_sweep(primes, bytes_per_call, reps)
    settings = {}
    for b, p in zip(bits, primes):
        mine = [r for r in rows if r["p"] == p]
        if mine:
            best = max(mine, key=lambda r: r["gelem_per_s"])
            settings[f"auto.rep.b{b}"] = ALGOS_REP[best["rep"]]
    return settings, rows


def apply(settings: dict) -> None:
    for k, v in settings.items():
        tune_set(k, v)


def write(path: str, settings: dict, comment: str = "") -> None:
    with open(path, "w") as fh:
        fh.write("# launch parameters chosen by paper_cs_0404008_amd.autotune\n")
        if comment:
            for line in comment.splitlines():
                fh.write(f"# {line}\n")
        for k in sorted(settings):
            fh.write(f"{k}={int(settings[k])}\n")


def read(path: str) -> dict:
    """Parses a file in the library's key=value format."""
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.startswith("#") or "=" not in line:
                continue
            k, v = line.split("=", 1)
            out[k.strip()] = int(v.strip())
    return out


def _batch(field: Field, ns, seed: int):
    from synth import fill_device  # the seeded input generator of this repository
    dt = field.dtype
    xs, ys = [], []
    m, lo = (field.p, 0) if field.rep != "centred" else (field.p, -((field.p - 1) // 2))
    for k, n in enumerate(ns):
        x = torch.empty(int(n), dtype=dt, device="cuda")
        y = torch.empty(int(n), dtype=dt, device="cuda")
        fill_device(x, seed, 2 * k, m, lo)
        fill_device(y, seed, 2 * k + 1, m, lo)
        xs.append(x)
        ys.append(y)
    return xs, ys, Field.make_desc(xs, ys)


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--out", required=True, help="tuning file to write (key=value lines)")
    ap.add_argument("--small", action="store_true", help="small shapes (quick check)")
    ap.add_argument("--no-gemm", action="store_true")
    ap.add_argument("--no-rep", action="store_true", help="skip the representation sweep")
    args = ap.parse_args(argv)
    import synth
    torch.cuda.set_device(0)
    count, lo_exp, hi_exp = (256, 3.0, 5.0) if args.small else (4096, 3.0, 6.0)
    ns = synth.log_uniform_lengths(2, 0, count, lo_exp, hi_exp)
    settings, log = {}, []
    for p, rep in [(65521, "zpz"), (2147483647, "mont"), (4294967291, "zpz"), (67108859, "fp64"),
                   (32749, "zech")]:
        F = Field(p, rep)
        xs, ys, desc = _batch(F, ns, 2)
        best, table = tune_batched(F, desc)
        settings.update(best)
        log.append(f"batched p={p} {rep}: " + ", ".join(
            f"{c} {t * 1e3:.3f} ms" for c, t in sorted(table, key=lambda x: x[1])[:3]))
        with _Settings(best):
            sched, stable = tune_schedule(F, desc)
        settings.update(sched)
        if stable:
            log.append(f"schedule p={p} {rep}: " + ", ".join(
                f"{c} {t * 1e3:.3f} ms" for c, t in stable))
        del xs, ys, desc
        n1 = 1 << 16 if args.small else 1_000_000
        x, y = (torch.empty(n1, dtype=F.dtype, device="cuda") for _ in range(2))
        m, lo = (p, 0) if rep != "centred" else (p, -((p - 1) // 2))
        synth.fill_device(x, 1, 0, m, lo)
        synth.fill_device(y, 1, 1, m, lo)
        best, table = tune_single(F, x, y)
        settings.update(best)
        log.append(f"single p={p} {rep} n={n1}: " + ", ".join(
            f"{c} {t * 1e6:.2f} us" for c, t in sorted(table, key=lambda x: x[1])[:3]))
        del x, y
        torch.cuda.empty_cache()
    if not args.no_gemm:
        n = 1024 if args.small else 8192
        for p, rep, dt in [(251, "centred", torch.int8), (1048573, "fp64", torch.float64)]:
            F = Field(p, rep)
            from synth import fill_device
            A = torch.empty((n, n), dtype=dt, device="cuda")
            B = torch.empty((n, n // 2), dtype=dt, device="cuda")
            m, lo = (p, 0) if rep != "centred" else (p, -((p - 1) // 2))
            fill_device(A, 4, 0, m, lo)
            fill_device(B, 4, 1, m, lo)
            best, table = tune_gemm(F, A, B)
            settings.update(best)
            log.append(f"fgemm p={p} {rep}: " + ", ".join(
                f"{c} {t * 1e3:.3f} ms" for c, t in sorted(table, key=lambda x: x[1])))
            del A, B
            torch.cuda.empty_cache()
        ssettings, stable = tune_split(sizes=(256, 512, 1024) if args.small else
                                       (256, 512, 768, 1024, 1536, 2048, 3072, 4096))
        settings.update(ssettings)
        for p, rep, d, n, tf, tdig in stable:
            log.append(f"split p={p} {rep} D={d} n={n}: fp64 {tf * 1e3:.3f} ms, digits {tdig * 1e3:.3f} ms")
    if not args.no_rep:
        bits = range(8, 33, 4) if args.small else range(8, 33)
        rsettings, rows = tune_representation(bits, (1 << 26) if args.small else (1 << 30))
        settings.update(rsettings)
        for r in rows:
            log.append(f"rep p={r['p']} {r['rep']}: {r['gelem_per_s']:.1f} Gelem/s")
    write(args.out, settings, "\n".join(log))
    print("\n".join(log))
    print(f"wrote {len(settings)} settings to {args.out}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
