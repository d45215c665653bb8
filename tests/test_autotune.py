"""The autotuner: its tuning file round-trips through the library's
FDOT_TUNE_FILE reader (CPU), and on the GPU every candidate it times gives
the default's result bit for bit and the chosen settings keep it."""
import os
import subprocess
import sys

import numpy as np
import pytest

from tests.conftest import ROOT

fd = pytest.importorskip("paper_cs_0404008_amd")
from paper_cs_0404008_amd import autotune  # noqa: E402


def test_tune_file_roundtrip(tmp_path):
    path = str(tmp_path / "tune.txt")
    settings = {"many.range.zpz": 524288, "wg_per_cu.zpz": 2, "auto.mont": 6, "gemm.i8.tile": 7}
    autotune.write(path, settings, "a comment\nover two lines")
    assert autotune.read(path) == settings
    # a fresh process picks the file up through FDOT_TUNE_FILE
    code = ("import paper_cs_0404008_amd as fd, json; "
            "print(json.dumps({k: fd.tune_get(k) for k in %r}))" % sorted(settings))
    env = dict(os.environ, FDOT_TUNE_FILE=path, PYTHONPATH=ROOT)
    out = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                         cwd=ROOT, timeout=300)
    assert out.returncode == 0, out.stderr
    import json
    assert json.loads(out.stdout.strip().splitlines()[-1]) == settings


@pytest.mark.gpu
def test_autotune_small_workloads():
    import torch
    import synth
    torch.cuda.set_device(0)
    ns = synth.log_uniform_lengths(7, 0, 64, 2.0, 5.0)
    for p, rep in [(65521, "zpz"), (2147483647, "mont"), (4294967291, "zpz"), (32749, "zech")]:
        F = fd.Field(p, rep)
        xs, ys, desc = autotune._batch(F, ns, 7)
        want = F.dot_many(desc).cpu().numpy()
        best, table = autotune.tune_batched(F, desc, ranges=(4096, 524288), wg_per_cu=(1, 2),
                                            slices=(1, 2), reps=1)
        assert len(table) == 8 and set(best) == {f"many.range.{rep}", f"wg_per_cu.{rep}",
                                                   f"many.slices.{rep}"}
        sched, stable = autotune.tune_schedule(F, desc, reps=1)
        assert (rep == "zpz" and p == 65521) or len(stable) >= 2
        old = {k: fd.tune_get(k) for k in list(best) + list(sched)}
        try:
            autotune.apply({**best, **sched})
            assert np.array_equal(F.dot_many(desc).cpu().numpy(), want)
        finally:
            autotune.apply(old)
    F = fd.Field(32749, "zpz")
    x = synth.uniform_int(7, 0, 100003, 32749).astype(np.uint32)
    y = synth.uniform_int(7, 1, 100003, 32749).astype(np.uint32)
    xd, yd = torch.from_numpy(x).cuda(), torch.from_numpy(y).cuda()
    best, table = autotune.tune_single(F, xd, yd, min_chunk=(256, 4096), spread=(1, 32), reps=1)
    assert len(table) == 4 and set(best) == {"min_chunk.zpz", "spread.zpz"}
    import oracle
    assert int(F.dot(xd, yd).cpu().numpy()[0]) == oracle.dot(32749, "zpz", x, y)
    for p, rep, dt in [(251, "centred", torch.int8), (1048573, "fp64", torch.float64)]:
        F = fd.Field(p, rep)
        m, lo = (p, 0) if rep != "centred" else (p, -((p - 1) // 2))
        A = torch.empty((512, 1024), dtype=dt, device="cuda")
        B = torch.empty((1024, 384), dtype=dt, device="cuda")
        synth.fill_device(A, 8, 0, m, lo)
        synth.fill_device(B, 8, 1, m, lo)
        best, table = autotune.tune_gemm(F, A, B, reps=1)
        assert len(table) >= 3 and len(best) == 1
    settings, table = autotune.tune_split(sizes=(256, 512), reps=1)
    assert len(table) == 6 and all(k.startswith("gemm.split.min_work.d") for k in settings)
