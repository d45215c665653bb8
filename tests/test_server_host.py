"""The request server's scheduling logic without a GPU (fake-device mode):
admission by footprint and slots, arrival order, batching, back-pressure,
rejection of requests that can never fit, exclusive long requests, and the
replay load generator."""
import time

import numpy as np
import pytest

fd = pytest.importorskip("paper_cs_0404008_amd")

F1 = fd.Field(32749, "zpz", host_only=True)
F2 = fd.Field(67108859, "fp64", host_only=True)
F3 = fd.Field(251, "centred", host_only=True)
FAKE = 1 << 20  # nonzero fake device addresses (never dereferenced)


def dot(F, n, fp=0):
    return fd.make_request("dot", F, FAKE, FAKE, FAKE, n=n, footprint=fp)


def test_host_only_field_refuses_compute():
    import ctypes
    L = fd.lib()
    assert L.fdot_modp(F1.handle, ctypes.c_void_p(FAKE), ctypes.c_void_p(FAKE), 10,
                       ctypes.c_void_p(FAKE), None) == -4
    assert F1.info["lambda_u64"] == 17200859919


def test_everything_completes_and_counts():
    srv = fd.Server(fake_device=True)
    tickets = [srv.submit(dot(F1, 1000 + i)) for i in range(200)]
    tickets += [srv.submit(fd.make_request("gemv", F2, FAKE, FAKE, FAKE, m=100, n=100))
                for _ in range(20)]
    tickets += [srv.submit(fd.make_request("gemm", F3, FAKE, FAKE, FAKE, m=64, n=64, k=64))
                for _ in range(5)]
    srv.drain(10000)
    for t in tickets:
        done, tm = srv.poll(t)
        assert done and tm.status == 0
        assert tm.submit_ns <= tm.admit_ns <= tm.launch_ns <= tm.done_ns
    st = srv.stats()
    assert st["submitted"] == st["completed"] == len(tickets)
    srv.close()


def test_budget_and_slots_are_respected():
    budget = 10_000
    srv = fd.Server(fake_device=True, hbm_budget=budget, max_inflight=3)
    reqs = [dot(F1, 10, fp=int(fp)) for fp in np.random.default_rng(1).integers(1000, 5000, 300)]
    for r in reqs:
        srv.submit(r)
    srv.drain(20000)
    st = srv.stats()
    assert st["peak_footprint"] <= budget
    assert st["peak_inflight"] <= 3
    assert st["completed"] == 300


def test_admission_keeps_arrival_order():
    srv = fd.Server(fake_device=True, hbm_budget=6000, max_inflight=4)
    fps = np.random.default_rng(2).integers(500, 5000, 200)
    tickets = [srv.submit(dot(F1, 10, fp=int(f))) for f in fps]
    srv.drain(20000)
    admits = [srv.poll(t)[1].admit_ns for t in tickets]
    assert all(a <= b for a, b in zip(admits, admits[1:]))


def test_batching_and_plain_mode():
    srv = fd.Server(fake_device=True, hbm_budget=1 << 40, max_inflight=1024)
    gemm = srv.submit(fd.make_request("gemm", F3, FAKE, FAKE, FAKE, m=2048, n=2048, k=2048))
    ts = [srv.submit(dot(F1, 1000)) for _ in range(300)]
    srv.drain(20000)
    sizes = [srv.poll(t)[1].batch_size for t in ts]
    assert max(sizes) > 1                   # same-field dots were fused
    assert srv.poll(gemm)[1].batch_size == 1
    plain = fd.Server(fake_device=True, plain=True)
    ts = [plain.submit(dot(F1, 1000)) for _ in range(50)]
    plain.drain(20000)
    assert all(plain.poll(t)[1].batch_size == 1 for t in ts)
    assert plain.stats()["launches"] == 50


def test_back_pressure_and_rejection():
    big = fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=4096, n=4096, k=4096)  # ~1.5 ms simulated
    # room for the product, its library scratch (digit planes, residue sum)
    # and the small requests, not for two products
    srv = fd.Server(fake_device=True, hbm_budget=2 * 3 * 4096 * 4096 * 8,
                    max_inflight=1, max_queue=4)
    srv.submit(big)
    statuses = [srv.try_submit(dot(F1, 10))[0] for _ in range(8)]
    assert statuses.count(0) <= 5 and -7 in statuses   # FDOT_E_BUSY once the queue is full
    too_big = fd.make_request("dot", F1, FAKE, FAKE, FAKE, n=10, footprint=1 << 50)
    assert srv.try_submit(too_big)[0] == -6             # FDOT_E_NOMEM: can never fit
    assert srv.stats()["rejected"] == 1
    with pytest.raises(fd.FdotError):
        srv.submit(fd.make_request("gemv", F1, FAKE, FAKE, FAKE, m=0, n=5))
    srv.drain(20000)


def test_replay_honours_arrivals():
    srv = fd.Server(fake_device=True)
    n = 200
    arrivals = np.cumsum(np.random.default_rng(3).exponential(1e-4, n))
    reqs = [dot(F1, 5000) for _ in range(n)]
    t0 = time.monotonic_ns()
    tm = srv.replay(reqs, arrivals)
    assert len(tm) == n and (tm["status"] == 0).all()
    start = tm["submit_ns"].min()
    offs = (tm["submit_ns"] - start) / 1e9
    # each request is submitted no earlier than its arrival (relative to the first)
    assert (offs + 1e-4 >= arrivals - arrivals[0]).all()
    assert (tm["done_ns"] >= tm["submit_ns"]).all()
    assert tm["submit_ns"].min() >= t0


def test_long_requests_run_alone():
    """A request estimated above exclusive_ns is admitted only once nothing
    else is in flight, and nothing is admitted while it runs."""
    heavy = lambda: fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=2000, n=2000, k=2000)
    light = lambda: dot(F1, 1000)
    order = ["l", "l", "l", "h", "l", "l", "h", "h", "l", "l", "l"]
    srv = fd.Server(fake_device=True, exclusive_ns=100_000, max_inflight=64)
    ts = [srv.submit(heavy() if k == "h" else light()) for k in order]
    srv.drain(20000)
    tm = [srv.poll(t)[1] for t in ts]
    for i, k in enumerate(order):
        if k != "h":
            continue
        assert tm[i].batch_size == 1
        assert all(tm[i].admit_ns >= tm[j].done_ns for j in range(i))
        assert all(tm[j].admit_ns >= tm[i].done_ns for j in range(i + 1, len(order)))
    # without the rule the light requests behind a long one overlap it
    srv2 = fd.Server(fake_device=True, max_inflight=64)  # rule off by default
    ts = [srv2.submit(heavy() if k == "h" else light()) for k in order]
    srv2.drain(20000)
    tm = [srv2.poll(t)[1] for t in ts]
    assert tm[4].admit_ns < tm[3].done_ns


def test_lanes_by_estimated_time():
    """With four streams: matrix products on stream 0, long streaming
    requests on stream 1, streaming requests estimated below short_ns on
    streams 2 and 3; plain mode keeps one stream."""
    srv = fd.Server(fake_device=True, streams=4, short_ns=100_000, max_inflight=64)
    long_gemm = srv.submit(fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=2048, n=2048, k=2048))
    long_gemv = srv.submit(fd.make_request("gemv", F2, FAKE, FAKE, FAKE, m=20000, n=20000))
    small_gemm = srv.submit(fd.make_request("gemm", F3, FAKE, FAKE, FAKE, m=64, n=64, k=64))
    small_gemv = srv.submit(fd.make_request("gemv", F1, FAKE, FAKE, FAKE, m=100, n=100))
    dots = [srv.submit(dot(F1, 1000)) for _ in range(5)]
    srv.drain(20000)
    lane = lambda t: srv.poll(t)[1].stream  # noqa: E731
    assert lane(long_gemm) == 0 and lane(long_gemv) == 1
    assert lane(small_gemm) == 0  # every matrix product on the matrix lane
    assert lane(small_gemv) in (2, 3)
    assert all(lane(t) in (2, 3) for t in dots)
    srv.close()
    plain = fd.Server(fake_device=True, plain=True)
    ts = [plain.submit(fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=2048, n=2048, k=2048)),
          plain.submit(dot(F1, 1000))]
    plain.drain(20000)
    assert all(plain.poll(t)[1].stream == 0 for t in ts)


def test_footprint_counts_library_scratch():
    """The admitted footprint of a matrix product includes the scratch the
    library takes for it (digit planes and the residue sum), so a budget of
    exactly its operand bytes refuses it."""
    m = n = k = 1024
    operands = (m * k + k * n + m * n) * 8
    srv = fd.Server(fake_device=True, hbm_budget=operands)
    assert srv.try_submit(fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=m, n=n, k=k))[0] == -6
    srv.close()


def test_matrix_products_shortest_first_with_aging():
    """matrix_depth = 1: one product outstanding at a time; of the waiting
    ones the shortest estimate goes next, so small products overtake a queue
    of large ones, and a large one still runs once it has waited long."""
    srv = fd.Server(fake_device=True, streams=4, matrix_depth=1, max_inflight=64)
    big = lambda: fd.make_request("gemm", F2, FAKE, FAKE, FAKE, m=1536, n=1536, k=1536)  # noqa: E731
    small = lambda: fd.make_request("gemm", F3, FAKE, FAKE, FAKE, m=64, n=64, k=64)  # noqa: E731
    order = ["b", "b", "b", "s", "s", "b", "s"]
    ts = [srv.submit(big() if k == "b" else small()) for k in order]
    srv.drain(60000)
    tm = [srv.poll(t)[1] for t in ts]
    # never two products outstanding at once
    spans = sorted((t.launch_ns, t.done_ns) for t in tm)
    assert all(a[1] <= b[0] for a, b in zip(spans, spans[1:]))
    # the small ones submitted behind large ones start before the later large ones
    for i in (3, 4, 6):
        assert tm[i].launch_ns < tm[5].launch_ns or tm[i].launch_ns < tm[2].launch_ns
    assert all(t.status == 0 and t.stream == 0 for t in tm)
    srv.close()
