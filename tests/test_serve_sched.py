"""Serving scheduler on the CPU: admission by footprint, strict arrival
order, batching rules, continuous joining of late arrivals, overlap of
different ring dimensions, error delivery; a stand-in backend replaces the
GPU (it sleeps for the batch's duration and records what it was given)."""
import threading
import time

import pytest

from paper_2305_17341_amd import inputs as I
from paper_2305_17341_amd import serve as S


class FakeBackend:
    def __init__(self, log_ns=(13, 14), cost=0.02, fail_d=None):
        self._log_ns = list(log_ns)
        self.cost = cost
        self.fail_d = fail_d
        self.calls = []
        self.lock = threading.Lock()
        self.started = threading.Event()   # set once the first batch is on the "device"

    def log_ns(self):
        return self._log_ns

    def footprint(self, r, budget=0):
        return r.d * 10

    def run(self, log_n, reqs):
        t0 = time.perf_counter()
        self.started.set()
        time.sleep(self.cost)
        with self.lock:
            self.calls.append((log_n, [(r.kind, r.d, r.id) for r in reqs], t0, time.perf_counter()))
        if self.fail_d is not None and reqs[0].d == self.fail_d:
            raise RuntimeError("device error")
        return [("out", r.id) for r in reqs]

    def release(self, log_n, keep_bytes):
        pass


def test_results_routed_to_their_requests():
    be = FakeBackend()
    srv = S.Server(be, hbm_budget=10_000)
    futs = [srv.submit("matmul", 13 + (i % 2), 16, (i,)) for i in range(12)]
    res = [f.result(timeout=10) for f in futs]
    srv.close()
    for i, r in enumerate(res):
        assert r == ("out", i)
    st = srv.stats()
    assert st["jobs"] == 12 and st["rejected"] == 0
    assert st["latency_s"]["p50"] <= st["latency_s"]["p99"] <= st["latency_s"]["max"]


def test_budget_never_exceeded_and_oversize_rejected():
    be = FakeBackend(cost=0.01)
    srv = S.Server(be, hbm_budget=500)
    big = srv.submit("matmul", 13, 64, ())         # 640 > 500: rejected at once
    with pytest.raises(S.AdmissionError):
        big.result(timeout=1)
    futs = [srv.submit("matmul", 13, 32, ()) for _ in range(10)]   # 320 each: one at a time
    for f in futs:
        f.result(timeout=10)
    srv.close()
    st = srv.stats()
    assert st["rejected"] == 1
    assert st["peak_admitted_bytes"] <= 500
    assert all(len(reqs) == 1 for _, reqs, _, _ in be.calls)


def test_strict_arrival_order_under_memory_pressure():
    be = FakeBackend(log_ns=(13,), cost=0.01)
    srv = S.Server(be, hbm_budget=400)
    ds = [32, 8, 32, 8, 16, 32]
    futs = [srv.submit("matmul", 13, d, ()) for d in ds]
    for f in futs:
        f.result(timeout=10)
    srv.close()
    started = [rid for _, reqs, _, _ in sorted(be.calls, key=lambda c: c[2]) for _, _, rid in reqs]
    # a request never starts before an earlier one was admitted; with one worker the
    # first request of every batch is the oldest not yet started
    first_of_batch = [reqs[0][2] for _, reqs, _, _ in sorted(be.calls, key=lambda c: c[2])]
    assert first_of_batch == sorted(first_of_batch)
    assert sorted(started) == list(range(len(ds)))


def test_batches_take_products_of_any_d_up_to_max_batch_and_covariance_alone():
    be = FakeBackend(log_ns=(16,), cost=0.05)
    srv = S.Server(be, hbm_budget=10**9, max_batch=3)
    hold = srv.submit("matmul", 16, 8, ())      # occupies the worker while the rest queue up
    be.started.wait(5)
    futs = [srv.submit("matmul", 16, d, ()) for d in (16, 16, 32, 16, 16, 32)]
    cov = srv.submit("covariance", 16, 16, (None, 2, 2, 100))
    for f in [hold, cov] + futs:
        f.result(timeout=10)
    srv.close()
    for _, reqs, _, _ in be.calls:
        kinds = {k for k, _, _ in reqs}
        assert len(reqs) <= 3
        if "covariance" in kinds:
            assert len(reqs) == 1
    sizes = [len(reqs) for _, reqs, _, _ in be.calls]
    assert sizes.count(3) == 2      # the six queued products went as 3 + 3, sizes mixed
    assert any(len({d for _, d, _ in reqs}) > 1 for _, reqs, _, _ in be.calls)
    # arrival order inside and across batches
    ids = [i for _, reqs, _, _ in be.calls for k, _, i in reqs if k == "matmul"]
    assert ids == sorted(ids)


def test_late_arrivals_join_the_next_batch():
    be = FakeBackend(log_ns=(14,), cost=0.1)
    srv = S.Server(be, hbm_budget=10**9, max_batch=8)
    first = srv.submit("matmul", 14, 16, ())
    be.started.wait(5)               # the first batch is now running
    late = [srv.submit("matmul", 14, 16, ()) for _ in range(5)]
    for f in [first] + late:
        f.result(timeout=10)
    srv.close()
    assert [len(reqs) for _, reqs, _, _ in be.calls] == [1, 5]


def test_different_ring_dimensions_overlap():
    be = FakeBackend(log_ns=(13, 16), cost=0.2)
    srv = S.Server(be, hbm_budget=10**9)
    a = srv.submit("matmul", 13, 16, ())
    b = srv.submit("matmul", 16, 16, ())
    a.result(timeout=10)
    b.result(timeout=10)
    srv.close()
    (_, _, s0, e0), (_, _, s1, e1) = be.calls
    assert max(s0, s1) < min(e0, e1)


def test_backend_error_reaches_every_request_of_the_batch():
    be = FakeBackend(log_ns=(13,), cost=0.05, fail_d=32)
    srv = S.Server(be, hbm_budget=10**9, max_batch=3)
    hold = srv.submit("matmul", 13, 16, ())
    be.started.wait(5)
    bad = [srv.submit("matmul", 13, 32, ()) for _ in range(3)]    # one batch of three, which fails
    good = srv.submit("matmul", 13, 16, ())                       # the next batch
    hold.result(timeout=10)
    for f in bad:
        with pytest.raises(RuntimeError):
            f.result(timeout=10)
    assert good.result(timeout=10)[0] == "out"
    srv.close()


def test_footprint_model_shapes():
    ch = I.LARGE
    a = len(ch.p_bits)
    f128 = S.product_footprint(ch.log_n, ch.top_level, a, 128)
    # 128 column- and 128 row-shifted ciphertexts of ~29-30 limbs of 512 KiB dominate: 7-12 GiB
    assert 7 * 2**30 < f128 < 12 * 2**30
    assert S.product_footprint(ch.log_n, ch.top_level, a, 128, batch=4) == pytest.approx(4 * f128, rel=1e-9)
    fs = [S.product_footprint(ch.log_n, ch.top_level, a, d) for d in (16, 32, 64, 128)]
    assert fs == sorted(fs)
    small = S.product_footprint(I.SMALL.log_n, I.SMALL.top_level, 1, 16)
    assert small < fs[0]
    assert S.covariance_footprint(ch.log_n, ch.top_level, a, 128, 2) > 1.5 * f128


def test_valid_pairs_match_the_fourteen_served_shapes():
    pairs = S.valid_pairs([I.SMALL, I.MID, I.SERVE15, I.LARGE])
    assert len(pairs) == 14
    assert all(d * d <= (1 << ln) // 2 for d, ln in pairs)


class ChunkedBackend(FakeBackend):
    """a covariance job takes `chunks` calls (None until the last), as the
    library's covariance in parts does"""

    def __init__(self, chunks=3, **kw):
        super().__init__(**kw)
        self.chunks = chunks

    def run(self, log_n, reqs):
        if reqs[0].kind == "covariance":
            t0 = time.perf_counter()
            self.started.set()
            time.sleep(self.cost)
            with self.lock:
                self.calls.append((log_n, [(r.kind, r.d, r.id) for r in reqs], t0, time.perf_counter()))
            reqs[0].cursor += 1
            return None if reqs[0].cursor < self.chunks else [("cov", reqs[0].id)]
        return super().run(log_n, reqs)


def test_products_run_between_covariance_chunks():
    """A covariance job runs a chunk at a time; products that arrive meanwhile
    get a batch between its chunks instead of waiting for the whole job,
    and the job still completes with its result."""
    be = ChunkedBackend(chunks=4, log_ns=(16,), cost=0.03)
    srv = S.Server(be, hbm_budget=100_000)
    cov = srv.submit("covariance", 16, 128, ())
    assert be.started.wait(5)
    mats = [srv.submit("matmul", 16, 16, (i,)) for i in range(3)]
    assert cov.result(timeout=10) == ("cov", 0)
    for f in mats:
        f.result(timeout=10)
    srv.close()
    kinds = [reqs[0][0] for _, reqs, _, _ in sorted(be.calls, key=lambda c: c[2])]
    assert kinds.count("covariance") == 4
    first_mat = kinds.index("matmul")
    assert first_mat < len(kinds) - 1 and "covariance" in kinds[first_mat + 1:], kinds
    st = srv.stats()
    assert st["covariance_chunks"] == 4 and st["jobs"] == 4
    assert srv.stats()["peak_admitted_bytes"] >= 128 * 10
