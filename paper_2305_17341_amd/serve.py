"""Serving layer: continuous batching of homomorphic matrix products and
covariance jobs over device-resident keys and ciphertexts.

Model (the client/cloud split of the paper's experimental section): clients
encrypt their matrices and hand the ciphertexts to the server; the server
keeps one context per ring dimension N (keys, plaintext diagonals and the
submitted ciphertexts stay in HBM) and returns result ciphertexts.

Scheduling
  * Admission by HBM footprint: every request carries the working-set bytes
    its computation will allocate (`product_footprint`,
    `covariance_footprint`).  Requests are admitted strictly in arrival
    order while the admitted footprints fit the budget; a request larger
    than the whole budget is rejected at submission.
  * Continuous batching: one worker per context.  Whenever a worker is free
    it takes the oldest admitted request of its N together with the other
    admitted products of that N, of any size (up to `max_batch`), and runs
    them as one merged batch: products of equal d are stacked, and the
    stacks of different d run together with their key inner products merged
    into shared launches (HE_MM_MERGED).  Requests that arrived while earlier
    work was on the device join the next batch.  Workers of different N run
    concurrently, each on its context's stream, so their kernels overlap on
    the GPU.  Memory freed by a finished batch admits waiting requests.
  * A covariance job runs in chunks of row blocks (he_covariance_begin /
    add / end, `cov_chunk` row blocks a call).  Between two chunks a worker
    runs up to `cov_yield` batches of the products waiting on its N, so a
    long covariance does not hold them back, and it still advances while
    products keep arriving.  Its residues do not depend on the chunks (the
    sums over row blocks are exact).
  * The merged path gives the same residues as running a product alone, so
    a result does not depend on what it was batched with.

Latency is measured per request from submission to the host seeing its
batch complete; `Server.stats()` reports p50/p99 latency and jobs/s.
"""
from __future__ import annotations

import collections
import math
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

BATCHED = 1  # HE_MM_BATCHED
LAZY_RELIN = 2  # HE_MM_LAZY_RELIN
FUSED_RESCALE = 4  # HE_MM_FUSED_RESCALE
MERGED = 64  # HE_MM_MERGED
POOL_SLACK = 1.25  # a cached device block is reused for requests down to 1/1.25 of its size


class AdmissionError(RuntimeError):
    pass


def default_n1(d: int) -> int:
    return 1 << ((max(d - 1, 1).bit_length() + 1) // 2)


def _qp(level: int, alpha: int) -> int:
    return level + 1 + alpha


def _beta(level: int, alpha: int) -> int:
    return -(-(level + 1) // alpha)


def product_footprint(log_n: int, top_level: int, alpha: int, d: int, batch: int = 1) -> int:
    """Upper bound on the device bytes one d x d product (inputs at
    `top_level`, no decomposition) allocates beyond what is resident, times
    `batch` stacked members: the n column-shifted A_k (level l-2) and the n
    row-shifted B_k (level l-1) held together before the products, plus the
    largest transient of a linear transform (n1 baby-step rotations in
    R_{Q_l P}, or the 2 n1 of the column shifts, the digits of one
    decomposition and a few accumulators), plus stacked copies of the
    inputs and the output."""
    l = top_level
    n1 = default_n1(d)
    sides = d * 2 * (l - 1) + d * 2 * l
    trans = 2 * (2 * n1 + 4) * _qp(l, alpha) + _beta(l, alpha) * _qp(l, alpha) + 6 * (l + 1)
    io = 4 * (l + 1) + 2 * (l - 2)
    words = batch * (sides + trans + io) << log_n
    return int(math.ceil(words * 8 * POOL_SLACK))


def covariance_footprint(log_n: int, top_level: int, alpha: int, d: int, k: int, row_blocks: int = 1,
                         stacked: int = 4) -> int:
    """Upper bound for the block covariance of k feature blocks: the A and B
    sides of all k blocks are held for the row blocks stacked into one batch
    (min(row_blocks, stacked): the library's "cov_row_blocks"; one-to-many
    reuse), plus the k^2 accumulators and one batch's transient."""
    l = top_level
    n1 = default_n1(d)
    g = max(1, min(row_blocks, stacked))
    sides = 2 * k * d * 2 * l * g
    acc = k * k * 2 * l
    trans = g * (2 * (2 * n1 + 4) * _qp(l, alpha) + _beta(l, alpha) * _qp(l, alpha) + 8 * (l + 1))
    words = (sides + acc + trans) << log_n
    return int(math.ceil(words * 8 * POOL_SLACK))


@dataclass
class Request:
    kind: str                       # "matmul" | "covariance"
    log_n: int
    d: int
    args: tuple                     # (a, b) or (blocks, row_blocks, k, n_samples)
    id: int = 0
    footprint: int = 0
    t_submit: float = 0.0
    t_admit: float = 0.0
    t_start: float = 0.0
    t_done: float = 0.0
    batch: int = 0
    future: Future = field(default_factory=Future)
    state: object = None            # covariance in parts: the library's state
    cursor: int = 0                 # covariance in parts: row blocks done
    cov_g: int = 0                  # covariance: row blocks stacked per batch (its footprint's g)

    @property
    def latency(self) -> float:
        return self.t_done - self.t_submit


class HeBackend:
    """One context per ring dimension, keys for every served product size."""

    def __init__(self, chains, ds_by_log_n, seed=1, covariance_d=(), lazy_relin=True, cov_chunk=8):
        from . import he
        self.cov_chunk = cov_chunk
        # the benchmark headline's variants: lazy relinearisation and one
        # rounding for the A side's ModDown and Rescale
        self.relin_flags = LAZY_RELIN | FUSED_RESCALE if lazy_relin else 0
        self.contexts = {}
        self.chains = {}
        for chain in chains:
            ctx = he.chain_context(chain, seed=seed)
            steps = set()
            for d in ds_by_log_n.get(chain.log_n, ()):
                steps |= set(ctx.matmul_rot_steps(d))
            if chain.log_n in dict(covariance_d):
                steps |= set(ctx.transpose_rot_steps(dict(covariance_d)[chain.log_n]))
            ctx.keygen(sorted(steps))
            self.contexts[chain.log_n] = ctx
            self.chains[chain.log_n] = chain

    def log_ns(self):
        return sorted(self.contexts)

    def footprint(self, r: Request, budget: int = 0) -> int:
        """device bytes the request's computation allocates.  A covariance
        stacks as many row blocks per batch (the library's cov_row_blocks,
        halved down to 1) as keep it within half the budget, so that
        products still find memory beside it."""
        ch = self.chains[r.log_n]
        if r.kind == "matmul":
            return product_footprint(r.log_n, ch.top_level, len(ch.p_bits), r.d)
        from . import he
        _, rb, k, _ = r.args
        g = he.knob_get("cov_row_blocks")
        while True:
            fp = covariance_footprint(r.log_n, ch.top_level, len(ch.p_bits), r.d, k, rb, g)
            if g == 1 or not budget or 2 * fp <= budget:
                r.cov_g = g
                return fp
            g = max(1, g // 2)

    def run(self, log_n: int, reqs):
        """Runs a merged batch of products, or the next chunk of a covariance
        job; returns the results, or None while a covariance is unfinished."""
        ctx = self.contexts[log_n]
        if reqs[0].kind == "covariance":
            r = reqs[0]
            blocks, rb, k, n_samples = r.args
            if r.state is None:
                r.state = ctx.covariance_begin(k, r.d, n_samples, opts={"flags": self.relin_flags})
            g = min(self.cov_chunk, rb - r.cursor)
            from . import he
            old = he.knob_get("cov_row_blocks")
            he.knob_set("cov_row_blocks", r.cov_g or old)
            try:
                r.state.add(blocks[r.cursor * k:(r.cursor + g) * k], g)
            finally:
                he.knob_set("cov_row_blocks", old)
            r.cursor += g
            if r.cursor < rb:
                ctx.sync()
                return None
            out = [r.state.end()]
            r.state.free()
            r.state = None
        else:
            out = ctx.matmul_batch([r.args[0] for r in reqs], [r.args[1] for r in reqs], [r.d for r in reqs],
                                   opts={"flags": BATCHED | MERGED | self.relin_flags})
        ctx.sync()
        return out

    def release(self, log_n: int, keep_bytes: int):
        """once the context is idle, give its cached device blocks back if
        they exceed `keep_bytes` (other contexts may need the memory)"""
        ctx = self.contexts[log_n]
        _, cached, _ = ctx.mem_info()
        if cached > keep_bytes:
            ctx.trim()


class Server:
    def __init__(self, backend, hbm_budget: int, max_batch: int = 8, trim_when_idle: bool = True,
                 cov_yield: int = 4):
        self.backend = backend
        self.cov_yield = cov_yield
        self.budget = int(hbm_budget)
        self.max_batch = max_batch
        self.trim_when_idle = trim_when_idle
        self._cv = threading.Condition()
        self._pending = collections.deque()
        self._ready = {n: [] for n in backend.log_ns()}
        self._in_use = 0
        self._peak = 0
        self._stop = False
        self._next_id = 0
        self._done = []
        self._rejected = 0
        self._batches = []
        self._cov_chunks = 0
        self._since_chunk = {n: 0 for n in backend.log_ns()}   # product batches since the last chunk
        self._workers = [threading.Thread(target=self._work, args=(n,), daemon=True) for n in backend.log_ns()]
        for w in self._workers:
            w.start()

    # -- client side --------------------------------------------------------
    def submit(self, kind: str, log_n: int, d: int, args: tuple) -> Future:
        if log_n not in self._ready:
            raise ValueError(f"no context for N = 2^{log_n}")
        r = Request(kind, log_n, d, args)
        r.footprint = self.backend.footprint(r, self.budget)
        r.t_submit = time.perf_counter()
        with self._cv:
            r.id = self._next_id
            self._next_id += 1
            if r.footprint > self.budget:
                self._rejected += 1
                r.future.set_exception(AdmissionError(
                    f"request {r.id} needs {r.footprint} B of device memory; the budget is {self.budget} B"))
                return r.future
            if self._stop:
                raise RuntimeError("server is stopping")
            self._pending.append(r)
            self._admit()
            self._cv.notify_all()
        return r.future

    def close(self):
        with self._cv:
            self._stop = True
            self._cv.notify_all()
        for w in self._workers:
            w.join()

    def stats(self) -> dict:
        with self._cv:
            done = list(self._done)
            batches = list(self._batches)
            peak, rejected = self._peak, self._rejected
        if not done:
            return {"jobs": 0, "rejected": rejected}

        def pct(rs):
            lat = sorted(r.latency for r in rs)

            def q(p):
                return lat[min(len(lat) - 1, max(0, int(math.ceil(p / 100.0 * len(lat))) - 1))]
            return {"p50": q(50), "p99": q(99), "max": lat[-1]}

        def rate(rs):
            span = max(r.t_done for r in rs) - min(r.t_submit for r in rs)
            return len(rs) / span if span > 0 else None
        prods = [r for r in done if r.kind == "matmul"]
        return {
            "jobs": len(done),
            "rejected": rejected,
            "jobs_per_s": rate(done),
            "latency_s": pct(done),
            # the products alone: a long covariance job would otherwise set
            # the span and the tail of every trace it is part of
            "products_per_s": rate(prods) if prods else None,
            "product_latency_s": pct(prods) if prods else None,
            "covariance_latency_s": [r.latency for r in done if r.kind != "matmul"],
            "mean_batch": sum(batches) / len(batches) if batches else None,
            "batches": len(batches),
            "covariance_chunks": self._cov_chunks,
            "peak_admitted_bytes": peak,
            "budget_bytes": self.budget,
        }

    # -- scheduler ------------------------------------------------------------
    def _admit(self):
        # strict arrival order: the head waits until it fits, nothing overtakes it
        while self._pending and self._pending[0].footprint <= self.budget - self._in_use:
            r = self._pending.popleft()
            self._in_use += r.footprint
            self._peak = max(self._peak, self._in_use)
            r.t_admit = time.perf_counter()
            self._ready[r.log_n].append(r)

    def _take(self, log_n):
        ready = self._ready[log_n]
        mats = [r for r in ready if r.kind == "matmul"]
        head = ready[0]
        # between two covariance chunks, up to cov_yield batches of products
        if head.kind != "matmul" and not (mats and self._since_chunk[log_n] < self.cov_yield):
            group = [head]
            self._since_chunk[log_n] = 0
        else:
            group = mats[: self.max_batch]
            self._since_chunk[log_n] += 1
        ids = {id(r) for r in group}
        self._ready[log_n] = [r for r in ready if id(r) not in ids]
        return group

    def _work(self, log_n):
        while True:
            with self._cv:
                while not self._ready[log_n]:
                    if self._stop and not any(p.log_n == log_n for p in self._pending):
                        return
                    self._cv.wait()
                group = self._take(log_n)
            t0 = time.perf_counter()
            err, out = None, None
            try:
                out = self.backend.run(log_n, group)
            except Exception as e:  # delivered to every request of the batch
                err = e
                for r in group:
                    if r.state is not None:
                        r.state.free()
                        r.state = None
            t1 = time.perf_counter()
            if err is None and out is None:
                # a covariance chunk: the job goes back to the head of its
                # queue, still holding its admitted memory
                with self._cv:
                    self._cov_chunks += 1
                    if group[0].t_start == 0.0:
                        group[0].t_start = t0
                    self._ready[log_n].insert(0, group[0])
                    self._cv.notify_all()
                continue
            with self._cv:
                for r in group:
                    self._in_use -= r.footprint
                    r.t_start, r.t_done, r.batch = r.t_start or t0, t1, len(group)
                    if err is None:
                        self._done.append(r)
                if group[0].kind == "matmul":
                    self._batches.append(len(group))
                else:
                    self._cov_chunks += 1
                self._admit()
                idle = not self._ready[log_n]
                # an idle context gives its cached blocks back only while
                # other contexts have work waiting that may need the memory
                others_busy = bool(self._pending) or any(self._ready[n] for n in self._ready if n != log_n)
                self._cv.notify_all()
            for i, r in enumerate(group):
                if err is None:
                    r.future.set_result(out[i])
                else:
                    r.future.set_exception(err)
            if idle and others_busy and self.trim_when_idle:
                self.backend.release(log_n, self.budget // len(self._ready))


def valid_pairs(chains, ds=(16, 32, 64, 128)):
    """(d, log_n) with d^2 <= N/2 (one matrix per ciphertext) and depth 3 available"""
    out = []
    for ch in chains:
        for d in ds:
            if d * d <= ch.N // 2 and ch.top_level >= 3:
                out.append((d, ch.log_n))
    return out


def run_trace(server, jobs, payloads, extra=()):
    """Submit `jobs` at their arrival times (seconds from now); `payloads[i]`
    is (kind, log_n, d, args) of job i; `extra` lists (arrival, payload)
    submitted alongside.  Returns the futures in submission order."""
    events = sorted([(j.arrival, p) for j, p in zip(jobs, payloads)] + list(extra), key=lambda e: e[0])
    t0 = time.perf_counter()
    futs = []
    for at, (kind, log_n, d, args) in events:
        delay = at - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        futs.append(((kind, log_n, d, args), server.submit(kind, log_n, d, args)))
    return futs


def main(argv=None):
    import json
    print(json.dumps(serve_bench(argv)), flush=True)


def serve_bench(argv=None):
    """Poisson mixes of products over every (d, N) pair with d in {16, 32, 64,
    128}, N in {2^13 .. 2^16} and d^2 <= N/2, plus one block-covariance job
    at N = 2^16.  First the batched capacity: every job of a trace offered at
    once (served jobs/s and mean batch); then the offered load swept as
    fractions of that capacity (each load a trace of its own, the covariance
    job in the middle of the last one); each reports served jobs/s, p50/p99
    latency and the mean batch.  Returns one dict (printed by main())."""
    import argparse
    import sys

    import numpy as np

    from . import inputs as I, packing

    ap = argparse.ArgumentParser()
    ap.add_argument("--jobs", type=int, default=300, help="jobs per trace (capacity run and each load)")
    ap.add_argument("--loads", default="0.2,0.6,1.0,1.2",
                    help="offered rates as fractions of the measured batched capacity")
    ap.add_argument("--budget-gib", type=float, default=0.0,
                    help="0: 3/4 of the device memory free once a trace's inputs are resident")
    ap.add_argument("--seed", type=int, default=11)
    ap.add_argument("--no-covariance", action="store_true")
    ap.add_argument("--cov-samples", type=int, default=256,
                    help="rows of the covariance job's dataset (256 features; the workload's job has 60000)")
    args = ap.parse_args(argv)
    loads = [float(x) for x in args.loads.split(",") if x]

    def log(m):
        print(m, file=sys.stderr, flush=True)

    chains = [I.SMALL, I.MID, I.SERVE15, I.LARGE]
    pairs = valid_pairs(chains)
    ds_by = {}
    for d, ln in pairs:
        ds_by.setdefault(ln, []).append(d)
    cov_n = 128
    t0 = time.perf_counter()
    backend = HeBackend(chains, ds_by, seed=args.seed, covariance_d=() if args.no_covariance else ((16, cov_n),))
    log(f"[serve] contexts and keys for {len(pairs)} (d, N) pairs in {time.perf_counter() - t0:.1f} s")

    # the NTT stage split of each ring size that has an alternative, tuned on a
    # batch of four of its largest products
    from . import autotune
    tuned = {}
    for ln, ctx in backend.contexts.items():
        d = max(ds_by[ln])
        A = I.uniform_matrix(3, d)
        cs = [ctx.encrypt_matrix(A, nonce=50 + i) for i in range(4)]
        ctx.matmul_batch(cs, cs, [d] * 4, opts={"flags": BATCHED | backend.relin_flags})   # warm caches
        best, tt = autotune.autotune_ntt_split(ctx, cs, cs, d, opts={"flags": BATCHED | backend.relin_flags},
                                               log=log)
        tuned.update({k: {"value": v, "ms": tt[k]} for k, v in best.items()})
        del cs

    # warm-up: every pair once alone (fills the plaintext caches), then its solo latency
    solo = {}
    for d, ln in pairs:
        ctx = backend.contexts[ln]
        A = I.uniform_matrix(1, d)
        ca, cb = ctx.encrypt_matrix(A, nonce=1), ctx.encrypt_matrix(A, nonce=2)
        for rep in range(2):
            t = time.perf_counter()
            r = ctx.matmul(ca, cb, d, opts={"flags": backend.relin_flags})
            ctx.sync()
            solo[(d, ln)] = time.perf_counter() - t
            del r
    one_at_a_time = len(pairs) / sum(solo.values())
    log(f"[serve] solo latency per pair (ms): " + ", ".join(f"d={d}/2^{ln}: {1e3 * s:.1f}"
                                                          for (d, ln), s in sorted(solo.items())))
    ctx16 = backend.contexts[16]

    def budget_now():
        """the admission budget: --budget-gib, else 3/4 of the device memory
        free once the trace's inputs are resident and cached blocks are back"""
        if args.budget_gib > 0:
            return int(args.budget_gib * 2**30)
        from . import he
        for c in backend.contexts.values():
            c.sync()
            c.trim()
        free, _ = he.device_memory()
        return int(0.75 * free)
    X = I.centre(I.dataset(args.seed, args.cov_samples, 2 * cov_n)) if not args.no_covariance else None

    def trace(seed, rate, with_cov):
        """one trace of --jobs products at `rate` (inf: all at once); returns (stats, max sampled error)"""
        jobs = I.poisson_jobs(seed, args.jobs, rate if np.isfinite(rate) else 1e9, pairs)
        payloads, plain = [], []
        for j in jobs:
            ctx = backend.contexts[j.log_n]
            A, B = I.uniform_matrix(j.seed, j.d), I.uniform_matrix(j.seed + 1, j.d)
            payloads.append(("matmul", j.log_n, j.d,
                             (ctx.encrypt_matrix(A, nonce=2 * j.seed), ctx.encrypt_matrix(B, nonce=2 * j.seed + 1))))
            plain.append(A @ B)
        extra = []
        if with_cov:
            # cov_samples x 256 uniform[0,1] dataset, centred on the client, as
            # row blocks x 2 blocks of 128 x 128 (the last row block zero-padded)
            cov_rb = -(-args.cov_samples // cov_n)
            blk = packing.blocks(X, cov_n)
            cts = [ctx16.encrypt_matrix(blk[r, c], nonce=10**6 + 2 * r + c) for r in range(cov_rb) for c in range(2)]
            extra.append((jobs[len(jobs) // 2].arrival, ("covariance", 16, cov_n, (cts, cov_rb, 2, X.shape[0]))))
            del blk
        budget = budget_now()
        srv = Server(backend, hbm_budget=budget)
        futs = run_trace(srv, jobs, payloads, extra)
        results = [f.result() for _, f in futs]
        srv.close()
        st = srv.stats()
        # client side: every 8th product and the covariance decrypted against FP64
        errs = []
        for (kind, ln, d, a), res in zip([p for p, _ in futs], results):
            if kind == "matmul":
                idx = next(i for i, p in enumerate(payloads) if p[3] is a)
                if idx % 8 == 0:
                    got = backend.contexts[ln].decrypt(res, d * d)
                    errs.append(float(np.max(np.abs(got - plain[idx].ravel()))))
            else:
                ref = X.T @ X / X.shape[0]
                for i, c in enumerate(res):
                    a_, b_ = divmod(i, 2)
                    got = ctx16.decrypt(c, cov_n * cov_n).reshape(cov_n, cov_n)
                    errs.append(float(np.max(np.abs(got - ref[a_ * cov_n:(a_ + 1) * cov_n,
                                                                b_ * cov_n:(b_ + 1) * cov_n]))))
        return st, (max(errs) if errs else None)

    def summary(st, rate, err):
        return {"offered_rate": None if not np.isfinite(rate) else round(rate, 3),
                "jobs_per_s": round(st["jobs_per_s"], 3),
                "latency_ms": {k2: round(1e3 * v, 2) for k2, v in st["latency_s"].items()},
                "products_per_s": round(st["products_per_s"], 3),
                "product_latency_ms": {k2: round(1e3 * v, 2) for k2, v in st["product_latency_s"].items()},
                "covariance_latency_s": [round(v, 3) for v in st["covariance_latency_s"]],
                "mean_batch": round(st["mean_batch"], 3), "batches": st["batches"], "jobs": st["jobs"],
                "rejected": st["rejected"], "peak_admitted_gib": round(st["peak_admitted_bytes"] / 2**30, 2),
                "budget_gib": round(st["budget_bytes"] / 2**30, 2), "covariance_chunks": st["covariance_chunks"],
                "max_abs_err_sampled": err}

    log(f"[serve] batched capacity: {args.jobs} jobs offered at once")
    st, err = trace(args.seed, float("inf"), False)
    capacity = st["jobs_per_s"]
    cap = summary(st, float("inf"), err)
    log(f"[serve] capacity {capacity:.2f} jobs/s (one at a time {one_at_a_time:.2f}), mean batch "
        f"{st['mean_batch']:.2f}, budget {cap['budget_gib']:.1f} GiB")
    sweep = []
    for k, load in enumerate(loads):
        rate = load * capacity
        with_cov = X is not None and k == len(loads) - 1
        st, err = trace(args.seed + 1 + k, rate, with_cov)
        row = dict(summary(st, rate, err), load=load, covariance_job=with_cov)
        sweep.append(row)
        log(f"[serve] load {load}: offered {rate:.2f}/s, products served {row['products_per_s']:.2f}/s, p50 "
            f"{row['product_latency_ms']['p50']:.1f} ms, p99 {row['product_latency_ms']['p99']:.1f} ms, mean batch "
            f"{row['mean_batch']:.2f}" + (f", covariance job {row['covariance_latency_s'][0]:.1f} s in "
                                          f"{row['covariance_chunks']} chunks" if row['covariance_latency_s'] else ""))
    for c in backend.contexts.values():
        c.close()
    head = max(sweep, key=lambda r: r["load"]) if sweep else cap
    errs = [r["max_abs_err_sampled"] for r in sweep + [cap] if r["max_abs_err_sampled"] is not None]
    return {
        "metric": "served HE jobs/s and latency percentiles (Poisson mix of d x d products over 14 (d, N) pairs"
                  + ("" if args.no_covariance else f" + one {args.cov_samples}x256 block covariance") + ")",
        "jobs_per_s": head["jobs_per_s"],
        "latency_ms": head["latency_ms"],
        "products_per_s": head["products_per_s"],
        "product_latency_ms": head["product_latency_ms"],
        "mean_batch": head["mean_batch"],
        "one_at_a_time_rate": round(one_at_a_time, 3),
        "batched_capacity": cap,
        "capacity_vs_one_at_a_time": round(capacity / one_at_a_time, 3),
        "load_sweep": sweep,
        "jobs_total": cap["jobs"] + sum(r["jobs"] for r in sweep),
        "max_abs_err_sampled": max(errs) if errs else None,
        "solo_ms": {f"d{d}_n{ln}": round(1e3 * s, 2) for (d, ln), s in sorted(solo.items())},
        "ntt_split_autotune": tuned,
    }


if __name__ == "__main__":
    main()
