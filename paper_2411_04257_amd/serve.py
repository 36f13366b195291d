"""Served form: a continuous-batching request loop over the batched pipeline.

Requests (each a run of consecutive documents of one host CSR corpus, so that
ticket order equals the stream order of Section 2.1) arrive at scheduled
times.  The scheduler admits waiting requests first-come first-served while
the pipeline has a free slot and the bytes of in-flight batches (tokens,
signatures, flags) stay within an HBM budget; everything admitted together
forms one batch.  A completion thread polls the pipeline and stamps each
request's finish time.  Because the pipeline runs MinHash of a new batch
while the previous batch's query-insert is still on the GPU, requests that
arrive during GPU work are admitted and overlapped as soon as a slot frees.

`PlainServer` is the baseline: one request at a time, synchronously, through
the same pipeline with a single batch in flight.
"""

from __future__ import annotations

import math
import threading
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np
import torch

from . import lshbloom


@dataclass
class Request:
    rid: int
    arrival: float  # seconds after the start of the run
    lo: int  # first document (index into the corpus)
    hi: int  # one past the last document
    finish: float = math.nan
    batch: int = -1


@dataclass
class ServeResult:
    requests: list
    wall_s: float
    docs: int
    batches: int
    latencies_ms: np.ndarray = field(default_factory=lambda: np.zeros(0))

    def summary(self) -> dict:
        lat = self.latencies_ms
        return {
            "docs": self.docs,
            "requests": len(self.requests),
            "batches": self.batches,
            "docs_per_s": self.docs / self.wall_s if self.wall_s > 0 else 0.0,
            "p50_ms": float(np.percentile(lat, 50)) if len(lat) else math.nan,
            "p99_ms": float(np.percentile(lat, 99)) if len(lat) else math.nan,
            "mean_ms": float(lat.mean()) if len(lat) else math.nan,
            "max_ms": float(lat.max()) if len(lat) else math.nan,
        }


def poisson_requests(n_requests: int, docs_per_s: float, size_lo: int, size_hi: int, first_doc: int,
                     rng: np.random.Generator) -> list:
    """Poisson arrivals; sizes log-uniform in [size_lo, size_hi]; consecutive documents."""
    sizes = np.floor(np.exp(rng.uniform(math.log(size_lo), math.log(size_hi + 1), n_requests))).astype(np.int64)
    sizes = np.clip(sizes, size_lo, size_hi)
    mean_size = (size_hi + 1 - size_lo) / math.log((size_hi + 1) / size_lo)
    rate = docs_per_s / mean_size  # requests per second
    gaps = rng.exponential(1.0 / rate, n_requests)
    arrivals = np.cumsum(gaps) - gaps[0]
    reqs, d = [], first_doc
    for i in range(n_requests):
        reqs.append(Request(i, float(arrivals[i]), d, d + int(sizes[i])))
        d += int(sizes[i])
    return reqs


def _report(done: int, total: int, now: float) -> None:
    import sys

    print(f"[serve] {done}/{total} requests finished after {now:.0f} s", file=sys.stderr, flush=True)


class Server:
    """Continuous batching with HBM-budget admission over a Pipeline."""

    def __init__(self, index: lshbloom.LSHBloom, max_docs: int, max_tokens: int, hbm_budget: int,
                 use_graph: bool = True, max_inflight: int = 2):
        self.index = index
        self.max_docs, self.max_tokens = max_docs, max_tokens
        self.hbm_budget = hbm_budget
        self.max_inflight = max_inflight
        self.pipe = lshbloom.Pipeline(index, max_docs=max_docs, max_tokens=max_tokens, use_graph=use_graph,
                                      autotune=False, n_buckets=1)

    def batch_bytes(self, docs: int, tokens: int) -> int:
        return tokens * 4 + docs * (self.index.num_perm * 4 + 1)

    def run(self, reqs: list, offsets: torch.Tensor, tokens: torch.Tensor, flags: torch.Tensor,
            progress_s: float = 0.0) -> ServeResult:
        """offsets/tokens/flags: host tensors (pinned for DMA) covering every request's documents.
        progress_s > 0: print the number of finished requests to stderr that often."""
        off = offsets.numpy()
        lock = threading.Lock()
        inflight = deque()  # (ticket, [requests], bytes)
        state = {"bytes": 0, "done": 0, "batches": 0}
        stop = threading.Event()
        t0 = time.perf_counter()

        def completer():
            while not stop.is_set():
                with lock:
                    head = inflight[0] if inflight else None
                if head is None:
                    time.sleep(20e-6)
                    continue
                ticket, rs, nbytes = head
                if self.pipe.poll(ticket):
                    now = time.perf_counter() - t0
                    for r in rs:
                        r.finish = now
                    with lock:
                        inflight.popleft()
                        state["bytes"] -= nbytes
                        state["done"] += len(rs)
                else:
                    time.sleep(20e-6)

        th = threading.Thread(target=completer, daemon=True)
        th.start()
        waiting = deque()
        nxt = 0
        last_report = 0.0
        try:
            while True:
                now = time.perf_counter() - t0
                if progress_s > 0 and now - last_report >= progress_s:
                    last_report = now
                    _report(state["done"], len(reqs), now)
                while nxt < len(reqs) and reqs[nxt].arrival <= now:
                    waiting.append(reqs[nxt])
                    nxt += 1
                with lock:
                    free = len(inflight) < self.max_inflight
                    used = state["bytes"]
                    finished = state["done"] == len(reqs)
                if finished:
                    break
                if waiting and free:
                    batch, docs, toks = [], 0, 0
                    while waiting:
                        r = waiting[0]
                        d = r.hi - r.lo
                        tk = int(off[r.hi] - off[r.lo])
                        nb = self.batch_bytes(docs + d, toks + tk)
                        if batch and (docs + d > self.max_docs or toks + tk > self.max_tokens or
                                      used + nb > self.hbm_budget):
                            break
                        if not batch and used + nb > self.hbm_budget and used > 0:
                            break  # wait for memory to free up
                        batch.append(waiting.popleft())
                        docs += d
                        toks += tk
                    if batch:
                        lo, hi = batch[0].lo, batch[-1].hi
                        ticket = self.pipe.submit(offsets[lo:hi + 1], tokens, flags[lo:hi])
                        for r in batch:
                            r.batch = ticket
                        with lock:
                            inflight.append((ticket, batch, self.batch_bytes(docs, toks)))
                            state["bytes"] += self.batch_bytes(docs, toks)
                            state["batches"] += 1
                        continue
                if nxt < len(reqs) and not waiting:
                    # sleep until the next arrival (or briefly, to watch completions)
                    time.sleep(max(0.0, min(reqs[nxt].arrival - (time.perf_counter() - t0), 200e-6)))
                else:
                    time.sleep(20e-6)
        finally:
            stop.set()
            th.join()
        wall = max(r.finish for r in reqs) - reqs[0].arrival
        lat = np.array([(r.finish - r.arrival) * 1e3 for r in reqs])
        return ServeResult(reqs, wall, sum(r.hi - r.lo for r in reqs), state["batches"], lat)

    def close(self):
        self.pipe.close()


class PlainServer:
    """Baseline: one request per batch, one batch at a time, no overlap."""

    def __init__(self, index: lshbloom.LSHBloom, max_docs: int, max_tokens: int, use_graph: bool = False):
        self.pipe = lshbloom.Pipeline(index, max_docs=max_docs, max_tokens=max_tokens, use_graph=use_graph,
                                      autotune=False, n_buckets=1)

    def run(self, reqs: list, offsets: torch.Tensor, tokens: torch.Tensor, flags: torch.Tensor,
            progress_s: float = 0.0) -> ServeResult:
        t0 = time.perf_counter()
        last_report = 0.0
        for q, r in enumerate(reqs):
            now = time.perf_counter() - t0
            if progress_s > 0 and now - last_report >= progress_s:
                last_report = now
                _report(q, len(reqs), now)
            if r.arrival > now:
                time.sleep(r.arrival - now)
            t = self.pipe.submit(offsets[r.lo:r.hi + 1], tokens, flags[r.lo:r.hi])
            self.pipe.wait(t)
            r.finish = time.perf_counter() - t0
            r.batch = t
        wall = max(r.finish for r in reqs) - reqs[0].arrival
        lat = np.array([(r.finish - r.arrival) * 1e3 for r in reqs])
        return ServeResult(reqs, wall, sum(r.hi - r.lo for r in reqs), len(reqs), lat)

    def close(self):
        self.pipe.close()


def preload(index: lshbloom.LSHBloom, n_docs: int, seed: int, chunk: int = 1 << 20) -> None:
    """Insert n_docs uniformly random signatures (stand-ins for already-ingested documents)."""
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    done = 0
    while done < n_docs:
        c = min(chunk, n_docs - done)
        sigs = torch.randint(-2**31, 2**31 - 1, (c, index.num_perm), generator=g, device="cuda", dtype=torch.int32)
        index.insert(sigs)
        done += c
    torch.cuda.synchronize()
