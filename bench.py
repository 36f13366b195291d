#!/usr/bin/env python3
"""End-to-end LSHBloom throughput on one MI355X.

A step is one pass of the whole hot path over one batch of documents:
MinHash signatures of the batch, then the in-order query-insert against the
per-band Bloom filters (which keep growing across steps, as in a real
stream).  The default workload is the batched form on the 10M-document
configuration: synthetic documents (Zipf(1.1) tokens over a 50k vocabulary,
Pareto(1.5, min 20) lengths capped at 200,000, 25% near-duplicates), 5-token
shingles, num_perm = 256, 32 bands x 8 rows, filters sized for n = 1e8 at a
per-band fp rate of 1e-8 (15.3 GB), batches of 2M documents handed over as
host CSR arrays and flags returned to host memory (the pipeline overlaps the
copies, length-bucketed MinHash and the query-insert).  Beside it the same
host batches go through plain per-batch calls, and the same batches through
plain calls on inputs already in HBM.

Prints one JSON line with docs/s, the dominant stage's roofline (the
query-insert, timed with HIP events on the stream it runs on) and the CPU
oracle timed on a bounded prefix of the same stream.
"""

from __future__ import annotations

import argparse
import dataclasses
import hashlib
import json
import os
import re
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

CSRC = os.path.join(ROOT, "paper_2411_04257_amd", "csrc")
PROFILES = os.path.join(ROOT, "profiles")
INT32_VALU_PEAK = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 3.93e13 lane-ops/s
HBM_PEAK = 8e12
CACHE_BYTES = 256e6


def source_tag(*files) -> str:
    """First 16 hex digits of the SHA-256 of the named kernel sources: the
    version of the kernels a counter profile was taken of."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def profile_rows(name: str, tag: str) -> dict:
    """Rows `| key | tag | v1 | v2 | ... |` of profiles/<name> whose tag is
    `tag` (key -> list of floats); rows of other kernel versions are ignored."""
    path = os.path.join(PROFILES, name)
    out = {}
    if not os.path.exists(path):
        return out
    pat = re.compile(r"^\|\s*(\S+)\s*\|\s*([0-9a-f]{16})\s*\|((?:\s*[-+0-9.eE]+\s*\|)+)\s*$")
    with open(path) as fh:
        for line in fh:
            m = pat.match(line.strip())
            if m and m.group(2) == tag:
                out[m.group(1)] = [float(v) for v in m.group(3).split("|") if v.strip()]
    return out


def qi_traffic(key: str):
    """HBM bytes per batch of the query-insert kernels from the counter runs
    in profiles/query_insert_counters.md (FETCH_SIZE and WRITE_SIZE, scaled by
    a plain copy), for the kernel version built here and the workload and
    batch size `key` names ("<workload>_b<documents per batch>"); None
    otherwise."""
    rows = profile_rows("query_insert_counters.md", source_tag("qi_binned.hip", "qi_binned.h", "device_math.h", "launch_order.h"))
    r = rows.get(key)
    return None if r is None else r[0] + r[1]


def minhash_ops_per_shingle(workload: str, ppl: int, w: int):
    """VALU lane-operations the k_minhash<PPL, w> instance issues per shingle
    on `workload`'s documents (SQ_INSTS_VALU x 64 / shingles, from the counter
    runs in profiles/k_minhash_valu_counters.md) for the kernel version built
    here; None otherwise."""
    rows = profile_rows("k_minhash_valu_counters.md", source_tag("kernels.hip", "device_math.h"))
    r = rows.get(f"{workload}_ppl{ppl}_w{w}")
    return None if r is None else r[0]


def minhash_ppl(num_perm: int) -> int:
    """Permutations per lane of the k_minhash instance launched for num_perm."""
    return (num_perm + 63) // 64


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c3", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--loads", default="1000,2000,10000,50000,250000,1000000,2000000",
                    help="c5: offered loads in docs/s")
    ap.add_argument("--requests", type=int, default=1000, help="c5: requests per offered load")
    ap.add_argument("--preload", type=int, default=None, help="c5: documents inserted before serving")
    ap.add_argument("--cpu-sample-docs", type=int, default=None,
                    help="documents the single-thread oracle is timed on (default: the workload's)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--qi-mode", type=int, default=0, help="0 automatic, 1 direct, 2 binned query-insert")
    ap.add_argument("--form", default=None, choices=["plain", "batched", "fidelity"],
                    help="batched (default for c3): host CSR in, host flags out through the pipeline "
                         "(length buckets, overlapping slots, hipGraph, autotuner), beside plain per-batch calls "
                         "fed the same host batches and plain calls on inputs already in HBM; plain (default "
                         "for c2): per-batch calls on HBM-resident inputs; fidelity: LSHBloom against the exact "
                         "MinHashLSH band index on the same signatures, scored on the corpus's near-dup labels")
    ap.add_argument("--full-stream", action="store_true",
                    help="c4: run the whole 1e9-signature stream (1,000 batches) and check the flagged fraction "
                         "of unique signatures against the p_eff composition law")
    ap.add_argument("--wide", action="store_true",
                    help="plain form: the wide-value variant (61-bit MinHash values, their band keys, "
                         "query-insert from keys) in each step")
    ap.add_argument("--batch", type=int, default=None,
                    help="documents per batch (default: the workload's)")
    ap.add_argument("--chunk-docs", type=int, default=None,
                    help="documents per in-order query-insert chunk (default: the batch)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, one device-to-device copy of this many bytes "
                         "(calibrates the HBM byte counters against a plain copy)")
    ap.add_argument("--probe-hbm", type=int, default=0, metavar="GB",
                    help="instead of a workload: measure the memory system's ceilings with torch's own kernels "
                         "(streaming copy, random 8-byte gather and scatter over a GB-sized buffer) and exit")
    a = ap.parse_args()
    if a.form is None:
        a.form = "batched" if a.workload == "c3" else "plain"
    default_steps = {"c2": (13, 2), "c3": (20, 5), "c4": (20, 2), "c5": (0, 0)}[a.workload]
    if a.steps is None:
        a.steps = default_steps[0]
    if a.warmup is None:
        a.warmup = default_steps[1]
    if a.cpu_sample_docs is None:
        a.cpu_sample_docs = {"c2": 3072, "c3": 20000}.get(a.workload, 3072)
    return a


def shingle_count(lengths, w=5):
    import numpy as np

    return int(np.where(lengths >= w, lengths - w + 1, np.minimum(lengths, 1)).sum())


def cpu_baseline(wl, h_off, h_tok, n_docs):
    """The oracle, single-threaded, over the first n_docs documents of the
    same stream (MinHash + in-order query-insert with full-size filters), and
    the same oracle with its MinHash over the host's cores on 8x as many."""
    import numpy as np

    import oracle

    off = np.ascontiguousarray(h_off[: n_docs + 1])
    tok = h_tok[: int(off[-1])].view(np.uint32)
    o = oracle.OracleIndex(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    t0 = time.perf_counter()
    sigs = o.minhash(off, tok)
    o.query_insert(sigs)
    dt = time.perf_counter() - t0
    o.close()
    out = {"value": n_docs / dt, "unit": "docs/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n_docs} documents of the same stream ({int(off[-1])} tokens), "
                     f"MinHash + in-order query-insert against full-size filters, single thread, {dt:.1f} s"}

    # The same oracle with MinHash shared out over the host's cores (each
    # document still the sequential per-document definition) and the
    # query-insert sequential, as the paper's own system runs the CPU path.
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    n_par = min(len(h_off) - 1, 8 * n_docs)
    off = np.ascontiguousarray(h_off[: n_par + 1])
    tok = h_tok[: int(off[-1])].view(np.uint32)
    o = oracle.OracleIndex(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    t0 = time.perf_counter()
    sigs = o.minhash_threads(off, tok, threads)
    o.query_insert(sigs)
    dt = time.perf_counter() - t0
    o.close()
    out["parallel_minhash"] = {
        "value": n_par / dt, "unit": "docs/s", "cores": threads,
        "sample": f"first {n_par} documents of the same stream ({int(off[-1])} tokens), MinHash over "
                  f"{threads} host threads + sequential in-order query-insert, {dt:.1f} s"}
    return out


SECTOR = 64  # bytes per random HBM access


def qi_algorithmic_bytes(steps, batch, probes, new_bits, num_perm):
    """Algorithmic HBM bytes of `steps` query-insert batches: one sector read
    per probe, one sector write per newly set bit, the signatures read once
    and one flag byte per document."""
    return SECTOR * (steps * probes + new_bits) + steps * batch * (4 * num_perm + 1)


def qi_roofline(wl, args, batch, probes, new_bits, qi_ms, filter_bytes, traffic_key):
    """Roofline object of the query-insert stage: algorithmic bytes per batch
    over the mean stage time measured with HIP events on its stream."""
    import numpy as np

    steps = len(qi_ms)
    per_batch = qi_algorithmic_bytes(steps, batch, probes, new_bits, wl.num_perm) / steps
    ach = per_batch / (float(np.mean(qi_ms)) * 1e-3)
    traffic = qi_traffic(f"{traffic_key}_b{batch}") if traffic_key else None
    roof = {
        "bound": "hbm",
        "kernel": "query-insert (all kernels of a batch's in-order test-and-set)",
        "achieved": ach / 1e9, "peak": HBM_PEAK / 1e9, "unit": "GB/s", "frac": ach / HBM_PEAK,
        "traffic": traffic,
        "algorithmic_bytes_per_batch": per_batch,
        "new_bits_per_batch": new_bits / steps,
        "probes_per_batch": probes,
        "stage_ms_mean": float(np.mean(qi_ms)),
        "probes_per_s": probes / (float(np.mean(qi_ms)) * 1e-3),
    }
    if traffic:
        roof["traffic_GBps"] = traffic / (float(np.mean(qi_ms)) * 1e-3) / 1e9
        roof["traffic_over_algorithmic"] = traffic / per_batch
    if filter_bytes < CACHE_BYTES:
        roof["note"] = "filters fit the 256 MB last-level cache: random reads are served by the cache"
    return roof


def minhash_roofline(wl, workload, shingles, mh_ms, kernel):
    """Roofline object of the MinHash stage.  `shingle_perm_per_s` is the
    algorithmic rate (shingle x permutation evaluations per second).
    `achieved` prices each shingle at the VALU lane-operations its k_minhash
    instance issues per shingle on this workload (SQ_INSTS_VALU of this
    kernel version), so `frac` is the stage's share of the INT32 VALU issue
    peak (None when the instance has no counter profile)."""
    import numpy as np

    per_s = float(np.mean([sh * wl.num_perm / (t * 1e-3) for sh, t in zip(shingles, mh_ms)]))
    ops = minhash_ops_per_shingle(workload, minhash_ppl(wl.num_perm), 5)
    roof = {"bound": "alu", "kernel": kernel, "achieved": None, "peak": INT32_VALU_PEAK / 1e12,
            "unit": "TOPS (int32 VALU lane-ops/s)", "frac": None, "traffic": None,
            "shingle_perm_per_s": per_s, "stage_ms_mean": float(np.mean(mh_ms))}
    if ops:
        ach = float(np.mean([sh * ops / (t * 1e-3) for sh, t in zip(shingles, mh_ms)]))
        roof.update(achieved=ach / 1e12, frac=ach / INT32_VALU_PEAK, ops_per_shingle=ops)
    return roof


def _events(n):
    import torch

    return [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(n)]


def _index(args, wl, lshbloom):
    chunk = wl.batch if args.chunk_docs is None else args.chunk_docs
    # binned workspace: 24 bytes per probe of a chunk
    budget = 24 * chunk * wl.bands * 40 + (64 << 20)
    return lshbloom.LSHBloom(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed,
                             chunk_docs=chunk if args.qi_mode != 1 else 0, qi_mode=args.qi_mode,
                             workspace_budget=budget)


def make_stream(args, wl, torch, synth, dev):
    """The workload's recipe drawn for warmup + steps batches (beyond the
    configuration's own document count when more batches are asked for: the
    near-duplicate sources then range over the whole longer stream)."""
    n = wl.batch * (args.warmup + args.steps)
    t = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=n)
    torch.cuda.synchronize()
    return corpus, time.perf_counter() - t


def run_plain_device(args, wl, torch, np, lshbloom, corpus, steps, warmup, wide=False):
    """Plain per-batch calls on inputs in HBM: MinHash + query-insert of each
    batch on torch's current stream, each stage bracketed by HIP events."""
    B = wl.batch
    n_batches = warmup + steps
    dev = corpus.offsets.device
    idx = _index(args, wl, lshbloom)
    sigs = torch.empty((B, wl.num_perm), dtype=torch.int64 if wide else torch.int32, device=dev)
    flags = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    offs = [corpus.offsets[b * B:(b + 1) * B + 1] for b in range(n_batches)]

    def mh(b):
        if wide:
            idx.minhash61(offs[b], corpus.tokens, out=sigs)
        else:
            idx.minhash(offs[b], corpus.tokens, out=sigs)

    def qi(b):
        if wide:
            idx.query_insert_keys(idx.band_keys61(sigs), out=flags[b])
        else:
            idx.query_insert(sigs, out=flags[b])

    for b in range(warmup):
        mh(b)
        qi(b)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = _events(steps)
    bits0 = sum(idx.count_set_bits())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(steps):
        b = warmup + s
        ev[s][0].record(stream)
        mh(b)
        ev[s][1].record(stream)
        qi(b)
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    new_bits = sum(idx.count_set_bits()) - bits0
    idx.sync()
    mh_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(steps)]
    qi_ms = [ev[s][1].elapsed_time(ev[s][2]) for s in range(steps)]
    out = {"elapsed": elapsed, "mh_ms": mh_ms, "qi_ms": qi_ms, "new_bits": new_bits, "k": idx.k,
           "filter_bytes": idx.info()["filter_bytes"], "flags": flags}
    idx.close()
    return out


def run_corpus(args, wl, torch, np, lshbloom, synth, dev):
    """Plain per-batch form over a synthetic stream already in HBM."""
    B = wl.batch
    corpus, t_gen = make_stream(args, wl, torch, synth, dev)
    lengths = torch.diff(corpus.offsets).cpu().numpy()
    r = run_plain_device(args, wl, torch, np, lshbloom, corpus, args.steps, args.warmup, wide=args.wide)
    timed = range(args.warmup, args.warmup + args.steps)
    shingles = [shingle_count(lengths[b * B:(b + 1) * B]) for b in timed]
    tokens = [int(lengths[b * B:(b + 1) * B].sum()) for b in timed]
    probes = B * wl.bands * r["k"]
    minhash_roof = minhash_roofline(wl, args.workload, shingles, r["mh_ms"], "k_minhash (incl. its 0xFFFFFFFF pre-fill)")
    qi_roof = qi_roofline(wl, args, B, probes, r["new_bits"], r["qi_ms"], r["filter_bytes"],
                          None if args.wide else args.workload)
    if args.wide:
        # the wide kernel does more than the 32-bit operation count per
        # evaluation: its VALU fraction is not reported on that count
        minhash_roof = dict(minhash_roof, kernel="k_minhash (wide values)", achieved=None, frac=None)
        qi_roof = dict(qi_roof, kernel="band keys of wide values + query-insert from keys")
    dominant = minhash_roof if np.mean(r["mh_ms"]) >= np.mean(r["qi_ms"]) else qi_roof
    res = {
        "value": args.steps * B / r["elapsed"],
        "ms_per_step": r["elapsed"] * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "tokens_per_step": float(np.mean(tokens)),
        "text_GBps": float(np.sum(tokens)) * 4 / r["elapsed"] / 1e9,
        "stage_ms": {"minhash": float(np.mean(r["mh_ms"])), "query_insert": float(np.mean(r["qi_ms"]))},
        "roofline": dominant,
        "other_rooflines": [x for x in (minhash_roof, qi_roof) if x is not dominant],
        "flagged_frac": float(r["flags"][args.warmup:].float().mean().item()),
        "corpus_gen_s": t_gen,
    }
    if args.wide:
        res["variant"] = "wide (61-bit MinHash values, band keys of them, query-insert from keys)"
    h_off = corpus.offsets.cpu().numpy()
    h_tok = corpus.tokens[: int(h_off[min(len(h_off) - 1, 8 * args.cpu_sample_docs)])].cpu().numpy()
    return res, (h_off, h_tok)


def run_batched(args, wl, torch, np, lshbloom, synth, dev):
    """Batched form (the headline): host CSR batches through the pipeline,
    beside the plain per-batch calls fed the same host batches (H2D, MinHash,
    query-insert, D2H, one batch at a time) and plain calls on the same
    batches already in HBM, each with its own index."""
    B = wl.batch
    n_batches = args.warmup + args.steps
    corpus, t_gen = make_stream(args, wl, torch, synth, dev)
    lengths = torch.diff(corpus.offsets).cpu().numpy()

    # plain calls on inputs in HBM (the device-resident rate)
    dres = run_plain_device(args, wl, torch, np, lshbloom, corpus, args.steps, args.warmup)
    dev_flags = dres.pop("flags")[args.warmup:].cpu()

    # host copies of the stream (pinned, so the pipeline moves tokens by DMA)
    t_pin = time.perf_counter()
    h_off = torch.empty(corpus.offsets.numel(), dtype=torch.int64, pin_memory=True)
    h_off.copy_(corpus.offsets)
    h_tok = torch.empty(corpus.tokens.numel(), dtype=torch.int32, pin_memory=True)
    h_tok.copy_(corpus.tokens)
    torch.cuda.synchronize()
    t_pin = time.perf_counter() - t_pin
    del corpus
    torch.cuda.empty_cache()
    max_tok = int(max(lengths[b * B:(b + 1) * B].sum() for b in range(n_batches)))
    offs = [h_off[b * B:(b + 1) * B + 1].clone().pin_memory() for b in range(n_batches)]

    # batched form
    idx = _index(args, wl, lshbloom)
    pl = lshbloom.Pipeline(idx, max_docs=B, max_tokens=max_tok, use_graph=True, autotune=True)
    flags = torch.zeros((n_batches, B), dtype=torch.uint8).pin_memory()
    for b in range(args.warmup):
        pl.wait(pl.submit(offs[b], h_tok, flags[b]))
    inf0 = pl.info()
    bits0 = sum(idx.count_set_bits())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    tickets = [pl.submit(offs[b], h_tok, flags[b]) for b in range(args.warmup, n_batches)]
    for t in tickets:
        pl.wait(t)
    elapsed = time.perf_counter() - t0
    torch.cuda.synchronize()
    inf1 = pl.info()
    new_bits = sum(idx.count_set_bits()) - bits0
    pl.close()
    idx.sync()
    filter_bytes = idx.info()["filter_bytes"]
    k = idx.k
    batched_flags = flags[args.warmup:].clone()
    idx.close()
    nb = inf1["timed_batches"] - inf0["timed_batches"]
    qi_ms_mean = (inf1["qi_ms_total"] - inf0["qi_ms_total"]) / nb
    mh_ms_mean = (inf1["minhash_ms_total"] - inf0["minhash_ms_total"]) / nb

    # plain per-batch calls on the same host batches
    idx = _index(args, wl, lshbloom)
    sigs = torch.empty((B, wl.num_perm), dtype=torch.int32, device=dev)
    pflags = torch.zeros((n_batches, B), dtype=torch.uint8).pin_memory()

    def plain(b):
        o = offs[b]
        doff = (o - o[0]).to(dev, non_blocking=True)
        dtok = h_tok[int(o[0]):int(o[-1])].to(dev, non_blocking=True)
        idx.minhash(doff, dtok, out=sigs)
        pflags[b].copy_(idx.query_insert(sigs), non_blocking=True)
        torch.cuda.synchronize()

    for b in range(args.warmup):
        plain(b)
    t1 = time.perf_counter()
    for b in range(args.warmup, n_batches):
        plain(b)
    plain_elapsed = time.perf_counter() - t1
    idx.sync()
    idx.close()

    timed = range(args.warmup, n_batches)
    tokens = [int(lengths[b * B:(b + 1) * B].sum()) for b in timed]
    shingles = [shingle_count(lengths[b * B:(b + 1) * B]) for b in timed]
    probes = B * wl.bands * k
    qi_roof = qi_roofline(wl, args, B, probes, new_bits, [qi_ms_mean] * args.steps, filter_bytes, args.workload)
    qi_roof["timing"] = ("HIP events on the pipeline's query-insert stream around each batch's query-insert "
                         f"kernels, mean over the {nb} timed batches")
    mh_roof = minhash_roofline(wl, args.workload, shingles, [mh_ms_mean] * args.steps,
                               "k_minhash, one launch per length bucket (incl. the signature pre-fill)")
    mh_roof["timing"] = "HIP events on the pipeline's MinHash stream around each batch's MinHash stage"
    dominant, other = (qi_roof, mh_roof) if qi_ms_mean >= mh_ms_mean else (mh_roof, qi_roof)
    same = bool(torch.equal(batched_flags, pflags[args.warmup:])) and bool(torch.equal(batched_flags, dev_flags))
    res = {
        "value": args.steps * B / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "tokens_per_step": float(np.mean(tokens)),
        "text_GBps": float(np.sum(tokens)) * 4 / elapsed / 1e9,
        "form": "batched (host CSR in, host flags out; length buckets, 2 overlapping slots, hipGraph, autotuner)",
        "stage_ms": {"minhash": mh_ms_mean, "query_insert": qi_ms_mean},
        "roofline": dominant,
        "other_rooflines": [other],
        "plain_per_batch_from_host": {"value": args.steps * B / plain_elapsed,
                                      "ms_per_step": plain_elapsed * 1e3 / args.steps,
                                      "form": "per batch: H2D copy, MinHash, query-insert, D2H flags, synchronise"},
        "plain_device_resident": {"value": args.steps * B / dres["elapsed"],
                                  "ms_per_step": dres["elapsed"] * 1e3 / args.steps,
                                  "stage_ms": {"minhash": float(np.mean(dres["mh_ms"])),
                                               "query_insert": float(np.mean(dres["qi_ms"]))},
                                  "form": "per batch: MinHash + query-insert on inputs already in HBM"},
        "speedup_vs_plain_from_host": plain_elapsed / elapsed,
        "flags_identical_across_forms": same,
        "pipeline": {k_: v for k_, v in inf1.items() if k_ not in ("minhash_ms_total", "qi_ms_total")},
        "flagged_frac": float(batched_flags.float().mean().item()),
        "corpus_gen_s": t_gen,
        "host_copy_s": t_pin,
    }
    n_cpu = min(len(h_off) - 1, 8 * args.cpu_sample_docs)
    return res, (h_off.numpy(), h_tok[: int(h_off[n_cpu])].numpy())


def _scores(flags, truth):
    tp = int((flags & truth).sum())
    fp = int((flags & ~truth).sum())
    fn = int((~flags & truth).sum())
    prec = tp / (tp + fp) if tp + fp else 1.0
    rec = tp / (tp + fn) if tp + fn else 1.0
    f1 = 2 * prec * rec / (prec + rec) if prec + rec else 0.0
    return {"flagged": int(flags.sum()), "tp": tp, "fp": fp, "fn": fn, "precision": prec, "recall": rec, "f1": f1}


def _recall_by_j(np, target_j, truth, fb, fe):
    """Recall of each index per band of the generator's target Jaccard."""
    out = []
    for lo, hi in [(0.6, 0.7), (0.7, 0.8), (0.8, 0.9), (0.9, 0.951)]:
        sel = truth & (target_j >= lo) & (target_j < hi)
        k = int(sel.sum())
        out.append({"target_j": [lo, min(hi, 0.95)], "near_dups": k,
                    "lshbloom": float(fb[sel].mean()) if k else None, "exact": float(fe[sel].mean()) if k else None})
    return out


def run_fidelity(args, wl, torch, np, lshbloom, synth, dev):
    """LSHBloom against the exact MinHashLSH band index (Section 2's index,
    which LSHBloom replaces) on the same GPU signatures of a labelled corpus:
    precision, recall and F1 of each against the generator's near-duplicate
    labels (a document is a near-duplicate iff it was made from an earlier
    one), the documents only LSHBloom flags, and each index's query-insert
    time and size."""
    B = wl.batch
    n_batches = args.warmup + args.steps
    n = B * n_batches
    corpus, t_gen = make_stream(args, wl, torch, synth, dev)
    truth = np.asarray(corpus.is_dup[:n]).astype(bool)

    idx = _index(args, wl, lshbloom)
    ex = lshbloom.ExactLSH(wl.num_perm, wl.bands, wl.rows, capacity_docs=n)
    sigs = torch.empty((B, wl.num_perm), dtype=torch.int32, device=dev)
    fb = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    fe = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    stream = torch.cuda.current_stream()
    ev = _events(n_batches)
    for b in range(n_batches):
        idx.minhash(corpus.offsets[b * B:(b + 1) * B + 1], corpus.tokens, out=sigs)
        ev[b][0].record(stream)
        idx.query_insert(sigs, out=fb[b])
        ev[b][1].record(stream)
        ex.query_insert(sigs, out=fe[b])
        ev[b][2].record(stream)
    torch.cuda.synchronize()
    timed = range(args.warmup, n_batches)
    bloom_ms = float(np.mean([ev[b][0].elapsed_time(ev[b][1]) for b in timed]))
    exact_ms = float(np.mean([ev[b][1].elapsed_time(ev[b][2]) for b in timed]))
    fb_h = fb.cpu().numpy().reshape(-1).astype(bool)
    fe_h = fe.cpu().numpy().reshape(-1).astype(bool)
    sb, se = _scores(fb_h, truth), _scores(fe_h, truth)
    inf = idx.info()
    bloom_bytes = inf["m_bits"] // 8 * wl.bands
    st = ex.stats()
    res = {
        "value": sb["f1"] - se["f1"],
        "ms_per_step": bloom_ms,
        "docs_timed": args.steps * B,
        "labelled_near_dups": int(truth.sum()),
        "lshbloom": dict(sb, qi_ms_per_batch=bloom_ms, docs_per_s=B / (bloom_ms * 1e-3), index_bytes=bloom_bytes),
        "exact_minhashlsh": dict(se, qi_ms_per_batch=exact_ms, docs_per_s=B / (exact_ms * 1e-3),
                                 index_bytes=st["table_bytes"], fingerprints_shared=st["fp_shared"]),
        "recall_by_target_jaccard": _recall_by_j(np, corpus.target_j[:n], truth, fb_h, fe_h),
        "exact_flags_missing_from_lshbloom": int((fe_h & ~fb_h).sum()),
        "lshbloom_only_flags": int((fb_h & ~fe_h).sum()),
        "index_size_ratio": st["table_bytes"] / bloom_bytes,
        "corpus_gen_s": t_gen,
    }
    ex.close()
    return res, None


def run_signatures(args, wl, torch, np, lshbloom, synth, dev):
    """Filter-scale query-insert: batches of precomputed signatures only."""
    if args.full_stream:
        return run_signature_stream(args, wl, torch, np, lshbloom, synth, dev)
    B = wl.batch
    n_batches = args.warmup + args.steps
    idx = _index(args, wl, lshbloom)
    ex = wl.extra
    t_gen = time.perf_counter()
    batches = [synth.signature_batch(b * B, B, wl.num_perm, wl.bands, wl.rows, B, ex["repeat_frac"],
                                     ex["in_batch_frac"], wl.corpus_seed, device=dev) for b in range(n_batches)]
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    flags = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    for b in range(args.warmup):
        idx.query_insert(batches[b], out=flags[b])
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = _events(args.steps)
    bits0 = sum(idx.count_set_bits())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        b = args.warmup + s
        ev[s][0].record(stream)
        idx.query_insert(batches[b], out=flags[b])
        ev[s][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    new_bits = sum(idx.count_set_bits()) - bits0
    idx.sync()
    qi_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]
    probes = B * wl.bands * idx.k
    rep, _ = synth.signature_repeat_info(args.warmup * B, args.steps * B, wl.bands, B, ex["repeat_frac"],
                                         ex["in_batch_frac"], wl.corpus_seed, device=dev)
    fl = flags[args.warmup:].reshape(-1)
    res = {
        "value": args.steps * B / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "stage_ms": {"query_insert": float(np.mean(qi_ms))},
        "roofline": qi_roofline(wl, args, B, probes, new_bits, qi_ms, idx.info()["filter_bytes"], "c4"),
        "repeats_flagged": float(fl[rep].float().mean().item()),
        "non_repeats_flagged": float(fl[~rep].float().mean().item()),
        "filter_bytes": idx.info()["filter_bytes"],
        "sig_gen_s": t_gen,
    }
    idx.close()
    return res, None


def run_signature_stream(args, wl, torch, np, lshbloom, synth, dev):
    """The whole filter-scale stream: wl.n_docs signatures in batches of
    wl.batch, generated on the device one batch ahead of its query-insert.
    Every repeat (a band copied from an earlier signature) must be flagged;
    the flags of the other signatures are false positives, whose count is
    compared with the p_eff composition law (Section 4.3): a unique signature
    arriving when band j's filter has X_j of its m bits set is flagged with
    probability 1 - prod_j (1 - (X_j / m)^k), X_j read every `every` batches
    and interpolated linearly in between."""
    import math

    B = wl.batch
    n_batches = wl.n_docs // B
    ex = wl.extra
    idx = _index(args, wl, lshbloom)
    k, m = idx.k, idx.m_bits
    every = 25
    flags = torch.empty(B, dtype=torch.uint8, device=dev)
    missed = torch.zeros((), dtype=torch.int64, device=dev)
    fp_flags = torch.zeros((), dtype=torch.int64, device=dev)
    n_rep = torch.zeros((), dtype=torch.int64, device=dev)
    expect = 0.0
    reps_seen = 0
    fill = [np.zeros(wl.bands)]
    stream = torch.cuda.current_stream()
    qi_ms = []
    t0 = time.perf_counter()
    nxt = synth.signature_batch(0, B, wl.num_perm, wl.bands, wl.rows, B, ex["repeat_frac"], ex["in_batch_frac"],
                                wl.corpus_seed, device=dev)
    for b in range(n_batches):
        sigs = nxt
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        idx.query_insert(sigs, out=flags)
        e1.record(stream)
        qi_ms.append((e0, e1))
        rep, _ = synth.signature_repeat_info(b * B, B, wl.bands, B, ex["repeat_frac"], ex["in_batch_frac"],
                                             wl.corpus_seed, device=dev)
        missed += (flags[rep] == 0).sum()
        fp_flags += flags[~rep].sum(dtype=torch.int64)
        n_rep += rep.sum()
        if b + 1 < n_batches:
            nxt = synth.signature_batch((b + 1) * B, B, wl.num_perm, wl.bands, wl.rows, B, ex["repeat_frac"],
                                        ex["in_batch_frac"], wl.corpus_seed, device=dev)
        if (b + 1) % every == 0 or b + 1 == n_batches:
            x1 = np.array(idx.count_set_bits(), dtype=np.float64)
            x0 = fill[-1]
            nb = (b + 1) - (len(fill) - 1) * every
            reps_now = int(n_rep.item())
            uniq = B * nb - (reps_now - reps_seen)
            reps_seen = reps_now
            # expected false flags of the unique signatures of these batches
            # (midpoint rule over the interval's fill)
            steps = 64
            p_sum = 0.0
            for q in range(steps):
                x = x0 + (x1 - x0) * (q + 0.5) / steps
                p_band = (x / m) ** k
                p_sum += -math.expm1(float(np.sum(np.log1p(-p_band))))
            expect += p_sum / steps * uniq
            fill.append(x1)
            print(f"[c4 stream] {b + 1}/{n_batches} batches, {time.perf_counter() - t0:.0f} s, "
                  f"fill {x1.mean() / m:.4f}, missed repeats {int(missed.item())}, "
                  f"false flags {int(fp_flags.item())} (expected so far {expect:.3f})", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    idx.sync()
    ms = [a_.elapsed_time(b_) for a_, b_ in qi_ms]
    n_unique = wl.n_docs - int(n_rep.item())
    obs = int(fp_flags.item())
    # two-sided 99.9% Poisson interval for the observed count given the expectation
    from scipy.stats import poisson
    lo, hi = poisson.ppf(0.0005, expect), poisson.ppf(0.9995, expect)
    res = {
        "value": wl.n_docs / elapsed,
        "ms_per_step": elapsed * 1e3 / n_batches,
        "docs_timed": wl.n_docs,
        "stage_ms": {"query_insert": float(np.mean(ms))},
        "full_stream": {
            "signatures": wl.n_docs, "batches": n_batches, "repeats": int(n_rep.item()),
            "repeats_not_flagged": int(missed.item()), "unique": n_unique,
            "unique_flagged": obs, "unique_flagged_expected_p_eff": expect,
            "poisson_99_9_interval": [float(lo), float(hi)],
            "p9_holds": bool(lo <= obs <= hi), "final_fill": float(fill[-1].mean() / m),
            "elapsed_s_incl_generation": elapsed, "query_insert_ms_mean": float(np.mean(ms)),
        },
        "filter_bytes": idx.info()["filter_bytes"],
    }
    idx.close()
    return res, None


def run_serve(args, wl, torch, np, lshbloom, synth, dev):
    """Served form: Poisson request streams at several offered loads against
    filters preloaded with 1e8 documents; continuous batching vs one request
    at a time (the plain per-batch form).  Every run starts from the same
    preloaded filter state (restored from a device snapshot) and serves the
    same documents."""
    import copy

    from paper_2411_04257_amd import serve

    loads = [float(x) for x in args.loads.split(",")]
    n_reqs = [args.requests for _ in loads]
    preload_n = wl.extra["preload"] if args.preload is None else args.preload
    rng = np.random.default_rng(wl.corpus_seed)
    warm = serve.poisson_requests(8, 10000.0, wl.extra["req_min"], wl.extra["req_max"], 0, rng)
    sizes = serve.poisson_requests(max(n_reqs), 1.0, wl.extra["req_min"], wl.extra["req_max"], warm[-1].hi, rng)
    n_docs = sizes[-1].hi
    t_gen = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=n_docs)
    h_off = corpus.offsets.cpu().pin_memory()
    h_tok = corpus.tokens.cpu().pin_memory()
    del corpus
    t_gen = time.perf_counter() - t_gen
    max_docs = 16384
    max_tokens = int(max_docs * 8000)

    idx_b = lshbloom.LSHBloom(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    idx_p = lshbloom.LSHBloom(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    t_pre = time.perf_counter()
    serve.preload(idx_b, preload_n, 1)
    t_pre = time.perf_counter() - t_pre
    snap = idx_b.read_filters()
    srv = serve.Server(idx_b, max_docs, max_tokens, hbm_budget=2 << 30)
    plain = serve.PlainServer(idx_p, max_docs, max_tokens)
    fb = torch.zeros(n_docs, dtype=torch.uint8).pin_memory()
    fp_ = torch.zeros(n_docs, dtype=torch.uint8).pin_memory()
    rows = []
    for ld, nr in [(10000.0, None)] + list(zip(loads, n_reqs)):
        if nr is None:
            reqs = warm  # warm-up stream: first-use costs, not reported
        else:
            base = serve.poisson_requests(nr, ld, wl.extra["req_min"], wl.extra["req_max"], 0,
                                          np.random.default_rng(int(ld)))
            reqs = [serve.Request(q.rid, b.arrival, q.lo, q.hi) for q, b in zip(sizes[:nr], base)]
        for idx in (idx_b, idx_p):
            idx.write_filters(snap, docs_inserted=preload_n)
        torch.cuda.synchronize()
        print(f"[c5] offered {ld:.0f} docs/s: {len(reqs)} requests, continuous batching", file=sys.stderr, flush=True)
        rb = srv.run(copy.deepcopy(reqs), h_off, h_tok, fb, progress_s=30.0).summary()
        print(f"[c5] offered {ld:.0f} docs/s: one request per batch", file=sys.stderr, flush=True)
        rp = plain.run(copy.deepcopy(reqs), h_off, h_tok, fp_, progress_s=30.0).summary()
        if nr is None:
            continue
        lo, hi = reqs[0].lo, reqs[-1].hi
        rows.append({"offered_docs_per_s": ld, "requests": len(reqs), "docs": int(hi - lo),
                     "tokens": int(h_off[hi] - h_off[lo]),
                     "continuous_batching": rb, "plain_one_request_per_batch": rp,
                     "flags_identical": bool(torch.equal(fb[lo:hi], fp_[lo:hi]))})
    srv.close()
    plain.close()
    assert idx_b.info()["device_status"] == 0 and idx_p.info()["device_status"] == 0
    top = rows[-1]
    res = {
        "value": top["continuous_batching"]["p99_ms"],
        "ms_per_step": top["continuous_batching"]["mean_ms"],
        "docs_timed": int(sum(r["docs"] for r in rows)),
        "loads": rows,
        "preload_docs": preload_n,
        "preload_s": t_pre,
        "filter_bytes": idx_b.info()["filter_bytes"],
        "corpus_gen_s": t_gen,
    }
    idx_b.close()
    idx_p.close()
    return res, None


def probe_hbm(torch, gb):
    """Ceilings of the memory system, measured with torch's kernels (not this
    library's): a streaming device copy, and uniformly random 8-byte gathers
    and scatters over a `gb`-GB buffer.  Each random access touches its own
    64-byte sector; the gather also reads its index and writes its value
    sequentially (16 bytes per access)."""
    n = gb * (1 << 27)
    buf = torch.zeros(n, dtype=torch.int64, device="cuda")
    m = 1 << 27
    gen = torch.Generator(device="cuda")
    gen.manual_seed(5)
    idx = torch.randint(0, n, (m,), device="cuda", generator=gen)
    vals = torch.empty(m, dtype=torch.int64, device="cuda")
    src = torch.ones(1 << 30, dtype=torch.int64, device="cuda")
    dst = torch.empty_like(src)

    def timed(fn, reps=5):
        fn()
        torch.cuda.synchronize()
        ms = []
        for _ in range(reps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            fn()
            b.record()
            b.synchronize()
            ms.append(a.elapsed_time(b))
        return min(ms)

    t_copy = timed(lambda: dst.copy_(src))
    t_gather = timed(lambda: torch.index_select(buf, 0, idx, out=vals))
    t_scatter = timed(lambda: buf.index_copy_(0, idx, vals))
    # random read-modify-writes: accumulate into random words (device atomics)
    t_atomic = timed(lambda: buf.index_put_((idx,), vals, accumulate=True))
    # The same random accesses into a buffer the size of the 1M-document
    # workload's filters (57.5 MB), which the 256 MB last-level cache holds.
    small_n = 57_510_400 // 8
    small = torch.zeros(small_n, dtype=torch.int64, device="cuda")
    sidx = torch.randint(0, small_n, (m,), device="cuda", generator=gen)
    t_sgather = timed(lambda: torch.index_select(small, 0, sidx, out=vals))
    t_sscatter = timed(lambda: small.index_copy_(0, sidx, vals))
    return {
        "probe": "hbm ceilings with torch kernels",
        "buffer_GB": gb,
        "copy_GBps_read_plus_write": 2 * src.numel() * 8 / (t_copy * 1e-3) / 1e9,
        "gather_accesses_per_s": m / (t_gather * 1e-3),
        "gather_GBps_at_64B_sectors": m * 64 / (t_gather * 1e-3) / 1e9,
        "scatter_accesses_per_s": m / (t_scatter * 1e-3),
        "atomic_add_accesses_per_s": m / (t_atomic * 1e-3),
        "cache_resident_buffer_MB": small_n * 8 / 1e6,
        "cache_resident_gather_accesses_per_s": m / (t_sgather * 1e-3),
        "cache_resident_scatter_accesses_per_s": m / (t_sscatter * 1e-3),
        "accesses": m,
    }


DESCRIPTIONS = {
    "c2": "plain method on GPU: 1M-doc synthetic corpus (Zipf(1.1)/50k-vocab uint32 tokens, lognormal lengths "
          "median 3000 sigma 0.8 cap 50000, 20% near-dups J 0.6-0.95), 5-shingles, num_perm 128, 16 bands x 8 rows, "
          "filters n=1M fp=1e-6, batches of {batch:,}",
    "c3": "batched-form configuration (c3): synthetic corpus with Pareto(1.5, min 20, cap 200k) lengths, "
          "Zipf(1.1)/50k vocab, 25% near-dups; num_perm 256, 32 bands x 8 rows, filters n=100M fp=1e-8 per band "
          "(15.3 GB), batches of {batch:,}",
    "c4": "filter-scale query-insert: 1B-signature stream of uniform uint32 (256 wide) with 30% one-band repeats, "
          "32 bands x 8 rows, filters n=1e9 fp=1e-10 per band (191.7 GB in HBM), batches of {batch:,}",
    "c5": "serving: Poisson arrivals of 1-4096-document requests (log-uniform), lognormal lengths median 2000 "
          "sigma 0.8, Zipf(1.1)/50k vocab, 15% near-dups of earlier served docs; filters preloaded with 1e8 "
          "documents (num_perm 128, 16 bands x 8 rows, fp 1e-8 per band, 7.7 GB); continuous batching with "
          "HBM-budget admission vs one request per batch",
}


def stream_note(args, wl) -> str:
    if args.workload == "c4":
        return "; the whole 1e9-signature stream" if args.full_stream else "; a timed prefix of the stream"
    if args.workload not in ("c2", "c3"):
        return ""
    n = wl.batch * (args.warmup + args.steps)
    note = (f"; stream: {args.warmup + args.steps} full batches ({n:,} documents: {args.warmup} warmup, "
            f"{args.steps} timed) drawn from this recipe")
    if n > wl.n_docs:
        note += (f", past the configuration's {wl.n_docs:,} documents (near-duplicate sources range over the "
                 f"whole stream; the filters are sized for n = {wl.expected_n:,})")
    return note


def main():
    args = parse()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on exactly one GPU: the LSHBloom hot path here is single-GPU "
              "(multi-GPU band sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_2411_04257_amd import lshbloom, synth

    torch.cuda.set_device(0)
    dev = torch.device("cuda:0")
    if args.probe_hbm:
        print(json.dumps(probe_hbm(torch, args.probe_hbm)), flush=True)
        return
    wl = synth.WORKLOADS[args.workload]
    if args.batch:
        wl = dataclasses.replace(wl, batch=args.batch)
    higher = True
    if args.workload == "c4":
        res, host_stream = run_signatures(args, wl, torch, np, lshbloom, synth, dev)
        metric = "signatures/sec query-insert (band Bloom), bit-exact flags"
        unit = "sigs/s"
    elif args.workload == "c5":
        res, host_stream = run_serve(args, wl, torch, np, lshbloom, synth, dev)
        metric = "p99 serve latency (ms) at the highest offered load, continuous batching"
        unit = "ms"
        higher = False
    elif args.form == "fidelity":
        res, host_stream = run_fidelity(args, wl, torch, np, lshbloom, synth, dev)
        metric = "F1 gap, LSHBloom minus exact MinHashLSH, on the same signatures (near-dup labels)"
        unit = "F1"
    elif args.form == "batched":
        res, host_stream = run_batched(args, wl, torch, np, lshbloom, synth, dev)
        metric = "docs/sec end-to-end (MinHash+band Bloom), bit-exact flags"
        unit = "docs/s"
    else:
        res, host_stream = run_corpus(args, wl, torch, np, lshbloom, synth, dev)
        metric = "docs/sec end-to-end (MinHash+band Bloom), bit-exact flags"
        unit = "docs/s"

    if args.workload == "c4" and args.full_stream:
        args.steps, args.warmup = wl.n_docs // wl.batch, 0
    out = {
        "metric": metric,
        "value": res.pop("value"),
        "unit": unit,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res.pop("ms_per_step"),
        "higher_is_better": higher,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": DESCRIPTIONS[args.workload].format(batch=wl.batch) + stream_note(args, wl),
            "global_batch": wl.batch if args.workload != "c5" else None,
            "docs_timed": res.pop("docs_timed"),
            "parallelism": "single-gpu",
        },
    }
    if "tokens_per_step" in res:
        out["config"]["tokens_per_step"] = res.pop("tokens_per_step")
    out.update(res)
    if args.copy_bytes:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device=dev).fill_(7)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_bytes"] = args.copy_bytes
    if host_stream is not None and not args.no_cpu_baseline:
        h_off, h_tok = host_stream
        out["cpu_baseline"] = cpu_baseline(wl, h_off, h_tok, min(args.cpu_sample_docs, len(h_off) - 1))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
