#!/usr/bin/env python3
"""End-to-end LSHBloom throughput on one MI355X.

A step is one pass of the whole hot path over one batch of documents already
resident in HBM: MinHash signatures of the batch, then the in-order
query-insert against the per-band Bloom filters (which keep growing across
steps, as in a real stream).  The default workload is the plain method on
GPU: a 1M-document synthetic corpus (Zipf(1.1) tokens over a 50k vocabulary,
lognormal lengths with median 3,000 and sigma 0.8 capped at 50,000, 20%
near-duplicates with Jaccard 0.6-0.95), num_perm = 128, 16 bands x 8 rows,
filters sized for n = 1M at a per-band fp rate of 1e-6, batches of 65,536.

Prints one JSON line (rank 0) with docs/s, the MinHash kernel's ALU roofline
and the CPU oracle timed on a bounded prefix of the same stream.
"""

from __future__ import annotations

import argparse
import dataclasses
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Per-unit VALU lane-operation counts of the MinHash hot loops (gfx950 ISA of
# k_minhash<PPL=2, w=5>): one SHA-1 shingle hash of a 5-token shingle (573),
# and one exact (a*x+b) mod (2^61-1) evaluation in a full 64-shingle tile with
# its share of the running min and of the flag test (3 v_mad_u64_u32 + 1 add,
# 1/2 of a v_min3 and 1/2 of a v_max3, each folding two evaluations: 80
# instructions per 16 evaluations).
OPS_PER_SHINGLE_HASH = 573
OPS_PER_SHINGLE_PERM = 5.0
INT32_VALU_PEAK = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 3.93e13 lane-ops/s
# HBM bytes per token that k_minhash moved, from rocprofv3 FETCH_SIZE (x2.0) and
# WRITE_SIZE (x1.0) scaled by a 1 GiB copy (profiles/k_minhash_c2_counters.md):
# 1.1747e9 B for a 2.717e8-token batch (65,536 waves).  Valid for the kernel
# version and grid sizing profiled.
MINHASH_HBM_BYTES_PER_TOKEN = 1.1747e9 / 2.7175e8
# Random 8-byte gathers per second into a 57.5 MB buffer that the 256 MB
# last-level cache holds, measured with torch's index_select
# (`bench.py --probe-hbm 48`, profiles/hbm_ceilings_probe.md): the rate
# c2's query-insert probes are compared with, its filters being that size.
CACHE_RESIDENT_GATHER_PER_S = 5.33e10
CACHE_BYTES = 256e6


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", default="c2", choices=["c2", "c3", "c4", "c5"])
    ap.add_argument("--loads", default="2000,10000,50000,250000,1000000,2000000",
                    help="c5: offered loads in docs/s")
    ap.add_argument("--preload", type=int, default=None, help="c5: documents inserted before serving")
    ap.add_argument("--cpu-sample-docs", type=int, default=3072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--qi-mode", type=int, default=0, help="0 automatic, 1 direct, 2 binned query-insert")
    ap.add_argument("--form", default="plain", choices=["plain", "batched", "fidelity"],
                    help="plain: per-batch calls on HBM-resident inputs; batched: the host-to-host pipeline "
                         "(length buckets, overlapping slots, hipGraph, autotuner) compared with per-batch "
                         "calls that copy the same host batches; fidelity: LSHBloom against the exact "
                         "MinHashLSH band index on the same signatures, scored on the corpus's near-dup labels")
    ap.add_argument("--wide", action="store_true",
                    help="plain form: the wide-value variant (61-bit MinHash values, their band keys, "
                         "query-insert from keys) in each step")
    ap.add_argument("--batch", type=int, default=None,
                    help="documents per batch (default: the workload's; c3 leaves it open)")
    ap.add_argument("--chunk-docs", type=int, default=None,
                    help="documents per in-order query-insert chunk (default: the batch)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, one device-to-device copy of this many bytes "
                         "(calibrates the HBM byte counters against a plain copy)")
    ap.add_argument("--probe-hbm", type=int, default=0, metavar="GB",
                    help="instead of a workload: measure the memory system's ceilings with torch's own kernels "
                         "(streaming copy, random 8-byte gather and scatter over a GB-sized buffer) and exit")
    a = ap.parse_args()
    default_steps = {"c2": (13, 2), "c3": (9, 1), "c4": (20, 2), "c5": (0, 0)}[a.workload]
    if a.steps is None:
        a.steps = default_steps[0]
    if a.warmup is None:
        a.warmup = default_steps[1]
    return a


def shingle_count(lengths, w=5):
    import numpy as np

    return int(np.where(lengths >= w, lengths - w + 1, np.minimum(lengths, 1)).sum())


def cpu_baseline(wl, corpus, n_docs):
    """The oracle, single-threaded, over the first n_docs documents of the
    same stream (MinHash + in-order query-insert with full-size filters)."""
    import numpy as np

    import oracle

    off = corpus.offsets[: n_docs + 1].cpu().numpy()
    tok = corpus.tokens[: int(off[-1])].cpu().numpy().view(np.uint32)
    o = oracle.OracleIndex(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    t0 = time.perf_counter()
    sigs = o.minhash(off, tok)
    o.query_insert(sigs)
    dt = time.perf_counter() - t0
    o.close()
    out = {"value": n_docs / dt, "unit": "docs/s", "cores": 1, "kind": "oracle",
           "sample": f"first {n_docs} documents of the same stream ({int(off[-1])} tokens), "
                     f"MinHash + in-order query-insert, single thread, {dt:.1f} s"}

    # The same oracle with MinHash shared out over the host's cores (each
    # document still the sequential per-document definition) and the
    # query-insert sequential, as the paper's own system runs the CPU path.
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    n_par = min(corpus.n_docs, 8 * n_docs)
    off = corpus.offsets[: n_par + 1].cpu().numpy()
    tok = corpus.tokens[: int(off[-1])].cpu().numpy().view(np.uint32)
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


def run_corpus(args, wl, torch, np, lshbloom, synth, dev):
    """Plain per-batch form over a synthetic corpus: MinHash + query-insert per batch."""
    B = wl.batch
    n_batches = args.warmup + args.steps
    if B * n_batches > wl.n_docs:
        print(f"warmup + steps exceed the {wl.n_docs // B} full batches of the corpus", file=sys.stderr)
        sys.exit(2)
    n_docs = B * n_batches
    t_gen = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=n_docs)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    idx = _index(args, wl, lshbloom)
    sigs = torch.empty((B, wl.num_perm), dtype=torch.int64 if args.wide else torch.int32, device=dev)
    flags = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    offs = [corpus.offsets[b * B:(b + 1) * B + 1] for b in range(n_batches)]
    lengths = torch.diff(corpus.offsets).cpu().numpy()

    def mh(b):
        if args.wide:
            idx.minhash61(offs[b], corpus.tokens, out=sigs)
        else:
            idx.minhash(offs[b], corpus.tokens, out=sigs)

    def qi(b):
        if args.wide:
            idx.query_insert_keys(idx.band_keys61(sigs), out=flags[b])
        else:
            idx.query_insert(sigs, out=flags[b])

    for b in range(args.warmup):
        mh(b)
        qi(b)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = _events(args.steps)
    bits0 = sum(idx.count_set_bits())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        b = args.warmup + s
        ev[s][0].record(stream)
        mh(b)
        ev[s][1].record(stream)
        qi(b)
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    new_bits = sum(idx.count_set_bits()) - bits0
    assert idx.info()["device_status"] == 0

    mh_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]
    qi_ms = [ev[s][1].elapsed_time(ev[s][2]) for s in range(args.steps)]
    timed = range(args.warmup, n_batches)
    shingles = [shingle_count(lengths[b * B:(b + 1) * B]) for b in timed]
    tokens = [int(lengths[b * B:(b + 1) * B].sum()) for b in timed]
    ops = [sh * (OPS_PER_SHINGLE_HASH + wl.num_perm * OPS_PER_SHINGLE_PERM) for sh in shingles]
    mh_achieved = float(np.mean([o / (t * 1e-3) for o, t in zip(ops, mh_ms)]))
    probes = B * wl.bands * idx.k
    qi_bytes = qi_algorithmic_bytes(args.steps, B, probes, new_bits, wl.num_perm)
    qi_achieved = qi_bytes / (float(np.sum(qi_ms)) * 1e-3)
    minhash_roof = {
        "bound": "alu",
        "kernel": "k_minhash (incl. its 0xFFFFFFFF pre-fill)",
        "achieved": mh_achieved / 1e12,
        "peak": INT32_VALU_PEAK / 1e12,
        "unit": "TOPS (int32 VALU lane-ops/s)",
        "frac": mh_achieved / INT32_VALU_PEAK,
        "traffic": float(np.mean(tokens)) * MINHASH_HBM_BYTES_PER_TOKEN if wl.num_perm == 128 else None,
        "shingle_perm_per_s": float(np.mean([sh * wl.num_perm / (t * 1e-3) for sh, t in zip(shingles, mh_ms)])),
    }
    qi_roof = {
        "bound": "hbm",
        "kernel": "query-insert (all kernels of a batch's in-order test-and-set)",
        "achieved": qi_achieved / 1e9,
        "peak": 8000.0,
        "unit": "GB/s",
        "frac": qi_achieved / 8e12,
        "traffic": None,
        "algorithmic_bytes_per_batch": qi_bytes / args.steps,
        "new_bits_per_batch": new_bits / args.steps,
        "probes_per_s": float(np.mean([probes / (t * 1e-3) for t in qi_ms])),
    }
    if idx.info()["filter_bytes"] < CACHE_BYTES:
        qi_roof["cache_resident_gather_per_s"] = CACHE_RESIDENT_GATHER_PER_S
        qi_roof["probes_frac_of_cache_gather_rate"] = qi_roof["probes_per_s"] / CACHE_RESIDENT_GATHER_PER_S
    if args.wide:
        # the wide kernel does more than the 32-bit operation count per
        # evaluation: its VALU fraction is not reported on that count
        minhash_roof = dict(minhash_roof, kernel="k_minhash (wide values)", achieved=None, frac=None, traffic=None)
        qi_roof = dict(qi_roof, kernel="band keys of wide values + query-insert from keys")
    dominant = minhash_roof if np.mean(mh_ms) >= np.mean(qi_ms) else qi_roof
    res = {
        "value": args.steps * B / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "tokens_per_step": float(np.mean(tokens)),
        "text_GBps": float(np.sum(tokens)) * 4 / elapsed / 1e9,
        "stage_ms": {"minhash": float(np.mean(mh_ms)), "query_insert": float(np.mean(qi_ms))},
        "roofline": dominant,
        "other_rooflines": [r for r in (minhash_roof, qi_roof) if r is not dominant],
        "flagged_frac": float(flags[args.warmup:].float().mean().item()),
        "corpus_gen_s": t_gen,
    }
    if args.wide:
        res["variant"] = "wide (61-bit MinHash values, band keys of them, query-insert from keys)"
    return res, corpus, idx


def run_batched(args, wl, torch, np, lshbloom, synth, dev):
    """Batched form: host CSR batches through the pipeline, against the plain
    per-batch calls fed the same host batches (H2D, MinHash, query-insert,
    D2H, one batch at a time), each with its own index."""
    B = wl.batch
    n_batches = args.warmup + args.steps
    if B * n_batches > wl.n_docs:
        print(f"warmup + steps exceed the {wl.n_docs // B} full batches of the corpus", file=sys.stderr)
        sys.exit(2)
    t_gen = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=B * n_batches)
    h_off = corpus.offsets.cpu().pin_memory()
    h_tok = corpus.tokens.cpu().pin_memory()
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
    lengths = torch.diff(corpus.offsets).cpu().numpy()
    max_tok = int(max(lengths[b * B:(b + 1) * B].sum() for b in range(n_batches)))
    del corpus

    # batched form
    idx = _index(args, wl, lshbloom)
    pl = lshbloom.Pipeline(idx, max_docs=B, max_tokens=max_tok, use_graph=True, autotune=True)
    flags = torch.zeros((n_batches, B), dtype=torch.uint8).pin_memory()
    offs = [h_off[b * B:(b + 1) * B + 1].clone().pin_memory() for b in range(n_batches)]
    for b in range(args.warmup):
        pl.wait(pl.submit(offs[b], h_tok, flags[b]))
    t0 = time.perf_counter()
    tickets = [pl.submit(offs[b], h_tok, flags[b]) for b in range(args.warmup, n_batches)]
    for t in tickets:
        pl.wait(t)
    elapsed = time.perf_counter() - t0
    info = pl.info()
    pl.close()
    assert idx.info()["device_status"] == 0
    batched_flags = flags[args.warmup:].clone()
    idx.close()
    del idx

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
    assert idx.info()["device_status"] == 0
    same = bool(torch.equal(batched_flags, pflags[args.warmup:]))
    idx.close()
    tokens = [int(lengths[b * B:(b + 1) * B].sum()) for b in range(args.warmup, n_batches)]
    res = {
        "value": args.steps * B / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "tokens_per_step": float(np.mean(tokens)),
        "text_GBps": float(np.sum(tokens)) * 4 / elapsed / 1e9,
        "form": "batched (host CSR in, host flags out; length buckets, 2 overlapping slots, hipGraph, autotuner)",
        "plain_per_batch_from_host": {"value": args.steps * B / plain_elapsed,
                                      "ms_per_step": plain_elapsed * 1e3 / args.steps},
        "speedup_vs_plain_from_host": plain_elapsed / elapsed,
        "flags_identical_to_plain": same,
        "pipeline": info,
        "flagged_frac": float(batched_flags.float().mean().item()),
        "corpus_gen_s": t_gen,
    }
    return res, None, None


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
    if B * n_batches > wl.n_docs:
        print(f"warmup + steps exceed the {wl.n_docs // B} full batches of the corpus", file=sys.stderr)
        sys.exit(2)
    n = B * n_batches
    t_gen = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=n)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen
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
    return res, None, None


def run_signatures(args, wl, torch, np, lshbloom, synth, dev):
    """Filter-scale query-insert: batches of precomputed signatures only."""
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
    assert idx.info()["device_status"] == 0
    qi_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]
    probes = B * wl.bands * idx.k
    qi_bytes = qi_algorithmic_bytes(args.steps, B, probes, new_bits, wl.num_perm)
    ach = qi_bytes / (float(np.sum(qi_ms)) * 1e-3)
    rep, _ = synth.signature_repeat_info(args.warmup * B, args.steps * B, wl.bands, B, ex["repeat_frac"],
                                         ex["in_batch_frac"], wl.corpus_seed, device=dev)
    fl = flags[args.warmup:].reshape(-1)
    res = {
        "value": args.steps * B / elapsed,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "docs_timed": args.steps * B,
        "stage_ms": {"query_insert": float(np.mean(qi_ms))},
        "roofline": {
            "bound": "hbm",
            "kernel": "query-insert (all kernels of a batch's in-order test-and-set)",
            "achieved": ach / 1e9, "peak": 8000.0, "unit": "GB/s", "frac": ach / 8e12, "traffic": None,
            "algorithmic_bytes_per_batch": qi_bytes / args.steps,
            "new_bits_per_batch": new_bits / args.steps,
            "probes_per_s": float(np.mean([probes / (t * 1e-3) for t in qi_ms])),
        },
        "repeats_flagged": float(fl[rep].float().mean().item()),
        "non_repeats_flagged": float(fl[~rep].float().mean().item()),
        "filter_bytes": idx.info()["filter_bytes"],
        "sig_gen_s": t_gen,
    }
    return res, None, idx


def run_serve(args, wl, torch, np, lshbloom, synth, dev):
    """Served form: Poisson request streams at several offered loads against
    filters preloaded with 1e8 documents; continuous batching vs one request
    at a time (the plain per-batch form).  Every run starts from the same
    preloaded filter state (restored from a device snapshot) and serves the
    same documents."""
    import copy

    from paper_2411_04257_amd import serve

    loads = [float(x) for x in args.loads.split(",")]
    n_reqs = [int(max(40, min(1000, ld / 100))) for ld in loads]
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
        rb = srv.run(copy.deepcopy(reqs), h_off, h_tok, fb).summary()
        rp = plain.run(copy.deepcopy(reqs), h_off, h_tok, fp_).summary()
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
    return res, None, None


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
        "cache_resident_buffer_MB": small_n * 8 / 1e6,
        "cache_resident_gather_accesses_per_s": m / (t_sgather * 1e-3),
        "cache_resident_scatter_accesses_per_s": m / (t_sscatter * 1e-3),
        "accesses": m,
    }


DESCRIPTIONS = {
    "c2": "plain method on GPU: 1M-doc synthetic corpus (Zipf(1.1)/50k-vocab uint32 tokens, lognormal lengths "
          "median 3000 sigma 0.8 cap 50000, 20% near-dups J 0.6-0.95), 5-shingles, num_perm 128, 16 bands x 8 rows, "
          "filters n=1M fp=1e-6, batches of 65,536",
    "c3": "10M-doc synthetic corpus with Pareto(1.5, min 20, cap 200k) lengths, Zipf(1.1)/50k vocab, 25% near-dups; "
          "num_perm 256, 32 bands x 8 rows, filters n=100M fp=1e-8 (15.3 GB), batches of 1M",
    "c4": "filter-scale query-insert: 1B-signature stream of uniform uint32 (256 wide) with 30% one-band repeats, "
          "32 bands x 8 rows, filters n=1e9 fp=1e-10 per band (191.7 GB in HBM), batches of 1M (timed prefix)",
    "c5": "serving: Poisson arrivals of 1-4096-document requests (log-uniform), lognormal lengths median 2000 "
          "sigma 0.8, Zipf(1.1)/50k vocab, 15% near-dups of earlier served docs; filters preloaded with 1e8 "
          "documents (num_perm 128, 16 bands x 8 rows, fp 1e-8 per band, 7.7 GB); continuous batching with "
          "HBM-budget admission vs one request per batch",
}


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
        res, corpus, idx = run_signatures(args, wl, torch, np, lshbloom, synth, dev)
        metric = "signatures/sec query-insert (band Bloom), bit-exact flags"
        unit = "sigs/s"
    elif args.workload == "c5":
        res, corpus, idx = run_serve(args, wl, torch, np, lshbloom, synth, dev)
        metric = "p99 serve latency (ms) at the highest offered load, continuous batching"
        unit = "ms"
        higher = False
    elif args.form == "fidelity":
        res, corpus, idx = run_fidelity(args, wl, torch, np, lshbloom, synth, dev)
        metric = "F1 gap, LSHBloom minus exact MinHashLSH, on the same signatures (near-dup labels)"
        unit = "F1"
    elif args.form == "batched":
        res, corpus, idx = run_batched(args, wl, torch, np, lshbloom, synth, dev)
        metric = "docs/sec end-to-end (MinHash+band Bloom), bit-exact flags"
        unit = "docs/s"
    else:
        res, corpus, idx = run_corpus(args, wl, torch, np, lshbloom, synth, dev)
        metric = "docs/sec end-to-end (MinHash+band Bloom), bit-exact flags"
        unit = "docs/s"

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
            "workload": DESCRIPTIONS[args.workload],
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
    if corpus is not None and not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, corpus, min(args.cpu_sample_docs, corpus.n_docs))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
