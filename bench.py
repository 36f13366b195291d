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
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Per-unit VALU lane-operation counts of the MinHash hot loops (gfx950 ISA of
# k_minhash<PPL=2, w=5>): one SHA-1 shingle hash of a 5-token shingle (573),
# and one exact (a*x+b) mod (2^61-1) evaluation with its share of the running
# min (8 + 1/2 of a v_min3 shared by two shingles).
OPS_PER_SHINGLE_HASH = 573
OPS_PER_SHINGLE_PERM = 8.5
INT32_VALU_PEAK = 256 * 4 * 16 * 2.4e9  # CUs x SIMDs x lanes x clock = 3.93e13 lane-ops/s
# HBM bytes per token that k_minhash moved, from rocprofv3 FETCH_SIZE (x2.0) and
# WRITE_SIZE (x1.0) scaled by a 1 GiB copy (profiles/k_minhash_c2_counters.md):
# 1.126e9 B for a 2.72e8-token batch.  Valid for the kernel version profiled.
MINHASH_HBM_BYTES_PER_TOKEN = 1.126e9 / 2.7207e8


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=13)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="c2", choices=["c2"])
    ap.add_argument("--cpu-sample-docs", type=int, default=3072)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="after the timed steps, one device-to-device copy of this many bytes "
                         "(calibrates the HBM byte counters against a plain copy)")
    return ap.parse_args()


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
    return {"value": n_docs / dt, "unit": "docs/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n_docs} documents of the same stream ({int(off[-1])} tokens), "
                      f"MinHash + in-order query-insert, single thread, {dt:.1f} s"}


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
    wl = synth.WORKLOADS[args.workload]
    B = wl.batch
    n_batches = args.warmup + args.steps
    n_docs = min(wl.n_docs, B * n_batches)
    if B * n_batches > wl.n_docs:
        print(f"warmup + steps exceed the {wl.n_docs // B} full batches of the corpus", file=sys.stderr)
        sys.exit(2)
    t_gen = time.perf_counter()
    corpus = synth.make_corpus(wl, device=dev, n_docs=n_docs)
    torch.cuda.synchronize()
    t_gen = time.perf_counter() - t_gen

    idx = lshbloom.LSHBloom(wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate, wl.index_seed)
    sigs = torch.empty((B, wl.num_perm), dtype=torch.int32, device=dev)
    flags = torch.empty((n_batches, B), dtype=torch.uint8, device=dev)
    offs = [corpus.offsets[b * B:(b + 1) * B + 1] for b in range(n_batches)]
    lengths = torch.diff(corpus.offsets).cpu().numpy()

    def step(b):
        idx.minhash(offs[b], corpus.tokens, out=sigs)
        idx.query_insert(sigs, out=flags[b])

    for b in range(args.warmup):
        step(b)
    torch.cuda.synchronize()

    stream = torch.cuda.current_stream()
    ev = [[torch.cuda.Event(enable_timing=True) for _ in range(3)] for _ in range(args.steps)]
    t0 = time.perf_counter()
    for s in range(args.steps):
        b = args.warmup + s
        ev[s][0].record(stream)
        idx.minhash(offs[b], corpus.tokens, out=sigs)
        ev[s][1].record(stream)
        idx.query_insert(sigs, out=flags[b])
        ev[s][2].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0

    mh_ms = [ev[s][0].elapsed_time(ev[s][1]) for s in range(args.steps)]
    qi_ms = [ev[s][1].elapsed_time(ev[s][2]) for s in range(args.steps)]
    timed = range(args.warmup, n_batches)
    shingles = [shingle_count(lengths[b * B:(b + 1) * B]) for b in timed]
    tokens = [int(lengths[b * B:(b + 1) * B].sum()) for b in timed]
    ops = [s * (OPS_PER_SHINGLE_HASH + wl.num_perm * OPS_PER_SHINGLE_PERM) for s in shingles]
    achieved = float(np.mean([o / (t * 1e-3) for o, t in zip(ops, mh_ms)]))
    docs = args.steps * B
    value = docs / elapsed
    info = idx.info()
    assert info["device_status"] == 0

    out = {
        "metric": "docs/sec end-to-end (MinHash+band Bloom), bit-exact flags",
        "value": value,
        "unit": "docs/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u32",
        "data": "synthetic",
        "config": {
            "workload": "plain method on GPU: 1M-doc synthetic corpus (Zipf(1.1)/50k-vocab uint32 tokens, "
                        "lognormal lengths median 3000 sigma 0.8 cap 50000, 20% near-dups J 0.6-0.95), "
                        "5-shingles, num_perm 128, 16 bands x 8 rows, filters n=1M fp=1e-6, batches of 65,536",
            "global_batch": B,
            "docs_timed": docs,
            "tokens_per_step": float(np.mean(tokens)),
            "parallelism": "single-gpu",
        },
        "text_GBps": float(np.sum(tokens)) * 4 / elapsed / 1e9,
        "stage_ms": {"minhash": float(np.mean(mh_ms)), "query_insert": float(np.mean(qi_ms))},
        "roofline": {
            "bound": "alu",
            "kernel": "k_minhash (incl. its 0xFFFFFFFF pre-fill)",
            "achieved": achieved / 1e12,
            "peak": INT32_VALU_PEAK / 1e12,
            "unit": "TOPS (int32 VALU lane-ops/s)",
            "frac": achieved / INT32_VALU_PEAK,
            "traffic": float(np.mean(tokens)) * MINHASH_HBM_BYTES_PER_TOKEN,
            "shingle_perm_per_s": float(np.mean([s * wl.num_perm / (t * 1e-3) for s, t in zip(shingles, mh_ms)])),
        },
        "flagged_frac": float(flags[args.warmup:].float().mean().item()),
        "corpus_gen_s": t_gen,
    }
    if args.copy_bytes:
        src = torch.empty(args.copy_bytes // 4, dtype=torch.int32, device=dev).fill_(7)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        out["copy_bytes"] = args.copy_bytes
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, corpus, min(args.cpu_sample_docs, n_docs))
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
