"""Seeded synthetic workloads (inputs only: no hashing, no MinHash, no Bloom).

The paper measures on peS2o and on labelled PDF-derived duplicate sets, none
of which exist here; these generators stand in for them with documents of
uint32 token ids drawn from a Zipf law over a 50,000-token vocabulary and
near-duplicates made by editing a copy of an earlier original document.

Both the CPU oracle and the GPU library consume the arrays produced here;
this module is the only code they share and it holds none of the method's
arithmetic.  Every generator takes a `device` so large corpora can be made
directly in HBM; CPU and GPU draws use different random streams, so a corpus
is identified by (config, seed, device, n_docs).

Recipe
------
* token id = Zipf rank - 1, P(rank) proportional to rank^-1.1 over ranks
  1..50,000, sampled by inverse CDF.
* document lengths per config: uniform [lo, hi]; lognormal with a median and
  sigma, capped; Pareto(alpha, min) capped.
* near-duplicates: each document after the first is, with probability
  `dup_frac`, an edited copy of a uniformly chosen earlier *original*
  (non-near-duplicate) document.  Edits per source token: substitution by a
  fresh Zipf token, or insertion of a fresh Zipf token before it.  For a
  target Jaccard J on 5-token shingle sets the per-token edit rate is
  e = 1 - (2J/(1+J))^(1/5) (a fraction (1-e)^5 of shingles survives and
  J = f/(2-f)), split half substitution and half insertion.
"""

from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import torch

VOCAB = 50_000
ZIPF_S = 1.1


@dataclass(frozen=True)
class Workload:
    name: str
    n_docs: int
    length: tuple  # ("uniform", lo, hi) | ("lognormal", median, sigma, cap) | ("pareto", alpha, min, cap)
    dup_frac: float
    edit: tuple  # ("sub", rate) | ("jaccard", j_lo, j_hi)
    num_perm: int
    bands: int
    rows: int
    expected_n: int
    fp_rate: float
    batch: int
    corpus_seed: int
    index_seed: int = 42
    extra: dict = field(default_factory=dict)


# The five workloads (sizes, distributions and index parameters as specified
# for this implementation; see the design notes for the reading of each).
WORKLOADS = {
    "c1": Workload("c1-plain-2k", 2_000, ("uniform", 50, 500), 0.10, ("sub", 0.05),
                   128, 16, 8, 2_000, 1e-5, 2_000, corpus_seed=2),
    "c2": Workload("c2-plain-1M", 1_000_000, ("lognormal", 3000.0, 0.8, 50_000), 0.20, ("jaccard", 0.6, 0.95),
                   128, 16, 8, 1_000_000, 1e-6, 65_536, corpus_seed=3),
    "c3": Workload("c3-batched-10M", 10_000_000, ("pareto", 1.5, 20, 200_000), 0.25, ("jaccard", 0.6, 0.95),
                   256, 32, 8, 100_000_000, 1e-8, 2_000_000, corpus_seed=4),
    "c4": Workload("c4-filter-1B", 1_000_000_000, ("none",), 0.0, ("none",),
                   256, 32, 8, 1_000_000_000, 1e-10, 1_000_000, corpus_seed=5,
                   extra={"repeat_frac": 0.30, "in_batch_frac": 0.5}),
    "c5": Workload("c5-serve", 0, ("lognormal", 2000.0, 0.8, 50_000), 0.15, ("jaccard", 0.6, 0.95),
                   128, 16, 8, 100_000_000, 1e-8, 4_096, corpus_seed=6,
                   extra={"preload": 100_000_000, "req_min": 1, "req_max": 4096}),
}


def _gen(seed: int, device) -> torch.Generator:
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    return g


def zipf_cdf(device, vocab: int = VOCAB, s: float = ZIPF_S) -> torch.Tensor:
    ranks = torch.arange(1, vocab + 1, dtype=torch.float64, device=device)
    w = ranks.pow(-s)
    cdf = torch.cumsum(w, 0)
    return cdf / cdf[-1]


def zipf_tokens(n: int, gen: torch.Generator, cdf: torch.Tensor, chunk: int = 1 << 26) -> torch.Tensor:
    """n token ids (int32; ids < 50,000 so the bits equal the uint32 value)."""
    out = torch.empty(n, dtype=torch.int32, device=cdf.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        u = torch.rand(e - s, generator=gen, device=cdf.device, dtype=torch.float64)
        idx = torch.searchsorted(cdf, u, right=True)
        out[s:e] = idx.clamp_(max=cdf.numel() - 1).to(torch.int32)
    return out


def draw_lengths(spec: tuple, n: int, gen: torch.Generator, device) -> torch.Tensor:
    kind = spec[0]
    if kind == "uniform":
        lo, hi = spec[1], spec[2]
        return torch.randint(lo, hi + 1, (n,), generator=gen, device=device, dtype=torch.int64)
    if kind == "lognormal":
        median, sigma, cap = spec[1], spec[2], spec[3]
        z = torch.randn(n, generator=gen, device=device, dtype=torch.float64)
        L = torch.exp(math.log(median) + sigma * z).round().to(torch.int64)
        return L.clamp_(1, cap)
    if kind == "pareto":
        alpha, lmin, cap = spec[1], spec[2], spec[3]
        u = torch.rand(n, generator=gen, device=device, dtype=torch.float64)
        L = torch.floor(lmin * torch.pow(1.0 - u, -1.0 / alpha)).to(torch.int64)
        return L.clamp_(lmin, cap)
    raise ValueError(f"unknown length spec {spec}")


def edit_rate_for_jaccard(J: torch.Tensor, w: int = 5) -> torch.Tensor:
    return 1.0 - torch.pow(2.0 * J / (1.0 + J), 1.0 / w)


def _dup_plan(n: int, dup_frac: float, rng: np.random.Generator):
    """is_dup[i] and source[i] (an earlier original, or -1)."""
    is_dup = rng.random(n) < dup_frac
    if n:
        is_dup[0] = False
    orig_idx = np.flatnonzero(~is_dup)
    # number of originals strictly before i
    n_before = np.cumsum(~is_dup) - (~is_dup)
    src = np.full(n, -1, dtype=np.int64)
    d = np.flatnonzero(is_dup)
    pick = np.floor(rng.random(len(d)) * n_before[d]).astype(np.int64)
    src[d] = orig_idx[pick]
    return is_dup, src


@dataclass
class Corpus:
    offsets: torch.Tensor  # int64 [n+1]
    tokens: torch.Tensor  # int32 [T] (uint32 bit pattern)
    is_dup: np.ndarray  # bool [n]
    source: np.ndarray  # int64 [n], -1 for originals
    target_j: np.ndarray  # float64 [n], nan for originals

    @property
    def n_docs(self) -> int:
        return self.offsets.numel() - 1

    def batch(self, start: int, stop: int):
        """CSR view of documents [start, stop) with offsets rebased to 0."""
        off = self.offsets[start:stop + 1]
        base = int(off[0])
        end = int(off[-1])
        return off - base, self.tokens[base:end]


def make_corpus(wl: Workload, device="cpu", n_docs: int | None = None, seed: int | None = None,
                dup_chunk_tokens: int = 1 << 27) -> Corpus:
    n = wl.n_docs if n_docs is None else int(n_docs)
    seed = wl.corpus_seed if seed is None else int(seed)
    device = torch.device(device)
    gen = _gen(seed, device)
    rng = np.random.default_rng(seed)
    cdf = zipf_cdf(device)

    is_dup, src = _dup_plan(n, wl.dup_frac, rng)
    target_j = np.full(n, np.nan)
    rate = np.zeros(n)
    d_idx = np.flatnonzero(is_dup)
    if wl.edit[0] == "sub":
        rate[d_idx] = wl.edit[1]
        sub_share = 1.0
        f = (1.0 - wl.edit[1]) ** 5
        target_j[d_idx] = f / (2.0 - f)
    elif wl.edit[0] == "jaccard":
        J = wl.edit[1] + (wl.edit[2] - wl.edit[1]) * rng.random(len(d_idx))
        target_j[d_idx] = J
        rate[d_idx] = edit_rate_for_jaccard(torch.from_numpy(J)).numpy()
        sub_share = 0.5
    else:
        sub_share = 1.0

    L = draw_lengths(wl.length, n, gen, device)
    L_cpu = L.cpu().numpy()

    # Per-dup edit decisions on the source tokens: 0 keep, 1 substitute, 2 insert-before.
    src_len = np.where(is_dup, L_cpu[np.maximum(src, 0)], 0)
    dup_src_len = src_len[d_idx]
    # Decide edits in chunks of documents so per-token temporaries stay bounded.
    ins_counts = np.zeros(n, dtype=np.int64)
    edit_chunks = []
    start = 0
    while start < len(d_idx):
        acc = 0
        stop = start
        while stop < len(d_idx) and (acc == 0 or acc + dup_src_len[stop] <= dup_chunk_tokens):
            acc += dup_src_len[stop]
            stop += 1
        docs = d_idx[start:stop]
        lens = torch.from_numpy(dup_src_len[start:stop]).to(device)
        rates = torch.from_numpy(rate[docs]).to(device)
        per_tok_rate = torch.repeat_interleave(rates, lens)
        u = torch.rand(int(acc), generator=gen, device=device, dtype=torch.float64)
        op = torch.zeros(int(acc), dtype=torch.int8, device=device)
        op[u < per_tok_rate * sub_share] = 1
        op[(u >= per_tok_rate * sub_share) & (u < per_tok_rate)] = 2
        doc_of_tok = torch.repeat_interleave(torch.arange(len(docs), device=device), lens)
        ins = torch.zeros(len(docs), dtype=torch.int64, device=device)
        ins.index_add_(0, doc_of_tok, (op == 2).to(torch.int64))
        ins_counts[docs] = ins.cpu().numpy()
        edit_chunks.append((docs, lens, op))
        start = stop

    final_len = np.where(is_dup, src_len + ins_counts, L_cpu)
    offsets_cpu = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(final_len, out=offsets_cpu[1:])
    offsets = torch.from_numpy(offsets_cpu).to(device)
    tokens = torch.empty(int(offsets_cpu[-1]), dtype=torch.int32, device=device)

    # Originals: fresh Zipf tokens in place.
    o_idx = np.flatnonzero(~is_dup)
    o_len = torch.from_numpy(final_len[o_idx]).to(device)
    o_start = torch.from_numpy(offsets_cpu[o_idx]).to(device)
    total_o = int(o_len.sum()) if len(o_idx) else 0
    step = 1 << 26
    o_cum = torch.cumsum(o_len, 0)
    for s in range(0, total_o, step):
        e = min(total_o, s + step)
        pos = torch.arange(s, e, device=device, dtype=torch.int64)
        doc = torch.searchsorted(o_cum, pos, right=True)
        within = pos - (o_cum[doc] - o_len[doc])
        tokens[o_start[doc] + within] = zipf_tokens(e - s, gen, cdf)

    # Near-duplicates: edited copies of their (original) sources.
    for docs, lens, op in edit_chunks:
        docs_t = torch.from_numpy(docs).to(device)
        src_start = offsets[torch.from_numpy(src[docs]).to(device)]
        dst_start = offsets[docs_t]
        first = torch.cumsum(lens, 0) - lens
        doc_of_tok = torch.repeat_interleave(torch.arange(len(docs), device=device), lens)
        t_in_doc = torch.arange(op.numel(), device=device) - first[doc_of_tok]
        vals = tokens[src_start[doc_of_tok] + t_in_doc]
        subs = op == 1
        vals[subs] = zipf_tokens(int(subs.sum()), gen, cdf)
        is_ins = (op == 2).to(torch.int64)
        ins_incl = torch.cumsum(is_ins, 0)
        ins_before_doc = (ins_incl - is_ins)[first] if op.numel() else ins_incl
        ins_in_doc_incl = ins_incl - ins_before_doc[doc_of_tok]
        out_pos = dst_start[doc_of_tok] + t_in_doc + ins_in_doc_incl
        tokens[out_pos] = vals
        ins_pos = out_pos[op == 2] - 1
        tokens[ins_pos] = zipf_tokens(ins_pos.numel(), gen, cdf)

    return Corpus(offsets, tokens, is_dup, src, target_j)


def random_tokens_doc(length: int, rng: np.random.Generator) -> np.ndarray:
    """One document of Zipf tokens drawn with numpy (small tests)."""
    ranks = np.arange(1, VOCAB + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** -ZIPF_S)
    cdf /= cdf[-1]
    idx = np.searchsorted(cdf, rng.random(length), side="right")
    return np.minimum(idx, VOCAB - 1).astype(np.uint32)


# --------------------------------------------------------------------------
# Filter-scale signature stream: uniform uint32 values from a counter-based
# generator, so that any earlier signature can be regenerated on demand, with
# a fraction of signatures repeating one band of an earlier original.
# --------------------------------------------------------------------------
_M32 = 0xFFFFFFFF


def _lowbias32(x: torch.Tensor) -> torch.Tensor:
    """Wellons' 'lowbias32' integer hash on int64 tensors holding uint32 values."""
    x = x & _M32
    x = x ^ (x >> 16)
    x = (x * 0x7FEB352D) & _M32
    x = x ^ (x >> 15)
    x = (x * 0x846CA68B) & _M32
    x = x ^ (x >> 16)
    return x


def _counter_u32(seed: int, stream: int, idx: torch.Tensor, col: torch.Tensor) -> torch.Tensor:
    h = _lowbias32(idx & _M32 ^ (seed * 0x9E3779B1 + stream * 0x85EBCA77))
    h = _lowbias32(h ^ (idx >> 32) ^ 0x27D4EB2F)
    return _lowbias32(h ^ (col * 0x165667B1))


def signature_batch(start: int, count: int, num_perm: int, bands: int, rows: int, batch: int,
                    repeat_frac: float, in_batch_frac: float, seed: int, device="cpu") -> torch.Tensor:
    """Signatures [start, start+count) as int32 [count, num_perm] (uint32 bits).

    Signature i is an 'original' unless its repeat draw (< repeat_frac) selects
    it; a repeat copies one band (rows values) of an earlier original chosen
    uniformly from its own batch with probability in_batch_frac, else from all
    earlier batches (four candidates are tried; if none is an original the
    signature stays an original)."""
    device = torch.device(device)
    idx = torch.arange(start, start + count, device=device, dtype=torch.int64)
    cols = torch.arange(num_perm, device=device, dtype=torch.int64)
    base = _counter_u32(seed, 0, idx[:, None], cols[None, :])

    def is_repeat(i):
        u = _counter_u32(seed, 1, i, torch.zeros_like(i)).to(torch.float64) / 4294967296.0
        return (u < repeat_frac) & (i > 0)

    rep = is_repeat(idx)
    batch_start = (idx // batch) * batch
    u_loc = _counter_u32(seed, 2, idx, torch.zeros_like(idx)).to(torch.float64) / 4294967296.0
    local = (u_loc < in_batch_frac) & (idx > batch_start)
    local = local | (batch_start == 0)
    lo = torch.where(local, batch_start, torch.zeros_like(idx))
    hi = torch.where(local, idx, batch_start)  # exclusive
    span = (hi - lo).clamp(min=1)
    src = torch.full_like(idx, -1)
    for c in range(4):
        u = _counter_u32(seed, 3 + c, idx, torch.zeros_like(idx)).to(torch.float64) / 4294967296.0
        cand = lo + torch.floor(u * span.to(torch.float64)).to(torch.int64)
        ok = (src < 0) & ~is_repeat(cand)
        src = torch.where(ok, cand, src)
    rep = rep & (src >= 0) & (hi > lo)
    band = _counter_u32(seed, 7, idx, torch.zeros_like(idx)) % bands
    out = base
    r_idx = torch.nonzero(rep).flatten()
    if r_idx.numel():
        s = src[r_idx]
        bcols = band[r_idx][:, None] * rows + torch.arange(rows, device=device)[None, :]
        vals = _counter_u32(seed, 0, s[:, None], bcols)
        out[r_idx[:, None], bcols] = vals
    return out.to(torch.int32) if out.dtype != torch.int32 else out


def signature_repeat_info(start: int, count: int, bands: int, batch: int, repeat_frac: float,
                          in_batch_frac: float, seed: int, device="cpu"):
    """(is_repeat, source) for signatures [start, start+count), as drawn by
    signature_batch (used by tests to know which flags must be 1)."""
    device = torch.device(device)
    idx = torch.arange(start, start + count, device=device, dtype=torch.int64)

    def is_repeat(i):
        u = _counter_u32(seed, 1, i, torch.zeros_like(i)).to(torch.float64) / 4294967296.0
        return (u < repeat_frac) & (i > 0)

    rep = is_repeat(idx)
    batch_start = (idx // batch) * batch
    u_loc = _counter_u32(seed, 2, idx, torch.zeros_like(idx)).to(torch.float64) / 4294967296.0
    local = (u_loc < in_batch_frac) & (idx > batch_start)
    local = local | (batch_start == 0)
    lo = torch.where(local, batch_start, torch.zeros_like(idx))
    hi = torch.where(local, idx, batch_start)
    span = (hi - lo).clamp(min=1)
    src = torch.full_like(idx, -1)
    for c in range(4):
        u = _counter_u32(seed, 3 + c, idx, torch.zeros_like(idx)).to(torch.float64) / 4294967296.0
        cand = lo + torch.floor(u * span.to(torch.float64)).to(torch.int64)
        ok = (src < 0) & ~is_repeat(cand)
        src = torch.where(ok, cand, src)
    rep = rep & (src >= 0) & (hi > lo)
    return rep, torch.where(rep, src, torch.full_like(src, -1))
