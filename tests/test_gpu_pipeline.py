"""GPU tests of the batched form (length buckets, two overlapping slots,
hipGraph replay, autotuner): every configuration must give the oracle's
stream result bit for bit."""

import os

import numpy as np
import pytest
import torch

import oracle
from paper_2411_04257_amd import synth

pytestmark = pytest.mark.gpu

P, B, R = 256, 32, 8


def _corpus(n_docs, seed):
    wl = synth.WORKLOADS["c3"]
    c = synth.make_corpus(wl, n_docs=n_docs, seed=seed)
    return c.offsets.numpy(), c.tokens.numpy().view(np.uint32)


def _oracle_stream(off, tok, batches, n=20_000, fp=1e-3, seed=42):
    o = oracle.OracleIndex(P, B, R, n, fp, seed)
    sigs = o.minhash(off, tok)
    flags = o.query_insert(sigs)
    return flags, o.filters()


def _split(off, batches):
    out, s = [], 0
    for b in batches:
        out.append((s, s + b))
        s += b
    return out


def _run_pipeline(gpu, off, tok, batches, pinned=False, n=20_000, fp=1e-3, seed=42, **kw):
    g = gpu.LSHBloom(P, B, R, n, fp, seed)
    pl = gpu.Pipeline(g, max_docs=max(batches), max_tokens=int(off[-1]) + 1, **kw)
    flags = np.zeros(len(off) - 1, np.uint8)
    tickets = []
    outs = []
    for a, b in _split(off, batches):
        o = (off[a:b + 1]).astype(np.int64)
        t = tok
        f = np.zeros(b - a, np.uint8)
        if pinned:
            o = torch.from_numpy(o).pin_memory()
            t = torch.from_numpy(tok.view(np.int32)).pin_memory()
            f = torch.zeros(b - a, dtype=torch.uint8).pin_memory()
        tickets.append(pl.submit(o, t, f))
        outs.append((a, b, f))
    for t in tickets:
        pl.wait(t)
    for a, b, f in outs:
        flags[a:b] = f.numpy() if isinstance(f, torch.Tensor) else f
    info = pl.info()
    pl.close()
    words = g.read_filters().cpu().numpy().view(np.uint64)
    assert g.info()["device_status"] == 0
    g.close()
    return flags, words, info


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
@pytest.mark.parametrize("buckets", ["one", "three", "auto"])
def test_pipeline_matches_oracle(gpu, use_graph, buckets):
    off, tok = _corpus(7000, seed=31)
    batches = [3000, 2500, 1500]
    want_flags, want_words = _oracle_stream(off, tok, batches)
    kw = {"one": dict(n_buckets=1, autotune=False),
          "three": dict(n_buckets=3, bucket_edges=(32, 64, 0), waves_per_cu=(8, 16, 24, 0), autotune=False),
          "auto": dict(autotune=True)}[buckets]
    flags, words, info = _run_pipeline(gpu, off, tok, batches, use_graph=use_graph, **kw)
    np.testing.assert_array_equal(flags, want_flags)
    np.testing.assert_array_equal(words, want_words)
    assert want_flags.sum() > 100
    if use_graph:
        assert info["graph_launches"] >= 6
        assert info["graph_updates"] + info["graph_instantiations"] == info["graph_launches"]
    if buckets == "auto":
        assert info["tuned"] == 1


@pytest.mark.parametrize("use_graph", [False, True], ids=["eager", "graph"])
def test_pipeline_binned_query_insert_matches_oracle(gpu, use_graph):
    """Batches above the binned path's threshold (4,096 documents): its
    kernels run inside the captured graphs and replay with new batches."""
    off, tok = _corpus(20000, seed=35)
    batches = [6000, 5000, 9000]
    want_flags, want_words = _oracle_stream(off, tok, batches, n=50_000)
    flags, words, info = _run_pipeline(gpu, off, tok, batches, n=50_000, use_graph=use_graph, autotune=False)
    np.testing.assert_array_equal(flags, want_flags)
    np.testing.assert_array_equal(words, want_words)
    assert want_flags.sum() > 1000


def test_pipeline_pinned_inputs_and_many_graph_replays(gpu):
    off, tok = _corpus(9000, seed=32)
    batches = [1500] * 6
    want_flags, want_words = _oracle_stream(off, tok, batches)
    flags, words, info = _run_pipeline(gpu, off, tok, batches, pinned=True, use_graph=True, autotune=False)
    np.testing.assert_array_equal(flags, want_flags)
    np.testing.assert_array_equal(words, want_words)
    assert info["graph_updates"] >= 4  # same topology: the executable graphs are updated in place


def test_pipeline_interleaves_with_direct_calls(gpu):
    """Pipeline batches and direct calls on the same index keep host call order."""
    off, tok = _corpus(4000, seed=33)
    o = oracle.OracleIndex(P, B, R, 20_000, 1e-3, 42)
    sigs = o.minhash(off, tok)
    want = o.query_insert(np.concatenate([sigs[:2000], sigs[1000:3000], sigs[3000:4000]]))
    g = gpu.LSHBloom(P, B, R, 20_000, 1e-3, 42)
    pl = gpu.Pipeline(g, max_docs=2000, max_tokens=int(off[-1]) + 1, autotune=False)
    f1 = np.zeros(2000, np.uint8)
    t1 = pl.submit(off[:2001].copy(), tok, f1)
    pl.wait(t1)
    doff = torch.as_tensor(off[1000:3001].copy()).cuda()
    dtok = torch.as_tensor(tok.view(np.int32)).cuda()
    f2 = g.query_insert(g.minhash(doff, dtok)).cpu().numpy()
    f3 = np.zeros(1000, np.uint8)
    t3 = pl.submit(off[3000:4001].copy(), tok, f3)
    pl.wait(t3)
    np.testing.assert_array_equal(np.concatenate([f1, f2, f3]), want)
    assert want[2000:3000].all()  # repeats of documents 1000..1999
    pl.close()
    g.close()


def test_pipeline_rejects_bad_batches(gpu):
    g = gpu.LSHBloom(P, B, R, 1000, 1e-3)
    pl = gpu.Pipeline(g, max_docs=10, max_tokens=100, autotune=False)
    tok = np.arange(200, dtype=np.uint32)
    with pytest.raises(gpu.LSHBloomError):
        pl.submit(np.array([0, 5, 3], np.int64), tok, np.zeros(2, np.uint8))  # decreasing offsets
    with pytest.raises(gpu.LSHBloomError):
        pl.submit(np.arange(12, dtype=np.int64), tok, np.zeros(11, np.uint8))  # more than max_docs
    with pytest.raises(gpu.LSHBloomError):
        pl.submit(np.array([0, 150], np.int64), tok, np.zeros(1, np.uint8))  # more than max_tokens
    t = pl.submit(np.array([0], np.int64), tok, np.zeros(0, np.uint8))  # empty batch
    pl.wait(t)
    pl.close()
    g.close()


def test_pipeline_tune_cache_round_trip(gpu, tmp_path):
    off, tok = _corpus(3000, seed=34)
    cache = str(tmp_path / "tune.txt")
    g = gpu.LSHBloom(P, B, R, 20_000, 1e-3, 42)
    pl = gpu.Pipeline(g, max_docs=3000, max_tokens=int(off[-1]) + 1, autotune=True, tune_cache=cache)
    f = np.zeros(3000, np.uint8)
    pl.wait(pl.submit(off.copy(), tok, f))
    first = pl.info()
    pl.close()
    g.close()
    assert os.path.exists(cache) and first["tuned"] == 1
    g = gpu.LSHBloom(P, B, R, 20_000, 1e-3, 42)
    pl = gpu.Pipeline(g, max_docs=3000, max_tokens=int(off[-1]) + 1, autotune=True, tune_cache=cache)
    f2 = np.zeros(3000, np.uint8)
    pl.wait(pl.submit(off.copy(), tok, f2))
    second = pl.info()
    pl.close()
    g.close()
    assert second["tune_best_ms"] == 0.0  # loaded from the cache, not re-timed
    assert (second["n_buckets"], second["bucket_edges"], second["waves_per_cu"]) == \
        (first["n_buckets"], first["bucket_edges"], first["waves_per_cu"])
    np.testing.assert_array_equal(f, f2)
