"""The served form at the serving configuration's size, against the oracle.

Filters (num_perm 128, 16 bands x 8 rows, n = 1e8 at a per-band rate of
1e-8: 7.7 GB) are preloaded with 1e8 random-signature documents and saved
with lshbloom_save; the serving index and the oracle both load that file.
Poisson requests of 1-4,096 documents (lognormal lengths, median 2,000
tokens) then go through the continuous-batching server at an offered load
where batches mix several requests, and through the one-request-per-batch
server on a third index loaded from the same file.  The served flags must
equal the oracle's replay of the ticket-ordered stream (Section 2.1), in the
mix and alone, and the final filters must equal the oracle's.
"""

import os
import shutil
import tempfile

import numpy as np
import pytest
import torch

import oracle
from paper_2411_04257_amd import serve, synth

pytestmark = pytest.mark.gpu


def _threads():
    n = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS", "").isdigit():
        n = min(n, int(os.environ["OMP_NUM_THREADS"]))
    return max(1, min(n, 32))


def _scratch_dir(need):
    for d in ("/dev/shm", tempfile.gettempdir()):
        if os.path.isdir(d) and shutil.disk_usage(d).free > 2 * need:
            return tempfile.mkdtemp(dir=d)
    pytest.skip(f"no scratch space for a {need / 1e9:.1f} GB index file")


def test_served_stream_after_full_preload_matches_oracle(gpu):
    wl = synth.WORKLOADS["c5"]
    P, b, r, n, p = wl.num_perm, wl.bands, wl.rows, wl.expected_n, wl.fp_rate
    pre = wl.extra["preload"]
    print(f"c5 at size: preload {pre} documents into {b} x 479 MB filters", flush=True)
    g = gpu.LSHBloom(P, b, r, n, p, wl.index_seed)
    serve.preload(g, pre, 1)
    d = _scratch_dir(g.info()["filter_bytes"])
    path = os.path.join(d, "preloaded.lshbloom")
    try:
        g.save(path)
        g.close()
        rng = np.random.default_rng(wl.corpus_seed)
        reqs = serve.poisson_requests(240, 1_000_000.0, wl.extra["req_min"], wl.extra["req_max"], 0, rng)
        n_docs = reqs[-1].hi
        corpus = synth.make_corpus(wl, device="cuda", n_docs=n_docs)
        h_off = corpus.offsets.cpu().pin_memory()
        h_tok = corpus.tokens.cpu().pin_memory()
        del corpus

        srv_idx = gpu.LSHBloom(P, b, r, n, p, wl.index_seed)
        srv_idx.load(path)
        srv = serve.Server(srv_idx, 16384, 16384 * 8000, hbm_budget=2 << 30)
        fb = torch.zeros(n_docs, dtype=torch.uint8).pin_memory()
        res = srv.run(reqs, h_off, h_tok, fb)
        srv.close()
        srv_idx.sync()
        assert res.batches < len(reqs), "the offered load should make batches of several requests"

        one_idx = gpu.LSHBloom(P, b, r, n, p, wl.index_seed)
        one_idx.load(path)
        plain = serve.PlainServer(one_idx, 16384, 16384 * 8000)
        fp_ = torch.zeros(n_docs, dtype=torch.uint8).pin_memory()
        import copy
        plain.run(copy.deepcopy(reqs), h_off, h_tok, fp_)
        plain.close()
        one_idx.sync()
        one_idx.close()

        o = oracle.OracleIndex(P, b, r, n, p, wl.index_seed)
        o.load_file(path)
        assert o.docs_inserted == pre
        sigs = o.minhash_threads(h_off.numpy(), h_tok.numpy().view(np.uint32), _threads())
        want = o.query_insert_by_band(sigs, _threads())
        got = fb.numpy()
        bad = np.flatnonzero(got != want)
        assert len(bad) == 0, f"{len(bad)} served flags differ from the oracle, first {bad[:5]}"
        assert np.array_equal(fp_.numpy(), want), "one-request-per-batch flags differ from the oracle"
        assert want.sum() > 0.02 * n_docs
        wv = o.filters_view()
        for j in range(b):
            got_w = torch.empty(srv_idx.words_per_band, dtype=torch.int64)
            import ctypes
            rc = gpu.load().lshbloom_read_filters(srv_idx._h, ctypes.c_void_p(got_w.data_ptr()),
                                                  j * srv_idx.words_per_band * 8, srv_idx.words_per_band * 8, None)
            assert rc == 0
            assert np.array_equal(got_w.numpy().view(np.uint64), wv[j]), f"band {j} filter differs"
        o.close()
        srv_idx.close()
    finally:
        shutil.rmtree(d, ignore_errors=True)
