"""A device status raised by a query-insert becomes an error on the host.

The kernels raise bits of a status word when their own bookkeeping fails; the
host copies it after every query-insert call.  The condition is forced from
the host (LSHBLOOM_STATUS_AT=n makes the n-th query-insert call of a handle
write a nonzero status with a plain fill kernel after its work), so every
kernel runs and exits normally.
"""

import os

import numpy as np
import pytest
import torch

from paper_2411_04257_amd import synth

pytestmark = pytest.mark.gpu

P, B, R, N, FP = 128, 16, 8, 100_000, 1e-6


def _sigs(start, count):
    return synth.signature_batch(start, count, P, B, R, count, 0.3, 0.5, 3, device="cuda")


@pytest.fixture
def status_at(monkeypatch):
    def set_at(n):
        monkeypatch.setenv("LSHBLOOM_STATUS_AT", str(n))
    yield set_at


def test_status_reported_by_sync_then_poisoned(gpu, status_at):
    status_at(2)
    idx = gpu.LSHBloom(P, B, R, N, FP, 42)
    os.environ.pop("LSHBLOOM_STATUS_AT", None)
    idx.query_insert(_sigs(0, 5000))
    idx.sync()  # the first call is clean
    idx.query_insert(_sigs(5000, 5000))  # enqueued; raises the status on the device
    with pytest.raises(gpu.LSHBloomError) as ei:
        idx.sync()
    assert ei.value.code == gpu.EDEVICE and "inconsistency" in str(ei.value)
    with pytest.raises(gpu.LSHBloomError) as ei:
        idx.query_insert(_sigs(10000, 100))
    assert ei.value.code == gpu.EPOISONED
    assert idx.info()["poisoned"] == 1
    idx.close()


def test_status_reported_by_next_call_after_host_wait(gpu, status_at):
    status_at(1)
    idx = gpu.LSHBloom(P, B, R, N, FP, 42)
    idx.query_insert_noalloc(_sigs(0, 300), torch.empty(300, dtype=torch.uint8, device="cuda"))
    torch.cuda.synchronize()
    with pytest.raises(gpu.LSHBloomError) as ei:
        idx.minhash(torch.zeros(2, dtype=torch.int64, device="cuda"), torch.zeros(1, dtype=torch.int32, device="cuda"))
    assert ei.value.code == gpu.EDEVICE
    idx.close()


def test_status_reported_by_pipeline_wait(gpu, status_at):
    status_at(2)
    idx = gpu.LSHBloom(P, B, R, N, FP, 42)
    pl = gpu.Pipeline(idx, max_docs=2000, max_tokens=2000 * 600, autotune=False, n_buckets=1)
    wl = synth.WORKLOADS["c1"]
    c = synth.make_corpus(wl, n_docs=3000)
    off = c.offsets.numpy()
    tok = c.tokens.numpy()
    f1 = np.zeros(1500, np.uint8)
    f2 = np.zeros(1500, np.uint8)
    t1 = pl.submit(np.ascontiguousarray(off[:1501]), tok, f1)
    pl.wait(t1)
    t2 = pl.submit(np.ascontiguousarray(off[1500:]), tok, f2)
    with pytest.raises(gpu.LSHBloomError) as ei:
        pl.wait(t2)
    assert ei.value.code == gpu.EDEVICE
    with pytest.raises(gpu.LSHBloomError) as ei:
        pl.submit(np.ascontiguousarray(off[:11]), tok, np.zeros(10, np.uint8))
    assert ei.value.code == gpu.EPOISONED
    pl.close()
    idx.close()


def test_no_status_without_forcing(gpu):
    idx = gpu.LSHBloom(P, B, R, N, FP, 42)
    for s in range(3):
        idx.query_insert(_sigs(s * 20000, 20000))
    idx.sync()
    assert idx.info()["device_status"] == 0 and idx.info()["poisoned"] == 0
    idx.close()
