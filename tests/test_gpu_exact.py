"""GPU parity of the exact MinHashLSH band index (the comparison baseline)
against the CPU reference `oracle.ExactLSHOracle`, through the C ABI.

Flags are compared bit for bit on seeded signature streams with band repeats
(inside a call and across calls) and whole repeated documents, over calls of
uneven sizes; with few fingerprint bits, so that different band values share
fingerprints and take the exact settling path; across the 2^20-document
chunks of one call (against the same stream in other splits and the oracle on
a prefix); and against LSHBloom on the same stream (containment).
"""

import numpy as np
import pytest
import torch

from oracle.exact_lsh import ExactLSHOracle
from paper_2411_04257_amd import synth

pytestmark = pytest.mark.gpu


def _sigs(n, num_perm, bands, rows, seed, start=0, whole=50):
    """Signatures with band repeats (synth's counter-based generator) and one
    whole repeated document in `whole`."""
    s = synth.signature_batch(start, n, num_perm, bands, rows, n, 0.3, 0.5, seed).numpy().view(np.uint32).copy()
    rng = np.random.default_rng(seed + 1)
    if n > 1 and whole:
        for i in rng.choice(np.arange(1, n), size=max(1, n // whole), replace=False):
            s[i] = s[rng.integers(0, i)]
    return s


def _dev(s: np.ndarray) -> torch.Tensor:
    return torch.from_numpy(np.ascontiguousarray(s).view(np.int32)).cuda()


@pytest.mark.parametrize("num_perm,bands,rows", [(128, 16, 8), (256, 32, 8), (16, 5, 3), (512, 64, 8)])
def test_exact_matches_oracle_over_uneven_calls(gpu, num_perm, bands, rows):
    s = _sigs(6000, num_perm, bands, rows, seed=bands)
    cuts = [0, 1, 1, 38, 1038, 1039, 4200, 6000]
    print(f"exact parity P={num_perm} b={bands} r={rows}", flush=True)
    x = gpu.ExactLSH(num_perm, bands, rows, capacity_docs=6000)
    o = ExactLSHOracle(num_perm, bands, rows)
    for a, b in zip(cuts[:-1], cuts[1:]):
        got = x.query_insert(_dev(s[a:b])).cpu().numpy() if b > a else np.zeros(0, np.uint8)
        want = o.query_insert(s[a:b])
        assert got.tolist() == want.tolist(), (a, b)
    st = x.stats()
    assert st["docs_inserted"] == 6000 and st["fp_shared"] == 0
    x.close()


@pytest.mark.parametrize("fp_bits", [1, 4, 8])
def test_exact_with_shared_fingerprints(gpu, fp_bits):
    """Few fingerprint bits: most slots' fingerprints are shared by different
    band values, which the settling pass places by full comparison."""
    s = _sigs(1500, 128, 16, 8, seed=fp_bits)
    print(f"exact fp_bits={fp_bits}", flush=True)
    x = gpu.ExactLSH(128, 16, 8, capacity_docs=1500, fp_bits=fp_bits)
    o = ExactLSHOracle(128, 16, 8)
    for a, b in [(0, 700), (700, 701), (701, 1500)]:
        got = x.query_insert(_dev(s[a:b])).cpu().numpy()
        assert got.tolist() == o.query_insert(s[a:b]).tolist(), (a, b)
    assert x.stats()["fp_shared"] > 0
    x.close()


def test_exact_identical_documents(gpu):
    """A batch of one document repeated: all but the first are flagged, and
    the next call flags every copy."""
    one = _sigs(1, 128, 16, 8, seed=9, whole=0)
    s = np.repeat(one, 300, axis=0)
    x = gpu.ExactLSH(128, 16, 8, capacity_docs=600)
    f1 = x.query_insert(_dev(s)).cpu().numpy()
    f2 = x.query_insert(_dev(s)).cpu().numpy()
    assert f1[0] == 0 and f1[1:].all() and f2.all()
    x.close()


def test_exact_chunks_of_one_call(gpu):
    """A call of 1.2M documents spans two 2^20-document chunks: the flags
    equal the same stream in calls of other sizes and the oracle's on a
    prefix."""
    n = 1_200_000
    s = _sigs(n, 128, 16, 8, seed=3, whole=200)
    d = _dev(s)
    print("exact chunks: one call", flush=True)
    x1 = gpu.ExactLSH(128, 16, 8, capacity_docs=n)
    f1 = x1.query_insert(d).cpu().numpy()
    x1.close()
    print("exact chunks: uneven calls", flush=True)
    x2 = gpu.ExactLSH(128, 16, 8, capacity_docs=n)
    cuts = [0, 65_536, 65_537, 700_000, n]
    f2 = np.concatenate([x2.query_insert(d[a:b]).cpu().numpy() for a, b in zip(cuts[:-1], cuts[1:])])
    x2.close()
    assert f1.tolist() == f2.tolist()
    m = 60_000
    assert f1[:m].tolist() == ExactLSHOracle(128, 16, 8).query_insert(s[:m]).tolist()
    assert 0.2 < f1.mean() < 0.5


def test_exact_capacity_is_enforced(gpu):
    x = gpu.ExactLSH(128, 16, 8, capacity_docs=100)
    s = _sigs(120, 128, 16, 8, seed=4)
    x.query_insert(_dev(s[:100]))
    with pytest.raises(gpu.LSHBloomError):
        x.query_insert(_dev(s[100:]))
    assert x.stats()["docs_inserted"] == 100
    x.close()


def test_lshbloom_flags_contain_exact_flags(gpu):
    """On the same stream LSHBloom flags every document the exact index
    flags (equal band values give equal band keys, and Bloom filters have no
    false negatives); the excess is the filters' false positives (Section
    3.2), a handful at this fill."""
    n = 200_000
    s = _sigs(n, 128, 16, 8, seed=8, whole=100)
    d = _dev(s)
    x = gpu.ExactLSH(128, 16, 8, capacity_docs=n)
    bl = gpu.LSHBloom(128, 16, 8, n, 1e-6, 42)
    fe = x.query_insert(d).cpu().numpy()
    fb = bl.query_insert(d).cpu().numpy()
    assert (fb >= fe).all()
    assert fe.sum() > 10_000
    assert fb.sum() - fe.sum() <= 20
    x.close()
    bl.close()
