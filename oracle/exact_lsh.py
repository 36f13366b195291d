"""Exact MinHashLSH band index, CPU reference (test infrastructure only).

MinHashLSH as the paper describes it (Section 2.3, "MinHashLSH for Text
Deduplication"; Section 4, opening paragraphs of the method): the signature
matrix is cut into b bands of r rows, and two documents whose signatures are
identical over all r rows of some band are a candidate pair, taken here as a
duplicate.  The traditional index keeps, per band, a hash map keyed by the
band's r values.  In a stream, document i is flagged iff some band of its
signature equals the same band of an earlier document's signature; every
document is inserted after its query (flagged or not), the same order the
LSHBloom reference follows, so that the two indexes answer the same question
and differ only by the Bloom filters' false positives (Section 4.3, Eq. 3).

Plain Python dictionaries keyed by the band's bytes; no hashing of the band
values of our own, no batching: one document after the other.  Only the
tests and the benchmark's fidelity leg use it; the GPU library never does.
"""

from __future__ import annotations

import numpy as np


class ExactLSHOracle:
    """Per band: {band values as bytes: index of the first document with them}."""

    def __init__(self, num_perm: int, bands: int, rows: int):
        if bands * rows > num_perm or bands == 0 or rows == 0:
            raise ValueError("need 0 < bands * rows <= num_perm")
        self.num_perm, self.bands, self.rows = num_perm, bands, rows
        self.tables = [dict() for _ in range(bands)]
        self.docs_inserted = 0

    def query_insert(self, sigs: np.ndarray) -> np.ndarray:
        """Flags of the documents of `sigs` (uint32 [n][num_perm]) in order."""
        sigs = np.ascontiguousarray(sigs).view(np.uint32).reshape(-1, self.num_perm)
        n = sigs.shape[0]
        flags = np.zeros(n, dtype=np.uint8)
        r = self.rows
        for i in range(n):
            doc = self.docs_inserted + i
            hit = False
            for j, table in enumerate(self.tables):
                key = sigs[i, j * r:(j + 1) * r].tobytes()
                if key in table:
                    hit = True
                else:
                    table[key] = doc
            flags[i] = hit
        self.docs_inserted += n
        return flags


def brute_force_flags(sigs: np.ndarray, bands: int, rows: int) -> np.ndarray:
    """The same flags by comparing every pair of documents (i' < i) band by
    band: O(n^2), for tiny inputs only."""
    sigs = np.ascontiguousarray(sigs).view(np.uint32)
    n = sigs.shape[0]
    flags = np.zeros(n, dtype=np.uint8)
    for j in range(bands):
        band = sigs[:, j * rows:(j + 1) * rows]
        eq = (band[:, None, :] == band[None, :, :]).all(axis=2)  # eq[i, i']
        earlier = np.tril(eq, k=-1).any(axis=1)
        flags |= earlier.astype(np.uint8)
    return flags
