"""LSHBloom CPU oracle (test infrastructure only).

A plain sequential reference of the LSHBloom hot path, written in C
(`lshbloom_oracle.c`) and wrapped here with ctypes, and of the exact
MinHashLSH band index it replaces (`exact_lsh.py`, plain Python).  Only the tests, the smoke
check and the benchmark's CPU-baseline leg may import it; the GPU library never
does, and the two share no code.
"""

from .oracle import (  # noqa: F401
    P61,
    OracleIndex,
    band_key,
    band_key61,
    build,
    fmix64,
    fn_lsh,
    fp_lsh,
    lib,
    minhash_doc,
    minhash_doc61,
    optimal_br,
    p_band_from_eff,
    p_eff_from_band,
    params,
    perm,
    perm61,
    positions,
    sha1,
    shingle_hash,
    splitmix64_stream,
)
from .exact_lsh import ExactLSHOracle, brute_force_flags  # noqa: F401,E402
