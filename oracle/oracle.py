"""ctypes binding of the C oracle (test infrastructure only).

Every function maps one-to-one onto a function of ``lshbloom_oracle.c``; the
paper passage each follows is stated there.
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lshbloom_oracle.c")
_LIB = os.path.join(_HERE, "liblshbloom_oracle.so")

P61 = (1 << 61) - 1

_u8p = ctypes.POINTER(ctypes.c_uint8)
_u32p = ctypes.POINTER(ctypes.c_uint32)
_u64p = ctypes.POINTER(ctypes.c_uint64)
_i64p = ctypes.POINTER(ctypes.c_int64)


def build(force: bool = False) -> str:
    """Compile the oracle into ``oracle/liblshbloom_oracle.so`` with gcc."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        L = _lib
        L.ora_sha1.argtypes = [_u8p, ctypes.c_uint64, _u8p]
        L.ora_shingle_hash.argtypes = [_u32p, ctypes.c_uint32]
        L.ora_shingle_hash.restype = ctypes.c_uint32
        L.ora_fmix64.argtypes = [ctypes.c_uint64]
        L.ora_fmix64.restype = ctypes.c_uint64
        L.ora_splitmix64_next.argtypes = [_u64p]
        L.ora_splitmix64_next.restype = ctypes.c_uint64
        L.ora_perm.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.ora_perm.restype = ctypes.c_uint32
        L.ora_minhash_doc.argtypes = [_u32p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, _u64p, _u64p, _u32p]
        L.ora_band_key.argtypes = [_u32p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
        L.ora_band_key.restype = ctypes.c_uint64
        L.ora_positions.argtypes = [ctypes.c_uint64] * 4 + [ctypes.c_uint32, _u64p]
        L.ora_params.argtypes = [ctypes.c_uint64, ctypes.c_double, _u64p, _u32p]
        L.ora_params.restype = ctypes.c_int
        L.ora_p_band_from_eff.argtypes = [ctypes.c_double, ctypes.c_uint32]
        L.ora_p_band_from_eff.restype = ctypes.c_double
        L.ora_p_eff_from_band.argtypes = [ctypes.c_double, ctypes.c_uint32]
        L.ora_p_eff_from_band.restype = ctypes.c_double
        L.ora_fp_lsh.argtypes = [ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32]
        L.ora_fp_lsh.restype = ctypes.c_double
        L.ora_fn_lsh.argtypes = [ctypes.c_double, ctypes.c_uint32, ctypes.c_uint32]
        L.ora_fn_lsh.restype = ctypes.c_double
        L.ora_optimal_br.argtypes = [ctypes.c_double, ctypes.c_uint32, ctypes.c_double, ctypes.c_double,
                                     ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint32)]
        L.ora_create.argtypes = [ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32]
        L.ora_create.restype = ctypes.c_void_p
        L.ora_destroy.argtypes = [ctypes.c_void_p]
        L.ora_minhash.argtypes = [ctypes.c_void_p, _i64p, _u32p, ctypes.c_int64, _u32p]
        L.ora_minhash.restype = ctypes.c_int
        L.ora_minhash_threads.argtypes = [ctypes.c_void_p, _i64p, _u32p, ctypes.c_int64, _u32p, ctypes.c_int]
        L.ora_minhash_threads.restype = ctypes.c_int
        L.ora_perm61.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_uint32]
        L.ora_perm61.restype = ctypes.c_uint64
        L.ora_minhash_doc61.argtypes = [_u32p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint32, _u64p, _u64p, _u64p]
        L.ora_minhash61.argtypes = [ctypes.c_void_p, _i64p, _u32p, ctypes.c_int64, _u64p]
        L.ora_minhash61.restype = ctypes.c_int
        L.ora_band_key61.argtypes = [_u64p, ctypes.c_uint32, ctypes.c_uint32, ctypes.c_uint64]
        L.ora_band_key61.restype = ctypes.c_uint64
        L.ora_band_keys61.argtypes = [ctypes.c_void_p, _u64p, ctypes.c_int64, _u64p]
        L.ora_query_insert_keys.argtypes = [ctypes.c_void_p, _u64p, ctypes.c_int64, _u8p]
        L.ora_query_insert_keys.restype = ctypes.c_int
        L.ora_query_insert.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int64, _u8p]
        L.ora_query_insert.restype = ctypes.c_int
        L.ora_query.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int64, _u8p]
        L.ora_query.restype = ctypes.c_int
        L.ora_insert.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int64]
        L.ora_insert.restype = ctypes.c_int
        L.ora_m_bits.argtypes = [ctypes.c_void_p]
        L.ora_m_bits.restype = ctypes.c_uint64
        L.ora_k.argtypes = [ctypes.c_void_p]
        L.ora_k.restype = ctypes.c_uint32
        L.ora_words_per_band.argtypes = [ctypes.c_void_p]
        L.ora_words_per_band.restype = ctypes.c_uint64
        L.ora_filters.argtypes = [ctypes.c_void_p]
        L.ora_filters.restype = _u64p
        L.ora_docs_inserted.argtypes = [ctypes.c_void_p]
        L.ora_docs_inserted.restype = ctypes.c_uint64
        L.ora_coeffs.argtypes = [ctypes.c_void_p, _u64p, _u64p, _u64p]
        L.ora_band_keys.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int64, _u64p]
        L.ora_query_insert_band.argtypes = [ctypes.c_void_p, _u32p, ctypes.c_int64, ctypes.c_uint32, _u8p]
        L.ora_query_insert_band.restype = ctypes.c_int
        L.ora_count_docs.argtypes = [ctypes.c_void_p, ctypes.c_uint64]
    return _lib


def _ptr(arr: np.ndarray, ctype):
    return arr.ctypes.data_as(ctypes.POINTER(ctype))


def sha1(data: bytes) -> bytes:
    buf = np.frombuffer(data, dtype=np.uint8).copy() if len(data) else np.zeros(1, np.uint8)
    out = np.zeros(20, np.uint8)
    lib().ora_sha1(_ptr(buf, ctypes.c_uint8), len(data), _ptr(out, ctypes.c_uint8))
    return out.tobytes()


def shingle_hash(tokens) -> int:
    t = np.ascontiguousarray(tokens, dtype=np.uint32)
    return int(lib().ora_shingle_hash(_ptr(t, ctypes.c_uint32), len(t)))


def fmix64(z: int) -> int:
    return int(lib().ora_fmix64(z & (2**64 - 1)))


def splitmix64_stream(seed: int, n: int) -> list[int]:
    s = ctypes.c_uint64(seed & (2**64 - 1))
    return [int(lib().ora_splitmix64_next(ctypes.byref(s))) for _ in range(n)]


def perm(a: int, b: int, x: int) -> int:
    return int(lib().ora_perm(a, b, x))


def perm61(a: int, b: int, x: int) -> int:
    return int(lib().ora_perm61(a, b, x))


def minhash_doc61(tokens, w: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    tok = np.ascontiguousarray(tokens, dtype=np.uint32)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    sig = np.zeros(len(a), np.uint64)
    tp = _ptr(tok, ctypes.c_uint32) if len(tok) else _ptr(np.zeros(1, np.uint32), ctypes.c_uint32)
    lib().ora_minhash_doc61(tp, len(tok), w, len(a), _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64),
                            _ptr(sig, ctypes.c_uint64))
    return sig


def band_key61(sig: np.ndarray, band: int, rows: int, salt_m: int) -> int:
    sig = np.ascontiguousarray(sig, dtype=np.uint64)
    return int(lib().ora_band_key61(_ptr(sig, ctypes.c_uint64), band, rows, salt_m))


def minhash_doc(tokens, w: int, a: np.ndarray, b: np.ndarray) -> np.ndarray:
    t = np.ascontiguousarray(tokens, dtype=np.uint32)
    a = np.ascontiguousarray(a, dtype=np.uint64)
    b = np.ascontiguousarray(b, dtype=np.uint64)
    sig = np.zeros(len(a), np.uint32)
    tp = _ptr(t, ctypes.c_uint32) if len(t) else None
    lib().ora_minhash_doc(tp, len(t), w, len(a), _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64),
                          _ptr(sig, ctypes.c_uint32))
    return sig


def band_key(sig: np.ndarray, band: int, rows: int, salt_m: int) -> int:
    s = np.ascontiguousarray(sig, dtype=np.uint32)
    return int(lib().ora_band_key(_ptr(s, ctypes.c_uint32), band, rows, salt_m))


def positions(key: int, salt1: int, salt2: int, m: int, k: int) -> np.ndarray:
    g = np.zeros(k, np.uint64)
    lib().ora_positions(key, salt1, salt2, m, k, _ptr(g, ctypes.c_uint64))
    return g


def params(n: int, p: float) -> tuple[int, int]:
    m = ctypes.c_uint64()
    k = ctypes.c_uint32()
    if lib().ora_params(n, p, ctypes.byref(m), ctypes.byref(k)) != 0:
        raise ValueError("invalid n or p")
    return int(m.value), int(k.value)


def p_band_from_eff(p_eff: float, bands: int) -> float:
    return float(lib().ora_p_band_from_eff(p_eff, bands))


def p_eff_from_band(p: float, bands: int) -> float:
    return float(lib().ora_p_eff_from_band(p, bands))


def fp_lsh(T: float, b: int, r: int) -> float:
    return float(lib().ora_fp_lsh(T, b, r))


def fn_lsh(T: float, b: int, r: int) -> float:
    return float(lib().ora_fn_lsh(T, b, r))


def optimal_br(T: float, num_perm: int, w_fp: float = 0.5, w_fn: float = 0.5) -> tuple[int, int]:
    b = ctypes.c_uint32()
    r = ctypes.c_uint32()
    lib().ora_optimal_br(T, num_perm, w_fp, w_fn, ctypes.byref(b), ctypes.byref(r))
    return int(b.value), int(r.value)


class OracleIndex:
    """The sequential LSHBloom index: b Bloom filters, one per band."""

    def __init__(self, num_perm: int, bands: int, rows: int, expected_n: int, fp_rate: float, seed: int,
                 w: int = 5):
        self._h = lib().ora_create(num_perm, bands, rows, expected_n, fp_rate, seed, w)
        if not self._h:
            raise ValueError("invalid oracle parameters")
        self.num_perm, self.bands, self.rows, self.w = num_perm, bands, rows, w
        self.m_bits = int(lib().ora_m_bits(self._h))
        self.k = int(lib().ora_k(self._h))
        self.words_per_band = int(lib().ora_words_per_band(self._h))

    def close(self):
        if self._h:
            lib().ora_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def coeffs(self):
        a = np.zeros(self.num_perm, np.uint64)
        b = np.zeros(self.num_perm, np.uint64)
        s = np.zeros(3, np.uint64)
        lib().ora_coeffs(self._h, _ptr(a, ctypes.c_uint64), _ptr(b, ctypes.c_uint64), _ptr(s, ctypes.c_uint64))
        return a, b, [int(v) for v in s]

    def minhash(self, offsets: np.ndarray, tokens: np.ndarray) -> np.ndarray:
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        tokens = np.ascontiguousarray(tokens, dtype=np.uint32)
        n = len(offsets) - 1
        sigs = np.zeros((max(n, 0), self.num_perm), np.uint32)
        tp = _ptr(tokens, ctypes.c_uint32) if len(tokens) else _ptr(np.zeros(1, np.uint32), ctypes.c_uint32)
        rc = lib().ora_minhash(self._h, _ptr(offsets, ctypes.c_int64), tp, n, _ptr(sigs, ctypes.c_uint32))
        if rc != 0:
            raise ValueError("bad CSR batch")
        return sigs

    def minhash_threads(self, offsets: np.ndarray, tokens: np.ndarray, threads: int) -> np.ndarray:
        """minhash() with documents shared out over host threads (same output)."""
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        tokens = np.ascontiguousarray(tokens, dtype=np.uint32)
        n = len(offsets) - 1
        sigs = np.zeros((max(n, 0), self.num_perm), np.uint32)
        tp = _ptr(tokens, ctypes.c_uint32) if len(tokens) else _ptr(np.zeros(1, np.uint32), ctypes.c_uint32)
        rc = lib().ora_minhash_threads(self._h, _ptr(offsets, ctypes.c_int64), tp, n, _ptr(sigs, ctypes.c_uint32),
                                       int(threads))
        if rc != 0:
            raise ValueError("bad CSR batch or thread count")
        return sigs

    def query_insert(self, sigs: np.ndarray) -> np.ndarray:
        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        flags = np.zeros(len(sigs), np.uint8)
        if len(sigs):
            lib().ora_query_insert(self._h, _ptr(sigs, ctypes.c_uint32), len(sigs), _ptr(flags, ctypes.c_uint8))
        return flags

    def query_insert_band(self, sigs: np.ndarray, band: int) -> np.ndarray:
        """Hits of one band over the stream (that band's filter only)."""
        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        hits = np.zeros(len(sigs), np.uint8)
        if len(sigs):
            rc = lib().ora_query_insert_band(self._h, _ptr(sigs, ctypes.c_uint32), len(sigs), band,
                                             _ptr(hits, ctypes.c_uint8))
            if rc != 0:
                raise ValueError("bad band")
        return hits

    def query_insert_by_band(self, sigs: np.ndarray, threads: int = 1) -> np.ndarray:
        """query_insert computed one band at a time (bands on up to `threads`
        host threads, each band's stream sequential); flags = OR of the hits."""
        from concurrent.futures import ThreadPoolExecutor

        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        with ThreadPoolExecutor(max_workers=max(1, int(threads))) as ex:
            hits = list(ex.map(lambda j: self.query_insert_band(sigs, j), range(self.bands)))
        lib().ora_count_docs(self._h, len(sigs))
        flags = np.zeros(len(sigs), np.uint8)
        for h in hits:
            flags |= h
        return flags

    def filters_view(self) -> np.ndarray:
        """The filter words in place (no copy), shape [bands, words_per_band];
        valid while the index is open."""
        n = self.bands * self.words_per_band
        p = lib().ora_filters(self._h)
        return np.ctypeslib.as_array(p, shape=(n,)).reshape(self.bands, self.words_per_band)

    def load_file(self, path: str) -> None:
        """Replace the filters with those of an index file in the documented
        layout (an 80-byte little-endian header: "LSHBLM01", num_perm, bands,
        rows, shingle width as u32; expected_n u64; fp_rate f64; seed, m_bits
        u64; k, 0 u32; docs_inserted, words_per_band u64; then the band-major
        filter words), after checking that it describes this index."""
        import struct

        with open(path, "rb") as f:
            hd = f.read(80)
            if len(hd) != 80 or hd[:8] != b"LSHBLM01":
                raise ValueError(f"{path} is not an index file")
            P, b, r, w, n, p, seed, m, k, _, docs, wpb = struct.unpack("<4IQdQQIIQQ", hd[8:])
            if (P, b, r, w, m, k, wpb) != (self.num_perm, self.bands, self.rows, self.w, self.m_bits, self.k,
                                           self.words_per_band):
                raise ValueError(f"{path} holds an index of other parameters")
            view = self.filters_view().reshape(-1)
            step = 1 << 24
            for a in range(0, view.size, step):
                chunk = np.frombuffer(f.read(8 * min(step, view.size - a)), dtype="<u8")
                if chunk.size != min(step, view.size - a):
                    raise ValueError(f"{path} is shorter than its header says")
                view[a:a + chunk.size] = chunk
        lib().ora_count_docs(self._h, docs - self.docs_inserted)

    def query(self, sigs: np.ndarray) -> np.ndarray:
        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        flags = np.zeros(len(sigs), np.uint8)
        if len(sigs):
            lib().ora_query(self._h, _ptr(sigs, ctypes.c_uint32), len(sigs), _ptr(flags, ctypes.c_uint8))
        return flags

    def insert(self, sigs: np.ndarray) -> None:
        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        if len(sigs):
            lib().ora_insert(self._h, _ptr(sigs, ctypes.c_uint32), len(sigs))

    def band_keys(self, sigs: np.ndarray) -> np.ndarray:
        sigs = np.ascontiguousarray(sigs, dtype=np.uint32).reshape(-1, self.num_perm)
        keys = np.zeros((len(sigs), self.bands), np.uint64)
        if len(sigs):
            lib().ora_band_keys(self._h, _ptr(sigs, ctypes.c_uint32), len(sigs), _ptr(keys, ctypes.c_uint64))
        return keys

    # -- wide-value variant (61-bit signature values) ------------------------
    def minhash61(self, offsets: np.ndarray, tokens: np.ndarray) -> np.ndarray:
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        tokens = np.ascontiguousarray(tokens, dtype=np.uint32)
        n = len(offsets) - 1
        sigs = np.zeros((max(n, 0), self.num_perm), np.uint64)
        tp = _ptr(tokens, ctypes.c_uint32) if len(tokens) else _ptr(np.zeros(1, np.uint32), ctypes.c_uint32)
        rc = lib().ora_minhash61(self._h, _ptr(offsets, ctypes.c_int64), tp, n, _ptr(sigs, ctypes.c_uint64))
        if rc != 0:
            raise ValueError("bad CSR batch")
        return sigs

    def band_keys61(self, sigs: np.ndarray) -> np.ndarray:
        sigs = np.ascontiguousarray(sigs, dtype=np.uint64).reshape(-1, self.num_perm)
        keys = np.zeros((len(sigs), self.bands), np.uint64)
        if len(sigs):
            lib().ora_band_keys61(self._h, _ptr(sigs, ctypes.c_uint64), len(sigs), _ptr(keys, ctypes.c_uint64))
        return keys

    def query_insert_keys(self, keys: np.ndarray) -> np.ndarray:
        keys = np.ascontiguousarray(keys, dtype=np.uint64).reshape(-1, self.bands)
        flags = np.zeros(len(keys), np.uint8)
        if len(keys):
            lib().ora_query_insert_keys(self._h, _ptr(keys, ctypes.c_uint64), len(keys), _ptr(flags, ctypes.c_uint8))
        return flags

    def filters(self) -> np.ndarray:
        """A copy of the filter words, shape [bands, words_per_band]."""
        n = self.bands * self.words_per_band
        p = lib().ora_filters(self._h)
        arr = np.ctypeslib.as_array(p, shape=(n,))
        return arr.copy().reshape(self.bands, self.words_per_band)

    def set_filters(self, words: np.ndarray) -> None:
        n = self.bands * self.words_per_band
        src = np.ascontiguousarray(words, dtype=np.uint64).reshape(-1)
        if len(src) != n:
            raise ValueError("filter size mismatch")
        p = lib().ora_filters(self._h)
        np.ctypeslib.as_array(p, shape=(n,))[:] = src

    @property
    def docs_inserted(self) -> int:
        return int(lib().ora_docs_inserted(self._h))
