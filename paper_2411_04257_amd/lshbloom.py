"""Python binding of liblshbloom.so (argument marshalling only).

Every method maps onto one C-ABI entry point of include/lshbloom.h; all
per-document work runs in the library's HIP kernels.  Tensors are torch CUDA
tensors (PyTorch provides device memory and streams); each call is enqueued on
torch's current stream.  If the library is not built or cannot be loaded the
binding raises: there is no fallback path.
"""

from __future__ import annotations

import ctypes
import os

import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liblshbloom.so")

OK, EINVAL, ENOMEM, EHIP, EPOISONED, EIO, EDEVICE = 0, -1, -2, -3, -4, -5, -6
QI_AUTO, QI_DIRECT, QI_BINNED = 0, 1, 2
_CODES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EHIP: "EHIP", EPOISONED: "EPOISONED", EIO: "EIO",
          EDEVICE: "EDEVICE"}


class LSHBloomError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODES.get(code, code)}: {msg}")
        self.code = code


class Params(ctypes.Structure):
    _fields_ = [
        ("num_perm", ctypes.c_uint32),
        ("bands", ctypes.c_uint32),
        ("rows", ctypes.c_uint32),
        ("expected_n", ctypes.c_uint64),
        ("fp_rate", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("shingle_width", ctypes.c_uint32),
        ("hbm_budget", ctypes.c_uint64),
        ("chunk_docs", ctypes.c_uint64),
        ("qi_mode", ctypes.c_uint32),
        ("workspace_budget", ctypes.c_uint64),
    ]


class Info(ctypes.Structure):
    _fields_ = [
        ("num_perm", ctypes.c_uint32),
        ("bands", ctypes.c_uint32),
        ("rows", ctypes.c_uint32),
        ("shingle_width", ctypes.c_uint32),
        ("k", ctypes.c_uint32),
        ("m_bits", ctypes.c_uint64),
        ("words_per_band", ctypes.c_uint64),
        ("filter_bytes", ctypes.c_uint64),
        ("workspace_bytes", ctypes.c_uint64),
        ("chunk_docs", ctypes.c_uint64),
        ("binned_chunk_docs", ctypes.c_uint64),
        ("fp_rate", ctypes.c_double),
        ("p_eff", ctypes.c_double),
        ("docs_inserted", ctypes.c_uint64),
        ("seed", ctypes.c_uint64),
        ("poisoned", ctypes.c_int),
        ("device_status", ctypes.c_uint32),
        ("general_path_bins", ctypes.c_uint64),
    ]


class PipelineParams(ctypes.Structure):
    _fields_ = [
        ("max_docs", ctypes.c_uint64),
        ("max_tokens", ctypes.c_uint64),
        ("n_buckets", ctypes.c_uint32),
        ("bucket_edges", ctypes.c_uint64 * 3),
        ("waves_per_cu", ctypes.c_uint32 * 4),
        ("use_graph", ctypes.c_uint32),
        ("autotune", ctypes.c_uint32),
        ("tune_cache", ctypes.c_char_p),
    ]


class PipelineInfo(ctypes.Structure):
    _fields_ = [
        ("n_buckets", ctypes.c_uint32),
        ("bucket_edges", ctypes.c_uint64 * 3),
        ("waves_per_cu", ctypes.c_uint32 * 4),
        ("tuned", ctypes.c_int),
        ("tune_best_ms", ctypes.c_float),
        ("batches", ctypes.c_uint64),
        ("graph_launches", ctypes.c_uint64),
        ("graph_updates", ctypes.c_uint64),
        ("graph_instantiations", ctypes.c_uint64),
        ("timed_batches", ctypes.c_uint64),
        ("minhash_ms_total", ctypes.c_double),
        ("qi_ms_total", ctypes.c_double),
    ]


# Every symbol the header declares.
EXPORTS = [
    "lshbloom_create", "lshbloom_create_ex", "lshbloom_destroy", "lshbloom_minhash", "lshbloom_query_insert",
    "lshbloom_query", "lshbloom_insert", "lshbloom_band_keys", "lshbloom_read_filters", "lshbloom_write_filters",
    "lshbloom_count_set_bits", "lshbloom_save", "lshbloom_load", "lshbloom_info", "lshbloom_p_band_from_eff", "lshbloom_optimal_bands", "lshbloom_last_error",
    "lshbloom_pipeline_create", "lshbloom_pipeline_submit", "lshbloom_pipeline_wait", "lshbloom_pipeline_poll",
    "lshbloom_pipeline_info", "lshbloom_pipeline_destroy",
    "lshbloom_exact_create", "lshbloom_exact_destroy", "lshbloom_exact_query_insert", "lshbloom_exact_stats",
    "lshbloom_query_insert_keys", "lshbloom_minhash61", "lshbloom_band_keys61",
    "lshbloom_query_insert_noalloc", "lshbloom_sync",
]
NOALLOC_MAX_DOCS = 65536

_lib = None


def load(path: str = LIB_PATH):
    """Load liblshbloom.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build the HIP library first (__graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i64, u32, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64
    L.lshbloom_create.argtypes = [u32, u32, u32, u64, ctypes.c_double, u64]
    L.lshbloom_create.restype = vp
    L.lshbloom_create_ex.argtypes = [ctypes.POINTER(Params)]
    L.lshbloom_create_ex.restype = vp
    L.lshbloom_destroy.argtypes = [vp]
    L.lshbloom_destroy.restype = None
    L.lshbloom_minhash.argtypes = [vp, vp, vp, i64, vp, vp]
    L.lshbloom_query_insert.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_query_insert_noalloc.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_query.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_insert.argtypes = [vp, vp, i64, vp]
    L.lshbloom_band_keys.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_read_filters.argtypes = [vp, vp, u64, u64, vp]
    L.lshbloom_write_filters.argtypes = [vp, vp, u64, u64, u64, vp]
    L.lshbloom_count_set_bits.argtypes = [vp, vp, vp]
    L.lshbloom_save.argtypes = [vp, ctypes.c_char_p, vp]
    L.lshbloom_load.argtypes = [vp, ctypes.c_char_p, vp]
    L.lshbloom_info.argtypes = [vp, ctypes.POINTER(Info)]
    L.lshbloom_sync.argtypes = [vp]
    L.lshbloom_p_band_from_eff.argtypes = [ctypes.c_double, u32]
    L.lshbloom_p_band_from_eff.restype = ctypes.c_double
    L.lshbloom_optimal_bands.argtypes = [ctypes.c_double, u32, ctypes.c_double, ctypes.c_double,
                                         ctypes.POINTER(u32), ctypes.POINTER(u32)]
    L.lshbloom_pipeline_create.argtypes = [vp, ctypes.POINTER(PipelineParams)]
    L.lshbloom_pipeline_create.restype = vp
    L.lshbloom_pipeline_submit.argtypes = [vp, vp, vp, i64, vp]
    L.lshbloom_pipeline_submit.restype = i64
    L.lshbloom_pipeline_wait.argtypes = [vp, i64]
    L.lshbloom_pipeline_wait.restype = ctypes.c_int
    L.lshbloom_pipeline_poll.argtypes = [vp, i64]
    L.lshbloom_pipeline_poll.restype = ctypes.c_int
    L.lshbloom_pipeline_info.argtypes = [vp, ctypes.POINTER(PipelineInfo)]
    L.lshbloom_pipeline_info.restype = ctypes.c_int
    L.lshbloom_pipeline_destroy.argtypes = [vp]
    L.lshbloom_pipeline_destroy.restype = None
    L.lshbloom_query_insert_keys.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_query_insert_keys.restype = ctypes.c_int
    L.lshbloom_minhash61.argtypes = [vp, vp, vp, i64, vp, vp]
    L.lshbloom_minhash61.restype = ctypes.c_int
    L.lshbloom_band_keys61.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_band_keys61.restype = ctypes.c_int
    L.lshbloom_exact_create.argtypes = [u32, u32, u32, u64, u32]
    L.lshbloom_exact_create.restype = vp
    L.lshbloom_exact_destroy.argtypes = [vp]
    L.lshbloom_exact_destroy.restype = None
    L.lshbloom_exact_query_insert.argtypes = [vp, vp, i64, vp, vp]
    L.lshbloom_exact_query_insert.restype = ctypes.c_int
    L.lshbloom_exact_stats.argtypes = [vp, vp, vp, vp]
    L.lshbloom_exact_stats.restype = ctypes.c_int
    L.lshbloom_last_error.argtypes = []
    L.lshbloom_last_error.restype = ctypes.c_char_p
    for name in ("lshbloom_minhash", "lshbloom_query_insert", "lshbloom_query_insert_noalloc", "lshbloom_query",
                 "lshbloom_insert",
                 "lshbloom_band_keys", "lshbloom_read_filters", "lshbloom_write_filters",
                 "lshbloom_count_set_bits", "lshbloom_save", "lshbloom_load", "lshbloom_info", "lshbloom_optimal_bands",
                 "lshbloom_sync"):
        getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def last_error() -> str:
    return load().lshbloom_last_error().decode()


def _check(rc: int):
    if rc != OK:
        raise LSHBloomError(rc, last_error())


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _dev_ptr(t: torch.Tensor, dtypes, name: str):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a CUDA tensor")
    if t.dtype not in dtypes:
        raise ValueError(f"{name} has dtype {t.dtype}, expected one of {dtypes}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


_U32 = (torch.int32, torch.uint32)


def p_band_from_eff(p_eff: float, bands: int) -> float:
    return float(load().lshbloom_p_band_from_eff(p_eff, bands))


def optimal_bands(threshold: float, num_perm: int, w_fp: float = 0.5, w_fn: float = 0.5) -> tuple[int, int]:
    b, r = ctypes.c_uint32(), ctypes.c_uint32()
    _check(load().lshbloom_optimal_bands(threshold, num_perm, w_fp, w_fn, ctypes.byref(b), ctypes.byref(r)))
    return int(b.value), int(r.value)


class LSHBloom:
    """An LSHBloom index on the current GPU: one Bloom filter per band."""

    def __init__(self, num_perm: int, bands: int, rows: int, expected_n: int, fp_rate: float, seed: int = 42,
                 shingle_width: int = 5, hbm_budget: int = 0, chunk_docs: int = 0, qi_mode: int = 0,
                 workspace_budget: int = 0):
        L = load()
        p = Params(num_perm, bands, rows, int(expected_n), float(fp_rate), int(seed), shingle_width,
                   int(hbm_budget), int(chunk_docs), int(qi_mode), int(workspace_budget))
        self._h = L.lshbloom_create_ex(ctypes.byref(p))
        if not self._h:
            raise LSHBloomError(EINVAL, last_error())
        self.num_perm, self.bands, self.rows = num_perm, bands, rows
        inf = self.info()
        self.k, self.m_bits, self.words_per_band = inf["k"], inf["m_bits"], inf["words_per_band"]

    # -- lifecycle -----------------------------------------------------------
    def close(self):
        if getattr(self, "_h", None):
            load().lshbloom_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    # -- hot path ------------------------------------------------------------
    def minhash(self, offsets: torch.Tensor, tokens: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = offsets.numel() - 1
        if out is None:
            out = torch.empty((max(n, 0), self.num_perm), dtype=torch.int32, device=offsets.device)
        if n <= 0:
            return out
        if out.shape != (n, self.num_perm):
            raise ValueError("out must have shape [n_docs, num_perm]")
        _check(load().lshbloom_minhash(self._h, _dev_ptr(offsets, (torch.int64,), "offsets"),
                                       _dev_ptr(tokens, _U32, "tokens") if tokens.numel() else ctypes.c_void_p(
                                           offsets.data_ptr()),
                                       n, _dev_ptr(out, _U32, "out"), _stream()))
        return out

    def query_insert(self, sigs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = self._rows_of(sigs)
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=sigs.device)
        if n:
            _check(load().lshbloom_query_insert(self._h, _dev_ptr(sigs, _U32, "sigs"), n,
                                                _dev_ptr(out, (torch.uint8,), "out"), _stream()))
        return out

    def query_insert_noalloc(self, sigs: torch.Tensor, out: torch.Tensor) -> torch.Tensor:
        """query_insert through the allocation-free entry point (out must be given)."""
        n = self._rows_of(sigs)
        if out.numel() != n:
            raise ValueError("out must hold one flag per document")
        _check(load().lshbloom_query_insert_noalloc(self._h, _dev_ptr(sigs, _U32, "sigs") if n else None, n,
                                                    _dev_ptr(out, (torch.uint8,), "out") if n else None, _stream()))
        return out

    def query(self, sigs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        n = self._rows_of(sigs)
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=sigs.device)
        if n:
            _check(load().lshbloom_query(self._h, _dev_ptr(sigs, _U32, "sigs"), n,
                                         _dev_ptr(out, (torch.uint8,), "out"), _stream()))
        return out

    def insert(self, sigs: torch.Tensor) -> None:
        n = self._rows_of(sigs)
        if n:
            _check(load().lshbloom_insert(self._h, _dev_ptr(sigs, _U32, "sigs"), n, _stream()))

    def band_keys(self, sigs: torch.Tensor) -> torch.Tensor:
        n = self._rows_of(sigs)
        out = torch.empty((n, self.bands), dtype=torch.int64, device=sigs.device)
        if n:
            _check(load().lshbloom_band_keys(self._h, _dev_ptr(sigs, _U32, "sigs"), n,
                                             _dev_ptr(out, (torch.int64,), "out"), _stream()))
        return out

    def query_insert_keys(self, keys: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Query-insert from band keys int64 [n, bands] (uint64 bit patterns)."""
        if keys.dim() != 2 or keys.shape[1] != self.bands:
            raise ValueError("keys must have shape [n_docs, bands]")
        n = keys.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=keys.device)
        if n:
            _check(load().lshbloom_query_insert_keys(self._h, _dev_ptr(keys, (torch.int64, torch.uint64), "keys"), n,
                                                     _dev_ptr(out, (torch.uint8,), "out"), _stream()))
        return out

    # -- wide-value variant (61-bit signature values) --------------------------
    def minhash61(self, offsets: torch.Tensor, tokens: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        """Signatures int64 [n_docs, num_perm] of whole 61-bit permutation values."""
        n = offsets.numel() - 1
        if out is None:
            out = torch.empty((max(n, 0), self.num_perm), dtype=torch.int64, device=offsets.device)
        if n <= 0:
            return out
        if out.shape != (n, self.num_perm):
            raise ValueError("out must have shape [n_docs, num_perm]")
        _check(load().lshbloom_minhash61(self._h, _dev_ptr(offsets, (torch.int64,), "offsets"),
                                         _dev_ptr(tokens, _U32, "tokens") if tokens.numel() else ctypes.c_void_p(
                                             offsets.data_ptr()),
                                         n, _dev_ptr(out, (torch.int64, torch.uint64), "out"), _stream()))
        return out

    def band_keys61(self, sigs: torch.Tensor) -> torch.Tensor:
        if sigs.dim() != 2 or sigs.shape[1] != self.num_perm:
            raise ValueError("sigs must have shape [n_docs, num_perm]")
        n = sigs.shape[0]
        out = torch.empty((n, self.bands), dtype=torch.int64, device=sigs.device)
        if n:
            _check(load().lshbloom_band_keys61(self._h, _dev_ptr(sigs, (torch.int64, torch.uint64), "sigs"), n,
                                               _dev_ptr(out, (torch.int64,), "out"), _stream()))
        return out

    # -- filters -------------------------------------------------------------
    def read_filters(self, out: torch.Tensor | None = None) -> torch.Tensor:
        """Filter words as int64 [bands, words_per_band] (uint64 bit patterns)."""
        if out is None:
            out = torch.empty((self.bands, self.words_per_band), dtype=torch.int64, device="cuda")
        nbytes = out.numel() * 8
        ptr = out.data_ptr()
        _check(load().lshbloom_read_filters(self._h, ctypes.c_void_p(ptr), 0, nbytes, _stream()))
        return out

    def save(self, path: str) -> None:
        """Write the index (header + filter words) to `path` (synchronous)."""
        _check(load().lshbloom_save(self._h, str(path).encode(), _stream()))

    def load(self, path: str) -> None:
        """Replace the filters and docs_inserted from a file written by save()."""
        _check(load().lshbloom_load(self._h, str(path).encode(), _stream()))

    def count_set_bits(self) -> list:
        """Set bits of each band's filter (synchronous)."""
        out = (ctypes.c_uint64 * self.bands)()
        _check(load().lshbloom_count_set_bits(self._h, ctypes.cast(out, ctypes.c_void_p), _stream()))
        return [int(v) for v in out]

    def write_filters(self, words: torch.Tensor, docs_inserted: int | None = None) -> None:
        if not words.is_contiguous():
            raise ValueError("words must be contiguous")
        di = (1 << 64) - 1 if docs_inserted is None else int(docs_inserted)
        _check(load().lshbloom_write_filters(self._h, ctypes.c_void_p(words.data_ptr()), 0, words.numel() * 8, di,
                                             _stream()))

    def sync(self) -> None:
        """Wait for the handle's calls; raises EDEVICE if a kernel reported an inconsistency."""
        _check(load().lshbloom_sync(self._h))

    def info(self) -> dict:
        inf = Info()
        _check(load().lshbloom_info(self._h, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in Info._fields_}

    def _rows_of(self, sigs: torch.Tensor) -> int:
        if sigs.dim() != 2 or sigs.shape[1] != self.num_perm:
            raise ValueError(f"signatures must have shape [n, {self.num_perm}]")
        return int(sigs.shape[0])


class Pipeline:
    """Batched form: host CSR batches in, host flags out, through one index.

    Length-bucketed persistent MinHash, in-order query-insert, two slots so
    that consecutive batches overlap, optional hipGraph replay and autotuning
    (all inside the C library)."""

    def __init__(self, index: LSHBloom, max_docs: int, max_tokens: int, n_buckets: int = 0,
                 bucket_edges=(0, 0, 0), waves_per_cu=(0, 0, 0, 0), use_graph: bool = True,
                 autotune: bool = True, tune_cache: str | None = None):
        L = load()
        self.index = index
        self._cache = tune_cache.encode() if tune_cache else None
        p = PipelineParams(int(max_docs), int(max_tokens), int(n_buckets),
                           (ctypes.c_uint64 * 3)(*[int(e) for e in bucket_edges]),
                           (ctypes.c_uint32 * 4)(*[int(w) for w in waves_per_cu]),
                           int(bool(use_graph)), int(bool(autotune)), self._cache)
        self._p = L.lshbloom_pipeline_create(ctypes.c_void_p(index._h), ctypes.byref(p))
        if not self._p:
            raise LSHBloomError(EINVAL, last_error())
        self._keep = {}

    def submit(self, offsets, tokens, flags_out) -> int:
        """offsets: int64 host array [n+1]; tokens: uint32/int32 host array;
        flags_out: uint8 host array [n] (filled when the ticket completes).
        numpy arrays or CPU torch tensors (pinned ones are copied by DMA)."""
        import numpy as np

        def ptr(a):
            if isinstance(a, torch.Tensor):
                if a.is_cuda or not a.is_contiguous():
                    raise ValueError("pipeline buffers must be contiguous host tensors")
                return a.data_ptr()
            if not (isinstance(a, np.ndarray) and a.flags["C_CONTIGUOUS"]):
                raise ValueError("pipeline buffers must be contiguous numpy arrays or host tensors")
            return a.ctypes.data

        n = (offsets.numel() if isinstance(offsets, torch.Tensor) else len(offsets)) - 1
        t = load().lshbloom_pipeline_submit(self._p, ctypes.c_void_p(ptr(offsets)), ctypes.c_void_p(ptr(tokens)),
                                            n, ctypes.c_void_p(ptr(flags_out)))
        if t < 0:
            raise LSHBloomError(int(t), last_error())
        self._keep[t] = (offsets, tokens, flags_out)  # keep the buffers alive until waited
        return int(t)

    def wait(self, ticket: int) -> None:
        _check(load().lshbloom_pipeline_wait(self._p, ticket))
        self._keep.pop(ticket, None)

    def poll(self, ticket: int) -> bool:
        """True once the batch is done (its flags are then in place)."""
        rc = load().lshbloom_pipeline_poll(self._p, ticket)
        if rc < 0:
            raise LSHBloomError(rc, last_error())
        if rc == 1:
            self._keep.pop(ticket, None)
        return rc == 1

    def info(self) -> dict:
        inf = PipelineInfo()
        _check(load().lshbloom_pipeline_info(self._p, ctypes.byref(inf)))
        d = {name: getattr(inf, name) for name, _ in PipelineInfo._fields_}
        d["bucket_edges"] = list(d["bucket_edges"])
        d["waves_per_cu"] = list(d["waves_per_cu"])
        return d

    def close(self):
        if getattr(self, "_p", None):
            load().lshbloom_pipeline_destroy(self._p)
            self._p = None
            self._keep.clear()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class ExactLSH:
    """The exact MinHashLSH band index (the comparison baseline) on the
    current GPU: per band a table keyed by the band's r values."""

    def __init__(self, num_perm: int, bands: int, rows: int, capacity_docs: int, fp_bits: int = 0):
        L = load()
        self._x = L.lshbloom_exact_create(num_perm, bands, rows, int(capacity_docs), int(fp_bits))
        if not self._x:
            raise LSHBloomError(EINVAL, last_error())
        self.num_perm, self.bands, self.rows = num_perm, bands, rows

    def query_insert(self, sigs: torch.Tensor, out: torch.Tensor | None = None) -> torch.Tensor:
        if sigs.dim() != 2 or sigs.shape[1] != self.num_perm:
            raise ValueError("sigs must have shape [n_docs, num_perm]")
        n = sigs.shape[0]
        if out is None:
            out = torch.empty(n, dtype=torch.uint8, device=sigs.device)
        if n:
            _check(load().lshbloom_exact_query_insert(self._x, _dev_ptr(sigs, _U32, "sigs"), n,
                                                      _dev_ptr(out, (torch.uint8,), "out"), _stream()))
        return out

    def stats(self) -> dict:
        d, t, f = ctypes.c_uint64(), ctypes.c_uint64(), ctypes.c_uint64()
        _check(load().lshbloom_exact_stats(self._x, ctypes.byref(d), ctypes.byref(t), ctypes.byref(f)))
        return {"docs_inserted": d.value, "table_bytes": t.value, "fp_shared": f.value}

    def close(self):
        if getattr(self, "_x", None):
            load().lshbloom_exact_destroy(self._x)
            self._x = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
