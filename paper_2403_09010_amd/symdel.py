"""Python binding of libsymdel.so (ctypes; argument marshalling only).

Every step of the search runs in the library's HIP kernels. PyTorch is used
for device tensors and the current HIP stream; numpy arrays are passed as
host memory. The binding has no fallback: if the library is not built or
cannot be loaded, ``Context()`` raises.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsymdel.so")

SD_OK = 0
ERRORS = {
    -1: "SD_E_INVAL", -2: "SD_E_ALPHABET", -3: "SD_E_LENGTH", -4: "SD_E_TOO_MANY",
    -5: "SD_E_NOMEM", -6: "SD_E_HIP", -7: "SD_E_CANCELLED", -8: "SD_E_STATE",
}
OPT_TIMING = 1
OPT_PATH = 2
OPT_GROUP_CAP = 3
OPT_GROUP_BITS = 4
OPT_SORT_ITEMS = 5
MAX_STAGES = 16


class SymdelError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{ERRORS.get(code, code)}: {msg}")
        self.code = code
        self.name = ERRORS.get(code, str(code))


class _Seqs(ctypes.Structure):
    _fields_ = [("codes", ctypes.c_void_p), ("offsets", ctypes.c_void_p),
                ("n", ctypes.c_int64), ("on_device", ctypes.c_int32)]


class _Pairs(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("i", ctypes.c_void_p), ("j", ctypes.c_void_p),
                ("d", ctypes.c_void_p), ("on_device", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class _Stats(ctypes.Structure):
    _fields_ = [("n_seqs", ctypes.c_int64), ("n_keys", ctypes.c_int64),
                ("n_cand_raw", ctypes.c_int64), ("n_cand_unique", ctypes.c_int64),
                ("n_pairs", ctypes.c_int64), ("n_stages", ctypes.c_int32),
                ("n_sort_passes", ctypes.c_int32), ("n_big_segments", ctypes.c_int64),
                ("stage_name", (ctypes.c_char * 24) * MAX_STAGES),
                ("stage_ms", ctypes.c_double * MAX_STAGES),
                ("stage_bytes", ctypes.c_double * MAX_STAGES),
                ("stage_launches", ctypes.c_int32 * MAX_STAGES)]


_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsymdel.so (raises OSError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run __graft_entry__.build() first")
    lib = ctypes.CDLL(path)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.sd_create.argtypes = [ctypes.POINTER(P), I, ctypes.c_uint64]
    lib.sd_create.restype = I
    lib.sd_destroy.argtypes = [P]
    lib.sd_destroy.restype = None
    lib.sd_set_option.argtypes = [P, I, I64]
    lib.sd_set_option.restype = I
    lib.sd_self_search.argtypes = [P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_self_search.restype = I
    lib.sd_pair_distance.argtypes = [P, ctypes.POINTER(_Seqs), ctypes.POINTER(_Seqs), P, P, I64,
                                     P, P]
    lib.sd_pair_distance.restype = I
    lib.sd_get_stats.argtypes = [P, ctypes.POINTER(_Stats)]
    lib.sd_get_stats.restype = I
    lib.sd_pairs_copy.argtypes = [P, ctypes.POINTER(_Pairs), P, P, P, I, P]
    lib.sd_pairs_copy.restype = I
    lib.sd_pairs_free.argtypes = [P, ctypes.POINTER(_Pairs)]
    lib.sd_pairs_free.restype = None
    lib.sd_strerror.argtypes = [I]
    lib.sd_strerror.restype = ctypes.c_char_p
    lib.sd_last_error.argtypes = [P]
    lib.sd_last_error.restype = ctypes.c_char_p
    _lib = lib
    return lib


def _is_torch(x) -> bool:
    return type(x).__module__.startswith("torch")


def _stream_handle(stream, device_inputs: bool):
    if stream is not None:
        return stream if isinstance(stream, int) else int(stream.cuda_stream)
    if device_inputs:
        import torch
        return int(torch.cuda.current_stream().cuda_stream)
    return None


@dataclass
class Pairs:
    """Result triplets; arrays are numpy (host) or torch tensors (device)."""
    i: object
    j: object
    d: object

    def __len__(self):
        return len(self.i)

    def numpy(self):
        if _is_torch(self.i):
            return self.i.cpu().numpy(), self.j.cpu().numpy(), self.d.cpu().numpy()
        return self.i, self.j, self.d


class Context:
    """A library context on one HIP device (see sd_create)."""

    def __init__(self, device: int = 0, hbm_budget: int = 0):
        self._lib = load_library()
        self._h = ctypes.c_void_p()
        rc = self._lib.sd_create(ctypes.byref(self._h), device, hbm_budget)
        if rc != SD_OK:
            raise SymdelError(rc, f"sd_create(device={device}) failed")
        self.device = device

    # ------------------------------------------------------------ plumbing
    def close(self):
        if self._h:
            self._lib.sd_destroy(self._h)
            self._h = ctypes.c_void_p()

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc: int, what: str):
        if rc != SD_OK:
            msg = self._lib.sd_last_error(self._h).decode() or self._lib.sd_strerror(rc).decode()
            raise SymdelError(rc, f"{what}: {msg}")

    def set_option(self, option: int, value: int):
        self._check(self._lib.sd_set_option(self._h, option, int(value)), "sd_set_option")

    def _seqs(self, codes, offsets):
        """(sd_seqs, keepalive, on_device) for numpy arrays or torch tensors."""
        if _is_torch(codes):
            import torch
            assert codes.dtype == torch.uint8 and offsets.dtype == torch.int64
            assert codes.is_cuda == offsets.is_cuda
            codes, offsets = codes.contiguous(), offsets.contiguous()
            s = _Seqs(codes.data_ptr() if codes.numel() else None, offsets.data_ptr(),
                      offsets.numel() - 1, 1 if codes.is_cuda else 0)
            return s, (codes, offsets), bool(codes.is_cuda)
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        s = _Seqs(codes.ctypes.data if codes.size else None, offsets.ctypes.data,
                  len(offsets) - 1, 0)
        return s, (codes, offsets), False

    def _take(self, p: _Pairs, device_output: bool, stream) -> Pairs:
        n = p.n
        try:
            if device_output:
                import torch
                dev = torch.device("cuda", self.device)
                i = torch.empty(n, dtype=torch.int32, device=dev)
                j = torch.empty(n, dtype=torch.int32, device=dev)
                d = torch.empty(n, dtype=torch.uint8, device=dev)
                if n:
                    self._check(self._lib.sd_pairs_copy(self._h, ctypes.byref(p), i.data_ptr(),
                                                        j.data_ptr(), d.data_ptr(), 1, stream),
                                "sd_pairs_copy")
                return Pairs(i, j, d)
            i = np.empty(n, dtype=np.uint32)
            j = np.empty(n, dtype=np.uint32)
            d = np.empty(n, dtype=np.uint8)
            if n:
                self._check(self._lib.sd_pairs_copy(self._h, ctypes.byref(p), i.ctypes.data,
                                                    j.ctypes.data, d.ctypes.data, 0, stream),
                            "sd_pairs_copy")
            return Pairs(i, j, d)
        finally:
            self._lib.sd_pairs_free(self._h, ctypes.byref(p))

    # ------------------------------------------------------------ searches
    def self_search(self, codes, offsets, k: int, device_output: bool | None = None,
                    stream=None) -> Pairs:
        """All i < j with Levenshtein(S_i, S_j) <= k, sorted by (i, j)."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        if device_output is None:
            device_output = on_dev
        p = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        rc = self._lib.sd_self_search(self._h, ctypes.byref(s), int(k), ctypes.byref(p), st)
        self._check(rc, "sd_self_search")
        return self._take(p, device_output, st)

    def self_search_raw(self, s: _Seqs, k: int, stream) -> _Pairs:
        """Device-resident result left in library memory (free with free_pairs)."""
        p = _Pairs(0, None, None, None, 1, 0)
        self._check(self._lib.sd_self_search(self._h, ctypes.byref(s), int(k), ctypes.byref(p),
                                             stream), "sd_self_search")
        return p

    def free_pairs(self, p: _Pairs):
        self._lib.sd_pairs_free(self._h, ctypes.byref(p))

    def pair_distance(self, a, b, ia, ib):
        """Levenshtein distance of pairs (ia[t], ib[t]); ia, ib are int32 cuda tensors."""
        import torch
        sa, ka, _ = self._seqs(*a)
        sb, kb, _ = self._seqs(*b)
        ia = ia.contiguous()
        ib = ib.contiguous()
        n = ia.numel()
        d = torch.empty(n, dtype=torch.uint8, device=ia.device)
        st = _stream_handle(None, True)
        self._check(self._lib.sd_pair_distance(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                               ia.data_ptr() if n else None,
                                               ib.data_ptr() if n else None, n,
                                               d.data_ptr() if n else None, st),
                    "sd_pair_distance")
        return d

    def stats(self) -> dict:
        st = _Stats()
        self._check(self._lib.sd_get_stats(self._h, ctypes.byref(st)), "sd_get_stats")
        stages = []
        for x in range(st.n_stages):
            stages.append(dict(name=bytes(st.stage_name[x]).split(b"\0")[0].decode(),
                               ms=st.stage_ms[x], bytes=st.stage_bytes[x],
                               launches=st.stage_launches[x]))
        return dict(n_seqs=st.n_seqs, n_keys=st.n_keys, n_cand_raw=st.n_cand_raw,
                    n_cand_unique=st.n_cand_unique, n_pairs=st.n_pairs,
                    n_sort_passes=st.n_sort_passes, n_big_segments=st.n_big_segments,
                    stages=stages)
