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
SD_E_INVAL, SD_E_ALPHABET, SD_E_LENGTH, SD_E_TOO_MANY = -1, -2, -3, -4
SD_E_NOMEM, SD_E_HIP, SD_E_CANCELLED, SD_E_STATE = -5, -6, -7, -8
NOALLOC_MAX_SEQS = 16384
OPT_TIMING = 1
OPT_PATH = 2
OPT_GROUP_CAP = 3
OPT_GROUP_BITS = 4
OPT_SORT_ITEMS = 5
OPT_BATCH_TILE = 6
OPT_PROBE = 7
OPT_GROUP_BATCHES = 8
OPT_PAIR_SORT = 9
OPT_METRIC = 10
OPT_STREAM = 11
OPT_STREAM_ELEMS = 12
OPT_GROUP_SHAPE = 13
OPT_BATCH_GRAPH = 14
OPT_JOIN_ELEMS = 15
METRIC_LEVENSHTEIN = 0
METRIC_HAMMING = 1
MAX_STAGES = 16
MLP_HIDDEN = 32
MLP_PARAMS = 3 * MLP_HIDDEN + 1


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
                ("n_probe_steps", ctypes.c_int64), ("n_stream_groups", ctypes.c_int64),
                ("n_graph_captures", ctypes.c_int64), ("n_graph_launches", ctypes.c_int64),
                ("n_graph_retries", ctypes.c_int64),
                ("n_pair_buckets", ctypes.c_int64), ("n_pair_fallbacks", ctypes.c_int64),
                ("stage_name", (ctypes.c_char * 24) * MAX_STAGES),
                ("stage_ms", ctypes.c_double * MAX_STAGES),
                ("stage_bytes", ctypes.c_double * MAX_STAGES),
                ("stage_launches", ctypes.c_int32 * MAX_STAGES)]


class _LearnedConfig(ctypes.Structure):
    _fields_ = [("leaves_log2", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("lr", ctypes.c_float), ("samples", ctypes.c_uint32),
                ("use_init", ctypes.c_int32), ("init", ctypes.c_float * MLP_PARAMS)]


class _LearnedInfo(ctypes.Structure):
    _fields_ = [("leaves", ctypes.c_int32), ("steps", ctypes.c_int32),
                ("max_eps", ctypes.c_uint32), ("empty_leaves", ctypes.c_uint32),
                ("mean_eps", ctypes.c_double), ("mean_window_log2", ctypes.c_double),
                ("loss_first", ctypes.c_float), ("loss_last", ctypes.c_float),
                ("train_ms", ctypes.c_double), ("fit_ms", ctypes.c_double),
                ("params", ctypes.c_float * MLP_PARAMS)]


class _TuneResult(ctypes.Structure):
    _fields_ = [("trials", ctypes.c_int32), ("path", ctypes.c_int32),
                ("group_cap", ctypes.c_int32), ("sort_items", ctypes.c_int32),
                ("batch_tile", ctypes.c_int64), ("best_s", ctypes.c_double),
                ("default_s", ctypes.c_double), ("group_bits", ctypes.c_int32),
                ("pair_sort", ctypes.c_int32), ("group_shape", ctypes.c_int32),
                ("batch_graph", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


# allocator hook signatures (sd_alloc_fn, sd_free_fn)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p)

_lib = None


def load_library(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libsymdel.so (raises OSError if it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise OSError(f"{path} is not built; run __graft_entry__.build() first")
    # torch ships its own HIP runtime under the same soname; importing it first
    # makes the library bind to that runtime, so torch streams and device
    # pointers are valid in both and torch still initialises afterwards.
    import torch  # noqa: F401
    lib = ctypes.CDLL(path)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.sd_create.argtypes = [ctypes.POINTER(P), I, ctypes.c_uint64]
    lib.sd_create.restype = I
    lib.sd_destroy.argtypes = [P]
    lib.sd_destroy.restype = None
    lib.sd_set_option.argtypes = [P, I, I64]
    lib.sd_set_option.restype = I
    lib.sd_set_allocator.argtypes = [P, ALLOC_FN, FREE_FN, P]
    lib.sd_set_allocator.restype = I
    lib.sd_self_search.argtypes = [P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_self_search.restype = I
    lib.sd_self_search_hamming.argtypes = [P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_self_search_hamming.restype = I
    lib.sd_paired_self_search.argtypes = [P, ctypes.POINTER(_Seqs), ctypes.POINTER(_Seqs), I,
                                          ctypes.POINTER(_Pairs), P]
    lib.sd_paired_self_search.restype = I
    lib.sd_self_search_noalloc.argtypes = [P, ctypes.POINTER(_Seqs), I, P, P, P, I64,
                                           ctypes.POINTER(I64), P]
    lib.sd_self_search_noalloc.restype = I
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
    lib.sd_index_build.argtypes = [P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(P), P]
    lib.sd_index_build.restype = I
    lib.sd_index_free.argtypes = [P]
    lib.sd_index_free.restype = None
    lib.sd_index_info.argtypes = [P, P, P, P, P]
    lib.sd_index_info.restype = I
    lib.sd_query.argtypes = [P, P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_query.restype = I
    lib.sd_query_hamming.argtypes = [P, P, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_query_hamming.restype = I
    lib.sd_query_batch.argtypes = [P, P, I, ctypes.POINTER(_Seqs), I, ctypes.POINTER(_Pairs), P]
    lib.sd_query_batch.restype = I
    lib.sd_query_weighted.argtypes = [P, P, ctypes.POINTER(_Seqs), P, I, I,
                                      ctypes.POINTER(_Pairs), P]
    lib.sd_query_weighted.restype = I
    lib.sd_index_build_learned.argtypes = [P, ctypes.POINTER(_Seqs), I,
                                           ctypes.POINTER(_LearnedConfig), ctypes.POINTER(P), P]
    lib.sd_index_build_learned.restype = I
    lib.sd_index_learned_info.argtypes = [P, ctypes.POINTER(_LearnedInfo), P, ctypes.c_int32]
    lib.sd_index_learned_info.restype = I
    lib.sd_mlp_gradients.argtypes = [P, P, P, P, ctypes.c_uint32, P, P, P]
    lib.sd_mlp_gradients.restype = I
    lib.sd_autotune.argtypes = [P, P, I, ctypes.POINTER(_Seqs), I, I,
                                ctypes.POINTER(_TuneResult), P]
    lib.sd_autotune.restype = I
    lib.sd_autotune_cache.argtypes = [P, ctypes.c_char_p]
    lib.sd_autotune_cache.restype = I
    _lib = lib
    return lib


class Index:
    """A device-resident reference deletion index (see sd_index_build)."""

    def __init__(self, lib, handle: ctypes.c_void_p):
        self._lib = lib
        self._h = handle

    @property
    def handle(self):
        return self._h

    def info(self) -> dict:
        n_ref, n_keys, nbytes = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        k = ctypes.c_int32()
        self._lib.sd_index_info(self._h, ctypes.byref(n_ref), ctypes.byref(n_keys),
                                ctypes.byref(k), ctypes.byref(nbytes))
        return dict(n_ref=n_ref.value, n_keys=n_keys.value, k=k.value, bytes=nbytes.value)

    def learned_info(self) -> dict:
        """Model of a learned index (sd_index_learned_info), with the loss curve."""
        inf = _LearnedInfo()
        rc = self._lib.sd_index_learned_info(self._h, ctypes.byref(inf), None, 0)
        if rc != SD_OK:
            raise SymdelError(rc, "sd_index_learned_info: not a learned index")
        curve = np.zeros(max(inf.steps, 0), dtype=np.float32)
        if inf.steps:
            self._lib.sd_index_learned_info(self._h, ctypes.byref(inf), curve.ctypes.data,
                                            inf.steps)
        out = {f: getattr(inf, f) for f, _ in _LearnedInfo._fields_ if f != "params"}
        out["params"] = np.ctypeslib.as_array(inf.params).copy()
        out["loss_curve"] = curve
        return out

    def free(self):
        if self._h:
            self._lib.sd_index_free(self._h)
            self._h = ctypes.c_void_p()

    def __del__(self):
        try:
            self.free()
        except Exception:
            pass


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

    def set_allocator(self, alloc, free):
        """Device memory from Python callables (sd_set_allocator): alloc(nbytes)
        returns a device address (0 or None when it cannot), free(address)
        gives it back. Both None: the library's own pool again."""
        if alloc is None and free is None:
            cb = (ALLOC_FN(), FREE_FN())
        else:
            def _alloc(nbytes, _user):
                try:
                    return alloc(int(nbytes)) or None
                except Exception:  # noqa: BLE001 - a failed allocation is reported as NULL
                    return None

            def _free(ptr, _user):
                free(int(ptr))
            cb = (ALLOC_FN(_alloc), FREE_FN(_free))
        self._check(self._lib.sd_set_allocator(self._h, cb[0], cb[1], None), "sd_set_allocator")
        # the library calls these until the hook is replaced; indexes built
        # with them keep calling free until they are released
        self._alloc_cb = cb
        self._alloc_cbs = getattr(self, "_alloc_cbs", []) + [cb]

    def use_torch_allocator(self, stream=None):
        """Take every device allocation of this context from PyTorch's caching
        allocator, on `stream` (default: the current stream of the device)."""
        import torch
        dev = self.device
        st = stream if stream is not None else torch.cuda.current_stream(dev)
        self.set_allocator(lambda n: torch.cuda.caching_allocator_alloc(n, dev, st),
                           torch.cuda.caching_allocator_delete)

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
                    stream=None, hamming: bool = False) -> Pairs:
        """All i < j with Levenshtein(S_i, S_j) <= k, sorted by (i, j); with
        hamming, equal-length pairs with Hamming distance <= k instead."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        if device_output is None:
            device_output = on_dev
        p = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        fn = self._lib.sd_self_search_hamming if hamming else self._lib.sd_self_search
        rc = fn(self._h, ctypes.byref(s), int(k), ctypes.byref(p), st)
        self._check(rc, "sd_self_search_hamming" if hamming else "sd_self_search")
        return self._take(p, device_output, st)

    def paired_self_search(self, a, b, k: int, device_output: bool | None = None,
                           stream=None) -> Pairs:
        """Paired-chain records (a[i], b[i]), each a (codes, offsets) pair: all
        i < j with Lev(a_i, a_j) + Lev(b_i, b_j) <= k (sd_paired_self_search)."""
        sa, keep_a, on_dev = self._seqs(*a)
        sb, keep_b, on_dev_b = self._seqs(*b)
        st = _stream_handle(stream, on_dev or on_dev_b)
        if device_output is None:
            device_output = on_dev
        p = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        self._check(self._lib.sd_paired_self_search(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                                    int(k), ctypes.byref(p), st),
                    "sd_paired_self_search")
        return self._take(p, device_output, st)

    def paired_self_search_raw(self, sa: _Seqs, sb: _Seqs, k: int, stream) -> _Pairs:
        """Paired-chain search with the device result left in library memory."""
        p = _Pairs(0, None, None, None, 1, 0)
        self._check(self._lib.sd_paired_self_search(self._h, ctypes.byref(sa), ctypes.byref(sb),
                                                    int(k), ctypes.byref(p), stream),
                    "sd_paired_self_search")
        return p

    def self_search_raw(self, s: _Seqs, k: int, stream) -> _Pairs:
        """Device-resident result left in library memory (free with free_pairs)."""
        p = _Pairs(0, None, None, None, 1, 0)
        self._check(self._lib.sd_self_search(self._h, ctypes.byref(s), int(k), ctypes.byref(p),
                                             stream), "sd_self_search")
        return p

    def self_search_noalloc(self, codes, offsets, k: int, out_i, out_j, out_d,
                            stream=None) -> int:
        """sd_self_search_noalloc: the self search into caller-owned device
        tensors (int32 i, int32 j, uint8 d of equal length = the capacity),
        with no allocation by the library; returns the number of pairs."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, True)
        cap = int(out_i.numel())
        assert out_j.numel() == cap and out_d.numel() == cap
        n = ctypes.c_int64(0)
        rc = self._lib.sd_self_search_noalloc(
            self._h, ctypes.byref(s), int(k), out_i.data_ptr() if cap else None,
            out_j.data_ptr() if cap else None, out_d.data_ptr() if cap else None, cap,
            ctypes.byref(n), st)
        if rc != SD_OK:
            err = SymdelError(rc, "sd_self_search_noalloc: " + (
                self._lib.sd_last_error(self._h).decode() or self._lib.sd_strerror(rc).decode()))
            err.needed = int(n.value)
            raise err
        return int(n.value)

    def free_pairs(self, p: _Pairs):
        self._lib.sd_pairs_free(self._h, ctypes.byref(p))

    # ------------------------------------------------------------ queries
    def build_index(self, codes, offsets, k: int, stream=None) -> Index:
        """Reference deletion index of a sequence set (sd_index_build)."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        h = ctypes.c_void_p()
        self._check(self._lib.sd_index_build(self._h, ctypes.byref(s), int(k), ctypes.byref(h), st),
                    "sd_index_build")
        return Index(self._lib, h)

    def build_learned_index(self, codes, offsets, k: int, leaves_log2: int = 0, steps: int = -1,
                            lr: float = 0.0, samples: int = 0, init=None, stream=None) -> Index:
        """Learned reference index (sd_index_build_learned); steps=-1 takes the default."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        cfg = _LearnedConfig()
        cfg.leaves_log2, cfg.steps, cfg.lr, cfg.samples = leaves_log2, steps, lr, samples
        if init is not None:
            cfg.use_init = 1
            v = np.ascontiguousarray(np.asarray(init, dtype=np.float32).reshape(MLP_PARAMS))
            ctypes.memmove(cfg.init, v.ctypes.data, MLP_PARAMS * 4)
        h = ctypes.c_void_p()
        self._check(self._lib.sd_index_build_learned(self._h, ctypes.byref(s), int(k),
                                                     ctypes.byref(cfg), ctypes.byref(h), st),
                    "sd_index_build_learned")
        return Index(self._lib, h)

    def autotune(self, sets, k: int, index: Index | None = None, reps: int = 2,
                 stream=None) -> dict:
        """Tune the context's options on sample set(s) (sd_autotune); returns the choice."""
        n = len(sets)
        arr = (_Seqs * max(n, 1))()
        keep = []
        on_dev = False
        for x, (codes, offsets) in enumerate(sets):
            s, kp, od = self._seqs(codes, offsets)
            arr[x] = s
            keep.append(kp)
            on_dev = on_dev or od
        st = _stream_handle(stream, on_dev)
        res = _TuneResult()
        self._check(self._lib.sd_autotune(self._h, index.handle if index is not None else None, n,
                                          arr, int(k), int(reps), ctypes.byref(res), st),
                    "sd_autotune")
        return {f: getattr(res, f) for f, _ in _TuneResult._fields_ if f != "reserved"}

    def set_tune_cache(self, path: str | None):
        """Use the JSON file at `path` as the autotuner's cache (None: no cache)."""
        self._check(self._lib.sd_autotune_cache(
            self._h, None if path is None else os.fsencode(path)), "sd_autotune_cache")

    def mlp_gradients(self, params, x, y):
        """(grad, loss) of the stage-1 training loss from the device kernels."""
        p = np.ascontiguousarray(np.asarray(params, dtype=np.float32).reshape(MLP_PARAMS))
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.ascontiguousarray(y, dtype=np.float32)
        assert x.shape == y.shape and x.ndim == 1
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        loss = ctypes.c_float()
        self._check(self._lib.sd_mlp_gradients(self._h, p.ctypes.data, x.ctypes.data,
                                               y.ctypes.data, len(x), g.ctypes.data,
                                               ctypes.byref(loss), None), "sd_mlp_gradients")
        return g, float(loss.value)

    def query(self, index: Index, codes, offsets, k: int, device_output: bool | None = None,
              stream=None, hamming: bool = False) -> Pairs:
        """All (q, r) with Levenshtein(Q_q, R_r) <= k, sorted by (q, r); with
        hamming, equal-length pairs with Hamming distance <= k instead."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        if device_output is None:
            device_output = on_dev
        p = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        fn = self._lib.sd_query_hamming if hamming else self._lib.sd_query
        self._check(fn(self._h, index.handle, ctypes.byref(s), int(k), ctypes.byref(p), st),
                    "sd_query_hamming" if hamming else "sd_query")
        return self._take(p, device_output, st)

    def query_batch(self, index: Index, sets, k: int, device_output: bool | None = None,
                    stream=None) -> list:
        """Results of many query sets against one index (sd_query_batch)."""
        n = len(sets)
        arr = (_Seqs * max(n, 1))()
        keep = []
        on_dev = False
        for x, (codes, offsets) in enumerate(sets):
            s, kp, od = self._seqs(codes, offsets)
            arr[x] = s
            keep.append(kp)
            on_dev = on_dev or od
        st = _stream_handle(stream, on_dev)
        if device_output is None:
            device_output = on_dev
        outs = (_Pairs * max(n, 1))()
        for x in range(n):
            outs[x] = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        self._check(self._lib.sd_query_batch(self._h, index.handle, n, arr, int(k), outs, st),
                    "sd_query_batch")
        return [self._take(outs[x], device_output, st) for x in range(n)]

    def query_batch_raw(self, index: Index, arr, n: int, k: int, stream):
        """Device-resident per-set results left in library memory (free with free_pairs)."""
        outs = (_Pairs * max(n, 1))()
        for x in range(n):
            outs[x] = _Pairs(0, None, None, None, 1, 0)
        self._check(self._lib.sd_query_batch(self._h, index.handle, n, arr, int(k), outs, stream),
                    "sd_query_batch")
        return outs

    def query_weighted(self, index: Index, codes, offsets, subst, indel: int, max_score: int,
                       device_output: bool | None = None, stream=None) -> Pairs:
        """Weighted rescoring of the index's Levenshtein candidates (d = score)."""
        s, keep, on_dev = self._seqs(codes, offsets)
        st = _stream_handle(stream, on_dev)
        if device_output is None:
            device_output = on_dev
        sub = np.ascontiguousarray(np.asarray(subst, dtype=np.uint8).reshape(400))
        p = _Pairs(0, None, None, None, 1 if device_output else 0, 0)
        self._check(self._lib.sd_query_weighted(self._h, index.handle, ctypes.byref(s),
                                                sub.ctypes.data, int(indel), int(max_score),
                                                ctypes.byref(p), st), "sd_query_weighted")
        return self._take(p, device_output, st)

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
                    n_probe_steps=st.n_probe_steps, n_stream_groups=st.n_stream_groups,
                    n_graph_captures=st.n_graph_captures, n_graph_launches=st.n_graph_launches,
                    n_graph_retries=st.n_graph_retries,
                    n_pair_buckets=st.n_pair_buckets, n_pair_fallbacks=st.n_pair_fallbacks,
                    stages=stages)


class _ServerConfig(ctypes.Structure):
    _fields_ = [("k", ctypes.c_int32), ("workers", ctypes.c_int32),
                ("max_batch_requests", ctypes.c_int32), ("weighted", ctypes.c_int32),
                ("hbm_budget", ctypes.c_uint64), ("subst", ctypes.c_uint8 * 400),
                ("indel", ctypes.c_int32), ("max_score", ctypes.c_int32),
                ("probe", ctypes.c_int32)]


class Server:
    """Continuous-batching query server over one index (sd_server_*).

    Requests are host query sets; results are host numpy triplets equal to
    querying each set alone.
    """

    def __init__(self, index: Index, k: int, device: int = 0, workers: int = 2,
                 max_batch_requests: int = 0, hbm_budget: int = 0, subst=None, indel: int = 8,
                 max_score: int = 8, probe: int = 0):
        lib = load_library()
        self._lib = lib
        P, I = ctypes.c_void_p, ctypes.c_int
        lib.sd_server_create.argtypes = [P, I, ctypes.POINTER(_ServerConfig), ctypes.POINTER(P)]
        lib.sd_server_create.restype = I
        lib.sd_server_submit.argtypes = [P, ctypes.POINTER(_Seqs), ctypes.POINTER(ctypes.c_uint64)]
        lib.sd_server_submit.restype = I
        lib.sd_server_poll.argtypes = [P, ctypes.c_uint64, I, ctypes.POINTER(_Pairs),
                                       ctypes.POINTER(ctypes.c_double)]
        lib.sd_server_poll.restype = I
        lib.sd_server_cancel.argtypes = [P, ctypes.c_uint64]
        lib.sd_server_cancel.restype = I
        lib.sd_server_stats.argtypes = [P, P, P, P]
        lib.sd_server_stats.restype = I
        lib.sd_server_free_pairs.argtypes = [ctypes.POINTER(_Pairs)]
        lib.sd_server_free_pairs.restype = None
        lib.sd_server_destroy.argtypes = [P]
        lib.sd_server_destroy.restype = None
        cfg = _ServerConfig()
        cfg.k, cfg.workers, cfg.max_batch_requests = k, workers, max_batch_requests
        cfg.hbm_budget = hbm_budget
        cfg.weighted = 1 if subst is not None else 0
        if subst is not None:
            sub = np.ascontiguousarray(np.asarray(subst, dtype=np.uint8).reshape(400))
            ctypes.memmove(cfg.subst, sub.ctypes.data, 400)
        cfg.indel, cfg.max_score, cfg.probe = indel, max_score, probe
        self._index = index  # the index must outlive the server
        self._h = ctypes.c_void_p()
        rc = lib.sd_server_create(index.handle, device, ctypes.byref(cfg), ctypes.byref(self._h))
        if rc != SD_OK:
            raise SymdelError(rc, "sd_server_create failed")

    def submit(self, codes, offsets) -> int:
        codes = np.ascontiguousarray(codes, dtype=np.uint8)
        offsets = np.ascontiguousarray(offsets, dtype=np.int64)
        s = _Seqs(codes.ctypes.data if codes.size else None, offsets.ctypes.data,
                  len(offsets) - 1, 0)
        rid = ctypes.c_uint64()
        rc = self._lib.sd_server_submit(self._h, ctypes.byref(s), ctypes.byref(rid))
        if rc != SD_OK:
            raise SymdelError(rc, "sd_server_submit failed")
        return rid.value

    def poll(self, request_id: int, timeout_ms: int = -1):
        """(Pairs, latency seconds); raises SymdelError on failure or timeout."""
        p = _Pairs()
        lat = ctypes.c_double()
        rc = self._lib.sd_server_poll(self._h, request_id, timeout_ms, ctypes.byref(p),
                                      ctypes.byref(lat))
        if rc != SD_OK:
            raise SymdelError(rc, f"request {request_id}")
        n = p.n
        i = np.empty(n, dtype=np.uint32)
        j = np.empty(n, dtype=np.uint32)
        d = np.empty(n, dtype=np.uint8)
        if n:
            ctypes.memmove(i.ctypes.data, p.i, n * 4)
            ctypes.memmove(j.ctypes.data, p.j, n * 4)
            ctypes.memmove(d.ctypes.data, p.d, n)
        self._lib.sd_server_free_pairs(ctypes.byref(p))
        return Pairs(i, j, d), lat.value

    def cancel(self, request_id: int) -> int:
        return self._lib.sd_server_cancel(self._h, request_id)

    def stats(self) -> dict:
        b, r, m = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int64()
        self._lib.sd_server_stats(self._h, ctypes.byref(b), ctypes.byref(r), ctypes.byref(m))
        return dict(batches=b.value, requests=r.value, max_batch=m.value)

    def close(self):
        if self._h:
            self._lib.sd_server_destroy(self._h)
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
