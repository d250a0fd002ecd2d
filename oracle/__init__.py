"""CPU ORACLE for symmetric-deletion neighbour search -- TEST INFRASTRUCTURE.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package. The product path (the HIP library and
its Python binding) never imports, links or calls it, and the two share no
code: the oracle works on plain byte strings with ``std::string`` deletion
variants, a ``std::unordered_map`` multi-value hash map and the full
Wagner-Fischer table (paper, Section II A; SymDel step list of Appendix A;
Fig. 1).

Functions return ``(a, b, d)`` numpy arrays sorted by ``(a, b)``:
  * ``self_search(codes, offsets, k)``: all i < j with Lev <= k.
  * ``self_search_sharded(codes, offsets, k, shards, threads)``: the same
    result on several threads with bounded memory (variant space split into
    shards by a hash of the variant string).
  * ``query_search(ref, qry, k)``: all (q, r) with Lev(Q_q, R_r) <= k.
  * ``paired_self_search(a, b, k)``: paired-chain records (Discussion: both
    chains joined by a non-deletable token); distance Lev(a) + Lev(b).
  * ``self_search_hamming`` / ``query_search_hamming``: Hamming mode
    (Section III C): the same candidates, kept when the lengths are equal and
    at most k positions differ.
  * ``query_weighted(ref, qry, subst, indel, max_score)``: SymDel candidates
    at Levenshtein radius 2, kept when the weighted alignment cost is
    <= max_score (Section III D: a Levenshtein prefilter, then a finer
    substitution-weighted score).
  * ``brute_*``: the definitions written out over every pair, for pinning.
Every function here is pinned by ``tests/test_oracle_pins.py``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "symdel_oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None


def build() -> str:
    """Compile the oracle with g++ (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["g++", "-O2", "-std=c++17", "-pthread", "-fPIC", "-shared", "-o", tmp, _SRC])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P, I, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64
    lib.or_lev.restype = I
    lib.or_lev.argtypes = [P, I, P, I]
    lib.or_weighted.restype = I
    lib.or_weighted.argtypes = [P, I, P, I, P, I]
    lib.or_lev_one_to_many.argtypes = [P, I, P, P, I64, P]
    lib.or_variants.restype = I64
    lib.or_variants.argtypes = [P, I, I, P, P, I64]
    lib.or_hamming.restype = I
    lib.or_hamming.argtypes = [P, I, P, I]
    for name in ("or_self_search", "or_self_candidates", "or_brute_self", "or_self_search_hamming",
                 "or_brute_self_hamming"):
        getattr(lib, name).restype = P
        getattr(lib, name).argtypes = [P, P, I64, I]
    lib.or_self_search_sharded.restype = P
    lib.or_self_search_sharded.argtypes = [P, P, I64, I, I, I]
    for name in ("or_query_search", "or_brute_query", "or_query_search_hamming",
                 "or_brute_query_hamming"):
        getattr(lib, name).restype = P
        getattr(lib, name).argtypes = [P, P, I64, P, P, I64, I]
    for name in ("or_paired_self_search", "or_brute_paired"):
        getattr(lib, name).restype = P
        getattr(lib, name).argtypes = [P, P, P, P, I64, I]
    lib.or_paired_variant_count.restype = I64
    lib.or_paired_variant_count.argtypes = [P, I, P, I, I]
    lib.or_query_weighted.restype = P
    lib.or_query_weighted.argtypes = [P, P, I64, P, P, I64, I, P, I, I]
    lib.or_brute_weighted.restype = P
    lib.or_brute_weighted.argtypes = [P, P, I64, P, P, I64, P, I, I]
    lib.or_size.restype = I64
    lib.or_size.argtypes = [P]
    lib.or_raw.restype = I64
    lib.or_raw.argtypes = [P]
    lib.or_copy.argtypes = [P, P, P, P]
    lib.or_free.argtypes = [P]
    _lib = lib
    return lib


def _u8(x) -> np.ndarray:
    if isinstance(x, (bytes, bytearray)):
        return np.frombuffer(bytes(x), dtype=np.uint8).copy()
    return np.ascontiguousarray(x, dtype=np.uint8)


def _i64(x) -> np.ndarray:
    return np.ascontiguousarray(x, dtype=np.int64)


def _take(h, with_raw=False):
    lib = _load()
    n = lib.or_size(h)
    a = np.empty(n, dtype=np.uint32)
    b = np.empty(n, dtype=np.uint32)
    d = np.empty(n, dtype=np.int32)
    if n:
        lib.or_copy(h, a.ctypes.data, b.ctypes.data, d.ctypes.data)
    raw = lib.or_raw(h)
    lib.or_free(h)
    return (a, b, d, raw) if with_raw else (a, b, d)


def lev(a, b) -> int:
    """Wagner-Fischer edit distance of two code sequences (bytes or arrays)."""
    a, b = _u8(a), _u8(b)
    return _load().or_lev(a.ctypes.data, len(a), b.ctypes.data, len(b))


def hamming(a, b) -> int:
    """Mismatching positions of two equal-length code sequences; -1 if the lengths differ."""
    a, b = _u8(a), _u8(b)
    return _load().or_hamming(a.ctypes.data, len(a), b.ctypes.data, len(b))


def weighted(a, b, subst: np.ndarray, indel: int) -> int:
    a, b = _u8(a), _u8(b)
    s = _u8(np.asarray(subst).reshape(-1))
    return _load().or_weighted(a.ctypes.data, len(a), b.ctypes.data, len(b), s.ctypes.data, indel)


def lev_one_to_many(a, codes, offsets) -> np.ndarray:
    a, codes, offsets = _u8(a), _u8(codes), _i64(offsets)
    out = np.empty(len(offsets) - 1, dtype=np.int32)
    _load().or_lev_one_to_many(a.ctypes.data, len(a), codes.ctypes.data, offsets.ctypes.data,
                               len(offsets) - 1, out.ctypes.data)
    return out


def variants(s, k: int) -> list[bytes]:
    """All deletion variants (with multiplicity) of one sequence, in enumeration order."""
    s = _u8(s)
    cap = 1 << 16
    out = np.zeros(cap * 32, dtype=np.uint8)
    lens = np.zeros(cap, dtype=np.int32)
    n = _load().or_variants(s.ctypes.data, len(s), k, out.ctypes.data, lens.ctypes.data, cap)
    assert n <= cap
    return [out[v * 32: v * 32 + lens[v]].tobytes() for v in range(n)]


def self_search(codes, offsets, k: int):
    codes, offsets = _u8(codes), _i64(offsets)
    h = _load().or_self_search(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1, k)
    return _take(h)


def host_threads() -> int:
    """Host threads the sharded oracle uses by default: OMP_NUM_THREADS if set
    (the share of the host a job is given), else every hardware thread."""
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit() and int(env) > 0:
        return int(env)
    return os.cpu_count() or 1


def self_search_sharded(codes, offsets, k: int, shards: int = 0, threads: int = 0):
    """self_search on several threads with bounded memory: the variant space is
    split into `shards` parts by a hash of the variant string (0: one per
    thread); at most min(threads, shards) threads run (0: host_threads()).
    Returns the same triplets as self_search."""
    codes, offsets = _u8(codes), _i64(offsets)
    threads = threads or host_threads()
    h = _load().or_self_search_sharded(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1,
                                       k, int(shards), int(threads))
    return _take(h)


def self_candidates(codes, offsets, k: int):
    """Unique candidate pairs before verification, plus the count with multiplicity."""
    codes, offsets = _u8(codes), _i64(offsets)
    h = _load().or_self_candidates(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1, k)
    a, b, _, raw = _take(h, with_raw=True)
    return a, b, raw


def self_search_hamming(codes, offsets, k: int):
    """Hamming mode (Section III C): SymDel candidates kept when the lengths are
    equal and at most k positions differ."""
    codes, offsets = _u8(codes), _i64(offsets)
    h = _load().or_self_search_hamming(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1, k)
    return _take(h)


def brute_self_hamming(codes, offsets, k: int):
    codes, offsets = _u8(codes), _i64(offsets)
    h = _load().or_brute_self_hamming(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1, k)
    return _take(h)


def query_search_hamming(ref, qry, k: int):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    h = _load().or_query_search_hamming(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                                        qo.ctypes.data, len(qo) - 1, k)
    return _take(h)


def brute_query_hamming(ref, qry, k: int):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    h = _load().or_brute_query_hamming(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                                       qo.ctypes.data, len(qo) - 1, k)
    return _take(h)


def paired_self_search(a, b, k: int):
    """Paired-chain mode (Discussion): records (a_i, b_i) from two CSR sets
    with the same count; variants keep a joining token and delete at most k
    positions in total; kept when Lev(a_i, a_j) + Lev(b_i, b_j) <= k."""
    (ac, ao), (bc, bo) = (_u8(a[0]), _i64(a[1])), (_u8(b[0]), _i64(b[1]))
    assert len(ao) == len(bo)
    h = _load().or_paired_self_search(ac.ctypes.data, ao.ctypes.data, bc.ctypes.data,
                                      bo.ctypes.data, len(ao) - 1, k)
    return _take(h)


def brute_paired(a, b, k: int):
    (ac, ao), (bc, bo) = (_u8(a[0]), _i64(a[1])), (_u8(b[0]), _i64(b[1]))
    assert len(ao) == len(bo)
    h = _load().or_brute_paired(ac.ctypes.data, ao.ctypes.data, bc.ctypes.data, bo.ctypes.data,
                                len(ao) - 1, k)
    return _take(h)


def paired_variant_count(a, b, k: int) -> int:
    a, b = _u8(a), _u8(b)
    return _load().or_paired_variant_count(a.ctypes.data, len(a), b.ctypes.data, len(b), k)


def brute_self(codes, offsets, k: int):
    codes, offsets = _u8(codes), _i64(offsets)
    h = _load().or_brute_self(codes.ctypes.data, offsets.ctypes.data, len(offsets) - 1, k)
    return _take(h)


def query_search(ref, qry, k: int):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    h = _load().or_query_search(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                                qo.ctypes.data, len(qo) - 1, k)
    return _take(h)


def brute_query(ref, qry, k: int):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    h = _load().or_brute_query(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                               qo.ctypes.data, len(qo) - 1, k)
    return _take(h)


def query_weighted(ref, qry, subst, indel: int, max_score: int, k: int = 2):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    s = _u8(np.asarray(subst).reshape(-1))
    h = _load().or_query_weighted(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                                  qo.ctypes.data, len(qo) - 1, k, s.ctypes.data, indel, max_score)
    return _take(h)


def brute_weighted(ref, qry, subst, indel: int, max_score: int):
    (rc, ro), (qc, qo) = (_u8(ref[0]), _i64(ref[1])), (_u8(qry[0]), _i64(qry[1]))
    s = _u8(np.asarray(subst).reshape(-1))
    h = _load().or_brute_weighted(rc.ctypes.data, ro.ctypes.data, len(ro) - 1, qc.ctypes.data,
                                  qo.ctypes.data, len(qo) - 1, s.ctypes.data, indel, max_score)
    return _take(h)
