"""Seeded synthetic CDR3-like inputs (test and benchmark data only).

The generator stands in for the TCR-beta CDR3 data set the paper measures on
(Section III A: valid sequences, de-duplicated, lengths up to 18); that data
set is not available here. Its recipe is stated in ``cdr3gen.c``. Nothing in
this module computes any part of the search method; the CPU oracle and the
GPU library both read its output.

Sequences are returned as ``(codes, offsets)``: a uint8 array of residue codes
0..19 in the order ``ACDEFGHIKLMNPQRSTVWY`` and an int64 CSR offset array of
length n + 1.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

ALPHABET = "ACDEFGHIKLMNPQRSTVWY"
_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cdr3gen.c")
_LIB = os.path.join(_HERE, "libcdr3gen.so")
_lib = None

# Named workloads: (seed, n, fresh fraction). A 40 % cluster fraction means
# 60 % fresh sequences.
PLAIN_CONFIGS = {
    "plain_10k": (1, 10_000, 0.7),
    "plain_1m": (2, 1_000_000, 0.7),
    "plain_10m": (3, 10_000_000, 0.6),
}
BATCHED = dict(ref_seed=4, ref_n=2_000_000, sets=512, size_seed=5, size_lo=1_000,
               size_hi=200_000, set_seed_base=1000, ref_mut_frac=0.1)
SERVED = dict(ref_seed=6, ref_n=5_000_000, arrival_seed=7, size_lo=100, size_hi=50_000,
              cost_seed=8, cost_lo=3, cost_hi=4, indel=8, max_score=8)


def build() -> str:
    """Compile the generator with gcc (always rebuilds)."""
    tmp = _LIB + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fPIC", "-shared", "-std=c11", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    P = ctypes.c_void_p
    lib.cdr3_generate.restype = ctypes.c_int64
    lib.cdr3_generate.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, P, P]
    lib.cdr3_generate_query.restype = ctypes.c_int64
    lib.cdr3_generate_query.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                        ctypes.c_double, P, P, ctypes.c_int64, P, P]
    lib.cdr3_loguniform_sizes.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double,
                                          ctypes.c_double, P]
    lib.cdr3_poisson_arrivals.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, P]
    lib.cdr3_cost_matrix.argtypes = [ctypes.c_uint64, ctypes.c_int, ctypes.c_int, P]
    lib.cdr3_residue_probs.argtypes = [P]
    lib.cdr3_generate_paired.argtypes = [ctypes.c_uint64, ctypes.c_int64, ctypes.c_double, P, P,
                                         P, P]
    _lib = lib
    return lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


def paired(seed: int, n: int, fresh_frac: float = 0.7):
    """n paired-chain records: ((codes_a, offsets_a), (codes_b, offsets_b))."""
    lib = _load()
    ca = np.empty(max(24 * n, 1), dtype=np.uint8)
    cb = np.empty(max(24 * n, 1), dtype=np.uint8)
    oa = np.empty(n + 1, dtype=np.int64)
    ob = np.empty(n + 1, dtype=np.int64)
    lib.cdr3_generate_paired(seed, n, fresh_frac, _ptr(ca), _ptr(oa), _ptr(cb), _ptr(ob))
    return (ca[:oa[-1]].copy(), oa), (cb[:ob[-1]].copy(), ob)


def generate(seed: int, n: int, fresh_frac: float = 0.7):
    """n CDR3-like sequences from the seeded recipe."""
    lib = _load()
    codes = np.empty(max(24 * n, 1), dtype=np.uint8)
    offsets = np.empty(n + 1, dtype=np.int64)
    total = lib.cdr3_generate(seed, n, fresh_frac, _ptr(codes), _ptr(offsets))
    return codes[:total].copy(), offsets


def generate_query(seed: int, n: int, ref_codes: np.ndarray, ref_offsets: np.ndarray,
                   ref_mut_frac: float = 0.1, fresh_frac: float = 0.7):
    """A query set whose sequences are reference mutants with probability ref_mut_frac."""
    lib = _load()
    ref_codes = np.ascontiguousarray(ref_codes, dtype=np.uint8)
    ref_offsets = np.ascontiguousarray(ref_offsets, dtype=np.int64)
    codes = np.empty(max(24 * n, 1), dtype=np.uint8)
    offsets = np.empty(n + 1, dtype=np.int64)
    total = lib.cdr3_generate_query(seed, n, fresh_frac, ref_mut_frac, _ptr(ref_codes),
                                    _ptr(ref_offsets), len(ref_offsets) - 1, _ptr(codes),
                                    _ptr(offsets))
    return codes[:total].copy(), offsets


def plain(name: str):
    seed, n, fresh = PLAIN_CONFIGS[name]
    return generate(seed, n, fresh)


def loguniform_sizes(seed: int, count: int, lo: float, hi: float) -> np.ndarray:
    out = np.empty(count, dtype=np.int64)
    _load().cdr3_loguniform_sizes(seed, count, lo, hi, _ptr(out))
    return out


def batched_sets(ref, nsets: int = BATCHED["sets"], scale: float = 1.0):
    """The batched workload's query sets: log-uniform sizes in [1e3, 2e5]
    (seeded, times `scale`), each with 10% mutants of the reference."""
    p = BATCHED
    sizes = loguniform_sizes(p["size_seed"], nsets, p["size_lo"], p["size_hi"])
    sizes = np.maximum(1, (sizes * scale).astype(np.int64))
    return [generate_query(p["set_seed_base"] + q, int(n), *ref, ref_mut_frac=p["ref_mut_frac"])
            for q, n in enumerate(sizes)]


def poisson_arrivals(seed: int, count: int, rate: float) -> np.ndarray:
    out = np.empty(count, dtype=np.float64)
    _load().cdr3_poisson_arrivals(seed, count, rate, _ptr(out))
    return out


def cost_matrix(seed: int = SERVED["cost_seed"], lo: int = 3, hi: int = 4) -> np.ndarray:
    out = np.empty(400, dtype=np.uint8)
    _load().cdr3_cost_matrix(seed, lo, hi, _ptr(out))
    return out.reshape(20, 20)


def residue_probs() -> np.ndarray:
    out = np.empty(20, dtype=np.float64)
    _load().cdr3_residue_probs(_ptr(out))
    return out


def subset(codes: np.ndarray, offsets: np.ndarray, n: int):
    """The first n sequences of a CSR set."""
    end = int(offsets[n])
    return codes[:end].copy(), offsets[: n + 1].copy()


def to_strings(codes: np.ndarray, offsets: np.ndarray) -> list[str]:
    b = codes.tobytes()
    table = bytes.maketrans(bytes(range(20)), ALPHABET.encode())
    s = b.translate(table).decode()
    return [s[offsets[i]:offsets[i + 1]] for i in range(len(offsets) - 1)]


def from_strings(seqs: list[str]):
    """CSR codes for strings over ALPHABET (raises on any other letter)."""
    idx = {c: i for i, c in enumerate(ALPHABET)}
    offsets = np.zeros(len(seqs) + 1, dtype=np.int64)
    buf = bytearray()
    for i, s in enumerate(seqs):
        buf.extend(idx[c] for c in s)
        offsets[i + 1] = len(buf)
    return np.frombuffer(bytes(buf), dtype=np.uint8).copy(), offsets
