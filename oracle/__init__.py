"""CPU oracle for exact multi-pattern matching.

TEST INFRASTRUCTURE, NOT PRODUCT.  Only the test suite, the smoke check and
the benchmark's CPU-baseline leg may import this package.  It shares no code
with the GPU library (``paper_1702_03657_amd``) and never imports it.

Contents (each cites the passage it follows):

* ``brute``, ``bucketed``, ``aho_corasick`` (C, ``oracle.c``): the match set
  M(T) = {(i, j) : T[i .. i+|P_j|) == P_j} of the problem statement
  (Background, "Multi-Pattern Matching"), which the failure-less walk of
  Background, "Parallel Failure-Less Aho-Corasick" reaches exactly.
* ``counts``: per-position match counts, count[i] = |{j : (i, j) in M}|.
* ``canonical_trie``: the compressed-row-storage trie of Design and
  Implementation (steps I, II and VI plus the CRS step), defined directly:
  nodes are the distinct prefixes of the patterns (the empty one is the root)
  in breadth-first order with children by ascending unsigned label; the CRS
  vectors are row_ptr (one row per node), the column index (edge label) and
  the value (child node).
* ``footprint``: storage of the dense node x 256 transition table, of the
  36-byte bitmapped node of Results, and of the CRS form (2 nnz + n + 1
  elements, Design and Implementation).
"""

from __future__ import annotations

import ctypes
import os
import subprocess
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")

ORC_BRUTE, ORC_BUCKETED, ORC_AC = 1, 2, 3

_lib = None


def build(force: bool = False) -> str:
    """Compile ``oracle.c`` into ``liboracle.so`` next to it (gcc, -O2)."""
    if force or not os.path.exists(_LIB_PATH) or (
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC)):
        tmp = _LIB_PATH + f".tmp{os.getpid()}"
        subprocess.check_call(["gcc", "-O2", "-std=gnu11", "-shared", "-fPIC", "-pthread",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    u8p = ctypes.POINTER(ctypes.c_uint8)
    u64p = ctypes.POINTER(ctypes.c_uint64)
    u32p = ctypes.POINTER(ctypes.c_uint32)
    lib.orc_match.restype = ctypes.c_void_p
    lib.orc_match.argtypes = [ctypes.c_int, u8p, u64p, ctypes.c_uint32, u8p, u64p,
                              ctypes.c_uint32, ctypes.c_uint64, ctypes.c_uint64,
                              ctypes.c_int, ctypes.c_uint64,
                              ctypes.POINTER(ctypes.c_double)]
    lib.orc_count.restype = ctypes.c_uint64
    lib.orc_count.argtypes = [ctypes.c_void_p]
    lib.orc_copy.restype = None
    lib.orc_copy.argtypes = [ctypes.c_void_p, u64p, u32p, u32p]
    lib.orc_free.restype = None
    lib.orc_free.argtypes = [ctypes.c_void_p]
    lib.orc_exhaustive.restype = ctypes.c_int64
    lib.orc_exhaustive.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   ctypes.c_int, u64p]
    _lib = lib
    return lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def _patterns(patterns) -> Tuple[np.ndarray, np.ndarray]:
    """Accept a sequence of bytes or an object with ``data``/``offsets``."""
    if hasattr(patterns, "data") and hasattr(patterns, "offsets"):
        data = np.ascontiguousarray(patterns.data, dtype=np.uint8)
        offs = np.ascontiguousarray(patterns.offsets, dtype=np.uint64)
    else:
        pats = [bytes(p) for p in patterns]
        offs = np.zeros(len(pats) + 1, dtype=np.uint64)
        if pats:
            offs[1:] = np.cumsum([len(p) for p in pats])
        data = np.frombuffer(b"".join(pats), dtype=np.uint8).copy()
    if len(offs) > 1 and np.any(np.diff(offs) == 0):
        raise ValueError("empty pattern: the match set is defined for non-empty patterns")
    if data.size == 0:
        data = np.zeros(1, dtype=np.uint8)
    return data, offs


def _texts(text, offsets) -> Tuple[np.ndarray, np.ndarray]:
    if isinstance(text, (bytes, bytearray, memoryview)):
        t = np.frombuffer(bytes(text), dtype=np.uint8)
    else:
        t = np.ascontiguousarray(text, dtype=np.uint8).reshape(-1)
    if offsets is None:
        offs = np.array([0, t.size], dtype=np.uint64)
    else:
        offs = np.ascontiguousarray(offsets, dtype=np.uint64)
    if t.size == 0:
        t = np.zeros(1, dtype=np.uint8)
    return t, offs


class Matches(dict):
    """Result arrays: 'text' (uint32), 'pos' (uint64), 'id' (uint32), sorted by (text, pos, id)."""

    def __repr__(self):
        return f"Matches(n={self.n})"

    @property
    def n(self) -> int:
        return int(self["pos"].size)

    def pairs(self) -> List[Tuple[int, int]]:
        return list(zip(self["pos"].tolist(), self["id"].tolist()))

    def triples(self) -> List[Tuple[int, int, int]]:
        return list(zip(self["text"].tolist(), self["pos"].tolist(), self["id"].tolist()))


def match(algo: int, text, patterns, offsets=None, lo: int = 0,
          hi: Optional[int] = None, threads: int = 1, chunk: int = 0,
          timing: Optional[list] = None) -> Matches:
    """Match set of every text (start positions in [lo, hi) of each text)."""
    lib = _load()
    t, toff = _texts(text, offsets)
    pdata, poff = _patterns(patterns)
    n_texts = len(toff) - 1
    k = len(poff) - 1
    tm = (ctypes.c_double * 2)()
    h = lib.orc_match(algo, _ptr(t, ctypes.c_uint8), _ptr(toff, ctypes.c_uint64), n_texts,
                      _ptr(pdata, ctypes.c_uint8), _ptr(poff, ctypes.c_uint64), k,
                      lo, (2 ** 64 - 1) if hi is None else hi, int(threads), int(chunk), tm)
    if not h:
        raise MemoryError("oracle failed (out of memory or bad input)")
    try:
        n = lib.orc_count(h)
        pos = np.empty(n, dtype=np.uint64)
        ids = np.empty(n, dtype=np.uint32)
        tid = np.empty(n, dtype=np.uint32)
        if n:
            lib.orc_copy(h, _ptr(pos, ctypes.c_uint64), _ptr(ids, ctypes.c_uint32),
                         _ptr(tid, ctypes.c_uint32))
    finally:
        lib.orc_free(h)
    if timing is not None:
        timing[:] = [tm[0], tm[1]]
    return Matches(text=tid, pos=pos, id=ids)


def brute(text, patterns, offsets=None, **kw) -> Matches:
    """Literal definition: every pattern compared at every start position."""
    return match(ORC_BRUTE, text, patterns, offsets, **kw)


def bucketed(text, patterns, offsets=None, **kw) -> Matches:
    """Definition with a sound first-m-bytes filter, m = min(shortest pattern, 8)."""
    return match(ORC_BUCKETED, text, patterns, offsets, **kw)


def aho_corasick(text, patterns, offsets=None, **kw) -> Matches:
    """Textbook goto/failure/output automaton of Aho & Corasick (1975)."""
    return match(ORC_AC, text, patterns, offsets, **kw)


def counts(n: int, m: Matches, text_id: int = 0) -> np.ndarray:
    """count[i] = number of patterns matching at position i of one text."""
    sel = m["text"] == text_id
    return np.bincount(m["pos"][sel].astype(np.int64), minlength=n).astype(np.uint32)[:max(n, 0)]


def exhaustive(sigma: int, max_plen: int, max_npat: int, max_tlen: int,
               threads: int = 4) -> Tuple[int, int]:
    """(disagreements, cases) of brute vs bucketed vs Aho-Corasick on every small case."""
    lib = _load()
    nc = ctypes.c_uint64(0)
    bad = lib.orc_exhaustive(sigma, max_plen, max_npat, max_tlen, threads, ctypes.byref(nc))
    if bad < 0:
        raise ValueError("exhaustive: parameters out of range")
    return int(bad), int(nc.value)


# ------------------------------------------------------------------ trie


def canonical_trie(patterns: Sequence[bytes]) -> Dict[str, np.ndarray]:
    """CRS trie defined from the distinct prefixes of the patterns.

    Steps I and II of Design and Implementation number the trie breadth
    first, level by level, in a row-major array; step VI views it as a
    node x symbol matrix, and the CRS step stores that matrix as row_ptr
    (one row per node), col_ind (the symbol, i.e. the edge label) and val
    (the child node).  Sorting the distinct prefixes by (length, bytes) is that
    breadth-first order with children by ascending label.
    """
    pats = [bytes(p) for p in patterns]
    prefixes = {b""}
    for p in pats:
        for d in range(1, len(p) + 1):
            prefixes.add(p[:d])
    order = sorted(prefixes, key=lambda s: (len(s), s))
    index = {s: v for v, s in enumerate(order)}
    N = len(order)
    parent = np.array([index[s[:-1]] for s in order[1:]], dtype=np.int64)
    row_ptr = np.zeros(N + 1, dtype=np.uint32)
    np.add.at(row_ptr, parent + 1, 1)
    row_ptr = np.cumsum(row_ptr).astype(np.uint32)
    labels = np.array([s[-1] for s in order[1:]], dtype=np.uint8)
    child = np.array([index[s] for s in order[1:]], dtype=np.uint32)
    by_node: Dict[int, List[int]] = {}
    for j, p in enumerate(pats):
        by_node.setdefault(index[p], []).append(j)
    term_ptr = np.zeros(N + 1, dtype=np.uint32)
    term_ids: List[int] = []
    for v in range(N):
        ids = sorted(by_node.get(v, []))
        term_ids.extend(ids)
        term_ptr[v + 1] = len(term_ids)
    depth = np.array([len(s) for s in order], dtype=np.uint32)
    return {
        "row_ptr": row_ptr,
        "labels": labels,
        "child": child,
        "term_ptr": term_ptr,
        "term_ids": np.array(term_ids, dtype=np.uint32),
        "depth": depth,
    }


def footprint(n_nodes: int, n_patterns: int) -> Dict[str, int]:
    """Storage of the three trie forms, in bytes (and CRS elements).

    * dense: 256 int32 transitions per node (node x symbol matrix, step VI);
    * bitmap36: 256-bit child bitmap + 4-byte first-child offset per node
      (Results: 36 bytes per node);
    * crs_elements: 2 nnz + n + 1 with nnz = N - 1 edges and n = N rows
      (Design and Implementation);
    * crs_bytes: row_ptr and term_ptr as N+1 uint32, labels as nnz bytes,
      child as nnz uint32, term_ids as k uint32.
    """
    N = int(n_nodes)
    nnz = max(N - 1, 0)
    return {
        "dense": 1024 * N,
        "bitmap36": 36 * N,
        "crs_elements": 2 * nnz + N + 1,
        "crs_bytes": 4 * (N + 1) + nnz + 4 * nnz + 4 * (N + 1) + 4 * int(n_patterns),
    }
