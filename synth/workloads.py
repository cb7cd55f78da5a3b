"""Workload recipes for the five scan configurations.

Every generator uses ``numpy.random.Generator(MT19937(SEED_BASE + index))``.
The paper picks its patterns with the Mersenne Twister (Results section); its
King James Bible text is not available here, so seeded synthetic bytes stand
in for it, with the sizes and byte distributions of the five configurations:

==  ==========================================================================
C1  100 patterns, lengths U{4..16}, bytes U{0..255}; 1 MiB text, same bytes;
    1000 planted copies at uniform offsets.
C2  10,000 patterns, lengths U{8..64}; each byte is printable ASCII
    (U{0x20..0x7E}) with probability 0.7, else U{0..255}; 256 MiB text of the
    same mix; copies planted with geometric gaps of mean 4096 bytes.
C3  100,000 patterns, lengths U{20..32} over {A,C,G,T}; 1 GiB uniform ACGT
    text; 10,000 copies at uniform offsets.
C4  20,000 patterns, lengths U{8..64}, bytes U{0..255}; 65,536 small texts
    with lengths clip(round(lognormal(ln 512, 0.75)), 64, 1500) plus 64 large
    texts with lengths U{1 MiB..64 MiB} placed at seeded positions; every text
    gets Poisson(len / 2048) copies.
C5  50,000 patterns, lengths U{8..64}, bytes U{0..255}; requests with sizes
    floor(exp(U(ln 1 KiB, ln 64 MiB))), Poisson(size / 2048) copies each.
==  ==========================================================================

Copies are written in draw order, so a later copy may overwrite part of an
earlier one; the manifest lists every copy that was written.  Sizes can be
scaled down for tests; the distributions stay the same.
"""

from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

SEED_BASE = 1702036570
_CHUNK = 1 << 26  # bytes drawn per generator call, bounds the temporaries
_ACGT = np.frombuffer(b"ACGT", dtype=np.uint8)

MiB = 1 << 20
GiB = 1 << 30


def rng_for(index: int) -> np.random.Generator:
    return np.random.Generator(np.random.MT19937(SEED_BASE + int(index)))


@dataclasses.dataclass
class PatternSet:
    """``k`` byte strings stored back to back: pattern j is data[offsets[j]:offsets[j+1]]."""

    data: np.ndarray      # uint8
    offsets: np.ndarray   # uint64, length k + 1

    @classmethod
    def from_list(cls, pats: Sequence[bytes]) -> "PatternSet":
        lens = np.array([len(p) for p in pats], dtype=np.uint64)
        offs = np.zeros(len(pats) + 1, dtype=np.uint64)
        if len(pats):
            offs[1:] = np.cumsum(lens)
        data = np.frombuffer(b"".join(bytes(p) for p in pats), dtype=np.uint8).copy()
        return cls(data=data, offsets=offs)

    def __len__(self) -> int:
        return len(self.offsets) - 1

    def __getitem__(self, j: int) -> bytes:
        return self.data[int(self.offsets[j]):int(self.offsets[j + 1])].tobytes()

    @property
    def lengths(self) -> np.ndarray:
        return np.diff(self.offsets).astype(np.uint64)

    def as_list(self) -> List[bytes]:
        return [self[j] for j in range(len(self))]


@dataclasses.dataclass
class Workload:
    """Patterns plus one or more texts stored back to back.

    Text i is ``text[offsets[i]:offsets[i+1]]``.  ``plants`` is an (m, 3)
    uint64 array of (text_id, position within the text, pattern_id) in the
    order the copies were written.
    """

    name: str
    patterns: PatternSet
    text: np.ndarray       # uint8, all texts concatenated
    offsets: np.ndarray    # uint64, n_texts + 1
    plants: np.ndarray     # uint64 (m, 3)

    @property
    def n_texts(self) -> int:
        return len(self.offsets) - 1

    def text_of(self, i: int) -> np.ndarray:
        return self.text[int(self.offsets[i]):int(self.offsets[i + 1])]


# ---------------------------------------------------------------- bytes


def draw_bytes(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    """``n`` bytes from ``dist``: 'uniform', 'mix' (70% printable) or 'acgt'."""
    out = np.empty(n, dtype=np.uint8)
    for lo in range(0, n, _CHUNK):
        m = min(_CHUNK, n - lo)
        if dist == "uniform":
            out[lo:lo + m] = rng.integers(0, 256, m, dtype=np.uint8)
        elif dist == "mix":
            printable = rng.integers(0x20, 0x7F, m, dtype=np.uint8)
            anybyte = rng.integers(0, 256, m, dtype=np.uint8)
            sel = rng.integers(0, 10, m, dtype=np.uint8) < 7
            out[lo:lo + m] = np.where(sel, printable, anybyte)
        elif dist == "acgt":
            out[lo:lo + m] = _ACGT[rng.integers(0, 4, m, dtype=np.uint8)]
        else:
            raise ValueError(f"unknown byte distribution {dist!r}")
    return out


def make_patterns(rng: np.random.Generator, k: int, len_lo: int, len_hi: int,
                  dist: str) -> PatternSet:
    lens = rng.integers(len_lo, len_hi + 1, k).astype(np.uint64)
    offs = np.zeros(k + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    data = draw_bytes(rng, int(offs[-1]), dist)
    return PatternSet(data=data, offsets=offs)


def make_text(rng: np.random.Generator, n: int, dist: str) -> np.ndarray:
    return draw_bytes(rng, n, dist)


def plant(text: np.ndarray, pats: PatternSet, text_id: int, base: int,
          positions: np.ndarray, ids: np.ndarray, text_len: int) -> List[tuple]:
    """Write pattern ``ids[r]`` at ``base + positions[r]`` in draw order.

    A copy that would run past ``text_len`` is skipped.  Returns the manifest
    rows that were written.
    """
    rows = []
    lens = pats.lengths
    for pos, j in zip(positions.tolist(), ids.tolist()):
        ln = int(lens[j])
        if pos + ln > text_len:
            continue
        a = int(pats.offsets[j])
        text[base + pos:base + pos + ln] = pats.data[a:a + ln]
        rows.append((text_id, pos, j))
    return rows


def _manifest(rows: List[tuple]) -> np.ndarray:
    if not rows:
        return np.zeros((0, 3), dtype=np.uint64)
    return np.asarray(rows, dtype=np.uint64)


def _single(name, pats, text, rows) -> Workload:
    return Workload(name=name, patterns=pats, text=text,
                    offsets=np.array([0, len(text)], dtype=np.uint64),
                    plants=_manifest(rows))


# ---------------------------------------------------------------- configs


def c1_plain_small(n_text: int = 1 * MiB, k: int = 100, n_plants: int = 1000) -> Workload:
    rng = rng_for(0)
    pats = make_patterns(rng, k, 4, 16, "uniform")
    text = make_text(rng, n_text, "uniform")
    ids = rng.integers(0, k, n_plants)
    highs = np.maximum(n_text - pats.lengths[ids].astype(np.int64) + 1, 1)
    pos = rng.integers(0, highs)
    rows = plant(text, pats, 0, 0, pos, ids, n_text)
    return _single("c1", pats, text, rows)


def c2_signature_set(n_text: int = 256 * MiB, k: int = 10_000,
                     mean_gap: int = 4096) -> Workload:
    rng = rng_for(1)
    pats = make_patterns(rng, k, 8, 64, "mix")
    text = make_text(rng, n_text, "mix")
    n_draw = int(n_text / mean_gap * 1.2) + 16
    gaps = rng.geometric(1.0 / mean_gap, n_draw)
    pos = np.cumsum(gaps) - 1
    pos = pos[pos < n_text]
    ids = rng.integers(0, k, len(pos))
    rows = plant(text, pats, 0, 0, pos, ids, n_text)
    return _single("c2", pats, text, rows)


def c3_dna(n_text: int = 1 * GiB, k: int = 100_000, n_plants: int = 10_000) -> Workload:
    rng = rng_for(2)
    pats = make_patterns(rng, k, 20, 32, "acgt")
    text = make_text(rng, n_text, "acgt")
    ids = rng.integers(0, k, n_plants)
    highs = np.maximum(n_text - pats.lengths[ids].astype(np.int64) + 1, 1)
    pos = rng.integers(0, highs)
    rows = plant(text, pats, 0, 0, pos, ids, n_text)
    return _single("c3", pats, text, rows)


def _batch_texts(rng, pats: PatternSet, lens: np.ndarray, rate: float,
                 name: str) -> Workload:
    offs = np.zeros(len(lens) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens.astype(np.uint64))
    text = make_text(rng, int(offs[-1]), "uniform")
    counts = rng.poisson(lens.astype(np.float64) * rate)
    rows: List[tuple] = []
    k = len(pats)
    plens = pats.lengths.astype(np.int64)
    for i in np.nonzero(counts)[0].tolist():
        c = int(counts[i])
        ids = rng.integers(0, k, c)
        highs = np.maximum(int(lens[i]) - plens[ids] + 1, 1)
        pos = rng.integers(0, highs)
        rows.extend(plant(text, pats, i, int(offs[i]), pos, ids, int(lens[i])))
    return Workload(name=name, patterns=pats, text=text, offsets=offs,
                    plants=_manifest(rows))


def c4_batched(n_small: int = 65_536, n_large: int = 64, large_lo: int = 1 * MiB,
               large_hi: int = 64 * MiB, k: int = 20_000, rate: float = 1 / 2048) -> Workload:
    rng = rng_for(3)
    pats = make_patterns(rng, k, 8, 64, "uniform")
    small = np.clip(np.rint(rng.lognormal(math.log(512), 0.75, n_small)), 64, 1500)
    large = rng.integers(large_lo, large_hi + 1, n_large)
    n = n_small + n_large
    where = np.sort(rng.choice(n, n_large, replace=False)) if n_large else np.zeros(0, int)
    lens = np.empty(n, dtype=np.int64)
    is_large = np.zeros(n, dtype=bool)
    is_large[where] = True
    lens[is_large] = large
    lens[~is_large] = small.astype(np.int64)
    return _batch_texts(rng, pats, lens, rate, "c4")


def c5_requests(n_requests: int = 2000, lo: int = 1024, hi: int = 64 * MiB,
                k: int = 50_000, rate: float = 1 / 2048,
                sizes_only: bool = False):
    """Pattern set and request texts for the serving configuration.

    With ``sizes_only`` the texts are not drawn: returns (patterns, sizes).
    """
    rng = rng_for(4)
    pats = make_patterns(rng, k, 8, 64, "uniform")
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n_requests))).astype(np.int64)
    if sizes_only:
        return pats, sizes
    return _batch_texts(rng, pats, sizes, rate, "c5")


def workload(name: str, **kw) -> Workload:
    return {
        "c1": c1_plain_small,
        "c2": c2_signature_set,
        "c3": c3_dna,
        "c4": c4_batched,
        "c5": c5_requests,
    }[name](**kw)


def poisson_arrivals(n: int, rate_per_s: float, seed: Optional[int] = None) -> np.ndarray:
    """Arrival times (seconds from 0) of a Poisson process with the given rate."""
    rng = rng_for(100 if seed is None else seed)
    return np.cumsum(rng.exponential(1.0 / rate_per_s, n))
