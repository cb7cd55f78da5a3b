"""Seeded random parity: many small pattern sets and texts drawn over
alphabets of 2 to 256 bytes, pattern lengths that do and do not reach the
filters' minimum lengths, planted copies and partial copies, scanned by the
tile kernel (first levels through the level index or the bitmapped nodes,
whole, truncated or merged into a DAG),
the fused wave kernel and the split wave kernels (with each of their second
filter stages), single and batched, each against the oracle's
brute force."""

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from tests.gpu_util import assert_same, gpu_scan, gpu_scan_batch, say

pytestmark = pytest.mark.gpu

ALPHABETS = [b"\x00\x01", b"ACG", b"ACGT", bytes(range(97, 113)), bytes(range(256))]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _case(seed):
    rng = np.random.default_rng(1000 + seed)
    alpha = np.frombuffer(ALPHABETS[seed % len(ALPHABETS)], dtype=np.uint8)
    k = int(rng.integers(1, 400))
    lo = int(rng.choice([1, 2, 4, 16, 20]))
    hi = lo + int(rng.integers(0, 40))
    pats = [bytes(rng.choice(alpha, int(rng.integers(lo, hi + 1)))) for _ in range(k)]
    n = int(rng.integers(0, 200_000)) // (4 if alpha.size <= 4 else 1)
    text = rng.choice(alpha, n).astype(np.uint8)
    for _ in range(int(rng.integers(0, 300))):  # copies and prefixes of patterns
        p = pats[int(rng.integers(0, k))]
        if n > len(p):
            cut = int(rng.integers(1, len(p) + 1))
            at = int(rng.integers(0, n - cut + 1))
            text[at:at + cut] = np.frombuffer(p[:cut], dtype=np.uint8)
    return pats, text


TUNINGS = [dict(kernel=0), dict(kernel=1, child_check=1), dict(kernel=2, child_check=0),
           dict(kernel=2, child_check=1), dict(kernel=2, child_check=2, chunks_per_unit=4),
           dict(kernel=0, index_bits=8, top_nodes=1),
           dict(kernel=0, index_bits=16, top_nodes=0, trunc_depth=3),
           dict(kernel=0, index_bits=16, top_nodes=0, trunc_depth=0, dag=1)]


@pytest.mark.parametrize("seed", range(20))
def test_random_sets_every_kernel(seed):
    pats, text = _case(seed)
    want = oracle.brute(text, pats, threads=8)
    trie = pf.Trie(pats)
    say(f"random seed={seed}: k={len(pats)} n={text.size} alphabet={len(set(b''.join(pats)))} "
        f"matches={want.n}")
    for t in TUNINGS:
        trie.set_tuning(**t)
        got, counts = gpu_scan(trie, text, pad_front=seed % 16)
        assert_same(got, want)
        if text.size:
            assert np.array_equal(counts, oracle.counts(text.size, want)), t


@pytest.mark.parametrize("seed", range(20, 30))
def test_random_batches(seed):
    pats, text = _case(seed)
    rng = np.random.default_rng(seed)
    cuts = np.sort(rng.integers(0, text.size + 1, int(rng.integers(1, 300))))
    offs = np.concatenate([[0], cuts, [text.size]]).astype(np.uint64)
    want = oracle.brute(text, pats, offsets=offs, threads=8)
    trie = pf.Trie(pats)
    say(f"random batch seed={seed}: k={len(pats)} texts={len(offs) - 1} matches={want.n}")
    for t in TUNINGS:
        trie.set_tuning(**t)
        got, n = gpu_scan_batch(trie, text, offs, pad_front=(seed * 7) % 16)
        assert n == want.n
        assert_same(got, want, with_text=True)
