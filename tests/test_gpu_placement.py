"""Trie placement (how many trie levels the level index resolves in LDS, down
to none): every depth the benchmark's placement ablation measures gives the
oracle's match list, on each workload's pattern set at a reduced text size,
single texts and batches, for the tile kernel (level index or bitmapped
nodes) and for the wave kernels with the filter at depth 0 and 1."""

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from bench import lds_depth_tuning
from synth import workloads
from tests.gpu_util import assert_same, gpu_scan, gpu_scan_batch, say

pytestmark = pytest.mark.gpu

KiB, MiB = 1 << 10, 1 << 20

SCALED = {
    "c1": lambda: workloads.c1_plain_small(n_text=256 * KiB + 19, n_plants=300),
    "c2": lambda: workloads.c2_signature_set(n_text=2 * MiB + 3, mean_gap=2048),
    "c3": lambda: workloads.c3_dna(n_text=1 * MiB + 7, k=20_000, n_plants=1500),
    "c4": lambda: workloads.c4_batched(n_small=3000, n_large=3, large_lo=64 * KiB,
                                       large_hi=512 * KiB, rate=1 / 512),
    "c5": lambda: workloads.c5_requests(12, hi=1 * MiB, rate=1 / 512),
}


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _points(st):
    pts = []
    for d in range(10):
        t = lds_depth_tuning(st, d)
        if t is not None:
            pts.append((d, t))
    # the tile kernel with the first levels through the bitmapped nodes
    for d in range(1, 10):
        t = lds_depth_tuning(st, d)
        if t is not None:
            pts.append((d, dict(t, top_nodes=1)))
    # the wave kernels with the filter on the root's children only, and one level
    for d in (0, 1):
        t = lds_depth_tuning(st, d)
        if t is not None:
            for k in (1, 2):
                pts.append((d, dict(t, kernel=k, fold_bits=0, chunks_per_unit=8)))
    return pts


@pytest.mark.parametrize("name", sorted(SCALED))
def test_every_lds_depth(name):
    wl = SCALED[name]()
    offs = wl.offsets.astype(np.uint64)
    n_texts = len(offs) - 1
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets if n_texts > 1 else None,
                           threads=8)
    trie = pf.Trie(wl.patterns)
    st = trie.stats()
    pts = _points(st)
    assert any(d == 0 for d, _ in pts) and len(pts) >= 3
    say(f"placement {name}: {n_texts} texts, {wl.text.size} bytes, {want.n} matches, "
        f"{len(pts)} points")
    assert want.n > 0
    for d, t in pts:
        try:
            trie.set_tuning(**t)
        except pf.PfacError:
            # bitmapped top nodes too large for LDS: refused, tuning unchanged
            assert t.get("top_nodes") and trie.stats()["bytes_top_nodes"] > 0
            say(f"  depth {d} {t}: refused (LDS)")
            continue
        assert trie.stats()["index_depth"] == d, t
        say(f"  depth {d} {t}")
        if n_texts > 1:
            got, n = gpu_scan_batch(trie, wl.text, offs)
            assert n == want.n
            assert_same(got, want, with_text=True)
        else:
            got, counts = gpu_scan(trie, wl.text)
            assert_same(got, want)
            assert np.array_equal(counts, oracle.counts(wl.text.size, want))
