"""Seeded parity sweep: random pattern sets and texts (alphabets of 2 to 256
bytes, planted copies and prefixes) scanned under random launch tunings
(kernel, tile size, level-index bits, fold width, occupancy, waves, unit
size with odd sizes and the default's 63 and 64, second filter stage,
bitmapped top nodes, truncated and merged images), every result against
the oracle's brute force.  Single texts start
at any alignment and get an output buffer that may be too small (the exact
count comes back, then a retry); batches run as one launch, one launch per
text, or a graph replayed twice; one workspace serves all tunings of a case.
Tunings the library refuses are skipped; every accepted one must give the
oracle's list and, for single texts, its per-position counts."""

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from tests.gpu_util import gpu_scan, gpu_scan_batch, say
from tests.test_gpu_random import _case

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _tuning(rng):
    t = dict(kernel=int(rng.integers(0, 3)), bytes_per_lane=int(rng.choice([4, 8, 16])),
             index_bits=int(rng.choice([1, 8, 12, 16, 18])), fold_bits=int(rng.choice([0, 8, 16])),
             wg_per_cu=int(rng.integers(0, 3)), waves_per_wg=int(rng.choice([4, 8, 12, 16])),
             chunks_per_unit=int(rng.choice([1, 2, 3, 4, 8, 16, 32, 63, 64])),
             child_check=int(rng.integers(0, 3)),
             top_nodes=0, trunc_depth=0, dag=0)
    v = int(rng.integers(0, 5))
    if v == 1:
        t.update(top_nodes=1)
    elif v == 2:
        t.update(trunc_depth=int(rng.integers(1, 20)))
    elif v == 3:
        t.update(dag=1)
    return t


@pytest.mark.parametrize("block", range(6))
def test_random_sets_random_tunings(block):
    runs = 0
    for seed in range(5001 + 50 * block, 5051 + 50 * block):
        pats, text = _case(seed)
        rng = np.random.default_rng(seed * 7 + 1)
        offs = None
        if seed % 3 == 0:
            cuts = np.sort(rng.integers(0, text.size + 1, int(rng.integers(1, 300))))
            offs = np.concatenate([[0], cuts, [text.size]]).astype(np.uint64)
        want = oracle.brute(text, pats, offsets=offs, threads=8)
        trie = pf.Trie(pats)
        ws = pf.Workspace()
        pad = seed % 16
        for _ in range(5):
            t = _tuning(rng)
            try:
                trie.set_tuning(**t)
            except pf.PfacError:
                continue
            runs += 1
            where = f"seed {seed} tuning {t} k {len(pats)} n {text.size}"
            if offs is not None:
                mode = int(rng.integers(0, 3))
                where += f" batch mode {mode}"
                if mode == 2:
                    res, n = gpu_scan_batch(trie, text, offs, ws=ws, pad_front=pad, graph_replays=2,
                                            capacity=want.n + 16)
                    got = res[-1]
                    assert np.array_equal(res[0], got), where
                else:
                    got, n = gpu_scan_batch(trie, text, offs, ws=ws, pad_front=pad, plain=mode == 1)
                assert n == want.n, where
                assert np.array_equal(got["text_id"], want["text"]), where
            else:
                cap = [None, 1, want.n // 2 + 1][int(rng.integers(0, 3))]
                got, counts = gpu_scan(trie, text, ws=ws, pad_front=pad, capacity=cap)
                assert got.size == want.n, where
                if text.size:
                    assert np.array_equal(counts, oracle.counts(text.size, want)), where
            assert np.array_equal(got["pos"], want["pos"]), where
            assert np.array_equal(got["pattern_id"], want["id"]), where
    say(f"fuzz block {block}: {runs} scans")
    assert runs > 100
