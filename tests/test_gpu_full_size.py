"""Parity at the benchmark's full sizes, in the launch configurations bench.py
times: the 256 MiB signature-set scan (c2), the 1 GiB DNA scan (c3), the
65,600-text batch in one graph-captured launch (c4) and 200 serving requests
(c5), each compared with the oracle's complete match list."""

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from synth import workloads
from tests.gpu_util import assert_same, say

pytestmark = pytest.mark.gpu

# the tunings bench.py's autotuner settles on for these workloads
C2_TUNING = dict(kernel=2, bytes_per_lane=16, index_bits=16, fold_bits=8, wg_per_cu=0,
                 waves_per_wg=16, chunks_per_unit=32, child_check=2)
C3_TUNING = dict(kernel=2, bytes_per_lane=16, index_bits=18, fold_bits=8, wg_per_cu=0,
                 waves_per_wg=16, chunks_per_unit=16, child_check=1)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _scan_whole(trie, text_host, capacity):
    import torch
    text = torch.from_numpy(text_host).cuda()
    ws = pf.Workspace()
    out = torch.empty(capacity * 16, dtype=torch.uint8, device="cuda")
    rc, n = pf.pfac_scan_sync(trie, ws, text, text.numel(), out, capacity)
    assert rc == pf.PFAC_OK, (rc, n)
    got = pf.matches_to_numpy(out, n)
    del text, out
    return got


@pytest.mark.parametrize("name", ["c2", "c3"])
def test_full_size_single_text(name):
    wl = workloads.c2_signature_set() if name == "c2" else workloads.c3_dna()
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(**(C2_TUNING if name == "c2" else C3_TUNING))
    st = trie.stats()
    say(f"full {name}: {wl.text.size} bytes, {len(wl.patterns)} patterns, kernel {st['scan_kernel']} "
        f"stage1 {st['stage1']} stage2 {st['stage2']}")
    want = oracle.bucketed(wl.text, wl.patterns, threads=16)
    assert want.n > 5000
    got = _scan_whole(trie, wl.text, want.n + 1024)
    assert_same(got, want)
    # every planted copy that survived later plants is in the list (manifest
    # rows: text id, position, pattern id)
    found = set(zip(got["pos"].tolist(), got["pattern_id"].tolist()))
    p = wl.patterns.as_list()
    kept = [(int(pos), int(j)) for _, pos, j in wl.plants.tolist()
            if bytes(wl.text[int(pos):int(pos) + len(p[int(j)])]) == p[int(j)]]
    assert len(kept) > 0.9 * len(wl.plants)
    assert all(k in found for k in kept)


def test_full_size_batch_graph():
    wl = workloads.c4_batched()
    trie = pf.Trie(wl.patterns)
    offs = wl.offsets.astype(np.uint64)
    say(f"full c4: {len(offs) - 1} texts, {wl.text.size} bytes")
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=16)
    import torch
    text = torch.from_numpy(wl.text).cuda()
    offs_dev = torch.from_numpy(offs.view(np.int64)).cuda()
    cap = want.n + 1024
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    ws = pf.Workspace()
    g = pf.Graph(trie, ws, text, offs_dev, len(offs) - 1, int(offs[-1]), out, cap, cnt, s)
    for _ in range(2):
        out.fill_(0xAB)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        assert int(cnt.item()) == want.n
        assert_same(pf.matches_to_numpy(out, want.n), want, with_text=True)
    g.close()


def test_full_size_serving_requests():
    import torch
    wl = workloads.c5_requests(200)
    offs = wl.offsets.astype(np.int64)
    sizes = np.diff(offs)
    say(f"serving c5: {len(sizes)} requests, {int(offs[-1])} bytes")
    trie = pf.Trie(wl.patterns)
    budget = 1 << 30
    arena = torch.empty(budget + (256 << 20), dtype=torch.uint8, device="cuda")
    srv = pf.Server(trie, arena, budget, 64, torch.cuda.Stream(), torch.cuda.Stream())
    ids = [srv.submit(wl.text[offs[i]:offs[i + 1]]) for i in range(len(sizes))]
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=16)
    for i, rid in enumerate(ids):
        got, _ = srv.wait(rid, capacity=1 << 22)
        sel = want["text"] == i
        assert got.size == int(sel.sum()), i
        assert np.array_equal(got["pos"], want["pos"][sel]), i
        assert np.array_equal(got["pattern_id"], want["id"][sel]), i
    srv.close()


def test_positions_beyond_4_gib():
    """64-bit positions: a text of 2^32 + 2^20 + 4,109 bytes (zeros, with a random
    stretch across byte 2^32 and planted copies straddling it, at both ends
    and inside the stretch), scanned whole and as a batch of three texts
    whose boundaries lie on both sides of 2^32, against the oracle's lists."""
    import torch
    rng = np.random.default_rng(77)
    pats = workloads.make_patterns(rng, 300, 6, 24, "uniform")
    plist = pats.as_list()
    n = (1 << 32) + (1 << 20) + 4096 + 13
    text = np.zeros(n, dtype=np.uint8)
    lo = (1 << 32) - (1 << 20)
    text[lo:lo + (2 << 20)] = rng.integers(0, 256, 2 << 20, dtype=np.uint8)
    at = [0, (1 << 32) - 3, (1 << 32) - 1, 1 << 32, (1 << 32) + 7, n - len(plist[5])]
    at += rng.integers(lo, lo + (2 << 20) - 32, 200).tolist()
    for i, p in enumerate(at):
        q = plist[(5 + 7 * i) % len(plist)] if p != n - len(plist[5]) else plist[5]
        text[p:p + len(q)] = np.frombuffer(q, dtype=np.uint8)
    say(f"beyond 4 GiB: {n} bytes, {len(at)} plants")
    want = oracle.bucketed(text, pats, threads=16)
    assert (want["pos"] >= (1 << 32)).sum() > 50 and want.n > 150
    trie = pf.Trie(pats)
    dev = torch.from_numpy(text).cuda()
    cap = want.n + 1024
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    ws = pf.Workspace()
    default = trie.tuning()
    for tn in (default, dict(default, kernel=0)):  # the library's choice, then the tile kernel
        trie.set_tuning(**tn)
        say(f"  kernel {trie.stats()['scan_kernel']}")
        rc, got_n = pf.pfac_scan_sync(trie, ws, dev, n, out, cap)
        assert rc == pf.PFAC_OK and got_n == want.n
        assert_same(pf.matches_to_numpy(out, got_n), want)
    trie.set_tuning(**default)
    # the same bytes as three texts: [0, 2^32 - 5), [2^32 - 5, 2^32 + 100), the rest
    offs = np.array([0, (1 << 32) - 5, (1 << 32) + 100, n], dtype=np.uint64)
    want_b = oracle.bucketed(text, pats, offsets=offs, threads=16)
    offs_dev = torch.from_numpy(offs.view(np.int64)).cuda()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.current_stream()
    pf.pfac_scan_batch(trie, ws, dev, offs_dev, 3, n, out, cap, cnt, s)
    torch.cuda.synchronize()
    assert int(cnt.item()) == want_b.n
    assert_same(pf.matches_to_numpy(out, want_b.n), want_b, with_text=True)
    del dev, out
