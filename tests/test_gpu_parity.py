"""GPU parity: the HIP scan through the C ABI against the CPU oracle, bit-exact
on the sorted (text, pos, pattern_id) list and on per-position counts."""

import itertools

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from synth import PatternSet, workloads
from tests.gpu_util import assert_same, gpu_scan, gpu_scan_batch, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def test_c1_full_size_against_brute_force():
    wl = workloads.c1_plain_small()
    say(f"c1 full: {wl.text.size} bytes, {len(wl.patterns)} patterns")
    trie = pf.Trie(wl.patterns)
    got, counts = gpu_scan(trie, wl.text)
    want = oracle.brute(wl.text, wl.patterns, threads=8)
    assert want.n >= 900
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(wl.text.size, want))


TUNINGS = (
    [dict(kernel=0, bytes_per_lane=bpl, index_bits=bits) for bpl in (4, 8, 16) for bits in (8, 12, 16, 18)]
    + [dict(kernel=1, index_bits=bits, fold_bits=fold, waves_per_wg=w, chunks_per_unit=g, child_check=cc)
       for bits in (8, 12, 16, 18) for fold in (0, 8, 16) for (w, g, cc) in ((4, 1, 0), (16, 16, 1), (12, 64, 1), (12, 16, 2))]
    # split filter + walk kernels
    + [dict(kernel=2, index_bits=bits, fold_bits=fold, waves_per_wg=w, chunks_per_unit=g, child_check=cc)
       for bits in (8, 12, 16, 18) for fold in (0, 8, 16) for (w, g, cc) in ((4, 1, 0), (16, 32, 1), (16, 16, 2), (8, 4, 2))]
)


def _tid(t):
    return "-".join(f"{k[0]}{v}" for k, v in t.items())


@pytest.mark.parametrize("tuning", TUNINGS, ids=_tid)
def test_every_tuning_point_c1(tuning):
    wl = workloads.c1_plain_small(n_text=(1 << 18) + 77, k=100, n_plants=400)
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(**tuning)
    say(f"tuning {tuning} K={trie.stats()['index_depth']}")
    got, counts = gpu_scan(trie, wl.text)
    want = oracle.brute(wl.text, wl.patterns, threads=8)
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(wl.text.size, want))


DNA_TUNINGS = [
    dict(kernel=0, bytes_per_lane=16, index_bits=16), dict(kernel=0, bytes_per_lane=8, index_bits=18, wg_per_cu=2),
    dict(kernel=0, bytes_per_lane=4, index_bits=12, wg_per_cu=1), dict(kernel=0, bytes_per_lane=16, index_bits=8, wg_per_cu=4),
    dict(kernel=1, index_bits=16, fold_bits=8), dict(kernel=1, index_bits=16, fold_bits=16),
    dict(kernel=1, index_bits=12, fold_bits=16, waves_per_wg=8), dict(kernel=1, index_bits=18, fold_bits=0),
    dict(kernel=1, index_bits=14, fold_bits=8, waves_per_wg=4, wg_per_cu=1),
    dict(kernel=1, index_bits=16, fold_bits=8, chunks_per_unit=1, child_check=0),
    dict(kernel=1, index_bits=12, fold_bits=8, chunks_per_unit=64, child_check=1),
    dict(kernel=2, index_bits=16, fold_bits=8), dict(kernel=2, index_bits=18, fold_bits=0),
    dict(kernel=2, index_bits=12, fold_bits=16, waves_per_wg=8, chunks_per_unit=2),
]


@pytest.mark.parametrize("tuning", DNA_TUNINGS, ids=_tid)
def test_dna_tuning_points(tuning):
    wl = workloads.c3_dna(n_text=(1 << 20) + 5, k=20_000, n_plants=2000)
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(**tuning)
    st = trie.stats()
    say(f"dna {tuning} K={st['index_depth']} b={st['symbol_bits']}")
    got, counts = gpu_scan(trie, wl.text)
    want = oracle.bucketed(wl.text, wl.patterns, threads=8)
    assert want.n >= 1800
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(wl.text.size, want))


@pytest.mark.parametrize("case", ["dirty_text", "three_letters", "batch", "short_units"])
def test_four_symbol_filter(case):
    """The split kernel's 16-symbol filter: texts with bytes outside the
    alphabet (which the symbol arithmetic aliases), a smaller alphabet,
    batches of uneven texts and one-chunk units."""
    rng = np.random.default_rng(17)
    if case == "three_letters":
        pats = [bytes(rng.choice(list(b"ACG"), int(n)).astype(np.uint8)) for n in rng.integers(16, 40, 3000)]
        text = rng.choice(list(b"ACGT"), 300_000, p=[0.33, 0.33, 0.33, 0.01]).astype(np.uint8)
    else:
        wl = workloads.c3_dna(n_text=(1 << 19) + 3, k=5000, n_plants=800)
        pats, text = wl.patterns.as_list(), wl.text.copy()
    if case == "dirty_text":
        # 'N', lower case and other bytes, some inside planted copies
        bad = rng.integers(0, text.size, 4000)
        text[bad] = rng.choice(list(b"Nacgt\x00\xff@"), bad.size).astype(np.uint8)
    # every 16-symbol prefix of some pattern appears too (filter hits that
    # fail later), and exact copies
    for _ in range(300):
        p = pats[int(rng.integers(0, len(pats)))]
        at = int(rng.integers(0, text.size - len(p)))
        cut = int(rng.integers(16, len(p) + 1))
        text[at:at + cut] = np.frombuffer(p[:cut], dtype=np.uint8)
    trie = pf.Trie(pats)
    trie.set_tuning(kernel=2, chunks_per_unit=1 if case == "short_units" else 16)
    say(f"four-symbol {case}: n={text.size} k={len(pats)} K={trie.stats()['index_depth']}")
    if case == "batch":
        lens = rng.integers(0, 5000, 200)
        offs = np.zeros(lens.size + 1, dtype=np.uint64)
        offs[1:] = np.cumsum(lens)
        t = text[: int(offs[-1])]
        want = oracle.bucketed(t, pats, offsets=offs, threads=8)
        got, n = gpu_scan_batch(trie, t, offs, pad_front=5)
        assert n == want.n
        assert_same(got, want, with_text=True)
        return
    got, counts = gpu_scan(trie, text)
    want = oracle.bucketed(text, pats, threads=8)
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(text.size, want))


def test_four_symbol_filter_graph_replays():
    rng = np.random.default_rng(23)
    wl = workloads.c3_dna(n_text=(1 << 20), k=8000, n_plants=1500)
    lens = rng.integers(0, 40_000, 60)
    offs = np.zeros(lens.size + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    text = wl.text[: int(offs[-1])]
    trie = pf.Trie(wl.patterns)
    assert trie.stats()["stage1"] == 3
    want = oracle.bucketed(text, wl.patterns, offsets=offs, threads=8)
    say(f"four-symbol graph: {lens.size} texts, {want.n} matches")
    results, n = gpu_scan_batch(trie, text, offs, graph_replays=3)
    assert n == want.n
    for r in results:
        assert_same(r, want, with_text=True)


@pytest.mark.parametrize("kernel", [1, 2])
def test_c2_scaled_full_pattern_set(kernel):
    wl = workloads.c2_signature_set(n_text=16 << 20, k=10_000)
    say(f"c2 scaled: {wl.text.size} bytes, kernel {kernel}")
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(kernel=kernel, chunks_per_unit=32)
    got, counts = gpu_scan(trie, wl.text)
    want = oracle.bucketed(wl.text, wl.patterns, threads=8)
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(wl.text.size, want))


@pytest.mark.parametrize("pad", [1, 3, 7, 8, 13, 15])
def test_misaligned_text_addresses(pad):
    wl = workloads.c1_plain_small(n_text=50_001, k=100, n_plants=200)
    trie = pf.Trie(wl.patterns)
    got, counts = gpu_scan(trie, wl.text, pad_front=pad)
    want = oracle.brute(wl.text, wl.patterns, threads=8)
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(wl.text.size, want))


@pytest.mark.parametrize("kernel", [0, 1, 2, "0t", "0d", "0g"])
@pytest.mark.parametrize("case", [
    "empty_text", "short_text", "no_patterns", "length_one", "duplicates", "nested_runs",
    "all_windows", "sigma1_long", "long_patterns", "match_at_end", "dense_candidates",
])
def test_edge_cases(case, kernel):
    rng = np.random.default_rng(hash(case) & 0xffff)
    if case == "empty_text":
        pats, text = [b"abc", b"x"], b""
    elif case == "short_text":
        pats, text = [b"abcdef", b"bcdefg"], b"abcde"
    elif case == "no_patterns":
        pats, text = [], bytes(rng.integers(0, 256, 10_000).astype(np.uint8))
    elif case == "length_one":
        pats = [bytes([c]) for c in rng.choice(256, 30, replace=False)] + [b"\x01\x02"]
        text = bytes(rng.integers(0, 256, 70_000).astype(np.uint8))
    elif case == "duplicates":
        pats = [b"ab", b"xyz", b"ab", b"b", b"ab", b"abxyz", b"xyz"]
        text = bytes(rng.choice(list(b"abxyz"), 30_000).astype(np.uint8))
    elif case == "nested_runs":
        # every position matches many patterns: the dense-tile path
        pats = [b"a" * d for d in range(1, 40)]
        text = b"a" * 20_000 + b"b" + b"a" * 5000
    elif case == "all_windows":
        pats = [bytes(t) for t in itertools.product(b"ACGT", repeat=5)]
        text = bytes(rng.choice(list(b"ACGT"), 100_000).astype(np.uint8))
    elif case == "sigma1_long":
        pats = [b"\x00" * 17, b"\x00" * 3]
        text = b"\x00" * 9999
    elif case == "long_patterns":
        # longer than the LDS halo: walks continue in global memory
        base = bytes(rng.integers(0, 4, 5000).astype(np.uint8))
        pats = [base[:3000], base[:2000] + b"\xff", base[1000:4500], base[4000:4003]]
        text = (base * 7)[: 30_000]
    elif case == "dense_candidates":
        # every position passes both filter stages: candidate lists overflow
        pats = [b"aaaab", b"aaab", b"aabx"]
        text = (b"a" * 3000 + b"b") * 12
    else:  # match_at_end
        pats = [b"tail!", b"l!"]
        text = bytes(rng.integers(0, 200, 8191).astype(np.uint8)) + b"tail!"
    text = np.frombuffer(text, dtype=np.uint8).copy()
    trie = pf.Trie(pats)
    if kernel == "0t":  # tile kernel, first levels through the bitmapped nodes
        trie.set_tuning(kernel=0, index_bits=8, top_nodes=1)
    elif kernel == "0d":  # image truncated at depth 2, tails verified
        trie.set_tuning(kernel=0, trunc_depth=2)
    elif kernel == "0g":  # merged DAG image, ranks on the edges
        trie.set_tuning(kernel=0, dag=1)
    else:
        trie.set_tuning(kernel=kernel)
    say(f"edge {case} kernel {kernel}: n={text.size} k={len(pats)} K={trie.stats()['index_depth']}")
    got, counts = gpu_scan(trie, text)
    want = oracle.brute(text, pats, threads=8)
    assert_same(got, want)
    if text.size:
        assert np.array_equal(counts, oracle.counts(text.size, want))


TRUNC_CASES = {
    "c1": lambda: workloads.c1_plain_small(n_text=(1 << 18) + 77, k=100, n_plants=400),
    "c2": lambda: workloads.c2_signature_set(n_text=(1 << 21) + 5, mean_gap=1024),
    "c3": lambda: workloads.c3_dna(n_text=(1 << 20) + 5, k=20_000, n_plants=2000),
    "c4": lambda: workloads.c4_batched(n_small=2000, n_large=2, large_lo=1 << 16,
                                       large_hi=1 << 18, rate=1 / 256),
}


@pytest.mark.parametrize("name", sorted(TRUNC_CASES))
def test_truncated_images(name):
    """Images truncated at several depths (tails verified against the
    pattern bytes) give the oracle's list, single texts and batches."""
    wl = TRUNC_CASES[name]()
    offs = wl.offsets.astype(np.uint64)
    batch = len(offs) > 2
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets if batch else None, threads=8)
    assert want.n > 100
    trie = pf.Trie(wl.patterns)
    for D in (1, 2, 3, 5, 8, 12, 20, 40):
        trie.set_tuning(kernel=0, trunc_depth=D, index_bits=16)
        st = trie.stats()
        say(f"truncated {name} D={D}: depth {st['trunc_depth']} K={st['index_depth']} "
            f"nodes {st['bytes_nodes']} tails {st['bytes_tails']}")
        if batch:
            got, n = gpu_scan_batch(trie, wl.text, offs)
            assert n == want.n
            assert_same(got, want, with_text=True)
        else:
            got, counts = gpu_scan(trie, wl.text, pad_front=D % 16)
            assert_same(got, want)
            assert np.array_equal(counts, oracle.counts(wl.text.size, want))


@pytest.mark.parametrize("name", sorted(TRUNC_CASES))
def test_merged_dag_images(name):
    """The merged DAG image (equal subtries shared, pattern ids recovered
    from the ranks on the edges) gives the oracle's list at several level
    index depths and tile sizes, single texts and batches."""
    wl = TRUNC_CASES[name]()
    offs = wl.offsets.astype(np.uint64)
    batch = len(offs) > 2
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets if batch else None, threads=8)
    trie = pf.Trie(wl.patterns)
    full = trie.stats()
    for bits, bpl in ((1, 16), (8, 4), (16, 16), (18, 8)):
        trie.set_tuning(kernel=0, dag=1, index_bits=bits, bytes_per_lane=bpl)
        st = trie.stats()
        say(f"dag {name} bits={bits} bpl={bpl}: K={st['index_depth']} dag nodes {st['dag_nodes']} "
            f"of {full['nodes']}, image {st['bytes_device']} vs {full['bytes_device']}")
        if batch:
            got, n = gpu_scan_batch(trie, wl.text, offs)
            assert n == want.n
            assert_same(got, want, with_text=True)
        else:
            got, counts = gpu_scan(trie, wl.text, pad_front=bits % 16)
            assert_same(got, want)
            assert np.array_equal(counts, oracle.counts(wl.text.size, want))


@pytest.mark.parametrize("kernel", [1, 2])
def test_capacity_overflow_reports_exact_count(kernel):
    wl = workloads.c1_plain_small(n_text=200_000, k=100, n_plants=2000)
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(kernel=kernel)
    want = oracle.brute(wl.text, wl.patterns, threads=8)
    ws = pf.Workspace()
    import torch
    t = torch.from_numpy(wl.text).cuda()
    out = torch.empty(16 * 100, dtype=torch.uint8, device="cuda")
    rc, cnt = pf.pfac_scan_sync(trie, ws, t, t.numel(), out, 100)
    assert rc == pf.PFAC_ETRUNC and cnt == want.n
    rc, cnt = pf.pfac_scan_sync(trie, ws, t, t.numel(), None, 0)
    assert rc == pf.PFAC_ETRUNC and cnt == want.n
    # the same workspace then serves a full scan
    got, _ = gpu_scan(trie, wl.text, ws=ws, counts=False, capacity=want.n)
    assert_same(got, want)


def _random_batch(rng, n_texts, max_len, alphabet):
    lens = rng.integers(0, max_len + 1, n_texts)
    lens[rng.integers(0, n_texts, max(1, n_texts // 10))] = 0   # some empty texts
    offs = np.zeros(n_texts + 1, dtype=np.uint64)
    offs[1:] = np.cumsum(lens)
    text = rng.choice(alphabet, int(offs[-1])).astype(np.uint8)
    return text, offs


BATCH_TUNINGS = [dict(kernel=1), dict(kernel=0, bytes_per_lane=8),
                 dict(kernel=1, chunks_per_unit=1, child_check=0, waves_per_wg=4),
                 dict(kernel=1, chunks_per_unit=64, fold_bits=0),
                 dict(kernel=2), dict(kernel=2, chunks_per_unit=1, child_check=0, waves_per_wg=4)]


@pytest.mark.parametrize("seed", range(len(BATCH_TUNINGS)))
def test_batch_matches_oracle_and_plain(seed):
    rng = np.random.default_rng(seed)
    alphabet = np.frombuffer(b"abcd", dtype=np.uint8)
    text, offs = _random_batch(rng, 3000, 700, alphabet)
    pats = [bytes(rng.choice(alphabet, int(rng.integers(2, 9))).astype(np.uint8)) for _ in range(300)]
    trie = pf.Trie(pats)
    trie.set_tuning(**BATCH_TUNINGS[seed])
    say(f"batch seed={seed}: {len(offs) - 1} texts, {offs[-1]} bytes")
    want = oracle.brute(text, pats, offsets=offs, threads=8)
    got, n = gpu_scan_batch(trie, text, offs, pad_front=seed * 5)
    assert n == want.n
    assert_same(got, want, with_text=True)
    got_plain, n2 = gpu_scan_batch(trie, text, offs, plain=True)
    assert n2 == want.n
    assert_same(got_plain, want, with_text=True)


@pytest.mark.parametrize("tuning", BATCH_TUNINGS, ids=_tid)
def test_batch_long_patterns_small_texts(tuning):
    wl = workloads.c4_batched(n_small=3000, n_large=2, large_lo=1 << 15, large_hi=1 << 16,
                              k=3000, rate=1 / 256)
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(**tuning)
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=8)
    say(f"batch long {tuning}: {wl.n_texts} texts, {want.n} matches")
    got, n = gpu_scan_batch(trie, wl.text, wl.offsets, pad_front=3)
    assert n == want.n
    assert_same(got, want, with_text=True)


GRAPH_TUNINGS = {"1": dict(kernel=1), "2": dict(kernel=2), "0": dict(kernel=0),
                 "0t": dict(kernel=0, index_bits=8, top_nodes=1), "0d": dict(kernel=0, trunc_depth=6),
                 "0g": dict(kernel=0, dag=1)}


@pytest.mark.parametrize("kernel", sorted(GRAPH_TUNINGS))
def test_batch_graph_replays_are_identical(kernel):
    rng = np.random.default_rng(9)
    wl = workloads.c4_batched(n_small=2000, n_large=3, large_lo=1 << 16, large_hi=1 << 18,
                              k=2000, rate=1 / 512)
    trie = pf.Trie(wl.patterns)
    trie.set_tuning(**GRAPH_TUNINGS[kernel])
    want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=8)
    say(f"graph: {wl.n_texts} texts {wl.text.size} bytes, {want.n} matches")
    results, n = gpu_scan_batch(trie, wl.text, wl.offsets, graph_replays=4)
    assert n == want.n
    for r in results:
        assert_same(r, want, with_text=True)
    del rng


def test_exhaustive_binary_alphabet_batched():
    """All multisets of <= 3 patterns of length 1..3 over {0,1}, every text of
    length 0..8, one batched launch per pattern set."""
    strs = [bytes(t) for L in range(1, 4) for t in itertools.product(b"\x00\x01", repeat=L)]
    texts = [bytes(t) for L in range(0, 9) for t in itertools.product(b"\x00\x01", repeat=L)]
    offs = np.zeros(len(texts) + 1, dtype=np.uint64)
    offs[1:] = np.cumsum([len(t) for t in texts])
    text = np.frombuffer(b"".join(texts), dtype=np.uint8).copy()
    sets = []
    for r in (1, 2, 3):
        sets.extend(itertools.combinations_with_replacement(range(len(strs)), r))
    assert len(sets) == 679
    ws = pf.Workspace()
    say(f"exhaustive: {len(sets)} pattern sets x {len(texts)} texts")
    for i_set, s in enumerate(sets):
        pats = [strs[i] for i in s]
        trie = pf.Trie(pats)
        trie.set_tuning(kernel=1 + i_set % 2)  # fused and split wave kernels alternate
        got, n = gpu_scan_batch(trie, text, offs, ws=ws, capacity=4096)
        want = oracle.brute(text, pats, offsets=offs)
        assert n == want.n, pats
        assert_same(got, want, with_text=True)
        trie.close()


def test_autotune_keeps_results():
    wl = workloads.c2_signature_set(n_text=4 << 20, k=2000)
    trie = pf.Trie(wl.patterns)
    import torch
    t = torch.from_numpy(wl.text).cuda()
    ws = pf.Workspace()
    best = pf.pfac_autotune(trie, ws, t, t.numel())
    say(f"autotune best: {best}")
    assert best["bytes_per_lane"] in (4, 8, 16)
    got, _ = gpu_scan(trie, wl.text, ws=ws, counts=False)
    want = oracle.bucketed(wl.text, wl.patterns, threads=8)
    assert_same(got, want)


FALLBACKS = {
    # the four-symbol fold table at K = 9 alone is 256 KiB
    "k1_index18": dict(kernel=1, index_bits=18, fold_bits=8),
    # tails and the merged DAG are walked by the tile kernel only
    "k2_trunc8": dict(kernel=2, index_bits=16, fold_bits=8, trunc_depth=8),
    "k2_dag": dict(kernel=2, index_bits=16, fold_bits=8, trunc_depth=0, dag=1),
}


@pytest.mark.parametrize("name", sorted(FALLBACKS) + ["k2_long_pattern"])
def test_wave_tunings_that_cannot_apply(name):
    """Wave-kernel tunings whose kernel cannot run select the tile kernel,
    which must then scan with its own LDS layout: single texts and batches
    against the oracle."""
    rng = np.random.default_rng(61)
    if name == "k2_long_pattern":
        # a pattern over 65,535 bytes: beyond the wave kernels' 16-bit limits
        base = bytes(rng.integers(0, 4, 70_001).astype(np.uint8))
        pats = [base, base[:40], base[5:30], b"\x00\x01\x02"]
        text = np.frombuffer((base * 3)[:180_000], dtype=np.uint8).copy()
        tn = dict(kernel=2)
    else:
        pats = workloads.make_patterns(rng, 3000, 20, 32, "acgt").as_list()
        text = rng.choice(np.frombuffer(b"ACGT", dtype=np.uint8), 300_000).astype(np.uint8)
        for at in rng.integers(0, text.size - 40, 400):
            p = pats[int(rng.integers(0, len(pats)))]
            text[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
        tn = FALLBACKS[name]
    trie = pf.Trie(pats)
    trie.set_tuning(**tn)
    st = trie.stats()
    say(f"fallback {name}: kernel {st['scan_kernel']}, lds {st['lds_bytes']}, K {st['index_depth']}")
    assert st["scan_kernel"] == 0
    want = oracle.bucketed(text, pats, threads=8)
    assert want.n > 0
    got, counts = gpu_scan(trie, text)
    assert_same(got, want)
    assert np.array_equal(counts, oracle.counts(text.size, want))
    offs = np.array([0, 1000, 1000, 77_777, text.size], dtype=np.uint64)
    want_b = oracle.bucketed(text, pats, offsets=offs, threads=8)
    got_b, n = gpu_scan_batch(trie, text, offs)
    assert n == want_b.n
    assert_same(got_b, want_b, with_text=True)


def test_graph_owns_its_scratch_and_pins_the_image():
    """A captured graph keeps replaying correctly while the workspace passed
    at capture serves larger scans (the graph has scratch of its own), and
    the trie's image cannot be rebuilt under it (PFAC_EBUSY) until it is
    freed."""
    import torch
    rng = np.random.default_rng(91)
    pats = workloads.make_patterns(rng, 500, 4, 24, "uniform").as_list()
    small = rng.integers(0, 256, 100_000, dtype=np.uint8)
    for at in rng.integers(0, small.size - 30, 300):
        p = pats[int(rng.integers(0, len(pats)))]
        small[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
    offs = np.array([0, 40_000, 40_000, small.size], dtype=np.uint64)
    want = oracle.bucketed(small, pats, offsets=offs, threads=8)
    trie = pf.Trie(pats)
    ws = pf.Workspace()
    text = torch.from_numpy(small).cuda()
    offs_dev = torch.from_numpy(offs.view(np.int64)).cuda()
    cap = want.n + 64
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    g = pf.Graph(trie, ws, text, offs_dev, 3, small.size, out, cap, cnt, s)
    big = np.tile(small, 80)  # 8 MB: the same workspace grows for it
    want_big = oracle.bucketed(big, pats, threads=8)
    for rep in range(2):
        got_big, _ = gpu_scan(trie, big, ws=ws, counts=False, capacity=want_big.n + 64)
        assert_same(got_big, want_big)
        out.fill_(0xAB)
        torch.cuda.synchronize()
        g.launch(s)
        s.synchronize()
        assert int(cnt.item()) == want.n, rep
        assert_same(pf.matches_to_numpy(out, want.n), want, with_text=True)
    tn = trie.tuning()
    with pytest.raises(pf.PfacError) as e:
        trie.set_tuning(index_bits=8 if tn["index_bits"] != 8 else 16)
    assert e.value.code == pf.PFAC_EBUSY
    trie.set_tuning(kernel=0)  # no rebuild: allowed, the graph keeps its own launch
    g.launch(s)
    s.synchronize()
    assert int(cnt.item()) == want.n
    g.close()
    trie.set_tuning(index_bits=8 if tn["index_bits"] != 8 else 16)  # free to rebuild now
    got, _ = gpu_scan(trie, small[:40_000], counts=False)
    assert_same(got, oracle.bucketed(small[:40_000], pats, threads=8))


def test_graph_records_timing_events_in_every_replay():
    """A graph captured from a workspace with timing events records them
    around its main scan kernel at every replay; pfac_graph_set_timing moves
    later replays to other events; the results stay the oracle's."""
    import torch
    rng = np.random.default_rng(93)
    pats = workloads.make_patterns(rng, 800, 6, 30, "uniform").as_list()
    text = rng.integers(0, 256, 3_000_000, dtype=np.uint8)
    for at in rng.integers(0, text.size - 40, 2000):
        p = pats[int(rng.integers(0, len(pats)))]
        text[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
    offs = np.array([0, 1000, 1_000_000, 1_000_000, text.size], dtype=np.uint64)
    want = oracle.bucketed(text, pats, offsets=offs, threads=8)
    trie = pf.Trie(pats)
    ws = pf.Workspace()
    dev = torch.from_numpy(text).cuda()
    offs_dev = torch.from_numpy(offs.view(np.int64)).cuda()
    cap = want.n + 64
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    s = torch.cuda.Stream()
    ev = [torch.cuda.Event(enable_timing=True) for _ in range(6)]
    for e in ev:
        e.record(s)
    ws.set_timing(ev[0], ev[1])
    g = pf.Graph(trie, ws, dev, offs_dev, 4, text.size, out, cap, cnt, s)
    ws.set_timing(None, None)
    step = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    step[0].record(s)
    for i in range(3):
        g.set_timing(ev[2 * i], ev[2 * i + 1])
        g.launch(s)
        step[i + 1].record(s)
    s.synchronize()
    for i in range(3):
        k = ev[2 * i].elapsed_time(ev[2 * i + 1])
        whole = step[i].elapsed_time(step[i + 1])
        say(f"replay {i}: kernel {k:.4f} ms of {whole:.4f} ms")
        assert 0 < k <= whole
    assert int(cnt.item()) == want.n
    assert_same(pf.matches_to_numpy(out, want.n), want, with_text=True)
    g.close()
    # a graph captured without timing events has no nodes to move
    g2 = pf.Graph(trie, ws, dev, offs_dev, 4, text.size, out, cap, cnt, s)
    with pytest.raises(pf.PfacError) as e:
        g2.set_timing(ev[0], ev[1])
    assert e.value.code == pf.PFAC_EINVAL
    g2.close()
