"""Pins for the CPU oracle: it is checked against things other than itself.

* a worked example printed by the Aho-Corasick paper (tests/golden);
* agreement of three different algorithms (literal definition, bucketed
  definition, textbook Aho-Corasick) on every case of tiny alphabets;
* closed forms: one pattern reduces to repeated ``bytes.find``; length-1
  patterns to set membership; all strings of length L give one match at every
  position that fits; {a, aa, ..., a^L} over a^n gives min(L, n - i);
* planted copies that survived later overwrites must be found;
* the trie definition against an independent insertion-built trie, its
  invariants, and the CRS storage identity 2 nnz + n + 1.
"""

import itertools
import os

import numpy as np
import pytest
from hypothesis import given, settings, strategies as st

import oracle
from synth import PatternSet, workloads

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ALGOS = [oracle.brute, oracle.bucketed, oracle.aho_corasick]


def _read_golden(name):
    pats, text, rows = None, None, []
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            if line.startswith("patterns:"):
                pats = [w.encode() for w in line.split(":", 1)[1].split()]
            elif line.startswith("text:"):
                text = line.split(":", 1)[1].strip().encode()
            else:
                a, b = line.split()
                rows.append((int(a), int(b)))
    return pats, text, rows


@pytest.mark.parametrize("algo", ALGOS)
def test_golden_aho_corasick_example(oracle_lib, algo):
    pats, text, rows = _read_golden("ac1975_ushers.txt")
    assert algo(text, pats).pairs() == rows


def test_exhaustive_binary(oracle_lib):
    bad, cases = oracle.exhaustive(2, 3, 3, 8, threads=8)
    n_sets = 14 + 14 * 15 // 2 + 14 * 15 * 16 // 6   # multisets of 1..3 of 14 strings
    assert cases == n_sets * (2 ** 9 - 1)
    assert bad == 0


def test_exhaustive_ternary(oracle_lib):
    # all multisets of <= 2 strings of length 1..3 over {0,1,2}; texts <= 7
    bad, cases = oracle.exhaustive(3, 3, 2, 7, threads=8)
    n_strs = 3 + 9 + 27
    n_sets = n_strs + n_strs * (n_strs + 1) // 2
    assert cases == n_sets * sum(3 ** L for L in range(8))
    assert bad == 0


def test_single_pattern_is_repeated_find(oracle_lib):
    rng = np.random.default_rng(5)
    for trial in range(40):
        sigma = int(rng.integers(1, 4))
        text = bytes(rng.integers(0, sigma, int(rng.integers(0, 300))).astype(np.uint8))
        pat = bytes(rng.integers(0, sigma, int(rng.integers(1, 6))).astype(np.uint8))
        want, i = [], text.find(pat)
        while i >= 0:
            want.append((i, 0))
            i = text.find(pat, i + 1)
        for algo in ALGOS:
            assert algo(text, [pat]).pairs() == want


def test_length_one_patterns_are_membership(oracle_lib):
    rng = np.random.default_rng(6)
    text = rng.integers(0, 256, 5000).astype(np.uint8)
    alphabet = rng.choice(256, 40, replace=False).astype(np.uint8)
    pats = [bytes([int(c)]) for c in alphabet]
    pos_of = {int(c): j for j, c in enumerate(alphabet)}
    want = [(i, pos_of[int(c)]) for i, c in enumerate(text.tolist()) if int(c) in pos_of]
    for algo in ALGOS:
        assert algo(text, pats).pairs() == want


@pytest.mark.parametrize("L", [1, 2, 3])
def test_all_strings_of_length_L(oracle_lib, L):
    sigma = 3
    pats = [bytes(t) for t in itertools.product(range(sigma), repeat=L)]
    rng = np.random.default_rng(L)
    n = 400
    text = rng.integers(0, sigma, n).astype(np.uint8)
    for algo in ALGOS:
        m = algo(text, pats)
        c = oracle.counts(n, m)
        assert np.all(c[:n - L + 1] == 1) and np.all(c[n - L + 1:] == 0)
        # and the id is the base-sigma value of the window
        for i, j in m.pairs():
            assert pats[j] == text[i:i + L].tobytes()


def test_nested_runs(oracle_lib):
    L, n = 7, 50
    pats = [b"a" * d for d in range(1, L + 1)]
    text = b"a" * n
    for algo in ALGOS:
        c = oracle.counts(n, algo(text, pats))
        assert c.tolist() == [min(L, n - i) for i in range(n)]


def test_duplicates_report_every_id(oracle_lib):
    pats = [b"ab", b"xyz", b"ab", b"b", b"ab"]
    text = b"zabxyzab"
    want = [(1, 0), (1, 2), (1, 4), (2, 3), (3, 1), (6, 0), (6, 2), (6, 4), (7, 3)]
    for algo in ALGOS:
        assert algo(text, pats).pairs() == want


def test_edge_cases(oracle_lib):
    for algo in ALGOS:
        assert algo(b"", [b"a"]).n == 0              # empty text
        assert algo(b"abc", []).n == 0               # no patterns
        assert algo(b"ab", [b"abc"]).n == 0          # text shorter than the pattern
        assert algo(b"abc", [b"abc"]).pairs() == [(0, 0)]
        assert algo(b"\x00\xff\x00", [b"\xff\x00", b"\x00"]).pairs() == [(0, 1), (1, 0), (2, 1)]
    with pytest.raises(ValueError):
        oracle.brute(b"abc", [b""])


def test_no_match_crosses_a_text_boundary(oracle_lib):
    text = b"abcdxbcd"
    offs = np.array([0, 2, 2, 5, 8], dtype=np.uint64)   # "ab" | "" | "cdx" | "bcd"
    for algo in ALGOS:
        m = algo(text, [b"bc", b"cd", b"b"], offsets=offs)
        got = sorted(m.triples())
        assert got == [(0, 1, 2), (2, 0, 1), (3, 0, 0), (3, 0, 2), (3, 1, 1)]
        assert m.triples() == got


@settings(max_examples=60, deadline=None)
@given(st.integers(1, 3), st.lists(st.binary(min_size=1, max_size=6), min_size=0, max_size=12),
       st.binary(min_size=0, max_size=400), st.integers(0, 2 ** 31))
def test_three_algorithms_agree(oracle_lib, sigma, raw_pats, raw_text, seed):
    # squash bytes into a small alphabet so that matches are frequent
    pats = [bytes(b % (sigma + 1) for b in p) for p in raw_pats]
    text = bytes(b % (sigma + 1) for b in raw_text)
    a = oracle.brute(text, pats)
    for algo in (oracle.bucketed, oracle.aho_corasick):
        assert algo(text, pats).pairs() == a.pairs()
    # windows and threading do not change the set
    lo = seed % (len(text) + 1)
    hi = lo + (seed // 7) % (len(text) + 1)
    w = oracle.aho_corasick(text, pats, lo=lo, hi=hi, threads=3, chunk=17)
    assert w.pairs() == [(i, j) for i, j in a.pairs() if lo <= i < hi]


def test_threads_and_chunks_do_not_change_results(oracle_lib):
    wl = workloads.c1_plain_small(n_text=1 << 16, k=60, n_plants=300)
    ref = oracle.brute(wl.text, wl.patterns)
    for algo in ALGOS:
        for threads, chunk in [(1, 0), (4, 1000), (8, 4096)]:
            m = algo(wl.text, wl.patterns, threads=threads, chunk=chunk)
            assert m.pairs() == ref.pairs()


@pytest.mark.parametrize("make", [
    lambda: workloads.c1_plain_small(n_text=1 << 17, k=100, n_plants=500),
    lambda: workloads.c2_signature_set(n_text=1 << 18, k=500, mean_gap=512),
    lambda: workloads.c3_dna(n_text=1 << 18, k=2000, n_plants=300),
    lambda: workloads.c4_batched(n_small=300, n_large=2, large_lo=1 << 14, large_hi=1 << 15,
                                 k=400, rate=1 / 1024),
])
def test_planted_copies_are_found(oracle_lib, make):
    wl = make()
    m = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=4)
    found = set(m.triples())
    survived = 0
    for tid, pos, j in wl.plants.tolist():
        t = wl.text_of(tid)
        if t[pos:pos + len(wl.patterns[j])].tobytes() == wl.patterns[j]:
            assert (tid, pos, j) in found
            survived += 1
    assert survived > 0.9 * len(wl.plants)
    # every reported match verifies byte for byte, and the three algorithms agree
    for tid, pos, j in list(found)[:2000]:
        assert wl.text_of(tid)[pos:pos + len(wl.patterns[j])].tobytes() == wl.patterns[j]
    ac = oracle.aho_corasick(wl.text, wl.patterns, offsets=wl.offsets, threads=4)
    assert ac.triples() == m.triples()


def test_brute_equals_bucketed_on_config_windows(oracle_lib):
    wl = workloads.c2_signature_set(n_text=1 << 20, k=2000, mean_gap=1024)
    for lo in (0, 300_000, (1 << 20) - 5000):
        a = oracle.brute(wl.text, wl.patterns, lo=lo, hi=lo + 5000)
        b = oracle.bucketed(wl.text, wl.patterns, lo=lo, hi=lo + 5000)
        assert a.pairs() == b.pairs()


# ------------------------------------------------------------------- trie


def _naive_trie(pats):
    """Independent construction: insert into nested dicts, then BFS."""
    root = {}
    ends = {}
    for j, p in enumerate(pats):
        node = root
        for c in p:
            node = node.setdefault(c, {})
        ends.setdefault(id(node), []).append(j)
    order, queue = [], [root]
    while queue:
        nxt = []
        for node in queue:
            order.append(node)
            for c in sorted(node):
                nxt.append(node[c])
        queue = nxt
    idx = {id(n): v for v, n in enumerate(order)}
    row_ptr, labels, child, term_ptr, term_ids = [0], [], [], [0], []
    for node in order:
        for c in sorted(node):
            labels.append(c)
            child.append(idx[id(node[c])])
        row_ptr.append(len(labels))
        term_ids.extend(sorted(ends.get(id(node), [])))
        term_ptr.append(len(term_ids))
    return row_ptr, labels, child, term_ptr, term_ids


@pytest.mark.parametrize("seed", range(6))
def test_canonical_trie_matches_insertion_trie(seed):
    rng = np.random.default_rng(seed)
    sigma = [2, 4, 256][seed % 3]
    k = int(rng.integers(0, 60))
    pats = [bytes(rng.integers(0, sigma, int(rng.integers(1, 9))).astype(np.uint8))
            for _ in range(k)]
    if k > 3:
        pats[1] = pats[0]                 # a duplicate
        pats[2] = pats[0][:max(1, len(pats[0]) - 1)]   # a prefix of another
    t = oracle.canonical_trie(pats)
    row_ptr, labels, child, term_ptr, term_ids = _naive_trie(pats)
    assert t["row_ptr"].tolist() == row_ptr
    assert t["labels"].tolist() == labels
    assert t["child"].tolist() == child
    assert t["term_ptr"].tolist() == term_ptr
    assert t["term_ids"].tolist() == term_ids


def test_canonical_trie_invariants():
    wl = workloads.c1_plain_small(n_text=1024, k=300, n_plants=0)
    pats = wl.patterns.as_list() + [b"\x00", b"\x00\x01"]
    t = oracle.canonical_trie(pats)
    N = len(t["row_ptr"]) - 1
    nnz = len(t["labels"])
    prefixes = {p[:d] for p in pats for d in range(1, len(p) + 1)}
    assert N == len(prefixes) + 1 and nnz == N - 1
    rp = t["row_ptr"].astype(np.int64)
    assert rp[0] == 0 and rp[-1] == nnz and np.all(np.diff(rp) >= 0)
    assert t["child"].tolist() == list(range(1, N))          # BFS numbering
    for v in range(N):
        lab = t["labels"][rp[v]:rp[v + 1]].astype(int)
        assert np.all(np.diff(lab) > 0)
    assert t["term_ptr"][-1] == len(pats)
    assert sorted(t["term_ids"].tolist()) == list(range(len(pats)))
    # CRS storage of Design and Implementation: 2 nnz + n + 1 elements
    fp = oracle.footprint(N, len(pats))
    assert fp["crs_elements"] == len(t["row_ptr"]) + len(t["labels"]) + len(t["child"])
    assert fp["dense"] == 256 * 4 * N and fp["bitmap36"] == (256 // 8 + 4) * N


def _footprint_sets():
    dna = workloads.make_patterns(workloads.rng_for(300), 400, 20, 32, "acgt").as_list()
    uni = workloads.make_patterns(workloads.rng_for(301), 300, 4, 16, "uniform").as_list()
    return {
        "empty": [],
        "duplicates": [b"abc", b"abc", b"abc", b"x"],
        "nested prefixes": [b"a", b"ab", b"abc", b"abcd", b"b", b"bc"],
        "c1-like": uni,
        "c3-like": dna,
    }


@pytest.mark.parametrize("name", list(_footprint_sets()))
def test_footprint_is_the_size_of_the_structures(name):
    """Design and Implementation (CRS paragraph; Results, 36-byte node):
    each footprint figure equals the byte size of that structure, built out
    of the trie and checked to encode it, not a restated formula."""
    pats = _footprint_sets()[name]
    t = oracle.canonical_trie(pats)
    N, k = len(t["row_ptr"]) - 1, len(pats)
    fp = oracle.footprint(N, k)
    stored = ("row_ptr", "labels", "child", "term_ptr", "term_ids")
    assert fp["crs_bytes"] == sum(t[a].nbytes for a in stored)
    assert fp["crs_elements"] == t["row_ptr"].size + t["labels"].size + t["child"].size
    rp = t["row_ptr"].astype(np.int64)
    parent = np.repeat(np.arange(N), np.diff(rp))
    # the uncompressed node x symbol table (step VI): one int32 per symbol
    dense = np.full((N, 256), -1, dtype=np.int32)
    dense[parent, t["labels"]] = t["child"]
    assert fp["dense"] == dense.nbytes
    assert np.count_nonzero(dense >= 0) == t["labels"].size
    # bitmapped nodes: a 256-bit child bitmap and the first child's index;
    # every child is the first child plus the set bits below its label
    node_t = np.dtype([("bitmap", "<u4", (8,)), ("first", "<u4")])
    nodes = np.zeros(N, dtype=node_t)
    lab = t["labels"].astype(np.int64)
    np.bitwise_or.at(nodes["bitmap"], (parent, lab >> 5),
                     (np.uint32(1) << (lab & 31).astype(np.uint32)))
    has = np.diff(rp) > 0
    nodes["first"][has] = t["child"][rp[:-1][has]]
    assert fp["bitmap36"] == nodes.nbytes
    for e in range(t["labels"].size):
        v, c = parent[e], int(lab[e])
        words = nodes["bitmap"][v]
        below = sum(bin(int(words[i])).count("1") for i in range(c >> 5))
        below += bin(int(words[c >> 5]) & ((1 << (c & 31)) - 1)).count("1")
        assert nodes["first"][v] + below == t["child"][e]


def test_patternset_roundtrip():
    pats = [b"abc", b"\x00", b"zz" * 10]
    ps = PatternSet.from_list(pats)
    assert ps.as_list() == pats and len(ps) == 3
