"""CPU tests of the host side of the library: the CRS builder (against the
oracle's trie definition), footprint arithmetic, C-ABI argument checks and
that every symbol of include/pfac.h is exported.  No GPU call is made."""

import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from synth import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pfac.h")


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(pf._pfac.LIB_PATH):
        from paper_1702_03657_amd import build
        build.build()
    return pf.load()


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\s*\*?\s*(pfac_[a-z_0-9]+)\s*\(", src, flags=re.M)
    return sorted(set(names))


def test_header_symbols_are_exported(lib):
    declared = _declared_functions()
    assert len(declared) >= 20
    out = subprocess.check_output(["nm", "-D", "--defined-only", pf._pfac.LIB_PATH], text=True)
    exported = {line.split()[-1] for line in out.splitlines() if line.strip()}
    missing = [n for n in declared if n not in exported]
    assert not missing, missing
    # and the binding knows every one of them
    assert sorted(n for n, _, _ in pf.SIGNATURES) == declared


@pytest.mark.parametrize("make", [
    lambda: workloads.c1_plain_small(n_text=64, k=100, n_plants=0).patterns.as_list(),
    lambda: workloads.c2_signature_set(n_text=64, k=800).patterns.as_list(),
    lambda: workloads.c3_dna(n_text=64, k=3000, n_plants=0).patterns.as_list(),
    lambda: [b"a", b"ab", b"abc", b"ab", b"b", b"\x00", b"\xff\x00", b"a"],
    lambda: [],
])
def test_builder_equals_canonical_trie(lib, make):
    pats = make()
    t = pf.Trie(pats, host_only=True)
    got = t.export()
    want = oracle.canonical_trie(pats)
    for key in ("row_ptr", "labels", "child", "term_ptr", "term_ids"):
        assert np.array_equal(got[key], want[key]), key
    st = t.stats()
    N = len(want["row_ptr"]) - 1
    fp = oracle.footprint(N, len(pats))
    assert st["nodes"] == N and st["edges"] == max(N - 1, 0)
    assert st["bytes_dense256"] == fp["dense"]
    assert st["bytes_bitmap36"] == fp["bitmap36"]
    assert st["crs_elements"] == fp["crs_elements"]
    assert st["bytes_crs"] == fp["crs_bytes"]
    if pats:
        assert st["max_len"] == max(len(p) for p in pats)
        assert st["min_len"] == min(len(p) for p in pats)
    assert st["bytes_device"] == 0  # host-only build


def test_level_index_choice(lib):
    # full-byte alphabet: K = 2 at 16 bits; DNA: 2-bit symbols, K = 8
    t = pf.Trie(workloads.c1_plain_small(n_text=64, k=100, n_plants=0).patterns, host_only=True)
    s = t.stats()
    assert (s["symbol_bits"], s["index_depth"]) == (8, 2)
    t = pf.Trie(workloads.c3_dna(n_text=64, k=3000, n_plants=0).patterns, host_only=True)
    s = t.stats()
    assert (s["alphabet_size"], s["symbol_bits"], s["index_depth"]) == (4, 2, 8)
    t.set_tuning(index_bits=18)
    assert t.stats()["index_depth"] == 9
    # the index never reaches a pattern end: K <= shortest - 1
    t = pf.Trie([b"abc", b"abcdef"], host_only=True)
    assert t.stats()["index_depth"] == 2
    t = pf.Trie([b"a", b"abcdef"], host_only=True)
    assert t.stats()["index_depth"] == 0


def test_error_codes(lib):
    import ctypes
    h = ctypes.c_void_p()
    data = np.frombuffer(b"abcd", dtype=np.uint8).copy()
    offs = np.array([0, 2, 2, 4], dtype=np.uint64)  # second pattern empty
    rc = lib.pfac_build_packed(data.ctypes.data, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                               3, pf.PFAC_BUILD_HOST_ONLY, ctypes.byref(h))
    assert rc == pf.PFAC_EEMPTY
    assert lib.pfac_build_packed(None, None, 1, pf.PFAC_BUILD_HOST_ONLY, ctypes.byref(h)) == pf.PFAC_EINVAL
    assert lib.pfac_build_packed(data.ctypes.data, offs.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)),
                                 0, 1 << 5, ctypes.byref(h)) == pf.PFAC_EINVAL
    assert lib.pfac_trie_stats(None, None) == pf.PFAC_EINVAL
    lib.pfac_trie_free(None)
    lib.pfac_workspace_free(None)
    lib.pfac_graph_free(None)
    lib.pfac_server_free(None)
    assert lib.pfac_server_cancel(None, 1) == pf.PFAC_EINVAL
    t = pf.Trie([b"abc"], host_only=True)
    # a host-only trie cannot scan
    rc = lib.pfac_scan(t.handle, None, None, 0, None, 0, None, None, None)
    assert rc == pf.PFAC_EINVAL
    with pytest.raises(pf.PfacError):
        t.set_tuning(bytes_per_lane=5)
    assert pf.strerror(pf.PFAC_ETRUNC) == "more matches than capacity"


def test_pattern_pointer_build(lib):
    import ctypes
    pats = [b"he", b"she", b"his", b"hers"]
    bufs = [ctypes.create_string_buffer(p, len(p)) for p in pats]
    ptrs = (ctypes.c_void_p * len(pats))(*[ctypes.addressof(b) for b in bufs])
    lens = (ctypes.c_uint64 * len(pats))(*[len(p) for p in pats])
    h = ctypes.c_void_p()
    assert lib.pfac_build(ptrs, lens, len(pats), pf.PFAC_BUILD_HOST_ONLY, ctypes.byref(h)) == 0
    st = pf._pfac.pfac_stats()
    assert lib.pfac_trie_stats(h, ctypes.byref(st)) == 0
    assert st.nodes == len(oracle.canonical_trie(pats)["row_ptr"]) - 1
    lib.pfac_trie_free(h)


def test_default_launch_and_filters(lib):
    """The build picks the split kernels and the matching filter stages; the
    tuning can switch them."""
    t = pf.Trie(workloads.c2_signature_set(n_text=64, k=2000).patterns, host_only=True)
    s = t.stats()
    assert (s["scan_kernel"], s["stage1"], s["stage2"]) == (2, 1, 2)  # two-byte table, prefix-4
    t.set_tuning(child_check=1)
    assert t.stats()["stage2"] == 1                                 # child labels
    t.set_tuning(fold_bits=0, child_check=0)
    assert (t.stats()["stage1"], t.stats()["stage2"]) == (0, 0)
    t.set_tuning(kernel=0)
    assert t.stats()["scan_kernel"] == 0
    # DNA: 16-symbol filter with its second stage
    t = pf.Trie(workloads.c3_dna(n_text=64, k=3000, n_plants=0).patterns, host_only=True)
    s = t.stats()
    assert (s["scan_kernel"], s["stage1"], s["stage2"]) == (2, 3, 3)
    t.set_tuning(kernel=1)
    assert (t.stats()["scan_kernel"], t.stats()["stage1"]) == (1, 0)  # fused: rolling code
    # patterns shorter than 16 symbols: no 16-symbol filter
    short = [bytes(p) for p in np.random.default_rng(1).choice(list(b"ACGT"), (500, 12)).astype(np.uint8)]
    s = pf.Trie(short, host_only=True).stats()
    assert s["stage1"] != 3
    # patterns shorter than 4 bytes: no prefix-4 filter
    s = pf.Trie([b"abc", b"abcdef", b"xyz"], host_only=True).stats()
    assert s["stage2"] != 2


def test_launch_kernel_by_size(lib):
    """Kernel 3 (the default) resolves by launch size: the tile kernel with 4
    bytes per lane below 1 MiB and 8 below 8 MiB, then the split kernels with
    64-chunk units (fewer when the launch has under two units per resident
    wave of the device's CUs); an explicit kernel is kept at every size."""
    t = pf.Trie(workloads.c2_signature_set(n_text=64, k=2000).patterns, host_only=True)
    assert t.tuning()["kernel"] == 3
    k, tn = t.launch_kernel(64 << 10)
    assert (k, tn["kernel"], tn["bytes_per_lane"]) == (0, 0, 4)
    k, tn = t.launch_kernel((8 << 20) - 1)
    assert (k, tn["kernel"], tn["bytes_per_lane"]) == (0, 0, 8)
    k, tn = t.launch_kernel(8 << 20)
    assert (k, tn["kernel"]) == (2, 2) and 1 <= tn["chunks_per_unit"] <= 64  # by the CU count
    k, tn = t.launch_kernel(4 << 30)
    assert (k, tn["kernel"], tn["chunks_per_unit"]) == (2, 2, 64)
    assert t.stats()["scan_kernel"] == 2               # statistics: large launches
    t.set_tuning(kernel=1)
    assert [t.launch_kernel(n)[0] for n in (1 << 10, 1 << 30)] == [1, 1]
    t.set_tuning(kernel=0)
    assert [t.launch_kernel(n)[0] for n in (1 << 10, 1 << 30)] == [0, 0]
    k = ctypes.c_uint32()
    assert lib.pfac_trie_launch_kernel(None, 1, ctypes.byref(k), None) == pf.PFAC_EINVAL
    assert lib.pfac_trie_launch_kernel(t.handle, 1, None, None) == pf.PFAC_EINVAL


def _balanced_unit_chunks(chunks, waves, gmax):
    """Chunks per unit that spread a wave-kernel launch over the grid's
    waves: units go to the waves one by one, the most loaded wave bounds the
    filter kernel; the largest G whose most loaded wave is within 2% of the
    best G's (retyped here as the host rule the library documents)."""
    m = {}
    for g in range(1, gmax + 1):
        units = -(-chunks // g)
        k = -(-units // waves)
        nk = units - (k - 1) * waves
        last = chunks - (units - 1) * g
        m[g] = (k - 1) * g + last if nk == 1 else k * g
    best = min(m.values())
    return max(g for g in m if m[g] <= best + best // 50)


def test_units_balance_the_grid(lib):
    """Split launches take the chunks per unit that balance the grid's waves
    (a host-only trie counts one CU: 16 waves), never more than the tuning's."""
    t = pf.Trie(workloads.c2_signature_set(n_text=64, k=2000).patterns, host_only=True)
    for total in (8 << 20, (8 << 20) + 12345, 40 << 20, 100 << 20, 1 << 30, 3 << 30):
        chunks = (total + 15 + 1023) // 1024
        _, tn = t.launch_kernel(total)
        assert tn["chunks_per_unit"] == _balanced_unit_chunks(chunks, 16, 64), total
    # worked by hand on 4,096 waves: c4's small texts (39,968 chunks) take one
    # unit of 10 chunks a wave; the 2.2 GiB batch (2,302,146 chunks) 63 (567
    # chunks on the most loaded wave, 576 with 64, 563 at best with 1); a
    # 256 MiB text (262,145 chunks) 64 (65, as with every G)
    assert _balanced_unit_chunks(39968, 4096, 64) == 10
    assert _balanced_unit_chunks(2302146, 4096, 64) == 63
    assert _balanced_unit_chunks(262145, 4096, 64) == 64
    t.set_tuning(kernel=2, chunks_per_unit=8)
    assert t.launch_kernel(1 << 30)[1]["chunks_per_unit"] <= 8


def test_placement_depths_reach_the_requested_level_index():
    """The placement ablation's tunings resolve exactly the requested number
    of trie levels in LDS (0: none), for a byte alphabet and for DNA."""
    from bench import lds_depth_tuning
    from synth import workloads
    for wl, depths in ((workloads.c1_plain_small(n_text=1024), [0, 1, 2]),
                       (workloads.c3_dna(n_text=4096, k=3000, n_plants=10), list(range(10)))):
        t = pf.Trie(wl.patterns, host_only=True)
        st = t.stats()
        got = []
        for d in range(12):
            tn = lds_depth_tuning(st, d)
            if tn is None:
                continue
            t.set_tuning(**tn)
            assert t.stats()["index_depth"] == d
            got.append(d)
        assert got == depths
        t.close()


def test_bitmapped_top_nodes_footprint_and_limits():
    """The bitmapped-node encoding of the first K levels: its size is the
    number of nodes of depth < K times (bitmap words + first child), the
    narrow bitmapped footprint uses the alphabet's bits, and a tuning whose
    top nodes would not fit in LDS is refused without changing the trie."""
    from synth import workloads
    wl = workloads.c1_plain_small(n_text=1024)
    pats = wl.patterns.as_list()
    t = pf.Trie(pats, host_only=True)
    for bits, K in ((8, 1), (16, 2)):
        t.set_tuning(kernel=0, index_bits=bits, top_nodes=1)
        st = t.stats()
        assert st["index_depth"] == K
        upper = 1 + len({p[:d] for p in pats for d in range(1, K)})  # nodes of depth < K
        assert st["bytes_top_nodes"] == upper * 9 * 4
        assert st["bytes_level_index"] == 8 * ((1 << (8 * K)) // 32)
        assert st["bytes_bitmap_narrow"] == 36 * st["nodes"] == st["bytes_bitmap36"]
    t.close()

    dna = workloads.c3_dna(n_text=4096, k=30_000, n_plants=10)
    pats = dna.patterns.as_list()
    t = pf.Trie(pats, host_only=True)
    st = t.stats()
    assert st["bytes_bitmap_narrow"] == 5 * st["nodes"]  # 4-bit bitmap in one byte + 4
    t.set_tuning(kernel=0, index_bits=12, top_nodes=1)  # K = 6, two words per node
    st = t.stats()
    upper = 1 + len({p[:d] for p in pats for d in range(1, 6)})
    assert st["index_depth"] == 6 and st["bytes_top_nodes"] == upper * 8
    before = t.tuning()
    with pytest.raises(pf.PfacError):
        t.set_tuning(index_bits=18)  # K = 9: ~39,000 nodes x 8 bytes do not fit
    assert t.tuning() == before and t.stats()["index_depth"] == 6
    t.close()


def test_truncated_image_sizes():
    """A truncated image keeps the nodes of depths 0..D and, per distinct
    pattern longer than D, one 16-byte tail entry and its bytes after D;
    depths at or past the deepest node leave the whole trie, and the scan
    falls back to the tile kernel."""
    pats = [b"he", b"she", b"his", b"hers", b"hers", b"abcdefgh", b"abcdxyz", b"a"]
    t = pf.Trie(pats, host_only=True)
    full = t.stats()
    assert full["trunc_depth"] == 0 and full["bytes_tails"] == 40
    assert full["bytes_nodes"] == 16 * full["nodes"]
    distinct = set(pats)
    for D in range(1, 9):
        t.set_tuning(trunc_depth=D)
        st = t.stats()
        deeper = [p for p in distinct if len(p) > D]
        if max(len(p) for p in pats) <= D:
            assert st["trunc_depth"] == 0 and st["bytes_nodes"] == full["bytes_nodes"]
            continue
        kept = 1 + len({p[:d] for p in pats for d in range(1, min(len(p), D) + 1)})
        assert st["trunc_depth"] == D and st["scan_kernel"] == 0
        assert st["index_depth"] <= D
        assert st["bytes_nodes"] == 16 * kept
        assert st["bytes_tails"] == 16 * len(deeper) + sum(len(p) - D for p in deeper) + 40
    t.set_tuning(trunc_depth=0)
    assert t.stats()["bytes_nodes"] == full["bytes_nodes"]
    with pytest.raises(pf.PfacError):
        t.set_tuning(trunc_depth=256)
    t.close()


def _dag_size_reference(pats):
    """Nodes and edges of the trie with equal subtries merged, from a plain
    dict trie: a subtrie is named by (terminal?, sorted (label, child name))."""
    root = {}
    for p in pats:
        node = root
        for c in p:
            node = node.setdefault(c, {})
        node[None] = True
    names = {}

    def name(node):
        key = (None in node, tuple((c, name(ch)) for c, ch in sorted(
            (c, ch) for c, ch in node.items() if c is not None)))
        return names.setdefault(key, len(names))

    name(root)
    return len(names), sum(len(k[1]) for k in names)


def test_merged_dag_sizes():
    """Suffix and end-node merging: closed forms (all strings of length L over
    s symbols: L + 1 nodes, s * L edges; a single pattern stays a chain) and a
    dict-trie reference on random sets with shared suffixes and duplicates."""
    import itertools
    pats = [bytes(t) for t in itertools.product(b"ACGT", repeat=5)]
    st = pf.Trie(pats, host_only=True).stats()
    assert st["nodes"] == sum(4 ** d for d in range(6))
    assert (st["dag_nodes"], st["dag_edges"]) == (6, 4 * 5)
    st = pf.Trie([b"abcdef"], host_only=True).stats()
    assert (st["dag_nodes"], st["dag_edges"]) == (7, 6)
    rng = np.random.default_rng(11)
    for trial in range(5):
        suf = [bytes(rng.integers(97, 100, int(n)).astype(np.uint8)) for n in rng.integers(1, 6, 20)]
        pats = [bytes(rng.integers(97, 101, int(n)).astype(np.uint8)) + suf[int(rng.integers(0, 20))]
                for n in rng.integers(0, 6, 300)]
        pats += pats[:10]  # duplicates
        st = pf.Trie(pats, host_only=True).stats()
        assert (st["dag_nodes"], st["dag_edges"]) == _dag_size_reference(pats), trial
        assert st["bytes_dag_crs"] == 8 * (st["dag_nodes"] + 1) + 9 * st["dag_edges"] + 4 * len(pats)
    t = pf.Trie([b"ab", b"cb"], host_only=True)
    with pytest.raises(pf.PfacError):
        t.set_tuning(dag=1, top_nodes=1)
    with pytest.raises(pf.PfacError):
        t.set_tuning(dag=1, trunc_depth=1)
    t.set_tuning(dag=1)
    assert t.stats()["scan_kernel"] == 0
    t.close()


def test_host_allocation_failure_reports_enomem():
    """An allocation the host cannot satisfy fails the build with PFAC_ENOMEM
    and the library keeps working: a child process caps its address space a
    little above its current size, builds a trie that needs more (300,000
    patterns, about 12 M nodes), then a small one."""
    import sys
    script = r'''
import resource, sys
sys.path.insert(0, sys.argv[1])
import ctypes

import numpy as np
import paper_1702_03657_amd as pf
from synth import workloads
pats = workloads.make_patterns(np.random.default_rng(3), 300_000, 24, 64, "uniform")
size = [int(l.split()[1]) * 1024 for l in open("/proc/self/status") if l.startswith("VmSize:")][0]
cap = size + (256 << 20)
resource.setrlimit(resource.RLIMIT_AS, (cap, cap))
try:
    pf.Trie(pats, host_only=True)
    print("no failure")
except pf.PfacError as e:
    print("code", e.code)
print("small", pf.Trie([b"abc", b"bcd"], host_only=True).stats()["nodes"])
'''
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    run = subprocess.run([sys.executable, "-c", script, root], capture_output=True, text=True,
                         timeout=300)
    assert run.returncode == 0, run.stderr[-2000:]
    assert f"code {pf.PFAC_ENOMEM}" in run.stdout, run.stdout
    assert "small 7" in run.stdout, run.stdout


FALLBACK_TUNINGS = [
    # the four-symbol fold table at K = 9 alone is 256 KiB
    dict(kernel=1, index_bits=18, fold_bits=8),
    # tails and the merged DAG are walked by the tile kernel only
    dict(kernel=2, index_bits=16, fold_bits=8, trunc_depth=8),
    dict(kernel=2, index_bits=16, fold_bits=8, trunc_depth=0, dag=1),
]


def test_wave_tunings_that_cannot_apply_run_the_tile_kernel():
    """A wave-kernel tuning whose kernel cannot run (tables too large for
    LDS, a truncated or merged image, a pattern over 65,535 bytes) selects
    the tile kernel with the tile kernel's own LDS layout, within the limit."""
    pats = workloads.make_patterns(np.random.default_rng(4), 2000, 20, 32, "acgt")
    t = pf.Trie(pats, host_only=True)
    for tn in FALLBACK_TUNINGS:
        t.set_tuning(**tn)
        st = t.stats()
        assert st["scan_kernel"] == 0 and 0 < st["lds_bytes"] <= 160 * 1024, (tn, st["lds_bytes"])
    t.set_tuning(kernel=2, trunc_depth=0, dag=0)
    assert t.stats()["scan_kernel"] == 2
    long = pf.Trie([b"ab" * 35_000, b"abc"], host_only=True)
    long.set_tuning(kernel=2)
    st = long.stats()
    assert st["scan_kernel"] == 0 and st["lds_bytes"] <= 160 * 1024
