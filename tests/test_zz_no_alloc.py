"""pfac_scan_noalloc (scratch in the library's per-device array, nothing
allocated) against pfac_scan (workspace scratch) and the oracle, through the
C ABI: two calls in a row, the second on a smaller text, and a text whose
scratch would not fit."""

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from synth import workloads
from tests.gpu_util import assert_same, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _both(trie, text, cap):
    """(matches, counts) of pfac_scan_noalloc and of pfac_scan on the same
    device text, each with its own output buffers."""
    import torch
    n = len(text)
    dev = torch.zeros(n + 16, dtype=torch.uint8, device="cuda")
    dev[3:3 + n] = torch.from_numpy(text)   # misaligned on purpose
    t = dev[3:3 + n]
    res = []
    for which in ("noalloc", "scan"):
        out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        counts = torch.full((n,), 7, dtype=torch.int32, device="cuda")
        s = torch.cuda.current_stream()
        if which == "noalloc":
            pf.pfac_scan_noalloc(trie, t, n, out, cap, cnt, counts, s)
        else:
            pf.pfac_scan(trie, pf.Workspace(), t, n, out, cap, cnt, counts, s)
        torch.cuda.synchronize()
        k = int(cnt.item())
        assert k <= cap
        res.append((pf.matches_to_numpy(out, k), counts.cpu().numpy().view(np.uint32)))
    return res


@pytest.mark.parametrize("kernel", [2, 1, 0])
def test_noalloc_matches_pfac_scan_twice(kernel):
    rng = np.random.default_rng(7 + kernel)
    pats = workloads.make_patterns(rng, 2000, 8, 40, "mix").as_list()
    trie = pf.Trie(pats)
    trie.set_tuning(kernel=kernel)
    for n in (3_000_001, 777_777):   # the second call smaller than the first
        text = rng.integers(32, 127, n, dtype=np.uint8)
        for at in rng.integers(0, n - 64, n // 2048):
            p = pats[int(rng.integers(0, len(pats)))]
            text[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
        want = oracle.bucketed(text, pats, threads=8)
        say(f"noalloc kernel {kernel}: {n} bytes, {want.n} matches")
        (m0, c0), (m1, c1) = _both(trie, text, want.n + 100)
        assert_same(m0, want)
        assert_same(m1, want)
        assert np.array_equal(c0, c1)
        assert np.array_equal(c0, oracle.counts(n, want))


def test_noalloc_refuses_scratch_beyond_its_array():
    import torch
    pats = [b"abcdefgh", b"bcdefghi"]
    trie = pf.Trie(pats)
    buf = torch.zeros(64, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    # far past the array: refused before anything reaches the device
    with pytest.raises(pf.PfacError) as e:
        pf.pfac_scan_noalloc(trie, buf, 1 << 40, buf, 0, cnt)
    assert e.value.code == pf.PFAC_EINVAL
    with pytest.raises(pf.PfacError) as e:
        pf.pfac_scan_noalloc(trie, buf, 16, buf, 1 << 30, cnt)
    assert e.value.code == pf.PFAC_EINVAL
    # and the next call works
    text = np.frombuffer(b"xxabcdefghixx", dtype=np.uint8).copy()
    dev = torch.from_numpy(text).cuda()
    out = torch.empty(16 * 16, dtype=torch.uint8, device="cuda")
    pf.pfac_scan_noalloc(trie, dev, text.size, out, 16, cnt)
    torch.cuda.synchronize()
    got = pf.matches_to_numpy(out, int(cnt.item()))
    assert got["pos"].tolist() == [2, 3] and got["pattern_id"].tolist() == [0, 1]
