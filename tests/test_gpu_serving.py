"""GPU tests of the serving loop (pfac_server_*): every request's result is
the same as the oracle's for that text alone and as a scan of it alone on the
GPU, whatever the mix it was batched with, the ring wrap-around, the budget,
the overflow fallback and the cancellation of other requests."""

import math

import numpy as np
import pytest

import oracle
import paper_1702_03657_amd as pf
from synth import workloads
from tests.gpu_util import assert_same, gpu_scan, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    # torch takes the device first, then the library
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    pf.load()


def _requests(seed, n, lo, hi, pats, rate=1 / 1024):
    """Seeded request texts of log-uniform sizes with planted pattern copies."""
    rng = np.random.default_rng(seed)
    sizes = np.floor(np.exp(rng.uniform(math.log(lo), math.log(hi), n))).astype(np.int64)
    texts = []
    for s in sizes:
        t = rng.integers(0, 256, int(s), dtype=np.uint8)
        for _ in range(rng.poisson(s * rate)):
            p = pats[int(rng.integers(0, len(pats)))]
            if len(p) <= s:
                at = int(rng.integers(0, s - len(p) + 1))
                t[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
        texts.append(t)
    return texts


def _server(trie, budget, arena, max_batch):
    import torch
    buf = torch.empty(arena, dtype=torch.uint8, device="cuda")
    cs, xs = torch.cuda.Stream(), torch.cuda.Stream()
    return pf.Server(trie, buf, budget, max_batch, cs, xs), buf


SERVER_TUNINGS = {"1": dict(kernel=1), "2": dict(kernel=2), "0d": dict(kernel=0, trunc_depth=8),
                  "0g": dict(kernel=0, dag=1)}


@pytest.mark.parametrize("kernel", sorted(SERVER_TUNINGS))
def test_mix_equals_alone(kernel):
    pats = workloads.make_patterns(np.random.default_rng(5), 2000, 8, 64, "uniform")
    texts = _requests(11, 48, 1024, 512 * 1024, pats)
    trie = pf.Trie(pats)
    trie.set_tuning(**SERVER_TUNINGS[kernel])
    budget = 2 << 20  # smaller than the sum: several batches and ring wrap-around
    srv, _buf = _server(trie, budget, budget + (16 << 20), 16)
    say(f"server kernel {kernel}: {len(texts)} requests, {sum(t.size for t in texts)} bytes")
    ids = [srv.submit(t) for t in texts]
    lat = []
    for t, rid in zip(texts, ids):
        got, l = srv.wait(rid, capacity=1 << 16)
        lat.append(l)
        want = oracle.bucketed(t, pats, threads=8)
        assert_same(got, want)
        alone, _ = gpu_scan(trie, t, counts=False)
        assert np.array_equal(got, alone)
    st = srv.stats()
    say(f"stats {st}, latency max {max(lat):.4f}s")
    assert st["requests"] == len(texts)
    assert st["batches"] > 1 and st["batches"] < len(texts)  # batched, more than once
    srv.close()


def test_overflow_falls_back_to_single_scans():
    # dense matches overflow the small per-batch output: each request is then
    # scanned alone with an exact-size buffer
    pats = [b"aa", b"aaa", b"ab"]
    rng = np.random.default_rng(3)
    texts = [np.frombuffer((b"a" * int(n)) + b"b", dtype=np.uint8).copy()
             for n in rng.integers(2000, 9000, 6)]
    trie = pf.Trie(pats)
    budget = 1 << 20
    srv, _buf = _server(trie, budget, budget + (256 << 10), 8)
    ids = [srv.submit(t) for t in texts]
    for t, rid in zip(texts, ids):
        got, _ = srv.wait(rid, capacity=1 << 16)
        assert_same(got, oracle.brute(t, pats))
    srv.close()


def test_empty_request_and_limits():
    pats = [b"abc", b"bcd"]
    trie = pf.Trie(pats)
    budget = 1 << 16
    srv, _buf = _server(trie, budget, budget + (1 << 20), 4)
    rid = srv.submit(np.zeros(0, dtype=np.uint8))
    got, _ = srv.wait(rid)
    assert got.size == 0
    with pytest.raises(pf.PfacError):
        srv.submit(np.zeros(budget + 1, dtype=np.uint8))  # larger than the ring
    t = np.frombuffer(b"xxabcdxx" * 100, dtype=np.uint8).copy()
    rid = srv.submit(t)
    with pytest.raises(pf.PfacError):
        srv.wait(rid, capacity=4)  # more matches than the caller's buffer
    rid = srv.submit(t)
    got, _ = srv.wait(rid, capacity=1024)
    assert_same(got, oracle.brute(t, pats))
    srv.close()


def test_allocation_failure_leaves_the_workspace_usable():
    """A reservation the device cannot hold fails with PFAC_ENOMEM (the
    allocator's refusal, forced from the host with an impossible size) and the
    same workspace then scans normally."""
    pats = [b"abc", b"bcd", b"cd"]
    trie = pf.Trie(pats)
    ws = pf.Workspace()
    # 1 TiB of staging (beyond the device), and sizes refused before any allocation
    for max_bytes, max_matches in ((1 << 20, 1 << 36), (1 << 62, 1), (1 << 20, 1 << 62)):
        with pytest.raises(pf.PfacError) as e:
            ws.reserve(max_bytes, 1, max_matches)
        assert e.value.code == pf.PFAC_ENOMEM
    t = np.frombuffer(b"xabcdx" * 1000, dtype=np.uint8).copy()
    got, _ = gpu_scan(trie, t, ws=ws)
    assert_same(got, oracle.brute(t, pats))


def test_cancel_leaves_the_rest_exact():
    """Requests cancelled while queued behind a text that holds the whole
    budget, while in flight and after completion: their ids are released,
    every other request gets the oracle's matches, and the server keeps
    serving with a consistent ring."""
    pats = workloads.make_patterns(np.random.default_rng(7), 500, 6, 32, "uniform")
    budget = 16 << 20
    rng = np.random.default_rng(23)
    big = rng.integers(0, 256, budget, dtype=np.uint8)
    for at in rng.integers(0, budget - 64, 200):
        p = pats[int(rng.integers(0, len(pats)))]
        big[at:at + len(p)] = np.frombuffer(p, dtype=np.uint8)
    small = _requests(22, 30, 4096, 256 * 1024, pats)
    trie = pf.Trie(pats)
    srv, _buf = _server(trie, budget, budget + (16 << 20), 8)
    texts = {srv.submit(big): big}
    first = srv.submit(small[0])
    srv.cancel(first)  # the big text holds the whole budget: still queued
    ids = [srv.submit(t) for t in small[1:]]
    texts.update(zip(ids, small[1:]))
    cancelled = [first] + ids[2::3]
    for rid in cancelled[1:]:
        srv.cancel(rid)
        del texts[rid]
    # one waited for with a zero timeout first (pending behind the big text), then cancelled
    late = srv.submit(big)
    try:
        srv.wait(late, timeout_ms=0)
    except pf.PfacError as e:
        assert e.code == pf.PFAC_EBUSY
        srv.cancel(late)
    cancelled.append(late)
    say(f"cancel: {len(texts)} kept, {len(cancelled)} cancelled")
    for rid, t in texts.items():
        got, _ = srv.wait(rid, capacity=1 << 16)
        assert_same(got, oracle.bucketed(t, pats, threads=8))
    # requests never scanned are not counted
    assert srv.stats()["requests"] < len(texts) + len(cancelled)
    for rid in cancelled:
        for call in (srv.wait, srv.cancel):
            with pytest.raises(pf.PfacError) as e:
                call(rid)
            assert e.value.code == pf.PFAC_EINVAL
    done = srv.submit(small[1])
    import time
    time.sleep(0.2)
    srv.cancel(done)  # completed and never waited for: the matches are dropped
    # the ring is consistent: a second pass over every small text is exact
    again = [srv.submit(t) for t in small]
    for rid, t in zip(again, small):
        got, _ = srv.wait(rid, capacity=1 << 16)
        assert_same(got, oracle.bucketed(t, pats, threads=8))
    srv.close()


def test_random_submit_wait_cancel():
    """A seeded random mix of submits, zero-timeout waits, waits and cancels
    over a small ring: every request that is waited for gets the oracle's
    matches, whatever was cancelled around it and in whatever state."""
    pats = workloads.make_patterns(np.random.default_rng(8), 300, 4, 24, "uniform")
    texts = _requests(31, 120, 256, 96 * 1024, pats, rate=1 / 256)
    trie = pf.Trie(pats)
    budget = 256 << 10
    srv, _buf = _server(trie, budget, budget + (8 << 20), 6)
    rng = np.random.default_rng(41)
    pending = {}  # id -> text index
    n_checked = n_cancelled = 0
    for i, t in enumerate(texts):
        pending[srv.submit(t)] = i
        for _ in range(int(rng.integers(0, 3))):
            if not pending:
                break
            rid = list(pending)[int(rng.integers(0, len(pending)))]
            op = int(rng.integers(0, 3))
            if op == 0:
                srv.cancel(rid)
                del pending[rid]
                n_cancelled += 1
                continue
            try:
                got, _ = srv.wait(rid, capacity=1 << 14, timeout_ms=0 if op == 1 else -1)
            except pf.PfacError as e:
                assert op == 1 and e.code == pf.PFAC_EBUSY
                continue
            assert_same(got, oracle.bucketed(texts[pending.pop(rid)], pats, threads=8))
            n_checked += 1
    for rid, i in pending.items():
        got, _ = srv.wait(rid, capacity=1 << 14)
        assert_same(got, oracle.bucketed(texts[i], pats, threads=8))
        n_checked += 1
    say(f"random serving: {n_checked} checked, {n_cancelled} cancelled")
    assert n_checked + n_cancelled == len(texts) and n_cancelled > 10
    srv.close()


def test_random_servers_with_cancellation():
    """Many small servers over seeded random pattern sets, launch tunings,
    budgets and batch limits; requests are random slices of a random text,
    a quarter of them cancelled right after a later submit (in whatever
    state they are in), the rest waited for (with a time limit, so a lost
    request fails instead of hanging) and compared with the oracle.  A
    request cancelled or waited for while earlier ones still hold the ring
    stays valid until it leaves the ring."""
    import torch
    from tests.test_gpu_fuzz import _tuning
    from tests.test_gpu_random import _case
    checked = cancelled = 0
    for seed in range(7001, 7061):
        pats, text = _case(seed)
        if text.size < 64:
            continue
        rng = np.random.default_rng(seed)
        trie = pf.Trie(pats)
        for _ in range(10):
            try:
                trie.set_tuning(**_tuning(rng))
                break
            except pf.PfacError:
                pass
        budget = int(rng.integers(text.size // 4 + 64, text.size + 1))
        max_batch = int(rng.choice([1, 2, 4, 16, 64]))
        buf = torch.empty(budget + (8 << 20), dtype=torch.uint8, device="cuda")
        srv = pf.Server(trie, buf, budget, max_batch, torch.cuda.Stream(), torch.cuda.Stream())
        reqs, pending = [], {}
        for i in range(int(rng.integers(5, 60))):
            a = int(rng.integers(0, text.size))
            b = min(text.size, a + int(rng.integers(0, min(budget, text.size) + 1)))
            reqs.append(text[a:b].copy())
            pending[srv.submit(reqs[-1])] = i
            if rng.integers(0, 4) == 0:
                rid = list(pending)[int(rng.integers(0, len(pending)))]
                srv.cancel(rid)
                del pending[rid]
                cancelled += 1
        for rid, i in pending.items():
            want = oracle.brute(reqs[i], pats, threads=8)
            got, _ = srv.wait(rid, capacity=want.n + 1, timeout_ms=30_000)
            assert_same(got, want)
            checked += 1
        srv.close()
        del buf
    say(f"random servers: {checked} checked, {cancelled} cancelled")
    assert checked > 500 and cancelled > 150


def test_server_pins_the_trie_image():
    """While a server runs, a tuning that would rebuild its trie's device
    image is refused (PFAC_EBUSY) and requests keep their results; after the
    server is freed the image can be rebuilt."""
    pats = [b"abc", b"bcd", b"zz"]
    trie = pf.Trie(pats)
    srv, _buf = _server(trie, 1 << 16, (1 << 16) + (1 << 20), 4)
    t = np.frombuffer(b"xxabcdzzz" * 500, dtype=np.uint8).copy()
    rid = srv.submit(t)
    bits = trie.tuning()["index_bits"]
    with pytest.raises(pf.PfacError) as e:
        trie.set_tuning(index_bits=8 if bits != 8 else 16)
    assert e.value.code == pf.PFAC_EBUSY
    got, _ = srv.wait(rid, capacity=1 << 14)
    assert_same(got, oracle.brute(t, pats))
    srv.close()
    trie.set_tuning(index_bits=8 if bits != 8 else 16)
    got, _ = gpu_scan(trie, t, counts=False)
    assert_same(got, oracle.brute(t, pats))


def test_server_fixes_the_whole_tuning():
    """The server's worker reads the trie's tuning at every launch: while it
    runs, any tuning change (a kernel switch needs no new image) and the
    autotuners are refused with PFAC_EBUSY, an unchanged tuning is accepted,
    and requests keep their results."""
    import torch
    pats = [b"abcd", b"bcde", b"zzzz"]
    trie = pf.Trie(pats)
    srv, _buf = _server(trie, 1 << 16, (1 << 16) + (1 << 20), 4)
    t = np.frombuffer(b"xxabcdezzzzz" * 500, dtype=np.uint8).copy()
    rid = srv.submit(t)
    tn = trie.tuning()
    for change in (dict(kernel=0 if tn["kernel"] else 2), dict(chunks_per_unit=4),
                   dict(waves_per_wg=8 if tn["waves_per_wg"] != 8 else 16)):
        with pytest.raises(pf.PfacError) as e:
            trie.set_tuning(**change)
        assert e.value.code == pf.PFAC_EBUSY, change
    trie.set_tuning(**tn)  # the same tuning: nothing changes, accepted
    dev = torch.from_numpy(t).cuda()
    with pytest.raises(pf.PfacError) as e:
        pf.pfac_autotune(trie, pf.Workspace(), dev, t.size)
    assert e.value.code == pf.PFAC_EBUSY
    got, _ = srv.wait(rid, capacity=1 << 14)
    assert_same(got, oracle.brute(t, pats))
    assert trie.tuning() == tn
    srv.close()
    trie.set_tuning(kernel=0)
    got, _ = gpu_scan(trie, t, counts=False)
    assert_same(got, oracle.brute(t, pats))


def test_server_keeps_its_trie_and_arena_alive():
    """A server built from temporaries (trie, arena, streams) holds them
    until it is closed: garbage collection in between frees none of them."""
    import gc

    import torch
    pats = [b"abcd", b"cdef", b"efgh"]
    t = np.frombuffer(b"abcdefgh" * 4096, dtype=np.uint8).copy()
    srv = pf.Server(pf.Trie(pats), torch.empty((1 << 16) + (1 << 20), dtype=torch.uint8, device="cuda"),
                    1 << 16, 4, torch.cuda.Stream(), torch.cuda.Stream())
    gc.collect()
    torch.cuda.empty_cache()
    # other allocations now, which would reuse a freed arena
    junk = torch.full((4 << 20,), 0x61, dtype=torch.uint8, device="cuda")
    ids = [srv.submit(t) for _ in range(6)]
    want = oracle.brute(t, pats)
    for rid in ids:
        got, _ = srv.wait(rid, capacity=1 << 16)
        assert_same(got, want)
    st = srv.stats()
    assert st["device_bytes"] > 0 and st["requests"] == 6
    srv.close()
    del junk
