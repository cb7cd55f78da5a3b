"""Helpers shared by the GPU tests: run the HIP path through the C ABI and
compare with the oracle, record by record."""

import sys

import numpy as np

import oracle
import paper_1702_03657_amd as pf


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def device_text(text: np.ndarray, pad_front: int = 0):
    """Copy a host text to the device, optionally at a misaligned address."""
    import torch
    buf = torch.zeros(len(text) + pad_front + 16, dtype=torch.uint8, device="cuda")
    if len(text):
        buf[pad_front:pad_front + len(text)] = torch.from_numpy(np.ascontiguousarray(text))
    return buf, buf[pad_front:pad_front + len(text)]


def gpu_scan(trie, text: np.ndarray, ws=None, counts=True, pad_front=0, capacity=None):
    import torch
    ws = ws or pf.Workspace()
    _, t = device_text(text, pad_front)
    n = len(text)
    cap = capacity if capacity is not None else max(256, n // 32)
    cdev = torch.full((max(n, 1),), 7, dtype=torch.int32, device="cuda") if counts else None
    while True:
        out = torch.empty(max(cap, 1) * 16, dtype=torch.uint8, device="cuda")
        rc, cnt = pf.pfac_scan_sync(trie, ws, t if n else None, n, out, cap,
                                    cdev[:n] if (counts and n) else None)
        if rc == pf.PFAC_OK:
            break
        assert rc == pf.PFAC_ETRUNC and cnt > cap
        cap = cnt
    m = pf.matches_to_numpy(out, cnt)
    c = cdev[:n].cpu().numpy().view(np.uint32) if counts else None
    return m, c


def gpu_scan_batch(trie, text: np.ndarray, offsets: np.ndarray, ws=None, pad_front=0,
                   capacity=None, plain=False, graph_replays=0):
    import torch
    ws = ws or pf.Workspace()
    _, t = device_text(text, pad_front)
    offs = torch.from_numpy(np.ascontiguousarray(offsets, dtype=np.uint64).view(np.int64)).to("cuda")
    n_texts = len(offsets) - 1
    total = int(offsets[-1])
    cap = capacity if capacity is not None else max(256, total // 32)
    cnt_dev = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty(max(cap, 1) * 16, dtype=torch.uint8, device="cuda")
    if plain:
        pf.pfac_scan_batch_plain(trie, ws, t if total else None, offsets, n_texts, out, cap, cnt_dev)
    elif graph_replays:
        s = torch.cuda.Stream()
        g = pf.Graph(trie, ws, t if total else None, offs, n_texts, total, out, cap, cnt_dev, s)
        results = []
        for _ in range(graph_replays):
            out.fill_(0xAB)
            torch.cuda.synchronize()
            g.launch(s)
            s.synchronize()
            n = int(cnt_dev.item())
            results.append(pf.matches_to_numpy(out, min(n, cap)))
        g.close()
        return results, int(cnt_dev.item())
    else:
        pf.pfac_scan_batch(trie, ws, t if total else None, offs, n_texts, total, out, cap, cnt_dev)
    torch.cuda.synchronize()
    n = int(cnt_dev.item())
    if n > cap:  # grow the output and scan again: the count is exact either way
        return gpu_scan_batch(trie, text, offsets, ws, pad_front, n, plain, graph_replays)
    return pf.matches_to_numpy(out, n), n


def assert_same(got: np.ndarray, want: "oracle.Matches", with_text=False):
    assert got.size == want.n, f"count {got.size} != oracle {want.n}"
    assert np.array_equal(got["pos"], want["pos"]), "positions differ"
    assert np.array_equal(got["pattern_id"], want["id"]), "pattern ids differ"
    if with_text:
        assert np.array_equal(got["text_id"], want["text"]), "text ids differ"
    else:
        assert np.all(got["text_id"] == 0)
