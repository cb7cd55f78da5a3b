#!/usr/bin/env python3
"""Throughput of the failure-less Aho-Corasick scan on one MI355X.

Default (``--workload c4``, the headline): one step is one replay of a
hipGraph-captured persistent launch that scans a batch of 65,600 texts
(65,536 of 64-1500 bytes and 64 of 1-64 MiB, 2.36 GB) through the C ABI
(``pfac_graph_create_batch``: batch plan, filter kernel, walk kernel,
finisher), with the texts and the trie already resident in HBM.  Prints one
JSON line:

* ``value``: Gbit/s of text scanned (8 * text bytes / step time);
* ``roofline``: the main scan kernel alone, timed by HIP events that the
  graph records around it in every replay (``pfac_graph_set_timing``),
  against the MI355X HBM peak, with the algorithmic bytes of one launch
  (every text byte once + the CRS trie once; + 16 B per match for kernels
  that write them); ``traffic`` comes from committed rocprofv3 FETCH_SIZE /
  WRITE_SIZE counts when they were taken on the current kernel source;
* ``cpu_baseline``: the oracle's bucketed matcher over the whole batch on the
  machine's host cores (with the textbook Aho-Corasick automaton's rate);
* ``parity_with_oracle``: the replayed graph's list equals the oracle's,
  record by record;
* ``batched_vs_plain``: the same batch as one launch per text, and the
  small and large texts alone, every list compared record by record;
* ``single_text``: c2 (10,000 patterns, 256 MiB text) scanned by pfac_scan,
  with its own roofline, CPU baseline and parity;
* ``serving``: c5, the serving loop's p50/p99 latency against one request at
  a time at 0.5 / 0.8 / 0.95 of the measured capacity, every request's list
  compared with the other path's and the oracle's.

Every scan runs with the library's default launch (kernel 3: the launch
shape by size); ``--autotune`` autotunes instead (cached per workload and
device), ``--tuning`` sets one.  ``--workload c1|c2|c3`` makes one text the
headline instead; ``--no-extras`` / ``--no-serving`` / ``--no-cpu-baseline``
leave parts out.

``--placement c1,c2,...`` prints instead one line with the trie-placement
ablation: the tile kernel with 0, 1, 2, ... trie levels resolved in LDS by
the level index or by bitmapped nodes (the rest walked through the node
records in global memory), images truncated at depths 4, 8 and 16 (tails
verified against the pattern bytes), the merged DAG image, the default
launch and the autotuned one, on each workload, every point checked against
the oracle, with the trie's footprint in each encoding.  ``--footprint
1000,10000,...`` prints the footprint curve (host only, no GPU).
"""

from __future__ import annotations

import argparse
import hashlib
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0   # MI355X HBM3E, GB/s
HIP_EVENT_DISABLE_SYSTEM_FENCE = 0x20000000


class TimingEvent:
    """A HIP timing event created with hipEventDisableSystemFence: recording
    it does not write L2 back to memory, so events between the kernels of a
    step do not stretch the step.  Same interface as torch.cuda.Event
    (``record``, ``elapsed_time``, ``cuda_event``)."""

    _hip = None

    def __init__(self):
        import ctypes
        if TimingEvent._hip is None:
            # the HIP runtime torch has loaded (same soname: dlopen returns it)
            h = ctypes.CDLL("libamdhip64.so.7")
            h.hipEventCreateWithFlags.argtypes = [ctypes.POINTER(ctypes.c_void_p), ctypes.c_uint]
            h.hipEventRecord.argtypes = [ctypes.c_void_p, ctypes.c_void_p]
            h.hipEventElapsedTime.argtypes = [ctypes.POINTER(ctypes.c_float), ctypes.c_void_p,
                                              ctypes.c_void_p]
            h.hipEventDestroy.argtypes = [ctypes.c_void_p]
            TimingEvent._hip = h
        ev = ctypes.c_void_p()
        rc = self._hip.hipEventCreateWithFlags(ctypes.byref(ev), HIP_EVENT_DISABLE_SYSTEM_FENCE)
        if rc != 0:
            raise RuntimeError(f"hipEventCreateWithFlags failed: {rc}")
        self.cuda_event = ev.value

    def record(self, stream):
        rc = self._hip.hipEventRecord(self.cuda_event, stream.cuda_stream)
        if rc != 0:
            raise RuntimeError(f"hipEventRecord failed: {rc}")

    def elapsed_time(self, end: "TimingEvent") -> float:
        import ctypes
        ms = ctypes.c_float(0.0)
        rc = self._hip.hipEventElapsedTime(ctypes.byref(ms), self.cuda_event, end.cuda_event)
        if rc != 0:
            raise RuntimeError(f"hipEventElapsedTime failed: {rc}")
        return float(ms.value)

    def __del__(self):
        try:
            if self.cuda_event:
                self._hip.hipEventDestroy(self.cuda_event)
        except Exception:
            pass


def timing_event():
    """A fence-free HIP timing event, or torch's default one when the HIP
    runtime cannot be reached through ctypes (the line then says so)."""
    global TIMING_EVENTS
    try:
        ev = TimingEvent()
        TIMING_EVENTS = "hip, no system fence"
        return ev
    except (OSError, AttributeError, RuntimeError):
        import torch
        TIMING_EVENTS = "torch default"
        return torch.cuda.Event(enable_timing=True)


TIMING_EVENTS = None
CSRC = os.path.join(ROOT, "paper_1702_03657_amd", "csrc")
# sources each scan kernel is compiled from (the traffic counts are tied to them)
KERNEL_SOURCES = {
    "scan_waves": ("scan_wave.hip", "kernels.hpp", "device_common.hpp"),
    "scan_tiles": ("kernels.hip", "kernels.hpp", "device_common.hpp"),
}

WORKLOADS = {
    "c1": ("c1: 100 patterns len U[4,16] bytes U[0,255]; 1 MiB uniform text, 1000 planted copies",
           lambda w: w.c1_plain_small()),
    "c2": ("c2: 10,000 patterns len U[8,64], 70% printable bytes; 256 MiB text of the same mix, "
           "one planted copy per ~4 KiB", lambda w: w.c2_signature_set()),
    "c3": ("c3: 100,000 patterns len U[20,32] over ACGT; 1 GiB uniform ACGT text, "
           "10,000 planted copies", lambda w: w.c3_dna()),
}


def kernel_hash(kernel: str) -> str:
    h = hashlib.sha256()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def tuning_cache_path():
    return os.environ.get("PFAC_TUNING_CACHE",
                          os.path.join(os.path.expanduser("~"), ".cache", "pfac_tuning.json"))


def choose_tuning(pf, trie, ws, text_dev, n, workload, device_name, retune, offsets=None,
                  n_texts=0):
    """Autotune once per (workload, device) (the batched launch when `offsets`
    are given); later runs reuse the cached choice."""
    path = tuning_cache_path()
    key = f"{workload}|{n}"
    cache = {}
    if os.path.exists(path):
        try:
            with open(path) as f:
                cache = json.load(f)
        except (OSError, ValueError):
            cache = {}
    if key in cache and not retune:
        t = cache[key]
        trie.set_tuning(**t)
        return t, False
    t0 = time.time()
    if offsets is not None:
        best = pf.pfac_autotune_batch(trie, ws, text_dev, offsets, n_texts, n)
    else:
        best = pf.pfac_autotune(trie, ws, text_dev, n)
    log(f"autotune {workload}: {best} in {time.time() - t0:.1f}s")
    cache[key] = best
    try:
        os.makedirs(os.path.dirname(path), exist_ok=True)
        with open(path, "w") as f:
            json.dump(cache, f)
    except OSError:
        pass
    return best, True


def profile_counts(kernel, workload, tuning):
    """Committed counter summary of a scan kernel (HBM bytes, VALU
    instructions per launch), when it was taken on the current source of that
    kernel with the same tuning; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel}_{workload}.json")
    if not os.path.exists(path):
        return None
    try:
        with open(path) as f:
            d = json.load(f)
    except (OSError, ValueError):
        return None
    if d.get("kernel_sha256_16") != kernel_hash(kernel):
        return None  # the kernel changed since the counters were taken
    if d.get("tuning") != {k: int(v) for k, v in tuning.items()}:
        return None  # taken with another launch configuration
    return d


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(oracle, wl, threads, batch=False):
    """Bucketed oracle over the whole text (or batch) on `threads` host
    threads, and the textbook Aho-Corasick automaton (one thread per
    contiguous range of start positions) beside it."""
    offsets = wl.offsets if batch else None
    tm = [0.0, 0.0]
    m = oracle.bucketed(wl.text, wl.patterns, offsets=offsets, threads=threads, timing=tm)
    gbps = wl.text.size * 8 / tm[1] / 1e9
    ta = [0.0, 0.0]
    ac = oracle.aho_corasick(wl.text, wl.patterns, offsets=offsets, threads=threads, timing=ta)
    extra = {}
    if wl.text.size <= (8 << 20):
        # small texts: the literal definition (every pattern at every position) too
        tb = [0.0, 0.0]
        br = oracle.brute(wl.text, wl.patterns, threads=threads, timing=tb)
        extra = {"brute_force_gbit_s": round(wl.text.size * 8 / tb[1] / 1e9, 3),
                 "brute_force_same_matches": bool(br.n == m.n)}
    return {"value": round(gbps, 3), "unit": "Gbit/s", "cores": threads, "kind": "oracle",
            "sample": f"bucketed matcher (first-min(len,8)-byte index + memcmp) over the whole "
                      f"{wl.text.size} B " + (f"batch of {len(wl.offsets) - 1} texts" if batch
                                             else "text") +
                      f"; index build {tm[0]:.3f}s excluded; {m.n} matches",
            "nproc": os.cpu_count(), "cpu_model": cpu_model(),
            "aho_corasick_gbit_s": round(wl.text.size * 8 / ta[1] / 1e9, 3),
            "aho_corasick_same_matches": bool(ac.n == m.n), **extra}, m


def streaming_probe(torch, text, reps=10):
    """Read-only streaming rate of the device: torch's float32 sum over the text's
    bytes read as float32 words (the values do not matter, only the reads)."""
    x = text[: (text.numel() // 4) * 4].view(torch.float32)
    for _ in range(2):
        x.sum()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    for _ in range(reps):
        x.sum()
    e1.record()
    torch.cuda.synchronize()
    return x.numel() * 4 / (e0.elapsed_time(e1) / reps / 1e3) / 1e9


def run_copy_probe(torch, nbytes):
    """A plain device copy of known size, to calibrate the HBM byte counters."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"copy probe: 3 copies of {nbytes} bytes")


def same_list(got, want, with_text=True) -> bool:
    """Record-by-record equality of a GPU match list (structured array) with
    the oracle's (pos, id, text) columns."""
    import numpy as np
    return bool(got.size == want.n and np.array_equal(got["pos"], want["pos"])
                and np.array_equal(got["pattern_id"], want["id"])
                and (not with_text or np.array_equal(got["text_id"], want["text"])))


def same_records(a, b) -> bool:
    """Record-by-record equality of two GPU match lists."""
    import numpy as np
    return bool(a.size == b.size and np.array_equal(a, b))


def _graph_vs_plain(pf, torch, trie, ws, text_host, offs_host, steps, cap, text_dev=None):
    """One graph-captured batched launch vs one plain launch per text, on the
    same device copy of a batch: (batched ms, plain ms, batched list, plain
    list, batched count, plain count)."""
    import numpy as np
    text = text_dev if text_dev is not None else torch.from_numpy(text_host).cuda()
    offs = torch.from_numpy(offs_host.view(np.int64)).cuda()
    n_texts = len(offs_host) - 1
    total = int(offs_host[-1])
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        g = pf.Graph(trie, ws, text, offs, n_texts, total, out, cap, cnt, stream)
        g.launch(stream)
        stream.synchronize()
        n_batched = int(cnt.item())
        batched_list = pf.matches_to_numpy(out, min(n_batched, cap))
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            g.launch(stream)
        e1.record(stream)
        stream.synchronize()
        ms_b = e0.elapsed_time(e1) / steps
        out.fill_(0xAB)
        pf.pfac_scan_batch_plain(trie, ws, text, offs_host, n_texts, out, cap, cnt, stream)
        stream.synchronize()
        n_plain = int(cnt.item())
        plain_list = pf.matches_to_numpy(out, min(n_plain, cap))
        plain_steps = max(1, min(steps, 2))
        e0.record(stream)
        for _ in range(plain_steps):
            pf.pfac_scan_batch_plain(trie, ws, text, offs_host, n_texts, out, cap, cnt, stream)
        e1.record(stream)
        stream.synchronize()
        ms_p = e0.elapsed_time(e1) / plain_steps
    g.close()
    return ms_b, ms_p, batched_list, plain_list, n_batched, n_plain


def batched_vs_plain(pf, torch, wl, trie, ws, text_dev, steps, cap, want):
    """C4: one graph-captured persistent launch vs one launch per text, for
    all texts, the small texts only and the large texts only; every list is
    compared record by record with the other launch's and with the oracle's."""
    import numpy as np
    offs_host = wl.offsets.astype(np.uint64)
    total = int(offs_host[-1])
    res = {"texts": wl.n_texts, "text_bytes": total}
    ms_b, ms_p, bl, pl, nb, npl = _graph_vs_plain(pf, torch, trie, ws, wl.text, offs_host, steps,
                                                  cap, text_dev)
    log(f"c4 batched {ms_b:.3f} ms vs plain {ms_p:.1f} ms")
    res.update({
        "matches": nb,
        "batched_equals_plain_records": same_records(bl, pl),
        "batched_equals_oracle_records": same_list(bl, want) if want is not None else None,
        "plain_equals_oracle_records": same_list(pl, want) if want is not None else None,
        "batched_ms": round(ms_b, 4), "plain_ms": round(ms_p, 4),
        "batched_gbit_s": round(total * 8 / ms_b / 1e6, 2),
        "plain_gbit_s": round(total * 8 / ms_p / 1e6, 2),
        "speedup": round(ms_p / ms_b, 2),
    })
    del bl, pl
    # the same comparison on each kind of text alone
    lens = np.diff(offs_host.astype(np.int64))
    for name, sel in (("small_texts", lens <= 1500), ("large_texts", lens > 1500)):
        idx = np.nonzero(sel)[0]
        parts = [wl.text[int(offs_host[i]):int(offs_host[i + 1])] for i in idx]
        sub = np.concatenate(parts) if parts else np.zeros(0, np.uint8)
        del parts
        so = np.zeros(len(idx) + 1, dtype=np.uint64)
        so[1:] = np.cumsum(lens[idx])
        b, p, sbl, spl, snb, snp = _graph_vs_plain(pf, torch, trie, ws, sub, so, steps, cap)
        entry = {"texts": int(len(idx)), "text_bytes": int(so[-1]), "matches": snb,
                 "batched_equals_plain_records": same_records(sbl, spl),
                 "batched_gbit_s": round(int(so[-1]) * 8 / b / 1e6, 2),
                 "plain_gbit_s": round(int(so[-1]) * 8 / p / 1e6, 2),
                 "speedup": round(p / b, 2)}
        if want is not None:
            # the oracle's records of these texts, renumbered in sub-batch order
            keep = sel[want["text"].astype(np.int64)]
            remap = np.full(len(lens), -1, dtype=np.int64)
            remap[idx] = np.arange(len(idx))
            ok = (sbl.size == int(keep.sum())
                  and np.array_equal(sbl["pos"], want["pos"][keep])
                  and np.array_equal(sbl["pattern_id"], want["id"][keep])
                  and np.array_equal(sbl["text_id"].astype(np.int64),
                                     remap[want["text"][keep].astype(np.int64)]))
            entry["batched_equals_oracle_records"] = bool(ok)
        res[name] = entry
        del sub, sbl, spl
    return res


def _percentiles(lat_s):
    import numpy as np
    a = np.asarray(lat_s) * 1e3
    return round(float(np.percentile(a, 50)), 3), round(float(np.percentile(a, 99)), 3)


def extras_serving(pf, torch, n_requests, rates, budget_bytes, rhos=(0.5, 0.8, 0.95),
                   oracle_threads=0):
    """C5: Poisson arrivals into the continuous-batching server, against one
    request at a time (copy in, scan, copy out, next) on the same arrival
    trace.  The offered rates are `rates` (requests/s) when given, else the
    fractions `rhos` of the measured capacity (host-to-device copy plus one
    batched scan of every request).  Latency percentiles leave out the first
    5% of the requests.  Every request's list from the server and from the
    one-at-a-time path is compared record by record with the other's and,
    with `oracle_threads`, with the oracle's list for that request."""
    import threading

    import numpy as np
    from synth import workloads
    t0 = time.time()
    wl = workloads.c5_requests(n_requests)
    log(f"c5 generated in {time.time() - t0:.1f}s: {n_requests} requests, {wl.text.size} bytes")
    want_by_req = None
    if oracle_threads:
        import oracle
        t0 = time.time()
        want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets, threads=oracle_threads)
        cuts = np.searchsorted(want["text"], np.arange(n_requests + 1))
        want_by_req = [(want["pos"][cuts[i]:cuts[i + 1]], want["id"][cuts[i]:cuts[i + 1]])
                       for i in range(n_requests)]
        log(f"c5 oracle in {time.time() - t0:.1f}s: {want.n} matches")

    def check_lists(lists):
        """(requests equal to the oracle's lists, requests checked)."""
        if want_by_req is None:
            return None, 0
        ok = sum(1 for i, m in enumerate(lists)
                 if m is not None and np.array_equal(m["pos"], want_by_req[i][0])
                 and np.array_equal(m["pattern_id"], want_by_req[i][1])
                 and np.all(m["text_id"] == 0))
        return ok, len(lists)
    offs = wl.offsets.astype(np.int64)
    sizes = np.diff(offs)
    total = int(offs[-1])
    host = torch.from_numpy(wl.text).pin_memory()  # request bodies in pinned host memory
    base_ptr = host.data_ptr()
    trie = pf.Trie(wl.patterns)
    max_n = int(sizes.max())
    res = {"workload": f"c5: {n_requests} requests, sizes log-uniform [1 KiB, 64 MiB] "
                       f"(mean {sizes.mean() / 2**20:.2f} MiB), 50,000 patterns len U[8,64], "
                       f"copies 1 per 2 KiB; Poisson arrivals; latency = arrival to results "
                       f"in host memory",
           "hbm_budget_bytes": budget_bytes, "max_batch": 64, "points": []}

    # one request at a time
    stream = torch.cuda.Stream()
    ws = pf.Workspace()
    dev = torch.empty(max_n + 16, dtype=torch.uint8, device="cuda")
    cap = 1 << 22
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    out_host = torch.empty(cap * 16, dtype=torch.uint8).pin_memory()
    ws.reserve(max_n, 1, cap)

    def serve_one(i):
        """Copy in, scan, copy the matches out: the request's list."""
        a, b = int(offs[i]), int(offs[i + 1])
        with torch.cuda.stream(stream):
            dev[:b - a].copy_(host[a:b], non_blocking=True)
            pf.pfac_scan(trie, ws, dev, b - a, out, cap, cnt, None, stream)
            n = int(cnt.item())  # synchronizes the stream
            if n > cap:
                raise SystemExit(f"request {i}: {n} matches over the {cap}-record buffer")
            if n:
                out_host[:16 * n].copy_(out[:16 * n])
        return out_host[:16 * n].numpy().view(pf.MATCH_DTYPE).copy()

    # capacity: every request body copied in, then scanned as one batch
    allreq = torch.empty(total + 16, dtype=torch.uint8, device="cuda")
    offs_dev = torch.from_numpy(offs.astype(np.int64)).cuda()
    e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
    cap_b = 1 << 23
    out_b = torch.empty(cap_b * 16, dtype=torch.uint8, device="cuda")
    ws_b = pf.Workspace()
    with torch.cuda.stream(stream):
        for rep in range(2):  # the second pass is the measured one
            e0.record(stream)
            allreq[:total].copy_(host, non_blocking=True)
            e1.record(stream)
            pf.pfac_scan_batch(trie, ws_b, allreq, offs_dev, n_requests, total, out_b, cap_b, cnt, stream)
            e2.record(stream)
            stream.synchronize()
    h2d_s, scan_s = e0.elapsed_time(e1) / 1e3, e1.elapsed_time(e2) / 1e3
    capacity = total / (h2d_s + scan_s)  # bytes per second
    res["capacity"] = {"h2d_gbit_s": round(total * 8 / h2d_s / 1e9, 2),
                       "batched_scan_gbit_s": round(total * 8 / scan_s / 1e9, 2),
                       "capacity_gbit_s": round(capacity * 8 / 1e9, 2)}
    del allreq, out_b
    ws_b.close()
    if not rates:
        rates = [round(r * capacity / float(sizes.mean()), 1) for r in rhos]
        res["rho"] = list(rhos)

    # the server
    arena = torch.empty(budget_bytes + (256 << 20), dtype=torch.uint8, device="cuda")
    cs, xs = torch.cuda.Stream(), torch.cuda.Stream()
    srv = pf.Server(trie, arena, budget_bytes, 64, cs, xs)
    serve_one(0)  # warm-ups
    srv.wait(srv.submit_ptr(base_ptr, int(sizes[0])), capacity=cap)

    # the arrival loop spins holding the GIL: switch threads often so that the
    # waiting thread collects results without a 5 ms scheduling quantum
    switch = sys.getswitchinterval()
    sys.setswitchinterval(2e-4)
    for rate in rates:
        arrivals = workloads.poisson_arrivals(n_requests, rate)
        lat_base, lists_base = [], []
        start = time.perf_counter()
        for i in range(n_requests):
            due = start + arrivals[i]
            while time.perf_counter() < due:
                pass
            lists_base.append(serve_one(i))
            lat_base.append(time.perf_counter() - due)
        end_base = time.perf_counter() - start

        b0 = srv.stats()["batches"]
        ids = [None] * n_requests
        lat_srv = [0.0] * n_requests
        late = [0.0] * n_requests  # arrival to submit: the submitting thread's own delay
        lists_srv = [None] * n_requests
        ready = threading.Semaphore(0)

        def waiter():
            for i in range(n_requests):
                ready.acquire()
                m, lat = srv.wait(ids[i], capacity=cap)
                lat_srv[i] = late[i] + lat  # the server times submit to completion
                lists_srv[i] = m

        th = threading.Thread(target=waiter)
        th.start()
        start = time.perf_counter()
        for i in range(n_requests):
            due = start + arrivals[i]
            while time.perf_counter() < due:
                pass
            late[i] = time.perf_counter() - due
            ids[i] = srv.submit_ptr(base_ptr + int(offs[i]), int(sizes[i]))
            ready.release()
        th.join()
        end_srv = time.perf_counter() - start
        skip = n_requests // 20  # warm-up requests left out of the percentiles
        p50b, p99b = _percentiles(lat_base[skip:])
        p50s, p99s = _percentiles(lat_srv[skip:])
        same = sum(1 for a, b in zip(lists_srv, lists_base)
                   if a is not None and same_records(a, b))
        ok_srv, n_chk = check_lists(lists_srv)
        ok_base, _ = check_lists(lists_base)
        n_matches = sum(m.size for m in lists_base)
        del lists_srv, lists_base
        res["points"].append({
            "offered_req_s": rate,
            "offered_gbit_s": round(sizes.mean() * 8 * rate / 1e9, 2),
            "one_at_a_time": {"p50_ms": p50b, "p99_ms": p99b,
                              "served_gbit_s": round(total * 8 / end_base / 1e9, 2)},
            "server": {"p50_ms": p50s, "p99_ms": p99s,
                       "served_gbit_s": round(total * 8 / end_srv / 1e9, 2),
                       "batches": srv.stats()["batches"] - b0},
            "matches": n_matches,
            "server_equals_one_at_a_time_records": f"{same}/{n_requests}",
            "server_equals_oracle_records": None if ok_srv is None else f"{ok_srv}/{n_chk}",
            "one_at_a_time_equals_oracle_records": None if ok_base is None else f"{ok_base}/{n_chk}",
            "parity": bool(same == n_requests and (ok_srv is None or
                                                   (ok_srv == n_chk and ok_base == n_chk))),
        })
        log(f"serving at {rate} req/s: server p50/p99 {p50s}/{p99s} ms, one at a time "
            f"{p50b}/{p99b} ms, records equal {same}/{n_requests}, oracle {ok_srv}/{ok_base}")
    sys.setswitchinterval(switch)
    res["server_device_bytes"] = srv.stats()["device_bytes"]
    srv.close()
    return res


def lds_depth_tuning(stats, depth):
    """Tile-kernel tuning whose level index resolves `depth` trie levels in
    LDS (0: nothing of the trie in LDS, every start position walks from the
    root through the node records in global memory), or None if the pattern
    set does not allow that depth."""
    alpha = max(1, int(stats["alphabet_size"]))
    b = max(1, (alpha - 1).bit_length())
    b = 8 if b >= 8 else b
    if depth == 0:
        if b < 2:
            return None  # one bit already resolves a level of a binary alphabet
        bits = 1
    else:
        bits = depth * b
    if bits > 18 or depth > int(stats["min_len"]) - 1:
        return None
    return dict(kernel=0, bytes_per_lane=16, index_bits=bits, fold_bits=0, wg_per_cu=0,
                child_check=0, top_nodes=0, trunc_depth=0, dag=0)


PLACEMENT_WORKLOADS = {
    "c1": lambda w: w.c1_plain_small(),
    "c2": lambda w: w.c2_signature_set(),
    "c3": lambda w: w.c3_dna(),
    "c4": lambda w: w.c4_batched(),
    # the serving pattern set over its first 64 requests, as one batch
    "c5": lambda w: w.c5_requests(64),
}


FOOTPRINT_FAMILIES = {
    # name: (pattern lengths, byte distribution, numpy seed index)
    "c1-like": ((4, 16), "uniform", 0),
    "c2-like": ((8, 64), "mix", 1),
    "c3-like": ((20, 32), "acgt", 2),
}


def footprint_curve(pf, ks):
    """Trie footprints against the number of patterns (host only): the CRS
    trie, the merged DAG in CRS form, 36-byte bitmapped nodes and the dense
    256-entry table, for seeded pattern sets of each family."""
    from synth import workloads
    rows = []
    for fam, ((lo, hi), dist, idx) in FOOTPRINT_FAMILIES.items():
        for k in ks:
            pats = workloads.make_patterns(workloads.rng_for(200 + idx), k, lo, hi, dist)
            t = pf.Trie(pats, host_only=True)
            st = t.stats()
            rows.append({"family": fam, "k": k, "nodes": int(st["nodes"]),
                         "dag_nodes": int(st["dag_nodes"]), "dag_edges": int(st["dag_edges"]),
                         "bytes_crs": int(st["bytes_crs"]), "bytes_dag_crs": int(st["bytes_dag_crs"]),
                         "bytes_bitmap36": int(st["bytes_bitmap36"]),
                         "bytes_bitmap_narrow": int(st["bytes_bitmap_narrow"]),
                         "bytes_dense256": int(st["bytes_dense256"])})
            log(f"footprint {fam} k={k}: nodes {st['nodes']} dag {st['dag_nodes']} "
                f"crs {st['bytes_crs']} dag_crs {st['bytes_dag_crs']}")
            t.close()
    return rows


def placement_ablation(pf, torch, names, steps, warmup, threads):
    """Trie placement: the tile kernel with 0, 1, 2, ... trie levels resolved
    from the level index in LDS (the rest walked through the node records in
    global memory), the library's default launch and the autotuned one, on
    each workload; every point's match list is checked against the oracle."""
    import numpy as np

    import oracle
    from synth import workloads
    rows = []
    for name in names:
        t0 = time.time()
        wl = PLACEMENT_WORKLOADS[name](workloads)
        offs_host = wl.offsets.astype(np.uint64)
        n_texts = len(offs_host) - 1
        n = int(offs_host[-1])
        log(f"placement {name}: generated in {time.time() - t0:.1f}s, {n_texts} texts, {n} bytes")
        want = oracle.bucketed(wl.text, wl.patterns, offsets=wl.offsets if n_texts > 1 else None,
                               threads=threads)
        trie = pf.Trie(wl.patterns)
        st = trie.stats()
        default = trie.tuning()
        ws = pf.Workspace()
        text = torch.from_numpy(wl.text).cuda()
        offs = torch.from_numpy(offs_host.view(np.int64)).cuda()
        cap = max(1024, want.n)
        out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
        cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
        ws.reserve(n, n_texts, cap)
        stream = torch.cuda.current_stream()

        def scan():
            if n_texts > 1:
                pf.pfac_scan_batch(trie, ws, text, offs, n_texts, n, out, cap, cnt, stream)
            else:
                pf.pfac_scan(trie, ws, text, n, out, cap, cnt, None, stream)

        points = [(f"tile kernel, LDS depth {d}", lds_depth_tuning(st, d)) for d in range(0, 10)]
        # the same depths through the bitmapped nodes (where they fit in LDS)
        points += [(f"tile kernel, bitmapped nodes depth {d}", t and dict(t, top_nodes=1))
                   for d, t in ((d, lds_depth_tuning(st, d)) for d in range(1, 10))]
        # images truncated at depth D (tails verified), level index as deep as allowed up to 8
        deep = max([d for d in range(1, 9) if lds_depth_tuning(st, d) is not None], default=0)
        for D in (4, 8, 16):
            t = lds_depth_tuning(st, min(deep, D))
            points.append((f"tile kernel, image truncated at depth {D}", t and dict(t, trunc_depth=D, dag=0)))
        # the merged DAG image (suffix and end-node merging, ids from edge ranks)
        t = lds_depth_tuning(st, deep)
        points.append(("tile kernel, merged DAG image", t and dict(t, dag=1)))
        points = [(lab, t) for lab, t in points if t is not None]
        points.append(("library default", default))
        trie.set_tuning(**default)
        points.append(("autotuned", pf.pfac_autotune(trie, ws, text, n)))
        res = {"workload": name, "texts": n_texts, "text_bytes": n, "patterns": len(wl.patterns),
               "alphabet": int(st["alphabet_size"]), "matches": int(want.n),
               "footprint_bytes": {"crs": int(st["bytes_crs"]), "dense256": int(st["bytes_dense256"]),
                                   "bitmap36": int(st["bytes_bitmap36"]),
                                   "bitmap_narrow": int(st["bytes_bitmap_narrow"]),
                                   "dag_crs": int(st["bytes_dag_crs"]),
                                   "device_image": int(st["bytes_device"])},
               "nodes": int(st["nodes"]), "dag_nodes": int(st["dag_nodes"]),
               "points": []}
        for label, tn in points:
            try:
                trie.set_tuning(**tn)
            except pf.PfacError:
                log(f"  {label:28s} does not fit in LDS")
                continue
            s2 = trie.stats()
            for _ in range(warmup):
                scan()
            kev = [(timing_event(), timing_event()) for _ in range(steps)]
            for a, b in kev:
                a.record(stream)
                b.record(stream)
            e0, e1 = timing_event(), timing_event()
            torch.cuda.synchronize()
            e0.record(stream)
            for i in range(steps):
                ws.set_timing(kev[i][0], kev[i][1])
                scan()
            e1.record(stream)
            torch.cuda.synchronize()
            ws.set_timing(None, None)
            ms = e0.elapsed_time(e1) / steps
            kms = statistics.mean(a.elapsed_time(b) for a, b in kev)
            got_n = int(cnt.item())
            got = pf.matches_to_numpy(out, min(got_n, cap))
            same = bool(got_n == want.n and np.array_equal(got["pos"], want["pos"])
                        and np.array_equal(got["pattern_id"], want["id"])
                        and (n_texts == 1 or np.array_equal(got["text_id"], want["text"])))
            gbit = n * 8 / ms / 1e6
            res["points"].append({
                "placement": label, "index_depth": int(s2["index_depth"]),
                "lds_bytes": int(s2["lds_bytes"]), "scan_kernel": int(s2["scan_kernel"]),
                "top_lds_bytes": int(s2["bytes_top_nodes"] if tn.get("top_nodes")
                                     else s2["bytes_level_index"]),
                "image_bytes": int(s2["bytes_device"]), "node_bytes": int(s2["bytes_nodes"]),
                "tail_bytes": int(s2["bytes_tails"]), "dag_nodes": int(s2["dag_nodes"]),
                "tuning": {k: int(v) for k, v in tn.items()},
                "ms_per_scan": round(ms, 5), "gbit_s": round(gbit, 2),
                "hbm_frac": round(n / ms / 1e6 / HBM_PEAK_GBS, 4),
                "main_kernel_ms": round(kms, 5), "parity_with_oracle": same})
            log(f"  {label:28s} K={int(s2['index_depth'])} {gbit:10.2f} Gbit/s "
                f"({ms:.4f} ms/scan, kernel {kms:.4f} ms) image {int(s2['bytes_device'])} B "
                f"parity={same}")
        rows.append(res)
        del text, offs, out
        trie.close()
        ws.close()
        torch.cuda.empty_cache()
    return rows


def valu_issue(counts, n_cu, kernel_ms):
    """The filter's other ceiling: VALU issue (wave64 instructions, 4 cycles
    each on one of 4 SIMDs per CU: CUs * 2.4 GHz instructions per second)."""
    if not counts or not counts.get("valu_insts_per_launch"):
        return None
    issue_ms = counts["valu_insts_per_launch"] / (n_cu * 2.4e9) * 1e3
    return {"valu_insts_per_launch": counts["valu_insts_per_launch"], "cus": n_cu,
            "issue_bound_ms": round(issue_ms, 5), "frac": round(issue_ms / kernel_ms, 4)}


def kernel_of(stats):
    """(name, split) of the main scan kernel of a launch; `stats` carries
    "launch_kernel", the kernel a launch of the measured size runs."""
    k = int(stats["launch_kernel"])
    return ("scan_waves" if k in (1, 2) else "scan_tiles"), k == 2


def alg_bytes_of(stats, text_bytes, n_matches):
    """Algorithmic bytes of one launch of the main scan kernel: every text
    byte read once and the CRS trie read once; the tile and fused wave
    kernels also write the 16-byte match records (on the split path the walk
    kernel writes them)."""
    _, split = kernel_of(stats)
    return text_bytes + int(stats["bytes_crs"]) + (0 if split else 16 * n_matches)


def roofline_entry(stats, workload, tuning, text_bytes, n_matches, kernel_ms, step_ms, probe, n_cu):
    kernel_name, split = kernel_of(stats)
    alg = alg_bytes_of(stats, text_bytes, n_matches)
    achieved = alg / (kernel_ms / 1e3) / 1e9
    step_bytes = text_bytes + int(stats["bytes_crs"]) + 16 * n_matches
    counts = profile_counts(kernel_name, workload, tuning)
    return {
        "bound": "hbm",
        "achieved": round(achieved, 1),
        "peak": HBM_PEAK_GBS,
        "unit": "GB/s",
        "frac": round(achieved / HBM_PEAK_GBS, 4),
        "traffic": counts.get("hbm_bytes_per_launch") if counts else None,
        "kernel": kernel_name + (" (split filter)" if split else ""),
        "kernel_source_sha256_16": kernel_hash(kernel_name),
        "kernel_ms": round(kernel_ms, 5),
        "algorithmic_bytes_per_launch": alg,
        "algorithmic_bytes": "text bytes + CRS trie bytes" + ("" if split else " + 16 B per match"),
        "whole_step": {"algorithmic_bytes": step_bytes,
                       "achieved": round(step_bytes / (step_ms / 1e3) / 1e9, 1),
                       "frac": round(step_bytes / (step_ms / 1e3) / 1e9 / HBM_PEAK_GBS, 4)},
        "streaming_probe_gb_s": round(probe, 1),
        "frac_of_probe": round(achieved / probe, 4),
        "valu_issue": valu_issue(counts, n_cu, kernel_ms),
    }


def trie_entry(st):
    return {"nodes": int(st["nodes"]), "bytes_crs": int(st["bytes_crs"]),
            "bytes_dense256": int(st["bytes_dense256"]),
            "bytes_bitmap36": int(st["bytes_bitmap36"]),
            "bytes_device": int(st["bytes_device"]),
            "build_s": round(st["build_seconds"], 3)}


def timed_steps(torch, stream, steps, one_step, set_kernel_events):
    """Run `steps` steps back to back on `stream`, each bracketed by fence-free
    HIP events, with a fresh event pair handed to `set_kernel_events` before
    each step (recorded by the library around the main scan kernel).
    Returns (mean ms per step, per-step ms, per-step kernel ms)."""
    kev = [(timing_event(), timing_event()) for _ in range(steps)]
    for a, b in kev:  # the library re-records them around the kernel
        a.record(stream)
        b.record(stream)
    sev = [timing_event() for _ in range(steps + 1)]
    torch.cuda.synchronize()
    sev[0].record(stream)
    for i in range(steps):
        set_kernel_events(*kev[i])
        one_step()
        sev[i + 1].record(stream)
    torch.cuda.synchronize()
    step_ms = [sev[i].elapsed_time(sev[i + 1]) for i in range(steps)]
    kms = [a.elapsed_time(b) for a, b in kev]
    return sev[0].elapsed_time(sev[-1]) / steps, step_ms, kms


def measure_single(pf, torch, name, args, dev_name, threads, steps, headline=False):
    """One text scanned by pfac_scan per step (workloads c1-c3): the line's
    fields for it, and the oracle's list."""
    import numpy as np
    from synth import workloads
    desc, make = WORKLOADS[name]
    t0 = time.time()
    wl = make(workloads)
    log(f"{name} generated in {time.time() - t0:.1f}s: {wl.text.size} bytes, "
        f"{len(wl.patterns)} patterns")
    n = int(wl.text.size)
    trie = pf.Trie(wl.patterns)
    ws = pf.Workspace()

    # host -> device copy of the text, timed separately (not part of `value`)
    host = torch.from_numpy(wl.text).pin_memory()
    text = torch.empty(n, dtype=torch.uint8, device="cuda")
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record()
    text.copy_(host, non_blocking=True)
    h1.record()
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1)
    del host

    if args.tuning and headline:
        trie.set_tuning(**parse_tuning(args.tuning))
        tuning, tuned_now = trie.tuning(), False
    elif args.autotune:
        tuning, tuned_now = choose_tuning(pf, trie, ws, text, n, name, dev_name, args.retune)
    else:
        tuning, tuned_now = trie.tuning(), False
    st = trie.stats()
    st["launch_kernel"] = trie.launch_kernel(n)[0]

    stream = torch.cuda.current_stream()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    rc, n_matches = pf.pfac_scan_sync(trie, ws, text, n, None, 0)
    cap = max(1024, n_matches)
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    ws.reserve(n, 1, cap)
    for _ in range(args.warmup):
        pf.pfac_scan(trie, ws, text, n, out, cap, cnt, None, stream)
    torch.cuda.synchronize()
    ms_per_step, step_ms, kms = timed_steps(
        torch, stream, steps, lambda: pf.pfac_scan(trie, ws, text, n, out, cap, cnt, None, stream),
        lambda a, b: ws.set_timing(a, b))
    ws.set_timing(None, None)
    got = int(cnt.item())
    if got != n_matches:
        raise SystemExit(f"match count changed between runs: {got} != {n_matches}")
    if args.copy_probe:
        run_copy_probe(torch, n)
    probe = streaming_probe(torch, text)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    res = {
        "metric": "Gbit/s scanned on 1 MI355X (plain PFAC scan of one text, text resident in HBM)",
        "value": round(n * 8 / (ms_per_step / 1e3) / 1e9, 2),
        "unit": "Gbit/s",
        "steps": steps,
        "ms_per_step": round(ms_per_step, 5),
        "ms_per_step_median": round(statistics.median(step_ms), 5),
        "ms_per_step_min": round(min(step_ms), 5),
        "config": {"workload": desc, "text_bytes": n, "patterns": len(wl.patterns),
                   "matches": n_matches, "tuning": {k: int(v) for k, v in tuning.items()},
                   "autotuned_this_run": tuned_now, "index_depth": int(st["index_depth"]),
                   "symbol_bits": int(st["symbol_bits"]), "device": dev_name},
        "roofline": roofline_entry(st, name, tuning, n, n_matches, statistics.mean(kms),
                                   ms_per_step, probe, n_cu),
        "h2d_gbit_s": round(n * 8 / (h2d_ms / 1e3) / 1e9, 2),
        "trie": trie_entry(st),
    }
    want = None
    if not args.no_cpu_baseline:
        import oracle
        cb, want = cpu_baseline(oracle, wl, threads)
        res["cpu_baseline"] = cb
        # the timed run's list equals the oracle's, record by record
        res["parity_with_oracle"] = same_list(pf.matches_to_numpy(out, n_matches), want,
                                              with_text=False)
    del text, out
    trie.close()
    ws.close()
    torch.cuda.empty_cache()
    return res, want


def measure_batch(pf, torch, args, dev_name, threads):
    """C4, the headline: every text of the batch scanned by one replay of a
    graph-captured persistent launch per step; the main scan kernel timed by
    events recorded inside each replay."""
    import numpy as np
    from synth import workloads
    t0 = time.time()
    wl = workloads.c4_batched()
    offs_host = wl.offsets.astype(np.uint64)
    total = int(offs_host[-1])
    n_texts = wl.n_texts
    log(f"c4 generated in {time.time() - t0:.1f}s: {n_texts} texts, {total} bytes")
    trie = pf.Trie(wl.patterns)
    ws = pf.Workspace()
    host = torch.from_numpy(wl.text).pin_memory()
    text = torch.empty(total, dtype=torch.uint8, device="cuda")
    h0, h1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    h0.record()
    text.copy_(host, non_blocking=True)
    h1.record()
    torch.cuda.synchronize()
    h2d_ms = h0.elapsed_time(h1)
    del host
    offs = torch.from_numpy(offs_host.view(np.int64)).cuda()

    if args.tuning:
        trie.set_tuning(**parse_tuning(args.tuning))
        tuning, tuned_now = trie.tuning(), False
    elif args.autotune:
        tuning, tuned_now = choose_tuning(pf, trie, ws, text, total, "c4", dev_name, args.retune,
                                          offsets=offs, n_texts=n_texts)
    else:
        tuning, tuned_now = trie.tuning(), False
    st = trie.stats()
    st["launch_kernel"] = trie.launch_kernel(total)[0]
    stream = torch.cuda.Stream()
    cnt = torch.zeros(1, dtype=torch.int64, device="cuda")
    with torch.cuda.stream(stream):
        pf.pfac_scan_batch(trie, ws, text, offs, n_texts, total, None, 0, cnt, stream)
        stream.synchronize()
    n_matches = int(cnt.item())
    cap = max(1024, n_matches)
    out = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")

    # the graph takes over the workspace's timing events: event-record nodes
    # around its main scan kernel, re-pointed at a fresh pair every step
    ev0, ev1 = timing_event(), timing_event()
    ws.set_timing(ev0, ev1)
    g = pf.Graph(trie, ws, text, offs, n_texts, total, out, cap, cnt, stream)
    ws.set_timing(None, None)
    for _ in range(args.warmup):
        g.launch(stream)
    stream.synchronize()
    kernel_timing = "events recorded by the graph around its main scan kernel in every timed replay"
    try:
        g.set_timing(ev0, ev1)
        set_events = lambda a, b: g.set_timing(a, b)  # noqa: E731
    except pf.PfacError:
        kernel_timing = None
        set_events = lambda a, b: None  # noqa: E731
    ms_per_step, step_ms, kms = timed_steps(torch, stream, args.steps, lambda: g.launch(stream),
                                            set_events)
    got_n = int(cnt.item())
    if got_n != n_matches:
        raise SystemExit(f"match count changed between runs: {got_n} != {n_matches}")
    graph_list = pf.matches_to_numpy(out, n_matches)
    g.close()
    if kernel_timing is None:
        # the runtime kept no event nodes in the graph: time the same launch
        # issued directly (pfac_scan_batch), with the workspace's events
        kernel_timing = "events around the main scan kernel of pfac_scan_batch (no graph)"
        with torch.cuda.stream(stream):
            _, _, kms = timed_steps(
                torch, stream, args.steps,
                lambda: pf.pfac_scan_batch(trie, ws, text, offs, n_texts, total, out, cap, cnt,
                                           stream),
                lambda a, b: ws.set_timing(a, b))
        ws.set_timing(None, None)
    kernel_ms = statistics.mean(kms)
    if not (0 < kernel_ms <= max(step_ms)):
        raise SystemExit(f"kernel events out of range: {kernel_ms} ms against steps {step_ms}")
    del out
    if args.copy_probe:
        run_copy_probe(torch, total)
    probe = streaming_probe(torch, text)
    n_cu = torch.cuda.get_device_properties(0).multi_processor_count
    desc = ("c4: 65,536 texts lognormal(512, 0.75) clipped [64,1500] B + 64 texts U[1,64] MiB, "
            "uniform bytes, copies 1 per 2 KiB; 20,000 patterns len U[8,64]; one graph replay "
            "of the persistent batched launch per step")
    line = {
        "metric": "Gbit/s scanned on 1 MI355X, batched vs plain PFAC; p50/p99 scan latency",
        "value": round(total * 8 / (ms_per_step / 1e3) / 1e9, 2),
        "unit": "Gbit/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 5),
        "ms_per_step_median": round(statistics.median(step_ms), 5),
        "ms_per_step_min": round(min(step_ms), 5),
        "timing_events": TIMING_EVENTS,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": desc, "texts": n_texts, "text_bytes": total,
                   "patterns": len(wl.patterns), "matches": n_matches, "launch": "hipGraph replay",
                   "tuning": {k: int(v) for k, v in tuning.items()},
                   "autotuned_this_run": tuned_now, "index_depth": int(st["index_depth"]),
                   "symbol_bits": int(st["symbol_bits"]), "device": dev_name},
        "roofline": dict(roofline_entry(st, "c4", tuning, total, n_matches, kernel_ms,
                                        ms_per_step, probe, n_cu), kernel_timing=kernel_timing),
        "h2d_gbit_s": round(total * 8 / (h2d_ms / 1e3) / 1e9, 2),
        "trie": trie_entry(st),
    }
    want = None
    if not args.no_cpu_baseline:
        import oracle
        cb, want = cpu_baseline(oracle, wl, threads, batch=True)
        line["cpu_baseline"] = cb
        line["parity_with_oracle"] = same_list(graph_list, want, with_text=True)
    del graph_list
    if not args.no_extras:
        line["batched_vs_plain"] = batched_vs_plain(pf, torch, wl, trie, ws, text,
                                                    max(3, min(10, args.steps // 5)), cap, want)
    del text, offs, want
    trie.close()
    ws.close()
    torch.cuda.empty_cache()
    return line


TUNING_FIELDS = ["kernel", "bytes_per_lane", "index_bits", "fold_bits", "wg_per_cu", "waves_per_wg",
                 "chunks_per_unit", "child_check", "top_nodes", "trunc_depth", "dag"]


def parse_tuning(text):
    return dict(zip(TUNING_FIELDS, (int(x) for x in text.split(","))))


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS) + ["c4"],
                    help="c4 (default): the batched graph launch; c1-c3: one text")
    ap.add_argument("--autotune", action="store_true",
                    help="autotune the launches (cached per workload and device) instead of "
                         "the library's default launch")
    ap.add_argument("--retune", action="store_true", help="with --autotune: ignore the cached choice")
    ap.add_argument("--tuning", default=None,
                    help="kernel,bytes_per_lane,index_bits,fold_bits,wg_per_cu,waves_per_wg,"
                         "chunks_per_unit,child_check[,top_nodes[,trunc_depth[,dag]]]")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the batched-vs-plain comparison (c4)")
    ap.add_argument("--no-serving", action="store_true",
                    help="skip the serving loop (c5) against one request at a time")
    ap.add_argument("--serving-requests", type=int, default=2000)
    ap.add_argument("--serving-rates", default=None,
                    help="offered requests per second, one measurement per rate (default: the "
                         "--serving-rho fractions of the measured capacity)")
    ap.add_argument("--serving-rho", default="0.5,0.8,0.95",
                    help="offered load as fractions of the measured capacity")
    ap.add_argument("--serving-budget", type=int, default=8 << 30, help="HBM bytes for request texts")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain copy of the text size (counter calibration)")
    ap.add_argument("--footprint", default=None, metavar="k1,k2,...",
                    help="instead of the headline line: trie footprints (CRS, merged DAG, bitmapped, "
                         "dense) for seeded pattern sets of these sizes, host only, one JSON line")
    ap.add_argument("--placement", default=None, metavar="c1,c2,...",
                    help="instead of the headline line: the trie-placement ablation (LDS depth "
                         "0, 1, 2, ... of the tile kernel, default and autotuned launches) on "
                         "these workloads, one JSON line")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this benchmark runs on exactly one GPU: the scan shards by "
                                   "text range with no exchange, so more GPUs are not measured "
                                   "here (run with --gpus 1)"}))
        sys.exit(2)

    if args.footprint:
        import paper_1702_03657_amd as pf
        rows = footprint_curve(pf, [int(x) for x in args.footprint.split(",")])
        print(json.dumps({"footprint_curve": rows}), flush=True)
        return

    import numpy as np
    import torch

    import paper_1702_03657_amd as pf
    from synth import workloads

    torch.cuda.set_device(0)
    dev_name = torch.cuda.get_device_name(0)
    if args.placement:
        names = args.placement.split(",")
        bad = [x for x in names if x not in PLACEMENT_WORKLOADS]
        if bad:
            raise SystemExit(f"unknown workloads {bad}; choose from {sorted(PLACEMENT_WORKLOADS)}")
        threads = args.cpu_threads or min(16, os.cpu_count() or 1)
        rows = placement_ablation(pf, torch, names, args.steps, args.warmup, threads)
        print(json.dumps({"placement_ablation": rows, "device": dev_name, "steps": args.steps,
                          "warmup": args.warmup, "hbm_peak_gb_s": HBM_PEAK_GBS}), flush=True)
        return
    threads = args.cpu_threads or min(16, os.cpu_count() or 1)
    if args.workload == "c4":
        line = measure_batch(pf, torch, args, dev_name, threads)
        if not args.no_extras:
            single, _ = measure_single(pf, torch, "c2", args, dev_name, threads,
                                       steps=max(20, min(args.steps, 200)))
            line["single_text"] = {"c2": single}
    else:
        single, _ = measure_single(pf, torch, args.workload, args, dev_name, threads,
                                   steps=args.steps, headline=True)
        line = {"metric": single.pop("metric"), "value": single.pop("value"),
                "unit": single.pop("unit"), "n_gpus": 1, "steps": args.steps,
                "warmup": args.warmup, "ms_per_step": single.pop("ms_per_step"),
                "timing_events": TIMING_EVENTS, "higher_is_better": True, "scaling": "weak",
                "vs_baseline": None, "dtype": "u8", "data": "synthetic", **single}
    if not args.no_serving:
        line["serving"] = extras_serving(
            pf, torch, args.serving_requests,
            [float(x) for x in args.serving_rates.split(",")] if args.serving_rates else None,
            args.serving_budget, [float(x) for x in args.serving_rho.split(",")],
            0 if args.no_cpu_baseline else threads)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
