"""The workload generator's file output (``python -m synth``): the files hold
the same texts, offsets and patterns as the in-memory generator, and every
copy in the manifest that later copies did not overwrite is in the text."""

import json
import os
import subprocess
import sys

import numpy as np

from synth import workloads

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_cli_writes_the_workload(tmp_path):
    out = tmp_path / "c4"
    subprocess.run([sys.executable, "-m", "synth", "c4", "--out", str(out), "--scale", "0.01"],
                   check=True, cwd=ROOT, capture_output=True)
    m = json.loads((out / "manifest.json").read_text())
    wl = workloads.c4_batched(n_small=int(65_536 * 0.01), n_large=int(64 * 0.01))
    text = np.fromfile(out / "text.bin", dtype=np.uint8)
    toff = np.fromfile(out / "text_offsets.bin", dtype=np.uint64)
    pdata = np.fromfile(out / "patterns.bin", dtype=np.uint8)
    poff = np.fromfile(out / "pattern_offsets.bin", dtype=np.uint64)
    assert np.array_equal(text, wl.text) and np.array_equal(toff, wl.offsets)
    assert np.array_equal(pdata, wl.patterns.data) and np.array_equal(poff, wl.patterns.offsets)
    assert m["seed"] == workloads.SEED_BASE + 3 and m["texts"] == len(toff) - 1
    assert len(m["plants"]) == len(wl.plants) > 0
    intact = 0
    for tid, pos, j in m["plants"]:
        p = pdata[int(poff[j]):int(poff[j + 1])]
        a = int(toff[tid]) + pos
        intact += bool(np.array_equal(text[a:a + len(p)], p))
    assert intact > 0.9 * len(m["plants"])
