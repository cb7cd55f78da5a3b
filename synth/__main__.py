"""Write a workload to files: ``python -m synth c2 --out DIR [--scale F]``.

Files: ``text.bin`` (all texts back to back), ``text_offsets.bin`` (uint64,
n_texts + 1), ``patterns.bin`` and ``pattern_offsets.bin`` (uint64, k + 1),
``manifest.json`` (name, seed, sizes, and every planted copy as
[text id, position, pattern id]).  ``--scale`` shrinks the text sizes (the
distributions stay the same).
"""

import argparse
import json
import os

import numpy as np

from . import workloads


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("config", choices=["c1", "c2", "c3", "c4", "c5"])
    ap.add_argument("--out", required=True)
    ap.add_argument("--scale", type=float, default=1.0, help="text size factor (default 1)")
    ap.add_argument("--requests", type=int, default=200, help="c5: number of requests")
    args = ap.parse_args()
    s = args.scale
    MiB = workloads.MiB
    if args.config == "c1":
        wl = workloads.c1_plain_small(n_text=max(1, int(MiB * s)))
    elif args.config == "c2":
        wl = workloads.c2_signature_set(n_text=max(1, int(256 * MiB * s)))
    elif args.config == "c3":
        wl = workloads.c3_dna(n_text=max(1, int(workloads.GiB * s)))
    elif args.config == "c4":
        wl = workloads.c4_batched(n_small=max(1, int(65_536 * s)), n_large=max(0, int(64 * s)))
    else:
        wl = workloads.c5_requests(args.requests, hi=max(1024, int(64 * MiB * s)))
    os.makedirs(args.out, exist_ok=True)
    wl.text.tofile(os.path.join(args.out, "text.bin"))
    np.asarray(wl.offsets, dtype=np.uint64).tofile(os.path.join(args.out, "text_offsets.bin"))
    wl.patterns.data.tofile(os.path.join(args.out, "patterns.bin"))
    np.asarray(wl.patterns.offsets, dtype=np.uint64).tofile(os.path.join(args.out, "pattern_offsets.bin"))
    index = {"c1": 0, "c2": 1, "c3": 2, "c4": 3, "c5": 4}[args.config]
    manifest = {"name": wl.name, "seed": workloads.SEED_BASE + index, "scale": s,
                "texts": int(len(wl.offsets) - 1), "text_bytes": int(wl.text.size),
                "patterns": int(len(wl.patterns)), "plants": wl.plants.astype(np.int64).tolist()}
    with open(os.path.join(args.out, "manifest.json"), "w") as f:
        json.dump(manifest, f)
    print(f"{args.config}: {manifest['texts']} texts, {manifest['text_bytes']} bytes, "
          f"{manifest['patterns']} patterns, {len(manifest['plants'])} copies -> {args.out}")


if __name__ == "__main__":
    main()
