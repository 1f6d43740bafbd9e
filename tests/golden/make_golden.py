"""Writes the stored oracle results for the large workloads.

Runs the CPU oracle (and nothing else: no GPU code is imported) on the seeded
synthetic workloads and stores, per workload, the input hash, the oracle
source hash, the iteration count, hashes of the final image and of the
per-iteration log, and a sample of log records.  The GPU parity tests compare
the HIP path's full runs against these.

    python tests/golden/make_golden.py small vga hd9 hd9w hd13 hd13w batch:0-31 serve:0-15
"""
from __future__ import annotations

import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from paper_1403_4238_amd import synth  # noqa: E402

LOG_FIELDS = ("target_index", "source_index", "ssd", "known_k", "n_filled",
              "priority", "confidence", "data_term", "remaining")


def log_matrix(log) -> np.ndarray:
    """Log records as an int64 matrix (doubles by their bit patterns)."""
    cols = []
    for f in LOG_FIELDS:
        a = np.asarray(log[f])
        if a.dtype == np.float64:
            a = a.view(np.int64)
        cols.append(a.astype(np.int64))
    return np.stack(cols, axis=1) if cols[0].size else np.zeros((0, len(LOG_FIELDS)), np.int64)


def log_sha256(log) -> str:
    return hashlib.sha256(np.ascontiguousarray(log_matrix(log)).tobytes()).hexdigest()


def oracle_sha256() -> str:
    with open(oracle.SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def workload(name: str):
    if name == "small":
        return [synth.small()]
    if name == "vga":
        return [synth.vga()]
    if name.startswith("hd"):
        win = name.endswith("w")
        patch = int(name[2:].rstrip("w"))
        return [synth.hd(patch=patch, window=win)]
    for prefix, gen in (("batch", synth.batch), ("serve", synth.serving)):
        if name.startswith(prefix):
            jobs = gen()
            if ":" in name:
                lo, hi = (int(v) for v in name.split(":")[1].split("-"))
                return [(prefix, i, jobs[i]) for i in range(lo, hi + 1)]
            return [(prefix, i, j) for i, j in enumerate(jobs)]
    raise ValueError(name)


def golden_path(key: str) -> str:
    return os.path.join(HERE, f"oracle_{key}.json")


def run_one(key: str, job: synth.Job) -> dict:
    t0 = time.time()
    o = oracle.Oracle(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha)
    log = o.run()
    dt = time.time() - t0
    rgb, _, hole, _ = o.read()
    assert hole.sum() == 0
    m = log_matrix(log)
    n = len(log)
    x0, y0, x1, y1 = o.rect()
    n_cand = int(o.valid_map()[y0:y1, x0:x1].sum())
    sample_idx = sorted(set(list(range(min(n, 64))) + list(range(0, n, 16)) + [n - 1]))
    rec = {
        "workload": job.name,
        "width": job.width, "height": job.height,
        "patch_radius": job.patch_radius, "search_mode": job.search_mode,
        "alpha": list(job.alpha), "rect": list(o.rect()),
        "input_sha256": job.sha256(),
        "oracle_c_sha256": oracle_sha256(),
        "iterations": n,
        "hole_pixels": int(job.mask.sum()),
        "final_rgb_sha256": hashlib.sha256(rgb.tobytes()).hexdigest(),
        "log_sha256": log_sha256(log),
        "log_fields": list(LOG_FIELDS),
        "log_sample": {str(i): [int(v) for v in m[i]] for i in sample_idx},
        "oracle_seconds_1thread": round(dt, 3),
        "candidates_per_search": n_cand,
        "candidate_evals": n * n_cand,
    }
    with open(golden_path(key), "w") as f:
        json.dump(rec, f, indent=1)
    print(f"{key}: {job.name} iters={n} {dt:.1f}s", flush=True)
    return rec


def main(names):
    for name in names:
        for item in workload(name):
            if isinstance(item, tuple):
                prefix, i, job = item
                run_one(f"{prefix}{i:02d}", job)
            else:
                run_one(name, item)


if __name__ == "__main__":
    main(sys.argv[1:] or ["small"])
