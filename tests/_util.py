"""Helpers shared by the GPU parity tests (no method arithmetic here)."""
import hashlib
import json
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden")

LOG_FIELDS = ("target_index", "source_index", "ssd", "known_k", "n_filled",
              "priority", "confidence", "data_term", "remaining")


def log_matrix(log) -> np.ndarray:
    cols = []
    for f in LOG_FIELDS:
        a = np.asarray(log[f])
        if a.dtype == np.float64:
            a = a.view(np.int64)
        cols.append(a.astype(np.int64))
    if not len(log):
        return np.zeros((0, len(LOG_FIELDS)), np.int64)
    return np.stack(cols, axis=1)


def log_sha256(log) -> str:
    return hashlib.sha256(np.ascontiguousarray(log_matrix(log)).tobytes()).hexdigest()


def assert_logs_equal(got, want, label=""):
    """Bit-exact comparison of two fill logs, naming the first divergence."""
    g, w = log_matrix(got), log_matrix(want)
    n = min(len(g), len(w))
    diff = np.nonzero((g[:n] != w[:n]).any(axis=1))[0]
    if len(diff):
        i = int(diff[0])
        cols = [LOG_FIELDS[c] for c in np.nonzero(g[i] != w[i])[0]]
        raise AssertionError(f"{label}: first divergence at iteration {i} in {cols}: "
                             f"got {dict(zip(LOG_FIELDS, g[i]))} want {dict(zip(LOG_FIELDS, w[i]))}")
    assert len(g) == len(w), f"{label}: {len(g)} iterations vs {len(w)}"


def load_golden(key: str):
    path = os.path.join(GOLDEN, f"oracle_{key}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        return json.load(f)


def assert_matches_golden(gold, log, rgb, label=""):
    """Compares a full run against stored oracle results (hashes + samples)."""
    m = log_matrix(log)
    for i, row in gold["log_sample"].items():
        i = int(i)
        assert i < len(m), f"{label}: run shorter than the oracle's ({len(m)} <= {i})"
        if list(m[i]) != row:
            cols = [LOG_FIELDS[c] for c in range(len(row)) if m[i][c] != row[c]]
            raise AssertionError(f"{label}: sampled iteration {i} differs in {cols}: got "
                                 f"{dict(zip(LOG_FIELDS, m[i]))} want {dict(zip(LOG_FIELDS, row))}")
    assert len(m) == gold["iterations"], f"{label}: {len(m)} iterations vs {gold['iterations']}"
    assert log_sha256(log) == gold["log_sha256"], f"{label}: log hash differs"
    assert hashlib.sha256(np.ascontiguousarray(rgb).tobytes()).hexdigest() == gold["final_rgb_sha256"], \
        f"{label}: final image differs"
