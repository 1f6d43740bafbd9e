"""Benchmark: masked-SSD patch evaluations/s and ms per removal on one MI355X.

A step is one complete object removal (fill front, FP64 priority, exemplar
search, copy/confidence update, repeated until the hole is empty) of the
1920x1080 synthetic workload with a 9x9 patch and a full-image search.  The
image and mask are uploaded and initialised before the timed region (each
timed removal has its own pre-created context, so the inputs are resident in
HBM when timing starts).

    python bench.py [--gpus 1] [--steps K] [--warmup W]
                    [--form persistent|stream|plain] [--path mfma|simt]
                    [--workload hd|vga|small|big|batch|serve|sweep|copy|resume]
                    [--patch 9|13|17] [--window]
                    [--dispatch-iters 1024] [--iters-per-check 128]
                    [--no-other-form] [--no-cpu-baseline] [--no-end-to-end]

Prints one JSON line.  Besides the headline it reports the other forms
(stream = search and commit launches enqueued ahead, checked every few
iterations; graph = hipGraph replay of G iterations), the live-measured
roofline of the dominant kernel, and the CPU oracle timed on a bounded prefix
of the same removal.  `--workload copy` times a plain 256 MiB device copy: its
HBM byte counters calibrate those of the fill kernels.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# MI355X (gfx950) public figures used for the roofline.
CUS, LANES_PER_CU_CYCLE, CLOCK_HZ = 256, 64, 2.4e9
VALU_LANE_OPS = CUS * LANES_PER_CU_CYCLE * CLOCK_HZ          # 39.32e12 lane-instructions/s
# A term is one (offset, channel, candidate) product of the cross term.  The
# SIMT search does one v_dot4_u32_u8 per (known offset, candidate); the
# instruction forms 4 int8 products per lane, so the VALU's dot4 peak is
# 4 products per lane-instruction (157.3e12/s), against which the SIMT
# roofline fraction is reported.  The RGBX layout uses 3 of the 4 (the
# fourth byte is 0), so 3 terms per lane-instruction (117.96e12/s) is the
# layout-limited ceiling, reported beside it.  The square term costs
# O(column runs) by running sums and is not counted.
PRODUCTS_PER_DOT4 = 4.0
TERM_PEAK = VALU_LANE_OPS * PRODUCTS_PER_DOT4                # 157.3e12 products/s
TERM_PEAK_LAYOUT = VALU_LANE_OPS * 3.0                       # 117.96e12 RGB terms/s
# int8 MFMA, dense: 5.0 POP/s = 2.5e15 multiply-accumulates (terms) per second.
MFMA_TERM_PEAK = 2.5e15
# The roofline is reported in ops: a term is two (a subtract and a
# multiply-accumulate on the SIMT path, an int8 multiply and its add on MFMA).
OPS_PER_TERM = 2.0
HBM_PEAK_GBS = 8000.0

# HBM bytes per launch of a kernel on a workload, from rocprofv3 FETCH_SIZE
# and WRITE_SIZE passes on this bench command (per-dispatch averages in KiB),
# scaled by what the same counters read for a plain 256 MiB device copy
# (`--workload copy`: FETCH x 2.0, WRITE x 1.0).  Each entry holds the hash of
# the kernel's sources it was taken on; once they change it reports null.
TRAFFIC_BYTES_PER_LAUNCH = {
    ("k_fill_mfma<R=4>", "hd-1920x1080-p9-full", 128): {
        "bytes": 36393574, "fetch_kib": 16208.05, "write_kib": 3124.5,
        "sources": ["inpaint_dev.h", "search_tile.h", "search_mfma_tile.h", "fill.hip"],
        "sha256_16": "af19dc1c885c4e90"},
    ("k_fill_mfma<R=4>", "hd-1920x1080-p9-full", 1024): {
        "bytes": 70608384, "fetch_kib": 22792.69, "write_kib": 23368.12,
        "sources": ["inpaint_dev.h", "search_tile.h", "search_mfma_tile.h", "fill.hip"],
        "sha256_16": "af19dc1c885c4e90"},
}


def checks(a, form):
    """Iterations per host check of a form: the persistent form's dispatch
    length, or what the stream and graph forms enqueue per check."""
    return a.dispatch_iters if form == "persistent" else a.iters_per_check


def traffic_for(kernel, workload, iters_per_launch):
    """Calibrated HBM bytes per launch, or None if not measured on the
    current kernel sources."""
    e = TRAFFIC_BYTES_PER_LAUNCH.get((kernel, workload, iters_per_launch))
    if e is None:
        return None
    h = hashlib.sha256()
    for f in e["sources"]:
        with open(os.path.join(ROOT, "paper_1403_4238_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return e["bytes"] if h.hexdigest()[:16] == e["sha256_16"] else None


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="hd", choices=["hd", "vga", "small", "big", "batch", "serve", "sweep", "copy", "resume"])
    ap.add_argument("--jobs", type=int, default=128, help="serve: number of jobs")
    ap.add_argument("--workers", type=int, default=1, help="serve: admission worker threads (0: on the loop)")
    ap.add_argument("--graph-iters", type=int, default=64, help="batch: iterations per step")
    ap.add_argument("--serve-iters", type=int, default=128, help="serve: iterations per batch step")
    ap.add_argument("--serve-form", default="persistent", choices=["persistent", "graph", "auto"],
                    help="serve: batch form")
    ap.add_argument("--tiles-per-group", type=int, default=0,
                    help="serve: attach a job only while the running jobs' search tiles fit this many per "
                         "search work-group (0: whenever a slot is free)")
    ap.add_argument("--batch-form", default="auto", choices=["auto", "persistent", "graph"],
                    help="batch: form of the batch steps")
    ap.add_argument("--capacity", type=int, default=16, help="serve: batch slots")
    ap.add_argument("--budget-gb", type=float, default=4.0, help="serve: device memory budget")
    ap.add_argument("--patch", type=int, default=9)
    ap.add_argument("--window", action="store_true", help="alpha = 1 search window (3x the hole bbox)")
    ap.add_argument("--form", default="persistent", choices=["persistent", "stream", "plain"],
                    help="timed form (kernel events need a non-graph form)")
    ap.add_argument("--iters-per-check", type=int, default=128,
                    help="stream / graph forms: iterations enqueued per host check")
    ap.add_argument("--dispatch-iters", type=int, default=1024,
                    help="persistent form: iterations per dispatch (one host check each)")
    ap.add_argument("--tile-rows", type=int, default=0)
    ap.add_argument("--path", default="mfma", choices=["mfma", "simt", "direct"],
                    help="exemplar-search kernel (direct: SIMT without LDS staging)")
    ap.add_argument("--source-policy", default="original", choices=["original", "current"],
                    help="candidate domain: filled pixels become sources (current)")
    ap.add_argument("--scoring", default="whole", choices=["whole", "intersect"],
                    help="candidate domain: score overlapping candidates on the known intersection")
    ap.add_argument("--sweep-part", default="both", choices=["both", "alpha", "lds"],
                    help="sweep: the persistent alpha x P timings, the LDS staging study, or both")
    ap.add_argument("--no-other-form", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-end-to-end", action="store_true",
                    help="skip the removal from host buffers (create, upload, read-back)")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    return ap.parse_args()


def make_job(a):
    from paper_1403_4238_amd import synth
    if a.workload == "hd":
        return synth.hd(patch=a.patch, window=a.window)
    if a.workload == "vga":
        return synth.vga()
    if a.workload == "big":
        # the first serving job: 1992x1221, 7x7 patch, more search tiles than
        # resident work-groups (the persistent form spreads them)
        return synth.serving()[0]
    return synth.small()


def path_id(name):
    from paper_1403_4238_amd import binding as B
    return {"mfma": B.PATH_MFMA, "simt": B.PATH_SIMT, "direct": B.PATH_SIMT_DIRECT}[name]


def search_kernel_name(path, r, tile_rows):
    if path == "mfma":
        return f"k_search_mfma<R={r}>"
    return f"k_search{'_direct' if path == 'direct' else ''}<R={r},NY={tile_rows or 8}>"


def timed_removals(job, n_steps, n_warmup, form, iters_per_check, tile_rows, timing=True, path="simt",
                   domain=("original", "whole")):
    """Runs n_warmup + n_steps removals; times the last n_steps together."""
    import torch
    from paper_1403_4238_amd import binding as B
    policy = B.SOURCE_CURRENT if domain[0] == "current" else B.SOURCE_ORIGINAL
    scoring = B.SCORE_INTERSECT if domain[1] == "intersect" else B.SCORE_WHOLE
    ctxs = [B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect,
                        form=form, iters_per_check=iters_per_check, tile_rows=tile_rows,
                        path=path_id(path), source_policy=policy, scoring=scoring)
            for _ in range(n_warmup + n_steps)]
    for c in ctxs[:n_warmup]:
        c.run()
    for c in ctxs[n_warmup:]:
        c.profile_search(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    iters = []
    for c in ctxs[n_warmup:]:
        st, n, _ = c.run()
        assert st == B.DONE
        iters.append(n)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kernel_ms = sum(c.search_time()[0] for c in ctxs[n_warmup:])
    searches = sum(c.search_time()[1] for c in ctxs[n_warmup:])
    last = ctxs[-1]
    log = last.read_log(0, iters[-1])
    out = last.read_image()
    rect, cands = last.search_info()
    run_form = last.run_form()
    for c in ctxs:
        c.close()
    return dict(seconds=dt, iters=iters, kernel_ms=kernel_ms, searches=searches, log=log, image=out,
                candidates=cands, rect=rect, ws_bytes=ctxs[0].ws_bytes, run_form=run_form)


def end_to_end_removal(job, form, iters_per_check, tile_rows, path, n=2):
    """Wall time of whole removals from host buffers: create (upload and
    initialisation), run, and read-back of the final image and the fill log,
    each synchronised; the mean over n (after the timed region)."""
    import torch
    from paper_1403_4238_amd import binding as B
    ts = []
    for _ in range(n):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        c = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect, form=form,
                        iters_per_check=iters_per_check, tile_rows=tile_rows, path=path_id(path))
        st, it, _ = c.run()
        c.read_image()
        c.read_log(0, it)
        torch.cuda.synchronize()
        ts.append(time.perf_counter() - t0)
        c.close()
    return round(1000 * sum(ts) / len(ts), 3)


def cpu_baseline(job, seconds):
    """The oracle as it stands, single-threaded, on a prefix of the removal."""
    import oracle
    oracle.build()
    t0 = time.perf_counter()
    o = oracle.Oracle(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect)
    t_create = time.perf_counter() - t0
    x0, y0, x1, y1 = o.rect()
    ncand = int(o.valid_map()[y0:y1, x0:x1].sum())
    n = 0
    t1 = time.perf_counter()
    while time.perf_counter() - t1 < seconds:
        if o.step() is None:
            break
        n += 1
    dt = time.perf_counter() - t1
    return {
        "value": round(n * ncand / dt, 1), "unit": "patch evals/s", "cores": 1, "kind": "oracle",
        "sample": f"first {n} fill iterations of the same removal ({n * ncand} patch evals), "
                  f"oracle create excluded ({t_create:.2f}s)",
        "ms_per_iteration": round(1000 * dt / max(n, 1), 2),
        "host_cpu": _cpu_name(), "host_nproc": os.cpu_count(),
        "all_cores": cpu_baseline_all_cores(job, 2.0, min(16, os.cpu_count() or 1), ncand),
    }


def cpu_baseline_all_cores(job, seconds, threads, ncand):
    """The same oracle on `threads` host threads at once, each running its own
    copy of the removal from the start for `seconds` (the C oracle holds no
    global state and ctypes releases the GIL during its calls): the host's
    aggregate oracle rate."""
    import threading
    import oracle
    olist = [None] * threads
    counts = [0] * threads

    def make(i):
        olist[i] = oracle.Oracle(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, rect=job.rect)

    def run(i):
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < seconds:
            if olist[i].step() is None:
                break
            counts[i] += 1

    for fn in (make, run):
        ts = [threading.Thread(target=fn, args=(i,)) for i in range(threads)]
        t0 = time.perf_counter()
        for t in ts:
            t.start()
        for t in ts:
            t.join()
        dt = time.perf_counter() - t0
    n = sum(counts)
    return {"value": round(n * ncand / dt, 1), "unit": "patch evals/s", "cores": threads, "kind": "oracle",
            "sample": f"{threads} threads, each the first {min(counts)}-{max(counts)} fill iterations of its own "
                      f"copy of the removal ({n * ncand} patch evals in {dt:.2f}s)"}


def _cpu_name():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def golden_check(job, a, log, image, workload=None):
    wl = workload or a.workload
    key = {("hd", 9, False): "hd9", ("hd", 9, True): "hd9w", ("hd", 13, False): "hd13",
           ("hd", 13, True): "hd13w"}.get((wl, a.patch, a.window), "serve00" if wl == "big" else wl)
    path = os.path.join(ROOT, "tests", "golden", f"oracle_{key}.json")
    if not os.path.exists(path):
        return "no stored oracle result"
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _util import log_sha256
    with open(path) as f:
        gold = json.load(f)
    ok = (gold["input_sha256"] == job.sha256() and gold["iterations"] == len(log)
          and gold["log_sha256"] == log_sha256(log)
          and gold["final_rgb_sha256"] == hashlib.sha256(image.tobytes()).hexdigest())
    return "bit-exact vs stored oracle" if ok else "MISMATCH vs stored oracle"


def sweep_bench(a):
    """The paper's trade-off study in kind: search factor alpha x patch size on
    stand-ins shaped like its four photographs (Table 3).  One warm-up and one
    timed removal per configuration, persistent form; the MFMA search for
    P <= 13, the SIMT search for P = 17.  Each configuration also runs its
    local-memory study: one stream-form removal with the SIMT search staged
    in LDS and one reading device memory directly, timing every search
    launch (both must give the same fill log)."""
    import torch
    from paper_1403_4238_amd import binding as B
    from paper_1403_4238_amd import synth
    alphas = [(1, 20), (1, 5), (1, 2), (1, 1), (2, 1), None]
    rows = []
    t_all = time.perf_counter()
    for name, *_ in synth.PAPER_IMAGES:
        for patch in (9, 13, 17):
            for alpha in alphas:
                job = synth.paper(name, patch=patch, alpha=alpha)
                path = B.PATH_MFMA if patch <= 13 else B.PATH_SIMT
                mk = lambda: B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha,
                                         form="persistent", iters_per_check=a.iters_per_check, path=path)
                row = {"image": name, "patch": patch, "alpha": None if alpha is None else f"{alpha[0]}/{alpha[1]}"}
                try:
                    mk().close()
                except B.InpaintError as e:   # no candidate window fits (thin strip, small alpha)
                    row["error"] = B.inpaint_status_string(e.status)
                    rows.append(row)
                    continue
                log = None
                if a.sweep_part != "lds":
                    w = mk()
                    w.run()
                    w.close()
                    g = mk()
                    torch.cuda.synchronize()
                    t0 = time.perf_counter()
                    st, n, _ = g.run()
                    torch.cuda.synchronize()
                    dt = time.perf_counter() - t0
                    log = g.read_log(0, n)
                    rect, cands = g.search_info()
                    k = np.asarray(log["known_k"], dtype=np.float64)
                    row.update({
                        "search_area": [rect[2] - rect[0], rect[3] - rect[1]],
                        "candidates_per_search": cands, "iterations": n,
                        "ms_per_removal": round(1000 * dt, 3),
                        "patch_evals_per_s": round(n * cands / dt, 1),
                        "mean_ssd_per_known_value": round(float(np.mean(np.asarray(log["ssd"], dtype=np.float64) / (3 * k))), 3),
                        "path": "mfma" if path == B.PATH_MFMA else "simt", "form": g.run_form()})
                    g.close()
                if a.sweep_part != "alpha":
                    lds = {}
                    for pth in ("simt", "direct"):
                        o = timed_removals(job, 1, 0, "stream", a.iters_per_check, 0, timing=True, path=pth)
                        lds[pth] = {"search_us": round(1000 * o["kernel_ms"] / max(o["searches"], 1), 3),
                                    "ms_per_removal": round(1000 * o["seconds"], 3)}
                        if log is None:
                            log = o["log"]
                        lds[pth]["same_log"] = bool(np.array_equal(o["log"], log))
                    row["lds_study"] = {"staged": lds["simt"], "direct": lds["direct"],
                                        "search_time_ratio": round(lds["direct"]["search_us"] / lds["simt"]["search_us"], 3)}
                rows.append(row)
    print(json.dumps({"metric": "alpha x patch-size sweep on paper-shaped stand-ins (ms per removal)",
                      "unit": "ms per removal", "n_gpus": 1, "data": "synthetic (seeded)",
                      "seconds_total": round(time.perf_counter() - t_all, 2), "sweep": rows}), flush=True)


def resume_bench(a):
    """Iterative editing / resume at 1080p: the removal is stopped half way,
    exported (image, hole, confidences, iteration count), imported into a
    new context created from the checkpoint image and finished there; the
    joined fill log and final image must match the stored oracle result."""
    import torch
    from paper_1403_4238_amd import binding as B
    job = synth_hd(a)
    kw = dict(form=a.form, iters_per_check=a.iters_per_check, path=path_id(a.path))
    full = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, **kw)
    full.run()                                   # warm-up of the same removal
    full.close()
    g1 = B.Inpainter(job.rgb, job.mask, job.patch_radius, job.search_mode, job.alpha, **kw)
    half = 1878
    _, n1, log1 = g1.run(max_iters=half, log_cap=half)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ck = g1.export_state()
    t1 = time.perf_counter()
    g2 = B.Inpainter(ck[0], job.mask, job.patch_radius, job.search_mode, job.alpha, **kw)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    g2.import_state(*ck)
    torch.cuda.synchronize()
    t3 = time.perf_counter()
    st, n2, log2 = g2.run(log_cap=job.mask.size)
    torch.cuda.synchronize()
    t4 = time.perf_counter()
    log = np.concatenate([log1, log2])
    parity = golden_check(job, a, log, g2.read_image(), workload="hd")
    print(json.dumps({"metric": "resume from a checkpoint (1080p 9x9 full search, stopped half way)",
                      "value": round(1000 * (t3 - t2), 3), "unit": "ms per import", "n_gpus": 1,
                      "higher_is_better": False, "data": "synthetic (seeded)",
                      "config": {"workload": f"{job.name}, checkpoint after {n1} of {n1 + n2} iterations, "
                                             f"{g2.run_form()} form"},
                      "export_ms": round(1000 * (t1 - t0), 3), "create_ms": round(1000 * (t2 - t1), 3),
                      "import_ms": round(1000 * (t3 - t2), 3), "finish_ms": round(1000 * (t4 - t3), 3),
                      "parity": parity}), flush=True)


def synth_hd(a):
    from paper_1403_4238_amd import synth
    return synth.hd(patch=a.patch, window=a.window)


def copy_bench(a):
    """A plain device-to-device copy of 256 MiB (HIP's blit copy kernel), three
    times: the reference reading of the HBM byte counters."""
    import torch
    n = 256 << 20
    src = torch.full((n,), 1, dtype=torch.uint8, device="cuda")
    dst = torch.empty_like(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms = []
    for _ in range(3):
        e0.record()
        dst.copy_(src)
        e1.record()
        e1.synchronize()
        ms.append(e0.elapsed_time(e1))
    assert bool((dst[:: 1 << 20] == 1).all())
    best = min(ms)
    print(json.dumps({"metric": "device copy bandwidth (read + write)", "value": round(2 * n / best / 1e6, 1),
                      "unit": "GB/s", "n_gpus": 1, "bytes_read": n, "bytes_written": n,
                      "ms": [round(m, 4) for m in ms], "data": "synthetic"}), flush=True)


def batch_bench(a):
    """64 images of uneven size: the batched forms vs one image after another."""
    import torch
    from paper_1403_4238_amd import binding as B
    from paper_1403_4238_amd import synth
    jobs = synth.batch()
    tune = os.environ.get("INPAINT_TUNE_CACHE")   # optional file that keeps the autotuner's choices
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _util import load_golden, log_sha256

    def make(form="plain", path="mfma"):
        return [B.Inpainter(j.rgb, j.mask, j.patch_radius, form=form, iters_per_check=a.iters_per_check,
                            path=path_id(path)) for j in jobs]

    def batched(bform, path):
        """Runs the whole batch in one form; returns (seconds, iterations, evals, steps, ok, checked)."""
        batch = B.Batch(capacity=len(jobs), graph_iters=a.graph_iters, autotune=True, tune_cache=tune, form=bform)
        # warm-up set: the first step plans (and, in the graph form, tunes and captures)
        warm = make(path=path)
        for c in warm:
            batch.attach(c)
        batch.step()
        for c in warm:
            batch.detach(c)
            c.close()
        del warm
        ctxs = make(path=path)
        for c in ctxs:
            batch.attach(c)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        steps = 0
        while batch.step() > 0:
            steps += 1
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        ran = batch.last_form()
        iters = [c.progress()[0] for c in ctxs]
        cands = [c.search_info()[1] for c in ctxs]
        evals = sum(i * n for i, n in zip(iters, cands))
        checked = ok = 0
        terms = 0
        for i, (j, c) in enumerate(zip(jobs, ctxs)):
            log = c.read_log(0, iters[i])
            # Eq. 4's terms: 3 channels x known offsets x candidates, per iteration
            terms += 3 * int(np.asarray(log["known_k"], dtype=np.int64).sum()) * cands[i]
            gold = load_golden(f"batch{i:02d}")
            if gold is None:
                continue
            checked += 1
            ok += (gold["input_sha256"] == j.sha256() and gold["log_sha256"] == log_sha256(log)
                   and gold["final_rgb_sha256"] == hashlib.sha256(c.read_image().tobytes()).hexdigest())
        for c in ctxs:
            batch.detach(c)
            c.close()
        batch.close()
        return dict(seconds=dt, iters=iters, evals=evals, terms=terms, steps=steps + 1, ok=ok, checked=checked,
                    form=ran)

    head = batched(a.batch_form, a.path)
    forms = {}
    if not a.no_other_form:
        for name, bform, path in (("persistent_simt", "persistent", "simt"), ("graph_simt", "graph", "simt"),
                                  ("graph_mfma", "graph", "mfma")):
            if (bform, path) == (head["form"], a.path):
                continue
            r = batched(bform, path)
            forms[name] = {"ms": round(1000 * r["seconds"], 2), "patch_evals_per_s": round(r["evals"] / r["seconds"], 1),
                           "parity": f"{r['ok']}/{r['checked']} bit-exact vs stored oracle", "form": r["form"]}
    # one image after another: two launches + one host check per iteration
    # (plain), or the search and commit launches enqueued ahead (stream)
    one = {}
    for form in ("plain", "stream", "persistent"):
        cs = make(form)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for c in cs:
            c.run()
        torch.cuda.synchronize()
        one[form] = time.perf_counter() - t1
        for c in cs:
            c.close()
    dt, evals = head["seconds"], head["evals"]
    line = {
        "metric": "masked-SSD patch evals/s (batch of 64 images, batched persistent form)",
        "value": round(evals / dt, 1), "unit": "patch evals/s", "n_gpus": 1, "steps": 1, "warmup": 1,
        "ms_per_step": round(1000 * dt, 3), "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 (SSD: u8 x u8 -> u32 exact; priority: f64)", "data": "synthetic (seeded)",
        "config": {"workload": "batch of 64 RGB u8 images 320x240..1280x720, 1-3 blobs covering 2-10%, "
                               f"9x9 patch, full search, {a.path} search; batch form {head['form']} "
                               f"({a.graph_iters} iterations per step)",
                   "images": len(jobs), "total_iterations": int(sum(head["iters"])), "batch_steps": head["steps"],
                   "max_iterations_per_image": int(max(head["iters"]))},
        "batched_ms": round(1000 * dt, 2),
        # over the whole batch's wall time (commits, host checks and the
        # graph / persistent switch included), so a lower bound for its
        # search kernels
        "roofline": {"bound": "mfma", "kernel": "whole batch (graph steps: k_search_batched + k_commit_batched, "
                                                "then k_fill_multi_mfma)",
                     "achieved": round(OPS_PER_TERM * head["terms"] / dt / 1e12, 3), "peak": MFMA_TERM_PEAK * OPS_PER_TERM / 1e12,
                     "unit": "TOP/s", "frac": round(head["terms"] / dt / MFMA_TERM_PEAK, 5),
                     "frac_of_valu_dot4": round(head["terms"] / dt / TERM_PEAK, 5), "traffic": None},
        "other_batch_forms": forms,
        "one_by_one": {f: {"ms": round(1000 * t, 2), "patch_evals_per_s": round(evals / t, 1)}
                       for f, t in one.items()},
        "speedup_vs_plain": round(one["plain"] / dt, 3),
        "speedup_vs_one_by_one_persistent": round(one["persistent"] / dt, 3),
        "parity": f"{head['ok']}/{head['checked']} images bit-exact vs stored oracle",
    }
    print(json.dumps(line), flush=True)


def serve_bench(a):
    """Poisson arrivals, memory-admitted continuous batching: p50/p99 latency."""
    import torch
    from paper_1403_4238_amd import binding as B
    from paper_1403_4238_amd import serve, synth
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from _util import load_golden, log_sha256
    jobs = synth.serving(n=a.jobs)
    budget = int(a.budget_gb * (1 << 30))

    def run(js, keep=False):
        eng = serve.GpuEngine(capacity=a.capacity, graph_iters=a.serve_iters, autotune=True, log=keep,
                              form=a.serve_form, tiles_per_group=a.tiles_per_group,
                              path=a.path)
        srv = serve.Server(eng, budget, a.capacity, a.serve_iters, keep_results=True, workers=a.workers)
        torch.cuda.synchronize()
        recs = srv.run(js)
        torch.cuda.synchronize()
        return srv, recs

    # capacity: everything arrives at once
    sat_jobs = synth.rescaled_arrivals(jobs, 1e9)
    run(sat_jobs[:2])   # warm-up (tuning, graph capture)
    srv_sat, recs_sat = run(sat_jobs)
    sat = serve.summarize(recs_sat)
    rate = 0.7 * sat["jobs_per_s"]
    srv_p, recs_p = run(synth.rescaled_arrivals(jobs, rate), keep=True)
    poisson = serve.summarize(recs_p)
    # the workload's own arrival rate (fixed)
    srv_f, recs_f = run(jobs)
    fixed = serve.summarize(recs_f)
    # every served job equals the same job run alone; the first ones also
    # equal their stored oracle results
    same = gold_ok = gold_n = 0
    differ = []

    def alone_run(j, form):
        alone = B.Inpainter(j.rgb, j.mask, j.patch_radius, form=form, iters_per_check=256,
                            log_capacity=int(j.mask.sum()),
                            path=B.PATH_MFMA if j.patch_radius <= 6 else B.PATH_SIMT)
        st, n, log = alone.run(log_cap=int(j.mask.sum()))
        img = alone.read_image()
        alone.close()
        return log, img

    for i, (j, r) in enumerate(zip(jobs, recs_p)):
        log, img = alone_run(j, "persistent")
        ok = bool(r.status == "done" and (img == r.result["image"]).all()
                  and log_sha256(log) == log_sha256(r.result["log"]))
        same += ok
        if not ok and r.status == "done":
            # where the two differ, and which side a third run (stream form) takes
            from _util import log_matrix
            a_m, b_m = log_matrix(log), log_matrix(r.result["log"])
            n = min(len(a_m), len(b_m))
            dv = np.nonzero((a_m[:n] != b_m[:n]).any(axis=1))[0]
            log3, img3 = alone_run(j, "stream")
            differ.append({"job": i, "name": j.name, "iters_alone": len(a_m), "iters_served": len(b_m),
                           "first_divergence": int(dv[0]) if len(dv) else None,
                           "image_equal": bool((img == r.result["image"]).all()),
                           "stream_equals_alone": bool(log_sha256(log3) == log_sha256(log)),
                           "stream_equals_served": bool(log_sha256(log3) == log_sha256(r.result["log"]))})
        gold = load_golden(f"serve{i:02d}")
        if gold is not None and r.status == "done":
            gold_n += 1
            gold_ok += (gold["input_sha256"] == j.sha256() and gold["log_sha256"] == log_sha256(r.result["log"])
                        and gold["final_rgb_sha256"] == hashlib.sha256(r.result["image"].tobytes()).hexdigest())
    line = {
        "metric": "serving: jobs/s and p50/p99 latency (Poisson arrivals at 0.7x measured capacity)",
        "value": poisson["jobs_per_s"], "unit": "jobs/s", "n_gpus": 1, "steps": len(jobs), "warmup": 2,
        "ms_per_step": poisson["mean_latency_ms"], "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u8 (SSD: u8 x u8 -> u32 exact; priority: f64)",
        "data": "synthetic (seeded)",
        "config": {"workload": f"{len(jobs)} removal jobs, RGB u8 256x256..2048x1536, holes 1-10% (1-3 blobs), "
                               "patch 7/9/11, full search; admission by workspace bytes "
                               f"(budget {a.budget_gb} GiB), {a.capacity} slots, {a.serve_form} form, G={a.serve_iters}, "
                               f"tiles per search group {a.tiles_per_group or 'unbounded'}, "
                               f"{a.workers} admission worker(s), {a.path} search",
                   "rate_jobs_per_s": round(rate, 3), "fixed_rate_jobs_per_s": 20.0},
        "poisson": poisson, "fixed_rate": fixed, "saturation": sat,
        "peak_active": srv_p.peak_active, "peak_bytes": srv_p.peak_used,
        "mix_equals_alone": f"{same}/{len(jobs)}",
        "mix_differs": differ,
        "not_done": [{"run": name, "job": r.index, "name": r.name, "status": r.status, "error": r.error}
                     for name, rs in (("saturation", recs_sat), ("poisson", recs_p), ("fixed_rate", recs_f))
                     for r in rs if r.status != "done"],
        "parity": f"{gold_ok}/{gold_n} served jobs bit-exact vs stored oracle",
    }
    print(json.dumps(line), flush=True)


def main():
    a = parse()
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(independent jobs would be placed one per GPU; see the design notes).", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if a.workload == "batch":
        return batch_bench(a)
    if a.workload == "serve":
        return serve_bench(a)
    if a.workload == "sweep":
        return sweep_bench(a)
    if a.workload == "copy":
        return copy_bench(a)
    if a.workload == "resume":
        return resume_bench(a)
    job = make_job(a)
    domain = (a.source_policy, a.scoring)
    if domain != ("original", "whole") and (a.path == "mfma" or a.form == "persistent"):
        sys.exit("the candidate-domain variants run on the SIMT search (--path simt|direct) in the "
                 "plain / stream / graph forms")
    res = timed_removals(job, a.steps, a.warmup, a.form, checks(a, a.form), a.tile_rows, path=a.path,
                         domain=domain)
    n_steps = a.steps
    evals = sum(res["iters"]) * res["candidates"]
    value = evals / res["seconds"]
    ms_per_step = 1000 * res["seconds"] / n_steps

    log = res["log"]
    terms_per_removal = 3 * int(np.asarray(log["known_k"], dtype=np.int64).sum()) * res["candidates"]
    # Timed launches: one per search in the stream / plain forms, one per
    # dispatch of up to iters_per_check whole iterations in the persistent form.
    avg_kernel_ms = res["kernel_ms"] / max(res["searches"], 1)
    terms_per_launch = terms_per_removal * n_steps / max(res["searches"], 1)
    achieved = terms_per_launch / (avg_kernel_ms * 1e-3)
    persistent = res["run_form"] == "persistent"
    peak = MFMA_TERM_PEAK if a.path == "mfma" else TERM_PEAK
    r = job.patch_radius
    kernel = ((f"k_fill_mfma<R={r}>" if a.path == "mfma" else f"k_fill<R={r}>") if persistent else
              search_kernel_name(a.path, r, a.tile_rows))
    # HBM bytes a search must move at least: the RGBX words of the candidate
    # windows' rows once (the frame is read through L2 / MALL every search).
    rx0, ry0, rx1, ry1 = res["rect"]
    bytes_per_launch = 4 * (min(rx1 + r, job.width) - max(rx0 - r, 0)) * (min(ry1 + r, job.height) - max(ry0 - r, 0))

    # The other forms.  The stream form runs the one-search-per-launch kernels,
    # so it also gives the search kernel's own launch time and rate; the
    # graph form replays them as a hipGraph (no events inside).
    others = {}
    if not a.no_other_form:
        # (name, form, path): the same search path in the stream, graph and
        # plain (one search launch and one host check per iteration) forms,
        # and the persistent form on the other search path.
        other_path = "simt" if a.path == "mfma" else "mfma"
        variants = [("stream", "stream", a.path), ("graph", "graph", a.path), ("plain", "plain", a.path)]
        if domain == ("original", "whole") and a.path != "direct" and (other_path == "simt" or r <= 6):
            variants.append((f"persistent_{other_path}", "persistent", other_path))
        for name, form, opath in variants:
            if form == res["run_form"] and opath == a.path:
                continue
            o = timed_removals(job, 1, 0, form, checks(a, form), a.tile_rows, timing=(form != "graph"),
                               path=opath, domain=domain)
            rec = {"ms_per_removal": round(1000 * o["seconds"], 2),
                   "patch_evals_per_s": round(sum(o["iters"]) * o["candidates"] / o["seconds"], 1),
                   "form": o["run_form"], "path": opath,
                   "bit_exact_vs_headline": bool(len(o["log"]) == len(log) and (o["log"] == log).all()
                                                 and (o["image"] == res["image"]).all())}
            opeak = MFMA_TERM_PEAK if opath == "mfma" else TERM_PEAK
            if form != "graph":
                k_ms = o["kernel_ms"] / max(o["searches"], 1)
                k_terms = terms_per_removal / max(o["searches"], 1)
                k_rate = k_terms / (k_ms * 1e-3)
                kname = ((f"k_fill_mfma<R={r}>" if opath == "mfma" else f"k_fill<R={r}>")
                         if o["run_form"] == "persistent" else search_kernel_name(opath, r, a.tile_rows))
                rec["kernel"] = {
                    "kernel": kname, "bound": "mfma" if opath == "mfma" else "alu",
                    "avg_launch_us": round(1000 * k_ms, 3), "launches_timed": o["searches"],
                    "achieved": round(OPS_PER_TERM * k_rate / 1e12, 3),
                    "peak": round(OPS_PER_TERM * opeak / 1e12, 2), "unit": "TOP/s", "frac": round(k_rate / opeak, 5)}
                if opath != "mfma":
                    rec["kernel"]["frac_of_rgb_layout_ceiling"] = round(k_rate / TERM_PEAK_LAYOUT, 5)
            others[name] = rec

    line = {
        "metric": "masked-SSD patch evals/s (ms per 1080p removal alongside)",
        "value": round(value, 1),
        "unit": "patch evals/s",
        "n_gpus": 1, "steps": n_steps, "warmup": a.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "u8 (SSD: u8 x u8 -> u32 exact; priority: f64)",
        "data": "synthetic (seeded)",
        "config": {
            "workload": f"{job.name}: {job.width}x{job.height} RGB u8, hole {int(job.mask.sum())} px, "
                        f"{2 * r + 1}x{2 * r + 1} patch, "
                        f"{'alpha=1 window' if a.window else 'full search'}, "
                        f"{'int8-MFMA' if a.path == 'mfma' else 'SIMT dot4'} search, "
                        + ("" if domain == ("original", "whole") else
                           f"candidate domain {a.source_policy} sources / {a.scoring} scoring, ") +
                        f"{res['run_form']} form" + (f" ({checks(a, a.form)} iterations per host check)"
                                                     if a.form != "plain" else ""),
            "width": job.width, "height": job.height, "patch": 2 * r + 1,
            "search_rect": list(res["rect"]), "candidates_per_search": res["candidates"],
            "iterations_per_removal": res["iters"][-1], "form": res["run_form"],
            "workspace_bytes": res["ws_bytes"],
        },
        "ms_per_removal": round(ms_per_step, 3),
        # the same removal from host buffers: create, upload and read-back included
        "ms_per_removal_end_to_end": (None if a.no_end_to_end else
                                      end_to_end_removal(job, a.form, checks(a, a.form), a.tile_rows, a.path)),
        "iterations_per_s": round(sum(res["iters"]) / res["seconds"], 1),
        # Eq. 4's terms (3 channels x known offsets) and the dense equivalent
        # (3 x P^2 per candidate), per second over the timed removals
        "algorithmic_terms_per_s": round(terms_per_removal * n_steps / res["seconds"], 1),
        "dense_equivalent_terms_per_s": round(3 * (2 * r + 1) ** 2 * evals / res["seconds"], 1),
        "parity": (golden_check(job, a, log, res["image"]) if domain == ("original", "whole")
                   else "no stored oracle result for this candidate domain (parity: tests/test_domains_gpu.py)"),
        "roofline": {
            "bound": "mfma" if a.path == "mfma" else "alu",
            "kernel": kernel,
            "achieved": round(OPS_PER_TERM * achieved / 1e12, 3), "peak": round(OPS_PER_TERM * peak / 1e12, 2),
            "unit": "TOP/s", "frac": round(achieved / peak, 5),
            "traffic": traffic_for(kernel, job.name, checks(a, a.form)) if persistent else None,
            "avg_launch_us": round(1000 * avg_kernel_ms, 3), "launches_timed": res["searches"],
            "terms_per_launch": round(terms_per_launch),
            "min_hbm_bytes_per_launch": bytes_per_launch,
            "hbm_frac_if_streamed": round(bytes_per_launch / (avg_kernel_ms * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "timed_kernel_share_of_step": round(res["kernel_ms"] / (1000 * res["seconds"]), 4),
        },
        "other_forms": others,
    }
    if "plain" in others:
        line["speedup_vs_plain"] = round(others["plain"]["ms_per_removal"] / ms_per_step, 3)
    if a.path != "mfma":
        line["roofline"]["frac_of_rgb_layout_ceiling"] = round(achieved / TERM_PEAK_LAYOUT, 5)
    if not a.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(job, a.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
