#!/usr/bin/env python3
"""Benchmark of the fragment-history-volume hot path on one MI355X.

One step = capture of a 200,000-triangle procedural scene into per-octant
fragment lists at octree depth 9 (512^3 leaves, 1024 samples per cube side,
tangent-space rasterization), compaction into per-octant arrays, point
splats of three 1920x1080 novel views at 0, 30 and 60 degrees, and the
learned fill (4-level U-Net, bf16 matrix cores) of those three views.
Inputs are uploaded before the timed region; every buffer is allocated once.

Prints one JSON line: whole-step fragments captured per second (`value`),
1080p views per second, per-kernel times from HIP events over the timed
region, the roofline of the dominant kernel, the learned fill's training
throughput and its PSNR gain over the plain splat (a short training run on
separate scenes, evaluated on held-out views), and the CPU oracle timed on
one host core beside it.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload pofl200k|batch64|large5m]

The other workloads (a batch of 64 scenes through one graph per step; one
5M-triangle scene at octree depth 11 with 16 4K views) print a line of the
same form for their own configuration.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0            # MI355X HBM3E, vendor figure
MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense bf16 matrix cores, vendor figure
LEVELS = 9
N_TRI = 200_000
SEED = 0
THETAS = (0.0, 30.0, 60.0)
W_OUT, H_OUT = 1920, 1080
WORKLOAD = ("pofl->pofa: 200k-tri procedural scene (seed 0), octree depth 9, "
            "3 x 1920x1080 splats at 0/30/60 deg + learned fill of the 3 views")


def host_info():
    model = ""
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                model = ln.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "cpu": model or platform.processor()}


def algorithmic_bytes(F: int, n_occ: int, n_tri: int, n_head: int, n_views: int, pix: int,
                      key_bytes: int = 4, link: bool = True, covered: int | None = None) -> dict:
    """Bytes each kernel scope must read and write at minimum, per launch
    (one step), as (read, written).

    capture.reset    4 per head entry written (8 for the counter alone when
                     no lists are linked)
    capture.setup    3 x (12 + 4) vertex bytes + 12 index bytes read, 128
                     record + 8 tile count written per triangle
    capture.raster   per fragment: 16 record + key (4, or 8 beyond 2^32
                     keys) written, 4 read and 4 written by the head exchange
                     when linking; 128 per triangle record read
    compact.hist     one key read per fragment
    compact.scatter  per fragment: 16 record + key read, 16 staged record
                     written
    compact.brick    per fragment 16 read + 16 written; 16 per table row
                     written
    splat.bin        the chunk boxes: 16 per fragment and 8 per table key
                     read (the arrays once)
    splat.splat      the tiles: 16 per fragment and 8 per table key read
                     once; per pixel and view 8 key + 4 colour + 4 depth + 1
                     coverage written and the winner's 4-byte colour read
                     (covered pixels; all pixels when `covered` is None)
    """
    n_brick = (n_head + 511) // 512
    cov = n_views * pix if covered is None else covered
    return {
        "capture.reset": (0, 4 * n_head if link else 8),
        "capture.setup": (n_tri * (3 * 16 + 12), n_tri * (128 + 8)),
        "capture.raster": (128 * n_tri + (4 * F if link else 0), F * (16 + key_bytes + (4 if link else 0))),
        "compact.hist": (key_bytes * F, 0),
        "compact.scan": (2 * 4 * n_brick, 2 * 4 * n_brick),
        "compact.scatter": (F * (16 + key_bytes), 16 * F),
        "compact.brick": (16 * F, 16 * F + 16 * n_occ),
        "splat.bin": (16 * F + 8 * n_occ, 0),
        "splat.splat": (16 * F + 8 * n_occ + 4 * cov, n_views * pix * (8 + 4 + 4 + 1)),
    }


def survey_bytes(F: int, n_occ: int, levels: int, n_views: int, pix: int) -> dict:
    """The algorithmic bytes of compaction and splat as the method's
    measurement defines them: B_c = 16F read + 16F written + 16 per table
    row + 8 per brick of 512 keys (counts and offsets); per view B_s = 16F/V
    (the fragment stream shared by the views) + 8 WH clear + 8 WH resolve
    read + 4 WH colour written + 4 WH winner gathered."""
    b_c = 32 * F + 16 * n_occ + 8 * 8 ** max(levels - 3, 0)
    b_s = 16 * F + n_views * 24 * pix
    return {"B_c": b_c, "B_s": b_s}


def compact_splat_fracs(algo: dict, F: int, n_occ: int, levels: int, n_views: int, pix: int,
                        compact_ms: float, splat_ms: float) -> dict:
    """Compaction plus splat against the HBM peak: with the method's
    algorithmic bytes B_c + sum of B_s (the headline figure), and with the
    bytes these kernels must move as built (`impl`)."""
    sb = survey_bytes(F, n_occ, levels, n_views, pix)
    t = (compact_ms + splat_ms) * 1e-3
    impl = sum(r + w for k, (r, w) in algo.items() if k.startswith(("compact.", "splat.")))
    return {"compact_splat_hbm_frac": (sb["B_c"] + sb["B_s"]) / t / 1e9 / HBM_PEAK_GBS,
            "compact_splat_bytes": {"B_c": sb["B_c"], "B_s": sb["B_s"], "impl": impl,
                                    "impl_hbm_frac": impl / t / 1e9 / HBM_PEAK_GBS,
                                    "splat_hbm_frac": sb["B_s"] / (splat_ms * 1e-3) / 1e9 / HBM_PEAK_GBS,
                                    "compact_hbm_frac": sb["B_c"] / (compact_ms * 1e-3) / 1e9 / HBM_PEAK_GBS}}


# kernel-name prefixes behind each timed scope (POFL mode)
SCOPE_KERNELS = {
    "fill.conv": ("k_conv",),
    "capture.setup": ("k_setup",), "capture.raster": ("k_raster",),
    "compact.hist": ("k_hist",), "compact.scatter": ("k_scatter",),
    "compact.brick": ("k_brick_wave", "k_brick"),
    "splat.bin": ("k_chunk_box", "k_node_box"), "splat.est": ("k_tile_est",), "splat.splat": ("k_tile_splat",),
    "ray.occupancy": ("k_occ_build",), "ray.cast": ("k_raycast",),
}


def src_digest() -> str:
    """sha256 over the HIP sources in name order (ties counter data to code)."""
    import glob
    import hashlib
    h = hashlib.sha256()
    for f in sorted(glob.glob(os.path.join(ROOT, "paper_2211_15460_amd", "csrc", "*"))):
        h.update(open(f, "rb").read())
    return h.hexdigest()


TRAFFIC_JSON = os.path.join(ROOT, "profiles", "traffic.json")


def measured_scope(scope: str):
    """(scope's counter figures, calibration) from profiles/traffic.json, or
    (None, None) when the kernels have changed since they were taken."""
    if not os.path.exists(TRAFFIC_JSON):
        return None, None
    t = json.load(open(TRAFFIC_JSON))
    if t.get("src_sha256") != src_digest():
        return None, None
    return t.get("scopes", {}).get(scope), t.get("calibration", {})


def measured_traffic(scope: str):
    """HBM bytes per launch of a scope from the committed rocprofv3 counter
    summary (profiles/traffic.json), or None when the kernels have changed
    since the counters were taken."""
    if not os.path.exists(TRAFFIC_JSON):
        return None
    t = json.load(open(TRAFFIC_JSON))
    if t.get("src_sha256") != src_digest() or scope not in t.get("scopes", {}):
        return None
    sc = t["scopes"][scope]
    return sc["read_bytes"] + sc["write_bytes"]


def _scope_of(kernel: str):
    for scope, prefixes in SCOPE_KERNELS.items():
        if any(kernel.startswith(p) for p in prefixes):
            return scope
    return None


def traffic_from(fetch_dir: str, write_dir: str, copy_mib: int, atomic_dir: str | None = None) -> dict:
    """Per-scope HBM bytes per launch from two rocprofv3 --pmc runs of this
    benchmark (FETCH_SIZE, then WRITE_SIZE; --output-format csv), each
    calibrated by what the counter reads for the plain device copy of
    copy_mib MiB that the benchmark runs first. Uses the dispatches of the
    last step (from the last triangle setup on); run with --no-train.

    With atomic_dir (a third run, counter TCC_ATOMIC_sum, with the ceiling
    probes on), each scope also gets the memory-side atomic requests per
    launch, and the calibration the requests per atomic operation of the
    probes: one per 128-byte line ("sparse", the add probe on HBM lines) and
    one per 8-byte word ("dense", the minimum probe on HBM words)."""
    import csv
    import glob
    import re

    def load(d, counter):
        f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
        if not f:
            raise SystemExit(f"no counter_collection.csv under {d}")
        per = {}
        for r in csv.DictReader(open(f[0])):
            if r["Counter_Name"] not in (counter, counter + "_sum"):
                continue
            did = int(r["Dispatch_Id"])
            name = re.sub(r"^void ", "", r["Kernel_Name"])
            name = re.sub(r"^(fhv::)?(nn::)?(\(anonymous namespace\)::)?", "", name)
            nm, v = per.get(did, (name, 0.0))
            per[did] = (nm, v + float(r["Counter_Value"]))
        return [per[k] for k in sorted(per)]

    out = {"src_sha256": src_digest(), "calibration": {}, "scopes": {}}
    for counter, d, key in (("FETCH_SIZE", fetch_dir, "read_bytes"), ("WRITE_SIZE", write_dir, "write_bytes")):
        rows = load(d, counter)
        # the calibration copy is the largest device copy of the run
        copies = [v for n, v in rows if n.startswith("__amd_rocclr_copyBuffer")]
        if not copies:
            raise SystemExit("the calibration copy is missing from the trace")
        big = max(copies)
        scale = copy_mib * 1024.0 / max(big, 1e-9)
        out["calibration"][counter] = {"copy_kib": big, "bytes_per_kib": scale * 1024.0}
        last = max(i for i, (n, _) in enumerate(rows) if n.startswith("k_setup"))
        start = last
        while start > 0 and rows[start - 1][0].startswith(("k_fill_u32", "k_fill_u64")):
            start -= 1
        acc = {}
        for n, v in rows[start:]:
            sc = _scope_of(n)
            if sc is None:
                continue
            b, c = acc.get(sc, (0.0, 0))
            acc[sc] = (b + v * scale * 1024.0, c + 1)
        for sc, (b, c) in acc.items():
            ent = out["scopes"].setdefault(sc, {"launches_per_step": c})
            ent[key] = b / c
    if atomic_dir:
        rows = load(atomic_dir, "TCC_ATOMIC")
        add = [v for n, v in rows if n.startswith("k_probe_atomic<1")]
        mn = [v for n, v in rows if n.startswith("k_probe_atomic<3")]
        if len(add) < 6 or len(mn) < 18:
            raise SystemExit("the ceiling probes are missing from the atomic-counter run")
        # probe order per operation: hbm, llc, dense_hbm, dense_llc, one
        # warm-up and five timed launches each (see ceilings())
        sparse_ops, dense_ops = (2 << 30) // 128, (2 << 30) // 8
        out["calibration"]["TCC_ATOMIC"] = {
            "requests_per_op_sparse": sum(add[1:6]) / 5 / sparse_ops,
            "requests_per_op_dense": sum(mn[13:18]) / 5 / dense_ops}
        last = max(i for i, (n, _) in enumerate(rows) if n.startswith("k_setup"))
        acc = {}
        for n, v in rows[last:]:
            sc = _scope_of(n)
            if sc is None:
                continue
            b, c = acc.get(sc, (0.0, 0))
            acc[sc] = (b + v, c + 1)
        for sc, (b, c) in acc.items():
            out["scopes"].setdefault(sc, {"launches_per_step": c})["atomic_requests"] = b / c
    return out


def unet_flops_per_pixel(levels: int = 4, training: bool = False) -> float:
    """Multiply-adds x 2 per level-0 pixel of the fill network's matrix
    products: 3x3 convs 2*9*Cin*Cout and transposed convs 2*Cin*Cout per
    output pixel of their level, the 1x1 head 2*32*3. Training adds the
    weight gradients (same count) and the input gradients (same count, all
    but the first layer)."""
    ch = [32 << l for l in range(levels)]
    fwd, first = 0.0, 0.0
    cin = 6
    for l in range(levels):
        a = 2 * 9 * cin * ch[l] / 4 ** l
        first = a if l == 0 else first
        fwd += a + 2 * 9 * ch[l] * ch[l] / 4 ** l
        cin = ch[l]
    for l in range(levels - 1):
        fwd += 2 * ch[l + 1] * ch[l] / 4 ** l + 2 * 9 * 2 * ch[l] * ch[l] / 4 ** l + 2 * 9 * ch[l] * ch[l] / 4 ** l
    fwd += 2 * 32 * 3
    return 3 * fwd - first if training else fwd


def learned_fill_report(torch, fhv, scenes, n_crops: int = 20000, eval_seeds: int = 10):
    """Train the fill on splats of the benchmark's scene family (seeds
    100-115, 1080p, two random orbit views per scene at octree depths 9 and
    8) against reference renders of the same views (the library's per-pixel
    capture of the triangles, nearest fragment kept; the tests check it
    against the oracle's direct raster), on n_crops distinct random 256x256
    crops in batches of 8; then compare PSNR of fill and plain splat on
    held-out scenes (seeds 0..eval_seeds-1, which no training scene uses) at
    30 and 60 degrees, at depth 9 (the timed step's configuration) and 8.
    Returns the report and the trained model."""
    import numpy as np
    from paper_2211_15460_amd import learned_fill as LF
    rng = np.random.default_rng(0)
    t0 = time.perf_counter()
    ts = LF.training_set(LF.gpu_reference, range(100, 116), (9, 8), 2, rng)
    torch.cuda.synchronize()
    t_data = time.perf_counter() - t0
    model = LF.FillModel(4, 0)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record()
    steps = LF.train(model, ts, n_crops, 8, 256, rng)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res = {"crops": n_crops, "train_steps": steps, "batch": "8 x 256 x 256",
           "train_views": len(ts.views), "train_scenes": "pofl_scene seeds 100-115, depths 9 and 8",
           "data_s": t_data, "train_ms_per_step": ms,
           "train_tflops": unet_flops_per_pixel(4, True) * 8 * 256 * 256 / (ms * 1e-3) / 1e12,
           "what": "train step time includes cutting the batch's crops on the device"}
    del ts
    for L, key in ((9, "eval"), (8, "eval_depth8")):
        ev = LF.evaluate(model, LF.gpu_reference, range(eval_seeds), L)
        gain = np.array([e["psnr_fill_db"] - e["psnr_splat_db"] for e in ev])
        res[key] = {"levels": L, "views": ev, "margin_db": float(gain.min()),
                    "gain_db": {"mean": float(gain.mean()), "std": float(gain.std()), "min": float(gain.min()),
                                "max": float(gain.max()), "n": int(gain.size),
                                "over": f"held-out scenes of seeds 0..{eval_seeds - 1} at 30 and 60 degrees"}}
    res["reference"] = ("library per-pixel capture of the triangles in the view, nearest fragment kept "
                        "(tests/test_learned_fill_psnr.py checks it against the oracle's direct raster)")
    return res, model


def raycast_report(torch, fhv, scenes, mesh, views, reps: int = 10) -> dict:
    """Ray casting (Sec. 3.3) of the step's scene into the same views:
    simple ray casting (R, nearest fragment) and ray casting with
    transparency (R/T, front to back until the transmittance is below
    1/256). The scene's own colours are opaque, so both run on the same
    scene with a seeded random alpha per vertex. Each figure is the mean of
    `reps` calls after two warm-ups (HIP events around the library's
    launches); a call rebuilds the octree's occupancy levels from the table
    and then casts one ray per pixel of every view."""
    import numpy as np
    rng = np.random.default_rng(7)
    alpha = rng.integers(0, 256, mesh.rgba.size, dtype=np.uint32)
    amesh = scenes.Mesh(mesh.pos, (mesh.rgba & 0x00FFFFFF) | (alpha << 24), mesh.tri, mesh.obj)
    d = fhv.desc(fhv.FHV_POFL, levels=LEVELS)
    dm = fhv.to_device(amesh)
    probe = fhv.alloc_lists(d, 1 << 16)
    fhv.capture(dm, d, probe)
    torch.cuda.synchronize()
    F = int(probe.counter.item())
    del probe
    lists = fhv.alloc_lists(d, F)
    fhv.capture(dm, d, lists)
    pofa = fhv.alloc_pofa(F)
    fhv.compact(lists, d, pofa)
    del lists
    W, H = views[0].width, views[0].height
    out = torch.empty((len(views), H, W, 4), dtype=torch.float32, device="cuda")
    ws = torch.empty(fhv.raycast_workspace(d), dtype=torch.uint8, device="cuda")
    vs = fhv.views_struct(views)
    res = {"views": len(views), "view_size": [W, H], "fragments": F, "levels": LEVELS, "tau_rt": 1.0 / 256}
    for mode, tau, name in ((fhv.FHV_RAY_NEAREST, 0.0, "R"), (fhv.FHV_RAY_BLEND, 1.0 / 256, "RT")):
        for _ in range(2):
            fhv.raycast(pofa, d, views, mode, tau, out, ws, vs)
        torch.cuda.synchronize()
        fhv.profile_begin()
        for _ in range(reps):
            fhv.raycast(pofa, d, views, mode, tau, out, ws, vs)
        prof = fhv.profile_end()
        occ = prof["ray.occupancy"][1] / reps
        cast = prof["ray.cast"][1] / reps
        res[name] = {"ms_per_call": occ + cast, "occupancy_ms": occ, "cast_ms": cast,
                     "views_per_s": len(views) / ((occ + cast) * 1e-3),
                     "rays_per_s": len(views) * W * H / (cast * 1e-3)}
    return res


def capture_variants_report(torch, fhv, mesh, reps: int = 10) -> dict:
    """The capture variants of Table 2 on the step's scene (octree depth 9):
    fragments captured and capture time (list reset, setup, scan and raster,
    summed over the passes) for 1-Pass/Normal (the step's own), 1-Pass/View,
    3-Pass/1-Way and 1-Pass/3-Way; means of `reps` captures after one
    warm-up, HIP events around the library's launches."""
    dm = fhv.to_device(mesh)
    names = {fhv.FHV_PROJ_NORMAL: "1-Pass/Normal", fhv.FHV_PROJ_VIEW: "1-Pass/View",
             fhv.FHV_PROJ_AXES_3PASS: "3-Pass/1-Way", fhv.FHV_PROJ_AXES_1PASS: "1-Pass/3-Way"}
    res = {}
    for proj, name in names.items():
        d = fhv.desc(fhv.FHV_POFL, levels=LEVELS, projection=proj)
        probe = fhv.alloc_lists(d, 1 << 16)
        fhv.capture(dm, d, probe)
        torch.cuda.synchronize()
        F = int(probe.counter.item())
        del probe
        lists = fhv.alloc_lists(d, F)
        ws = torch.empty(fhv.capture_workspace(d, mesh.n_tri), dtype=torch.uint8, device="cuda")
        fhv.capture(dm, d, lists, ws)
        torch.cuda.synchronize()
        fhv.profile_begin()
        for _ in range(reps):
            fhv.capture(dm, d, lists, ws)
        prof = fhv.profile_end()
        ms = sum(t for k, (n, t) in prof.items() if k.startswith("capture.")) / reps
        res[name] = {"fragments": F, "capture_ms": ms, "fragments_per_s": F / (ms * 1e-3),
                     "raster_launches": prof["capture.raster"][0] // reps}
        del lists, ws
    base = res["1-Pass/Normal"]
    for name, r in res.items():
        r["fragments_vs_normal"] = r["fragments"] / base["fragments"]
        r["time_vs_normal"] = r["capture_ms"] / base["capture_ms"]
    return res


def arrays_report(torch, fhv, mesh, reps: int = 10) -> dict:
    """The paper's way of creating the per-octant arrays (Sec. 3.2: count
    pass, scan, insert pass; fhv_capture_arrays) against the step's lists
    then compaction (fhv_capture + fhv_compact), on the step's scene; means
    of `reps` calls after one warm-up, HIP events around the library's
    launches. Both give the same arrays."""
    d = fhv.desc(fhv.FHV_POFL, levels=LEVELS)
    dm = fhv.to_device(mesh)
    probe = fhv.alloc_lists(d, 1 << 16)
    fhv.capture(dm, d, probe)
    torch.cuda.synchronize()
    F = int(probe.counter.item())
    del probe
    out = fhv.alloc_pofa(F)
    ws = torch.empty(fhv.capture_arrays_workspace(d, mesh.n_tri, F), dtype=torch.uint8, device="cuda")
    fhv.capture_arrays(dm, d, out, ws)
    torch.cuda.synchronize()
    assert int(out.n_frag.item()) == F
    fhv.profile_begin()
    for _ in range(reps):
        fhv.capture_arrays(dm, d, out, ws)
    prof = fhv.profile_end()
    per = {k: t / reps for k, (n, t) in prof.items() if k.startswith("arrays.")}
    return {"two_pass_ms": sum(per.values()), "stages_ms": per, "fragments": F,
            "what": "count rasterization, scans, insert rasterization, per-brick sort; compare with "
                    "stage_ms capture + compact (lists, then compaction)"}


def cpu_baseline(mesh, views, min_seconds: float = 10.0):
    """The CPU oracle, single-threaded, on the same workload: full steps
    (capture, compaction, three splats) repeated for at least min_seconds."""
    import oracle
    oracle.lib()
    n, t_all = 0, 0.0
    while t_all < min_seconds:
        t0 = time.perf_counter()
        head, pool, F = oracle.capture_pofl(mesh, LEVELS, 8 << 20)
        r = oracle.compact(head, pool, F)
        oracle.splat(1, r["key"], r["frag"], views, levels=LEVELS)
        t_all += time.perf_counter() - t0
        n += 1
        del head, pool, r
    dt = t_all / n
    return {"value": F / dt, "unit": "fragments/s", "cores": 1, "kind": "oracle",
            "sample": f"{n} full steps of the same workload ({F} fragments, 3 views each), "
                      f"{t_all:.1f} s on one core, {dt:.3f} s per step"}


def kernel_table(prof: dict, algo: dict) -> dict:
    kernels = {}
    for name, (launches, tot) in prof.items():
        avg = tot / max(launches, 1)
        r, w = algo.get(name, (0, 0))
        b = r + w
        kernels[name] = {"avg_ms": round(avg, 5), "launches": launches, "algo_bytes": b,
                         "read_bytes": r, "write_bytes": w,
                         "gbs": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 and b else None}
    return kernels


def hbm_roofline(kernels: dict) -> dict:
    """Roofline entry of the kernel scope with the largest total time; HBM
    bytes from counters are not taken for this workload (null)."""
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    return {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": dk["gbs"] / HBM_PEAK_GBS if dk["gbs"] else None, "traffic": None}


def ceilings(torch, fhv, reps: int = 5) -> dict:
    """Measured ceilings beside the vendor peaks (fhv_probe): plain copy
    bandwidth over 2 GiB, and the rate of uncontended device-scope atomics
    on a 2 GiB buffer (lines in HBM, one pass) and a 64 MiB one (lines held
    by the last-level cache, 32 passes): one atomic per 128-byte line
    ("sparse", as list-head exchanges land), or on every 8-byte word
    ("dense", as neighbouring pixels of a z-buffer do). Each figure is the
    mean of `reps` launches after one warm-up, from HIP events on the launch
    stream; the atomic probes' buffers are reset before every launch,
    outside the timing."""
    big = torch.empty(2 << 30, dtype=torch.uint8, device="cuda")
    small = torch.empty(64 << 20, dtype=torch.uint8, device="cuda")
    mid = big[:512 << 20]
    cases = [("copy", fhv.FHV_PROBE_COPY, big, 128, 1, "probe.copy"),
             ("read", fhv.FHV_PROBE_READ, big, 128, 1, "probe.read"),
             ("write", fhv.FHV_PROBE_WRITE, big, 128, 1, "probe.write"),
             ("copy_cached", fhv.FHV_PROBE_COPY_CACHED, big, 128, 1, "probe.copy_cached"),
             ("read_cached", fhv.FHV_PROBE_READ_CACHED, big, 128, 1, "probe.read_cached"),
             ("write_cached", fhv.FHV_PROBE_WRITE_CACHED, big, 128, 1, "probe.write_cached"),
             ("write_512mib", fhv.FHV_PROBE_WRITE, mid, 128, 1, "probe.write"),
             ("write_cached_512mib", fhv.FHV_PROBE_WRITE_CACHED, mid, 128, 1, "probe.write_cached"),
             ("write_cached_512mib_clean", fhv.FHV_PROBE_WRITE_CACHED, mid, 128, 1, "probe.write_cached")]
    for op, kind, scope in (("add_u32", fhv.FHV_PROBE_ADD_U32, "probe.add_u32"),
                            ("exch_u32", fhv.FHV_PROBE_EXCH_U32, "probe.exch_u32"),
                            ("min_u64", fhv.FHV_PROBE_MIN_U64, "probe.min_u64")):
        cases.append((op + ".hbm", kind, big, 128, 1, scope))
        cases.append((op + ".llc", kind, small, 128, 32, scope))
        if kind != fhv.FHV_PROBE_EXCH_U32:
            cases.append((op + ".dense_hbm", kind, big, 8, 1, scope))
            cases.append((op + ".dense_llc", kind, small, 8, 32, scope))
    streams = (fhv.FHV_PROBE_COPY, fhv.FHV_PROBE_READ, fhv.FHV_PROBE_WRITE, fhv.FHV_PROBE_COPY_CACHED,
               fhv.FHV_PROBE_READ_CACHED, fhv.FHV_PROBE_WRITE_CACHED)
    res = {}
    for name, kind, buf, line, passes, scope in cases:
        tot = 0.0
        # a stream runs as in a steady state, launch after launch on a buffer
        # filled once (a fill right before each launch would leave its own
        # written lines in the caches for the probe to write back); the
        # atomic probes start from a freshly filled buffer every time
        if kind in streams:
            buf.fill_(0xFF)
        for r in range(reps + 1):
            if kind not in streams:
                buf.fill_(0xFF)
            if name.endswith("_clean"):
                # a read-only stream over the rest of the 2 GiB buffer first,
                # untimed: the previous launch's written lines leave the
                # caches and the write starts with none to write back
                fhv.probe(fhv.FHV_PROBE_READ, big[512 << 20:])
            torch.cuda.synchronize()
            fhv.profile_begin()
            fhv.probe(kind, buf, line, passes)
            prof = fhv.profile_end()
            if r > 0:
                tot += prof[scope][1]
        ms = tot / reps
        if kind in streams:
            res.setdefault("streams_gbs", {})[name] = buf.numel() / (ms * 1e-3) / 1e9
        else:
            res.setdefault("atomics_g_per_s", {})[name] = buf.numel() // line * passes / (ms * 1e-3) / 1e9
    del big, small, mid
    # the stream ceilings over 2 GiB (far beyond the last-level cache): the
    # faster of the two access forms
    st = res["streams_gbs"]
    for k in ("copy", "read", "write"):
        res[k + "_gbs"] = max(st[k], st[k + "_cached"])
    # the matrix cores' practical rate: the vendor library's bf16 GEMM
    # (torch.matmul, fp32 accumulation) on 8192^3, the best case for it
    n = 8192
    ga = torch.randn(n, n, dtype=torch.bfloat16, device="cuda")
    gb = torch.randn(n, n, dtype=torch.bfloat16, device="cuda")
    for _ in range(3):
        torch.matmul(ga, gb)
    ms = timed(torch, lambda: torch.matmul(ga, gb), 10)
    res["gemm_bf16_tflops"] = 2.0 * n ** 3 / (ms * 1e-3) / 1e12
    del ga, gb
    res["note"] = ("copy: GB/s read+written over 2 GiB; read, write: GB/s of a read-only and a write-only "
                   "stream over 2 GiB; each the faster of non-temporal and ordinary accesses (streams_gbs: "
                   "both forms, and the write-only stream over 512 MiB, also right after a read of other memory (_clean), "
                   "as a kernel that follows kernels writing little starts); "
                   "atomics: G ops/s; hbm = 2 GiB buffer, one pass; "
                   "llc = 64 MiB buffer, 32 passes; one atomic per 128-B line, or per 8-B word (dense); "
                   "exch returns its value; gemm: the vendor library's bf16 matmul, 8192^3, TFLOP/s")
    return res


def add_ceilings(args, out: dict, torch, fhv, kernels: dict, n_exch: int | None, counters: bool = False):
    """Adds the measured ceilings, the streaming kernels' fraction of the
    measured copy bandwidth and, when the capture keeps list heads, the
    raster's head exchanges (one returning u32 atomic per fragment, on a head
    array in HBM) against the measured exchange rate. `counters`: the
    committed counter figures were taken on this workload, so the splat's
    measured atomic requests are reported too."""
    if args.no_ceilings:
        return
    ceil = ceilings(torch, fhv)
    out["ceilings"] = ceil
    # each streaming kernel against the stream ceiling of its own mix of
    # reads and writes: the time the read-only and write-only probes would
    # take for its bytes, added
    sf = {}
    for k in ("capture.reset", "compact.hist", "compact.scatter", "compact.brick", "splat.bin", "splat.splat"):
        kk = kernels.get(k, {})
        if not kk.get("avg_ms") or not (kk.get("read_bytes") or kk.get("write_bytes")):
            continue
        r, w = kk["read_bytes"], kk["write_bytes"]
        t_ceil = r / (ceil["read_gbs"] * 1e9) + w / (ceil["write_gbs"] * 1e9)
        sf[k] = t_ceil / (kk["avg_ms"] * 1e-3)
    out["stream_frac"] = sf
    if kernels.get("fill.conv", {}).get("tflops"):
        out["gemm_frac"] = {"fill.conv": kernels["fill.conv"]["tflops"] / ceil["gemm_bf16_tflops"]}
    r_ms = kernels.get("capture.raster", {}).get("avg_ms")
    if n_exch and r_ms:
        # one exchange per fragment; samples next to each other in a tile
        # often hit one 64-byte line and share a memory-side request, so the
        # request count (from the committed counters, when they were taken
        # on this workload) is what meets the ceiling
        ops = n_exch / (r_ms * 1e-3) / 1e9
        peak = ceil["atomics_g_per_s"]["exch_u32.hbm"]     # one request per exchange there
        sc, cal = measured_scope("capture.raster") if counters else (None, None)
        if sc and sc.get("atomic_requests"):
            req = sc["atomic_requests"] / (r_ms * 1e-3) / 1e9
            out["atomic_roofline"] = {"kernel": "capture.raster", "achieved": req, "peak": peak,
                                      "unit": "G memory-side atomic requests/s", "frac": req / peak,
                                      "exchanges_g_per_s": ops,
                                      "what": "the raster's memory-side atomic requests (list-head exchanges "
                                              "and counters, from the counter run) against the measured rate "
                                              "of uncontended returning u32 exchanges, one request each"}
        else:
            out["atomic_roofline"] = {"kernel": "capture.raster", "achieved": None, "peak": peak,
                                      "unit": "G memory-side atomic requests/s", "frac": None,
                                      "exchanges_g_per_s": ops,
                                      "what": "requests not counted for this workload; exchanges per second "
                                              "exceed the one-request-per-exchange rate where samples share "
                                              "lines"}


def timed(torch, fn, steps: int) -> float:
    """Milliseconds per call of fn over `steps` calls, HIP events on the
    current stream."""
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    ev0.record()
    for _ in range(steps):
        fn()
    ev1.record()
    torch.cuda.synchronize()
    return ev0.elapsed_time(ev1) / steps


def bench_batch64(args, torch, fhv, scenes):
    """64 scenes (triangle counts log-uniform in [1e3, 5e5]) at octree depth
    9, 8 views each at 1280x720 (45 degrees apart): capture, compaction and
    splat of the whole batch per step, through fhv_batch_run. The launch
    choices are autotuned on the batch first; the timed steps replay the
    recorded graph (eager launches are timed and profiled separately)."""
    import numpy as np
    L, V, W, H = 9, 8, 1280, 720
    meshes = scenes.batched_scenes(SEED, 64)
    n_tri = sum(m.tri.shape[0] for m in meshes)
    b = fhv.to_device_batch(meshes, L)
    views = [[scenes.cube_view(45.0 * v, L, W, H) for v in range(V)] for _ in meshes]
    vm = fhv.batch_view_matrices(views)
    k = views[0][0].splat_px
    img = fhv.alloc_images(len(meshes) * V, W, H)
    probe, probe_pofa = fhv.alloc_batch_lists(b, 1 << 16), fhv.alloc_pofa(1 << 16)
    fhv.batch_run(b, vm, W, H, k, probe, probe_pofa, img)
    torch.cuda.synchronize()
    F = int(probe.counter.item())
    del probe, probe_pofa
    cap = ((F >> 20) + 1) << 20
    lists, pofa = fhv.alloc_batch_lists(b, cap), fhv.alloc_pofa(cap)
    ws = fhv.batch_run(b, vm, W, H, k, lists, pofa, img, flags=fhv.FHV_BATCH_TUNE)
    tuning = fhv.get_tuning()
    eager = lambda: fhv.batch_run(b, vm, W, H, k, lists, pofa, img, ws=ws)
    graph = lambda: fhv.batch_run(b, vm, W, H, k, lists, pofa, img, ws=ws, flags=fhv.FHV_BATCH_GRAPH)
    for _ in range(args.warmup):
        eager()
    fhv.profile_begin()
    ms_eager = timed(torch, eager, args.steps)
    prof = fhv.profile_end()
    for _ in range(args.warmup):
        graph()
    t0 = time.perf_counter()
    ms_graph = timed(torch, graph, args.steps)
    wall = time.perf_counter() - t0
    assert int(lists.counter.item()) == F
    n_occ = int(pofa.n_occ.item())
    n_views = len(meshes) * V
    algo = algorithmic_bytes(F, n_occ, n_tri, len(meshes) * 8 ** L, n_views, W * H, key_bytes=8,
                             link=False)
    kernels = kernel_table(prof, algo)
    for kk in kernels.values():
        kk["launches_per_step"] = kk["launches"] / args.steps
    stage = lambda pre: sum(kernels[k]["avg_ms"] * kernels[k]["launches"] / args.steps
                            for k in kernels if k.startswith(pre))
    out = {
        "metric": "fragments captured/s; 1080p novel views/s; learned-fill vs plain-splat PSNR",
        "value": F / (ms_graph * 1e-3), "unit": "fragments/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_graph, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "batched: 64 procedural scenes (seed 0), triangle counts log-uniform in "
                               "[1e3, 5e5], octree depth 9, 8 views each at 1280x720, one graph per step",
                   "scenes": len(meshes), "n_tri": n_tri, "levels": L, "fragments": F,
                   "occupied_octants": n_occ, "views": n_views, "view_size": [W, H]},
        "scenes_per_s": len(meshes) / (ms_graph * 1e-3),
        "views_per_s_720p": n_views / (ms_graph * 1e-3),
        "ms_per_step_eager": ms_eager,
        "graph_saves_ms": ms_eager - ms_graph,
        "stage_ms": {"capture": stage("capture."), "compact": stage("compact."), "splat": stage("splat.")},
        **compact_splat_fracs(algo, F, n_occ, L, n_views, W * H, stage("compact."), stage("splat.")),
        "tuning": tuning,
        "kernels": kernels,
        "roofline": hbm_roofline(kernels),
        "wall_s_timed": wall,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
    }
    add_ceilings(args, out, torch, fhv, kernels, None)     # a batch keeps no list heads
    if not args.no_cpu_baseline:
        import oracle
        oracle.lib()
        n_s, n_f, t_all = 0, 0, 0.0
        for m, vs in zip(meshes, views):
            t1 = time.perf_counter()
            head, pool, Fs = oracle.capture_pofl(m, L, 32 << 20)
            r = oracle.compact(head, pool, Fs)
            oracle.splat(1, r["key"], r["frag"], vs, levels=L)
            t_all += time.perf_counter() - t1
            n_s, n_f = n_s + 1, n_f + Fs
            del head, pool, r
            if t_all >= 10.0:
                break
        out["cpu_baseline"] = {"value": n_f / t_all, "unit": "fragments/s", "cores": 1, "kind": "oracle",
                               "sample": f"the first {n_s} scenes of the batch, each captured, compacted "
                                         f"and splatted into its 8 views ({n_f} fragments, {t_all:.1f} s "
                                         "on one core)"}
    return out


def bench_ppfl64(args, torch, fhv, scenes):
    """The per-pixel case: 64 random clip-space triangles captured into
    per-pixel fragment lists at 128x128 (pool of 2^18 records), compacted
    into per-pixel arrays and splatted at 30 degrees into one 128x128 view.
    About 80k fragments: a latency-bound correctness configuration, timed
    for completeness (the roofline entry is the dominant kernel's, with no
    claim of being near it)."""
    Wc = Hc = 128
    cap = 1 << 18
    mesh = scenes.ppfl_plain(SEED)
    views = [scenes.ppfl_view(30.0, Wc, Hc)]
    d = fhv.desc(fhv.FHV_PPFL, Wc, Hc)
    dm = fhv.to_device(mesh)
    lists = fhv.alloc_lists(d, cap)
    pofa = fhv.alloc_pofa(cap)
    imgs = fhv.alloc_images(1, Wc, Hc)
    ws_c = torch.empty(fhv.capture_workspace(d, mesh.n_tri), dtype=torch.uint8, device="cuda")
    ws_k = torch.empty(fhv.compact_workspace(d, cap), dtype=torch.uint8, device="cuda")
    ws_s = torch.empty(fhv.splat_workspace(cap, 1, Wc, Hc), dtype=torch.uint8, device="cuda")
    vs = fhv.views_struct(views)

    def step():
        fhv.capture(dm, d, lists, ws_c)
        fhv.compact(lists, d, pofa, ws_k)
        fhv.splat(pofa, d, views, imgs, vs, ws_s)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    F = int(lists.counter.item())
    assert 0 < F <= cap
    fhv.profile_begin()
    t0 = time.perf_counter()
    ms = timed(torch, step, args.steps)
    wall = time.perf_counter() - t0
    prof = fhv.profile_end()
    n_occ = int(pofa.n_occ.item())
    algo = algorithmic_bytes(F, n_occ, mesh.n_tri, Wc * Hc, 1, Wc * Hc)
    kernels = kernel_table(prof, algo)
    stage = lambda pre: sum(kernels[k]["avg_ms"] * kernels[k]["launches"] / args.steps
                            for k in kernels if k.startswith(pre))
    out = {
        "metric": "fragments captured/s; 1080p novel views/s; learned-fill vs plain-splat PSNR",
        "value": F / (ms * 1e-3), "unit": "fragments/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "ppfl plain: 64 random clip-space triangles (seed 0), 128x128 per-pixel "
                               "lists, pool 2^18, one 128x128 splat at 30 deg",
                   "n_tri": mesh.n_tri, "fragments": F, "occupied_pixels": n_occ, "views": 1,
                   "view_size": [Wc, Hc]},
        "stage_ms": {"capture": stage("capture."), "compact": stage("compact."), "splat": stage("splat.")},
        "kernels": kernels,
        "roofline": hbm_roofline(kernels),
        "wall_s_timed": wall,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
    }
    if not args.no_cpu_baseline:
        import oracle
        oracle.lib()
        n, t_all = 0, 0.0
        while t_all < 10.0:
            t1 = time.perf_counter()
            oh, op, Fs = oracle.capture_ppfl(mesh, Wc, Hc, cap)
            r = oracle.compact(oh, op, Fs)
            oracle.splat(0, r["key"], r["frag"], views, width_cap=Wc)
            t_all += time.perf_counter() - t1
            n += 1
        out["cpu_baseline"] = {"value": Fs * n / t_all, "unit": "fragments/s", "cores": 1, "kind": "oracle",
                               "sample": f"the whole step ({Fs} fragments), {n} runs, {t_all:.1f} s on one core"}
    return out


def bench_large5m(args, torch, fhv, scenes):
    """One 5M-triangle scene (20,000 objects) at octree depth 11 (2048^3
    leaves, 64-bit keys), about 0.9e9 fragments; 16 views at 3840x2160,
    22.5 degrees apart. Each step: capture, compaction, splat of the 16
    views."""
    import numpy as np
    L, V, W, H = 11, 16, 3840, 2160
    mesh = scenes.large_scene(SEED)
    views = [scenes.cube_view(22.5 * v, L, W, H) for v in range(V)]
    d = fhv.desc(fhv.FHV_POFL, levels=L)
    dm = fhv.to_device(mesh)
    head = torch.empty(8 ** L, dtype=torch.int32, device="cuda")
    probe = fhv.Lists(head, torch.empty((1 << 16, 4), dtype=torch.int32, device="cuda"),
                      torch.empty(1 << 16, dtype=torch.int64, device="cuda"),
                      torch.zeros(1, dtype=torch.int64, device="cuda"), 1 << 16)
    fhv.capture(dm, d, probe)
    torch.cuda.synchronize()
    F = int(probe.counter.item())
    del probe
    cap = ((F >> 20) + 1) << 20
    lists = fhv.Lists(head, torch.empty((cap, 4), dtype=torch.int32, device="cuda"),
                      torch.empty(cap, dtype=torch.int64, device="cuda"),
                      torch.zeros(1, dtype=torch.int64, device="cuda"), cap)
    pofa = fhv.alloc_pofa(cap)
    imgs = fhv.alloc_images(V, W, H)
    ws_c = torch.empty(fhv.capture_workspace(d, mesh.n_tri), dtype=torch.uint8, device="cuda")
    ws_k = torch.empty(fhv.compact_workspace(d, cap), dtype=torch.uint8, device="cuda")
    ws_s = torch.empty(fhv.splat_workspace(cap, V, W, H), dtype=torch.uint8, device="cuda")
    vs = fhv.views_struct(views)

    def step():
        fhv.capture(dm, d, lists, ws_c)
        fhv.compact(lists, d, pofa, ws_k)
        fhv.splat(pofa, d, views, imgs, vs, ws_s)

    for _ in range(args.warmup):
        step()
    fhv.profile_begin()
    t0 = time.perf_counter()
    ms = timed(torch, step, args.steps)
    wall = time.perf_counter() - t0
    prof = fhv.profile_end()
    assert int(lists.counter.item()) == F
    n_occ = int(pofa.n_occ.item())
    algo = algorithmic_bytes(F, n_occ, mesh.n_tri, 8 ** L, V, W * H, key_bytes=8)
    kernels = kernel_table(prof, algo)
    stage = lambda pre: sum(kernels[k]["avg_ms"] * kernels[k]["launches"] / args.steps
                            for k in kernels if k.startswith(pre))
    out = {
        "metric": "fragments captured/s; 1080p novel views/s; learned-fill vs plain-splat PSNR",
        "value": F / (ms * 1e-3), "unit": "fragments/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int64", "data": "synthetic",
        "config": {"workload": "large pofa: 5M-tri procedural scene (seed 0, 20k objects), octree depth 11, "
                               "16 x 3840x2160 splats 22.5 deg apart",
                   "n_tri": mesh.n_tri, "levels": L, "fragments": F, "occupied_octants": n_occ,
                   "views": V, "view_size": [W, H]},
        "views_per_s_4k": V / (ms * 1e-3),
        "stage_ms": {"capture": stage("capture."), "compact": stage("compact."), "splat": stage("splat.")},
        **compact_splat_fracs(algo, F, n_occ, L, V, W * H, stage("compact."), stage("splat.")),
        "kernels": kernels,
        "roofline": hbm_roofline(kernels),
        "wall_s_timed": wall,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
    }
    add_ceilings(args, out, torch, fhv, kernels, F)
    if not args.no_cpu_baseline:
        # the oracle cannot hold 8^11 list heads: it captures the keys of one
        # level-3 sub-cube (8^8 keys) from the triangles whose snapped
        # bounding box meets that sub-cube, and compacts them
        import oracle
        oracle.lib()
        G = 2 ** (L + 8)
        sh = L + 8 - 3
        g = np.minimum(np.floor(mesh.pos.astype(np.float64) * G), G - 1).astype(np.int64)
        tg = g[mesh.tri]                                   # [nt, 3, 3]
        lo_c, hi_c = tg.min(axis=1) >> sh, tg.max(axis=1) >> sh
        top = g[mesh.tri[0, 0]] >> sh
        sel = np.all((lo_c <= top) & (hi_c >= top), axis=1)
        sub = scenes.Mesh(mesh.pos, mesh.rgba, mesh.tri[sel], mesh.obj[sel])
        span = 8 ** (L - 3)
        key_lo = oracle.morton3(int(top[0]), int(top[1]), int(top[2]), 3) * span
        n, t_all = 0, 0.0
        while t_all < 10.0:
            t1 = time.perf_counter()
            oh, op, Fs = oracle.capture_pofl_range(sub, L, key_lo, key_lo + span, 64 << 20)
            oracle.compact(oh, op, Fs)
            t_all += time.perf_counter() - t1
            n += 1
        out["cpu_baseline"] = {"value": Fs * n / t_all, "unit": "fragments/s", "cores": 1, "kind": "oracle",
                               "sample": f"capture and compaction of one level-3 sub-cube (8^8 keys, {Fs} "
                                         f"fragments) from the {int(sel.sum())} triangles meeting it, {n} "
                                         f"runs, {t_all:.1f} s on one core"}
    return out


WORKLOADS = {"pofl200k": None, "batch64": bench_batch64, "large5m": bench_large5m, "ppfl64": bench_ppfl64}
DEFAULT_STEPS = {"pofl200k": (50, 5), "batch64": (10, 2), "large5m": (4, 1), "ppfl64": (200, 20)}


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None)
    ap.add_argument("--warmup", type=int, default=None)
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="pofl200k",
                    help="pofl200k (default): 200k triangles, depth 9, 3 x 1080p views + fill; "
                         "batch64: 64 scenes x 8 views at 720p in one graph; "
                         "large5m: 5M triangles, depth 11, 16 x 4K views; "
                         "ppfl64: 64 triangles, per-pixel lists at 128x128")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-train", action="store_true", help="skip the learned-fill training report")
    ap.add_argument("--no-raycast", action="store_true", help="skip the ray casting report")
    ap.add_argument("--no-variants", action="store_true", help="skip the capture-variant report")
    ap.add_argument("--no-ceilings", action="store_true",
                    help="skip the measured copy and atomic ceilings (fhv_probe)")
    ap.add_argument("--copy-mib", type=int, default=256,
                    help="size of a plain device copy run once before the steps, so that "
                         "hardware byte counters can be calibrated against a known size")
    ap.add_argument("--traffic-from", nargs="+", metavar="DIR",
                    help="write profiles/traffic.json from rocprofv3 --pmc runs of this benchmark "
                         "(FETCH_SIZE dir, WRITE_SIZE dir[, TCC_ATOMIC_sum dir]; csv output) and exit")
    args = ap.parse_args()
    if args.traffic_from:
        if len(args.traffic_from) not in (2, 3):
            raise SystemExit("--traffic-from takes two or three directories")
        t = traffic_from(*args.traffic_from[:2], args.copy_mib,
                         args.traffic_from[2] if len(args.traffic_from) == 3 else None)
        json.dump(t, open(TRAFFIC_JSON, "w"), indent=1)
        print(json.dumps(t["scopes"]))
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: this path runs on a single MI355X; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    ds, dw = DEFAULT_STEPS[args.workload]
    args.steps = ds if args.steps is None else args.steps
    args.warmup = dw if args.warmup is None else args.warmup

    import torch
    from paper_2211_15460_amd import fhv, scenes

    torch.cuda.set_device(0)
    if WORKLOADS[args.workload] is not None:
        print(json.dumps(WORKLOADS[args.workload](args, torch, fhv, scenes)), flush=True)
        return
    mesh = scenes.pofl_scene(SEED, N_TRI)
    views = [scenes.cube_view(th, LEVELS, W_OUT, H_OUT) for th in THETAS]
    d = fhv.desc(fhv.FHV_POFL, levels=LEVELS)
    dm = fhv.to_device(mesh)

    # size the pool from a first capture, as a caller would after overflow
    probe = fhv.alloc_lists(d, 1 << 16)
    fhv.capture(dm, d, probe)
    torch.cuda.synchronize()
    F = int(probe.counter.item())
    del probe
    cap = ((F >> 20) + 1) << 20
    lists = fhv.alloc_lists(d, cap)
    pofa = fhv.alloc_pofa(cap)
    imgs = fhv.alloc_images(len(views), W_OUT, H_OUT)
    ws_c = torch.empty(fhv.capture_workspace(d, mesh.n_tri), dtype=torch.uint8, device="cuda")
    ws_k = torch.empty(fhv.compact_workspace(d, cap), dtype=torch.uint8, device="cuda")
    ws_s = torch.empty(fhv.splat_workspace(cap, len(views), W_OUT, H_OUT), dtype=torch.uint8, device="cuda")
    vs = fhv.views_struct(views)
    from paper_2211_15460_amd import learned_fill as LF
    lf_report = None
    if not args.no_train:
        # the fill is trained first, so that the timed step runs the trained
        # network
        lf_report, lf_model = learned_fill_report(torch, fhv, scenes)
        fill_params = lf_model.params
    else:
        fill_params = torch.from_numpy(LF.init_params(0, 4)).cuda()
    ws_f = torch.empty(fhv.fill_workspace(4, len(views), H_OUT, W_OUT, False), dtype=torch.uint8,
                       device="cuda")

    def step():
        fhv.capture(dm, d, lists, ws_c)
        fhv.compact(lists, d, pofa, ws_k)
        fhv.splat(pofa, d, views, imgs, vs, ws_s)
        fhv.fill(fill_params, imgs.rgba, imgs.depth, imgs.cov, 4, ws=ws_f)

    if args.copy_mib > 0:
        src = torch.empty(args.copy_mib << 20, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    assert int(lists.counter.item()) == F
    n_occ = int(pofa.n_occ.item())

    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    fhv.profile_begin()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record()
    for _ in range(args.steps):
        step()
    ev1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    prof = fhv.profile_end()
    ms_step = ev0.elapsed_time(ev1) / args.steps

    n_head = 8 ** LEVELS
    pix = W_OUT * H_OUT
    algo = algorithmic_bytes(F, n_occ, mesh.n_tri, n_head, len(views), pix)
    fill_flops = unet_flops_per_pixel(4) * len(views) * pix      # per step
    kernels = {}
    for name, (launches, tot) in prof.items():
        per_step = launches / args.steps
        avg = tot / max(launches, 1)
        if name == "fill.conv":
            fl = fill_flops / per_step      # matrix-product flops per launch, averaged
            kernels[name] = {"avg_ms": round(avg, 5), "launches": launches, "algo_flops": fl,
                             "tflops": round(fl / (avg * 1e-3) / 1e12, 2) if avg > 0 else None}
            continue
        r, w = algo.get(name, (0, 0))
        b = r + w
        kernels[name] = {"avg_ms": round(avg, 5), "launches": launches, "algo_bytes": b,
                         "read_bytes": r, "write_bytes": w,
                         "gbs": round(b / (avg * 1e-3) / 1e9, 1) if avg > 0 else None}
    dom = max(kernels, key=lambda k: kernels[k]["avg_ms"] * kernels[k]["launches"])
    dk = kernels[dom]
    stage = lambda pre: sum(kernels[k]["avg_ms"] * kernels[k]["launches"] / args.steps
                            for k in kernels if k.startswith(pre))
    splat_ms, capture_ms, compact_ms, fill_ms = stage("splat."), stage("capture."), stage("compact."), stage("fill.")
    if dom == "fill.conv":
        roof = {"bound": "mfma", "kernel": "k_conv (fill.conv)", "achieved": dk["tflops"],
                "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": dk["tflops"] / MFMA_BF16_PEAK_TFLOPS if dk["tflops"] else None,
                "traffic": measured_traffic(dom)}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": dk["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": dk["gbs"] / HBM_PEAK_GBS if dk["gbs"] else None,
                "traffic": measured_traffic(dom)}
    out = {
        "metric": "fragments captured/s; 1080p novel views/s; learned-fill vs plain-splat PSNR",
        "value": F / (ms_step * 1e-3),
        "unit": "fragments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int64",
        "data": "synthetic",
        "config": {"workload": WORKLOAD, "n_tri": mesh.n_tri, "levels": LEVELS,
                   "fragments": F, "occupied_octants": n_occ, "views": len(views),
                   "view_size": [W_OUT, H_OUT],
                   "fill_weights": "trained (learned_fill)" if lf_report is not None else "untrained (--no-train)"},
        "views_per_s_1080p": len(views) / (ms_step * 1e-3),
        "splat_views_per_s_1080p": len(views) / (splat_ms * 1e-3),
        "capture_fragments_per_s": F / (capture_ms * 1e-3),
        "fill_ms_per_1080p_view": fill_ms / len(views),
        "fill_tflops": fill_flops / (fill_ms * 1e-3) / 1e12 if fill_ms else None,
        "stage_ms": {"capture": capture_ms, "compact": compact_ms, "splat": splat_ms, "fill": fill_ms},
        **compact_splat_fracs(algo, F, n_occ, LEVELS, len(views), pix, compact_ms, splat_ms),
        "kernels": kernels,
        "roofline": roof,
        "wall_s_timed": wall,
        "host": host_info(),
        "device": torch.cuda.get_device_name(0),
    }
    add_ceilings(args, out, torch, fhv, kernels, F, counters=True)
    if not args.no_raycast:
        out["raycast"] = raycast_report(torch, fhv, scenes, mesh, views)
    if not args.no_variants:
        out["capture_variants"] = capture_variants_report(torch, fhv, mesh)
        out["pofa_two_pass"] = arrays_report(torch, fhv, mesh)
        # Blinn-Phong shading of the step's three splats (Sec. 5)
        import numpy as np
        lights = np.stack([fhv.light_vectors(v, (0.3, 1.0, -0.5)) for v in views])
        fhv.shade(pofa, imgs, lights)
        torch.cuda.synchronize()
        fhv.profile_begin()
        for _ in range(10):
            fhv.shade(pofa, imgs, lights)
        sh = fhv.profile_end()["shade"][1] / 10
        out["shade"] = {"ms_per_call": sh, "views": len(views), "views_per_s": len(views) / (sh * 1e-3),
                        "bytes": len(views) * W_OUT * H_OUT * (8 + 16),
                        "gbs": len(views) * W_OUT * H_OUT * (8 + 16) / (sh * 1e-3) / 1e9,
                        "what": "per pixel: z-buffer key read, float4 written (plus the winner's record)"}
    if lf_report is not None:
        # the timed step's own three views: plain splat and trained fill
        # against the reference render
        fimg, _ = fhv.fill(fill_params, imgs.rgba, imgs.depth, imgs.cov, 4, ws=ws_f)
        torch.cuda.synchronize()
        lf_report["step_views"] = [
            {"theta": th, "psnr_splat_db": LF.psnr_rgb(imgs.rgba[i], ref),
             "psnr_fill_db": LF.psnr_rgb(fimg[i], ref)}
            for i, (th, ref) in enumerate((th, LF.gpu_reference(mesh, LEVELS, v)) for th, v in zip(THETAS, views))]
        out["learned_fill"] = lf_report
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(mesh, views)
        # the oracle's step has no fill: the GPU's time for the same work
        gpu_ms = capture_ms + compact_ms + splat_ms
        out["cpu_baseline"]["gpu_same_work"] = {
            "value": F / (gpu_ms * 1e-3), "unit": "fragments/s", "ms": gpu_ms,
            "what": "capture + compaction + three splats of the timed step (no fill), as the oracle's step"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
