"""Throughput of the volumetric filtering hot path on one MI355X.

Default workload ("headline"): the precision form at full size.  A 2048^3
porous phantom with values in [0, 1] sits in HBM; one timed step = Gaussian
smoothing with sigma 1 and sigma 4 (truncate 3, reflect) in plain FP32;
value = output voxels per second of that step (2 x 2048^3 per step), in
GVox/s.  The same two filters with the volume stored in BF16 and in FP16
(FP32 accumulation) are timed too, and every filter's max / mean relative
error against the FP64 oracle on sampled blocks is reported beside its rate.
The resident 1024^3 FP32 ops (Gaussian sigma 1, 2, 4, grayscale ball-3
erosion + dilation, binary erosion + dilation) ride along in ops.

Per-op times are measured with HIP events on the stream the library launches
on (torch's current stream).  The roofline block reports the dominant
kernel of the step: algorithmic flops (or bytes) per launch over its average
event-timed duration, against the MI355X peak.  The oracle legs (CPU
baseline: the FP64 oracle on a bounded sample of the same workload, timed on
this host's cores, all and one, median of 3; and the sampled accuracy
figures) are skipped with --no-cpu.

Other workloads (--workload): "resident" (the 1024^3 FP32 ops alone),
"precision" (2048^3 rates without the oracle), "chunked" (2048^3 uint16 in
pinned host memory, 8 GiB device budget, 512^3 bricks: Gaussian sigma 2 to
float32 and binary opening with the radius-2 ball on threshold 32768),
"batched" (64 uneven float32 crops, learnable-sigma Gaussian + box-5
dilation, forward + backward in one graph), "filters" (the next filters of
the suite at 1024^3).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# tiles chosen by the library's autotuner for these workloads on MI355X
# (written by `bench.py --tune`, loaded by every other run)
TILES = os.path.join(ROOT, "paper_2511_11890_amd", "tiles_mi355x.txt")

METRIC = "GVox/s plain FP32 vs BF16+fused fwd/bwd filter at stated err; % HBM peak"
HBM_PEAK_GBS = 8000.0
# fp32 vector peak of the chip: 256 CU x 4 SIMD x 16 lanes x 2 (packed dual
# FP32) x 2 flop per FMA x 2.4 GHz
FP32_VECTOR_PEAK_TFLOPS = 157.3

KERNEL_SOURCES = {
    "gauss": ["paper_2511_11890_amd/csrc/common.h", "paper_2511_11890_amd/csrc/gauss_grid.h",
              "paper_2511_11890_amd/csrc/gauss_impl.h", "paper_2511_11890_amd/csrc/gauss_f32.hip"],
    "morph": ["paper_2511_11890_amd/csrc/common.h", "paper_2511_11890_amd/csrc/morph_impl.h",
              "paper_2511_11890_amd/csrc/morph_f32.hip"],
    "bits": ["paper_2511_11890_amd/csrc/common.h", "paper_2511_11890_amd/csrc/morph_impl.h",
             "paper_2511_11890_amd/csrc/morph_bits_u8.hip", "paper_2511_11890_amd/csrc/morph_bits_u16.hip"],
}

# kernel-name fragments of the 2048^3 FP32 ops of the headline step
HEADLINE_KERNELS = {
    "f32_sigma1": ("gauss", "gauss_fused_kernel<float, float, 3,"),
    "f32_sigma4": ("gauss", "gauss_fused_kernel<float, float, 12,"),
}

# kernel-name fragments of the resident workload's ops (fused kernels), with
# their algorithmic bytes per voxel where the op is not f32 in, f32 out
RESIDENT_KERNELS = {
    "gauss_s1": ("gauss", "gauss_fused_kernel<float, float, 3,"),
    "gauss_s2": ("gauss", "gauss_fused_kernel<float, float, 6,"),
    "gauss_s4": ("gauss", "gauss_fused_kernel<float, float, 12,"),
    "erode_dilate_ball3": ("morph", "gray_kernel<float, 1, 3, true>"),
    "bin_u8_box1": ("bits", "bits_kernel<unsigned char, 0, 1, true>", 3),
    "bin_u16_ball2": ("bits", "bits_kernel<unsigned short, 1, 2, true>", 4),
}


def sources_sha(kind: str) -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES[kind]:
        with open(os.path.join(ROOT, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def traffic_for(op_name: str, kind: str, size: int):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if
    it was taken on the current kernel source at this size; else None."""
    for path in glob.glob(os.path.join(ROOT, "profiles", "*traffic*.json")):
        try:
            with open(path) as f:
                d = json.load(f)
        except (OSError, ValueError):
            continue
        op = d.get("ops", {}).get(op_name)
        if op and d.get("size") == size and d.get("source_sha", {}).get(kind) == sources_sha(kind):
            return op.get("hbm_bytes_per_launch")
    return None


def tiles_load(path: str) -> dict:
    """Load the autotuner's recorded tiles, if the file exists."""
    import paper_2511_11890_amd as h

    if not os.path.exists(path):
        return {"source": "heuristic"}
    h.tune_load(path)
    return {"source": os.path.relpath(path, ROOT), "entries": h.tune_entries()}


def tiles_merge_save(path: str) -> dict:
    """Merge the tiles recorded in this process into the tile file."""
    import paper_2511_11890_amd as h

    mine = os.path.join(os.path.dirname(path), ".tiles_new.txt")
    h.tune_save(mine)
    if os.path.exists(path):
        h.tune_load(path)   # older entries ...
        h.tune_load(mine)   # ... overridden by this run's
    h.tune_save(path)
    os.remove(mine)
    return {"source": "autotuned in this run, saved to " + os.path.relpath(path, ROOT),
            "entries": h.tune_entries()}


def _csv_rows(root: str, suffix: str):
    for path in sorted(glob.glob(os.path.join(root, "**", "*" + suffix), recursive=True)):
        with open(path) as f:
            yield from csv.DictReader(f)


def _short(name: str) -> str:
    s = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return s.split("(")[0]


def stats_summary(root: str, command: str, title: str) -> str:
    """Markdown tables of a `rocprofv3 --kernel-trace --stats --output-format
    csv` run under `root`: the library's kernels per (kernel, grid size) from
    kernel_trace.csv (one row per launch shape, so launches of different
    volume sizes are not averaged together), then the kernel_stats.csv
    summary of every kernel the command ran."""
    lines = ["# %s" % title, "", "command: `%s`" % command, "",
             "## Library kernels per launch shape", "",
             "| kernel | grid (threads) | workgroup | calls | avg us | min us | max us |",
             "|---|---|---|---|---|---|---|"]
    groups = {}
    for row in _csv_rows(root, "kernel_trace.csv"):
        name = _short(row["Kernel_Name"])
        if "harpia" not in name:
            continue
        key = (name, int(row["Grid_Size_X"]) * int(row["Grid_Size_Y"]) * int(row["Grid_Size_Z"]),
               int(row["Workgroup_Size_X"]) * int(row["Workgroup_Size_Y"]) * int(row["Workgroup_Size_Z"]))
        groups.setdefault(key, []).append((int(row["End_Timestamp"]) - int(row["Start_Timestamp"])) / 1e3)
    for (name, grid, wg), d in sorted(groups.items(), key=lambda kv: -sum(kv[1])):
        lines.append("| %s | %d | %d | %d | %.1f | %.1f | %.1f |" % (name, grid, wg, len(d), sum(d) / len(d), min(d),
                                                                      max(d)))
    lines += ["", "## All kernels (rocprofv3 --stats)", "",
              "| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for row in _csv_rows(root, "kernel_stats.csv"):
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.2f | %.1f |" % (
            _short(row["Name"]), row["Calls"], float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3,
            float(row["MaxNs"]) / 1e3, float(row["TotalDurationNs"]) / 1e6, float(row["Percentage"])))
    return "\n".join(lines) + "\n"


def traffic_summary(fetch_root: str, write_root: str, size: int, commands, kernels=None) -> dict:
    """HBM bytes per launch of the ops in `kernels` (default: the resident
    ops) from two `rocprofv3 --pmc` runs (FETCH_SIZE, then WRITE_SIZE; KiB
    per dispatch) of a bench command with --copy-ref.  Each counter is scaled
    by what it reads for the plain device copy of the volume in the same run
    (the largest copy dispatch: 4 * size^3 bytes read and written)."""
    kernels = RESIDENT_KERNELS if kernels is None else kernels
    vox = size ** 3
    copy_kib = 4.0 * vox / 1024.0
    out = {"size": size, "commands": list(commands), "source_sha": {k: sources_sha(k) for k in KERNEL_SOURCES},
           "copy_ref": {}, "ops": {}}
    per_op = {op: {} for op in kernels}
    for counter, root in (("FETCH_SIZE", fetch_root), ("WRITE_SIZE", write_root)):
        rows = [r for r in _csv_rows(root, "counter_collection.csv") if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not copies:
            raise SystemExit("no copy dispatch in %s" % root)
        ref = max(copies)
        scale = copy_kib / ref
        out["copy_ref"][counter] = {"kib": ref, "expected_kib": copy_kib, "scale": round(scale, 4)}
        for op, spec in kernels.items():
            vals = [float(r["Counter_Value"]) for r in rows if spec[1] in r["Kernel_Name"]]
            if vals:
                per_op[op][counter] = (sum(vals) / len(vals), len(vals), scale)
    for op, d in per_op.items():
        if len(d) != 2:
            continue
        nout = 2 if op.startswith("erode_dilate") else 1
        fetch = d["FETCH_SIZE"][0] * d["FETCH_SIZE"][2] * 1024.0
        write = d["WRITE_SIZE"][0] * d["WRITE_SIZE"][2] * 1024.0
        spec = kernels[op]
        alg = (spec[2] if len(spec) > 2 else 4.0 * (1 + nout)) * vox
        out["ops"][op] = {"fetch_kib_raw": round(d["FETCH_SIZE"][0], 1), "write_kib_raw": round(d["WRITE_SIZE"][0], 1),
                          "dispatches": d["FETCH_SIZE"][1], "hbm_bytes_per_launch": int(fetch + write),
                          "alg_bytes_per_launch": int(alg), "traffic_over_alg": round((fetch + write) / alg, 4)}
    return out


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def oracle_protocol(work_all, work_one, outputs_per_voxel: int, sample_all: str, sample_one: str, reps: int = 3):
    """The CPU-baseline protocol: the oracle timed on all of this host's
    cores and on one core, median of `reps` runs each.  work_*() runs the
    oracle on its bounded sample and returns the voxels it covered; the
    rate counts outputs_per_voxel outputs per voxel."""
    import oracle

    cores = len(os.sched_getaffinity(0))
    res = {}
    for label, fn, threads in (("all", work_all, cores), ("one", work_one, 1)):
        oracle.set_threads(threads)
        times, vox = [], 0
        for _ in range(reps):
            t0 = time.perf_counter()
            vox = fn()
            times.append(time.perf_counter() - t0)
        times.sort()
        res[label] = (times[len(times) // 2], vox, times, oracle.num_threads())
    oracle.set_threads(cores)
    t_all, v_all, runs_all, c_all = res["all"]
    t_one, v_one, runs_one, _ = res["one"]
    return {"value": round(outputs_per_voxel * v_all / t_all / 1e9, 6), "unit": "GVox/s", "cores": c_all,
            "kind": "oracle", "sample": "%s; median of %d runs (%s s)" % (
                sample_all, reps, ", ".join("%.2f" % t for t in runs_all)),
            "cpu_model": cpu_model(),
            "one_core": {"value": round(outputs_per_voxel * v_one / t_one / 1e9, 6), "unit": "GVox/s",
                         "sample": "%s; median of %d runs (%s s)" % (
                             sample_one, reps, ", ".join("%.2f" % t for t in runs_one))}}


def time_ops(ops, steps: int, warmup: int):
    """Warm-up, then `steps` timed passes over ops [(name, fn)]: returns
    (wall ms per pass, {name: mean event ms per launch}).  Events are
    recorded on torch's current stream, the stream the library launches on."""
    import torch

    for _ in range(warmup):
        for _, fn in ops:
            fn()
    torch.cuda.synchronize()
    events = {name: [] for name, _ in ops}
    t0 = time.perf_counter()
    for _ in range(steps):
        for name, fn in ops:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            events[name].append((e0, e1))
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - t0) * 1000.0 / max(1, steps)
    return wall_ms, {name: sum(a.elapsed_time(b) for a, b in ev) / len(ev) for name, ev in events.items()}


def sample_blocks(n: int, b: int, count: int = 32, seed: int = 2048):
    """Origins of `count` seeded b^3 blocks of an n^3 volume plus its 8
    corner blocks."""
    import numpy as np

    rng = np.random.default_rng(seed)
    out = [tuple(int(t) for t in rng.integers(0, n - b, size=3, endpoint=True)) for _ in range(count)]
    for cz in (0, n - b):
        for cy in (0, n - b):
            for cx in (0, n - b):
                out.append((cz, cy, cx))
    return out


def reflect_window(t, o, b: int, r: int):
    """t[o - r : o + b + r] per axis with half-sample reflection at the
    faces, gathered on the device, as float64 numpy."""
    import numpy as np
    import torch

    idx = []
    for k in range(3):
        n = t.shape[k]
        m = np.mod(np.arange(o[k] - r, o[k] + b + r), 2 * n)
        idx.append(torch.as_tensor(np.where(m < n, m, 2 * n - 1 - m), device=t.device))
    w = t.index_select(0, idx[0]).index_select(1, idx[1]).index_select(2, idx[2])
    return w.float().cpu().numpy().astype(np.float64)


def cpu_baseline(v_dev, slices_all: int = 48, slices_one: int = 3):
    """FP64 oracle on z-slabs of the resident phantom: Gaussian sigma 1, 2, 4
    (separable, pinned equal to the direct form) and ball-3 erosion and
    dilation (brute force), on all cores and on one core.  A slab is
    reflected at its own faces, which does not change the work per voxel."""
    import oracle

    va = v_dev[:slices_all].double().cpu().numpy()
    vo = v_dev[:slices_one].double().cpu().numpy()

    def work(v):
        for s in (1.0, 2.0, 4.0):
            oracle.gaussian3d(v, s, method="separable")
        oracle.erode3d(v, "ball", 3)
        oracle.dilate3d(v, "ball", 3)
        return v.size

    what = "slab of the %d^3 phantom: separable FP64 Gaussian sigma 1,2,4 + brute-force ball-3 erosion and dilation"
    n = v_dev.shape[1]
    return oracle_protocol(lambda: work(va), lambda: work(vo), 5,
                           "%dx%dx%d %s" % (va.shape + (what % n,)), "%dx%dx%d %s" % (vo.shape + (what % n,)))


def resident_measure(n: int, steps: int, warmup: int, tune: bool = False, copy_ref: bool = False,
                     tiles_path: str = TILES):
    """The resident single-GPU ops on an n^3 float32 porous phantom in HBM:
    Gaussian sigma 1, 2, 4, and grayscale erosion + dilation with the ball of
    radius 3 from one read (one launch, two outputs); plus binary erosion +
    dilation from one read (uint8 {0,1} input with the 3x3x3 box, uint16
    input thresholded at 32768 with the radius-2 ball).  Returns the
    phantom, the per-op figures, the wall ms of one pass over the first
    four ops, the plain device copy rate and the tile source."""
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    shape = (n, n, n)
    v = phantoms.porous(shape, seed=0, device=dev)
    vox = v.numel()
    outs = {s: torch.empty_like(v) for s in (1.0, 2.0, 4.0)}
    ero, dil = torch.empty_like(v), torch.empty_like(v)
    u8 = (v > 0.5).to(torch.uint8)
    u16 = torch.round(torch.clamp(v, 0.0, 1.0) * 65535.0).to(torch.int32).to(torch.uint16)
    be, bd = torch.empty_like(u8), torch.empty_like(u8)
    stream = lambda: torch.cuda.current_stream().cuda_stream  # noqa: E731
    lib = h._lib.load()

    def op_gauss(s):
        h.gaussian(v, s, out=outs[s])

    def op_pair(x, e, d, code, se, r, thr, flags):
        h._lib.check(lib.harpia_erode_dilate3d(
            x.data_ptr(), e.data_ptr(), d.data_ptr(), code, h._lib.i64_3(shape), se, h._lib.i32_3((r, r, r)),
            thr, 0, h._lib.make_exec(stream=stream(), flags=flags)))

    if copy_ref:
        # a plain device copy of the same volume (reference for HBM counters)
        ero.copy_(v)
        torch.cuda.synchronize()

    nan = float("nan")
    main = [("gauss_s1", lambda: op_gauss(1.0)), ("gauss_s2", lambda: op_gauss(2.0)),
            ("gauss_s4", lambda: op_gauss(4.0)),
            ("erode_dilate_ball3", lambda: op_pair(v, ero, dil, h._lib.HARPIA_F32, h._lib.HARPIA_SE_BALL, 3, nan, 0))]
    extra = [("bin_u8_box1", lambda: op_pair(u8, be, bd, h._lib.HARPIA_U8, h._lib.HARPIA_SE_BOX, 1, nan,
                                             h._lib.HARPIA_F_BINARY)),
             ("bin_u16_ball2", lambda: op_pair(u16, be, bd, h._lib.HARPIA_U16, h._lib.HARPIA_SE_BALL, 2, 32768.0, 0))]
    radius = {"gauss_s1": 3, "gauss_s2": 6, "gauss_s4": 12}
    # algorithmic bytes per voxel: one read, every output written once
    alg_b = {"gauss_s1": 8, "gauss_s2": 8, "gauss_s4": 8, "erode_dilate_ball3": 12, "bin_u8_box1": 3,
             "bin_u16_ball2": 4}
    n_out = {"erode_dilate_ball3": 2, "bin_u8_box1": 2, "bin_u16_ball2": 2}

    if tune:
        tuned = {}
        for s in (1.0, 2.0, 4.0):
            tuned["gauss_s%g" % s] = h.autotune_gaussian(v, s, out=outs[s])
        tuned["erode_dilate_ball3"] = h.autotune_erode_dilate(v, "ball", 3, ero=ero, dil=dil)
        tuned["bin_u8_box1"] = h.autotune_erode_dilate(u8, "box", 1, ero=be, dil=bd, binary=True)
        tuned["bin_u16_ball2"] = h.autotune_erode_dilate(u16, "ball", 2, ero=be, dil=bd, threshold=32768.0)
        tiles = tiles_merge_save(tiles_path)
        tiles["report"] = tuned
    else:
        tiles = tiles_load(tiles_path)

    # achievable HBM ceiling on this device: a plain device-to-device copy of
    # the volume (read + write bytes), timed the same way
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ero.copy_(v)
    c0.record()
    for _ in range(5):
        ero.copy_(v)
    c1.record()
    torch.cuda.synchronize()
    copy_gbs = 2 * 4 * vox * 5 / c0.elapsed_time(c1) / 1e6

    ms_step, ms = time_ops(main, steps, warmup)
    _, ms_x = time_ops(extra, steps, warmup)
    ms.update(ms_x)
    per_op = {}
    for name, t in ms.items():
        nout = n_out.get(name, 1)
        d = {"ms": round(t, 4), "gvox_s": round(nout * vox / t / 1e6, 2),
             "hbm_gbs": round(alg_b[name] * vox / t / 1e6, 1),
             "hbm_frac": round(alg_b[name] * vox / t / 1e6 / HBM_PEAK_GBS, 4), "alg_bytes_per_voxel": alg_b[name]}
        if name in radius:
            flops = 2 * 3 * (2 * radius[name] + 1) * vox  # separable form, one FMA = 2 flop
            d["tflops"] = round(flops / t / 1e9, 2)
            d["valu_frac"] = round(flops / t / 1e9 / FP32_VECTOR_PEAK_TFLOPS, 4)
        per_op[name] = d
    del u8, u16, be, bd, outs, ero, dil
    return v, per_op, ms_step, copy_gbs, tiles


def gauss_roofline(name: str, d: dict, r: int, vox: int, size: int, kind: str = "gauss"):
    """Roofline block of a Gaussian launch: ALU-bound when its separable
    flops take more of the FP32 vector peak than its bytes take of HBM."""
    alg_bytes = d["alg_bytes_per_voxel"] * vox
    flops = 2 * 3 * (2 * r + 1) * vox
    if d["hbm_frac"] < d.get("valu_frac", 0.0) * 2:
        roof = {"bound": "alu", "kernel": name, "achieved": d["tflops"], "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(d["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4),
                "per_launch": {"flops": flops, "bytes": alg_bytes, "ms": d["ms"]}}
    else:
        roof = {"bound": "hbm", "kernel": name, "achieved": d["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(d["hbm_gbs"] / HBM_PEAK_GBS, 4), "per_launch": {"bytes": alg_bytes, "ms": d["ms"]}}
    roof["traffic"] = traffic_for(name, kind, size)
    return roof


def run_resident(args):
    v, per_op, ms_step, copy_gbs, tiles = resident_measure(args.size, args.steps, args.warmup, args.tune,
                                                           args.copy_ref, args.tiles)
    vox = v.numel()
    n = args.size
    main = ["gauss_s1", "gauss_s2", "gauss_s4", "erode_dilate_ball3"]
    dom = max(main, key=lambda k: per_op[k]["ms"])
    dd = per_op[dom]
    if dom.startswith("gauss"):
        roof = gauss_roofline(dom, dd, {"gauss_s1": 3, "gauss_s2": 6, "gauss_s4": 12}[dom], vox, n)
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": dd["hbm_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": dd["hbm_frac"], "per_launch": {"bytes": 12 * vox, "ms": dd["ms"]},
                "traffic": traffic_for(dom, "morph", n)}
    outputs_per_step = 5
    value = outputs_per_step * vox / (ms_step / 1000.0) / 1e9
    line = {"metric": METRIC, "value": round(value, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "resident %d^3 float32 porous phantom: Gaussian sigma 1,2,4 + "
                                   "grayscale erode+dilate ball r=3" % n, "voxels": vox,
                       "outputs_per_step": outputs_per_step},
            "roofline": roof, "ops": per_op, "hbm_copy_gbs": round(copy_gbs, 1), "tiles": tiles}
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(v)
    return line


# 16-bit storage: unit roundoff of round-to-nearest-even (8 and 11
# significand bits); the end-to-end error bound is one rounding of the input
# plus one of the output, 2u relative (positive taps)
U_STORAGE = {"bf16": 2.0 ** -8, "f16": 2.0 ** -11}


def run_headline(args):
    """The precision workload at full size: a 2048^3 porous phantom with
    values in [0, 1], Gaussian sigma 1 and 4 (truncate 3, reflect) in plain
    FP32 (the timed step and `value`), and the same filters with the volume
    stored in BF16 and FP16 (FP32 accumulation, FP64 tap normalisation),
    each with its max / mean relative error against the FP64 oracle on
    sampled blocks.  The resident 1024^3 FP32 ops ride along in `ops`."""
    import numpy as np
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    n = args.size
    tiles = tiles_load(args.tiles)
    tuned = {}
    print("headline: phantom %d^3" % n, file=sys.stderr, flush=True)
    v = torch.clamp(phantoms.porous((n, n, n), seed=0, device=dev), 0.0, 1.0)
    vox = v.numel()
    out = torch.empty_like(v)
    radius = {1.0: 3, 4.0: 12}
    if args.tune:
        for s in radius:
            tuned["f32_sigma%g" % s] = h.autotune_gaussian(v, s, out=out)
    step_ops = [("f32_sigma1", lambda: h.gaussian(v, 1.0, out=out)), ("f32_sigma4", lambda: h.gaussian(v, 4.0, out=out))]
    ms_step, ms = time_ops(step_ops, args.steps, args.warmup)

    # oracle blocks: b^3 blocks with a 12-voxel reflected halo (enough for
    # both radii), from the unquantised volume and from each 16-bit copy
    b, rmax = 32, 12
    blocks = sample_blocks(n, b) if not args.no_cpu else []
    wins = [reflect_window(v, o, b, rmax) for o in blocks]
    want = {s: [oracle_gauss(w, s)[rmax:-rmax, rmax:-rmax, rmax:-rmax] for w in wins] for s in radius}

    def errors(y, s, ref=None):
        ref = want[s] if ref is None else ref
        if not blocks:
            return {}
        e = []
        for o, wt in zip(blocks, ref):
            g = y[o[0]:o[0] + b, o[1]:o[1] + b, o[2]:o[2] + b].float().cpu().numpy().astype(np.float64)
            e.append((np.abs(g - wt) / np.maximum(np.abs(wt), 1e-300)).ravel())
        e = np.concatenate(e)
        return {"err_max": float("%.3e" % e.max()), "err_mean": float("%.3e" % e.mean())}

    per_op = {}
    for s in radius:
        name = "f32_sigma%g" % s
        h.gaussian(v, s, out=out)
        torch.cuda.synchronize()
        t = ms[name]
        flops = 2 * 3 * (2 * radius[s] + 1) * vox
        per_op[name] = {"ms": round(t, 4), "gvox_s": round(vox / t / 1e6, 2), "hbm_gbs": round(8 * vox / t / 1e6, 1),
                        "hbm_frac": round(8 * vox / t / 1e6 / HBM_PEAK_GBS, 4), "alg_bytes_per_voxel": 8,
                        "tflops": round(flops / t / 1e9, 2),
                        "valu_frac": round(flops / t / 1e9 / FP32_VECTOR_PEAK_TFLOPS, 4),
                        "err_bound": 1e-5}
        per_op[name].update(errors(out, s))
    del out
    for tag, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        print("headline: %s" % tag, file=sys.stderr, flush=True)
        x = v.to(dt)
        y = torch.empty_like(x)
        if args.tune:
            for s in radius:
                tuned["%s_sigma%g" % (tag, s)] = h.autotune_gaussian(x, s, out=y)
        ops16 = [("%s_sigma%g" % (tag, s), (lambda s=s: h.gaussian(x, s, out=y))) for s in radius]
        _, ms16 = time_ops(ops16, args.steps, args.warmup)
        deq = [reflect_window(x, o, b, rmax) for o in blocks]
        for s in radius:
            name = "%s_sigma%g" % (tag, s)
            h.gaussian(x, s, out=y)
            torch.cuda.synchronize()
            t = ms16[name]
            flops = 2 * 3 * (2 * radius[s] + 1) * vox
            d = {"ms": round(t, 4), "gvox_s": round(vox / t / 1e6, 2), "hbm_gbs": round(4 * vox / t / 1e6, 1),
                 "hbm_frac": round(4 * vox / t / 1e6 / HBM_PEAK_GBS, 4), "alg_bytes_per_voxel": 4,
                 "tflops": round(flops / t / 1e9, 2),
                 "valu_frac": round(flops / t / 1e9 / FP32_VECTOR_PEAK_TFLOPS, 4),
                 "speedup_vs_f32": round(per_op["f32_sigma%g" % s]["ms"] / t, 3),
                 "err_bound": 2 * U_STORAGE[tag]}
            d.update(errors(y, s))
            if blocks:
                # against the oracle on the dequantised input: arithmetic and
                # output rounding only
                ref = [oracle_gauss(w, s)[rmax:-rmax, rmax:-rmax, rmax:-rmax] for w in deq]
                d["err_max_vs_dequantised"] = errors(y, s, ref)["err_max"]
            per_op[name] = d
        del x, y
    cpu = None
    if not args.no_cpu:
        print("headline: oracle timing", file=sys.stderr, flush=True)
        va = v[:24].double().cpu().numpy()
        vo = v[:2].double().cpu().numpy()

        def work(a):
            oracle_gauss(a, 1.0)
            oracle_gauss(a, 4.0)
            return a.size

        what = "slab of the %d^3 phantom: separable FP64 Gaussian sigma 1 and 4" % n
        cpu = oracle_protocol(lambda: work(va), lambda: work(vo), 2, "%dx%dx%d %s" % (va.shape + (what,)),
                              "%dx%dx%d %s" % (vo.shape + (what,)))
        del va, vo
    del v
    torch.cuda.empty_cache()
    print("headline: resident 1024^3 ops", file=sys.stderr, flush=True)
    vr, res_ops, res_ms_step, copy_gbs, res_tiles = resident_measure(1024, args.steps, args.warmup, tune=args.tune,
                                                                     tiles_path=args.tiles)
    if args.tune:
        tiles = res_tiles
        tiles["report"] = dict(tuned, resident_1024=res_tiles.get("report"))
    del vr
    torch.cuda.empty_cache()
    per_op["resident_1024"] = dict(res_ops, step_ms=round(res_ms_step, 3),
                                   step_gvox_s=round(5 * 1024 ** 3 / res_ms_step / 1e6, 2))

    roof = gauss_roofline("f32_sigma4", per_op["f32_sigma4"], 12, vox, n)
    line = {"metric": METRIC, "value": round(2 * vox / ms_step / 1e6, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "precision %d^3 porous phantom in [0,1]: Gaussian sigma 1 and 4 in plain FP32 "
                                   "(timed step; BF16 / FP16 storage in ops, with errors vs the FP64 oracle; "
                                   "resident 1024^3 ops in ops.resident_1024)" % n,
                       "voxels": vox, "outputs_per_step": 2},
            "roofline": roof, "ops": per_op, "hbm_copy_gbs": round(copy_gbs, 1), "tiles": tiles}
    if blocks:
        line["config"]["error_sample"] = "%d blocks of %d^3 (%d seeded + 8 corners), relative to the FP64 oracle " \
                                         "on the unquantised input" % (len(blocks), b, len(blocks) - 8)
    if cpu:
        line["cpu_baseline"] = cpu
    return line


def oracle_gauss(w, s):
    """Separable FP64 oracle Gaussian (truncate 3, reflect) of a window."""
    import oracle

    return oracle.gaussian3d(w, s, method="separable")


def run_precision(args):
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    n = args.size
    v = torch.clamp(phantoms.porous((n, n, n), seed=0, device=dev), 0, 1)
    tiles_load(args.tiles)
    if args.copy_ref:
        # a plain device copy of the volume (reference for HBM counters)
        w = torch.empty_like(v)
        w.copy_(v)
        torch.cuda.synchronize()
        del w
    res = {}
    for name, dt in (("f32", torch.float32), ("bf16", torch.bfloat16), ("f16", torch.float16)):
        x = v.to(dt)
        for s in (1.0, 4.0):
            out = torch.empty_like(x)
            for _ in range(args.warmup):
                h.gaussian(x, s, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(args.steps):
                h.gaussian(x, s, out=out)
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / args.steps
            es = x.element_size()
            res["%s_sigma%g" % (name, s)] = {"ms": round(ms, 3), "gvox_s": round(x.numel() / ms / 1e6, 1),
                                             "hbm_frac": round(2 * es * x.numel() / ms / 1e6 / HBM_PEAK_GBS, 4)}
            del out
        del x
    step_ms = sum(d["ms"] for k, d in res.items() if k.startswith("bf16"))
    return {"metric": METRIC, "value": round(2 * v.numel() / step_ms / 1e6, 2), "unit": "GVox/s",
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_ms, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
            "data": "synthetic",
            "config": {"workload": "precision: %d^3 bf16 Gaussian sigma 1 and 4 (f32, f16 for comparison)" % n},
            "ops": res}


def link_rates(nbytes: int = 4 << 30):
    """Pinned host <-> device copy rates (GB/s) of this box, timed with
    events around torch's copies (hipMemcpyAsync)."""
    import torch

    hbuf = torch.empty(nbytes, dtype=torch.uint8, pin_memory=True)
    dbuf = torch.empty(nbytes, dtype=torch.uint8, device="cuda:0")
    rates = {}
    for name, fn in (("h2d", lambda: dbuf.copy_(hbuf, non_blocking=True)),
                     ("d2h", lambda: hbuf.copy_(dbuf, non_blocking=True))):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(3):
            fn()
        e1.record()
        torch.cuda.synchronize()
        rates[name] = round(3 * nbytes / e0.elapsed_time(e1) / 1e6, 2)
    del hbuf, dbuf
    return rates


def run_chunked(args):
    """Out-of-core: a 2048^3 uint16 phantom in pinned host memory, 8 GiB
    device budget, 512^3 bricks (Section III-D streamed with halos):
    Gaussian sigma 2 to float32 and the binary opening with the radius-2 ball
    on v > 32768.  Rates are host-to-host (PCIe included).  Each op also runs
    as a z-slab plan and as one resident chunk (budget uncapped: one H2D,
    the kernels, one D2H), and reports the summed per-chunk kernel time
    against the resident kernel time."""
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    n = args.size
    dev = torch.device("cuda:0")
    print("chunked: phantom %d^3 u16" % n, file=sys.stderr, flush=True)
    v = phantoms.porous_u16((n, n, n), seed=0, device=dev)
    host = torch.empty((n, n, n), dtype=torch.uint16, pin_memory=True)
    host.copy_(v)
    del v
    torch.cuda.empty_cache()
    out_g = torch.empty((n, n, n), dtype=torch.float32, pin_memory=True)
    out_o = torch.empty((n, n, n), dtype=torch.uint8, pin_memory=True)
    rates = link_rates()
    budget = 8 << 30
    res = {}
    for name, fn in (("gauss_s2", lambda ex: h.gaussian(host, 2.0, out=out_g, ex=ex)),
                     ("open_ball2", lambda ex: h.opening(host, "ball", 2, threshold=32768.0, out=out_o, ex=ex))):
        for label, chunk, bud in (("chunked_512", (512, 512, 512), budget), ("chunked_zslab", (0, 0, 0), budget),
                                  ("resident", (n, n, n), 200 << 30)):
            print("chunked: %s %s" % (name, label), file=sys.stderr, flush=True)
            st = h.harpia_stats()
            fn(h.Exec(budget=bud, chunk=chunk, stats=st))
            t0 = time.perf_counter()
            st = h.harpia_stats()
            fn(h.Exec(budget=bud, chunk=chunk, stats=st))
            dt = time.perf_counter() - t0
            link_s = max(st.bytes_h2d / (rates["h2d"] * 1e9), st.bytes_d2h / (rates["d2h"] * 1e9))
            res["%s_%s" % (name, label)] = {"s": round(dt, 3), "gvox_s": round(n ** 3 / dt / 1e9, 2),
                                            "chunks": st.n_chunks, "peak_gib": round(st.peak_device_bytes / 2 ** 30, 2),
                                            "h2d_gb": round(st.bytes_h2d / 1e9, 2),
                                            "d2h_gb": round(st.bytes_d2h / 1e9, 2),
                                            "kernel_ms": round(st.kernel_ms, 2),
                                            "link_bound_s": round(link_s, 3),
                                            "link_frac": round(link_s / dt, 4)}
        r = res["%s_resident" % name]
        for label in ("chunked_512", "chunked_zslab"):
            c = res["%s_%s" % (name, label)]
            c["vs_resident_host_to_host"] = round(c["gvox_s"] / r["gvox_s"], 3)
            c["kernel_time_vs_resident"] = round(c["kernel_ms"] / r["kernel_ms"], 3) if r["kernel_ms"] else None
    tot = res["gauss_s2_chunked_512"]["s"] + res["open_ball2_chunked_512"]["s"]
    g = res["gauss_s2_chunked_512"]
    d2h_bound = g["d2h_gb"] / rates["d2h"] >= g["h2d_gb"] / rates["h2d"]
    roof = {"bound": "pcie", "kernel": "gauss_s2 chunked_512 (%s-bound)" % ("D2H" if d2h_bound else "H2D"),
            "achieved": round((g["d2h_gb"] if d2h_bound else g["h2d_gb"]) / g["s"], 2),
            "peak": rates["d2h"] if d2h_bound else rates["h2d"], "unit": "GB/s",
            "frac": g["link_frac"], "peak_source": "pinned hipMemcpyAsync measured in this run", "traffic": None}
    line = {"metric": METRIC, "value": round(2 * n ** 3 / tot / 1e9, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": round(tot * 1000, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
            "config": {"workload": "chunked %d^3 uint16 pinned host, 8 GiB budget, 512^3 bricks: Gaussian "
                                   "sigma 2 -> f32 + binary opening ball r=2 at 32768 (host to host)" % n},
            "roofline": roof, "link_gbs": rates, "ops": res}
    if not args.no_cpu:
        import oracle

        print("chunked: oracle timing", file=sys.stderr, flush=True)
        ba = host[:512, :512, :512].numpy().astype("float64")
        bo = host[:32, :512, :512].numpy().astype("float64")

        def work(a):
            oracle.gaussian3d(a, 2.0, method="separable")
            oracle.opening3d(oracle.threshold(a, 32768.0), "ball", 2)
            return a.size

        what = "brick of the %d^3 uint16 phantom: separable FP64 Gaussian sigma 2 + threshold and brute-force " \
               "ball-2 opening (rate extrapolates to the 64 bricks)" % n
        line["cpu_baseline"] = oracle_protocol(lambda: work(ba), lambda: work(bo), 2,
                                               "%dx%dx%d %s" % (ba.shape + (what,)),
                                               "%dx%dx%d %s" % (bo.shape + (what,)))
    return line


def run_batched(args):
    """64 float32 crops with seeded uneven extents in [64, 256] cut from the
    1024^3 phantom; learnable sigma 1.5 (radius 5) then dilation with the
    5x5x5 box; one step = forward + backward (input and sigma gradients) as
    one captured graph replay."""
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    parent = phantoms.porous((1024, 1024, 1024), seed=0, device=dev)
    boxes = phantoms.crop_boxes(64, 64, 256, parent=(1024, 1024, 1024), seed=0)
    xs = [parent[z:z + dz, y:y + dy, x:x + dx].contiguous() for (z, y, x), (dz, dy, dx) in boxes]
    del parent
    torch.cuda.empty_cache()
    cs = [phantoms.gaussian_noise(x.shape, seed=100 + i, device=dev) for i, x in enumerate(xs)]
    vox = sum(x.numel() for x in xs)
    b = h.GaussDilateBatch(xs, 1.5, "box", 2)
    if args.tune:
        tuned = b.autotune()
        tiles = tiles_merge_save(args.tiles)
        tiles["report"] = tuned
    else:
        tiles = tiles_load(args.tiles)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        for _ in range(max(1, args.warmup)):
            b.forward()
            b.backward(cs)
    torch.cuda.current_stream().wait_stream(s)
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.forward()
        b.backward(cs)
    for _ in range(args.warmup):
        g.replay()
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record()
    for _ in range(args.steps):
        g.replay()
    e1.record()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    # eager per-phase timing (not captured) for the breakdown
    phases = {}
    for name, fn in (("forward", lambda: b.forward()), ("backward", lambda: b.backward(cs))):
        fn()
        a0, a1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a0.record()
        for _ in range(5):
            fn()
        a1.record()
        torch.cuda.synchronize()
        phases[name + "_ms"] = round(a0.elapsed_time(a1) / 5, 3)
    # algorithmic bytes: forward 8 B (x in, d out) + backward 12 B (x, c in, grad_x out)
    alg = 20 * vox
    roof = {"bound": "hbm", "kernel": "forward + backward step (one graph replay)", "achieved": round(alg / ms / 1e6, 1),
            "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(alg / ms / 1e6 / HBM_PEAK_GBS, 4),
            "per_launch": {"bytes": alg, "bytes_per_voxel": 20, "ms": round(ms, 4)}, "traffic": None}
    line = {"metric": METRIC, "value": round(vox / ms / 1e6, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000 / args.steps, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "batched: 64 float32 crops, extents U[64,256], Gaussian sigma 1.5 (learnable) "
                                   "+ box-5 dilation, forward + backward per step, one graph replay",
                       "voxels": vox, "crops": len(xs)},
            "roofline": roof,
            "ops": dict(phases, graph_ms=round(ms, 3), hbm_frac_alg20=round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)),
            "tiles": tiles}
    if not args.no_cpu:
        import oracle

        order = sorted(range(len(xs)), key=lambda i: xs[i].numel())
        def pick(limit):
            out, tot = [], 0
            for i in order:
                if tot >= limit:
                    break
                out.append((xs[i].double().cpu().numpy(), cs[i].double().cpu().numpy()))
                tot += xs[i].numel()
            return out
        sa, so = pick(12_000_000), pick(800_000)

        def work(sample):
            for x, c in sample:
                oracle.gauss_dilate_loss_grad(x, c, 1.5, "box", 2)
            return sum(x.size for x, _ in sample)

        what = "smallest crops: FP64 forward (separable Gaussian sigma 1.5, brute-force box-5 dilation) and " \
               "analytic backward (routing, transposed Gaussian, d/d sigma)"
        line["cpu_baseline"] = oracle_protocol(
            lambda: work(sa), lambda: work(so), 1,
            "%d crops, %d voxels, %s" % (len(sa), sum(x.size for x, _ in sa), what),
            "%d crops, %d voxels, %s" % (len(so), sum(x.size for x, _ in so), what))
    return line


def run_filters(args):
    """The next filters of the suite on the resident 1024^3 float32 phantom:
    mean (box) filter r = 1 and 2, unsharp masking sigma 2 amount 1, Sobel
    gradient magnitude.  One step = the four filters; value = output voxels
    per second."""
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    n = args.size
    v = phantoms.porous((n, n, n), seed=0, device=dev)
    vox = v.numel()
    out = torch.empty_like(v)
    hout = torch.empty((6,) + tuple(v.shape), dtype=torch.float32, device=dev)
    bout = torch.empty(tuple(v.shape), dtype=torch.uint8, device=dev)
    v16 = phantoms.porous_u16((n, n, n), seed=0, device=dev)
    if args.tune:
        # the mean filter runs the fused kernel of radius r (sigma 0.34 and
        # 0.5 resolve to r = 1 and 2: same kernel, same workload key)
        tuned = {"r%d" % r: h.autotune_gaussian(v, sg, out=out) for r, sg in ((1, 0.34), (2, 0.5))}
        tiles = tiles_merge_save(args.tiles)
        tiles["report"] = tuned
    else:
        tiles = tiles_load(args.tiles)
    ops = [("mean_r1", lambda: h.mean(v, 1, out=out)), ("mean_r2", lambda: h.mean(v, 2, out=out)),
           ("unsharp_s2_a1", lambda: h.unsharp(v, 2.0, 1.0, out=out)), ("sobel", lambda: h.edge(v, "sobel", out=out)),
           ("hessian_s1_6out", lambda: h.hessian(v, 1.0, out=hout)),
           ("niblack_r2", lambda: h.local_threshold(v, "niblack", radius=2, k=-0.2, out=bout)),
           ("otsu_u16", lambda: h.otsu(v16, out=bout))]
    for _ in range(args.warmup):
        for _, fn in ops:
            fn()
    torch.cuda.synchronize()
    events = {name: [] for name, _ in ops}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for name, fn in ops:
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            events[name].append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per_op = {}
    for name, _ in ops:
        ms = sum(a.elapsed_time(b) for a, b in events[name]) / len(events[name])
        # algorithmic bytes: read once, write once (the unsharp epilogue's
        # read of the centre voxel is a re-read); the Hessian writes 6 outputs
        nout = 6 if name.startswith("hessian") else 1
        # thresholds write a byte; Otsu reads the u16 volume twice (histogram,
        # then the comparison) and writes a byte
        alg = {"niblack_r2": 5, "otsu_u16": 5}.get(name, 4 + 4 * nout)
        per_op[name] = {"ms": round(ms, 4), "gvox_s": round(nout * vox / ms / 1e6, 2),
                        "hbm_frac": round(alg * vox / ms / 1e6 / HBM_PEAK_GBS, 4)}
    ms_step = wall * 1000 / args.steps
    dom = max(per_op, key=lambda k: per_op[k]["ms"])
    d = per_op[dom]
    nb = (4 + 4 * (6 if dom.startswith("hessian") else 1)) * vox
    roof = {"bound": "hbm", "kernel": dom, "achieved": round(nb / d["ms"] / 1e6, 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": d["hbm_frac"], "per_launch": {"bytes": nb, "ms": d["ms"]}, "traffic": None}
    outputs = len(ops) + 5  # the Hessian has 6 outputs
    line = {"metric": METRIC, "value": round(outputs * vox / ms_step / 1e6, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(ms_step, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "filters: %d^3 float32 porous phantom, mean r=1,2 + unsharp sigma 2 amount 1 + "
                                   "Sobel magnitude + Hessian sigma 1 (6 outputs) + Niblack r=2 + Otsu (uint16 "
                                   "phantom)" % n,
                       "voxels": vox},
            "roofline": roof, "ops": per_op, "tiles": tiles}
    if not args.no_cpu:
        import oracle

        sa = v[:8].double().cpu().numpy()
        so = v[:1].double().cpu().numpy()

        def work(sl):
            oracle.mean3d(sl, 1, method="separable")
            oracle.mean3d(sl, 2, method="separable")
            oracle.unsharp3d(sl, 2.0, 1.0)
            oracle.edge3d(sl, "sobel")
            oracle.hessian3d(sl, 1.0)
            oracle.local_threshold3d(sl, "niblack", 2, k=-0.2)
            return sl.size

        what = "slab: separable FP64 mean r=1,2 + unsharp (direct FP64 Gaussian) sigma 2 + direct FP64 Sobel + " \
               "direct FP64 Hessian sigma 1 + Niblack r=2"
        line["cpu_baseline"] = oracle_protocol(lambda: work(sa), lambda: work(so), 11,
                                               "%dx%dx%d %s" % (sa.shape + (what,)),
                                               "%dx%dx%d %s" % (so.shape + (what,)))
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="headline",
                    choices=["headline", "resident", "precision", "chunked", "batched", "filters"])
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one plain device copy of the volume (counter reference)")
    ap.add_argument("--tune", action="store_true",
                    help="headline / resident / batched / filters: run the autotuner on the ops first and merge "
                         "its tiles into --tiles")
    ap.add_argument("--tiles", default=TILES, help="tile file of the autotuner (loaded if present)")
    ap.add_argument("--stats-summary", nargs=3, metavar=("CSV_DIR", "COMMAND", "TITLE"),
                    help="print a markdown summary of a rocprofv3 --stats csv run and exit (no GPU)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_CMD", "WRITE_CMD"),
                    help="print the HBM traffic JSON of two rocprofv3 --pmc runs and exit (no GPU)")
    ap.add_argument("--traffic-kernels", default="resident", choices=["resident", "headline"],
                    help="ops whose dispatches --traffic-summary reads (resident 1024^3 or headline 2048^3 FP32)")
    args = ap.parse_args()
    if args.stats_summary:
        print(stats_summary(*args.stats_summary), end="")
        return
    if args.traffic_summary:
        fr, wr, fc, wc = args.traffic_summary
        kern = HEADLINE_KERNELS if args.traffic_kernels == "headline" else RESIDENT_KERNELS
        size = args.size or (2048 if args.traffic_kernels == "headline" else 1024)
        print(json.dumps(traffic_summary(fr, wr, size, (fc, wc), kern), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs no multi-GPU path (one process, one device). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.size == 0:
        args.size = 1024 if args.workload in ("resident", "filters") else 2048
    fn = {"headline": run_headline, "resident": run_resident, "precision": run_precision, "chunked": run_chunked,
          "batched": run_batched, "filters": run_filters}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
