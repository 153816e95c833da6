"""Throughput of the volumetric filtering hot path on one MI355X.

Default workload (resident, one GPU): a 1024^3 float32 two-phase porous
phantom in HBM; one step = Gaussian smoothing with sigma 1, 2 and 4 (truncate
3, reflect) plus grayscale erosion and dilation with the ball of radius 3
(one fused launch, two outputs).  value = output voxels of the step (5 x
1024^3) per second, in GVox/s.

Per-op times are measured with HIP events on the stream the library launches
on (torch's current stream).  The roofline block reports the op with the
largest share of the step: algorithmic bytes (or multiply-adds) per launch
over its average event-timed duration, against the MI355X peak.  The CPU
baseline is the FP64 oracle on a bounded slab of the same phantom, timed on
this host's cores.

Other workloads (--workload): "precision" (2048^3 bf16 / f16 / f32 Gaussian
sigma 1 and 4), "chunked" (2048^3 uint16 in pinned host memory, 8 GiB device
budget, 512^3 bricks: Gaussian sigma 2 to float32 and binary opening with the
radius-2 ball on threshold 32768), "batched" (64 uneven float32 crops,
learnable-sigma Gaussian + box-5 dilation, forward + backward in one graph).
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
}

# kernel-name fragments of the resident workload's ops (f32, fused kernels)
RESIDENT_KERNELS = {
    "gauss_s1": ("gauss", "gauss_fused_kernel<float, float, 3,"),
    "gauss_s2": ("gauss", "gauss_fused_kernel<float, float, 6,"),
    "gauss_s4": ("gauss", "gauss_fused_kernel<float, float, 12,"),
    "erode_dilate_ball3": ("morph", "gray_kernel<float, 1, 3, true>"),
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
    """Markdown table of a `rocprofv3 --kernel-trace --stats --output-format
    csv` run (its kernel_stats.csv under `root`)."""
    lines = ["# %s" % title, "", "command: `%s`" % command, "",
             "| kernel | calls | avg us | min us | max us | total ms | % |", "|---|---|---|---|---|---|---|"]
    for row in _csv_rows(root, "kernel_stats.csv"):
        lines.append("| %s | %s | %.1f | %.1f | %.1f | %.2f | %.1f |" % (
            _short(row["Name"]), row["Calls"], float(row["AverageNs"]) / 1e3, float(row["MinNs"]) / 1e3,
            float(row["MaxNs"]) / 1e3, float(row["TotalDurationNs"]) / 1e6, float(row["Percentage"])))
    return "\n".join(lines) + "\n"


def traffic_summary(fetch_root: str, write_root: str, size: int, commands) -> dict:
    """HBM bytes per launch of the resident ops from two `rocprofv3 --pmc`
    runs (FETCH_SIZE, then WRITE_SIZE; KiB per dispatch) of
    `bench.py --copy-ref`.  Each counter is scaled by what it reads for the
    plain device copy of the volume in the same run (the largest copy
    dispatch: 4 * size^3 bytes read and written)."""
    vox = size ** 3
    copy_kib = 4.0 * vox / 1024.0
    out = {"size": size, "commands": list(commands), "source_sha": {k: sources_sha(k) for k in KERNEL_SOURCES},
           "copy_ref": {}, "ops": {}}
    per_op = {op: {} for op in RESIDENT_KERNELS}
    for counter, root in (("FETCH_SIZE", fetch_root), ("WRITE_SIZE", write_root)):
        rows = [r for r in _csv_rows(root, "counter_collection.csv") if r["Counter_Name"] == counter]
        copies = [float(r["Counter_Value"]) for r in rows if "copyBuffer" in r["Kernel_Name"]]
        if not copies:
            raise SystemExit("no copy dispatch in %s" % root)
        ref = max(copies)
        scale = copy_kib / ref
        out["copy_ref"][counter] = {"kib": ref, "expected_kib": copy_kib, "scale": round(scale, 4)}
        for op, (_, pat) in RESIDENT_KERNELS.items():
            vals = [float(r["Counter_Value"]) for r in rows if pat in r["Kernel_Name"]]
            if vals:
                per_op[op][counter] = (sum(vals) / len(vals), len(vals), scale)
    for op, d in per_op.items():
        if len(d) != 2:
            continue
        nout = 2 if op.startswith("erode_dilate") else 1
        fetch = d["FETCH_SIZE"][0] * d["FETCH_SIZE"][2] * 1024.0
        write = d["WRITE_SIZE"][0] * d["WRITE_SIZE"][2] * 1024.0
        alg = 4.0 * vox * (1 + nout)
        out["ops"][op] = {"fetch_kib_raw": round(d["FETCH_SIZE"][0], 1), "write_kib_raw": round(d["WRITE_SIZE"][0], 1),
                          "dispatches": d["FETCH_SIZE"][1], "hbm_bytes_per_launch": int(fetch + write),
                          "alg_bytes_per_launch": int(alg), "traffic_over_alg": round((fetch + write) / alg, 4)}
    return out


def cpu_baseline(v_dev, sample_slices: int = 160):
    """FP64 oracle on a z-slab of the phantom: Gaussian sigma 1, 2, 4
    (separable, pinned equal to the direct form) and ball-3 erosion and
    dilation (brute force).  The slab is reflected at its own faces, which
    does not change the work per voxel."""
    import numpy as np

    import oracle

    v = v_dev[:sample_slices].double().cpu().numpy()
    t0 = time.perf_counter()
    for s in (1.0, 2.0, 4.0):
        oracle.gaussian3d(v, s, method="separable")
    oracle.erode3d(v, "ball", 3)
    oracle.dilate3d(v, "ball", 3)
    dt = time.perf_counter() - t0
    vox = int(np.prod(v.shape))
    return {"value": round(5 * vox / dt / 1e9, 6), "unit": "GVox/s", "cores": oracle.num_threads(),
            "kind": "oracle",
            "sample": "%dx%dx%d slab of the 1024^3 phantom: separable FP64 Gaussian sigma 1,2,4 + "
                      "brute-force ball-3 erosion and dilation, %.1f s" % (v.shape + (dt,))}


def run_resident(args):
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    n = args.size
    shape = (n, n, n)
    v = phantoms.porous(shape, seed=0, device=dev)
    vox = v.numel()
    outs = {s: torch.empty_like(v) for s in (1.0, 2.0, 4.0)}
    ero, dil = torch.empty_like(v), torch.empty_like(v)

    def op_gauss(s):
        h.gaussian(v, s, out=outs[s])

    def op_morph():
        h._lib.check(h._lib.load().harpia_erode_dilate3d(
            v.data_ptr(), ero.data_ptr(), dil.data_ptr(), h._lib.HARPIA_F32, h._lib.i64_3(shape),
            h._lib.HARPIA_SE_BALL, h._lib.i32_3((3, 3, 3)), float("nan"), 0,
            h._lib.make_exec(stream=torch.cuda.current_stream().cuda_stream)))

    if args.copy_ref:
        # a plain device copy of the same volume (reference for HBM counters)
        ero.copy_(v)
        torch.cuda.synchronize()

    ops = [("gauss_s1", lambda: op_gauss(1.0), 3), ("gauss_s2", lambda: op_gauss(2.0), 6),
           ("gauss_s4", lambda: op_gauss(4.0), 12), ("erode_dilate_ball3", op_morph, 3)]
    outputs_per_step = 5

    if args.tune:
        tuned = {}
        for s in (1.0, 2.0, 4.0):
            tuned["gauss_s%g" % s] = h.autotune_gaussian(v, s, out=outs[s])
        tuned["erode_dilate_ball3"] = h.autotune_erode_dilate(v, "ball", 3, ero=ero, dil=dil)
        tiles = tiles_merge_save(args.tiles)
        tiles["report"] = tuned
    else:
        tiles = tiles_load(args.tiles)

    for _ in range(args.warmup):
        for _, fn, _ in ops:
            fn()
    torch.cuda.synchronize()

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

    events = {name: [] for name, _, _ in ops}
    t0 = time.perf_counter()
    for _ in range(args.steps):
        for name, fn, _ in ops:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            fn()
            e1.record()
            events[name].append((e0, e1))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1000.0 / args.steps

    per_op = {}
    for name, _, r in ops:
        ms = sum(a.elapsed_time(b) for a, b in events[name]) / len(events[name])
        nout = 2 if name.startswith("erode_dilate") else 1
        alg_bytes = vox * (4 + 4 * nout)
        d = {"ms": round(ms, 4), "gvox_s": round(nout * vox / ms / 1e6, 2),
             "hbm_gbs": round(alg_bytes / ms / 1e6, 1),
             "hbm_frac": round(alg_bytes / ms / 1e6 / HBM_PEAK_GBS, 4)}
        if name.startswith("gauss"):
            macs = 3 * (2 * r + 1) * vox  # multiply-adds of the separable form
            d["tflops"] = round(2 * macs / ms / 1e9, 2)
            d["valu_frac"] = round(2 * macs / ms / 1e9 / FP32_VECTOR_PEAK_TFLOPS, 4)
        per_op[name] = d

    dom = max(per_op, key=lambda k: per_op[k]["ms"])
    dd = per_op[dom]
    kind = "gauss" if dom.startswith("gauss") else "morph"
    nout = 2 if kind == "morph" else 1
    alg_bytes = vox * (4 + 4 * nout)
    if kind == "gauss" and dd["hbm_frac"] < dd["valu_frac"] * 2:
        r = dict((nm, rr) for nm, _, rr in ops)[dom]
        macs = 3 * (2 * r + 1) * vox
        roof = {"bound": "alu", "kernel": dom, "achieved": dd["tflops"], "peak": FP32_VECTOR_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": round(dd["tflops"] / FP32_VECTOR_PEAK_TFLOPS, 4),
                "per_launch": {"macs": macs, "bytes": alg_bytes, "ms": dd["ms"]}}
    else:
        roof = {"bound": "hbm", "kernel": dom, "achieved": dd["hbm_gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(dd["hbm_gbs"] / HBM_PEAK_GBS, 4),
                "per_launch": {"bytes": alg_bytes, "ms": dd["ms"]}}
    roof["traffic"] = traffic_for(dom, kind, n)

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


def run_precision(args):
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    dev = torch.device("cuda:0")
    n = args.size
    v = torch.clamp(phantoms.porous((n, n, n), seed=0, device=dev), 0, 1)
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


def run_chunked(args):
    import torch

    import paper_2511_11890_amd as h
    from paper_2511_11890_amd import phantoms

    n = args.size
    dev = torch.device("cuda:0")
    v = phantoms.porous_u16((n, n, n), seed=0, device=dev)
    host = torch.empty((n, n, n), dtype=torch.uint16, pin_memory=True)
    host.copy_(v)
    del v
    torch.cuda.empty_cache()
    out_g = torch.empty((n, n, n), dtype=torch.float32, pin_memory=True)
    out_o = torch.empty((n, n, n), dtype=torch.uint8, pin_memory=True)
    budget = 8 << 30
    res = {}
    for name, fn in (("gauss_s2", lambda ex: h.gaussian(host, 2.0, out=out_g, ex=ex)),
                     ("open_ball2", lambda ex: h.opening(host, "ball", 2, threshold=32768.0, out=out_o, ex=ex))):
        for label, chunk, bud in (("chunked_512", (512, 512, 512), budget), ("chunked_zslab", (0, 0, 0), budget),
                                  ("resident", (n, n, n), 200 << 30)):
            st = h.harpia_stats()
            fn(h.Exec(budget=bud, chunk=chunk, stats=st))
            t0 = time.perf_counter()
            st = h.harpia_stats()
            fn(h.Exec(budget=bud, chunk=chunk, stats=st))
            dt = time.perf_counter() - t0
            res["%s_%s" % (name, label)] = {"s": round(dt, 3), "gvox_s": round(n ** 3 / dt / 1e9, 2),
                                            "chunks": st.n_chunks, "peak_gib": round(st.peak_device_bytes / 2 ** 30, 2),
                                            "h2d_gb": round(st.bytes_h2d / 1e9, 2),
                                            "d2h_gb": round(st.bytes_d2h / 1e9, 2)}
    tot = res["gauss_s2_chunked_512"]["s"] + res["open_ball2_chunked_512"]["s"]
    return {"metric": METRIC, "value": round(2 * n ** 3 / tot / 1e9, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": 1, "warmup": 1, "ms_per_step": round(tot * 1000, 1), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u16", "data": "synthetic",
            "config": {"workload": "chunked %d^3 uint16 pinned host, 8 GiB budget, 512^3 bricks: Gaussian "
                                   "sigma 2 -> f32 + binary opening ball r=2 at 32768" % n},
            "ops": res}


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
    return {"metric": METRIC, "value": round(vox / ms / 1e6, 2), "unit": "GVox/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(wall * 1000 / args.steps, 3),
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": "batched: 64 float32 crops, extents U[64,256], Gaussian sigma 1.5 (learnable) "
                                   "+ box-5 dilation, forward + backward per step, one graph replay",
                       "voxels": vox, "crops": len(xs)},
            "ops": dict(phases, graph_ms=round(ms, 3), hbm_frac_alg20=round(alg / ms / 1e6 / HBM_PEAK_GBS, 4)),
            "tiles": tiles}


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

        sl = v[:32].double().cpu().numpy()
        t0 = time.perf_counter()
        oracle.mean3d(sl, 1, method="separable")
        oracle.mean3d(sl, 2, method="separable")
        oracle.unsharp3d(sl, 2.0, 1.0)
        oracle.edge3d(sl, "sobel")
        oracle.hessian3d(sl, 1.0)
        oracle.local_threshold3d(sl, "niblack", 2, k=-0.2)
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = {"value": round(11 * sl.size / dt / 1e9, 6), "unit": "GVox/s",
                                "cores": oracle.num_threads(), "kind": "oracle",
                                "sample": "%dx%dx%d slab: separable FP64 mean r=1,2 + unsharp (direct FP64 Gaussian) "
                                          "sigma 2 + direct FP64 Sobel + direct FP64 Hessian sigma 1 + Niblack r=2, %.1f s"
                                          % (sl.shape + (dt,))}
    return line


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="resident", choices=["resident", "precision", "chunked", "batched", "filters"])
    ap.add_argument("--size", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--copy-ref", action="store_true",
                    help="also run one plain device copy of the volume (counter reference)")
    ap.add_argument("--tune", action="store_true",
                    help="resident / batched / filters: run the autotuner on the ops first and merge its tiles "
                         "into --tiles")
    ap.add_argument("--tiles", default=TILES, help="tile file of the autotuner (loaded if present)")
    ap.add_argument("--stats-summary", nargs=3, metavar=("CSV_DIR", "COMMAND", "TITLE"),
                    help="print a markdown summary of a rocprofv3 --stats csv run and exit (no GPU)")
    ap.add_argument("--traffic-summary", nargs=4, metavar=("FETCH_DIR", "WRITE_DIR", "FETCH_CMD", "WRITE_CMD"),
                    help="print the HBM traffic JSON of two rocprofv3 --pmc runs and exit (no GPU)")
    args = ap.parse_args()
    if args.stats_summary:
        print(stats_summary(*args.stats_summary), end="")
        return
    if args.traffic_summary:
        fr, wr, fc, wc = args.traffic_summary
        print(json.dumps(traffic_summary(fr, wr, args.size or 1024, (fc, wc)), indent=1))
        return
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU: this build runs no multi-GPU path (one process, one device). "
              "Run with --gpus 1.", file=sys.stderr)
        sys.exit(2)
    if args.size == 0:
        args.size = 1024 if args.workload in ("resident", "filters") else 2048
    fn = {"resident": run_resident, "precision": run_precision, "chunked": run_chunked,
          "batched": run_batched, "filters": run_filters}[args.workload]
    print(json.dumps(fn(args)), flush=True)


if __name__ == "__main__":
    main()
