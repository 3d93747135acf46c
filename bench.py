"""Benchmark of the one-sided box filter on one MI355X.

Workload (one step): the plain FP32 forward of a 3x2048x2048 piecewise-constant
image (Voronoi K=64, levels U[0,1], Gaussian noise sigma=0.03), channels as
independent planes, replicate boundary, T=30 sweeps, once for each radius
r in {2, 5, 10}.  The metric is megapixel-iterations per second
(H*W*C*T summed over the three radii, per second) and its share of the HBM
roofline at 8 bytes per pixel-sweep (read and write one FP32 iterate).

The other forms of the filter are reported under "forms", each next to the
plain FP32 forward on the same workload:
  batched   256 images, H, W in [64, 1024], 1 or 3 channels, r in {1,2,4,8},
            T in [5, 30]; one prepared batch replayed as a HIP graph
  bf16/f16  1x8192x8192 stored as BF16 / FP16, r=16, T=20, with the max/mean
            error against the FP64 oracle on crops (storage-only and total)
            from the committed parity record (tests/parity_report.py)
  dram      1x8192x8192 FP32, r in {2,5,10}, T=10: the bench radii on an image
            whose 2 x 256 MiB ping-pong does not fit the 256 MiB Infinity Cache
  fwd_bwd   32x3x512x512, r=3, T=10, loss sum(W*U): forward with uint8
            selection maps + backward, and with a checkpoint every 5 sweeps
  variants  the bench workload through the fast approximation (Alg. 3) and
            the classical box filter, the paper's two timing comparisons
  volume    a 256^3 FP32 volume (3D Voronoi K=64, sigma 0.05) through the
            14-window volume filter, r in {1,2,3,4}, T=10
  gaussian  the bench image through the one-sided Gaussian filter (Sec. II-B),
            r in {2,5,8} with sigma = r/2, T=10, next to the box filter
  autotune  the bench workload with the plans osbf_autotune measures on this
            device, next to the measured table the timed step uses
  small     one 256x256 plane (12 rectangles, sigma 0.05), r=2, T=10: launch
            bound, so reported as microseconds per call, eager and replayed
            from a HIP graph, with the table plan and the autotuned one

"parity" carries that record's checks of the timed workload itself (near-tie
flips per sweep, end-to-end error after T sweeps, oracle replay of the GPU's
selection maps) while the forward kernels and plans are the ones it was
taken on; the oracle itself runs here only for the CPU baseline.

Prints one JSON line (see the repository's benchmark contract).  Inputs are
resident in HBM before every timed region; each timed region is bracketed by
device synchronisations.
"""
from __future__ import annotations

import argparse
import hashlib
import glob
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
BYTES_PER_PX_SWEEP = 8         # FP32 read + write of the iterate
RADII = (2, 5, 10)
T_SWEEPS = 30
H = W = 2048
C = 3


# sources that define the planar forward kernels (their launch shape is
# checked separately through the plans)
FWD_KERNEL_SOURCES = ("osbf_device.h", "osbf_fwd_device.h", "osbf_forward.hip", "osbf_stream_device.h",
                      "osbf_stream.hip")


def fwd_kernel_name(plan) -> str:
    """The forward kernel a plan launches: the row-streaming kernels have a
    tile height of 0 (rows chosen at launch), the fused two-sweep one for
    plans that fuse two sweeps."""
    if plan["tile"][1] == 0:
        return "osbf::fwd_stream2_kernel" if plan["fused"] == 2 else "osbf::fwd_stream_kernel"
    return "osbf::fwd_fixed_kernel"


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for name in FWD_KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2108_05021_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def plan_signature(plans) -> dict:
    return {str(r): [p["tile"][0], p["tile"][1], p["fused"]] for r, p in sorted(plans.items())}


def measured_traffic(config_key: str, plans):
    """HBM bytes per launch from the committed rocprofv3 counter summary, if it
    was taken on the current forward kernel sources with the same launch
    plans (else None)."""
    path = os.path.join(ROOT, "profiles", "fwd_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash() or d.get("plans") != plan_signature(plans):
        return None
    return d.get("per_launch_bytes", {}).get(config_key)


# VALU issue peak with packed FP32 disabled: 256 CUs x 4 SIMDs x 16 lanes x
# 2.4 GHz lane-operations per second
VALU_PEAK_TLANE_OPS = 256 * 4 * 16 * 2.4e9 / 1e12


def measured_valu(plans):
    """VALU lane-operations per pixel-sweep by radius from the committed
    rocprofv3 SQ_INSTS_VALU record, if it was taken on the current forward
    kernel sources with the same launch plans (else None)."""
    path = os.path.join(ROOT, "profiles", "fwd_valu.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash() or d.get("plans") != plan_signature(plans):
        return None
    ops = d.get("lane_ops_per_px_sweep", {})
    return {int(r): float(v) for r, v in ops.items()}


def parity_record(plans):
    """Parity of the GPU path against the FP64 oracle, from the committed
    record written by tests/parity_report.py, if it was taken on the current
    forward kernel sources with the same launch plans (else None)."""
    path = os.path.join(ROOT, "profiles", "parity_record.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        d = json.load(f)
    if d.get("kernel_hash") != kernel_source_hash() or d.get("plans") != plan_signature(plans):
        return None
    return d


def _counter_rows(path):
    """Per-kernel mean of every counter per dispatch from a rocprofv3
    --pmc --output-format csv directory."""
    import csv
    sums, disp = {}, {}
    for f in glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            for row in csv.DictReader(fh):
                k = row["Kernel_Name"]
                sums.setdefault(k, {}).setdefault(row["Counter_Name"], 0.0)
                sums[k][row["Counter_Name"]] += float(row["Counter_Value"])
                disp.setdefault(k, set()).add(row["Dispatch_Id"])
    return {k: {c: v / len(disp[k]) for c, v in cs.items()} for k, cs in sums.items()}, \
        {k: len(v) for k, v in disp.items()}


def write_counter_records(path, out_dir=None):
    """Write profiles/fwd_traffic.json and profiles/fwd_valu.json from the
    rocprofv3 counter runs of the timed step under `path` (subdirectories
    fetch, write: FETCH_SIZE / WRITE_SIZE of `bench.py --steps 1 --warmup 1
    --no-cpu-baseline --no-forms`; copy_fetch, copy_write: the same of
    `bench.py --copy-calibration`; sq: SQ_INSTS_VALU of the step).  The
    records carry the forward sources' hash and the plans, so bench.py uses
    them only while both still hold.  `out_dir` defaults to profiles/."""
    import re

    import torch

    from paper_2108_05021_amd import osbf
    plans = {r: osbf.forward_plan(C, H, W, torch.float32, r, T_SWEEPS) for r in RADII}
    pat = re.compile(r"osbf::fwd_(?:stream2?|fixed)_kernel<0, (\d+),")

    def by_radius(sub, counter):
        rows, _ = _counter_rows(os.path.join(path, sub))
        out = {}
        for k, cs in rows.items():
            m = pat.search(k)
            if m and counter in cs:
                out[int(m.group(1))] = cs[counter]
        return out

    def copy_kib(sub, counter):
        rows, _ = _counter_rows(os.path.join(path, sub))
        vals = [cs[counter] for k, cs in rows.items() if "copyBuffer" in k and counter in cs]
        if not vals:
            raise SystemExit(f"no device copy dispatch with {counter} under {sub}")
        return max(vals)

    copy_kib_total = (64 << 20) * 4 / 1024
    ff = copy_kib_total / copy_kib("copy_fetch", "FETCH_SIZE")
    wf = copy_kib_total / copy_kib("copy_write", "WRITE_SIZE")
    fetch, write = by_radius("fetch", "FETCH_SIZE"), by_radius("write", "WRITE_SIZE")
    per = {f"r{r}_k{plans[r]['fused']}": round((fetch[r] * ff + write[r] * wf) * 1024) for r in RADII}
    launches = sum(plans[r]["launches"] for r in RADII)
    per["rgb2048_T30"] = round(sum(per[f"r{r}_k{plans[r]['fused']}"] * plans[r]["launches"] for r in RADII)
                               / launches)
    step = "python bench.py --steps 1 --warmup 1 --no-cpu-baseline --no-forms"
    cmd = "rocprofv3 --pmc {c} --output-format csv -d " + path.rstrip("/") + "/{d} -o pmc -- {p}"
    common = {"kernel_hash": kernel_source_hash(), "plans": plan_signature(plans)}
    traffic = {
        "about": f"HBM-side bytes per launch of the forward kernels on the {C}x{H}x{W} FP32 workload "
                 f"(r in {set(RADII)}, T={T_SWEEPS}), from rocprofv3 FETCH_SIZE and WRITE_SIZE (KiB per "
                 f"dispatch) scaled by a plain 256 MiB device copy (factors {ff:.2f} and {wf:.2f}).  Valid "
                 "only for the forward kernel sources with this hash and these launch plans.",
        **common, "fetch_factor": round(ff, 4), "write_factor": round(wf, 4),
        "fetch_kib": {str(r): round(fetch[r], 1) for r in RADII},
        "write_kib": {str(r): round(write[r], 1) for r in RADII},
        "per_launch_bytes": per,
        "commands": [cmd.format(c="FETCH_SIZE", d="fetch", p=step), cmd.format(c="WRITE_SIZE", d="write", p=step),
                     cmd.format(c="FETCH_SIZE", d="copy_fetch", p="python bench.py --copy-calibration"),
                     cmd.format(c="WRITE_SIZE", d="copy_write", p="python bench.py --copy-calibration")]}
    valu = by_radius("sq", "SQ_INSTS_VALU")
    pxs = C * H * W
    valu_rec = {
        "about": f"VALU lane-operations per pixel-sweep of the forward kernels on the {C}x{H}x{W} FP32 workload: "
                 "rocprofv3 SQ_INSTS_VALU (wave instructions per dispatch) x 64 lanes / (pixels x sweeps "
                 "per launch).  Valid only for the forward kernel sources with this hash and these launch plans.",
        **common,
        "lane_ops_per_px_sweep": {str(r): round(valu[r] * 64 / (pxs * plans[r]["fused"]), 2) for r in RADII},
        "command": cmd.format(c="SQ_WAVES SQ_INSTS_VALU SQ_INSTS_LDS SQ_INSTS_SALU SQ_WAVE_CYCLES SQ_BUSY_CYCLES "
                                "SQ_INSTS_VMEM_RD SQ_INSTS_VMEM_WR", d="sq", p=step)}
    for name, rec in (("fwd_traffic.json", traffic), ("fwd_valu.json", valu_rec)):
        with open(os.path.join(out_dir or os.path.join(ROOT, "profiles"), name), "w") as f:
            json.dump(rec, f, indent=1)
            f.write("\n")
    print(json.dumps({"traffic": per, "valu": valu_rec["lane_ops_per_px_sweep"]}))


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


def copy_ceiling():
    """Device copy bandwidth (read + write bytes per second) of a plain D2D
    copy: 48 MiB, the size of one bench iterate (its ping-pong stays in the
    256 MiB Infinity Cache), and 1 GiB (DRAM)."""
    import torch
    res = {}
    for tag, nbytes in (("48MiB", 48 << 20), ("1GiB", 1 << 30)):
        a = torch.ones(nbytes // 4, device="cuda")
        b = torch.empty_like(a)
        best = 1e30
        for _ in range(3):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            b.copy_(a)
            e0.record()
            for _ in range(10):
                b.copy_(a)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) / 10)
        res[f"GBs_{tag}"] = round(2 * nbytes / (best * 1e-3) / 1e9, 1)
        del a, b
    torch.cuda.empty_cache()
    return res


def cpu_baseline(img, budget_s: float = 10.0):
    """The FP64 oracle on the host: the whole bench image (all planes), as
    many consecutive sweeps per radius as fit in budget_s / 3 seconds (at
    least one), scaled to MPix*it/s with the same equal mix of radii (each
    radius's time per sweep counts once per sweep of the bench)."""
    import numpy as np
    import oracle

    planes = np.ascontiguousarray(img, dtype=np.float64)
    threads = int(os.environ.get("OMP_NUM_THREADS", os.cpu_count() or 1))
    per_sweep = {}
    done = {}
    for r in RADII:
        cur = planes
        n, t_r = 0, 0.0
        while n == 0 or t_r < budget_s / len(RADII):
            t0 = time.perf_counter()
            cur = oracle.forward(cur, r, 1, nthreads=threads)
            t_r += time.perf_counter() - t0
            n += 1
        per_sweep[r] = t_r / n
        done[r] = n
    # one bench step = T_SWEEPS sweeps of each radius on the whole image
    step_s = sum(per_sweep[r] * T_SWEEPS for r in RADII)
    pxit = len(RADII) * C * H * W * T_SWEEPS
    total = sum(per_sweep[r] * done[r] for r in RADII)
    # the launch-bound single 256^2 plane (r=2, T=10) on one host thread
    from paper_2108_05021_amd import synth
    small = synth.workload_single().astype(np.float64)
    t0 = time.perf_counter()
    oracle.forward(small, 2, 10, nthreads=1)
    t_small = time.perf_counter() - t0
    return {"value": pxit / step_s / 1e6, "unit": "MPix*it/s", "cores": threads, "kind": "oracle",
            "cpu_model": cpu_model(),
            "sample": f"all {C} planes of the bench image; consecutive sweeps per r: "
                      + ", ".join(f"r={r}: {done[r]}" for r in RADII)
                      + f" of {T_SWEEPS} ({total:.1f} s wall on {threads} threads)",
            "single_thread_256x256_r2_T10": {"seconds": round(t_small, 4),
                                             "mpix_it_s": round(small.size * 10 / t_small / 1e6, 2)}}


def _timed(fn, reps, warmup=2, warm_s=0.05):
    """Seconds per call of fn over `reps` calls, after at least `warmup` calls
    and `warm_s` seconds of untimed calls (the device's first tens of
    milliseconds of work run measurably slower)."""
    import torch
    t_end = time.perf_counter() + warm_s
    n = 0
    while n < warmup or time.perf_counter() < t_end:
        fn()
        torch.cuda.synchronize()
        n += 1
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def form_batched(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    items = synth.workload_batched()
    xs = [torch.from_numpy(it["img"]).cuda() for it in items]
    rs = [it["r"] for it in items]
    ts = [it["T"] for it in items]
    pxit = sum(x.numel() * T for x, T in zip(xs, ts))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan = osbf.BatchPlan(xs, rs, ts)   # workspace, host planning and table upload, timed apart
    torch.cuda.synchronize()
    prepare_s = time.perf_counter() - t0
    plan.launch()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    st = torch.cuda.Stream()
    st.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(st):
        with torch.cuda.graph(g, stream=st):
            plan.launch()
    torch.cuda.current_stream().wait_stream(st)
    t_graph = _timed(g.replay, reps)
    t_eager = _timed(plan.launch, reps)
    outs = [torch.empty_like(x) for x in xs]

    def single():
        for x, y, r, T in zip(xs, outs, rs, ts):
            osbf.forward(x, r, T, out=y)
    t_single = _timed(single, max(1, reps // 2), warmup=1)
    # rows per work item tuned per radius on this device, then replayed again
    t0 = time.perf_counter()
    tuned_rows = osbf.batched_autotune(xs, rs, ts)
    tuning_s = time.perf_counter() - t0
    plan2 = osbf.BatchPlan(xs, rs, ts)
    plan2.launch()
    torch.cuda.synchronize()
    g2 = torch.cuda.CUDAGraph()
    with torch.cuda.stream(st):
        with torch.cuda.graph(g2, stream=st):
            plan2.launch()
    torch.cuda.current_stream().wait_stream(st)
    t_tuned = _timed(g2.replay, reps)
    osbf.autotune_clear()
    return {"workload": "256 images, H,W in [64,1024], C in {1,3}, Voronoi K=16 + N(0,0.05^2), "
                        "r in {1,2,4,8}, T in [5,30], f32",
            "mpix_it": round(pxit / 1e6, 1), "rounds": plan.batch.rounds, "grid": plan.batch.grid,
            "prepare_ms": round(prepare_s * 1e3, 2),
            "graph_ms": round(t_graph * 1e3, 3), "mpix_it_s": round(pxit / t_graph / 1e6, 1),
            "eager_launch_mpix_it_s": round(pxit / t_eager / 1e6, 1),
            "plain_fp32_forward_per_image_mpix_it_s": round(pxit / t_single / 1e6, 1),
            "vs_plain_fwd": round(t_single / t_graph, 3),
            "partition": "per round and kernel class, items grouped by image and split over the 8 XCDs by "
                         "estimated cost (LPT)",
            "autotuned": {"rows_per_item": {str(r): v for r, v in tuned_rows.items()},
                          "graph_mpix_it_s": round(pxit / t_tuned / 1e6, 1), "tuning_s": round(tuning_s, 2)}}


def form_precision(reps, errors=True):
    import torch
    from paper_2108_05021_amd import osbf, synth
    r, T = 16, 20
    img = synth.workload_precision()[0]
    x32 = torch.from_numpy(img).cuda()[None]
    pxit = x32.numel() * T
    t32 = _timed(lambda: osbf.forward(x32, r, T), reps)
    out = {"workload": "1x8192x8192 Voronoi K=256 + N(0,0.02^2), r=16, T=20",
           "plain_fp32_forward_mpix_it_s": round(pxit / t32 / 1e6, 1)}
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        xs = x32.to(dt)
        t = _timed(lambda: osbf.forward(xs, r, T), reps)
        out[name] = {"mpix_it_s": round(pxit / t / 1e6, 1), "vs_plain_fwd": round(t32 / t, 3)}
    if errors:
        # errors against the FP64 oracle come from the committed parity record
        # (tests/parity_report.py) while the kernels and plans it was taken on
        # are the current ones
        plans = {rr: osbf.forward_plan(C, H, W, torch.float32, rr, T_SWEEPS) for rr in RADII}
        rec = parity_record(plans)
        if rec is None:
            out["errors"] = None
        else:
            p = rec["precision"]
            out["f32_err_max"], out["f32_err_mean"] = p["f32_err_max"], p["f32_err_mean"]
            for name in ("bf16", "f16"):
                out[name].update(p[name])
            out["err_sample"] = p["crops"]
    return out


def form_dram(reps):
    """The bench radii on an image whose ping-pong (2 x 256 MiB) is larger than
    the 256 MiB Infinity Cache, so every sweep reads and writes DRAM (the
    bench image's 2 x 48 MiB stay in that cache)."""
    import torch
    from paper_2108_05021_amd import osbf, synth
    T = 10
    x = torch.from_numpy(synth.workload_precision()[0]).cuda()[None]
    pxit = x.numel() * T
    out = {"workload": "1x8192x8192 Voronoi K=256 + N(0,0.02^2), FP32, r in {2,5,10}, T=10 "
                       "(2 x 256 MiB ping-pong)"}
    for r in RADII:
        t = _timed(lambda: osbf.forward(x, r, T), reps)
        gbs = 8 * pxit / t / 1e9
        out[f"r{r}"] = {"mpix_it_s": round(pxit / t / 1e6, 1), "us_per_sweep": round(t / T * 1e6, 2),
                        "achieved_GBs": round(gbs, 1), "frac_hbm_peak": round(gbs / HBM_PEAK_GBS, 4)}
    return out


def form_fwd_bwd(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    r, T = 3, 10
    x_np, w_np = synth.workload_grad()
    x = torch.from_numpy(x_np).cuda()
    w = torch.from_numpy(w_np).cuda()
    pxit = x.numel() * T
    t_fwd = _timed(lambda: osbf.forward(x, r, T), reps)

    def maps():
        y, sel = osbf.forward(x, r, T, return_sel=True)
        return osbf.backward(w, r, T, sel=sel)

    def ckpt():
        y, ck = osbf.forward(x, r, T, ckpt_every=5)
        return osbf.backward(w, r, T, ckpt=ck, ck=5)
    t_maps = _timed(maps, reps)
    t_ck = _timed(ckpt, reps)
    _, sel = osbf.forward(x, r, T, return_sel=True)
    t_adj = _timed(lambda: osbf.backward(w, r, T, sel=sel), reps)
    return {"workload": "32x3x512x512 Voronoi K=64 + N(0,0.05^2), r=3, T=10, loss sum(W*U), W~N(0,1)",
            "plain_fp32_forward_mpix_it_s": round(pxit / t_fwd / 1e6, 1),
            "maps_u8": {"mpix_it_s": round(pxit / t_maps / 1e6, 1), "vs_plain_fwd": round(t_fwd / t_maps, 3),
                        "map_bytes": T * x.numel()},
            "ckpt_every_5": {"mpix_it_s": round(pxit / t_ck / 1e6, 1), "vs_plain_fwd": round(t_fwd / t_ck, 3)},
            "adjoint_only": {"mpix_it_s": round(pxit / t_adj / 1e6, 1),
                             "achieved_GBs": round(9 * pxit / t_adj / 1e9, 1), "bytes_per_px_sweep": 9}}


def form_gaussian(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    x = torch.from_numpy(synth.workload_rgb()).cuda()
    T = 10
    res = {"workload": "3x2048x2048 f32 (the bench image), T=10, sigma = r/2, replicate boundary"}
    for _ in range(8):  # the first radius timed must not pay for a cold device
        osbf.gaussian_forward(x, 5, 2.5, T)
    for r in (2, 5, 8):
        tg = _timed(lambda: osbf.gaussian_forward(x, r, r / 2.0, T), reps)
        tb = _timed(lambda: osbf.forward(x, r, T), reps)
        res[f"r{r}"] = {"mpix_it_s": round(x.numel() * T / tg / 1e6, 1),
                        "box_filter_mpix_it_s": round(x.numel() * T / tb / 1e6, 1),
                        "time_over_box_filter": round(tg / tb, 3)}
    return res


def form_small(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    x = torch.from_numpy(synth.workload_single()).cuda()
    planes, H, W = x.shape
    r, T = 2, 10
    out = torch.empty_like(x)
    ws = torch.empty(max(1, osbf.forward_workspace_size(planes, H, W, torch.float32, r, T)),
                     dtype=torch.uint8, device=x.device)
    res = {"workload": "1x256x256 f32, 12 rectangles on 0.5 + N(0,0.05^2), r=2, T=10, replicate boundary"}
    n = 40 * reps

    def measure(tag):
        def call():
            osbf.osbf_forward(x, out, r, T, ws=ws)
        call()
        torch.cuda.synchronize()
        want = out.clone()
        t_eager = _timed(call, n, warmup=20)
        g = torch.cuda.CUDAGraph()
        st = torch.cuda.Stream()
        st.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(st):
            with torch.cuda.graph(g, stream=st):
                call()
        torch.cuda.current_stream().wait_stream(st)
        for _ in range(3):  # every replay equals the eager result
            out.zero_()
            g.replay()
            torch.cuda.synchronize()
            if not torch.equal(out, want):
                raise RuntimeError("graph replay differs from the eager forward")
        t_graph = _timed(g.replay, n, warmup=20)
        # ten calls in one graph: a graph launch's fixed cost is then paid
        # once per ten calls
        g10 = torch.cuda.CUDAGraph()
        with torch.cuda.stream(st):
            with torch.cuda.graph(g10, stream=st):
                for _ in range(10):
                    call()
        torch.cuda.current_stream().wait_stream(st)
        out.zero_()
        g10.replay()
        torch.cuda.synchronize()
        if not torch.equal(out, want):
            raise RuntimeError("graph replay differs from the eager forward")
        t_graph10 = _timed(g10.replay, max(1, n // 10), warmup=3) / 10
        plan = osbf.forward_plan(planes, H, W, torch.float32, r, T)
        res[tag] = {"plan": {"tile": list(plan["tile"]), "fused": plan["fused"], "launches": plan["launches"]},
                    "eager_us": round(t_eager * 1e6, 2), "graph_us": round(t_graph * 1e6, 2),
                    "graph_10_calls_us_per_call": round(t_graph10 * 1e6, 2),
                    "graph_launch_overhead_us": round((t_graph - t_graph10) * 1e6 * 10 / 9, 2),
                    "eager_mpix_it_s": round(x.numel() * T / t_eager / 1e6, 1),
                    "graph_mpix_it_s": round(x.numel() * T / t_graph / 1e6, 1),
                    "graph_10_calls_mpix_it_s": round(x.numel() * T / t_graph10 / 1e6, 1)}

    measure("table")
    osbf.autotune(x, r, T)
    measure("autotuned")
    osbf.autotune_clear()
    return res


def form_autotune(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    x = torch.from_numpy(synth.workload_rgb()).cuda()
    res = {"workload": "the bench workload (3x2048x2048 f32, T=30)"}
    osbf.autotune_clear()
    for _ in range(8):  # the first plan timed must not pay for a cold device
        osbf.forward(x, RADII[0], T_SWEEPS)
    for r in RADII:
        table = osbf.forward_plan(C, H, W, torch.float32, r, T_SWEEPS)
        t_table = _timed(lambda: osbf.forward(x, r, T_SWEEPS), reps, warmup=4)
        t0 = time.perf_counter()
        tuned = osbf.autotune(x, r, T_SWEEPS)
        tune_s = time.perf_counter() - t0
        t_tuned = _timed(lambda: osbf.forward(x, r, T_SWEEPS), reps, warmup=4)
        res[f"r{r}"] = {"table_plan": {"tile": list(table["tile"]), "fused": table["fused"]},
                        "table_mpix_it_s": round(x.numel() * T_SWEEPS / t_table / 1e6, 1),
                        "tuned_plan": {"tile": list(tuned["tile"]), "fused": tuned["fused"]},
                        "tuned_mpix_it_s": round(x.numel() * T_SWEEPS / t_tuned / 1e6, 1),
                        "tuning_s": round(tune_s, 3)}
    osbf.autotune_clear()
    return res


def form_volume(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    x = torch.from_numpy(synth.workload_volume()).cuda()
    T = 10
    res = {"workload": "256^3 f32 volume, 3D Voronoi K=64 + N(0,0.05^2), T=10, 14 windows "
                       "(6 halves, 8 octants), replicate boundary"}
    for _ in range(8):  # the first radius timed must not pay for a cold device
        osbf.forward3d(x, 2, T)
    for r in (1, 2, 3, 4):
        t = _timed(lambda: osbf.forward3d(x, r, T), reps)
        res[f"r{r}"] = {"mvox_it_s": round(x.numel() * T / t / 1e6, 1),
                        "achieved_GBs": round(BYTES_PER_PX_SWEEP * x.numel() * T / t / 1e9, 1)}
    return res


def form_variants(reps):
    import torch
    from paper_2108_05021_amd import osbf, synth
    x = torch.from_numpy(synth.workload_rgb()).cuda()
    pxit = x.numel() * T_SWEEPS * len(RADII)
    t = {}
    for name, fn in (("exact", osbf.forward), ("fast", osbf.forward_fast), ("box", osbf.box_forward)):
        t[name] = _timed(lambda: [fn(x, r, T_SWEEPS) for r in RADII], reps)
    per_r = {}
    for r in RADII:
        te = _timed(lambda: osbf.forward(x, r, T_SWEEPS), reps)
        tb = _timed(lambda: osbf.box_forward(x, r, T_SWEEPS), reps)
        per_r[str(r)] = {"exact_mpix_it_s": round(x.numel() * T_SWEEPS / te / 1e6, 1),
                         "box_mpix_it_s": round(x.numel() * T_SWEEPS / tb / 1e6, 1),
                         "exact_time_over_box": round(te / tb, 3)}
    return {"workload": "3x2048x2048 f32, r in {2,5,10}, T=30 (the bench workload)",
            "exact_mpix_it_s": round(pxit / t["exact"] / 1e6, 1),
            "fast_mpix_it_s": round(pxit / t["fast"] / 1e6, 1),
            "box_mpix_it_s": round(pxit / t["box"] / 1e6, 1),
            "fast_time_over_exact": round(t["fast"] / t["exact"], 3),
            "exact_time_over_box": round(t["exact"] / t["box"], 3),
            "per_radius": per_r,
            "box_kernel": "separable two-pass box (vertical running sum in registers, horizontal in LDS)",
            "paper_context": "fast/exact ~0.6 and exact/box ~8 (MATLAB) or ~6 (C++) on a laptop CPU, r unstated"}


FORMS = ("batched", "precision", "dram", "fwd_bwd", "variants", "volume", "gaussian", "small", "autotune")


def run_form(name, args, reps=5):
    if name == "precision":
        return form_precision(reps, errors=not args.no_errors)
    return globals()["form_" + name](reps)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the batched/bf16/f16/fwd+bwd forms")
    ap.add_argument("--no-errors", action="store_true", help="skip the oracle error crops of the bf16/f16 form")
    ap.add_argument("--form", choices=sorted(FORMS), default=None,
                    help="run only this form (for profiling it) and print its result; no timed step")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 256 MiB device copy 5 times (for scaling HBM counters)")
    ap.add_argument("--counter-records", metavar="DIR", default=None,
                    help="write profiles/fwd_traffic.json and fwd_valu.json from the rocprofv3 counter "
                         "runs under DIR (no GPU needed)")
    args = ap.parse_args()
    if args.counter_records:
        write_counter_records(args.counter_records)
        return
    if args.copy_calibration:
        import torch
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": src.numel() * 4, "copies": 5}), flush=True)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (asked for {args.gpus}); the filter's multi-GPU "
              "sharding is a design note, not built.", file=sys.stderr)
        sys.exit(2)
    if args.form:
        print(json.dumps({"form": args.form, **run_form(args.form, args)}), flush=True)
        return

    import numpy as np
    import torch

    from paper_2108_05021_amd import osbf, synth

    dev = torch.device("cuda:0")
    img = synth.workload_rgb()
    x = torch.from_numpy(img).to(dev)
    out = torch.empty_like(x)
    ws = torch.empty(osbf.forward_workspace_size(C, H, W, torch.float32, max(RADII), T_SWEEPS),
                     dtype=torch.uint8, device=dev)
    plans = {r: osbf.forward_plan(C, H, W, torch.float32, r, T_SWEEPS) for r in RADII}
    stream = torch.cuda.current_stream(dev)

    def step(events=None):
        for i, r in enumerate(RADII):
            if events is not None:
                events[i][0].record(stream)
            osbf.osbf_forward(x, out, r, T_SWEEPS, ws=ws)
            if events is not None:
                events[i][1].record(stream)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # timed region: K steps, per-call events on the launch stream
    ev = [[[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in RADII] for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in range(args.steps):
        step(ev[s])
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0

    per_r_ms = {r: sum(ev[s][i][0].elapsed_time(ev[s][i][1]) for s in range(args.steps)) / args.steps
                for i, r in enumerate(RADII)}
    pxit_step = len(RADII) * C * H * W * T_SWEEPS
    ms_per_step = wall * 1e3 / args.steps
    value = pxit_step / (ms_per_step / 1e3) / 1e6

    kernels = []
    tot_bytes = tot_ms = 0.0
    for r in RADII:
        p = plans[r]
        launch_us = per_r_ms[r] * 1e3 / p["launches"]
        alg_bytes = BYTES_PER_PX_SWEEP * C * H * W * p["fused"]
        kernels.append({"r": r, "kernel": fwd_kernel_name(p), "tile": list(p["tile"]), "fused": p["fused"],
                        "launches": p["launches"],
                        "avg_launch_us": round(launch_us, 2),
                        "achieved_GBs": round(alg_bytes / launch_us / 1e3, 1),
                        "mpix_it_s": round(C * H * W * T_SWEEPS / (per_r_ms[r] / 1e3) / 1e6, 1)})
        tot_bytes += BYTES_PER_PX_SWEEP * C * H * W * T_SWEEPS
        tot_ms += per_r_ms[r]
    achieved = tot_bytes / (tot_ms / 1e3) / 1e9
    traffic = measured_traffic("rgb2048_T30", plans)
    # the kernels' own bound: VALU issue (lane-operations measured per
    # pixel-sweep, times the pixel-sweeps of each radius, over its time)
    valu = measured_valu(plans)
    alu = None
    if valu and all(r in valu for r in RADII):
        ops = sum(valu[r] * C * H * W * T_SWEEPS for r in RADII)
        a_t = ops / (tot_ms / 1e3) / 1e12
        alu = {"achieved": round(a_t, 2), "peak": round(VALU_PEAK_TLANE_OPS, 2), "unit": "Tlane-op/s",
               "frac": round(a_t / VALU_PEAK_TLANE_OPS, 4),
               "lane_ops_per_px_sweep": {str(r): valu[r] for r in RADII}}

    line = {
        "metric": "megapixel-iterations/s (fwd, batched, fwd+bwd) and % of HBM peak",
        "value": round(value, 1),
        "unit": "MPix*it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "3x2048x2048 f32 Voronoi(K=64)+N(0,0.03^2), r in {2,5,10}, T=30, "
                               "replicate boundary, plain forward",
                   "planes": C, "height": H, "width": W, "radii": list(RADII), "iterations": T_SWEEPS},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic,
                     "kernel": " + ".join(dict.fromkeys(k["kernel"] for k in kernels)), "kernels": kernels,
                     "bytes_per_px_sweep": BYTES_PER_PX_SWEEP, "valu_issue": alu},
    }
    rec = parity_record(plans)
    line["parity"] = None if rec is None else {
        "workload": "the timed workload; FP64 oracle on 32x32 crops (tests/parity_report.py)",
        "tolerance": "1e-5 abs on the selected window's mean; near-tie flips within "
                     "tau = 2^-19 N (1 + max|U|) are counted; end to end, 1e-5 outside the "
                     "dependency cones of the sweeps where the GPU's window had another mean",
        **{r: {"flips": v["teacher_forced"]["flips"], "flip_pixels_checked": v["teacher_forced"]["pixels"],
               "teacher_forced_max_err": v["teacher_forced"]["max_err"],
               "err_max": v["end_to_end"]["err_max"], "err_mean": v["end_to_end"]["err_mean"],
               "err_max_outside_flip_cones": v["end_to_end"].get("err_max_outside_flip_cones"),
               "flip_cone_fraction": v["end_to_end"].get("flip_cone_fraction"),
               "replay_outliers": v["replay"]["outliers"], "replay_max_dev": v["replay"]["max_dev"]}
           for r, v in rec["headline"].items()}}
    cc = copy_ceiling()
    line["roofline"]["copy_ceiling"] = cc
    line["roofline"]["frac_of_copy_48MiB"] = round(achieved / cc["GBs_48MiB"], 4)
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(img)
    if not args.no_forms:
        del x, out, ws
        torch.cuda.empty_cache()
        line["forms"] = {name: run_form(name, args) for name in FORMS}
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
