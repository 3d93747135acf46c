"""Parity record of the benchmark workloads against the FP64 oracle (run on a
GPU machine; test infrastructure, like the tests themselves).

Headline workload (3x2048x2048 FP32, r in {2, 5, 10}, T = 30), per radius:
  teacher_forced  every sweep of the GPU run, one sweep per call (the same
                  bits as the T = 30 call, which is checked), on six 32x32
                  crops grown by r: value-changing near-tie flips against the
                  oracle's own selection, and the largest |GPU - mean of the
                  GPU's window| (parity.sweep_region)
  end_to_end      the T = 30 GPU output against the untethered oracle run on
                  each crop grown by r*T (exact at the crop): max and mean
                  |GPU - oracle|, and the max outside the dependency cones
                  of the sweeps where the GPU chose a window of another mean
                  (parity.untethered_errors) with the share of the crop
                  those cones cover
  replay          the oracle replaying the GPU's 30 selection maps on those
                  grown crops (parity.replay_region): outliers must be 0
Precision workload (1x8192x8192, r = 16, T = 20): max / mean |GPU - oracle| of
FP32, BF16 and FP16 storage on three 32x32 crops grown by r*T, against the
oracle run on the cast input (storage error) and on the FP32 input (total).

    python tests/parity_report.py [--out profiles/parity_record.json]

The record carries the forward kernels' source hash and launch plans;
bench.py attaches it to its JSON line only while both match.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
sys.path[:0] = [ROOT, HERE]

import numpy as np  # noqa: E402
import torch  # noqa: E402

import bench  # noqa: E402
import oracle  # noqa: E402
import parity  # noqa: E402
from paper_2108_05021_amd import osbf, synth  # noqa: E402

SIZE = 32
# (plane, y0, x0): corner, centre, far corner, top edge, left edge, interior
CROPS = [(0, 0, 0), (1, 1008, 1008), (2, 2048 - SIZE, 2048 - SIZE), (0, 0, 1000), (1, 1000, 0), (2, 512, 1536)]


def headline(dev, log):
    x = torch.from_numpy(synth.workload_rgb()).to(dev)
    C, H, W = x.shape
    T = bench.T_SWEEPS
    out = {}
    for r in bench.RADII:
        t0 = time.time()
        cur = x
        tf = {"flips": 0, "pixels": 0, "max_err": 0.0}
        for t in range(T):
            nxt, sel = osbf.forward(cur, r, 1, return_sel=True)
            for (p, y0, x0) in CROPS:
                (ya, yb, xa, xb), cuts = parity.region_of(H, W, y0, x0, SIZE, r)
                f, px, d = parity.sweep_region(cur[p, ya:yb, xa:xb].cpu().numpy(),
                                               nxt[p, ya:yb, xa:xb].cpu().numpy(),
                                               sel[0, p, ya:yb, xa:xb].cpu().numpy(), r, cuts)
                tf["flips"] += f
                tf["pixels"] += px
                tf["max_err"] = max(tf["max_err"], d)
            cur = nxt
        y, sels = osbf.forward(x, r, T, return_sel=True)
        assert torch.equal(y, cur), "the T-sweep call differs from single-sweep calls"
        e2e, outside, in_cones = [], [], []
        rep = {"outliers": 0, "max_dev": 0.0, "flips": 0, "pixels": 0}
        for (p, y0, x0) in CROPS:
            (ya, yb, xa, xb), cuts = parity.region_of(H, W, y0, x0, SIZE, r * T)
            u0 = x[p, ya:yb, xa:xb].cpu().numpy()
            ug = y[p, ya:yb, xa:xb].cpu().numpy()
            n_bad, dmax, flips, px = parity.replay_region(u0, ug, sels[:, p, ya:yb, xa:xb].cpu().numpy(), r, cuts)
            rep["outliers"] += n_bad
            rep["max_dev"] = max(rep["max_dev"], dmax)
            rep["flips"] += flips
            rep["pixels"] += px
            # the oracle's own run on the crop grown by r*T (exact at the
            # crop), and the cones of the sweeps where the runs' windows had
            # different means (seeds outside the grown crop's exact region
            # never reach the crop)
            err, cone = parity.untethered_errors(u0, ug, sels[:, p, ya:yb, xa:xb].cpu().numpy(), r)
            cy, cx = y0 - ya, x0 - xa
            e_c, k_c = err[cy:cy + SIZE, cx:cx + SIZE], cone[cy:cy + SIZE, cx:cx + SIZE]
            e2e.append(e_c)
            outside.append(e_c[~k_c])
            in_cones.append(k_c)
        e = np.concatenate([v.ravel() for v in e2e])
        eo = np.concatenate(outside)
        kc = np.concatenate([v.ravel() for v in in_cones])
        out[str(r)] = {
            "teacher_forced": {"sweeps": T, "crops": len(CROPS), **tf},
            "end_to_end": {"err_max": float(e.max()), "err_mean": float(e.mean()), "pixels": int(e.size),
                           "margin": r * T,
                           "err_max_outside_flip_cones": float(eo.max()) if eo.size else 0.0,
                           "flip_cone_fraction": float(kc.mean())},
            "replay": rep,
        }
        log(f"headline r={r}: {out[str(r)]} ({time.time() - t0:.1f} s)")
    return out


def precision(dev, log):
    r, T = 16, 20
    img = synth.workload_precision()[0]
    H, W = img.shape
    crops = [(0, 0), (4000, 4100), (H - SIZE, W - SIZE)]
    x32 = torch.from_numpy(img).to(dev)[None]
    res = {"workload": "1x8192x8192 Voronoi K=256 + N(0,0.02^2), r=16, T=20",
           "crops": "3 crops of 32x32 (corner, centre, far corner), oracle on each grown by r*T"}
    cache = {}

    def oracle_crop(src_name, src, y0, x0):
        key = (src_name, y0, x0)
        if key not in cache:
            (ya, yb, xa, xb), _ = parity.region_of(H, W, y0, x0, SIZE, r * T)
            want = oracle.forward(src[ya:yb, xa:xb].astype(np.float64), r, T)
            cache[key] = want[y0 - ya:y0 - ya + SIZE, x0 - xa:x0 - xa + SIZE]
        return cache[key]

    def errs(gpu_out, src_name, src):
        e = np.concatenate([np.abs(gpu_out[y0:y0 + SIZE, x0:x0 + SIZE].astype(np.float64)
                                   - oracle_crop(src_name, src, y0, x0)).ravel() for (y0, x0) in crops])
        return float(e.max()), float(e.mean())

    y32 = osbf.forward(x32, r, T)[0].cpu().numpy()
    res["f32_err_max"], res["f32_err_mean"] = errs(y32, "f32", img)
    for name, dt in (("bf16", torch.bfloat16), ("f16", torch.float16)):
        xs = x32.to(dt)
        y = osbf.forward(xs, r, T)[0].float().cpu().numpy()
        cast_in = xs[0].float().cpu().numpy()
        d = {}
        d["storage_only_err_max"], d["storage_only_err_mean"] = errs(y, name + "_in", cast_in)
        d["total_err_max"], d["total_err_mean"] = errs(y, "f32", img)
        res[name] = d
    log(f"precision: {res}")
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=os.path.join(ROOT, "profiles", "parity_record.json"))
    args = ap.parse_args()
    dev = torch.device("cuda:0")

    def log(msg):
        print(msg, flush=True)

    plans = {r: osbf.forward_plan(3, bench.H, bench.W, torch.float32, r, bench.T_SWEEPS) for r in bench.RADII}
    rec = {"command": "python tests/parity_report.py",
           "kernel_hash": bench.kernel_source_hash(), "plans": bench.plan_signature(plans),
           "headline": headline(dev, log), "precision": precision(dev, log)}
    with open(args.out, "w") as f:
        json.dump(rec, f, indent=1)
    log(f"wrote {args.out}")


if __name__ == "__main__":
    main()
