"""bench.py's counter-record writer on synthetic rocprofv3 CSV output (CPU):
per-radius bytes are FETCH_SIZE and WRITE_SIZE scaled by what the same
counters read for the 256 MiB calibration copy, VALU lane-ops per
pixel-sweep are SQ_INSTS_VALU x 64 / pixels, and the records carry the
current kernel hash and plans (so bench.py accepts them)."""
import csv
import json
import os

import bench

FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "pmc_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, FIELDS)
        w.writeheader()
        for i, (kernel, counter, value) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value})


def test_counter_records_from_csv(tmp_path):
    import torch

    from paper_2108_05021_amd import osbf
    plans = {r: osbf.forward_plan(bench.C, bench.H, bench.W, torch.float32, r, bench.T_SWEEPS) for r in bench.RADII}
    name = {r: f"void osbf::fwd_stream_kernel<0, {r}, 192, {r}, false, 0>(osbf::FwdLaunch)" for r in bench.RADII}
    copy = "__amd_rocclr_copyBuffer"
    fetch = {2: 30000.0, 5: 31000.0, 10: 32000.0}       # KiB per dispatch
    valu = {2: 9.0e6, 5: 10.0e6, 10: 11.0e6}            # wave instructions per dispatch
    d = tmp_path / "pmc"
    # two dispatches per radius (averaged), a foreign kernel that must be ignored
    _csv(d / "fetch", [(name[r], "FETCH_SIZE", fetch[r]) for r in bench.RADII for _ in range(2)]
         + [("void other(int)", "FETCH_SIZE", 1.0)])
    _csv(d / "write", [(name[r], "WRITE_SIZE", 49152.0) for r in bench.RADII for _ in range(2)])
    _csv(d / "copy_fetch", [(copy, "FETCH_SIZE", 131072.0)])    # half the copied KiB: factor 2
    _csv(d / "copy_write", [(copy, "WRITE_SIZE", 262144.0)])    # factor 1
    _csv(d / "sq", [(name[r], "SQ_INSTS_VALU", valu[r]) for r in bench.RADII for _ in range(2)])
    out = tmp_path / "records"
    out.mkdir()
    bench.write_counter_records(str(d), out_dir=str(out))
    t = json.loads((out / "fwd_traffic.json").read_text())
    v = json.loads((out / "fwd_valu.json").read_text())
    assert t["kernel_hash"] == v["kernel_hash"] == bench.kernel_source_hash()
    assert t["plans"] == v["plans"] == bench.plan_signature(plans)
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    for r in bench.RADII:
        k = f"r{r}_k{plans[r]['fused']}"
        assert t["per_launch_bytes"][k] == round((fetch[r] * 2 + 49152.0) * 1024)
        assert v["lane_ops_per_px_sweep"][str(r)] == round(valu[r] * 64 / (bench.C * bench.H * bench.W * plans[r]["fused"]), 2)
