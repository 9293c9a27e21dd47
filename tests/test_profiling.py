"""The counter reduction used for the roofline's traffic figure (CPU only):
per-dispatch FETCH_SIZE/WRITE_SIZE rows scaled by a copy kernel of known size."""
import csv
import os

from paper_2308_08410_amd import profiling as P

HDR = ["Correlation_Id", "Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]


def _write(path, counter, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for i, (name, v) in enumerate(rows):
            w.writerow([i, i, name, counter, v])


def test_traffic_scaling(tmp_path):
    fetch, write = str(tmp_path / "f"), str(tmp_path / "w")
    # copy of 1 MiB reads as 512 KiB (scale 2) and writes 1024 KiB (scale 1)
    _write(fetch, "FETCH_SIZE", [("void k_sweep<false,16>(int)", 100.0), ("void k_sweep<false,16>(int)", 300.0),
                                 ("neg_kernel", 512.0), ("other", 9.0)])
    _write(write, "WRITE_SIZE", [("void k_sweep<false,16>(int)", 10.0), ("void k_sweep<false,16>(int)", 30.0),
                                 ("neg_kernel", 1024.0)])
    t = P.traffic(fetch, write, "k_sweep", "neg", copy_mib=1)
    assert t["dispatches"] == [2, 2]
    assert abs(t["fetch_scale"] - 2.0) < 1e-12 and abs(t["write_scale"] - 1.0) < 1e-12
    assert abs(t["bytes_per_launch"] - 1024 * (200.0 * 2 + 20.0)) < 1e-6
    out = tmp_path / "s.md"
    P.main(["--fetch", fetch, "--write", write, "--copy-mib", "1", "--out", str(out)])
    assert P.read_summary(str(out))["bytes_per_launch"] == t["bytes_per_launch"]


def test_valu_reduction(tmp_path):
    """Per-dispatch VALU and transcendental counts, averaged over dispatches, and
    the transcendental rate over the dispatch time against the quarter-rate peak."""
    d = str(tmp_path / "v")
    os.makedirs(d)
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]
    with open(os.path.join(d, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(hdr)
        for i, (valu, trans, busy) in enumerate(((1000.0, 100.0, 20.0), (3000.0, 300.0, 40.0))):
            w.writerow([i, "k_ecg_fwd(float const*)", "SQ_INSTS_VALU", valu, 0, 2000])
            w.writerow([i, "k_ecg_fwd(float const*)", "SQ_INSTS_VALU_TRANS_F32", trans, 0, 2000])
            w.writerow([i, "k_ecg_fwd(float const*)", "VALUBusy", busy, 0, 2000])
        w.writerow([9, "k_other", "SQ_INSTS_VALU", 5.0, 0, 10])
    t = P.valu(d, "k_ecg_fwd")
    assert t["dispatches"] == 2
    assert t["valu_insts_per_launch"] == 2000.0 and t["trans_insts_per_launch"] == 200.0
    assert t["trans_ops_per_launch"] == 64 * 200.0
    assert abs(t["trans_ops_per_s"] - 64 * 200.0 / 2e-6) < 1e-3
    assert abs(t["trans_frac"] - t["trans_ops_per_s"] / (256 * 4 * 4 * 2.4e9)) < 1e-15
    assert t["valu_busy_pct"] == 30.0
    out = tmp_path / "v.md"
    P.main(["--valu", d, "--kernel", "k_ecg_fwd", "--out", str(out)])
    assert P.read_summary(str(out))["trans_insts_per_launch"] == 200.0
