"""CPU tests of the profile summarisers on synthetic rocprofv3 CSV output with known answers."""
import argparse
import csv
import os

from paper_2608_15781_amd import profile_run

COUNTER_FIELDS = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _write_counters(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "run_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=COUNTER_FIELDS)
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(COUNTER_FIELDS, r)))


def test_summarize_scales_byte_counters_by_the_copy(tmp_path):
    """FETCH_SIZE per dispatch is averaged per kernel and scaled so that the last dispatch (the
    calibration copy) reads as copy_bytes: a copy of 512 MiB reading 262144 KiB gives factor 2."""
    out = str(tmp_path / "fetch")
    k = "void lbm::k_collide<1, false>(lbm::StepArgs<1>)"
    _write_counters(out, [
        (1, k, "FETCH_SIZE", 100.0, 0, 1000),
        (2, k, "FETCH_SIZE", 120.0, 2000, 3000),
        (3, "__amd_rocclr_copyBuffer", "FETCH_SIZE", 262144.0, 4000, 5000),
    ])
    stats = str(tmp_path / "fetch" / "run_kernel_stats.csv")
    with open(stats, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "AverageNs", "MinNs", "MaxNs"])
        w.writeheader()
        w.writerow(dict(Name=k, Calls=2, AverageNs=1000, MinNs=900, MaxNs=1100))
    res = profile_run.summarize(out, 512 << 20)
    c = res["counters"]["FETCH_SIZE"]
    assert c["copy_kernel"] == "__amd_rocclr_copyBuffer"
    assert abs(c["scale"] - 2.0) < 1e-12
    assert c["kib_per_dispatch"] == {"lbm::k_collide<1, false>": 110.0}
    assert res["kernels"]["lbm::k_collide<1, false>"]["avg_us"] == 1.0


def test_counters_report_normalises_by_duration_and_units(tmp_path, capsys):
    """TA busy = TA_TA_BUSY / (duration x clock x units), L2 hit = hit / (hit + miss), VMEM reads
    per wave = SQ_INSTS_VMEM_RD / SQ_WAVES, each averaged over the kernel's dispatches."""
    k = "void lbm::k_colour<1>(lbm::StepArgs<1>)"
    dur_ns = 10000  # 10 us
    busy = 0.5 * dur_ns * 1e-9 * profile_run.CLOCK_HZ * profile_run.N_CU
    _write_counters(str(tmp_path / "a"), [
        (1, k, "SQ_WAVES", 100.0, 0, dur_ns),
        (1, k, "SQ_INSTS_VMEM_RD", 5500.0, 0, dur_ns),
        (2, k, "SQ_WAVES", 100.0, 0, dur_ns),
        (2, k, "SQ_INSTS_VMEM_RD", 5500.0, 0, dur_ns),
    ])
    _write_counters(str(tmp_path / "b"), [
        (1, k, "TA_TA_BUSY", busy, 0, dur_ns),
        (1, k, "TA_ADDR_STALLED_BY_TC_CYCLES", 0.25 * busy, 0, dur_ns),
        (1, k, "TCC_HIT", 60.0, 0, dur_ns),
        (1, k, "TCC_HIT", 15.0, 0, dur_ns),  # a second hardware instance of the same counter
        (1, k, "TCC_MISS", 25.0, 0, dur_ns),
        (2, k, "TA_TA_BUSY", busy, 0, dur_ns),
        (2, k, "TA_ADDR_STALLED_BY_TC_CYCLES", 0.25 * busy, 0, dur_ns),
        (2, k, "TCC_HIT", 75.0, 0, dur_ns),
        (2, k, "TCC_MISS", 25.0, 0, dur_ns),
    ])
    args = argparse.Namespace(out=str(tmp_path / "a"), fetch=str(tmp_path / "b"), workload="bijel128",
                              precision="fp32", steps=5)
    profile_run.counters(args)
    text = capsys.readouterr().out
    assert "| `lbm::k_colour<1>` | 2 | 10.00 | 50% | 25% | 75% | 55.0 |" in text, text
    assert "- source_digest: " in text
