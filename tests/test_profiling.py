"""Host-side checks of the rocprofv3 summary helpers (paper_2601_18705_amd.profiling) on small
synthetic CSV files: the calibration scaling of the HBM counters, the per-kernel traffic table and
the kernel-time table with excluded kernels."""
import csv

from paper_2601_18705_amd import profiling

CALIB = "void at::native::vectorized_elementwise_kernel<4, at::native::AUnaryFunctor<float, float, float, MulFunctor<float> > >(int)"
SWEEP = "void dlr::(anonymous namespace)::k_sweep<float, 4>(dlr::SweepArgs<float> const*)"
SMALL = "void dlr::(anonymous namespace)::k_chol<32>(int)"


def write_counters(path, counter, values):
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for name, v in values:
            w.writerow({"Kernel_Name": name, "Counter_Name": counter, "Counter_Value": v})


def counter_files(tmp_path):
    fetch, write = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # the calibration kernel moves 256 MiB each way: FETCH reads half of it, WRITE all of it
    write_counters(fetch, "FETCH_SIZE", [(SWEEP, 100000.0), (SWEEP, 120000.0), (SMALL, 4.0), (CALIB, 131072.0)])
    write_counters(write, "WRITE_SIZE", [(SWEEP, 50000.0), (SWEEP, 50000.0), (SMALL, 2.0), (CALIB, 262144.0)])
    return fetch, write


def test_sweep_traffic_scales_by_the_calibration_kernel(tmp_path):
    fetch, write = counter_files(tmp_path)
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    rec = profiling.sweep_traffic(str(fetch), str(write), 256.0, str(src))
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["sweep_launches"] == 2
    assert rec["fetch_bytes_per_launch"] == 110000.0 * 1024 * 2
    assert rec["write_bytes_per_launch"] == 50000.0 * 1024
    assert rec["hbm_bytes_per_launch"] == rec["fetch_bytes_per_launch"] + rec["write_bytes_per_launch"]


def test_traffic_table_lists_kernels_above_the_threshold(tmp_path):
    fetch, write = counter_files(tmp_path)
    md = profiling.traffic_table_md(str(fetch), str(write), 256.0, "title", ["cmd one", "cmd two"])
    assert "cmd one" in md and "cmd two" in md
    row = [line for line in md.splitlines() if "k_sweep" in line]
    assert len(row) == 1
    cells = [c.strip() for c in row[0].strip("|").split("|")]
    assert cells[1] == "2"
    assert float(cells[2]) == round(110000.0 * 1024 * 2 / 1e6, 1)
    assert float(cells[3]) == round(50000.0 * 1024 / 1e6, 1)
    assert "k_chol" not in md            # below 20 MB per dispatch
    assert "MulFunctor" not in md.split("| kernel |")[1]   # the calibration kernel is not listed


def test_kernel_stats_exclusion_recomputes_the_shares(tmp_path):
    path = tmp_path / "stats.csv"
    rows = [("void dlr::(anonymous namespace)::k_sweep<float, 4>(int)", 8, 3e6),
            ("void dlr::(anonymous namespace)::k_q1_sweep<float>(int)", 5, 6e6),
            ("dlr::(anonymous namespace)::k_svd(int)", 4, 1e6)]
    with open(path, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs", "MinNs", "MaxNs",
                                           "Percentage"])
        w.writeheader()
        for name, calls, tot in rows:
            w.writerow({"Name": name, "Calls": calls, "TotalDurationNs": tot, "AverageNs": tot / calls,
                        "MinNs": tot / calls, "MaxNs": tot / calls, "Percentage": 100.0 * tot / 1e7})
    md = profiling.kernel_stats_md(str(path), "t", "c", exclude=("k_q1_sweep",))
    assert "k_q1_sweep" not in md
    shares = {line.split("`")[1]: float(line.strip().strip("|").split("|")[-1]) for line in md.splitlines()
              if "`k_" in line}
    assert shares == {"k_sweep<float, 4>": 75.0, "k_svd": 25.0}
