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


def test_mfma_table_rates_and_busy_fraction(tmp_path):
    """Flops = MOPS x 512 per dispatch, the rate over the kernel-trace average duration against the
    operand type's dense peak, busy = busy cycles / (GUI_ACTIVE summed over XCCs / XCCs x SIMDs)."""
    proj = "void dlr::(anonymous namespace)::k_project_mfma<2, float, false>(int)"
    gram = "void dlr::(anonymous namespace)::k_gram_mfma<double, 2>(long)"
    counters = tmp_path / "mfma.csv"
    with open(counters, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for disp, name, f32, f64, busy, gui in [(1, proj, 2.0e7, 0.0, 409.6e3, 8.0e3),
                                                (2, proj, 2.0e7, 0.0, 409.6e3, 8.0e3),
                                                (3, gram, 0.0, 1.0e6, 1024.0e3, 8.0e3)]:
            for cname, v in [("SQ_INSTS_VALU_MFMA_MOPS_F32", f32), ("SQ_INSTS_VALU_MFMA_MOPS_F64", f64),
                             ("SQ_VALU_MFMA_BUSY_CYCLES", busy), ("GRBM_GUI_ACTIVE", gui)]:
                w.writerow({"Dispatch_Id": disp, "Kernel_Name": name, "Counter_Name": cname, "Counter_Value": v})
    agent = tmp_path / "agent.csv"
    with open(agent, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Agent_Type", "Simd_Count", "Num_Xcc"])
        w.writeheader()
        w.writerow({"Agent_Type": "CPU", "Simd_Count": 0, "Num_Xcc": 0})
        w.writerow({"Agent_Type": "GPU", "Simd_Count": 1024, "Num_Xcc": 8})
    stats = tmp_path / "stats.csv"
    with open(stats, "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Name", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": proj, "AverageNs": 200000.0})   # 200 us
        w.writerow({"Name": gram, "AverageNs": 10000.0})    # 10 us
    md = profiling.mfma_md(str(counters), str(agent), str(stats), "t", ["cmd"])
    rows = {line.split("`")[1]: [c.strip() for c in line.strip().strip("|").split("|")] for line in md.splitlines()
            if "`k_" in line}
    p = rows["k_project_mfma<2, float, false>"]
    assert p[1] == "2" and p[2] == "F32"
    assert float(p[3]) == round(2.0e7 * 512 / 1e9, 3)                  # 10.240 GFLOP
    rate = 2.0e7 * 512 / 200e-6 / 1e12                                   # 51.2 TFLOP/s
    assert float(p[5]) == round(rate, 1) and float(p[6]) == round(100 * rate / 157.3, 1)
    assert float(p[7]) == round(100 * 409.6e3 / (8.0e3 / 8 * 1024), 1)   # 40 % of 1000 cycles x 1024 SIMDs
    g = rows["k_gram_mfma<double, 2>"]
    assert g[2] == "F64" and float(g[6]) == round(100 * (1.0e6 * 512 / 10e-6 / 1e12) / 78.6, 1)
