"""Host logic of the benchmark (no GPU): the mapping from profiler kernel
names to the library's timing-table names, and the conversion of two counter
runs into HBM bytes per dispatch scaled by the calibration copy."""
import csv
import json

import bench

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
       "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
       "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]

GEMM = "void lrr::(anonymous namespace)::k_dgemm<64, false, false, false>(lrr::GemmDesc const*, int, int, int)"
SYM = "void lrr::(anonymous namespace)::k_dgemm<64, true, false, true>(lrr::GemmDesc const*, int, int, int)"
EST = "void lrr::(anonymous namespace)::k_estep_w<4, true>(double*, double const*, double*, int, long)"
COPY = "__amd_rocclr_copyBuffer"


def test_kernel_names():
    assert bench.lib_kernel_name(GEMM) == "k_dgemm<false, false>"
    assert bench.lib_kernel_name(SYM) == "k_dgemm_sym"
    assert bench.lib_kernel_name(
        "void lrr::(anonymous namespace)::k_dgemm<32, true, true, false>(lrr::GemmDesc const*, int, int, int)"
    ) == "k_dgemm<true, true>"
    assert bench.lib_kernel_name(EST) == "k_estep"
    assert bench.lib_kernel_name("void lrr::(anonymous namespace)::k_update_Z_w<true>(double const*)") == "k_update_Z"
    assert bench.lib_kernel_name("void lrr::(anonymous namespace)::k_form_Y_w<false>(double const*)") == "k_form_Y"
    assert bench.lib_kernel_name("lrr::(anonymous namespace)::k_form_QT(double const*, double*)") == "k_form_QT"
    assert bench.lib_kernel_name(COPY) is None


def _write(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for did, name, val in rows:
            # two rows per dispatch (the counter is reported per XCD group): they add up
            for part in (0.25, 0.75):
                w.writerow([did, did, "Agent 1", 1, 1, 1, 256, 1, name, 256, 0, 0, 8, 0, 32, counter, val * part, 0, 1])


def test_traffic_from_counter_runs(tmp_path):
    # the copy moves 512 MiB each way; its FETCH_SIZE reads half (scale 2), WRITE_SIZE all (scale 1)
    fetch, write = tmp_path / "f.csv", tmp_path / "w.csv"
    _write(fetch, "FETCH_SIZE", [(1, GEMM, 1000.0), (2, GEMM, 3000.0), (3, EST, 500.0), (4, COPY, 262144.0)])
    _write(write, "WRITE_SIZE", [(1, GEMM, 100.0), (2, GEMM, 300.0), (3, EST, 800.0), (4, COPY, 524288.0)])
    out = tmp_path / "t.json"
    bench.traffic_from_pmc(str(fetch), str(write), str(out), "abc")
    t = json.load(open(out))
    assert t["_lib"] == "abc"
    assert abs(t["_scale"]["fetch"] - 2.0) < 1e-12 and abs(t["_scale"]["write"] - 1.0) < 1e-12
    # GEMM: mean fetch 2000 KiB x 2 + mean write 200 KiB x 1, in bytes
    assert t["k_dgemm<false, false>"] == round((2000.0 * 2 + 200.0) * 1024)
    assert t["k_estep"] == round((500.0 * 2 + 800.0) * 1024)
    assert "__amd_rocclr_copyBuffer" not in t
