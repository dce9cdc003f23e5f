"""The rocprofv3 summarizer: calibration scaling and the source-hash check
that keeps stale counters out of the bench line."""
import csv

from paper_2603_14641_amd import profsum

HDR = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size", "Kernel_Id",
       "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count",
       "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _csv(path, counter, rows):
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(HDR)
        for i, (name, val) in enumerate(rows):
            grid = 131072 if "copyBuffer" in name else 64
            w.writerow([i, i, "Agent 1", 1, 1, 1, grid, 1, name, 64, 0, 0, 8, 0, 16, counter, val, 0, 1])


def test_short_name():
    assert profsum.short_name("void sq::k_layer<2, 4>(unsigned long long*, sq::Group const*)") == "k_layer<2, 4>"
    assert profsum.short_name("__amd_rocclr_copyBuffer") == "__amd_rocclr_copyBuffer"


def test_hbm_scaling_and_staleness(tmp_path):
    layer = "void sq::k_layer<2, 4>(unsigned long long*, unsigned int)"
    fetch = tmp_path / "f.csv"
    write = tmp_path / "w.csv"
    # the copy moves 1 GiB each way but FETCH_SIZE reads half of it: factor 2;
    # a later, larger copy (4 GiB) must not be taken for the calibration
    cp = "__amd_rocclr_copyBuffer"
    _csv(fetch, "FETCH_SIZE", [(cp, 524288.0)] * 3 + [(layer, 100.0), (layer, 300.0), (cp, 2097152.0)])
    _csv(write, "WRITE_SIZE", [(cp, 1048576.0)] * 3 + [(layer, 50.0), (layer, 50.0), (cp, 4194304.0)])
    text = profsum.hbm_summary(str(fetch), str(write), "t", "cmd")
    summ = tmp_path / "s.md"
    summ.write_text(text)
    # (200 KiB * 2 + 50 KiB * 1) per dispatch
    assert profsum.traffic_per_dispatch("k_layer", str(summ)) == 400 * 1024 + 50 * 1024
    assert profsum.traffic_per_dispatch("k_rowsum", str(summ)) is None
    stale = text.replace(f"source={profsum.source_hash('k_layer<2, 4>')}", "source=0000000000000000")
    summ.write_text(stale)
    assert profsum.traffic_per_dispatch("k_layer", str(summ)) is None


def test_every_kernel_maps_to_a_source():
    import os
    import re
    names = set()
    for f in os.listdir(profsum.CSRC):
        if f.endswith(".hip"):
            with open(os.path.join(profsum.CSRC, f)) as fh:
                names |= set(re.findall(r"__global__.*?\bvoid\s+(k_\w+)", fh.read(), re.S))
    assert names
    for k in names:
        assert profsum.source_of(k) is not None, k
