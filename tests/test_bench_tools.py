"""The profile summaries that bench.py writes from rocprofv3 output (CPU only):
synthetic counter and trace files with known answers go through the same
code that made the committed files under profiles/."""
import csv
import os

import pytest

import bench

COPY = "void wd::k_stream_copy(HIP_vector_type<unsigned int, 4u> const*, HIP_vector_type<unsigned int, 4u>*, unsigned long)"
UPD = "void wd::k_cg_update_tiled<4, true>(wd::Geom, void const*, wd::SpinorBuf, wd::SpinorBuf, double)"
GIB8_KIB = (8 << 30) // 1024


def _write_counters(directory, rows):
    os.makedirs(directory, exist_ok=True)
    with open(os.path.join(directory, "p_counter_collection.csv"), "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for i, (kernel, counter, value, dur_ns) in enumerate(rows):
            w.writerow({"Dispatch_Id": i, "Kernel_Name": kernel, "Counter_Name": counter, "Counter_Value": value,
                        "Start_Timestamp": 1000, "End_Timestamp": 1000 + dur_ns})


def _read_kv(path):
    kv = {}
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            k, v = line.split(":", 1)
            kv[k.strip()] = v.strip()
    return kv


def test_traffic_from_request_sizes(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    os.makedirs(bench.PROFILES)
    # the copy: 8 GiB read in 128-byte requests (FETCH_SIZE reads half), 8 GiB written
    n128_copy = (8 << 30) // 128
    # the kernel: reads 300 MB as 128-byte lines plus some 64- and 32-byte pieces,
    # FETCH_SIZE counting the 128-byte ones as 64 bytes; writes 58 MiB
    n128, n64, n32 = 2_300_000, 1_000, 500
    fetch_kib = (64 * n128 + 64 * n64 + 32 * n32) / 1024
    write_kib = 59_392.0
    _write_counters(tmp_path / "fetch", [(COPY, "FETCH_SIZE", GIB8_KIB / 2, 3_000_000),
                                         (UPD, "FETCH_SIZE", fetch_kib, 90_000)])
    _write_counters(tmp_path / "write", [(COPY, "WRITE_SIZE", GIB8_KIB, 3_000_000),
                                         (UPD, "WRITE_SIZE", write_kib, 90_000)])
    rd = []
    for kernel, n in ((COPY, (n128_copy, 0, 0)), (UPD, (n128, n64, n32))):
        rd += [(kernel, "TCC_EA0_RDREQ_sum", sum(n), 1000), (kernel, "TCC_EA0_RDREQ_128B_sum", n[0], 1000),
               (kernel, "TCC_EA0_RDREQ_64B_sum", n[1], 1000), (kernel, "TCC_EA0_RDREQ_32B_sum", n[2], 1000)]
    _write_counters(tmp_path / "rdreq", rd)
    bench.summarize_traffic(str(tmp_path / "fetch"), str(tmp_path / "write"), str(tmp_path / "rdreq"))
    kv = _read_kv(os.path.join(bench.PROFILES, "traffic_k_cg_update_tiled_i8_rows2_32x32x32x64.txt"))
    reads = 128 * n128 + 64 * n64 + 32 * n32
    assert float(kv["read_bytes_per_launch"]) == pytest.approx(reads, rel=1e-9)
    assert float(kv["fetch_scale"]) == pytest.approx(2.0)
    assert float(kv["write_scale"]) == pytest.approx(1.0)
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx(reads + write_kib * 1024, rel=1e-9)
    V = 32 * 32 * 32 * 64
    assert int(kv["algorithmic_bytes_per_launch"]) == 180 * V
    # without the request-size pass: FETCH_SIZE scaled by the copy
    bench.summarize_traffic(str(tmp_path / "fetch"), str(tmp_path / "write"))
    kv = _read_kv(os.path.join(bench.PROFILES, "traffic_k_cg_update_tiled_i8_rows2_32x32x32x64.txt"))
    assert float(kv["traffic_bytes_per_launch"]) == pytest.approx((2 * fetch_kib + write_kib) * 1024, rel=1e-9)


def test_issue_summary(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path / "profiles"))
    os.makedirs(bench.PROFILES)
    waves, valu, xcds, simds = 32768, 1300, 8, 1024
    cycles = 220_000                     # per XCD: 91.7 us at 2.4 GHz
    dur = int(cycles / 2.4)              # ns
    vals = {"SQ_WAVES": waves, "SQ_INSTS_VALU": waves * valu, "SQ_INSTS_VMEM_RD": waves * 66,
            "SQ_INSTS_VMEM_WR": waves * 4, "SQ_INSTS_LDS": waves * 61, "SQ_INSTS_SALU": waves * 93,
            "SQ_WAIT_INST_ANY": 360, "SQ_WAVE_CYCLES": 1000, "GRBM_GUI_ACTIVE": cycles * xcds}
    d = tmp_path / "issue"
    os.makedirs(d)
    with open(d / "p_counter_collection.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value",
                                          "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        for name, v in vals.items():
            w.writerow({"Dispatch_Id": 7, "Kernel_Name": UPD, "Counter_Name": name, "Counter_Value": v,
                        "Start_Timestamp": 0, "End_Timestamp": dur})
    with open(d / "p_agent_info.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Agent_Type", "Simd_Count", "Num_Xcc"])
        w.writeheader()
        w.writerow({"Agent_Type": "GPU", "Simd_Count": simds, "Num_Xcc": xcds})
    bench.summarize_issue(str(d))
    lines = open(os.path.join(bench.PROFILES, "issue_hot_kernels_32x32x32x64.md")).read().splitlines()
    row = [l for l in lines if l.startswith("k_cg_update_tiled_i8_rows2 |")][0].split(" | ")
    assert row[1] == str(waves) and row[2] == str(valu)
    assert float(row[8]) == pytest.approx(2.4, abs=0.01)                 # clock
    assert float(row[9]) == pytest.approx(waves * valu * 4 / simds / cycles, abs=0.01)   # VALU-issue
    assert float(row[10]) == pytest.approx(0.36, abs=0.01)               # wait share


def test_trace_summary_per_grid(tmp_path, capsys):
    d = tmp_path / "trace"
    os.makedirs(d)
    with open(d / "t_kernel_trace.csv", "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X"])
        w.writeheader()
        for grid, us in ((663552, 30.0), (10616832, 400.0)):
            for _ in range(5):
                w.writerow({"Kernel_Name": UPD, "Start_Timestamp": 0, "End_Timestamp": int(us * 1000),
                            "Grid_Size_X": grid})
        w.writerow({"Kernel_Name": UPD, "Start_Timestamp": 0, "End_Timestamp": 3000, "Grid_Size_X": 663552})
    bench.summarize_trace(str(d))
    out = capsys.readouterr().out.splitlines()
    assert "k_cg_update_tiled<4, true> | grid 663552 | 6 | 5 | 30.0" in out   # a gated 3 us launch left out
    assert "k_cg_update_tiled<4, true> | grid 10616832 | 5 | 5 | 400.0" in out


def test_source_sha_ignores_comments_only(tmp_path, monkeypatch):
    assert bench.strip_c_comments('int a; // x "y"\n/* z\n */ const char* s = "//k /*"; char c = \'/\';') == \
        'int a; const char* s = "//k /*"; char c = \'/\';'
    src = os.path.normpath(os.path.join(bench.CSRC, ".."))
    pkg = tmp_path / "pkg"
    (pkg / "csrc").mkdir(parents=True)
    (tmp_path / "include").mkdir()
    for rel in bench.KERNEL_SOURCES:
        text = open(os.path.normpath(os.path.join(src, rel)), encoding="utf-8").read()
        open(os.path.normpath(os.path.join(pkg, rel)), "w", encoding="utf-8").write(text)
    monkeypatch.setattr(bench, "CSRC", str(pkg / "csrc"))
    base = bench.kernel_source_sha()
    k = pkg / "csrc" / "wd_kernels.hip"
    text = k.read_text(encoding="utf-8")
    k.write_text("// a new comment\n" + text.replace("\n", "  \n", 3), encoding="utf-8")
    assert bench.kernel_source_sha() == base
    k.write_text(text.replace("kForceSites = 64", "kForceSites = 32"), encoding="utf-8")
    assert bench.kernel_source_sha() != base
