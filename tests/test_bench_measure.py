"""The benchmark's measurement helpers on the CPU: algorithmic bytes per
launch (the per-row figures of the kernel table), the rocprofv3 counter and
trace summaries on small synthetic CSV files whose answers are worked out by
hand here, and the one-GPU guard of the command line."""
import csv
import os
import subprocess
import sys

import pytest

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
N = 1 << 20
# a 3-level hierarchy: (rows, entries) per level
LEVELS = [[N, 7 * N], [150_000, 1_800_000], [20_000, 300_000]]


def test_fine_kernel_bytes():
    assert bench.algorithmic_bytes("k_spmv_J<float>(x)", N) == 76 * N          # 56 J + 4 z + 8 q + 8 y
    assert bench.algorithmic_bytes("k_spmv_J<float>(x)", N, shifted=False) == 68 * N
    assert bench.algorithmic_bytes("k_st25<double, float, 0>(x)", N) == 32 * N  # 8 b + 16 M + 4 D + 4 r
    assert bench.algorithmic_bytes("k_st25<double, float, 0>(x)", N, mixed=False) == 56 * N
    assert bench.algorithmic_bytes("k_faces_tiled<false, false>(x)", N) == 32 * N
    assert bench.algorithmic_bytes("k_faces_tiled<true, false>(x)", N) == 132 * N
    assert bench.algorithmic_bytes("k_update_norm<7>(x)", N) == 8 * N * 9       # K vectors + w in and out
    assert bench.algorithmic_bytes("k_multidot<7>(x)", N) == 8 * N * 8
    # the post-smoother needs the hierarchy (a gather per coarse row)
    assert bench.algorithmic_bytes("k_st25<double, float, 1>(x)", N) is None
    assert bench.algorithmic_bytes("k_st25<double, float, 1>(x)", N, 0, LEVELS) == 36 * N + 4 * LEVELS[1][0]
    assert bench.algorithmic_bytes("k_block_update<10>(x)", N, 1024, LEVELS) is None


def test_coarse_kernel_bytes_found_by_block_count():
    n0, n1, n2 = LEVELS[0][0], LEVELS[1][0], LEVELS[2][0]
    nnz1 = LEVELS[1][1]
    # restriction 0 -> 1: one block per 256 coarse rows, padded to a multiple of 8
    b01 = -(-(-(-n1 // 256)) // 8) * 8
    assert bench.algorithmic_bytes("k_restrict<float>(x)", N, b01, LEVELS) == n0 * 8 + n1 * (12 + 8)
    # restriction 1 -> 2 stores no pre-smoothed iterate (level 2 is the coarsest)
    b12 = -(-(-(-n2 // 256)) // 8) * 8
    assert bench.algorithmic_bytes("k_restrict<float>(x)", N, b12, LEVELS) == n1 * 8 + n2 * 12
    # CSR-stream on level 1: one block per 1536 entries, padded to a multiple of 8
    bs = -(-(-(-nnz1 // 1536)) // 8) * 8
    pre = bench.algorithmic_bytes("k_csr_stream<2, float, float, false>(x)", N, bs, LEVELS)
    post = bench.algorithmic_bytes("k_csr_stream<2, float, float, true>(x)", N, bs, LEVELS)
    assert pre == nnz1 * 8 + n1 * 20
    assert post == nnz1 * 8 + n1 * 40 + n2 * 4
    assert bench.algorithmic_bytes("k_csr_stream<2, float, float, true>(x)", N, bs + 8, LEVELS) is None


def _write_counters(path, cname, rows):
    with open(path, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for k, grid, v in rows:
            w.writerow({"Kernel_Name": k, "Grid_Size": grid, "Counter_Name": cname, "Counter_Value": v})


def test_pmc_summary_calibration_and_family_ratio(tmp_path):
    """The copy of 1 GiB reads back as 0.5 GiB of FETCH_SIZE (factor 2) and
    1 GiB of WRITE_SIZE (factor 1); a J product whose calibrated traffic is
    1.25 x its 76 N algorithmic bytes must come out at 1.25."""
    kib = 1024.0
    alg = 76 * N
    fetch = [("__amd_rocclr_copyBuffer", 0, (1 << 30) / 2 / kib),
             ("k_spmv_J<float>(rich::Phys)", 65536, 1.25 * alg / 2 / 2 / kib),   # half of it fetched, x2 calibration
             ("k_spmv_J<float>(rich::Phys)", 65536, 1.25 * alg / 2 / 2 / kib)]
    write = [("__amd_rocclr_copyBuffer", 0, (1 << 30) / kib),
             ("k_spmv_J<float>(rich::Phys)", 65536, 1.25 * alg / 2 / kib),
             ("k_spmv_J<float>(rich::Phys)", 65536, 1.25 * alg / 2 / kib)]
    _write_counters(tmp_path / "f.csv", "FETCH_SIZE", fetch)
    _write_counters(tmp_path / "w.csv", "WRITE_SIZE", write)
    info = {"options": {"gmres_block": 10}}
    text = bench.pmc_summary(str(tmp_path / "f.csv"), str(tmp_path / "w.csv"), N, info=info)
    assert "FETCH_SIZE x2.0000, WRITE_SIZE x1.0000" in text
    fam = [ln.split() for ln in text.splitlines() if ln.startswith("family spmv_J")]
    assert len(fam) == 1
    assert fam[0][2] == "2" and float(fam[0][3]) == pytest.approx(1.25, abs=1e-4)
    assert fam[0][4] == "fine.hip" and fam[0][5] == bench.source_digest("fine.hip")


def test_stats_and_gaps_summaries(tmp_path):
    st = tmp_path / "stats.csv"
    with open(st, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Name", "Calls", "TotalDurationNs", "AverageNs"])
        w.writeheader()
        w.writerow({"Name": "void rich::(anonymous namespace)::k_a<1>(int)", "Calls": 2, "TotalDurationNs": 3000,
                    "AverageNs": 1500})
        w.writerow({"Name": "void rich::(anonymous namespace)::k_a<2>(int)", "Calls": 1, "TotalDurationNs": 1000,
                    "AverageNs": 1000})
        w.writerow({"Name": "k_b(int)", "Calls": 4, "TotalDurationNs": 4000, "AverageNs": 1000})
    text = bench.stats_summary(str(st))
    assert text.splitlines()[0] == "total kernel time 0.000 s"
    fam = {ln.split()[0]: ln.split() for ln in text.splitlines()[2:4]}
    assert fam["k_a"][1] == "3" and fam["k_a"][4] == "50.0%"
    assert fam["k_b"][1] == "4" and fam["k_b"][4] == "50.0%"
    tr = tmp_path / "trace.csv"
    with open(tr, "w", newline="") as f:
        w = csv.DictWriter(f, fieldnames=["Kernel_Name", "Start_Timestamp", "End_Timestamp"])
        w.writeheader()
        # k_a 0-100, k_b 150-250 (50 idle), k_a 240-300 (overlap), k_b 400-500 (100 idle)
        for k, s, e in (("k_a<1>(int)", 0, 100), ("k_b(int)", 150, 250), ("k_a<2>(int)", 240, 300),
                        ("k_b(int)", 400, 500)):
            w.writerow({"Kernel_Name": k, "Start_Timestamp": s, "End_Timestamp": e})
    lines = bench.trace_gaps(str(tr)).splitlines()
    assert lines[0].startswith("kernels 4, span 0.000 s")
    assert "(30.0%)" in lines[0]  # 150 ns idle of a 500 ns span
    # both gaps fall between the families k_a and k_b: one line, two gaps of 75 ns on average
    assert len(lines) == 3
    f = lines[2].split()
    assert f[0] == "k_a" and f[1] == "->" and f[2] == "k_b" and f[4] == "2" and f[5] == "0.1"


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""
