"""The rocprofv3 summary tool (paper_1612_04787_amd/counters.py) on synthetic
counter and trace files: kernel naming, the traffic calibration against a
reference kernel or a copy, the per-launch-size trace summary, and reading
the summaries back."""
import csv

from paper_1612_04787_amd import counters as K


def _pmc_csv(path, rows):
    """rows: (kernel name, grid size, counter, value)"""
    with open(path, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        for r in rows:
            w.writerow(r)


ROW_FWD = "void swift::k_row_fwd<512, 8, 11264, 5, false>(swift::MatchArgs)"
PROJ = "void swift::k_project<3>(unsigned char const*, long, long, int, int, int, unsigned char const*, unsigned char*)"
COPY = "void at::native::elementwise_kernel_manual_unroll<128, 8, at::native::direct_copy_kernel_cuda(...)>"


def test_short_names():
    assert K.short_name(ROW_FWD) == "k_row_fwd<512>"
    assert K.short_name("void swift::k_bwd_col<1024, true>(swift::BwdArgs)") == "k_cj_col<1024>"
    assert K.short_name("void swift::k_bwd_row<512, true, false>(swift::BwdArgs)") == "k_cj_row<512>"
    assert K.short_name("void swift::k_bwd_col<256, false>(swift::BwdArgs)") == "k_bwd_col<256>"
    assert K.short_name("void swift::k_col_pair<512, true>(swift::MatchArgs)") == "k_col_pair_pruned<512>"
    assert K.short_name("void swift::k_col_pair<1024, false>(swift::MatchArgs)") == "k_col_pair<1024>"
    assert K.short_name("void swift::k_row_inv<512, 16, true, false>(swift::MatchArgs)") == "k_row_inv_pruned<512>"
    assert K.short_name("void swift::k_row_inv<512, 16, true, true>(swift::MatchArgs)") == "k_row_inv_pearson<512>"
    assert K.short_name("void swift::k_row_fwd<512, 8, 11264, 5, true>(swift::MatchArgs)") == "k_row_fwd_pearson<512>"
    assert K.short_name(PROJ) == "k_project<3>"
    assert K.short_name("void foo<int>(int)") is None


def test_traffic_reference_kernel_full_size_launches(tmp_path):
    """The reference's full-size launches set the scale, not the smaller ones
    of the same grid; the scale applies per counter; rows are per launch of
    each kernel's largest grid."""
    gib = 1 << 30
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    # k_project<3>: two full launches (FETCH counts half the bytes) and one
    # quarter-size launch on the same grid
    _pmc_csv(f, [(PROJ, 1048576, "FETCH_SIZE", gib / 2048), (PROJ, 1048576, "FETCH_SIZE", gib / 2048),
                 (PROJ, 1048576, "FETCH_SIZE", gib / 8192),
                 (ROW_FWD, 33554432, "FETCH_SIZE", 1000.0), (ROW_FWD, 1024, "FETCH_SIZE", 5.0)])
    _pmc_csv(w, [(PROJ, 1048576, "WRITE_SIZE", gib / 1024), (PROJ, 1048576, "WRITE_SIZE", gib / 1024),
                 (PROJ, 1048576, "WRITE_SIZE", gib / 4096),
                 (ROW_FWD, 33554432, "WRITE_SIZE", 3000.0), (ROW_FWD, 1024, "WRITE_SIZE", 7.0)])
    out = K.traffic(str(f), str(w), gib, ref_kernel="k_project<3>", ref_bytes=gib)
    lines = {l.split()[0]: l.split() for l in out.splitlines() if l.split()}
    assert abs(float(lines["scale_fetch"][1]) - 2.0) < 1e-4
    assert abs(float(lines["scale_write"][1]) - 1.0) < 1e-4
    assert lines["source_digest"][1] == K.source_digest()
    rd, wr, tot = (float(x) for x in lines["k_row_fwd<512>"][1:4])
    assert abs(rd - 1000.0 * 1024 * 2) < 1e-6 * rd
    assert abs(wr - 3000.0 * 1024) < 1e-6 * wr
    assert abs(tot - (rd + wr)) < 1e-3 * tot


def test_traffic_copy_calibration(tmp_path):
    gib = 1 << 30
    f, w = tmp_path / "fetch.csv", tmp_path / "write.csv"
    _pmc_csv(f, [(COPY, 262144, "FETCH_SIZE", gib / 1024), (COPY, 256, "FETCH_SIZE", 1.0),
                 (ROW_FWD, 1024, "FETCH_SIZE", 10.0)])
    _pmc_csv(w, [(COPY, 262144, "WRITE_SIZE", gib / 1024), (COPY, 256, "WRITE_SIZE", 1.0),
                 (ROW_FWD, 1024, "WRITE_SIZE", 20.0)])
    out = K.traffic(str(f), str(w), gib)
    lines = {l.split()[0]: l.split() for l in out.splitlines() if l.split()}
    assert abs(float(lines["scale_fetch"][1]) - 1.0) < 1e-6
    rd, wr = float(lines["k_row_fwd<512>"][1]), float(lines["k_row_fwd<512>"][2])
    assert abs(rd - 10240.0) < 1e-3 and abs(wr - 20480.0) < 1e-3


def test_traffic_summary_round_trip(tmp_path):
    p = tmp_path / "traffic.txt"
    p.write_text("# header\nscale_fetch 2.0\nsource_digest abc123\n"
                 "kernel read_B/launch write_B/launch traffic_B/launch\n"
                 "k_row_fwd<512> 2.458e+09 8.607e+09 1.107e+10\n")
    assert K.read_traffic(str(p), "k_row_fwd<512>") == (1.107e10, "abc123")
    assert K.read_traffic(str(p), "k_col_pair<512>") == (None, "abc123")
    assert K.read_traffic(str(tmp_path / "missing.txt"), "k_row_fwd<512>") == (None, None)


def test_grids_one_line_per_launch_size(tmp_path):
    p = tmp_path / "trace.csv"
    with open(p, "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Grid_Size_X", "Workgroup_Size_X"])
        w.writerow([ROW_FWD, 0, 3_000_000, 256 * 262144, 256])
        w.writerow([ROW_FWD, 10, 5_000_010, 256 * 262144, 256])
        w.writerow([ROW_FWD, 0, 100_000, 256 * 2048, 256])
        w.writerow(["void at::native::something_else(float)", 0, 10, 64, 64])
    rows = [l.split() for l in K.grids(str(p)).splitlines()[1:]]
    assert rows[0] == ["k_row_fwd<512>", "262144", "2", "4.0000", "8.000"]
    assert rows[1] == ["k_row_fwd<512>", "2048", "1", "0.1000", "0.100"]
    assert len(rows) == 2
