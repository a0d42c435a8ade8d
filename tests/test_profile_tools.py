"""The profile summary tools on small synthetic rocprofv3 CSV files, and the
bench's lookup of recorded traffic (CPU)."""
import csv
import json

from paper_2606_08883_amd import profile_summary as PS
from paper_2606_08883_amd import trace_levels as TL


def _write(path, header, rows):
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_trace_levels_groups_interface_launches(tmp_path, capsys):
    hdr = ["Kernel_Name", "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Grid_Size_X"]
    rows, t = [], 0
    for _ in range(3):   # three applications: local, rhs, 2 fwd, 1 bwd, reconstruct
        for name, us, wgs in (("void mrcm::(anonymous namespace)::k_local<double>(int)", 50, 10),
                              ("mrcm::(anonymous namespace)::k_coarse_rhs(int)", 4, 2),
                              ("mrcm::(anonymous namespace)::k_coarse_fwd(int)", 10, 8),
                              ("mrcm::(anonymous namespace)::k_coarse_fwd(int)", 8, 4),
                              ("mrcm::(anonymous namespace)::k_coarse_bwd(int)", 6, 4),
                              ("void mrcm::(anonymous namespace)::k_reconstruct<double>(int)", 12, 10)):
            rows.append([name, t, t + us * 1000, 256, wgs * 256])
            t += us * 1000 + 500
    _write(tmp_path / "run_kernel_trace.csv", hdr, rows[::-1])   # out of order on purpose
    sv = TL.solves(str(tmp_path))
    assert len(sv) == 3 and [x[0] for x in sv[0]] == ["k_coarse_rhs", "k_coarse_fwd",
                                                       "k_coarse_fwd", "k_coarse_bwd"]
    assert sv[0][1][1:] == (8, 256, 10.0)
    assert TL.main(["trace_levels", str(tmp_path), "2"]) == 0
    out = capsys.readouterr().out
    assert "solve total (sum of launch means): 28.0 us" in out


def test_profile_summary_traffic_scales_by_the_copy(tmp_path, capsys):
    hdr = ["Kernel_Name", "Counter_Value"]
    for d in ("cf", "cw", "lf", "lw"):
        (tmp_path / d).mkdir()
    # the 1 GiB copy reads FETCH 524288 KiB (factor 2) and WRITE 1048576 KiB (factor 1)
    _write(tmp_path / "cf" / "run_counter_collection.csv", hdr,
           [["__amd_rocclr_copyBuffer", 524288.0]] * 2)
    _write(tmp_path / "cw" / "run_counter_collection.csv", hdr,
           [["__amd_rocclr_copyBuffer", 1048576.0]] * 2)
    _write(tmp_path / "lf" / "run_counter_collection.csv", hdr,
           [["void mrcm::(anonymous namespace)::k_patch<float, float, 36, 64>(int)", 1000.0]] * 2)
    _write(tmp_path / "lw" / "run_counter_collection.csv", hdr,
           [["void mrcm::(anonymous namespace)::k_patch<float, float, 36, 64>(int)", 100.0]] * 2)
    bj = tmp_path / "bench.json"
    bj.write_text("log line\n" + json.dumps({"phases": {"patch": {"algorithmic_bytes": 1050000}}})
                  + "\n")
    PS.traffic("k_patch", "w", "1", str(tmp_path / "lf"), str(tmp_path / "lw"),
               str(tmp_path / "cf"), str(tmp_path / "cw"), str(bj))
    out = capsys.readouterr().out
    expect = int((1000.0 * 2 + 100.0) * 1024)   # KiB scaled by the copy factors, in bytes
    assert f"traffic_bytes_per_launch: {expect}" in out
    ratio = [ln for ln in out.splitlines() if ln.strip().startswith("k_patch ") and "/" in ln]
    assert len(ratio) == 1 and ratio[0].rstrip().endswith(f"= {expect / 1050000:.2f}")
    assert f"source_sha256_16: {PS.kernel_source_hash()}" in out


def test_profile_summary_stats_table(tmp_path, capsys):
    hdr = ["Name", "Calls", "AverageNs", "TotalDurationNs", "Percentage"]
    _write(tmp_path / "run_kernel_stats.csv", hdr,
           [["void mrcm::(anonymous namespace)::k_patch<float>(int)", 18, 500000, 9000000, 60.0],
            ["void mrcm::(anonymous namespace)::k_factor_boxes<float>(int)", 1, 6000000, 6000000,
             40.0]])
    PS.stats(str(tmp_path), 9)
    out = capsys.readouterr().out.splitlines()
    assert out[1].startswith("k_patch<float>") and out[1].split()[-1] == "1000.00"
    assert out[2].startswith("k_factor_boxes<float>") and out[2].split()[-1] == "-"


def test_trace_levels_usage_and_missing_trace(tmp_path, capsys):
    assert TL.main(["trace_levels", "--help"]) == 0
    assert "Usage" in capsys.readouterr().out
    assert TL.main(["trace_levels"]) == 2
    assert TL.main(["trace_levels", str(tmp_path), "x"]) == 2
    capsys.readouterr()
    assert TL.main(["trace_levels", str(tmp_path)]) == 1
    assert "no kernel_trace.csv" in capsys.readouterr().err


def test_bench_reads_recorded_traffic_only_for_current_sources(tmp_path, monkeypatch):
    import bench
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))

    def write(source, precision=1):
        (prof / "k_patch_large4096_traffic.txt").write_text(
            "summary text\n  indented: ignored\nkernel: k_patch\nworkload: large4096\n"
            f"precision: {precision}\nsource_sha256_16: {source}\n"
            "traffic_bytes_per_launch: 123456\n")

    assert bench.recorded_traffic("k_patch", "large4096", 1) is None  # no summary
    write(PS.kernel_source_hash())
    assert bench.recorded_traffic("k_patch", "large4096", 1) == 123456
    assert bench.recorded_traffic("k_patch", "large4096", 2) is None  # other precision
    assert bench.recorded_traffic("k_local", "large4096", 1) is None  # other kernel
    write("0" * 16)
    assert bench.recorded_traffic("k_patch", "large4096", 1) is None  # stale sources
