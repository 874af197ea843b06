"""Host-side checks of bench.py that need no GPU: it refuses more than one
GPU with a message, and the hash that ties the committed HBM counter data to
the kernel sources ignores comments and layout but not code."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, cwd=ROOT, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in (r.stdout + r.stderr)


def test_sources_hash_ignores_comments_but_not_code():
    import bench
    a = "int f(int x) {  // twice\n  return 2 * x; /* doubled */\n}\n"
    b = "int f(int x)\n{\n    return 2*x;\n}"
    c = "int f(int x) { return 3 * x; }"
    assert bench.code_only(a) == bench.code_only(b)
    assert bench.code_only(a) != bench.code_only(c)
    h = bench.sources_hash()
    assert len(h) == 16 and h == bench.sources_hash()


def _write_trace(path, launches, counters=False):
    """A rocprofv3-style CSV of the given (kernel name, grid, duration) launches,
    with fill and transpose launches in between as a real sweep has."""
    import csv
    with open(path, "w", newline="") as f:
        if counters:
            w = csv.writer(f)
            w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
            for i, (name, grid, dur) in enumerate(launches):
                w.writerow([i + 1, grid, name, "TCC_HIT_sum", dur])
                w.writerow([i + 1, grid, name, "TCC_MISS_sum", 1])
        else:
            w = csv.writer(f)
            w.writerow(["Dispatch_Id", "Kernel_Name", "Grid_Size_X", "Start_Timestamp",
                        "End_Timestamp"])
            for i, (name, grid, dur) in enumerate(launches):
                w.writerow([i + 1, name, grid, 1000 * i, 1000 * i + dur])


def _sweep_launches(bench, sizes, ns, steps, dur):
    out = []
    names = {"soa": "void soax::soa_step_kernel<0, float, float, 1, false, false>(soax::SoaStepArgs)",
             "aos": "void soax::aos_step_kernel<0, float, float, true, false, false>(soax::AosStepArgs)",
             "aos_naive": "void soax::aos_naive_kernel<0, float, float, true>(soax::AosStepArgs)"}
    for size in sizes:
        for n in ns:
            out.append(("void soax::fill_kernel(soax::FillArgs)", n, 7))
            out.append(("void soax::soa_to_aos_kernel(soax::XposeArgs)", n, 7))
            for lay in bench.SWEEP_LAYOUTS:
                for k in range(bench.SWEEP_WARM + bench.sweep_steps(n, steps)):
                    # warm-up launches are slow; timed ones take dur(size, n, lay)
                    out.append((names[lay], n, 10 ** 6 if k < bench.SWEEP_WARM else
                                dur(size, n, lay)))
    return out


def test_sweep_report_reads_kernel_times_back_in_sweep_order(tmp_path):
    import bench
    sizes, ns, steps = (0, 32), (1000, 10000), 7
    lay_ns = {"soa": 2000, "aos": 3000, "aos_naive": 5000}
    dur = lambda size, n, lay: lay_ns[lay] + size + n // 1000  # noqa: E731
    _write_trace(str(tmp_path / "x_kernel_trace.csv"), _sweep_launches(bench, sizes, ns, steps, dur))
    rows = bench.sweep_report_rows([str(tmp_path)], sizes, ns, steps)
    assert [(r["SIZE"], r["N"]) for r in rows] == [(0, 1000), (0, 10000), (32, 1000), (32, 10000)]
    for r in rows:
        for lay in bench.SWEEP_LAYOUTS:
            assert r[lay]["kernel_ns"] == dur(r["SIZE"], r["N"], lay)
        assert abs(r["aos_over_soa"] - dur(r["SIZE"], r["N"], "aos") /
                   dur(r["SIZE"], r["N"], "soa")) < 1e-12


def test_sweep_report_counters_and_mismatch(tmp_path):
    import pytest

    import bench
    sizes, ns, steps = (0,), (1000,), 3
    dur = lambda size, n, lay: {"soa": 4, "aos": 6, "aos_naive": 8}[lay]  # noqa: E731
    launches = _sweep_launches(bench, sizes, ns, steps, dur)
    _write_trace(str(tmp_path / "c_counter_collection.csv"), launches, counters=True)
    rows = bench.sweep_report_rows([str(tmp_path)], sizes, ns, steps)
    assert rows[0]["aos"]["counters_per_launch"] == {"TCC_HIT_sum": 6.0, "TCC_MISS_sum": 1.0}
    # one launch missing: the report refuses to guess
    _write_trace(str(tmp_path / "c_counter_collection.csv"), launches[:-1], counters=True)
    with pytest.raises(SystemExit):
        bench.sweep_report_rows([str(tmp_path)], sizes, ns, steps)


def test_sweep_markdown_merges_time_and_counters(tmp_path):
    import bench
    sizes, ns, steps = (0,), (1000,), 3
    dur = lambda size, n, lay: {"soa": 4000, "aos": 6000, "aos_naive": 8000}[lay]  # noqa: E731
    launches = _sweep_launches(bench, sizes, ns, steps, dur)
    (tmp_path / "t").mkdir()
    (tmp_path / "c").mkdir()
    _write_trace(str(tmp_path / "t" / "x_kernel_trace.csv"), launches)
    _write_trace(str(tmp_path / "c" / "x_counter_collection.csv"), launches, counters=True)
    rows = bench.sweep_report_rows([str(tmp_path / "t"), str(tmp_path / "c")], sizes, ns, steps)
    assert rows[0]["soa"]["kernel_ns"] == 4000
    # TCC_HIT = the duration column of the fake counter file, TCC_MISS = 1
    assert rows[0]["soa"]["counters_per_launch"]["TCC_HIT_sum"] == 4000
    md = bench.sweep_markdown(rows)
    assert "| 0 | 1e+03 | 4.00 | 6.00 | 8.00 | 4.0000 | 1.50 | 2.00 |" in md
    assert "1.00/1.00/1.00" in md


def test_sweep_markdown_traffic_columns(tmp_path):
    import csv

    import bench
    sizes, ns, steps = (0,), (1000,), 2
    launches = _sweep_launches(bench, sizes, ns, steps, lambda size, n, lay: 1)
    with open(tmp_path / "x_counter_collection.csv", "w", newline="") as f:
        w = csv.writer(f)
        w.writerow(["Dispatch_Id", "Grid_Size", "Kernel_Name", "Counter_Name", "Counter_Value"])
        for i, (name, grid, _) in enumerate(launches):
            w.writerow([i + 1, grid, name, "WRITE_SIZE", 12.0])  # KiB per dispatch
    rows = bench.sweep_report_rows([str(tmp_path)], sizes, ns, steps)
    md = bench.sweep_markdown(rows)
    assert "read+write B/particle" in md
    # 12 KiB over 1000 particles with the committed write calibration
    import json
    cal = json.load(open(bench.PROFILE_TRAFFIC))["calibration"]["write_factor"]
    assert f"0.0+{12 * 1024 * cal / 1000:.1f}" in md
