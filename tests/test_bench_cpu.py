"""Host-side parts of bench.py: the one-GPU guard and the rocprofv3 CSV
summaries (no GPU needed)."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True, text=True,
                          timeout=120)


def test_more_than_one_gpu_exits_with_a_message():
    r = _run("--gpus", "2")
    assert r.returncode == 2
    assert "one GPU" in r.stdout


def test_trace_summary_groups_by_kernel_and_grid(tmp_path):
    p = tmp_path / "t.csv"
    p.write_text(
        '"Kind","Kernel_Name","Start_Timestamp","End_Timestamp","Grid_Size_X","Grid_Size_Y","Grid_Size_Z"\n'
        '"K","void mgf::(anonymous namespace)::k_a<double>(int)",1000,3000,64,4,1\n'
        '"K","void mgf::(anonymous namespace)::k_a<double>(int)",4000,8000,64,4,1\n'
        '"K","mgf::(anonymous namespace)::k_b(int)",9000,9500,32,1,1\n')
    r = _run("--trace-summary", str(p))
    assert r.returncode == 0, r.stderr
    lines = r.stdout.splitlines()
    top = lines[1].split()
    assert top[1] == "mgf::k_a<double>" and top[2] == "64x4x1" and top[3] == "2"
    assert abs(float(top[5]) - 3.0) < 1e-9  # average of 2 us and 4 us
    assert any("mgf::k_b" in ln for ln in lines)


def test_counter_summary_averages_per_dispatch(tmp_path):
    p = tmp_path / "c.csv"
    p.write_text(
        '"Dispatch_Id","Grid_Size","Kernel_Name","Counter_Name","Counter_Value"\n'
        '1,93024,"void mgf::(anonymous namespace)::k_s<double>(int)","FETCH_SIZE",10.0\n'
        '2,93024,"void mgf::(anonymous namespace)::k_s<double>(int)","FETCH_SIZE",30.0\n')
    r = _run("--trace-summary", str(p))
    assert r.returncode == 0, r.stderr
    row = r.stdout.splitlines()[1].split()
    assert row[2] == "93024" and row[3] == "FETCH_SIZE" and row[4] == "2" and float(row[5]) == 20.0


def test_trace_summary_reports_the_roofline_loop_tail(tmp_path):
    """The mean of the last dispatches of the one-sweep kernel on its largest
    grid (the roofline loop comes last in the benchmark); the two-sweep kernel
    and smaller grids are not counted."""
    p = tmp_path / "t.csv"
    rows = ['"Kind","Kernel_Name","Start_Timestamp","End_Timestamp","Grid_Size_X","Grid_Size_Y","Grid_Size_Z"']
    t = 0
    for d in (50000, 40000):  # early, slower dispatches of the large grid
        rows.append('"K","void mgf::(anonymous namespace)::k_block_rb_sweep<double, 8>(int)",%d,%d,288,363,1'
                    % (t, t + d))
        t += 100000
    rows.append('"K","void mgf::(anonymous namespace)::k_block_rb_sweep<double, 8>(int)",%d,%d,96,99,1'
                % (t, t + 3000))
    t += 100000
    rows.append('"K","void mgf::(anonymous namespace)::k_block_rb_sweep2<double, 8>(int)",%d,%d,1600,17,1'
                % (t, t + 9000))
    t += 100000
    for d in (7000, 8000, 9000):
        rows.append('"K","void mgf::(anonymous namespace)::k_block_rb_sweep<double, 8>(int)",%d,%d,288,363,1'
                    % (t, t + d))
        t += 100000
    p.write_text("\n".join(rows) + "\n")
    r = subprocess.run([sys.executable, "-c", "import sys; sys.path.insert(0, %r); import bench; "
                        "bench.trace_summary(%r, tail=3)" % (ROOT, str(p))], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 0, r.stderr
    last = r.stdout.splitlines()[-1]
    assert "288x363x1" in last and last.endswith("mean 8.000 us"), last


def test_fig1_rejects_grids_the_chain_cannot_reach():
    r = _run("--fig1", "--fig1-grids", "16,32")
    assert r.returncode != 0 and "powers of two above 16" in (r.stdout + r.stderr)
    r = _run("--fig1", "--fig1-grids", "48")
    assert r.returncode != 0 and "powers of two above 16" in (r.stdout + r.stderr)
