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
