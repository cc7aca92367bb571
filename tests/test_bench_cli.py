"""bench.py's command-line contract that needs no GPU."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=60)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout == ""


def test_sweep_grids_are_the_study_grids():
    sys.path.insert(0, ROOT)
    import bench
    # the parameter study of Sec 5.2: k x w grids of the two data sets, k' = k + r_ov
    assert bench.SWEEPS["P1"]["rs"] == [10, 20, 30, 40, 50] and bench.SWEEPS["P1"]["qs"] == [1, 2, 3, 4, 5]
    assert bench.SWEEPS["P2"]["rs"] == [50, 60, 70, 80, 90] and bench.SWEEPS["P2"]["qs"] == [1, 3, 5, 7, 9, 11]
    assert bench.SWEEPS["P1"]["r_ov"] == 25 - 20 and bench.SWEEPS["P2"]["r_ov"] == 72 - 60


def test_c3_has_a_stored_oracle_error_and_the_bench_can_select_it():
    """The c3 block times to eps = (1 + 1e-3) e_oracle(150 it): the value must be
    stored, and the workload and the opt-out flag must parse."""
    import json
    sys.path.insert(0, ROOT)
    import bench
    import datagen
    golden = json.load(open(bench.GOLDEN))
    assert golden["c3"]["iters"] == datagen.CONFIGS["c3"]["iters"] == 150
    assert 0.0 < golden["c3"]["e"] < 1.0
    old = sys.argv
    try:
        sys.argv = ["bench.py", "--workload", "c3", "--no-c3"]
        a = bench.parse()
    finally:
        sys.argv = old
    assert a.workload == "c3" and a.no_c3
