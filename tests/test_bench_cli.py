"""Host checks of bench.py's command line (no GPU): more than one GPU is
refused with a message before anything touches a device, and the workload
table is consistent with the oracle's cycle options."""
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_workloads_name_known_cycles():
    sys.path.insert(0, ROOT)
    import bench

    assert bench.DEFAULT in bench.WORKLOADS
    d = bench.WORKLOADS[bench.DEFAULT]
    assert (d["dim"], d["L"], d["prec"], d.get("nu")) == (3, 10, "fp64", 1)  # 1023^3 FP64 V(1,1)
    for name, spec in bench.WORKLOADS.items():
        # dim 0: the batch of problems of several sizes
        assert spec["dim"] in ((0,) if spec["rhs"] == "batch" else (2, 3)), name
        assert spec.get("smoother", "rbgs") in ("rbgs", "wj", "mcgs"), name
        assert spec["prec"] in ("fp64", "mixed"), name
