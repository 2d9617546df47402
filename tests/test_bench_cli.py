"""Host checks of bench.py (no GPU): more than one GPU is
refused with a message before anything touches a device, and the workload
table is consistent with the oracle's cycle options, and the committed
counter tables belong to the kernel sources in the tree."""
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


def test_traffic_tables_match_the_kernel_sources():
    """Every counter table bench.py reads was taken with the kernel sources
    in the tree (its sha256 record matches), so the bench line's `traffic`
    is filled; every entry lies between the algorithmic bytes and 6x them."""
    import json

    sys.path.insert(0, ROOT)
    import bench

    for (workload, cls), path in bench.TRAFFIC_PROFILES.items():
        rec_line = [l for l in open(path) if l.startswith("traffic-json: ")]
        assert rec_line, path
        rec = json.loads(rec_line[-1][len("traffic-json: "):])
        assert rec.get("sources_sha256"), path
        assert rec["tiles"], path
        key = next(iter(rec["tiles"]))
        parts = key.split("|")
        if cls == "smooth_cross_l0":
            tile, folded = tuple(int(x) for x in parts[1:4]), parts[4] == "1"
        else:
            tile, folded = tuple(int(x) for x in parts[1:4]), False
        got = bench.measured_traffic(workload, cls, tile, folded)
        assert got is not None, (
            "%s no longer matches the kernel sources: regenerate it with the commands it lists"
            % os.path.relpath(path, ROOT))
    text = open(os.path.join(ROOT, "profiles", "cross_pass_l0_poisson3d_1023_traffic.md")).read()
    for row in text.splitlines():
        if row.startswith("| cross|"):
            cells = [c.strip() for c in row.strip().strip("|").split("|")]
            traffic, alg = float(cells[-3]), float(cells[-2])  # the key holds '|' too
            assert alg < traffic < 6.0 * alg, row
