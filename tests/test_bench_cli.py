"""Host checks of bench.py's command-line contract (no GPU needed): it measures
one GPU and refuses more, and the committed counter summary it reads the
headline kernel's HBM traffic from parses."""
import os
import subprocess
import sys

ROOT = os.path.join(os.path.dirname(__file__), "..")


def test_more_than_one_gpu_is_refused():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert p.returncode != 0
    assert "one GPU" in (p.stdout + p.stderr)


def test_traffic_summary_parses():
    sys.path.insert(0, ROOT)
    import bench
    vals = {}
    with open(bench.TRAFFIC_FILE) as f:
        for line in f:
            if "=" in line and not line.lstrip().startswith("#"):
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
    assert int(vals["bytes_per_launch"]) > 0
    assert len(vals["kernel_source_sha"]) == 16
    # the traffic is reported only for the kernel sources it was counted on
    got = bench.measured_traffic()
    if vals["kernel_source_sha"] == bench.kernel_source_sha():
        assert got == int(vals["bytes_per_launch"])
    else:
        assert got is None
