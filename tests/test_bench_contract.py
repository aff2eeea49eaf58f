"""bench.py contract checks that need no GPU: more than one GPU is refused
with a message, and the roofline's measured traffic is tied to the kernel
source it was taken on."""
import json
import os
import subprocess
import sys

from conftest import ROOT


def test_more_than_one_gpu_is_refused():
    res = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                         capture_output=True, text=True, timeout=120)
    assert res.returncode == 2
    assert "one GPU" in res.stderr
    assert res.stdout.strip() == ""


def test_committed_traffic_is_tied_to_the_kernel_source():
    # The bench reports the counter traffic only while the headline kernel's
    # sources are the ones the counters were taken on, and null after a change.
    sys.path.insert(0, ROOT)
    import bench
    rec = json.load(open(bench.TRAFFIC_FILE))
    if rec["kernel_source_sha256_16"] == bench.kernel_source_hash():
        assert bench.measured_traffic() == rec["bytes_per_launch"]
    else:
        assert bench.measured_traffic() is None
    # the counters saw the algorithmic bytes (no re-reads) within 1 %
    assert abs(rec["bytes_per_launch"] / rec["algorithmic_bytes_per_launch"] - 1) < 0.01
