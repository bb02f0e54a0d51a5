"""bench.py's contract on the host: more than one GPU is refused with a JSON
message and exit status 2 before anything touches a GPU, and the counter
traffic it reports comes from the committed summary only for the launch
options the counters were taken with."""
import importlib.util
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench_module():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120, cwd=ROOT)
    assert r.returncode == 2
    line = json.loads(r.stdout.strip().splitlines()[-1])
    assert line["n_gpus"] == 2 and "one GPU" in line["error"]


def test_traffic_only_for_the_profiled_options():
    b = _bench_module()
    default = dict(max_batch=4194304, band_width=24, lane_load=32, sort_electrons=0, pipelines=2,
                   density_effect=0)
    got = b.measured_traffic("k_electron", default)
    assert got is None or got > 0
    for change in (dict(band_width=3), dict(sort_electrons=1), dict(lane_load=16)):
        assert b.measured_traffic("k_electron", dict(default, **change)) is None
    assert b.measured_traffic("k_no_such_kernel", default) is None
