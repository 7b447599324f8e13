"""Host logic of the benchmark script, without a GPU: the algorithmic byte
model behind the roofline figures, and the refusal of multi-GPU runs."""
import importlib.util
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _bench():
    spec = importlib.util.spec_from_file_location("bench_host", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_byte_model_128_elastic():
    bench = _bench()
    b, shared, u = bench.algorithmic_bytes(128)
    # one FP64 nodal field of 3 components; a half spectrum of 65 x 128 x 128
    # complex FP64 values per component; K^+ keeps 6 symmetric FP64 entries
    # per frequency; one phase byte per voxel
    assert u == dict(V=50_331_648, Sb=51_118_080, Kb=51_118_080, Pb=2_097_152)
    assert b["operator"] == 2 * 50_331_648       # read p, write q
    assert b["xfwd"] == 3 * 50_331_648 + 51_118_080
    assert b["yfwd"] == b["yinv"] == b["zsolve"] == 102_236_160
    assert b["xinv"] == 51_118_080 + 4 * 50_331_648
    # shared by the load cases of a launch: phases (operator), K^+ (z pass)
    assert shared == {"operator": 2_097_152, "zsolve": 51_118_080}
    # one load case per launch: about 18.2 nodal fields per iteration
    total = sum(b.values()) + sum(shared.values())
    assert total == 915_144_704
    assert abs(total / u["V"] - 18.18) < 0.01
    # six load cases per launch: K^+ and phases are read once
    assert bench.launch_bytes(b, shared, "zsolve", 6) == 6 * 102_236_160 + 51_118_080
    assert bench.launch_bytes(b, shared, "xinv", 6) == 6 * b["xinv"]
    assert bench.FLOOR_V * u["V"] == 654_311_424


def test_byte_model_scalar_256():
    b, shared, u = _bench().algorithmic_bytes(256, nd=1)
    assert u["V"] == 8 * 256 ** 3
    assert u["Sb"] == 16 * 129 * 256 * 256
    assert u["Kb"] == 8 * 129 * 256 * 256          # one entry per frequency
    assert b["zsolve"] == 2 * u["Sb"] and shared["zsolve"] == u["Kb"]


def test_multi_gpu_request_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=60)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""
