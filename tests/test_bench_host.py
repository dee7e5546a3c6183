"""Host-side logic of bench.py (no GPU): the one-GPU guard, the HBM traffic
figures read from the committed counter summary, and the serving cost model."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


@pytest.mark.parametrize("argv,env", [(["--gpus", "2"], {}), (["--gpus", "8"], {}),
                                      ([], {"WORLD_SIZE": "2"})])
def test_more_than_one_gpu_is_refused(argv, env):
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *argv], cwd=ROOT,
                       env={**os.environ, **env}, capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr and r.stdout == ""


def test_traffic_read_while_sources_match():
    for k in ("k_rform_f32 tile=32x4", "k_rform_f64 tile=32x4"):
        t = bench.measured_traffic(k)
        assert t is not None and t > 0
    assert bench.measured_traffic("k_rform_f32 tile=64x2") is None  # no such line


def test_traffic_dropped_once_sources_change(tmp_path, monkeypatch):
    changed = []
    for f in bench.RFORM_SOURCES:
        c = tmp_path / os.path.basename(f)
        c.write_bytes(open(f, "rb").read())
        changed.append(str(c))
    monkeypatch.setattr(bench, "RFORM_SOURCES", changed)
    assert bench.measured_traffic("k_rform_f32 tile=32x4") is not None  # same bytes, same hash
    with open(changed[0], "ab") as fh:
        fh.write(b"\n")
    assert bench.measured_traffic("k_rform_f32 tile=32x4") is None


def test_request_cost_counts_contraction_and_lu():
    class PW:
        nchan, npole = 3, 7
    # per energy: the symmetric half of the contraction, n (n + 1) M, and the LU, (2/3) n^3
    assert bench.request_cost(PW, 5) == pytest.approx(5 * (3 * 4 * 7 + 2.0 / 3.0 * 27))
    assert bench.request_cost(PW, 0) == 0.0
