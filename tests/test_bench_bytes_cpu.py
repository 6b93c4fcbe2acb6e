"""The algorithmic bytes per cell-update that the benchmark's roofline divides by,
and the gating of its measured-traffic field.

They count the state a step must read and write plus one read of a compact mesh
description per RHS evaluation (60 B per triangle: three neighbour indices, 1/A,
the centroid, the three entries of the least-squares matrix inverse, and half
of each face's normal-times-length and midpoint; 72 B per quadrilateral).  The
state part is 18 values per Euler step (read f, write f) and 99 per four-stage
RK step (the first stage reads f and writes a stage, the other three also read
the step's base f): 18 + 3 x 27.
"""
import hashlib
import importlib.util
import json
import os

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_module", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_mesh_bytes_from_their_parts(bench):
    f32, i32 = 4, 4
    tri = 3 * i32 + (1 + 2 + 3) * f32 + 0.5 * 3 * (2 + 2) * f32
    quad = 4 * i32 + (1 + 2 + 3) * f32 + 0.5 * 4 * (2 + 2) * f32
    assert bench.MESH_BYTES == {3: tri, 4: quad} == {3: 60, 4: 72}


def test_state_values_per_step(bench):
    assert bench.STATE_VALUES["euler"] == 9 + 9
    assert bench.STATE_VALUES["rk4"] == 18 + 3 * 27


@pytest.mark.parametrize("nf,scheme,storage,expected", [
    (3, "euler", "fp32dev", 132), (4, "euler", "fp32dev", 144),
    (3, "rk4", "fp32dev", 636), (4, "rk4", "fp32dev", 684),
    (3, "rk4", "fp32", 636),
    # FP16 deviations: 2 B per value plus the three FP16 moment-carry values,
    # read and rewritten once per step
    (3, "euler", "fp16dev", 36 + 60 + 12), (3, "rk4", "fp16dev", 198 + 240 + 12),
    # 16-bit block-scaled: nine int16 values and one exponent byte per cell
    (3, "rk4", "i16dev", 11 * 19 + 240),
])
def test_alg_bytes_per_update(bench, nf, scheme, storage, expected):
    assert bench.alg_bytes_per_update(nf, scheme, storage) == pytest.approx(expected, rel=1e-12)


def test_state_only_bytes(bench):
    assert bench.state_bytes_per_update("euler", "fp32dev") == 72
    assert bench.state_bytes_per_update("rk4", "fp32dev") == 396
    assert bench.state_bytes_per_update("rk4", "fp16dev") == 198 + 12


def test_traffic_is_reported_only_for_profiled_sources_and_schedules(bench, tmp_path, monkeypatch):
    """`roofline.traffic` comes from committed counter runs; a record whose sources
    no longer hash to the profiled ones, or a schedule it does not hold, gives None."""
    src = tmp_path / "kernel.hip"
    src.write_text("// a kernel\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()
    prof = tmp_path / "profiles"
    prof.mkdir()
    rec = {"sources": ["kernel.hip"], "source_sha256": sha,
           "per_schedule": {"hilbert:128,1,2": {"bytes_per_launch": 123},
                            "rk4_fp32dev:256,1,0": {"bytes_per_launch": 456}}}
    (prof / "k_tile_traffic_w.json").write_text(json.dumps(rec))
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    sched = {"block": 128, "xcd_remap": True, "persistent": 2}
    assert bench.measured_traffic("w", sched, "hilbert") == 123
    assert bench.measured_traffic("w", {"block": 256, "xcd_remap": True, "persistent": 0}, "rk4_fp32dev") == 456
    assert bench.measured_traffic("w", dict(sched, xcd_remap=False), "hilbert") is None      # not profiled
    assert bench.measured_traffic("absent", sched, "hilbert") is None
    src.write_text("// a changed kernel\n")
    assert bench.measured_traffic("w", sched, "hilbert") is None                              # stale record


def test_bench_refuses_more_than_one_gpu():
    """The benchmark runs on one GPU; asked for more it says so and exits non-zero
    before touching a device."""
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode != 0
    assert "one GPU" in (r.stdout + r.stderr)
