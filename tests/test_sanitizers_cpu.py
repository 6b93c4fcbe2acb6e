"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only).

Two drivers under tests/sanitize/ are built here with -fsanitize=address,undefined:
  * the FP64 oracle with every exported function called on each mesh (the
    mass after the steps must equal the unsanitized oracle's);
  * the library's host mesh code (topology, validation, every cell order, tile
    and halo tables at six tile sizes), built for the host only.
Any memory error, leak or undefined behaviour aborts the driver with a report.
A malformed mesh must be rejected cleanly by both.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_1812_00390_amd import meshgen as mg

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = os.path.join(ROOT, "tests", "sanitize")
CSRC = os.path.join(ROOT, "paper_1812_00390_amd", "csrc")
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")


def write_mesh(m, path):
    g = m.groups
    with open(path, "wb") as fp:
        fp.write(np.asarray([m.n_nodes, m.n_cells, m.cell_nodes.size, m.bface_nodes.shape[0], len(g),
                             m.periodic.shape[0]], np.int32).tobytes())
        fp.write(np.ascontiguousarray(m.nodes, np.float64).tobytes())
        fp.write(np.ascontiguousarray(m.cell_ptr, np.int32).tobytes())
        fp.write(np.ascontiguousarray(m.cell_nodes, np.int32).tobytes())
        fp.write(np.ascontiguousarray(m.bface_nodes, np.int32).reshape(-1).tobytes())
        fp.write(np.ascontiguousarray(m.bface_group, np.int32).tobytes())
        fp.write(np.asarray([x.kind for x in g], np.int32).tobytes())
        fp.write(np.asarray([x.internal for x in g], np.int32).tobytes())
        fp.write(np.asarray([c for x in g for c in x.u], np.float64).tobytes())
        fp.write(np.asarray([x.rho for x in g], np.float64).tobytes())
        fp.write(np.ascontiguousarray(m.periodic, np.int32).reshape(-1).tobytes())
        fp.write(np.ascontiguousarray(m.periodic_shift, np.float64).reshape(-1).tobytes())


def _wall_group(m):
    for k, g in enumerate(m.groups):
        if g.kind == 0:
            return k
    return -1


def _inverted(m):
    """The first cell with its corner order reversed (negative area)."""
    cn = m.cell_nodes.copy()
    a, b = m.cell_ptr[0], m.cell_ptr[1]
    cn[a:b] = cn[a:b][::-1]
    return mg.RawMesh(m.nodes, m.cell_ptr, cn, m.bface_nodes, m.bface_group, m.groups, m.periodic,
                      m.periodic_shift, name="inverted")


MESHES = {
    "cavity_tri": lambda: mg.cavity(n=14, jitter=0.2, seed=5),
    "channel_inlet_outlet_symmetry": lambda: mg.channel(16, 8, jitter=0.2, seed=6, tri=True, top="symmetry"),
    "channel_internal": lambda: mg.channel(12, 6, jitter=0.2, seed=7, tri=True, internal=1),
    "periodic_box": lambda: mg.periodic_box(9, 7, jitter=0.25, seed=8),
    "cylinder_quads": lambda: mg.cylinder(nr=12, nt=18, R=6.0, h0=0.05),
    "two_cylinders": lambda: mg.two_cylinders(nr=6, nt=16, half_width=8.0, height=8.0, h0=0.05),
    "hybrid": lambda: mg.hybrid(10),
    "couette": lambda: mg.couette(8, 8),
}


@pytest.fixture(scope="module")
def drivers(tmp_path_factory):
    d = tmp_path_factory.mktemp("san")
    out = {}
    if shutil.which("gcc"):
        exe = str(d / "oracle_driver")
        subprocess.check_call(["gcc", "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fno-omit-frame-pointer",
                               "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
                               "-o", exe, os.path.join(ROOT, "oracle", "fvlbm_oracle.c"),
                               os.path.join(SAN, "oracle_driver.c"), "-lm"])
        out["oracle"] = exe
    if shutil.which("hipcc"):
        exe = str(d / "mesh_driver")
        # host code only (-x c++): the sanitizer flags go to the host compiler
        subprocess.check_call(["hipcc", "-x", "c++", "-O1", "-g", "-std=c++17", "-fno-omit-frame-pointer",
                               "-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
                               "-Xarch_host", "-fno-sanitize-recover=all",
                               "-D__HIP_PLATFORM_AMD__", "-I", os.path.join(os.environ.get("ROCM_PATH", "/opt/rocm"), "include"),
                               "-I", os.path.join(ROOT, "include"), "-I", CSRC,
                               os.path.join(CSRC, "topology.cpp"), os.path.join(CSRC, "tiles.cpp"),
                               os.path.join(SAN, "mesh_driver.cpp"), "-o", exe])
        out["mesh"] = exe
    out["dir"] = d
    return out


def _clean(r):
    text = r.stdout + r.stderr
    assert "Sanitizer" not in text and "runtime error" not in text, text[-3000:]


@pytest.mark.parametrize("scheme", [0, 1, 2])
@pytest.mark.parametrize("name", list(MESHES))
def test_oracle_under_sanitizers(drivers, name, scheme):
    if "oracle" not in drivers:
        pytest.skip("no gcc")
    from oracle import oracle as O
    m = MESHES[name]()
    path = str(drivers["dir"] / f"{name}.mesh")
    write_mesh(m, path)
    tau, steps = 0.01, 12
    r = subprocess.run([drivers["oracle"], path, str(tau), str(scheme), str(steps), str(_wall_group(m))],
                       capture_output=True, text=True, env=ENV, timeout=120)
    _clean(r)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    mass = float(r.stdout.split("mass ")[1].split()[0])
    o = O.Oracle(m, tau=tau, cfl=0.5, u_ref=0.2, scheme=["euler", "rk4", "ab2"][scheme])
    o.init(rho0=1.0, u0=(0.0, 0.0))
    o.step(steps)
    assert mass == pytest.approx(o.mass(), rel=1e-13, abs=0.0)


@pytest.mark.parametrize("name", list(MESHES))
def test_mesh_code_under_sanitizers(drivers, name):
    if "mesh" not in drivers:
        pytest.skip("no hipcc")
    m = MESHES[name]()
    path = str(drivers["dir"] / f"m_{name}.mesh")
    write_mesh(m, path)
    r = subprocess.run([drivers["mesh"], path], capture_output=True, text=True, env=ENV, timeout=300)
    _clean(r)
    assert r.returncode == 0, r.stdout + r.stderr[-2000:]
    assert r.stdout.count("halo slots") == 4


def test_malformed_mesh_rejected_cleanly(drivers):
    m = _inverted(mg.cavity(n=6, jitter=0.0, seed=0))
    path = str(drivers["dir"] / "inverted.mesh")
    write_mesh(m, path)
    for key in ("oracle", "mesh"):
        if key not in drivers:
            continue
        args = [drivers[key], path] + (["0.01", "0", "1", "-1"] if key == "oracle" else [])
        r = subprocess.run(args, capture_output=True, text=True, env=ENV, timeout=120)
        _clean(r)
        assert r.returncode == 3, (key, r.stdout, r.stderr[-2000:])
