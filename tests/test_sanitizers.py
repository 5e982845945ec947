"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU).

The library's host sources (api.cpp, bvh.cpp, and the host side of the
kernel translation units) and the oracle are built with -fsanitize=address
and -fsanitize=undefined on the host code only (device code is built as in
the library), linked into tests/sanitize/sanitize_driver.cpp, and run over
scenes written here: the host BVH build at several leaf sizes and split
budgets on the small TPC, the DARWIN-scale mesh and the 4-pi SiPM variant;
the oracle's transport (brute force and BVH, scintillation times, spectrum,
gradient tallies) in its FP64 and FP32 builds; and the argument and state
checks of the C ABI that need no device.  Any sanitizer report fails the
test (UBSan is built without recovery, ASan aborts on its first error).
The large meshes run the default build options and the brute-force oracle
runs on the small TPC only, to keep the instrumented runs to about a minute.
"""
import os
import subprocess

import numpy as np
import pytest

from paper_2203_14354_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2203_14354_amd", "csrc")
OUT = os.path.join(ROOT, "_build", "sanitize")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=all", "-Xarch_host", "-fno-omit-frame-pointer"]
DEV = ["-x", "hip", "--offload-arch=gfx950", "-munsafe-fp-atomics", "-ffp-contract=on",
       "-fno-hip-fp32-correctly-rounded-divide-sqrt", "-fgpu-flush-denormals-to-zero",
       "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops"]
ENV = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
           UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")


def _run(cmd, **kw):
    r = subprocess.run(cmd, capture_output=True, text=True, **kw)
    assert r.returncode == 0, f"{' '.join(cmd[:3])} ...\n{r.stdout[-3000:]}\n{r.stderr[-6000:]}"
    return r


@pytest.fixture(scope="module")
def drivers():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    os.makedirs(OUT, exist_ok=True)
    inc = ["-I", os.path.join(ROOT, "include"), "-I", CSRC]
    objs = []
    for src in ("api.cpp", "bvh.cpp", "propagate.hip", "propagate_tally.hip"):
        o = os.path.join(OUT, src + ".o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-fPIC", *inc, *DEV, *SAN, "-c",
              os.path.join(CSRC, src), "-o", o])
        objs.append(o)
    do = os.path.join(OUT, "driver.o")
    _run([HIPCC, "-O1", "-g", "-std=c++17", "-x", "c++", *inc, *SAN, "-c",
          os.path.join(ROOT, "tests", "sanitize", "sanitize_driver.cpp"), "-o", do])
    out = {}
    for name, defs in (("fp64", []), ("fp32", ["-DXEORACLE_FP32"])):
        oo = os.path.join(OUT, f"oracle_{name}.o")
        _run([HIPCC, "-O1", "-g", "-std=c++17", "-x", "c++", *defs, *SAN, "-c",
              os.path.join(ROOT, "oracle", "xeoracle.cpp"), "-o", oo])
        exe = os.path.join(OUT, f"sanitize_driver_{name}")
        _run([HIPCC, "-fsanitize=address", "-fsanitize=undefined", "-fno-gpu-sanitize",
              "--offload-arch=gfx950", do, oo, *objs, "-o", exe])
        out[name] = exe
    return out


def _write_scene(path, mesh, cyl):
    from paper_2203_14354_amd.workloads import materials_array, surfaces_array
    sp, stags, sopt = surfaces_array(mesh.surfaces)
    mats = materials_array(mesh.materials)
    ch = np.arange(mesh.n_sensors, dtype=np.int32)
    hdr = np.array([len(mesh.vertices), len(mesh.triangles), len(mats), len(sp), mesh.n_sensors,
                    max(mesh.n_sensors, 1)], dtype=np.int64)
    with open(path, "wb") as f:
        for a, dt in ((hdr, np.int64), (mesh.vertices, np.float32), (mesh.triangles, np.int32),
                      (mesh.mat_inner, np.int32), (mesh.mat_outer, np.int32),
                      (mesh.surface, np.int32), (mesh.sensor, np.int32), (mats, np.float32),
                      (sp, np.float32), (stags, np.int32), (sopt, np.float32), (ch, np.int32),
                      (np.asarray(cyl, np.float32), np.float32)):
            f.write(np.ascontiguousarray(a, dtype=dt).tobytes())


DARWIN_CYL = (W.DARWIN_SRC_R, W.DARWIN_SRC_ZLO, W.DARWIN_SRC_ZHI)
# mesh, source cylinder, BVH options (leaf size:split budget), oracle photons and modes
SCENES = {
    "tpc1": (lambda: W.tpc1(plane=True), (W.TPC1_SRC_R, -W.TPC1_SRC_ZHALF, W.TPC1_SRC_ZHALF),
             ["1:0", "1:1", "4:4", "8:-1"], 20_000, ["brute", "bvh"]),
    "darwin": (lambda: W.darwin(), DARWIN_CYL, ["1:0", "8:-1"], 2_000, ["bvh"]),
    "sipm": (lambda: W.darwin(side_array="sipm"), DARWIN_CYL, ["1:0"], 0, []),
}


@pytest.mark.parametrize("scene", list(SCENES))
def test_host_bvh_build_under_sanitizers(drivers, scene, tmp_path):
    make, cyl, specs, _, _ = SCENES[scene]
    path = str(tmp_path / f"{scene}.bin")
    _write_scene(path, make(), cyl)
    r = _run([drivers["fp64"], "bvh", path, *specs], env=ENV, timeout=900)
    assert r.stdout.count("bvh leaf") == len(specs)


@pytest.mark.parametrize("build", ["fp64", "fp32"])
@pytest.mark.parametrize("scene", ["tpc1", "darwin"])
def test_oracle_under_sanitizers(drivers, scene, build, tmp_path):
    make, cyl, _, n, modes = SCENES[scene]
    path = str(tmp_path / f"{scene}.bin")
    _write_scene(path, make(), cyl)
    r = _run([drivers[build], "oracle", path, str(n), *modes], env=ENV, timeout=900)
    assert r.stdout.count("oracle ") == len(modes)


def test_api_checks_under_sanitizers(drivers):
    r = _run([drivers["fp64"], "api"], env=ENV, timeout=300)
    assert "api checks passed" in r.stdout
