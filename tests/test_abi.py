"""The C ABI library loads and exports every symbol include/xephot.h declares;
host-side argument validation works without a GPU."""
import ctypes
import os
import re
import subprocess

import numpy as np

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "xephot.h")


@pytest.fixture(scope="module")
def lib():
    from paper_2203_14354_amd import _lib
    if not os.path.exists(_lib.LIB_PATH):
        from paper_2203_14354_amd import build
        build.build()
    return _lib.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^\s*(?:const\s+)?[a-z_0-9]+\**\s+\**(xp_[a-z_0-9]+)\s*\(",
                                 text, flags=re.M)))


def test_header_functions_are_exported(lib):
    from paper_2203_14354_amd import _lib
    names = declared_functions()
    assert len(names) >= 15
    assert sorted(_lib.EXPORTS) == names
    out = subprocess.run(["nm", "-D", "--defined-only", _lib.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    exported = set(l.split()[-1] for l in out.splitlines() if " T " in l)
    for n in names:
        assert n in exported, n
        assert hasattr(lib, n)


def test_struct_layouts_match_header():
    from paper_2203_14354_amd import _lib
    assert ctypes.sizeof(_lib.Material) == 12
    assert ctypes.sizeof(_lib.Surface) == 48
    assert ctypes.sizeof(_lib.Sources) == 112
    assert ctypes.sizeof(_lib.ExtraTallies) == 24
    assert ctypes.sizeof(_lib.RunParams) == 32
    assert ctypes.sizeof(_lib.LaunchCfg) == 28
    assert ctypes.sizeof(_lib.BvhOptions) == 12
    assert ctypes.sizeof(_lib.BvhInfo) == 56
    assert _lib.RECORD_DTYPE.itemsize == 96


_C_STRUCTS = {"Material": "xp_material", "Surface": "xp_surface", "BvhOptions": "xp_bvh_options",
              "BvhInfo": "xp_bvh_info", "Sources": "xp_sources", "ExtraTallies": "xp_extra_tallies",
              "RunParams": "xp_run_params", "LaunchCfg": "xp_launch_cfg"}


def test_struct_offsets_match_header(tmp_path):
    """Every field of the ctypes mirrors (and of the photon-record dtype) has
    the offset and size the C compiler gives the header's struct member, and
    every struct has the header's size: a C program built against
    include/xephot.h prints them."""
    from paper_2203_14354_amd import _lib
    mirrors = {c: [(f, getattr(getattr(_lib, k), f).offset, getattr(getattr(_lib, k), f).size)
                   for f, _ in getattr(_lib, k)._fields_]
               for k, c in _C_STRUCTS.items()}
    mirrors["xp_photon_record"] = [(f, _lib.RECORD_DTYPE.fields[f][1],
                                    _lib.RECORD_DTYPE.fields[f][0].itemsize)
                                   for f in _lib.RECORD_DTYPE.names]
    sizes = {c: ctypes.sizeof(getattr(_lib, k)) for k, c in _C_STRUCTS.items()}
    sizes["xp_photon_record"] = _lib.RECORD_DTYPE.itemsize
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "xephot.h"',
             'int main(void) {']
    for c, fields in mirrors.items():
        lines.append(f'  printf("{c} sizeof %zu\\n", sizeof({c}));')
        for f, _, _ in fields:
            lines.append(f'  printf("{c} {f} %zu %zu\\n", offsetof({c}, {f}), '
                         f'sizeof((({c} *)0)->{f}));')
    lines += ['  return 0;', '}']
    src, exe = tmp_path / "layout.c", tmp_path / "layout"
    src.write_text("\n".join(lines) + "\n")
    subprocess.run(["gcc", "-std=c99", "-Wall", "-Werror", "-I", os.path.join(ROOT, "include"),
                    str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in filter(None, out):
        parts = line.split()
        if parts[1] == "sizeof":
            got[(parts[0], None)] = int(parts[2])
        else:
            got[(parts[0], parts[1])] = (int(parts[2]), int(parts[3]))
    for c, fields in mirrors.items():
        assert got[(c, None)] == sizes[c], c
        for f, off, size in fields:
            assert got[(c, f)] == (off, size), (c, f)


def test_argument_validation_without_device(lib):
    from paper_2203_14354_amd import _lib
    assert lib.xp_version().startswith(b"xephot")
    # null context / arguments are rejected before any device work
    assert lib.xp_load_mesh(None, None, 0, None, 0, None, None, None, None) == -1
    assert lib.xp_propagate(None, None, None, None, None, None, None, None, None) == -1
    assert lib.xp_backward(None, None, None, None, None, None, None) == -1
    assert lib.xp_set_materials(None, None, 0) == -1
    assert lib.xp_sample(9, 0, 0, 10, None, None, 0.0, 0.0, 0.0, None, None, None) == -1
    assert b"sampler" in lib.xp_last_error(None)
    assert lib.xp_sample(1, 0, 0, 10, None, None, 0.0, 0.0, 0.0, None, None, None) == -1
    out = ctypes.c_void_p()
    assert lib.xp_context_create(-1, ctypes.byref(out)) < 0
    assert out.value is None
    assert len(lib.xp_last_error(None)) > 0
    assert _lib.ERRORS[-3] == "XP_ERR_MESH"
    # extra tallies and their helpers validate before touching a device
    assert lib.xp_set_loss_groups(None, None, 0) == -1
    assert lib.xp_propagate_ex(None, None, None, None, None, None, None, None, None, None) == -1
    assert lib.xp_time_quantile(None, 1, 10, 1.0, 0.9, None, None) == -1
    assert lib.xp_time_quantile(None, 0, 10, 1.0, 1.5, None, None) == -1  # q outside (0, 1]
    assert lib.xp_time_quantile(None, 0, 10, 1.0, 0.9, None, None) == 0   # nothing to do
    assert lib.xp_sample_emission_time(0, 0, 10, 3.5, 24.0, 1.5, None, None, None) == -1
    assert lib.xp_sample_emission_time(0, 0, 0, 3.5, 24.0, 0.5, None, None, None) == 0
    assert lib.xp_set_material_dispersion(None, 0, 0, None, None, None, None) == -1
    assert lib.xp_sample_wavelength(0, 0, 10, 174.8, -1.0, None, None) == -1
    assert lib.xp_surface_reflectance(0, 1.69, 0.81, 1.86, 0, 0, 174.8, 0, None, None, None,
                                      None) == -1  # model 0 has no reflectance formula
    assert lib.xp_surface_reflectance(1, 1.69, 0.81, 1.86, 0, 0, 174.8, 0, None, None, None,
                                      None) == 0


def test_launch_dict_defaults():
    """A launch dict that leaves a field out gets the library default for it:
    lds_levels -1 (the default), not 0 (no staged levels)."""
    from paper_2203_14354_amd.runtime import launch_cfg
    assert launch_cfg(None) is None and launch_cfg({}) is None
    lc = launch_cfg({"wave_batch": 24})
    assert (lc.wave_batch, lc.lds_levels, lc.block_size, lc.stack_lds) == (24, -1, 0, 0)
    assert launch_cfg({"lds_levels": 0}).lds_levels == 0
