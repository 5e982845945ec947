"""The C ABI library loads and exports every symbol include/xephot.h declares;
host-side argument validation works without a GPU."""
import ctypes
import os
import re
import subprocess

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
    assert ctypes.sizeof(_lib.Surface) == 28
    assert ctypes.sizeof(_lib.Sources) == 88
    assert ctypes.sizeof(_lib.RunParams) == 32
    assert ctypes.sizeof(_lib.LaunchCfg) == 24
    assert _lib.RECORD_DTYPE.itemsize == 96


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
