"""The C-ABI libraries load and export every entry point their headers
declare (no GPU needed: nothing here launches a kernel)."""
import ctypes as C
import os
import re
import subprocess

import pytest

from paper_2511_02021_amd import _build, nhdc


def _declared(header):
    src = open(os.path.join(_build.INCLUDE, header)).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b((?:nhdc|nhgrid)_[a-z_]+)\s*\(", src)))


def _exported(path):
    out = subprocess.run(["nm", "-D", "--defined-only", path], capture_output=True, text=True,
                         check=True).stdout
    return {ln.split()[-1] for ln in out.splitlines() if " T " in ln}


def test_nhdc_exports_every_declared_symbol():
    lib = nhdc.lib()  # loads (and builds if absent) libnhdc.so
    declared = _declared("nhdc.h")
    assert len(declared) >= 10
    exported = _exported(_build.NHDC_SO)
    missing = [s for s in declared if s not in exported]
    assert not missing, missing
    for s in declared:
        assert hasattr(lib, s)


def test_nhgrid_exports_every_declared_symbol():
    from paper_2511_02021_amd.inputs import grid
    grid.lib()
    declared = _declared("nhgrid.h")
    exported = _exported(_build.INPUTS_SO)
    assert not [s for s in declared if s not in exported]


def test_library_has_gfx950_code_object(tmp_path):
    fat = tmp_path / "nhdc.fatbin"
    r = subprocess.run(["objcopy", f"--dump-section=.hip_fatbin={fat}", _build.NHDC_SO,
                        str(tmp_path / "copy.so")], capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("objcopy cannot extract the device code section")
    out = subprocess.run(["/opt/rocm/llvm/bin/clang-offload-bundler", "--list", "--type=o",
                          f"--input={fat}"], capture_output=True, text=True)
    assert out.returncode == 0 and "gfx950" in out.stdout


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(_build.PKG, "nhdc.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


def test_argument_errors_without_device():
    L = nhdc.lib()
    h = C.c_void_p()
    assert L.nhdc_create(None, 0, 0) == -1
    assert L.nhdc_create(C.byref(h), 7, 0) == -1
    assert L.nhdc_step(None, 1.0, 1, None) == -1
    assert L.nhdc_last_error(None) == b"no context"


def test_shape_calls_refuse_null_handles_without_device():
    L = nhdc.lib()
    buf = (C.c_int * 7)()
    assert L.nhdc_set_column_mode(None, 1) == -1
    assert L.nhdc_get_shapes(None, buf) == -1
    assert L.nhdc_batch_set_column_mode(None, 0) == -1
    assert L.nhdc_batch_get_shapes(None, buf) == -1
    assert L.nhdc_set_tiles(None, 0, 0, 0) == -1
    assert L.nhdc_set_block_sizes(None, 256, 64, 3) == -1


def test_noalloc_argument_errors_without_device():
    """The allocation-free entry point refuses NULL arrays, bad sizes and
    inputs beyond its fixed scratch before any device call."""
    L = nhdc.lib()
    fake = C.c_void_p(0x1000)  # never dereferenced: the checks come first
    assert L.nhdc_diag_noalloc(10, 5, None, fake, fake, fake, fake, None) == -1
    assert b"NULL" in L.nhdc_last_error(None)
    assert L.nhdc_diag_noalloc(0, 5, fake, fake, fake, fake, fake, None) == -1
    assert L.nhdc_diag_noalloc(10, 0, fake, fake, fake, fake, fake, None) == -1
    assert L.nhdc_diag_noalloc(10, 257, fake, fake, fake, fake, fake, None) == -1
    assert L.nhdc_diag_noalloc(nhdc.NOALLOC_MAX_CELLS + 1, 5, fake, fake, fake, fake, fake, None) == -7
    assert b"exceed the static scratch" in L.nhdc_last_error(None)
