"""The C-ABI library loads and exports what include/gwswig.h declares (CPU).

No compute call is made here; only argument checks that happen before any
HIP call, and the no-device error path when no GPU is visible.
"""
import ctypes
import os
import re

import numpy as np
import pytest

import gwsynth
from paper_2607_28265_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gwswig.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    names = re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\**\s*([A-Za-z_][A-Za-z0-9_]*)\s*\(", src, flags=re.M)
    return sorted(set(names))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(_lib.LIB_PATH):
        pytest.fail("libgwswig.so is not built (run python -m paper_2607_28265_amd.build)")
    return _lib.load()


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert {"loglike_batch", "gw_template", "heterodyne_setup", "loglike_batch_uneven", "slice_step"} <= set(names)
    for n in names:
        assert hasattr(lib, n), f"symbol {n} declared in gwswig.h but not exported"


def test_binding_covers_header():
    names = set(_declared_functions())
    assert names <= set(_lib._SIGS), names - set(_lib._SIGS)


def test_version(lib):
    assert "gfx950" in _lib.gw_version()


def test_ctx_create_argument_errors(lib):
    out = ctypes.c_void_p()
    assert lib.gw_ctx_create(None, 0, ctypes.byref(out)) == _lib.GW_EINVAL
    assert "problem is NULL" in _lib.gw_last_error()
    p = _lib.gw_problem(n_det=0)
    assert lib.gw_ctx_create(ctypes.byref(p), 0, ctypes.byref(out)) == _lib.GW_EINVAL
    assert "n_det" in _lib.gw_last_error()
    assert out.value is None


def test_ctx_create_rejects_bad_psd(lib):
    prob = gwsynth.make_problem(8.0, 20.0, 64.0)
    prob.psd = prob.psd.copy()
    prob.psd[1, 5] = -1.0
    with pytest.raises(_lib.GwError) as e:
        _lib.gw_ctx_create(prob)
    assert e.value.status == _lib.GW_EINVAL


def test_null_context_calls(lib):
    assert lib.loglike_batch(None, None, 0, 0, 0, 0, None, None) == _lib.GW_EINVAL
    assert lib.gw_ctx_destroy(None) == _lib.GW_OK
    v = ctypes.c_double()
    assert lib.gw_data_inner(None, ctypes.byref(v)) == _lib.GW_EINVAL


def test_no_device_is_reported(lib):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    prob = gwsynth.make_problem(8.0, 20.0, 64.0)
    with pytest.raises(_lib.GwError) as e:
        _lib.gw_ctx_create(prob)
    assert e.value.status == _lib.GW_EDEVICE


def test_struct_layouts_match_header(tmp_path):
    # The ctypes mirrors of the argument structs must have the C compiler's
    # size and field offsets (a shorter mirror would let the library read past
    # the caller's struct).
    import shutil
    import subprocess
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    structs = {"gw_problem": _lib.gw_problem, "gw_slice_args": _lib.gw_slice_args,
               "gw_sweep_args": _lib.gw_sweep_args, "gw_fiducial_args": _lib.gw_fiducial_args}
    lines = ['#include <stddef.h>', '#include <stdio.h>', '#include "gwswig.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'  printf("{name} size %zu\\n", sizeof({name}));')
        for f, _ in cls._fields_:
            lines.append(f'  printf("{name} {f} %zu\\n", offsetof({name}, {f}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run([cc, "-std=c11", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for name, cls in structs.items():
        assert got[(name, "size")] == ctypes.sizeof(cls), name
        for f, _ in cls._fields_:
            assert got[(name, f)] == getattr(cls, f).offset, (name, f)
