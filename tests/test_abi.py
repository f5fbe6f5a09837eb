"""The C-ABI library loads and exports every function its header declares (no GPU needed)."""
import ctypes
import os
import re
import subprocess

import pytest

import paper_1206_3710_amd as rt

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "rt.h")


def declared():
    txt = open(HEADER).read()
    return sorted(set(re.findall(r"^\s*(?:rt_status|const char\*)\s+(rt_\w+)\s*\(", txt, re.M)))


@pytest.fixture(scope="module")
def libpath():
    if not os.path.exists(rt.LIB_PATH):
        from paper_1206_3710_amd import build
        build.build()
    return rt.LIB_PATH


def test_header_declares_the_boundary():
    names = declared()
    for n in ("rt_build_tree", "rt_set_dust", "rt_trace_packets", "rt_solve_temperature",
              "rt_render_map", "rt_lambda_iterate", "rt_locate"):
        assert n in names
    assert names == sorted(rt.EXPORTS)


def test_library_exports_every_declared_symbol(libpath):
    lib = ctypes.CDLL(libpath)
    for n in declared():
        assert hasattr(lib, n), n
    out = subprocess.run(["nm", "-D", "--defined-only", libpath], capture_output=True, text=True).stdout
    syms = {l.split()[-1] for l in out.splitlines() if l.strip()}
    for n in declared():
        assert n in syms


def test_library_is_built_for_gfx950(libpath, tmp_path):
    """The embedded device-code bundle targets gfx950 (and nothing else)."""
    sec = tmp_path / "fatbin.bin"
    r = subprocess.run(["objcopy", "-O", "binary", "--only-section=.hip_fatbin", libpath, str(sec)],
                       capture_output=True, text=True)
    if r.returncode != 0:
        pytest.skip("objcopy unavailable")
    data = sec.read_bytes()
    targets = set(re.findall(rb"amdgcn-amd-amdhsa--(gfx[0-9a-z]+)", data))
    assert targets == {b"gfx950"}


def test_binding_refuses_without_gpu():
    import torch
    if torch.cuda.is_available():
        pytest.skip("GPU present")
    with pytest.raises(RuntimeError):
        rt.Context(0)
