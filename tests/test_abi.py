"""Host-side checks of the C ABI: the library loads and exports every function
include/pnp_cdft.h declares, and the host-only entry points answer without a
device (no compute calls here)."""
import ctypes
import os
import re

import pytest

import paper_1407_0674_amd as pkg
from paper_1407_0674_amd import binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pnp_cdft.h")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(pnp_[a-z0-9_]+)\s*\(", txt)))


def test_header_declares_expected_calls():
    names = declared_functions()
    for must in ("pnp_create", "pnp_cdft_mu_ex", "pnp_batch_mu_ex", "pnp_workspace_bytes",
                 "pnp_weighted_densities", "pnp_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for name in declared_functions():
        assert hasattr(lib, name), name
    assert sorted(binding.EXPORTED) == declared_functions()


@pytest.mark.parametrize("n,ok", [(8, 1), (16, 1), (24, 1), (48, 1), (64, 1), (256, 1), (50, 0), (512, 0), (0, 0)])
def test_supported_sizes(n, ok):
    assert binding.load_library().pnp_supported_size(n) == ok


def test_create_without_device_reports_device_error():
    try:
        import torch
        if torch.cuda.is_available():
            pytest.skip("a GPU is present")
    except ImportError:
        pass
    lib = binding.load_library()
    ctx = ctypes.c_void_p()
    assert lib.pnp_create(0, ctypes.byref(ctx)) == -7
    assert not ctx.value


def test_null_arguments_are_rejected_without_device():
    lib = binding.load_library()
    assert lib.pnp_create(0, None) == -1
    assert lib.pnp_workspace_bytes(None, None, 1, None, None) == -1


def test_struct_layouts_match_header():
    # natural C alignment: grid = 3 int32 + pad + double; params = 4 x 4 bytes + 5 x 8
    assert ctypes.sizeof(binding.Grid) == 24
    assert ctypes.sizeof(binding.SpeciesC) == 32
    assert ctypes.sizeof(binding.ParamsC) == 56
    assert binding.RequestC.status.offset == ctypes.sizeof(binding.RequestC) - 8
