"""The C ABI library: built, loadable, exporting every declared entry point."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "vesis.h")
NN_HEADER = os.path.join(ROOT, "include", "vesis_nn.h")


def declared_functions(header=HEADER):
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(vesis_[a-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary_calls():
    names = declared_functions()
    for required in ("vesis_set_atoms", "vesis_set_positions", "vesis_set_params",
                     "vesis_set_grid", "vesis_minimize_interface", "vesis_energy",
                     "vesis_forces", "vesis_atom_step"):
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2208_05524_amd import _lib
    lib = _lib.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(_lib.EXPORTS) == declared_functions()


def test_library_exports_every_network_layer():
    from paper_2208_05524_amd import _lib, nn
    lib = _lib.load()
    names = declared_functions(NN_HEADER)
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing
    assert sorted(nn.NN_EXPORTS) == names


def test_library_is_built_for_gfx950():
    from paper_2208_05524_amd import _lib
    data = open(_lib.LIB_PATH, "rb").read()
    assert b"gfx950" in data


def test_create_without_a_device_reports_no_device():
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    from paper_2208_05524_amd import _lib
    lib = _lib.load()
    h = ctypes.c_void_p()
    assert lib.vesis_create(0, None, ctypes.byref(h)) == -5
    assert not h.value


def test_product_package_does_not_import_the_oracle():
    pkg = os.path.join(ROOT, "paper_2208_05524_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp")):
                src = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in src.replace("oracles", ""), f


def test_new_calls_reject_bad_arguments_before_touching_a_device():
    """The solute-solute set-up calls refuse a null context, and the fused
    decoder convolution refuses odd or too narrow grids and channel counts
    that are not multiples of 16 (or of 32 for the outputs), all before any
    device work (so this runs without a GPU)."""
    from paper_2208_05524_amd import _lib, nn
    lib = _lib.load()
    one = (ctypes.c_int32 * 4)(0, 1, 2, 3)
    val = (ctypes.c_double * 7)(*([1.0] * 7))
    assert lib.vesis_set_angles(None, 1, one, val, val) == -1
    assert lib.vesis_set_torsions(None, 1, one, val, val) == -1
    assert lib.vesis_set_nonbonded(None, 1, None, None, 0, None) == -1
    L = nn.lib()
    p = ctypes.c_void_p(1 << 20)  # never dereferenced: every call below fails its checks
    bad = [(16, 64, 32, 32, 15),   # odd grid
           (16, 64, 32, 32, 8),    # narrower than 16
           (16, 60, 32, 32, 16),   # ca % 16
           (16, 64, 20, 32, 16),   # cb % 16
           (16, 64, 32, 48, 16)]   # cout % 32
    for d, ca, cb, cout, wd in bad:
        assert L.vesis_nn_conv3_fwd_upcat(None, p, ca, p, cb, p, None, p, 1, d, d, wd, cout,
                                          1) == -1
    assert L.vesis_nn_conv3_fwd_upcat(None, None, 64, p, 32, p, None, p, 1, 16, 16, 16, 32,
                                      1) == -1
