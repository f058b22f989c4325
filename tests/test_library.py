"""Host-side checks of the C-ABI library (no GPU compute calls)."""
import ctypes
import os
import re

import pytest

import dcsd_synth as synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "libdcsd.h")
LIB = os.path.join(ROOT, "paper_2401_11935_amd", "lib", "libdcsd.so")


def declared_functions():
    txt = open(HEADER).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(dcsd_[a-z_]+)\s*\(", txt)) - {"dcsd_iter_cb"})


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(LIB):
        pytest.skip("libdcsd.so not built (run __graft_entry__.build())")
    return ctypes.CDLL(LIB)


def test_header_declares_the_method_calls():
    names = declared_functions()
    for required in ("dcsd_init", "dcsd_residual", "dcsd_energy", "dcsd_solve", "dcsd_destroy",
                     "dcsd_last_error", "dcsd_amplitude_count", "dcsd_default_config"):
        assert required in names


def test_library_exports_every_declared_symbol(lib):
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_amplitude_count_and_defaults(lib):
    from paper_2401_11935_amd import libdcsd as L
    L.load(LIB)
    for nc, nv in ((0, 1), (3, 16), (12, 400)):
        assert L.amplitude_count(nc, nv, L.load(LIB)) == synth.amplitude_count(nc, nv)
    assert L.amplitude_count(-1, 3, L.load(LIB)) == -1
    c = L.default_config(L.load(LIB))
    assert c.method == 0 and c.diis_dim == 8 and c.max_iter == 200 and c.term_mask == L.TERM_ALL
    assert ctypes.sizeof(L.Config) == 64


def test_init_rejects_bad_arguments_without_touching_the_gpu(lib):
    from paper_2401_11935_amd import libdcsd as L
    lib2 = L.load(LIB)
    c = L.default_config(lib2, nc=2, nv=3, naux=5)
    c.nv = 0
    with pytest.raises(L.DcsdError) as e:
        L.Context(c, 1, 1, 0, lib2)
    assert e.value.status == L.DCSD_ERR_ARG
    c = L.default_config(lib2, nc=2, nv=3, naux=5, method=7)
    with pytest.raises(L.DcsdError):
        L.Context(c, 1, 1, 0, lib2)
    c = L.default_config(lib2, nc=2, nv=3, naux=5)
    with pytest.raises(L.DcsdError):
        L.Context(c, 0, 0, 0, lib2)      # NULL B and F
