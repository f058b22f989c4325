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
    assert c.adjoint == 0 and c.guard_iters == 10 and c.ladder_cache == 1


def test_ctypes_mirrors_match_the_header(tmp_path):
    """Sizes and field offsets of the binding's structs equal those the C compiler
    gives the header's structs."""
    import shutil
    import subprocess
    from paper_2401_11935_amd import libdcsd as L
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    structs = {"dcsd_config": L.Config, "dcsd_report": L.Report, "dcsd_energies": L.Energies,
               "dcsd_timing": L.Timing, "dcsd_kernel_time": L.KernelTime}
    lines = ["#include <stdio.h>", "#include <stddef.h>", f'#include "{HEADER}"', "int main(void) {"]
    for cname, py in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in py._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ["  return 0;", "}"]
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines) + "\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-o", str(exe), str(src)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    got = {tuple(x.split()[:2]): int(x.split()[2]) for x in out if x}
    for cname, py in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(py), cname
        for fname, _ in py._fields_:
            assert got[(cname, fname)] == getattr(py, fname).offset, (cname, fname)


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
    for bad in (dict(guard_iters=-1), dict(adjoint=2), dict(ladder_cache=3)):
        c = L.default_config(lib2, nc=2, nv=3, naux=5)
        for k, v in bad.items():
            setattr(c, k, v)
        with pytest.raises(L.DcsdError) as e:
            L.Context(c, 1, 1, 0, lib2)
        assert e.value.status == L.DCSD_ERR_ARG
