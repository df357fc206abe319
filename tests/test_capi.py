"""CPU-side checks of the C ABI: the library loads, exports every declared entry point, and rejects
invalid arguments before touching the GPU."""

import ctypes
import os
import re

import numpy as np
import pytest

from paper_2301_12836_amd import lsvie

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    text = open(os.path.join(ROOT, "include", "ls.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ls_[A-Za-z0-9_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("ls_setup", "ls_apply", "ls_solve", "ls_destroy", "ls_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    lib = lsvie.load()
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_functions()) == set(lsvie.EXPORTED)


def test_setup_rejects_bad_arguments_without_a_gpu():
    lib = lsvie.load()
    g = lsvie.Grid((ctypes.c_int * 3)(1, 8, 8), 10.0)      # an axis with one cell
    C0 = np.eye(6).ravel() * 1e10
    om = np.array([1.0])
    out = ctypes.c_void_p()
    dp = ctypes.POINTER(ctypes.c_double)
    rc = lib.ls_setup(ctypes.byref(g), C0.ctypes.data_as(dp), 2400.0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                      om.ctypes.data_as(dp), 1, None, None, ctypes.byref(out))
    assert rc == lsvie.LS_ERR_ARG
    assert b"grid size" in lib.ls_last_error()
    g = lsvie.Grid((ctypes.c_int * 3)(8, 8, 8), 10.0)
    rc = lib.ls_setup(ctypes.byref(g), C0.ctypes.data_as(dp), 2400.0, None, None, om.ctypes.data_as(dp), 1, None,
                      None, ctypes.byref(out))
    assert rc == lsvie.LS_ERR_ARG
    bad = C0.copy()
    bad[1] = 5.0                                          # C0[0][1] != C0[1][0]
    rc = lib.ls_setup(ctypes.byref(g), bad.ctypes.data_as(dp), 2400.0, ctypes.c_void_p(1), ctypes.c_void_p(1),
                      om.ctypes.data_as(dp), 1, None, None, ctypes.byref(out))
    assert rc == lsvie.LS_ERR_ARG and b"symmetric" in lib.ls_last_error()
    assert not out.value


def test_null_context_is_rejected():
    lib = lsvie.load()
    assert lib.ls_apply(None, 0, None, None, 1) == lsvie.LS_ERR_ARG
    assert lib.ls_solve(None, 0, None, 1, 1e-6, 10, 0, None, None, None) == lsvie.LS_ERR_ARG
    lib.ls_destroy(None)
    assert lib.ls_device_bytes(None) == 0


def test_output_buffers_are_checked_before_the_library_writes():
    """A caller-supplied output must match the input's dtype and shape exactly: the library writes
    complex128 or complex64 fields through a plain pointer sized by the grid and right-hand sides."""
    torch = pytest.importorskip("torch")
    dev = torch.device("cpu")
    shape = (2, 3, 4, 5, 6)
    good = torch.zeros(shape, dtype=torch.complex128)
    assert lsvie.check_buffer(good, shape, torch.complex128, dev) is good
    bad = [torch.zeros(shape, dtype=torch.complex64),             # half the bytes
           torch.zeros((1,) + shape[1:], dtype=torch.complex128),  # fewer right-hand sides
           torch.zeros(shape[::-1], dtype=torch.complex128).permute(4, 3, 2, 1, 0),  # not contiguous
           good.conj(),                                            # lazy conjugate view
           torch.zeros(shape, dtype=torch.float64)]
    for t in bad:
        with pytest.raises(ValueError):
            lsvie.check_buffer(t, shape, torch.complex128, dev)


def test_header_is_plain_c():
    """The boundary is a C ABI: the header compiles as C99 (and as C++) with no HIP or torch types."""
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    src = '#include "ls.h"\nint main(void) { ls_options o = {0}; ls_info i = {0}; ls_job j = {0};\n' \
          '  (void)o; (void)i; (void)j; return LS_OK; }\n'
    with tempfile.TemporaryDirectory() as d:
        for lang, comp, std in (("c", "gcc", "-std=c99"), ("c++", "g++", "-std=c++17")):
            f = os.path.join(d, "t." + ("c" if lang == "c" else "cpp"))
            open(f, "w").write(src)
            r = subprocess.run([comp, std, "-Wall", "-Werror", "-fsyntax-only", "-I", os.path.join(ROOT, "include"), f],
                               capture_output=True, text=True)
            assert r.returncode == 0, r.stderr


def test_ctypes_structures_match_the_header_layout():
    """The binding's ctypes mirrors of ls_grid, ls_options, ls_info and ls_job have the C layout: sizes and
    field offsets printed by a C program compiled against include/ls.h."""
    import ctypes
    import shutil
    import subprocess
    import tempfile
    if shutil.which("gcc") is None:
        pytest.skip("no host C compiler")
    from paper_2301_12836_amd import lsvie
    structs = {"ls_grid": lsvie.Grid, "ls_options": lsvie.Options, "ls_info": lsvie.Info, "ls_job": lsvie.Job}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "ls.h"', 'int main(void) {']
    for cname, cls in structs.items():
        lines.append(f'  printf("{cname} size %zu\\n", sizeof({cname}));')
        for fname, _ in cls._fields_:
            lines.append(f'  printf("{cname} {fname} %zu\\n", offsetof({cname}, {fname}));')
    lines += ['  return 0;', '}']
    with tempfile.TemporaryDirectory() as d:
        src = os.path.join(d, "layout.c")
        exe = os.path.join(d, "layout")
        open(src, "w").write("\n".join(lines) + "\n")
        r = subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), src, "-o", exe],
                           capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        out = subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {tuple(l.split()[:2]): int(l.split()[2]) for l in out if l.strip()}
    for cname, cls in structs.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for fname, _ in cls._fields_:
            assert got[(cname, fname)] == getattr(cls, fname).offset, (cname, fname)
