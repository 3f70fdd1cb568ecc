"""The C-ABI library loads and exports every entry point include/fmmbem.h
declares; host-side argument validation rejects bad input without touching
the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "fmmbem.h")
LIB = os.path.join(ROOT, "paper_1506_05957_amd", "libfmmbem.so")


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fmmbem_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = declared_functions()
    for required in ("fmmbem_build", "fmmbem_matvec", "fmmbem_solve", "fmmbem_solve_ctx", "fmmbem_get_stats",
                     "fmmbem_destroy", "fmmbem_last_error", "fmmbem_server_create", "fmmbem_submit",
                     "fmmbem_poll", "fmmbem_wait", "fmmbem_server_destroy"):
        assert required in names


def test_library_exports_every_declared_symbol():
    assert os.path.exists(LIB), "build first"
    lib = ctypes.CDLL(LIB)
    for name in declared_functions():
        assert hasattr(lib, name), name


def test_no_cpu_fallback_in_binding():
    src = open(os.path.join(ROOT, "paper_1506_05957_amd", "fmmbem.py")).read()
    assert "import oracle" not in src and "from oracle" not in src


@pytest.fixture(scope="module")
def fb():
    from paper_1506_05957_amd import fmmbem
    return fmmbem


def _build_rc(fb, xyz, tri, kernel=0, prm=None):
    m, keep = fb.make_mesh(xyz, tri)
    h = ctypes.c_void_p()
    rc = fb._lib.fmmbem_build(ctypes.byref(m), kernel, ctypes.byref(prm) if prm is not None else None,
                              ctypes.c_void_p(0), ctypes.byref(h))
    return rc, h


def test_build_rejects_bad_meshes(fb):
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    rc, h = _build_rc(fb, xyz, np.array([[0, 1, 3]], dtype=np.int32))
    assert rc == fb.EINVAL and not h.value
    assert "out of range" in fb.fmmbem_last_error()
    rc, h = _build_rc(fb, xyz, np.zeros((0, 3), dtype=np.int32))
    assert rc == fb.EINVAL
    bad = xyz.copy(); bad[1, 0] = np.nan
    rc, h = _build_rc(fb, bad, np.array([[0, 1, 2]], dtype=np.int32))
    assert rc == fb.EINVAL
    rc, h = _build_rc(fb, xyz, np.array([[0, 1, 2]], dtype=np.int32), kernel=7)
    assert rc == fb.EINVAL


def test_build_rejects_bad_params(fb):
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    for prm in (fb.params(theta=0.0), fb.params(theta=1.5), fb.params(ncrit=0), fb.params(p_max=21),
                fb.params(p_max=0), fb.params(mu=-1.0), fb.params(near_stored=2),
                fb.params(m2l_stored=3)):
        rc, h = _build_rc(fb, xyz, tri, prm=prm)
        assert rc == fb.EINVAL


def test_null_arguments(fb):
    assert fb._lib.fmmbem_build(None, 0, None, None, None) == fb.EINVAL
    assert fb._lib.fmmbem_matvec(None, 5, 0, None, None, None) == fb.EINVAL
    assert fb._lib.fmmbem_get_stats(None, None) == fb.EINVAL
    assert fb._lib.fmmbem_set_timing_stages(None, 1) == fb.EINVAL
    fb._lib.fmmbem_destroy(None)


def test_schedule_defaults(fb):
    s = fb.schedule(fb.STOKES)
    assert (s.p_init, s.p_min, s.restart, s.rule) == (16, 4, 50, fb.RELAX_BF)
    s = fb.schedule(fb.LAPLACE)
    assert (s.p_init, s.p_min) == (12, 3)


def test_binding_struct_layouts_match_the_header(fb, tmp_path):
    """Every field offset and struct size of the ctypes binding equals the C
    header's (a C program built against include/fmmbem.h prints them)."""
    import subprocess
    structs = {name: getattr(fb, name) for name in ("fmmbem_mesh", "fmmbem_params", "fmmbem_schedule",
                                                      "fmmbem_report", "fmmbem_stats", "fmmbem_server_params",
                                                      "fmmbem_request_info")}
    lines = ["#include <stdio.h>", "#include <stddef.h>", '#include "fmmbem.h"', "int main(void) {"]
    for name, cls in structs.items():
        lines.append(f'printf("{name} size %zu\\n", sizeof({name}));')
        for field, _ in cls._fields_:
            lines.append(f'printf("{name} {field} %zu\\n", offsetof({name}, {field}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout.split("\n")
    seen = 0
    for line in filter(None, out):
        name, field, value = line.split()
        cls = structs[name]
        got = ctypes.sizeof(cls) if field == "size" else getattr(cls, field).offset
        assert got == int(value), (name, field, got, value)
        seen += 1
    assert seen == sum(len(c._fields_) + 1 for c in structs.values())


def test_build_rejects_quadrature_it_does_not_implement(fb):
    xyz = np.array([[0.0, 0, 0], [1, 0, 0], [0, 1, 0]])
    tri = np.array([[0, 1, 2]], dtype=np.int32)
    for prm in (fb.params(quad_far=7), fb.params(quad_near=16), fb.params(near_factor=3.0)):
        rc, h = _build_rc(fb, xyz, tri, prm=prm)
        assert rc == fb.EINVAL and not h.value
    prm = fb.params()
    prm.alloc = fb.ALLOC_FN(lambda n, u: None)  # alloc without free
    rc, h = _build_rc(fb, xyz, tri, prm=prm)
    assert rc == fb.EINVAL and "together" in fb.fmmbem_last_error()
