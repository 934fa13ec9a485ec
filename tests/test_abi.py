"""The C-ABI library loads and exports every symbol include/ifmm.h declares (no GPU needed)."""
import os
import re

import pytest

from paper_1508_01835_amd import ifmm as binding

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "ifmm.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(ifmm_[a-z_]+)\s*\(", src)))


def test_header_declares_the_boundary():
    names = declared_symbols()
    for n in ["ifmm_build", "ifmm_factorize", "ifmm_solve", "ifmm_matvec", "ifmm_gmres", "ifmm_destroy"]:
        assert n in names


def test_library_exports_every_declared_symbol():
    lib = binding.load_library()
    for n in declared_symbols():
        assert hasattr(lib, n), n
    assert set(binding.EXPORTS) == set(declared_symbols())


def test_status_strings_and_defaults():
    import ctypes
    lib = binding.load_library()
    assert lib.ifmm_strerror(0) == b"ok"
    assert b"argument" in lib.ifmm_strerror(1)
    opt = binding.Options()
    lib.ifmm_default_options(ctypes.byref(opt))
    assert opt.precision == 64 and opt.leaf_max == 64 and opt.rank_max == 0


def test_null_arguments_rejected_without_gpu_work():
    import ctypes
    lib = binding.load_library()
    h = ctypes.c_void_p()
    k = binding.Kernel(0, 0.01, 1.0)
    rc = lib.ifmm_build(None, 10, 2, k, 3, 3, 1e-6, None, ctypes.byref(h))
    assert rc == 1 and not h.value
    assert lib.ifmm_factorize(None) == 1
    assert lib.ifmm_solve(None, None, None, 1, 1) == 1
    assert lib.ifmm_solve_noalloc(None, None, None, 1, 1) == 1
    assert lib.ifmm_query_ranks(None, 2, None, 0) == 1
    assert lib.ifmm_destroy(None) == 0


@pytest.mark.parametrize("cname,mirror", [("ifmm_options", "Options"), ("ifmm_stats", "Stats"),
                                          ("ifmm_kernel", "Kernel")])
def test_struct_layout_matches_header(tmp_path, cname, mirror):
    """The ctypes mirror of a header struct has its size and field offsets (gcc on the header)."""
    import ctypes
    import shutil
    import subprocess
    if shutil.which("gcc") is None:
        pytest.skip("no C compiler")
    cls = getattr(binding, mirror)
    names = [f[0] for f in cls._fields_]
    src = tmp_path / "layout.c"
    src.write_text('#include <stdio.h>\n#include <stddef.h>\n#include "ifmm.h"\nint main(void) {\n'
                   '  printf("%%zu\\n", sizeof(%s));\n' % cname +
                   "".join('  printf("%%zu\\n", offsetof(%s, %s));\n' % (cname, n) for n in names) +
                   "  return 0;\n}\n")
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-std=c99", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    got = [int(v) for v in subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(cls)
    assert got[1:] == [getattr(cls, n).offset for n in names]


def test_allocator_callbacks_default_null_and_come_in_pairs():
    import ctypes
    lib = binding.load_library()
    opt = binding.Options()
    lib.ifmm_default_options(ctypes.byref(opt))
    assert not opt.dev_alloc and not opt.dev_free and not opt.alloc_ctx
    opt.dev_alloc = binding.DevAllocFn(lambda n, c: None)   # dev_free left null: rejected before any GPU work
    pts = (ctypes.c_double * 20)()
    h = ctypes.c_void_p()
    rc = lib.ifmm_build(pts, 10, 2, binding.Kernel(0, 0.01, 1.0), 3, 3, 1e-6, ctypes.byref(opt), ctypes.byref(h))
    assert rc == 1 and not h.value
    assert b"dev_alloc" in lib.ifmm_last_error()
