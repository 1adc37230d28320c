"""Host-only checks of the C ABI library: it loads, exports every entry point
that include/mm.h declares, and rejects bad geometry before touching HIP."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    text = open(os.path.join(ROOT, "include", "mm.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(mm_[a-z_]+)\s*\(", text)))


def test_header_declares_the_boundary():
    syms = declared_symbols()
    for s in ["mm_create", "mm_build_tensor", "mm_compute_heff", "mm_step_llg", "mm_reduce",
              "mm_set_material", "mm_set_workspace", "mm_sync", "mm_last_error"]:
        assert s in syms


def test_library_exports_every_declared_symbol():
    from paper_1411_2565_amd import binding
    lib = binding.load()
    for s in declared_symbols():
        assert hasattr(lib, s), s


def test_bad_geometry_rejected_on_host():
    from paper_1411_2565_amd import binding
    lib = binding.load()
    for n, d in [((1, 4, 4), (5e-9,) * 3), ((4, 0, 4), (5e-9,) * 3), ((513, 4, 4), (5e-9,) * 3),
                 ((4, 4, 4), (0.0, 5e-9, 5e-9)), ((4, 4, 4), (5e-9, float("nan"), 5e-9))]:
        g = binding.mm_geometry(n[0], n[1], n[2], *d)
        ctx = ctypes.c_void_p()
        assert lib.mm_create(ctypes.byref(ctx), ctypes.byref(g), 0, None) == binding.MM_EINVAL
        assert not ctx.value


def test_batch_bad_sizes_rejected_on_host():
    from paper_1411_2565_amd import binding
    lib = binding.load()
    b = ctypes.c_void_p()
    for sizes, d in [([(64, 64, 1), (1, 8, 1)], (4e-9, 4e-9, 3e-9)), ([(600, 8, 1)], (4e-9, 4e-9, 3e-9)),
                     ([(64, 64, 1)], (4e-9, -1.0, 3e-9))]:
        arr = (ctypes.c_int32 * (3 * len(sizes)))(*[v for s in sizes for v in s])
        assert lib.mm_batch_create(ctypes.byref(b), len(sizes), arr, *d, 0, None) == binding.MM_EINVAL
        assert not b.value
    assert lib.mm_batch_create(ctypes.byref(b), 0, None, 4e-9, 4e-9, 3e-9, 0, None) == binding.MM_EINVAL


def test_null_arguments_rejected():
    from paper_1411_2565_amd import binding
    lib = binding.load()
    assert lib.mm_create(None, None, 0, None) == binding.MM_EINVAL
    assert lib.mm_destroy(None) == binding.MM_EINVAL
    assert lib.mm_sync(None) == binding.MM_EINVAL
    assert lib.mm_step_llg(None, None, 1, 1e-13, 0) == binding.MM_EINVAL
    assert lib.mm_diag_dot3(None, None, None, 1) == binding.MM_EINVAL


def test_product_path_does_not_import_oracle():
    """The GPU package never imports, includes or loads the CPU oracle."""
    pkg = os.path.join(ROOT, "paper_1411_2565_amd")
    pat = re.compile(r"^\s*(import\s+oracle|from\s+oracle|#include\s*[<\"].*oracle)|liboracle", re.M)
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".cpp", ".hip", ".hpp", ".h")):
                src = open(os.path.join(dirpath, f)).read()
                assert not pat.search(src), f
