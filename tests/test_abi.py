"""The C-ABI library: builds, loads, and exports every entry point that
include/mdx.h declares.  No compute calls here (no GPU needed)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def header_functions():
    src = open(os.path.join(ROOT, "include", "mdx.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(mdx_[a-z_0-9]+)\s*\(", src)))


def test_header_declares_the_entry_points():
    names = header_functions()
    for required in ["mdx_eri_batch", "mdx_eri_grad_batch", "mdx_boys", "mdx_create", "mdx_destroy",
                     "mdx_plan_create", "mdx_plan_execute", "mdx_eri_digest_batch", "mdx_one_body_batch",
                     "mdx_nuclear_batch"]:
        assert required in names


def test_library_exports_every_declared_symbol():
    from paper_2506_12501_amd import native
    L = native.lib()
    for name in header_functions():
        assert hasattr(L, name), name
    assert set(header_functions()) == set(native.EXPORTS), "binding and header disagree"


def test_status_strings():
    from paper_2506_12501_amd import native
    L = native.lib()
    for s, name in enumerate(["MDX_OK", "MDX_EINVAL", "MDX_EUNSUPPORTED", "MDX_EWORKSPACE", "MDX_ENOMEM",
                              "MDX_EDEVICE"]):
        assert L.mdx_status_string(s).decode() == name


def test_null_arguments_rejected_without_device_work():
    from paper_2506_12501_amd import native
    L = native.lib()
    assert L.mdx_boys(None, 4, None, 3, None, None) == native.MDX_EINVAL
    assert L.mdx_create(0, None) == native.MDX_EINVAL
    assert L.mdx_set_variant(None, 4, 0, 0, 0, 0, 0, 0) == native.MDX_EINVAL
    assert L.mdx_eri_workspace_size(None, None, 4, 1, None, 1, None, 0) == 0


def test_no_gpu_means_clean_error():
    from tests.conftest import gpu_available
    if gpu_available():
        pytest.skip("device present")
    from paper_2506_12501_amd import native
    h = ctypes.c_void_p()
    st = native.lib().mdx_create(0, ctypes.byref(h))
    assert st in (native.MDX_EINVAL, native.MDX_EDEVICE)


def test_every_entry_point_is_documented():
    """each declaration follows its contract comment: between the nearest
    comment block and the declaration stands at most one other declaration
    (a size query and its call share one contract)"""
    src = open(os.path.join(ROOT, "include", "mdx.h")).read()
    for name in header_functions():
        # the declaration: the first occurrence outside a comment line
        for m in re.finditer(r"\b" + name + r"\s*\(", src):
            line = src[src.rfind("\n", 0, m.start()) + 1:m.start()].strip()
            if not line.startswith(("*", "/*")):
                break
        i = m.start()
        gap = src[src.rfind("*/", 0, i):i]
        assert src.rfind("*/", 0, i) >= 0 and gap.count(";") <= 1, name
