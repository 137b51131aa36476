import os
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (HIP device) and the built libmdx.so")


def _ensure_oracle():
    lib = os.path.join(ROOT, "oracle", "liboracle_f64.so")
    libq = os.path.join(ROOT, "oracle", "liboracle_q.so")
    src = os.path.join(ROOT, "oracle", "mdx_oracle.c")
    if (not os.path.exists(lib) or not os.path.exists(libq)
            or os.path.getmtime(lib) < os.path.getmtime(src)):
        from oracle import build as ob
        ob.build()


_ensure_oracle()


def gpu_available() -> bool:
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def pytest_collection_modifyitems(config, items):
    if gpu_available():
        return
    skip = pytest.mark.skip(reason="no HIP device visible")
    for it in items:
        if "gpu" in it.keywords:
            it.add_marker(skip)
