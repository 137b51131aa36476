"""The compact [r]^(0) table layouts of the matrix-core kernels: every entry
(t, u, v), t + u + v <= L, of up to QMAX tables placed SIZE doubles apart
must have an address of its own, and the largest entry of a table must be
(L, 0, 0), which the kernels' LDS sizing assumes."""
import os
import re

import numpy as np

HDR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2506_12501_amd", "csrc", "cube_layouts.h")


def table():
    src = open(HDR).read()
    qmax = int(re.search(r"CUBE_COMPACT_QMAX = (\d+);", src).group(1))
    dmax = int(re.search(r"CUBE_COMPACT_DMAX = (\d+);", src).group(1))
    rows = [tuple(map(int, m)) for m in re.findall(r"\{(\d+), (\d+), (\d+), (\d+)\}", src)]
    return qmax, dmax, rows


def test_table_covers_every_order():
    qmax, dmax, rows = table()
    assert [r[0] for r in rows] == list(range(1, dmax + 1))
    assert dmax >= 18          # (gg|gg) has L = 16; the backward kernel reaches L + 1
    assert qmax >= 32


def test_layouts_are_injective_for_qmax_tables():
    qmax, _, rows = table()
    for D, su, st, size in rows:
        L = D - 1
        pts = np.array([(t, u, v) for t in range(D) for u in range(D - t) for v in range(D - t - u)])
        one = pts[:, 0] * st + pts[:, 1] * su + pts[:, 2]
        assert one.max() == L * st, D                      # span of a table ends at (L, 0, 0)
        allq = (one[None, :] + size * np.arange(qmax)[:, None]).ravel()
        assert len(np.unique(allq)) == allq.size, f"D={D}: tables overlap"


def test_layouts_are_smaller_than_the_dense_cube():
    _, _, rows = table()
    for D, su, st, size in rows[3:]:
        assert size < 0.6 * D ** 3, D
