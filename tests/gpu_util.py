"""Helpers shared by the GPU tests (no integral arithmetic here)."""
import numpy as np

ATOL = 1e-12   # per element: pass iff |gpu - oracle| <= ATOL or <= RTOL |oracle|
RTOL = 1e-10


def assert_close(got, ref, what=""):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    assert np.all(np.isfinite(got)), f"{what}: non-finite values"
    err = np.abs(got - ref)
    ok = (err <= ATOL) | (err <= RTOL * np.abs(ref))
    if not ok.all():
        idx = np.unravel_index(np.argmax(np.where(ok, 0, err)), err.shape)
        raise AssertionError(f"{what}: {np.count_nonzero(~ok)} of {ok.size} elements off; worst at {idx}: "
                             f"gpu {got[idx]!r} oracle {ref[idx]!r}")


def shells(batch_basis):
    from paper_2506_12501_amd import native
    return native.DeviceShells(batch_basis)
