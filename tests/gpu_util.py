"""Helpers shared by the GPU tests (no integral arithmetic here)."""
import numpy as np

ATOL = 1e-12   # per element: pass iff |gpu - oracle| <= ATOL or <= RTOL |oracle|
RTOL = 1e-10
SHELLSET_RTOL = 1e-10   # max |gpu - oracle| over a shellset / max |oracle| of that shellset


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


def assert_close_shellsets(got, ref, what="", block_axes=(1, 2)):
    """assert_close per element, plus the error relative to each shellset's
    largest element (block_axes: the [ab, cd] axes of one shellset), which
    must stay within SHELLSET_RTOL; returns and prints the worst ratio."""
    assert_close(got, ref, what)
    err = np.abs(np.asarray(got) - np.asarray(ref)).max(axis=block_axes)
    big = np.abs(np.asarray(ref)).max(axis=block_axes)
    rel = float(np.max(err / np.maximum(big, 1e-300)))
    print(f"{what}: max |err| / shellset max = {rel:.2e}")
    assert rel <= SHELLSET_RTOL, (what, rel)
    return rel


def shells(batch_basis):
    from paper_2506_12501_amd import native
    return native.DeviceShells(batch_basis)
