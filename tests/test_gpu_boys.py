"""mdx_boys on the GPU vs the CPU oracle (and closed forms)."""
import math

import numpy as np
import pytest

from oracle import oracle as O

pytestmark = pytest.mark.gpu

X_EDGE = [0.0, 1e-300, 1e-15, 1e-8, 0.0625 - 1e-12, 0.0625, 0.5, 1.0, 2.0, 10.0, 29.9, 36.0, 44.9375,
          44.99999999, 45.0, 45.000001, 50.0, 117.9, 118.0, 1e3, 1e5, 1e7, 1e12]


@pytest.mark.parametrize("mmax", [0, 1, 8, 16, 25, 32])
def test_boys_vs_oracle(mmax):
    import torch
    from paper_2506_12501_amd import native
    rng = np.random.default_rng(mmax)
    x = np.concatenate([X_EDGE, rng.uniform(0, 60, 2000), np.exp(rng.uniform(-20, 16, 500))])
    F = native.boys(torch.as_tensor(x, device="cuda"), mmax).cpu().numpy()
    ref = O.boys(x, mmax)
    rel = np.abs(F - ref) / np.maximum(np.abs(ref), 1e-300)
    assert np.all(np.isfinite(F))
    assert rel.max() < 5e-15, (rel.max(), np.unravel_index(np.argmax(rel), rel.shape))


def test_boys_closed_forms_on_gpu():
    import torch
    from paper_2506_12501_amd import native
    x = np.array([1e-3, 0.7, 3.0, 17.0, 44.0, 46.0, 400.0])
    F = native.boys(torch.as_tensor(x, device="cuda"), 3).cpu().numpy()
    f0 = np.array([math.sqrt(math.pi / (4 * v)) * math.erf(math.sqrt(v)) for v in x])
    assert np.allclose(F[0], f0, rtol=4e-16, atol=0)
    F0 = native.boys(torch.zeros(5, dtype=torch.float64, device="cuda"), 32).cpu().numpy()
    assert np.allclose(F0[:, 0], 1.0 / (2 * np.arange(33) + 1), rtol=2e-16, atol=0)


def test_boys_empty_and_errors():
    import torch
    from paper_2506_12501_amd import native
    F = native.boys(torch.zeros(0, dtype=torch.float64, device="cuda"), 4)
    assert F.shape == (5, 0)
    with pytest.raises(native.MdxError) as e:
        native.boys(torch.zeros(3, dtype=torch.float64, device="cuda"), 33)
    assert e.value.status == native.MDX_EUNSUPPORTED
