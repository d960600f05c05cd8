"""The soft histogram used for derivatives of a histogram of halo decorations (paper
Sec. 3.1): limits, totals and its gradient (CPU, float64)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def _soft():
    from paper_2510_26851_amd.autograd import soft_histogram
    return soft_histogram


def test_narrow_bins_give_the_ordinary_histogram():
    soft = _soft()
    rng = np.random.default_rng(5)
    v = rng.uniform(0.0, 10.0, 400)
    edges = np.linspace(0.0, 10.0, 11)
    v = v[np.min(np.abs(v[:, None] - edges[None]), axis=1) > 1e-3]  # away from every edge
    h = soft(torch.from_numpy(v), torch.from_numpy(edges), 1e-6).numpy()
    np.testing.assert_allclose(h, np.histogram(v, edges)[0], atol=1e-9)


def test_total_and_gradient():
    soft = _soft()
    v = torch.tensor([0.5, 1.9, 2.05, 3.3], dtype=torch.float64, requires_grad=True)
    edges = torch.tensor([-10.0, 1.0, 2.0, 3.0, 20.0], dtype=torch.float64)
    h = soft(v, edges, 0.1)
    # bins covering far beyond every value: the soft counts add up to the number of values
    assert abs(float(h.sum()) - 4.0) < 1e-12
    w = torch.tensor([0.3, -1.0, 2.0, 0.5], dtype=torch.float64)
    assert torch.autograd.gradcheck(lambda x: (soft(x, edges, 0.1) * w).sum(), (v,))
