"""Toy topology optimisation (paper Sec. 3.2): REINFORCE with the paper's Bernoulli form
(alpha = 0.5, S = 16 samples per step) inside an Adam loop lowers the toy loss."""
import numpy as np
import pytest

import workloads as W
from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def test_toy_loop_moves_mass_into_the_target():
    import torch
    from paper_2510_26851_amd.topology import halo_mass_loss, optimise

    # b = 0.4 of a mean spacing 1.05: the initial sampled graphs are below percolation, so
    # halos must be built (inside) rather than only shifted
    L, b, n = 12.0, 0.4, 1500
    pos = torch.from_numpy(W.uniform_box(n, (L,) * 3, 91)).cuda()
    inside = lambda c: c[:, 0] < L / 2            # Omega: the half-box x < L/2
    final, hist = optimise(pos, L, b, alpha=0.5, K=16, steps=60, lr=0.05, min_mass=5,
                           inside=inside, seed=7)
    say(f"toy loss: first {hist[:3]} last {hist[-3:]}")
    assert np.all(np.isfinite(hist))
    assert float(final.min()) >= 0.0 and float(final.max()) < L
    first, last = np.mean(hist[:5]), np.mean(hist[-5:])
    assert last < first - 0.5 * abs(first) - 50.0, (first, last)
    # the loss of the labels of a hard link on the final positions has the same sign pattern
    root = torch.arange(n, dtype=torch.int32, device="cuda").reshape(1, n)
    assert float(halo_mass_loss(final, root, L, 1, inside)[0]) == \
        float((final[:, 0] >= L / 2).sum() - (final[:, 0] < L / 2).sum())
