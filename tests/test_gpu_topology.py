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
    inside = lambda c: c[..., 0] < L / 2          # Omega: the half-box x < L/2
    final, hist = optimise(pos, L, b, alpha=0.5, K=16, steps=60, lr=0.05, min_mass=5,
                           inside=inside, seed=7)
    say(f"toy loss: first {hist[:3]} last {hist[-3:]}")
    assert np.all(np.isfinite(hist))
    assert float(final.min()) >= 0.0 and float(final.max()) < L
    first, last = np.mean(hist[:5]), np.mean(hist[-5:])
    assert last < first - 0.5 * abs(first) - 50.0, (first, last)
    # the toy loss of sampled graphs on the final positions, from the library's halo
    # tables, equals the oracle's: its sampled labels, catalogue and the same Omega test
    import oracle
    from oracle import reinforce as RF
    from paper_2510_26851_amd.reinforce import Sampler

    smp = Sampler(final, L, b, None, 8, 123, alpha=0.5)
    smp.sample()
    got = halo_mass_loss(smp.groups(5), inside).cpu().numpy()
    fpos = final.cpu().numpy()
    ei, ej, d2 = RF.candidate_edges(fpos, L, smp.r_cut)
    roots, _ = RF.sample_labels(n, ei, ej, RF.edge_prob_quadratic(d2, b, 0.5), 123, 8)
    for k in range(8):
        ref = oracle.groups(fpos, roots[k], L, 5)
        sign = np.where(ref["com"][:, 0] < L / 2, -1.0, 1.0)
        assert got[k] == float(np.sum(sign * ref["sizes"])), k
