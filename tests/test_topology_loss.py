"""The toy topology loss (paper Sec. 3.2): hand cases on the CPU."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_halo_mass_loss_hand_cases():
    from paper_2510_26851_amd.topology import halo_mass_loss

    L = 10.0
    # halo A (3 members) around (1, 1, 1); halo B (4 members) across the x = 0 face near
    # (9.9, 5, 5); one lone particle
    pos = torch.tensor([[1.0, 1.0, 1.0], [1.1, 1.0, 1.0], [1.0, 1.1, 1.0],
                        [9.8, 5.0, 5.0], [9.9, 5.0, 5.0], [0.1, 5.0, 5.0], [0.0, 5.1, 5.0],
                        [5.0, 5.0, 9.0]], dtype=torch.float32)
    root = torch.tensor([[0, 0, 0, 3, 3, 3, 3, 7],
                         [0, 0, 0, 3, 3, 5, 5, 7]], dtype=torch.int32)
    inside = lambda c: c[:, 0] < 5.0          # Omega: x < 5
    out = halo_mass_loss(pos, root, L, 2, inside).numpy()
    # sample 0: A (3, inside) and B (4; centre x = 9.95, outside): 4 - 3
    # sample 1: A inside, {3, 4} at x = 9.85 outside, {5, 6} at x = 0.05 inside: 2 - 3 - 2
    np.testing.assert_array_equal(out, [1.0, -3.0])
    # a mass cut of 3 drops the pairs
    np.testing.assert_array_equal(halo_mass_loss(pos, root, L, 3, inside).numpy(), [1.0, -3.0])
    np.testing.assert_array_equal(halo_mass_loss(pos, root, L, 4, inside).numpy(), [4.0, 0.0])
