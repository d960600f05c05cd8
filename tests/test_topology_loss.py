"""The toy topology loss (paper Sec. 3.2) on hand-made halo tables, on the CPU: the signed
sum of halo masses, negative inside Omega, over the groups each sample's table holds."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")


def test_halo_mass_loss_hand_cases():
    from paper_2510_26851_amd.topology import halo_mass_loss

    # sample 0: a 3-member halo at x = 1 (inside Omega: x < 5) and a 4-member one at x = 9.95
    # (outside); sample 1: three halos (3 inside, 2 outside, 2 inside across the x = 0 face)
    # and an unused table row that must not count
    halos = dict(
        cap=4,
        n_groups=torch.tensor([2, 3], dtype=torch.int32),
        sizes=torch.tensor([[3, 4, 99, 99], [3, 2, 2, 99]], dtype=torch.int32),
        com=torch.tensor([[[1.0, 1.0, 1.0], [9.95, 5.0, 5.0], [0.0] * 3, [0.0] * 3],
                          [[1.0, 1.0, 1.0], [9.85, 5.0, 5.0], [0.05, 5.05, 5.0], [9.0] * 3]],
                         dtype=torch.float64))
    inside = lambda c: c[..., 0] < 5.0
    np.testing.assert_array_equal(halo_mass_loss(halos, inside).numpy(), [1.0, -3.0])
    # no groups at all
    empty = dict(halos, n_groups=torch.tensor([0, 0], dtype=torch.int32))
    np.testing.assert_array_equal(halo_mass_loss(empty, inside).numpy(), [0.0, 0.0])


def test_sum_sq_sizes_counts_only_table_groups():
    from paper_2510_26851_amd.reinforce import sum_sq_sizes

    halos = dict(cap=3, n_groups=torch.tensor([1, 3, 0], dtype=torch.int32),
                 sizes=torch.tensor([[5, 7, 7], [2, 3, 4], [9, 9, 9]], dtype=torch.int32),
                 com=torch.zeros((3, 3, 3), dtype=torch.float64))
    np.testing.assert_array_equal(sum_sq_sizes(halos).numpy(), [25.0, 29.0, 0.0])
