"""Pins of the multi-threaded oracle labelling (``oracle.fof_par``), without a GPU.

It must give exactly the serial definition's labels and link count: against the O(N^2)
brute force with a library connected-components routine on small inputs, and against
``oracle.fof`` (itself pinned in ``test_oracle.py``) on boxes large enough that many
threads merge trees concurrently, at several thread counts.  Closed lattice cases and
degenerate inputs (empty box, one point, every particle at one point, fewer than three
cells per axis) are checked as well.
"""
import numpy as np
import pytest

import oracle
import workloads as W
from test_oracle import brute_labels, check_partition_invariants


@pytest.mark.parametrize("seed,n,L,b", [
    (1, 500, 10.0, 0.6),
    (3, 2000, (12.0, 9.0, 20.0), 0.7),
    (6, 200, 1.0, 0.4),        # two cells per axis: duplicate neighbours merged
    (8, 50, (0.7, 3.0, 5.0), 0.34),
])
@pytest.mark.parametrize("threads", [1, 3, 8])
def test_par_matches_brute_force(seed, n, L, b, threads):
    pos = W.uniform_box(n, np.broadcast_to(L, (3,)), seed)
    ref, nlinks = brute_labels(pos, L, b)
    got, nl = oracle.fof_par(pos, L, b, threads=threads)
    assert nl == nlinks
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("threads", [2, 8])
def test_par_matches_brute_force_clumpy(threads):
    pos = W.clumpy_box(2000, 24.0, 6, 11)
    ref, nlinks = brute_labels(pos, 24.0, 0.5)
    got, nl = oracle.fof_par(pos, 24.0, 0.5, threads=threads)
    assert nl == nlinks
    np.testing.assert_array_equal(got, ref)


@pytest.mark.parametrize("threads", [2, 5, 8])
def test_par_equals_serial_on_clumped_boxes(threads):
    """Many concurrent merges: 32768-particle clumped box (the small workload) and a
    denser 200k-particle one whose clumps span many cells."""
    box = W.config0()
    ref, nl_ref = oracle.fof(box.pos, box.L, box.b)
    got, nl = oracle.fof_par(box.pos, box.L, box.b, threads=threads)
    assert nl == nl_ref
    np.testing.assert_array_equal(got, ref)
    pos = W.clumpy_box(200_000, 40.0, 300, 7)
    ref, nl_ref = oracle.fof(pos, 40.0, 0.3)
    got, nl = oracle.fof_par(pos, 40.0, 0.3, threads=threads)
    assert nl == nl_ref
    np.testing.assert_array_equal(got, ref)
    check_partition_invariants(got)


def test_par_repeatable():
    pos = W.clumpy_box(100_000, 30.0, 200, 3)
    a, _ = oracle.fof_par(pos, 30.0, 0.3, threads=8)
    for _ in range(3):
        b, _ = oracle.fof_par(pos, 30.0, 0.3, threads=8)
        np.testing.assert_array_equal(a, b)


def test_par_lattices_closed_forms():
    pos = W.cubic_lattice(16, 0.375)           # spacing 0.375 < b = 0.4: one group
    root, nl = oracle.fof_par(pos, 6.0, 0.4, threads=8)
    assert np.all(root == 0)
    assert nl == 3 * 16 ** 3
    pos = W.cubic_lattice(16, 0.4375)          # spacing 0.4375 > b: all singletons
    root, nl = oracle.fof_par(pos, 7.0, 0.4, threads=8)
    np.testing.assert_array_equal(root, np.arange(pos.shape[0]))
    assert nl == 0


def test_par_degenerate_inputs():
    root, nl = oracle.fof_par(np.zeros((0, 3), np.float32), 10.0, 0.5, threads=4)
    assert root.shape == (0,) and nl == 0
    root, nl = oracle.fof_par(np.array([[1.0, 2.0, 3.0]], np.float32), 10.0, 0.5, threads=4)
    np.testing.assert_array_equal(root, [0]) and nl == 0
    n = 3000                                   # every particle at one point: one clique
    pos = np.full((n, 3), 2.5, np.float32)
    root, nl = oracle.fof_par(pos, 10.0, 0.5, threads=8)
    assert np.all(root == 0) and nl == n * (n - 1) // 2
    with pytest.raises(oracle.OracleError):
        oracle.fof_par(np.array([[10.0, 0.0, 0.0]], np.float32), 10.0, 0.5)


def test_max_threads_positive():
    assert oracle.max_threads() >= 1
