"""The link predicate's edge cases on the GPU (paper Sec. 2 step (iv): friends when the
periodic minimum-image separation is below b; strict '<' on the double-precision squared
separation of the float32 coordinates).

Every hand case of ``golden/predicate_cases.txt`` (squared separation exactly b^2, one float
ulp either side, float32(0.4) against b = 0.4, pairs across a face or a corner, |d| = L/2)
is placed in a box of its own length and linking length, among filler particles that link
to nothing, and run through the library in several launch configurations: the LDS-tiled
kernel, the clique-cell (dense) passes, and the per-particle global search.  The pair's
decision must equal the file's, and every label the oracle's.  A cubic lattice with dyadic
spacing exactly b must fall apart into singletons, and be one group at the next double
above b, on the same paths."""
import os

import numpy as np
import pytest

import oracle
import workloads as W
from gpu_util import run_gpu, say

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "predicate_cases.txt")

# launch configurations: default (tiled for the 64^3 boxes), clique cells for every cell
# holding two particles or more, large cells with clique tables (per-particle search for the
# rest), and no tiles at all
TUNES = [None, dict(dense_threshold=1), dict(cell_side=4.0, dense_threshold=1),
         dict(cell_side=4.0, dense_threshold=8), dict(flags=1)]


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def golden_cases():
    out = []
    for line in open(GOLDEN):
        if not line.strip() or line.startswith("#"):
            continue
        f = line.split()
        xi = np.array(f[0:3], dtype=np.float32)
        xj = np.array(f[3:6], dtype=np.float32)
        L = tuple(float(v) for v in f[6:9])
        out.append((xi, xj, L, float(f[9]), int(f[10]), " ".join(f[11:])))
    return out


def with_filler(xi, xj, L):
    """The pair as particles 0 and 1, then a lattice of filler at spacing 2 on the odd
    integers (a boxes of side 64): filler within 1.25 of the pair (per axis, minimum image)
    is dropped, so the filler links to nothing."""
    pair = np.stack([xi, xj])
    if min(L) < 16.0:
        return pair
    g = np.arange(1.0, L[0], 2.0)
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    keep = np.ones(q.shape[0], bool)
    Lv = np.asarray(L)
    for p in pair.astype(np.float64):
        d = np.abs(q - p)
        d = np.minimum(d, Lv - d)
        keep &= ~np.all(d < 1.25, axis=1)
    return np.concatenate([pair, q[keep].astype(np.float32)])


@pytest.mark.parametrize("case", range(len(golden_cases())))
def test_golden_pairs_on_every_path(case):
    xi, xj, L, b, expect, why = golden_cases()[case]
    pos = with_filler(xi, xj, L)
    ref, _ = oracle.fof(pos, L, b)
    assert (ref[0] == ref[1]) == bool(expect), why
    assert np.sum(ref == ref[0]) == (2 if expect else 1)     # the filler links to nothing
    for tune in TUNES:
        say(f"golden case {case} ({why}) n={pos.shape[0]} tune={tune}")
        root, g, status = run_gpu(pos, L, b, 2, tune=tune)
        assert status == 0
        np.testing.assert_array_equal(root, ref)
        assert g["n_groups"] == (1 if expect else 0)


@pytest.mark.parametrize("tune", [None, dict(cell_side=1.5, dense_threshold=4), dict(flags=1)])
def test_lattice_at_exactly_b(tune):
    """Spacing 0.375 (dyadic, so the float32 lattice is exact): at b = 0.375 every neighbour
    distance squared equals b^2 and nothing links; at the next double above 0.375 every
    axis neighbour links and the lattice is one group."""
    m, a = 32, 0.375
    pos = W.cubic_lattice(m, a)
    L = m * a
    say(f"lattice at b = spacing, tune={tune}")
    root, g, status = run_gpu(pos, L, a, 1, tune=tune)
    assert status == 0
    np.testing.assert_array_equal(root, np.arange(m ** 3))
    b_up = float(np.nextafter(a, 1.0))
    say(f"lattice at b = nextafter(spacing), tune={tune}")
    root, g, status = run_gpu(pos, L, b_up, 1, tune=tune)
    assert status == 0
    assert np.all(root == 0) and g["n_groups"] == 1 and g["sizes"][0] == m ** 3
