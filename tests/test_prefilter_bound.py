"""The float prefilter of the link predicate (used by the HIP kernels before the exact double
test) must never decide differently from the exact predicate.  Its bounds are derived in
the kernel source; here the same float32 arithmetic is replayed with numpy (no fused
multiply-add) on pairs drawn right at the linking length and near L/2, and every pair it
decides is compared with the oracle's double predicate."""
import numpy as np

import oracle


def prefilter(xi, xj, L, b):
    """Returns +1 (link), 0 (no link) or -1 (left to the double test), float32 steps."""
    halfL = 0.5 * np.asarray(L, dtype=np.float64)
    nowrap = (halfL * (1.0 - 2.0 ** -20)).astype(np.float32)
    b2 = b * b
    b2lo = np.float32(b2 * (1.0 - 2.0 ** -18))
    b2hi = np.float32(b2 * (1.0 + 2.0 ** -18))
    d = (xi.astype(np.float32) - xj.astype(np.float32)).astype(np.float32)
    near = np.all(np.abs(d) < nowrap, axis=-1)
    sq = (d * d).astype(np.float32)
    s = ((sq[..., 0] + sq[..., 1]).astype(np.float32) + sq[..., 2]).astype(np.float32)
    out = np.full(s.shape, -1, dtype=np.int64)
    out[near & (s < b2lo)] = 1
    out[near & (s > b2hi)] = 0
    return out


def exact(xi, xj, L, b):
    return np.array([oracle.dist2(a, c, L) < b * b for a, c in zip(xi, xj)])


def test_prefilter_agrees_with_the_double_predicate():
    rng = np.random.default_rng(11)
    checked = 0
    for L, b in [(64.0, 0.4), (512.0, 0.2), ((7.5, 9.0, 11.0), 0.37), (3.0, 1.2)]:
        L3 = np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))
        n = 20000
        xi = (rng.uniform(0, 1, (n, 3)) * L3).astype(np.float32)
        # partners at distance b (1 +- 1e-6 .. 1e-3) in random directions, some across the box
        u = rng.standard_normal((n, 3))
        u /= np.linalg.norm(u, axis=1, keepdims=True)
        r = b * (1.0 + rng.choice([-1, 1], n) * 10.0 ** rng.uniform(-7, -3, n))
        xj64 = (xi.astype(np.float64) + u * r[:, None]) % L3
        xj = xj64.astype(np.float32)
        xj[xj >= L3.astype(np.float32)] = 0.0
        dec = prefilter(xi, xj, L3, b)
        sel = dec >= 0
        ex = exact(xi[sel], xj[sel], tuple(L3), b)
        assert np.array_equal(dec[sel] == 1, ex)
        checked += int(sel.sum())
        # pairs near half the box on one axis: either left to the double test or agreeing
        xk = xi.copy()
        xk[:, 0] = ((xi[:, 0].astype(np.float64) + L3[0] / 2 * (1 + rng.uniform(-1e-6, 1e-6, n)))
                    % L3[0]).astype(np.float32)
        dec = prefilter(xi, xk, L3, b)
        sel = dec >= 0
        assert np.array_equal(dec[sel] == 1, exact(xi[sel], xk[sel], tuple(L3), b))
    assert checked > 50000


def test_coarse_index_by_multiply_high_is_exact():
    """The kernels take the coarse index f / m of a fine index f as the high word of
    f * ceil(2^32 / m) (m = 2..10 fine cells per coarse cell).  Exact for every fine index a
    box can have (nf <= 10 * 2^20), checked here for all of them."""
    import numpy as np

    f = np.arange(10 * 2 ** 20 + 1, dtype=np.uint64)
    for m in range(2, 11):
        M = np.uint64(((1 << 32) + m - 1) // m)
        np.testing.assert_array_equal((f * M) >> np.uint64(32), f // np.uint64(m))
