"""The float prefilter of the six-dimensional sub-halo metric (used by the HIP kernel before
its FP64 test) must never decide differently from the FP64 definition of the metric (the
oracle's: squared norms summed ((c0*c0 + c1*c1) + c2*c2) in FP64, divided by the factors).
The kernel's float steps are replayed here with numpy float32 (no fused multiply-add) on
pairs drawn right at the threshold, across the box faces and near half the box, with
several factors (one of them infinite), and every pair it decides is checked."""
import numpy as np


def prefilter(xi, xj, L3, norm_x, norm_v, bb):
    """+1 (friends), 0 (not), -1 (left to the FP64 test): the kernel's float32 steps."""
    rx = np.float32(1.0 / norm_x)
    rv = np.float32(1.0 / norm_v)
    lo = np.float32(bb * (1.0 - 2.0 ** -16))
    hi = np.float32(bb * (1.0 + 2.0 ** -16))
    nowrap = (0.5 * L3 * (1.0 - 2.0 ** -20)).astype(np.float32)

    def ok(f):
        return f == 0.0 or 1e-15 <= f <= 1e15

    assert 1e-15 <= bb <= 1e15 and ok(rx) and ok(rv)
    d = (xi - xj).astype(np.float32)
    near_wrap = np.any(~(np.abs(d[:, :3]) < nowrap), axis=1)
    sq = (d * d).astype(np.float32)
    sx = ((sq[:, 0] + sq[:, 1]).astype(np.float32) + sq[:, 2]).astype(np.float32)
    sv = ((sq[:, 3] + sq[:, 4]).astype(np.float32) + sq[:, 5]).astype(np.float32)
    with np.errstate(invalid="ignore", over="ignore"):
        e = ((sx * rx).astype(np.float32) + (sv * rv).astype(np.float32)).astype(np.float32)
    out = np.where(e < lo, 1, np.where(e > hi, 0, -1))
    out[near_wrap] = -1
    return out


def exact(xi, xj, L3, norm_x, norm_v, bb):
    """The metric's FP64 definition (the oracle's steps), per pair."""
    d = xi.astype(np.float64) - xj.astype(np.float64)
    half = 0.5 * L3
    dx = np.where(d[:, :3] > half, d[:, :3] - L3, np.where(d[:, :3] < -half, d[:, :3] + L3,
                                                            d[:, :3]))
    dv = d[:, 3:]
    sx = (dx[:, 0] * dx[:, 0] + dx[:, 1] * dx[:, 1]) + dx[:, 2] * dx[:, 2]
    sv = (dv[:, 0] * dv[:, 0] + dv[:, 1] * dv[:, 1]) + dv[:, 2] * dv[:, 2]
    return sx / norm_x + sv / norm_v < bb


def test_subhalo_prefilter_agrees_with_the_fp64_metric():
    rng = np.random.default_rng(23)
    checked = 0
    cases = [((96.0, 96.0, 96.0), 0.04, 1.0, 1.0), ((96.0, 96.0, 96.0), 1.0, np.inf, 0.04),
             ((7.5, 9.0, 11.0), 0.3, 2.5, 0.7), ((3.0, 3.0, 3.0), 1e-3, 1e3, 1e-2),
             ((512.0, 512.0, 512.0), 5.0, 0.02, 3.0)]
    for L, nx, nv, b6 in cases:
        L3 = np.asarray(L, dtype=np.float64)
        bb = b6 * b6
        n = 20000
        xi = np.empty((n, 6), dtype=np.float32)
        xi[:, :3] = (rng.uniform(0, 1, (n, 3)) * L3).astype(np.float32)
        xi[:, 3:] = rng.normal(0, 2, (n, 3)).astype(np.float32)
        # partners at metric distance b6 (1 +- 1e-8 .. 1e-3): split d^2 between the two
        # terms, random directions, positions wrapped into the box
        t = rng.uniform(0, 1, n) if np.isfinite(nv) else np.ones(n)
        r2 = bb * (1.0 + rng.choice([-1, 1], n) * 10.0 ** rng.uniform(-8, -3, n))
        ux = rng.standard_normal((n, 3))
        ux /= np.linalg.norm(ux, axis=1, keepdims=True)
        uv = rng.standard_normal((n, 3))
        uv /= np.linalg.norm(uv, axis=1, keepdims=True)
        dx = ux * np.sqrt(t * r2 * nx)[:, None]
        dv = uv * np.sqrt((1 - t) * r2 * (nv if np.isfinite(nv) else 1.0))[:, None]
        xj = np.empty_like(xi)
        xj[:, :3] = ((xi[:, :3].astype(np.float64) + dx) % L3).astype(np.float32)
        xj[:, :3][xj[:, :3] >= L3.astype(np.float32)] = 0.0
        xj[:, 3:] = (xi[:, 3:].astype(np.float64) + dv).astype(np.float32)
        dec = prefilter(xi, xj, L3, nx, nv, bb)
        sel = dec >= 0
        assert np.array_equal(dec[sel] == 1, exact(xi[sel], xj[sel], L3, nx, nv, bb))
        checked += int(sel.sum())
        # one axis near half the box: left to the FP64 test or agreeing with it
        xk = xj.copy()
        xk[:, 0] = ((xi[:, 0].astype(np.float64) + L3[0] / 2 * (1 + rng.uniform(-1e-6, 1e-6, n)))
                    % L3[0]).astype(np.float32)
        dec = prefilter(xi, xk, L3, nx, nv, bb)
        sel = dec >= 0
        assert np.array_equal(dec[sel] == 1, exact(xi[sel], xk[sel], L3, nx, nv, bb))
    assert checked > 40000


def test_subhalo_prefilter_catches_a_dropped_term():
    """A replay that forgets the velocity term disagrees with the FP64 metric on such pairs:
    the comparison above would notice a prefilter that drops a term."""
    rng = np.random.default_rng(5)
    L3 = np.full(3, 96.0)
    n = 2000
    xi = np.zeros((n, 6), dtype=np.float32)
    xi[:, :3] = 10.0
    xj = xi.copy()
    xj[:, 0] += np.float32(0.1)
    xj[:, 3] += rng.uniform(0.5, 2.0, n).astype(np.float32)
    dec = prefilter(xi, xj, L3, 0.04, 1.0, 1.0)
    ex = exact(xi, xj, L3, 0.04, 1.0, 1.0)
    assert np.array_equal(dec[dec >= 0] == 1, ex[dec >= 0])
    no_v = exact(xi, xj, L3, 0.04, np.inf, 1.0)
    assert not np.array_equal(no_v, ex)
