"""Seeded synthetic particle workloads for the Friends-of-Friends hot path.

These generators stand in for the paper's fastPM boxes (500 Mpc/h, 64^3..512^3 particles,
Sec. 2) and its b = 0.2 linking parameter (Sec. 3.1).  None of the paper's data is used.
They hold none of the halo finder's arithmetic: they only draw positions (and velocities)
and wrap them into the periodic box.  Both the CPU oracle and the GPU path consume the
arrays produced here.

Every array is drawn from ``numpy.random.default_rng(26851 + config)`` (PCG64) in the draw
order documented on each function.  Positions are built in float64, wrapped into [0, L),
cast to float32, and any float32 value that rounds to >= L is mapped to 0 so that every
coordinate satisfies 0 <= x < L exactly (the library rejects anything else).

Configurations (sizes as in the workload table of the design notes):
  0  clumps:     32768 particles, L = 64, b = 0.4, 50% uniform + 50% in 40 Gaussian clumps
  1  zeldovich:  256^3 lattice, L = 256, b = 0.2, displacement rms 0.5 spacing
  2  zeldovich:  512^3 lattice, L = 512, b = 0.2, rms 0.8 + 50,000 NFW clumps
  3  zeldovich:  128^3 lattice, L = 128, b = 0.2, rms 0.5, Gaussian velocities (sigma = 1)
  4  batch:      256 boxes, N_b log-uniform in [16^3, 128^3], clump generator per box
  5  zeldovich:  1024^3 lattice, L = 1024, b = 0.2, rms 0.8 + 400,000 NFW clumps (the 512^3
                 recipe at eight times the volume; about 80 GB of host memory while drawn)
"""
from __future__ import annotations

import dataclasses
import math
import os

import numpy as np

SEED_BASE = 26851
REINFORCE_SEED = SEED_BASE + 100


@dataclasses.dataclass
class Box:
    """One periodic box: float32 positions [n, 3] in [0, L) and the physical linking length."""
    pos: np.ndarray
    L: tuple
    b: float
    min_size: int
    vel: np.ndarray | None = None
    name: str = ""

    @property
    def n(self) -> int:
        return int(self.pos.shape[0])


def _threads() -> int:
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        n = os.cpu_count() or 1
    return max(1, min(16, n))


def wrap_to_f32(x64: np.ndarray, L) -> np.ndarray:
    """Wrap float64 coordinates into [0, L) and cast to float32 with every value < L."""
    L = np.asarray(L, dtype=np.float64).reshape(1, -1)
    x = np.mod(x64, L)
    x32 = x.astype(np.float32)
    bad = x32.astype(np.float64) >= L
    if bad.any():
        x32[bad] = 0.0
    return np.ascontiguousarray(x32)


def linking_length(bdim: float, L: float, n: int) -> float:
    """Physical linking length b * (V/N)^(1/3) for a cube, computed once on the host.

    Perfect cubes use the exact integer cube root so that e.g. 0.2*64/32 is exactly 0.4.
    """
    r = round(n ** (1.0 / 3.0))
    for c in (r - 1, r, r + 1):
        if c > 0 and c * c * c == n:
            return bdim * L / c
    return bdim * L / float(np.cbrt(n))


# --------------------------------------------------------------------------------------
# Gaussian-clump generator (config 0 and the per-box generator of config 4)
# --------------------------------------------------------------------------------------
def clump_positions(rng: np.random.Generator, n: int, L: float, n_clumps: int) -> np.ndarray:
    """Half uniform, half in Gaussian clumps; returns float64 [n, 3] (unwrapped).

    Draw order: uniform positions (n_uni, 3); clump centres (n_clumps, 3); clump sigma
    log-uniform on [0.2, 1.0] (n_clumps); member offsets standard normal (n_clump_members, 3).
    Clump members are shared equally, the first (members % n_clumps) clumps taking one more.
    """
    n_uni = n - n // 2
    n_mem = n // 2
    uni = rng.random((n_uni, 3)) * L
    centres = rng.random((n_clumps, 3)) * L
    sigma = np.exp(rng.uniform(math.log(0.2), math.log(1.0), n_clumps))
    counts = np.full(n_clumps, n_mem // n_clumps, dtype=np.int64)
    counts[: n_mem % n_clumps] += 1
    owner = np.repeat(np.arange(n_clumps), counts)
    off = rng.standard_normal((n_mem, 3))
    mem = centres[owner] + off * sigma[owner, None]
    return np.concatenate([uni, mem], axis=0)


def config0() -> Box:
    rng = np.random.default_rng(SEED_BASE + 0)
    n, L = 32768, 64.0
    x = clump_positions(rng, n, L, 40)
    return Box(wrap_to_f32(x, (L, L, L)), (L, L, L), linking_length(0.2, L, n), 20,
               name="clumps-32768-L64")


# --------------------------------------------------------------------------------------
# Zel'dovich lattice generator (configs 1-3)
# --------------------------------------------------------------------------------------
def _say(progress, msg):
    if progress is not None:
        progress(msg)


def zeldovich_displacement(rng: np.random.Generator, n: int, rms: float,
                           progress=None) -> np.ndarray:
    """Displacement field psi on an n^3 lattice (spacing 1) with P_psi(k) ~ k^-2.

    White noise w -> w_hat; psi_hat = i k w_hat / k^2 (so div psi = -delta with a white
    delta); k = 0 and every Nyquist plane are zeroed; psi is rescaled so that the vector rms
    sqrt(<|psi|^2>) equals ``rms``.  Returns float64 [n^3, 3] in lattice C order.
    """
    import scipy.fft as sfft

    w = rng.standard_normal((n, n, n))
    _say(progress, "white noise drawn")
    wk = sfft.rfftn(w, workers=_threads())
    _say(progress, "forward FFT done")
    del w
    k1 = 2.0 * np.pi * np.fft.fftfreq(n)
    kz1 = 2.0 * np.pi * np.fft.rfftfreq(n)
    kx = k1[:, None, None]
    ky = k1[None, :, None]
    kz = kz1[None, None, :]
    k2 = kx * kx + ky * ky + kz * kz
    k2[0, 0, 0] = 1.0
    wk /= k2
    wk[0, 0, 0] = 0.0
    if n % 2 == 0:
        wk[n // 2, :, :] = 0.0
        wk[:, n // 2, :] = 0.0
        wk[:, :, n // 2] = 0.0
    psi = np.empty((n * n * n, 3), dtype=np.float64)
    for c, kc in enumerate((kx, ky, kz)):
        comp = sfft.irfftn(1j * kc * wk, s=(n, n, n), workers=_threads())
        psi[:, c] = comp.reshape(-1)
        del comp
        _say(progress, f"displacement component {c} done")
    del wk
    cur = math.sqrt(float(np.mean(np.sum(psi * psi, axis=1))))
    psi *= rms / cur
    return psi


def lattice(n: int) -> np.ndarray:
    """Lagrangian lattice q = (i + 1/2, j + 1/2, k + 1/2), index (i*n + j)*n + k."""
    g = np.arange(n, dtype=np.float64) + 0.5
    q = np.empty((n, n, n, 3), dtype=np.float64)
    q[..., 0] = g[:, None, None]
    q[..., 1] = g[None, :, None]
    q[..., 2] = g[None, None, :]
    return q.reshape(-1, 3)


def nfw_radius(u: np.ndarray, c: float) -> np.ndarray:
    """Inverse enclosed-mass CDF of an NFW profile truncated at x = c, in units of r_s.

    m(x) = ln(1+x) - x/(1+x); solve m(x) = u*m(c) with x = -1/W0(-exp(-m-1)) - 1.
    """
    from scipy.special import lambertw

    mc = math.log1p(c) - c / (1.0 + c)
    m = u * mc
    w = lambertw(-np.exp(-m - 1.0), 0).real
    return -1.0 / w - 1.0


def config_zeldovich(cfg: int, n: int, rms: float, *, with_vel: bool = False,
                     n_nfw: int = 0, progress=None) -> Box:
    """Draw order: white noise (n^3); [velocities (n^3, 3)]; then for the NFW clumps:
    centres (n_nfw, 3), r200 log-uniform on [0.5, 3] (n_nfw), member counts from the
    truncated power law dN/dn ~ n^-2 on [100, 1e4] (n_nfw), a permutation of all particles
    (the first sum(counts) become clump members, clump by clump), member radii u (members),
    member directions standard normal (members, 3)."""
    rng = np.random.default_rng(SEED_BASE + cfg)
    L = float(n)
    psi = zeldovich_displacement(rng, n, rms, progress)
    x = lattice(n)
    x += psi
    del psi
    _say(progress, "lattice displaced")
    vel = None
    if with_vel:
        vel = rng.standard_normal((n * n * n, 3)).astype(np.float32)
    if n_nfw:
        centres = rng.random((n_nfw, 3)) * L
        r200 = np.exp(rng.uniform(math.log(0.5), math.log(3.0), n_nfw))
        lo, hi = 100.0, 1e4
        u = rng.random(n_nfw)
        cnt = np.rint(1.0 / (1.0 / lo - u * (1.0 / lo - 1.0 / hi))).astype(np.int64)
        total = int(cnt.sum())
        perm = rng.permutation(n * n * n)[:total]
        _say(progress, "clump members chosen")
        rad = nfw_radius(rng.random(total), 10.0)
        owner = np.repeat(np.arange(n_nfw), cnt)
        rad *= (r200 / 10.0)[owner]
        d = rng.standard_normal((total, 3))
        d /= np.sqrt(np.sum(d * d, axis=1))[:, None]
        x[perm] = centres[owner] + d * rad[:, None]
        del perm, rad, owner, d
        _say(progress, "clumps placed")
    b = linking_length(0.2, L, n ** 3)
    names = {1: "zeldovich-256^3", 2: "zeldovich-nfw-512^3", 3: "zeldovich-128^3-vel",
             5: "zeldovich-nfw-1024^3"}
    pos = wrap_to_f32(x, (L, L, L))
    del x
    _say(progress, "wrapped to float32")
    return Box(pos, (L, L, L), b, 2 if with_vel else 20, vel=vel,
               name=names.get(cfg, f"zeldovich-{n}^3"))


def config1() -> Box:
    return config_zeldovich(1, 256, 0.5)


def config2() -> Box:
    return config_zeldovich(2, 512, 0.8, n_nfw=50000)


def config5(progress=None) -> Box:
    return config_zeldovich(5, 1024, 0.8, n_nfw=400000, progress=progress)


def config3() -> Box:
    return config_zeldovich(3, 128, 0.5, with_vel=True)


# REINFORCE settings of config 3: tau = 0.05 b, candidate cut r_c = b + 10 tau, K samples.
CONFIG3_TAU_FRAC = 0.05
CONFIG3_K = 64


# --------------------------------------------------------------------------------------
# Batched boxes (config 4)
# --------------------------------------------------------------------------------------
def config4(nbox: int = 256, n_lo: int = 16 ** 3, n_hi: int = 128 ** 3) -> list:
    """Draw order: all box sizes first (log-uniform, rounded), then each box in turn with
    ``clump_positions`` (clump count round(40 N_b / 32768), at least 1)."""
    rng = np.random.default_rng(SEED_BASE + 4)
    sizes = np.rint(np.exp(rng.uniform(math.log(n_lo), math.log(n_hi), nbox))).astype(np.int64)
    boxes = []
    for i, nb in enumerate(sizes):
        nb = int(nb)
        cb = float(np.cbrt(nb))
        L = 2.0 * cb
        b = 0.2 * L / cb
        ncl = max(1, int(round(40 * nb / 32768)))
        x = clump_positions(rng, nb, L, ncl)
        boxes.append(Box(wrap_to_f32(x, (L, L, L)), (L, L, L), b, 20, name=f"box{i}"))
    return boxes


def make(cfg: int, progress=None, cache_dir=None):
    """Configuration `cfg` (0-5).  With `cache_dir`, single-box configurations are stored
    there as .npy files on first use and loaded afterwards (drawing 512^3 takes minutes)."""
    if cache_dir and cfg != 4:
        return _cached(cfg, progress, cache_dir)
    if cfg == 5:
        return config5(progress)
    return {0: config0, 1: config1, 2: config2, 3: config3, 4: config4}[cfg]()


def _cached(cfg: int, progress, cache_dir) -> Box:
    import json

    stem = os.path.join(cache_dir, f"config{cfg}")
    try:
        with open(stem + ".json") as f:
            meta = json.load(f)
        pos = np.load(stem + ".pos.npy", mmap_mode=None)
        vel = np.load(stem + ".vel.npy") if meta["has_vel"] else None
        _say(progress, f"loaded {stem}")
        return Box(pos, tuple(meta["L"]), meta["b"], meta["min_size"], vel=vel, name=meta["name"])
    except (OSError, ValueError, KeyError):
        pass
    box = make(cfg, progress)
    os.makedirs(cache_dir, exist_ok=True)
    np.save(stem + ".pos.npy", box.pos)
    if box.vel is not None:
        np.save(stem + ".vel.npy", box.vel)
    with open(stem + ".json", "w") as f:
        json.dump(dict(L=list(box.L), b=box.b, min_size=box.min_size, name=box.name,
                       has_vel=box.vel is not None), f)
    return box


# --------------------------------------------------------------------------------------
# Small structured inputs for tests
# --------------------------------------------------------------------------------------
def phase_space_hosts(n_hosts: int, L: float, seed: int, n_sub: int = 3,
                      members=(30, 400), n_background: int = 0):
    """Hosts made of sub-clumps that overlap in space but move apart in velocity, for the
    six-dimensional sub-halo pass (a stand-in for the paper's CAMELS halos).

    Draw order: host centres (n_hosts, 3) uniform in [0, L); member counts (n_hosts, n_sub)
    integers in [members[0], members[1]]; sub-clump offsets (n_hosts, n_sub, 3) normal with
    sigma 0.25; bulk velocities (n_hosts, n_sub, 3) normal with sigma 4; then per sub-clump,
    in order, member positions normal about its centre (sigma 0.12) and member velocities
    normal about its bulk velocity (sigma 0.3); finally n_background uniform positions with
    normal velocities (sigma 1).  Returns (pos float32 [n, 3], vel float32 [n, 3])."""
    rng = np.random.default_rng(seed)
    centres = rng.random((n_hosts, 3)) * L
    counts = rng.integers(members[0], members[1], (n_hosts, n_sub), endpoint=True)
    offs = rng.normal(0.0, 0.25, (n_hosts, n_sub, 3))
    bulk = rng.normal(0.0, 4.0, (n_hosts, n_sub, 3))
    xs, vs = [], []
    for h in range(n_hosts):
        for k in range(n_sub):
            c = int(counts[h, k])
            xs.append(centres[h] + offs[h, k] + rng.normal(0.0, 0.12, (c, 3)))
            vs.append(bulk[h, k] + rng.normal(0.0, 0.3, (c, 3)))
    if n_background:
        xs.append(rng.random((n_background, 3)) * L)
        vs.append(rng.normal(0.0, 1.0, (n_background, 3)))
    x = np.concatenate(xs)
    v = np.concatenate(vs).astype(np.float32)
    return wrap_to_f32(x, (L, L, L)), v


def uniform_box(n: int, L, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    L = np.asarray(L, dtype=np.float64).reshape(1, 3)
    return wrap_to_f32(rng.random((n, 3)) * L, L)


def clumpy_box(n: int, L: float, n_clumps: int, seed: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return wrap_to_f32(clump_positions(rng, n, L, n_clumps), (L, L, L))


def cubic_lattice(m: int, a: float, origin: float = 0.0) -> np.ndarray:
    """m^3 simple-cubic lattice with spacing a (use dyadic a so that the float32 lattice is
    exactly uniform); box side m*a."""
    g = origin + a * np.arange(m, dtype=np.float64)
    q = np.stack(np.meshgrid(g, g, g, indexing="ij"), axis=-1).reshape(-1, 3)
    return wrap_to_f32(q, (m * a,) * 3)
