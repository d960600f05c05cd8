"""CPU oracle for the Friends-of-Friends hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` may
import this package.  The product library never calls it, and it shares no code with the
GPU library (``fof_oracle.c`` is a separate plain-C implementation written from the paper).

Functions and the passages they follow (paper section / algorithm):
  linked, dist2          Sec. 2 step (iv) link criterion, minimum image; fixed FP64 reading
  fof                    Sec. 2 steps (i)-(v); Alg. 2 (cell list, labels = min index)
  fof_par                the same labels with the pair enumeration on OpenMP threads
  groups                 Sec. 2 step (vi) / Alg. 2 compaction; Sec. 3.1 halo position
  frozen_backward        Sec. 3.1 frozen assignment (gradients with memberships fixed)
  group_dispersion,
  dispersion_backward    Sec. 3.1 decorated frozen assignment: the particle standard
                         deviation of each halo as the decoration, and its gradient
  component              BFS closure of one particle under the same predicate (sampled checks)
  subhalos               Sec. 2 sub-halo finding: a second, six-dimensional pass inside
                         each host halo with the phase-space distance of that passage
  philox4x64, uniforms,
  candidate_edges,
  sample_labels,
  reinforce_enumerate    Sec. 3.2 REINFORCE estimator (see ``reinforce.py``)

Every function here is pinned by the ``-m "not gpu"`` tests in ``tests/test_oracle_*.py``
against brute force, library routines, closed forms and hand cases.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fof_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

CFLAGS = ["-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared", "-std=c11"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (IEEE double, no FMA contraction)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", *CFLAGS, "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(build())
        P = ctypes.c_void_p
        i64, i32, dbl = ctypes.c_int64, ctypes.c_int32, ctypes.c_double
        _lib.oracle_dist2.argtypes = [P, P, P]
        _lib.oracle_dist2.restype = dbl
        _lib.oracle_linked.argtypes = [P, P, P, dbl]
        _lib.oracle_linked.restype = ctypes.c_int
        _lib.oracle_fof.argtypes = [i64, P, P, dbl, P]
        _lib.oracle_fof.restype = i64
        _lib.oracle_fof_par.argtypes = [i64, P, P, dbl, P, ctypes.c_int]
        _lib.oracle_fof_par.restype = i64
        _lib.oracle_max_threads.argtypes = []
        _lib.oracle_max_threads.restype = ctypes.c_int
        _lib.oracle_index_build.argtypes = [i64, P, P, dbl]
        _lib.oracle_index_build.restype = P
        _lib.oracle_index_free.argtypes = [P]
        _lib.oracle_index_free.restype = None
        _lib.oracle_component.argtypes = [P, i64, P, i64, P]
        _lib.oracle_component.restype = i64
        _lib.oracle_groups.argtypes = [i64, P, P, P, P, i32, i32, P, P, P, P, P, P]
        _lib.oracle_groups.restype = ctypes.c_int
        _lib.oracle_frozen_backward.argtypes = [i64, P, P, i32, P, P, P, P, P, P, P, P]
        _lib.oracle_frozen_backward.restype = ctypes.c_int
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _pos(pos):
    pos = np.ascontiguousarray(pos, dtype=np.float32)
    assert pos.ndim == 2 and pos.shape[1] == 3
    return pos


def _L(L):
    L = np.ascontiguousarray(np.broadcast_to(np.asarray(L, dtype=np.float64), (3,)))
    return L


class OracleError(RuntimeError):
    pass


def dist2(xi, xj, L) -> float:
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    xj = np.ascontiguousarray(xj, dtype=np.float32)
    return lib().oracle_dist2(_ptr(xi), _ptr(xj), _ptr(_L(L)))


def linked(xi, xj, L, b) -> bool:
    xi = np.ascontiguousarray(xi, dtype=np.float32)
    xj = np.ascontiguousarray(xj, dtype=np.float32)
    return bool(lib().oracle_linked(_ptr(xi), _ptr(xj), _ptr(_L(L)), float(b)))


def fof(pos, L, b):
    """Return (root int32[n], n_links): root[i] = min index in i's component."""
    pos = _pos(pos)
    n = pos.shape[0]
    root = np.empty(n, dtype=np.int32)
    r = lib().oracle_fof(n, _ptr(pos), _ptr(_L(L)), float(b), _ptr(root))
    if r < 0:
        raise OracleError(f"oracle_fof failed ({r})")
    return root, int(r)


def fof_par(pos, L, b, threads: int = 0):
    """Multi-threaded form of ``fof`` (OpenMP): the same pairs, merged into one shared
    union-find whose roots only move to smaller indices, so (root, n_links) equal ``fof``'s
    exactly.  ``threads`` = 0 uses the OpenMP default."""
    pos = _pos(pos)
    n = pos.shape[0]
    root = np.empty(n, dtype=np.int32)
    r = lib().oracle_fof_par(n, _ptr(pos), _ptr(_L(L)), float(b), _ptr(root), int(threads))
    if r < 0:
        raise OracleError(f"oracle_fof_par failed ({r})")
    return root, int(r)


def max_threads() -> int:
    """Threads ``fof_par(..., threads=0)`` runs with."""
    return int(lib().oracle_max_threads())


class Index:
    """Cell list kept alive for repeated single-component queries."""

    def __init__(self, pos, L, b):
        self.pos = _pos(pos)
        self.L = _L(L)
        self.n = self.pos.shape[0]
        self.h = lib().oracle_index_build(self.n, _ptr(self.pos), _ptr(self.L), float(b))
        if not self.h:
            raise OracleError("oracle_index_build failed")
        self.mark = np.zeros(self.n, dtype=np.uint8)

    def component(self, seed: int, cap: int = 1 << 22) -> np.ndarray:
        out = np.empty(cap, dtype=np.int64)
        r = lib().oracle_component(self.h, int(seed), _ptr(out), cap, _ptr(self.mark))
        if r <= 0:
            raise OracleError(f"component too large or failed ({r})")
        return np.sort(out[:r])

    def close(self):
        if self.h:
            lib().oracle_index_free(self.h)
            self.h = None

    def __del__(self):
        self.close()


def groups(pos, root, L, min_size, vel=None, cap=None):
    """Return dict(group_id, n_groups, sizes, com, vmean, sigv) following C8/C9 readings."""
    pos = _pos(pos)
    n = pos.shape[0]
    root = np.ascontiguousarray(root, dtype=np.int32)
    if cap is None:
        cap = max(n, 1)
    gid = np.empty(n, dtype=np.int32)
    ng = np.zeros(1, dtype=np.int32)
    sizes = np.zeros(cap, dtype=np.int32)
    com = np.zeros((cap, 3), dtype=np.float64)
    vm = sv = None
    if vel is not None:
        vel = _pos(vel)
        vm = np.zeros((cap, 3), dtype=np.float64)
        sv = np.zeros(cap, dtype=np.float64)
    rc = lib().oracle_groups(n, _ptr(pos), _ptr(vel), _ptr(_L(L)), _ptr(root), int(min_size),
                             int(cap), _ptr(gid), _ptr(ng), _ptr(sizes), _ptr(com), _ptr(vm),
                             _ptr(sv))
    if rc not in (0, -3):
        raise OracleError(f"oracle_groups failed ({rc})")
    G = int(ng[0])
    k = min(G, cap)
    out = dict(group_id=gid, n_groups=G, sizes=sizes[:k], com=com[:k], overflow=(rc == -3))
    if vel is not None:
        out["vmean"] = vm[:k]
        out["sigv"] = sv[:k]
    return out


def frozen_backward(group_id, sizes, vmean=None, sigv=None, vel=None, g_mass=None,
                    g_com=None, g_sigv=None):
    """FP64 gradients (grad_pos[n,3], grad_vel[n,3]) with memberships frozen (Sec. 3.1)."""
    gid = np.ascontiguousarray(group_id, dtype=np.int32)
    n = gid.shape[0]
    sizes = np.ascontiguousarray(sizes, dtype=np.int32)
    G = sizes.shape[0]
    f64 = lambda a: None if a is None else np.ascontiguousarray(a, dtype=np.float64)
    velp = None if vel is None else _pos(vel)
    gp = np.zeros((n, 3), dtype=np.float64)
    gv = np.zeros((n, 3), dtype=np.float64)
    rc = lib().oracle_frozen_backward(n, _ptr(velp), _ptr(gid), G, _ptr(sizes), _ptr(f64(vmean)),
                                      _ptr(f64(sigv)), _ptr(f64(g_mass)), _ptr(f64(g_com)),
                                      _ptr(f64(g_sigv)), _ptr(gp), _ptr(gv))
    if rc:
        raise OracleError(f"oracle_frozen_backward failed ({rc})")
    return gp, gv


def _min_image(d, L3):
    """Per-axis minimum image of differences in (-L, L): wrapped once by +-L when |d| > L/2."""
    half = 0.5 * L3
    return np.where(d > half, d - L3, np.where(d < -half, d + L3, d))


def group_dispersion(pos, group_id, sizes, com, L):
    """Decoration of the decorated frozen assignment (Sec. 3.1): the particle standard
    deviation of each group about its centre of mass, read as the 1-D population value
        sigx_g = sqrt( sum_{i in g} sum_c mi(x_ic - com_gc)^2 / (3 n_g) ),
    mi the minimum image, FP64; 0 for groups of one.  Plain numpy definition."""
    pos = np.asarray(pos, dtype=np.float64)
    gid = np.asarray(group_id)
    sizes = np.asarray(sizes, dtype=np.int64)
    com = np.asarray(com, dtype=np.float64)
    G = sizes.shape[0]
    m = (gid >= 0) & (gid < G)
    d = _min_image(pos[m] - com[gid[m]], _L(L))
    s2 = np.zeros(G, dtype=np.float64)
    np.add.at(s2, gid[m], np.sum(d * d, axis=1))
    out = np.zeros(G, dtype=np.float64)
    many = sizes > 1
    out[many] = np.sqrt(s2[many] / (3.0 * sizes[many]))
    return out


def dispersion_backward(pos, group_id, sizes, com, sigx, g_sigx, L):
    """d(sum_g g_sigx_g sigx_g)/d x with memberships frozen (Sec. 3.1): the derivative of the
    definition above, mi(x_i - com_g) / (3 n_g sigx_g) per member (the terms through com_g
    vanish because the deviations of a group sum to zero); 0 where sigx_g = 0."""
    pos = np.asarray(pos, dtype=np.float64)
    gid = np.asarray(group_id)
    sizes = np.asarray(sizes, dtype=np.float64)
    com = np.asarray(com, dtype=np.float64)
    sigx = np.asarray(sigx, dtype=np.float64)
    g_sigx = np.asarray(g_sigx, dtype=np.float64)
    G = sizes.shape[0]
    grad = np.zeros_like(pos)
    m = (gid >= 0) & (gid < G)
    m[m] &= sigx[gid[m]] > 0.0
    g = gid[m]
    d = _min_image(pos[m] - com[g], _L(L))
    grad[m] = (g_sigx[g] / (3.0 * sizes[g] * sigx[g]))[:, None] * d
    return grad



def subhalos(pos, vel, group_id, norm_x, norm_v, b6, L):
    """Six-dimensional sub-halo pass (Sec. 2, sub-halo finding).

    Inside each host g (the particles with group_id == g >= 0) two particles are phase-space
    friends when d(i, j) < b6, where
        d^2 = |mi(x_i - x_j)|^2 / norm_x[g] + |v_i - v_j|^2 / norm_v[g],
    the paper's metric with its normalisation factors dividing the squared separations as
    printed; mi is the per-axis minimum image.  A host whose factors are not both positive
    is left as singletons (the metric is undefined there).  Particles of different hosts never link.
    Each squared norm is summed as ((c0*c0 + c1*c1) + c2*c2) in FP64 from the float32 inputs.
    Returns int32[n]: the smallest original index of the particle's phase-space component,
    -1 for particles outside every host.  Brute force over the pairs of each host (plain
    numpy + a library connected-components routine), so hosts must stay small (a few
    thousand members)."""
    from scipy.sparse import csr_matrix
    from scipy.sparse.csgraph import connected_components

    pos = _pos(pos)
    vel = np.asarray(vel, dtype=np.float32).reshape(-1, 3).astype(np.float64)
    gid = np.asarray(group_id, dtype=np.int64).reshape(-1)
    L3 = _L(L)
    n = pos.shape[0]
    out = np.full(n, -1, dtype=np.int32)
    bb = float(b6) * float(b6)
    for g in np.unique(gid[gid >= 0]):
        m = np.nonzero(gid == g)[0]
        if not (float(norm_x[g]) > 0.0 and float(norm_v[g]) > 0.0):
            out[m] = m
            continue
        x, v = pos[m].astype(np.float64), vel[m]
        dx = _min_image(x[:, None, :] - x[None, :, :], L3)
        sx = (dx[..., 0] * dx[..., 0] + dx[..., 1] * dx[..., 1]) + dx[..., 2] * dx[..., 2]
        del dx
        dv = v[:, None, :] - v[None, :, :]
        sv = (dv[..., 0] * dv[..., 0] + dv[..., 1] * dv[..., 1]) + dv[..., 2] * dv[..., 2]
        del dv
        d2 = sx / float(norm_x[g]) + sv / float(norm_v[g])
        _, lab = connected_components(csr_matrix(d2 < bb), directed=False)
        first = np.full(lab.max() + 1, m.size, dtype=np.int64)
        np.minimum.at(first, lab, np.arange(m.size))
        out[m] = m[first[lab]]
    return out
