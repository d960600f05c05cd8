"""Python front end of libfof.so.  torch supplies device memory and the current stream;
every step of the computation runs in the library's HIP kernels.

    plan = Plan([n], [(L, b)])              # host planning + device workspace
    plan.build_grid(pos)                    # pos: float32 [n, 3] on the GPU
    root = plan.link()                      # int32 [n] smallest member index per component
    out = plan.groups(min_size, vel=None)   # group ids, sizes, centres of mass, moments

``find_groups(pos, L, b, min_size)`` does all three for one box.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import check


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _need(t, name, dtype, shape, device, min_rows=None):
    """Raises ValueError unless t is a contiguous tensor of `dtype` on `device` with `shape`
    (or, with min_rows, a 1-D tensor of at least that many entries): the library would read
    a host pointer or a wrong element size as device memory."""
    if not isinstance(t, torch.Tensor):
        raise ValueError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if t.device != device:
        raise ValueError(f"{name} must be on {device}, got {t.device}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if min_rows is not None:
        if t.dim() != 1 or t.shape[0] < min_rows:
            raise ValueError(f"{name} needs at least {min_rows} entries, got {tuple(t.shape)}")
    elif tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


class Plan:
    """A planned batch of periodic boxes with its device workspace.

    counts: particles per box; boxes: (L, b) per box where L is a scalar or 3 sides and b
    the physical linking length.  tune: dict(cell_side=..., block=...), results do not
    depend on it.
    """

    def __init__(self, counts, boxes, device=None, tune=None):
        L = _lib.load()
        self.device = torch.device(device if device is not None else "cuda")
        with torch.cuda.device(self.device):
            _lib.init()  # helper stream of this device (once per process)
        counts = np.ascontiguousarray(np.asarray(counts, dtype=np.int64).reshape(-1))
        nbox = counts.shape[0]
        bx = (_lib.fof_box * nbox)()
        for k, (Lk, bk) in enumerate(boxes):
            Lk = np.broadcast_to(np.asarray(Lk, dtype=np.float64), (3,))
            bx[k].L[:] = [float(v) for v in Lk]
            bx[k].b = float(bk)
        self.boxes = [(tuple(float(v) for v in bx[k].L), float(bx[k].b)) for k in range(nbox)]
        self.counts = counts
        self.tune = _lib.fof_tune()
        for key, v in (tune or {}).items():
            setattr(self.tune, key, v)
        self.grid = _lib.fof_grid()
        check("fof_workspace_bytes",
              L.fof_workspace_bytes(nbox, counts.ctypes.data_as(ctypes.c_void_p), bx,
                                    ctypes.byref(self.tune), ctypes.byref(self.grid), None, 0))
        desc = np.zeros(self.grid.desc_bytes, dtype=np.uint8)
        check("fof_workspace_bytes",
              L.fof_workspace_bytes(nbox, counts.ctypes.data_as(ctypes.c_void_p), bx,
                                    ctypes.byref(self.tune), ctypes.byref(self.grid),
                                    desc.ctypes.data_as(ctypes.c_void_p), desc.shape[0]))
        self.n = int(self.grid.n)
        self.nbox = nbox
        self.ws_bytes = int(self.grid.ws_bytes)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        o = int(self.grid.off_desc)
        self.ws[o:o + desc.shape[0]].copy_(torch.from_numpy(desc))
        self._gref = ctypes.byref(self.grid)

    # -- stages ---------------------------------------------------------------------------
    def build_grid(self, pos, stream=None):
        _need(pos, "pos", torch.float32, (self.n, 3), self.ws.device)
        self._pos = pos
        check("fof_build_grid",
              _lib.load().fof_build_grid(self._gref, _ptr(pos), _ptr(self.ws), self.ws_bytes,
                                         _stream(stream)))

    def link(self, root=None, stream=None):
        if root is None:
            root = torch.empty(self.n, dtype=torch.int32, device=self.device)
        check("fof_link",
              _lib.load().fof_link(self._gref, _ptr(self.ws), self.ws_bytes, None, _ptr(root),
                                   _stream(stream)))
        return root

    def groups(self, min_size, vel=None, cap=None, out=None, stream=None):
        """Returns a dict of device tensors; n_groups stays on the device (one int32).
        Tensors passed in `out` (a previous result) are reused; they must have the shapes of
        this cap (by default the cap they were made for), else ValueError."""
        o = out or {}
        if cap is None:
            cap = int(o["cap"]) if "cap" in o else self.n
        cap = int(cap)
        d = self.device
        c1 = max(cap, 1)

        def buf(name, dtype, shape):
            t = o.get(name)
            if t is None:
                return torch.empty(shape, dtype=dtype, device=d)
            _need(t, name, dtype, shape, self.ws.device)
            return t

        gid = buf("group_id", torch.int32, (self.n,))
        ng = buf("n_groups", torch.int32, (1,))
        sizes = buf("sizes", torch.int32, (c1,))
        com = buf("com", torch.float64, (c1, 3))
        vm = sv = None
        if vel is not None:
            _need(vel, "vel", torch.float32, (self.n, 3), self.ws.device)
            vm = buf("vmean", torch.float64, (c1, 3))
            sv = buf("sigv", torch.float64, (c1,))
        check("fof_groups",
              _lib.load().fof_groups(self._gref, _ptr(self.ws), self.ws_bytes, None,
                                     int(min_size), _ptr(vel), cap,
                                     _ptr(gid), _ptr(ng), _ptr(sizes), _ptr(com), _ptr(vm),
                                     _ptr(sv), _stream(stream)))
        res = dict(group_id=gid, n_groups=ng, sizes=sizes, com=com, cap=cap)
        if vel is not None:
            res["vmean"] = vm
            res["sigv"] = sv
        return res

    def dispersion(self, res, sigx=None, stream=None):
        """Position dispersion per group (device float64 [cap]) for the result `res` of the
        last groups() call; groups of one get 0."""
        cap = res["cap"]
        if sigx is None:
            sigx = torch.empty(max(cap, 1), dtype=torch.float64, device=self.device)
        check("fof_group_dispersion",
              _lib.load().fof_group_dispersion(self._gref, _ptr(self.ws), self.ws_bytes,
                                               cap,
                                               _ptr(res["n_groups"]), _ptr(res["sizes"]),
                                               _ptr(res["com"]), _ptr(sigx), _stream(stream)))
        return sigx

    def backward_dispersion(self, pos, group_id, G, sizes, com, sigx, g_sigx, grad_pos,
                            stream=None):
        """Adds the frozen-assignment gradient of the dispersion to grad_pos (in place)."""
        d, G = self.ws.device, int(G)
        g_sigx = g_sigx.to(torch.float64).contiguous()
        _need(pos, "pos", torch.float32, (self.n, 3), d)
        _need(group_id, "group_id", torch.int32, (self.n,), d)
        _need(grad_pos, "grad_pos", torch.float32, (self.n, 3), d)
        _need(sizes, "sizes", torch.int32, None, d, min_rows=G)
        _need(sigx, "sigx", torch.float64, None, d, min_rows=G)
        _need(g_sigx, "g_sigx", torch.float64, None, d, min_rows=G)
        _need(com.reshape(-1), "com", torch.float64, None, d, min_rows=3 * G)
        check("fof_backward_dispersion",
              _lib.load().fof_backward_dispersion(self._gref, _ptr(self.ws), self.ws_bytes,
                                                  _ptr(pos),
                                                  _ptr(group_id), int(G), _ptr(sizes),
                                                  _ptr(com), _ptr(sigx), _ptr(g_sigx),
                                                  _ptr(grad_pos), _stream(stream)))
        return grad_pos

    def subhalo(self, pos, vel, group_id, G, sizes, norm_x, norm_v, b6, sub=None,
                stream=None):
        """Six-dimensional sub-halo labels (device int32 [n]) inside the G host groups that
        group_id / sizes describe (as groups() returns them): the smallest original index of
        each member's phase-space component, -1 outside the hosts.  norm_x, norm_v: one
        factor per host dividing the squared position and velocity separations."""
        G = int(G)
        d = self.ws.device
        _need(pos, "pos", torch.float32, (self.n, 3), d)
        _need(vel, "vel", torch.float32, (self.n, 3), d)
        _need(group_id, "group_id", torch.int32, (self.n,), d)
        _need(sizes, "sizes", torch.int32, None, d, min_rows=G)
        if sub is None:
            sub = torch.empty(max(self.n, 1), dtype=torch.int32, device=d)
        _need(sub, "sub", torch.int32, None, d, min_rows=self.n)
        lib = _lib.load()
        nbytes = int(lib.fof_subhalo_scratch_bytes(self.n, G))
        scratch = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-scratch.data_ptr()) % 256
        nx = torch.as_tensor(norm_x, dtype=torch.float64, device=self.device).reshape(-1)
        nv = torch.as_tensor(norm_v, dtype=torch.float64, device=self.device).reshape(-1)
        if G > 0 and (nx.numel() < G or nv.numel() < G):
            raise ValueError("norm_x and norm_v need one factor per host")
        check("fof_subhalo",
              lib.fof_subhalo(self._gref, _ptr(self.ws), self.ws_bytes, _ptr(pos), _ptr(vel),
                              _ptr(group_id),
                              G, _ptr(sizes), _ptr(nx), _ptr(nv), float(b6),
                              ctypes.c_void_p(scratch.data_ptr() + off), nbytes, _ptr(sub),
                              _stream(stream)))
        self._keep = (scratch, nx, nv)   # alive until the next call on this plan
        return sub

    def status(self) -> int:
        p = ctypes.c_void_p()
        check("fof_status", _lib.load().fof_status(self._gref, _ptr(self.ws), self.ws_bytes,
                                                   ctypes.byref(p)))
        off = p.value - self.ws.data_ptr()
        return int(self.ws[off:off + 4].view(torch.int32).item())

    def backward(self, group_id, G, sizes, vmean=None, sigv=None, vel=None, g_mass=None,
                 g_com=None, g_sigv=None, want_pos=True, want_vel=True, stream=None):
        d = self.ws.device
        G = int(G)
        _need(group_id, "group_id", torch.int32, (self.n,), d)
        _need(sizes, "sizes", torch.int32, None, d, min_rows=G)
        if g_sigv is not None:
            _need(vel, "vel", torch.float32, (self.n, 3), d)
            _need(vmean.reshape(-1), "vmean", torch.float64, None, d, min_rows=3 * G)
            _need(sigv, "sigv", torch.float64, None, d, min_rows=G)
        gp = torch.empty((self.n, 3), dtype=torch.float32, device=d) if want_pos else None
        gv = torch.empty((self.n, 3), dtype=torch.float32, device=d) if want_vel else None
        f64 = lambda t: None if t is None else t.to(torch.float64).contiguous()
        g_mass, g_com, g_sigv = f64(g_mass), f64(g_com), f64(g_sigv)
        for t, name, k in ((g_mass, "g_mass", 1), (g_com, "g_com", 3), (g_sigv, "g_sigv", 1)):
            if t is not None:
                _need(t.reshape(-1), name, torch.float64, None, d, min_rows=k * G)
        check("fof_backward",
              _lib.load().fof_backward(self._gref, _ptr(self.ws), self.ws_bytes,
                                       _lib.FOF_FROZEN, _ptr(group_id),
                                       int(G), _ptr(sizes), _ptr(vmean), _ptr(sigv), _ptr(vel),
                                       _ptr(g_mass), _ptr(g_com), _ptr(g_sigv), None, None, 0,
                                       _ptr(gp), _ptr(gv), _stream(stream)))
        return gp, gv


def trim(res):
    """Synchronise once and cut the group tables to n_groups (host-side convenience)."""
    G = int(res["n_groups"].item())
    k = min(G, res["cap"])
    out = dict(group_id=res["group_id"], n_groups=G, sizes=res["sizes"][:k], com=res["com"][:k])
    if "vmean" in res:
        out["vmean"] = res["vmean"][:k]
        out["sigv"] = res["sigv"][:k]
    return out


def find_groups(pos, L, b, min_size=20, vel=None, cap=None, tune=None):
    """One periodic box: returns (root, groups dict trimmed to n_groups)."""
    plan = Plan([pos.shape[0]], [(L, b)], device=pos.device, tune=tune)
    plan.build_grid(pos)
    root = plan.link()
    res = trim(plan.groups(min_size, vel=vel, cap=cap))
    return root, res


def _box(L, b):
    bx = _lib.fof_box()
    bx.L[:] = [float(v) for v in np.broadcast_to(np.asarray(L, dtype=np.float64), (3,))]
    bx.b = float(b)
    return bx


class Stream:
    """Streaming labels of one box in z-slabs (fof_stream_counts, fof_stream_workspace_bytes,
    fof_link_stream): the workspace holds one slab at a time, so it is bounded by the
    largest slab instead of the box.  `counts()` reads the slab sizes back to the host once
    (the only synchronisation); `labels()` then gives what fof_link gives for the whole box."""

    def __init__(self, pos, L, b, nslab=16, tune=None):
        _need(pos, "pos", torch.float32, (pos.shape[0], 3), pos.device)
        self.pos, self.n, self.nslab = pos, int(pos.shape[0]), int(nslab)
        self.box = _box(L, b)
        self.tune = _lib.fof_tune()
        for key, v in (tune or {}).items():
            setattr(self.tune, key, v)
        lib = _lib.load()
        counts = torch.empty(self.nslab, dtype=torch.int64, device=pos.device)
        check("fof_stream_counts",
              lib.fof_stream_counts(ctypes.byref(self.box), self.n, _ptr(pos), self.nslab,
                                    _ptr(counts), _stream()))
        self.counts = np.ascontiguousarray(counts.cpu().numpy(), dtype=np.int64)
        nbytes = ctypes.c_size_t()
        check("fof_stream_workspace_bytes",
              lib.fof_stream_workspace_bytes(ctypes.byref(self.box), self.n, self.nslab,
                                             self.counts.ctypes.data_as(ctypes.c_void_p),
                                             ctypes.byref(self.tune), ctypes.byref(nbytes)))
        self.ws_bytes = int(nbytes.value)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=pos.device)
        self.status_word = torch.zeros(1, dtype=torch.int32, device=pos.device)

    def labels(self, root=None, stream=None):
        if root is None:
            root = torch.empty(max(self.n, 1), dtype=torch.int32, device=self.pos.device)
        _need(root, "root", torch.int32, None, self.pos.device, min_rows=self.n)
        check("fof_link_stream",
              _lib.load().fof_link_stream(ctypes.byref(self.box), self.n, _ptr(self.pos),
                                          self.nslab,
                                          self.counts.ctypes.data_as(ctypes.c_void_p),
                                          ctypes.byref(self.tune), _ptr(self.ws), self.ws_bytes,
                                          _ptr(root), _ptr(self.status_word), _stream(stream)))
        return root

    def status(self) -> int:
        return int(self.status_word.item())
