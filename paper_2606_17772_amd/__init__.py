"""FD-CGKS on MI355X: Python binding of libfdcgks.so.

Argument marshalling only: every step of the method runs in the HIP kernels
behind the C ABI (include/fdcgks.h).  PyTorch provides device memory and the
stream; numpy arrays are accepted for host-side state exchange.

    from paper_2606_17772_amd import Problem
    pb = Problem(dim=2, nx=512, ny=512, lx=10.0, ly=10.0)
    pb.set_state(0, W, Wx, Wy); pb.set_state(1, Wd, Wxd, Wyd)
    t, n = pb.step(cfl=0.5, nsteps=10)
    W, Wx, Wy = pb.get_state(0)
"""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import _lib
from ._lib import (BC_NO_SLIP, BC_PERIODIC, BC_REFLECTING, BC_ZERO_GRADIENT, FLUX_6_2, FLUX_6_4, FLUX_LINEAR, FP32_FLUX, FP64,  # noqa: F401
                   GRAD_CARRIED, GRAD_REEVAL, RECON_CHARACTERISTIC, RECON_CONSERVATIVE, FdcgksError, Params,
                   Params3D)

__all__ = ["Problem", "Problem3D", "Batch", "Params", "Params3D", "FdcgksError", "default_params", "make_params",
           "make_params3d", "step1d_static"]

_VARIANTS = {"6-4": FLUX_6_4, "6-2": FLUX_6_2, "linear": FLUX_LINEAR}
_BCS = {"periodic": BC_PERIODIC, "zero_gradient": BC_ZERO_GRADIENT, "reflecting": BC_REFLECTING,
        "no_slip": BC_NO_SLIP}
_RECON = {"conservative": RECON_CONSERVATIVE, "characteristic": RECON_CHARACTERISTIC}


def default_params() -> Params:
    p = Params()
    _lib.load().fdcgks_default_params(C.byref(p))
    return p


def make_params(**kw) -> Params:
    """fdcgks_params from keywords (names of the C struct; also
    variant='6-4'|'6-2'|'linear', bc='periodic'|'zero_gradient'|'reflecting'|
    'no_slip', sides=(x-low, x-high, y-low, y-high) boundary names or codes,
    recon_vars='conservative'|'characteristic', fp32_flux=bool,
    flux_order=6|8)."""
    p = default_params()
    kw = dict(kw)
    if "variant" in kw:
        v = kw.pop("variant")
        p.flux_variant = _VARIANTS[v] if isinstance(v, str) else int(v)
    if "bc" in kw and isinstance(kw["bc"], str):
        kw["bc"] = _BCS[kw["bc"]]
    sides = kw.pop("sides", None)
    if sides is not None:
        p.side[:] = [_BCS[b] if isinstance(b, str) else int(b) for b in sides]
    if "recon_vars" in kw and isinstance(kw["recon_vars"], str):
        kw["recon_vars"] = _RECON[kw["recon_vars"]]
    if kw.pop("fp32_flux", False):
        p.flux_precision = FP32_FLUX
    if kw.pop("grad_carried", False):
        p.grad_update = GRAD_CARRIED
    if "dim" in kw and kw["dim"] == 1:
        kw.setdefault("ny", 1)
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    if p.dim == 2 and "ly" not in kw:
        p.ly = p.lx * p.ny / p.nx
    return p


def _torch():
    import torch  # noqa: PLC0415
    return torch


def _current_stream():
    try:
        torch = _torch()
        if torch.cuda.is_available():
            return C.c_void_p(torch.cuda.current_stream().cuda_stream)
    except ImportError:
        pass
    return C.c_void_p(None)


def _ptr(a, writable=False):
    """(pointer, on_device, keepalive) for a numpy array or torch tensor."""
    if isinstance(a, np.ndarray):
        if a.dtype != np.float64 or not a.flags.c_contiguous or (writable and not a.flags.writeable):
            raise TypeError("numpy state arrays must be contiguous float64")
        return C.c_void_p(a.ctypes.data), 0, a
    torch = _torch()
    if isinstance(a, torch.Tensor):
        if a.dtype != torch.float64 or not a.is_contiguous():
            raise TypeError("tensors must be contiguous float64")
        return C.c_void_p(a.data_ptr()), (1 if a.is_cuda else 0), a
    raise TypeError(f"unsupported array type {type(a)}")


def step1d_static(params: Params, state, nsteps=1, dt=0.0, cfl=0.5, t_end=0.0, t=0.0, stream=None):
    """fdcgks_step1d_static: a whole 1D run that allocates nothing on the
    device.  state: a contiguous float64 CUDA tensor of shape (lines, 6, nx)
    (lines = 2 with dual_1d), advanced in place.  Returns (t, steps_done)."""
    L = _lib.load()
    torch = _torch()
    if not (isinstance(state, torch.Tensor) and state.is_cuda and state.dtype == torch.float64
            and state.is_contiguous()):
        raise TypeError("state must be a contiguous float64 CUDA tensor")
    tt = C.c_double(t)
    n = C.c_int32()
    s = _current_stream() if stream is None else C.c_void_p(stream)
    _lib.check(L.fdcgks_step1d_static(C.byref(params), C.c_void_p(state.data_ptr()), dt, cfl, nsteps, t_end,
                                      C.byref(tt), C.byref(n), s))
    return tt.value, n.value


class Problem:
    """One FD-CGKS problem on the current HIP device (see fdcgks_create)."""

    def __init__(self, params: Params | None = None, stream=None, **kw):
        self._L = _lib.load()
        self.params = params if params is not None else make_params(**kw)
        self._h = C.c_void_p()
        s = _current_stream() if stream is None else C.c_void_p(stream)
        _lib.check(self._L.fdcgks_create(C.byref(self.params), s, C.byref(self._h)))
        p = self.params
        self.ncomp = 4 if p.dim == 2 else 3
        self.ngrid = 2 if (p.dim == 2 or p.dual_1d) else 1
        self.shape = (self.ncomp, p.ny, p.nx)
        # along a bounded 2D axis the dual grid has a node on each side
        side = [p.side[k] if p.side[k] >= 0 else p.bc for k in range(4)]
        self.bounded = (p.dim == 2 and side[0] != BC_PERIODIC, p.dim == 2 and side[2] != BC_PERIODIC)

    def grid_dims(self, grid):
        """(ny, nx) of the nodes of `grid`."""
        p = self.params
        return (p.ny + (grid == 1 and self.bounded[1]), p.nx + (grid == 1 and self.bounded[0]))

    def grid_shape(self, grid):
        return (self.ncomp,) + self.grid_dims(grid)

    # -- lifetime
    def close(self):
        if self._h:
            self._L.fdcgks_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st):
        return _lib.check(st, self._h)

    # -- state
    def set_state(self, grid, W, Wx, Wy=None, row_stride=0):
        """W, Wx[, Wy]: (ncomp, ny_g, nx_g) arrays of the grid (numpy, or torch
        on the device).  row_stride > 0: the arrays are flat with rows of
        row_stride elements (padded rows)."""
        pw, dev, k1 = _ptr(W)
        px, dev2, k2 = _ptr(Wx)
        py, dev3, k3 = _ptr(Wy) if Wy is not None else (C.c_void_p(None), dev, None)
        if len({dev, dev2, dev3}) != 1:
            raise TypeError("W, Wx, Wy must all live on the host or all on the device")
        shape = self.grid_shape(grid)
        need = int(np.prod(shape)) if not row_stride else shape[0] * shape[1] * int(row_stride)
        for a in (W, Wx) + ((Wy,) if Wy is not None else ()):
            if not row_stride and tuple(a.shape) not in (shape, (need,)):
                raise ValueError(f"state arrays of grid {grid} must have shape {shape}")
            if row_stride and int(np.prod(tuple(a.shape))) < need:
                raise ValueError(f"strided state arrays of grid {grid} need {need} elements")
        self._chk(self._L.fdcgks_set_state(self._h, grid, pw, px, py, int(row_stride), dev))

    def set_state_stacked(self, grid, S):
        """S: (12, ny, nx) (2D; the dual grid's own size along bounded axes) or
        (6, N) (1D) stacked W, Wx[, Wy]."""
        n = self.ncomp
        S = np.ascontiguousarray(S, dtype=np.float64).reshape((-1,) + self.grid_dims(grid))
        self.set_state(grid, np.ascontiguousarray(S[:n]), np.ascontiguousarray(S[n:2 * n]),
                       np.ascontiguousarray(S[2 * n:3 * n]) if self.params.dim == 2 else None)

    def get_state(self, grid, device=None):
        """Returns (W, Wx, Wy) as numpy (device=None) or torch tensors on `device`."""
        shape = self.grid_shape(grid)
        if device is None:
            out = [np.empty(shape) for _ in range(3 if self.params.dim == 2 else 2)]
        else:
            torch = _torch()
            out = [torch.empty(shape, dtype=torch.float64, device=device)
                   for _ in range(3 if self.params.dim == 2 else 2)]
        ptrs = [_ptr(a, True) for a in out]
        py = ptrs[2][0] if len(ptrs) == 3 else C.c_void_p(None)
        self._chk(self._L.fdcgks_get_state(self._h, grid, ptrs[0][0], ptrs[1][0], py, 0, ptrs[0][1]))
        return tuple(out)

    def get_state_strided(self, grid, row_stride):
        """(W, Wx[, Wy]) as flat numpy arrays with rows of row_stride elements
        (the padding is left as zeros)."""
        ny, nx = self.grid_dims(grid)
        out = [np.zeros(self.ncomp * ny * row_stride) for _ in range(3 if self.params.dim == 2 else 2)]
        py = C.c_void_p(out[2].ctypes.data) if len(out) == 3 else C.c_void_p(None)
        self._chk(self._L.fdcgks_get_state(self._h, grid, C.c_void_p(out[0].ctypes.data),
                                           C.c_void_p(out[1].ctypes.data), py, int(row_stride), 0))
        return tuple(out)

    def set_state_from_samples(self, S):
        """Every grid's state from samples of the initial field on the
        half-spacing lattice: (ncomp, 2 ny, 2 nx) in 2D, (ncomp, 2 nx) in 1D
        (fdcgks_set_state_from_samples; periodic problems)."""
        p = self.params
        shape = (self.ncomp, 2 * p.ny, 2 * p.nx) if p.dim == 2 else (self.ncomp, 2 * p.nx)
        if tuple(S.shape) != shape:
            raise ValueError(f"samples must have shape {shape}")
        if isinstance(S, np.ndarray):
            S = np.ascontiguousarray(S, dtype=np.float64)
        ps, dev, _ = _ptr(S)
        self._chk(self._L.fdcgks_set_state_from_samples(self._h, ps, dev))

    def get_state_stacked(self, grid):
        return np.concatenate(self.get_state(grid), axis=0)

    def set_state_all(self, S):
        """S: (ngrid, 12, ny, nx) (2D) stacked W, Wx, Wy of every grid, as a
        contiguous float64 numpy array or torch tensor (host or device);
        both grids must have the same size (no bounded axis)."""
        if any(self.bounded):
            raise ValueError("grids differ in size along bounded axes: use set_state per grid")
        n = self.ncomp
        for g in range(self.ngrid):
            if self.params.dim == 2:
                self.set_state(g, S[g, :n], S[g, n:2 * n], S[g, 2 * n:3 * n])
            else:
                self.set_state(g, S[g, :n], S[g, n:2 * n])

    def get_state_all(self, device=None):
        """(ngrid, 3*ncomp, ny, nx) as numpy (device=None) or a torch tensor on `device`."""
        if any(self.bounded):
            raise ValueError("grids differ in size along bounded axes: use get_state per grid")
        parts = [self.get_state(g, device) for g in range(self.ngrid)]
        if device is None:
            return np.stack([np.concatenate(p, axis=0) for p in parts])
        torch = _torch()
        return torch.stack([torch.cat(p, dim=0) for p in parts])

    def step_vjp(self, dt, lam_out):
        """J^T lam_out for one step of size dt from the current state (the
        state is not advanced).  lam_out: (2, 12, ny, nx) numpy array or
        torch tensor; the result has the same type and device.  With bounded
        axes the grids differ in size: lam_out is a pair of (12, ny_g, nx_g)
        arrays (grid_shape), and so is the result."""
        p = self.params
        if any(self.bounded):
            return self._step_vjp_bounded(dt, lam_out)
        shape = (self.ngrid, (3 if p.dim == 2 else 2) * self.ncomp, p.ny, p.nx)
        if tuple(lam_out.shape) != shape:
            raise ValueError(f"lam_out must have shape {shape}")
        if isinstance(lam_out, np.ndarray):
            lam_out = np.ascontiguousarray(lam_out, dtype=np.float64)
            lam_in = np.empty(shape)
        else:
            lam_out = lam_out.contiguous()
            lam_in = _torch().empty_like(lam_out)
        po, dev, _ = _ptr(lam_out)
        pi, dev2, _ = _ptr(lam_in, True)
        self._chk(self._L.fdcgks_step_vjp(self._h, dt, po, pi, dev))
        return lam_in

    def _step_vjp_bounded(self, dt, lam_out):
        shapes = [(3 * self.ncomp,) + self.grid_dims(g) for g in range(self.ngrid)]
        if len(lam_out) != self.ngrid or any(tuple(a.shape) != sh for a, sh in zip(lam_out, shapes)):
            raise ValueError(f"lam_out must be a pair of arrays of shapes {shapes}")
        sizes = [int(np.prod(sh)) for sh in shapes]
        if isinstance(lam_out[0], np.ndarray):
            flat = np.ascontiguousarray(np.concatenate([np.asarray(a, dtype=np.float64).ravel() for a in lam_out]))
            out = np.empty_like(flat)
            parts = np.split(out, [sizes[0]])
        else:
            torch = _torch()
            flat = torch.cat([a.reshape(-1) for a in lam_out]).contiguous()
            out = torch.empty_like(flat)
            parts = torch.split(out, sizes)
        po, dev, _ = _ptr(flat)
        pi, dev2, _ = _ptr(out, True)
        self._chk(self._L.fdcgks_step_vjp(self._h, dt, po, pi, dev))
        return [q.reshape(sh) for q, sh in zip(parts, shapes)]

    def diagnostics(self):
        """Conservation sums per grid ((ngrid, ncomp) array), smallest rho and
        smallest pressure of the current state (fdcgks_diagnostics)."""
        nq = self.ngrid * self.ncomp + 2
        out = (C.c_double * nq)()
        self._chk(self._L.fdcgks_diagnostics(self._h, out))
        v = np.array(list(out))
        return {"sums": v[:-2].reshape(self.ngrid, self.ncomp), "rho_min": float(v[-2]), "p_min": float(v[-1])}

    # -- time stepping
    def compute_dt(self, cfl):
        dt = C.c_double()
        self._chk(self._L.fdcgks_compute_dt(self._h, cfl, C.byref(dt)))
        return dt.value

    def step(self, nsteps=1, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
        """Advance up to nsteps; returns (t, steps_done)."""
        tt = C.c_double(t)
        n = C.c_int32()
        self._chk(self._L.fdcgks_step(self._h, dt, cfl, nsteps, t_end, C.byref(tt), C.byref(n)))
        return tt.value, n.value

    # -- launch options
    _TILES = {"edge": _lib.OPT_TILE_EDGE, "node": _lib.OPT_TILE_NODE, "update": _lib.OPT_TILE_UPDATE}

    @property
    def graph_steps(self):
        """Steps per captured HIP graph in fdcgks_step (0: separate launches)."""
        v = C.c_int64()
        self._chk(self._L.fdcgks_get_option(self._h, _lib.OPT_GRAPH, C.byref(v)))
        return v.value

    @graph_steps.setter
    def graph_steps(self, k):
        self._chk(self._L.fdcgks_set_option(self._h, _lib.OPT_GRAPH, int(k)))

    @property
    def use_graph(self):
        return self.graph_steps > 0

    @use_graph.setter
    def use_graph(self, on):
        self.graph_steps = max(1, self.graph_steps) if on else 0

    @property
    def fuse_nodes(self):
        """Node sweep evaluated inside the update kernel (2D steps)."""
        v = C.c_int64()
        self._chk(self._L.fdcgks_get_option(self._h, _lib.OPT_FUSE_NODES, C.byref(v)))
        return bool(v.value)

    @fuse_nodes.setter
    def fuse_nodes(self, on):
        self._chk(self._L.fdcgks_set_option(self._h, _lib.OPT_FUSE_NODES, 1 if on else 0))

    @property
    def fuse_stage(self):
        """Interface sweep and update in one marching kernel (2D steps):
        False / 0 off, True / 1 on, 2 (the default) where it pays."""
        v = C.c_int64()
        self._chk(self._L.fdcgks_get_option(self._h, _lib.OPT_FUSE_STAGE, C.byref(v)))
        return int(v.value)

    @fuse_stage.setter
    def fuse_stage(self, mode):
        self._chk(self._L.fdcgks_set_option(self._h, _lib.OPT_FUSE_STAGE, int(mode)))

    @property
    def fused_rows(self):
        """Node rows per block of the fused stage kernel (0: automatic)."""
        v = C.c_int64()
        self._chk(self._L.fdcgks_get_option(self._h, _lib.OPT_FUSED_ROWS, C.byref(v)))
        return v.value

    @fused_rows.setter
    def fused_rows(self, rows):
        self._chk(self._L.fdcgks_set_option(self._h, _lib.OPT_FUSED_ROWS, int(rows)))

    def tiles(self):
        """Block shapes {"edge": (x, y), "node": ..., "update": ...}."""
        out = {}
        for name, opt in self._TILES.items():
            v = C.c_int64()
            self._chk(self._L.fdcgks_get_option(self._h, opt, C.byref(v)))
            out[name] = (v.value & 0xFFFF, (v.value >> 16) & 0xFFFF)
        return out

    def set_tile(self, kernel, x, y):
        self._chk(self._L.fdcgks_set_option(self._h, self._TILES[kernel], int(x) | (int(y) << 16)))

    def autotune(self, reps=5):
        """Time the candidate block shapes and keep the fastest; returns tiles()."""
        self._chk(self._L.fdcgks_autotune(self._h, reps))
        return self.tiles()

    KERNEL_CLASSES = ("halo", "edge1", "node1", "update1", "edge2", "node2", "update2", "step")

    def step_timed(self, nsteps=1, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
        """step() with per-kernel device milliseconds: returns (t, steps, {class: ms})."""
        tt = C.c_double(t)
        n = C.c_int32()
        ms = (C.c_double * 8)()
        self._chk(self._L.fdcgks_step_timed(self._h, dt, cfl, nsteps, t_end, C.byref(tt), C.byref(n), ms))
        return tt.value, n.value, dict(zip(self.KERNEL_CLASSES, list(ms)))

    # -- diagnostics
    def debug_stage(self, stage, dt):
        """One stage without committing it: (state, accumulators) for stage 1,
        state for stage 2.  Each is an (ngrid, nf, ny, nx) array, or with
        bounded axes a tuple of one (nf, ny_g, nx_g) array per grid."""
        p = self.params
        nf = 12 if p.dim == 2 else 6
        sizes = [nf * int(np.prod(self.grid_dims(g))) for g in range(self.ngrid)]
        out = np.zeros(sum(sizes))
        acc = np.zeros_like(out)
        self._chk(self._L.fdcgks_debug_stage(self._h, stage, dt, C.c_void_p(out.ctypes.data),
                                             C.c_void_p(acc.ctypes.data)))

        def split(a):
            if not any(self.bounded):
                return a.reshape(self.ngrid, nf, p.ny, p.nx)
            parts = np.split(a, np.cumsum(sizes)[:-1])
            return tuple(q.reshape((nf,) + self.grid_dims(g)) for g, q in enumerate(parts))
        return (split(out), split(acc)) if stage == 1 else split(out)

    def debug_intermediates(self, dt):
        p = self.params
        ex = np.zeros((2, 25, p.ny, p.nx)); ey = np.zeros_like(ex)
        npp = np.zeros((16, p.ny, p.nx)); nd = np.zeros_like(npp)
        self._chk(self._L.fdcgks_debug_intermediates(self._h, dt, *(C.c_void_p(a.ctypes.data)
                                                                   for a in (ex, ey, npp, nd))))
        return ex, ey, npp, nd


class Batch:
    """Many independent 2D problems advanced together (fdcgks_batch_*):
    every launch covers every member (phased launches captured as graphs by
    default; see set_mode)."""

    def __init__(self, params_list, stream=None):
        self._L = _lib.load()
        n = len(params_list)
        arr = (Params * n)(*params_list)
        self.params = list(params_list)
        self.count = n
        self._h = C.c_void_p()
        s = _current_stream() if stream is None else C.c_void_p(stream)
        _lib.check(self._L.fdcgks_batch_create(n, arr, s, C.byref(self._h)), None, batch=True)

    def close(self):
        if self._h:
            self._L.fdcgks_batch_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def _chk(self, st):
        return _lib.check(st, self._h, batch=True)

    def set_state(self, member, grid, W, Wx, Wy):
        pw, dev, _ = _ptr(W)
        px, _, _ = _ptr(Wx)
        py, _, _ = _ptr(Wy)
        self._chk(self._L.fdcgks_batch_set_state(self._h, member, grid, pw, px, py, dev))

    def grid_dims(self, member, grid):
        """(ny, nx) of the nodes of `grid` of a member (the dual grid has one
        more row / column along a bounded axis)."""
        p = self.params[member]
        side = [p.side[k] if p.side[k] >= 0 else p.bc for k in range(4)]
        return (p.ny + (grid == 1 and side[2] != BC_PERIODIC), p.nx + (grid == 1 and side[0] != BC_PERIODIC))

    def set_state_stacked(self, member, grid, S):
        S = np.ascontiguousarray(S, dtype=np.float64).reshape((12,) + self.grid_dims(member, grid))
        self.set_state(member, grid, np.ascontiguousarray(S[:4]), np.ascontiguousarray(S[4:8]),
                       np.ascontiguousarray(S[8:12]))

    def get_state_stacked(self, member, grid):
        out = [np.empty((4,) + self.grid_dims(member, grid)) for _ in range(3)]
        self._chk(self._L.fdcgks_batch_get_state(self._h, member, grid, *(C.c_void_p(a.ctypes.data) for a in out), 0))
        return np.concatenate(out, axis=0)

    def set_mode(self, mode):
        """'graph' (one launch per phase, 16 steps per captured HIP graph;
        default), 'phased' (the same launches, not captured) or 'persistent'
        (one cooperative launch per stage)."""
        m = {"persistent": _lib.BATCH_PERSISTENT, "phased": _lib.BATCH_PHASED, "graph": _lib.BATCH_GRAPH}[mode]
        self._chk(self._L.fdcgks_batch_set_mode(self._h, m))

    def step(self, nsteps=1, cfl=0.5):
        """Returns (t[count], dt_last[count], steps_done)."""
        t = np.zeros(self.count)
        dt = np.zeros(self.count)
        n = C.c_int32()
        self._chk(self._L.fdcgks_batch_step(self._h, cfl, nsteps, t.ctypes.data_as(C.POINTER(C.c_double)),
                                            dt.ctypes.data_as(C.POINTER(C.c_double)), C.byref(n)))
        return t, dt, n.value


# ---------------------------------------------------------------------- 3D
def make_params3d(**kw) -> Params3D:
    """fdcgks3d_params from keywords (names of the C struct; also
    variant='6-4'|'6-2'|'linear', grad_carried=bool,
    recon_vars='conservative'|'characteristic')."""
    p = Params3D()
    _lib.load().fdcgks3d_default_params(C.byref(p))
    kw = dict(kw)
    if "recon_vars" in kw and isinstance(kw["recon_vars"], str):
        kw["recon_vars"] = _RECON[kw["recon_vars"]]
    if "variant" in kw:
        v = kw.pop("variant")
        p.flux_variant = _VARIANTS[v] if isinstance(v, str) else int(v)
    if kw.pop("grad_carried", False):
        p.grad_update = GRAD_CARRIED
    for k, v in kw.items():
        if not hasattr(p, k):
            raise TypeError(f"unknown parameter {k!r}")
        setattr(p, k, v)
    return p


class Problem3D:
    """One 3D FD-CGKS problem (four grids, periodic) on the current HIP device
    (see fdcgks3d_create).  A grid's state is a (20, nz, ny, nx) array: W[5],
    Wx[5], Wy[5], Wz[5]."""

    KERNEL_CLASSES = ("edge1", "node1", "update1", "edge2", "node2", "update2", "step")

    def __init__(self, params: Params3D | None = None, stream=None, **kw):
        self._L = _lib.load()
        self.params = params if params is not None else make_params3d(**kw)
        self._h = C.c_void_p()
        s = _current_stream() if stream is None else C.c_void_p(stream)
        _lib.check(self._L.fdcgks3d_create(C.byref(self.params), s, C.byref(self._h)), None, dim3=True)
        p = self.params
        self.shape = (20, p.nz, p.ny, p.nx)

    def close(self):
        if getattr(self, "_h", None) and self._h.value:
            self._L.fdcgks3d_destroy(self._h)
            self._h = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:  # noqa: BLE001
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()

    def _chk(self, st):
        return _lib.check(st, self._h, dim3=True)

    def set_state(self, grid, S):
        """S: (20, nz, ny, nx) numpy array or torch tensor on the device."""
        if isinstance(S, np.ndarray):
            S = np.ascontiguousarray(S, dtype=np.float64)
        if tuple(S.shape) != self.shape:
            raise ValueError(f"grid state must have shape {self.shape}")
        ptr, dev, keep = _ptr(S)
        self._chk(self._L.fdcgks3d_set_state(self._h, grid, ptr, dev))

    def set_state_all(self, S):
        """S: (4, 20, nz, ny, nx)."""
        for g in range(4):
            self.set_state(g, S[g])

    def get_state(self, grid, device=None):
        if device is None:
            out = np.empty(self.shape)
        else:
            out = _torch().empty(self.shape, dtype=_torch().float64, device=device)
        ptr, dev, keep = _ptr(out, True)
        self._chk(self._L.fdcgks3d_get_state(self._h, grid, ptr, dev))
        return out

    def get_state_all(self):
        return np.stack([self.get_state(g) for g in range(4)])

    def compute_dt(self, cfl):
        d = C.c_double()
        self._chk(self._L.fdcgks3d_compute_dt(self._h, cfl, C.byref(d)))
        return d.value

    def diagnostics(self):
        out = np.zeros(22)
        self._chk(self._L.fdcgks3d_diagnostics(self._h, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def step(self, nsteps=1, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
        """Returns (t, steps_done)."""
        tt = C.c_double(t)
        n = C.c_int32()
        self._chk(self._L.fdcgks3d_step(self._h, dt, cfl, nsteps, t_end, C.byref(tt), C.byref(n)))
        return tt.value, n.value

    def step_timed(self, nsteps=1, dt=0.0, cfl=0.5, t_end=0.0, t=0.0):
        """step() with per-kernel device milliseconds: (t, steps, {class: ms})."""
        tt = C.c_double(t)
        n = C.c_int32()
        ms = (C.c_double * 7)()
        self._chk(self._L.fdcgks3d_step_timed(self._h, dt, cfl, nsteps, t_end, C.byref(tt), C.byref(n), ms))
        return tt.value, n.value, dict(zip(self.KERNEL_CLASSES, list(ms)))

    def debug_stage(self, stage, dt):
        """(state, accumulators) of stage 1 or the state of stage 2, each
        (4, 20, nz, ny, nx), without committing the stage."""
        out = np.zeros((4,) + self.shape)
        acc = np.zeros_like(out)
        self._chk(self._L.fdcgks3d_debug_stage(self._h, stage, dt, C.c_void_p(out.ctypes.data),
                                               C.c_void_p(acc.ctypes.data)))
        return (out, acc) if stage == 1 else out

    def debug_intermediates(self, dt):
        """Stage-1 interface records (4 classes, 3 normals, 31, nz, ny, nx) and
        nodal fluxes (4 grids, 30, nz, ny, nx)."""
        p = self.params
        E = np.zeros((4, 3, 31, p.nz, p.ny, p.nx))
        N = np.zeros((4, 30, p.nz, p.ny, p.nx))
        self._chk(self._L.fdcgks3d_debug_intermediates(self._h, dt, C.c_void_p(E.ctypes.data),
                                                       C.c_void_p(N.ctypes.data)))
        return E, N
