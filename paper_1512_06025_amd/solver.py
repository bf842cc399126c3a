"""Torch-facing wrapper of libbbdg: marshals arrays and tensors into the C ABI."""
import ctypes

import numpy as np

from . import _lib
from ._lib import check, load


def np_count(N):
    n = load().bbdg_np(int(N))
    check(n if n < 0 else 0, "bbdg_np")
    return n


def alpha_table(N):
    """(Np, 4) int32 multi-indices in storage order."""
    out = np.zeros((np_count(N), 4), dtype=np.int32)
    check(load().bbdg_alpha_table(int(N), out.ctypes.data), "bbdg_alpha_table")
    return out


class MeshData:
    """Geometry and connectivity computed by bbdg_mesh_geometry (host arrays)."""

    def __init__(self, geo, EToE, EToF, EToO):
        self.geo, self.EToE, self.EToF, self.EToO = geo, EToE, EToF, EToO
        self.K = geo.shape[0]


def mesh_geometry(VX, EToV):
    VX = np.ascontiguousarray(VX, dtype=np.float64)
    EToV = np.ascontiguousarray(EToV, dtype=np.int32)
    K, Nv = EToV.shape[0], VX.shape[0]
    geo = np.zeros((K, 10), dtype=np.float64)
    EToE = np.zeros((K, 4), dtype=np.int32)
    EToF = np.zeros((K, 4), dtype=np.int8)
    EToO = np.zeros((K, 4), dtype=np.int8)
    check(load().bbdg_mesh_geometry(K, Nv, VX.ctypes.data, EToV.ctypes.data, geo.ctypes.data,
                                    EToE.ctypes.data, EToF.ctypes.data, EToO.ctypes.data),
          "bbdg_mesh_geometry")
    return MeshData(geo, EToE, EToF, EToO)


def _stream_ptr(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def nodal_operators(N):
    """(dr (3, Np, Np), lift (Np, 4 Nfp)) of the dense nodal comparator."""
    Np = np_count(N)
    Nfp = (N + 1) * (N + 2) // 2
    dr = np.zeros((3, Np, Np))
    lift = np.zeros((Np, 4 * Nfp))
    check(load().bbdg_nodal_operators(int(N), dr.ctypes.data, lift.ctypes.data), "bbdg_nodal_operators")
    return dr, lift


class Solver:
    """One solver handle: order N, element type, mesh, wavespeed, boundary condition.

    basis="bb" is the Bernstein-Bezier solver; basis="nodal" the dense nodal
    comparator (fields are then nodal values at the lattice points).
    Field tensors are torch CUDA tensors of shape (4, K, Np) with dtype
    float64 (dtype="f64") or float32 (dtype="f32")."""

    def __init__(self, N, mesh, c, dtype="f64", bc="rigid", device=0, basis="bb"):
        import torch
        self.N = int(N)
        self.dtype = dtype
        self.code = {"f64": _lib.BBDG_F64, "f32": _lib.BBDG_F32}[dtype]
        self.torch_dtype = torch.float64 if dtype == "f64" else torch.float32
        bcode = {"rigid": _lib.BBDG_BC_RIGID, "pressure_release": _lib.BBDG_BC_PRESSURE_RELEASE}[bc]
        self.K = mesh.K
        self.Np = np_count(self.N)
        self.device = torch.device("cuda", device)
        c = np.ascontiguousarray(np.broadcast_to(np.asarray(c, dtype=np.float64), (self.K,)))
        h = ctypes.c_void_p()
        create = {"bb": load().bbdg_create, "nodal": load().bbdg_nodal_create}[basis]
        self.basis = basis
        check(create(ctypes.byref(h), self.N, self.code, self.K,
                     mesh.EToE.ctypes.data, mesh.EToF.ctypes.data, mesh.EToO.ctypes.data,
                     mesh.geo.ctypes.data, c.ctypes.data, bcode, int(device)),
              "bbdg_create" if basis == "bb" else "bbdg_nodal_create")
        self._h = h
        self._work = None

    def _check_field(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == self.torch_dtype
                and tuple(t.shape) == (4, self.K, self.Np) and t.is_contiguous()):
            raise ValueError("expected a contiguous CUDA tensor (4, %d, %d) of %s"
                             % (self.K, self.Np, self.torch_dtype))

    def empty_field(self):
        import torch
        return torch.empty((4, self.K, self.Np), dtype=self.torch_dtype, device=self.device)

    def rhs(self, q, mode=_lib.BBDG_RHS_FULL, out=None, stream=None):
        self._check_field(q)
        out = self.empty_field() if out is None else out
        self._check_field(out)
        check(load().bbdg_rhs(self._h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(out.data_ptr()),
                              int(mode), _stream_ptr(stream)), "bbdg_rhs")
        return out

    def work(self):
        import torch
        if self._work is None:
            nbytes = load().bbdg_work_bytes(self._h)
            self._work = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=self.device)
        return self._work

    def run(self, q, dt, steps, t0=0.0, stream=None):
        """Advance q in place by `steps` LSRK4 steps of size dt."""
        self._check_field(q)
        w = self.work()
        check(load().bbdg_run(self._h, ctypes.c_void_p(q.data_ptr()), ctypes.c_void_p(w.data_ptr()),
                              float(t0), float(dt), int(steps), _stream_ptr(stream)), "bbdg_run")
        return q

    def close(self):
        if getattr(self, "_h", None):
            load().bbdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
