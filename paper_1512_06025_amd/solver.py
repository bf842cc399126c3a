"""Torch-facing wrapper of libbbdg: marshals arrays and tensors into the C ABI."""
import ctypes
import functools

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
    """Geometry and connectivity computed by bbdg_mesh_geometry (host arrays),
    with the vertex coordinates and element vertices it came from."""

    def __init__(self, geo, EToE, EToF, EToO, VX=None, EToV=None):
        self.geo, self.EToE, self.EToF, self.EToO = geo, EToE, EToF, EToO
        self.VX, self.EToV = VX, EToV
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
    return MeshData(geo, EToE, EToF, EToO, VX, EToV)


def locate_points(mesh, xyz):
    """(elem (n,) int32, bary (n, 4)) of points xyz (n, 3); raises if a point
    lies outside the mesh."""
    xyz = np.ascontiguousarray(np.atleast_2d(xyz), dtype=np.float64)
    n = xyz.shape[0]
    elem = np.zeros(n, dtype=np.int32)
    bary = np.zeros((n, 4))
    check(load().bbdg_locate_points(mesh.K, mesh.VX.shape[0], mesh.VX.ctypes.data, mesh.EToV.ctypes.data,
                                    n, xyz.ctypes.data, elem.ctypes.data, bary.ctypes.data),
          "bbdg_locate_points")
    return elem, bary


def bernstein_eval(N, bary):
    """(n, Np) Bernstein polynomials of order N at barycentric points (n, 4)."""
    bary = np.ascontiguousarray(np.atleast_2d(bary), dtype=np.float64)
    out = np.zeros((bary.shape[0], np_count(N)))
    check(load().bbdg_bernstein_eval(int(N), bary.shape[0], bary.ctypes.data, out.ctypes.data),
          "bbdg_bernstein_eval")
    return out


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
    comparator applied by MFMA, basis="nodal_ept" the element-per-thread one
    (fields are then nodal values at the lattice points).
    Field tensors are torch CUDA tensors of shape (K, 4, Np) (element-major:
    element k's p, u, v, w coefficients are q[k, 0..3, :]) with dtype
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
        create = {"bb": load().bbdg_create, "nodal": load().bbdg_nodal_create,
                  "nodal_ept": load().bbdg_nodal_ept_create}[basis]
        self.basis = basis
        check(create(ctypes.byref(h), self.N, self.code, self.K,
                     mesh.EToE.ctypes.data, mesh.EToF.ctypes.data, mesh.EToO.ctypes.data,
                     mesh.geo.ctypes.data, c.ctypes.data, bcode, int(device)),
              {"bb": "bbdg_create", "nodal": "bbdg_nodal_create", "nodal_ept": "bbdg_nodal_ept_create"}[basis])
        self._h = h
        self._work = None

    def _check_field(self, t):
        import torch
        if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == self.torch_dtype
                and tuple(t.shape) == (self.K, 4, self.Np) and t.is_contiguous()):
            raise ValueError("expected a contiguous CUDA tensor (%d, 4, %d) of %s"
                             % (self.K, self.Np, self.torch_dtype))

    def empty_field(self):
        import torch
        return torch.empty((self.K, 4, self.Np), dtype=self.torch_dtype, device=self.device)

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

    def set_store_policy(self, policy):
        """"auto", "plain" or "nontemporal" output stores of the FP64 stage
        (a performance choice; results are identical)."""
        code = {"auto": _lib.BBDG_STORES_AUTO, "plain": _lib.BBDG_STORES_PLAIN,
                "nontemporal": _lib.BBDG_STORES_NONTEMPORAL}[policy]
        check(load().bbdg_set_store_policy(self._h, code), "bbdg_set_store_policy")

    def nontemporal_stores(self):
        """True if run() launches the non-temporal-store stage variant."""
        r = load().bbdg_nontemporal_stores(self._h)
        check(r if r < 0 else 0, "bbdg_nontemporal_stores")
        return bool(r)

    def close(self):
        if getattr(self, "_h", None):
            load().bbdg_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchedSolver:
    """Independent shots on one mesh and wavespeed, advanced together in
    persistent kernel launches (up to 1024 steps each).

    sources: (S, 3) source positions (one Ricker point source per shot) or
    None; receivers: (R, 3) positions shared by all shots.  States are CUDA
    tensors (S, K, 4, Np); run() returns the receiver traces (steps, S, R).
    wpb = 0 lets bbdg_tune_batched pick the waves per workgroup on first use."""

    def __init__(self, N, mesh, c, shots, sources=None, receivers=None, f0=8.0, ts=0.125,
                 dtype="f32", bc="rigid", device=0, wpb=0):
        import torch
        self.solver = Solver(N, mesh, c, dtype=dtype, bc=bc, device=device)
        s = self.solver
        self.S = int(shots)
        self.f0, self.ts = float(f0), float(ts)
        self.wpb = int(wpb)
        dev = s.device
        self.src_elem = self.src_coef = None
        self._src = None
        if sources is not None:
            elem, bary = locate_points(mesh, sources)
            if elem.shape[0] != self.S:
                raise ValueError("need one source per shot")
            self._src = (elem, bary)
            self.src_elem = torch.from_numpy(elem).to(dev)
            self.update_sources()
        self.R = 0
        self.rec_elem = self.rec_coef = None
        if receivers is not None and len(receivers):
            elem, bary = locate_points(mesh, receivers)
            self.R = elem.shape[0]
            self.rec_elem = torch.from_numpy(elem).to(dev)
            self.rec_coef = torch.from_numpy(bernstein_eval(N, bary)).to(dev, s.torch_dtype)
        self._work = None

    def update_sources(self):
        """(Re)computes the source vectors, which scale with kappa of the source element."""
        import torch
        if self._src is None:
            return
        s = self.solver
        elem, bary = self._src
        coef = np.zeros((self.S, s.Np))
        check(load().bbdg_source_coeffs(s._h, self.S, elem.ctypes.data, bary.ctypes.data, coef.ctypes.data),
              "bbdg_source_coeffs")
        self.src_coef = torch.from_numpy(coef).to(s.device, s.torch_dtype)

    def empty_state(self):
        import torch
        s = self.solver
        return torch.zeros((self.S, s.K, 4, s.Np), dtype=s.torch_dtype, device=s.device)

    def _buffer(self, nbytes):
        import torch
        return torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=self.solver.device)

    def work(self):
        if self._work is None:
            self._work = self._buffer(load().bbdg_batched_work_bytes(self.solver._h, self.S))
        return self._work

    def tune(self, stream=None):
        """Times the launch shapes and keeps the fastest; returns waves per workgroup."""
        s = self.solver
        state = self.S * 4 * s.K * s.Np * (8 if s.dtype == "f64" else 4)
        scratch = self._buffer(load().bbdg_batched_work_bytes(s._h, self.S) + state + 256)
        out = ctypes.c_int(0)
        check(load().bbdg_tune_batched(s._h, self.S, ctypes.c_void_p(scratch.data_ptr()), ctypes.byref(out),
                                       _stream_ptr(stream)), "bbdg_tune_batched")
        del scratch
        self.wpb = out.value
        return self.wpb

    def run(self, q, dt, steps, t0=0.0, traces=None, stream=None):
        """Advance every shot of q in place; returns the traces (steps, S, R)."""
        import torch
        s = self.solver
        if not (isinstance(q, torch.Tensor) and q.is_cuda and q.dtype == s.torch_dtype and q.is_contiguous()
                and tuple(q.shape) == (self.S, s.K, 4, s.Np)):
            raise ValueError("expected a contiguous CUDA tensor (%d, %d, 4, %d) of %s"
                             % (self.S, s.K, s.Np, s.torch_dtype))
        if self.wpb == 0:
            self.tune(stream)
        if traces is None:
            traces = torch.empty((int(steps), self.S, self.R), dtype=s.torch_dtype, device=s.device)
        w = self.work()

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr() if t is not None else None)
        check(load().bbdg_run_batched(s._h, ptr(q), self.S, ptr(self.src_elem), ptr(self.src_coef),
                                      self.f0, self.ts, self.R, ptr(self.rec_elem), ptr(self.rec_coef),
                                      ptr(traces) if self.R else ctypes.c_void_p(None), ptr(w), float(t0),
                                      float(dt), int(steps), self.wpb, _stream_ptr(stream)), "bbdg_run_batched")
        return traces

    def set_barrier_timeout(self, seconds):
        """Longest wait at a grid barrier of the persistent launches (default 2 s)."""
        check(load().bbdg_set_barrier_timeout(self.solver._h, float(seconds)), "bbdg_set_barrier_timeout")

    def check(self):
        """Waits for the device; raises BBDGError (BBDG_E_TIMEOUT) if a grid
        barrier of a run since the last check timed out (outputs are NaN)."""
        check(load().bbdg_status(self.solver._h), "batched run")

    def close(self):
        self.solver.close()


class Misfit:
    """Receiver misfit J(m) = 1/2 sum (d(m) - d_obs)^2 of a batched forward run
    and its gradient in m = c^2 per element (discrete adjoint on the GPU).

    d_obs: CUDA tensor (steps, S, R) of the solver's element type.  evaluate(m)
    sets the wavespeed to sqrt(m), runs the forward problem keeping
    checkpoints every ckpt_every steps, and returns J (0-dim float64 CUDA
    tensor); gradient() then returns dJ/dm (K,) float64 at the model of the
    last evaluate() (it needs that run's checkpoints).  The work space holds
    the stage records of rec_segments checkpoint segments: the forward run
    records its last rec_segments segments and the reverse sweep recomputes
    only the others; "max" takes as many as fit in the free device memory
    less `reserve_bytes` (at least one).  `evaluations` counts the forward
    runs of this object."""

    def __init__(self, N, mesh, m, shots, sources, receivers, d_obs, dt, steps, t0=0.0, f0=8.0, ts=0.125,
                 ckpt_every=0, dtype="f32", bc="rigid", device=0, tune=True, rec_segments=1,
                 reserve_bytes=8 << 30):
        import torch
        m = np.asarray(m, dtype=np.float64)
        self.batched = BatchedSolver(N, mesh, np.sqrt(m), shots, sources=sources, receivers=receivers, f0=f0,
                                     ts=ts, dtype=dtype, bc=bc, device=device, wpb=4)
        if tune:
            self.batched.tune()   # the misfit runs use the handle's tuned launch shape
        s = self.batched.solver
        self.dt, self.steps, self.t0, self.ckpt = float(dt), int(steps), float(t0), int(ckpt_every)
        self.d_obs = d_obs.to(s.device, s.torch_dtype).contiguous()
        if tuple(self.d_obs.shape) != (self.steps, self.batched.S, self.batched.R):
            raise ValueError("d_obs must be (steps, shots, receivers)")
        def work_bytes(m):
            return load().bbdg_misfit_work_bytes(s._h, self.batched.S, self.batched.R, self.steps, self.ckpt, m)
        C = self.steps if self.ckpt <= 0 else min(self.ckpt, self.steps)
        nseg = (self.steps + C - 1) // C
        if rec_segments == "max":
            free = torch.cuda.mem_get_info(s.device)[0] - int(reserve_bytes)
            rec_segments = 1
            while rec_segments < nseg and work_bytes(rec_segments + 1) <= free:
                rec_segments += 1
        self.rec_segments = min(int(rec_segments), nseg)
        nbytes = work_bytes(self.rec_segments) if self.rec_segments >= 1 else 0
        if nbytes == 0:
            raise ValueError("invalid misfit sizes")
        self._work = torch.empty(nbytes // 8 + 32, dtype=torch.float64, device=s.device)
        self._J = torch.zeros((), dtype=torch.float64, device=s.device)
        self._evaluated = False
        self.evaluations = 0

    def _args(self):
        b = self.batched

        def ptr(t):
            return ctypes.c_void_p(t.data_ptr() if t is not None else None)
        return (b.solver._h, b.S, ctypes.c_void_p(None), ptr(b.src_elem), ptr(b.src_coef), b.f0, b.ts, b.R,
                ptr(b.rec_elem), ptr(b.rec_coef), ptr(self.d_obs), self.t0, self.dt, self.steps, self.ckpt,
                self.rec_segments)

    def set_m(self, m):
        import torch
        mh = m.detach().to("cpu", torch.float64).numpy() if isinstance(m, torch.Tensor) else np.asarray(m, np.float64)
        c = np.ascontiguousarray(np.sqrt(mh))
        check(load().bbdg_set_wavespeed(self.batched.solver._h, c.ctypes.data), "bbdg_set_wavespeed")
        self.batched.update_sources()
        self._evaluated = False   # the checkpoints belong to the previous model

    def evaluate(self, m=None, stream=None):
        if m is not None:
            self.set_m(m)
        check(load().bbdg_misfit(*self._args(), ctypes.c_void_p(self._J.data_ptr()),
                                 ctypes.c_void_p(self._work.data_ptr()), _stream_ptr(stream)), "bbdg_misfit")
        self._evaluated = True
        self.evaluations += 1
        return self._J.clone()

    def gradient(self, stream=None):
        import torch
        if not self._evaluated:
            raise RuntimeError("evaluate() first")
        g = torch.empty(self.batched.solver.K, dtype=torch.float64, device=self.batched.solver.device)
        check(load().bbdg_misfit_gradient(*self._args(), ctypes.c_void_p(g.data_ptr()),
                                          ctypes.c_void_p(self._work.data_ptr()), _stream_ptr(stream)),
              "bbdg_misfit_gradient")
        return g

    def check(self):
        """See BatchedSolver.check."""
        self.batched.check()

    def close(self):
        self.batched.close()


@functools.lru_cache(maxsize=None)
def _misfit_function():
    import torch

    class MisfitFunction(torch.autograd.Function):
        """J = MisfitFunction.apply(m, misfit): forward runs the forward
        problem (checkpointed) at m; backward runs the adjoint sweep at the
        same m (re-running the forward problem first if the Misfit was
        evaluated at another model in between), which recomputes each
        segment from its checkpoint, and returns
        grad_output * dJ/dm."""

        @staticmethod
        def forward(ctx, m, misfit):
            J = misfit.evaluate(m)
            ctx.misfit = misfit
            ctx.m = m.detach().clone()
            ctx.evaluation = misfit.evaluations
            return J

        @staticmethod
        def backward(ctx, grad_out):
            mf = ctx.misfit
            # the gradient needs the checkpoints of a forward run at this
            # graph's m; if the Misfit was evaluated since (another graph, a
            # line search), run the forward problem at this m again first
            if mf.evaluations != ctx.evaluation:
                mf.evaluate(ctx.m)
                ctx.evaluation = mf.evaluations
            return grad_out * mf.gradient(), None

    return MisfitFunction
