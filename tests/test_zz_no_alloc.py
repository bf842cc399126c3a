"""bbdg_run_noalloc: bbdg_run with its work space in the library's static
device array (for callers that cannot allocate), called through the C ABI.

It must give bbdg_run's results bit for bit (same kernels, same arithmetic;
only the work-space address differs), which in turn match the FP64 oracle to
1e-12 (FP64) / 1e-5 (FP32) relative L2.  Two calls in a row, the second on a
smaller problem, show that the array's leftover contents from the first call
do not leak into the second.  A problem whose work space exceeds the array is
refused before anything runs.
"""
import ctypes

import numpy as np
import pytest

import workload
from oracle import dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _create(lib, N, dtype, VX, EToV, c):
    from paper_1512_06025_amd import _lib
    import paper_1512_06025_amd as P
    mesh = P.mesh_geometry(VX, EToV)
    h = ctypes.c_void_p()
    code = _lib.BBDG_F64 if dtype == "f64" else _lib.BBDG_F32
    cc = np.ascontiguousarray(c, dtype=np.float64)
    _lib.check(lib.bbdg_create(ctypes.byref(h), N, code, mesh.K, mesh.EToE.ctypes.data, mesh.EToF.ctypes.data,
                               mesh.EToO.ctypes.data, mesh.geo.ctypes.data, cc.ctypes.data,
                               _lib.BBDG_BC_RIGID, 0), "bbdg_create")
    return h


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_noalloc_matches_run_twice(dtype):
    from paper_1512_06025_amd import _lib
    lib = _lib.load()
    tdt = torch.float64 if dtype == "f64" else torch.float32
    stream = torch.cuda.current_stream()
    sp = ctypes.c_void_p(stream.cuda_stream)
    # (cubes per edge, order, steps, elements dropped): the second call is the
    # smaller problem; odd step counts end on the second buffer (final copy)
    cases = [(5, 6, 3, 11), (2, 3, 2, 5)]
    for n, N, steps, drop in cases:
        VX, EToV = workload.kuhn_cube_mesh(n, 0.1, drop_last=drop)
        K = EToV.shape[0]
        c = workload.wavespeed(K, 1.0, 3.0)
        h = _create(lib, N, dtype, VX, EToV, c)
        try:
            Np = lib.bbdg_np(N)
            wb = lib.bbdg_work_bytes(h)
            assert 0 < wb <= _lib.BBDG_NOALLOC_WORK_BYTES
            q0 = workload.random_coeffs(K, Np, seed=70 + N)
            if dtype == "f32":
                q0 = q0.astype(np.float32).astype(np.float64)
            dt = 0.5 / (n * 3.0 * (N + 1) ** 2)
            # the library's element-major field layout (K, 4, Np)
            qa = torch.from_numpy(np.ascontiguousarray(np.swapaxes(q0, 0, 1))).to("cuda", tdt)
            qb = qa.clone()
            work = torch.empty(wb // qa.element_size(), dtype=tdt, device="cuda")
            _lib.check(lib.bbdg_run(h, qa.data_ptr(), work.data_ptr(), 0.0, dt, steps, sp), "bbdg_run")
            _lib.check(lib.bbdg_run_noalloc(h, qb.data_ptr(), 0.0, dt, steps, sp), "bbdg_run_noalloc")
            torch.cuda.synchronize()
            assert torch.equal(qa, qb), (n, N, dtype)
            prob = dg.Problem(VX, EToV, N, c)
            want = prob.lsrk4(q0, dt, steps)
            got = np.swapaxes(qb.to("cpu", torch.float64).numpy(), 0, 1)
            err = float(np.linalg.norm(got - want) / np.linalg.norm(want))
            assert err < TOL[dtype], (n, N, dtype, err)
            del work
        finally:
            lib.bbdg_destroy(h)


def test_noalloc_refuses_too_large():
    from paper_1512_06025_amd import _lib
    lib = _lib.load()
    # 16^3 x 6 = 24,576 tets at N = 5 in FP64: 2 x 4 K Np doubles = 88 MB of work
    VX, EToV = workload.kuhn_cube_mesh(16, 0.0)
    h = _create(lib, 5, "f64", VX, EToV, np.ones(EToV.shape[0]))
    try:
        assert lib.bbdg_work_bytes(h) > _lib.BBDG_NOALLOC_WORK_BYTES
        q = torch.zeros(1, dtype=torch.float64, device="cuda")
        rc = lib.bbdg_run_noalloc(h, q.data_ptr(), 0.0, 1e-3, 1, None)
        assert rc == -13 and _lib.ERRORS[rc] == "BBDG_E_TOOBIG"
        torch.cuda.synchronize()
        assert q.item() == 0.0
    finally:
        lib.bbdg_destroy(h)
