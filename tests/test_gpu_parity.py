"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Tolerances: relative L2 over all of q of 1e-12 in FP64 and 1e-5 in FP32.
In FP32 runs the oracle starts from the same float32-rounded input.
"""
import numpy as np
import pytest

import workload
from oracle import dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _setup(n, N, jitter=0.1, c=(1.0, 3.0), bc="rigid", drop_last=0):
    import paper_1512_06025_amd as P
    VX, EToV = workload.kuhn_cube_mesh(n, jitter, drop_last=drop_last)
    cc = workload.wavespeed(EToV.shape[0], *c)
    mesh = P.mesh_geometry(VX, EToV)
    prob = dg.Problem(VX, EToV, N, cc, bc)
    return P, mesh, cc, prob


def _to_dev(x, dtype):
    """Oracle state (4, K, Np) -> device field in the library's element-major
    layout (K, 4, Np)."""
    return torch.from_numpy(np.ascontiguousarray(np.swapaxes(x, 0, 1))).to(
        "cuda", torch.float64 if dtype == "f64" else torch.float32)


def _host(x):
    """Device field (K, 4, Np) -> oracle layout (4, K, Np), float64."""
    torch.cuda.synchronize()
    return np.swapaxes(x.detach().to("cpu", torch.float64).numpy(), 0, 1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", list(range(1, 10)))
def test_rhs_parity(N, dtype):
    # 2^3 cubes, 5 elements dropped: ragged element count, interior boundary faces
    P, mesh, c, prob = _setup(2, N, drop_last=5)
    q = workload.random_coeffs(prob.K, prob.Np)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
    s = P.Solver(N, mesh, c, dtype=dtype)
    qd = _to_dev(q, dtype)
    for mode, kw in ((P.BBDG_RHS_VOLUME, dict(surface=False)),
                     (P.BBDG_RHS_SURFACE, dict(volume=False)),
                     (P.BBDG_RHS_FULL, {})):
        got = _host(s.rhs(qd, mode))
        want = prob.rhs(q, **kw)
        err = _rel(got, want)
        assert err < TOL[dtype], (N, dtype, mode, err)
    s.close()


# Every stage-kernel instantiation that bbdg_run can launch: order N, element
# type, and for FP64 plain or non-temporal output stores (the latter is what
# meshes whose fields exceed the last-level cache get; forced here on a small
# mesh).  The instantiations differ in team size (N = 4, 6 and, in FP64,
# 8 and 9 share an element group between several waves), lift batch size,
# late residual loads (FP64 N >= 6, FP32 N >= 8) and stores.
STAGE_CASES = ([(N, "f64", "plain") for N in range(1, 10)] + [(N, "f64", "nontemporal") for N in range(1, 10)]
               + [(N, "f32", "plain") for N in range(1, 10)])


@pytest.mark.parametrize("N,dtype,policy", STAGE_CASES)
def test_stage_every_instantiation(N, dtype, policy):
    """One LSRK4 step (five fused stage launches; the first reads no
    residual) on 155 jittered tets with c ~ U[1,3] and interior boundary
    faces, every coefficient against the oracle."""
    P, mesh, c, prob = _setup(3, N, drop_last=7)
    q = workload.random_coeffs(prob.K, prob.Np, seed=50 + N)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
    s = P.Solver(N, mesh, c, dtype=dtype)
    s.set_store_policy(policy)
    assert s.nontemporal_stores() == (policy == "nontemporal")
    qd = _to_dev(q, dtype)
    dt = 0.4 / (3.0 * 3 * (N + 1) ** 2)
    s.run(qd, dt, 1)
    err = _rel(_host(qd), prob.lsrk4(q, dt, 1))
    assert err < TOL[dtype], (N, dtype, policy, err)
    s.close()


def test_store_policy_arguments():
    P, mesh, c, prob = _setup(2, 3)
    s = P.Solver(3, mesh, c, dtype="f64")
    assert not s.nontemporal_stores()          # 48 tets: auto picks plain stores
    s.set_store_policy("nontemporal")
    assert s.nontemporal_stores()
    from paper_1512_06025_amd import _lib
    assert _lib.load().bbdg_set_store_policy(s._h, 3) == -1
    s.close()
    s32 = P.Solver(3, mesh, c, dtype="f32")
    s32.set_store_policy("nontemporal")
    assert not s32.nontemporal_stores()       # FP32 has plain stores only
    s32.close()


@pytest.mark.parametrize("bc", ["rigid", "pressure_release"])
def test_rhs_parity_boundary_conditions(bc):
    P, mesh, c, prob = _setup(3, 4, bc=bc)
    q = workload.random_coeffs(prob.K, prob.Np)
    s = P.Solver(4, mesh, c, dtype="f64", bc=bc)
    got = _host(s.rhs(_to_dev(q, "f64")))
    assert _rel(got, prob.rhs(q)) < 1e-12
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_run_parity_c1(dtype):
    """384 tets, N=3, c=1, standing mode, rigid walls, dt = 0.5 h/(N+1)^2, 10 steps."""
    import paper_1512_06025_amd as P
    cfg, VX, EToV, c = workload.build_preset("c1")
    prob = dg.Problem(VX, EToV, cfg["N"], c)
    q0 = dg.initial_state(prob, workload.standing_mode_p0)
    if dtype == "f32":
        q0 = q0.astype(np.float32).astype(np.float64)
    want = prob.lsrk4(q0, cfg["dt"], cfg["steps"])
    s = P.Solver(cfg["N"], P.mesh_geometry(VX, EToV), c, dtype=dtype)
    qd = _to_dev(q0, dtype)
    s.run(qd, cfg["dt"], cfg["steps"])
    err = _rel(_host(qd), want)
    assert err < TOL[dtype], err
    s.close()


@pytest.mark.parametrize("steps", [0, 1, 2, 3])
def test_run_step_counts(steps):
    """Odd and even stage counts (the ping-pong buffer ends in either place)."""
    P, mesh, c, prob = _setup(2, 2, drop_last=1)
    q = workload.random_coeffs(prob.K, prob.Np)
    dt = 1e-3
    s = P.Solver(2, mesh, c)
    qd = _to_dev(q, "f64")
    s.run(qd, dt, steps)
    assert _rel(_host(qd), prob.lsrk4(q, dt, steps)) < 1e-12
    s.close()


def test_run_resume_is_bitwise():
    """run(10) equals run(4) followed by run(6) from t0 + 4 dt bit for bit:
    a run keeps no state between calls beyond q (the residual is
    overwritten by the first stage of every step)."""
    P, mesh, c, prob = _setup(2, 4, drop_last=3)
    q0 = workload.random_coeffs(prob.K, prob.Np, seed=91)
    dt = 2.0 ** -10
    for dtype in ("f64", "f32"):
        s = P.Solver(4, mesh, c, dtype=dtype)
        a = _to_dev(q0, dtype)
        b = a.clone()
        s.run(a, dt, 10)
        s.run(b, dt, 4)
        s.run(b, dt, 6, t0=4 * dt)
        torch.cuda.synchronize()
        assert torch.equal(a, b), dtype
        s.close()


def test_run_is_bitwise_repeatable():
    P, mesh, c, prob = _setup(3, 5)
    q = workload.random_coeffs(prob.K, prob.Np)
    s = P.Solver(5, mesh, c)
    a, b = _to_dev(q, "f64"), _to_dev(q, "f64")
    s.run(a, 1e-3, 3)
    s.run(b, 1e-3, 3)
    assert torch.equal(a, b)
    s.close()


# ---- dense nodal comparator -------------------------------------------------
# Nodal values are V c (V the Bernstein-Vandermonde matrix of the lattice);
# the comparator's result is compared with V (oracle RHS of c).  The change of
# basis (condition number of V up to ~1e3 at N = 9) loosens the FP64 bar to
# 1e-10; FP32 operators and dense sums of up to 4 Nfp terms give 1e-4.
NODAL_TOL = {"f64": 1e-10, "f32": 1e-4}


def _lattice_vandermonde(N):
    from oracle import bernstein as bb
    return dg.bernstein_eval(N, np.array(bb.multi_indices(N), float) / N)


NODAL_KINDS = ["nodal", "nodal_ept"]  # MFMA and element-per-thread comparators


@pytest.mark.parametrize("basis", NODAL_KINDS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", list(range(1, 10)))
def test_nodal_rhs_parity(N, dtype, basis):
    P, mesh, c, prob = _setup(2, N, drop_last=5)
    V = _lattice_vandermonde(N)
    cq = workload.random_coeffs(prob.K, prob.Np)
    x = cq @ V.T
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
        cq = x @ np.linalg.inv(V).T
    s = P.Solver(N, mesh, c, dtype=dtype, basis=basis)
    xd = _to_dev(x, dtype)
    for mode, kw in ((P.BBDG_RHS_VOLUME, dict(surface=False)),
                     (P.BBDG_RHS_SURFACE, dict(volume=False)),
                     (P.BBDG_RHS_FULL, {})):
        got = _host(s.rhs(xd, mode))
        want = prob.rhs(cq, **kw) @ V.T
        err = _rel(got, want)
        assert err < NODAL_TOL[dtype], (N, dtype, basis, mode, err)
    s.close()


@pytest.mark.parametrize("basis", NODAL_KINDS)
@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_nodal_run_parity_c1(dtype, basis):
    import paper_1512_06025_amd as P
    cfg, VX, EToV, c = workload.build_preset("c1")
    prob = dg.Problem(VX, EToV, cfg["N"], c)
    V = _lattice_vandermonde(cfg["N"])
    q0 = dg.initial_state(prob, workload.standing_mode_p0)
    x0 = q0 @ V.T
    if dtype == "f32":
        x0 = x0.astype(np.float32).astype(np.float64)
        q0 = x0 @ np.linalg.inv(V).T
    want = prob.lsrk4(q0, cfg["dt"], cfg["steps"]) @ V.T
    s = P.Solver(cfg["N"], P.mesh_geometry(VX, EToV), c, dtype=dtype, basis=basis)
    xd = _to_dev(x0, dtype)
    s.run(xd, cfg["dt"], cfg["steps"])
    err = _rel(_host(xd), want)
    assert err < NODAL_TOL[dtype], (basis, err)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [3, 6, 9])
def test_nodal_ept_stage_parity(N, dtype):
    """One LSRK4 step of the element-per-thread comparator (fused volume,
    flux, lift and update over several row blocks for N >= 3 in FP64) on a
    ragged jittered mesh with c ~ U[1,3], against V (oracle step)."""
    P, mesh, c, prob = _setup(3, N, drop_last=7)
    V = _lattice_vandermonde(N)
    cq = workload.random_coeffs(prob.K, prob.Np, seed=60 + N)
    x = cq @ V.T
    if dtype == "f32":
        x = x.astype(np.float32).astype(np.float64)
        cq = x @ np.linalg.inv(V).T
    dt = 0.5 / (3 * 3.0 * (N + 1) ** 2)
    want = prob.lsrk4(cq, dt, 1) @ V.T
    s = P.Solver(N, mesh, c, dtype=dtype, basis="nodal_ept")
    xd = _to_dev(x, dtype)
    s.run(xd, dt, 1)
    err = _rel(_host(xd), want)
    assert err < NODAL_TOL[dtype], (N, dtype, err)
    s.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [3, 5])
def test_set_wavespeed_then_step(N, dtype):
    """bbdg_set_wavespeed replaces the wavespeed of an existing handle (the
    upwind weights of the header and the per-element geometry the stage
    kernels load, precomputed on the host): one LSRK4 step after the switch
    matches the oracle built with the new wavespeed, on every coefficient."""
    from paper_1512_06025_amd import _lib
    P, mesh, c_old, _ = _setup(3, N, c=(1.0, 3.0), drop_last=7)
    c_new = np.ascontiguousarray(workload.wavespeed(c_old.shape[0], 0.5, 2.0, seed=123))
    assert np.abs(c_new - c_old).max() > 0.1
    VX, EToV = workload.kuhn_cube_mesh(3, 0.1, drop_last=7)
    prob = dg.Problem(VX, EToV, N, c_new)
    q = workload.random_coeffs(prob.K, prob.Np, seed=80 + N)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
    s = P.Solver(N, mesh, c_old, dtype=dtype)
    _lib.check(_lib.load().bbdg_set_wavespeed(s._h, c_new.ctypes.data), "bbdg_set_wavespeed")
    qd = _to_dev(q, dtype)
    dt = 0.4 / (3.0 * 3 * (N + 1) ** 2)
    s.run(qd, dt, 1)
    err = _rel(_host(qd), prob.lsrk4(q, dt, 1))
    assert err < TOL[dtype], (N, dtype, err)
    s.close()
