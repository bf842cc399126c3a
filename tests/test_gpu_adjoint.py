"""Misfit gradient (discrete adjoint on the GPU) against the FP64 oracle
adjoint, central differences of the GPU misfit, and the autograd wrapper."""
import numpy as np
import pytest

import workload
from oracle import adjoint

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

F0, TS = 8.0, 0.125


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _case(N, bc="rigid", shots=2, nrec=3, steps=6, seed=1):
    VX, EToV = workload.kuhn_cube_mesh(2, 0.1, drop_last=3)
    K = EToV.shape[0]
    m = workload.wavespeed(K, 1.0, 2.0) ** 2
    rng = np.random.default_rng(seed)
    src = rng.uniform(0.1, 0.45, (shots, 3))
    rec = rng.uniform(0.1, 0.45, (nrec, 3))
    obs = rng.standard_normal((steps, shots, nrec)) * 1e-3
    return VX, EToV, m, src, rec, obs


def _gpu_misfit(P, VX, EToV, m, src, rec, obs, N, dtype, ckpt, bc="rigid", dt=2e-3, t0=0.08, rec_segments=1):
    mesh = P.mesh_geometry(VX, EToV)
    d = torch.from_numpy(obs)
    return P.Misfit(N, mesh, m, src.shape[0], src, rec, d, dt, obs.shape[0], t0=t0, f0=F0, ts=TS,
                    ckpt_every=ckpt, dtype=dtype, bc=bc, rec_segments=rec_segments)


def _oracle(VX, EToV, m, src, rec, obs, N, bc="rigid", dt=2e-3, t0=0.08):
    A = adjoint.Adjoint(VX, EToV, N, m, bc)
    p = A.prob
    se, sl = p.locate(src)
    re, rl = p.locate(rec)
    q0 = np.zeros((src.shape[0], 4, p.K, p.Np))
    return A.gradient(q0, dt, obs.shape[0], se, sl, F0, TS, re, rl, obs, t0)


def _J_bar(VX, EToV, m, src, rec, obs, N, bc="rigid", dt=2e-3, t0=0.08, tol=1e-12):
    """Rounding bound of J = 1/2 sum r^2, r = d - d_obs: each trace d is a
    dot product of receiver weights and coefficients whose error is bounded
    by tol * sum_n |W_rn| |p_n| (its own terms, which cancel by up to a few
    hundred at N = 9), so |dJ| <= tol * sum |r| sum_n |W_rn| |p_n|, plus the
    summation of J itself."""
    A = adjoint.Adjoint(VX, EToV, N, m, bc)
    p = A.prob
    se, sl = p.locate(src)
    re, rl = p.locate(rec)
    q0 = np.zeros((src.shape[0], 4, p.K, p.Np))
    _, tr, sc = p.run_shots(q0, dt, obs.shape[0], se, sl, F0, TS, re, rl, t0, trace_scales=True)
    r = tr - obs
    return tol * float(np.sum(np.abs(r) * sc)) + 1e-13 * 0.5 * float(np.sum(r ** 2))


@pytest.mark.parametrize("N,ckpt,bc", [(1, 0, "rigid"), (2, 0, "rigid"), (3, 4, "rigid"), (4, 1, "rigid"),
                                       (5, 2, "rigid"), (3, 0, "pressure_release"), (6, 3, "rigid"),
                                       (7, 2, "rigid"), (8, 0, "rigid"), (9, 4, "pressure_release")])
def test_gradient_matches_oracle_fp64(N, ckpt, bc):
    import paper_1512_06025_amd as P
    VX, EToV, m, src, rec, obs = _case(N)
    J0, g0 = _oracle(VX, EToV, m, src, rec, obs, N, bc)
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, N, "f64", ckpt, bc)
    J = float(mf.evaluate().item())
    g = mf.gradient().cpu().numpy()
    bar = _J_bar(VX, EToV, m, src, rec, obs, N, bc)
    assert abs(J - J0) <= bar, (J, J0, bar)
    assert _rel(g, g0) < 1e-10, _rel(g, g0)
    # a second gradient of the same forward run: the last segment, which the
    # forward run recorded, is now recomputed (its records were overwritten
    # by the earlier segments) with the same arithmetic
    g2 = mf.gradient().cpu().numpy()
    assert np.array_equal(g, g2)
    mf.check()
    mf.close()


def test_gradient_fp32_states():
    """FP32 states with FP64 accumulation, against the FP64 oracle adjoint."""
    import paper_1512_06025_amd as P
    VX, EToV, m, src, rec, obs = _case(3)
    J0, g0 = _oracle(VX, EToV, m, src, rec, obs, 3)
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, 3, "f32", 2)
    J = float(mf.evaluate().item())
    g = mf.gradient().cpu().numpy()
    assert abs(J - J0) < 1e-5 * abs(J0)
    assert _rel(g, g0) < 1e-4, _rel(g, g0)
    mf.close()


@pytest.mark.parametrize("dtype,N", [("f64", 3), ("f32", 5)])
def test_record_slots(dtype, N):
    """Records of several checkpoint segments in the work space (7 steps,
    checkpoints every 2: four segments).  With M slots the forward run records
    the last M segments and the reverse sweep recomputes the others; the
    records of a segment come from the same recording launch on the same
    checkpoint either way, so J and dJ/dm match the one-slot run (up to the
    rounding of traces from the recording launch) and the FP64 oracle
    adjoint; a second gradient of the same forward run (slots reused in
    another order) is bitwise the first."""
    import paper_1512_06025_amd as P
    from paper_1512_06025_amd import _lib
    VX, EToV, m, src, rec, obs = _case(N, steps=7)
    J0, g0 = _oracle(VX, EToV, m, src, rec, obs, N)
    tol_same, tol_oracle = (1e-13, 1e-10) if dtype == "f64" else (1e-6, 1e-4)
    # one more slot adds one 2-step segment's records: the pressure right-hand
    # side of every element and the jumps of every distinct face (once)
    mesh = P.mesh_geometry(VX, EToV)
    EToE = np.asarray(mesh.EToE).reshape(-1, 4)
    K = EToE.shape[0]
    F = int(np.sum((EToE < 0) | (np.arange(K)[:, None] <= EToE)))
    Np, Nfp = (N + 1) * (N + 2) * (N + 3) // 6, (N + 1) * (N + 2) // 2
    w = 8 if dtype == "f64" else 4

    def al(b):
        return (b + 255) // 256 * 256
    S = src.shape[0]
    slot_p, slot_j = 5 * 2 * S * K * Np * w, 5 * 2 * S * F * 2 * Nfp * w  # bytes per slot
    ref = None
    for M in (1, 2, 3, 4, 9):
        mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, N, dtype, 2, rec_segments=M)
        assert mf.rec_segments == min(M, 4)
        lib, h = _lib.load(), mf.batched.solver._h
        b1 = lib.bbdg_misfit_work_bytes(h, S, rec.shape[0], 7, 2, 1)
        Mc = min(M, 4)
        grow = al(Mc * slot_p) + al(Mc * slot_j) - al(slot_p) - al(slot_j)
        assert lib.bbdg_misfit_work_bytes(h, S, rec.shape[0], 7, 2, M) - b1 == grow, (M, grow)
        J = float(mf.evaluate().item())
        g = mf.gradient().cpu().numpy()
        g2 = mf.gradient().cpu().numpy()
        assert np.array_equal(g, g2), M
        assert _rel(g, g0) < tol_oracle, (M, _rel(g, g0))
        if ref is None:
            ref = (J, g)
        else:
            assert abs(J - ref[0]) <= tol_same * abs(ref[0]), (M, J, ref[0])
            assert _rel(g, ref[1]) < tol_same, (M, _rel(g, ref[1]))
        if M == 2:
            # rec_segments below 1 is an argument error at the boundary
            args = list(mf._args())
            args[-1] = 0
            rc = _lib.load().bbdg_misfit(*args, _lib.ctypes.c_void_p(mf._J.data_ptr()),
                                         _lib.ctypes.c_void_p(mf._work.data_ptr()), _lib.ctypes.c_void_p(None))
            assert _lib.ERRORS[rc] == "BBDG_E_ARG"
        mf.check()
        mf.close()
    with pytest.raises(ValueError):
        _gpu_misfit(P, VX, EToV, m, src, rec, obs, N, dtype, 2, rec_segments=0)
    # "max": as many slots as the free device memory holds -- here all four
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, N, dtype, 2, rec_segments="max")
    assert mf.rec_segments == 4
    mf.evaluate()
    assert _rel(mf.gradient().cpu().numpy(), ref[1]) < tol_same
    mf.close()


def test_receivers_sharing_an_element():
    """Several receivers in one element (two at the same point): the adjoint
    source of that element sums all of their residuals."""
    import paper_1512_06025_amd as P
    VX, EToV, m, src, _, _ = _case(3)
    rec = np.array([[0.2, 0.2, 0.2], [0.2, 0.2, 0.2], [0.21, 0.2, 0.19], [0.4, 0.3, 0.2], [0.3, 0.1, 0.35]])
    obs = np.random.default_rng(5).standard_normal((6, src.shape[0], rec.shape[0])) * 1e-3
    re, _ = adjoint.Adjoint(VX, EToV, 3, m).prob.locate(rec)
    assert re[0] == re[1] == re[2], re
    J0, g0 = _oracle(VX, EToV, m, src, rec, obs, 3)
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, 3, "f64", 2)
    J = float(mf.evaluate().item())
    g = mf.gradient().cpu().numpy()
    assert abs(J - J0) <= _J_bar(VX, EToV, m, src, rec, obs, 3), (J, J0)
    assert _rel(g, g0) < 1e-10, _rel(g, g0)
    mf.check()
    mf.close()


def test_gradient_against_gpu_finite_differences():
    """Central differences of the GPU FP64 misfit at the elements with the largest gradient."""
    import paper_1512_06025_amd as P
    VX, EToV, m, src, rec, obs = _case(3)
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, 3, "f64", 0)
    mf.evaluate()
    g = mf.gradient().cpu().numpy()
    for k in np.argsort(-np.abs(g))[:4]:
        eps = 1e-4 * m[k]
        mp, mm = m.copy(), m.copy()
        mp[k] += eps
        mm[k] -= eps
        fd = (float(mf.evaluate(mp).item()) - float(mf.evaluate(mm).item())) / (2 * eps)
        assert abs(fd - g[k]) < 1e-6 * abs(g[k]), (k, fd, g[k])
    mf.close()


def test_autograd_two_graphs_before_backward():
    """Two forward evaluations at different models before either backward:
    each backward returns the gradient at its own model (the Misfit re-runs
    the forward problem when it was evaluated elsewhere in between)."""
    import paper_1512_06025_amd as P
    VX, EToV, m1, src, rec, obs = _case(2)
    m2 = m1 * (1.0 + 0.2 * np.sin(np.arange(m1.size)))
    mf = _gpu_misfit(P, VX, EToV, m1, src, rec, obs, 2, "f64", 2)
    t1 = torch.tensor(m1, dtype=torch.float64, device="cuda", requires_grad=True)
    t2 = torch.tensor(m2, dtype=torch.float64, device="cuda", requires_grad=True)
    J1 = P.MisfitFunction.apply(t1, mf)
    J2 = P.MisfitFunction.apply(t2, mf)
    J1.backward()
    J2.backward()
    for t, m, J in ((t1, m1, J1), (t2, m2, J2)):
        J0, g0 = _oracle(VX, EToV, m, src, rec, obs, 2)
        assert abs(float(J.item()) - J0) < 1e-12 * abs(J0)
        assert _rel(t.grad.cpu().numpy(), g0) < 1e-10
    # a gradient after set_m without a new forward run is refused
    mf.set_m(m1)
    with pytest.raises(RuntimeError):
        mf.gradient()
    mf.close()


def test_autograd_function():
    import paper_1512_06025_amd as P
    VX, EToV, m, src, rec, obs = _case(2)
    mf = _gpu_misfit(P, VX, EToV, m, src, rec, obs, 2, "f64", 0)
    mt = torch.tensor(m, dtype=torch.float64, device="cuda", requires_grad=True)
    J = P.MisfitFunction.apply(mt, mf)
    (3.0 * J).backward()
    J0, g0 = _oracle(VX, EToV, m, src, rec, obs, 2)
    assert abs(float(J.item()) - J0) < 1e-12 * abs(J0)
    assert _rel(mt.grad.cpu().numpy(), 3.0 * g0) < 1e-10
    mf.close()
