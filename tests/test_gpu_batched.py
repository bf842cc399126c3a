"""Batched shots (one persistent cooperative launch) against the FP64 oracle.

Each shot is an independent forward run with its own Ricker point source;
all shots share the receivers.  Final states and receiver traces are
compared with the oracle's per-shot runs (relative L2 1e-12 in FP64, 1e-5 in
FP32); source and receiver element ids must match exactly.
"""
import numpy as np
import pytest

import workload
from oracle import dg

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = {"f64": 1e-12, "f32": 1e-5}
F0, TS = 8.0, 0.125


def _rel(a, b):
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def _host(x):
    torch.cuda.synchronize()
    return x.detach().to("cpu", torch.float64).numpy()


def _host_state(q):
    """Device shots (S, K, 4, Np) -> oracle layout (S, 4, K, Np), float64."""
    return np.swapaxes(_host(q), 1, 2)


def _dev_state(q0, dtype):
    """Oracle shots (S, 4, K, Np) -> the library's element-major (S, K, 4, Np)."""
    return torch.from_numpy(np.ascontiguousarray(np.swapaxes(q0, 1, 2))).to("cuda", dtype)


def _case(N, n=2, drop_last=5, shots=4, nrec=5, seed=3):
    import paper_1512_06025_amd as P
    VX, EToV = workload.kuhn_cube_mesh(n, 0.1, drop_last=drop_last)
    c = workload.wavespeed(EToV.shape[0], 1.0, 3.0)
    mesh = P.mesh_geometry(VX, EToV)
    prob = dg.Problem(VX, EToV, N, c)
    rng = np.random.default_rng(seed)
    # keep points inside the part of the cube that drop_last leaves meshed
    src = rng.uniform(0.1, 0.45, (shots, 3))
    rec = rng.uniform(0.1, 0.45, (nrec, 3))
    return P, mesh, c, prob, src, rec


@pytest.mark.parametrize("wpb", [4])
@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [1, 3, 4, 6, 8, 9])
def test_batched_parity(N, dtype, wpb, steps=7):
    """N = 9 in FP64 with four waves per workgroup runs one element per
    four-wave team; the other cases one wave per element group."""
    P, mesh, c, prob, src, rec = _case(N)
    S, dt, t0 = src.shape[0], 2e-3, 0.08   # 7 steps, odd stage count: result in the second buffer
    bs = P.BatchedSolver(N, mesh, c, S, sources=src, receivers=rec, f0=F0, ts=TS, dtype=dtype, wpb=wpb)
    # shot S-1 has no source but a nonzero initial state
    bs.src_elem[S - 1] = -1
    q0 = np.zeros((S, 4, prob.K, prob.Np))
    q0[S - 1] = workload.random_coeffs(prob.K, prob.Np, seed=77)
    if dtype == "f32":
        q0 = q0.astype(np.float32).astype(np.float64)
    q = _dev_state(q0, bs.solver.torch_dtype)
    tr = bs.run(q, dt, steps, t0=t0)

    se, sl = prob.locate(src)
    re, rl = prob.locate(rec)
    np.testing.assert_array_equal(_host(bs.src_elem)[:-1], se[:-1])
    np.testing.assert_array_equal(_host(bs.rec_elem), re)
    se[-1] = -1
    want_q, want_tr, scale = prob.run_shots(q0, dt, steps, se, sl, F0, TS, re, rl, t0=t0, trace_scales=True)
    assert _rel(_host_state(q), want_q) < TOL[dtype]
    for s in range(S):
        assert _rel(_host_state(q)[s], want_q[s]) < TOL[dtype], s
    assert tr.shape == (steps, S, len(rec))
    # a trace is a linear functional sum_n W_rn p_n whose terms cancel (by a
    # factor of several hundred at N = 9 on this rough initial state), so the
    # rounding error of each trace is bounded relative to the size of its own
    # terms, sum_n |W_rn| |p_n| at that step and shot (from the oracle's
    # state), not relative to the trace; a trace whose terms are all zero
    # must be zero
    err = np.abs(_host(tr) - want_tr)
    bad = np.argwhere(err > TOL[dtype] * scale)
    assert bad.size == 0, [(tuple(i), err[tuple(i)], scale[tuple(i)]) for i in bad[:5]]
    bs.check()
    bs.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_batched_resume_is_bitwise(dtype):
    """A forced run of 10 steps equals 4 steps followed by 6 steps from
    t0 + 4 dt, bit for bit in states and traces: with dt a power of two the
    second launch's wavelet table sees exactly the same stage times."""
    P, mesh, c, prob, src, rec = _case(3)
    S, dt, t0 = src.shape[0], 2.0 ** -10, 0.0625
    bs = P.BatchedSolver(3, mesh, c, S, sources=src, receivers=rec, f0=F0, ts=TS, dtype=dtype, wpb=4)
    qa = bs.empty_state()
    qb = bs.empty_state()
    ta = bs.run(qa, dt, 10, t0=t0).clone()
    tb1 = bs.run(qb, dt, 4, t0=t0).clone()
    tb2 = bs.run(qb, dt, 6, t0=t0 + 4 * dt).clone()
    torch.cuda.synchronize()
    bs.check()
    assert torch.equal(qa, qb)
    assert torch.equal(ta, torch.cat([tb1, tb2]))
    assert float(qa.abs().max()) > 0  # the sources acted
    bs.close()


def test_barrier_timeout_drains_and_reports():
    """A zero barrier time limit (forced from the host) times every grid
    barrier out: the launch still ends, q and the traces come back NaN, the
    status reports BBDG_E_TIMEOUT once, and a run with the default limit is
    then correct again."""
    P, mesh, c, prob, src, rec = _case(3)
    S, dt, steps = src.shape[0], 2e-3, 3
    bs = P.BatchedSolver(3, mesh, c, S, sources=src, receivers=rec, f0=F0, ts=TS, dtype="f64", wpb=4)
    for bad in (-1.0, float("nan"), 1e9):
        with pytest.raises(P.BBDGError) as err:
            bs.set_barrier_timeout(bad)
        assert err.value.code == -1
    bs.set_barrier_timeout(0.0)
    q = bs.empty_state()
    tr = bs.run(q, dt, steps, t0=0.1)
    with pytest.raises(P.BBDGError) as err:
        bs.check()
    assert err.value.code == -12
    assert np.isnan(_host(q)).all() and np.isnan(_host(tr)).all()
    bs.check()   # the flag was cleared
    bs.set_barrier_timeout(2.0)
    q = bs.empty_state()
    tr = bs.run(q, dt, steps, t0=0.1)
    bs.check()
    se, sl = prob.locate(src)
    re, rl = prob.locate(rec)
    want_q, want_tr = prob.run_shots(np.zeros((S, 4, prob.K, prob.Np)), dt, steps, se, sl, F0, TS, re, rl, t0=0.1)
    assert _rel(_host_state(q), want_q) < TOL["f64"]
    bs.close()


def test_batched_parity_n9_one_wave_per_element():
    """N = 9 FP64 with two waves per workgroup: one wave per element."""
    test_batched_parity(9, "f64", 2)


def test_batched_parity_across_launches():
    """1027 steps: two persistent launches (1024 steps, then 3), each with its
    own wavelet table; the second ends on an odd stage count."""
    test_batched_parity(1, "f64", 4, steps=1027)


def test_launch_shapes_agree_bitwise():
    """Waves per workgroup change only the work distribution, not the arithmetic."""
    P, mesh, c, prob, src, rec = _case(3, n=3, drop_last=0, shots=3)
    outs = []
    for wpb in (2, 4, 8):
        bs = P.BatchedSolver(3, mesh, c, 3, sources=src, receivers=rec, dtype="f64", wpb=wpb)
        q = bs.empty_state()
        tr = bs.run(q, 1e-3, 4, t0=0.1)
        outs.append((q.clone(), tr.clone()))
        bs.close()
    for q, tr in outs[1:]:
        assert torch.equal(q, outs[0][0]) and torch.equal(tr, outs[0][1])


def test_autotuner_picks_a_candidate():
    P, mesh, c, prob, src, rec = _case(4, n=3, drop_last=0, shots=2)
    bs = P.BatchedSolver(4, mesh, c, 2, sources=src, receivers=rec, dtype="f32")
    assert bs.tune() in (2, 4, 8)
    q = bs.empty_state()
    tr = bs.run(q, 1e-3, 3, t0=0.1)
    assert torch.isfinite(tr).all() and torch.isfinite(q).all()
    bs.close()


def test_source_coefficients_match_oracle():
    from paper_1512_06025_amd import _lib
    P, mesh, c, prob, src, rec = _case(5, shots=6)
    s = P.Solver(5, mesh, c)
    elem, bary = P.locate_points(mesh, src)
    coef = np.zeros((len(elem), prob.Np))
    _lib.check(_lib.load().bbdg_source_coeffs(s._h, len(elem), elem.ctypes.data, bary.ctypes.data,
                                              coef.ctypes.data), "bbdg_source_coeffs")
    oe, ol = prob.locate(src)
    for i in range(len(elem)):
        want = prob.point_source_vector(oe[i], ol[i])
        np.testing.assert_allclose(coef[i], want, rtol=0, atol=1e-12 * np.abs(want).max())
    s.close()


def test_c4_full_size_sampled():
    """The 64-shot, 24,576-tet, N = 4 FP32 workload in the launch configuration
    the benchmark times (autotuned), two steps: the first and the last shot
    (smallest and largest offsets) re-run by the oracle, and for every shot the pressure integral,
    which only the source changes, against the same LSRK quadrature of the
    wavelet."""
    import paper_1512_06025_amd as P
    cfg, VX, EToV, c = workload.build_preset("c4")
    mesh = P.mesh_geometry(VX, EToV)
    S = cfg["shots"]
    src = workload.source_positions(S)
    rec = workload.receiver_grid()
    bs = P.BatchedSolver(cfg["N"], mesh, c, S, sources=src, receivers=rec, f0=cfg["f0"], ts=cfg["ts"],
                         dtype="f32")
    bs.tune()
    steps, t0, dt = 2, 0.1, cfg["dt"]
    q = bs.empty_state()
    tr = bs.run(q, dt, steps, t0=t0)
    bs.check()
    qh = _host_state(q)
    prob = dg.Problem(VX, EToV, cfg["N"], c)
    se, sl = prob.locate(src)
    re, rl = prob.locate(rec)
    for s in (0, S - 1):
        want, wtr = prob.run_shots(np.zeros((1, 4, prob.K, prob.Np)), dt, steps, se[s:s + 1], sl[s:s + 1],
                                   cfg["f0"], cfg["ts"], re, rl, t0=t0)
        assert _rel(qh[s], want[0]) < 1e-5, s
        # the receivers (z = 0.9) may not have been reached yet: compare absolutely
        got_tr = _host(tr)[:, s]
        assert np.abs(got_tr - wtr[:, 0]).max() <= 1e-5 * max(np.abs(wtr).max(), 1e-5 * np.abs(want[0][0]).max())
    # conservation for every shot
    I_res = 0.0
    I = 0.0
    for n in range(steps):
        for st in range(5):
            I_res = dg.LSRK_A[st] * I_res + dt * dg.ricker(t0 + n * dt + dg.LSRK_C[st] * dt, cfg["f0"], cfg["ts"])
            I += dg.LSRK_B[st] * I_res
    # FP32 rounding acts on every coefficient, so the bar scales with the sum
    # of the magnitudes of the integral's terms (the source vector oscillates)
    from oracle import bernstein as bb
    msum = bb.mass(cfg["N"]).sum(axis=1)
    for s in range(S):
        got = prob.pressure_integral(qh[s])
        scale = np.sum(np.abs(prob.geo.volume[:, None] * qh[s][0] * msum[None, :] / prob.kappa[:, None]))
        assert abs(got - I) < 1e-5 * scale, (s, got, I, scale)
    bs.close()


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_residency_bound(dtype):
    """For every order and batched launch shape, the co-residency bound that
    cooperative launches use never exceeds the occupancy query, is zero for
    a kernel that uses scratch memory and at least one otherwise; a shape
    with bound zero is refused before anything runs."""
    import ctypes

    import paper_1512_06025_amd as P
    from paper_1512_06025_amd import _lib
    lib = _lib.load()
    VX, EToV = workload.kuhn_cube_mesh(2, 0.0)
    mesh = P.mesh_geometry(VX, EToV)
    for N in range(1, 10):
        s = P.Solver(N, mesh, 1.0, dtype=dtype)
        for wpb in (2, 4, 8):
            for record in (0, 1):
                out = (ctypes.c_int32 * 6)()
                _lib.check(lib.bbdg_batched_occupancy(s._h, wpb, record, out), "bbdg_batched_occupancy")
                api, bound, vgprs, lds, scratch, cus = list(out)
                assert cus > 0 and vgprs > 0 and api >= 1, (N, wpb, record, list(out))
                assert 0 <= bound <= min(api, 8), (N, wpb, record, list(out))
                assert (bound == 0) == (scratch > 0), (N, wpb, record, list(out))
                assert lds <= 160 * 1024
                if record == 0 and bound == 0:
                    bs = P.BatchedSolver(N, mesh, 1.0, 1, dtype=dtype, wpb=wpb)
                    with pytest.raises(P.BBDGError) as err:
                        bs.run(bs.empty_state(), 1e-3, 1)
                    assert err.value.code == -11
                    bs.close()
        s.close()
