"""Parity at the full workload sizes, in the launch configurations the
benchmark times.

* c2 (24,576 jittered tets, N = 5): one LSRK4 step of bbdg_run against the
  oracle on every coefficient, FP64 (1e-12) and FP32 (1e-5); the same mesh
  at N = 7, 8, 9 in FP64, which take the non-temporal-store instantiations.
* c3 (196,608 tets, c ~ U[1,3], N = 1..9): one right-hand side of the whole
  mesh on the GPU, checked element by element on a seeded sample of
  elements.  The oracle evaluates the sample on a sub-mesh made of the
  sampled elements and their face neighbours: a sampled element sees exactly
  the same neighbours, wavespeeds and boundary faces as in the full mesh, so
  its right-hand side is the full-mesh one.
* c5 (24,576 tets, N = 5, 8 shots, 64 receivers): dJ/dm from the GPU
  adjoint against central differences of the GPU FP64 misfit on 20 seeded
  elements with |g_k| >= 1e-3 max|g|, over the workload's 500 steps.  The central
  difference with eps = 1e-4 m_k alone has a truncation error of up to
  ~2e-5 relative here (it falls as eps^2 towards the adjoint value), so one
  Richardson step with eps and eps/2 is taken.
"""
import numpy as np
import pytest

import workload
from oracle import dg

torch = pytest.importorskip("torch")
pytestmark = [pytest.mark.gpu, pytest.mark.slow]

TOL = {"f64": 1e-12, "f32": 1e-5}


def _rel(a, b):
    return float(np.linalg.norm(np.ravel(a - b)) / np.linalg.norm(np.ravel(b)))


def _host(x):
    torch.cuda.synchronize()
    return x.detach().to("cpu", torch.float64).numpy()


def _dev(q0, dtype):
    """Oracle state (4, K, Np) -> the library's element-major (K, 4, Np)."""
    return torch.from_numpy(np.ascontiguousarray(np.swapaxes(q0, 0, 1))).to("cuda", dtype)


def _host_field(q):
    """Device field (K, 4, Np) -> oracle layout (4, K, Np), float64."""
    return np.swapaxes(_host(q), 0, 1)


@pytest.mark.parametrize("dtype", ["f64", "f32"])
def test_c2_one_step(dtype):
    import paper_1512_06025_amd as P
    cfg, VX, EToV, c = workload.build_preset("c2")
    prob = dg.Problem(VX, EToV, cfg["N"], c)
    q0 = workload.random_coeffs(prob.K, prob.Np, seed=21)
    if dtype == "f32":
        q0 = q0.astype(np.float32).astype(np.float64)
    s = P.Solver(cfg["N"], P.mesh_geometry(VX, EToV), c, dtype=dtype)
    q = _dev(q0, s.torch_dtype)
    s.run(q, cfg["dt"], 1)
    want = prob.lsrk4(q0, cfg["dt"], 1)
    assert _rel(_host_field(q), want) < TOL[dtype]
    s.close()


@pytest.mark.parametrize("N", [7, 8, 9])
def test_c2_mesh_high_order_one_step_nontemporal_stores(N):
    """N = 7, 8, 9 on the 24,576-tet mesh, FP64: the three field sets (270 MiB
    and more) exceed the 256 MB last-level cache, so the stage runs the
    instantiation with non-temporal output stores and residual loads (at
    N = 8 and 9 with element groups shared by a team of waves); one LSRK4
    step on every coefficient against the oracle (1e-12)."""
    import paper_1512_06025_amd as P
    cfg, VX, EToV, c = workload.build_preset("c2", N=N)
    prob = dg.Problem(VX, EToV, N, c)
    assert 3 * 4 * prob.K * prob.Np * 8 > 256 * 1024 * 1024
    q0 = workload.random_coeffs(prob.K, prob.Np, seed=22)
    s = P.Solver(N, P.mesh_geometry(VX, EToV), c, dtype="f64")
    assert s.nontemporal_stores()
    q = _dev(q0, s.torch_dtype)
    s.run(q, cfg["dt"], 1)
    want = prob.lsrk4(q0, cfg["dt"], 1)
    assert _rel(_host_field(q), want) < TOL["f64"]
    s.close()


def _submesh(EToV, sample):
    """Elements of the sample and their face neighbours (elements sharing the
    three vertices of a face); index of each sampled element in the sub-mesh."""
    EToV = np.asarray(EToV)
    faces = np.sort(np.concatenate([np.delete(EToV, f, axis=1) for f in range(4)]), axis=1)  # (4K, 3)
    owner = np.tile(np.arange(EToV.shape[0]), 4)
    _, fid = np.unique(faces, axis=0, return_inverse=True)
    fid = fid.ravel()
    keep = set(int(k) for k in sample)
    wanted = set(fid[np.isin(owner, sample)].tolist())
    keep.update(int(k) for k in owner[np.isin(fid, list(wanted))])
    keep = np.array(sorted(keep))
    where = {k: i for i, k in enumerate(keep)}
    return keep, np.array([where[int(k)] for k in sample])


_C3 = {}


def _c3_mesh():
    if not _C3:
        import paper_1512_06025_amd as P
        cfg, VX, EToV, c = workload.build_preset("c3")
        mesh = P.mesh_geometry(VX, EToV)
        _C3.update(cfg=cfg, VX=VX, EToV=EToV, c=c, mesh=mesh)
    return _C3


@pytest.mark.parametrize("dtype", ["f64", "f32"])
@pytest.mark.parametrize("N", [1, 3, 5, 7, 9])
def test_c3_rhs_sampled(N, dtype):
    import paper_1512_06025_amd as P
    m = _c3_mesh()
    VX, EToV, c, mesh = m["VX"], m["EToV"], m["c"], m["mesh"]
    K = EToV.shape[0]
    Np = (N + 1) * (N + 2) * (N + 3) // 6
    q = workload.random_coeffs(K, Np, seed=30 + N)
    if dtype == "f32":
        q = q.astype(np.float32).astype(np.float64)
    s = P.Solver(N, mesh, c, dtype=dtype)
    got = _host_field(s.rhs(_dev(q, s.torch_dtype)))
    s.close()
    rng = np.random.default_rng(400 + N)
    # include elements on the domain boundary and the last element
    sample = np.unique(np.concatenate([rng.choice(K, 62, replace=False), [0, K - 1]]))
    keep, pos = _submesh(EToV, sample)
    sub = dg.Problem(VX, EToV[keep], N, c[keep])
    want = sub.rhs(q[:, keep])[:, pos]
    assert _rel(got[:, sample], want) < TOL[dtype], (N, dtype)


_C5 = {}


def _c5_gradient():
    """GPU FP64 misfit gradient of the full c5 workload (500 steps,
    checkpoints every 50), computed once for all chunks of elements."""
    if not _C5:
        import paper_1512_06025_amd as P
        cfg, VX, EToV, _ = workload.build_preset("c5")
        N, K, S, dt, steps = cfg["N"], cfg["K"], cfg["shots"], cfg["dt"], cfg["steps"]
        mesh = P.mesh_geometry(VX, EToV)
        src, rec = workload.plane_sources(S), workload.receiver_grid()
        m_true = workload.blob_model(VX, EToV)
        obs_run = P.BatchedSolver(N, mesh, np.sqrt(m_true), S, sources=src, receivers=rec, f0=cfg["f0"],
                                  ts=cfg["ts"], dtype="f64", wpb=4)
        d_obs = obs_run.run(obs_run.empty_state(), dt, steps).clone()
        obs_run.close()
        m0 = np.ones(K)
        mf = P.Misfit(N, mesh, m0, S, src, rec, d_obs, dt, steps, f0=cfg["f0"], ts=cfg["ts"],
                      ckpt_every=cfg["ckpt_every"], dtype="f64")
        J0 = float(mf.evaluate().item())
        g = mf.gradient().cpu().numpy()
        big = np.nonzero(np.abs(g) >= 1e-3 * np.abs(g).max())[0]
        pick = np.random.default_rng(workload.SEED_FD_ELEMENTS).choice(big, size=min(20, big.size), replace=False)
        _C5.update(mf=mf, m0=m0, J0=J0, g=g, pick=pick)
    return _C5


@pytest.mark.parametrize("chunk", [0, 1, 2, 3])
def test_c5_gradient_vs_finite_differences(chunk):
    """The full c5 workload (500 steps, checkpoints every 50): dJ/dm of the
    GPU adjoint against central differences of the GPU FP64 misfit on the 20
    seeded elements (five per chunk), to 1e-6 relative."""
    c5 = _c5_gradient()
    mf, m0, g = c5["mf"], c5["m0"], c5["g"]
    assert c5["J0"] > 0

    def central(k, eps):
        mp, mm = m0.copy(), m0.copy()
        mp[k] += eps
        mm[k] -= eps
        return (float(mf.evaluate(mp).item()) - float(mf.evaluate(mm).item())) / (2 * eps)
    worst = 0.0
    for k in c5["pick"][5 * chunk: 5 * chunk + 5]:
        eps = 1e-4 * m0[k]
        fd = (4.0 * central(k, eps / 2) - central(k, eps)) / 3.0
        worst = max(worst, abs(fd - g[k]) / abs(g[k]))
    if chunk == 3:
        mf.close()
        _C5.clear()
    assert worst < 1e-6, worst
