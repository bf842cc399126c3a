"""Host-side checks of libbbdg (no GPU): exported symbols, the coefficient
order, mesh geometry and connectivity against the oracle's own, and
argument validation (which runs before any device call)."""
import ctypes
import os
import re

import numpy as np
import pytest

import workload
from oracle.mesh import Geometry

P = pytest.importorskip("paper_1512_06025_amd")
from paper_1512_06025_amd import _lib  # noqa: E402

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def _declared_functions():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if fn.endswith(".h"):
            text = open(os.path.join(inc, fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(bbdg_[a-z_0-9]+)\s*\(", text))
    return names


def test_every_declared_symbol_is_exported(lib):
    names = _declared_functions()
    assert {"bbdg_create", "bbdg_rhs", "bbdg_run", "bbdg_destroy", "bbdg_mesh_geometry"} <= names
    for name in names:
        assert hasattr(lib, name), name
    # and the binding covers all of them
    assert names <= set(_lib.SIGNATURES)


def test_np_and_alpha_table(lib):
    for N in range(1, 10):
        Np = (N + 1) * (N + 2) * (N + 3) // 6
        assert lib.bbdg_np(N) == Np
        want = [(N - a1 - a2 - a3, a1, a2, a3)
                for a3 in range(N + 1) for a2 in range(N + 1 - a3) for a1 in range(N + 1 - a3 - a2)]
        assert [tuple(r) for r in P.alpha_table(N)] == want
    assert lib.bbdg_np(0) == -2
    assert lib.bbdg_np(10) == -2
    assert lib.bbdg_alpha_table(3, None) == -1


@pytest.mark.parametrize("drop", [0, 7])
def test_mesh_geometry_matches_oracle(drop):
    VX, EToV = workload.kuhn_cube_mesh(3, 0.1, drop_last=drop)
    m = P.mesh_geometry(VX, EToV)
    G = Geometry(VX, EToV)
    np.testing.assert_allclose(m.geo[:, :9].reshape(-1, 3, 3), G.grad_lambda[:, 1:], rtol=1e-13, atol=1e-13)
    np.testing.assert_allclose(m.geo[:, 9], 0.75 * G.volume, rtol=1e-13)
    np.testing.assert_array_equal(m.EToE, G.nbr)
    inner = G.nbr >= 0
    np.testing.assert_array_equal(m.EToF[inner], G.nbr_face[inner])
    assert np.all(m.EToF[~inner] == -1) and np.all(m.EToO[~inner] == -1)
    # orientation: own face vertex a_m is neighbour face vertex b_pi(m)
    perms = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]
    for k, f in zip(*np.nonzero(inner)):
        k2, f2 = m.EToE[k, f], m.EToF[k, f]
        a = [v for v in range(4) if v != f]
        b = [v for v in range(4) if v != f2]
        pi = perms[m.EToO[k, f]]
        for i in range(3):
            assert EToV[k, a[i]] == EToV[k2, b[pi[i]]]


def _good_mesh():
    VX, EToV = workload.kuhn_cube_mesh(2, 0.1)
    m = P.mesh_geometry(VX, EToV)
    c = np.ones(m.K)
    return m, c


def _create(lib, m, c, N=3, dtype=0, bc=0, K=None, geo=None, EToE=None, EToF=None, EToO=None):
    h = ctypes.c_void_p()
    arr = lambda x, d: x.ctypes.data if x is not None else None  # noqa: E731
    rc = lib.bbdg_create(ctypes.byref(h), N, dtype, m.K if K is None else K,
                         arr(m.EToE if EToE is None else EToE, 0), arr(m.EToF if EToF is None else EToF, 0),
                         arr(m.EToO if EToO is None else EToO, 0), arr(m.geo if geo is None else geo, 0),
                         arr(c, 0), bc, 0)
    return rc, h


def test_create_validation_errors(lib):
    m, c = _good_mesh()
    assert _create(lib, m, c, N=0)[0] == -2
    assert _create(lib, m, c, N=10)[0] == -2
    assert _create(lib, m, c, dtype=2)[0] == -5
    assert _create(lib, m, c, bc=5)[0] == -6
    assert _create(lib, m, c, K=0)[0] == -1
    bad = m.geo.copy()
    bad[3, 2] = np.nan
    assert _create(lib, m, c, geo=bad)[0] == -4
    bad = m.geo.copy()
    bad[4, 9] = -1.0
    assert _create(lib, m, c, geo=bad)[0] == -3
    assert _create(lib, m, np.zeros(m.K))[0] == -1
    e = m.EToE.copy()
    k, f = np.argwhere(e >= 0)[0]
    e[k, f] = (e[k, f] + 1) % m.K          # asymmetric connectivity
    assert _create(lib, m, c, EToE=e)[0] == -3
    o = m.EToO.copy()
    o[k, f] = (o[k, f] + 1) % 6            # inconsistent orientation
    assert _create(lib, m, c, EToO=o)[0] == -3
    e = m.EToE.copy()
    e[0, 0] = m.K                           # out of range
    assert _create(lib, m, c, EToE=e)[0] == -3
    h = ctypes.c_void_p()
    assert lib.bbdg_create(ctypes.byref(h), 3, 0, m.K, None, None, None, None, None, 0, 0) == -1


@pytest.mark.parametrize("N", list(range(1, 10)))
def test_create_builds_host_tables_before_the_device(lib, N):
    """Valid arguments to the three create calls: every host-side table (flux
    weights, index tables, the dense nodal operators in both comparator
    layouts) is built before the first device call, so without a GPU the
    calls build them and then fail with BBDG_E_DEVICE; with a GPU they
    succeed and the handle is destroyed."""
    VX, EToV = workload.kuhn_cube_mesh(2, 0.1, drop_last=3)
    m = P.mesh_geometry(VX, EToV)
    c = np.linspace(1.0, 2.0, m.K)
    for create in (lib.bbdg_create, lib.bbdg_nodal_create, lib.bbdg_nodal_ept_create):
        for dtype in (_lib.BBDG_F64, _lib.BBDG_F32):
            h = ctypes.c_void_p()
            rc = create(ctypes.byref(h), N, dtype, m.K, m.EToE.ctypes.data, m.EToF.ctypes.data,
                        m.EToO.ctypes.data, m.geo.ctypes.data, c.ctypes.data, _lib.BBDG_BC_RIGID, 0)
            assert rc in (0, -7), rc
            if rc == 0:
                assert lib.bbdg_destroy(h) == 0
            else:
                assert not h.value


def test_mesh_geometry_errors(lib):
    VX, EToV = workload.kuhn_cube_mesh(1)
    K, Nv = EToV.shape[0], VX.shape[0]
    out = [np.zeros((K, 10)), np.zeros((K, 4), np.int32), np.zeros((K, 4), np.int8), np.zeros((K, 4), np.int8)]
    ptrs = [o.ctypes.data for o in out]
    bad = EToV.copy()
    bad[0, [2, 3]] = bad[0, [3, 2]]         # negative orientation
    assert lib.bbdg_mesh_geometry(K, Nv, VX.ctypes.data, bad.ctypes.data, *ptrs) == -3
    bad = EToV.copy()
    bad[1, 0] = Nv                          # vertex id out of range
    assert lib.bbdg_mesh_geometry(K, Nv, VX.ctypes.data, bad.ctypes.data, *ptrs) == -3
    dup = np.concatenate([EToV, EToV[:1]])  # a face shared by three elements
    out2 = [np.zeros((K + 1, 10)), np.zeros((K + 1, 4), np.int32), np.zeros((K + 1, 4), np.int8),
            np.zeros((K + 1, 4), np.int8)]
    assert lib.bbdg_mesh_geometry(K + 1, Nv, VX.ctypes.data, dup.ctypes.data,
                                  *[o.ctypes.data for o in out2]) == -3
    nanv = VX.copy()
    nanv[0, 0] = np.inf
    assert lib.bbdg_mesh_geometry(K, Nv, nanv.ctypes.data, EToV.ctypes.data, *ptrs) == -4


def test_null_handles_and_strerror(lib):
    assert lib.bbdg_rhs(None, None, None, 0, None) == -1
    assert lib.bbdg_run(None, None, None, 0.0, 1.0, 1, None) == -1
    assert lib.bbdg_work_bytes(None) == 0
    assert lib.bbdg_destroy(None) == 0
    assert lib.bbdg_info(None, None, None, None, None) == -1
    for code in list(_lib.ERRORS):
        assert lib.bbdg_strerror(code)
    assert lib.bbdg_strerror(-99) == b"unknown error code"
    assert lib.bbdg_run_batched(None, None, 1, None, None, 8.0, 0.1, 0, None, None, None, None,
                                0.0, 1e-3, 1, 0, None) == -1
    assert lib.bbdg_tune_batched(None, 1, None, None, None) == -1
    assert lib.bbdg_batched_work_bytes(None, 4) == 0
    assert lib.bbdg_source_coeffs(None, 0, None, None, None) == -1
    assert lib.bbdg_status(None) == -1
    assert lib.bbdg_set_barrier_timeout(None, 1.0) == -1
    assert lib.bbdg_strerror(-12) != b"unknown error code"
    assert lib.bbdg_run_noalloc(None, None, 0.0, 1.0, 1, None) == -1
    assert lib.bbdg_strerror(-13) != b"unknown error code"


# -- host utilities of the batched path (no device involved) ---------------------

def test_locate_points_matches_oracle():
    from oracle import dg
    VX, EToV = workload.kuhn_cube_mesh(3, 0.1, drop_last=7)
    mesh = P.mesh_geometry(VX, EToV)
    prob = dg.Problem(VX, EToV, 2, np.ones(EToV.shape[0]))
    rng = np.random.default_rng(21)
    pts = rng.uniform(0.0, 1.0, (200, 3))
    oe, ol = prob.locate(pts)
    inside = oe >= 0
    e, l = P.locate_points(mesh, pts[inside])
    np.testing.assert_array_equal(e, oe[inside])
    np.testing.assert_allclose(l, ol[inside], atol=1e-13)
    # a point in the removed elements (or outside the cube) is an error
    if not inside.all():
        with pytest.raises(_lib.BBDGError):
            P.locate_points(mesh, pts)
    with pytest.raises(_lib.BBDGError):
        P.locate_points(mesh, [[1.2, 0.5, 0.5]])


@pytest.mark.parametrize("N", [1, 4, 9])
def test_bernstein_eval_matches_oracle(N):
    from oracle import dg
    rng = np.random.default_rng(N)
    lam = rng.dirichlet(np.ones(4), size=30)
    np.testing.assert_allclose(P.bernstein_eval(N, lam), dg.bernstein_eval(N, lam), rtol=1e-13, atol=1e-15)
    # partition of unity
    np.testing.assert_allclose(P.bernstein_eval(N, lam).sum(axis=1), 1.0, rtol=1e-14)


def test_initial_state_is_element_major():
    """The package's initial-state helper returns the solver's element-major
    field layout (K, 4, Np): element k's pressure coefficients at [k, 0].  For
    a polynomial of degree <= N its interpolation equals the oracle's L2
    projection (both reproduce the polynomial exactly)."""
    from oracle import dg
    from paper_1512_06025_amd import ic
    VX, EToV = workload.kuhn_cube_mesh(2, 0.1, drop_last=3)
    N = 3
    prob = dg.Problem(VX, EToV, N, np.ones(EToV.shape[0]))

    def p0(x, y, z):
        return 1.0 + 2.0 * x - y + 3.0 * z * x - 0.5 * y * y * z

    got = ic.initial_state(N, VX, EToV, p0)
    assert got.shape == (prob.K, 4, prob.Np)
    want = dg.initial_state(prob, p0)
    np.testing.assert_allclose(np.swapaxes(got, 0, 1), want, rtol=0, atol=1e-11)
