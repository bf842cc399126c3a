"""Pins of the oracle's discrete adjoint and misfit gradient.

* A^T against A by the dot-product identity <A q, r> = <q, A^T r> (random q, r,
  both boundary conditions, ragged meshes with interior boundary faces);
* dA/dm against central differences of A(m) q (Richardson-extrapolated);
* dJ/dm against central differences of J and a Taylor remainder of order 2;
* planted mistakes (a dropped tau derivative, a wrong boundary mirror in
  A^T) fail these pins.
"""
import numpy as np
import pytest

import workload
from oracle import adjoint

F0, TS = 8.0, 0.125


def _setup(N=2, n=2, drop_last=3, bc="rigid", crange=(1.0, 3.0)):
    VX, EToV = workload.kuhn_cube_mesh(n, 0.1, drop_last=drop_last)
    m = workload.wavespeed(EToV.shape[0], *crange) ** 2
    return VX, EToV, m, adjoint.Adjoint(VX, EToV, N, m, bc)


@pytest.mark.parametrize("bc", ["rigid", "pressure_release"])
@pytest.mark.parametrize("N", [1, 3, 4])
def test_dot_product_identity(N, bc):
    _, _, _, A = _setup(N, bc=bc)
    p = A.prob
    rng = np.random.default_rng(N)
    q = rng.standard_normal((4, p.K, p.Np))
    r = rng.standard_normal((4, p.K, p.Np))
    lhs = np.sum(p.rhs(q) * r)
    rhs = np.sum(q * A.rhs_transpose(r))
    assert abs(lhs - rhs) < 1e-13 * np.sqrt(np.sum(p.rhs(q) ** 2) * np.sum(r ** 2))
    # also the volume and surface parts separately
    for kw in (dict(surface=False), dict(volume=False)):
        assert abs(np.sum(p.rhs(q, **kw) * r) - np.sum(q * A.rhs_transpose(r, **kw))) < 1e-12 * abs(lhs)


@pytest.mark.parametrize("bc", ["rigid", "pressure_release"])
def test_operator_derivative_against_differences(bc):
    VX, EToV, m, A = _setup(3, bc=bc)
    p = A.prob
    rng = np.random.default_rng(4)
    q = rng.standard_normal((4, p.K, p.Np))
    r = rng.standard_normal((4, p.K, p.Np))
    dm = rng.standard_normal(p.K) * m * 0.1

    def d(eps):
        Ap = adjoint.Adjoint(VX, EToV, 3, m + eps * dm, bc).prob.rhs(q)
        Am = adjoint.Adjoint(VX, EToV, 3, m - eps * dm, bc).prob.rhs(q)
        return np.sum(r * (Ap - Am)) / (2 * eps)
    e = 1e-3
    fd = (4 * d(e / 2) - d(e)) / 3                   # O(e^4)
    an = A.rhs_dm(q, r) @ dm
    assert abs(fd - an) < 1e-9 * abs(an), (fd, an)


def _shots(A, S=2, R=3, seed=1):
    p = A.prob
    rng = np.random.default_rng(seed)
    se, sl = p.locate(rng.uniform(0.1, 0.45, (S, 3)))
    re, rl = p.locate(rng.uniform(0.1, 0.45, (R, 3)))
    return se, sl, re, rl


def test_gradient_against_finite_differences():
    VX, EToV, m, A = _setup(2, crange=(1.0, 2.0))
    p = A.prob
    se, sl, re, rl = _shots(A)
    q0 = np.zeros((2, 4, p.K, p.Np))
    dt, steps, t0 = 2e-3, 6, 0.08
    rng = np.random.default_rng(2)
    obs = rng.standard_normal((steps, 2, 3)) * 1e-3
    J, g = A.gradient(q0, dt, steps, se, sl, F0, TS, re, rl, obs, t0)
    assert J == pytest.approx(A.misfit(q0, dt, steps, se, sl, F0, TS, re, rl, obs, t0), rel=1e-14)

    def Jm(mm):
        return adjoint.Adjoint(VX, EToV, 2, mm).misfit(q0, dt, steps, se, sl, F0, TS, re, rl, obs, t0)
    big = np.nonzero(np.abs(g) >= 1e-3 * np.abs(g).max())[0]
    pick = np.random.default_rng(workload.SEED_FD_ELEMENTS).choice(big, size=min(6, big.size), replace=False)
    for k in pick:
        eps = 1e-4 * m[k]
        e = np.zeros(p.K)
        e[k] = eps
        fd = (Jm(m + e) - Jm(m - e)) / (2 * eps)
        assert abs(fd - g[k]) < 1e-6 * abs(g[k]), (k, fd, g[k])


def test_taylor_remainder_is_second_order():
    VX, EToV, m, A = _setup(2, crange=(1.0, 2.0))
    p = A.prob
    se, sl, re, rl = _shots(A, S=1)
    q0 = np.zeros((1, 4, p.K, p.Np))
    q0[0] = workload.random_coeffs(p.K, p.Np, seed=9) * 1e-2
    dt, steps, t0 = 2e-3, 4, 0.1
    obs = np.zeros((steps, 1, 3))
    J, g = A.gradient(q0, dt, steps, se, sl, F0, TS, re, rl, obs, t0)
    dm = np.random.default_rng(3).standard_normal(p.K) * m * 0.05

    def Jm(mm):
        return adjoint.Adjoint(VX, EToV, 2, mm).misfit(q0, dt, steps, se, sl, F0, TS, re, rl, obs, t0)
    rem = [abs(Jm(m + h * dm) - J - h * (g @ dm)) for h in (1e-1, 5e-2, 2.5e-2)]
    slopes = [np.log2(rem[i] / rem[i + 1]) for i in range(2)]
    assert all(1.8 < s < 2.2 for s in slopes), slopes


def test_pins_catch_a_dropped_tau_derivative(monkeypatch):
    """Planted mistake: ignoring that tau_p, tau_u depend on c."""
    VX, EToV, m, A = _setup(3)
    p = A.prob
    rng = np.random.default_rng(4)
    q = rng.standard_normal((4, p.K, p.Np))
    r = rng.standard_normal((4, p.K, p.Np))
    dm = rng.standard_normal(p.K) * m * 0.1
    good = A.rhs_dm(q, r) @ dm
    monkeypatch.setattr(adjoint.Adjoint, "_lift_T", lambda self, x: np.zeros((p.K, 4, p.Nfp)))
    # with the face adjoint zeroed, only the kappa part is left
    bad = A.rhs_dm(q, r) @ dm
    assert abs(bad - good) > 1e-6 * abs(good)


def test_pins_catch_a_wrong_boundary_mirror(monkeypatch):
    """Planted mistake: A^T built for the pressure-release mirror on a rigid problem."""
    _, _, _, A = _setup(2)
    p = A.prob
    rng = np.random.default_rng(8)
    q = rng.standard_normal((4, p.K, p.Np))
    r = rng.standard_normal((4, p.K, p.Np))
    lhs = np.sum(p.rhs(q) * r)
    monkeypatch.setattr(p, "bc", "pressure_release")
    rhs = np.sum(q * A.rhs_transpose(r))
    assert abs(lhs - rhs) > 1e-6 * abs(lhs)
