"""Pins of the oracle's point sources, receivers and forced time stepping.

The paper's experiments are unforced; the batched-shot path adds a Ricker
point source to the pressure equation and samples the pressure at receivers.
Each piece is pinned to something outside its own code: the wavelet to its
closed-form zeros and antiderivative, point location to the affine map, the
projected source to a quadrature mass matrix, receivers to polynomial
reproduction, and the forced solver to the conservation law that the upwind
scheme satisfies exactly (sum_k int p/kappa changes only through the source).
"""
import numpy as np
import pytest

import workload
from oracle import dg

F0, TS = 8.0, 0.125


def _ricker_antiderivative(t):
    a = (np.pi * F0 * (t - TS)) ** 2
    return (t - TS) * np.exp(-a)


def test_ricker_closed_forms():
    assert dg.ricker(TS, F0, TS) == 1.0
    z = 1.0 / (np.sqrt(2.0) * np.pi * F0)
    assert abs(dg.ricker(TS + z, F0, TS)) < 1e-15
    assert abs(dg.ricker(TS - z, F0, TS)) < 1e-15
    # antiderivative (t - ts) exp(-pi^2 f0^2 (t - ts)^2), by a fine trapezoid rule
    t = np.linspace(0.0, 0.4, 400001)
    w = dg.ricker(t, F0, TS)
    integral = np.sum(0.5 * (w[1:] + w[:-1]) * np.diff(t))
    assert abs(integral - (_ricker_antiderivative(0.4) - _ricker_antiderivative(0.0))) < 1e-9


def _problem(N=3, n=2, jitter=0.1):
    VX, EToV = workload.kuhn_cube_mesh(n, jitter)
    c = workload.wavespeed(EToV.shape[0], 1.0, 3.0)
    return dg.Problem(VX, EToV, N, c)


def test_locate_reproduces_points():
    prob = _problem()
    rng = np.random.default_rng(7)
    pts = rng.uniform(0.0, 1.0, (50, 3))
    elem, lam = prob.locate(pts)
    assert np.all(elem >= 0)
    np.testing.assert_allclose(np.einsum("pj,pjd->pd", lam, prob.geo.X[elem]), pts, atol=1e-14)
    assert np.all(lam >= 0) and np.allclose(lam.sum(axis=1), 1.0)
    # a mesh vertex is in many elements: the lowest id wins
    e_v, lam_v = prob.locate([[0.5, 0.5, 0.5]])
    owners = [k for k in range(prob.K) if np.any(np.all(np.abs(prob.geo.X[k] - 0.5) < 1e-14, axis=1))]
    if owners:  # jittered meshes move the interior vertex
        assert e_v[0] == min(owners)
    e_out, _ = prob.locate([[1.5, 0.2, 0.2]])
    assert e_out[0] == -1


@pytest.mark.parametrize("N", [1, 3, 4])
def test_point_source_is_the_projected_delta(N):
    """M^k s = kappa_k B(lambda_s), with M^k from a quadrature rule."""
    prob = _problem(N)
    elem, lam = prob.locate([[0.31, 0.62, 0.27]])
    k = elem[0]
    s = prob.point_source_vector(k, lam[0])
    ql, qw = dg.tet_quadrature(N + 2)
    B = dg.bernstein_eval(N, ql)
    Mk = prob.geo.volume[k] * (B.T @ (qw[:, None] * B))
    want = prob.kappa[k] * dg.bernstein_eval(N, lam)[0]
    np.testing.assert_allclose(Mk @ s, want, rtol=1e-11, atol=1e-11 * np.abs(want).max())


def test_receivers_reproduce_polynomials():
    N = 3
    prob = _problem(N)

    def f(x, y, z):
        return 1.0 + x - 2.0 * y * y + x * y * z

    coef = dg.project(prob, f)  # exact for a polynomial of degree <= N
    rng = np.random.default_rng(11)
    pts = rng.uniform(0.05, 0.95, (20, 3))
    elem, lam = prob.locate(pts)
    W = prob.receiver_weights(lam)
    got = np.einsum("rn,rn->r", coef[elem], W)
    np.testing.assert_allclose(got, f(*pts.T), atol=1e-12)


def _scalar_lsrk(t0, dt, steps):
    """The same LSRK4 applied to dI/dt = w(t)."""
    I, res = 0.0, 0.0
    for n in range(steps):
        for s in range(5):
            res = dg.LSRK_A[s] * res + dt * dg.ricker(t0 + n * dt + dg.LSRK_C[s] * dt, F0, TS)
            I += dg.LSRK_B[s] * res
    return I


def test_forced_run_conserves_pressure_integral():
    """sum_k int p/kappa grows exactly by the LSRK quadrature of w (rigid walls,
    heterogeneous c), which itself matches the closed-form antiderivative."""
    prob = _problem(N=3)
    elem, lam = prob.locate([[0.4, 0.55, 0.35]])
    q0 = np.zeros((1, 4, prob.K, prob.Np))
    t0, dt, steps = 0.05, 2e-3, 30
    out, _ = prob.run_shots(q0, dt, steps, elem, lam, F0, TS, [], np.zeros((0, 4)), t0=t0)
    gain = prob.pressure_integral(out[0])
    scalar = _scalar_lsrk(t0, dt, steps)
    assert abs(gain - scalar) < 1e-12 * max(1.0, abs(scalar))
    exact = _ricker_antiderivative(t0 + steps * dt) - _ricker_antiderivative(t0)
    assert abs(scalar - exact) < 1e-8
    assert abs(gain) > 1e-3  # the source did act


def test_run_shots_matches_single_runs_and_traces():
    prob = _problem(N=2)
    rng = np.random.default_rng(5)
    elem, lam = prob.locate(rng.uniform(0.1, 0.9, (2, 3)))
    relem, rlam = prob.locate(rng.uniform(0.1, 0.9, (3, 3)))
    q0 = np.zeros((2, 4, prob.K, prob.Np))
    dt, steps = 2e-3, 5
    out, tr = prob.run_shots(q0, dt, steps, elem, lam, F0, TS, relem, rlam, t0=0.08)
    for s in range(2):
        one = prob.lsrk4(q0[s], dt, steps, forcing=prob.point_source(elem[s], lam[s], F0, TS), t0=0.08)
        np.testing.assert_array_equal(out[s], one)
        W = dg.bernstein_eval(2, rlam)
        np.testing.assert_allclose(tr[-1, s], np.einsum("rn,rn->r", one[0][relem], W), rtol=1e-14, atol=0)


def test_pins_catch_a_missing_kappa(monkeypatch):
    """Planted mistake: dropping kappa from the source breaks the conservation pin."""
    good = dg.Problem.point_source_vector

    def bad(self, k, lam):
        return good(self, k, lam) / self.kappa[k]
    monkeypatch.setattr(dg.Problem, "point_source_vector", bad)
    with pytest.raises(AssertionError):
        test_forced_run_conserves_pressure_integral()


def test_pins_catch_a_wrong_stage_time(monkeypatch):
    """Planted mistake: evaluating the wavelet at t_n instead of t_n + c_s dt."""
    monkeypatch.setattr(dg, "LSRK_C", (0.0,) * 5)
    prob = _problem(N=2)
    elem, lam = prob.locate([[0.4, 0.55, 0.35]])
    q0 = np.zeros((1, 4, prob.K, prob.Np))
    t0, dt, steps = 0.05, 2e-3, 30
    out, _ = prob.run_shots(q0, dt, steps, elem, lam, F0, TS, [], np.zeros((0, 4)), t0=t0)
    exact = _ricker_antiderivative(t0 + steps * dt) - _ricker_antiderivative(t0)
    assert abs(prob.pressure_integral(out[0]) - exact) > 1e-6


def test_resume_is_bitwise():
    """A forced oracle run of 10 steps equals 4 steps followed by 6 steps from
    t0 + 4 dt, bit for bit (dt a power of two keeps the stage times exact),
    states and traces."""
    prob = _problem(N=2)
    rng = np.random.default_rng(9)
    elem, lam = prob.locate(rng.uniform(0.1, 0.9, (2, 3)))
    relem, rlam = prob.locate(rng.uniform(0.1, 0.9, (3, 3)))
    q0 = np.zeros((2, 4, prob.K, prob.Np))
    dt, t0 = 2.0 ** -10, 0.0625
    qa, ta = prob.run_shots(q0, dt, 10, elem, lam, F0, TS, relem, rlam, t0=t0)
    q1, t1 = prob.run_shots(q0, dt, 4, elem, lam, F0, TS, relem, rlam, t0=t0)
    qb, t2 = prob.run_shots(q1, dt, 6, elem, lam, F0, TS, relem, rlam, t0=t0 + 4 * dt)
    np.testing.assert_array_equal(qa, qb)
    np.testing.assert_array_equal(ta, np.concatenate([t1, t2]))
    assert np.abs(qa).max() > 0
