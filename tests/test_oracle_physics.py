"""Pins of the oracle's DG operator and time stepping (no GPU).

  * energy identity of the upwind scheme (energy estimate of Section 2),
    exact for the semi-discrete operator with exact integration;
  * reproduction of globally continuous polynomials of degree N (the
    derivative matrices and geometric factors of Section 3 are exact);
  * constant states are steady;
  * convergence O(h^{N+1}) to the standing-mode exact solution;
  * discrete energy does not grow over LSRK4 steps;
  * geometric identities and coincidence of matched face control points.
A few tests plant a mistake in a copy of the oracle and check that the pins
catch it.
"""
import numpy as np
import pytest

import workload
from oracle import dg
from oracle.mesh import Geometry
from oracle import bernstein as bb


def _problem(n=2, N=3, jitter=0.1, c=(1.0, 3.0), bc="rigid", drop_last=0):
    VX, EToV = workload.kuhn_cube_mesh(n, jitter, drop_last=drop_last)
    c = workload.wavespeed(EToV.shape[0], *c)
    return dg.Problem(VX, EToV, N, c, bc)


@pytest.mark.parametrize("bc", ["rigid", "pressure_release"])
@pytest.mark.parametrize("N", [1, 2, 4, 6])
def test_energy_identity(bc, N):
    P = _problem(N=N, bc=bc, drop_last=5)
    q = workload.random_coeffs(P.K, P.Np)
    rate, diss = P.energy_rate(q), P.jump_dissipation(q)
    assert diss < 0
    assert abs(rate - diss) <= 1e-12 * abs(diss)


@pytest.mark.parametrize("N", [1, 2, 3, 5])
def test_polynomial_exactness(N):
    """p a global polynomial of degree N, u = 0, rigid walls: no jumps, so
    dp/dt = 0 and du/dt = -grad p exactly."""
    P = _problem(N=N, c=(1.0, 1.0))
    rng = np.random.default_rng(7)
    terms = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a) for c in range(N + 1 - a - b)]
    coef = rng.standard_normal(len(terms))

    def p(x, y, z):
        return sum(k * x ** a * y ** b * z ** c for k, (a, b, c) in zip(coef, terms))

    def dp(d):
        def g(x, y, z):
            out = np.zeros_like(x)
            for k, (a, b, c) in zip(coef, terms):
                e = [a, b, c]
                if e[d] == 0:
                    continue
                f = e[d]
                e[d] -= 1
                out = out + k * f * x ** e[0] * y ** e[1] * z ** e[2]
            return out
        return g

    q = np.zeros((4, P.K, P.Np))
    q[0] = dg.project(P, p)
    r = P.rhs(q)
    # rounding of the projected coefficients is amplified by the lift
    tol = 1e-12 * np.abs(q[0]).max() * np.abs(P.L).max() * P.scale.max()
    assert np.abs(r[0]).max() < tol
    for d in range(3):
        want = -dg.project(P, dp(d))
        np.testing.assert_allclose(r[1 + d], want, atol=tol)


def test_constant_state_is_steady():
    P = _problem(N=4, c=(1.0, 2.0))
    q = np.zeros((4, P.K, P.Np))
    q[0] = 1.0
    assert np.abs(P.rhs(q)).max() < 1e-12


@pytest.mark.slow
@pytest.mark.parametrize("N", [1, 2, 3])
def test_standing_mode_convergence(N):
    errs = []
    for n in (2, 4, 8):
        P = _problem(n=n, N=N, jitter=0.0, c=(1.0, 1.0))
        q = dg.initial_state(P, workload.standing_mode_p0)
        T = 0.1
        dt = 0.5 / n / (N + 1) ** 2
        steps = int(np.ceil(T / dt))
        q = P.lsrk4(q, T / steps, steps)
        errs.append(dg.l2_error(P, q[0], dg.standing_mode_exact(T)[0]))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert rates[-1] > N + 0.8 and rates[-1] < N + 1.3, (errs, rates)


def test_pressure_release_standing_mode():
    """The paper's mirror condition p+ = -p- with its exact mode on [0,1]^3."""
    N = 3
    P = _problem(n=4, N=N, jitter=0.0, c=(1.0, 1.0), bc="pressure_release")
    pe0 = dg.standing_mode_exact(0.0, "pressure_release")[0]
    q = np.zeros((4, P.K, P.Np))
    q[0] = dg.project(P, pe0)
    T, steps = 0.05, 10
    q = P.lsrk4(q, T / steps, steps)
    ex = dg.standing_mode_exact(T, "pressure_release")
    for i in range(4):
        assert dg.l2_error(P, q[i], ex[i]) < 2e-3


def test_energy_does_not_grow():
    P = _problem(n=2, N=4, c=(1.0, 3.0))
    q = workload.random_coeffs(P.K, P.Np)
    dt = 0.5 * 0.5 / (3 * 25)
    E = [P.energy(q)]
    P.lsrk4(q, dt, 20, callback=lambda n, qq: E.append(P.energy(qq)))
    E = np.array(E)
    assert np.all(E[1:] <= E[:-1] * (1 + 1e-14))
    assert E[-1] < E[0]


def test_geometry_identities():
    VX, EToV = workload.kuhn_cube_mesh(3, 0.1)
    G = Geometry(VX, EToV)
    assert np.all(G.volume > 0)
    np.testing.assert_allclose(G.volume.sum(), 1.0, rtol=1e-13)
    # closed surface: sum_f A_f n_f = 0
    np.testing.assert_allclose(np.einsum("kf,kfd->kd", G.area, G.normal), 0.0, atol=1e-15)
    # n_f = -grad lambda_f / |grad lambda_f| and A_f / V = 3 |grad lambda_f|
    gl = G.grad_lambda
    norm = np.linalg.norm(gl, axis=2)
    np.testing.assert_allclose(G.normal, -gl / norm[..., None], atol=1e-13)
    np.testing.assert_allclose(G.area / G.volume[:, None], 3 * norm, rtol=1e-12)
    # neighbours are mutual and normals opposite
    k, f = np.nonzero(G.nbr >= 0)
    k2, f2 = G.nbr[k, f], G.nbr_face[k, f]
    assert np.all(G.nbr[k2, f2] == k)
    np.testing.assert_allclose(G.normal[k, f], -G.normal[k2, f2], atol=1e-13)
    # boundary faces lie on the cube surface
    kb, fb = np.nonzero(G.nbr < 0)
    assert kb.size == 6 * 2 * 9


@pytest.mark.parametrize("N", [1, 4, 7])
def test_matched_face_nodes_coincide(N):
    VX, EToV = workload.kuhn_cube_mesh(2, 0.15)
    G = Geometry(VX, EToV)
    own, other, bnd = G.face_node_maps(N)
    A = np.array(bb.multi_indices(N), dtype=float) / N
    pts = G.map_to_physical(A).reshape(-1, 3)        # control point positions
    inner = ~bnd
    np.testing.assert_allclose(pts[own[inner]], pts[other[inner]], atol=1e-14)
    assert not np.array_equal(own[inner], other[inner])


# -- planted mistakes ---------------------------------------------------------

def test_pins_catch_a_flipped_flux_sign(monkeypatch):
    P = _problem(N=3)
    q = workload.random_coeffs(P.K, P.Np)
    orig = dg.Problem.fluxes

    def bad(self, qq):
        Fp, Fu, jp, jun = orig(self, qq)
        return 0.5 * (self.tau_p[:, :, None] * jp + jun), Fu, jp, jun
    monkeypatch.setattr(dg.Problem, "fluxes", bad)
    rate, diss = P.energy_rate(q), P.jump_dissipation(q)
    assert abs(rate - diss) > 1e-8 * abs(diss)


def test_pins_catch_a_misoriented_face_map():
    P = _problem(N=3)
    q = workload.random_coeffs(P.K, P.Np)
    # reverse the face-local order of the neighbour nodes on interior faces
    inner = ~P.boundary
    P.other[inner] = P.other[inner][:, ::-1]
    rate, diss = P.energy_rate(q), P.jump_dissipation(q)
    assert abs(rate - diss) > 1e-8 * abs(diss)
    # a continuous field now shows jumps
    q = np.zeros((4, P.K, P.Np))
    q[0] = dg.project(P, lambda x, y, z: x * y + z)
    assert np.abs(P.rhs(q)[0]).max() > 1e-3


def test_pins_catch_a_transposed_derivative():
    P = _problem(N=3, c=(1.0, 1.0))
    P.D = np.transpose(P.D, (0, 2, 1)).copy()
    q = np.zeros((4, P.K, P.Np))
    q[0] = dg.project(P, lambda x, y, z: x * x + y * z)
    r = P.rhs(q)
    want = -dg.project(P, lambda x, y, z: 2 * x)
    assert np.abs(r[1] - want).max() > 1e-3
