"""Initial Bernstein-Bezier coefficients from an analytic field (host input prep).

The field is sampled at the equispaced lattice of every element (control
point positions sum_i alpha_i X_i / N) and the samples are converted to
Bernstein coefficients by solving with the Bernstein-Vandermonde matrix of
the lattice: nodal interpolation followed by a change of basis, the way the
paper prepares its initial conditions (Section 4.1), with the equispaced
lattice in place of the Warp & Blend nodes.
"""
from math import factorial

import numpy as np

from .solver import alpha_table


def _vandermonde(N):
    A = alpha_table(N).astype(np.float64)
    lam = A / N                                    # lattice points (barycentric)
    coef = np.array([factorial(N) / np.prod([factorial(int(x)) for x in a]) for a in A])
    # V[p, b] = C_b prod_i lam_p,i ^ b_i
    V = coef[None, :] * np.prod(lam[:, None, :] ** A[None, :, :], axis=2)
    return lam, V


def lattice_values(N, VX, EToV, func):
    """(K, Np) values of func at the lattice points (control-point positions)."""
    lam, _ = _vandermonde(N)
    X = np.asarray(VX, dtype=np.float64)[np.asarray(EToV)]
    pts = np.einsum("pi,kid->kpd", lam, X)
    return func(pts[..., 0], pts[..., 1], pts[..., 2])


def interpolate(N, VX, EToV, func):
    """(K, Np) Bernstein coefficients interpolating func(x, y, z) on each element."""
    lam, V = _vandermonde(N)
    X = np.asarray(VX, dtype=np.float64)[np.asarray(EToV)]          # (K, 4, 3)
    pts = np.einsum("pi,kid->kpd", lam, X)                          # (K, Np, 3)
    vals = func(pts[..., 0], pts[..., 1], pts[..., 2])               # (K, Np)
    return np.linalg.solve(V, vals.T).T


def initial_state(N, VX, EToV, p0, basis="bb"):
    """(K, 4, Np) float64 state, the solver's element-major field layout, with
    p interpolated from p0 and zero velocity: Bernstein coefficients
    (basis="bb") or lattice values (basis="nodal")."""
    K = np.asarray(EToV).shape[0]
    q = np.zeros((K, 4, alpha_table(N).shape[0]))
    q[:, 0] = interpolate(N, VX, EToV, p0) if basis == "bb" else lattice_values(N, VX, EToV, p0)
    return q
