"""Semi-discrete DG operator, LSRK4, energy and errors (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Fields are q = (p, u, v, w) with shape (4, K, Np) (Bernstein coefficients,
storage order of bernstein.multi_indices); rho = 1 and kappa = c^2 per element.

Right-hand side (Section 2 weak form, strong-form ODE system of Section 3
with M^{-1} applied):
  dp/dt   = kappa * ( -div u + sum_f (A_f/V) Lf [ 1/2 (tau_p [[p]] - n.[[u]]) ] )
  du_i/dt =           -d_i p + sum_f (A_f/V) n_i Lf [ 1/2 (tau_u n.[[u]] - [[p]]) ]
with [[a]] = a+ - a- (neighbour minus own), n the outward unit normal of the
own element, tau_p = 1/{{rho c}}, tau_u = {{rho c}} ({{.}} the arithmetic mean
of the two sides) and Lf the normalised lift of bernstein.lift.  The flux
coefficients are pointwise combinations of the face control points because
tau, n and A_f/V are constant on a face.

Physical gradients use the chain rule through the barycentric coordinates:
grad p = sum_{i=0..3} grad(lambda_i) (D^i p).

Domain boundary (exterior state built from the interior one):
  "rigid":            p+ = p-,  u+ = u- - 2 (n.u-) n   (u.n = 0 wall)
  "pressure_release": p+ = -p-, u+ = u-                (p = 0 mirror of Section 2)
with c+ = c- on the boundary.
"""
import numpy as np

from . import bernstein as bb
from .mesh import Geometry

# Carpenter-Kennedy five-stage fourth-order 2N-storage Runge-Kutta coefficients
# (the low-storage RK4 cited in Section 4.2).
LSRK_A = (0.0,
          -567301805773.0 / 1357537059087.0,
          -2404267990393.0 / 2016746695238.0,
          -3550918686646.0 / 2091501179385.0,
          -1275806237668.0 / 842570457699.0)
LSRK_B = (1432997174477.0 / 9575080441755.0,
          5161836677717.0 / 13612068292357.0,
          1720146321549.0 / 2090206949498.0,
          3134564353537.0 / 4481467310338.0,
          2277821191437.0 / 14882151754819.0)
LSRK_C = (0.0,
          1432997174477.0 / 9575080441755.0,
          2526269341429.0 / 6820363962896.0,
          2006345519317.0 / 3224310063776.0,
          2802321613138.0 / 2924317926251.0)

BOUNDARY_CONDITIONS = ("rigid", "pressure_release")


class Problem:
    """A mesh, an order N, per-element wavespeed and a boundary condition."""

    def __init__(self, VX, EToV, N, c, bc="rigid"):
        if bc not in BOUNDARY_CONDITIONS:
            raise ValueError("unknown boundary condition %r" % bc)
        self.N = N
        self.geo = Geometry(VX, EToV)
        self.K = self.geo.K
        self.Np = bb.np_count(N)
        self.Nfp = bb.nfp_count(N)
        self.c = np.asarray(c, dtype=np.float64).reshape(self.K)
        self.kappa = self.c ** 2
        self.bc = bc
        self.D = bb.bary_derivative(N)           # (4, Np, Np)
        self.L = bb.lift(N)                      # (4, Np, Np) normalised lifts
        self.own, self.other, self.boundary = self.geo.face_node_maps(N)
        self.face_ids = [bb.face_node_ids(N, f) for f in range(4)]
        g = self.geo
        self.scale = g.area / g.volume[:, None]  # A_f / V  (K, 4)
        nb = np.where(self.boundary, np.arange(self.K)[:, None], g.nbr)
        self.c_plus = self.c[nb]                 # (K, 4); c+ = c- on the boundary
        self.tau_p = 2.0 / (self.c[:, None] + self.c_plus)
        self.tau_u = 0.5 * (self.c[:, None] + self.c_plus)

    # -- building blocks ---------------------------------------------------
    def gradient(self, x):
        """Physical gradient coefficients of a scalar field x (K, Np): (3, K, Np)."""
        out = np.zeros((3,) + x.shape)
        for i in range(4):
            bary = x @ self.D[i].T                             # D^i x on every element
            for d in range(3):
                out[d] += self.geo.grad_lambda[:, i, d, None] * bary
        return out

    def traces(self, q):
        """Own and exterior traces on every face node: (4 fields, K, 4, Nfp) each."""
        flat = q.reshape(4, -1)
        qm = flat[:, self.own]
        qp = flat[:, self.other].copy()
        n = self.geo.normal                                  # (K, 4, 3)
        bmask = self.boundary[:, :, None]
        if self.bc == "rigid":
            un = np.einsum("kfd,dkfg->kfg", n, qm[1:4])
            mirror_u = qm[1:4] - 2.0 * np.einsum("kfg,kfd->dkfg", un, n)
            qp[0] = np.where(bmask, qm[0], qp[0])
            qp[1:4] = np.where(bmask[None], mirror_u, qp[1:4])
        else:
            qp[0] = np.where(bmask, -qm[0], qp[0])
            qp[1:4] = np.where(bmask[None], qm[1:4], qp[1:4])
        return qm, qp

    def fluxes(self, q):
        """Flux coefficients (F_p, F_u) on every face node, (K, 4, Nfp) each."""
        qm, qp = self.traces(q)
        n = self.geo.normal
        jp = qp[0] - qm[0]
        jun = np.einsum("kfd,dkfg->kfg", n, qp[1:4] - qm[1:4])
        Fp = 0.5 * (self.tau_p[:, :, None] * jp - jun)
        Fu = 0.5 * (self.tau_u[:, :, None] * jun - jp)
        return Fp, Fu, jp, jun

    def lift_faces(self, F):
        """sum_f (A_f/V) n-free lift of face data F (K, 4, Nfp) -> per face (4, K, Np)."""
        out = np.empty((4, self.K, self.Np))
        for f in range(4):
            full = np.zeros((self.K, self.Np))
            full[:, self.face_ids[f]] = F[:, f, :]
            out[f] = self.scale[:, f, None] * (full @ self.L[f].T)
        return out

    # -- operator ------------------------------------------------------------
    def rhs(self, q, volume=True, surface=True):
        """Semi-discrete right-hand side A(q), shape (4, K, Np)."""
        q = np.asarray(q, dtype=np.float64)
        out = np.zeros_like(q)
        kap = self.kappa[:, None]
        if volume:
            gp = self.gradient(q[0])
            div = sum(self.gradient(q[1 + d])[d] for d in range(3))
            out[0] -= kap * div
            out[1:4] -= gp
        if surface:
            Fp, Fu, _, _ = self.fluxes(q)
            lp = self.lift_faces(Fp)
            lu = self.lift_faces(Fu)
            out[0] += kap * lp.sum(axis=0)
            n = self.geo.normal
            for d in range(3):
                out[1 + d] += np.einsum("kf,fkn->kn", n[:, :, d], lu)
        return out

    # -- time stepping ---------------------------------------------------------
    def lsrk4(self, q, dt, steps, callback=None, forcing=None, t0=0.0):
        """Advance q by `steps` LSRK4 steps of size dt from time t0; returns the
        new q.  forcing(t), if given, is added to the right-hand side of the
        stage at time t = t_n + c_s dt (LSRK_C)."""
        q = np.array(q, dtype=np.float64, copy=True)
        res = np.zeros_like(q)
        for n in range(steps):
            for s in range(5):
                r = self.rhs(q)
                if forcing is not None:
                    r = r + forcing(t0 + n * dt + LSRK_C[s] * dt)
                res = LSRK_A[s] * res + dt * r
                q = q + LSRK_B[s] * res
            if callback is not None:
                callback(n + 1, q)
        return q

    # -- point sources and receivers -------------------------------------------
    # The paper's experiments are unforced; a seismic point source enters the
    # pressure equation as (1/kappa) p_t + div u = w(t) delta(x - x_s).  Its
    # Galerkin projection on the element k holding x_s (the same test
    # functions as the DG scheme, Section 2) is
    #   dp_k/dt += w(t) kappa_k (M^k)^{-1} B(lambda(x_s)),   M^k = V_k m.
    def locate(self, pts, tol=1e-10):
        """Lowest-numbered element containing each point, with its barycentric
        coordinates (negatives below tol set to 0, renormalised).  Returns
        (elem (P,), lam (P, 4)); elem is -1 for a point outside the mesh."""
        pts = np.atleast_2d(np.asarray(pts, dtype=np.float64))
        g = self.geo
        elem = np.full(pts.shape[0], -1, dtype=np.int64)
        lam = np.zeros((pts.shape[0], 4))
        for i, x in enumerate(pts):
            # lambda_j(x) = 1/4 + grad(lambda_j) . (x - centroid) is affine
            cen = g.X.mean(axis=1)
            L = 0.25 + np.einsum("kjd,kd->kj", g.grad_lambda, x[None, :] - cen)
            inside = np.nonzero(np.all(L >= -tol, axis=1))[0]
            if inside.size:
                k = inside[0]
                l = np.clip(L[k], 0.0, None)
                elem[i], lam[i] = k, l / l.sum()
        return elem, lam

    def point_source_vector(self, k, lam):
        """kappa_k (V_k m)^{-1} B(lambda): (Np,) pressure right-hand side of a
        unit point source in element k at barycentric coordinates lam."""
        m = bb.mass_exact(self.N)
        b = bernstein_eval(self.N, np.asarray(lam, dtype=np.float64)[None, :])[0]
        x = bb._ld_gauss_solve(bb._frac_to_ld(m), np.asarray(b, dtype=np.longdouble)[:, None])[:, 0]
        return (self.kappa[k] / self.geo.volume[k]) * np.asarray(x, dtype=np.float64)

    def point_source(self, k, lam, f0, ts):
        """forcing(t) for lsrk4: a Ricker point source in element k."""
        vec = self.point_source_vector(k, lam)

        def forcing(t):
            out = np.zeros((4, self.K, self.Np))
            out[0, k] = ricker(t, f0, ts) * vec
            return out
        return forcing

    def receiver_weights(self, lam):
        """B_alpha(lambda_r) for receivers at barycentric points lam (R, 4)."""
        return bernstein_eval(self.N, np.atleast_2d(np.asarray(lam, dtype=np.float64)))

    def run_shots(self, q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, t0=0.0,
                  trace_scales=False):
        """Independent shots, each with its own point source (src_elem[s] = -1:
        none), sharing the receivers.  q0: (S, 4, K, Np).  Returns the final
        states (S, 4, K, Np) and the traces (steps, S, R): the pressure at the
        receivers after every step.  With trace_scales=True also returns
        sum_n |W_rn| |p_n| for every trace (steps, S, R): the size of the
        terms each trace sums, which bounds its rounding error."""
        q0 = np.asarray(q0, dtype=np.float64)
        S, R = q0.shape[0], len(rec_elem)
        W = self.receiver_weights(rec_lam) if R else np.zeros((0, self.Np))
        traces = np.zeros((steps, S, R))
        scales = np.zeros((steps, S, R))
        out = np.empty_like(q0)
        for s in range(S):
            forcing = None if src_elem[s] < 0 else self.point_source(src_elem[s], src_lam[s], f0, ts)

            def record(n, q, s=s):
                for r in range(R):
                    traces[n - 1, s, r] = q[0, rec_elem[r]] @ W[r]
                    scales[n - 1, s, r] = np.abs(q[0, rec_elem[r]]) @ np.abs(W[r])
            out[s] = self.lsrk4(q0[s], dt, steps, callback=record, forcing=forcing, t0=t0)
        if trace_scales:
            return out, traces, scales
        return out, traces

    def pressure_integral(self, q):
        """sum_k int_{D^k} p / kappa: advanced only by the source term (the
        upwind flux telescopes across interior faces and vanishes on rigid
        walls), so under a point source its rate is w(t)."""
        m = bb.mass(self.N)
        return float(np.sum(self.geo.volume * (q[0] @ m.sum(axis=1)) / self.kappa))

    # -- diagnostics -----------------------------------------------------------
    def energy(self, q):
        """sum_k int (p^2/kappa + rho |u|^2)."""
        m = bb.mass(self.N)
        V = self.geo.volume
        e = np.einsum("kn,nm,km->k", q[0], m, q[0]) / self.kappa
        for d in range(1, 4):
            e += np.einsum("kn,nm,km->k", q[d], m, q[d])
        return float(np.sum(V * e))

    def energy_rate(self, q):
        """2 sum_k (p^T M^k rhs_p / kappa + u^T M^k rhs_u): d/dt of energy(q)."""
        r = self.rhs(q)
        m = bb.mass(self.N)
        V = self.geo.volume
        e = np.einsum("kn,nm,km->k", q[0], m, r[0]) / self.kappa
        for d in range(1, 4):
            e += np.einsum("kn,nm,km->k", q[d], m, r[d])
        return float(2.0 * np.sum(V * e))

    def jump_dissipation(self, q):
        """-1/2 sum_k sum_f int_f (tau_p [[p]]^2 + tau_u [[u.n]]^2), the energy
        rate that the upwind flux predicts (energy estimate of Section 2)."""
        _, _, jp, jun = self.fluxes(q)
        mf = bb.to_f64(bb.face_mass_2d_exact(self.N))
        A = self.geo.area
        tot = 0.0
        tot += np.sum(A * self.tau_p * np.einsum("kfg,gh,kfh->kf", jp, mf, jp))
        tot += np.sum(A * self.tau_u * np.einsum("kfg,gh,kfh->kf", jun, mf, jun))
        return -0.5 * float(tot)


# ---------------------------------------------------------------------------
# quadrature, projection and errors
# ---------------------------------------------------------------------------

def ricker(t, f0, ts):
    """Ricker wavelet (1 - 2 pi^2 f0^2 (t - ts)^2) exp(-pi^2 f0^2 (t - ts)^2)."""
    a = (np.pi * f0 * (t - ts)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def tet_quadrature(n):
    """Collapsed-coordinate Gauss-Jacobi rule on the unit simplex, exact for
    polynomials of degree <= 2n-1 in each collapsed variable.

    Returns (lam (P,4) barycentric points, w (P,) weights summing to 1)."""
    from scipy.special import roots_jacobi
    xa, wa = roots_jacobi(n, 2.0, 0.0)   # weight (1-x)^2
    xb, wb = roots_jacobi(n, 1.0, 0.0)   # weight (1-x)^1
    xc, wc = roots_jacobi(n, 0.0, 0.0)   # Legendre
    a = (1 + xa) / 2
    b = (1 + xb) / 2
    c = (1 + xc) / 2
    A, B, C = np.meshgrid(a, b, c, indexing="ij")
    WA, WB, WC = np.meshgrid(wa, wb, wc, indexing="ij")
    l1 = A
    l2 = B * (1 - A)
    l3 = C * (1 - A) * (1 - B)
    l0 = 1 - l1 - l2 - l3
    lam = np.stack([l0.ravel(), l1.ravel(), l2.ravel(), l3.ravel()], axis=1)
    w = (WA * WB * WC).ravel()
    return lam, w / w.sum()


def bernstein_eval(N, lam):
    """B_alpha at float barycentric points lam (P, 4): returns (P, Np)."""
    from math import factorial
    A = bb.multi_indices(N)
    out = np.empty((lam.shape[0], len(A)))
    for j, a in enumerate(A):
        coef = factorial(N)
        for x in a:
            coef //= factorial(x)
        out[:, j] = coef * np.prod(lam ** np.array(a)[None, :], axis=1)
    return out


def project(prob, func, qdeg=None):
    """L2 projection of func(x, y, z) onto each element: (K, Np) coefficients."""
    N = prob.N
    lam, w = tet_quadrature(qdeg or (N + 4))
    B = bernstein_eval(N, lam)                      # (P, Np)
    xyz = prob.geo.map_to_physical(lam)             # (K, P, 3)
    fv = func(xyz[..., 0], xyz[..., 1], xyz[..., 2])
    rhs = fv @ (w[:, None] * B)                     # (K, Np)
    return np.linalg.solve(bb.mass(N), rhs.T).T


def l2_error(prob, coeffs, func, qdeg=None):
    """sqrt(sum_k int (p_h - func)^2) for one field with coefficients (K, Np)."""
    N = prob.N
    lam, w = tet_quadrature(qdeg or (N + 4))
    B = bernstein_eval(N, lam)
    xyz = prob.geo.map_to_physical(lam)
    diff = coeffs @ B.T - func(xyz[..., 0], xyz[..., 1], xyz[..., 2])
    return float(np.sqrt(np.sum(prob.geo.volume * (diff ** 2 @ w))))


def standing_mode_exact(t, wall="rigid"):
    """Exact fields of the standing mode on [0,1]^3 with rho = kappa = 1.

    rigid walls:  p = cos(pi x) cos(pi y) cos(pi z) cos(sqrt3 pi t),
                  u = sin(sqrt3 pi t)/sqrt3 * (sin(pi x)cos(pi y)cos(pi z), ...);
    pressure release: the same with every cos(pi .) <-> sin(pi .) in space
    (p = sin sin sin, u_x = -sin(sqrt3 pi t)/sqrt3 cos(pi x) sin(pi y) sin(pi z), ...)."""
    w = np.sqrt(3.0) * np.pi
    ct, st = np.cos(w * t), np.sin(w * t) / np.sqrt(3.0)
    if wall == "rigid":
        def p(x, y, z):
            return np.cos(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z) * ct

        def u(x, y, z):
            return st * np.sin(np.pi * x) * np.cos(np.pi * y) * np.cos(np.pi * z)

        def v(x, y, z):
            return st * np.cos(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z)

        def ww(x, y, z):
            return st * np.cos(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z)
    else:
        def p(x, y, z):
            return np.sin(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z) * ct

        def u(x, y, z):
            return -st * np.cos(np.pi * x) * np.sin(np.pi * y) * np.sin(np.pi * z)

        def v(x, y, z):
            return -st * np.sin(np.pi * x) * np.cos(np.pi * y) * np.sin(np.pi * z)

        def ww(x, y, z):
            return -st * np.sin(np.pi * x) * np.sin(np.pi * y) * np.cos(np.pi * z)
    return p, u, v, ww


def initial_state(prob, p0):
    """(4, K, Np) state: p projected from p0(x, y, z), velocity zero."""
    q = np.zeros((4, prob.K, prob.Np))
    q[0] = project(prob, p0)
    return q
