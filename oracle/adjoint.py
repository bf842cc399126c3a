"""Discrete adjoint of the forced DG/LSRK4 solver and the gradient of a
receiver misfit with respect to m = c^2 (= kappa, rho = 1) per element
(oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The paper solves the forward problem only; the gradient is the standard
discrete adjoint ("first discretise, then differentiate") of exactly the
scheme of dg.Problem:
  * the semi-discrete operator A(m) of Sections 2-3 (strong form, upwind flux
    with tau_p = 2/(c- + c+), tau_u = (c- + c+)/2, c = sqrt(m)), whose
    transpose is assembled here from the transposes of its pieces: the
    barycentric derivatives D^i (Lemma 1), the face lifts L^f, the pointwise
    flux and the trace selections with the boundary mirror;
  * the point source kappa_k (M^k)^{-1} B(lambda_s) w(t) (linear in kappa_k);
  * the five-stage 2N-storage LSRK4 (Section 4.2), reversed stage by stage:
        forward  r <- a_s r + dt (A q + f(t_s)),   q <- q + b_s r
        reverse  rb <- rb + b_s qb,  qb <- qb + dt A^T rb,
                 g <- g + dt d(A q + f)/dm^T rb,  rb <- a_s rb
    with q the forward state entering the stage.
Misfit: J = 1/2 sum_{steps n} sum_{shots} sum_{receivers} (d - d_obs)^2,
d = the receiver pressures recorded after every step.

The derivative of A(m) q with respect to m_k has three parts: the factor
kappa_k of the pressure equation of element k; tau_p and tau_u of every face
of k, which depend on c_k + c_+ (on the domain boundary c_+ = c_k, so the sum
is 2 c_k); and the same taus seen from the neighbour across each interior
face.  The source adds f / kappa_k in its element.
"""
import numpy as np

from . import dg


class Adjoint:
    """A dg.Problem parameterised by m = c^2, with A^T and dA/dm."""

    def __init__(self, VX, EToV, N, m, bc="rigid"):
        self.m = np.asarray(m, dtype=np.float64).reshape(-1)
        self.prob = dg.Problem(VX, EToV, N, np.sqrt(self.m), bc)

    # -- transposes of the pieces of A ------------------------------------------
    def _dt_apply(self, i, x):
        """D^{iT} applied to every element's coefficients x (K, Np)."""
        return x @ self.prob.D[i]

    def _lift_T(self, x):
        """Per face f: scale_f (L^{fT} x) on the face nodes, (K, 4, Nfp)."""
        p = self.prob
        out = np.empty((p.K, 4, p.Nfp))
        for f in range(4):
            full = x @ p.L[f]                        # (L^{fT} x) for every element
            out[:, f, :] = p.scale[:, f, None] * full[:, p.face_ids[f]]
        return out

    def rhs_transpose(self, r, volume=True, surface=True):
        """A^T r for r of shape (4, K, Np)."""
        p = self.prob
        r = np.asarray(r, dtype=np.float64)
        out = np.zeros_like(r)
        kap = p.kappa[:, None]
        gl = p.geo.grad_lambda                        # (K, 4, 3)
        if volume:
            # rhs_p = -kappa sum_d sum_i gl[i,d] D^i u_d ; rhs_ud = -sum_i gl[i,d] D^i p
            for i in range(4):
                kr = self._dt_apply(i, kap * r[0])
                for d in range(3):
                    out[1 + d] -= gl[:, i, d, None] * kr
                out[0] -= self._dt_apply(i, sum(gl[:, i, d, None] * r[1 + d] for d in range(3)))
        if surface:
            n = p.geo.normal                          # (K, 4, 3)
            zp = self._lift_T(kap * r[0])            # adjoint of F_p on face nodes
            zu = sum(n[:, :, d, None] * self._lift_T(r[1 + d]) for d in range(3))
            tp, tu = p.tau_p[:, :, None], p.tau_u[:, :, None]
            # F_p = (tau_p jp - jun)/2, F_u = (tau_u jun - jp)/2
            jpb = 0.5 * tp * zp - 0.5 * zu
            junb = -0.5 * zp + 0.5 * tu * zu
            # jp = p+ - p-, jun = n.(u+ - u-)
            qmb = np.zeros((4, p.K, 4, p.Nfp))
            qpb = np.zeros((4, p.K, 4, p.Nfp))
            qmb[0] -= jpb
            qpb[0] += jpb
            for d in range(3):
                qmb[1 + d] -= n[:, :, d, None] * junb
                qpb[1 + d] += n[:, :, d, None] * junb
            bmask = p.boundary[:, :, None]
            # boundary exterior state is a function of the interior one
            if p.bc == "rigid":
                # p+ = p-, u+ = u- - 2 (n.u-) n
                qmb[0] += np.where(bmask, qpb[0], 0.0)
                nub = np.einsum("kfd,dkfg->kfg", n, qpb[1:4])
                for d in range(3):
                    qmb[1 + d] += np.where(bmask, qpb[1 + d] - 2.0 * n[:, :, d, None] * nub, 0.0)
            else:
                # p+ = -p-, u+ = u-
                qmb[0] -= np.where(bmask, qpb[0], 0.0)
                qmb[1:4] += np.where(bmask[None], qpb[1:4], 0.0)
            qpb = np.where(bmask[None], 0.0, qpb)
            flat = out.reshape(4, -1)
            for fld in range(4):
                np.add.at(flat[fld], p.own.ravel(), qmb[fld].ravel())
                np.add.at(flat[fld], p.other.ravel(), qpb[fld].ravel())
        return out

    # -- dA/dm ---------------------------------------------------------------------
    def rhs_dm(self, q, r):
        """g_k = r^T d(A(m) q)/dm_k for every element, (K,)."""
        p = self.prob
        q = np.asarray(q, dtype=np.float64)
        r = np.asarray(r, dtype=np.float64)
        K = p.K
        # kappa_k multiplies the whole pressure equation of element k (taus fixed)
        div = sum(p.gradient(q[1 + d])[d] for d in range(3))
        Fp, Fu, jp, jun = p.fluxes(q)
        lp = p.lift_faces(Fp).sum(axis=0)
        g = np.einsum("kn,kn->k", r[0], -div + lp)
        # tau_p, tau_u depend on s = c_k + c_+ of the face
        n = p.geo.normal
        zp = self._lift_T(p.kappa[:, None] * r[0])
        zu = sum(n[:, :, d, None] * self._lift_T(r[1 + d]) for d in range(3))
        s = p.c[:, None] + p.c_plus                   # (K, 4)
        dtp = -2.0 / s ** 2
        dtu = 0.5
        T = np.einsum("kfg,kfg->kf", zp, 0.5 * dtp[:, :, None] * jp) + np.einsum("kfg,kfg->kf", zu, 0.5 * dtu * jun)
        dcdm = 0.5 / p.c                              # c = sqrt(m)
        ds_own = np.where(p.boundary, 2.0, 1.0)       # boundary: s = 2 c_k
        g += dcdm * np.sum(T * ds_own, axis=1)
        nb = p.geo.nbr
        inner = ~p.boundary
        np.add.at(g, nb[inner], (dcdm[nb[inner]] * T[inner]))
        return g

    # -- misfit and gradient ----------------------------------------------------------
    def forward(self, q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, t0=0.0, keep=False):
        """Per-shot forward runs: traces (steps, S, R) and, with keep, the
        stage-input states of every stage of every shot."""
        p = self.prob
        S = q0.shape[0]
        W = p.receiver_weights(rec_lam)
        traces = np.zeros((steps, S, len(rec_elem)))
        stages = [] if keep else None
        for sh in range(S):
            vec = None if src_elem[sh] < 0 else p.point_source_vector(src_elem[sh], src_lam[sh])
            q = np.array(q0[sh], dtype=np.float64)
            res = np.zeros_like(q)
            kept = []
            for n_ in range(steps):
                for s in range(5):
                    if keep:
                        kept.append(q.copy())
                    rr = p.rhs(q)
                    if vec is not None:
                        rr[0, src_elem[sh]] += dg.ricker(t0 + n_ * dt + dg.LSRK_C[s] * dt, f0, ts) * vec
                    res = dg.LSRK_A[s] * res + dt * rr
                    q = q + dg.LSRK_B[s] * res
                traces[n_, sh] = np.einsum("rn,rn->r", q[0, rec_elem], W)
            if keep:
                stages.append(kept)
        return traces, stages

    def misfit(self, q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, d_obs, t0=0.0):
        tr, _ = self.forward(q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, t0)
        return 0.5 * float(np.sum((tr - d_obs) ** 2))

    def gradient(self, q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, d_obs, t0=0.0):
        """(J, dJ/dm (K,)) by the discrete adjoint."""
        p = self.prob
        tr, stages = self.forward(q0, dt, steps, src_elem, src_lam, f0, ts, rec_elem, rec_lam, t0, keep=True)
        resid = tr - d_obs
        J = 0.5 * float(np.sum(resid ** 2))
        W = p.receiver_weights(rec_lam)
        g = np.zeros(p.K)
        for sh in range(q0.shape[0]):
            ks = src_elem[sh]
            vec = None if ks < 0 else p.point_source_vector(ks, src_lam[sh])
            qb = np.zeros((4, p.K, p.Np))
            rb = np.zeros_like(qb)
            for n_ in reversed(range(steps)):
                for r_, k in enumerate(rec_elem):
                    qb[0, k] += resid[n_, sh, r_] * W[r_]
                for s in reversed(range(5)):
                    rb = rb + dg.LSRK_B[s] * qb
                    qb = qb + dt * self.rhs_transpose(rb)
                    g += dt * self.rhs_dm(stages[sh][5 * n_ + s], rb)
                    if vec is not None:
                        w = dg.ricker(t0 + n_ * dt + dg.LSRK_C[s] * dt, f0, ts)
                        g[ks] += dt * w * (rb[0, ks] @ vec) / p.kappa[ks]
                    rb = dg.LSRK_A[s] * rb
        return J, g

