"""Affine tetrahedral geometry and face matching (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Each element is the affine image of the reference tetrahedron (Section 3):
x = sum_i lambda_i X_i with barycentric coordinates lambda_i and vertices
X_0..X_3 taken in the element's vertex order.  From that:
  * grad lambda_i (i=1..3) are the rows of the inverse of [X1-X0, X2-X0, X3-X0],
    grad lambda_0 = -(grad lambda_1 + grad lambda_2 + grad lambda_3);
  * V = det[X1-X0, X2-X0, X3-X0] / 6 > 0 is the element volume;
  * face f is the face opposite vertex f; its area A_f and outward unit normal
    n_f are computed from the cross product of two face edges, oriented away
    from vertex f.

Faces are matched through their sets of global vertex ids.  Face control
points of neighbouring elements coincide (Section 3.1): the control point of
multi-index alpha sits at sum_i alpha_i X_i / N, so a face node is identified
by the multiset {global vertex id -> alpha component} of its face vertices.
"""
import numpy as np

from .bernstein import face_vertices, multi_indices, tri_indices


class Geometry:
    """Per-element geometric factors and face connectivity of a mesh."""

    def __init__(self, VX, EToV):
        VX = np.asarray(VX, dtype=np.float64)
        EToV = np.asarray(EToV, dtype=np.int64)
        K = EToV.shape[0]
        X = VX[EToV]                                   # (K, 4, 3)
        Jm = np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], axis=2)  # columns
        det = np.linalg.det(Jm)
        if np.any(det <= 0):
            raise ValueError("element with non-positive orientation")
        inv = np.linalg.inv(Jm)                        # rows = grad lambda_1..3
        grad = np.empty((K, 4, 3))
        grad[:, 1:] = inv
        grad[:, 0] = -inv.sum(axis=1)
        self.K = K
        self.X = X
        self.volume = det / 6.0
        self.grad_lambda = grad                        # (K, 4, 3)

        area = np.empty((K, 4))
        normal = np.empty((K, 4, 3))
        for f in range(4):
            a, b, c = face_vertices(f)
            cr = np.cross(X[:, b] - X[:, a], X[:, c] - X[:, a])
            nrm = np.linalg.norm(cr, axis=1)
            area[:, f] = 0.5 * nrm
            n = cr / nrm[:, None]
            # orient away from the opposite vertex
            s = np.sign(np.einsum("kd,kd->k", n, X[:, a] - X[:, f]))
            normal[:, f] = n * s[:, None]
        self.area = area
        self.normal = normal

        # face connectivity by global vertex sets
        faces = {}
        for k in range(K):
            for f in range(4):
                key = tuple(sorted(int(EToV[k, v]) for v in face_vertices(f)))
                faces.setdefault(key, []).append((k, f))
        nbr = -np.ones((K, 4), dtype=np.int64)
        nbr_face = -np.ones((K, 4), dtype=np.int64)
        for key, lst in faces.items():
            if len(lst) > 2:
                raise ValueError("non-conforming mesh: face shared by more than two elements")
            if len(lst) == 2:
                (k1, f1), (k2, f2) = lst
                nbr[k1, f1], nbr_face[k1, f1] = k2, f2
                nbr[k2, f2], nbr_face[k2, f2] = k1, f1
        self.nbr = nbr
        self.nbr_face = nbr_face
        self.EToV = EToV

    def face_node_maps(self, N):
        """Index maps for face traces at degree N.

        Returns (own, other, boundary):
          own[k, f, g]   flat index k*Np + a of the own node of face-local node g
          other[k, f, g] flat index k'*Np + a' of the coinciding node of the
                         neighbour (own index again on boundary faces)
          boundary[k, f] True where face f of k is on the domain boundary.

        The neighbour's multi-index a' gives each of its face vertices the
        component that the own multi-index gives the same global vertex."""
        A = multi_indices(N)
        Np = len(A)
        lookup = -np.ones((N + 1,) * 4, dtype=np.int64)
        for i, a in enumerate(A):
            lookup[a] = i
        T = np.array(tri_indices(N))                   # (Nfp, 3)
        Nfp = T.shape[0]
        K = self.K
        ks = np.arange(K)
        own = np.empty((K, 4, Nfp), dtype=np.int64)
        other = np.empty((K, 4, Nfp), dtype=np.int64)
        boundary = self.nbr < 0
        for f in range(4):
            fv = face_vertices(f)
            a = np.zeros((Nfp, 4), dtype=np.int64)
            a[:, list(fv)] = T
            own_local = lookup[a[:, 0], a[:, 1], a[:, 2], a[:, 3]]
            own[:, f, :] = ks[:, None] * Np + own_local[None, :]
            k2 = np.where(boundary[:, f], ks, self.nbr[:, f])
            b = np.zeros((K, Nfp, 4), dtype=np.int64)
            for m in range(3):
                gid = self.EToV[:, fv[m]]                      # global id of own face vertex m
                hit = self.EToV[k2] == gid[:, None]            # (K, 4) which neighbour vertex it is
                ok = hit.sum(axis=1) == 1
                if not np.all(ok | boundary[:, f]):
                    raise ValueError("face vertices do not match across a face")
                loc = np.argmax(hit, axis=1)
                b[ks, :, loc] = T[None, :, m]
            nb_local = lookup[b[..., 0], b[..., 1], b[..., 2], b[..., 3]]
            other[:, f, :] = np.where(boundary[:, f, None], own[:, f, :], k2[:, None] * Np + nb_local)
        return own, other, boundary

    def map_to_physical(self, lam):
        """Physical points of barycentric points lam (P, 4): returns (K, P, 3)."""
        return np.einsum("pi,kid->kpd", lam, self.X)
