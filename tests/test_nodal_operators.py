"""The dense nodal comparator's operators (built in libbbdg from its own BB
formulas) against operators derived from the oracle's dense BB matrices:
V (D^i - D^0) V^{-1} and V L^f Vf^{-1}, V and Vf the Bernstein-Vandermonde
matrices of the volume and face lattices (no GPU)."""
import numpy as np
import pytest

from oracle import bernstein as bb
from oracle import dg

P = pytest.importorskip("paper_1512_06025_amd")


@pytest.mark.parametrize("N", list(range(1, 10)))
def test_nodal_operators_match_oracle(N):
    dr, lift = P.nodal_operators(N)
    V = dg.bernstein_eval(N, np.array(bb.multi_indices(N), float) / N)
    Vi = np.linalg.inv(V)
    D = bb.bary_derivative(N)
    for i in range(1, 4):
        ref = V @ (D[i] - D[0]) @ Vi
        assert np.abs(dr[i - 1] - ref).max() <= 1e-12 * np.abs(ref).max()
    L = bb.lift(N) * 1.5  # reference lift M^{-1} M^f (area-2 reference faces)
    T = np.array(bb.tri_indices(N), float) / N
    Nfp = T.shape[0]
    for f in range(4):
        ids = bb.face_node_ids(N, f)
        lamf = np.zeros((Nfp, 4))
        lamf[:, list(bb.face_vertices(f))] = T
        Vf = dg.bernstein_eval(N, lamf)[:, ids]
        ref = V @ L[f][:, ids] @ np.linalg.inv(Vf)
        got = lift[:, f * Nfp:(f + 1) * Nfp]
        assert np.abs(got - ref).max() <= 1e-11 * np.abs(ref).max()
