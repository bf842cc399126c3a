"""Pins of the oracle's dense Bernstein-Bezier operators against what the
paper and standard mathematics fix (no GPU).

Each pin compares an oracle matrix, built by monomial evaluation and exact
simplex integrals, with an independent statement: the sparse derivative
formula of Lemma 1 (row form of Appendix A.1), the lift factorisation of
Section 3.1.2 / Appendix A.3, the printed values of Figures 4 and 5, the
eigenvalue formulas of Appendix A.3, quadrature, and the LSRK4 stability
polynomial.
"""
import os
from fractions import Fraction
from math import comb, factorial

import numpy as np
import pytest

from oracle import bernstein as bb
from oracle import dg

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")
ORDERS = list(range(1, 10))


def _load(name):
    return np.loadtxt(os.path.join(GOLDEN, name), comments="#")


# -- test-local index helpers (written from the definitions, not imported) --

def _vol_alphas(N):
    return [(N - a1 - a2 - a3, a1, a2, a3)
            for a3 in range(N + 1) for a2 in range(N + 1 - a3) for a1 in range(N + 1 - a3 - a2)]


def _tri(m):
    return [(m - g1 - g2, g1, g2) for g2 in range(m + 1) for g1 in range(m + 1 - g2)]


def _elevation(m):
    """One-degree elevation E^m_{m-1} on a triangle (rows degree m, cols m-1):
    B^{m-1}_b = sum_k (b_k+1)/m B^m_{b+e_k} (Appendix A, degree elevation)."""
    rows = {g: i for i, g in enumerate(_tri(m))}
    cols = _tri(m - 1)
    E = [[Fraction(0)] * len(cols) for _ in rows]
    for j, b in enumerate(cols):
        for k in range(3):
            g = list(b)
            g[k] += 1
            E[rows[tuple(g)]][j] += Fraction(b[k] + 1, m)
    return E


def _matmul(A, B):
    return [[sum(A[i][k] * B[k][j] for k in range(len(B)) if A[i][k] and B[k][j]) or Fraction(0)
             for j in range(len(B[0]))] for i in range(len(A))]


def _transpose(A):
    return [list(r) for r in zip(*A)]


def _paper_L0(N):
    E = _elevation(N + 1)
    EtE = _matmul(_transpose(E), E)
    s = Fraction((N + 1) ** 2, 2)
    return [[s * x for x in row] for row in EtE]


def _paper_EL(N, f):
    """E_L^f (Np x Nfp, volume row order): layer i (alpha_f = i) holds
    ell_i (E^N_{N-i})^T with ell_i = (-1)^i C(N,i)/(1+i) (Section 3.1.2)."""
    fv = [v for v in range(4) if v != f]
    red = {0: [[Fraction(int(i == j)) for j in range(len(_tri(N)))] for i in range(len(_tri(N)))]}
    for i in range(1, N + 1):
        # (E^N_{N-i})^T = (E^{N-i+1}_{N-i})^T (E^N_{N-i+1})^T
        red[i] = _matmul(_transpose(_elevation(N - i + 1)), red[i - 1])
    out = []
    for a in _vol_alphas(N):
        i = a[f]
        ell = Fraction((-1) ** i * comb(N, i), 1 + i)
        pos = {g: j for j, g in enumerate(_tri(N - i))}[tuple(a[v] for v in fv)]
        out.append([ell * x for x in red[i][pos]])
    return out


def _face_cols(N, f):
    A = _vol_alphas(N)
    index = {a: i for i, a in enumerate(A)}
    fv = [v for v in range(4) if v != f]
    ids = []
    for g in _tri(N):
        a = [0, 0, 0, 0]
        for m in range(3):
            a[fv[m]] = g[m]
        ids.append(index[tuple(a)])
    return ids


def _cond(A):
    s = np.linalg.svd(A, compute_uv=False)
    s = s[s > s[0] * 1e-12]
    return s[0] / s[-1]


# -- pins --------------------------------------------------------------------

def test_storage_order_is_documented_order():
    for N in ORDERS:
        assert bb.multi_indices(N) == _vol_alphas(N)
        assert len(bb.multi_indices(N)) == (N + 1) * (N + 2) * (N + 3) // 6


@pytest.mark.parametrize("N", ORDERS)
def test_dense_derivative_equals_sparse_lemma(N):
    """Lemma 1, row form (Appendix A.1): D^i[a, a + e_i - e_j] = a_j, j = 0..3,
    and no other nonzero; at most 4 nonzeros per row."""
    D = bb.bary_derivative_exact(N)
    A = _vol_alphas(N)
    index = {a: n for n, a in enumerate(A)}
    for i in range(4):
        S = [[Fraction(0)] * len(A) for _ in A]
        for r, a in enumerate(A):
            for j in range(4):
                if a[j] == 0:
                    continue
                b = list(a)
                b[i] += 1
                b[j] -= 1
                S[r][index[tuple(b)]] += a[j]
        assert D[i] == S, "D^%d differs from the sparse formula at N=%d" % (i, N)
        nnz = [sum(1 for x in row if x != 0) for row in D[i]]
        assert max(nnz) <= 4
        assert nnz == [sum(1 for x in a if x) for a in A]


@pytest.mark.parametrize("N", ORDERS)
def test_lift_factorisation(N):
    """L^f = E_L^f L_0 exactly (Section 3.1.2, Appendix A.3) on every face."""
    L0 = _paper_L0(N)
    for f in range(4):
        L = bb.reference_lift_exact(N, f)
        cols = _face_cols(N, f)
        Lf = [[row[c] for c in cols] for row in L]
        EL = _paper_EL(N, f)
        assert _matmul(EL, L0) == Lf
        # columns off face f are zero
        off = [c for c in range(len(L)) if c not in set(cols)]
        assert all(L[r][c] == 0 for r in range(len(L)) for c in off)


def test_figure5_min_max():
    tab = _load("fig5_minmax.txt")
    for row in tab:
        N = int(row[0])
        Ls = [bb.to_f64(bb.reference_lift_exact(N, f)) for f in range(4)]
        allL = np.concatenate(Ls)
        cols = _face_cols(N, 0)
        Lf = Ls[0][:, cols]
        L0 = Lf[cols, :]
        EL = Lf @ np.linalg.inv(L0)
        got = [allL.min(), allL.max(), EL.min(), EL.max(), L0.min(), L0.max()]
        np.testing.assert_allclose(got, row[1:], rtol=1e-5, atol=1e-12, err_msg="N=%d" % N)


def test_figure4_condition_numbers():
    tab = _load("fig4_condition.txt")
    for row in tab:
        N = int(row[0])
        cols = _face_cols(N, 0)
        Lf = bb.to_f64(bb.reference_lift_exact(N, 0))[:, cols]
        L0 = Lf[cols, :]
        EL = Lf @ np.linalg.inv(L0)
        D0 = bb.bary_derivative(N)[0]
        got = [_cond(Lf), _cond(D0), _cond(L0), _cond(EL)]
        np.testing.assert_allclose(got, row[1:], rtol=5e-6, err_msg="N=%d" % N)
        # closed forms behind two of the series
        assert abs(_cond(D0) - np.sqrt(N * (N + 3) / (2.0 * (N + 1)))) < 1e-12
        assert abs(_cond(L0) - (N + 1) * (N + 3) / (2.0 * N + 3)) < 1e-12


@pytest.mark.parametrize("N", ORDERS)
def test_L0_eigenvalues(N):
    """eig(L_0) = (N+i+3)(N+1-i)/2, i = 0..N, multiplicity i+1 (Appendix A.3, d=3)."""
    cols = _face_cols(N, 0)
    L0 = bb.to_f64(bb.reference_lift_exact(N, 0))[np.ix_(cols, cols)]
    ev = np.sort(np.linalg.eigvals(L0).real)
    want = np.sort(np.concatenate([[(N + i + 3) * (N + 1 - i) / 2.0] * (i + 1) for i in range(N + 1)]))
    np.testing.assert_allclose(ev, want, rtol=1e-11)


@pytest.mark.parametrize("N", [1, 2, 3, 5, 7])
def test_mass_eigenvalues(N):
    """Distinct eigenvalues of the degree-N Bernstein mass matrix (Appendix A.3):
    |T| (N!)^2 d! / ((N+i+d)! (N-i)!), each with the multiplicity of the
    degree-i orthogonal modes; here |T| = 1 (normalised)."""
    for d, M, mult in ((3, bb.mass(N), lambda i: (i + 1) * (i + 2) // 2),
                       (2, bb.to_f64(bb.face_mass_2d_exact(N)), lambda i: i + 1)):
        ev = np.sort(np.linalg.eigvalsh(M))
        want = np.sort(np.concatenate([[factorial(N) ** 2 * factorial(d) /
                                        (factorial(N + i + d) * factorial(N - i))] * mult(i)
                                       for i in range(N + 1)]))
        np.testing.assert_allclose(ev, want, rtol=1e-9)


@pytest.mark.parametrize("N", [1, 3, 5])
def test_mass_matrices_against_quadrature(N):
    lam, w = dg.tet_quadrature(N + 2)
    B = dg.bernstein_eval(N, lam)
    np.testing.assert_allclose(B.T @ (w[:, None] * B), bb.mass(N), atol=1e-15, rtol=1e-13)
    # face f: integrate over the face lambda_f = 0 with a triangle rule
    from scipy.special import roots_jacobi
    xa, wa = roots_jacobi(N + 2, 1.0, 0.0)
    xb, wb = roots_jacobi(N + 2, 0.0, 0.0)
    a, b = (1 + xa) / 2, (1 + xb) / 2
    A_, B_ = np.meshgrid(a, b, indexing="ij")
    W = np.outer(wa, wb).ravel()
    W /= W.sum()
    s1, s2 = A_.ravel(), (B_ * (1 - A_)).ravel()
    for f in range(4):
        fv = [v for v in range(4) if v != f]
        lamf = np.zeros((s1.size, 4))
        lamf[:, fv[0]] = 1 - s1 - s2
        lamf[:, fv[1]] = s1
        lamf[:, fv[2]] = s2
        Bf = dg.bernstein_eval(N, lamf)
        np.testing.assert_allclose(Bf.T @ (W[:, None] * Bf), bb.face_mass(N, f), atol=1e-15, rtol=1e-13)


@pytest.mark.parametrize("N", ORDERS)
def test_sparsity_counts(N):
    """L_0 has at most 7 nonzeros per row (7 once N >= 2 gives interior
    face nodes); E_L^f rows hold (a_f+1)(a_f+2)/2 nonzeros, the concatenated
    E_L at most Nfp + 3 (Section 3.1.2)."""
    Nfp = (N + 1) * (N + 2) // 2
    cols = _face_cols(N, 0)
    L0 = bb.to_f64(bb.reference_lift_exact(N, 0))[np.ix_(cols, cols)]
    nnz0 = (np.abs(L0) > 0).sum(axis=1)
    assert nnz0.max() <= 7
    if N >= 3:
        assert nnz0.max() == 7
    A = _vol_alphas(N)
    total = np.zeros(len(A), dtype=int)
    for f in range(4):
        c = _face_cols(N, f)
        Lf = bb.to_f64(bb.reference_lift_exact(N, f))[:, c]
        EL = Lf @ np.linalg.inv(Lf[c, :])
        rown = (np.abs(EL) > 1e-9).sum(axis=1)
        assert list(rown) == [(a[f] + 1) * (a[f] + 2) // 2 for a in A]
        total += rown
    assert total.max() <= Nfp + 3


def test_lsrk4_stability_polynomial():
    """The five-stage scheme applied to y' = z y gives
    R(z) = 1 + z + z^2/2 + z^3/6 + z^4/24 + z^5/200 (fourth order)."""
    def padd(p, q):
        n = max(len(p), len(q))
        return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0) for i in range(n)]
    y, res = [Fraction(1)], [Fraction(0)]
    for a, b in zip(dg.LSRK_A, dg.LSRK_B):
        res = padd([Fraction(a) * x for x in res], [Fraction(0)] + y)
        y = padd(y, [Fraction(b) * x for x in res])
    want = [1, 1, 1 / 2, 1 / 6, 1 / 24, 1 / 200]
    np.testing.assert_allclose([float(x) for x in y], want, rtol=1e-13, atol=1e-15)
    # stage times: for y' = 1 the stage-s input equals c_s (dt = 1)
    q, r = 0.0, 0.0
    for s in range(5):
        assert abs(q - dg.LSRK_C[s]) < 1e-15
        r = dg.LSRK_A[s] * r + 1.0
        q += dg.LSRK_B[s] * r
    assert abs(q - 1.0) < 1e-15
