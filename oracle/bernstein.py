"""Dense Bernstein-Bezier operators on the reference tetrahedron (oracle).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Definitions followed (Section 3, Section 3.1):
  * barycentric coordinates of the bi-unit reference tetrahedron
      lambda0 = -(1+r+s+t)/2, lambda1 = (1+r)/2, lambda2 = (1+s)/2, lambda3 = (1+t)/2;
  * B_alpha = N!/(alpha!) lambda^alpha for |alpha| = N (scaled monomials);
  * mass matrix M_ij = int B_i B_j over the element, face mass M^f over face f
    (face f is the face opposite vertex f, where lambda_f = 0);
  * the derivative matrix of a coordinate is the operator mapping the
    coefficients of p to those of the derivative of p;
  * lift L^f = M^{-1} M^f.

Exactness: every matrix here is computed exactly in rationals.  Integrals
use the simplex moment formula  int_T lambda^g = |T| d! g! / (|g| + d)!.
Linear solves take a candidate from Gaussian elimination in 80-bit floating
point, round it to the nearest multiple of 1/den, and then verify A X = B
exactly modulo three primes near 2^25; any mismatch raises.  (A wrong
candidate cannot pass all three congruences except with probability
~2^-75.)  Float64 versions are the exact rationals rounded once.

Coefficient order (shared convention of the whole project): alpha =
(a0, a1, a2, a3), |alpha| = N, enumerated with a3 slowest, then a2, then a1
fastest; a0 = N - a1 - a2 - a3.  Face-local order on a triangle of degree m:
(g0, g1, g2) with g2 slowest, then g1 fastest.
"""
from fractions import Fraction
from functools import lru_cache
from math import factorial, gcd

import numpy as np


# ---------------------------------------------------------------------------
# multi-indices
# ---------------------------------------------------------------------------

def multi_indices(N):
    """All (a0,a1,a2,a3) with sum N in storage order."""
    out = []
    for a3 in range(N + 1):
        for a2 in range(N + 1 - a3):
            for a1 in range(N + 1 - a3 - a2):
                out.append((N - a1 - a2 - a3, a1, a2, a3))
    return out


def tri_indices(m):
    """All (g0,g1,g2) with sum m in face-local order."""
    out = []
    for g2 in range(m + 1):
        for g1 in range(m + 1 - g2):
            out.append((m - g1 - g2, g1, g2))
    return out


def np_count(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def nfp_count(N):
    return (N + 1) * (N + 2) // 2


def face_vertices(f):
    """Local vertices of face f (the face opposite vertex f), increasing."""
    return tuple(v for v in range(4) if v != f)


def face_node_ids(N, f):
    """Volume indices of the nodes on face f, in face-local order.

    Face-local node (g0,g1,g2) is the volume node with alpha_f = 0 and
    alpha[face_vertices(f)[m]] = g_m."""
    index = {a: i for i, a in enumerate(multi_indices(N))}
    fv = face_vertices(f)
    ids = []
    for g in tri_indices(N):
        a = [0, 0, 0, 0]
        for m in range(3):
            a[fv[m]] = g[m]
        ids.append(index[tuple(a)])
    return np.array(ids, dtype=np.int64)


def _multinomial(a):
    r = factorial(sum(a))
    for x in a:
        r //= factorial(x)
    return r


def _fact_prod(a):
    r = 1
    for x in a:
        r *= factorial(x)
    return r


# ---------------------------------------------------------------------------
# exact linear algebra
# ---------------------------------------------------------------------------

_PRIMES = (33554393, 33554383, 33554371)  # primes just below 2^25


def _lcm_upto(n):
    r = 1
    for k in range(2, n + 1):
        r = r * k // gcd(r, k)
    return r


def _to_modp(F, p):
    """Fraction matrix -> int64 residues mod p (denominators must be units)."""
    out = np.empty((len(F), len(F[0])), dtype=np.int64)
    for i, row in enumerate(F):
        for j, x in enumerate(row):
            out[i, j] = (x.numerator % p) * pow(x.denominator % p, -1, p) % p
    return out


def _matmul_modp(A, B, p):
    # entries < 2^25, so every product < 2^50 and a row of <= 2^12 terms fits int64
    return (A @ B) % p


def _ld_gauss_solve(A, B):
    """Gaussian elimination with partial pivoting in np.longdouble."""
    A = A.copy()
    B = B.copy()
    n = A.shape[0]
    for c in range(n):
        piv = c + int(np.argmax(np.abs(A[c:, c])))
        if piv != c:
            A[[c, piv]] = A[[piv, c]]
            B[[c, piv]] = B[[piv, c]]
        f = A[c + 1:, c] / A[c, c]
        A[c + 1:, c:] -= np.outer(f, A[c, c:])
        B[c + 1:] -= np.outer(f, B[c])
    X = np.zeros_like(B)
    for c in range(n - 1, -1, -1):
        X[c] = (B[c] - A[c, c + 1:] @ X[c + 1:]) / A[c, c]
    return X


def _frac_to_ld(F):
    out = np.empty((len(F), len(F[0])), dtype=np.longdouble)
    for i, row in enumerate(F):
        for j, x in enumerate(row):
            out[i, j] = np.longdouble(x.numerator) / np.longdouble(x.denominator)
    return out


def exact_solve(A, B, den):
    """Exact rational X with A X = B (A square, nonsingular; lists of Fractions).

    X is found as the nearest multiples of 1/den to an extended-precision
    solution and then checked exactly modulo three primes."""
    Xld = _ld_gauss_solve(_frac_to_ld(A), _frac_to_ld(B))
    scaled = np.rint(Xld * np.longdouble(den))
    X = [[Fraction(int(v), den) for v in row] for row in scaled]
    for p in _PRIMES:
        lhs = _matmul_modp(_to_modp(A, p), _to_modp(X, p), p)
        if not np.array_equal(lhs, _to_modp(B, p)):
            raise ArithmeticError("exact_solve: candidate rational solution fails verification")
    return X


def to_f64(F):
    return np.array([[float(x) for x in row] for row in F], dtype=np.float64)


# ---------------------------------------------------------------------------
# dense operators
# ---------------------------------------------------------------------------

def bernstein_values(N, lam):
    """B_alpha(lam) for exact barycentric points lam (list of 4-tuples of Fractions).

    Returns a list (points) of lists (alpha) of Fractions."""
    A = multi_indices(N)
    rows = []
    for l in lam:
        row = []
        for a in A:
            v = Fraction(_multinomial(a))
            for li, ai in zip(l, a):
                v *= li ** ai
            row.append(v)
        rows.append(row)
    return rows


def bernstein_bary_derivative_values(N, lam, i):
    """d/d(lambda_i) B_alpha at points lam, differentiating the monomial
    lambda^alpha with the power rule (lambda treated as 4 independent variables)."""
    A = multi_indices(N)
    rows = []
    for l in lam:
        row = []
        for a in A:
            if a[i] == 0:
                row.append(Fraction(0))
                continue
            v = Fraction(_multinomial(a) * a[i])
            for j, (lj, aj) in enumerate(zip(l, a)):
                v *= lj ** (aj - 1 if j == i else aj)
            row.append(v)
        rows.append(row)
    return rows


def lattice_points(N):
    """Equispaced lattice lambda = alpha / N (unisolvent for degree N)."""
    return [tuple(Fraction(x, N) for x in a) for a in multi_indices(N)]


@lru_cache(maxsize=None)
def bary_derivative_exact(N):
    """Exact dense barycentric derivative matrices D^0..D^3 (Np x Np each).

    Column beta of V holds B_beta at the lattice points; column beta of V_i
    holds d B_beta / d lambda_i there.  The coefficients of d p / d lambda_i
    are D^i c with V D^i = V_i."""
    lam = lattice_points(N)
    V = bernstein_values(N, lam)
    den = 2 * _lcm_upto(2 * N + 4)
    return tuple(exact_solve(V, bernstein_bary_derivative_values(N, lam, i), den) for i in range(4))


@lru_cache(maxsize=None)
def mass_exact(N):
    """Volume mass matrix of the unit-volume-normalised simplex:
    m_ab = (1/|T|) int_T B_a B_b = (N!)^2/(a! b!) * 3! (a+b)!/(2N+3)!."""
    A = multi_indices(N)
    fN2 = factorial(N) ** 2
    return [[Fraction(fN2 * 6 * _fact_prod([x + y for x, y in zip(a, b)]),
                      _fact_prod(a) * _fact_prod(b) * factorial(2 * N + 3)) for b in A] for a in A]


@lru_cache(maxsize=None)
def face_mass_exact(N, f):
    """Face mass matrix over face f normalised by the face area (Np x Np, zero
    off the face): (1/|F|) int_F B_a B_b = (N!)^2/(a! b!) * 2! (a+b)!/(2N+2)!
    when a_f = b_f = 0 (on the face lambda_f = 0 the other three barycentric
    coordinates are the face's own)."""
    A = multi_indices(N)
    fN2 = factorial(N) ** 2
    out = []
    for a in A:
        row = []
        for b in A:
            if a[f] or b[f]:
                row.append(Fraction(0))
            else:
                row.append(Fraction(fN2 * 2 * _fact_prod([x + y for x, y in zip(a, b)]),
                                    _fact_prod(a) * _fact_prod(b) * factorial(2 * N + 2)))
        out.append(row)
    return out


@lru_cache(maxsize=None)
def lift_exact(N, f):
    """Normalised lift m^{-1} m^f (Np x Np), with m, m^f the area/volume-normalised
    mass matrices above.  On an element of volume V with face area A_f the
    physical lift is (A_f / V) times this matrix."""
    den = 6 * _lcm_upto(2 * N + 4)
    return exact_solve(mass_exact(N), face_mass_exact(N, f), den)


@lru_cache(maxsize=None)
def reference_lift_exact(N, f):
    """L^f = M^{-1} M^f on the bi-unit reference tetrahedron (volume 4/3) with
    every reference face measured on a triangle of area 2, i.e. (2/(4/3)) times
    the normalised lift."""
    return [[Fraction(3, 2) * x for x in row] for row in lift_exact(N, f)]


# float64 views ---------------------------------------------------------------

@lru_cache(maxsize=None)
def bary_derivative(N):
    """float64 (4, Np, Np): D[i] maps coefficients to those of d/d lambda_i."""
    return np.stack([to_f64(D) for D in bary_derivative_exact(N)])


@lru_cache(maxsize=None)
def mass(N):
    return to_f64(mass_exact(N))


@lru_cache(maxsize=None)
def face_mass(N, f):
    return to_f64(face_mass_exact(N, f))


@lru_cache(maxsize=None)
def lift(N):
    """float64 (4, Np, Np): normalised lifts m^{-1} m^f for f = 0..3."""
    return np.stack([to_f64(lift_exact(N, f)) for f in range(4)])


def face_mass_2d_exact(m):
    """Area-normalised mass matrix of degree-m Bernstein polynomials on a triangle."""
    T = tri_indices(m)
    fm2 = factorial(m) ** 2
    return [[Fraction(fm2 * 2 * _fact_prod([x + y for x, y in zip(a, b)]),
                      _fact_prod(a) * _fact_prod(b) * factorial(2 * m + 2)) for b in T] for a in T]
