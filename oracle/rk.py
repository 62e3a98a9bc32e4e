"""Runge-Kutta schemes of the paper, in exact rational arithmetic.

* Classical RK4 -- Sec. 2 names it as one of the solver's integrators; the
  coefficients are the textbook Butcher tableau.
* LSERK (2N-storage) -- Sec. 2, Eq. (3):
      Q^(m) = A_m Q^(m-1) + dt R(U^(m-1)),   U^(m) = U^(m-1) + B_m Q^(m).
  LSERK2: A = {0, -1/2}, B = {1/2, 1}  (App. B).
  LSERK4: the five-stage coefficients of App. B, Table 4, as printed (8 digits).

``stage_polynomials`` returns, for every stage input e = 0..s-1, the
polynomial in z = lambda*dt that the scheme produces for the linear test
equation y' = lambda*y.  Its coefficients are the nu_j^e of Sec. 3.1
(Eqs. 9-10): nu_0^e = 1, nu_1^e is the stage abscissa, nu_e^e is the product
of the B's.  Where the text elides the middle coefficients, this reading
(coefficient of z^j in stage e's polynomial) reproduces the printed first and
last ones.
"""
from fractions import Fraction as Fr

RK4 = "rk4"
LSERK4 = "lserk4"
LSERK2 = "lserk2"

# Classical RK4 Butcher tableau.
RK4_A = [[Fr(0), Fr(0), Fr(0), Fr(0)],
         [Fr(1, 2), Fr(0), Fr(0), Fr(0)],
         [Fr(0), Fr(1, 2), Fr(0), Fr(0)],
         [Fr(0), Fr(0), Fr(1), Fr(0)]]
RK4_B = [Fr(1, 6), Fr(1, 3), Fr(1, 3), Fr(1, 6)]

# App. B, Table 4 (LSERK4), exactly as printed.
LSERK4_A = [Fr("0"), Fr("-0.4812317"), Fr("-1.0495626"), Fr("-1.6025296"),
            Fr("-1.7782672")]
LSERK4_B = [Fr("0.09761835"), Fr("0.41225329"), Fr("0.44021696"),
            Fr("1.42631146"), Fr("0.19787605")]

# App. B (LSERK2).
LSERK2_A = [Fr(0), Fr(-1, 2)]
LSERK2_B = [Fr(1, 2), Fr(1)]


def lserk_coeffs(scheme):
    if scheme == LSERK4:
        return LSERK4_A, LSERK4_B
    if scheme == LSERK2:
        return LSERK2_A, LSERK2_B
    raise ValueError(scheme)


def n_stages(scheme):
    return {RK4: 4, LSERK4: 5, LSERK2: 2}[scheme]


def _padd(p, q):
    n = max(len(p), len(q))
    return [(p[i] if i < len(p) else 0) + (q[i] if i < len(q) else 0)
            for i in range(n)]


def _pscale(p, a):
    return [a * c for c in p]


def _pshift(p):
    """Multiply a polynomial in z by z."""
    return [Fr(0)] + list(p)


def stage_polynomials(scheme):
    """(stages, step): stages[e] = coefficients of the stage-e input U^(e)
    (e = 0..s-1) as a polynomial in z; step = the one-step amplification
    polynomial U^(s)."""
    if scheme == RK4:
        Y = []
        for e in range(4):
            acc = [Fr(0)]
            for j in range(e):
                acc = _padd(acc, _pscale(Y[j], RK4_A[e][j]))
            Y.append(_padd([Fr(1)], _pshift(acc)))
        acc = [Fr(0)]
        for j in range(4):
            acc = _padd(acc, _pscale(Y[j], RK4_B[j]))
        return Y, _padd([Fr(1)], _pshift(acc))
    A, B = lserk_coeffs(scheme)
    U = [Fr(1)]
    Q = [Fr(0)]
    stages = [U]
    for m in range(len(A)):
        Q = _padd(_pscale(Q, A[m]), _pshift(U))
        U = _padd(U, _pscale(Q, B[m]))
        if m < len(A) - 1:
            stages.append(U)
    return stages, U


def nu(scheme):
    """nu[e][j] -- the coefficients of Eq. (9) for stage e."""
    stages, _ = stage_polynomials(scheme)
    return [list(p) for p in stages]


def lserk_to_butcher(scheme):
    """Butcher (a, b, c) of a 2N-storage scheme.

    Unrolling Eq. (3): Q^(m) = sum_{j<=m} (prod_{r=j+1..m} A_r) dt R(U^(j-1)),
    so U^(m) = U^(0) + dt sum_{j=1..m} R(U^(j-1)) sum_{i=j..m} B_i prod_{r=j+1..i} A_r.
    """
    A, B = lserk_coeffs(scheme)
    s = len(A)

    def coeff(m, j):  # weight of R(U^(j-1)) in U^(m); 1-based m, j
        tot = Fr(0)
        for i in range(j, m + 1):
            prod = Fr(1)
            for r in range(j + 1, i + 1):
                prod *= A[r - 1]
            tot += B[i - 1] * prod
        return tot

    a = [[coeff(m, j + 1) if j < m else Fr(0) for j in range(s)]
         for m in range(s)]            # row m = stage input U^(m), m = 0..s-1
    b = [coeff(s, j + 1) for j in range(s)]
    c = [sum(row) for row in a]
    return a, b, c


def butcher(scheme):
    if scheme == RK4:
        a = RK4_A
        b = RK4_B
        return a, b, [sum(r) for r in a]
    return lserk_to_butcher(scheme)


def order_condition_residuals(scheme):
    """The eight classical order conditions up to order 4 (Butcher trees),
    returned as residuals (value - target)."""
    a, b, c = butcher(scheme)
    s = len(b)

    def ac(vec):
        return [sum(a[i][j] * vec[j] for j in range(s)) for i in range(s)]

    def dot(u, v):
        return sum(x * y for x, y in zip(u, v))

    one = [Fr(1)] * s
    c2 = [x * x for x in c]
    c3 = [x * x * x for x in c]
    acv = ac(c)
    res = [
        dot(b, one) - 1,
        dot(b, c) - Fr(1, 2),
        dot(b, c2) - Fr(1, 3),
        dot(b, acv) - Fr(1, 6),
        dot(b, c3) - Fr(1, 4),
        dot(b, [ci * x for ci, x in zip(c, acv)]) - Fr(1, 8),
        dot(b, ac(c2)) - Fr(1, 12),
        dot(b, ac(acv)) - Fr(1, 24),
    ]
    return res
