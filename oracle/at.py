"""Asynchrony-tolerant (AT) coefficients, exact rational arithmetic.

Notation.  A buffer (halo) point holds C delayed levels
U^{n-k}, U^{n-k-1}, ..., U^{n-k-C+1}, where k is the delay (k-tilde in the
paper) and level l (l = 0..C-1) sits at time t_n - (k+l) dt.  All weights
below act on that vector of C levels.  Time is measured in units of dt, so a
temporal-derivative coefficient returned here multiplies 1/dt.

Three objects of Sec. 3 are computed:

1. PE-boundary stencil (Eqs. 4-7).  With the spatial stencil kept and only
   the buffer values taken at C delayed levels, Eq. (7) writes the boundary
   derivative as c(k)^T Phi(k).  The Taylor constraints of Eq. (6) then
   reduce to the time moments sum_l c_l (-(k+l))^theta / theta! = delta_{theta,0}
   for theta = 0..C-1 (``boundary_coefficients``).  The result equals the
   Lagrange extrapolation of the buffer value to t_n (Eqs. 14-15,
   ``lagrange_extrapolation``).

2. Buffer temporal derivative at stage e (Eqs. 8-13): the constraints of
   Eq. (12), sum_l c_l (-(k+l))^theta/theta! = nu_{theta-1}^e for
   theta = 1..e+1 and 0 for theta = 0 and e+1 < theta < q/r+1
   (``buffer_derivative``).

3. The halo value used at stage e.  Stage 0 uses the extrapolation; later
   stages run the RK recursion of Eq. (8) on the buffer with the
   temporal derivative in place of the spatial residual.  Every stage value is
   therefore a fixed linear combination W[e][l] of the C levels.
   ``halo_weights_literal`` runs that recursion in weight space;
   ``halo_weights_closed`` uses the closed form
       W_e = sum_j nu_j^e * d^j/dtau^j p(tau)|_{tau=0},
   p being the degree-(C-1) interpolant of the C levels.  Both must agree
   exactly.

Reading (paper is ambiguous): the second AT4 weight is printed with 25 k^2
both in Eq. (7)'s AT4 vector and in Eq. (15); the weights only sum to one
(and match the Lagrange form) with 26 k^2.  The oracle uses the derived
(26) value; the printed form is kept in the golden fixture and the test shows
it is inconsistent.
"""
from fractions import Fraction as Fr
from math import factorial

from . import rk as rkmod

AT2_C = 3   # (d, q, r) = (1, 2, 1)
AT4_C = 5   # (d, q, r) = (1, 4, 1)


def solve_exact(M, rhs):
    """Gauss-Jordan elimination over the rationals."""
    n = len(M)
    A = [[Fr(x) for x in row] + [Fr(rhs[i])] for i, row in enumerate(M)]
    for col in range(n):
        piv = next(r for r in range(col, n) if A[r][col] != 0)
        A[col], A[piv] = A[piv], A[col]
        p = A[col][col]
        A[col] = [x / p for x in A[col]]
        for r in range(n):
            if r != col and A[r][col] != 0:
                f = A[r][col]
                A[r] = [x - f * y for x, y in zip(A[r], A[col])]
    return [A[i][n] for i in range(n)]


def _moment_matrix(k, C):
    """Row theta, column l: (-(k+l))^theta / theta!  (Eq. 5 / Eq. 10 with dt=1)."""
    return [[Fr(-(k + l)) ** th / factorial(th) for l in range(C)]
            for th in range(C)]


def boundary_coefficients(k, C):
    """c(k) of Eq. (7) from the time-moment constraints (Eq. 6 reduced)."""
    rhs = [Fr(1)] + [Fr(0)] * (C - 1)
    return solve_exact(_moment_matrix(k, C), rhs)


def lagrange_extrapolation(k, C):
    """Weights of the Lagrange extrapolation to tau = 0 from the nodes
    tau_l = -(k+l), l = 0..C-1 (Eqs. 14-15 closed form)."""
    w = []
    for l in range(C):
        num = Fr(1)
        for m in range(C):
            if m != l:
                num *= Fr(0 - (-(k + m)), (-(k + l)) - (-(k + m)))
        w.append(num)
    return w


def buffer_derivative(k, C, nu_e):
    """Coefficients (times 1/dt) of the stage-e temporal derivative, Eq. (12).

    nu_e = [nu_0^e, ..., nu_e^e].  Requires e + 1 <= C - 1.
    """
    e = len(nu_e) - 1
    if e + 1 > C - 1:
        raise ValueError("stage too high for C levels")
    rhs = [Fr(0)] * C
    for j in range(e + 1):
        rhs[j + 1] = Fr(nu_e[j])
    return solve_exact(_moment_matrix(k, C), rhs)


def _lagrange_basis_poly(k, C, l):
    """Coefficients (in tau, ascending) of the Lagrange basis polynomial L_l."""
    nodes = [Fr(-(k + m)) for m in range(C)]
    poly = [Fr(1)]
    denom = Fr(1)
    for m in range(C):
        if m == l:
            continue
        # multiply by (tau - node_m)
        new = [Fr(0)] * (len(poly) + 1)
        for i, c in enumerate(poly):
            new[i + 1] += c
            new[i] -= nodes[m] * c
        poly = new
        denom *= nodes[l] - nodes[m]
    return [c / denom for c in poly]


def interpolant_derivative_weights(k, C, j):
    """Weights over the C levels of p^{(j)}(0), p the degree-(C-1) interpolant."""
    out = []
    for l in range(C):
        poly = _lagrange_basis_poly(k, C, l)
        out.append(poly[j] * factorial(j) if j < len(poly) else Fr(0))
    return out


def halo_weights_literal(scheme, k, C):
    """W[e][l], e = 0..s-1, by running the buffer recursion of Eq. (8).

    Stage 0: extrapolation (Eqs. 14-15).  Stage e >= 1: the RK recursion with
    dt*dU/dt|^(e-1) given by ``buffer_derivative`` (Eq. 12).
    """
    s = rkmod.n_stages(scheme)
    nus = rkmod.nu(scheme)
    u0 = boundary_coefficients(k, C)
    derivs = [buffer_derivative(k, C, nus[e]) for e in range(s - 1)]
    W = [u0]
    if scheme == rkmod.RK4:
        a, _, _ = rkmod.butcher(scheme)
        for e in range(1, s):
            w = list(u0)
            for j in range(e):
                w = [x + a[e][j] * d for x, d in zip(w, derivs[j])]
            W.append(w)
        return W
    A, B = rkmod.lserk_coeffs(scheme)
    q = [Fr(0)] * C
    u = list(u0)
    for m in range(1, s):            # Eq. (8) for m = 1..s-1
        q = [A[m - 1] * qq + d for qq, d in zip(q, derivs[m - 1])]
        u = [uu + B[m - 1] * qq for uu, qq in zip(u, q)]
        W.append(list(u))
    return W


def halo_weights_closed(scheme, k, C):
    """W[e][l] = sum_j nu_j^e p^{(j)}(0) weights (closed form)."""
    s = rkmod.n_stages(scheme)
    nus = rkmod.nu(scheme)
    D = [interpolant_derivative_weights(k, C, j) for j in range(C)]
    W = []
    for e in range(s):
        w = [Fr(0)] * C
        for j, nj in enumerate(nus[e]):
            if j < C:
                w = [x + nj * d for x, d in zip(w, D[j])]
        W.append(w)
    return W


SA, AS, AT = "sa", "as", "at"


def halo_table(scheme, mode, C, kmax):
    """float table W[e][k][l] for k = 0..kmax used by the solver.

    AT: closed form above.  AS (standard stencil on stale data, Table 1 cases
    2 and 5): W = delta_{l,0} at every stage.  SA has no table.
    """
    import numpy as np
    s = rkmod.n_stages(scheme)
    T = np.zeros((s, kmax + 1, C))
    for k in range(kmax + 1):
        if mode == AT:
            W = halo_weights_closed(scheme, k, C)
            for e in range(s):
                T[e, k, :] = [float(x) for x in W[e]]
        elif mode == AS:
            T[:, k, 0] = 1.0
        else:
            raise ValueError(mode)
    return T
