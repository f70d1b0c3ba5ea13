"""Dense Galerkin system (Sec. 2.3, linear system A x = b with blocks A11..A22).

A11 = (1+eps)/2 diag(A) - (eps I3 - I2)     A12 = -I1
A21 = -I6                                    A22 = (1+1/eps)/2 diag(A) - (I4 - I5/eps)
(eps = eps_out/eps_in; the integral terms of the boundary integral equations
enter with a minus sign once moved to the left-hand side; the printed entry
formulas show plus signs, which contradict the integral equations and the
variational form - the minus reading reproduces the Born solution).
Every pair (i, j) is integrated with the rule its class selects (``pairs``).
"""
import numpy as np

from .kernels import combine
from .pairs import pair_integrals


def integrals(P, kappa, near_ratio=2.0, n=7, rows=None):
    N = P.n
    rows = np.arange(N) if rows is None else np.asarray(rows)
    ii = np.repeat(rows, N)
    jj = np.tile(np.arange(N), len(rows))
    I, cls = pair_integrals(P, ii, jj, kappa, near_ratio, n)
    return I.reshape(len(rows), N, 6), cls.reshape(len(rows), N)


def assemble(P, eps, kappa, near_ratio=2.0, n=7):
    N = P.n
    I, _ = integrals(P, kappa, near_ratio, n)
    B = combine(I, eps)
    A = np.zeros((2 * N, 2 * N))
    A[:N, :N] = B[..., 0] + np.diag(0.5 * (1.0 + eps) * P.area)
    A[:N, N:] = B[..., 1]
    A[N:, :N] = B[..., 2]
    A[N:, N:] = B[..., 3] + np.diag(0.5 * (1.0 + 1.0 / eps) * P.area)
    return A


def rows_matvec(P, eps, kappa, x, rows, near_ratio=2.0, n=7):
    """(A x) restricted to the given panel rows, for both equation blocks,
    without storing A: returns (y1[rows], y2[rows])."""
    N = P.n
    I, _ = integrals(P, kappa, near_ratio, n, rows)
    B = combine(I, eps)
    phi, dphi = x[:N], x[N:]
    y1 = B[..., 0] @ phi + B[..., 1] @ dphi + 0.5 * (1.0 + eps) * P.area[rows] * phi[rows]
    y2 = B[..., 2] @ phi + B[..., 3] @ dphi + 0.5 * (1.0 + 1.0 / eps) * P.area[rows] * dphi[rows]
    return y1, y2
