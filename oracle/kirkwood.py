"""Solvation energy of point charges inside a dielectric sphere in a screened
solvent (Kirkwood's sphere, the analytic test case of Sec. 3.1), as a series in
Legendre polynomials.

Matching the interior potential (Coulomb source plus regular reaction field
B_n r^n P_n) to an exterior field C_n k_n(kappa r) P_n (k_n the modified
spherical Bessel function of the second kind) through continuity of phi and of
eps dphi/dr at r = a gives, per degree n,
    reaction factor C_n = (eps2 R_n + eps1 (n+1)) / (eps1 n - eps2 R_n),
    R_n = x k_n'(x)/k_n(x) = n - x rho_n,  rho_n = k_{n+1}(x)/k_n(x),
    rho_0 = 1 + 1/x,  rho_n = 1/rho_{n-1} + (2n+1)/x,  x = kappa a,
and the energy (kcal/mol, charges in e, lengths in Angstrom)
    E = 332.0716/2 sum_j sum_k q_j q_k/(eps1 a) sum_n (r_j r_k/a^2)^n P_n(cos g_jk) C_n.
"""
import numpy as np


def reaction_factors(a, eps1, eps2, kappa, nmax):
    n = np.arange(nmax + 1)
    if kappa == 0.0:
        Rn = -(n + 1.0)
    else:
        x = kappa * a
        rho = np.empty(nmax + 1)
        rho[0] = 1.0 + 1.0 / x
        for k in range(1, nmax + 1):
            rho[k] = 1.0 / rho[k - 1] + (2 * k + 1) / x
        Rn = n - x * rho
    return (eps2 * Rn + eps1 * (n + 1)) / (eps1 * n - eps2 * Rn)


def legendre(nmax, t):
    P = np.zeros((nmax + 1,) + np.shape(t))
    P[0] = 1.0
    if nmax >= 1:
        P[1] = t
    for n in range(1, nmax):
        P[n + 1] = ((2 * n + 1) * t * P[n] - n * P[n - 1]) / (n + 1)
    return P


def energy(xq, q, a, eps1, eps2, kappa, nmax=60):
    xq = np.atleast_2d(np.asarray(xq, np.float64))
    q = np.asarray(q, np.float64)
    r = np.linalg.norm(xq, axis=1)
    C = reaction_factors(a, eps1, eps2, kappa, nmax)
    rr = np.outer(r, r)
    with np.errstate(invalid="ignore", divide="ignore"):
        cosg = (xq @ xq.T) / rr
    cosg = np.where(rr > 0, np.clip(cosg, -1.0, 1.0), 1.0)
    Pn = legendre(nmax, cosg)
    s = rr / (a * a)
    tot = np.zeros_like(rr)
    sp = np.ones_like(rr)
    for n in range(nmax + 1):
        tot += sp * Pn[n] * C[n]
        sp = sp * s
    return 0.5 * 332.0716 * float(q @ tot @ q) / (eps1 * a)


def born(q, a, eps1, eps2, kappa):
    """single central charge: the n = 0 term alone"""
    return 0.5 * 332.0716 * q * q / a * (1.0 / (eps2 * (1.0 + kappa * a)) - 1.0 / eps1)
