"""Cartesian treecode for the solvation energy (Sec. 2.5, "Cartesian
treecode": the particle-cluster form of the energy sum, the acceptance
criterion r_c / R <= theta and the addCluster recursion).

Test infrastructure: plain FP64 numpy, slow and obviously correct; only the
tests, the smoke check and the benchmark's CPU baseline use it.

The energy is E = 1/2 * 4 pi 332.0716 * sum_n q_n V_n with V_n the integral
over the surface of K1(x_n, y) dphi(y) + K2(x_n, y) phi(y) (Sec. 2.3), i.e.
the potential at x_n of the two FMM channels: Coulomb with the moments
M0 = m_s(dphi) - m_d(phi) and screened with Mk = -m_s(dphi) + eps m_d(phi).

Readings (one choice, used by the GPU path as well):
  * the moments m'_c are the FMM's: leaf moments by the 3-point rule and the
    MtM upward pass, order p_l on level l; a particle-cluster term is the MtL
    row alpha = 0 at the point x_n:
        V_n += sum_|b|<=p_l (-1)^|b| [F_b(x_n - x_c; 0) M0_b + F_b(x_n - x_c; kappa) Mk_b] / (4 pi)
    with F_b the Taylor coefficients of exp(-kappa r)/r (oracle.taylor);
  * x_c is the cube centre and r_c the level's radius rho_l (the largest
    cluster radius of the level, so acceptance is never looser than with the
    cluster's own radius); the criterion rho_l / R <= theta is evaluated as
    rho_l^2 <= theta^2 ((dx^2 + dy^2) + dz^2) in that order;
  * the recursion starts from every cluster of level min(l_min, L), the
    coarsest level that carries moments (for charges inside the molecule no
    coarser cluster can pass the criterion);
  * a leaf that fails the criterion is summed directly with the 3-point rule,
    with the integrand of the direct energy sum (oracle.solve.energy);
  * an optional order cap p_max evaluates the terms |b| <= min(p_l, p_max)
    only (the leading terms of the level's moments).

The right-hand side (Sec. 2.2 source terms, b1 = (1/eps_in) int psi_i
sum_n q_n G0(x, x_n), b2 likewise with dG0/dn_x) by the same visit run in
reverse: a charge accepted by a cluster adds its particle-to-local expansion
q_n F_a(x_c - x_n; 0) / 4 pi to the cluster's Coulomb local expansion (the
MtL column beta = 0 of a point source), a leaf that fails is summed directly
(the integrand of oracle.solve.rhs), then the far field's LtL takes the
locals down to the leaves and LtP tests them with the single- and double-
layer moments of each panel (step 6 of the FMM).
"""
import numpy as np

from . import taylor
from .fmm import downward, upward
from .solve import UNIT_KCAL

FOUR_PI = 4.0 * np.pi


def _direct(P, ids, xn, phi, dphi, eps, kappa):
    """sum over the panels ids of the 3-point rule of K1 dphi + K2 phi at x_n."""
    r = xn[None, None, :] - P.qp[ids]                       # x_n - y_q
    rr = np.sqrt((r * r).sum(-1))
    u = kappa * rr
    em1 = np.expm1(-u)
    E = em1 + 1.0
    rny = (r * P.normal[ids][:, None, :]).sum(-1)
    k1 = -em1 / (FOUR_PI * rr)
    k2 = (eps * E * (1.0 + u) - 1.0) * rny / (FOUR_PI * rr ** 3)
    return float((P.qw[ids] * (k1 * dphi[ids][:, None] + k2 * phi[ids][:, None])).sum())


def _far(d, m0, mk, kappa, p):
    """particle-cluster terms of the clusters at offsets d = x_n - x_c [m, 3]."""
    mi = taylor.multi_indices(p)
    F0 = taylor.coefficients(d, 0.0, p)
    Fk = taylor.coefficients(d, kappa, p)
    v = np.zeros(len(d))
    for t, k in enumerate(mi):
        s = -1.0 if sum(k) & 1 else 1.0
        v += s * (F0[k] * m0[:, t] + Fk[k] * mk[:, t])
    return v / FOUR_PI


def potentials(F, x, xq, theta, moments=None, p_max=None):
    """V_n for every charge by the treecode, and the number of particle-cluster
    terms and of directly summed leaves (per charge)."""
    P, tree, eps, kappa, pl = F.P, F.tree, F.eps, F.kappa, F.orders
    N = P.n
    phi, dphi = x[:N], x[N:]
    M0, Mk = moments if moments is not None else upward(F, phi, dphi)
    L, levels, perm = tree.L, tree.levels, tree.perm
    l0 = min(tree.lmin, L)
    xq = np.atleast_2d(np.asarray(xq, np.float64))
    V = np.zeros(len(xq))
    n_far = np.zeros(len(xq), np.int64)
    n_leaf = np.zeros(len(xq), np.int64)
    th2 = theta * theta
    for n in range(len(xq)):
        xn = xq[n]
        front = np.arange(levels[l0].n)
        for l in range(l0, L + 1):
            if len(front) == 0:
                break
            cl = levels[l]
            d = xn[None, :] - cl.center[front]
            R2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            acc = cl.rho * cl.rho <= th2 * R2
            if acc.any():
                a = front[acc]
                p = pl[l] if p_max is None else min(pl[l], p_max)
                T = len(taylor.multi_indices(p))
                V[n] += _far(d[acc], M0[l][a][:, :T], Mk[l][a][:, :T], kappa, p).sum()
                n_far[n] += len(a)
            rest = front[~acc]
            if l < L:
                front = np.concatenate([np.arange(cl.child_start[c], cl.child_end[c]) for c in rest]) \
                    if len(rest) else rest
            else:
                for c in rest:
                    V[n] += _direct(P, perm[cl.start[c]:cl.end[c]], xn, phi, dphi, eps, kappa)
                n_leaf[n] += len(rest)
    return V, n_far, n_leaf


def energy(F, x, xq, q, theta, p_max=None):
    """E_sol in kcal/mol by the treecode (theta = 0 accepts no cluster: the
    direct sum)."""
    V, _, _ = potentials(F, x, xq, theta, p_max=p_max)
    return 0.5 * UNIT_KCAL * float(np.dot(np.asarray(q, np.float64), V))


def rhs(F, xq, q, theta, eps_in, p_max=None):
    """b = [b1; b2] (panel order) by the reverse treecode (theta = 0: the
    direct sum of oracle.solve.rhs)."""
    P, tree, pl = F.P, F.tree, F.orders
    N = P.n
    L, levels, perm = tree.L, tree.levels, tree.perm
    l0 = min(tree.lmin, L)
    xq = np.atleast_2d(np.asarray(xq, np.float64))
    q = np.asarray(q, np.float64)
    lam = {l: np.zeros((levels[l].n, len(taylor.multi_indices(pl[l])))) for l in range(l0, L + 1)}
    b1 = np.zeros(N)
    b2 = np.zeros(N)
    th2 = theta * theta
    for n in range(len(xq)):
        xn = xq[n]
        front = np.arange(levels[l0].n)
        for l in range(l0, L + 1):
            if len(front) == 0:
                break
            cl = levels[l]
            d = xn[None, :] - cl.center[front]
            R2 = (d[:, 0] * d[:, 0] + d[:, 1] * d[:, 1]) + d[:, 2] * d[:, 2]
            acc = cl.rho * cl.rho <= th2 * R2
            if acc.any():
                a = front[acc]
                p = pl[l] if p_max is None else min(pl[l], p_max)
                Fc = taylor.coefficients(-d[acc], 0.0, p)           # at x_c - x_n
                for t, k in enumerate(taylor.multi_indices(p)):
                    lam[l][a, t] += q[n] * Fc[k] / FOUR_PI
            rest = front[~acc]
            if l < L:
                front = np.concatenate([np.arange(cl.child_start[c], cl.child_end[c]) for c in rest]) \
                    if len(rest) else rest
            else:
                for c in rest:
                    ids = perm[cl.start[c]:cl.end[c]]
                    r = P.qp[ids] - xn[None, None, :]                # y_q - x_n
                    rr = np.sqrt((r * r).sum(-1))
                    g0 = 1.0 / (FOUR_PI * rr)
                    dg0 = -(r * P.normal[ids][:, None, :]).sum(-1) / (FOUR_PI * rr ** 3)
                    b1[ids] += q[n] * (P.qw[ids] * g0).sum(1)
                    b2[ids] += q[n] * (P.qw[ids] * dg0).sum(1)
    downward(F, lam, l0)
    f = lam[L][F.owner]                                             # tree order
    b1[perm] += (f * F.ms).sum(1)
    b2[perm] += (f * F.md).sum(1)
    return np.concatenate([b1, b2]) / eps_in
