"""Right-hand side, solvation energy, block-diagonal preconditioner and GMRES.

* RHS (Sec. 2.2 source terms, tested with the box functions of Sec. 2.3):
    b1_i = sum_q w_q (1/eps_in) sum_k q_k G0(x_q, y_k)
    b2_i = sum_q w_q (1/eps_in) sum_k q_k dG0(x_q, y_k)/dn_x
  with the same 3-point rule as the regular near field.
* Energy (Sec. 2.3 discrete solvation energy and the unit factor 4 pi 332.0716
  of Sec. 3):
    E = 4 pi 332.0716 * 1/2 sum_n q_n sum_i sum_q w_q
          [K1(x_n, y_q) dphi_i + K2(x_n, y_q) phi_i]      (kcal/mol)
  K1 = G0 - Gk, K2 = eps dGk/dn_y - dG0/dn_y at the panel point y_q.
* Block-diagonal preconditioner (Sec. 2.6): M keeps the entries of A between
  panels of the same leaf cube (identity terms included); each leaf block
  [phi_c; dphi_c] is solved directly.
* GMRES (Sec. 2.3 closing paragraph): right-preconditioned, x0 = 0, no
  restart, modified Gram-Schmidt, Givens rotations; stops when the residual
  estimate drops below tol * ||b||.
"""
import numpy as np

from .kernels import FOUR_PI

UNIT_KCAL = 4.0 * np.pi * 332.0716


def rhs(P, xq, q, eps_in):
    xq = np.atleast_2d(xq)
    r = P.qp[:, :, None, :] - xq[None, None, :, :]         # [N,3,Nc,3]
    rr = np.sqrt((r * r).sum(-1))
    g0 = 1.0 / (FOUR_PI * rr)
    dg0 = -(r * P.normal[:, None, None, :]).sum(-1) / (FOUR_PI * rr ** 3)
    b1 = (P.qw * (g0 @ q)).sum(1) / eps_in
    b2 = (P.qw * (dg0 @ q)).sum(1) / eps_in
    return np.concatenate([b1, b2])


def energy(P, x, xq, q, eps, kappa):
    N = P.n
    phi, dphi = x[:N], x[N:]
    xq = np.atleast_2d(xq)
    total = 0.0
    for n in range(len(q)):
        r = xq[n][None, None, :] - P.qp                     # x_n - y_q
        rr = np.sqrt((r * r).sum(-1))
        u = kappa * rr
        em1 = np.expm1(-u)
        E = em1 + 1.0
        rny = (r * P.normal[:, None, :]).sum(-1)
        k1 = -em1 / (FOUR_PI * rr)
        k2 = (eps * E * (1.0 + u) - 1.0) * rny / (FOUR_PI * rr ** 3)
        pot = (P.qw * (k1 * dphi[:, None] + k2 * phi[:, None])).sum()
        total += q[n] * pot
    return 0.5 * UNIT_KCAL * total


def block_preconditioner(P, tree, eps, kappa, near_ratio=2.0, n=7, group_max=0):
    """Returns a function z -> M^{-1} z (dense solves per block), Sec. 2.6.

    Blocks: one per leaf (group_max = 0), or groups of consecutive leaves in
    tree order holding at most group_max panels.  A block [phi_g; dphi_g]
    holds the operator entries of every pair of its panels whose leaves are
    neighbours (the pairs the near field stores); other pairs are far field
    and left out."""
    from .pairs import pair_integrals
    from .kernels import combine
    N = P.n
    leaf = tree.levels[tree.L]
    groups, cur, cnt = [], [], 0
    for c in range(leaf.n):
        nc = leaf.end[c] - leaf.start[c]
        if cur and (group_max == 0 or cnt + nc > group_max):
            groups.append(cur)
            cur, cnt = [], 0
        cur.append(c)
        cnt += nc
    groups.append(cur)
    blocks = []
    for g in groups:
        ids = tree.perm[leaf.start[g[0]]:leaf.end[g[-1]]]
        lf = np.concatenate([np.full(leaf.end[c] - leaf.start[c], c) for c in g])
        m = len(ids)
        ra, rb = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
        ra, rb = ra.ravel(), rb.ravel()
        near = np.array([lf[b] in set(leaf.nbr[lf[a]].tolist()) for a, b in zip(ra, rb)], bool)
        B = np.zeros((m * m, 4))
        if near.any():
            I, _ = pair_integrals(P, ids[ra[near]], ids[rb[near]], kappa, near_ratio, n)
            B[near] = combine(I, eps)
        B = B.reshape(m, m, 4)
        M = np.zeros((2 * m, 2 * m))
        M[:m, :m] = B[..., 0] + np.diag(0.5 * (1 + eps) * P.area[ids])
        M[:m, m:] = B[..., 1]
        M[m:, :m] = B[..., 2]
        M[m:, m:] = B[..., 3] + np.diag(0.5 * (1 + 1 / eps) * P.area[ids])
        blocks.append((ids, M))

    def apply(z):
        y = np.zeros_like(z)
        for ids, M in blocks:
            rhs_ = np.concatenate([z[ids], z[N + ids]])
            s = np.linalg.solve(M, rhs_)
            y[ids] = s[:len(ids)]
            y[N + ids] = s[len(ids):]
        return y

    return apply


def gmres(matvec, b, tol=1e-6, max_iter=200, precond=None):
    """Returns (x, iterations, residual-estimate history relative to ||b||)."""
    n = len(b)
    M = precond or (lambda v: v)
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n), 0, [0.0]
    V = np.zeros((max_iter + 1, n))
    Z = np.zeros((max_iter, n))
    H = np.zeros((max_iter + 1, max_iter))
    cs = np.zeros(max_iter)
    sn = np.zeros(max_iter)
    g = np.zeros(max_iter + 1)
    g[0] = beta
    V[0] = b / beta
    hist = [1.0]
    k = 0
    for k in range(max_iter):
        Z[k] = M(V[k])
        w = matvec(Z[k])
        for i in range(k + 1):
            H[i, k] = w @ V[i]
            w = w - H[i, k] * V[i]
        H[k + 1, k] = np.linalg.norm(w)
        if H[k + 1, k] > 0:
            V[k + 1] = w / H[k + 1, k]
        for i in range(k):
            t = cs[i] * H[i, k] + sn[i] * H[i + 1, k]
            H[i + 1, k] = -sn[i] * H[i, k] + cs[i] * H[i + 1, k]
            H[i, k] = t
        den = np.hypot(H[k, k], H[k + 1, k])
        cs[k] = H[k, k] / den
        sn[k] = H[k + 1, k] / den
        H[k, k] = den
        H[k + 1, k] = 0.0
        g[k + 1] = -sn[k] * g[k]
        g[k] = cs[k] * g[k]
        hist.append(abs(g[k + 1]) / beta)
        if hist[-1] <= tol:
            break
    m = k + 1
    y = np.linalg.solve(np.triu(H[:m, :m]), g[:m])
    x = Z[:m].T @ y
    return x, m, hist
