"""Cartesian Taylor FMM matrix-vector product for the Galerkin PB operator
(Sec. 2.4: moments, MtM, MtL, LtL, LtP and the six-step algorithm).

Readings (one choice, used everywhere):
  * order convention: |alpha| <= p_l for locals and |alpha| + |beta| <= p_l in
    MtL (the truncation written in the MtL formula; its (-1)^beta is read as
    (-1)^|beta|, which follows from G(x, y) = f(x - y));
  * LtL sums over alpha >= beta (componentwise), |alpha| <= p_l;
  * variable order: MtM builds a parent's moments up to p_l from its children's
    moments of order p_{l+1} (missing terms are zero); LtL truncates the
    shifted parent locals to the child order;
  * the interaction phase runs over c in C_l and c' in I(c) for
    l = l_min..L;
  * leaf moments of a panel use the same 3-point rule as the regular near field;
  * only two expansion channels are needed.  With phi, dphi the two unknown
    blocks and m_s / m_d the single / double layer moments,
        M0 = m_s(dphi) - m_d(phi)        (Coulomb kernel G0)
        Mk = -m_s(dphi) + eps m_d(phi)   (screened kernel Gk)
    row 1 of the far field is -(lambda0 + lambdak) tested with m_s, row 2 is
    -(lambda0 + lambdak/eps) tested with m_d (the kernels K1..K4 of Sec. 2.2).
"""
import numpy as np
from math import comb, factorial
from types import SimpleNamespace

from . import taylor
from .kernels import combine
from .pairs import pair_integrals

FOUR_PI = 4.0 * np.pi


def _mi(p):
    mi = taylor.multi_indices(p)
    return mi, {k: n for n, k in enumerate(mi)}


def panel_moments(P, ids, centers, p):
    """Single- and double-layer moments of the basis functions psi_i about the
    given centres with the 3-point rule:  m_s^b = sum_q w_q (y_q - x_c)^b,
    m_d^b = sum_q w_q n . grad (y - x_c)^b at y_q.  Returns [n, T], [n, T]."""
    mi, _ = _mi(p)
    d = P.qp[ids] - centers[:, None, :]              # [n,3,3] (q, dim)
    pw = np.ones((len(ids), 3, 3, p + 1))            # [n, q, dim, power]
    for e in range(1, p + 1):
        pw[..., e] = pw[..., e - 1] * d
    nrm = P.normal[ids]
    w = P.qw[ids]
    ms = np.zeros((len(ids), len(mi)))
    md = np.zeros((len(ids), len(mi)))
    for t, (a, b, c) in enumerate(mi):
        mono = pw[:, :, 0, a] * pw[:, :, 1, b] * pw[:, :, 2, c]
        ms[:, t] = (w * mono).sum(1)
        g = np.zeros_like(mono)
        if a:
            g += a * nrm[:, 0, None] * pw[:, :, 0, a - 1] * pw[:, :, 1, b] * pw[:, :, 2, c]
        if b:
            g += b * nrm[:, 1, None] * pw[:, :, 0, a] * pw[:, :, 1, b - 1] * pw[:, :, 2, c]
        if c:
            g += c * nrm[:, 2, None] * pw[:, :, 0, a] * pw[:, :, 1, b] * pw[:, :, 2, c - 1]
        md[:, t] = (w * g).sum(1)
    return ms, md


def shift_matrix(dvec, p_big, p_small):
    """S[alpha, beta] = C(alpha, beta) d^(alpha - beta) for beta <= alpha,
    |alpha| <= p_big, |beta| <= p_small.  MtM: M_parent = S M_child;
    LtL: lambda_child = S^T lambda_parent (multivariate binomial formula)."""
    ma, _ = _mi(p_big)
    mb, _ = _mi(p_small)
    S = np.zeros((len(ma), len(mb)))
    for i, al in enumerate(ma):
        for j, be in enumerate(mb):
            if all(be[k] <= al[k] for k in range(3)):
                v = 1.0
                for k in range(3):
                    v *= comb(al[k], be[k]) * dvec[k] ** (al[k] - be[k])
                S[i, j] = v
    return S


def m2l_matrices(x0s, kappa, p):
    """m2l_matrix for several offsets at once: x0s [m, 3] -> [m, T, T].  Every
    entry is the same expression as in m2l_matrix, evaluated elementwise."""
    mi, pos = _mi(p)
    x0s = np.atleast_2d(np.asarray(x0s, np.float64))
    F = taylor.coefficients(x0s, kappa, p)
    T = np.zeros((len(x0s), len(mi), len(mi)))
    for i, al in enumerate(mi):
        for j, be in enumerate(mi):
            if sum(al) + sum(be) <= p:
                g = (al[0] + be[0], al[1] + be[1], al[2] + be[2])
                c = taylor.mfact(g) / (taylor.mfact(al) * taylor.mfact(be)) * (-1.0) ** sum(be)
                T[:, i, j] = c * F[g] / FOUR_PI
    return T


def m2l_matrix(x0, kappa, p):
    """T[alpha, beta] = (alpha+beta)!/(alpha! beta!) (-1)^|beta| F_{alpha+beta}(x0)/(4 pi)
    for |alpha| + |beta| <= p (the MtL translation, x0 = x_c - x_c')."""
    return m2l_matrices(np.asarray(x0)[None, :], kappa, p)[0]


def setup(P, tree, eps, kappa, p_leaf=4, adaptive=False, p_max=8,
          near_ratio=2.0, n_duffy=7, with_near=True):
    """Precompute panel moments and the near-field blocks (per leaf c and each
    c' in N(c), the combined 4-entry blocks of every panel pair)."""
    from .tree import orders
    L = tree.L
    pl = orders(tree, p_leaf, adaptive, p_max)
    leaf = tree.levels[L]
    perm = tree.perm
    owner = np.repeat(np.arange(leaf.n), leaf.end - leaf.start)   # tree order
    ms, md = panel_moments(P, perm, leaf.center[owner], pl[L])
    F = SimpleNamespace(P=P, tree=tree, eps=eps, kappa=kappa, orders=pl,
                        ms=ms, md=md, owner=owner)
    if with_near:
        ii, jj = [], []
        for c in range(leaf.n):
            tgt = perm[leaf.start[c]:leaf.end[c]]
            for c2 in leaf.nbr[c]:
                src = perm[leaf.start[c2]:leaf.end[c2]]
                a, b = np.meshgrid(tgt, src, indexing="ij")
                ii.append(a.ravel())
                jj.append(b.ravel())
        ii = np.concatenate(ii)
        jj = np.concatenate(jj)
        I, cls = pair_integrals(P, ii, jj, kappa, near_ratio, n_duffy)
        F.near_i, F.near_j, F.near_B, F.near_cls = ii, jj, combine(I, eps), cls
    return F


def matvec(F, x, far=True, near=True):
    """y = A x, x = [phi (N); dphi (N)] in panel order."""
    P, tree, eps, kappa = F.P, F.tree, F.eps, F.kappa
    N = P.n
    phi, dphi = x[:N], x[N:]
    y1 = 0.5 * (1.0 + eps) * P.area * phi
    y2 = 0.5 * (1.0 + 1.0 / eps) * P.area * dphi
    if near:
        B = F.near_B
        y1 = y1 + np.bincount(F.near_i, B[:, 0] * phi[F.near_j] + B[:, 1] * dphi[F.near_j],
                              minlength=N)
        y2 = y2 + np.bincount(F.near_i, B[:, 2] * phi[F.near_j] + B[:, 3] * dphi[F.near_j],
                              minlength=N)
    if far and tree.lmin <= tree.L:
        f1, f2 = far_field(F, phi, dphi)
        y1 = y1 + f1
        y2 = y2 + f2
    return np.concatenate([y1, y2])


def upward(F, phi, dphi):
    """Steps 2 and 3: leaf moments of the two channels and the MtM upward pass.
    Returns dicts level -> [n_l, T(p_l)] of M0 and Mk for l = l_min..L."""
    tree, eps = F.tree, F.eps
    L, perm = tree.L, tree.perm
    # step 2: leaf moments (two channels)
    a = phi[perm]
    b = dphi[perm]
    c0 = F.ms * b[:, None] - F.md * a[:, None]
    ck = -F.ms * b[:, None] + eps * F.md * a[:, None]
    leaf = tree.levels[L]
    M0L = np.zeros((leaf.n, F.ms.shape[1]))
    MkL = np.zeros((leaf.n, F.ms.shape[1]))
    np.add.at(M0L, F.owner, c0)
    np.add.at(MkL, F.owner, ck)
    return upward_pass(F, M0L, MkL)


def upward_pass(F, M0L, MkL):
    """Step 3 from the leaf moments M0L, MkL [n_L, T(p_L)]: dicts level ->
    moments for l = l_min..L."""
    tree, pl = F.tree, F.orders
    L = tree.L
    levels = tree.levels
    M0 = {L: M0L}
    Mk = {L: MkL}
    for l in range(L - 1, tree.lmin - 1, -1):
        ch, pa = levels[l + 1], levels[l]
        T = len(_mi(pl[l])[0])
        M0[l] = np.zeros((pa.n, T))
        Mk[l] = np.zeros((pa.n, T))
        octant = ch.idx & 1
        for o in np.unique(octant[:, 0] * 4 + octant[:, 1] * 2 + octant[:, 2]):
            sel = np.nonzero(octant[:, 0] * 4 + octant[:, 1] * 2 + octant[:, 2] == o)[0]
            dvec = (np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1]) - 0.5) * ch.h
            S = shift_matrix(dvec, pl[l], pl[l + 1])
            np.add.at(M0[l], ch.parent[sel], M0[l + 1][sel] @ S.T)
            np.add.at(Mk[l], ch.parent[sel], Mk[l + 1][sel] @ S.T)
    return M0, Mk


def downward(F, lam, l_from):
    """Step 5 for one channel: lam[l + 1] += LtL(lam[l]) for l = l_from..L-1
    (dict level -> [n_l, T(p_l)], updated in place)."""
    tree, pl = F.tree, F.orders
    levels = tree.levels
    for l in range(l_from, tree.L):
        ch = levels[l + 1]
        octant = ch.idx & 1
        for o in np.unique(octant[:, 0] * 4 + octant[:, 1] * 2 + octant[:, 2]):
            sel = np.nonzero(octant[:, 0] * 4 + octant[:, 1] * 2 + octant[:, 2] == o)[0]
            dvec = (np.array([(o >> 2) & 1, (o >> 1) & 1, o & 1]) - 0.5) * ch.h
            S = shift_matrix(dvec, pl[l], pl[l + 1])
            lam[l + 1][sel] += lam[l][ch.parent[sel]] @ S


def interaction(F, M0, Mk, l, targets=None):
    """Step 4 on level l: the locals lambda_c = sum_{c' in I(c)} T(x_c - x_c') M_c'
    of both channels, one MtL matrix per offset, for every cluster of the
    level (or only the given targets, whose rows are the only non-zero ones).
    Returns [n_l, T(p_l)] arrays lam0, lamk."""
    tree, kappa, pl = F.tree, F.kappa, F.orders
    cl = tree.levels[l]
    T = len(_mi(pl[l])[0])
    lam0 = np.zeros((cl.n, T))
    lamk = np.zeros((cl.n, T))
    cs = np.arange(cl.n) if targets is None else np.asarray(targets, np.int64)
    tgt = np.concatenate([np.full(len(cl.inter[c]), c) for c in cs] + [np.zeros(0)]).astype(np.int64)
    src = np.concatenate([cl.inter[c] for c in cs] + [np.zeros(0)]).astype(np.int64)
    if len(tgt) == 0:
        return lam0, lamk
    off = cl.idx[tgt] - cl.idx[src]              # x_c - x_c' = off * h
    uo, inv = np.unique(off, axis=0, return_inverse=True)
    inv = inv.ravel()
    T0s = m2l_matrices(uo * cl.h, 0.0, pl[l])
    Tks = m2l_matrices(uo * cl.h, kappa, pl[l])
    for k in range(len(uo)):
        sel = np.nonzero(inv == k)[0]
        np.add.at(lam0, tgt[sel], M0[l][src[sel]] @ T0s[k].T)
        np.add.at(lamk, tgt[sel], Mk[l][src[sel]] @ Tks[k].T)
    return lam0, lamk


def far_field(F, phi, dphi):
    M0, Mk = upward(F, phi, dphi)
    # steps 4 and 5, then step 6: evaluation
    return evaluate(F, *leaf_locals(F, M0, Mk))


def leaf_locals(F, M0, Mk):
    """Steps 4 and 5: the interaction phase on every level and the downward
    pass; returns the leaf locals (lam0, lamk) [n_L, T(p_L)]."""
    tree = F.tree
    L = tree.L
    lam0, lamk = {}, {}
    for l in range(tree.lmin, L + 1):
        lam0[l], lamk[l] = interaction(F, M0, Mk, l)
    downward(F, lam0, tree.lmin)
    downward(F, lamk, tree.lmin)
    return lam0[L], lamk[L]


def evaluate(F, lam0_leaf, lamk_leaf):
    """Step 6: the far field at every panel from the leaf locals, row 1
    -(lambda0 + lambdak) tested with m_s, row 2 -(lambda0 + lambdak/eps)
    tested with m_d.  Returns (y1, y2) in panel order."""
    l0 = lam0_leaf[F.owner]
    lk = lamk_leaf[F.owner]
    f1 = -((l0 + lk) * F.ms).sum(1)
    f2 = -((l0 + lk / F.eps) * F.md).sum(1)
    y1 = np.zeros(F.P.n)
    y2 = np.zeros(F.P.n)
    y1[F.tree.perm] = f1
    y2[F.tree.perm] = f2
    return y1, y2


def coverage(tree):
    """Count, for every ordered leaf pair, how many times the near field or a
    far-field translation (at any level) accounts for it.  Returns [nleaf,
    nleaf] counts (each must be exactly one)."""
    L = tree.L
    leaf = tree.levels[L]
    C = np.zeros((leaf.n, leaf.n), np.int64)
    # descendants at leaf level of each cluster per level
    desc = {L: [np.array([c]) for c in range(leaf.n)]}
    for l in range(L - 1, -1, -1):
        pa = tree.levels[l]
        desc[l] = [np.concatenate([desc[l + 1][k] for k in
                                   range(pa.child_start[c], pa.child_end[c])])
                   for c in range(pa.n)]
    for c in range(leaf.n):
        C[c, leaf.nbr[c]] += 1
    for l in range(L + 1):
        cl = tree.levels[l]
        for c in range(cl.n):
            for c2 in cl.inter[c]:
                C[np.ix_(desc[l][c], desc[l][c2])] += 1
    return C


def far_field_rows(F, phi, dphi, leaves):
    """The far field of far_field() at the panels of the given leaves only:
    the full upward pass (steps 2, 3), then the interaction phase (step 4) for
    the ancestors of these leaves alone, the downward pass (step 5) along their
    ancestor chains and the evaluation (step 6) at their panels.  Every
    computed local is the same sum as in far_field (one matrix per offset),
    taken for fewer targets.  Returns (panel ids [m], f1 [m], f2 [m])."""
    tree, eps = F.tree, F.eps
    L, perm = tree.L, tree.perm
    M0, Mk = upward(F, phi, dphi)
    anc, lam0, lamk = leaf_locals_at(F, M0, Mk, leaves)
    leaf = tree.levels[L]
    ids, f1, f2 = [], [], []
    for k, c in enumerate(anc):
        tpos = np.arange(leaf.start[c], leaf.end[c])
        ids.append(perm[tpos])
        f1.append(-((lam0[k] + lamk[k]) * F.ms[tpos]).sum(1))
        f2.append(-((lam0[k] + lamk[k] / eps) * F.md[tpos]).sum(1))
    return np.concatenate(ids), np.concatenate(f1), np.concatenate(f2)


def leaf_locals_at(F, M0, Mk, leaves):
    """Steps 4 and 5 for the given leaves only (from the moments of every
    level): the interaction phase at the ancestors of these leaves and the
    downward pass along their chains.  Returns (leaves, sorted unique [m],
    lam0 [m, T(p_L)], lamk [m, T(p_L)])."""
    tree, kappa, pl = F.tree, F.kappa, F.orders
    L = tree.L
    levels = tree.levels
    anc = {L: np.unique(np.asarray(leaves, np.int64))}
    for l in range(L - 1, tree.lmin - 1, -1):
        anc[l] = np.unique(levels[l + 1].parent[anc[l + 1]])
    lam0, lamk = {}, {}
    for l in range(tree.lmin, L + 1):
        cl = levels[l]
        T = len(_mi(pl[l])[0])
        lam0[l] = np.zeros((len(anc[l]), T))
        lamk[l] = np.zeros((len(anc[l]), T))
        for k, c in enumerate(anc[l]):
            src = np.asarray(cl.inter[c], np.int64)
            if len(src) == 0:
                continue
            x0 = (cl.idx[c][None, :] - cl.idx[src]) * cl.h
            T0s = m2l_matrices(x0, 0.0, pl[l])
            Tks = m2l_matrices(x0, kappa, pl[l])
            lam0[l][k] = np.einsum("sab,sb->a", T0s, M0[l][src])
            lamk[l][k] = np.einsum("sab,sb->a", Tks, Mk[l][src])
    for l in range(tree.lmin, L):
        ch = levels[l + 1]
        where = {c: k for k, c in enumerate(anc[l])}
        for k, c in enumerate(anc[l + 1]):
            o = ch.idx[c] & 1
            dvec = (o - 0.5) * ch.h
            S = shift_matrix(dvec, pl[l], pl[l + 1])
            p = where[ch.parent[c]]
            lam0[l + 1][k] += lam0[l][p] @ S
            lamk[l + 1][k] += lamk[l][p] @ S
    if tree.lmin > L:
        T = len(_mi(pl[L])[0])
        return anc[L], np.zeros((len(anc[L]), T)), np.zeros((len(anc[L]), T))
    return anc[L], lam0[L], lamk[L]
