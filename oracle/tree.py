"""Cluster tree of panel centroids (Sec. 2.4, cluster tree and separation ratio).

Readings of points the paper leaves open (one choice, used everywhere):
  * level-0 cube: centred on the vertex bounding box, side = largest extent
    times (1 + 1e-12); corner = centre - side/2;
  * uniform depth: the leaf level L is the smallest l whose fullest cube holds
    at most ``leaf_size`` centroids; empty cubes are dropped;
  * a panel sits in cube floor((c - corner) / h_l) of level l (h_l = side/2^l),
    clamped to [0, 2^l - 1];
  * cluster centre x_c = the cube centre, and one radius per level,
    rho_l = max over level-l clusters of the farthest quadrature point of a
    member panel from the cube centre (so the separation ratio of two level-l
    clusters is 2 rho_l / |x_c - x_c'| and depends only on their index
    offset).  The far field is the FMM of the 3-point-rule interaction, whose
    sources and targets are exactly these points, so this radius bounds every
    point the expansions are evaluated at;
  * c' is a neighbour of c iff it is a child of a neighbour of c's parent and
    eta(c, c') > eta0 (c is its own neighbour); the interaction list I(c) holds
    the other children of the parent's neighbours.

Shrunk radii (``radii="cluster"``), after the shrink scheme of Sec. 2.4, which
replaces a cluster's cube by the tight box around its panels: here the
centre stays the cube centre (so that the offsets between clusters of a level
stay on the cube lattice and translations remain shared per offset) and each
cluster gets its own radius rho_c, the farthest vertex of a member panel from
that centre (the ball holds the cluster's panels whole, as the paper's box
does).  The separation ratio becomes (rho_c + rho_c') / |x_c - x_c'|; lists
are built by the same recursion.  Every quadrature point of c lies within
rho_c of x_c, so the expansions converge under the same condition
eta <= eta0 < 1; and two panels sharing a vertex v always land in
neighbouring clusters, since |x_c - x_c'| <= |x_c - v| + |v - x_c'| <=
rho_c + rho_c' gives eta >= 1.
"""
import numpy as np
from types import SimpleNamespace


def _spread3(v):
    """interleave: bit b of v goes to bit 3b"""
    v = v.astype(np.uint64)
    out = np.zeros_like(v)
    for b in range(21):
        out |= ((v >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def morton(idx):
    return (_spread3(idx[:, 0]) << np.uint64(2)) | (_spread3(idx[:, 1]) << np.uint64(1)) \
        | _spread3(idx[:, 2])


def cube_index(c, corner, side, level):
    h = side / float(2 ** level)
    k = np.floor((c - corner) / h)
    return np.clip(k, 0, 2 ** level - 1).astype(np.int64)


def build(P, leaf_size=32, eta0=0.8, max_level=20, radii="level"):
    V = P.verts[np.unique(P.tris)]
    lo, hi = V.min(0), V.max(0)
    center = 0.5 * (lo + hi)
    side = (hi - lo).max() * (1.0 + 1e-12)
    corner = center - 0.5 * side
    c = P.centroid
    L = None
    for lev in range(max_level + 1):
        key = morton(cube_index(c, corner, side, lev))
        _, cnt = np.unique(key, return_counts=True)
        if cnt.max() <= leaf_size:
            L = lev
            break
    if L is None:
        raise ValueError("leaf size not reached by level %d" % max_level)
    idxL = cube_index(c, corner, side, L)
    keyL = morton(idxL)
    perm = np.argsort(keyL, kind="stable")          # tree order -> panel id
    keyS = keyL[perm]
    idxS = idxL[perm]
    levels = []
    for lev in range(L + 1):
        k = keyS >> np.uint64(3 * (L - lev))
        start = np.concatenate([[0], np.nonzero(k[1:] != k[:-1])[0] + 1])
        end = np.concatenate([start[1:], [len(k)]])
        idx = idxS[start] >> (L - lev)
        h = side / float(2 ** lev)
        ctr = corner + (idx + 0.5) * h
        # radius: farthest quadrature point of a member panel from its cube
        # centre (the far field only ever evaluates the 3-point rule)
        memb = np.repeat(np.arange(len(start)), end - start)
        vv = P.qp[perm]                                   # [N,3,3]
        dist = np.linalg.norm(vv - ctr[memb][:, None, :], axis=2).max(1)
        dvert = np.linalg.norm(P.corners[perm] - ctr[memb][:, None, :], axis=2).max(1)
        rho_c = np.zeros(len(start))
        np.maximum.at(rho_c, memb, dvert)
        levels.append(SimpleNamespace(level=lev, start=start, end=end, idx=idx,
                                      h=h, center=ctr, rho=dist.max(), rho_c=rho_c,
                                      key=k[start], n=len(start)))
    # parents / children
    for lev in range(1, L + 1):
        ch, pa = levels[lev], levels[lev - 1]
        parent = np.searchsorted(pa.key, ch.key >> np.uint64(3))
        ch.parent = parent
        cstart = np.searchsorted(parent, np.arange(pa.n), side="left")
        cend = np.searchsorted(parent, np.arange(pa.n), side="right")
        pa.child_start, pa.child_end = cstart, cend
    levels[0].parent = np.array([-1])
    # neighbour and interaction lists
    levels[0].nbr = [np.array([0])]
    levels[0].inter = [np.array([], np.int64)]
    for lev in range(1, L + 1):
        cl, pa = levels[lev], levels[lev - 1]
        nbr, inter = [], []
        for ci in range(cl.n):
            p = cl.parent[ci]
            cand = np.concatenate([np.arange(pa.child_start[q], pa.child_end[q])
                                   for q in pa.nbr[p]])
            d = np.sqrt(((cl.center[ci] - cl.center[cand]) ** 2).sum(1))
            if radii == "cluster":
                num = cl.rho_c[ci] + cl.rho_c[cand]
            elif radii == "level":
                num = cl.rho + cl.rho
            else:
                raise ValueError("radii must be 'level' or 'cluster'")
            with np.errstate(divide="ignore"):
                eta = num / d
            isn = eta > eta0
            nbr.append(cand[isn])
            inter.append(cand[~isn])
        cl.nbr, cl.inter = nbr, inter
    lmin = next((l for l in range(L + 1)
                 if any(len(x) for x in levels[l].inter)), L + 1)
    return SimpleNamespace(L=L, levels=levels, perm=perm, corner=corner,
                           side=side, lmin=lmin, leaf_size=leaf_size, eta0=eta0,
                           radii=radii)


def orders(tree, p_leaf, adaptive, p_max):
    """Expansion order per level: p_l = min(p_L + L - l, p_max) when adaptive
    (Sec. 2.4, variable order), p_L at every level otherwise."""
    L = tree.L
    if adaptive:
        return [min(p_leaf + L - l, p_max) for l in range(L + 1)]
    return [p_leaf] * (L + 1)
