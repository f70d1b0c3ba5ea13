"""Continuous piecewise-linear Galerkin discretisation S^1_h (Sec. 2.3, the
space of continuous functions that are linear on every flat panel, spanned by
the vertex hat functions; projection error O(h^2) against O(h) for the box
functions of the piecewise-constant space).

TEST INFRASTRUCTURE ONLY (see the package docstring).

Unknowns: the nodal values of phi and dphi at the V mesh vertices,
x = [phi_1..phi_V, dphi_1..dphi_V].  On a panel tau with corners (c0, c1, c2)
in its own order, the hat function of the vertex at corner a restricts to the
barycentric coordinate lambda_a.  The system is the box-function system of
``dense`` with hat functions as test and trial functions:
  A11 = (1+eps)/2 M - (eps I3 - I2),  A12 = -I1,
  A21 = -I6,                          A22 = (1+1/eps)/2 M - (I4 - I5/eps),
  I_m[i, j] = int int phi_i(x) k_m(x, y) phi_j(y) dy dx
            = sum over panels tau at vertex i (corner a), sigma at vertex j
              (corner b) of the corner integrals
              J_m[tau, sigma, a, b] = int_tau int_sigma lambda_a(x) k_m(x, y) lambda_b(y),
  M_ij = int phi_i phi_j  (per panel A (1 + delta_ab) / 12).

Corner integrals, by the rules of ``pairs`` with the basis products inside:
  REGULAR, CLOSE, VERTEX: each quadrature point of the rule carries the
      barycentric coordinates of its two points; their products multiply the
      kernel.  The 3-point rule's point k has lambda = 2/3 at corner k and 1/6
      at the others.
  IDENT: the rule runs over z = y - x; for fixed z the x-integral over the
      shrunken triangle T(z) = {x : x and x + z in the reference triangle} is
      the integral of lambda_a(x) lambda_b(x + z), a quadratic in x, taken by
      the 3-point rule on T(z) (exact).  With a = max(0, -z2),
      b = max(0, z2 - z1), c = max(0, z1), T(z) has the corners (a + b, a),
      (1 - c, a), (1 - c, 1 - c - b) and area (1 - sigma)^2 / 2.
  EDGE: the rule runs over (z1 = y1 - x1, x2, y2); the x1-integral over
      [max(x2, y2 - z1), 1 - max(0, z1)] (length 1 - sigma) of the product,
      a quadratic in x1, is taken by 2-point Gauss-Legendre (exact).
Reference coordinates: chi(x) = u + x1 (v - u) + x2 (w - v) on
{0 <= x2 <= x1 <= 1}, so lambda_u = 1 - x1, lambda_v = x1 - x2, lambda_w = x2.
Since the hat functions of a panel sum to one, sum_ab J[a, b] is the
box-function integral of ``pairs`` with the same rule (pinned).
"""
import numpy as np

from . import fmm
from .kernels import FOUR_PI, combine, kernel6
from .pairs import (CLOSE, EDGE, IDENT, REGULAR, VERTEX, _HEX, classify, gauss01)
from .solve import UNIT_KCAL

# LAM[k, a]: barycentric coordinate of corner a at point k of the 3-point rule
LAM = np.full((3, 3), 1.0 / 6.0) + np.eye(3) * 0.5


def _bary(x1, x2):
    """barycentric coordinates (lambda_u, lambda_v, lambda_w) of reference
    coordinates (x1, x2): [..., 3]"""
    return np.stack([1.0 - x1, x1 - x2, x2], axis=-1)


def _accumulate(r, w, lx, ly, nx, ny, kappa, kern):
    """sum_k w[p,k] lx[p,k,a] ly[p,k,b] kern(r[p,k])[m] -> [p, 3, 3, m]"""
    K = (kern or kernel6)(r, nx[:, None, :], ny[:, None, :], kappa)     # [p,k,m]
    wk = w[:, :, None] * K
    out = np.empty((r.shape[0], 3, 3, K.shape[-1]))
    for a in range(3):
        out[:, a] = np.einsum("pkb,pkm->pbm", ly, lx[:, :, a, None] * wk)
    return out


def _scatter_corners(vals, order_i, order_j):
    """vals [p, 3, 3, m] in the rule's corner order -> the triangles' own
    corner order: row order_i[p, a] is the triangle corner of rule corner a"""
    out = np.empty_like(vals)
    r = np.arange(vals.shape[0])
    for a in range(3):
        for b in range(3):
            out[r, order_i[:, a], order_j[:, b]] = vals[:, a, b]
    return out


def regular(P, i, j, kappa, kern=None):
    r = P.qp[i][:, :, None, :] - P.qp[j][:, None, :, :]          # [p, kx, ky, 3]
    w = P.qw[i][:, :, None] * P.qw[j][:, None, :]
    p = len(i)
    lx = np.broadcast_to(LAM[:, None, :], (3, 3, 3)).reshape(9, 3)   # point (kx, ky) -> lambda(x_kx)
    ly = np.broadcast_to(LAM[None, :, :], (3, 3, 3)).reshape(9, 3)
    return _accumulate(r.reshape(p, 9, 3), w.reshape(p, 9), np.broadcast_to(lx, (p, 9, 3)),
                       np.broadcast_to(ly, (p, 9, 3)), P.normal[i], P.normal[j], kappa, kern)


def _duffy(corners, n):
    """Duffy-collapsed n x n rule: points [p, n*n, 3], weights, barycentrics"""
    g, gw = gauss01(n)
    s = np.repeat(g, n)
    t = np.tile(g, n)
    w = np.repeat(gw, n) * np.tile(gw, n) * s
    u, v, ww = corners[:, 0], corners[:, 1], corners[:, 2]
    pts = (u[:, None, :] + s[None, :, None] * (v - u)[:, None, :]
           + (s * t)[None, :, None] * (ww - v)[:, None, :])
    two_a = np.linalg.norm(np.cross(v - u, ww - u), axis=1)
    return pts, two_a[:, None] * w[None, :], _bary(s, s * t)


def close(P, i, j, kappa, n, kern=None):
    xi, wx, bx = _duffy(P.corners[i], n)
    yj, wy, by = _duffy(P.corners[j], n)
    m = n * n
    p = len(i)
    r = (xi[:, :, None, :] - yj[:, None, :, :]).reshape(p, m * m, 3)
    w = (wx[:, :, None] * wy[:, None, :]).reshape(p, m * m)
    lx = np.broadcast_to(bx[:, None, :], (m, m, 3)).reshape(m * m, 3)
    ly = np.broadcast_to(by[None, :, :], (m, m, 3)).reshape(m * m, 3)
    return _accumulate(r, w, np.broadcast_to(lx, (p, m * m, 3)), np.broadcast_to(ly, (p, m * m, 3)),
                       P.normal[i], P.normal[j], kappa, kern)


def _ident_samples(n):
    """z-samples of the identical-pair rule and, per sample, the 3-point rule on
    T(z): z [K, 2], weights [K] (with the area of T(z)), Q [K, 3, 3] with
    Q[a, b] = mean over the rule's points x of lambda_a(x) lambda_b(x + z)"""
    g, gw = gauss01(n)
    xi = np.repeat(g, n)
    t = np.tile(g, n)
    wq = np.repeat(gw, n) * np.tile(gw, n) * 0.5 * (1.0 - xi) ** 2 * xi
    zs = []
    for Pq, Qq in _HEX:
        Pq = np.array(Pq, float)
        Qq = np.array(Qq, float)
        zs.append(xi[:, None] * ((1.0 - t)[:, None] * Pq + t[:, None] * Qq))
    z = np.concatenate(zs)
    w = np.tile(wq, 6)
    a = np.maximum(0.0, -z[:, 1])
    b = np.maximum(0.0, z[:, 1] - z[:, 0])
    c = np.maximum(0.0, z[:, 0])
    V = np.stack([np.stack([a + b, a], -1), np.stack([1 - c, a], -1), np.stack([1 - c, 1 - c - b], -1)], 1)
    Q = np.zeros((len(z), 3, 3))
    for k in range(3):
        x = (2.0 / 3.0) * V[:, k] + (1.0 / 6.0) * (V[:, (k + 1) % 3] + V[:, (k + 2) % 3])
        lx = _bary(x[:, 0], x[:, 1])
        ly = _bary(x[:, 0] + z[:, 0], x[:, 1] + z[:, 1])
        Q += lx[:, :, None] * ly[:, None, :] / 3.0
    return z, w, Q


def ident(P, i, kappa, n, kern=None):
    z, w, Q = _ident_samples(n)
    c = P.corners[i]
    e1 = c[:, 1] - c[:, 0]
    e2 = c[:, 2] - c[:, 1]
    r = -(z[None, :, 0, None] * e1[:, None, :] + z[None, :, 1, None] * e2[:, None, :])
    K = (kern or kernel6)(r, P.normal[i][:, None, :], P.normal[i][:, None, :], kappa)   # [p,K,m]
    scale = 4.0 * P.area[i] ** 2
    out = np.einsum("k,kab,pkm->pabm", w, Q, K) * scale[:, None, None, None]
    if kern is None:
        out[..., 1:5] = 0.0          # r.n = 0 on a flat panel
    return out


def _edge_order(P, i, j):
    """Per pair the triangle corners of P, Q (the shared edge, in the order
    they appear in triangle i) and R_i, and of P, Q, R_j in triangle j."""
    ti, tj = P.tris[i], P.tris[j]
    in_j = (ti[:, :, None] == tj[:, None, :]).any(2)
    oi = np.argsort(~in_j, axis=1, kind="stable")       # shared first (order of i), then R_i
    r = np.arange(len(i))
    Pv = ti[r, oi[:, 0]]
    Qv = ti[r, oi[:, 1]]
    pj = np.argmax(tj == Pv[:, None], axis=1)
    qj = np.argmax(tj == Qv[:, None], axis=1)
    rj = 3 - pj - qj
    return oi, np.stack([pj, qj, rj], 1)


def _edge_samples(n):
    """(z1, x2, y2) samples of the edge rule with their weights (including the
    x1-length 1 - sigma), and per sample Q[a, b] = mean over the 2-point rule
    in x1 of lambda_a(x) lambda_b(y) in the corner order (P, Q, R)"""
    g, gw = gauss01(n)
    XI, W1, W2 = np.meshgrid(g, g, g, indexing="ij")
    WXI, WW1, WW2 = np.meshgrid(gw, gw, gw, indexing="ij")
    XI, W1, W2 = XI.ravel(), W1.ravel(), W2.ravel()
    wbase = (WXI * WW1 * WW2).ravel() * (1.0 - XI) * XI ** 2
    pieces = [(XI * W1, XI * (1 - W1), XI * W2, wbase),
              (XI * W1 * (1 - W2), XI * W1 * W2, XI, wbase * W1),
              (-XI * W1 * (1 - W2), XI, XI * W1 * W2, wbase * W1),
              (-XI * W1, XI * W2, XI * (1 - W1), wbase)]
    z1 = np.concatenate([p[0] for p in pieces])
    x2 = np.concatenate([p[1] for p in pieces])
    y2 = np.concatenate([p[2] for p in pieces])
    w = np.concatenate([p[3] for p in pieces])
    lo = np.maximum(x2, y2 - z1)
    hi = 1.0 - np.maximum(0.0, z1)
    g2, gw2 = gauss01(2)
    Q = np.zeros((len(z1), 3, 3))
    for k in range(2):
        x1 = lo + (hi - lo) * g2[k]
        lx = _bary(x1, x2)
        ly = _bary(x1 + z1, y2)
        Q += gw2[k] * lx[:, :, None] * ly[:, None, :]
    return z1, x2, y2, w, Q


def edge(P, i, j, kappa, n, kern=None):
    oi, oj = _edge_order(P, i, j)
    r_ = np.arange(len(i))
    V = P.verts
    Pv = V[P.tris[i][r_, oi[:, 0]]]
    Qv = V[P.tris[i][r_, oi[:, 1]]]
    Ri = V[P.tris[i][r_, oi[:, 2]]]
    Rj = V[P.tris[j][r_, oj[:, 2]]]
    e = Qv - Pv
    a = Ri - Qv
    b = Rj - Qv
    z1, x2, y2, w, Q = _edge_samples(n)
    r = (-z1[None, :, None] * e[:, None, :] + x2[None, :, None] * a[:, None, :]
         - y2[None, :, None] * b[:, None, :])
    K = (kern or kernel6)(r, P.normal[i][:, None, :], P.normal[j][:, None, :], kappa)
    scale = 4.0 * P.area[i] * P.area[j]
    out = np.einsum("k,kab,pkm->pabm", w, Q, K) * scale[:, None, None, None]
    return _scatter_corners(out, oi, oj)


def _vertex_order(P, i, j):
    """triangle corners of (S, V, W) in each triangle: S the shared vertex, V
    and W the others in their order of appearance"""
    ti, tj = P.tris[i], P.tris[j]
    in_j = (ti[:, :, None] == tj[:, None, :]).any(2)
    in_i = (tj[:, :, None] == ti[:, None, :]).any(2)
    oi = np.argsort(~in_j, axis=1, kind="stable")
    oj = np.argsort(~in_i, axis=1, kind="stable")
    return oi, oj


def vertex(P, i, j, kappa, n, kern=None):
    oi, oj = _vertex_order(P, i, j)
    r_ = np.arange(len(i))
    V = P.verts
    S = V[P.tris[i][r_, oi[:, 0]]]
    Vi, Wi = V[P.tris[i][r_, oi[:, 1]]], V[P.tris[i][r_, oi[:, 2]]]
    Vj, Wj = V[P.tris[j][r_, oj[:, 1]]], V[P.tris[j][r_, oj[:, 2]]]
    g, gw = gauss01(n)
    XI, ETA, T1, T2 = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.ones_like(XI)
    for wv in np.meshgrid(gw, gw, gw, gw, indexing="ij"):
        W = W * wv
    XI, ETA, T1, T2, W = (q.ravel() for q in (XI, ETA, T1, T2, W))
    W = W * XI ** 3 * ETA
    al = (Vi - S)[:, None, :] + T1[None, :, None] * (Wi - Vi)[:, None, :]
    be = (Vj - S)[:, None, :] + T2[None, :, None] * (Wj - Vj)[:, None, :]
    # half 1: x1 = xi, y1 = xi eta; half 2: x1 = xi eta, y1 = xi
    r = np.concatenate([XI[None, :, None] * al - (XI * ETA)[None, :, None] * be,
                        (XI * ETA)[None, :, None] * al - XI[None, :, None] * be], axis=1)
    x1 = np.concatenate([XI, XI * ETA])
    y1 = np.concatenate([XI * ETA, XI])
    t1 = np.concatenate([T1, T1])
    t2 = np.concatenate([T2, T2])
    w = np.concatenate([W, W])
    lx = _bary(x1, x1 * t1)          # (S, V, W) of triangle i
    ly = _bary(y1, y1 * t2)
    p = len(i)
    K = (kern or kernel6)(r, P.normal[i][:, None, :], P.normal[j][:, None, :], kappa)
    scale = 4.0 * P.area[i] * P.area[j]
    out = np.einsum("k,ka,kb,pkm->pabm", w, lx, ly, K) * scale[:, None, None, None]
    assert out.shape[0] == p
    return _scatter_corners(out, oi, oj)


def pair_integrals(P, i, j, kappa, near_ratio=2.0, n=7, cls=None, kern=None):
    """Corner integrals J[p, a, b, m] of the ordered pairs (i[p], j[p]) (a the
    corner of panel i, b of panel j, each in its triangle's order) and the
    pair classes.  Touching and close pairs are integrated for the member with
    the lower panel index and mirrored (J_ji[b, a] = J_ij[a, b] with I2 <-> I4,
    I3 <-> I5), as in ``pairs``."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    if cls is None:
        cls = classify(P, i, j, near_ratio)
    m = 6 if kern is None else kern(np.ones((1, 3)), np.ones((1, 3)), np.ones((1, 3)), 0.0).shape[-1]
    out = np.zeros((len(i), 3, 3, m))
    rules = {REGULAR: (lambda a, b: regular(P, a, b, kappa, kern), 16384),
             IDENT: (lambda a, b: ident(P, a, kappa, n, kern), 1024),
             EDGE: (lambda a, b: edge(P, a, b, kappa, n, kern), 256),
             VERTEX: (lambda a, b: vertex(P, a, b, kappa, n, kern), 32),
             CLOSE: (lambda a, b: close(P, a, b, kappa, n, kern), 32)}
    mirror = (cls >= EDGE) & (i > j)
    a = np.where(mirror, j, i)
    b = np.where(mirror, i, j)
    for c, (fn, ch) in rules.items():
        sel = np.nonzero(cls == c)[0]
        for s in range(0, len(sel), ch):
            k = sel[s:s + ch]
            out[k] = fn(a[k], b[k])
    if mirror.any():
        swap = [0, 3, 4, 1, 2, 5] if m == 6 else list(range(m))
        out[mirror] = out[mirror].transpose(0, 2, 1, 3)[..., swap]
    return out, cls


def mass_diag_blocks(P):
    """per panel the 3 x 3 mass matrix int lambda_a lambda_b = A (1 + delta_ab) / 12"""
    return P.area[:, None, None] * (np.ones((3, 3)) + np.eye(3))[None] / 12.0


def _add_blocks(A, rows, cols, B, eps, V):
    """add the four operator blocks B [p, 3, 3, 4] at vertex rows [p, 3] and
    columns [p, 3] of the 2V x 2V matrix A"""
    R = np.broadcast_to(rows[:, :, None], B.shape[:3])
    C = np.broadcast_to(cols[:, None, :], B.shape[:3])
    np.add.at(A, (R, C), B[..., 0])
    np.add.at(A, (R, V + C), B[..., 1])
    np.add.at(A, (V + R, C), B[..., 2])
    np.add.at(A, (V + R, V + C), B[..., 3])


def assemble(P, eps, kappa, near_ratio=2.0, n=7, rows_chunk=64):
    """dense 2V x 2V hat-function system"""
    N = P.n
    V = len(P.verts)
    A = np.zeros((2 * V, 2 * V))
    for r0 in range(0, N, rows_chunk):
        rows = np.arange(r0, min(N, r0 + rows_chunk))
        ii = np.repeat(rows, N)
        jj = np.tile(np.arange(N), len(rows))
        J, _ = pair_integrals(P, ii, jj, kappa, near_ratio, n)
        _add_blocks(A, P.tris[ii], P.tris[jj], combine(J, eps), eps, V)
    Mb = mass_diag_blocks(P)
    R = np.broadcast_to(P.tris[:, :, None], Mb.shape)
    C = np.broadcast_to(P.tris[:, None, :], Mb.shape)
    np.add.at(A, (R, C), 0.5 * (1.0 + eps) * Mb)
    np.add.at(A, (V + R, V + C), 0.5 * (1.0 + 1.0 / eps) * Mb)
    return A


def mass_matvec(P, u):
    """M u for the hat-function mass matrix (panel by panel)"""
    V = len(P.verts)
    y = np.zeros(V)
    Mb = mass_diag_blocks(P)
    np.add.at(y, P.tris, np.einsum("pab,pb->pa", Mb, u[P.tris]))
    return y


# ---------------------------------------------------------------------------
# FMM (Sec. 2.4) with hat functions: the far field is the box-function far
# field with one moment set per panel corner, m_s[tau, a]^b = sum_q w_q
# lambda_a(y_q) (y_q - x_c)^b (m_d likewise), source strengths taken from the
# corner's vertex values and the tested results summed into the vertices.
# ---------------------------------------------------------------------------
def _weighted(P, a):
    from types import SimpleNamespace
    return SimpleNamespace(qp=P.qp, qw=P.qw * LAM[:, a][None, :], normal=P.normal)


def setup(P, tree, eps, kappa, p_leaf=4, adaptive=False, p_max=8, near_ratio=2.0, n_duffy=7, with_near=True):
    F = fmm.setup(P, tree, eps, kappa, p_leaf=p_leaf, adaptive=adaptive, p_max=p_max,
                  near_ratio=near_ratio, n_duffy=n_duffy, with_near=False)
    L = tree.L
    leaf = tree.levels[L]
    ms3, md3 = [], []
    for a in range(3):
        s_, d_ = fmm.panel_moments(_weighted(P, a), tree.perm, leaf.center[F.owner], F.orders[L])
        ms3.append(s_)
        md3.append(d_)
    F.ms3 = np.stack(ms3, 1)         # [N tree order, 3, T]
    F.md3 = np.stack(md3, 1)
    F.V = len(P.verts)
    if with_near:
        ii, jj = [], []
        for c in range(leaf.n):
            tgt = tree.perm[leaf.start[c]:leaf.end[c]]
            for c2 in leaf.nbr[c]:
                src = tree.perm[leaf.start[c2]:leaf.end[c2]]
                x_, y_ = np.meshgrid(tgt, src, indexing="ij")
                ii.append(x_.ravel())
                jj.append(y_.ravel())
        ii = np.concatenate(ii)
        jj = np.concatenate(jj)
        J, cls = pair_integrals(P, ii, jj, kappa, near_ratio, n_duffy)
        F.near_i, F.near_j, F.near_B, F.near_cls = ii, jj, combine(J, eps), cls
    return F


def far_field(F, u, v):
    """far field of the hat-function operator at the vertices: (y1 [V], y2 [V])"""
    P, tree, eps = F.P, F.tree, F.eps
    L = tree.L
    tri = P.tris[tree.perm]                 # vertex of each corner, tree order
    a, b = u[tri], v[tri]                   # [N, 3]
    c0 = np.einsum("pat,pa->pt", F.ms3, b) - np.einsum("pat,pa->pt", F.md3, a)
    ck = -np.einsum("pat,pa->pt", F.ms3, b) + eps * np.einsum("pat,pa->pt", F.md3, a)
    leaf = tree.levels[L]
    M0L = np.zeros((leaf.n, F.ms3.shape[2]))
    MkL = np.zeros((leaf.n, F.ms3.shape[2]))
    np.add.at(M0L, F.owner, c0)
    np.add.at(MkL, F.owner, ck)
    M0, Mk = fmm.upward_pass(F, M0L, MkL)
    lam0, lamk = fmm.leaf_locals(F, M0, Mk)
    l0 = lam0[F.owner]
    lk = lamk[F.owner]
    f1 = -np.einsum("pt,pat->pa", l0 + lk, F.ms3)
    f2 = -np.einsum("pt,pat->pa", l0 + lk / eps, F.md3)
    y1 = np.zeros(F.V)
    y2 = np.zeros(F.V)
    np.add.at(y1, tri, f1)
    np.add.at(y2, tri, f2)
    return y1, y2


def _leaf_of_panels(F):
    """leaf of every panel (caller order)"""
    owner = np.empty(F.P.n, np.int64)
    owner[F.tree.perm] = F.owner
    return owner


def panels_at(P, verts):
    """the panels having a corner at one of the given vertices"""
    return np.nonzero(np.isin(P.tris, np.asarray(verts)).any(1))[0]


def near_rows(F, u, v, verts, near_ratio=2.0, n=7):
    """the near part of A x (identity terms included) at the given vertices:
    the stored pairs of the panels at those vertices (sources: every panel of
    the neighbour leaves of their leaf), integrated pair by pair.  Returns
    (y1 [m], y2 [m]) in the order of verts."""
    P, tree, eps = F.P, F.tree, F.eps
    leaf = tree.levels[tree.L]
    owner = _leaf_of_panels(F)
    verts = np.asarray(verts)
    y1 = np.zeros(len(verts))
    y2 = np.zeros(len(verts))
    Mb = mass_diag_blocks(P)
    for k, vx in enumerate(verts):
        for t_ in panels_at(P, [vx]):
            a = int(np.nonzero(P.tris[t_] == vx)[0][0])
            c = owner[t_]
            src = np.concatenate([tree.perm[leaf.start[c2]:leaf.end[c2]] for c2 in leaf.nbr[c]])
            J, _ = pair_integrals(P, np.full(len(src), t_), src, F.kappa, near_ratio, n)
            B = combine(J[:, a], eps)                  # [s, b, 4]
            ub, vb = u[P.tris[src]], v[P.tris[src]]    # [s, b]
            y1[k] += (B[..., 0] * ub).sum() + (B[..., 1] * vb).sum()
            y2[k] += (B[..., 2] * ub).sum() + (B[..., 3] * vb).sum()
            y1[k] += 0.5 * (1.0 + eps) * (Mb[t_, a] * u[P.tris[t_]]).sum()
            y2[k] += 0.5 * (1.0 + 1.0 / eps) * (Mb[t_, a] * v[P.tris[t_]]).sum()
    return y1, y2


def far_rows(F, u, v, verts):
    """the far field of A x at the given vertices: the full upward pass, the
    locals of the leaves holding the vertices' panels only, and the corner
    results of those panels summed into the vertices.  Returns (y1, y2)."""
    P, tree, eps = F.P, F.tree, F.eps
    L = tree.L
    tri = P.tris[tree.perm]
    a, b = u[tri], v[tri]
    c0 = np.einsum("pat,pa->pt", F.ms3, b) - np.einsum("pat,pa->pt", F.md3, a)
    ck = -np.einsum("pat,pa->pt", F.ms3, b) + eps * np.einsum("pat,pa->pt", F.md3, a)
    leaf = tree.levels[L]
    M0L = np.zeros((leaf.n, F.ms3.shape[2]))
    MkL = np.zeros((leaf.n, F.ms3.shape[2]))
    np.add.at(M0L, F.owner, c0)
    np.add.at(MkL, F.owner, ck)
    M0, Mk = fmm.upward_pass(F, M0L, MkL)
    verts = np.asarray(verts)
    owner = _leaf_of_panels(F)
    pans = panels_at(P, verts)
    anc, lam0, lamk = fmm.leaf_locals_at(F, M0, Mk, owner[pans])
    row = {int(c): k for k, c in enumerate(anc)}
    pos = np.empty(P.n, np.int64)
    pos[tree.perm] = np.arange(P.n)                  # tree position of each panel
    y1 = np.zeros(len(verts))
    y2 = np.zeros(len(verts))
    for k, vx in enumerate(verts):
        for t_ in panels_at(P, [vx]):
            a_ = int(np.nonzero(P.tris[t_] == vx)[0][0])
            r = row[int(owner[t_])]
            y1[k] -= ((lam0[r] + lamk[r]) * F.ms3[pos[t_], a_]).sum()
            y2[k] -= ((lam0[r] + lamk[r] / eps) * F.md3[pos[t_], a_]).sum()
    return y1, y2


def near_matvec(F, u, v):
    P, V = F.P, F.V
    ti, tj = P.tris[F.near_i], P.tris[F.near_j]
    B = F.near_B
    y1 = np.zeros(V)
    y2 = np.zeros(V)
    np.add.at(y1, ti, np.einsum("pab,pb->pa", B[..., 0], u[tj]) + np.einsum("pab,pb->pa", B[..., 1], v[tj]))
    np.add.at(y2, ti, np.einsum("pab,pb->pa", B[..., 2], u[tj]) + np.einsum("pab,pb->pa", B[..., 3], v[tj]))
    return y1, y2


def matvec(F, x, far=True, near=True):
    """y = A x for x = [phi (V); dphi (V)] (identity terms with the near part)"""
    P, eps, V = F.P, F.eps, F.V
    u, v = x[:V], x[V:]
    y1 = np.zeros(V)
    y2 = np.zeros(V)
    if near:
        y1 += 0.5 * (1.0 + eps) * mass_matvec(P, u)
        y2 += 0.5 * (1.0 + 1.0 / eps) * mass_matvec(P, v)
        n1, n2 = near_matvec(F, u, v)
        y1 += n1
        y2 += n2
    if far and F.tree.lmin <= F.tree.L:
        f1, f2 = far_field(F, u, v)
        y1 += f1
        y2 += f2
    return np.concatenate([y1, y2])


def diagonal(F):
    """the diagonal of A (near entries between a vertex's own corners, plus
    the mass terms): the Jacobi preconditioner's divisors"""
    P, eps, V = F.P, F.eps, F.V
    ti, tj = P.tris[F.near_i], P.tris[F.near_j]
    same = ti[:, :, None] == tj[:, None, :]            # [p, a, b]
    d1 = np.zeros(V)
    d2 = np.zeros(V)
    R = np.broadcast_to(ti[:, :, None], same.shape)
    np.add.at(d1, R[same], F.near_B[..., 0][same])
    np.add.at(d2, R[same], F.near_B[..., 3][same])
    Mb = mass_diag_blocks(P)
    np.add.at(d1, P.tris, 0.5 * (1.0 + eps) * Mb[:, np.arange(3), np.arange(3)])
    np.add.at(d2, P.tris, 0.5 * (1.0 + 1.0 / eps) * Mb[:, np.arange(3), np.arange(3)])
    return np.concatenate([d1, d2])


def rhs(P, xq, q, eps_in):
    """b_i = (1/eps_in) int phi_i sum_k q_k G0(x, x_k) (and dG0/dn_x), by the
    3-point rule with the hat functions' values at its points"""
    V = len(P.verts)
    xq = np.atleast_2d(xq)
    r = P.qp[:, :, None, :] - xq[None, None, :, :]
    rr = np.sqrt((r * r).sum(-1))
    g0 = (1.0 / (FOUR_PI * rr)) @ q                                   # [N, 3 points]
    dg0 = (-(r * P.normal[:, None, None, :]).sum(-1) / (FOUR_PI * rr ** 3)) @ q
    b1 = np.zeros(V)
    b2 = np.zeros(V)
    np.add.at(b1, P.tris, np.einsum("pk,ka->pa", P.qw * g0, LAM) / eps_in)
    np.add.at(b2, P.tris, np.einsum("pk,ka->pa", P.qw * dg0, LAM) / eps_in)
    return np.concatenate([b1, b2])


def energy(P, x, xq, q, eps, kappa):
    """the discrete energy of ``solve.energy`` with phi, dphi interpolated by
    the hat functions at the 3-point rule's points"""
    V = len(P.verts)
    u, v = x[:V], x[V:]
    phi = np.einsum("ka,pa->pk", LAM, u[P.tris])          # [N, 3 points]
    dphi = np.einsum("ka,pa->pk", LAM, v[P.tris])
    xq = np.atleast_2d(xq)
    total = 0.0
    for n in range(len(q)):
        r = xq[n][None, None, :] - P.qp
        rr = np.sqrt((r * r).sum(-1))
        uu = kappa * rr
        em1 = np.expm1(-uu)
        E = em1 + 1.0
        rny = (r * P.normal[:, None, :]).sum(-1)
        k1 = -em1 / (FOUR_PI * rr)
        k2 = (eps * E * (1.0 + uu) - 1.0) * rny / (FOUR_PI * rr ** 3)
        total += q[n] * (P.qw * (k1 * dphi + k2 * phi)).sum()
    return 0.5 * UNIT_KCAL * total


# ---------------------------------------------------------------------------
# The Cartesian treecode (Sec. 2.5) with hat functions: the visit of
# ``treecode`` with the moments of the hat-function far field (corner moments,
# MtM) and, at leaves that fail the criterion, the direct sums with the nodal
# values interpolated at the 3-point rule's points (energy), or the per-point
# source terms distributed to the panel's corners with lambda_a (RHS; the far
# part by LtL and LtP with the corner moments).
# ---------------------------------------------------------------------------
def _hat_moments(F, u, v):
    P, tree, eps = F.P, F.tree, F.eps
    tri = P.tris[tree.perm]
    a, b = u[tri], v[tri]
    c0 = np.einsum("pat,pa->pt", F.ms3, b) - np.einsum("pat,pa->pt", F.md3, a)
    ck = -np.einsum("pat,pa->pt", F.ms3, b) + eps * np.einsum("pat,pa->pt", F.md3, a)
    leaf = tree.levels[tree.L]
    M0L = np.zeros((leaf.n, F.ms3.shape[2]))
    MkL = np.zeros((leaf.n, F.ms3.shape[2]))
    np.add.at(M0L, F.owner, c0)
    np.add.at(MkL, F.owner, ck)
    return fmm.upward_pass(F, M0L, MkL)


def treecode_energy(F, x, xq, q, theta, p_max=None):
    """E_sol (kcal/mol) by the treecode with hat functions (theta = 0: the
    direct sum of ``energy``)."""
    from .treecode import _far
    from . import taylor
    P, tree, eps, kappa, pl = F.P, F.tree, F.eps, F.kappa, F.orders
    V = F.V
    u, v = x[:V], x[V:]
    M0, Mk = _hat_moments(F, u, v)
    phi = np.einsum("ka,pa->pk", LAM, u[P.tris])          # [N, 3 points]
    dphi = np.einsum("ka,pa->pk", LAM, v[P.tris])
    L, levels, perm = tree.L, tree.levels, tree.perm
    l0 = min(tree.lmin, L)
    xq = np.atleast_2d(np.asarray(xq, np.float64))
    Vn = np.zeros(len(xq))
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
                Vn[n] += _far(d[acc], M0[l][a][:, :T], Mk[l][a][:, :T], kappa, p).sum()
            rest = front[~acc]
            if l < L:
                front = np.concatenate([np.arange(cl.child_start[c], cl.child_end[c]) for c in rest]) \
                    if len(rest) else rest
            else:
                for c in rest:
                    ids = perm[cl.start[c]:cl.end[c]]
                    r = xn[None, None, :] - P.qp[ids]
                    rr = np.sqrt((r * r).sum(-1))
                    uu = kappa * rr
                    em1 = np.expm1(-uu)
                    E = em1 + 1.0
                    rny = (r * P.normal[ids][:, None, :]).sum(-1)
                    k1 = -em1 / (FOUR_PI * rr)
                    k2 = (eps * E * (1.0 + uu) - 1.0) * rny / (FOUR_PI * rr ** 3)
                    Vn[n] += float((P.qw[ids] * (k1 * dphi[ids] + k2 * phi[ids])).sum())
    return 0.5 * UNIT_KCAL * float(np.dot(np.asarray(q, np.float64), Vn))


def treecode_rhs(F, xq, q, theta, eps_in, p_max=None):
    """b = [b1; b2] (vertex order) by the reverse treecode with hat functions
    (theta = 0: the direct sum of ``rhs``)."""
    from . import taylor
    P, tree, pl = F.P, F.tree, F.orders
    N, V = P.n, F.V
    L, levels, perm = tree.L, tree.levels, tree.perm
    l0 = min(tree.lmin, L)
    xq = np.atleast_2d(np.asarray(xq, np.float64))
    q = np.asarray(q, np.float64)
    lam = {l: np.zeros((levels[l].n, len(taylor.multi_indices(pl[l])))) for l in range(l0, L + 1)}
    c1 = np.zeros((N, 3))          # per panel corner (caller order)
    c2 = np.zeros((N, 3))
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
                Fc = taylor.coefficients(-d[acc], 0.0, p)
                for t, k in enumerate(taylor.multi_indices(p)):
                    lam[l][a, t] += q[n] * Fc[k] / FOUR_PI
            rest = front[~acc]
            if l < L:
                front = np.concatenate([np.arange(cl.child_start[c], cl.child_end[c]) for c in rest]) \
                    if len(rest) else rest
            else:
                for c in rest:
                    ids = perm[cl.start[c]:cl.end[c]]
                    r = P.qp[ids] - xn[None, None, :]
                    rr = np.sqrt((r * r).sum(-1))
                    g0 = 1.0 / (FOUR_PI * rr)
                    dg0 = -(r * P.normal[ids][:, None, :]).sum(-1) / (FOUR_PI * rr ** 3)
                    c1[ids] += q[n] * np.einsum("pk,ka->pa", P.qw[ids] * g0, LAM)
                    c2[ids] += q[n] * np.einsum("pk,ka->pa", P.qw[ids] * dg0, LAM)
    fmm.downward(F, lam, l0)
    f = lam[L][F.owner]                                             # tree order
    c1[perm] += np.einsum("pt,pat->pa", f, F.ms3)
    c2[perm] += np.einsum("pt,pat->pa", f, F.md3)
    b1 = np.zeros(V)
    b2 = np.zeros(V)
    np.add.at(b1, P.tris, c1)
    np.add.at(b2, P.tris, c2)
    return np.concatenate([b1, b2]) / eps_in
