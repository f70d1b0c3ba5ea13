"""Galerkin panel-pair integrals I1..I6 = int_{tau_i} int_{tau_j} k_m(x, y) dy dx.

Classes (decided from shared vertex indices and centroid distance):
  IDENT  i == j
  EDGE   two shared vertices
  VERTEX one shared vertex
  CLOSE  no shared vertex, |c_i - c_j| < near_ratio * max(h_i, h_j)
  REGULAR otherwise

Rules (n = Gauss-Legendre points per dimension, 7 by default):
  REGULAR  product of the panels' regular rules (3 x 3 points; 1 x 1 with
           the one-point panel rule), Sec. 2.3 regular quadrature.
  CLOSE    Duffy-collapsed n x n Gauss rule on each triangle (n^4 points).
  IDENT/EDGE/VERTEX: the singularity-removing relative-coordinate transforms of
  Sauter and Schwab (Sec. 2.3, "cubature"), written out below from their
  mathematics.  Each panel is parameterised over the reference triangle
  {0 <= x2 <= x1 <= 1} by chi(x) = u + x1 (v - u) + x2 (w - v), Jacobian 2A.

  IDENT: the integrand depends only on z = y - x.  For fixed z the admissible
  x form a copy of the reference triangle scaled by (1 - sigma(z)), with
  sigma(z) = max(0,-z2) + max(0, z2-z1) + max(0, z1), so
      int int f = int_{hexagon} (1 - sigma)^2 / 2 * f(z) dz .
  The hexagon splits into six triangles (0, P_s, Q_s) on which sigma is linear;
  z = xi ((1-t) P_s + t Q_s) gives dz = xi dxi dt, sigma = xi.  The 1/|z|
  singularity cancels against xi.  n^2 points per sector.

  EDGE (shared edge P->Q, both panels chi = P + x1 (Q-P) + x2 (R - Q)): the
  integrand depends on (z1 = y1 - x1, x2, y2) only; the x1-range has length
  1 - sigma with sigma = max(0, z1) + max(x2, y2 - z1).  Four pyramids on which
  sigma is linear, each parameterised radially (xi times a point of the face
  sigma = 1) with Jacobian xi^2 (times s on the two triangular faces, which are
  Duffy-collapsed).  n^3 points per pyramid.

  VERTEX (shared vertex S at the reference origin of both panels): Duffy on
  each triangle (x = x1 (1, t)), then the square (x1, y1) is split along its
  diagonal and each half collapsed towards the origin (weight xi^3 eta).
  n^4 points per half.

On flat panels I2..I5 of an identical pair vanish identically (r.n = 0); they
are set to exactly zero.  Touching and close pairs are integrated once, for
the ordering with the lower first index, and the other ordering is filled in
by the exact symmetries of the kernels (Sec. 2.2: every kernel depends on
x - y): I1, I6 symmetric, I2 <-> I4 and I3 <-> I5 transposed.
"""
import numpy as np

from .kernels import kernel6

REGULAR, IDENT, EDGE, VERTEX, CLOSE = 0, 1, 2, 3, 4


def gauss01(n):
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def shared_count(tris, i, j):
    ti, tj = tris[i], tris[j]
    return (ti[:, :, None] == tj[:, None, :]).any(2).sum(1)


def classify(P, i, j, near_ratio):
    i = np.asarray(i)
    j = np.asarray(j)
    s = shared_count(P.tris, i, j)
    cls = np.full(i.shape, REGULAR, np.int64)
    d = np.linalg.norm(P.centroid[i] - P.centroid[j], axis=1)
    close = d < near_ratio * np.maximum(P.h[i], P.h[j])
    cls[close] = CLOSE
    cls[s == 1] = VERTEX
    cls[s == 2] = EDGE
    cls[i == j] = IDENT
    return cls


def _integrate(r, wts, nx, ny, kappa, kern=None):
    """sum_k wts[p,k] * kern(r[p,k]) -> [p, m] (kern defaults to kernel6)"""
    K = (kern or kernel6)(r, nx[:, None, :], ny[:, None, :], kappa)
    return np.einsum("pk,pkm->pm", wts, K)


def regular(P, i, j, kappa, kern=None):
    m = P.qp.shape[1]
    r = P.qp[i][:, :, None, :] - P.qp[j][:, None, :, :]
    w = P.qw[i][:, :, None] * P.qw[j][:, None, :]
    return _integrate(r.reshape(len(i), m * m, 3), w.reshape(len(i), m * m),
                      P.normal[i], P.normal[j], kappa, kern)


def _duffy_points(corners, n):
    """Duffy-collapsed n x n rule on triangles: points [p, n*n, 3], weights."""
    g, gw = gauss01(n)
    s = np.repeat(g, n)
    t = np.tile(g, n)
    w = np.repeat(gw, n) * np.tile(gw, n) * s
    u, v, ww = corners[:, 0], corners[:, 1], corners[:, 2]
    pts = (u[:, None, :] + s[None, :, None] * (v - u)[:, None, :]
           + (s * t)[None, :, None] * (ww - v)[:, None, :])
    two_a = np.linalg.norm(np.cross(v - u, ww - u), axis=1)
    return pts, two_a[:, None] * w[None, :]


def close(P, i, j, kappa, n, kern=None):
    xi, wx = _duffy_points(P.corners[i], n)
    yj, wy = _duffy_points(P.corners[j], n)
    m = n * n
    r = xi[:, :, None, :] - yj[:, None, :, :]
    w = wx[:, :, None] * wy[:, None, :]
    return _integrate(r.reshape(len(i), m * m, 3), w.reshape(len(i), m * m),
                      P.normal[i], P.normal[j], kappa, kern)


_HEX = [((1, 0), (1, 1)), ((1, 1), (0, 1)), ((0, 1), (-1, 0)),
        ((-1, 0), (-1, -1)), ((-1, -1), (0, -1)), ((0, -1), (1, 0))]


def ident(P, i, kappa, n, kern=None):
    g, gw = gauss01(n)
    xi = np.repeat(g, n)
    t = np.tile(g, n)
    wq = np.repeat(gw, n) * np.tile(gw, n) * 0.5 * (1.0 - xi) ** 2 * xi
    zs, ws = [], []
    for Pq, Qq in _HEX:
        Pq = np.array(Pq, float)
        Qq = np.array(Qq, float)
        z = xi[:, None] * ((1.0 - t)[:, None] * Pq + t[:, None] * Qq)
        zs.append(z)
        ws.append(wq)
    z = np.concatenate(zs)          # [6 n^2, 2]
    w = np.concatenate(ws)
    c = P.corners[i]
    e1 = c[:, 1] - c[:, 0]
    e2 = c[:, 2] - c[:, 1]
    # r = chi(x) - chi(x + z) = -(z1 e1 + z2 e2)
    r = -(z[None, :, 0, None] * e1[:, None, :] + z[None, :, 1, None] * e2[:, None, :])
    scale = 4.0 * P.area[i] ** 2
    I = _integrate(r, scale[:, None] * w[None, :], P.normal[i], P.normal[i], kappa, kern)
    if kern is None:
        I[:, 1:5] = 0.0
    return I


def _reorder_edge(P, i, j):
    """Per pair: P, Q (the shared edge, in the order they appear in triangle
    i) and the opposite vertices R_i, R_j."""
    ti, tj = P.tris[i], P.tris[j]
    in_j = (ti[:, :, None] == tj[:, None, :]).any(2)   # [p,3] which of ti shared
    in_i = (tj[:, :, None] == ti[:, None, :]).any(2)
    oi = np.argsort(~in_j, axis=1, kind="stable")       # shared first, in order
    oj = np.argsort(in_i, axis=1, kind="stable")        # unshared first
    r = np.arange(len(i))
    V = P.verts
    return (V[ti[r, oi[:, 0]]], V[ti[r, oi[:, 1]]], V[ti[r, oi[:, 2]]],
            V[tj[r, oj[:, 0]]])


def edge(P, i, j, kappa, n, kern=None):
    Pv, Qv, Ri, Rj = _reorder_edge(P, i, j)
    e = Qv - Pv
    a = Ri - Qv
    b = Rj - Qv
    g, gw = gauss01(n)
    XI, W1, W2 = np.meshgrid(g, g, g, indexing="ij")
    WXI, WW1, WW2 = np.meshgrid(gw, gw, gw, indexing="ij")
    XI, W1, W2 = XI.ravel(), W1.ravel(), W2.ravel()
    wbase = (WXI * WW1 * WW2).ravel() * (1.0 - XI) * XI ** 2
    pieces = []
    # A: (z1, x2, y2) = xi (w1, 1 - w1, w2)
    pieces.append((XI * W1, XI * (1 - W1), XI * W2, wbase))
    # B: (z1, x2, y2) = xi (s(1-q), s q, 1), extra weight s
    pieces.append((XI * W1 * (1 - W2), XI * W1 * W2, XI, wbase * W1))
    # C: (z1, x2, y2) = xi (-s(1-q), 1, s q), extra weight s
    pieces.append((-XI * W1 * (1 - W2), XI, XI * W1 * W2, wbase * W1))
    # D: (z1, x2, y2) = xi (-w1, w2, 1 - w1)
    pieces.append((-XI * W1, XI * W2, XI * (1 - W1), wbase))
    z1 = np.concatenate([p[0] for p in pieces])
    x2 = np.concatenate([p[1] for p in pieces])
    y2 = np.concatenate([p[2] for p in pieces])
    w = np.concatenate([p[3] for p in pieces])
    r = (-z1[None, :, None] * e[:, None, :] + x2[None, :, None] * a[:, None, :]
         - y2[None, :, None] * b[:, None, :])
    scale = 4.0 * P.area[i] * P.area[j]
    return _integrate(r, scale[:, None] * w[None, :], P.normal[i], P.normal[j], kappa, kern)


def _reorder_vertex(P, i, j):
    """Per pair: the shared vertex S and the other two vertices of each
    triangle in their order of appearance."""
    ti, tj = P.tris[i], P.tris[j]
    in_j = (ti[:, :, None] == tj[:, None, :]).any(2)
    in_i = (tj[:, :, None] == ti[:, None, :]).any(2)
    oi = np.argsort(~in_j, axis=1, kind="stable")
    oj = np.argsort(~in_i, axis=1, kind="stable")
    r = np.arange(len(i))
    V = P.verts
    return (V[ti[r, oi[:, 0]]], V[ti[r, oi[:, 1]]], V[ti[r, oi[:, 2]]],
            V[tj[r, oj[:, 1]]], V[tj[r, oj[:, 2]]])


def vertex(P, i, j, kappa, n, kern=None):
    S, Vi, Wi, Vj, Wj = _reorder_vertex(P, i, j)
    g, gw = gauss01(n)
    XI, ETA, T1, T2 = np.meshgrid(g, g, g, g, indexing="ij")
    W = np.ones_like(XI)
    for ax, wv in enumerate(np.meshgrid(gw, gw, gw, gw, indexing="ij")):
        W = W * wv
    XI, ETA, T1, T2, W = (a.ravel() for a in (XI, ETA, T1, T2, W))
    W = W * XI ** 3 * ETA
    # alpha(t) = (V - S) + t (W - V)
    al = (Vi - S)[:, None, :] + T1[None, :, None] * (Wi - Vi)[:, None, :]
    be = (Vj - S)[:, None, :] + T2[None, :, None] * (Wj - Vj)[:, None, :]
    r1 = XI[None, :, None] * al - (XI * ETA)[None, :, None] * be
    r2 = (XI * ETA)[None, :, None] * al - XI[None, :, None] * be
    r = np.concatenate([r1, r2], axis=1)
    w = np.concatenate([W, W])
    scale = 4.0 * P.area[i] * P.area[j]
    return _integrate(r, scale[:, None] * w[None, :], P.normal[i], P.normal[j], kappa, kern)


def pair_integrals(P, i, j, kappa, near_ratio=2.0, n=7, cls=None, chunk=2048):
    """I1..I6 for the ordered pairs (i[k], j[k]): returns ([p, 6], classes)."""
    i = np.asarray(i, np.int64)
    j = np.asarray(j, np.int64)
    if cls is None:
        cls = classify(P, i, j, near_ratio)
    out = np.zeros((len(i), 6))
    rules = {REGULAR: (lambda a, b: regular(P, a, b, kappa), 65536),
             IDENT: (lambda a, b: ident(P, a, kappa, n), 4096),
             EDGE: (lambda a, b: edge(P, a, b, kappa, n), 1024),
             VERTEX: (lambda a, b: vertex(P, a, b, kappa, n), 256),
             CLOSE: (lambda a, b: close(P, a, b, kappa, n), 128)}
    # touching and close pairs are integrated for the member with the lower
    # panel index and mirrored: I1, I6 are symmetric and I2/I4, I3/I5 swap
    # (the kernels depend on x - y only), which the cubature would otherwise
    # satisfy only to its own error
    mirror = (cls >= EDGE) & (i > j)
    a = np.where(mirror, j, i)
    b = np.where(mirror, i, j)
    for c, (fn, ch) in rules.items():
        sel = np.nonzero(cls == c)[0]
        for s in range(0, len(sel), ch):
            k = sel[s:s + ch]
            out[k] = fn(a[k], b[k])
    out[mirror] = out[mirror][:, [0, 3, 4, 1, 2, 5]]
    return out, cls
