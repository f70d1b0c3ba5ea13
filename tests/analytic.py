"""Closed forms used to pin the oracle's singular quadrature (test helpers only).

* ``potential_1_over_r``: int_T 1/|x - y| dA_y over a flat triangle, in closed
  form (Wilton et al. 1984, IEEE Trans. Antennas Propag. 32, 276): a sum over the
  edges of a logarithmic term and an arctangent height correction.
* ``solid_angle``: the signed solid angle of a triangle seen from x (Van
  Oosterom & Strackee 1983, IEEE Trans. Biomed. Eng. 30, 125):
  tan(Omega/2) = a.(b x c) / (abc + (a.b)c + (a.c)b + (b.c)a),  a = p1 - x, ...
  Omega = int_T (y - x).n / |y - x|^3 dA_y for counter-clockwise vertices.
* ``composite_outer``: a composite rule on a triangle (4**levels congruent
  sub-triangles, each with a Duffy-collapsed Gauss rule) for the outer
  integral of a function that is smooth inside but not at the edges.
"""
import numpy as np


def potential_1_over_r(x, tri):
    """x: [m,3], tri: [3,3] -> [m]"""
    p = np.asarray(tri, np.float64)
    n = np.cross(p[1] - p[0], p[2] - p[0])
    n /= np.linalg.norm(n)
    d = (x - p[0]) @ n
    rho = x - d[:, None] * n
    ad = np.abs(d)
    out = np.zeros(len(x))
    for k in range(3):
        a, b = p[k], p[(k + 1) % 3]
        L = b - a
        lh = L / np.linalg.norm(L)
        uh = np.cross(lh, n)
        lp = (b - rho) @ lh
        lm = (a - rho) @ lh
        P0 = (a - rho) @ uh
        R02 = P0 * P0 + d * d
        Rp = np.sqrt(lp * lp + R02)
        Rm = np.sqrt(lm * lm + R02)
        with np.errstate(divide="ignore", invalid="ignore"):
            lg = np.where(np.abs(P0) > 0, P0 * np.log((Rp + lp) / (Rm + lm)), 0.0)
            at = np.arctan2(P0 * lp, R02 + ad * Rp) - np.arctan2(P0 * lm, R02 + ad * Rm)
        out += lg - ad * at
    return out


def solid_angle(x, tri):
    p = np.asarray(tri, np.float64)
    a = p[0] - x
    b = p[1] - x
    c = p[2] - x
    la, lb, lc = (np.linalg.norm(v, axis=1) for v in (a, b, c))
    num = np.einsum("ij,ij->i", a, np.cross(b, c))
    den = (la * lb * lc + np.einsum("ij,ij->i", a, b) * lc
           + np.einsum("ij,ij->i", a, c) * lb + np.einsum("ij,ij->i", b, c) * la)
    return 2.0 * np.arctan2(num, den)


def composite_outer(tri, levels=3, n=8):
    """Points [m,3] and weights [m] of a composite rule on the triangle."""
    tris = [np.asarray(tri, np.float64)]
    for _ in range(levels):
        nxt = []
        for t in tris:
            m01, m12, m20 = (t[0] + t[1]) / 2, (t[1] + t[2]) / 2, (t[2] + t[0]) / 2
            nxt += [np.array([t[0], m01, m20]), np.array([m01, t[1], m12]),
                    np.array([m20, m12, t[2]]), np.array([m01, m12, m20])]
        tris = nxt
    x, w = np.polynomial.legendre.leggauss(n)
    g, gw = 0.5 * (x + 1), 0.5 * w
    s = np.repeat(g, n)
    tt = np.tile(g, n)
    ww = np.repeat(gw, n) * np.tile(gw, n) * s
    pts, wts = [], []
    for t in tris:
        two_a = np.linalg.norm(np.cross(t[1] - t[0], t[2] - t[0]))
        pts.append(t[0] + s[:, None] * (t[1] - t[0]) + (s * tt)[:, None] * (t[2] - t[1]))
        wts.append(two_a * ww)
    return np.concatenate(pts), np.concatenate(wts)
