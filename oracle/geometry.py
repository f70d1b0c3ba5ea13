"""Flat triangle panels (Sec. 2.3, reference triangle and affine parameterisation).

A panel tau_i with vertices u, v, w has area A_i = |(v-u) x (w-u)|/2, unit normal
n_i = (v-u) x (w-u)/(2A_i) (outward for counter-clockwise vertices seen from the
solvent side), centroid (u+v+w)/3 and local size h_i = sqrt(A_i).

Regular Galerkin quadrature: the symmetric three-point rule with barycentric
points (2/3,1/6,1/6) and permutations and weights A_i/3 (exact for quadratics;
its points stay in the interior so neighbouring panels never share one).
``points=1`` gives the one-point (centroid, weight A_i) rule instead, the
reading of the paper's "single point" regular quadrature that the tests
compare against its printed Kirkwood energies.
"""
import numpy as np
from types import SimpleNamespace


def panels(verts, tris, points=3):
    verts = np.asarray(verts, np.float64)
    tris = np.asarray(tris, np.int64)
    u, v, w = verts[tris[:, 0]], verts[tris[:, 1]], verts[tris[:, 2]]
    cr = np.cross(v - u, w - u)
    two_a = np.linalg.norm(cr, axis=1)
    area = 0.5 * two_a
    normal = cr / two_a[:, None]
    centroid = (u + v + w) / 3.0
    corners = np.stack([u, v, w], 1)
    # quadrature point k sits at 2/3 of corner k and 1/6 of the others
    if points == 3:
        qp = np.empty((len(tris), 3, 3))
        for k in range(3):
            qp[:, k] = (2.0 / 3.0) * corners[:, k] + (1.0 / 6.0) * (
                corners[:, (k + 1) % 3] + corners[:, (k + 2) % 3])
        qw = np.repeat((area / 3.0)[:, None], 3, axis=1)
    elif points == 1:
        qp = centroid[:, None, :].copy()
        qw = area[:, None].copy()
    else:
        raise ValueError("points must be 1 or 3")
    return SimpleNamespace(verts=verts, tris=tris, area=area, normal=normal,
                           centroid=centroid, h=np.sqrt(area), corners=corners,
                           qp=qp, qw=qw, n=len(tris))
