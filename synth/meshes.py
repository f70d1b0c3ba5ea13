"""Closed, conforming, outward-oriented triangle meshes for the test workloads.

* ``icosphere``: an icosahedron refined by edge bisection with every vertex
  pushed onto the sphere (20 * 4**level flat triangles).
* ``isosurface_mesh``: the level set rho(x) = iso of a sum of Gaussian atom
  densities, triangulated by marching tetrahedra on a uniform grid (each cube
  cut into the six Kuhn tetrahedra around its main diagonal, which tile space
  conformingly, so the extracted surface is closed and welded).

Vertices are shared (welded) between triangles, triangles are counter-clockwise
seen from outside, so (v1-v0) x (v2-v0) points out of the enclosed volume.
"""
import numpy as np


# ----------------------------------------------------------------------------
# icosphere
# ----------------------------------------------------------------------------
def _icosahedron():
    from scipy.spatial import ConvexHull
    g = (1.0 + 5.0 ** 0.5) / 2.0
    v = []
    for a in (-1.0, 1.0):
        for b in (-g, g):
            v += [(0.0, a, b), (a, b, 0.0), (b, 0.0, a)]
    v = np.array(v)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = ConvexHull(v).simplices.astype(np.int64)
    return v, _orient_outward_convex(v, f)


def _orient_outward_convex(v, f):
    n = np.cross(v[f[:, 1]] - v[f[:, 0]], v[f[:, 2]] - v[f[:, 0]])
    c = v[f].mean(axis=1)
    flip = np.einsum("ij,ij->i", n, c) < 0
    f = f.copy()
    f[flip] = f[flip][:, [0, 2, 1]]
    return f


def _bisect(v, f):
    nv, nf = len(v), len(f)
    e = np.concatenate([f[:, [0, 1]], f[:, [1, 2]], f[:, [2, 0]]])
    es = np.sort(e, axis=1)
    key = es[:, 0] * nv + es[:, 1]
    uk, inv = np.unique(key, return_inverse=True)
    mid = 0.5 * (v[uk // nv] + v[uk % nv])
    ab, bc, ca = (nv + inv[:nf], nv + inv[nf:2 * nf], nv + inv[2 * nf:])
    a, b, c = f[:, 0], f[:, 1], f[:, 2]
    nf_ = np.concatenate([np.stack([a, ab, ca], 1), np.stack([ab, b, bc], 1),
                          np.stack([ca, bc, c], 1), np.stack([ab, bc, ca], 1)])
    return np.concatenate([v, mid]), nf_


def icosphere(level, radius=1.0, center=(0.0, 0.0, 0.0)):
    """Geodesic sphere with 20*4**level flat triangles inscribed in a sphere of
    the given radius.  Returns (verts f64[nv,3], tris i32[nt,3])."""
    v, f = _icosahedron()
    for _ in range(level):
        v, f = _bisect(v, f)
        v /= np.linalg.norm(v, axis=1, keepdims=True)
    v = v * radius + np.asarray(center, dtype=np.float64)
    return np.ascontiguousarray(v), np.ascontiguousarray(f.astype(np.int32))


# ----------------------------------------------------------------------------
# Gaussian-density isosurface
# ----------------------------------------------------------------------------
def gaussian_density(grid_lo, h, shape, centers, radii, sigma):
    """rho on the grid points grid_lo + h*(i,j,k): sum over atoms of
    exp(-(|x-c|^2 - R^2) / (2 sigma^2)), truncated where a term is < 1e-7."""
    rho = np.zeros(shape, dtype=np.float64)
    s2 = 2.0 * sigma * sigma
    for c, r in zip(centers, radii):
        cut = np.sqrt(r * r + s2 * np.log(1e7))
        lo = np.maximum(np.floor((c - cut - grid_lo) / h).astype(int), 0)
        hi = np.minimum(np.ceil((c + cut - grid_lo) / h).astype(int) + 1,
                        np.array(shape))
        xs = [grid_lo[d] + h * np.arange(lo[d], hi[d]) - c[d] for d in range(3)]
        d2 = (xs[0][:, None, None] ** 2 + xs[1][None, :, None] ** 2
              + xs[2][None, None, :] ** 2)
        rho[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += np.exp(-(d2 - r * r) / s2)
    return rho


# the six Kuhn tetrahedra of the unit cube: walk from (0,0,0) to (1,1,1)
# along the axes in every order
_PERMS = [(0, 1, 2), (0, 2, 1), (1, 0, 2), (1, 2, 0), (2, 0, 1), (2, 1, 0)]


def _marching_tets(f, grid_lo, h, t_clamp):
    """Extract the zero level set of the grid function f (positive inside)."""
    nx, ny, nz = f.shape
    inside = f > 0
    corners = [inside[i:nx - 1 + i, j:ny - 1 + j, k:nz - 1 + k]
               for i in (0, 1) for j in (0, 1) for k in (0, 1)]
    anyin = np.logical_or.reduce(corners)
    allin = np.logical_and.reduce(corners)
    ci, cj, ck = np.nonzero(anyin & ~allin)
    base = np.stack([ci, cj, ck], 1)

    def gid(p):
        return (p[:, 0] * ny + p[:, 1]) * nz + p[:, 2]

    tris_e = []      # per triangle: three edges as (g_lo, g_hi) pairs
    dirs = []        # outward reference direction per triangle
    eye = np.eye(3, dtype=np.int64)
    lone_other = np.array([[1, 2, 3], [0, 2, 3], [0, 1, 3], [0, 1, 2]])
    # for a 2-2 split: code (bitmask of inside vertices) -> (a, b, c, d)
    pair_tab = {3: (0, 1, 2, 3), 5: (0, 2, 1, 3), 6: (1, 2, 0, 3),
                9: (0, 3, 1, 2), 10: (1, 3, 0, 2), 12: (2, 3, 0, 1)}
    for perm in _PERMS:
        o = [np.zeros(3, np.int64)]
        o.append(o[0] + eye[perm[0]])
        o.append(o[1] + eye[perm[1]])
        o.append(o[2] + eye[perm[2]])
        P = np.stack([base + oo for oo in o], 1)           # [M,4,3]
        G = np.stack([gid(P[:, q]) for q in range(4)], 1)  # [M,4]
        S = np.stack([inside[P[:, q, 0], P[:, q, 1], P[:, q, 2]]
                      for q in range(4)], 1)
        nin = S.sum(1)
        code = (S * (1 << np.arange(4))).sum(1)
        X = P.astype(np.float64)
        # one vertex alone on its side
        m1 = (nin == 1) | (nin == 3)
        if m1.any():
            Sl, Gl, Xl = S[m1], G[m1], X[m1]
            lone = np.where(nin[m1] == 1, np.argmax(Sl, 1), np.argmax(~Sl, 1))
            oth = lone_other[lone]
            a = Gl[np.arange(len(lone)), lone]
            e = [np.stack([a, Gl[np.arange(len(lone)), oth[:, q]]], 1)
                 for q in range(3)]
            tris_e.append(np.stack(e, 1))
            xin = np.where(S[m1][:, :, None], Xl, 0).sum(1) / nin[m1][:, None]
            xout = np.where(~S[m1][:, :, None], Xl, 0).sum(1) / (4 - nin[m1])[:, None]
            dirs.append(xout - xin)
        m2 = nin == 2
        if m2.any():
            c2 = code[m2]
            tab = np.zeros((16, 4), np.int64)
            for k, v in pair_tab.items():
                tab[k] = v
            abcd = tab[c2]
            G2, X2 = G[m2], X[m2]
            r = np.arange(len(c2))
            ga, gb, gc, gd = (G2[r, abcd[:, q]] for q in range(4))
            ac = np.stack([ga, gc], 1)
            ad = np.stack([ga, gd], 1)
            bd = np.stack([gb, gd], 1)
            bc = np.stack([gb, gc], 1)
            tris_e.append(np.stack([ac, ad, bd], 1))
            tris_e.append(np.stack([ac, bd, bc], 1))
            xin = 0.5 * (X2[r, abcd[:, 0]] + X2[r, abcd[:, 1]])
            xout = 0.5 * (X2[r, abcd[:, 2]] + X2[r, abcd[:, 3]])
            dirs.append(xout - xin)
            dirs.append(xout - xin)
    TE = np.concatenate(tris_e)             # [F,3,2] grid ids
    D = np.concatenate(dirs)
    lo = TE.min(axis=2)
    hi = TE.max(axis=2)
    ng = nx * ny * nz
    key = lo * ng + hi
    uk, inv = np.unique(key.ravel(), return_inverse=True)
    glo, ghi = uk // ng, uk % ng

    def unr(g):
        k = g % nz
        j = (g // nz) % ny
        i = g // (ny * nz)
        return np.stack([i, j, k], 1)

    plo, phi = unr(glo), unr(ghi)
    flat = f.ravel()
    flo, fhi = flat[glo], flat[ghi]
    t = np.clip(flo / (flo - fhi), t_clamp, 1.0 - t_clamp)
    verts = grid_lo + h * (plo + t[:, None] * (phi - plo))
    tris = inv.reshape(-1, 3)
    n = np.cross(verts[tris[:, 1]] - verts[tris[:, 0]],
                 verts[tris[:, 2]] - verts[tris[:, 0]])
    flip = np.einsum("ij,ij->i", n, D) < 0
    tris[flip] = tris[flip][:, [0, 2, 1]]
    return verts, tris


def largest_component(verts, tris):
    """Keep the connected surface piece with the most triangles (drops interior
    cavity surfaces and detached specks) and renumber its vertices."""
    from scipy.sparse import coo_matrix
    from scipy.sparse.csgraph import connected_components
    nv = len(verts)
    r = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2]])
    c = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0]])
    g = coo_matrix((np.ones(len(r)), (r, c)), shape=(nv, nv))
    ncomp, lab = connected_components(g, directed=False)
    tl = lab[tris[:, 0]]
    best = np.bincount(tl, minlength=ncomp).argmax()
    tris = tris[tl == best]
    used = np.unique(tris)
    remap = -np.ones(nv, np.int64)
    remap[used] = np.arange(len(used))
    return np.ascontiguousarray(verts[used]), remap[tris]


def _smooth(verts, tris, f_grid, grid_lo, h, iters):
    """Tangential Laplacian relaxation followed by a Newton projection back onto
    the level set (density interpolated trilinearly).  Improves triangle shape
    without changing the connectivity."""
    nv = len(verts)
    from scipy.sparse import coo_matrix
    r = np.concatenate([tris[:, 0], tris[:, 1], tris[:, 2], tris[:, 1], tris[:, 2], tris[:, 0]])
    c = np.concatenate([tris[:, 1], tris[:, 2], tris[:, 0], tris[:, 0], tris[:, 1], tris[:, 2]])
    A = coo_matrix((np.ones(len(r)), (r, c)), shape=(nv, nv)).tocsr()
    A.data[:] = 1.0
    deg = np.asarray(A.sum(1)).ravel()
    shape = np.array(f_grid.shape)

    def interp(p):
        u = (p - grid_lo) / h
        i0 = np.clip(np.floor(u).astype(np.int64), 0, shape - 2)
        w = u - i0
        val = np.zeros(len(p))
        grad = np.zeros((len(p), 3))
        for dx in (0, 1):
            for dy in (0, 1):
                for dz in (0, 1):
                    fv = f_grid[i0[:, 0] + dx, i0[:, 1] + dy, i0[:, 2] + dz]
                    wx = w[:, 0] if dx else 1 - w[:, 0]
                    wy = w[:, 1] if dy else 1 - w[:, 1]
                    wz = w[:, 2] if dz else 1 - w[:, 2]
                    val += fv * wx * wy * wz
                    sx = 1.0 if dx else -1.0
                    sy = 1.0 if dy else -1.0
                    sz = 1.0 if dz else -1.0
                    grad[:, 0] += fv * sx * wy * wz / h
                    grad[:, 1] += fv * wx * sy * wz / h
                    grad[:, 2] += fv * wx * wy * sz / h
        return val, grad

    v = verts.copy()
    for _ in range(iters):
        avg = (A @ v) / deg[:, None]
        _, g = interp(v)
        gn = g / np.maximum(np.linalg.norm(g, axis=1, keepdims=True), 1e-30)
        d = avg - v
        d -= np.einsum("ij,ij->i", d, gn)[:, None] * gn   # tangential part
        v = v + 0.5 * d
        for _ in range(2):
            val, g = interp(v)
            g2 = np.maximum(np.einsum("ij,ij->i", g, g), 1e-30)
            step = (val / g2)[:, None] * g
            step = np.clip(step, -0.25 * h, 0.25 * h)
            v = v - step
    return v


def isosurface_mesh(centers, radii, sigma=1.0, iso=1.0, spacing=0.5,
                    t_clamp=0.05, smooth_iters=3):
    """Triangulated surface rho(x) = iso of the Gaussian atom density.

    rho(x) = sum_i exp(-(|x - c_i|^2 - R_i^2) / (2 sigma^2)): a lone atom's
    surface sits at |x - c| = R.  Returns the largest closed component as
    (verts f64[nv,3], tris i32[nt,3]), outward oriented."""
    centers = np.asarray(centers, np.float64)
    radii = np.asarray(radii, np.float64)
    pad = radii.max() + 4.0 * sigma + 2.0 * spacing
    lo = centers.min(0) - pad
    hi = centers.max(0) + pad
    shape = tuple((np.ceil((hi - lo) / spacing).astype(int) + 1).tolist())
    rho = gaussian_density(lo, spacing, shape, centers, radii, sigma)
    f = rho - iso
    f[f == 0.0] = -1e-12
    v, t = _marching_tets(f, lo, spacing, t_clamp)
    v, t = largest_component(v, t)
    if smooth_iters:
        v = _smooth(v, t, f, lo, spacing, smooth_iters)
    return np.ascontiguousarray(v), np.ascontiguousarray(t.astype(np.int32))


def mesh_report(verts, tris):
    """Closedness/orientation/quality summary of a triangle mesh."""
    tris = np.asarray(tris, np.int64)
    nv = len(verts)
    e = np.concatenate([tris[:, [0, 1]], tris[:, [1, 2]], tris[:, [2, 0]]])
    dkey = e[:, 0] * nv + e[:, 1]
    ukey = np.sort(e, axis=1)
    ukey = ukey[:, 0] * nv + ukey[:, 1]
    _, ucnt = np.unique(ukey, return_counts=True)
    _, dcnt = np.unique(dkey, return_counts=True)
    a = verts[tris]
    n = np.cross(a[:, 1] - a[:, 0], a[:, 2] - a[:, 0])
    area = 0.5 * np.linalg.norm(n, axis=1)
    L = np.stack([np.linalg.norm(a[:, 1] - a[:, 0], axis=1),
                  np.linalg.norm(a[:, 2] - a[:, 1], axis=1),
                  np.linalg.norm(a[:, 0] - a[:, 2], axis=1)], 1)
    # quality 1 for equilateral, -> 0 for slivers
    q = 4.0 * np.sqrt(3.0) * area / (L ** 2).sum(1)
    vol = np.einsum("ij,ij->i", a[:, 0], np.cross(a[:, 1], a[:, 2])).sum() / 6.0
    return {
        "n_tris": int(len(tris)), "n_verts": int(nv),
        "n_edges": int(len(ucnt)),
        "euler": int(nv - len(ucnt) + len(tris)),
        "closed_manifold": bool((ucnt == 2).all()),
        "consistently_oriented": bool((dcnt == 1).all()),
        "volume": float(vol),
        "area_total": float(area.sum()),
        "area_min": float(area.min()), "area_mean": float(area.mean()),
        "quality_min": float(q.min()), "quality_mean": float(q.mean()),
        "h_mean": float(L.max(1).mean()),
    }
