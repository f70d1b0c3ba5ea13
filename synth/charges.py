"""Seeded atoms and point charges for the synthetic workloads (numpy PCG64).

Workloads (sizes in Angstrom, charges in units of e):
  kirkwood1  : 1,280-triangle icosphere, R = 2, one +1 e at the centre.
  kirkwood2  : 81,920-triangle icosphere, R = 20, 50 charges uniform in a
               ball of radius 15, q ~ N(0, 0.5^2).
  globule200k: 2,000 atoms in a random compact packing (random sequential
               addition, min spacing 2.0) at protein-like number density
               0.055 per A^3, i.e. a ball of radius 20.6 (about 25 A with the
               atom radii and density tails); radii U[1.4, 2.0],
               q ~ N(0, 0.4^2) shifted to net -3 e; Gaussian isosurface with
               ~200k triangles.
  ellipsoid  : 20,000 atoms packed the same way in an ellipsoid with the
               80:60:50 aspect ratio scaled to the same number density
               (semi-axes 57.0 x 42.8 x 35.6), net -15 e; grid spacing chosen
               for a target triangle count (about 500k for the headline
               workload, 1M for the largest).
  At the nominal 25-A / 80x60x50-A sizes these atom counts are too sparse for
  sigma = 1 densities to close up: the isosurface becomes a sponge (genus in
  the thousands), which is nothing like a protein surface.
"""
import numpy as np

from .meshes import icosphere, isosurface_mesh


def ball_charges(n, radius, q_sigma, seed):
    """n charges uniform in a ball: r = radius*u^(1/3) with an isotropic
    direction; q ~ N(0, q_sigma^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    d = rng.standard_normal((n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    r = radius * rng.random(n) ** (1.0 / 3.0)
    x = d * r[:, None]
    q = rng.normal(0.0, q_sigma, n)
    return np.ascontiguousarray(x), np.ascontiguousarray(q)


def _packed(n, inside, sample, min_dist, rng, batch=4096):
    """Rejection-sample n points (from `sample`, filtered by `inside`) with
    pairwise distance >= min_dist (grid hashing)."""
    cell = min_dist
    pts = []
    grid = {}

    def ok(p):
        key = tuple(np.floor(p / cell).astype(int))
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                for dz in (-1, 0, 1):
                    for q in grid.get((key[0] + dx, key[1] + dy, key[2] + dz), ()):
                        if np.sum((q - p) ** 2) < min_dist * min_dist:
                            return False
        return True

    tries = 0
    while len(pts) < n:
        cand = sample(rng, batch)
        cand = cand[inside(cand)]
        for p in cand:
            tries += 1
            if ok(p):
                pts.append(p)
                key = tuple(np.floor(p / cell).astype(int))
                grid.setdefault(key, []).append(p)
                if len(pts) == n:
                    break
        if tries > 200 * n:
            raise RuntimeError("packing too dense")
    return np.array(pts)


def _atom_props(n, net_charge, rng):
    radii = rng.uniform(1.4, 2.0, n)
    q = rng.normal(0.0, 0.4, n)
    q -= (q.sum() - net_charge) / n
    return radii, q


NUMBER_DENSITY = 0.055   # atoms per cubic Angstrom, protein-like


def packed_atoms_ball(n=2000, radius=None, min_dist=2.0, net_charge=-3.0, seed=3):
    if radius is None:
        radius = (3.0 * n / (4.0 * np.pi * NUMBER_DENSITY)) ** (1.0 / 3.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = _packed(n, lambda p: np.einsum("ij,ij->i", p, p) <= radius * radius,
                lambda g, m: g.uniform(-radius, radius, (m, 3)), min_dist, rng)
    radii, q = _atom_props(n, net_charge, rng)
    return x, radii, q


def packed_atoms_ellipsoid(n=20000, aspect=(80.0, 60.0, 50.0), min_dist=2.0,
                           net_charge=-15.0, seed=5):
    a = np.asarray(aspect, np.float64)
    vol = 4.0 / 3.0 * np.pi * a.prod()
    a = a * (n / (NUMBER_DENSITY * vol)) ** (1.0 / 3.0)
    rng = np.random.Generator(np.random.PCG64(seed))
    x = _packed(n, lambda p: ((p / a) ** 2).sum(1) <= 1.0,
                lambda g, m: g.uniform(-1.0, 1.0, (m, 3)) * a, min_dist, rng)
    radii, q = _atom_props(n, net_charge, rng)
    return x, radii, q


# grid spacings (Angstrom) that put the triangle counts in the stated ranges
_SPACING = {"globule200k": 0.548, "ellipsoid500k": 0.748, "ellipsoid1m": 0.529}


def workload(name, spacing=None):
    """Return dict(verts, tris, xq, q, eps_in, eps_out, kappa, name)."""
    eps_in, eps_out, kappa = 1.0, 80.0, 0.1257
    if name == "kirkwood1":
        v, t = icosphere(3, 2.0)
        xq = np.zeros((1, 3))
        q = np.array([1.0])
    elif name.startswith("icosphere"):
        # icosphereL_R: level L, radius R, one +1 e at the centre
        lvl, rad = name[len("icosphere"):].split("_")
        v, t = icosphere(int(lvl), float(rad))
        xq = np.zeros((1, 3))
        q = np.array([1.0])
    elif name == "kirkwood2":
        v, t = icosphere(6, 20.0)
        xq, q = ball_charges(50, 15.0, 0.5, seed=2)
    elif name == "globule200k":
        x, r, q = packed_atoms_ball()
        v, t = isosurface_mesh(x, r, spacing=spacing or _SPACING[name])
        xq = x
    elif name in ("ellipsoid500k", "ellipsoid1m"):
        x, r, q = packed_atoms_ellipsoid()
        v, t = isosurface_mesh(x, r, spacing=spacing or _SPACING[name])
        xq = x
    else:
        raise ValueError(name)
    return {"name": name, "verts": np.ascontiguousarray(v, np.float64),
            "tris": np.ascontiguousarray(t, np.int32),
            "xq": np.ascontiguousarray(xq, np.float64),
            "q": np.ascontiguousarray(q, np.float64),
            "eps_in": eps_in, "eps_out": eps_out, "kappa": kappa}
