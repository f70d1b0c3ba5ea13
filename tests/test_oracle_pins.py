"""Pins of the FP64 oracle against things other than itself: closed forms,
finite differences, symbolic derivatives, invariants and the paper's printed
Kirkwood-sphere values.  CPU only."""
import numpy as np
import pytest

from analytic import composite_outer, potential_1_over_r, solid_angle
from oracle import dense, fmm, kirkwood, pairs, solve, taylor
from oracle import tree as otree
from oracle.geometry import panels
from oracle.kernels import kernel6
from synth import icosphere


def _golden(name):
    import os
    out = {}
    with open(os.path.join(os.path.dirname(__file__), "golden", name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            k, n, v = line.split()
            out[(k, n)] = float(v)
    return out


def _three_panels():
    verts = np.array([[0, 0, 0], [1.0, 0, 0], [0.4, 0.8, 0.1], [0.5, -0.7, 0.3],
                      [-0.6, 0.5, -0.2]])
    tris = np.array([[0, 1, 2], [1, 0, 3], [0, 4, 2]])
    return panels(verts, tris)


def _g0_kernels(r, nx, ny, kappa):
    rr = np.sqrt((r * r).sum(-1))
    return np.stack([1.0 / (4 * np.pi * rr), (r * ny).sum(-1) / (4 * np.pi * rr ** 3)], -1)


def _reference(P, i, j):
    """outer composite rule at two refinements, Richardson-extrapolated (the
    outer integrand is smooth inside but its gradient is log-singular at the
    panel edges, so the composite error falls by about 4 per level)"""
    vals = []
    for lev in (4, 5):
        pts, w = composite_outer(P.corners[i], lev, 8)
        s = np.sum(w * potential_1_over_r(pts, P.corners[j])) / (4 * np.pi)
        d = -np.sum(w * solid_angle(pts, P.corners[j])) / (4 * np.pi)
        vals.append((s, d))
    (s4, d4), (s5, d5) = vals
    return s5 + (s5 - s4) / 3.0, d5 + (d5 - d4) / 3.0


def test_gauss_legendre_exactness():
    g, w = pairs.gauss01(7)
    for k in range(14):
        assert abs((w * g ** k).sum() - 1.0 / (k + 1)) < 1e-14


def test_three_point_rule_exact_for_quadratics():
    P = panels(np.array([[0, 0, 0], [2.0, 0, 0], [0.5, 1.5, 0]]), np.array([[0, 1, 2]]))
    # int x^2 over the triangle by a fine composite rule as the check
    pts, w = composite_outer(P.corners[0], 3, 6)
    for f in (lambda p: p[..., 0] ** 2, lambda p: p[..., 0] * p[..., 1], lambda p: p[..., 1]):
        ref = (w * f(pts)).sum()
        got = (P.qw[0] * f(P.qp[0])).sum()
        assert abs(got - ref) < 1e-12 * max(1, abs(ref))


@pytest.mark.parametrize("case", ["ident", "edge01", "edge10", "edge02", "vertex12"])
def test_singular_rules_match_closed_forms(case):
    """Single layer against the Wilton closed form, double layer against the
    Van Oosterom-Strackee solid angle (outer integral by a fine composite rule)."""
    P = _three_panels()
    spec = {"ident": (0, 0), "edge01": (0, 1), "edge10": (1, 0), "edge02": (0, 2),
            "vertex12": (1, 2)}[case]
    i, j = np.array([spec[0]]), np.array([spec[1]])
    if case == "ident":
        I = pairs.ident(P, i, 0.0, 7, kern=_g0_kernels)[0]
    elif case.startswith("edge"):
        I = pairs.edge(P, i, j, 0.0, 7, kern=_g0_kernels)[0]
    else:
        I = pairs.vertex(P, i, j, 0.0, 7, kern=_g0_kernels)[0]
    s, d = _reference(P, spec[0], spec[1])
    assert abs(I[0] - s) < 2e-8 * abs(s)
    if case != "ident":      # the solid angle is two-valued on the panel itself
        assert abs(I[1] - d) < 1e-7 * abs(d)
    else:
        assert I[1] == pytest.approx(0.0, abs=1e-12)


def test_kernel6_matches_finite_differences():
    """k2..k6 are normal derivatives of G0/Gk: check against central differences."""
    rng = np.random.default_rng(1)
    kappa = 0.37
    x = rng.standard_normal(3)
    y = rng.standard_normal(3) + np.array([1.5, 0, 0])
    nx = rng.standard_normal(3); nx /= np.linalg.norm(nx)
    ny = rng.standard_normal(3); ny /= np.linalg.norm(ny)

    def G(a, b, k):
        r = np.linalg.norm(a - b)
        return np.exp(-k * r) / (4 * np.pi * r)

    h = 1e-4
    dy = lambda k: (G(x, y + h * ny, k) - G(x, y - h * ny, k)) / (2 * h)
    dx = lambda k: (G(x + h * nx, y, k) - G(x - h * nx, y, k)) / (2 * h)

    def dxy(k):
        f = lambda a, b: G(x + a * nx, y + b * ny, k)
        return (f(h, h) - f(h, -h) - f(-h, h) + f(-h, -h)) / (4 * h * h)

    K = kernel6(x - y, nx, ny, kappa)
    ref = [G(x, y, 0) - G(x, y, kappa), dy(0), dy(kappa), dx(0), dx(kappa), dxy(kappa) - dxy(0)]
    for m in range(6):
        assert abs(K[m] - ref[m]) < 1e-6 * max(abs(ref[m]), 1e-3), m


@pytest.mark.parametrize("kappa", [0.0, 0.4])
def test_taylor_recurrence_matches_sympy(kappa):
    import sympy as sp
    X, Y, Z = sp.symbols("X Y Z", real=True)
    r = sp.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    f = sp.exp(-sp.Rational(kappa).limit_denominator(1000) * r) / r
    x0 = np.array([0.7, -1.1, 0.4])
    F = taylor.coefficients(x0, float(sp.Rational(kappa).limit_denominator(1000)), 5)
    sub = {X: sp.Rational(7, 10), Y: sp.Rational(-11, 10), Z: sp.Rational(2, 5)}
    for k in taylor.multi_indices(5):
        d = sp.diff(f, X, k[0], Y, k[1], Z, k[2]) if sum(k) else f
        ref = float(d.subs(sub).evalf(30)) / taylor.mfact(k)
        assert abs(F[k][0] - ref) < 1e-12 * max(abs(ref), 1e-8), k


def test_taylor_coefficients_reflect_with_the_axes():
    """Both kernels depend on |r| only, so reflecting axis a multiplies the
    coefficient of k by (-1)^k_a: F_k(x0) = (-1)^(k . s) F_k(|x0|) with s the
    signs of x0's components (the octant tables of the GPU's order-4 MtL rest
    on this).  An index mixed up between axes in the recurrence breaks it; the
    values themselves are pinned against sympy above."""
    rng = np.random.default_rng(8)
    x0 = rng.uniform(-4.0, 4.0, (40, 3))
    x0[np.abs(x0) < 0.3] = 0.7
    for kappa in (0.0, 0.1257):
        F = taylor.coefficients(x0, kappa, 7)
        Fa = taylor.coefficients(np.abs(x0), kappa, 7)
        neg = (x0 < 0).astype(int)
        for k in taylor.multi_indices(7):
            sign = (-1.0) ** (neg @ np.array(k))
            scale = np.abs(Fa[k]).max()
            assert np.abs(F[k] - sign * Fa[k]).max() <= 1e-14 * scale, (kappa, k)


def test_shift_matrices_are_exact_translations():
    """MtM of moments equals the moments taken about the new centre, and LtL
    of a local expansion evaluates to the same polynomial (binomial formula)."""
    rng = np.random.default_rng(2)
    p = 5
    mi = taylor.multi_indices(p)
    pts = rng.standard_normal((20, 3)) * 0.3
    w = rng.standard_normal(20)
    c1 = np.array([0.1, -0.2, 0.05])
    c2 = c1 + np.array([0.25, -0.25, 0.25])
    mom = lambda c: np.array([(w * np.prod((pts - c) ** np.array(a), 1)).sum() for a in mi])
    S = fmm.shift_matrix(c1 - c2, p, p)
    assert np.allclose(S @ mom(c1), mom(c2), rtol=1e-12, atol=1e-14)
    lam = rng.standard_normal(len(mi))
    x = rng.standard_normal(3) * 0.2
    ev = lambda l, c: sum(l[t] * np.prod((x - c) ** np.array(a)) for t, a in enumerate(mi))
    S2 = fmm.shift_matrix(c2 - c1, p, p)   # parent c1 -> child c2
    assert abs(ev(S2.T @ lam, c2) - ev(lam, c1)) < 1e-12


def test_m2l_converges_to_direct_sum():
    rng = np.random.default_rng(3)
    src = rng.uniform(-0.5, 0.5, (30, 3))
    tgt = rng.uniform(-0.5, 0.5, (10, 3)) + np.array([3.0, 0, 0])
    q = rng.standard_normal(30)
    kappa = 0.3
    cs, ct = np.zeros(3), np.array([3.0, 0, 0])
    direct = np.array([(q * np.exp(-kappa * np.linalg.norm(t - src, axis=1))
                        / (4 * np.pi * np.linalg.norm(t - src, axis=1))).sum() for t in tgt])
    errs = []
    for p in (2, 4, 6, 8):
        mi = taylor.multi_indices(p)
        M = np.array([(q * np.prod((src - cs) ** np.array(a), 1)).sum() for a in mi])
        lam = fmm.m2l_matrix(ct - cs, kappa, p) @ M
        approx = np.array([sum(lam[t] * np.prod((x - ct) ** np.array(a)) for t, a in enumerate(mi))
                           for x in tgt])
        errs.append(np.abs(approx - direct).max() / np.abs(direct).max())
    assert all(errs[k + 1] < 0.5 * errs[k] for k in range(3)), errs
    assert errs[-1] < 1e-4


@pytest.fixture(scope="module")
def sphere320():
    v, t = icosphere(2, 2.0)
    P = panels(v, t)
    I, cls = dense.integrals(P, 0.1257)
    return P, I


def test_gauss_double_layer_identity(sphere320):
    """sum_j int_i int_j dG0/dn_y = -A_i/2 on a closed surface (Gauss)."""
    P, I = sphere320
    s = I[..., 1].sum(1) / P.area
    assert np.abs(s + 0.5).max() < 2e-3


def test_pair_symmetries(sphere320):
    P, I = sphere320
    # the product rules are symmetric; touching/close pairs are mirrored
    for a, b in ((0, 0), (5, 5), (3, 1), (4, 2)):
        scale = np.abs(I[..., a]).max()
        assert np.abs(I[..., a] - I[..., b].T).max() < 1e-14 * scale


def test_sphere_constant_density_operators(sphere320):
    """Unit density on a sphere of radius a: int G0 = a, int Gk = (1 - e^{-2 k a})/(2k),
    int dGk/dn = -(1 - e^{-2ka}(1+ka))/(2ka); flat 320-panel sphere agrees to O(h^2)."""
    P, I = sphere320
    a, k = 2.0, 0.1257
    V0 = a
    Vk = (1 - np.exp(-2 * k * a)) / (2 * k)
    Kk = -(1 - np.exp(-2 * k * a) * (1 + k * a)) / (2 * k * a)
    A = P.area
    assert abs((I[..., 0].sum(1) / A).mean() - (V0 - Vk)) < 0.02 * (V0 - Vk)
    assert abs((I[..., 2].sum(1) / A).mean() - Kk) < 0.01 * abs(Kk)


def test_born_and_kirkwood_series_agree():
    for kap in (0.0, 0.1257):
        assert kirkwood.energy(np.zeros((1, 3)), [1.0], 2.0, 1.0, 80.0, kap) == pytest.approx(
            kirkwood.born(1.0, 2.0, 1.0, 80.0, kap), rel=1e-13)
    g = _golden("kirkwood_paper_table2.txt")
    assert kirkwood.born(50.0, 50.0, 1.0, 40.0, 0.1257) == pytest.approx(g[("exact", "inf")], abs=0.02)


def test_kirkwood_series_properties():
    from scipy.special import spherical_kn
    x = 0.8
    for n in range(6):
        Rn = x * spherical_kn(n, x, derivative=True) / spherical_kn(n, x)
        # reaction factor from the library's Bessel ratio
        C = (80.0 * Rn + 2.0 * (n + 1)) / (2.0 * n - 80.0 * Rn)
        assert kirkwood.reaction_factors(x / 0.4, 2.0, 80.0, 0.4, 5)[n] == pytest.approx(C, rel=1e-12)
    # kappa = 0 reduces to the classical (n+1)(e1-e2)/(n e1 + (n+1) e2)
    C0 = kirkwood.reaction_factors(3.0, 2.0, 80.0, 0.0, 5)
    for n in range(6):
        assert C0[n] == pytest.approx((n + 1) * (2.0 - 80.0) / (n * 2.0 + (n + 1) * 80.0), rel=1e-14)
    rng = np.random.default_rng(4)
    xq = rng.uniform(-1, 1, (5, 3))
    q = rng.standard_normal(5)
    e1 = kirkwood.energy(xq, q, 3.0, 1.0, 80.0, 0.1)
    p = rng.permutation(5)
    assert kirkwood.energy(xq[p], q[p], 3.0, 1.0, 80.0, 0.1) == pytest.approx(e1, rel=1e-13)


def test_paper_sphere_energy_matches_table2():
    """Dense oracle on the paper's sphere (R=50, q=50, eps 1/40) with 320 panels
    lands within 0.05% of the paper's high-order quadrature value."""
    g = _golden("kirkwood_paper_table2.txt")
    v, t = icosphere(2, 50.0)
    P = panels(v, t)
    A = dense.assemble(P, 40.0, 0.1257)
    b = solve.rhs(P, np.zeros((1, 3)), np.array([50.0]), 1.0)
    x, it, _ = solve.gmres(lambda z: A @ z, b, 1e-10)
    E = solve.energy(P, x, np.zeros((1, 3)), np.array([50.0]), 40.0, 0.1257)
    assert abs(E - g[("table2_order4", "320")]) < 5e-4 * abs(E)
    assert abs(E - g[("table2_order3", "320")]) < 5e-4 * abs(E)
    # and the discretisation error is below the paper's one-point-rule error
    assert abs(E - g[("exact", "inf")]) < abs(g[("table1_order1", "320")] - g[("exact", "inf")])


def test_regular_rule_reading_against_tables():
    """Reading of the paper's regular quadrature (Sec. 2.3; Tables 1-2 print
    energies for orders 2-4 of the touching-pair cubature): on its 320-panel
    sphere the three-point panel rule lands within 0.05 % of the printed
    entries for orders 3 and 4, while a one-point (centroid) rule for the
    regular pairs, the right-hand side and the energy lands 1.6 % away from
    them and farther than the three-point rule for every order 2-4."""
    g = _golden("kirkwood_paper_table2.txt")
    v, t = icosphere(2, 50.0)
    err = {}
    for pts in (3, 1):
        P = panels(v, t, points=pts)
        b = solve.rhs(P, np.zeros((1, 3)), np.array([50.0]), 1.0)
        for n in (2, 3, 4):
            A = dense.assemble(P, 40.0, 0.1257, n=n)
            x = np.linalg.solve(A, b)
            E = solve.energy(P, x, np.zeros((1, 3)), np.array([50.0]), 40.0, 0.1257)
            ref = g[("table2_order%d" % n, "320")]
            err[(pts, n)] = abs(E - ref) / abs(ref)
    for n in (2, 3, 4):
        assert err[(3, n)] < err[(1, n)], (n, err)
        assert err[(1, n)] > 1e-2, (n, err)
    assert err[(3, 3)] < 5e-4 and err[(3, 4)] < 5e-4, err


def test_born_surface_values():
    """Solved surface potential/derivative vs the exact Born values on C1-like sphere."""
    v, t = icosphere(2, 2.0)
    P = panels(v, t)
    eps, kap = 80.0, 0.1257
    A = dense.assemble(P, eps, kap)
    b = solve.rhs(P, np.zeros((1, 3)), np.array([1.0]), 1.0)
    x, it, _ = solve.gmres(lambda z: A @ z, b, 1e-10)
    N = P.n
    phi_ex = 1.0 / (4 * np.pi * 2.0 * eps * (1 + kap * 2.0))
    dphi_ex = -1.0 / (4 * np.pi * 4.0)
    assert np.abs(x[:N] / phi_ex - 1).max() < 0.05
    # flat panels sit inside the sphere (centroid radius ~1.5% short at 320
    # panels), so the flux density is a few percent high
    assert np.abs(x[N:] / dphi_ex - 1).max() < 0.05
    assert np.linalg.norm(A @ x - b) < 1e-9 * np.linalg.norm(b)


@pytest.fixture(scope="module")
def sphere1280_dense():
    v, t = icosphere(3, 2.0)
    P = panels(v, t)
    return P, dense.assemble(P, 80.0, 0.1257)


def test_tree_coverage_and_fmm_convergence(sphere1280_dense):
    P, A = sphere1280_dense
    tr = otree.build(P, 32, 0.8)
    assert (fmm.coverage(tr) == 1).all()
    # a deeper tree on a smaller leaf size also covers every pair once
    tr8 = otree.build(P, 8, 0.8)
    assert tr8.L > tr.L and (fmm.coverage(tr8) == 1).all()
    rng = np.random.default_rng(5)
    x = rng.standard_normal(2 * P.n)
    F = fmm.setup(P, tr8, 80.0, 0.1257, p_leaf=2, with_near=False)
    near = fmm.setup(P, tr8, 80.0, 0.1257, p_leaf=2)
    ref = A @ x
    errs = []
    for p in (2, 4, 6):
        F = fmm.setup(P, tr8, 80.0, 0.1257, p_leaf=p, with_near=False)
        F.near_i, F.near_j, F.near_B = near.near_i, near.near_j, near.near_B
        errs.append(np.linalg.norm(fmm.matvec(F, x) - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
    # far field off + every pair near (eta0 = 0) is the dense operator exactly
    tr0 = otree.build(P, 32, 0.0)
    F0 = fmm.setup(P, tr0, 80.0, 0.1257, p_leaf=2)
    assert np.linalg.norm(fmm.matvec(F0, x) - ref) < 1e-13 * np.linalg.norm(ref)


def test_cluster_radii_tree_pins(sphere1280_dense):
    """Per-cluster radii (the shrink scheme of Sec. 2.4 with the cube centre
    kept), checked from the member panels' own vertices rather than from the
    radii the tree stores: every neighbour pair inadmissible and every
    interaction pair admissible, every leaf pair covered once, panels that
    share a vertex always in neighbouring leaves, the FMM converging to the
    dense operator as p grows, and eta0 = 0 giving the dense operator."""
    P, A = sphere1280_dense
    rng = np.random.default_rng(7)
    x = rng.standard_normal(2 * P.n)
    ref = A @ x
    # panel pairs sharing a vertex
    inc = {}
    for i, tri in enumerate(P.tris):
        for v in tri:
            inc.setdefault(int(v), []).append(i)
    touching = {(a, b) for ps in inc.values() for a in ps for b in ps}
    for leaf_size, eta0 in ((8, 0.8), (4, 0.6)):
        tr = otree.build(P, leaf_size, eta0, radii="cluster")
        assert (fmm.coverage(tr) == 1).all()
        for l in range(1, tr.L + 1):
            cl = tr.levels[l]
            rad = np.array([np.linalg.norm(P.corners[tr.perm[cl.start[c]:cl.end[c]]] - cl.center[c], axis=2).max()
                            for c in range(cl.n)])
            for c in range(cl.n):
                d = np.linalg.norm(cl.center[cl.inter[c]] - cl.center[c], axis=1)
                assert (rad[c] + rad[cl.inter[c]] <= eta0 * d).all()
                nb = cl.nbr[c][cl.nbr[c] != c]
                d = np.linalg.norm(cl.center[nb] - cl.center[c], axis=1)
                assert (rad[c] + rad[nb] > eta0 * d).all()
        leaf = tr.levels[tr.L]
        own = np.empty(P.n, np.int64)
        own[tr.perm] = np.repeat(np.arange(leaf.n), leaf.end - leaf.start)
        nbrs = [set(map(int, leaf.nbr[c])) for c in range(leaf.n)]
        assert all(int(own[b]) in nbrs[own[a]] for a, b in touching)
    tr = otree.build(P, 8, 0.8, radii="cluster")
    near = fmm.setup(P, tr, 80.0, 0.1257, p_leaf=2)
    errs = []
    for p in (2, 4, 6):
        F = fmm.setup(P, tr, 80.0, 0.1257, p_leaf=p, with_near=False)
        F.near_i, F.near_j, F.near_B = near.near_i, near.near_j, near.near_B
        errs.append(np.linalg.norm(fmm.matvec(F, x) - ref) / np.linalg.norm(ref))
    assert errs[1] < 0.5 * errs[0] and errs[2] < 0.5 * errs[1], errs
    tr0 = otree.build(P, 32, 0.0, radii="cluster")
    F0 = fmm.setup(P, tr0, 80.0, 0.1257, p_leaf=2)
    assert np.linalg.norm(fmm.matvec(F0, x) - ref) < 1e-13 * np.linalg.norm(ref)


def test_gmres_matches_direct_solve():
    rng = np.random.default_rng(6)
    A = np.eye(40) * 3 + rng.standard_normal((40, 40)) * 0.2
    b = rng.standard_normal(40)
    x, it, _ = solve.gmres(lambda z: A @ z, b, 1e-12, 40)
    assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)
    D = np.diag(A)
    x2, it2, _ = solve.gmres(lambda z: A @ z, b, 1e-12, 40, precond=lambda z: z / D)
    assert np.allclose(x2, np.linalg.solve(A, b), rtol=1e-9, atol=1e-11)


def _close_panels():
    """three mutually non-touching, non-coplanar triangles at 1.5-2.5 h"""
    verts = np.array([[0, 0, 0], [1.0, 0, 0], [0.4, 0.8, 0.1],
                      [1.25, 0.1, 0.05], [2.0, 0.6, 0.3], [1.3, 0.9, -0.15],
                      [0.2, -0.35, 0.0], [1.1, -0.5, 0.2], [0.6, -1.2, -0.1]])
    return panels(verts, np.array([[0, 1, 2], [3, 4, 5], [7, 6, 8]]))


@pytest.mark.parametrize("pair", [(0, 1), (0, 2), (1, 0)])
def test_close_rule_matches_closed_forms(pair):
    """The close-pair rule (Duffy-collapsed Gauss rule on both triangles)
    against the Wilton single-layer and Van Oosterom-Strackee double-layer
    closed forms integrated over the target by a fine composite rule: the
    pairs are closer than 2 h, so the rule's class is CLOSE, and the error
    falls geometrically with n."""
    P = _close_panels()
    i, j = np.array([pair[0]]), np.array([pair[1]])
    assert pairs.classify(P, i, j, 2.0)[0] == pairs.CLOSE
    s, d = _reference(P, pair[0], pair[1])
    err = {}
    for n in (3, 5, 7):
        I = pairs.close(P, i, j, 0.0, n, kern=_g0_kernels)[0]
        err[n] = (abs(I[0] - s) / abs(s), abs(I[1] - d) / abs(d))
    assert err[7][0] < 1e-8 and err[7][1] < 1e-6, err
    assert err[7][0] < 1e-2 * err[3][0] and err[7][1] < 1e-2 * err[3][1], err


def test_touching_and_close_rules_symmetric_under_swap(sphere320):
    """The rules applied with the two panels exchanged (no mirroring) give the
    transposed integrals to the rules' own accuracy: I1, I6 symmetric,
    I2 <-> I4 and I3 <-> I5 (the kernels depend on x - y only).  The mirrored
    values the oracle stores are therefore the integrals of either order."""
    P, _ = sphere320
    kap = 0.1257
    swap = [0, 3, 4, 1, 2, 5]
    tris = P.tris
    sh = (tris[:, None, :, None] == tris[None, :, None, :]).any(3).sum(2)
    for rule, cnt, tol in ((pairs.edge, 2, 1e-8), (pairs.vertex, 1, 1e-8)):
        ii, jj = np.nonzero(sh == cnt)
        ii, jj = ii[:40], jj[:40]
        a = rule(P, ii, jj, kap, 7)
        b = rule(P, jj, ii, kap, 7)[:, swap]
        scale = np.abs(a).max(0)
        assert (np.abs(a - b) / scale).max() < tol
    Pc = _close_panels()
    a = pairs.close(Pc, np.array([0, 0]), np.array([1, 2]), kap, 7)
    b = pairs.close(Pc, np.array([1, 2]), np.array([0, 0]), kap, 7)[:, swap]
    assert (np.abs(a - b) / np.abs(a).max(0)).max() < 1e-12


def _precond_matrix(Minv, n2):
    """the matrix M of a preconditioner from its inverse's columns"""
    Mi = np.stack([Minv(np.eye(n2)[k]) for k in range(n2)], 1)
    return np.linalg.inv(Mi)


def test_block_preconditioner_pins():
    """Sec. 2.6 block-diagonal preconditioner against the dense operator A:
    (1) one leaf holding every panel with eta0 = 0: M = A, so M^{-1} A x = x;
    (2) leaf blocks: M_ij = A_ij for panels of one leaf (in both unknown
        blocks, identity terms included), 0 elsewhere;
    (3) groups of consecutive leaves (tree order) of at most 32 panels: M_ij =
        A_ij for panels of one group whose leaves are neighbours, 0 elsewhere,
        and each group is maximal (the next leaf would exceed 32 panels)."""
    v, t = icosphere(1, 2.0)
    P = panels(v, t)
    N = P.n
    eps, kap = 80.0, 0.1257
    A = dense.assemble(P, eps, kap)
    x = np.random.default_rng(8).standard_normal(2 * N)
    one = otree.build(P, N, 0.0)
    assert one.L == 0
    Minv = solve.block_preconditioner(P, one, eps, kap)
    assert np.linalg.norm(Minv(A @ x) - x) < 1e-12 * np.linalg.norm(x)
    tr = otree.build(P, 8, 0.8)
    leaf = tr.levels[tr.L]
    lf = np.empty(N, np.int64)
    lf[tr.perm] = np.repeat(np.arange(leaf.n), leaf.end - leaf.start)
    same2 = lambda m: np.block([[m, m], [m, m]])
    M = _precond_matrix(solve.block_preconditioner(P, tr, eps, kap), 2 * N)
    keep = same2(lf[:, None] == lf[None, :])
    scale = np.abs(A).max()
    assert np.abs(M[keep] - A[keep]).max() < 1e-13 * scale
    assert np.abs(M[~keep]).max() < 1e-13 * scale
    # groups: greedy runs of consecutive leaves up to 32 panels
    sizes = leaf.end - leaf.start
    grp, g, cnt = np.empty(leaf.n, np.int64), 0, 0
    for c in range(leaf.n):
        if cnt and cnt + sizes[c] > 32:
            g, cnt = g + 1, 0
        grp[c] = g
        cnt += sizes[c]
    for k in range(g):       # maximal: the next group's first leaf does not fit
        assert sizes[grp == k].sum() + sizes[np.nonzero(grp == k + 1)[0][0]] > 32
    nb = np.zeros((leaf.n, leaf.n), bool)
    for c in range(leaf.n):
        nb[c, leaf.nbr[c]] = True
    M = _precond_matrix(solve.block_preconditioner(P, tr, eps, kap, group_max=32), 2 * N)
    keep = same2((grp[lf][:, None] == grp[lf][None, :]) & nb[lf][:, lf])
    assert np.abs(M[keep] - A[keep]).max() < 1e-13 * scale
    assert np.abs(M[~keep]).max() < 1e-13 * scale
    assert (grp[lf][:, None] == grp[lf][None, :]).sum() > (lf[:, None] == lf[None, :]).sum()


def test_far_field_rows_equal_far_field():
    """The restricted far field (ancestor chains of a few leaves) equals the
    full far field at those panels, at adaptive orders 5..8."""
    v, t = icosphere(3, 2.0)
    P = panels(v, t)
    tr = otree.build(P, 4, 0.8)
    O = fmm.setup(P, tr, 80.0, 0.1257, p_leaf=5, adaptive=1, p_max=8, with_near=False)
    x = np.random.default_rng(9).standard_normal(2 * P.n)
    f1, f2 = fmm.far_field(O, x[:P.n], x[P.n:])
    leaves = np.random.default_rng(10).choice(tr.levels[tr.L].n, 10, replace=False)
    ids, g1, g2 = fmm.far_field_rows(O, x[:P.n], x[P.n:], leaves)
    assert len(ids) == (tr.levels[tr.L].end - tr.levels[tr.L].start)[leaves].sum()
    assert np.abs(g1 - f1[ids]).max() < 1e-13 * np.abs(f1).max()
    assert np.abs(g2 - f2[ids]).max() < 1e-13 * np.abs(f2).max()
