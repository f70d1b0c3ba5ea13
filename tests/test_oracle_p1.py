"""Pins of the oracle's piecewise-linear (hat-function) discretisation against
things other than itself: the box-function integrals (hat functions sum to
one on a panel), closed forms of the single- and double-layer potentials of a
flat triangle with a hat-function weight on the outer panel, brute-force
cubature of the smooth kernel, Gauss's double-layer identity, the dense
operator, and the analytic Kirkwood sphere (the projection rates of Sec. 2.3:
O(h^2) for S^1_h against O(h) for the box functions).  CPU only."""
import numpy as np
import pytest

from analytic import composite_outer, potential_1_over_r, solid_angle
from oracle import dense, kirkwood, p1, pairs, solve
from oracle import tree as otree
from oracle.geometry import panels
from synth import icosphere, isosurface_mesh, packed_atoms_ball


def _three_panels():
    verts = np.array([[0, 0, 0], [1.0, 0, 0], [0.4, 0.8, 0.1], [0.5, -0.7, 0.3],
                      [-0.6, 0.5, -0.2]])
    tris = np.array([[0, 1, 2], [1, 0, 3], [0, 4, 2]])
    return panels(verts, tris)


def _g0_kernels(r, nx, ny, kappa):
    rr = np.sqrt((r * r).sum(-1))
    return np.stack([1.0 / (4 * np.pi * rr), (r * ny).sum(-1) / (4 * np.pi * rr ** 3)], -1)


def _bary(tri, pts):
    """barycentric coordinates of points in the plane of a triangle"""
    T = np.stack([tri[1] - tri[0], tri[2] - tri[0]], 1)
    c, *_ = np.linalg.lstsq(T, (pts - tri[0]).T, rcond=None)
    return np.stack([1 - c[0] - c[1], c[0], c[1]], 1)


def _weighted_closed_forms(P, i, j):
    """int_{tau_i} lambda_a(x) [S_j(x), D_j(x)] dx for a = 0..2, with S_j, D_j
    the single- and double-layer potentials of panel j in closed form (outer
    composite rule, Richardson over two refinements)"""
    vals = []
    for lev in (4, 5):
        pts, w = composite_outer(P.corners[i], lev, 8)
        lam = _bary(P.corners[i], pts)
        s = (w[:, None] * lam * potential_1_over_r(pts, P.corners[j])[:, None]).sum(0) / (4 * np.pi)
        d = -(w[:, None] * lam * solid_angle(pts, P.corners[j])[:, None]).sum(0) / (4 * np.pi)
        vals.append((s, d))
    (s4, d4), (s5, d5) = vals
    return s5 + (s5 - s4) / 3.0, d5 + (d5 - d4) / 3.0


def test_corner_sums_reproduce_box_integrals():
    """sum_ab J[a, b] = the box-function integral of the same pair, every class"""
    x, r, q = packed_atoms_ball(n=16, radius=None, seed=11)
    v, t = isosurface_mesh(x, r, spacing=1.0)
    P = panels(v, t)
    rng = np.random.default_rng(0)
    ii = list(rng.integers(0, P.n, 600))
    jj = list(rng.integers(0, P.n, 600))
    at = {}
    for k in range(P.n):
        for vv in P.tris[k]:
            at.setdefault(int(vv), []).append(k)
    for vv in list(at)[:40]:
        for a in at[vv]:
            for b in at[vv]:
                ii.append(a)
                jj.append(b)
    ii, jj = np.array(ii), np.array(jj)
    J, cls = p1.pair_integrals(P, ii, jj, 0.1257, 2.0, 7)
    I, cls0 = pairs.pair_integrals(P, ii, jj, 0.1257, 2.0, 7)
    assert np.array_equal(cls, cls0)
    S = J.sum((1, 2))
    for c in range(5):
        sel = cls == c
        assert sel.sum() > 0, c
        scale = np.abs(I[sel]).max(0)
        scale[scale == 0] = 1.0
        assert (np.abs(S[sel] - I[sel]).max(0) / scale).max() < 1e-13, c


@pytest.mark.parametrize("i,j,rule", [(0, 0, "ident"), (0, 1, "edge"), (1, 0, "edge"), (0, 2, "edge"),
                                      (2, 0, "edge"), (1, 2, "vertex"), (2, 1, "vertex")])
def test_hat_weighted_sides_match_closed_forms(i, j, rule):
    """sum_b J[a, b] (test side: hat function a on panel i, unit density on
    panel j) and sum_a J[a, b] (trial side) of the Laplace single layer, and
    the test side of the double layer, against the closed-form potentials"""
    P = _three_panels()
    a, b = np.array([i]), np.array([j])
    if rule == "ident":
        J = p1.ident(P, a, 0.0, 7, kern=_g0_kernels)[0]
    else:
        J = getattr(p1, rule)(P, a, b, 0.0, 7, kern=_g0_kernels)[0]
    s, d = _weighted_closed_forms(P, i, j)
    st, _ = _weighted_closed_forms(P, j, i)
    assert np.abs(J[:, :, 0].sum(1) - s).max() < 5e-8 * np.abs(s).max()
    assert np.abs(J[:, :, 0].sum(0) - st).max() < 5e-8 * np.abs(st).max()
    if rule != "ident":      # the solid angle is two-valued on the panel itself
        assert np.abs(J[:, :, 1].sum(1) - d).max() < 1e-6 * np.abs(d).max()


def _brute_smooth(P, i, j, kappa, lev):
    """int int lambda_a(x) (G0 - Gk)(x, y) lambda_b(y) by a composite rule on
    both panels (the kernel is continuous, kappa / 4 pi at r = 0)"""
    px, wx = composite_outer(P.corners[i], lev, 4)
    py, wy = composite_outer(P.corners[j], lev, 4)
    lx, ly = _bary(P.corners[i], px), _bary(P.corners[j], py)
    out = np.zeros((3, 3))
    for s in range(0, len(px), 512):
        r = px[s:s + 512, None, :] - py[None, :, :]
        rr = np.sqrt((r * r).sum(-1))
        safe = np.where(rr > 0, rr, 1.0)
        k = np.where(rr > 0, -np.expm1(-kappa * safe) / (4 * np.pi * safe), kappa / (4 * np.pi))
        out += np.einsum("x,xa,xy,y,yb->ab", wx[s:s + 512], lx[s:s + 512], k, wy, ly)
    return out


@pytest.mark.parametrize("i,j,rule,tol", [(0, 0, "ident", 5e-6), (0, 1, "edge", 1e-8), (1, 2, "vertex", 1e-8)])
def test_corner_split_of_touching_rules_brute_force(i, j, rule, tol):
    """the whole 3 x 3 corner split of the smooth channel G0 - Gk"""
    P = _three_panels()
    kappa = 1.0
    a, b = np.array([i]), np.array([j])
    J = (p1.ident(P, a, kappa, 7) if rule == "ident" else getattr(p1, rule)(P, a, b, kappa, 7))[0, :, :, 0]
    ref = _brute_smooth(P, i, j, kappa, 4)
    assert np.abs(J - ref).max() < tol * np.abs(J).max()


def test_close_and_regular_corner_integrals_brute_force():
    """all six kernels with the hat-function weights, for a close and a
    regular (well separated) pair, against a fine product rule"""
    v = np.array([[0, 0, 0], [1.0, 0, 0], [0.3, 0.9, 0.2], [0.4, 0.3, 1.1], [1.3, 0.5, 1.0], [0.6, 1.2, 1.4],
                  [4.0, 0.2, 0.5], [4.8, 0.9, 0.3], [4.1, 1.1, 1.2]])
    t = np.array([[0, 1, 2], [3, 4, 5], [6, 7, 8]])
    P = panels(v, t)
    kappa = 0.4
    from oracle.kernels import kernel6
    for (i, j, rule) in ((0, 1, "close"), (0, 2, "regular")):
        a, b = np.array([i]), np.array([j])
        J = (p1.close(P, a, b, kappa, 7) if rule == "close" else p1.regular(P, a, b, kappa))[0]
        px, wx = composite_outer(P.corners[i], 3, 6)
        py, wy = composite_outer(P.corners[j], 3, 6)
        lx, ly = _bary(P.corners[i], px), _bary(P.corners[j], py)
        K = kernel6(px[:, None, :] - py[None, :, :], P.normal[i], P.normal[j], kappa)
        ref = np.einsum("x,xa,xym,y,yb->abm", wx, lx, K, wy, ly)
        # the n = 7 Duffy rule reaches 5.5e-9 here (5e-13 with n = 10); the 3 x 3
        # regular rule at 5.8 h about 6e-4
        tol = 2e-8 if rule == "close" else 5e-3
        assert np.abs(J - ref).max() < tol * np.abs(ref).max(), rule


@pytest.fixture(scope="module")
def sphere320_p1():
    v, t = icosphere(2, 2.0)
    P = panels(v, t)
    N = P.n
    ii, jj = np.repeat(np.arange(N), N), np.tile(np.arange(N), N)
    J, _ = p1.pair_integrals(P, ii, jj, 0.1257, 2.0, 7)
    return P, J.reshape(N, N, 3, 3, 6)


def test_gauss_identity_and_mass(sphere320_p1):
    """int phi_i(x) int_S dG0/dn_y = -1/2 int phi_i on a closed polyhedron, test
    side (I2) and trial side (I4, with dG0/dn_x); mass matrix row sums"""
    P, J = sphere320_p1
    test = J[..., 1].sum((1, 3))          # [panel, corner a]
    trial = J[..., 3].sum((0, 2))         # [panel, corner b]
    # int lambda_a = A / 3 per corner
    assert np.abs(test / (P.area[:, None] / 3.0) + 0.5).max() < 2e-3
    assert np.abs(trial / (P.area[:, None] / 3.0) + 0.5).max() < 2e-3
    V = len(P.verts)
    u = np.ones(V)
    lumped = np.zeros(V)
    np.add.at(lumped, P.tris, np.repeat(P.area[:, None] / 3.0, 3, 1))
    assert np.allclose(p1.mass_matvec(P, u), lumped, rtol=1e-14, atol=0)


def test_dense_operator_from_corner_integrals(sphere320_p1):
    """the dense hat-function matrix against the corner integrals gathered by
    hand for a few vertex pairs"""
    P, J = sphere320_p1
    eps, kappa = 80.0, 0.1257
    A = p1.assemble(P, eps, kappa)
    V = len(P.verts)
    Mb = p1.mass_diag_blocks(P)
    rng = np.random.default_rng(5)
    for vi, vj in zip(rng.integers(0, V, 6), list(rng.integers(0, V, 5)) + [0]):
        ref = np.zeros((2, 2))
        for s in range(P.n):
            for a in range(3):
                if P.tris[s, a] != vi:
                    continue
                for s2 in range(P.n):
                    for b in range(3):
                        if P.tris[s2, b] != vj:
                            continue
                        I = J[s, s2, a, b]
                        ref += np.array([[-(eps * I[2] - I[1]), -I[0]], [-I[5], -(I[3] - I[4] / eps)]])
                        if s == s2:
                            ref += np.diag([0.5 * (1 + eps), 0.5 * (1 + 1 / eps)]) * Mb[s, a, b]
        got = np.array([[A[vi, vj], A[vi, V + vj]], [A[V + vi, vj], A[V + vi, V + vj]]])
        assert np.abs(got - ref).max() < 1e-13 * np.abs(ref).max()


def _kirkwood_case():
    R, e1, e2, kap = 2.0, 1.0, 80.0, 0.1257
    xq = np.array([[0.0, 0.0, 0.9], [0.7, -0.3, -0.5], [-0.4, 0.6, 0.2]])
    q = np.array([1.0, -0.7, 0.5])
    return R, e1, e2, kap, xq, q


def _kirkwood_surface_potential(x, R, e1, e2, kap, xq, q, nmax=60):
    """interior potential on the sphere |x| = R (at the radial projection of
    x), in the units of the discrete unknowns (the Coulomb part is
    q / (4 pi eps1 r)): the series of ``kirkwood`` evaluated at r = R"""
    C = kirkwood.reaction_factors(R, e1, e2, kap, nmax)
    xs = R * x / np.linalg.norm(x, axis=-1, keepdims=True)
    out = np.zeros(xs.shape[:-1])
    for k in range(len(q)):
        rk = np.linalg.norm(xq[k])
        d = np.linalg.norm(xs - xq[k], axis=-1)
        Pn = kirkwood.legendre(nmax, (xs @ xq[k]) / (R * rk))
        s = sum(C[n] * (rk / R) ** n * Pn[n] for n in range(nmax + 1))
        out += q[k] / (4 * np.pi * e1) * (1.0 / d + s / R)
    return out


def test_kirkwood_projection_rates():
    """On the Kirkwood sphere with three off-centre charges: the L2 error of
    the surface potential falls like h^2 with hat functions and like h with
    box functions (Sec. 2.3), and both energies converge to the series."""
    R, e1, e2, kap, xq, q = _kirkwood_case()
    eps = e2 / e1
    Eref = kirkwood.energy(xq, q, R, e1, e2, kap)
    err1, err0, eE1 = [], [], []
    for lev in (1, 2):
        v, t = icosphere(lev, R)
        P = panels(v, t)
        V = len(v)
        x1 = np.linalg.solve(p1.assemble(P, eps, kap), p1.rhs(P, xq, q, e1))
        x0 = np.linalg.solve(dense.assemble(P, eps, kap), solve.rhs(P, xq, q, e1))
        ex = _kirkwood_surface_potential(P.qp, R, e1, e2, kap, xq, q)
        nrm = np.sqrt((P.qw * ex ** 2).sum())
        u1 = np.einsum("ka,pa->pk", p1.LAM, x1[:V][P.tris])
        err1.append(np.sqrt((P.qw * (u1 - ex) ** 2).sum()) / nrm)
        err0.append(np.sqrt((P.qw * (x0[:P.n, None] - ex) ** 2).sum()) / nrm)
        eE1.append(abs(p1.energy(P, x1, xq, q, eps, kap) - Eref) / abs(Eref))
    print("L2 errors hat %s, box %s; energy errors hat %s" % (err1, err0, eE1))
    assert err1[0] / err1[1] > 3.5          # O(h^2): h halves per level
    assert err0[0] / err0[1] < 2.6          # O(h)
    assert err1[1] < 0.35 * err0[1]
    assert eE1[0] / eE1[1] > 3.5 and eE1[1] < 0.03


def test_fmm_converges_to_dense_operator():
    v, t = icosphere(2, 2.0)
    P = panels(v, t)
    eps, kap = 80.0, 0.1257
    A = p1.assemble(P, eps, kap)
    rng = np.random.default_rng(3)
    x = rng.standard_normal(2 * len(v))
    ref = A @ x
    errs = []
    for pl in (2, 4, 6):
        F = p1.setup(P, otree.build(P, 8, 0.8), eps, kap, p_leaf=pl)
        errs.append(np.linalg.norm(p1.matvec(F, x) - ref) / np.linalg.norm(ref))
    assert errs[0] > 2 * errs[1] > 4 * errs[2] and errs[2] < 1e-3, errs
    # everything near: the FMM operator is the dense one
    F = p1.setup(P, otree.build(P, 8, 0.0), eps, kap, p_leaf=4)
    assert np.linalg.norm(p1.matvec(F, x) - ref) < 1e-13 * np.linalg.norm(ref)
    # the Jacobi divisors are the dense diagonal
    assert np.abs(p1.diagonal(F) - np.diag(A)).max() < 1e-13 * np.abs(np.diag(A)).max()


def test_hat_treecodes():
    """Treecode energy and RHS with hat functions (Sec. 2.5): theta = 0 gives the
    direct sums; the error falls with theta for smooth nodal values; constant
    nodal values give the box-function treecode's energy and the same total
    right-hand side (the hat functions of a panel sum to one)."""
    from oracle import fmm, treecode
    x_, r_, q_ = packed_atoms_ball(n=16, radius=None, seed=11)
    v, t = isosurface_mesh(x_, r_, spacing=1.0)
    P = panels(v, t)
    V = len(v)
    tr = otree.build(P, 16, 0.8)
    F1 = p1.setup(P, tr, 80.0, 0.1257, p_leaf=4, adaptive=1, p_max=8, with_near=False)
    c = v.mean(0)
    u = np.cos(0.3 * (v - c) @ np.array([1.0, 0.5, -0.2]))
    w = np.sin(0.25 * (v - c) @ np.array([-0.3, 1.0, 0.4]))
    x = np.concatenate([u, w])
    Ed = p1.energy(P, x, x_, q_, 80.0, 0.1257)
    bd = p1.rhs(P, x_, q_, 1.0)
    assert abs(p1.treecode_energy(F1, x, x_, q_, 0.0) - Ed) < 1e-13 * abs(Ed)
    assert np.linalg.norm(p1.treecode_rhs(F1, x_, q_, 0.0, 1.0) - bd) < 1e-13 * np.linalg.norm(bd)
    eE = [abs(p1.treecode_energy(F1, x, x_, q_, th) - Ed) / abs(Ed) for th in (0.7, 0.5, 0.3)]
    eb = [np.linalg.norm(p1.treecode_rhs(F1, x_, q_, th, 1.0) - bd) / np.linalg.norm(bd) for th in (0.7, 0.5, 0.3)]
    print("hat treecode energy errors %s, rhs errors %s" % (eE, eb))
    assert eE[0] > eE[1] > eE[2] and eE[2] < 5e-5
    assert eb[0] > eb[1] > eb[2] and eb[2] < 1e-4
    F0 = fmm.setup(P, tr, 80.0, 0.1257, p_leaf=4, adaptive=1, p_max=8, with_near=False)
    for c1, c2 in ((1.0, 0.0), (0.3, -0.8)):
        xh = np.concatenate([np.full(V, c1), np.full(V, c2)])
        xb = np.concatenate([np.full(P.n, c1), np.full(P.n, c2)])
        Eh = p1.treecode_energy(F1, xh, x_, q_, 0.5, p_max=6)
        Eb = treecode.energy(F0, xb, x_, q_, 0.5, p_max=6)
        assert abs(Eh - Eb) < 1e-12 * abs(Eb), (Eh, Eb)
    bh = p1.treecode_rhs(F1, x_, q_, 0.5, 1.0, p_max=6)
    bb = treecode.rhs(F0, x_, q_, 0.5, 1.0, p_max=6)
    for ch in range(2):
        sh, sb = bh[ch * V:(ch + 1) * V].sum(), bb[ch * P.n:(ch + 1) * P.n].sum()
        assert abs(sh - sb) < 1e-12 * np.abs(bb[ch * P.n:(ch + 1) * P.n]).sum()
