"""The continuous piecewise-linear basis (FAGBI_BASIS_S1, hat functions at the
vertices; Sec. 2.3) against the oracle's hat-function discretisation.

* the operator: FP64 to 1e-11 and FP32 to 1e-6 (relative L2 and largest row),
  near part (with the mass terms) and far part separately, on the icosphere
  and on an irregular isosurface globule with close pairs (one tree with
  per-cluster radii);
* the right-hand side and the energy to 1e-12, the Jacobi divisors to 1e-12;
* solves: with every pair near (eta0 = 0) the GPU solution equals the oracle's
  dense solve; on the Kirkwood sphere the surface potential's L2 error falls
  like h^2 (against h with box functions) and the FP32-inner solve agrees with
  the FP64 one;
* the treecode energy and RHS with hat functions against the oracle's;
* error paths of the parameters the basis excludes."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import dense, kirkwood, p1  # noqa: E402
from oracle import solve as osolve  # noqa: E402
from oracle import tree as otree  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere, isosurface_mesh, packed_atoms_ball  # noqa: E402

pytestmark = pytest.mark.gpu
EPS, KAP = 80.0, 0.1257
DEV = "cuda:0"
HAT = F.BASIS_S1


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def maxrow(a, b):
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def gpu_matvec(h, x, precision=F.FP64, parts=F.PART_ALL):
    xd = dev(x)
    y = torch.empty_like(xd)
    h.matvec(xd, y, precision, parts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.fixture(scope="module")
def sphere1280():
    v, t = icosphere(3, 2.0)
    return v, t, panels(v, t)


@pytest.fixture(scope="module")
def globule():
    x, r, q = packed_atoms_ball(n=16, radius=None, seed=11)
    v, t = isosurface_mesh(x, r, spacing=1.0)     # 2,388 panels with close pairs
    return v, t, panels(v, t)


@pytest.mark.parametrize("mesh,cfg", [
    ("sphere", dict(leaf_size=8, p_leaf=3, adaptive=1, p_max=6)),
    ("globule", dict(leaf_size=16, p_leaf=4, adaptive=0, quad_duffy=4)),
    ("globule", dict(leaf_size=4, p_leaf=3, adaptive=1, p_max=8, quad_duffy=4)),
    ("globule", dict(leaf_size=8, p_leaf=3, adaptive=1, p_max=8, quad_duffy=4, radii=F.RADII_CLUSTER)),
])
def test_hat_operator_matches_oracle(sphere1280, globule, mesh, cfg):
    v, t, P = sphere1280 if mesh == "sphere" else globule
    h = F.Handle(eta0=0.8, basis=HAT, precond=F.PRECOND_DIAG, **cfg).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, cfg["leaf_size"], 0.8, radii="cluster" if cfg.get("radii") else "level")
    O = p1.setup(P, tr, EPS, KAP, p_leaf=cfg["p_leaf"], adaptive=cfg["adaptive"], p_max=cfg.get("p_max", 8),
                 n_duffy=cfg.get("quad_duffy", 7))
    V = len(v)
    rng = np.random.default_rng(21)
    x = rng.standard_normal(2 * V)
    ref = p1.matvec(O, x)
    y64, y32 = gpu_matvec(h, x), gpu_matvec(h, x, F.MIXED)
    print("%s %s: %d vertices, fp64 %.2e / %.2e, fp32 %.2e / %.2e"
          % (mesh, cfg, V, rel(y64, ref), maxrow(y64, ref), rel(y32, ref), maxrow(y32, ref)))
    assert rel(y64, ref) < 1e-11 and maxrow(y64, ref) < 1e-11
    assert rel(y32, ref) < 1e-6 and maxrow(y32, ref) < 1e-6
    assert rel(gpu_matvec(h, x, parts=F.PART_NEAR), p1.matvec(O, x, far=False)) < 1e-11
    assert rel(gpu_matvec(h, x, parts=F.PART_FAR), np.concatenate(p1.far_field(O, x[:V], x[V:]))) < 1e-11
    # Jacobi divisors
    z = rng.standard_normal(2 * V)
    y = torch.empty(2 * V, dtype=torch.float64, device=DEV)
    h.precond_apply(dev(z), y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), z / p1.diagonal(O)) < 1e-12
    h.close()


def test_hat_rhs_and_energy(globule):
    v, t, P = globule
    V = len(v)
    x_, r_, q_ = packed_atoms_ball(n=16, radius=None, seed=11)
    h = F.Handle(leaf_size=16, basis=HAT, precond=F.PRECOND_DIAG, quad_duffy=4).build_tree(v, t)
    h.assemble_nearfield()
    b = torch.empty(2 * V, dtype=torch.float64, device=DEV)
    h.rhs(x_, q_, b)
    torch.cuda.synchronize()
    ref = p1.rhs(P, x_, q_, 1.0)
    assert rel(b.cpu().numpy(), ref) < 1e-12 and maxrow(b.cpu().numpy(), ref) < 1e-12
    rng = np.random.default_rng(4)
    x = rng.standard_normal(2 * V)
    E = h.solvation_energy(dev(x), x_, q_)
    Eref = p1.energy(P, x, x_, q_, EPS, KAP)
    assert abs(E - Eref) < 1e-12 * abs(Eref)
    h.close()


def _kirkwood_case():
    R, e1, e2, kap = 2.0, 1.0, 80.0, 0.1257
    xq = np.array([[0.0, 0.0, 0.9], [0.7, -0.3, -0.5], [-0.4, 0.6, 0.2]])
    q = np.array([1.0, -0.7, 0.5])
    return R, e1, e2, kap, xq, q


def test_hat_solve_equals_dense_oracle():
    """every pair near (eta0 = 0): the GPU operator is the dense matrix, and the
    FP64 solve to 1e-12 reproduces the oracle's direct solve and energy"""
    R, e1, e2, kap, xq, q = _kirkwood_case()
    v, t = icosphere(2, R)
    P = panels(v, t)
    V = len(v)
    A = p1.assemble(P, e2 / e1, kap)
    b = p1.rhs(P, xq, q, e1)
    xref = np.linalg.solve(A, b)
    Eref = p1.energy(P, xref, xq, q, e2 / e1, kap)
    h = F.Handle(eps_in=e1, eps_out=e2, kappa=kap, eta0=0.0, leaf_size=8, basis=HAT,
                 precond=F.PRECOND_DIAG, tol=1e-12, max_iter=300)
    h.build_tree(v, t).assemble_nearfield()
    rng = np.random.default_rng(2)
    z = rng.standard_normal(2 * V)
    assert rel(gpu_matvec(h, z), A @ z) < 1e-12
    x = torch.zeros(2 * V, dtype=torch.float64, device=DEV)
    code, info = h.solve(xq, q, x)
    assert code == 0 and info.rel_residual <= 1e-12
    E = h.solvation_energy(x, xq, q)
    print("dense hat system: %d iterations, solution rel diff %.2e, energy %.10f vs %.10f"
          % (info.inner_iterations, rel(x.cpu().numpy(), xref), E, Eref))
    assert rel(x.cpu().numpy(), xref) < 1e-10
    assert abs(E - Eref) < 1e-10 * abs(Eref)
    h.close()


def _surface_potential(pts, R, e1, e2, kap, xq, q, nmax=60):
    C = kirkwood.reaction_factors(R, e1, e2, kap, nmax)
    xs = R * pts / np.linalg.norm(pts, axis=-1, keepdims=True)
    out = np.zeros(xs.shape[:-1])
    for k in range(len(q)):
        rk = np.linalg.norm(xq[k])
        d = np.linalg.norm(xs - xq[k], axis=-1)
        Pn = kirkwood.legendre(nmax, (xs @ xq[k]) / (R * rk))
        out += q[k] / (4 * np.pi * e1) * (1.0 / d + sum(C[n] * (rk / R) ** n * Pn[n] for n in range(nmax + 1)) / R)
    return out


def test_hat_kirkwood_projection_rates_on_gpu():
    """FMM solves on the Kirkwood sphere at 320 / 1,280 / 5,120 panels: the
    surface potential's L2 error falls like h^2 with hat functions and like h
    with box functions; the energies converge to the series; the FP32-inner
    solve agrees with the FP64 one.  The expansions (order 7 at the leaves,
    eta0 0.6) keep the FMM's error far below the discretisation's (with order
    4 at eta0 0.8 the hat error levels off near 1e-3 from 5,120 panels on)."""
    R, e1, e2, kap, xq, q = _kirkwood_case()
    Eref = kirkwood.energy(xq, q, R, e1, e2, kap)
    prm = dict(eps_in=e1, eps_out=e2, kappa=kap, leaf_size=16, eta0=0.6, p_leaf=7, adaptive=1, p_max=8,
               tol=1e-8, max_iter=300, inner_tol=5e-9)
    e_hat, e_box, E_hat = [], [], []
    for lev in (2, 3, 4):
        v, t = icosphere(lev, R)
        P = panels(v, t)
        V, N = len(v), len(t)
        ex = _surface_potential(P.qp, R, e1, e2, kap, xq, q)
        nrm = np.sqrt((P.qw * ex ** 2).sum())
        sol = {}
        for basis, prec, pc in ((HAT, F.FP64, F.PRECOND_DIAG), (HAT, F.MIXED, F.PRECOND_DIAG),
                                (F.BASIS_S0, F.FP64, F.PRECOND_BLOCK)):
            print("solve: %d panels, basis %d, precision %d" % (N, basis, prec), flush=True)
            h = F.Handle(basis=basis, precision=prec, precond=pc, **prm).build_tree(v, t).assemble_nearfield()
            n = V if basis == HAT else N
            x = torch.zeros(2 * n, dtype=torch.float64, device=DEV)
            code, info = h.solve(xq, q, x)
            assert code == 0, (basis, prec)
            sol[(basis, prec)] = (x.cpu().numpy(), h.solvation_energy(x, xq, q), info.inner_iterations)
            h.close()
        xh, Eh, ith = sol[(HAT, F.FP64)]
        xb, Eb, itb = sol[(F.BASIS_S0, F.FP64)]
        uh = np.einsum("ka,pa->pk", p1.LAM, xh[:V][P.tris])
        e_hat.append(np.sqrt((P.qw * (uh - ex) ** 2).sum()) / nrm)
        e_box.append(np.sqrt((P.qw * (xb[:N, None] - ex) ** 2).sum()) / nrm)
        E_hat.append(abs(Eh - Eref) / abs(Eref))
        Em = sol[(HAT, F.MIXED)][1]
        print("%d panels: L2 hat %.3e box %.3e, energy hat %.6f box %.6f series %.6f (mixed %.6f), "
              "iterations hat %d box %d" % (N, e_hat[-1], e_box[-1], Eh, Eb, Eref, Em, ith, itb))
        assert abs(Em - Eh) < 1e-7 * abs(Eh)
    assert e_hat[0] / e_hat[1] > 3.5 and e_hat[1] / e_hat[2] > 3.5
    assert e_box[0] / e_box[1] < 2.6 and e_box[1] / e_box[2] < 2.6
    assert e_hat[2] < 0.2 * e_box[2]
    assert E_hat[0] / E_hat[1] > 3.5 and E_hat[1] / E_hat[2] > 3.5


def test_hat_error_paths(sphere1280):
    v, t, P = sphere1280
    for kw in (dict(mlp_mode=F.MLP_GATED), dict(precond=F.PRECOND_BLOCK), dict(precond=F.PRECOND_GROUP),
               dict(basis=2)):
        args = dict(basis=HAT, precond=F.PRECOND_DIAG)
        args.update(kw)
        with pytest.raises(F.FagbiError) as e:
            F.Handle(**args)
        assert e.value.code == -1, kw
    # a vertex on no triangle carries a hat function of zero support
    v2 = np.vstack([v, [[10.0, 0.0, 0.0]]])
    with pytest.raises(F.FagbiError) as e:
        F.Handle(basis=HAT, precond=F.PRECOND_DIAG).build_tree(v2, t)
    assert e.value.code == -2
    h = F.Handle(basis=HAT, precond=F.PRECOND_DIAG).build_tree(v, t)
    b = torch.zeros(2 * len(v), dtype=torch.float64, device=DEV)
    with pytest.raises(F.FagbiError) as e:      # before the assembly
        h.rhs(np.zeros((1, 3)), np.ones(1), b)
    assert e.value.code == -3
    h.assemble_nearfield()
    x = torch.zeros(2 * len(v), dtype=torch.float64, device=DEV)
    chg = torch.zeros((1, 4), dtype=torch.float64, device=DEV)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    with pytest.raises(F.FagbiError) as e:      # the allocation-free energy is box-only
        h.solvation_energy_noalloc(x, chg, E)
    assert e.value.code == -1
    h.close()


def test_hat_treecodes_match_oracle(globule):
    """treecode energy and RHS with hat functions (theta 0.5, order cap 6, and
    theta 0 = the direct sums) against the oracle's hat treecodes, and a solve
    with the treecode right-hand side"""
    v, t, P = globule
    V = len(v)
    x_, r_, q_ = packed_atoms_ball(n=16, radius=None, seed=11)
    cfg = dict(leaf_size=16, p_leaf=4, adaptive=1, p_max=8, quad_duffy=4)
    h = F.Handle(eta0=0.8, basis=HAT, precond=F.PRECOND_DIAG, rhs_theta=0.5, rhs_pmax=6, **cfg)
    h.build_tree(v, t).assemble_nearfield()
    O = p1.setup(P, otree.build(P, 16, 0.8), EPS, KAP, p_leaf=4, adaptive=1, p_max=8, with_near=False)
    c = v.mean(0)
    x = np.concatenate([np.cos(0.3 * (v - c) @ np.array([1.0, 0.5, -0.2])),
                        np.sin(0.25 * (v - c) @ np.array([-0.3, 1.0, 0.4]))])
    for theta, pmax in ((0.5, 6), (0.3, 8), (0.0, 8)):
        E = h.solvation_energy_treecode(dev(x), x_, q_, theta, p_max=pmax)
        Eref = p1.treecode_energy(O, x, x_, q_, theta, p_max=pmax)
        b = torch.empty(2 * V, dtype=torch.float64, device=DEV)
        h.rhs_treecode(x_, q_, theta, b, p_max=pmax)
        torch.cuda.synchronize()
        bref = p1.treecode_rhs(O, x_, q_, theta, 1.0, p_max=pmax)
        print("theta %.1f: energy %.3e, rhs %.3e / %.3e" % (theta, abs(E - Eref) / abs(Eref),
                                                           rel(b.cpu().numpy(), bref), maxrow(b.cpu().numpy(), bref)))
        assert abs(E - Eref) < 1e-11 * abs(Eref)
        assert rel(b.cpu().numpy(), bref) < 1e-11 and maxrow(b.cpu().numpy(), bref) < 1e-11
    Ed = h.solvation_energy(dev(x), x_, q_)
    assert abs(h.solvation_energy_treecode(dev(x), x_, q_, 0.0) - Ed) < 1e-12 * abs(Ed)
    xs = torch.zeros(2 * V, dtype=torch.float64, device=DEV)
    code, info = h.solve(x_, q_, xs)
    assert code == 0 and info.rel_residual <= 1e-6
    h.close()


# the benchmark's tree and expansion settings on its 491,088-panel workload
BIG = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8, quad_duffy=7, near_ratio=2.0)


@pytest.fixture(scope="module")
def big_hat():
    from synth import workload
    w = workload("ellipsoid500k")
    P = panels(w["verts"], w["tris"])
    eps = w["eps_out"] / w["eps_in"]
    tr = otree.build(P, BIG["leaf_size"], BIG["eta0"])
    O = p1.setup(P, tr, eps, w["kappa"], p_leaf=BIG["p_leaf"], adaptive=BIG["adaptive"], p_max=BIG["p_max"],
                 with_near=False)
    h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], basis=HAT, precond=F.PRECOND_DIAG,
                 **BIG).build_tree(w["verts"], w["tris"]).assemble_nearfield()
    yield dict(w=w, P=P, O=O, h=h)
    h.close()


def test_hat_full_size_rows_and_invariant(big_hat):
    """491,088 panels (245,546 vertices): near and far rows of 12 sampled
    vertices against the oracle (FP64 to 1e-11, the FP32 operator to 1e-6 of
    the largest row), and the box-function invariant: for constant nodal
    values the sum of A x over the vertices equals the box operator's sum over
    the panels (the hat functions of a panel sum to one)"""
    w, P, O, h = big_hat["w"], big_hat["P"], big_hat["O"], big_hat["h"]
    V = len(w["verts"])
    rng = np.random.default_rng(31)
    x = rng.standard_normal(2 * V)
    yn = gpu_matvec(h, x, parts=F.PART_NEAR)
    yf = gpu_matvec(h, x, parts=F.PART_FAR)
    y32 = gpu_matvec(h, x, F.MIXED)
    verts = rng.choice(V, 12, replace=False)
    n1, n2 = p1.near_rows(O, x[:V], x[V:], verts)
    f1, f2 = p1.far_rows(O, x[:V], x[V:], verts)
    near = np.concatenate([n1, n2])
    far = np.concatenate([f1, f2])
    idx = np.concatenate([verts, V + verts])
    print("491k hat rows: near %.2e, far %.2e, fp32 %.2e"
          % (maxrow(yn[idx], near), maxrow(yf[idx], far), maxrow(y32[idx], near + far)))
    assert maxrow(yn[idx], near) < 1e-11 and maxrow(yf[idx], far) < 1e-11
    assert maxrow(y32[idx], near + far) < 1e-6
    hb = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], precond=F.PRECOND_DIAG, **BIG)
    hb.build_tree(w["verts"], w["tris"]).assemble_nearfield()
    N = len(w["tris"])
    for c1, c2 in ((1.0, 0.0), (0.0, 1.0), (0.7, -0.3)):
        s_hat = gpu_matvec(h, np.concatenate([np.full(V, c1), np.full(V, c2)]))
        s_box = gpu_matvec(hb, np.concatenate([np.full(N, c1), np.full(N, c2)]))
        for ch in range(2):
            a, b = s_hat[ch * V:(ch + 1) * V].sum(), s_box[ch * N:(ch + 1) * N].sum()
            print("constant (%.1f, %.1f) channel %d: hat %.12e box %.12e" % (c1, c2, ch, a, b))
            assert abs(a - b) < 1e-11 * np.abs(s_box[ch * N:(ch + 1) * N]).sum()
    hb.close()


def test_hat_full_size_solves(big_hat):
    """both precisions to a 1e-6 true residual on the 491,088-panel workload,
    energies within 1e-5 of each other and within 5e-3 of the box-function
    FP64 energy: the two discretisations of the same problem, each with an
    O(h^2) energy error (measured 1.9e-3 apart here; 3.8e-3 apart on the
    320-panel Kirkwood sphere, 2.4e-4 at 5,120 panels)"""
    w = big_hat["w"]
    V, N = len(w["verts"]), len(w["tris"])
    E = {}
    for basis, prec, pc in ((HAT, F.FP64, F.PRECOND_DIAG), (HAT, F.MIXED, F.PRECOND_DIAG),
                            (F.BASIS_S0, F.FP64, F.PRECOND_GROUP)):
        print("solve: basis %d precision %d" % (basis, prec), flush=True)
        h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], basis=basis, precision=prec,
                     precond=pc, tol=1e-6, max_iter=300, max_outer=5, inner_tol=5e-7, **BIG)
        h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
        n = V if basis == HAT else N
        x = torch.zeros(2 * n, dtype=torch.float64, device=DEV)
        code, info = h.solve(w["xq"], w["q"], x)
        assert code == 0 and info.rel_residual <= 1e-6, (basis, prec)
        E[(basis, prec)] = h.solvation_energy(x, w["xq"], w["q"])
        print("basis %d precision %d: %d inner iterations, energy %.6f"
              % (basis, prec, info.inner_iterations, E[(basis, prec)]))
        if basis == HAT and prec == F.FP64:
            # the treecode energy (theta 0.5, order cap 6) against the direct sum
            Et = h.solvation_energy_treecode(x, w["xq"], w["q"], 0.5, p_max=6)
            print("hat treecode energy %.6f (rel. diff %.2e)" % (Et, abs(Et - E[(basis, prec)]) / abs(E[(basis, prec)])))
            assert abs(Et - E[(basis, prec)]) < 1e-5 * abs(E[(basis, prec)])
        h.close()
    e64 = E[(HAT, F.FP64)]
    assert abs(E[(HAT, F.MIXED)] - e64) < 1e-5 * abs(e64)
    assert abs(E[(F.BASIS_S0, F.FP64)] - e64) < 5e-3 * abs(e64)
