"""Treecode solvation energy (Sec. 2.5) on the GPU against the oracle's
treecode: same moments (FP64 upward pass of the far field), same acceptance
decisions, same direct leaves, so the two agree to rounding (1e-11 relative).
At the benchmark's size a sample of charges is checked (the energy of a
subset of charges is the sum of their terms)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import fmm as ofmm  # noqa: E402
from oracle import tree as otree  # noqa: E402
from oracle import treecode as otc  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere, workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS_IN, EPS_OUT, KAP = 1.0, 80.0, 0.1257


def smooth_x(P, scale):
    c = P.centroid / scale
    return np.concatenate([1.0 + 0.3 * c[:, 0] + 0.2 * c[:, 1] ** 2, -0.5 + 0.1 * c[:, 2]])


@pytest.mark.parametrize("p_leaf,adaptive", [(3, 1), (8, 0)])
def test_small_sphere_matches_oracle(p_leaf, adaptive):
    v, t = icosphere(3, 10.0)
    P = panels(v, t)
    prm = dict(leaf_size=8, eta0=0.8, p_leaf=p_leaf, adaptive=adaptive, p_max=8)
    h = F.Handle(eps_in=EPS_IN, eps_out=EPS_OUT, kappa=KAP, **prm)
    h.build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 8, 0.8)
    Fo = ofmm.setup(P, tr, EPS_OUT / EPS_IN, KAP, p_leaf=p_leaf, adaptive=adaptive, p_max=8, with_near=False)
    rng = np.random.default_rng(p_leaf)
    x = smooth_x(P, 10.0)
    xq = rng.uniform(-5.0, 5.0, (70, 3))     # a ragged second wave of charges
    q = rng.standard_normal(70)
    xd = torch.tensor(x, device=DEV)
    for theta in (0.0, 0.3, 0.5):
        E = h.solvation_energy_treecode(xd, xq, q, theta)
        Eo = otc.energy(Fo, x, xq, q, theta)
        print("theta %.1f  gpu %.15e  oracle %.15e" % (theta, E, Eo))
        assert abs(E - Eo) <= 1e-11 * abs(Eo), theta
    # theta = 0 is the direct sum of the other entry point
    assert abs(h.solvation_energy_treecode(xd, xq, q, 0.0) - h.solvation_energy(xd, xq, q)) <= \
        1e-12 * abs(h.solvation_energy(xd, xq, q))
    h.close()


def test_single_leaf_mesh():
    v, t = icosphere(0, 1.5)
    P = panels(v, t)
    h = F.Handle(eps_in=EPS_IN, eps_out=EPS_OUT, kappa=KAP, p_leaf=3, adaptive=1, p_max=8)
    h.build_tree(v, t).assemble_nearfield()
    assert h.tree_info().levels == 0
    tr = otree.build(P, 32, 0.8)
    Fo = ofmm.setup(P, tr, EPS_OUT / EPS_IN, KAP, p_leaf=3, adaptive=1, p_max=8, with_near=False)
    x = smooth_x(P, 1.5)
    xq = np.array([[0.1, 0.0, 0.2], [9.0, 1.0, 0.0]])   # inside, and far enough to accept the leaf
    q = np.array([1.0, -0.5])
    E = h.solvation_energy_treecode(torch.tensor(x, device=DEV), xq, q, 0.5)
    Eo = otc.energy(Fo, x, xq, q, 0.5)
    assert abs(E - Eo) <= 1e-11 * abs(Eo)
    h.close()


def test_full_size_sampled_charges_and_pair_limit():
    w = workload("ellipsoid500k")
    P = panels(w["verts"], w["tris"])
    prm = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8)
    h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], **prm)
    h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
    tr = otree.build(P, 32, 0.8)
    eps = w["eps_out"] / w["eps_in"]
    Fo = ofmm.setup(P, tr, eps, w["kappa"], p_leaf=3, adaptive=1, p_max=8, with_near=False)
    x = smooth_x(P, 40.0)
    xd = torch.tensor(x, device=DEV)
    rng = np.random.default_rng(8)
    sel = rng.choice(len(w["q"]), 24, replace=False)
    xq, q = w["xq"][sel], w["q"][sel]
    for theta in (0.3, 0.5):
        E = h.solvation_energy_treecode(xd, xq, q, theta)
        Eo = otc.energy(Fo, x, xq, q, theta)
        assert abs(E - Eo) <= 1e-11 * abs(Eo), theta
    # theta = 0 visits every leaf: the direct sum, also on the big tree
    E0 = h.solvation_energy_treecode(xd, xq[:2], q[:2], 0.0)
    Ed = h.solvation_energy(xd, xq[:2], q[:2])
    assert abs(E0 - Ed) <= 1e-12 * abs(Ed)
    # with every charge it would need more than 2^26 (charge, cluster) pairs on
    # one level: refused on the host, before any allocation
    with pytest.raises(F.FagbiError) as e:
        h.solvation_energy_treecode(xd, w["xq"], w["q"], 0.0)
    assert e.value.code == -1
    # the handle is still usable
    assert np.isfinite(h.solvation_energy_treecode(xd, xq[:2], q[:2], 0.5))
    h.close()


@pytest.mark.parametrize("p_leaf,adaptive", [(3, 1), (8, 0)])
def test_rhs_small_sphere_matches_oracle(p_leaf, adaptive):
    """right-hand side by the reverse treecode against the oracle's (the
    atomics change the summation order only: 1e-11 of max |b|)"""
    v, t = icosphere(3, 10.0)
    P = panels(v, t)
    prm = dict(leaf_size=8, eta0=0.8, p_leaf=p_leaf, adaptive=adaptive, p_max=8)
    h = F.Handle(eps_in=2.0, eps_out=EPS_OUT, kappa=KAP, **prm)
    h.build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 8, 0.8)
    Fo = ofmm.setup(P, tr, EPS_OUT / 2.0, KAP, p_leaf=p_leaf, adaptive=adaptive, p_max=8, with_near=False)
    rng = np.random.default_rng(10 + p_leaf)
    xq = rng.uniform(-5.0, 5.0, (70, 3))
    q = rng.standard_normal(70)
    b = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    for theta in (0.0, 0.3, 0.5):
        h.rhs_treecode(xq, q, theta, b)
        bo = otc.rhs(Fo, xq, q, theta, 2.0)
        err = np.abs(b.cpu().numpy() - bo).max() / np.abs(bo).max()
        print("theta %.1f  max rel %.2e" % (theta, err))
        assert err <= 1e-11, theta
    bd = torch.empty_like(b)
    h.rhs(xq, q, bd)
    h.rhs_treecode(xq, q, 0.0, b)
    assert (b - bd).abs().max().item() <= 1e-12 * bd.abs().max().item()
    h.close()


def test_rhs_full_size_sampled_charges_and_solve():
    w = workload("ellipsoid500k")
    P = panels(w["verts"], w["tris"])
    prm = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8)
    h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], **prm)
    h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
    tr = otree.build(P, 32, 0.8)
    eps = w["eps_out"] / w["eps_in"]
    Fo = ofmm.setup(P, tr, eps, w["kappa"], p_leaf=3, adaptive=1, p_max=8, with_near=False)
    rng = np.random.default_rng(9)
    sel = rng.choice(len(w["q"]), 16, replace=False)
    b = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    h.rhs_treecode(w["xq"][sel], w["q"][sel], 0.5, b)
    bo = otc.rhs(Fo, w["xq"][sel], w["q"][sel], 0.5, w["eps_in"])
    assert np.abs(b.cpu().numpy() - bo).max() <= 1e-11 * np.abs(bo).max()
    # whole RHS of all charges against the direct sum (the treecode's own error)
    bd = torch.empty_like(b)
    h.rhs(w["xq"], w["q"], bd)
    h.rhs_treecode(w["xq"], w["q"], 0.5, b)
    err = ((b - bd).norm() / bd.norm()).item()
    print("treecode RHS against the direct sum: %.2e" % err)
    assert err < 1e-3
    h.close()
    # a solve with the treecode right-hand side
    E = {}
    for th in (0.0, 0.5):
        hs = F.Handle(precision=F.FP64, eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], tol=1e-6,
                      rhs_theta=th, quad_duffy=7, near_ratio=2.0, **prm)
        hs.build_tree(w["verts"], w["tris"]).assemble_nearfield()
        x = torch.zeros(2 * P.n, dtype=torch.float64, device=DEV)
        code, info = hs.solve(w["xq"], w["q"], x)
        assert code == 0
        E[th] = hs.solvation_energy(x, w["xq"], w["q"])
        hs.close()
    print("energy with the treecode RHS against the direct RHS: %.2e" % (abs(E[0.5] - E[0.0]) / abs(E[0.0])))
    assert abs(E[0.5] - E[0.0]) < 1e-4 * abs(E[0.0])


def test_order_cap_matches_oracle():
    v, t = icosphere(3, 10.0)
    P = panels(v, t)
    prm = dict(leaf_size=8, eta0=0.8, p_leaf=3, adaptive=1, p_max=8)
    h = F.Handle(eps_in=2.0, eps_out=EPS_OUT, kappa=KAP, **prm)
    h.build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 8, 0.8)
    Fo = ofmm.setup(P, tr, EPS_OUT / 2.0, KAP, p_leaf=3, adaptive=1, p_max=8, with_near=False)
    rng = np.random.default_rng(12)
    x = smooth_x(P, 10.0)
    xq = rng.uniform(-5.0, 5.0, (40, 3))
    q = rng.standard_normal(40)
    xd = torch.tensor(x, device=DEV)
    b = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    for cap in (3, 5):
        E = h.solvation_energy_treecode(xd, xq, q, 0.4, p_max=cap)
        Eo = otc.energy(Fo, x, xq, q, 0.4, p_max=cap)
        assert abs(E - Eo) <= 1e-11 * abs(Eo), cap
        h.rhs_treecode(xq, q, 0.4, b, p_max=cap)
        bo = otc.rhs(Fo, xq, q, 0.4, 2.0, p_max=cap)
        assert np.abs(b.cpu().numpy() - bo).max() <= 1e-11 * np.abs(bo).max(), cap
    h.close()
