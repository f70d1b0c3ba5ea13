"""Parity of the HIP library (through its C ABI) with the FP64 CPU oracle.

Tolerances (relative L2 unless stated): FP64 path 1e-11 against the oracle's
same algorithm (same tree, orders and quadrature); mixed path 1e-6 against the
same FP64 oracle."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import dense as odense  # noqa: E402
from oracle import fmm as ofmm  # noqa: E402
from oracle import solve as osolve  # noqa: E402
from oracle import tree as otree  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere, isosurface_mesh, packed_atoms_ball  # noqa: E402

pytestmark = pytest.mark.gpu
EPS, KAP = 80.0, 0.1257
DEV = "cuda:0"


def rel(a, b):
    return float(np.linalg.norm(np.asarray(a) - np.asarray(b)) / np.linalg.norm(b))


def maxrow(a, b):
    """largest row error relative to the largest row"""
    return float(np.abs(np.asarray(a) - np.asarray(b)).max() / np.abs(np.asarray(b)).max())


def dev(x):
    return torch.tensor(np.asarray(x), dtype=torch.float64, device=DEV)


def gpu_matvec(h, x, precision=F.FP64, parts=F.PART_ALL):
    y = torch.empty(len(x), dtype=torch.float64, device=DEV)
    h.matvec(dev(x), y, precision, parts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.fixture(scope="module")
def sphere1280():
    v, t = icosphere(3, 2.0)
    return v, t, panels(v, t)


@pytest.fixture(scope="module")
def dense1280(sphere1280):
    v, t, P = sphere1280
    return odense.assemble(P, EPS, KAP)


def test_tree_order_matches_oracle(sphere1280):
    v, t, P = sphere1280
    for leaf, eta in ((32, 0.8), (8, 0.8), (4, 0.6)):
        h = F.Handle(leaf_size=leaf, eta0=eta).build_tree(v, t)
        tr = otree.build(P, leaf, eta)
        ti = h.tree_info()
        assert ti.levels == tr.L and ti.lmin == tr.lmin
        assert np.array_equal(h.permutation(), tr.perm)
        assert ti.m2l_pairs == sum(sum(len(x) for x in lv.inter) for lv in tr.levels)
        h.close()


def test_nearfield_all_pairs_equals_dense(sphere1280, dense1280):
    """eta0 = 0 makes every pair near: the GPU operator is the dense one."""
    v, t, P = sphere1280
    h = F.Handle(eta0=0.0).build_tree(v, t).assemble_nearfield()
    rng = np.random.default_rng(1)
    for _ in range(2):
        x = rng.standard_normal(2 * P.n)
        ref = dense1280 @ x
        assert rel(gpu_matvec(h, x), ref) < 1e-11
        assert rel(gpu_matvec(h, x, F.MIXED), ref) < 1e-6
    h.close()


# (leaf 4 at fixed order 3: the LtL into the leaves folded into the LtP with
# parents of order 3; the adaptive trees fold it from order 4)
@pytest.mark.parametrize("cfg", [dict(leaf_size=32, p_leaf=4, adaptive=0),
                                 dict(leaf_size=8, p_leaf=3, adaptive=1, p_max=6),
                                 dict(leaf_size=4, p_leaf=2, adaptive=1, p_max=5),
                                 dict(leaf_size=4, p_leaf=3, adaptive=0)])
def test_fmm_matches_oracle_fmm(sphere1280, cfg):
    v, t, P = sphere1280
    h = F.Handle(eta0=0.8, **cfg).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, cfg["leaf_size"], 0.8)
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=cfg["p_leaf"], adaptive=cfg["adaptive"],
                   p_max=cfg.get("p_max", 8))
    rng = np.random.default_rng(2)
    x = rng.standard_normal(2 * P.n)
    ref = ofmm.matvec(O, x)
    y64, y32 = gpu_matvec(h, x), gpu_matvec(h, x, F.MIXED)
    assert rel(y64, ref) < 1e-11 and maxrow(y64, ref) < 1e-11
    assert rel(y32, ref) < 1e-6 and maxrow(y32, ref) < 1e-6
    # near and far parts separately: the near part carries the identity
    # terms (folded into the stored diagonal), the far part is the far field
    # alone (steps 2-6 of the FMM)
    assert rel(gpu_matvec(h, x, parts=F.PART_NEAR), ofmm.matvec(O, x, far=False)) < 1e-11
    far = np.concatenate(ofmm.far_field(O, x[:P.n], x[P.n:]))
    assert rel(gpu_matvec(h, x, parts=F.PART_FAR), far) < 1e-11
    assert rel(gpu_matvec(h, x, F.MIXED, parts=F.PART_FAR), far) < 2e-6
    h.close()


@pytest.mark.parametrize("leaf", [8, 4])
def test_grouped_preconditioner_matches_oracle(sphere1280, leaf):
    """blocks over consecutive leaves up to 32 panels (small leaves, so the
    groups mix neighbouring and non-neighbouring leaves)"""
    v, t, P = sphere1280
    h = F.Handle(leaf_size=leaf, precond=F.PRECOND_GROUP).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, leaf, 0.8)
    Minv = osolve.block_preconditioner(P, tr, EPS, KAP, group_max=32)
    rng = np.random.default_rng(4)
    z = rng.standard_normal(2 * P.n)
    y = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    h.precond_apply(dev(z), y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), Minv(z)) < 1e-11
    h.close()


def test_precond_and_rhs_and_energy(sphere1280):
    v, t, P = sphere1280
    h = F.Handle().build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 32, 0.8)
    Minv = osolve.block_preconditioner(P, tr, EPS, KAP)
    rng = np.random.default_rng(3)
    z = rng.standard_normal(2 * P.n)
    y = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    h.precond_apply(dev(z), y)
    torch.cuda.synchronize()
    assert rel(y.cpu().numpy(), Minv(z)) < 1e-11
    xq = rng.uniform(-1, 1, (7, 3))
    q = rng.standard_normal(7)
    b = torch.empty(2 * P.n, dtype=torch.float64, device=DEV)
    h.rhs(xq, q, b)
    torch.cuda.synchronize()
    assert rel(b.cpu().numpy(), osolve.rhs(P, xq, q, 1.0)) < 1e-12
    E = h.solvation_energy(dev(z), xq, q)
    Eref = osolve.energy(P, z, xq, q, EPS, KAP)
    assert abs(E - Eref) < 1e-11 * abs(Eref)
    h.close()


@pytest.mark.parametrize("precision", [F.FP64, F.MIXED])
def test_solve_kirkwood_c1(sphere1280, dense1280, precision):
    v, t, P = sphere1280
    h = F.Handle(precision=precision, tol=1e-6).build_tree(v, t).assemble_nearfield()
    xq, q = np.zeros((1, 3)), np.array([1.0])
    x = torch.zeros(2 * P.n, dtype=torch.float64, device=DEV)
    code, info = h.solve(xq, q, x)
    assert code == 0 and info.rel_residual <= 1e-6
    E = h.solvation_energy(x, xq, q)
    from oracle import kirkwood
    Eb = kirkwood.born(1.0, 2.0, 1.0, EPS, KAP)
    assert abs(E - Eb) < 0.007 * abs(Eb)          # paper's N=1280 error band
    # against the dense oracle's solution of its own system
    b = osolve.rhs(P, xq, q, 1.0)
    xo = np.linalg.solve(dense1280, b)
    Eo = osolve.energy(P, xo, xq, q, EPS, KAP)
    assert abs(E - Eo) < 2e-4 * abs(Eo)            # FMM truncation + tol 1e-6
    h.close()


def test_solve_c1_same_algorithm_1e9(sphere1280):
    """C1 (1,280 panels, +1 e at the centre): the GPU FP64 solve to 1e-11
    against the oracle's GMRES on the oracle's same-algorithm operator (same
    tree, order, rules) to 1e-13: solution vectors and energies agree to 1e-9.
    The mixed path (FP64 flexible GMRES around FP32 inner solves) reaches the
    same FP64 solution once its outer tolerance is below the FP32 level."""
    v, t, P = sphere1280
    tr = otree.build(P, 32, 0.8)
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=4)
    xq, q = np.zeros((1, 3)), np.array([1.0])
    b = osolve.rhs(P, xq, q, 1.0)
    xo, it, _ = osolve.gmres(lambda z: ofmm.matvec(O, z), b, 1e-13, 200)
    Eo = osolve.energy(P, xo, xq, q, EPS, KAP)
    for prec, tol, bound in ((F.FP64, 1e-11, 1e-9), (F.MIXED, 1e-10, 1e-8)):
        h = F.Handle(precision=prec, tol=tol, max_outer=8).build_tree(v, t).assemble_nearfield()
        x = torch.zeros(2 * P.n, dtype=torch.float64, device=DEV)
        code, info = h.solve(xq, q, x)
        assert code == 0 and info.rel_residual <= tol
        E = h.solvation_energy(x, xq, q)
        ex = rel(x.cpu().numpy(), xo)
        print("C1 %s: solution rel-L2 %.2e, energy rel %.2e"
              % ("fp64" if prec == F.FP64 else "mixed", ex, abs(E - Eo) / abs(Eo)))
        assert ex < bound and abs(E - Eo) < bound * abs(Eo)
        h.close()


def test_irregular_globule_fmm():
    """isosurface mesh: slivers, close pairs and an uneven tree."""
    x, r, q = packed_atoms_ball(n=40, radius=None, seed=11)
    v, t = isosurface_mesh(x, r, spacing=0.9)
    P = panels(v, t)
    h = F.Handle(leaf_size=16, p_leaf=4, eta0=0.8).build_tree(v, t).assemble_nearfield()
    ti = h.tree_info()
    assert ti.singular_pairs[3] > 0          # close pairs present
    tr = otree.build(P, 16, 0.8)
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=4)
    rng = np.random.default_rng(4)
    xx = rng.standard_normal(2 * P.n)
    ref = ofmm.matvec(O, xx)
    assert rel(gpu_matvec(h, xx), ref) < 1e-11
    assert rel(gpu_matvec(h, xx, F.MIXED), ref) < 1e-6
    h.close()


def test_error_paths():
    v, t = icosphere(1, 1.0)
    h = F.Handle()
    with pytest.raises(F.FagbiError) as e:
        h.assemble_nearfield()
    assert e.value.code == -3
    with pytest.raises(F.FagbiError) as e:         # open mesh
        h.build_tree(v, t[:-1])
    assert e.value.code == -2
    with pytest.raises(F.FagbiError) as e:         # inward orientation
        h.build_tree(v, t[:, ::-1])
    assert e.value.code == -2
    with pytest.raises(F.FagbiError):
        F.Handle(p_leaf=12)
    with pytest.raises(F.FagbiError) as e:         # unknown cluster-radius mode
        F.Handle(radii=2)
    assert e.value.code == -1
    h.build_tree(v, t).assemble_nearfield()
    x = torch.zeros(2 * len(t), dtype=torch.float64, device=DEV)
    with pytest.raises(F.FagbiError):
        h.matvec(x, x)
    h.close()
