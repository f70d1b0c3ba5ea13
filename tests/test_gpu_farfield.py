"""The far field alone (FAGBI_PART_FAR: moments, MtM, MtL, LtL, LtP; no near
field, no identity terms) against the oracle's far field (Sec. 2.4, steps 2-6)
on trees whose interaction levels run every MtL order from 3 to 8, i.e. every
translation kernel the benchmark dispatches (register, LDS-table and slot
kernels, FP32 and FP64).  Errors are measured as relative L2 over the vector
and as the largest row error relative to the largest row (a single bad row
cannot hide under the norm).  Tolerances: FP64 1e-11.  FP32 expansions: the
whole mixed operator within 1e-6 of the FP64 one; the far field alone within
2e-6 (L2) and 4e-6 (largest row) of the oracle's: FP32 rounding of order-8
expansions is ~1e-6 of the far field alone (measured 6.6e-7 to 9.5e-7 L2 and
1.0e-6 to 1.6e-6 max-row at orders 5-8), and the far field is a fraction of
the operator's norm."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import fmm as ofmm  # noqa: E402
from oracle import tree as otree  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere  # noqa: E402

pytestmark = pytest.mark.gpu
EPS, KAP = 80.0, 0.1257
DEV = "cuda:0"


def errs(got, ref):
    d = np.asarray(got) - np.asarray(ref)
    return (float(np.linalg.norm(d) / np.linalg.norm(ref)),
            float(np.abs(d).max() / np.abs(ref).max()))


def far_gpu(h, x, prec, parts=F.PART_FAR):
    xd = torch.tensor(x, dtype=torch.float64, device=DEV)
    y = torch.empty_like(xd)
    h.matvec(xd, y, prec, parts)
    torch.cuda.synchronize()
    return y.cpu().numpy()


@pytest.fixture(scope="module")
def sphere5120():
    v, t = icosphere(4, 2.0)
    return v, t, panels(v, t)


# 5,120 panels, leaf 4: levels 2..5 interact; p_leaf 3 gives MtL orders
# 6, 5, 4, 3 and p_leaf 5 gives 8, 7, 6, 5 (adaptive, p_max 8)
@pytest.mark.parametrize("p_leaf", [3, 5])
def test_far_field_every_order(sphere5120, p_leaf):
    v, t, P = sphere5120
    prm = dict(leaf_size=4, eta0=0.8, p_leaf=p_leaf, adaptive=1, p_max=8)
    h = F.Handle(eps_out=EPS, kappa=KAP, **prm).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 4, 0.8)
    ti = h.tree_info()
    orders = otree.orders(tr, p_leaf, 1, 8)
    used = {orders[l] for l in range(tr.lmin, tr.L + 1) if ti.lev_pairs[l] > 0}
    assert used == ({3, 4, 5, 6} if p_leaf == 3 else {5, 6, 7, 8}), used
    assert [ti.lev_order[l] for l in range(tr.L + 1)] == orders
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=p_leaf, adaptive=1, p_max=8, with_near=False)
    rng = np.random.default_rng(30 + p_leaf)
    for _ in range(2):
        x = rng.standard_normal(2 * P.n)
        ref = np.concatenate(ofmm.far_field(O, x[:P.n], x[P.n:]))
        e64 = errs(far_gpu(h, x, F.FP64), ref)
        e32 = errs(far_gpu(h, x, F.MIXED), ref)
        print("p_leaf %d: FP64 rel-L2 %.2e max-row %.2e; mixed rel-L2 %.2e max-row %.2e"
              % (p_leaf, e64[0], e64[1], e32[0], e32[1]))
        assert e64[0] < 1e-11 and e64[1] < 1e-11, e64
        assert e32[0] < 2e-6 and e32[1] < 4e-6, e32
        ew = errs(far_gpu(h, x, F.MIXED, F.PART_ALL), far_gpu(h, x, F.FP64, F.PART_ALL))
        print("  whole operator, mixed vs FP64: rel-L2 %.2e max-row %.2e" % ew)
        assert ew[0] < 1e-6 and ew[1] < 1e-6, ew
    h.close()


def test_far_field_grouped_coarse_levels(sphere5120):
    """leaf 2, p_leaf 4: L = 6, interactions from level 2, orders 8, 7, 6, 5, 4
    on levels 2..6.  The finest two levels' MtL run on their own stream, level
    4 on the main one, and in FP32 the coarse levels 2 and 3 (orders 8 and 7)
    are one launch of the multi-level slot kernel (two levels with different
    slot rounds); FP64 runs them one launch per level."""
    v, t, P = sphere5120
    prm = dict(leaf_size=2, eta0=0.8, p_leaf=4, adaptive=1, p_max=8)
    h = F.Handle(eps_out=EPS, kappa=KAP, **prm).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, 2, 0.8)
    ti = h.tree_info()
    orders = otree.orders(tr, 4, 1, 8)
    assert (tr.L, tr.lmin) == (6, 2) and orders == [8, 8, 8, 7, 6, 5, 4], (tr.L, tr.lmin, orders)
    assert [ti.lev_order[l] for l in range(tr.L + 1)] == orders
    assert all(ti.lev_pairs[l] > 0 for l in range(2, 7))
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=4, adaptive=1, p_max=8, with_near=False)
    x = np.random.default_rng(50).standard_normal(2 * P.n)
    ref = np.concatenate(ofmm.far_field(O, x[:P.n], x[P.n:]))
    e64 = errs(far_gpu(h, x, F.FP64), ref)
    e32 = errs(far_gpu(h, x, F.MIXED), ref)
    print("grouped coarse levels: FP64 rel-L2 %.2e max-row %.2e; mixed rel-L2 %.2e max-row %.2e"
          % (e64[0], e64[1], e32[0], e32[1]))
    assert e64[0] < 1e-11 and e64[1] < 1e-11, e64
    assert e32[0] < 2e-6 and e32[1] < 4e-6, e32
    h.close()


def test_far_field_fixed_order8(sphere5120):
    """fixed order 8 on every level (the slot MtM / LtL kernels at 8 -> 8)"""
    v, t, P = sphere5120
    h = F.Handle(eps_out=EPS, kappa=KAP, leaf_size=8, eta0=0.8, p_leaf=8, adaptive=0).build_tree(v, t)
    h.assemble_nearfield()
    tr = otree.build(P, 8, 0.8)
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=8, adaptive=0, with_near=False)
    x = np.random.default_rng(40).standard_normal(2 * P.n)
    ref = np.concatenate(ofmm.far_field(O, x[:P.n], x[P.n:]))
    e64 = errs(far_gpu(h, x, F.FP64), ref)
    e32 = errs(far_gpu(h, x, F.MIXED), ref)
    print("fixed p 8: FP64 rel-L2 %.2e max-row %.2e; mixed rel-L2 %.2e max-row %.2e"
          % (e64[0], e64[1], e32[0], e32[1]))
    assert e64[0] < 1e-11 and e64[1] < 1e-11, e64
    assert e32[0] < 2e-6 and e32[1] < 4e-6, e32
    ew = errs(far_gpu(h, x, F.MIXED, F.PART_ALL), far_gpu(h, x, F.FP64, F.PART_ALL))
    print("  whole operator, mixed vs FP64: rel-L2 %.2e max-row %.2e" % ew)
    assert ew[0] < 1e-6 and ew[1] < 1e-6, ew
    h.close()


@pytest.mark.parametrize("mesh", ["sphere", "globule"])
def test_leaf_mtl_on_matrix_cores(sphere5120, mesh, monkeypatch):
    """The order-3 leaf-level FP32 MtL on the matrix cores (FAGBI_M2L_MFMA=1,
    v_mfma_f32_16x16x4f32) against the oracle's far field (the FP32 bounds
    above) and against the vector-unit kernel on the same tiles (both FP32,
    different summation order: 1e-6)."""
    from synth import isosurface_mesh, packed_atoms_ball
    if mesh == "sphere":
        v, t, P = sphere5120
        leaf = 4
    else:
        xa, ra, _ = packed_atoms_ball(n=40, radius=None, seed=11)
        v, t = isosurface_mesh(xa, ra, spacing=0.9)
        P = panels(v, t)
        leaf = 8
    prm = dict(eps_out=EPS, kappa=KAP, leaf_size=leaf, eta0=0.8, p_leaf=3, adaptive=1, p_max=8)
    monkeypatch.setenv("FAGBI_M2L_MFMA", "1")
    hm = F.Handle(**prm).build_tree(v, t).assemble_nearfield()
    monkeypatch.setenv("FAGBI_M2L_MFMA", "0")
    hv = F.Handle(**prm).build_tree(v, t).assemble_nearfield()
    tr = otree.build(P, leaf, 0.8)
    assert hm.tree_info().lev_order[tr.L] == 3
    O = ofmm.setup(P, tr, EPS, KAP, p_leaf=3, adaptive=1, p_max=8, with_near=False)
    rng = np.random.default_rng(44)
    x = rng.standard_normal(2 * P.n)
    ref = np.concatenate(ofmm.far_field(O, x[:P.n], x[P.n:]))
    ym, yv = far_gpu(hm, x, F.MIXED), far_gpu(hv, x, F.MIXED)
    em, ev, emv = errs(ym, ref), errs(yv, ref), errs(ym, yv)
    print("%s (%d panels): matrix cores vs oracle %.2e / %.2e, vector units vs oracle %.2e / %.2e, "
          "between them %.2e / %.2e" % (mesh, P.n, em[0], em[1], ev[0], ev[1], emv[0], emv[1]))
    assert em[0] < 2e-6 and em[1] < 4e-6, em
    assert emv[0] < 1e-6 and emv[1] < 2e-6, emv
    hm.close()
    hv.close()
