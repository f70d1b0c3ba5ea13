"""Parity at the benchmark's full size: the 491,088-panel ellipsoid globule in
the launch configuration the benchmark times (leaf 32, eta0 0.8, adaptive
orders 3..8).  The oracle cannot run the whole operator at this size, so:

* the cluster tree: permutation and interaction-pair count bit for bit;
* the near field: sampled rows (every panel of randomly drawn leaves) against
  the oracle's pair integrals over the oracle tree's neighbour lists, FP64 to
  1e-11 and FP32 to 1e-6;
* the far field: rows of FAGBI_PART_FAR at every panel of 24 randomly drawn
  leaves against the oracle's far field restricted to those leaves (its full
  upward pass, then MtL for their ancestors, LtL down their ancestor chains
  and LtP at their panels): every MtL order 3..8 and the benchmark's launch
  configuration, FP64 to 1e-11 and FP32 to 1e-6 (relative L2 and the largest
  row error relative to the largest row);
* the whole operator: FP32 against FP64 (property: same algorithm, so the
  difference is rounding), and sampled rows against the dense oracle rows
  within a bound far above the Taylor truncation and far below what a lost
  level, list or sign gives;
* repeated FP32 products with alternating inputs: bitwise equal (the leaf
  MtL's claimed tiles are each processed once per launch);
* the solve: true residuals and the energy of both precisions.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import dense as odense  # noqa: E402
from oracle import fmm as ofmm  # noqa: E402
from oracle import tree as otree  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from oracle.kernels import combine  # noqa: E402
from oracle.pairs import pair_integrals  # noqa: E402
from synth import workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
# the benchmark's tree and expansion settings
PARAMS = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8, quad_duffy=7, near_ratio=2.0)


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.fixture(scope="module")
def big():
    w = workload("ellipsoid500k")
    P = panels(w["verts"], w["tris"])
    eps = w["eps_out"] / w["eps_in"]
    h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], **PARAMS)
    h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
    tr = otree.build(P, PARAMS["leaf_size"], PARAMS["eta0"])
    yield dict(w=w, P=P, eps=eps, h=h, tr=tr)
    h.close()


def gpu_matvec(h, x, prec, parts=F.PART_ALL):
    xd = torch.tensor(x, dtype=torch.float64, device=DEV)
    yd = torch.empty_like(xd)
    h.matvec(xd, yd, prec, parts)
    return yd.cpu().numpy()


def test_tree_matches_oracle_at_full_size(big):
    h, tr = big["h"], big["tr"]
    ti = h.tree_info()
    assert ti.levels == tr.L and ti.lmin == tr.lmin
    assert np.array_equal(h.permutation(), tr.perm)
    assert ti.m2l_pairs == sum(sum(len(x) for x in lv.inter) for lv in tr.levels)


def test_sampled_near_rows_match_oracle(big):
    P, tr, h, eps, w = big["P"], big["tr"], big["h"], big["eps"], big["w"]
    N = P.n
    rng = np.random.default_rng(21)
    x = rng.standard_normal(2 * N)
    leaf = tr.levels[tr.L]
    perm = tr.perm
    rows, ii, jj = [], [], []
    for c in rng.choice(leaf.n, 12, replace=False):
        tgt = perm[leaf.start[c]:leaf.end[c]]
        src = np.concatenate([perm[leaf.start[c2]:leaf.end[c2]] for c2 in leaf.nbr[c]])
        a, b = np.meshgrid(tgt, src, indexing="ij")
        ii.append(a.ravel())
        jj.append(b.ravel())
        rows.append(tgt)
    rows, ii, jj = np.concatenate(rows), np.concatenate(ii), np.concatenate(jj)
    I, _ = pair_integrals(P, ii, jj, w["kappa"], PARAMS["near_ratio"], PARAMS["quad_duffy"])
    B = combine(I, eps)
    phi, dphi = x[:N], x[N:]
    y1 = 0.5 * (1.0 + eps) * P.area * phi
    y2 = 0.5 * (1.0 + 1.0 / eps) * P.area * dphi
    y1 = y1 + np.bincount(ii, B[:, 0] * phi[jj] + B[:, 1] * dphi[jj], minlength=N)
    y2 = y2 + np.bincount(ii, B[:, 2] * phi[jj] + B[:, 3] * dphi[jj], minlength=N)
    ref = np.concatenate([y1[rows], y2[rows]])
    for prec, tol in ((F.FP64, 1e-11), (F.MIXED, 1e-6)):
        y = gpu_matvec(h, x, prec, F.PART_NEAR)
        got = np.concatenate([y[rows], y[N + rows]])
        assert rel(got, ref) < tol, prec


def test_sampled_far_field_rows_match_oracle(big):
    P, tr, h, eps, w = big["P"], big["tr"], big["h"], big["eps"], big["w"]
    N = P.n
    orders = otree.orders(tr, PARAMS["p_leaf"], PARAMS["adaptive"], PARAMS["p_max"])
    ti = h.tree_info()
    assert {orders[l] for l in range(tr.lmin, tr.L + 1) if ti.lev_pairs[l] > 0} == {3, 4, 5, 6, 7, 8}
    O = ofmm.setup(P, tr, eps, w["kappa"], p_leaf=PARAMS["p_leaf"], adaptive=PARAMS["adaptive"],
                   p_max=PARAMS["p_max"], with_near=False)
    rng = np.random.default_rng(23)
    x = rng.standard_normal(2 * N)
    leaves = rng.choice(tr.levels[tr.L].n, 24, replace=False)
    ids, f1, f2 = ofmm.far_field_rows(O, x[:N], x[N:], leaves)
    ref = np.concatenate([f1, f2])
    for prec, tol in ((F.FP64, 1e-11), (F.MIXED, 1e-6)):
        y = gpu_matvec(h, x, prec, F.PART_FAR)
        got = np.concatenate([y[ids], y[N + ids]])
        e = rel(got, ref)
        em = np.abs(got - ref).max() / np.abs(ref).max()
        print("far-field rows (%d panels), %s: rel-L2 %.2e, max-row %.2e"
              % (len(ids), "fp64" if prec == F.FP64 else "fp32", e, em))
        assert e < tol and em < tol, prec


def test_full_operator_precisions_and_sampled_dense_rows(big):
    P, h, eps, w = big["P"], big["h"], big["eps"], big["w"]
    N = P.n
    rng = np.random.default_rng(22)
    x = rng.standard_normal(2 * N)
    y64 = gpu_matvec(h, x, F.FP64)
    y32 = gpu_matvec(h, x, F.MIXED)
    assert np.isfinite(y64).all()
    assert rel(y32, y64) < 1e-6
    # whole rows against the dense oracle (all 491k sources per row).  The far
    # field is the same algorithm as the oracle's FMM (checked to 1e-11 on the
    # small cases); what separates it from the dense rows is the Taylor
    # truncation at p_leaf = 3, eta0 = 0.8 (measured 1.7e-3 here).  The bound
    # catches a lost level, list or sign, which give O(1) differences.
    rows = rng.choice(N, 3, replace=False)
    r1, r2 = odense.rows_matvec(P, eps, w["kappa"], x, rows, PARAMS["near_ratio"], PARAMS["quad_duffy"])
    ref = np.concatenate([r1, r2])
    got = np.concatenate([y64[rows], y64[N + rows]])
    err = rel(got, ref)
    print("sampled dense rows: relative difference %.2e" % err)
    assert err < 1e-2


def test_repeated_fp32_products_reproduce_bit_for_bit(big):
    """The leaf MtL's blocks claim tiles through counters that the launch's
    last block clears for the next launch; which block takes a tile does not
    change its arithmetic, so repeated products are bitwise equal.  Inputs
    alternate (and an FP64 product runs in between), so a tile skipped or
    left from the launch before would show as a changed row."""
    P, h = big["P"], big["h"]
    rng = np.random.default_rng(26)
    xs = [rng.standard_normal(2 * P.n) for _ in range(2)]
    first = [gpu_matvec(h, x, F.MIXED) for x in xs]
    for k in range(12):
        y = gpu_matvec(h, xs[k % 2], F.MIXED)
        assert np.array_equal(y, first[k % 2]), (k, int(np.sum(y != first[k % 2])))
        if k == 5:
            gpu_matvec(h, xs[0], F.FP64)
    assert not np.array_equal(first[0], first[1])


def test_full_size_solves(big):
    w = big["w"]
    N = big["P"].n
    res = {}
    for prec in (F.FP64, F.MIXED):
        h = F.Handle(precision=prec, eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], tol=1e-6,
                     max_iter=200, max_outer=5, inner_tol=5e-7, **PARAMS)
        h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
        x = torch.zeros(2 * N, dtype=torch.float64, device=DEV)
        code, info = h.solve(w["xq"], w["q"], x)
        assert code == 0 and info.rel_residual <= 1e-6
        res[prec] = h.solvation_energy(x, w["xq"], w["q"])
        h.close()
    assert abs(res[F.MIXED] - res[F.FP64]) < 1e-5 * abs(res[F.FP64])


def test_leaf_mtl_on_matrix_cores_full_size(big, monkeypatch):
    """At full size the matrix-core leaf MtL (FAGBI_M2L_MFMA=1) gives the same
    FP32 far field as the vector-unit kernel (1e-6) and stays within the FP32
    bound of the FP64 far field (itself equal to the oracle's to 1e-11)."""
    P, h, w = big["P"], big["h"], big["w"]
    N = P.n
    monkeypatch.setenv("FAGBI_M2L_MFMA", "1")
    hm = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], **PARAMS)
    hm.build_tree(w["verts"], w["tris"]).assemble_nearfield()
    rng = np.random.default_rng(25)
    x = rng.standard_normal(2 * N)
    ym = gpu_matvec(hm, x, F.MIXED, F.PART_FAR)
    yv = gpu_matvec(h, x, F.MIXED, F.PART_FAR)
    y64 = gpu_matvec(h, x, F.FP64, F.PART_FAR)
    e_mv, e_m64 = rel(ym, yv), rel(ym, y64)
    mr = np.abs(ym - yv).max() / np.abs(yv).max()
    print("full size far field: matrix cores vs vector units rel-L2 %.2e max-row %.2e; vs FP64 %.2e"
          % (e_mv, mr, e_m64))
    assert e_mv < 1e-6 and mr < 2e-6 and e_m64 < 2e-6
    yall = gpu_matvec(hm, x, F.MIXED)
    assert rel(yall, gpu_matvec(h, x, F.FP64)) < 1e-6
    hm.close()
