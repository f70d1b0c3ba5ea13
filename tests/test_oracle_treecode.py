"""Pins of the oracle's Cartesian treecode for the solvation energy (Sec. 2.5).

* theta = 0 accepts no cluster: every leaf is summed directly exactly once, so
  the result is the direct energy sum (oracle.solve.energy, itself pinned by
  the Kirkwood sphere) up to rounding;
* the particle-cluster expansion converges to the direct sum as the Taylor
  order grows and as theta shrinks (a dropped term, a wrong sign or index in
  the moments or the coefficients leaves an error of the size of that term,
  which stops the convergence);
* every charge's potential is covered: far terms and direct leaves together
  account for the whole surface (checked through theta = 0 and the counts).
"""
import numpy as np
import pytest

from oracle import fmm as ofmm
from oracle import solve as osolve
from oracle import tree as otree
from oracle import treecode as otc
from oracle.geometry import panels
from synth import icosphere

EPS, KAP = 80.0, 0.1257


@pytest.fixture(scope="module")
def sphere():
    v, t = icosphere(3, 10.0)
    P = panels(v, t)
    tr = otree.build(P, 8, 0.8)
    rng = np.random.default_rng(3)
    c = P.centroid
    # smooth surface densities (as a solution is), charges inside the sphere
    x = np.concatenate([1.0 + 0.3 * c[:, 0] / 10 + 0.2 * (c[:, 1] / 10) ** 2, -0.5 + 0.1 * c[:, 2] / 10])
    xq = rng.uniform(-5.0, 5.0, (12, 3))
    q = rng.standard_normal(12)
    Vd = np.array([otc._direct(P, np.arange(P.n), xn, x[:P.n], x[P.n:], EPS, KAP) for xn in xq])
    return P, tr, x, xq, q, Vd


def setup(P, tr, p, adaptive=0):
    return ofmm.setup(P, tr, EPS, KAP, p_leaf=p, adaptive=adaptive, p_max=8, with_near=False)


def test_theta_zero_is_the_direct_sum(sphere):
    P, tr, x, xq, q, Vd = sphere
    F = setup(P, tr, 3, 1)
    V, nf, nl = otc.potentials(F, x, xq, 0.0)
    assert (nf == 0).all() and (nl == tr.levels[tr.L].n).all()
    E = otc.energy(F, x, xq, q, 0.0)
    Ed = osolve.energy(P, x, xq, q, EPS, KAP)
    assert abs(E - Ed) <= 1e-13 * abs(Ed)
    assert np.abs(V - Vd).max() <= 1e-13 * np.abs(Vd).max()


def test_converges_with_order(sphere):
    P, tr, x, xq, q, Vd = sphere
    errs = []
    for p in (1, 3, 5, 7):
        V, nf, _ = otc.potentials(setup(P, tr, p), x, xq, 0.4)
        assert nf.sum() > 0
        errs.append(np.abs(V - Vd).max() / np.abs(Vd).max())
    assert all(b < 0.5 * a for a, b in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs


def test_converges_with_theta(sphere):
    P, tr, x, xq, q, Vd = sphere
    F = setup(P, tr, 5)
    errs = []
    for th in (0.7, 0.5, 0.3):
        V, _, _ = otc.potentials(F, x, xq, th)
        errs.append(np.abs(V - Vd).max() / np.abs(Vd).max())
    assert errs[0] > errs[1] > errs[2], errs
    assert errs[2] < 1e-4, errs


def test_adaptive_orders_energy(sphere):
    """the FMM's variable orders (p_l = p_L + L - l) as the moments' orders"""
    P, tr, x, xq, q, Vd = sphere
    F = setup(P, tr, 3, 1)
    Ed = osolve.energy(P, x, xq, q, EPS, KAP)
    E = otc.energy(F, x, xq, q, 0.3)
    assert abs(E - Ed) < 3e-3 * abs(Ed)


def test_rhs_theta_zero_is_the_direct_sum(sphere):
    P, tr, x, xq, q, Vd = sphere
    F = setup(P, tr, 3, 1)
    b = otc.rhs(F, xq, q, 0.0, 2.0)
    bd = osolve.rhs(P, xq, q, 2.0)
    assert np.abs(b - bd).max() <= 1e-13 * np.abs(bd).max()


def test_rhs_converges_with_order_and_theta(sphere):
    P, tr, x, xq, q, Vd = sphere
    bd = osolve.rhs(P, xq, q, 1.0)
    errs = []
    for p in (1, 3, 5, 7):
        b = otc.rhs(setup(P, tr, p), xq, q, 0.4, 1.0)
        errs.append(np.linalg.norm(b - bd) / np.linalg.norm(bd))
    assert all(e2 < 0.5 * e1 for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 1e-4, errs
    F = setup(P, tr, 5)
    et = [np.linalg.norm(otc.rhs(F, xq, q, th, 1.0) - bd) / np.linalg.norm(bd) for th in (0.7, 0.5, 0.3)]
    assert et[0] > et[1] > et[2], et


def test_order_cap(sphere):
    """a cap at or above every level's order is no cap; a cap p evaluates the
    same terms as moments of order p on every level above it"""
    P, tr, x, xq, q, Vd = sphere
    F = setup(P, tr, 3, 1)
    assert otc.energy(F, x, xq, q, 0.4, p_max=8) == otc.energy(F, x, xq, q, 0.4)
    Fc = setup(P, tr, 4, 0)   # fixed order 4 on every level
    E4 = otc.energy(Fc, x, xq, q, 0.4)
    Fa = setup(P, tr, 4, 1)   # orders 4.. upwards, capped at 4
    assert abs(otc.energy(Fa, x, xq, q, 0.4, p_max=4) - E4) <= 1e-12 * abs(E4)
    # capped locals are polynomials of degree 4: LtL shifts them exactly, so
    # the right-hand side equals the fixed-order one too
    b4 = otc.rhs(Fc, xq, q, 0.4, 1.0)
    assert np.abs(otc.rhs(Fa, xq, q, 0.4, 1.0, p_max=4) - b4).max() <= 1e-12 * np.abs(b4).max()
