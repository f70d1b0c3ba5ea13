"""Learned near-field surrogate on the GPU: training kernels against the FP64
reference network, training on cubature labels, the error gate, and what the
network changes in a solve (iterations, cubature work, energy)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import mlp as omlp  # noqa: E402
from synth import isosurface_mesh, packed_atoms_ball  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"


def test_gradient_matches_reference_network():
    rng = np.random.default_rng(11)
    theta = (rng.standard_normal(omlp.n_params()) * 0.15).astype(np.float32)
    for n in (64, 1000):
        X = rng.standard_normal((n, 16)).astype(np.float32)
        T = rng.standard_normal((n, 6)).astype(np.float32)
        h = F.Handle()
        loss, g = h.mlp_grad(theta, torch.tensor(X, device=DEV), torch.tensor(T, device=DEV))
        l_ref, g_ref = omlp.loss_and_grad(theta.astype(np.float64), X.astype(np.float64), T.astype(np.float64))
        assert abs(loss - l_ref) < 1e-5 * abs(l_ref)
        assert np.abs(g - g_ref).max() < 1e-4 * np.abs(g_ref).max()
        h.close()


def test_forward_matches_reference_network():
    """fused inference kernel (matrix cores) against the FP64 reference
    network, with input standardisation and per-class output scaling; 1000
    rows leave a ragged last tile"""
    rng = np.random.default_rng(12)
    theta = (rng.standard_normal(omlp.n_params()) * 0.15).astype(np.float32)
    mu_in, sd_in = rng.standard_normal(16) * 0.3, 0.5 + rng.random(16)
    mu_in[13:], sd_in[13:] = 0.0, 1.0
    mu_out, sd_out = rng.standard_normal((3, 6)), 0.5 + rng.random((3, 6))
    ncal = 3 * 9 + 3 * 8
    blob = np.concatenate([theta, mu_in, sd_in, mu_out.ravel(), sd_out.ravel(), np.zeros(ncal)]).astype(np.float32)
    assert blob.size == 36093
    n = 1000
    X = rng.standard_normal((n, 16)).astype(np.float32)
    cls = rng.integers(0, 3, n)
    X[:, 13:] = 0.0
    X[np.arange(n), 13 + cls] = 1.0
    h = F.Handle()
    h.mlp_set_weights(blob)
    Y = h.mlp_forward(torch.tensor(X, device=DEV)).cpu().numpy()
    h.close()
    xs = (X.astype(np.float64) - mu_in) / sd_in
    ref = omlp.forward(theta.astype(np.float64), xs)[-1] * sd_out[cls] + mu_out[cls]
    assert np.abs(Y - ref).max() < 1e-5 * np.abs(ref).max()


@pytest.fixture(scope="module")
def trained():
    x, r, q = packed_atoms_ball(n=150, seed=7)
    v, t = isosurface_mesh(x, r, spacing=0.75)
    h = F.Handle().build_tree(v, t).assemble_nearfield()
    X, T, A = h.mlp_dataset(200000)
    hist = h.mlp_train(X.contiguous(), T.contiguous(), A.contiguous(), epochs=60, batch=1024,
                       lr=3e-3, seed=5)
    blob = h.mlp_get_weights()
    return dict(v=v, t=t, xq=x, q=q, h=h, X=X, T=T, A=A, hist=hist, blob=blob)


def test_training_reduces_loss_and_predicts_held_out_pairs(trained):
    hist = trained["hist"]
    assert np.isfinite(hist).all()
    assert hist[-1] < 0.3 * hist[0], hist
    X, T, A = trained["X"], trained["T"], trained["A"]
    n = X.shape[0]
    val = np.arange(9, n, 10)          # the rows held out from training
    Y = trained["h"].mlp_forward(X[val].contiguous()).cpu().numpy()
    t = T[val].cpu().numpy()
    full = A[val, 2:].cpu().numpy()
    cls = A[val, 0].cpu().numpy()
    assert set(np.unique(cls)) == {0.0, 1.0, 2.0}
    # error relative to the full integral (floor 10% of its rms), worst of
    # the six outputs per pair
    rms = np.sqrt((full ** 2).mean(0))
    e = (np.abs(Y - t) / (np.abs(full) + 0.1 * rms)).max(1)
    e0 = (np.abs(t) / (np.abs(full) + 0.1 * rms)).max(1)   # no correction at all
    for c in (0, 1, 2):
        assert np.median(e[cls == c]) < 0.1
    # edge-adjacent pairs, where the 3x3 rule is worst, are corrected well
    assert np.median(e[cls == 0]) < 0.5 * np.median(e0[cls == 0])
    print("held-out median error edge/vertex/close: %.4f %.4f %.4f (no correction: %.4f %.4f %.4f)"
          % tuple([np.median(e[cls == c]) for c in (0, 1, 2)] + [np.median(e0[cls == c]) for c in (0, 1, 2)]))


def _solve(w, mode, blob=None, gate=1e-3):
    h = F.Handle(mlp_mode=mode, mlp_gate_tol=gate)
    if blob is not None:
        h.mlp_set_weights(blob)
    h.build_tree(w["v"], w["t"]).assemble_nearfield()
    x = torch.zeros(2 * len(w["t"]), dtype=torch.float64, device=DEV)
    code, info = h.solve(w["xq"], w["q"], x)
    E = h.solvation_energy(x, w["xq"], w["q"])
    stats = h.mlp_stats() if mode != F.MLP_OFF else (0, 0)
    h.close()
    return code, info, E, stats


def test_surrogate_in_preconditioner_and_gated_near_field(trained):
    w = trained
    c0, i0, E0, _ = _solve(w, F.MLP_OFF)
    assert c0 == 0
    # preconditioner built from the network: same operator, so the same
    # solution; the network's error only costs iterations
    c1, i1, E1, _ = _solve(w, F.MLP_PRECOND, w["blob"])
    assert c1 == 0 and i1.rel_residual <= 1e-6
    assert abs(E1 - E0) < 1e-5 * abs(E0)
    assert i1.inner_iterations <= 2 * i0.inner_iterations + 5
    # gated near field: some cubature replaced; the energy moves by a bounded
    # amount against the all-cubature operator
    c2, i2, E2, (gated, cand) = _solve(w, F.MLP_GATED, w["blob"], gate=0.15)
    assert c2 == 0
    assert 0 < gated <= cand
    assert abs(E2 - E0) < 5e-3 * abs(E0)
    # a zero tolerance gates nothing and reproduces the cubature operator
    c3, i3, E3, (g3, _) = _solve(w, F.MLP_GATED, w["blob"], gate=0.0)
    assert g3 == 0 and abs(E3 - E0) < 1e-9 * abs(E0)
    print("surrogate: candidates %d, gated %d at tol 0.15; iterations off/precond/gated %d/%d/%d; "
          "E off %.6f precond %.6f gated %.6f" % (cand, gated, i0.inner_iterations, i1.inner_iterations,
                                                   i2.inner_iterations, E0, E1, E2))
