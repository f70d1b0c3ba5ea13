"""What the trained near-field network gains on the ~200k-panel globule.

The network is trained on the GPU (the library's own MFMA training kernels)
on every near-singular pair of the 81,920-panel sphere and the globule,
labelled by the cubature (120 epochs, as the benchmark trains it).  The
globule is then solved in the mixed-precision path with the gated surrogate
(near-singular pairs whose calibrated error estimate passes the gate take
the network's integrals; cubature elsewhere) and without it.  Stated and
checked: the assembly time of the near field (cubature + surrogate stages)
is lower with the network, the iterations rise by at most 10 %, and the
energy error against the no-surrogate path and the surrogate solution's
true residual under the cubature operator are printed and bounded (the
network's per-pair error is about the gate, so the operator moves by about
1e-3; the time-to-1e-6 of the surrogate path is to its own operator)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from synth import workload  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
PRM = dict(leaf_size=32, eta0=0.8, p_leaf=3, adaptive=1, p_max=8, precond=3, tol=1e-6, max_iter=200,
           max_outer=5, inner_tol=5e-7, precision=1)
GATE = 0.05


@pytest.fixture(scope="module")
def trained_blob():
    Xs, Ts, As = [], [], []
    for name in ("kirkwood2", "globule200k"):
        w = workload(name)
        h = F.Handle().build_tree(w["verts"], w["tris"]).assemble_nearfield()
        X, T, A = h.mlp_dataset(2000000)     # every near-singular pair of the mesh
        Xs.append(X.clone()); Ts.append(T.clone()); As.append(A.clone())
        h.close()
    h = F.Handle()
    hist = h.mlp_train(torch.cat(Xs).contiguous(), torch.cat(Ts).contiguous(), torch.cat(As).contiguous(),
                       epochs=120, batch=4096, lr=3e-3, seed=5)
    assert np.isfinite(hist).all() and hist[-1] < 0.3 * hist[0]
    blob = h.mlp_get_weights()
    h.close()
    return blob


def _run(w, blob, gated):
    extra = dict(mlp_mode=F.MLP_GATED, mlp_gate_tol=GATE) if gated else {}
    out = None
    times = []
    for _ in range(4):          # the first run warms the caches; median of the others
        h = F.Handle(eps_in=w["eps_in"], eps_out=w["eps_out"], kappa=w["kappa"], **PRM, **extra)
        if gated:
            h.mlp_set_weights(blob)
        h.set_profiling(True)
        h.build_tree(w["verts"], w["tris"]).assemble_nearfield()
        x = torch.zeros(2 * len(w["tris"]), dtype=torch.float64, device=DEV)
        code, info = h.solve(w["xq"], w["q"], x)
        E = h.solvation_energy(x, w["xq"], w["q"])
        pr = h.profile()
        stats = h.mlp_stats() if gated else (0, 0)
        if out is not None:
            out["h"].close()
        out = dict(h=h, x=x, code=code, info=info, E=E, stats=stats)
        times.append(pr["ms_singular"] + pr["ms_surrogate"])
    out["asm"] = float(np.median(times[1:]))
    return out


def test_gated_surrogate_gain_on_globule(trained_blob):
    w = workload("globule200k")
    off = _run(w, None, False)
    on = _run(w, trained_blob, True)
    assert off["code"] == 0 and on["code"] == 0
    gated, cand = on["stats"]
    # the surrogate solution under the cubature operator (the no-surrogate
    # handle's FP64 operator and right-hand side)
    N = len(w["tris"])
    b = torch.empty(2 * N, dtype=torch.float64, device=DEV)
    off["h"].rhs(w["xq"], w["q"], b)
    y = torch.empty_like(b)
    off["h"].matvec(on["x"], y, F.FP64)
    res = float(torch.linalg.norm(b - y) / torch.linalg.norm(b))
    dE = abs(on["E"] - off["E"]) / abs(off["E"])
    print("globule %d panels: gated %d of %d near-singular pairs; near-field assembly %.2f ms with the network, "
          "%.2f ms without; inner iterations %d / %d; energy %.6f / %.6f (rel. diff %.2e); true residual of "
          "the surrogate solution under the cubature operator %.2e"
          % (N, gated, cand, on["asm"], off["asm"], on["info"].inner_iterations, off["info"].inner_iterations,
             on["E"], off["E"], dE, res))
    assert 0 < gated <= cand
    assert on["asm"] < off["asm"]
    assert on["info"].inner_iterations <= 1.1 * off["info"].inner_iterations + 1
    assert dE < 1e-4
    assert res < 1e-2
    on["h"].close()
    off["h"].close()
