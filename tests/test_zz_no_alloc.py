"""The allocation-free energy entry point (fagbi_solvation_energy_noalloc,
its partial sums in a static device array) against the allocating
fagbi_solvation_energy (same kernels and summation order) and the FP64
oracle, on two calls in a row, the second with a smaller mesh and fewer
charges (the shared array keeps the first call's partial sums beyond the
second call's blocks)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import solve as osolve  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere  # noqa: E402

pytestmark = pytest.mark.gpu
DEV = "cuda:0"
EPS, KAP = 80.0, 0.1257


def test_noalloc_energy_matches_allocating_entry_point():
    rng = np.random.default_rng(50)
    E_dev = torch.zeros(1, dtype=torch.float64, device=DEV)
    for sub, nc in ((4, 300), (2, 7)):
        v, t = icosphere(sub, 2.0)
        P = panels(v, t)
        h = F.Handle().build_tree(v, t)
        N = len(t)
        xh = rng.standard_normal(2 * N)
        x = torch.tensor(xh, dtype=torch.float64, device=DEV)
        xq = rng.uniform(-1, 1, (nc, 3))
        q = rng.standard_normal(nc)
        E_ref = h.solvation_energy(x, xq, q)
        chg = torch.tensor(np.concatenate([xq, q[:, None]], 1), dtype=torch.float64, device=DEV).contiguous()
        E_dev.fill_(float("nan"))
        h.solvation_energy_noalloc(x, chg, E_dev)
        torch.cuda.synchronize()
        E = float(E_dev.item())
        print("N %d, %d charges: no-alloc %.17g, allocating %.17g" % (N, nc, E, E_ref))
        assert abs(E - E_ref) <= 1e-13 * abs(E_ref)
        Eo = osolve.energy(P, xh, xq, q, EPS, KAP)
        assert abs(E - Eo) <= 1e-11 * abs(Eo)
        h.close()


def test_noalloc_energy_rejects_bad_arguments():
    v, t = icosphere(1, 2.0)
    h = F.Handle().build_tree(v, t)
    x = torch.zeros(2 * len(t), dtype=torch.float64, device=DEV)
    E = torch.zeros(1, dtype=torch.float64, device=DEV)
    flat = torch.zeros(4 * 3 + 1, dtype=torch.float64, device=DEV)
    with pytest.raises(F.FagbiError) as e:     # 8-byte offset: not 32-byte aligned
        h.solvation_energy_noalloc(x, flat[1:].view(3, 4), E)
    assert e.value.code == -1          # FAGBI_E_ARG
    h.close()
