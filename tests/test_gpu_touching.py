"""Touching-pair cubature (identical panels, shared edge, shared vertex) on the
GPU against the dense FP64 oracle, entry by entry.

The GPU sums the radial coordinate of these transforms in closed form: a power
series in kappa |R_hat| whose degree grows with the pair's size, and the
n-point rule beyond the series' range.  A coarse sphere (R = 20 A, 320 panels,
edges up to 6.5 A) with kappa from 0.02 to 1 takes the pairs' bound on
kappa |R_hat| from about 0.25 (degree ~13) through the whole table (degree 24)
to beyond it (point by point), and mixes both within one mesh at kappa 0.2.
With eta0 = 0 every pair is near, so the GPU operator's columns (unit-vector
matvecs) are the oracle's dense matrix; each block's off-diagonal and diagonal
entries must agree to 1e-12 of that part's largest entry.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

import paper_2110_13778_amd as F  # noqa: E402
from oracle import dense as odense  # noqa: E402
from oracle.geometry import panels  # noqa: E402
from synth import icosphere  # noqa: E402

pytestmark = pytest.mark.gpu
EPS = 80.0
DEV = "cuda:0"


@pytest.fixture(scope="module")
def coarse_sphere():
    v, t = icosphere(2, 20.0)
    return v, t, panels(v, t)


def gpu_columns(h, n2):
    A = np.empty((n2, n2))
    x = torch.zeros(n2, dtype=torch.float64, device=DEV)
    y = torch.empty(n2, dtype=torch.float64, device=DEV)
    for j in range(n2):
        x.zero_()
        x[j] = 1.0
        h.matvec(x, y, F.FP64, F.PART_NEAR)
        A[:, j] = y.cpu().numpy()
    return A


def check_blocks(A, R, N):
    """every operator block's off-diagonal and diagonal entries to 1e-12 of
    that part's largest oracle entry"""
    off = ~np.eye(N, dtype=bool)
    for bi in range(2):
        for bj in range(2):
            G = A[bi * N:(bi + 1) * N, bj * N:(bj + 1) * N]
            O = R[bi * N:(bi + 1) * N, bj * N:(bj + 1) * N]
            for mask in (off, ~off):
                scale = np.abs(O[mask]).max()
                err = np.abs(G[mask] - O[mask]).max()
                assert err <= 1e-12 * scale, (bi, bj, mask is off, err / scale)


@pytest.mark.parametrize("n,kappa", [(7, 0.02), (7, 0.1257), (7, 0.2), (7, 1.0), (3, 0.1257), (4, 0.3)])
def test_touching_pairs_entrywise(coarse_sphere, n, kappa):
    v, t, P = coarse_sphere
    N = P.n
    print("touching pairs: n %d kappa %g" % (n, kappa), flush=True)
    h = F.Handle(eta0=0.0, eps_in=1.0, eps_out=EPS, kappa=kappa, quad_duffy=n)
    h.build_tree(v, t).assemble_nearfield()
    A = gpu_columns(h, 2 * N)   # caller order, as the oracle's
    h.close()
    R = odense.assemble(P, EPS, kappa, n=n)
    check_blocks(A, R, N)


@pytest.mark.parametrize("level,n,kappa", [(2, 1, 0.1257), (1, 16, 0.02)])
def test_touching_pairs_extreme_orders(level, n, kappa):
    """the smallest and the largest accepted rule orders (1 and 16; the
    coarser mesh keeps the oracle's 2 n^4 vertex points affordable)"""
    v, t = icosphere(level, 20.0)
    P = panels(v, t)
    N = P.n
    print("touching pairs: level %d n %d kappa %g" % (level, n, kappa), flush=True)
    h = F.Handle(eta0=0.0, eps_in=1.0, eps_out=EPS, kappa=kappa, quad_duffy=n)
    h.build_tree(v, t).assemble_nearfield()
    A = gpu_columns(h, 2 * N)
    h.close()
    R = odense.assemble(P, EPS, kappa, n=n)
    check_blocks(A, R, N)
