"""The six panel-pair integrands (Sec. 2.2, kernels K1..K4).

With r = x - y, r = |r|, E = exp(-kappa r), G0 = 1/(4 pi r), Gk = E/(4 pi r):
  k1 = G0 - Gk                              (K1)
  k2 = dG0/dn_y = (r.n_y)/(4 pi r^3)
  k3 = dGk/dn_y = E (1 + kappa r)(r.n_y)/(4 pi r^3)
  k4 = dG0/dn_x = -(r.n_x)/(4 pi r^3)
  k5 = dGk/dn_x = -E (1 + kappa r)(r.n_x)/(4 pi r^3)
  k6 = d2(Gk - G0)/dn_x dn_y
     = [c1 (n_x.n_y) - c2 (r.n_x)(r.n_y)/r^2] / (4 pi r^3)
    with u = kappa r, c1 = E(1+u) - 1, c2 = E(3(1+u) + u^2) - 3
so that K1 = k1, K2 = eps k3 - k2, K3 = k4 - k5/eps, K4 = k6.
c1 and c2 vanish like u^2 and are formed from expm1 to keep their leading digits.
"""
import numpy as np

FOUR_PI = 4.0 * np.pi


def kernel6(r, nx, ny, kappa):
    """r, nx, ny: [..., 3] arrays (broadcastable).  Returns [..., 6]."""
    rr = np.sqrt(np.sum(r * r, axis=-1))
    u = kappa * rr
    em1 = np.expm1(-u)              # E - 1
    E = em1 + 1.0
    inv4pr = 1.0 / (FOUR_PI * rr)
    inv4pr3 = inv4pr / (rr * rr)
    rny = np.sum(r * ny, axis=-1)
    rnx = np.sum(r * nx, axis=-1)
    nxny = np.sum(nx * ny, axis=-1)
    k1 = -em1 * inv4pr
    k2 = rny * inv4pr3
    k3 = E * (1.0 + u) * rny * inv4pr3
    k4 = -rnx * inv4pr3
    k5 = -E * (1.0 + u) * rnx * inv4pr3
    c1 = em1 + u * E                          # E(1+u) - 1
    c2 = 3.0 * em1 + 3.0 * u * E + u * u * E  # E(3(1+u)+u^2) - 3
    k6 = (c1 * nxny - c2 * rnx * rny / (rr * rr)) * inv4pr3
    return np.stack([k1, k2, k3, k4, k5, k6], axis=-1)


def combine(I, eps):
    """Map the six integrals to the four operator blocks (Sec. 2.3, linear
    system entries, with the integral terms on the right-hand side of the
    integral equations moved to the left, i.e. subtracted):
      B11 = -(eps I3 - I2), B12 = -I1, B21 = -I6, B22 = -(I4 - I5/eps)."""
    I = np.asarray(I)
    return np.stack([-(eps * I[..., 2] - I[..., 1]), -I[..., 0], -I[..., 5],
                     -(I[..., 3] - I[..., 4] / eps)], axis=-1)
