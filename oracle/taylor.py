"""Taylor coefficients of the Coulomb / screened Coulomb kernel (Sec. 2.4: the
derivatives D^gamma G are produced by recurrence rather than closed forms).

F_k(x0) = D^k f(x0) / k!  for f(x) = exp(-kappa |x|)/|x|, and H_k likewise for
h(x) = exp(-kappa |x|).  Contracting r^2 grad f = -x (f + kappa h) and
grad h = -kappa x f with the Euler operator and comparing coefficients of
delta^k in the expansions about x0 gives, for |k| >= 1,
  |k| r0^2 F_k + (2|k|-1) sum_i x0_i F_{k-e_i} + (|k|-1) sum_i F_{k-2e_i}
        = -kappa [ sum_i x0_i H_{k-e_i} + sum_i H_{k-2e_i} ]
  |k| H_k = -kappa [ sum_i x0_i F_{k-e_i} + sum_i F_{k-2e_i} ]
with F_0 = exp(-kappa r0)/r0, H_0 = exp(-kappa r0) and terms with a negative
index equal to zero.  Then G(x, y) = f(x - y)/(4 pi).
"""
import numpy as np
from math import factorial


def multi_indices(p):
    """All (a, b, c) with a+b+c <= p, by total degree then lexicographically
    descending in a, then b."""
    out = []
    for d in range(p + 1):
        for a in range(d, -1, -1):
            for b in range(d - a, -1, -1):
                out.append((a, b, d - a - b))
    return out


def mfact(k):
    return factorial(k[0]) * factorial(k[1]) * factorial(k[2])


def coefficients(x0, kappa, p):
    """x0: [m, 3].  Returns dict k -> F_k [m] for |k| <= p."""
    x0 = np.atleast_2d(np.asarray(x0, np.float64))
    r2 = (x0 * x0).sum(1)
    r0 = np.sqrt(r2)
    F = {(0, 0, 0): np.exp(-kappa * r0) / r0}
    H = {(0, 0, 0): np.exp(-kappa * r0)}
    zero = np.zeros(len(x0))
    E = np.eye(3, dtype=int)

    def get(D, k):
        return D.get(k, zero) if min(k) >= 0 else zero

    for k in multi_indices(p)[1:]:
        n = sum(k)
        s1f = sum(x0[:, i] * get(F, tuple(np.array(k) - E[i])) for i in range(3))
        s2f = sum(get(F, tuple(np.array(k) - 2 * E[i])) for i in range(3))
        s1h = sum(x0[:, i] * get(H, tuple(np.array(k) - E[i])) for i in range(3))
        s2h = sum(get(H, tuple(np.array(k) - 2 * E[i])) for i in range(3))
        F[k] = (-kappa * (s1h + s2h) - (2 * n - 1) * s1f - (n - 1) * s2f) / (n * r2)
        H[k] = -kappa * (s1f + s2f) / n
    return F
