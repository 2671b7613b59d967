"""Low-storage five-stage fourth-order Runge-Kutta (paper, Section 5.2:
the 2D and 3D experiments are integrated with the low-storage 4th-order
five-stage scheme of Carpenter and Kennedy).

The paper cites the scheme without printing its coefficients; the values
below are the published Carpenter-Kennedy (1994) 2N-storage table, checked
by the tests against the eight fourth-order conditions through the Butcher
tableau this module derives from them.

2N-storage form, stage i = 1..5 (the system here is autonomous, so the
stage times C_i are not needed by the right-hand side):

    res <- A_i res + dt f(y)
    y   <- y + B_i res
"""

from fractions import Fraction as F

import numpy as np

A_RAT = [F(0), F(-567301805773, 1357537059087), F(-2404267990393, 2016746695238),
         F(-3550918686646, 2091501179385), F(-1275806237668, 842570457699)]
B_RAT = [F(1432997174477, 9575080441755), F(5161836677717, 13612068292357),
         F(1720146321549, 2090206949498), F(3134564353537, 4481467310338),
         F(2277821191437, 14882151754819)]
C_RAT = [F(0), F(1432997174477, 9575080441755), F(2526269341429, 6820363962896),
         F(2006345519317, 3224310063776), F(2802321613138, 2924317926251)]


class LSRK54:
    A = np.array([float(a) for a in A_RAT])
    B = np.array([float(b) for b in B_RAT])
    C = np.array([float(c) for c in C_RAT])
    stages = 5


def butcher_tableau(exact=False):
    """Butcher form (a, b, c) of the 2N-storage scheme.

    With k_j = dt f(Y_j): res_i = sum_{j<=i} (prod_{l=j+1..i} A_l) k_j and
    Y_{i+1} = y0 + sum_{m<=i} B_m res_m, so
    a_{i+1,j} = sum_{m=j..i} B_m prod_{l=j+1..m} A_l and b_j = a_{6,j}.
    """
    A = A_RAT if exact else [float(a) for a in A_RAT]
    B = B_RAT if exact else [float(b) for b in B_RAT]
    s = 5
    zero = F(0) if exact else 0.0
    one = F(1) if exact else 1.0
    full = [[zero] * s for _ in range(s + 1)]    # rows: Y_1..Y_5, then b
    for i in range(s):            # after stage i (0-based) -> row i+1
        for j in range(i + 1):
            tot = zero
            for m in range(j, i + 1):
                prod = one
                for l in range(j + 1, m + 1):
                    prod *= A[l]
                tot += B[m] * prod
            full[i + 1][j] = tot
    a = [row[:] for row in full[:s]]
    b = full[s][:]
    c = [sum(row) for row in a]
    return a, b, c


def stability_polynomial_coeffs():
    """Coefficients gamma_0..gamma_5 of R(z) = sum gamma_k z^k for y' = lambda y,
    from the Butcher form: gamma_0 = 1, gamma_k = b^T a^{k-1} 1 (exact)."""
    a, b, _ = butcher_tableau(exact=True)
    s = 5
    vec = [F(1)] * s
    coeffs = [F(1)]
    for _ in range(s):
        coeffs.append(sum(bi * vi for bi, vi in zip(b, vec)))
        vec = [sum(a[i][j] * vec[j] for j in range(s)) for i in range(s)]
    return coeffs


def lsrk_integrate(f, y0, dt, nsteps, callback=None):
    """Advance y' = f(y) by ``nsteps`` steps of size ``dt``; plain loop.

    ``callback(n, y)`` (optional) is called after every full step n = 1..nsteps.
    """
    y = np.array(y0, copy=True)
    if not np.iscomplexobj(y):
        y = y.astype(np.float64)
    res = np.zeros_like(y)
    for n in range(nsteps):
        for i in range(LSRK54.stages):
            res = LSRK54.A[i] * res + dt * f(y)
            y = y + LSRK54.B[i] * res
        if callback is not None:
            callback(n + 1, y)
    return y
