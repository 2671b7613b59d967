"""Parareal iteration over time slices -- oracle (test infrastructure).

The paper does not define a parallel-in-time correction; this is the
standard parareal iteration (Lions, Maday, Turinici 2001) written from its
definition, with the paper's WADG-LSRK sweep as both propagators:

    U_0^k = y0 for all k,
    U_{s+1}^0 = G(U_s^0),
    U_{s+1}^{k+1} = G(U_s^{k+1}) + F(U_s^k) - G(U_s^k),    s = 0..S-1,

F = fine propagator over one slice (nsteps_fine LSRK steps of dt),
G = coarse propagator over the same slice (nsteps_coarse steps of
nsteps_fine*dt/nsteps_coarse).  The iteration stops when the largest
relative change max_s ||U_s^{k+1} - U_s^k|| / ||U_s^{k+1}|| (s = 1..S) is
<= tol, or after max_iter iterations.  By construction U_s^k equals the
serial fine solution F^s(y0) exactly (up to rounding) for s <= k.
"""

import numpy as np


def parareal(F, G, y0, S, max_iter, tol):
    """Serial reference implementation.  F, G: callables on one state.
    Returns (U [S+1 states], iterations done, last relative change)."""
    y0 = np.array(y0, copy=True)
    U = [y0 if np.iscomplexobj(y0) else y0.astype(np.float64)]
    Gold = []
    for s in range(S):
        g = G(U[s])
        Gold.append(g)
        U.append(g)
    it, change = 0, np.inf
    for k in range(max_iter):
        Fv = [F(U[s]) for s in range(S)]          # independent: the parallel part
        Unew = [U[0]]
        for s in range(S):
            g = G(Unew[s])
            Unew.append(g + Fv[s] - Gold[s])
            Gold[s] = g
        change = max(np.linalg.norm(Unew[s] - U[s]) / np.linalg.norm(Unew[s])
                     for s in range(1, S + 1))
        U = Unew
        it = k + 1
        if change <= tol:
            break
    return np.stack(U), it, change


def wadg_propagators(oracle, dt, nsteps_fine, nsteps_coarse):
    """F and G built from a WADGOracle: both advance one slice of length
    dT = dt * nsteps_fine, G with nsteps_coarse larger steps."""
    dT = dt * nsteps_fine
    F = lambda q: oracle.integrate(q, dt, nsteps_fine)                      # noqa: E731
    G = lambda q: oracle.integrate(q, dT / nsteps_coarse, nsteps_coarse)    # noqa: E731
    return F, G
