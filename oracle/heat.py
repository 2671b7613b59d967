"""1D periodic heat equation u_t = u_xx by second-order central differences:
the method-of-lines system used to pin the time stepper against exact
Fourier-mode decay (test infrastructure).

On the grid x_i = i h, h = 1/n, the discrete Laplacian maps the Fourier mode
sin(2 pi k x + phi) to lambda_k times itself with
lambda_k = -(4/h^2) sin^2(pi k h); the semi-discrete solution of each mode is
therefore exp(lambda_k t), and one LSRK step multiplies it by R(dt lambda_k).
"""

import numpy as np

from .lsrk import lsrk_integrate


def heat_rhs(y, h):
    """(y_{i-1} - 2 y_i + y_{i+1}) / h^2 with periodic wrap."""
    return (np.roll(y, 1) - 2.0 * y + np.roll(y, -1)) / (h * h)


def heat_eigenvalues(n):
    k = np.arange(n)
    h = 1.0 / n
    return -(4.0 / h ** 2) * np.sin(np.pi * k * h) ** 2


def heat_integrate(y0, dt, nsteps):
    n = len(y0)
    h = 1.0 / n
    return lsrk_integrate(lambda y: heat_rhs(y, h), y0, dt, nsteps)
