"""Independent one-dimensional Maxwell--Stefan solver (test helper).

Solves the Stefan--Maxwell relations at uniform pressure and temperature,
    d_x X_a = sum_b (X_a N_b - X_b N_a) / (c D_ab),
with zero net molar flux (closed tube, uniform molar density c), and
    d_t (c X_a) = - d_x N_a
by explicit finite volumes with zero-flux walls. This is the continuum limit
that the species kinetic model recovers (eqs constit2 and
smDiffusionCoefficients2 of the paper, Sec. 2.3); it shares nothing with the
lattice Boltzmann oracle.
"""
from __future__ import annotations

import numpy as np


def fluxes(X: np.ndarray, D: np.ndarray, c: float, dx: float) -> np.ndarray:
    """Molar fluxes N[M, n-1] at the interior faces of mole fractions X[M, n]."""
    M = X.shape[0]
    Xf = 0.5 * (X[:, 1:] + X[:, :-1])
    dX = (X[:, 1:] - X[:, :-1]) / dx
    nf = Xf.shape[1]
    # Unknowns N_1..N_{M-1}; N_M = -sum of the others. Row a (a < M):
    #   sum_{b != a} (X_a N_b - X_b N_a) / D_ab = c dX_a
    A = np.zeros((nf, M - 1, M - 1))
    for a in range(M - 1):
        for b in range(M):
            if b == a:
                continue
            if b < M - 1:
                A[:, a, b] += Xf[a] / D[a, b]
            else:
                A[:, a, :] -= (Xf[a] / D[a, b])[:, None]
            A[:, a, a] -= Xf[b] / D[a, b]
    rhs = (c * dX[: M - 1]).T[:, :, None]
    N = np.zeros((M, nf))
    N[: M - 1] = np.linalg.solve(A, rhs)[:, :, 0].T
    N[M - 1] = -N[: M - 1].sum(axis=0)
    return N


def solve(X0: np.ndarray, D: np.ndarray, t_end: float, dx: float = 1.0, c: float = 1.0,
          dt: float = 0.25, sample_every: float | None = None):
    """Integrate X[M, n] from t = 0 to t_end with forward Euler steps of dt.

    Returns (times, list of X arrays) sampled every ``sample_every`` (and at the end).
    """
    X = np.array(X0, dtype=np.float64)
    t = 0.0
    times, out = [0.0], [X.copy()]
    next_sample = sample_every
    while t < t_end - 1e-12:
        h = min(dt, t_end - t)
        N = fluxes(X, D, c, dx)
        div = np.zeros_like(X)
        div[:, :-1] += N
        div[:, 1:] -= N
        X = X - h * div / (c * dx)
        t += h
        if next_sample is not None and t >= next_sample - 1e-9:
            times.append(t)
            out.append(X.copy())
            next_sample += sample_every
    if times[-1] != t:
        times.append(t)
        out.append(X.copy())
    return np.array(times), out
