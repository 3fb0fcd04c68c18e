"""Small physical set-ups used to pin the oracle (test helper).

Each builder returns (params, fields) for a one-dimensional periodic run along x
and a closed-form expectation from the paper's hydrodynamic limit (Secs. 2.3, 3.3)
or from textbook linear acoustics of a viscous, heat-conducting ideal gas.
"""
from __future__ import annotations

import numpy as np

PR = 0.71


def species_block(masses, cv_over_R, mu_rel, P0, D, pr=PR, lam_rel=None):
    """Species data in lattice units (R_U = 1): cv_a = cv_over_R[a] / m_a;
    mu_a = mu_rel[a] * P0 (so omega = 2/(1 + 2 mu_rel) for a pure species);
    lambda_a = mu_a c_{p,a} / pr, or lam_rel[a] * P0 when given."""
    m = np.asarray(masses, dtype=np.float64)
    M = len(m)
    cv = np.asarray(cv_over_R, dtype=np.float64) / m
    cp = cv + 1.0 / m
    mu = np.asarray(mu_rel, dtype=np.float64) * P0
    lam = mu * cp / pr if lam_rel is None else np.asarray(lam_rel, dtype=np.float64) * P0
    Dm = np.full((M, M), float(D)) if np.isscalar(D) else np.asarray(D, dtype=np.float64)
    return {"M": M, "molar_mass": m, "cv": cv, "D": Dm, "mu": mu, "lambda": lam}


def mixture_props(masses, cv_over_R, X):
    m = np.asarray(masses, dtype=np.float64)
    X = np.asarray(X, dtype=np.float64)
    mbar = float(X @ m)
    Y = X * m / mbar
    cv = np.asarray(cv_over_R, dtype=np.float64) / m
    Cv = float(Y @ cv)
    R = 1.0 / mbar
    Cp = Cv + R
    return {"mbar": mbar, "R": R, "Cv": Cv, "Cp": Cp, "gamma": Cp / Cv}


def line_fields(M, nx, X, p, T, u):
    """Broadcast 1-D profiles of length nx (or scalars) onto a (1, 1, nx) grid."""
    def f(v):
        return np.broadcast_to(np.asarray(v, dtype=np.float64), (nx,)).reshape(1, 1, nx).copy()
    Xf = np.stack([f(X[a]) for a in range(M)])
    uf = np.stack([f(u[k]) for k in range(3)])
    return {"X": Xf, "p": f(p), "T": f(T), "u": uf}


def zero_crossings(a):
    return np.array([i + a[i] / (a[i] - a[i + 1]) for i in range(len(a) - 1) if a[i] * a[i + 1] < 0])


def fit_decay(ts, amps, skip=0):
    """Exponential decay rate from log-linear least squares."""
    ts = np.asarray(ts, dtype=np.float64)[skip:]
    amps = np.abs(np.asarray(amps, dtype=np.float64))[skip:]
    return -np.polyfit(ts, np.log(amps), 1)[0]
