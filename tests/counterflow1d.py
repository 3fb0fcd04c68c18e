"""Independent planar counterflow similarity solver (test helper).

Two opposed plug-flow jets at x = 0 and x = L, steady, isothermal, at the
pressure p0 (low Mach). Along the stagnation line the fields are taken in the
similarity form u = u(x), v = y V(x), T = T0, X_a = X_a(x), with the transverse
pressure gradient -dp/dy = y Lambda (Lambda an unknown constant):

    d(rho u)/dx          = -rho V                              (continuity)
    rho u dV/dx + rho V^2 = Lambda + d/dx (mu dV/dx)          (transverse momentum)
    d(rho u Y_a + j_a)/dx = -rho V Y_a                          (species)
    dX_a/dx = (m/rho) sum_b (X_a j_b / m_b - X_b j_a / m_a) / D_ab   (Stefan--Maxwell)

with rho = p0 m / T0 (R_U = 1), m the mean molar mass, j_a the diffusive mass
fluxes (sum zero) and mu Wilke's mixture viscosity. Boundary conditions: the
given mass fluxes rho u at both ends, V = 0 (plug flow), and the flux form of the
inlet composition, rho u Y_a + j_a = rho u Y_a,in. This is the one-dimensional
reduction that counterflow solvers use for opposed jets (the paper compares its
opposed jets, Sec. 4.3, with such a solution); it shares nothing with the lattice
Boltzmann oracle. Solved with scipy's collocation solver.
"""
from __future__ import annotations

import numpy as np
from scipy.integrate import solve_bvp


def wilke_mu(X, m, mu):
    """Wilke's mixture viscosity of mole fractions X[M, n]."""
    M = len(m)
    out = np.zeros(X.shape[1])
    for a in range(M):
        den = np.zeros(X.shape[1])
        for b in range(M):
            phi = (1.0 + np.sqrt(mu[a] / mu[b]) * (m[b] / m[a]) ** 0.25) ** 2 / np.sqrt(8.0 * (1.0 + m[a] / m[b]))
            den += phi * X[b]
        out += mu[a] * X[a] / den
    return out


def solve(L, F0, FL, XL, XR, m, D, mu, p0, T0, n=201, tol=1e-8, composition="flux"):
    """Steady counterflow between x = 0 (mass flux F0 > 0, inlet mole fractions
    XL) and x = L (mass flux FL < 0, inlet XR). composition "flux": the inlet
    composition enters by convection and diffusion (rho u Y + j = rho u Y_in);
    "dirichlet": X = XL and XR at the ends. Returns (x, u, V, X[M, n], Lambda)."""
    m = np.asarray(m, float)
    D = np.asarray(D, float)
    mu = np.asarray(mu, float)
    M = len(m)
    XL = np.asarray(XL, float)
    XR = np.asarray(XR, float)
    YL = XL * m / np.dot(XL, m)
    YR = XR * m / np.dot(XR, m)

    def unpack(y):
        F, V, W = y[0], y[1], y[2]
        Lam = y[3]
        Xa = y[4:4 + M - 1]
        ja = y[4 + M - 1:4 + 2 * (M - 1)]
        X = np.vstack([Xa, 1.0 - Xa.sum(axis=0)])
        j = np.vstack([ja, -ja.sum(axis=0)])
        return F, V, W, Lam, X, j

    def rhs(x, y):
        F, V, W, Lam, X, j = unpack(y)
        mbar = m @ X
        rho = p0 * mbar / T0
        dV = W / wilke_mu(X, m, mu)
        dX = np.zeros_like(X)
        for a in range(M):
            for b in range(M):
                if b != a:
                    dX[a] += (X[a] * j[b] / m[b] - X[b] * j[a] / m[a]) / D[a, b]
            dX[a] *= mbar / rho
        dmbar = m @ dX
        dY = (m[:, None] * dX * mbar - (m[:, None] * X) * dmbar) / mbar ** 2
        dF = -rho * V
        dW = F * dV + rho * V * V - Lam
        dj = -F * dY[:M - 1]
        return np.vstack([dF, dV, dW, np.zeros_like(Lam), dX[:M - 1], dj])

    def bc(ya, yb):
        Fa, Va, _, _, Xa, ja = unpack(ya[:, None])
        Fb, Vb, _, _, Xb, jb = unpack(yb[:, None])
        Ya = (Xa[:, 0] * m) / np.dot(Xa[:, 0], m)
        Yb = (Xb[:, 0] * m) / np.dot(Xb[:, 0], m)
        res = [Fa[0] - F0, Va[0], Fb[0] - FL, Vb[0]]
        if composition == "dirichlet":
            res += list(Xa[:M - 1, 0] - XL[:M - 1])
            res += list(Xb[:M - 1, 0] - XR[:M - 1])
        else:
            res += list(F0 * Ya[:M - 1] + ja[:M - 1, 0] - F0 * YL[:M - 1])
            res += list(FL * Yb[:M - 1] + jb[:M - 1, 0] - FL * YR[:M - 1])
        return np.array(res)

    x = np.linspace(0.0, L, n)
    s = x / L
    y0 = np.zeros((4 + 2 * (M - 1), n))
    y0[0] = F0 + (FL - F0) * s
    rho0 = p0 * np.dot(0.5 * (XL + XR), m) / T0
    y0[1] = (F0 - FL) / (L * rho0) * 6 * s * (1 - s)      # V ~ the strain, zero at the nozzles
    y0[3] = 0.0
    for a in range(M - 1):
        y0[4 + a] = XL[a] + (XR[a] - XL[a]) * s
    sol = solve_bvp(rhs, bc, x, y0, tol=tol, max_nodes=100000)
    if not sol.success:
        raise RuntimeError("counterflow solver: " + sol.message)
    F, V, W, Lam, X, j = unpack(sol.sol(x))
    rho = p0 * (m @ X) / T0
    return x, F / rho, V, X, float(Lam[0])
