"""Pins of the oracle's opposed jets (Sec. 4.3): two nozzles (equilibrium inlets)
on the rows nozzle_y0 <= y < nozzle_y1 of both x faces, free-slip walls on the
other rows of those faces, zero-gradient outlets at both y ends (wall_x = 3,
wall_y = 2; readings R24, R25).

What fixes the results: a gas at rest fed at its own state through both nozzles
stays put; two identical jets give a flow that is the mirror image of itself
about the mid-plane; and the steady counterflow on the stagnation line follows
the planar similarity solution of an independent one-dimensional solver
(tests/counterflow1d.py: continuity, transverse momentum with its pressure
eigenvalue, Stefan--Maxwell species fluxes), as the paper's lattice solution
follows its one-dimensional reference.
"""
import numpy as np
import pytest

from paper_2004_11286_amd import workloads as W

XL = np.array([0.1, 0.4, 0.5])
XR = np.array([0.0, 0.5, 0.5])


def jets(nx, ny, U=0.04, xl=XL, xr=XR, T0=1.0 / 3.0):
    params, _ = W.ternary_tube(nx=nx, ny=ny, nz=1, T0=T0)
    P0 = params["P0"]
    p = dict(params, wall_x=3, wall_y=2, nozzle=(ny // 10, ny - ny // 10),
             inlet=np.concatenate([xl, [P0, T0, U, 0.0, 0.0]]),
             inlet_right=np.concatenate([xr, [P0, T0, -U, 0.0, 0.0]]))
    M = params["M"]
    X = np.broadcast_to((0.5 * (xl + xr))[:, None, None, None], (M, 1, ny, nx)).copy()
    fields = {"X": X, "p": np.full((1, ny, nx), P0), "T": np.full((1, ny, nx), T0), "u": np.zeros((3, 1, ny, nx))}
    return p, fields


def test_jets_at_rest_fed_with_their_own_state_stay_put(oracle_mod):
    p, f = jets(12, 20, U=0.0, xl=XL, xr=XL)
    f["X"][:] = XL[:, None, None, None]
    o = oracle_mod.OracleSim(p)
    o.init_fields(**f)
    a = o.read_moments()
    o.step(200)
    b = o.read_moments()
    for k in a:
        np.testing.assert_allclose(b[k], a[k], rtol=0, atol=1e-12 * max(np.abs(a[k]).max(), 1e-3), err_msg=k)


def test_identical_jets_are_mirror_symmetric(oracle_mod):
    p, f = jets(14, 24, xl=XL, xr=XL)
    f["X"][:] = XL[:, None, None, None]
    o = oracle_mod.OracleSim(p)
    o.init_fields(**f)
    o.step(300)
    m = o.read_moments()
    assert np.abs(m["u"][0]).max() > 1e-3                    # the jets flow
    for k in ("X", "rho", "p", "T"):
        v = m[k]
        np.testing.assert_allclose(v, v[..., ::-1], rtol=0, atol=1e-12 * np.abs(v).max(), err_msg=k)
    ux = m["u"][0]
    np.testing.assert_allclose(ux, -ux[..., ::-1], rtol=0, atol=1e-12 * np.abs(ux).max())
    uy = m["u"][1]
    np.testing.assert_allclose(uy, uy[..., ::-1], rtol=0, atol=1e-12 * np.abs(uy).max())


def test_stagnation_line_follows_the_counterflow_similarity_solution(oracle_mod):
    """32 x 64 nodes, nozzles on 52 of the 64 rows, jets of 0.04 with different
    compositions (one species only in the left jet, as H2 in the paper's case),
    2500 steps (the profiles are steady well before). The 1D solver takes the
    lattice's mass fluxes and compositions at the first and last node of the
    stagnation line as its boundary values; its axial velocity and mole
    fractions are compared with the lattice's on that line. Measured: u within
    1.8-3.5% of its range, X within 0.013 (0.008 at 48 x 96)."""
    import counterflow1d as CF

    nx, ny = 32, 64
    p, f = jets(nx, ny)
    M = p["M"]
    o = oracle_mod.OracleSim(p)
    o.init_fields(**f)
    o.step(2500)
    m = o.read_moments()
    yc = ny // 2
    rho, u, X = m["rho"][0, yc], m["u"][0, 0, yc], m["X"][:, 0, yc]
    xs, uc, _, Xc, _ = CF.solve(nx - 1, rho[0] * u[0], rho[-1] * u[-1], X[:, 0], X[:, -1], p["molar_mass"], p["D"],
                                p["mu"], float(m["p"][0, yc].mean()), 1.0 / 3.0, composition="dirichlet")
    xi = np.arange(nx, dtype=float)
    du = np.abs(np.interp(xi, xs, uc) - u).max() / np.ptp(u)
    dX = max(np.abs(np.interp(xi, xs, Xc[k]) - X[k]).max() for k in range(M))
    print("u error / range", du, "largest X error", dX)
    assert du < 0.05
    assert dX < 0.02
    # the species of the left jet alone reaches across the stagnation point
    assert X[0, -1] < 1e-3 < X[0, nx // 2]
