"""Pins of the oracle's free-slip y walls (wall_y = 1: specular reflection at the
half-way walls y = -1/2 and y = ny - 1/2; the stencils mirror the boundary node,
with the y component of Phi odd), the lateral boundary of the opposed-jet setup
(Sec. 4.3).

What fixes the results: a plug flow parallel to the walls is a fixed point; the
walls exchange no tangential momentum, so mass, energy and the x and z momenta
are conserved exactly while the y momentum is not; and a shear mode whose
profile has zero slope at both walls, u_x = A cos(pi (y + 1/2) / ny), decays at
nu (pi / ny)^2, the free-slip (Neumann) eigenvalue. The fixed point and the
conservation laws hold under weak coupling and with temperature-dependent heat
capacities and transport as well.
"""
import numpy as np
import pytest

import physics_cases as pc
from paper_2004_11286_amd import workloads as W
from test_oracle_physics import wilke_mu


def test_plug_flow_between_free_slip_walls_is_fixed_point(oracle_mod):
    params, _ = W.ternary_tube(nx=6, ny=8, nz=3)
    X, P0, T0, u = [0.3, 0.3, 0.4], params["P0"], 1 / 3, (0.05, 0.0, 0.02)
    params = dict(params, wall_x=0, wall_y=1)
    s = oracle_mod.OracleSim(params)
    s.init_fields(**W.uniform_state(params, 6, 8, 3, X=X, p=P0, T=T0, u=u))
    p0 = s.populations()
    s.step(200)
    p1 = s.populations()
    stored = [0, 1, 3, 4]
    assert np.abs(p1[stored] - p0[stored]).max() <= 1e-13 * np.abs(p0[stored]).max()


@pytest.mark.parametrize("wall_x", [0, 1])
def test_free_slip_conserves_tangential_momentum(oracle_mod, wall_x):
    """Mass and energy are conserved with free-slip y walls (and x walls); with
    periodic x the x and z momenta are conserved too."""
    params, _ = W.ternary_tube(nx=10, ny=8, nz=4)
    params = dict(params, wall_x=wall_x, wall_y=1)
    f = W.random_near_equilibrium(params, 10, 8, 4, seed=13, X0=[0.3, 0.3, 0.4], p0=params["P0"], T0=1 / 3,
                                  amp=0.05, uamp=0.03)
    s = oracle_mod.OracleSim(params)
    s.init_fields(**f)
    c0 = s.conservation()
    s.step(200)
    c1 = s.conservation()
    M = params["M"]
    mass_like = list(range(M + 1)) + [M + 4]
    np.testing.assert_allclose(c1[mass_like], c0[mass_like], rtol=1e-12)
    if not wall_x:
        # periodic x: the free-slip walls exchange no x or z momentum (no-slip
        # bounce-back x walls would take both)
        np.testing.assert_allclose(c1[[M + 1, M + 3]], c0[[M + 1, M + 3]], atol=1e-12 * c0[M])
    assert abs(c1[M + 2] - c0[M + 2]) > 1e-6 * c0[M]              # the walls take y momentum


def test_neumann_shear_mode_decays_at_free_slip_rate(oracle_mod):
    ny, T0 = 64, 1.0 / 3.0
    masses, X, cvr = [2.0, 40.0], [0.5, 0.5], [2.5, 1.5]
    props = pc.mixture_props(masses, cvr, X)
    P0 = T0 / props["mbar"]
    params = {"nx": 1, "ny": ny, "nz": 1, "wall_x": 0, "wall_y": 1,
              **pc.species_block(masses, cvr, [0.5, 0.5], P0, 0.05)}
    k = np.pi / ny
    y = np.arange(ny, dtype=np.float64) + 0.5
    mode = np.cos(k * y)
    shape = (1, ny, 1)
    f = {"X": np.stack([np.full(shape, x) for x in X]), "p": np.full(shape, P0), "T": np.full(shape, T0),
         "u": np.stack([1e-4 * mode.reshape(shape), np.zeros(shape), np.zeros(shape)])}
    s = oracle_mod.OracleSim(params)
    s.init_fields(**f)
    ts, amps = [], []
    for t in range(0, 800, 50):
        amps.append(np.dot(s.read_moments()["u"][0, 0, :, 0], mode) * 2 / ny)
        ts.append(t)
        s.step(50)
    G = pc.fit_decay(ts, amps)
    rho = P0 / (props["R"] * T0)
    nu = wilke_mu(params["mu"], params["molar_mass"], X) / rho
    print("decay", G, "free-slip", nu * k * k)
    assert G / (nu * k * k) == pytest.approx(1.0, abs=0.01)


def _with_mode(params, weak, props, T=1 / 3):
    params = dict(params, weak=weak)
    if props:
        M = params["M"]
        cv = np.asarray(params["cv"], dtype=np.float64)
        params["cv_coef"] = np.stack([cv[a] * np.array([1.0, 0.4 / T, 0.1 / T ** 2, 0.05 * (a + 1) / T ** 3])
                                      for a in range(M)])
        params["transport_exp"] = np.concatenate([0.7 + 0.1 * np.arange(M), 0.8 + 0.05 * np.arange(M),
                                                  [1.75, T / 1.2]])
    return params


MODES = [(1, False), (0, True), (1, True)]


@pytest.mark.parametrize("weak,props", MODES)
def test_plug_flow_fixed_point_other_modes(oracle_mod, weak, props):
    """The plug flow between free-slip walls stays put under weak coupling (every
    lattice, species M's included, reflected) and with C_v(T) and T-dependent
    transport."""
    params, _ = W.ternary_tube(nx=6, ny=8, nz=3)
    X, P0, T0, u = [0.3, 0.3, 0.4], params["P0"], 1 / 3, (0.05, 0.0, 0.02)
    params = _with_mode(dict(params, wall_x=0, wall_y=1), weak, props)
    s = oracle_mod.OracleSim(params)
    s.init_fields(**W.uniform_state(params, 6, 8, 3, X=X, p=P0, T=T0, u=u))
    p0 = s.populations()
    s.step(200)
    p1 = s.populations()
    stored = list(range(5)) if weak else [0, 1, 3, 4]
    assert np.abs(p1[stored] - p0[stored]).max() <= 1e-13 * np.abs(p0[stored]).max()


@pytest.mark.parametrize("weak,props", MODES)
def test_free_slip_conservation_other_modes(oracle_mod, weak, props):
    """Periodic x, free-slip y walls: every species' mass, the mixture's mass and
    energy, and the x and z momenta are conserved in every mode; the walls take
    y momentum."""
    params, _ = W.ternary_tube(nx=10, ny=8, nz=4)
    params = _with_mode(dict(params, wall_x=0, wall_y=1), weak, props)
    f = W.random_near_equilibrium(params, 10, 8, 4, seed=23, X0=[0.3, 0.3, 0.4], p0=params["P0"], T0=1 / 3,
                                  amp=0.05, uamp=0.03)
    s = oracle_mod.OracleSim(params)
    s.init_fields(**f)
    c0 = s.conservation()
    s.step(200)
    c1 = s.conservation()
    M = params["M"]
    mass_like = list(range(M + 1)) + [M + 4]
    np.testing.assert_allclose(c1[mass_like], c0[mass_like], rtol=1e-12)
    np.testing.assert_allclose(c1[[M + 1, M + 3]], c0[[M + 1, M + 3]], atol=1e-12 * c0[M])
    assert abs(c1[M + 2] - c0[M + 2]) > 1e-6 * c0[M]
