"""The physical-unit front end (acoustic scaling, Sec. 4.1).

Inputs are synthetic but of realistic size (an H2 / Ar / CH4 mixture near 300 K
and 1 atm, the species of the Loschmidt experiment of Sec. 4.2; transport values
of the usual magnitudes, not data from a mechanism file). What fixes the
results: the dimensionless groups are the same before and after conversion;
the lattice gas constants and speed of sound map back exactly; and the oracle's
standing wave, run on the converted parameters, propagates at the physical
sqrt(gamma R T) once converted back (eq soundSpeed).
"""
import numpy as np
import pytest

import physics_cases as pc
from paper_2004_11286_amd import units as U

# H2, CH4, Ar: the species with most of the mass last (it is the slaved one under
# strong coupling, Sec. 3.5.2)
SPECIES = {
    "molar_mass": np.array([2.016, 16.043, 39.948]),        # g/mol
    "cv_molar": np.array([2.5, 3.3, 1.5]),
    "D": np.array([[1.5e-4, 7.7e-5, 8.3e-5], [7.7e-5, 2.2e-5, 2.2e-5], [8.3e-5, 2.2e-5, 1.8e-5]]),
    "mu": np.array([8.9e-6, 1.1e-5, 2.27e-5]),               # Pa s
    "lambda": np.array([0.18, 0.034, 0.0177]),              # W/(m K)
}
X_REF = np.array([0.3, 0.4, 0.3])
T_REF, P_REF = 300.0, 101325.0


def _convert(dx=7e-7, T_lat=0.3):
    return U.to_lattice(SPECIES, X_REF, T_REF, P_REF, dx=dx, T_lat=T_lat)


def _groups(m_g, cv, D, mu, lam, rho, p, T, u, L, Rgas):
    """Pr_a, Sc_ab, gamma_a, Mach, Reynolds and Peclet_ab of one unit system
    (cv mass based, Rgas the universal gas constant of the system)."""
    R_a = Rgas / m_g
    cp = cv + R_a
    pr = mu * cp / lam
    sc = mu[0] / (rho * D)
    gam = cp / cv
    Y = X_REF * m_g / (X_REF @ m_g)
    cvm, Rm = Y @ cv, Y @ R_a
    cs = np.sqrt((cvm + Rm) / cvm * Rm * T)
    return np.concatenate([pr, sc.ravel(), gam, [u / cs, rho * u * L / mu[0]], (u * L / D).ravel(),
                           [p / (rho * Rm * T)]])


def test_dimensionless_groups_are_invariant():
    params, s = _convert()
    m_kg = SPECIES["molar_mass"] / 1000.0
    cv_si = SPECIES["cv_molar"] * U.R_U_SI / m_kg
    rho = U.mixture_density(SPECIES["molar_mass"], X_REF, P_REF, T_REF)
    u_si, L_si = 12.0, 64 * s.dx
    si = _groups(m_kg, cv_si, SPECIES["D"], SPECIES["mu"], SPECIES["lambda"], rho, P_REF, T_REF, u_si, L_si,
                 U.R_U_SI)
    lat = _groups(params["molar_mass"], params["cv"], params["D"], params["mu"], params["lambda"], 1.0,
                  params["P0"], T_REF / s.temperature, u_si / s.velocity, 64.0, 1.0)
    np.testing.assert_allclose(lat, si, rtol=1e-12)


def test_scales_are_acoustic():
    """Each species' gas constant maps onto its lattice value 1/m_a, so the speed
    of sound scales with the velocity scale; the reference state has lattice
    density 1 and the chosen lattice temperature."""
    params, s = _convert()
    for m in SPECIES["molar_mass"]:
        assert U.R_U_SI / (m / 1000) == pytest.approx((1.0 / m) * s.specific_heat, rel=1e-13)
    cs_si = U.sound_speed(SPECIES["molar_mass"], SPECIES["cv_molar"], X_REF, T_REF)
    mbar = X_REF @ SPECIES["molar_mass"]
    cvm = X_REF @ SPECIES["cv_molar"]
    cs_lat = np.sqrt((cvm + 1) / cvm / mbar * 0.3)
    assert cs_lat * s.velocity == pytest.approx(cs_si, rel=1e-13)
    assert params["P0"] * mbar / 0.3 == pytest.approx(1.0, rel=1e-13)
    assert s.dt == pytest.approx(s.dx / s.velocity, rel=1e-15)


def test_fields_round_trip():
    _, s = _convert()
    rng = np.random.default_rng(1)
    X = rng.dirichlet([2, 2, 2], size=(4, 3, 2)).transpose(3, 0, 1, 2)
    p = P_REF * (1 + 0.01 * rng.uniform(-1, 1, (4, 3, 2)))
    T = T_REF * (1 + 0.05 * rng.uniform(-1, 1, (4, 3, 2)))
    u = rng.uniform(-20, 20, (3, 4, 3, 2))
    lat = U.fields_to_lattice(s, X, p, T, u)
    back = U.fields_to_physical(s, lat)
    for k, v in (("p", p), ("T", T), ("u", u), ("X", X)):
        np.testing.assert_allclose(back[k], v, rtol=1e-14)


def test_converted_mixture_carries_sound_at_physical_speed(oracle_mod):
    """The oracle run on the converted parameters: a 1e-5 standing pressure wave
    on a 64-node periodic line; its lattice speed times the velocity scale is
    sqrt(gamma R T) of the physical mixture within 1%."""
    params, s = _convert()
    nx = 64
    params = dict(params, nx=nx, ny=1, nz=1, wall_x=0)
    T_lat = T_REF / s.temperature
    P0 = params["P0"]
    x = np.arange(nx, dtype=np.float64)
    k = 2 * np.pi / nx
    sim = oracle_mod.OracleSim(params)
    sim.init_fields(**pc.line_fields(3, nx, X_REF, P0 * (1 + 1e-5 * np.cos(k * x)), T_lat, (0, 0, 0)))
    cs_si = U.sound_speed(SPECIES["molar_mass"], SPECIES["cv_molar"], X_REF, T_REF)
    nsteps = int(1.5 * nx / (cs_si / s.velocity))
    amp = np.zeros(nsteps)
    for t in range(nsteps):
        p = sim.read_moments()["p"][0, 0]
        amp[t] = np.dot(p - p.mean(), np.cos(k * x)) * 2 / nx
        sim.step(1)
    zc = pc.zero_crossings(amp)
    c_lat = np.pi / np.mean(np.diff(zc)) / k
    print("sound speed (m/s)", c_lat * s.velocity, "expected", cs_si, "lattice D", params["D"][0, 1],
          "mu/P0", params["mu"] / P0)
    assert c_lat * s.velocity / cs_si == pytest.approx(1.0, abs=0.01)


def test_rejects_bad_input():
    with pytest.raises(ValueError):
        U.make_scales(300.0, 0.0, 1e-6, 1.0)
    bad = dict(SPECIES, D=SPECIES["D"] + np.triu(np.ones((3, 3)) * 1e-6, 1))
    with pytest.raises(ValueError):
        U.to_lattice(bad, X_REF, T_REF, P_REF, dx=1e-6, T_lat=0.3)
