"""Physical-unit front end: acoustic scaling of species and transport data into
the lattice units of the library (Sec. 4.1 of the paper: the speed of sound at a
reference composition and temperature makes velocities non-dimensional, and the
transport coefficients are converted with the same scaling).

Lattice units: dx = dt = 1, R_U = 1 and molar masses in g/mol, so a species of
molar mass m_a has gas constant 1/m_a. Physical units: SI, with R_U = 8.314...
J/(mol K) and molar masses in kg/mol.

Scales. The user picks the lattice temperature T_lat that the reference
temperature T_ref maps to (this sets how far the lattice state sits from the
stability limit R_a T + u^2 < 1), the grid spacing dx, and the lattice density
of the reference state (1 by default). Because the gas constant of every species
must map onto its lattice value,
    R_phys = R_lat U^2 / Theta,    Theta = T_ref / T_lat,
the velocity scale is U = sqrt(1000 R_U Theta) m/s per lattice unit and the
time step dt = dx / U. The speed of sound sqrt(gamma R T), with gamma the same
number in both unit systems, then scales by U: acoustic scaling. Every other
quantity follows from U, dx, Theta and the density scale rho_s:
    pressure        rho_s U^2          diffusivity     U dx
    viscosity       rho_s U dx         specific heat   U^2 / Theta
    conductivity    rho_s U dx U^2 / Theta
so the dimensionless groups (Mach, Reynolds, Prandtl, Schmidt, Peclet, gamma)
are the same in both systems.

This module only converts numbers; it holds none of the lattice arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

R_U_SI = 8.314462618          # J / (mol K)


@dataclass(frozen=True)
class Scales:
    """Physical value = lattice value x scale."""
    dx: float                  # m
    dt: float                  # s
    velocity: float            # m/s
    temperature: float         # K
    density: float             # kg/m^3
    pressure: float            # Pa
    diffusivity: float         # m^2/s
    viscosity: float           # Pa s
    conductivity: float        # W/(m K)
    specific_heat: float       # J/(kg K)


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def make_scales(T_ref: float, T_lat: float, dx: float, rho_ref: float, rho_lat: float = 1.0) -> Scales:
    """Scales of acoustic scaling for a reference temperature T_ref (K) mapped to
    the lattice temperature T_lat, grid spacing dx (m), and a reference density
    rho_ref (kg/m^3) mapped to rho_lat."""
    if not (T_ref > 0 and T_lat > 0 and dx > 0 and rho_ref > 0 and rho_lat > 0):
        raise ValueError("T_ref, T_lat, dx and the densities must be positive")
    theta = T_ref / T_lat
    U = np.sqrt(1000.0 * R_U_SI * theta)        # molar masses: g/mol on the lattice, kg/mol in SI
    rho_s = rho_ref / rho_lat
    return Scales(dx=dx, dt=dx / U, velocity=U, temperature=theta, density=rho_s, pressure=rho_s * U * U,
                  diffusivity=U * dx, viscosity=rho_s * U * dx, conductivity=rho_s * U * dx * U * U / theta,
                  specific_heat=U * U / theta)


def mixture_density(molar_mass_g, X, p: float, T: float) -> float:
    """Ideal-gas density (kg/m^3) of a mixture of mole fractions X at p (Pa), T (K)."""
    m = float(_f64(X) @ _f64(molar_mass_g)) / 1000.0   # kg/mol
    return p * m / (R_U_SI * T)


def to_lattice(species: dict, X_ref, T_ref: float, p_ref: float, dx: float, T_lat: float, rho_lat: float = 1.0):
    """Lattice parameter block and scales from physical species data.

    species: "molar_mass" [M] g/mol; "cv_molar" [M] molar heat capacity at
    constant volume over R_U (C_v / R_U, e.g. 1.5 for a monatomic gas);
    "D" [M, M] binary diffusivities (m^2/s) at (T_ref, p_ref), symmetric, the
    diagonal the self-diffusivity (for the sums over b = a); "mu" [M] Pa s;
    "lambda" [M] W/(m K). X_ref: the reference composition; T_ref (K), p_ref (Pa).

    Returns (params, scales): params holds M, molar_mass, cv, D, mu, lambda in
    lattice units and P0, the lattice pressure of the reference state (with the
    reference density mapped to rho_lat), ready for mclbm.Sim once nx, ny, nz
    are added."""
    m = _f64(species["molar_mass"])
    M = len(m)
    cvm = _f64(species["cv_molar"])
    D = _f64(species["D"]).reshape(M, M)
    mu, lam = _f64(species["mu"]), _f64(species["lambda"])
    if not np.allclose(D, D.T, rtol=0, atol=0):
        raise ValueError("D must be symmetric")
    rho_ref = mixture_density(m, X_ref, p_ref, T_ref)
    s = make_scales(T_ref, T_lat, dx, rho_ref, rho_lat)
    cv_si = cvm * R_U_SI / (m / 1000.0)          # J/(kg K)
    params = {"M": M, "molar_mass": m.copy(), "cv": cv_si / s.specific_heat, "D": D / s.diffusivity,
              "mu": mu / s.viscosity, "lambda": lam / s.conductivity, "P0": p_ref / s.pressure}
    return params, s


def fields_to_lattice(s: Scales, X, p, T, u) -> dict:
    """Physical fields (p in Pa, T in K, u in m/s) in lattice units."""
    return {"X": _f64(X), "p": _f64(p) / s.pressure, "T": _f64(T) / s.temperature, "u": _f64(u) / s.velocity}


def fields_to_physical(s: Scales, fields: dict) -> dict:
    """Lattice fields (as read back by mclbm.Sim.read_moments) in SI units."""
    out = dict(fields)
    for k, scale in (("p", s.pressure), ("T", s.temperature), ("u", s.velocity), ("rho", s.density)):
        if k in fields:
            out[k] = _f64(fields[k]) * scale
    return out


def sound_speed(molar_mass_g, cv_molar, X, T: float) -> float:
    """sqrt(gamma R T) (eq soundSpeed) in SI for a mixture of mole fractions X at T (K),
    with constant molar heat capacities."""
    X = _f64(X)
    m = float(X @ _f64(molar_mass_g)) / 1000.0
    cv_molar_mix = float(X @ _f64(cv_molar))
    gamma = (cv_molar_mix + 1.0) / cv_molar_mix
    return float(np.sqrt(gamma * R_U_SI / m * T))
