"""Seeded synthetic workloads: species parameters and initial fields.

This module is shared by the GPU path's tests and benchmark and by the CPU
oracle's tests. It holds configuration recipes only (grid sizes, species data,
initial mole fractions, pressure, temperature and velocity fields) and none of
the lattice Boltzmann arithmetic. Every array it returns is float64; fields are
shaped ``[..., nz, ny, nx]`` (x fastest in memory).

Units are lattice units with R_U = 1: a species of molar mass m_a has gas
constant 1/m_a, and a pressure p at temperature T and mean molar mass m gives
density p m / T.

The paper (Sec. 4) runs physical setups (a Loschmidt tube, a three-band shear
layer) with transport data from GRI-Mech 3.0, which is not available here. The
recipes below keep the structure of those setups (sizes, walls, band layout,
composition contrast) with lattice-unit species data chosen to be stable.
"""
from __future__ import annotations

import numpy as np

PRANDTL = 0.71


def _species(masses, gamma=5.0 / 3.0, D=None, P0=None, mu=None, pr=PRANDTL):
    """Species parameter block. cv_a = 1/((gamma-1) m_a) (mass based, R_U = 1);
    lambda_a = mu_a c_{p,a} / Pr with c_{p,a} = gamma cv_a."""
    m = np.asarray(masses, dtype=np.float64)
    g = np.broadcast_to(np.asarray(gamma, dtype=np.float64), m.shape)
    cv = 1.0 / ((g - 1.0) * m)
    cp = g * cv
    mu = np.broadcast_to(np.asarray(mu, dtype=np.float64), m.shape).copy()
    lam = mu * cp / pr
    return {"M": len(m), "molar_mass": m, "cv": cv, "D": np.asarray(D, dtype=np.float64),
            "mu": mu, "lambda": lam}


def full_D(offdiag: dict, M: int) -> np.ndarray:
    """Symmetric diffusivity matrix from {(a, b): D_ab} (0-based, a != b); the
    diagonal (self-diffusivity, needed by the sums over b = a) is the mean of
    the row's off-diagonal entries."""
    D = np.zeros((M, M))
    for (a, b), v in offdiag.items():
        D[a, b] = D[b, a] = v
    for a in range(M):
        D[a, a] = np.mean([D[a, b] for b in range(M) if b != a])
    return D


def _grid(nx, ny, nz):
    z, y, x = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    return x.astype(np.float64), y.astype(np.float64), z.astype(np.float64)


def _pack(params, X, p, T, u, **meta):
    params = dict(params)
    params.update(meta)
    return params, {"X": np.ascontiguousarray(X), "p": np.ascontiguousarray(p),
                    "T": np.ascontiguousarray(T), "u": np.ascontiguousarray(u)}


# ----------------------------------------------------------------------------- C1
def binary_interdiffusion(nx=64, ny=8, nz=8, D12=0.05, T0=1.0 / 3.0, x_left=0.8, x_right=0.2,
                          masses=(2.0, 40.0), omega0=1.0):
    """Binary interdiffusion of a step on a periodic grid (masses 2 and 40 by
    default, gamma = 5/3, D_12 = 0.05, T = 1/3). X_1 = x_left for x < nx/2, else
    x_right; uniform pressure chosen so the mean density is 1; zero velocity.
    Viscosities give omega = omega0 at the mean pressure."""
    mbar = 0.5 * (x_left * masses[0] + (1 - x_left) * masses[1]) + \
        0.5 * (x_right * masses[0] + (1 - x_right) * masses[1])
    P0 = T0 / mbar
    mu = (1.0 / omega0 - 0.5) * P0
    M = 2
    D = np.full((M, M), D12)
    sp = _species(masses, D=D, mu=mu)
    x, y, z = _grid(nx, ny, nz)
    X1 = np.where(x < nx // 2, x_left, x_right)
    X = np.stack([X1, 1.0 - X1])
    shape = x.shape
    return _pack(sp, X, np.full(shape, P0), np.full(shape, T0), np.zeros((3,) + shape),
                 nx=nx, ny=ny, nz=nz, wall_x=0, slaved=1, P0=P0,
                 workload=f"binary interdiffusion {nx}x{ny}x{nz} periodic")


# ----------------------------------------------------------------------------- C2
TERNARY_D = {(0, 1): 0.083, (0, 2): 0.068, (1, 2): 0.017}


def ternary_tube(nx=256, ny=4, nz=4, T0=1.0 / 3.0, masses=(2.0, 16.0, 40.0),
                 x_left=(0.0, 0.5, 0.5), x_right=(0.5, 0.0, 0.5), Doff=None, omega0=1.0):
    """Ternary uphill-diffusion tube (the structure of the paper's Loschmidt-tube
    runs, Sec. 4.2): walls at both x ends, periodic in y and z, left half and
    right half at different compositions, uniform pressure and temperature, zero
    velocity. The last species is the one slaved to the mixture (largest mass
    fraction everywhere)."""
    Doff = TERNARY_D if Doff is None else Doff
    M = len(masses)
    D = full_D(Doff, M)
    ml = float(np.dot(x_left, masses))
    mr = float(np.dot(x_right, masses))
    P0 = T0 / (0.5 * (ml + mr))
    mu = (1.0 / omega0 - 0.5) * P0
    sp = _species(masses, D=D, mu=mu)
    x, y, z = _grid(nx, ny, nz)
    left = x < nx // 2
    X = np.stack([np.where(left, x_left[a], x_right[a]) for a in range(M)])
    shape = x.shape
    return _pack(sp, X, np.full(shape, P0), np.full(shape, T0), np.zeros((3,) + shape),
                 nx=nx, ny=ny, nz=nz, wall_x=1, slaved=M - 1, P0=P0,
                 workload=f"ternary uphill-diffusion tube {nx}x{ny}x{nz} walls")


# ----------------------------------------------------------------------------- C3
def shear_layer(nx=256, ny=256, nz=256, seed=2004, T0=1.0, masses=(2.0, 28.0), D12=0.1,
                omega0=1.0, u0=0.1, x_outer=0.9, x_middle=0.1, delta=4.0, noise=1e-3, modes=8, kmax=4):
    """Three-band Kelvin--Helmholtz shear layer (the layout of Sec. 4.5, eq icKHI):
    periodic box, interfaces at y = ny/4 and 3 ny/4 with tanh profiles of
    thickness ``delta``; u_x = +u0 in the outer bands and -u0 in the middle band;
    X_1 = x_outer outside and x_middle inside along the same profile; uniform
    pressure and temperature.

    Perturbation: seeded and band-limited, like the paper's long-wave sinusoids
    (eqs uyKHI, uzKHI): on every velocity component a sum of ``modes`` Fourier
    modes with integer wavenumbers |k_x|, |k_y|, |k_z| <= kmax, uniform random
    amplitudes and phases, scaled to a maximum of ``noise``. (White noise at the
    grid scale is not used: it drives the scheme unstable within tens of steps.)

    Defaults: T = 1 (sound speed 1/3 at X = 0.5, so u0 = 0.1 is Mach 0.3), D_12 =
    0.1, omega = 1 at the mean pressure. With D_12 = 0.05 the light species'
    lattice (R_a T = 0.5 in the hydrogen-rich band) becomes unstable, and with
    omega above about 1.3 the layer blows up within a few hundred steps."""
    M = 2
    D = np.full((M, M), D12)
    mhalf = 0.5 * (masses[0] + masses[1])
    P0 = T0 / mhalf
    mu = (1.0 / omega0 - 0.5) * P0
    sp = _species(masses, D=D, mu=mu)
    x, y, z = _grid(nx, ny, nz)
    y1, y2 = ny / 4.0, 3.0 * ny / 4.0
    # band indicator: 0 in the outer bands, 1 in the middle band
    s = 0.5 * (np.tanh((y - y1) / delta) - np.tanh((y - y2) / delta))
    ux = u0 * (1.0 - 2.0 * s)
    X1 = x_outer + (x_middle - x_outer) * s
    X = np.stack([X1, 1.0 - X1])
    rng = np.random.Generator(np.random.PCG64(seed))
    u = np.stack([ux, np.zeros_like(ux), np.zeros_like(ux)])
    if noise > 0.0:
        for c in range(3):
            pert = np.zeros_like(ux)
            for _ in range(modes):
                k = rng.integers(-kmax, kmax + 1, size=3)
                amp = rng.uniform(-1.0, 1.0)
                ph = rng.uniform(0.0, 2.0 * np.pi)
                pert += amp * np.sin(2.0 * np.pi * (k[0] * x / nx + k[1] * y / ny + k[2] * z / nz) + ph)
            m = np.abs(pert).max()
            if m > 0:
                u[c] += noise * pert / m
    shape = x.shape
    return _pack(sp, X, np.full(shape, P0), np.full(shape, T0), u,
                 nx=nx, ny=ny, nz=nz, wall_x=0, slaved=1, P0=P0,
                 workload=f"binary Kelvin-Helmholtz shear layer {nx}x{ny}x{nz} periodic")


# ----------------------------------------------------------------------------- C4
SLAVED_MIN_Y = 0.3           # minimum mass fraction of the slaved species in the ensemble
ENSEMBLE_MASSES = (2.0, 16.0, 28.0, 40.0)


def tube_ensemble(ntubes=512, ny=16, nz=16, lmin=32, lmax=256, seed=11286, T0=1.0 / 3.0,
                  omega0=1.0, min_slaved_y=SLAVED_MIN_Y):
    """Independent ternary tubes with walls at both x ends (the Loschmidt-tube
    structure of Sec. 4.2), one species set and composition per tube: three
    distinct molar masses from {2, 16, 28, 40}, D_ab ~ U[0.01, 0.1], left and
    right mole fractions ~ Dirichlet(1, 1, 1), uniform pressure giving mean
    density 1, T = 1/3, zero velocity. The slaved species is the one with the
    largest minimum mass fraction. Strong coupling (Sec. 3.5.2) needs the slaved
    species to carry a good part of the mass everywhere: compositions whose
    slaved species falls below ``min_slaved_y`` in mass fraction on either side
    are drawn again. Of unconditioned Dirichlet(1, 1, 1) draws about 10% have the
    slaved species under 0.2 and 23% under 0.3 somewhere; in the oracle itself,
    tubes whose slaved species was near 0.1 to 0.2 on one side went negative at
    the interface within a hundred steps.
    Returns a list of (params, fields)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    tubes = []
    for _ in range(ntubes):
        L = int(rng.integers(lmin, lmax + 1))
        masses = np.sort(rng.choice(ENSEMBLE_MASSES, size=3, replace=False))
        d = rng.uniform(0.01, 0.1, size=3)
        while True:
            xl = rng.dirichlet([1.0, 1.0, 1.0])
            xr = rng.dirichlet([1.0, 1.0, 1.0])
            yl = xl * masses / np.dot(xl, masses)
            yr = xr * masses / np.dot(xr, masses)
            ymin = np.minimum(yl, yr)
            if ymin.max() >= min_slaved_y:
                break
        # order species so the slaved one (largest minimum mass fraction) is last
        order = np.argsort(ymin, kind="stable")
        masses, xl, xr = masses[order], xl[order], xr[order]
        Doff = {}
        pairs = [(0, 1), (0, 2), (1, 2)]
        inv = {int(o): k for k, o in enumerate(order)}
        for (a, b), v in zip(pairs, d):
            Doff[(min(inv[a], inv[b]), max(inv[a], inv[b]))] = float(v)
        tubes.append(ternary_tube(nx=L, ny=ny, nz=nz, T0=T0, masses=tuple(masses),
                                  x_left=tuple(xl), x_right=tuple(xr), Doff=Doff,
                                  omega0=omega0))
    return tubes


# ----------------------------------------------------------------------------- opposed jets
# Species of the opposed jets of Sec. 4.3, ordered so that N2 (the carrier of both
# jets, slaved under strong coupling) is last: H2, O2, H2O, N2.
JETS_SPECIES = ("H2", "O2", "H2O", "N2")
JETS_MASSES = (2.0, 32.0, 18.0, 28.0)
JETS_LEFT = (0.1, 0.0, 0.05, 0.85)      # the jet at x = 0 (Sec. 4.3)
JETS_RIGHT = (0.0, 0.1, 0.0, 0.9)       # the jet at x = nx - 1
# Binary diffusivities near 300 K and 1 atm in cm^2/s, rounded (orders of
# magnitude from gas-kinetic tables), in the species order above; scaled
# uniformly into lattice units by the recipe.
JETS_D_PHYS = {(0, 1): 0.81, (0, 2): 0.95, (0, 3): 0.78, (1, 2): 0.26, (1, 3): 0.21, (2, 3): 0.26}


def opposed_jets(nx=200, ny=400, nz=1, U=0.04, T0=1.0, omega0=1.0, d_max=0.05, gamma=1.4, nozzle_frac=0.1):
    """The planar opposed jets of Sec. 4.3: 200 x 400 x 1 nodes, the nozzles
    nx - 1 apart on the rows nozzle_frac ny <= y < (1 - nozzle_frac) ny of both x
    faces, free-slip walls beside them, zero-gradient outlets at both y ends
    (wall_x = 3, wall_y = 2). The jets carry the paper's compositions with equal
    momentum (the left one at U, the right one at U sqrt(rho_l / rho_r)) at the
    common pressure and temperature; the interior starts at rest at the mean
    composition. Lattice-unit species data: the diffusivities of JETS_D_PHYS
    scaled so the largest is d_max, one ratio of specific heats for all species,
    viscosities giving omega = omega0 at the mean state."""
    M = len(JETS_MASSES)
    m = np.asarray(JETS_MASSES)
    xl, xr = np.asarray(JETS_LEFT), np.asarray(JETS_RIGHT)
    scale = d_max / max(JETS_D_PHYS.values())
    D = full_D({k: v * scale for k, v in JETS_D_PHYS.items()}, M)
    x0 = 0.5 * (xl + xr)
    P0 = T0 / float(np.dot(x0, m))                  # mean density 1
    mu = (1.0 / omega0 - 0.5) * P0
    sp = _species(JETS_MASSES, gamma=gamma, D=D, mu=mu)
    ur = U * np.sqrt(float(np.dot(xl, m)) / float(np.dot(xr, m)))
    noz = (int(round(nozzle_frac * ny)), int(round((1.0 - nozzle_frac) * ny)))
    x, y, z = _grid(nx, ny, nz)
    shape = x.shape
    X = np.broadcast_to(x0[:, None, None, None], (M,) + shape)
    return _pack(sp, X, np.full(shape, P0), np.full(shape, T0), np.zeros((3,) + shape),
                 nx=nx, ny=ny, nz=nz, wall_x=3, wall_y=2, nozzle=noz, slaved=M - 1, P0=P0,
                 inlet=np.concatenate([xl, [P0, T0, U, 0.0, 0.0]]),
                 inlet_right=np.concatenate([xr, [P0, T0, -ur, 0.0, 0.0]]),
                 workload=f"opposed jets {nx}x{ny}x{nz} (H2/O2/H2O/N2)")


# ----------------------------------------------------------------------------- helpers
def uniform_state(params: dict, nx, ny, nz, X, p, T, u=(0.0, 0.0, 0.0)):
    """Uniform fields (used for fixed-point and single-node tests)."""
    shape = (nz, ny, nx)
    M = params["M"]
    Xf = np.stack([np.full(shape, float(X[a])) for a in range(M)])
    uf = np.stack([np.full(shape, float(c)) for c in u])
    return {"X": Xf, "p": np.full(shape, float(p)), "T": np.full(shape, float(T)), "u": uf}


def random_near_equilibrium(params: dict, nx, ny, nz, seed, X0, p0, T0, amp=0.02, uamp=0.02):
    """Smoothly random fields around (X0, p0, T0, 0); relative amplitude ``amp``."""
    rng = np.random.Generator(np.random.PCG64(seed))
    shape = (nz, ny, nx)
    M = params["M"]
    X = np.stack([float(X0[a]) * (1.0 + amp * rng.uniform(-1, 1, shape)) for a in range(M)])
    X = X / X.sum(axis=0, keepdims=True)
    p = p0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    T = T0 * (1.0 + amp * rng.uniform(-1, 1, shape))
    u = uamp * rng.uniform(-1, 1, (3,) + shape)
    return {"X": X, "p": p, "T": T, "u": u}
