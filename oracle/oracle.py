"""ctypes shim for the FP64 CPU oracle (``oracle/liboracle.so``).

TEST INFRASTRUCTURE: only the test suite, the smoke check and the benchmark's
CPU-baseline leg import this module. It never loads the GPU library, and the GPU
library never loads it.

The oracle computes one time step of the consistent multicomponent lattice
Boltzmann model of Sawant, Dorschner and Karlin (arXiv 2004.11286) literally,
in FP64; see ``mclbm_oracle.c`` for the step and the readings of the paper.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
MAXM = 8

DROP_QDIFF = 1
DROP_QCORR = 2
DROP_XCORR = 4
DROP_UPNEQ = 8
DROP_FSOURCE = 16
WEAK_MIXTURE_U = 32
WEAK_MIXTURE_P = 64
CVT_HA_CPT = 128


class _Params(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("wall_x", C.c_int32), ("keep_slaved", C.c_int32), ("debug_flags", C.c_int32),
        ("weak", C.c_int32),
        ("molar_mass", C.POINTER(C.c_double)), ("cv", C.POINTER(C.c_double)),
        ("D", C.POINTER(C.c_double)), ("mu", C.POINTER(C.c_double)),
        ("lam", C.POINTER(C.c_double)), ("cv_coef", C.POINTER(C.c_double)),
        ("inlet", C.POINTER(C.c_double)), ("transport_exp", C.POINTER(C.c_double)),
        ("wall_y", C.c_int32), ("reserved2", C.c_int32),
        ("inlet_right", C.POINTER(C.c_double)), ("nozzle_y0", C.c_int32), ("nozzle_y1", C.c_int32),
    ]


class NodeInfo(C.Structure):
    _fields_ = [
        ("rho", C.c_double), ("u", C.c_double * 3), ("rhoE", C.c_double), ("T", C.c_double),
        ("P", C.c_double), ("R", C.c_double), ("Cv", C.c_double), ("Cp", C.c_double),
        ("H", C.c_double), ("mu", C.c_double), ("lam", C.c_double), ("omega", C.c_double),
        ("omega1", C.c_double),
        ("rho_a", C.c_double * MAXM), ("Y", C.c_double * MAXM), ("X", C.c_double * MAXM),
        ("j_a", (C.c_double * 3) * MAXM), ("beta", C.c_double * MAXM),
        ("V", (C.c_double * 3) * MAXM), ("K", (C.c_double * MAXM) * MAXM),
    ]


def build(force: bool = False) -> str:
    """Compile the oracle with its Makefile (gcc -O2 -ffp-contract=off)."""
    src = os.path.join(_HERE, "mclbm_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        subprocess.run(["make", "-B" if force else "-s", "-C", _HERE], check=True,
                       stdout=subprocess.DEVNULL)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        dp = C.POINTER(C.c_double)
        L.oracle_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_void_p)]
        L.oracle_destroy.argtypes = [C.c_void_p]
        L.oracle_destroy.restype = None
        L.oracle_init_fields.argtypes = [C.c_void_p, dp, dp, dp, dp]
        L.oracle_step.argtypes = [C.c_void_p, C.c_int64]
        L.oracle_read_moments.argtypes = [C.c_void_p, dp, dp, dp, dp, dp]
        L.oracle_conservation.argtypes = [C.c_void_p, dp]
        L.oracle_get_populations.argtypes = [C.c_void_p, dp]
        L.oracle_set_populations.argtypes = [C.c_void_p, dp]
        L.oracle_node_info_at.argtypes = [C.c_void_p, C.c_int32, C.c_int32, C.c_int32,
                                          C.POINTER(NodeInfo)]
        L.oracle_set_threads.argtypes = [C.c_int32]
        L.oracle_velocities.argtypes = [C.POINTER(C.c_int32)]
        L.oracle_velocities.restype = None
        L.oracle_psi.argtypes = [dp, C.c_double, dp]
        L.oracle_psi.restype = None
        L.oracle_weights.argtypes = [C.c_double, dp]
        L.oracle_weights.restype = None
        L.oracle_gansatz.argtypes = [C.c_double, C.c_double, dp, dp, dp]
        L.oracle_gansatz.restype = None
        L.oracle_tables.argtypes = [dp, dp]
        L.oracle_tables.restype = None
        L.oracle_gradient.argtypes = [C.c_int32, C.c_int32, C.c_int32, dp, dp]
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


# ---------------------------------------------------------------- building blocks
def velocities() -> np.ndarray:
    out = np.zeros(27 * 3, dtype=np.int32)
    lib().oracle_velocities(out.ctypes.data_as(C.POINTER(C.c_int32)))
    return out.reshape(27, 3)


def psi(xi, zeta) -> np.ndarray:
    xi = _f64(xi)
    out = np.zeros(27)
    lib().oracle_psi(_dp(xi), float(zeta), _dp(out))
    return out


def weights(theta) -> np.ndarray:
    out = np.zeros(27)
    lib().oracle_weights(float(theta), _dp(out))
    return out


def gansatz(theta, M0, m, Mt) -> np.ndarray:
    m = _f64(m)
    Mt = _f64(Mt).reshape(9)
    out = np.zeros(27)
    lib().oracle_gansatz(float(theta), float(M0), _dp(m), _dp(Mt), _dp(out))
    return out


def tables():
    A = np.zeros(81)
    B = np.zeros(81)
    lib().oracle_tables(_dp(A), _dp(B))
    return A.reshape(27, 3), B.reshape(27, 3)


def gradient(phi: np.ndarray) -> np.ndarray:
    """Isotropic gradient of a periodic field ``phi[nz, ny, nx]`` -> ``[3, nz, ny, nx]``."""
    phi = _f64(phi)
    nz, ny, nx = phi.shape
    out = np.zeros((3,) + phi.shape)
    rc = lib().oracle_gradient(nx, ny, nz, _dp(phi), _dp(out))
    assert rc == 0
    return out


def set_threads(n: int) -> None:
    lib().oracle_set_threads(int(n))


def threads() -> int:
    return int(lib().oracle_threads())


# ---------------------------------------------------------------- simulation
class OracleError(RuntimeError):
    pass


class OracleSim:
    """One FP64 oracle simulation. Fields are numpy arrays shaped ``[..., nz, ny, nx]``."""

    def __init__(self, params: dict, keep_slaved: bool = False, debug_flags: int = 0):
        self.M = int(params["M"])
        self.nx, self.ny, self.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
        self.n = self.nx * self.ny * self.nz
        self._arrays = [_f64(params["molar_mass"]), _f64(params["cv"]),
                        _f64(params["D"]).reshape(-1), _f64(params["mu"]),
                        _f64(params["lambda"])]
        cvc = params.get("cv_coef")
        cvc = None if cvc is None else _f64(cvc).reshape(self.M * 4)
        inl = params.get("inlet")
        inl = None if inl is None else _f64(inl).reshape(self.M + 5)
        tex = params.get("transport_exp")
        tex = None if tex is None else _f64(tex).reshape(2 * self.M + 2)
        inr = params.get("inlet_right")
        inr = None if inr is None else _f64(inr).reshape(self.M + 5)
        self._arrays += [a for a in (cvc, inl, tex, inr) if a is not None]
        noz = params.get("nozzle", (0, 0))
        p = _Params(self.M, self.nx, self.ny, self.nz, int(params.get("wall_x", 0)),
                    int(keep_slaved), int(debug_flags), int(params.get("weak", 0)),
                    *[_dp(a) for a in self._arrays[:5]],
                    *[_dp(a) if a is not None else None for a in (cvc, inl, tex)],
                    int(params.get("wall_y", 0)), 0, _dp(inr) if inr is not None else None,
                    int(noz[0]), int(noz[1]))
        h = C.c_void_p()
        rc = lib().oracle_create(C.byref(p), C.byref(h))
        if rc != 0:
            raise OracleError(f"oracle_create failed ({rc})")
        self._h = h

    def close(self):
        if getattr(self, "_h", None):
            lib().oracle_destroy(self._h)
            self._h = None

    def __del__(self):
        self.close()

    def _check(self, rc, what):
        if rc != 0:
            raise OracleError(f"{what} failed ({rc})")

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def init_fields(self, X, p, T, u):
        X = _f64(X).reshape(self.M, self.n)
        p = _f64(p).reshape(self.n)
        T = _f64(T).reshape(self.n)
        u = _f64(u).reshape(3, self.n)
        self._check(lib().oracle_init_fields(self._h, _dp(X), _dp(p), _dp(T), _dp(u)), "init_fields")

    def step(self, nsteps: int = 1):
        self._check(lib().oracle_step(self._h, int(nsteps)), "step")

    def read_moments(self) -> dict:
        X = np.zeros((self.M,) + self.shape)
        rho = np.zeros(self.shape)
        u = np.zeros((3,) + self.shape)
        p = np.zeros(self.shape)
        T = np.zeros(self.shape)
        self._check(lib().oracle_read_moments(self._h, _dp(X), _dp(rho), _dp(u), _dp(p), _dp(T)),
                    "read_moments")
        return {"X": X, "rho": rho, "u": u, "p": p, "T": T}

    def conservation(self) -> np.ndarray:
        out = np.zeros(self.M + 5)
        self._check(lib().oracle_conservation(self._h, _dp(out)), "conservation")
        return out

    def populations(self) -> np.ndarray:
        out = np.zeros((self.M + 2, 27) + self.shape)
        self._check(lib().oracle_get_populations(self._h, _dp(out)), "get_populations")
        return out

    def set_populations(self, pops: np.ndarray):
        pops = _f64(pops)
        assert pops.size == (self.M + 2) * 27 * self.n
        self._check(lib().oracle_set_populations(self._h, _dp(pops)), "set_populations")

    def node_info(self, x=0, y=0, z=0) -> dict:
        info = NodeInfo()
        self._check(lib().oracle_node_info_at(self._h, x, y, z, C.byref(info)), "node_info")
        M = self.M
        return {
            "rho": info.rho, "u": np.array(info.u[:]), "rhoE": info.rhoE, "T": info.T,
            "P": info.P, "R": info.R, "Cv": info.Cv, "Cp": info.Cp, "H": info.H,
            "mu": info.mu, "lambda": info.lam, "omega": info.omega, "omega1": info.omega1,
            "rho_a": np.array(info.rho_a[:M]), "Y": np.array(info.Y[:M]),
            "X": np.array(info.X[:M]), "beta": np.array(info.beta[:M]),
            "j_a": np.array([list(info.j_a[a]) for a in range(M)]),
            "V": np.array([list(info.V[a]) for a in range(M)]),
            "K": np.array([list(info.K[a])[:M] for a in range(M)]),
        }
