"""Helpers shared by the GPU tests: per-field comparison and checkpoint decoding."""
from __future__ import annotations

import numpy as np

FIELDS = ("X", "rho", "u", "p", "T")

# Checkpoint written by mclbm_save (see mclbm.hip): a header (magic[8], M,
# wall_x, precision, ntubes, weak, cvt as int32, int64 step count, the caller's
# 0-based index of the slaved species and a pad word), then per tube
# its size, its fixed-point range flag and its reference tables (10 lattices: up
# to 8 species, f, g; fixed-point factors per lattice and direction class), then
# the stored populations of all tubes (M-1 species lattices under strong
# coupling, M under weak coupling, then f and g).
_MAXL = 10
_NCLS = 8
_HDR = np.dtype([("magic", "S8"), ("M", "<i4"), ("wall_x", "<i4"), ("precision", "<i4"),
                 ("ntubes", "<i4"), ("weak", "<i4"), ("cvt", "<i4"), ("steps", "<i8"),
                 ("slaved", "<i4"), ("pad", "<i4")])
_TUBE = np.dtype([("nx", "<i4"), ("ny", "<i4"), ("nz", "<i4"), ("range_flag", "<u4"),
                  ("ref", "<f8", (_MAXL, 27)), ("ref0", "<f8", (_MAXL,)), ("ref2", "<f8", (_MAXL, 3)),
                  ("scale", "<f8", (_MAXL,)), ("qs", "<f8", (_MAXL, _NCLS)), ("inv_qs", "<f8", (_MAXL, _NCLS))])
_STORE = {0: np.float64, 1: np.float32, 2: np.float32, 3: np.float16, 5: np.int16}
# direction class (equal |c_x|, |c_y|, |c_z|) of the 27 directions, i = 9 (c_x+1) + 3 (c_y+1) + (c_z+1)
_CLS = np.array([(i // 9 != 1) + 2 * ((i // 3) % 3 != 1) + 4 * (i % 3 != 1) for i in range(27)])


def absolute_populations(hdr: dict, vals: np.ndarray) -> np.ndarray:
    """Stored values [L][27][...] of a decoded checkpoint as absolute populations in
    FP64, for every storage type."""
    L = vals.shape[0]
    out = np.empty(vals.shape, dtype=np.float64)
    shape = (27,) + (1,) * (vals.ndim - 2)
    for l in range(L):
        if int(hdr["precision"]) == 5:
            dec = hdr["inv_qs"][l][_CLS]
        else:
            dec = np.full(27, 1.0 / hdr["scale"][l])
        out[l] = hdr["ref"][l].reshape(shape) + vals[l].astype(np.float64) * dec.reshape(shape)
    return out


def rel_linf(a: np.ndarray, b: np.ndarray) -> float:
    """max |a - b| / max |b| (absolute when b is identically zero)."""
    den = float(np.abs(b).max())
    return float(np.abs(a - b).max() / (den if den > 0 else 1.0))


def field_errors(gpu: dict, ref: dict, u_floor: float = 0.0) -> dict:
    """Relative L-infinity error per field. With u_floor > 0 the velocity error is
    taken against max(max |u_ref|, u_floor) instead of max |u_ref|: in a tube whose
    flow is driven by diffusion alone the velocity decays towards zero, and the
    floor (1e-3 in the tests, a fraction of a percent of the sound speed) gives
    the error a scale there."""
    out = {k: rel_linf(np.asarray(gpu[k]), np.asarray(ref[k])) for k in FIELDS}
    if u_floor > 0.0:
        du = float(np.abs(np.asarray(gpu["u"]) - np.asarray(ref["u"])).max())
        out["u"] = du / max(float(np.abs(np.asarray(ref["u"])).max()), u_floor)
    return out


def decode_checkpoint(buf, tube: int = 0) -> tuple[dict, np.ndarray]:
    """Header dict of one tube and its stored values as an array [L][27][nz][ny][nx]."""
    h = np.frombuffer(buf, dtype=_HDR, count=1)[0]
    M, prec, ntubes = int(h["M"]), int(h["precision"]), int(h["ntubes"])
    L = M + 2 if int(h["weak"]) else M + 1
    tubes = np.frombuffer(buf, dtype=_TUBE, count=ntubes, offset=_HDR.itemsize)
    sizes = [int(t["nx"]) * int(t["ny"]) * int(t["nz"]) for t in tubes]
    start = L * 27 * sum(sizes[:tube])
    count = L * 27 * sizes[tube]
    off = _HDR.itemsize + _TUBE.itemsize * ntubes
    if prec == 4:
        raw = np.frombuffer(buf, dtype=np.uint16, offset=off, count=start + count)[start:]
        vals = (raw.astype(np.uint32) << 16).view(np.float32)
    else:
        vals = np.frombuffer(buf, dtype=_STORE[prec], offset=off, count=start + count)[start:]
    t = tubes[tube]
    hdr = {k: h[k] for k in _HDR.names}
    hdr.update({k: t[k] for k in _TUBE.names})
    return hdr, vals.reshape(L, 27, int(t["nz"]), int(t["ny"]), int(t["nx"]))


def oracle_window(hdr: dict, vals: np.ndarray, center, radius: int) -> np.ndarray:
    """Absolute populations of a periodic (2 radius + 1)^3 window around ``center``
    in the oracle's layout [(M+2)][27][w][w][w]; the slaved species' lattice
    (never read under strong coupling) is left at zero."""
    M = int(hdr["M"])
    L = vals.shape[0]
    nz, ny, nx = vals.shape[2:]
    x0, y0, z0 = center
    ix = np.arange(x0 - radius, x0 + radius + 1) % nx
    iy = np.arange(y0 - radius, y0 + radius + 1) % ny
    iz = np.arange(z0 - radius, z0 + radius + 1) % nz
    w = 2 * radius + 1
    out = np.zeros((M + 2, 27, w, w, w))
    sub = absolute_populations(hdr, vals[np.ix_(np.arange(L), np.arange(27), iz, iy, ix)])
    for l in range(L):
        # GPU lattices: species 1..M-1 (1..M under weak coupling), f, g
        dst = l if (L == M + 2 or l < M - 1) else l + 1
        out[dst] = sub[l]
    return out


# The coupling and property modes beyond strong coupling with constant
# properties: (weak, temperature-dependent heat capacities and transport).
OTHER_MODES = [(1, False), (0, True), (1, True)]


def with_mode(params, weak, props, T=0.3):
    """params with weak coupling and/or cubic C_{a,v}(T) (different per species)
    and transport coefficients as powers of T / T_ref, T_ref = T / 1.2."""
    params = dict(params, weak=int(weak))
    if props:
        M = params["M"]
        cv = np.asarray(params["cv"], dtype=np.float64)
        params["cv_coef"] = np.stack([cv[a] * np.array([1.0, 0.4 / T, 0.1 / T ** 2, 0.05 * (a + 1) / T ** 3])
                                      for a in range(M)])
        params["transport_exp"] = np.concatenate([0.7 + 0.1 * np.arange(M), 0.8 + 0.05 * np.arange(M),
                                                  [1.75, T / 1.2]])
    return params


def stored_population_error(hdr, vals, oracle_pops, M, weak):
    """Relative L-inf error of every stored lattice of a checkpoint against the
    oracle's populations (all M + 2 under weak coupling; the slaved species'
    lattice is not stored under strong coupling)."""
    L = vals.shape[0]
    gp = absolute_populations(hdr, vals)
    ref = oracle_pops if weak else np.concatenate([oracle_pops[:M - 1], oracle_pops[M:M + 2]])
    return float(np.abs(gp - ref).max() / np.abs(ref).max())
