"""Thin ctypes binding of libmclbm (include/mclbm.h).

Functions keep the C names and only marshal arguments; every step of the time
step runs in the library's HIP kernels. PyTorch supplies device memory (the
workspace and optional device field buffers) and the HIP stream.

Importing this module raises if ``libmclbm.so`` has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmclbm.so")

MCLBM_OK = 0
MCLBM_EARG = -1
MCLBM_ESTATE = -2
MCLBM_EDEVICE = -3
MCLBM_ENAN = -4
MCLBM_EUNSUPPORTED = -6

MCLBM_FP64 = 0
MCLBM_FP32 = 1
MCLBM_FP32_FP32 = 2
MCLBM_FP16 = 3
MCLBM_BF16 = 4
MCLBM_I16 = 5
PRECISIONS = {"fp64": MCLBM_FP64, "fp32": MCLBM_FP32, "fp32_fp32": MCLBM_FP32_FP32,
              "fp16": MCLBM_FP16, "bf16": MCLBM_BF16, "i16": MCLBM_I16}
STORAGE_BYTES = {MCLBM_FP64: 8, MCLBM_FP32: 4, MCLBM_FP32_FP32: 4, MCLBM_FP16: 2, MCLBM_BF16: 2, MCLBM_I16: 2}

MCLBM_K_MOMENTS = 0
MCLBM_K_GFIELD = 1
MCLBM_K_COLLIDE = 2


def kernel_count() -> int:
    """Number of kernel identifiers mclbm_kernel_stats knows (MCLBM_K_*)."""
    return 3

EXPORTS = ["mclbm_workspace_bytes", "mclbm_batch_workspace_bytes", "mclbm_create", "mclbm_batch_create",
           "mclbm_destroy", "mclbm_last_error", "mclbm_tube_count", "mclbm_node_count",
           "mclbm_init_fields", "mclbm_step", "mclbm_read_moments", "mclbm_read_fields_f32",
           "mclbm_conservation", "mclbm_step_count", "mclbm_range_refits", "mclbm_state_bytes", "mclbm_save", "mclbm_load",
           "mclbm_set_timing", "mclbm_kernel_stats", "mclbm_get_launch", "mclbm_set_launch",
           "mclbm_autotune", "mclbm_stream_copy", "mclbm_half_tube_moles", "mclbm_create_static"]
NN_EXPORTS = ["mclbm_nn_workspace_bytes", "mclbm_nn_create", "mclbm_nn_destroy", "mclbm_nn_last_error",
              "mclbm_nn_param_count", "mclbm_nn_set_params", "mclbm_nn_get_params", "mclbm_nn_get_grads",
              "mclbm_nn_set_norm", "mclbm_nn_set_conditioning", "mclbm_nn_io", "mclbm_nn_forward", "mclbm_nn_loss", "mclbm_nn_backward",
              "mclbm_nn_zero_grad", "mclbm_nn_clip_grad_norm", "mclbm_nn_adam_step", "mclbm_nn_mole_residual",
              "mclbm_nn_advance"]


class mclbm_params(C.Structure):
    _fields_ = [
        ("M", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
        ("wall_x", C.c_int32), ("precision", C.c_int32), ("weak", C.c_int32),
        ("wall_y", C.c_int32),
        ("molar_mass", C.POINTER(C.c_double)), ("cv", C.POINTER(C.c_double)),
        ("D", C.POINTER(C.c_double)), ("mu", C.POINTER(C.c_double)),
        ("lam", C.POINTER(C.c_double)), ("cv_coef", C.POINTER(C.c_double)),
        ("inlet", C.POINTER(C.c_double)), ("transport_exp", C.POINTER(C.c_double)),
        ("inlet_right", C.POINTER(C.c_double)), ("nozzle_y0", C.c_int32), ("nozzle_y1", C.c_int32),
        ("slaved", C.c_int32),
    ]


class mclbm_launch(C.Structure):
    _fields_ = [("variant", C.c_int32), ("swizzle", C.c_int32), ("order", C.c_int32),
                ("graph_steps", C.c_int32), ("sequential", C.c_int32), ("split", C.c_int32),
                ("three_pass", C.c_int32), ("shape", C.c_int32)]


LAUNCH_KEYS = ("variant", "swizzle", "order", "graph_steps", "sequential", "split", "three_pass", "shape")


class MclbmError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libmclbm error {code}: {msg}")
        self.code = code


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2004_11286_amd.build` "
                          "(there is no CPU fallback)")
    # torch ships its own HIP runtime under the unversioned file names its libraries
    # ask for; loaded first, it is the process's one and this library binds to it by
    # its soname. Loaded the other way round, the process would hold two runtimes and
    # device memory from torch would be foreign to this library.
    import torch  # noqa: F401

    L = C.CDLL(LIB_PATH)
    dp = C.POINTER(C.c_double)
    vp = C.c_void_p
    P = C.POINTER(mclbm_params)
    L.mclbm_workspace_bytes.argtypes = [P]
    L.mclbm_workspace_bytes.restype = C.c_size_t
    L.mclbm_create.argtypes = [P, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.mclbm_create_static.argtypes = [P, vp, C.POINTER(vp)]
    L.mclbm_batch_workspace_bytes.argtypes = [P, C.c_int32]
    L.mclbm_batch_workspace_bytes.restype = C.c_size_t
    L.mclbm_batch_create.argtypes = [P, C.c_int32, vp, C.c_size_t, vp, C.POINTER(vp)]
    L.mclbm_tube_count.argtypes = [vp]
    L.mclbm_tube_count.restype = C.c_int32
    L.mclbm_node_count.argtypes = [vp]
    L.mclbm_node_count.restype = C.c_int64
    L.mclbm_read_fields_f32.argtypes = [vp, vp, C.c_int]
    L.mclbm_get_launch.argtypes = [vp, C.POINTER(mclbm_launch)]
    L.mclbm_set_launch.argtypes = [vp, C.POINTER(mclbm_launch)]
    L.mclbm_autotune.argtypes = [vp, C.c_int32, C.c_char_p, C.c_size_t]
    ip = C.POINTER(C.c_int32)
    fp = C.POINTER(C.c_float)
    L.mclbm_nn_workspace_bytes.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, ip, C.c_int32]
    L.mclbm_nn_workspace_bytes.restype = C.c_size_t
    L.mclbm_nn_create.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_int32, C.c_int32, ip, C.c_int32, vp,
                                  C.c_size_t, vp, C.POINTER(vp)]
    L.mclbm_nn_set_conditioning.argtypes = [vp, fp]
    L.mclbm_nn_destroy.argtypes = [vp]
    L.mclbm_nn_destroy.restype = None
    L.mclbm_nn_last_error.argtypes = [vp]
    L.mclbm_nn_last_error.restype = C.c_char_p
    L.mclbm_nn_param_count.argtypes = [vp]
    L.mclbm_nn_param_count.restype = C.c_int64
    for name in ("mclbm_nn_set_params", "mclbm_nn_get_params", "mclbm_nn_get_grads"):
        getattr(L, name).argtypes = [vp, fp]
    L.mclbm_nn_set_norm.argtypes = [vp, fp, fp, fp]
    L.mclbm_nn_io.argtypes = [vp, C.POINTER(vp), C.POINTER(vp)]
    L.mclbm_nn_forward.argtypes = [vp]
    L.mclbm_nn_loss.argtypes = [vp, vp, fp, dp]
    L.mclbm_nn_backward.argtypes = [vp]
    L.mclbm_nn_zero_grad.argtypes = [vp]
    L.mclbm_nn_adam_step.argtypes = [vp, C.c_float, C.c_float, C.c_float, C.c_float]
    L.mclbm_nn_clip_grad_norm.argtypes = [vp, C.c_double, dp]
    L.mclbm_nn_mole_residual.argtypes = [vp, C.c_int32, vp, vp, dp]
    L.mclbm_nn_advance.argtypes = [vp, vp, C.c_int32, C.c_double, C.c_double, ip, dp, dp]
    L.mclbm_destroy.argtypes = [vp]
    L.mclbm_destroy.restype = None
    L.mclbm_last_error.argtypes = [vp]
    L.mclbm_last_error.restype = C.c_char_p
    L.mclbm_init_fields.argtypes = [vp, vp, vp, vp, vp, C.c_int]
    L.mclbm_step.argtypes = [vp, C.c_int64]
    L.mclbm_read_moments.argtypes = [vp, vp, vp, vp, vp, vp, C.c_int]
    L.mclbm_conservation.argtypes = [vp, dp]
    L.mclbm_step_count.argtypes = [vp]
    L.mclbm_step_count.restype = C.c_int64
    L.mclbm_range_refits.argtypes = [vp]
    L.mclbm_range_refits.restype = C.c_int64
    L.mclbm_state_bytes.argtypes = [vp]
    L.mclbm_state_bytes.restype = C.c_size_t
    L.mclbm_save.argtypes = [vp, vp, C.c_size_t]
    L.mclbm_load.argtypes = [vp, vp, C.c_size_t]
    L.mclbm_set_timing.argtypes = [vp, C.c_int]
    L.mclbm_kernel_stats.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64), C.POINTER(C.c_char_p)]
    L.mclbm_stream_copy.argtypes = [vp, vp, C.c_size_t, vp]
    L.mclbm_half_tube_moles.argtypes = [vp, dp]
    return L


lib = _load()


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


def make_params(params: dict, precision: int):
    """mclbm_params from a workload dict (``weak``: 1 for weak coupling, default 0;
    ``slaved``: the 0-based index of the slaved species, default the last (the C
    field is 1-based, 0 meaning the last); the opposed jets
    add ``inlet_right`` and ``nozzle`` = (y0, y1)); returns (struct, arrays kept
    alive)."""
    M = int(params["M"])
    arrs = [_f64(params["molar_mass"]), _f64(params["cv"]), _f64(params["D"]).reshape(M * M),
            _f64(params["mu"]), _f64(params["lambda"])]
    dp = C.POINTER(C.c_double)
    cvc = params.get("cv_coef")
    cvc = None if cvc is None else _f64(cvc).reshape(M * 4)
    inl = params.get("inlet")
    inl = None if inl is None else _f64(inl).reshape(M + 5)
    tex = params.get("transport_exp")
    tex = None if tex is None else _f64(tex).reshape(2 * M + 2)
    inr = params.get("inlet_right")
    inr = None if inr is None else _f64(inr).reshape(M + 5)
    noz = params.get("nozzle", (0, 0))
    arrs += [a for a in (cvc, inl, tex, inr) if a is not None]
    p = mclbm_params(M, int(params["nx"]), int(params["ny"]), int(params["nz"]),
                     int(params.get("wall_x", 0)), int(precision), int(params.get("weak", 0)),
                     int(params.get("wall_y", 0)),
                     *[a.ctypes.data_as(dp) for a in arrs[:5]],
                     *[a.ctypes.data_as(dp) if a is not None else None for a in (cvc, inl, tex, inr)],
                     int(noz[0]), int(noz[1]), 0 if params.get("slaved") is None else int(params["slaved"]) + 1)
    return p, arrs


def make_param_array(tubes: list, precision: int):
    """Array of mclbm_params for a batch; returns (array, arrays kept alive)."""
    arr = (mclbm_params * len(tubes))()
    keep = []
    for t, params in enumerate(tubes):
        arr[t], k = make_params(params, precision)
        keep.append(k)
    return arr, keep


def mclbm_stream_copy(dst_ptr: int, src_ptr: int, nbytes: int, stream: int = 0) -> None:
    rc = lib.mclbm_stream_copy(C.c_void_p(dst_ptr), C.c_void_p(src_ptr), nbytes, C.c_void_p(stream or None))
    if rc != MCLBM_OK:
        raise MclbmError(rc, "mclbm_stream_copy: size not a multiple of 16, misaligned or overlapping buffers")


def stream_copy(dst, src, stream=None) -> None:
    """mclbm_stream_copy of the bytes of device tensor src into dst (same size)."""
    nbytes = src.numel() * src.element_size()
    if dst.numel() * dst.element_size() != nbytes or not (src.is_cuda and dst.is_cuda):
        raise ValueError("stream_copy needs two device tensors of the same size")
    mclbm_stream_copy(dst.data_ptr(), src.data_ptr(), nbytes, 0 if stream is None else stream.cuda_stream)


def _check(ctx, rc: int):
    if rc != MCLBM_OK:
        msg = lib.mclbm_last_error(ctx)
        raise MclbmError(rc, msg.decode() if msg else "")


# ------------------------------------------------------------------ C-named calls
def mclbm_workspace_bytes(params: dict, precision: int) -> int:
    p, _keep = make_params(params, precision)
    n = lib.mclbm_workspace_bytes(C.byref(p))
    if n == 0:
        raise MclbmError(MCLBM_EARG, lib.mclbm_last_error(None).decode())
    return int(n)


def mclbm_create(params: dict, precision: int, workspace_ptr: int, nbytes: int, stream: int) -> C.c_void_p:
    p, _keep = make_params(params, precision)
    h = C.c_void_p()
    _check(None, lib.mclbm_create(C.byref(p), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream),
                                  C.byref(h)))
    return h


def mclbm_create_static(params: dict, precision: int, stream: int) -> C.c_void_p:
    """A context over the library's static workspace (no device allocation)."""
    p, _keep = make_params(params, precision)
    h = C.c_void_p()
    _check(None, lib.mclbm_create_static(C.byref(p), C.c_void_p(stream), C.byref(h)))
    return h


# Bytes of the library's static workspace (MCLBM_STATIC_WORKSPACE_BYTES in include/mclbm.h).
MCLBM_STATIC_WORKSPACE_BYTES = 64 << 20


def mclbm_batch_workspace_bytes(tubes: list, precision: int) -> int:
    arr, _keep = make_param_array(tubes, precision)
    n = lib.mclbm_batch_workspace_bytes(arr, len(tubes))
    if n == 0:
        raise MclbmError(MCLBM_EARG, lib.mclbm_last_error(None).decode())
    return int(n)


def mclbm_batch_create(tubes: list, precision: int, workspace_ptr: int, nbytes: int, stream: int) -> C.c_void_p:
    arr, _keep = make_param_array(tubes, precision)
    h = C.c_void_p()
    _check(None, lib.mclbm_batch_create(arr, len(tubes), C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream),
                                        C.byref(h)))
    return h


def mclbm_tube_count(ctx) -> int:
    return int(lib.mclbm_tube_count(ctx))


def mclbm_node_count(ctx) -> int:
    return int(lib.mclbm_node_count(ctx))


def mclbm_read_fields_f32(ctx, out_ptr: int, on_device: int) -> None:
    _check(ctx, lib.mclbm_read_fields_f32(ctx, C.c_void_p(out_ptr), int(on_device)))


def mclbm_get_launch(ctx) -> dict:
    lc = mclbm_launch()
    _check(ctx, lib.mclbm_get_launch(ctx, C.byref(lc)))
    return {k: int(getattr(lc, k)) for k in LAUNCH_KEYS}


def mclbm_set_launch(ctx, **kw) -> None:
    cur = mclbm_get_launch(ctx)
    cur.update({k: int(v) for k, v in kw.items()})
    lc = mclbm_launch(*[cur[k] for k in LAUNCH_KEYS])
    _check(ctx, lib.mclbm_set_launch(ctx, C.byref(lc)))


def mclbm_autotune(ctx, trial_steps: int) -> str:
    buf = C.create_string_buffer(16384)
    _check(ctx, lib.mclbm_autotune(ctx, int(trial_steps), buf, len(buf)))
    return buf.value.decode()


def mclbm_destroy(ctx) -> None:
    lib.mclbm_destroy(ctx)


def mclbm_last_error(ctx) -> str:
    m = lib.mclbm_last_error(ctx)
    return m.decode() if m else ""


def mclbm_init_fields(ctx, X_ptr: int, p_ptr: int, T_ptr: int, u_ptr: int, on_device: int) -> None:
    _check(ctx, lib.mclbm_init_fields(ctx, C.c_void_p(X_ptr), C.c_void_p(p_ptr), C.c_void_p(T_ptr),
                                      C.c_void_p(u_ptr), int(on_device)))


def mclbm_step(ctx, nsteps: int) -> None:
    _check(ctx, lib.mclbm_step(ctx, int(nsteps)))


def mclbm_read_moments(ctx, X_ptr, rho_ptr, u_ptr, p_ptr, T_ptr, on_device: int) -> None:
    ptrs = [C.c_void_p(v) if v else None for v in (X_ptr, rho_ptr, u_ptr, p_ptr, T_ptr)]
    _check(ctx, lib.mclbm_read_moments(ctx, *ptrs, int(on_device)))


def mclbm_conservation(ctx, M: int) -> np.ndarray:
    """Per-tube FP64 sums, shape [ntubes][M+5]."""
    out = np.zeros((mclbm_tube_count(ctx), M + 5))
    _check(ctx, lib.mclbm_conservation(ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def mclbm_half_tube_moles(ctx, M: int) -> np.ndarray:
    """Per-tube moles of every species in each x half, shape [ntubes][2][M]."""
    out = np.zeros((mclbm_tube_count(ctx), 2, M))
    _check(ctx, lib.mclbm_half_tube_moles(ctx, out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def mclbm_step_count(ctx) -> int:
    return int(lib.mclbm_step_count(ctx))


def mclbm_range_refits(ctx) -> int:
    return int(lib.mclbm_range_refits(ctx))


def mclbm_state_bytes(ctx) -> int:
    return int(lib.mclbm_state_bytes(ctx))


def mclbm_save(ctx) -> bytearray:
    n = mclbm_state_bytes(ctx)
    buf = bytearray(n)
    _check(ctx, lib.mclbm_save(ctx, (C.c_char * n).from_buffer(buf), n))
    return buf


def mclbm_load(ctx, buf: bytearray) -> None:
    n = len(buf)
    _check(ctx, lib.mclbm_load(ctx, (C.c_char * n).from_buffer(buf), n))


def mclbm_set_timing(ctx, enable: bool) -> None:
    _check(ctx, lib.mclbm_set_timing(ctx, int(bool(enable))))


def mclbm_kernel_stats(ctx, kernel: int):
    ms = C.c_double()
    launches = C.c_int64()
    name = C.c_char_p()
    _check(ctx, lib.mclbm_kernel_stats(ctx, int(kernel), C.byref(ms), C.byref(launches), C.byref(name)))
    return ms.value, launches.value, name.value.decode()


# ------------------------------------------------------------------ convenience wrapper
class Sim:
    """A context plus its torch-owned device workspace on ``device``."""

    def __init__(self, params: dict, precision: int | str = MCLBM_FP32, device: str = "cuda:0", stream=None,
                 static_workspace: bool = False):
        """static_workspace: use the library's static workspace (mclbm_create_static)
        instead of a torch-allocated one."""
        import torch

        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.params = dict(params)
        self.precision = int(precision)
        self.M = int(params["M"])
        self.nx, self.ny, self.nz = int(params["nx"]), int(params["ny"]), int(params["nz"])
        self.n = self.nx * self.ny * self.nz
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        if static_workspace:
            self.workspace = None
            with torch.cuda.device(self.device):
                self.ctx = mclbm_create_static(params, self.precision, self.stream.cuda_stream)
            return
        nbytes = mclbm_workspace_bytes(params, self.precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        with torch.cuda.device(self.device):
            self.ctx = mclbm_create(params, self.precision, self.workspace.data_ptr(), nbytes,
                                    self.stream.cuda_stream)

    @property
    def shape(self):
        return (self.nz, self.ny, self.nx)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            mclbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_fields(self, X, p, T, u):
        """Fields as numpy arrays (host) or CUDA tensors (device), shaped [..., nz, ny, nx]."""
        import torch

        if all(isinstance(a, torch.Tensor) and a.is_cuda for a in (X, p, T, u)):
            t = [a.to(torch.float64).contiguous() for a in (X, p, T, u)]
            mclbm_init_fields(self.ctx, *[a.data_ptr() for a in t], 1)
            return
        a = [_f64(v) for v in (X, p, T, u)]
        assert a[0].size == self.M * self.n and a[3].size == 3 * self.n
        mclbm_init_fields(self.ctx, *[v.ctypes.data for v in a], 0)

    def step(self, nsteps: int = 1):
        mclbm_step(self.ctx, nsteps)

    def read_moments(self, on_device: bool = False) -> dict:
        if on_device:
            import torch

            kw = dict(dtype=torch.float64, device=self.device)
            out = {"X": torch.empty((self.M,) + self.shape, **kw), "rho": torch.empty(self.shape, **kw),
                   "u": torch.empty((3,) + self.shape, **kw), "p": torch.empty(self.shape, **kw),
                   "T": torch.empty(self.shape, **kw)}
            mclbm_read_moments(self.ctx, *[out[k].data_ptr() for k in ("X", "rho", "u", "p", "T")], 1)
            return out
        out = {"X": np.zeros((self.M,) + self.shape), "rho": np.zeros(self.shape),
               "u": np.zeros((3,) + self.shape), "p": np.zeros(self.shape), "T": np.zeros(self.shape)}
        mclbm_read_moments(self.ctx, *[out[k].ctypes.data for k in ("X", "rho", "u", "p", "T")], 0)
        return out

    def conservation(self) -> np.ndarray:
        return mclbm_conservation(self.ctx, self.M)[0]

    def half_tube_moles(self) -> np.ndarray:
        """[2][M]: moles of every species in the x < nx/2 and x >= nx/2 halves."""
        return mclbm_half_tube_moles(self.ctx, self.M)[0]

    @property
    def step_count(self) -> int:
        return mclbm_step_count(self.ctx)

    def range_refits(self) -> int:
        return mclbm_range_refits(self.ctx)

    def launch(self) -> dict:
        return mclbm_get_launch(self.ctx)

    def set_launch(self, **kw) -> None:
        mclbm_set_launch(self.ctx, **kw)

    def autotune(self, trial_steps: int = 10) -> str:
        return mclbm_autotune(self.ctx, trial_steps)

    def save(self) -> bytearray:
        return mclbm_save(self.ctx)

    def load(self, buf) -> None:
        mclbm_load(self.ctx, buf)

    def set_timing(self, enable: bool) -> None:
        mclbm_set_timing(self.ctx, enable)

    def kernel_stats(self, kernel: int):
        return mclbm_kernel_stats(self.ctx, kernel)


class Batch:
    """A context over independent tubes (one workload dict each) plus its
    torch-owned workspace. Per-node arrays are the concatenation over tubes of
    each tube's own array (see include/mclbm.h); the helpers below split and
    join them."""

    def __init__(self, tubes: list, precision: int | str = MCLBM_FP32, device: str = "cuda:0", stream=None):
        import torch

        if isinstance(precision, str):
            precision = PRECISIONS[precision]
        self.tubes = [dict(t) for t in tubes]
        self.precision = int(precision)
        self.M = int(tubes[0]["M"])
        self.shapes = [(int(t["nz"]), int(t["ny"]), int(t["nx"])) for t in tubes]
        self.sizes = [int(np.prod(s)) for s in self.shapes]
        self.offsets = np.concatenate([[0], np.cumsum(self.sizes)]).astype(np.int64)
        self.n = int(self.offsets[-1])
        self.device = torch.device(device)
        nbytes = mclbm_batch_workspace_bytes(self.tubes, self.precision)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.ctx = mclbm_batch_create(self.tubes, self.precision, self.workspace.data_ptr(), nbytes,
                                          self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            mclbm_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- layout helpers
    def join(self, per_tube: list, comps: int) -> np.ndarray:
        """Concatenate per-tube arrays of shape [comps, nz, ny, nx] (or [nz, ny, nx])."""
        return np.concatenate([_f64(a).reshape(comps * n) for a, n in zip(per_tube, self.sizes)])

    def split(self, flat: np.ndarray, comps: int) -> list:
        out = []
        for t, sh in enumerate(self.shapes):
            a = flat[comps * self.offsets[t]:comps * self.offsets[t + 1]]
            out.append(a.reshape(((comps,) if comps > 1 else ()) + sh))
        return out

    def init_fields(self, fields: list):
        """fields: one dict (X, p, T, u) per tube, numpy arrays."""
        X = self.join([f["X"] for f in fields], self.M)
        p = self.join([f["p"] for f in fields], 1)
        T = self.join([f["T"] for f in fields], 1)
        u = self.join([f["u"] for f in fields], 3)
        mclbm_init_fields(self.ctx, X.ctypes.data, p.ctypes.data, T.ctypes.data, u.ctypes.data, 0)

    def step(self, nsteps: int = 1):
        mclbm_step(self.ctx, nsteps)

    def read_moments(self) -> list:
        """One dict of numpy fields per tube."""
        flat = {"X": np.zeros(self.M * self.n), "rho": np.zeros(self.n), "u": np.zeros(3 * self.n),
                "p": np.zeros(self.n), "T": np.zeros(self.n)}
        mclbm_read_moments(self.ctx, *[flat[k].ctypes.data for k in ("X", "rho", "u", "p", "T")], 0)
        comps = {"X": self.M, "rho": 1, "u": 3, "p": 1, "T": 1}
        parts = {k: self.split(v, comps[k]) for k, v in flat.items()}
        return [{k: parts[k][t] for k in flat} for t in range(len(self.shapes))]

    def read_fields_f32(self, out=None):
        """FP32 trajectory fields (X_1..X_M, T, u, p) into a CUDA tensor of M+5 values per node."""
        import torch

        if out is None:
            out = torch.empty((self.M + 5) * self.n, dtype=torch.float32, device=self.device)
        mclbm_read_fields_f32(self.ctx, out.data_ptr(), 1)
        return out

    def conservation(self) -> np.ndarray:
        return mclbm_conservation(self.ctx, self.M)

    def half_tube_moles(self) -> np.ndarray:
        """[ntubes][2][M]: moles of every species in each x half of every tube."""
        return mclbm_half_tube_moles(self.ctx, self.M)

    @property
    def step_count(self) -> int:
        return mclbm_step_count(self.ctx)

    def range_refits(self) -> int:
        return mclbm_range_refits(self.ctx)

    def launch(self) -> dict:
        return mclbm_get_launch(self.ctx)

    def set_launch(self, **kw) -> None:
        mclbm_set_launch(self.ctx, **kw)

    def autotune(self, trial_steps: int = 10) -> str:
        return mclbm_autotune(self.ctx, trial_steps)

    def save(self) -> bytearray:
        return mclbm_save(self.ctx)

    def load(self, buf) -> None:
        mclbm_load(self.ctx, buf)

    def set_timing(self, enable: bool) -> None:
        mclbm_set_timing(self.ctx, enable)

    def kernel_stats(self, kernel: int):
        return mclbm_kernel_stats(self.ctx, kernel)


# ------------------------------------------------------------------ surrogate (include/mclbm_nn.h)
def _nn_check(net, rc: int):
    if rc != MCLBM_OK:
        msg = lib.mclbm_nn_last_error(net)
        raise MclbmError(rc, msg.decode() if msg else "")


def _dims_array(dims):
    d = np.ascontiguousarray(np.asarray(dims, dtype=np.int32).reshape(-1))
    return d, d.ctypes.data_as(C.POINTER(C.c_int32))


def _f32p(a):
    return a.ctypes.data_as(C.POINTER(C.c_float))


def mclbm_nn_workspace_bytes(channels: int, two_term: int, conditioning: int, species: int, depth: int,
                             dims) -> int:
    d, dp_ = _dims_array(dims)
    n = lib.mclbm_nn_workspace_bytes(int(channels), int(two_term), int(conditioning), int(species), int(depth),
                                     dp_, d.size // 3)
    if n == 0:
        raise MclbmError(MCLBM_EARG, lib.mclbm_nn_last_error(None).decode())
    return int(n)


def mclbm_nn_create(channels: int, two_term: int, conditioning: int, species: int, depth: int, dims,
                    workspace_ptr: int, nbytes: int, stream: int):
    d, dp_ = _dims_array(dims)
    h = C.c_void_p()
    _nn_check(None, lib.mclbm_nn_create(int(channels), int(two_term), int(conditioning), int(species), int(depth),
                                        dp_, d.size // 3, C.c_void_p(workspace_ptr), nbytes, C.c_void_p(stream),
                                        C.byref(h)))
    return h


def mclbm_nn_set_conditioning(net, values: np.ndarray) -> None:
    a = np.ascontiguousarray(values, dtype=np.float32)
    _nn_check(net, lib.mclbm_nn_set_conditioning(net, _f32p(a)))


def mclbm_nn_destroy(net) -> None:
    lib.mclbm_nn_destroy(net)


def mclbm_nn_last_error(net) -> str:
    m = lib.mclbm_nn_last_error(net)
    return m.decode() if m else ""


def mclbm_nn_param_count(net) -> int:
    return int(lib.mclbm_nn_param_count(net))


def mclbm_nn_set_params(net, params: np.ndarray) -> None:
    a = np.ascontiguousarray(params, dtype=np.float32)
    assert a.size == mclbm_nn_param_count(net)
    _nn_check(net, lib.mclbm_nn_set_params(net, _f32p(a)))


def mclbm_nn_get_params(net) -> np.ndarray:
    a = np.zeros(mclbm_nn_param_count(net), dtype=np.float32)
    _nn_check(net, lib.mclbm_nn_get_params(net, _f32p(a)))
    return a


def mclbm_nn_get_grads(net) -> np.ndarray:
    a = np.zeros(mclbm_nn_param_count(net), dtype=np.float32)
    _nn_check(net, lib.mclbm_nn_get_grads(net, _f32p(a)))
    return a


def mclbm_nn_set_norm(net, in_shift, in_scale, out_scale) -> None:
    arrs = [np.ascontiguousarray(v, dtype=np.float32) for v in (in_shift, in_scale, out_scale)]
    _nn_check(net, lib.mclbm_nn_set_norm(net, *[_f32p(a) for a in arrs]))


def mclbm_nn_io(net):
    a, b = C.c_void_p(), C.c_void_p()
    _nn_check(net, lib.mclbm_nn_io(net, C.byref(a), C.byref(b)))
    return a.value, b.value


def mclbm_nn_forward(net) -> None:
    _nn_check(net, lib.mclbm_nn_forward(net))


def mclbm_nn_loss(net, target_ptr: int, channel_weight=None) -> float:
    out = C.c_double()
    w = None if channel_weight is None else np.ascontiguousarray(channel_weight, dtype=np.float32)
    _nn_check(net, lib.mclbm_nn_loss(net, C.c_void_p(target_ptr), None if w is None else _f32p(w), C.byref(out)))
    return out.value


def mclbm_nn_backward(net) -> None:
    _nn_check(net, lib.mclbm_nn_backward(net))


def mclbm_nn_zero_grad(net) -> None:
    _nn_check(net, lib.mclbm_nn_zero_grad(net))


def mclbm_nn_clip_grad_norm(net, max_norm: float) -> float:
    out = C.c_double()
    _nn_check(net, lib.mclbm_nn_clip_grad_norm(net, float(max_norm), C.byref(out)))
    return out.value


def mclbm_nn_adam_step(net, lr: float, beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    _nn_check(net, lib.mclbm_nn_adam_step(net, float(lr), float(beta1), float(beta2), float(eps)))


def mclbm_nn_mole_residual(net, species: int, a_ptr: int, b_ptr: int, ntubes: int) -> np.ndarray:
    out = np.zeros(ntubes)
    _nn_check(net, lib.mclbm_nn_mole_residual(net, int(species), C.c_void_p(a_ptr), C.c_void_p(b_ptr),
                                              out.ctypes.data_as(C.POINTER(C.c_double))))
    return out


def mclbm_nn_advance(ctx, net, K: int, resid_tol: float, change_tol: float = float("inf")):
    used = C.c_int32()
    res = C.c_double()
    chg = C.c_double()
    _check(ctx, lib.mclbm_nn_advance(ctx, net, int(K), float(resid_tol), float(change_tol), C.byref(used),
                                     C.byref(res), C.byref(chg)))
    return bool(used.value), res.value, chg.value


class Net:
    """A surrogate network over a set of tubes plus its torch-owned workspace.
    fields_in / fields_out are views of the network's own device buffers
    ([channels][n] per tube, concatenated)."""

    def __init__(self, channels: int, depth: int, dims, conditioning: int = 0, two_term: int = 0, species: int = 0,
                 device: str = "cuda:0", stream=None):
        import torch

        self.C = int(channels)
        self.P = int(two_term)
        self.S = int(conditioning)
        self.Ms = int(species)
        self.Cout = 3 * self.Ms + 4 if self.Ms else self.C
        self.depth = int(depth)
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.sizes = [nx * ny * nz for nx, ny, nz in self.dims]
        self.n = int(sum(self.sizes))
        self.device = torch.device(device)
        nbytes = mclbm_nn_workspace_bytes(self.C, self.P, self.S, self.Ms, self.depth, self.dims)
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        with torch.cuda.device(self.device):
            self.net = mclbm_nn_create(self.C, self.P, self.S, self.Ms, self.depth, self.dims,
                                       self.workspace.data_ptr(), nbytes, self.stream.cuda_stream)
        pin, pout = mclbm_nn_io(self.net)
        base = self.workspace.data_ptr()
        count = self.C * self.n
        as_f32 = self.workspace.view(torch.float32) if nbytes % 4 == 0 else None
        assert as_f32 is not None and (pin - base) % 4 == 0 and (pout - base) % 4 == 0
        self.fields_in = as_f32[(pin - base) // 4:(pin - base) // 4 + count]
        self.fields_out = as_f32[(pout - base) // 4:(pout - base) // 4 + count]

    def close(self):
        if getattr(self, "net", None) is not None:
            mclbm_nn_destroy(self.net)
            self.net = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @property
    def param_count(self) -> int:
        return mclbm_nn_param_count(self.net)

    def set_params(self, p):
        mclbm_nn_set_params(self.net, p)

    def get_params(self):
        return mclbm_nn_get_params(self.net)

    def get_grads(self):
        return mclbm_nn_get_grads(self.net)

    def set_norm(self, in_shift, in_scale, out_scale):
        mclbm_nn_set_norm(self.net, in_shift, in_scale, out_scale)

    def set_conditioning(self, values):
        """values: [ntubes][conditioning] floats."""
        mclbm_nn_set_conditioning(self.net, values)

    def forward(self, fields=None):
        """fields: a CUDA float32 tensor of channels * n values (copied in), or None
        to use what fields_in holds. Returns fields_out."""
        if fields is not None:
            self.fields_in.copy_(fields.reshape(-1))
        mclbm_nn_forward(self.net)
        return self.fields_out

    def loss(self, target, channel_weight=None) -> float:
        t = target.reshape(-1).contiguous()
        return mclbm_nn_loss(self.net, t.data_ptr(), channel_weight)

    def backward(self):
        mclbm_nn_backward(self.net)

    def zero_grad(self):
        mclbm_nn_zero_grad(self.net)

    def clip_grad_norm(self, max_norm: float = 0.0) -> float:
        """Global gradient norm; gradients scaled down to max_norm when above it (> 0)."""
        return mclbm_nn_clip_grad_norm(self.net, max_norm)

    def adam_step(self, lr, beta1=0.9, beta2=0.999, eps=1e-8):
        mclbm_nn_adam_step(self.net, lr, beta1, beta2, eps)

    def mole_residual(self, species, a, b) -> np.ndarray:
        a = a.reshape(-1).contiguous()
        b = b.reshape(-1).contiguous()
        return mclbm_nn_mole_residual(self.net, species, a.data_ptr(), b.data_ptr(), len(self.dims))

    def advance(self, sim, K: int, resid_tol: float, change_tol: float = float("inf")):
        """Advance a Sim or Batch by K steps; returns (used_fallback, max_residual, max_change)."""
        return mclbm_nn_advance(sim.ctx, self.net, K, resid_tol, change_tol)
