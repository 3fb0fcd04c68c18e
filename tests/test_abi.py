"""The C ABI library loads, exports every symbol include/mclbm.h declares, and
validates its arguments on the host (no GPU needed for these calls)."""
import os
import re

import numpy as np
import pytest

from paper_2004_11286_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            src = open(os.path.join(ROOT, "include", h)).read()
            src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
            names |= set(re.findall(r"\b(mclbm_[a-z0-9_]+)\s*\(", src))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    names = declared_functions()
    assert len(names) >= 14
    for name in names:
        assert hasattr(m.lib, name), name
    assert sorted(m.EXPORTS + m.NN_EXPORTS) == names


def test_binding_names_match_c_names():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    for name in declared_functions():
        assert callable(getattr(m, name)), name


def test_workspace_bytes_and_validation():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.binary_interdiffusion()
    sizes = {prec: m.mclbm_workspace_bytes(p, prec) for prec in range(5)}
    n = 64 * 8 * 8
    # two population buffers of 27 (M+1) values dominate
    assert sizes[m.MCLBM_FP64] > 2 * 27 * 3 * n * 8
    assert sizes[m.MCLBM_FP32] > 2 * 27 * 3 * n * 4
    assert sizes[m.MCLBM_FP16] < sizes[m.MCLBM_FP32]
    bad = dict(p)
    bad["D"] = np.array([[0.05, 0.04], [0.05, 0.05]])      # not symmetric
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_workspace_bytes(bad, 1)
    assert "symmetric" in str(e.value)
    bad = dict(p)
    bad["mu"] = np.array([0.0, 1.0])
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(bad, 1)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(p, 7)                         # unknown precision
    tube, _ = W.ternary_tube(nx=1)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(tube, 1)                      # walls need nx >= 2


def test_weak_coupling_workspace_and_validation():
    """Weak coupling stores one more lattice (species M) in both population
    buffers and four more record fields (rho_M and the species velocity u_s); it
    is compiled for FP64 arithmetic and for FP16 storage, and a batch cannot mix
    couplings."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.binary_interdiffusion()
    n = 64 * 8 * 8
    for prec, s_bytes, r_bytes in ((m.MCLBM_FP64, 8, 8), (m.MCLBM_FP32, 4, 4), (m.MCLBM_FP16, 2, 4)):
        strong = m.mclbm_workspace_bytes(p, prec)
        weak = m.mclbm_workspace_bytes(dict(p, weak=1), prec)
        assert weak - strong == 2 * 27 * n * s_bytes + 4 * n * r_bytes
    for prec in (m.MCLBM_FP32_FP32, m.MCLBM_BF16):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(dict(p, weak=1), prec)
        assert "weak coupling" in str(e.value)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(dict(p, weak=2), m.MCLBM_FP32)
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_batch_workspace_bytes([p, dict(p, weak=1)], m.MCLBM_FP32)
    assert "weak" in str(e.value)


def test_fixed16_workspace_and_validation():
    """16-bit fixed-point storage takes the workspace of FP16 storage (two bytes a
    population, FP32 record); it is compiled for both couplings with constant
    properties and periodic or walled x ends only."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.binary_interdiffusion()
    tube, _ = W.ternary_tube(nx=16, ny=2, nz=2)
    for q in (p, dict(p, weak=1), tube, dict(tube, weak=1)):
        assert m.mclbm_workspace_bytes(q, m.MCLBM_I16) == m.mclbm_workspace_bytes(q, m.MCLBM_FP16)
    inlet = np.array([0.3, 0.3, 0.4, tube["P0"], 1 / 3, 0.05, 0.0, 0.0])
    for bad, what in ((dict(tube, wall_x=2, inlet=inlet), "open x ends"), (dict(tube, wall_y=1), "free-slip"),
                      (dict(tube, cv_coef=np.ones((3, 4))), "")):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(bad, m.MCLBM_I16)
        assert what in str(e.value)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(p, m.MCLBM_I16 + 1)             # unknown precision


def test_cv_of_T_workspace_and_validation():
    """Temperature-dependent specific heats add M - 1 mass-fraction fields to the
    node record; the coefficients must give a positive, non-decreasing C_v; the
    kernels exist for strong coupling with FP64 arithmetic only; a batch cannot
    mix constant and polynomial heat capacities."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.ternary_tube(nx=16, ny=4, nz=4)
    n = 16 * 4 * 4
    cvc = np.array([[c, 0.5 * c, 0.0, 0.1 * c] for c in p["cv"]])
    for prec, r_bytes in ((m.MCLBM_FP64, 8), (m.MCLBM_FP32, 4)):
        assert (m.mclbm_workspace_bytes(dict(p, cv_coef=cvc), prec) - m.mclbm_workspace_bytes(p, prec)
                == 2 * n * r_bytes)                          # M - 1 = 2 more record fields
    for bad in (np.array([[0.0, 1.0, 0.0, 0.0]] * 3), np.array([[1.0, -0.1, 0.0, 0.0]] * 3),
                np.array([[1.0, np.nan, 0.0, 0.0]] * 3)):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(dict(p, cv_coef=bad), m.MCLBM_FP64)
        assert "cv_coef" in str(e.value)
    for prec, r_bytes in ((m.MCLBM_FP64, 8), (m.MCLBM_FP32, 4)):      # with weak coupling too
        assert (m.mclbm_workspace_bytes(dict(p, cv_coef=cvc, weak=1), prec)
                - m.mclbm_workspace_bytes(dict(p, weak=1), prec) == 2 * n * r_bytes)
    for q, prec in ((dict(p, cv_coef=cvc, weak=1), m.MCLBM_FP16), (dict(p, cv_coef=cvc), m.MCLBM_FP16),
                    (dict(p, cv_coef=cvc), m.MCLBM_FP32_FP32)):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(q, prec)
        assert "compiled for MCLBM_FP64 and MCLBM_FP32 only" in str(e.value)
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_batch_workspace_bytes([p, dict(p, cv_coef=cvc)], m.MCLBM_FP32)
    assert "cv_coef" in str(e.value)
    tex = np.array([0.7, 0.7, 0.7, 0.8, 0.8, 0.8, 1.75, 0.25])
    assert m.mclbm_workspace_bytes(dict(p, transport_exp=tex), m.MCLBM_FP64) == \
        m.mclbm_workspace_bytes(dict(p, cv_coef=cvc), m.MCLBM_FP64)
    for bad in (np.concatenate([tex[:-1], [0.0]]), np.concatenate([[np.inf], tex[1:]])):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(dict(p, transport_exp=bad), m.MCLBM_FP64)
        assert "transport_exp" in str(e.value)
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_workspace_bytes(dict(p, transport_exp=tex), m.MCLBM_FP16)
    assert "temperature-dependent transport" in str(e.value)


def test_open_ends_validation():
    """Open x ends (wall_x = 2) need inlet fields with mole fractions summing to 1
    and positive p and T; they are compiled for strong coupling with constant
    heat capacities and FP64 arithmetic."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.ternary_tube(nx=16, ny=2, nz=2)
    inlet = np.array([0.3, 0.3, 0.4, p["P0"], 1 / 3, 0.05, 0.0, 0.0])
    q = dict(p, wall_x=2, inlet=inlet)
    assert m.mclbm_workspace_bytes(q, m.MCLBM_FP32) == m.mclbm_workspace_bytes(dict(p, wall_x=1), m.MCLBM_FP32)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(dict(p, wall_x=2), m.MCLBM_FP32)              # no inlet
    for bad in (np.array([0.3, 0.3, 0.3, p["P0"], 1 / 3, 0, 0, 0]), np.array([0.3, 0.3, 0.4, -1.0, 1 / 3, 0, 0, 0]),
                np.array([0.3, 0.3, 0.4, p["P0"], np.nan, 0, 0, 0])):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(dict(q, inlet=bad), m.MCLBM_FP32)
        assert "inlet" in str(e.value)
    # with either coupling and either kind of properties: the workspace of the walled tube
    for r in (dict(q, weak=1), dict(q, cv_coef=np.ones((3, 4))), dict(q, weak=1, cv_coef=np.ones((3, 4)))):
        w = dict(r, wall_x=1)
        del w["inlet"]
        assert m.mclbm_workspace_bytes(r, m.MCLBM_FP64) == m.mclbm_workspace_bytes(w, m.MCLBM_FP64)
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_workspace_bytes(q, m.MCLBM_FP16)
    assert "open x ends" in str(e.value)
    with pytest.raises(m.MclbmError):
        m.mclbm_workspace_bytes(dict(p, wall_x=4), m.MCLBM_FP32)


def test_opposed_jets_validation():
    """The opposed jets (wall_x = 3) need both inlets, nozzle rows inside
    1 <= y0 < y1 <= ny - 1 and outlets at the y ends (wall_y = 2, which goes with
    them only); they are compiled for strong coupling, constant properties and
    FP64 arithmetic, and take the workspace of the walled tube."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.ternary_tube(nx=16, ny=8, nz=2)
    left = np.array([0.3, 0.3, 0.4, p["P0"], 1 / 3, 0.04, 0.0, 0.0])
    right = np.array([0.2, 0.3, 0.5, p["P0"], 1 / 3, -0.04, 0.0, 0.0])
    q = dict(p, wall_x=3, wall_y=2, inlet=left, inlet_right=right, nozzle=(2, 6))
    for prec in (m.MCLBM_FP64, m.MCLBM_FP32):
        assert m.mclbm_workspace_bytes(q, prec) == m.mclbm_workspace_bytes(dict(p, wall_x=1), prec)
    assert m.mclbm_workspace_bytes(dict(q, nozzle=(1, 7)), m.MCLBM_FP32) > 0
    for bad in (dict(q, inlet_right=None), dict(q, wall_y=0), dict(q, wall_y=1), dict(q, nozzle=(0, 4)),
                dict(q, nozzle=(3, 8)), dict(q, nozzle=(4, 4)), dict(p, wall_y=2),
                dict(q, inlet_right=np.array([0.2, 0.3, 0.4, p["P0"], 1 / 3, 0, 0, 0]))):
        with pytest.raises(m.MclbmError):
            m.mclbm_workspace_bytes(bad, m.MCLBM_FP32)
    for bad, prec in ((dict(q, weak=1), m.MCLBM_FP64), (dict(q, cv_coef=np.ones((3, 4))), m.MCLBM_FP64),
                      (q, m.MCLBM_FP16), (q, m.MCLBM_FP32_FP32)):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(bad, prec)
        assert "jets" in str(e.value)


def test_free_slip_validation():
    """Free-slip y walls need ny >= 2 and are compiled for periodic or walled x
    ends and FP64 arithmetic, with either coupling and either kind of properties."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.ternary_tube(nx=16, ny=4, nz=2)
    assert m.mclbm_workspace_bytes(dict(p, wall_y=1), m.MCLBM_FP32) == m.mclbm_workspace_bytes(p, m.MCLBM_FP32)
    for bad in (dict(p, wall_y=2), dict(p, ny=1, wall_y=1)):
        with pytest.raises(m.MclbmError):
            m.mclbm_workspace_bytes(bad, m.MCLBM_FP32)
    inlet = np.array([0.3, 0.3, 0.4, p["P0"], 1 / 3, 0.05, 0.0, 0.0])
    for q in (dict(p, weak=1), dict(p, cv_coef=np.ones((3, 4))), dict(p, weak=1, wall_x=1)):
        assert m.mclbm_workspace_bytes(dict(q, wall_y=1), m.MCLBM_FP64) == m.mclbm_workspace_bytes(q, m.MCLBM_FP64)
    for q, prec in ((dict(p, wall_y=1, weak=1), m.MCLBM_FP32_FP32), (dict(p, wall_y=1), m.MCLBM_BF16),
                    (dict(p, wall_y=1, wall_x=2, inlet=inlet), m.MCLBM_FP64)):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(q, prec)
        assert "free-slip" in str(e.value)


def test_create_rejects_bad_workspace():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    p, _ = W.binary_interdiffusion()
    with pytest.raises(m.MclbmError):
        m.mclbm_create(p, 1, 0, 1 << 30, 0)                   # NULL workspace
    with pytest.raises(m.MclbmError):
        m.mclbm_create(p, 1, 0x1000, 16, 0)                   # too small (never dereferenced)


def test_batch_workspace_and_validation():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    tubes = [t for t, _ in W.tube_ensemble(ntubes=5, ny=4, nz=4, lmin=8, lmax=40)]
    total = m.mclbm_batch_workspace_bytes(tubes, 1)
    singles = [m.mclbm_workspace_bytes(t, 1) for t in tubes]
    n = sum(t["nx"] * t["ny"] * t["nz"] for t in tubes)
    assert total > 2 * 27 * 4 * n * 4                        # two FP32 buffers of 4 lattices
    assert total < sum(singles)                              # one set of staging buffers
    # a batch of one tube is a single context
    assert m.mclbm_batch_workspace_bytes(tubes[:1], 1) == singles[0]
    mixed = [tubes[0], dict(W.binary_interdiffusion(nx=8, ny=4, nz=4)[0])]
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_batch_workspace_bytes(mixed, 1)               # M differs
    assert "share" in str(e.value)
    periodic = dict(tubes[1])
    periodic["wall_x"] = 0
    with pytest.raises(m.MclbmError):
        m.mclbm_batch_workspace_bytes([tubes[0], periodic], 1)
    bad = dict(tubes[2])
    bad["D"] = np.array(bad["D"]) * np.array([[1, 1, 1], [1, 1, 2], [1, 1, 1]])
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_batch_workspace_bytes([tubes[0], tubes[1], bad], 1)
    assert "tube 2" in str(e.value)
    with pytest.raises(m.MclbmError):
        m.mclbm_batch_workspace_bytes([], 1)


def test_launch_struct_matches_header():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    import ctypes

    src = open(os.path.join(ROOT, "include", "mclbm.h")).read()
    body = re.search(r"typedef struct \{([^{}]*)\} mclbm_launch;", src).group(1)
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    fields = re.findall(r"int32_t\s+(\w+)(?:\[(\d+)\])?;", body)
    assert [f for f, _ in fields] == [f for f, *_ in m.mclbm_launch._fields_]
    assert ctypes.sizeof(m.mclbm_launch) == 4 * sum(int(k or 1) for _, k in fields)


def test_params_struct_matches_header():
    """The binding's mclbm_params has the header's fields in order, and the layout a
    C compiler gives the header's struct (size and every offset)."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    import ctypes
    import shutil
    import subprocess
    import tempfile

    src = open(os.path.join(ROOT, "include", "mclbm.h")).read()
    end = src.index("} mclbm_params;")
    body = src[src.rindex("typedef struct {", 0, end) + len("typedef struct {"):end]
    body = re.sub(r"/\*.*?\*/", "", body, flags=re.S)
    names = []
    for decl in body.split(";"):
        decl = decl.strip()
        if decl:
            rest = re.match(r"(?:const\s+)?\w+\s+(.*)", decl, re.S).group(1)
            names += [v.strip().lstrip("*").strip() for v in rest.split(",")]
    binding = [f for f, *_ in m.mclbm_params._fields_]
    assert [n if n != "lambda" else "lam" for n in names] == binding
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler")
    with tempfile.TemporaryDirectory() as d:
        prog = os.path.join(d, "layout.c")
        with open(prog, "w") as fh:
            fh.write('#include <stdio.h>\n#include <stddef.h>\n#include "mclbm.h"\nint main(void){printf("%zu", sizeof(mclbm_params));')
            for n in names:
                fh.write(f'printf(" %zu", offsetof(mclbm_params, {n}));')
            fh.write("return 0;}\n")
        exe = os.path.join(d, "layout")
        subprocess.run([cc, "-I" + os.path.join(ROOT, "include"), prog, "-o", exe], check=True)
        got = [int(v) for v in subprocess.run([exe], capture_output=True, text=True, check=True).stdout.split()]
    assert got[0] == ctypes.sizeof(m.mclbm_params)
    assert got[1:] == [getattr(m.mclbm_params, b).offset for b in binding]


def test_slaved_species_validation():
    """The slaved species (C field: 0 for species M, or 1..M; the binding's dict
    key is 0-based) is checked; weak coupling slaves none; the tubes of a batch
    agree on it; the workspace does not depend on it."""
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    tube, _ = W.ternary_tube(nx=16, ny=2, nz=2)
    assert m.make_params(tube, m.MCLBM_FP32)[0].slaved == 3          # the workload's slaved species, the last
    assert m.make_params({k: v for k, v in tube.items() if k != "slaved"}, m.MCLBM_FP32)[0].slaved == 0
    base = m.mclbm_workspace_bytes(tube, m.MCLBM_FP32)
    for k in (0, 1, 2):
        assert m.mclbm_workspace_bytes(dict(tube, slaved=k), m.MCLBM_FP32) == base
    for bad in (-2, 3):
        with pytest.raises(m.MclbmError) as e:
            m.mclbm_workspace_bytes(dict(tube, slaved=bad), m.MCLBM_FP32)
        assert "slaved" in str(e.value)
    assert m.mclbm_workspace_bytes(dict(tube, weak=1, slaved=2), m.MCLBM_FP32) > base
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_workspace_bytes(dict(tube, weak=1, slaved=0), m.MCLBM_FP32)
    assert "weak" in str(e.value)
    with pytest.raises(m.MclbmError) as e:
        m.mclbm_batch_workspace_bytes([tube, dict(tube, slaved=1)], m.MCLBM_FP32)
    assert "slaved" in str(e.value)


def test_nn_workspace_and_validation():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    dims = [(13, 4, 3), (40, 2, 5)]
    b = m.mclbm_nn_workspace_bytes(7, 0, 0, 0, 6, dims)
    n = 13 * 12 + 40 * 10
    assert b > 5 * n * 64 * 2                     # the hidden activations dominate
    assert b < m.mclbm_nn_workspace_bytes(7, 0, 0, 0, 6, dims + [(64, 8, 8)])
    assert m.mclbm_nn_workspace_bytes(7, 3, 6, 0, 6, dims) >= b
    assert m.mclbm_nn_workspace_bytes(8, 3, 6, 3, 6, dims) > 0            # conservative: 3 species, 13 outputs
    assert m.mclbm_nn_workspace_bytes(8, 3, 6, 0, 6, dims) > 0            # 17 input channels fit in 32
    for bad in [(0, 0, 0, 0, 6, dims), (17, 0, 0, 0, 6, dims), (16, 16, 1, 0, 6, dims), (7, 8, 0, 0, 6, dims),
                (7, 0, -1, 0, 6, dims), (7, 0, 0, 0, 1, dims), (7, 0, 0, 0, 6, [(0, 4, 4)]),
                (7, 0, 0, 3, 6, dims), (15, 0, 0, 10, 6, dims)]:
        with pytest.raises(m.MclbmError):
            m.mclbm_nn_workspace_bytes(*bad)


def test_nn_param_count_matches_the_oracle():
    """Parameter count of the library's layout equals the oracle's (host order)."""
    from oracle import surrogate_oracle as S

    assert S.param_count(7, 6) == 27 * (7 * 64 + 4 * 64 * 64 + 64 * 7) + 5 * 64 + 7
    assert S.param_count(7, 6, S=6) == 27 * (13 * 64 + 4 * 64 * 64 + 64 * 7) + 5 * 64 + 7


def test_stream_copy_rejects_bad_sizes_without_a_device():
    m = pytest.importorskip("paper_2004_11286_amd.mclbm")
    with pytest.raises(m.MclbmError):
        m.mclbm_stream_copy(4096, 8192, 15)          # not a multiple of 16
    with pytest.raises(m.MclbmError):
        m.mclbm_stream_copy(4100, 8192, 16)          # misaligned
    with pytest.raises(m.MclbmError):
        m.mclbm_stream_copy(4096, 4096 + 16, 64)     # overlapping
    with pytest.raises(m.MclbmError):
        m.mclbm_stream_copy(0, 4096, 16)             # null


def test_binding_loads_torch_runtime_first():
    # importing the package before torch must still leave one HIP runtime in the process
    import subprocess
    import sys

    code = ("import paper_2004_11286_amd.mclbm, sys; "
            "maps = open('/proc/self/maps').read(); "
            "paths = {l.split()[-1] for l in maps.splitlines() if 'libamdhip64' in l}; "
            "print(len(paths)); sys.exit(0 if len(paths) == 1 else 1)")
    r = subprocess.run([sys.executable, "-c", code], cwd=os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
