"""Benchmark: D3Q27 mixture lattice Boltzmann step on one MI355X.

Workload: the binary Kelvin--Helmholtz shear layer on a 256^3 periodic grid
(molar masses 2 and 28, u_x = +-0.1 with tanh profiles, seeded noise), FP32
population storage. A step is one pass of the whole path: moments, stencil
field, collide-and-stream over all 16.8 M nodes.

Prints one JSON line (the last line of stdout) with MLUPS, the HBM roofline of
the dominant kernel (timed with HIP events on the library's stream), the other
storage precisions measured side by side with their per-field error against the
FP32 run, and the FP64 CPU oracle timed on a bounded crop of the same workload.

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--precision fp32|fp32_fp32|fp16|bf16|fp64]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
PROFILES = os.path.join(ROOT, "profiles")
KERNEL_SOURCES = ["lattice.hpp", "node_ops.hpp", "device_ops.hpp", "kernels.hpp", "inst_fp64.hip",
                  "inst_fp32_fp64.hip", "inst_weak.hip", "inst_cvt.hip", "inst_weak_cvt.hip", "inst_fp32.hip",
                  "inst_fp16.hip", "inst_bf16.hip"]


def record_fields(M: int, weak: bool = False, cvt: bool = False) -> int:
    """Node record: Phi (3), omega, C_p, rho, u (3), T, omega_1, q_neq (3), rho_a (M-1;
    M under weak coupling), V_a (3 M), under weak coupling u_s (3), and with
    temperature-dependent heat capacities Y_a (M-1)."""
    return 14 + (M if weak else M - 1) + 3 * M + (3 if weak else 0) + (M - 1 if cvt else 0)


def algorithmic_bytes(M: int, s_bytes: int, r_bytes: int, weak: bool = False, cvt: bool = False) -> dict:
    """Bytes each kernel must move per node, every value read or written once:
    k_moments reads the populations and writes the record; k_gfield reads Phi and
    omega and writes G; k_collide reads the populations, the record except Phi,
    and G, and writes the populations. Stored lattices: M + 1 (strong coupling),
    M + 2 (weak)."""
    L = M + 2 if weak else M + 1
    pops = L * 27 * s_bytes
    rec = record_fields(M, weak, cvt) * r_bytes
    return {
        "k_moments": pops + rec,
        "k_gfield": 4 * r_bytes + 3 * r_bytes,
        "k_collide": 2 * pops + (rec - 3 * r_bytes) + 3 * r_bytes,
        "step": 3 * pops + 2 * rec + 7 * r_bytes,
        "method_min": 2 * pops,
    }


def record_bytes(precision: int, mc) -> int:
    return 8 if precision == mc.MCLBM_FP64 else 4


def kernel_source_hash() -> str:
    import hashlib

    h = hashlib.sha256()
    for name in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_2004_11286_amd", "csrc", name), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel: str, precision: str):
    """HBM bytes per launch from the committed counter summary, if it was taken
    on the current kernel sources (else None)."""
    path = os.path.join(PROFILES, f"{kernel}_shear256_{precision}_hbm_counters.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    return float(vals["hbm_bytes_per_launch"])


def copy_ceiling_gbs(gib: int = 4, reps: int = 10) -> dict:
    """Read + write bandwidth of two device-to-device copies, the practical
    streaming ceilings next to the 8 TB/s peak: the runtime's copy kernel and the
    library's 16-byte nontemporal copy (mclbm_stream_copy)."""
    import torch

    from paper_2004_11286_amd import mclbm as mc

    n = gib << 28
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    out = {}
    for name, fn in (("runtime_copy_GBs", lambda: b.copy_(a)), ("stream_copy_GBs", lambda: mc.stream_copy(b, a))):
        fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        e1.synchronize()
        out[name] = 8.0 * n / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a, b
    torch.cuda.empty_cache()
    return out


def time_run(mc, params, fields, precision, steps, warmup):
    import torch

    sim = mc.Sim(params, precision)
    sim.init_fields(**fields)
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    stats = {}
    for k in (mc.MCLBM_K_MOMENTS, mc.MCLBM_K_GFIELD, mc.MCLBM_K_COLLIDE):
        ms, launches, name = sim.kernel_stats(k)
        stats[name] = {"total_ms": ms, "launches": launches, "avg_ms": ms / max(launches, 1)}
    sim.set_timing(False)
    return sim, t1 - t0, stats


def cpu_baseline(seconds_target: float = 15.0):
    """The FP64 oracle, unchanged, on a 32 x 256 x 8 box of the shear-layer recipe
    (the full band geometry across y, a thin slab in x and z, long-wave
    perturbation), timed over whole steps."""
    from oracle import oracle as O
    from paper_2004_11286_amd import workloads as W

    O.build()
    params, fields = W.shear_layer(nx=32, ny=256, nz=8, kmax=1)
    o = O.OracleSim(params)
    o.init_fields(**fields)
    o.step(1)                                  # first touch
    n = 32 * 256 * 8
    steps, elapsed = 0, 0.0
    while elapsed < seconds_target and steps < 200:
        t0 = time.perf_counter()
        o.step(1)
        elapsed += time.perf_counter() - t0
        steps += 1
    cpu_model = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            cpu_model = next((ln.split(":", 1)[1].strip() for ln in fh if ln.startswith("model name")), cpu_model)
    except OSError:
        pass
    return {"value": n * steps / elapsed / 1e6, "unit": "MLUPS", "cores": O.threads(), "kind": "oracle",
            "sample": f"FP64 oracle, {steps} steps of a 32x256x8 box of the shear-layer recipe "
                      f"({elapsed:.1f} s)", "cpu_model": cpu_model}


def ensemble_bench(mc, steps: int = 50, seq_steps: int = 10, trial_steps: int = 10):
    """The batched ensemble: 512 independent ternary tubes, L ~ U{32..256} x 16 x
    16 with walls (18.9 M nodes), FP32 storage, all tubes in one context.
    Aggregate MLUPS of the autotuned batched launch, of plain batched launches,
    of a replayed HIP graph, and of one launch triplet per tube and step (the
    unbatched reference), all timed with HIP events on the context's stream."""
    import torch

    from paper_2004_11286_amd import workloads as W

    tubes = W.tube_ensemble()
    b = mc.Batch([p for p, _ in tubes], mc.MCLBM_FP32)
    b.init_fields([f for _, f in tubes])
    n = b.n

    def timed(k, **launch):
        b.set_launch(**launch)
        b.step(2 if not launch.get("graph_steps") else launch["graph_steps"])   # warm-up / graph build
        if b.step_count % 2:
            b.step(1)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(b.stream)
        b.step(k)
        e1.record(b.stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1)
        return {"MLUPS": n * k / (ms * 1e-3) / 1e6, "ms_per_step": ms / k}

    base = dict(variant=0, swizzle=0, order=0, graph_steps=0, sequential=0, split=0)
    out = {"workload": "512 ternary tubes L~U{32..256}x16x16 with walls, FP32 storage, one context",
           "nodes": n, "tubes": len(tubes)}
    out["sequential"] = timed(seq_steps, **dict(base, sequential=1))
    out["batched"] = timed(steps, **base)
    out["batched_graph"] = timed(steps, **dict(base, graph_steps=10))
    out["batched_split"] = timed(steps, **dict(base, split=1))
    report = b.autotune(trial_steps)
    out["autotune_report"] = report.strip().splitlines()
    chosen = b.launch()
    out["autotuned"] = timed(steps, **chosen)
    out["autotuned"]["launch"] = chosen
    out["speedup_batched_vs_sequential"] = out["autotuned"]["MLUPS"] / out["sequential"]["MLUPS"]
    c = b.conservation()
    out["finite"] = bool(np.isfinite(c).all())
    b.close()
    del b
    torch.cuda.empty_cache()
    return out


BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16 matrix-core peak


def surrogate_bench(train_iters: int = 36000):
    """The learned surrogate: trained by the library's BF16 MFMA kernels on
    trajectories of a 2048-tube ensemble (every 100 steps up to 5000; the tubes
    are one-dimensional, uniform in y and z, so a one-node cross-section carries
    all of their physics), then judged by the lattice on eight held-out
    128 x 32 x 32 ternary tubes (1 M nodes): mole-fraction L-infinity and RMS
    errors of one 100-step hop, the same for the persistence prediction, the
    mole residual and whether the advance entry point accepted the hop (residual
    <= 1e-4) or fell back to the lattice, and the times of the forward pass, of
    the whole advance and of the 100 lattice steps. The conv roofline: forward
    FLOP / forward time against the BF16 peak."""
    from paper_2004_11286_amd import surrogate as SG
    from paper_2004_11286_amd import workloads as W

    t0 = time.perf_counter()
    train_tubes = W.tube_ensemble(ntubes=2048, ny=1, nz=1, seed=11286)
    snaps, dims = SG.trajectories(train_tubes, K=100, nsnap=50)
    M = 3
    C = SG.channels(M)
    st = SG.channel_stats(snaps, dims, M)
    norm = SG.norm_from_stats(st, M)
    pw = SG.pair_weights(st, M)
    net = SG.build_net(dims, [p for p, _ in train_tubes], norm, M)
    ms_train_step, _ = SG.timed_train_step(net, snaps, pw)
    net.set_params(SG.he_init(C, 6, SG.DEPTH, 0, 3 * M + 4))
    losses = SG.train(net, snaps, train_iters, pw, lr=2e-4, clip=2.0)
    params = net.get_params()
    n_train = sum(a * b * c for a, b, c in dims)
    net.close()
    del snaps
    train_s = time.perf_counter() - t0
    eval_tubes = W.tube_ensemble(ntubes=8, ny=32, nz=32, lmin=128, lmax=128, seed=2025)
    res = SG.evaluate(params, norm, eval_tubes, K=100, starts=(0, 1000, 3000), resid_tol=1e-4)
    n_eval = sum(p["nx"] * p["ny"] * p["nz"] for p, _ in eval_tubes)
    fpn = SG.conv_flops_per_node(C, M + 6, 3 * M + 4)
    flops = fpn * n_eval
    ms_fwd = float(np.median([r["ms_forward"] for r in res]))
    achieved = flops / (ms_fwd * 1e-3) / 1e12
    train_flops = 3 * fpn * n_train
    return {
        "workload": "train: 2048 ternary tubes L~U{32..256}x1x1, 50 snapshots every 100 steps; "
                    "apply: 8 held-out ternary tubes 128x32x32, one 100-step hop from t0 = 0, 1000, 3000",
        "network": {"layers": SG.DEPTH, "width": 64, "kernel": "3x3x3", "params": int(params.size),
                    "input": "X_a, T, u, p (+ second BF16 terms of X_a, 6 tube constants)",
                    "output": "conservative: face fluxes of the molar densities p X_a / T, changes of T and u",
                    "padding": "replicate at the x walls, periodic in y and z",
                    "loss": "molar densities, T, u, and the x fluxes the target change implies (weight 0.1)",
                    "dtype": "bf16 weights/activations, fp32 accumulate"},
        "train": {"iters": train_iters, "lr": 2e-4, "clip_times_mean_norm": 2.0, "seconds": train_s, "loss_first100": float(np.mean(losses[:100])),
                  "loss_last100": float(np.mean(losses[-100:])), "ms_per_step": ms_train_step,
                  "TFLOPs_per_step_approx": train_flops / (ms_train_step * 1e-3) / 1e12},
        "eval": res,
        "hops_within_1e-3_linf": [{"t0": r["t0"], "X_linf": r["X_linf"],
                                   "speedup_advance_vs_lattice": r["ms_lattice"] / r["ms_advance"]}
                                  for r in res if r["X_linf"] <= 1e-3],
        "speedup_forward_vs_lattice": float(np.median([r["ms_lattice"] / r["ms_forward"] for r in res])),
        "speedup_advance_vs_lattice": float(np.median([r["ms_lattice"] / r["ms_advance"] for r in res])),
        "roofline_conv_forward": {"bound": "mfma", "achieved": achieved, "peak": BF16_PEAK_TFLOPS,
                                  "unit": "TFLOP/s", "frac": achieved / BF16_PEAK_TFLOPS,
                                  "flop_per_node": fpn, "nodes": n_eval},
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--precision", default="fp32")
    ap.add_argument("--n", type=int, default=256, help="cube edge")
    ap.add_argument("--no-variants", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-ensemble", action="store_true")
    ap.add_argument("--no-surrogate", action="store_true")
    ap.add_argument("--surrogate-iters", type=int, default=36000)
    ap.add_argument("--copy-calibrate", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB mebibytes five times (to scale HBM counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU slab decomposition is a design, not an implementation)", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_2004_11286_amd import mclbm as mc
    from paper_2004_11286_amd import workloads as W

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    torch.cuda.set_device(0)
    if args.copy_calibrate:
        nbytes = args.copy_calibrate << 20
        src = torch.ones(nbytes, dtype=torch.uint8, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        el = (time.perf_counter() - t0) / 5
        print(json.dumps({"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "copies": 5,
                          "GBs_read_plus_write": 2 * nbytes / el / 1e9}))
        return
    copies = copy_ceiling_gbs()
    copy_gbs = max(copies.values())
    params, fields = W.shear_layer(nx=args.n, ny=args.n, nz=args.n)
    M = params["M"]
    n = args.n ** 3
    prec = mc.PRECISIONS[args.precision]
    sim, elapsed, stats = time_run(mc, params, fields, prec, args.steps, args.warmup)
    mlups = n * args.steps / elapsed / 1e6
    sb, rb = mc.STORAGE_BYTES[prec], record_bytes(prec, mc)
    ab = algorithmic_bytes(M, sb, rb)
    col = stats["k_collide"]
    achieved = ab["k_collide"] * n / (col["avg_ms"] * 1e-3) / 1e9
    kernel_gbs = {k: ab[k] * n / (v["avg_ms"] * 1e-3) / 1e9 for k, v in stats.items()}
    ref = sim.read_moments()
    base_count = sim.step_count
    sim.close()
    del sim
    torch.cuda.empty_cache()

    variants = {}
    if not args.no_variants:
        for name in ("fp32_fp32", "fp16", "bf16"):
            if mc.PRECISIONS[name] == prec:
                continue
            v, el, st = time_run(mc, params, fields, mc.PRECISIONS[name], args.steps, args.warmup)
            assert v.step_count == base_count
            got = v.read_moments()
            errs = {}
            for k in ("X", "rho", "u", "p", "T"):
                den = np.abs(ref[k]).max()
                errs[k] = float(np.abs(got[k] - ref[k]).max() / den)
            variants[name] = {"MLUPS": n * args.steps / el / 1e6, "speedup_vs_" + args.precision:
                              (n * args.steps / el / 1e6) / mlups,
                              "rel_linf_vs_" + args.precision: errs,
                              "collide_avg_ms": st["k_collide"]["avg_ms"]}
            v.close()
            del v
            torch.cuda.empty_cache()

    weak = None
    if not args.no_variants:
        # weak coupling (all M species lattices evolved) on the same workload: a
        # different model from strong coupling, so its fields are not compared
        wp = dict(params, weak=1)
        v, el, st = time_run(mc, wp, fields, prec, args.steps, args.warmup)
        wab = algorithmic_bytes(M, sb, rb, weak=True)
        wcol = st["k_collide"]["avg_ms"]
        wgbs = wab["k_collide"] * n / (wcol * 1e-3) / 1e9
        weak = {"MLUPS": n * args.steps / el / 1e6, "ms_per_step": el / args.steps * 1e3,
                "stored_lattices": M + 2, "launch": v.launch(), "collide_avg_ms": wcol,
                "collide_algorithmic_bytes_per_node": wab["k_collide"], "collide_GBs": wgbs,
                "collide_frac_of_hbm_peak": wgbs / HBM_PEAK_GBS,
                "kernels_avg_ms": {k: x["avg_ms"] for k, x in st.items()}}
        v.close()
        del v
        torch.cuda.empty_cache()

    weak_fp16 = None
    if not args.no_variants:
        # weak coupling with FP16 deviation storage and FP32 arithmetic
        v, el, st = time_run(mc, dict(params, weak=1), fields, mc.MCLBM_FP16, args.steps, args.warmup)
        hab = algorithmic_bytes(M, 2, 4, weak=True)
        hcol = st["k_collide"]["avg_ms"]
        weak_fp16 = {"MLUPS": n * args.steps / el / 1e6, "ms_per_step": el / args.steps * 1e3,
                     "launch": v.launch(), "collide_avg_ms": hcol,
                     "collide_algorithmic_bytes_per_node": hab["k_collide"],
                     "collide_GBs": hab["k_collide"] * n / (hcol * 1e-3) / 1e9,
                     "kernels_avg_ms": {k: x["avg_ms"] for k, x in st.items()}}
        v.close()
        del v
        torch.cuda.empty_cache()

    cv_of_T = None
    if not args.no_variants:
        # temperature-dependent heat capacities (cubic C_{a,v}(T), about twice the
        # constant part at the shear layer's T = 1) on the same workload
        cv = np.asarray(params["cv"], dtype=np.float64)
        shapes = [[1.0, 0.6, 0.1, 0.3], [1.0, 0.0, 0.4, 0.0]]
        cp_ = dict(params, cv_coef=np.stack([cv[a] * np.asarray(shapes[a]) for a in range(M)]))
        v, el, st = time_run(mc, cp_, fields, prec, args.steps, args.warmup)
        cab = algorithmic_bytes(M, sb, rb, cvt=True)
        ccol = st["k_collide"]["avg_ms"]
        cgbs = cab["k_collide"] * n / (ccol * 1e-3) / 1e9
        cv_of_T = {"MLUPS": n * args.steps / el / 1e6, "ms_per_step": el / args.steps * 1e3,
                   "cv_coef_shape": shapes, "collide_avg_ms": ccol,
                   "collide_algorithmic_bytes_per_node": cab["k_collide"], "collide_GBs": cgbs,
                   "collide_frac_of_hbm_peak": cgbs / HBM_PEAK_GBS,
                   "kernels_avg_ms": {k: x["avg_ms"] for k, x in st.items()}}
        v.close()
        del v
        torch.cuda.empty_cache()

    weak_cv_of_T = None
    if not args.no_variants:
        # weak coupling with the same temperature-dependent heat capacities
        v, el, st = time_run(mc, dict(cp_, weak=1), fields, prec, args.steps, args.warmup)
        wcab = algorithmic_bytes(M, sb, rb, weak=True, cvt=True)
        wccol = st["k_collide"]["avg_ms"]
        wcgbs = wcab["k_collide"] * n / (wccol * 1e-3) / 1e9
        weak_cv_of_T = {"MLUPS": n * args.steps / el / 1e6, "ms_per_step": el / args.steps * 1e3,
                        "launch": v.launch(), "collide_avg_ms": wccol,
                        "collide_algorithmic_bytes_per_node": wcab["k_collide"], "collide_GBs": wcgbs,
                        "collide_frac_of_hbm_peak": wcgbs / HBM_PEAK_GBS,
                        "kernels_avg_ms": {k: x["avg_ms"] for k, x in st.items()}}
        v.close()
        del v
        torch.cuda.empty_cache()

    open_x = None
    if not args.no_variants:
        # open x ends: the same 256^3 binary fields carried through the domain by a
        # mean flow u_x = 0.05, fed at x = 0 with the mean composition and state
        Xm = [float(fields["X"][a].mean()) for a in range(M)]
        Xm[-1] = 1.0 - sum(Xm[:-1])
        op_ = dict(params, wall_x=2,
                   inlet=np.array(Xm + [float(fields["p"].mean()), float(fields["T"].mean()), 0.05, 0.0, 0.0]))
        of = dict(fields, u=fields["u"] + np.array([0.05, 0.0, 0.0])[:, None, None, None])
        v, el, st = time_run(mc, op_, of, prec, args.steps, args.warmup)
        oc = st["k_collide"]["avg_ms"]
        open_x = {"MLUPS": n * args.steps / el / 1e6, "ms_per_step": el / args.steps * 1e3, "collide_avg_ms": oc,
                  "collide_GBs": ab["k_collide"] * n / (oc * 1e-3) / 1e9,
                  "kernels_avg_ms": {k: x["avg_ms"] for k, x in st.items()}}
        v.close()
        del v
        torch.cuda.empty_cache()

    ensemble = None if args.no_ensemble else ensemble_bench(mc)
    surrogate = None if args.no_surrogate else surrogate_bench(args.surrogate_iters)
    cpu = None if args.no_cpu else cpu_baseline()
    out = {
        "metric": "D3Q27 mixture MLUPS & % HBM roofline; FP16-store and surrogate vs FP32 plain",
        "value": mlups,
        "unit": "MLUPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp32": "f32-store/f64-collide", "fp32_fp32": "f32", "fp64": "f64",
                  "fp16": "f16-store/f32-collide", "bf16": "bf16-store/f32-collide"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"binary Kelvin-Helmholtz shear layer {args.n}^3 periodic, D3Q27, "
                               f"{M} species + momentum + energy lattices, strong coupling",
                   "nodes": n, "species": M, "precision": args.precision, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": "k_collide", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": measured_traffic("k_collide", args.precision),
                     "algorithmic_bytes_per_node": ab["k_collide"],
                     "algorithmic_bytes_per_launch": ab["k_collide"] * n,
                     **copies, "frac_of_best_copy": achieved / copy_gbs},
        "kernels": {k: {"avg_ms": v["avg_ms"], "launches": v["launches"], "GBs": kernel_gbs[k],
                        "algorithmic_bytes_per_node": ab[k]} for k, v in stats.items()},
        "step_effective_GBs": {"step_bytes_per_node": ab["step"], "GBs": ab["step"] * mlups * 1e6 / 1e9,
                               "method_min_bytes_per_node": ab["method_min"],
                               "method_min_frac": ab["method_min"] * mlups * 1e6 / 1e9 / HBM_PEAK_GBS},
        "variants": variants,
        "weak_coupling": weak,
        "weak_fp16": weak_fp16,
        "cv_of_T": cv_of_T,
        "weak_cv_of_T": weak_cv_of_T,
        "open_x": open_x,
        "ensemble": ensemble,
        "surrogate": surrogate,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out))


if __name__ == "__main__":
    main()
