"""sn-K exchange build benchmark on one MI355X.

A step is one full build K[P] of the 1000-atom water-like cluster (config 5: 9,676 Cartesian
s/p/d functions, 50x194 grid per atom = 9.7 M points in 256-point batches, molecule-local
density) in the mixed-precision + learned-screening form: collocation, F = P Phi, the learned
screen, the 3c-CP A.F digestion, K~ = G Phi^T, symmetrisation and E_x, with basis screening
(eps_B = 1e-9) and P and K resident in HBM.  The plain FP64 build of the same workload (no
density screening) is the reference for the speed-up and for dE_x and max|dK|.  Prints one
JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu-baseline] [--no-extras]

`value` counts the workload's shell-pair x grid-point units (every unique shell pair with a
surviving primitive pair, at every grid point: the work the plain FP64 build evaluates) per
second of the timed build.  The extra keys carry the FP64 + learned build of the same
workload, the 150-atom cluster (config 3: mixed + learned against plain FP64), and the 30-atom
cluster (config 2: plain FP64, the oracle-parity workload).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sn-K build time + shell-pair·gridpoint ints/s; mixed+learned vs FP64 at 1e-6 Eh"
CLASSES = ("ss", "ps", "pp", "ds", "dp", "dd")
GEMM_KINDS = ("F product, FP64 matrix cores", "F product, FP32 matrix cores", "K~ product, FP64 matrix cores",
              "K~ product, FP32 matrix cores")
EPS_BASIS = 1e-9


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(system, pairs_per_point: float):
    """The CPU oracle (plain sn-K: every shell pair at every point, FP64) timed on a bounded
    sample of the same workload: one evenly spaced grid point per host thread (the oracle
    parallelises over points, and one point of this system is tens of seconds of one core's
    work), in the units of `value`: the GPU's count of surviving shell pairs per point times the
    points evaluated, per second."""
    import numpy as np
    from oracle import oracle as O
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    n = max(1, min(64, nthreads))
    stride = max(1, system.npts // n)
    sample = system.subset_points(np.arange(stride // 2, system.npts, stride)[:n])
    t = time.perf_counter()
    O.snk(sample, nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": pairs_per_point * sample.npts / dt, "unit": "shell-pair·gridpoints/s", "cores": nthreads,
            "kind": "oracle",
            "sample": "%d evenly spaced grid points of the same workload (every %d-th of %d), %.0f surviving shell "
                      "pairs per point counted as on the GPU, %.1f s" % (sample.npts, stride, system.npts,
                                                                          pairs_per_point, dt)}


def time_builds(ctx, P, K, stream, steps, warmup):
    """Mean time of `steps` builds after `warmup` (HIP events on the build's stream, and the
    host clock around the same region; the larger of the two)."""
    import torch
    for i in range(warmup):
        ctx.build_device(P.data_ptr(), K.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(steps):
        ctx.build_device(P.data_ptr(), K.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    return max(e0.elapsed_time(e1) / steps, 1000.0 * (time.perf_counter() - t0) / steps)


def phases(st):
    return {"collocate": st["t_collocate_ms"], "fgemm": st["t_fgemm_ms"], "screen": st["t_screen_ms"],
            "afg": st["t_afg_ms"], "kgemm": st["t_kgemm_ms"], "finish": st["t_finish_ms"]}


# HBM bytes per launch of a dominant kernel from the copy-calibrated FETCH_SIZE + WRITE_SIZE
# counter runs of the same build (profiles/gsplit_config5_mixed_learned.md,
# profiles/afg_config2_fp64.md); valid only for the kernel code and batch groups those runs
# measured, so an entry goes when its kernel changes
PROFILED_TRAFFIC = {"gsplit_kernel (F product, FP32 matrix cores)": 6.764e9,   # config 5, mixed + learned
                    "afg_kernel<1,0> (ps, A.F digestion)": 2.821e10}           # config 2, plain FP64


def dominant_kernel(st):
    """The kernel family with the most GPU time in a statistics build (per-class A.F kernels and
    the four grouped product kinds, all timed by the library with HIP events on its stream),
    with its algorithmic work per launch, average launch time and the roofline it sits under."""
    from paper_2303_14280_amd import flops
    cands = []
    groups = max(1, int(st["n_groups"]))
    for c in range(6):
        if st["t_afg_class_ms"][c] <= 0:
            continue
        work = flops.class_flops(c, st["pair_points"][c], st["prim_pair_points"][c])
        cands.append((st["t_afg_class_ms"][c], "afg_kernel<%d,%d> (%s, A.F digestion)" % (flops.CLASS_L[c] + (CLASSES[c],)),
                      work, groups, "alu", flops.PEAK_FP64_VALU_TFLOPS))
    for k in range(4):
        if st["t_gemm_ms"][k] <= 0:
            continue
        f64, f32 = st["gemm_kind_flops"][k]
        # a product with parts on both kinds of matrix cores is priced at its combined peak: the
        # flops over the time the two parts take at their own peaks
        ideal_s = f64 / (flops.PEAK_FP64_MFMA_TFLOPS * 1e12) + f32 / (flops.PEAK_FP32_MFMA_TFLOPS * 1e12)
        peak = (f64 + f32) / ideal_s / 1e12 if ideal_s > 0 else flops.PEAK_FP64_MFMA_TFLOPS
        cands.append((st["t_gemm_ms"][k], "%s (%s)" % ("gsplit_kernel" if f64 > 0 and f32 > 0 else "ggemm_kernel",
                                                       GEMM_KINDS[k]),
                      f64 + f32, max(1, st["gemm_launches"][k]), "mfma", peak))
    t, name, work, launches, bound, peak = max(cands, key=lambda x: x[0])
    launch_ms = t / launches
    achieved = work / launches / (launch_ms * 1e-3) / 1e12
    return {"bound": bound, "kernel": name, "achieved": achieved, "peak": peak, "unit": "TFLOP/s",
            "frac": achieved / peak, "traffic": PROFILED_TRAFFIC.get(name), "launch_ms": launch_ms,
            "algorithmic_flops": work / launches, "launches_per_build": launches}


# Device memory the library may use for batch groups: a fixed figure rather than a share of
# what is free at the time (the library's own default, 0.45 of it), so that every run, profiled
# or not, splits a workload into the same groups.  Two thirds of an MI355X's 268 GiB leaves room
# for the buffers outside the budget (lists, partial products, the benchmark's tensors); larger
# groups mean fewer launch tails (1000-atom build: 19 groups 370 ms, 13 groups 348 ms).
DEVICE_BUDGET = 180 << 30


def make_ctx(s, stream, mlp, **kw):
    from paper_2303_14280_amd import snk
    kw.setdefault("max_device_bytes", DEVICE_BUDGET)
    return snk.Context(s, flags=snk.SNK_DEVICE_PTRS, stream=stream.cuda_stream, device=0, screener=mlp, **kw)


def run_variant(name, s, P, stream, mlp, steps, warmup, ref=None, **kw):
    """Create a context, time `steps` builds, then one statistics build; errors against ref."""
    import torch
    t = time.perf_counter()
    ctx = make_ctx(s, stream, mlp, **kw)
    t_create = time.perf_counter() - t
    K = torch.empty_like(P)
    if steps > 0:
        ms = time_builds(ctx, P, K, stream, steps, warmup)
    st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
    torch.cuda.synchronize()
    if steps <= 0:
        ms = st["t_total_ms"]
    ctx.close()
    ints = float(sum(st["pair_points"]) + st["pair_points_skipped"])
    g64, g32 = st["gemm_flops_fp64"], st["gemm_flops_fp32"]
    r = {"ms_per_step": ms, "create_s": t_create, "ex": st["ex"], "phases_ms": phases(st),
         "skipped_pair_points_fraction": st["pair_points_skipped"] / max(1.0, ints),
         "fp32_afg_pair_points_fraction": st["pair_points_lowprec"] / max(1.0, ints),
         "fp32_gemm_flops_fraction": g32 / max(1.0, g64 + g32), "gemm_flops": g64 + g32,
         "fp32_gemm_energy_bound": st["lowprec_bound"], "skipped_rigorous_bound_sum": st["skipped_bound"],
         "shell_pair_points": ints, "effective_rate": ints / (ms * 1e-3),
         "tile_functions": st["tile_functions"], "tile_f_rows": st["tile_frows"], "tile_g_rows": st["tile_grows"]}
    if ref is not None:
        K0, ms0, ex0 = ref
        r["speedup_vs_fp64"] = ms0 / ms
        r["dE_x_vs_fp64"] = st["ex"] - ex0
        r["max_dK_vs_fp64"] = float((K - K0).abs().max().item())
    log("%s: %.1f ms/step, E_x %.10f%s" % (name, ms, st["ex"], "" if ref is None else
                                            ", dE_x %.2e, max|dK| %.2e, x%.2f vs FP64" %
                                            (r["dE_x_vs_fp64"], r["max_dK_vs_fp64"], r["speedup_vs_fp64"])))
    return r, K, st


def headline(args, stream):
    """config 5: plain FP64 (one build, the reference), FP64 + learned, mixed + learned."""
    import torch
    from paper_2303_14280_amd import snk, synth
    t = time.perf_counter()
    s = synth.make_system(5)
    log("config 5 generated in %.1f s" % (time.perf_counter() - t))
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    mlp = snk.load_screener(device=0)
    out = {"system": s}
    r0, K0, st0 = run_variant("config 5 fp64 (plain, reference)", s, P, stream, mlp, 0, 0, eps_basis=EPS_BASIS)
    ref = (K0, r0["ms_per_step"], r0["ex"])
    out["fp64"] = r0
    out["fp64+learned"], _, _ = run_variant("config 5 fp64+learned", s, P, stream, mlp, max(2, args.steps // 2), 1,
                                            ref=ref, eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED,
                                            eps_skip_energy=args.eps)
    r, K, st = run_variant("config 5 mixed+learned", s, P, stream, mlp, args.steps, args.warmup, ref=ref,
                           eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED, precision=snk.SNK_MIXED,
                           eps_skip_energy=args.eps, eps_lowprec_energy=args.eps)
    r["speedup_vs_fp64_learned"] = out["fp64+learned"]["ms_per_step"] / r["ms_per_step"]
    out["mixed+learned"] = r
    out["stats"] = st
    out["ints"] = r0["shell_pair_points"]
    del P, K0, K
    torch.cuda.empty_cache()
    return out


def config3(args, stream):
    """150-atom cluster, delocalised density: mixed + learned against plain FP64."""
    import torch
    from paper_2303_14280_amd import snk, synth
    s = synth.make_system(3)
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    mlp = snk.load_screener(device=0)
    res = {"workload": "config3: %d atoms, %d functions, %d grid points, %s density, eps_basis %g"
                       % (len(s.atom_Z), s.nbf, s.npts, s.density, EPS_BASIS)}
    r0, K0, _ = run_variant("config 3 fp64", s, P, stream, mlp, 0, 0, eps_basis=EPS_BASIS)
    ref = (K0, r0["ms_per_step"], r0["ex"])
    res["fp64"] = r0
    res["fp64+learned"], _, _ = run_variant("config 3 fp64+learned", s, P, stream, mlp, 2, 1, ref=ref,
                                            eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED,
                                            eps_skip_energy=args.eps)
    res["mixed+learned"], _, _ = run_variant("config 3 mixed+learned", s, P, stream, mlp, 2, 1, ref=ref,
                                             eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED,
                                             precision=snk.SNK_MIXED, eps_skip_energy=args.eps,
                                             eps_lowprec_energy=args.eps)
    return res


def dfj_config2(args, stream):
    """The density-fitted Coulomb matrix (Sec. II.B) of config 2 with the seeded auxiliary basis:
    set-up (metric and its Cholesky factor) once, then timed builds J[P]."""
    import torch
    from paper_2303_14280_amd import snk, synth
    s = synth.make_system(2)
    aux = synth.make_aux_basis(s)
    t = time.perf_counter()
    ctx = snk.DfJ(s, aux, stream=stream.cuda_stream)
    t_create = time.perf_counter() - t
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    J = torch.empty_like(P)
    for _ in range(args.warmup):
        ctx.build_device(P.data_ptr(), J.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        ctx.build_device(P.data_ptr(), J.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1) / args.steps, 1000.0 * (time.perf_counter() - t0) / args.steps)
    ej = ctx.build_device(P.data_ptr(), J.data_ptr(), energy=True)
    ctx.close()
    log("DF-J config 2: %d functions, %d auxiliary functions: %.2f ms/build (set-up %.2f s), E_J %.10f" %
        (s.nbf, aux.nfunc, ms, t_create, ej))
    return {"workload": "config2 density-fitted Coulomb matrix: %d functions, %d auxiliary functions "
                        "(seeded even-tempered s/p/d set), FP64, no screening" % (s.nbf, aux.nfunc),
            "ms_per_step": ms, "create_s": t_create, "e_j": ej}


def config2(args, stream):
    """30-atom cluster: the plain FP64 build (the oracle-parity workload) and mixed + learned."""
    import torch
    from paper_2303_14280_amd import snk, synth
    s = synth.make_system(2)
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    mlp = snk.load_screener(device=0)
    res = {"workload": "config2: %d atoms, %d functions, %d grid points, %s density, no basis screening"
                       % (len(s.atom_Z), s.nbf, s.npts, s.density)}
    r0, K0, st0 = run_variant("config 2 fp64", s, P, stream, mlp, args.steps, args.warmup)
    res["fp64"] = r0
    res["fp64"]["dominant_kernel"] = dominant_kernel(st0)
    res["mixed+learned"], _, _ = run_variant("config 2 mixed+learned", s, P, stream, mlp, args.steps, args.warmup,
                                             ref=(K0, r0["ms_per_step"], r0["ex"]), screen=snk.SNK_SCREEN_LEARNED,
                                             precision=snk.SNK_MIXED, eps_skip_energy=args.eps,
                                             eps_lowprec_energy=args.eps)
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the config 3 and config 2 comparisons")
    ap.add_argument("--eps", type=float, default=5e-6,
                    help="estimate budget (Eh) of the learned screen's skipped blocks and of the FP32 blocks")
    ap.add_argument("--profile", choices=("config5", "config2", "dfj2", "xc2", "deloc4"), default=None,
                    help="only time one build for profiler runs (no JSON): config5 = the headline build "
                         "(mixed + learned), config2 = the plain FP64 build of config 2, dfj2 = the "
                         "density-fitted Coulomb build of config 2, xc2 = the PBE potential of config 2, "
                         "deloc4 = FP64 + learned on config 4 with a delocalised density")
    ap.add_argument("--delocalised", type=int, default=0, metavar="CONFIG",
                    help="only compare plain FP64 with FP64 + learned and mixed + learned on config 4 or 5 "
                         "with a delocalised density (one JSON line of its own)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of this many MiB (HBM counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 8
        a = torch.ones(n, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        torch.cuda.synchronize()
        b.copy_(a)
        torch.cuda.synchronize()
        log("copied %d MiB" % args.calibrate_copy)
        return
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path (the build would "
              "shard by grid batch and all-reduce K); rerun with --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2303_14280_amd import snk

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        raise SystemExit("the trained screener weights are missing (%s)" % snk.SCREENER_WEIGHTS)
    stream = torch.cuda.Stream(device=dev)          # default priority
    torch.cuda.set_stream(stream)

    if args.delocalised:
        from paper_2303_14280_amd import synth
        if args.delocalised not in (4, 5):
            raise SystemExit("--delocalised takes 4 or 5")
        s = synth.make_system(args.delocalised, density="delocalised")
        P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
        mlp = snk.load_screener(device=0)
        r0, K0, _ = run_variant("config %d delocalised fp64" % args.delocalised, s, P, stream, mlp, 0, 0,
                                eps_basis=EPS_BASIS)
        ref = (K0, r0["ms_per_step"], r0["ex"])
        rl, _, _ = run_variant("config %d delocalised fp64+learned" % args.delocalised, s, P, stream, mlp, 2, 1,
                               ref=ref, eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED, eps_skip_energy=args.eps)
        rm, _, _ = run_variant("config %d delocalised mixed+learned" % args.delocalised, s, P, stream, mlp, 2, 1,
                               ref=ref, eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED, precision=snk.SNK_MIXED,
                               eps_skip_energy=args.eps, eps_lowprec_energy=args.eps)
        print(json.dumps({"workload": "config%d with a delocalised density: %d functions, %d grid points"
                                      % (args.delocalised, s.nbf, s.npts),
                          "fp64": r0, "fp64+learned": rl, "mixed+learned": rm}), flush=True)
        return
    if args.profile:
        from paper_2303_14280_amd import synth
        if args.profile == "dfj2":
            r = dfj_config2(args, stream)
            log("profile run: %.2f ms/step" % r["ms_per_step"])
            return
        if args.profile == "xc2":
            s = synth.make_system(2)
            P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
            ctx = make_ctx(s, stream, None)
            V = torch.empty_like(P)
            for _ in range(args.warmup):
                ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(args.steps):
                ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - t0) / args.steps
            exc, nel = ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE, scalars=True)
            ctx.close()
            log("profile run: %.2f ms/step (PBE potential of config 2: E_xc %.10f, N_el %.6f)" % (ms, exc, nel))
            return
        if args.profile == "deloc4":
            s = synth.make_system(4, density="delocalised")
            P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
            r, _, _ = run_variant("config 4 delocalised fp64+learned", s, P, stream, snk.load_screener(device=0),
                                  args.steps, args.warmup, eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED,
                                  eps_skip_energy=args.eps)
            log("profile run: %.1f ms/step, phases %s" % (r["ms_per_step"], r["phases_ms"]))
            return
        cfg = 5 if args.profile == "config5" else 2
        s = synth.make_system(cfg)
        P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
        mlp = snk.load_screener(device=0)
        if cfg == 5:
            r, _, _ = run_variant("config 5 mixed+learned", s, P, stream, mlp, args.steps, args.warmup,
                                  eps_basis=EPS_BASIS, screen=snk.SNK_SCREEN_LEARNED, precision=snk.SNK_MIXED,
                                  eps_skip_energy=args.eps, eps_lowprec_energy=args.eps)
        else:
            r, _, _ = run_variant("config 2 fp64", s, P, stream, mlp, args.steps, args.warmup)
        log("profile run: %.1f ms/step, phases %s" % (r["ms_per_step"], r["phases_ms"]))
        return
    h = headline(args, stream)
    s = h["system"]
    m = h["mixed+learned"]
    ms = m["ms_per_step"]
    ints = h["ints"]
    out = {
        "metric": METRIC,
        "value": ints / (ms * 1e-3),
        "unit": "shell-pair·gridpoints/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": "config5: %d-atom water-like cluster (333 waters + 1 O, 38 A box), %d Cartesian "
                               "s/p/d functions, 50x194 grid per atom = %d points in 256-point batches, "
                               "molecule-local density; mixed precision + learned screen, eps_basis %g"
                               % (len(s.atom_Z), s.nbf, s.npts, EPS_BASIS),
                   "atoms": int(len(s.atom_Z)), "nbf": s.nbf, "grid_points": s.npts,
                   "shell_pair_points": ints, "precision": "mixed", "screen": "learned",
                   "eps_skip_energy": args.eps, "eps_lowprec_energy": args.eps, "parallelism": "single GPU"},
        "roofline": dominant_kernel(h["stats"]),
        "speedup_vs_fp64": m["speedup_vs_fp64"],
        "speedup_vs_fp64_learned": m["speedup_vs_fp64_learned"],
        "dE_x_vs_fp64": m["dE_x_vs_fp64"],
        "max_dK_vs_fp64": m["max_dK_vs_fp64"],
        "ex": m["ex"],
        "config5": {"fp64": h["fp64"], "fp64+learned": h["fp64+learned"], "mixed+learned": m},
    }
    out["roofline"]["traffic_unit"] = "bytes per launch"
    log("value %.4g shell-pair·gridpoints/s at %.1f ms/step (x%.1f vs plain FP64, x%.2f vs FP64+learned); "
        "dominant kernel %s at %.1f%% of %.1f TFLOP/s" %
        (out["value"], ms, m["speedup_vs_fp64"], m["speedup_vs_fp64_learned"], out["roofline"]["kernel"],
         100 * out["roofline"]["frac"], out["roofline"]["peak"]))
    if not args.no_extras:
        out["config3"] = config3(args, stream)
        out["config2"] = config2(args, stream)
        out["dfj_config2"] = dfj_config2(args, stream)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(s, ints / s.npts)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
