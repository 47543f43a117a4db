"""sn-K exchange build benchmark on one MI355X.

A step is one full build K[P] (collocation, F GEMM, 3c-CP A.F digestion, K GEMM,
symmetrisation and E_x) for the 30-atom water cluster (config 2: 290 Cartesian
s/p/d functions, 75x302 grid per atom = 679,500 points, FP64, no screening) with
P and K resident in HBM.  Prints one JSON line.

    python bench.py [--gpus 1] [--steps 5] [--warmup 2] [--no-cpu-baseline] [--large 4,5]

The JSON line also carries the mixed-precision and learned-screen builds of the same
workload, a molecule-local density on the same geometry, the exchange-correlation potential
matrix (Slater, LDA, PBE) of the same density and grid, and (--large) the 500- and
1000-atom clusters with basis and density screening.
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


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(system, target_s: float = 20.0):
    """The CPU oracle timed on a bounded sample of the same workload (every k-th grid point)."""
    import numpy as np
    from oracle import oracle as O
    nthreads = int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or (os.cpu_count() or 1)
    npair = system.nshell * (system.nshell + 1) // 2
    probe = system.subset_points(np.arange(0, system.npts, max(1, system.npts // 64)))
    t = time.perf_counter()
    O.snk(probe, nthreads=nthreads)
    dt = max(time.perf_counter() - t, 1e-3)
    rate = npair * probe.npts / dt
    n = int(min(system.npts, max(probe.npts, rate * target_s / npair)))
    stride = max(1, system.npts // n)
    sample = system.subset_points(np.arange(0, system.npts, stride))
    t = time.perf_counter()
    O.snk(sample, nthreads=nthreads)
    dt = time.perf_counter() - t
    return {"value": npair * sample.npts / dt, "unit": "shell-pair·gridpoints/s", "cores": nthreads,
            "kind": "oracle",
            "sample": "every %d-th grid point of the same workload (%d of %d points, %d shell pairs), %.1f s"
                      % (stride, sample.npts, system.npts, npair, dt)}


def afg_source_sha() -> str:
    import hashlib
    d = os.path.join(ROOT, "paper_2303_14280_amd", "csrc")
    src = b"".join(open(os.path.join(d, f), "rb").read() for f in ("k_afg.hip", "os3c.h", "snk_internal.h"))
    return hashlib.sha256(src).hexdigest()[:16]


def measured_traffic(kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 summaries, or None when the
    kernel source has changed since the counters were taken."""
    import glob
    import re
    sha = afg_source_sha()
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        for line in open(path):
            m = re.match(r"traffic: kernel=(\S+) sha=(\w+) read_bytes=(\S+) write_bytes=(\S+)", line.strip())
            if m and m.group(1) == kernel and m.group(2) == sha:
                return float(m.group(3)) + float(m.group(4)), os.path.basename(path)
    return None, None


def time_builds(ctx, P, K, stream, steps, warmup):
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


def mixed_learned(s, P, K64, stream, args, ms64, ex64, ints):
    """The mixed-precision + learned-screen build of the same workload, timed the same way,
    with its errors against the FP64 build (max|dK|, dE_x) and its screen statistics."""
    import numpy as np
    import torch
    from paper_2303_14280_amd import snk
    res = {}
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        return {"error": "no trained screener weights"}
    mlp = snk.load_screener(device=0)
    K = torch.empty_like(P)
    D, R = snk.SNK_DEVICE_PTRS, snk.SNK_DEVICE_PTRS
    variants = [("mixed+learned", dict(precision=snk.SNK_MIXED, screen=snk.SNK_SCREEN_LEARNED, flags=R)),
                ("mixed+learned+fp32gemm", dict(precision=snk.SNK_MIXED, screen=snk.SNK_SCREEN_LEARNED,
                                                flags=D | snk.SNK_FP32_GEMM)),
                ("fp64+learned", dict(precision=snk.SNK_FP64, screen=snk.SNK_SCREEN_LEARNED, flags=R)),
                ("fp64, two groups overlapped", dict(precision=snk.SNK_FP64, screen=snk.SNK_SCREEN_NONE,
                                                     flags=R | snk.SNK_OVERLAP_GROUPS)),
                ("fp64 native GEMM", dict(precision=snk.SNK_FP64, screen=snk.SNK_SCREEN_NONE, flags=D)),
                ("fp32gemm", dict(precision=snk.SNK_MIXED, screen=snk.SNK_SCREEN_NONE, flags=D | snk.SNK_FP32_GEMM)),
                ("fp64+bound", dict(precision=snk.SNK_FP64, screen=snk.SNK_SCREEN_BOUND, flags=R)),
                ("fp64+link (paper, 1e-9)", dict(precision=snk.SNK_FP64, screen=snk.SNK_SCREEN_LINK, flags=R,
                                                 eps_skip_energy=1e-9))]
    for name, kw in variants:
        kw = dict(kw)
        eps_skip = kw.pop("eps_skip_energy", args.eps)
        ctx = snk.Context(s, stream=stream.cuda_stream, device=0, screener=mlp, eps_skip_energy=eps_skip,
                          eps_lowprec_energy=args.eps, **kw)
        steps = args.steps if name == "mixed+learned" else max(2, args.steps // 2)
        ms = time_builds(ctx, P, K, stream, steps, args.warmup)
        st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
        torch.cuda.synchronize()
        dK = float((K - K64).abs().max().item())
        evaluated = float(sum(st["pair_points"]))
        r = {"ms_per_step": ms, "speedup_vs_fp64": ms64 / ms, "dE_x_vs_fp64": st["ex"] - ex64,
             "max_dK_vs_fp64": dK, "skipped_pair_points_fraction": st["pair_points_skipped"] / max(1.0, ints),
             "fp32_pair_points_fraction": st["pair_points_lowprec"] / max(1.0, ints),
             "skipped_energy_estimate": st["skipped_bound"], "shell_pair_points_evaluated": evaluated,
             "effective_rate": ints / (ms * 1e-3),
             "phases_ms": {"collocate": st["t_collocate_ms"], "fgemm": st["t_fgemm_ms"],
                           "screen": st["t_screen_ms"], "afg": st["t_afg_ms"], "kgemm": st["t_kgemm_ms"],
                           "finish": st["t_finish_ms"]},
             "afg_class_ms": dict(zip(CLASSES, st["t_afg_class_ms"])),
             "afg_class_pair_points": dict(zip(CLASSES, st["pair_points"]))}
        log("%s: %.3f ms/step (x%.2f vs FP64), dE_x %.2e, max|dK| %.2e, skipped %.3f, FP32 %.3f" %
            (name, ms, ms64 / ms, r["dE_x_vs_fp64"], dK, r["skipped_pair_points_fraction"],
             r["fp32_pair_points_fraction"]))
        res[name] = r
        ctx.close()
    res["eps_skip_energy"] = args.eps
    res["eps_lowprec_energy"] = args.eps
    res["target"] = "|dE_x| <= 1e-6 Eh at >= 3x the FP64 build"
    return res


def xc_potential(s, P, stream, args, ms64):
    """The exchange-correlation potential matrix (Sec. II.C) of the same workload: Slater, LDA
    and PBE through snk_vxc_build (device pointers, F GEMM through rocBLAS), timed like the sn-K
    builds, with E_xc and the electron count; then K and the PBE V^xc of the same density in one
    call (snk_ctx_build_kxc, collocation and F shared) against the two builds apart."""
    import torch
    from paper_2303_14280_amd import snk
    ctx = snk.Context(s, flags=snk.SNK_DEVICE_PTRS, stream=stream.cuda_stream, device=0)
    V = torch.empty_like(P)
    res = {"grid_points": s.npts, "nbf": ctx.nbf,
           "gemm_flops": 4.0 * ctx.nbf * ctx.nbf * ctx.nbatches * 256}
    for name, fn in (("slater", snk.SNK_XC_SLATER), ("lda", snk.SNK_XC_LDA), ("pbe", snk.SNK_XC_PBE)):
        for i in range(args.warmup):
            ctx.vxc_device(P.data_ptr(), V.data_ptr(), fn)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for i in range(args.steps):
            ctx.vxc_device(P.data_ptr(), V.data_ptr(), fn)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = max(e0.elapsed_time(e1) / args.steps, 1000.0 * (time.perf_counter() - t0) / args.steps)
        exc, nel = ctx.vxc_device(P.data_ptr(), V.data_ptr(), fn, scalars=True)
        res[name] = {"ms_per_build": ms, "exc": exc, "nel": nel}
        log("XC %s: %.3f ms/build, E_xc %.10f, N_el %.8f" % (name, ms, exc, nel))
    # K and V^xc (PBE) of the same density in one call, sharing Phi and F
    K = torch.empty_like(P)
    for i in range(args.warmup):
        ctx.build_kxc_device(P.data_ptr(), K.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        ctx.build_kxc_device(P.data_ptr(), K.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = max(e0.elapsed_time(e1) / args.steps, 1000.0 * (time.perf_counter() - t0) / args.steps)
    res["k_and_pbe_one_pass"] = {"ms_per_build": ms, "separate_ms": ms64 + res["pbe"]["ms_per_build"]}
    log("K + V^xc (PBE) in one pass: %.3f ms/build (separately %.3f)" % (ms, ms64 + res["pbe"]["ms_per_build"]))
    ctx.close()
    return res


def local_density_comparison(s, stream, args):
    """The same geometry and grid with a molecule-local density (each water's five occupied
    orbitals on its own functions, P block-diagonal by molecule): FP64 build against the
    mixed + learned build, both timed like the headline build."""
    import torch
    from paper_2303_14280_amd import snk, synth
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        return {"error": "no trained screener weights"}
    sl = s.with_density(synth.make_density(s, s.n_occ, "local", [args.config, 2]))
    P = torch.tensor(sl.P, dtype=torch.float64, device="cuda")
    mlp = snk.load_screener(device=0)
    R = snk.SNK_DEVICE_PTRS
    res = {"density": "molecule-local (block-diagonal by molecule)"}
    K64 = torch.empty_like(P)
    ctx = snk.Context(sl, flags=R, stream=stream.cuda_stream, device=0)
    ms64 = time_builds(ctx, P, K64, stream, args.steps, args.warmup)
    st64 = ctx.build_device(P.data_ptr(), K64.data_ptr(), stats=True)
    ctx.close()
    res["fp64"] = {"ms_per_step": ms64, "ex": st64["ex"]}
    K = torch.empty_like(P)
    ctx = snk.Context(sl, flags=R, stream=stream.cuda_stream, device=0, screener=mlp, precision=snk.SNK_MIXED,
                      screen=snk.SNK_SCREEN_LEARNED, eps_skip_energy=args.eps, eps_lowprec_energy=args.eps)
    ms = time_builds(ctx, P, K, stream, args.steps, args.warmup)
    st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
    torch.cuda.synchronize()
    ctx.close()
    ints = float(sum(st["pair_points"]) + st["pair_points_skipped"])
    res["mixed+learned"] = {
        "ms_per_step": ms, "speedup_vs_fp64": ms64 / ms, "dE_x_vs_fp64": st["ex"] - st64["ex"],
        "max_dK_vs_fp64": float((K - K64).abs().max().item()),
        "skipped_pair_points_fraction": st["pair_points_skipped"] / max(1.0, ints),
        "fp32_pair_points_fraction": st["pair_points_lowprec"] / max(1.0, ints),
        "phases_ms": {"collocate": st["t_collocate_ms"], "fgemm": st["t_fgemm_ms"], "screen": st["t_screen_ms"],
                      "afg": st["t_afg_ms"], "kgemm": st["t_kgemm_ms"], "finish": st["t_finish_ms"]}}
    log("local density: FP64 %.3f ms, mixed+learned %.3f ms (x%.2f), dE_x %.2e" %
        (ms64, ms, ms64 / ms, res["mixed+learned"]["dE_x_vs_fp64"]))
    return res


def large_system(config, stream, args):
    """A large cluster with molecule-local density (500 or 1000 atoms), all builds with basis
    screening (eps_basis 1e-9): the plain FP64 build (no density screen; one timed build, the
    reference for E_x and K), FP64 with the rigorous density screen (5e-7 Eh), and the learned
    screen in FP64 and in the mixed build, each timed over `args.large_steps` builds after one
    warm-up; then the basis-screened PBE exchange-correlation potential of the same density."""
    import torch
    from paper_2303_14280_amd import snk, synth
    if not os.path.exists(snk.SCREENER_WEIGHTS):
        return {"error": "no trained screener weights"}
    t = time.perf_counter()
    s = synth.make_system(config)
    log("config %d generated in %.1f s" % (config, time.perf_counter() - t))
    P = torch.tensor(s.P, dtype=torch.float64, device="cuda")
    mlp = snk.load_screener(device=0)
    R = snk.SNK_DEVICE_PTRS
    res = {"workload": "config%d: %d atoms, %d functions, %d grid points, %s density"
                       % (config, len(s.atom_Z), s.nbf, s.npts, s.density)}
    variants = [("fp64", dict(screen=snk.SNK_SCREEN_NONE)),
                ("fp64+bound", dict(screen=snk.SNK_SCREEN_BOUND, eps_skip_energy=5e-7)),
                ("fp64+link (paper, 1e-9)", dict(screen=snk.SNK_SCREEN_LINK, eps_skip_energy=1e-9)),
                ("fp64+learned", dict(screen=snk.SNK_SCREEN_LEARNED, eps_skip_energy=args.eps)),
                ("mixed+learned", dict(screen=snk.SNK_SCREEN_LEARNED, precision=snk.SNK_MIXED,
                                       eps_skip_energy=args.eps, eps_lowprec_energy=args.eps))]
    K0 = None
    for name, kw in variants:
        t = time.perf_counter()
        ctx = snk.Context(s, flags=R, stream=stream.cuda_stream, device=0, screener=mlp, eps_basis=1e-9, **kw)
        t_create = time.perf_counter() - t
        K = torch.empty_like(P)
        if name == "fp64":
            # one build (tens of seconds), timed on the host clock around the synchronous call
            torch.cuda.synchronize()
            t = time.perf_counter()
            st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
            torch.cuda.synchronize()
            ms = 1000.0 * (time.perf_counter() - t)
        else:
            ms = time_builds(ctx, P, K, stream, args.large_steps, 1)
            st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
            torch.cuda.synchronize()
        ctx.close()
        ints = float(sum(st["pair_points"]) + st["pair_points_skipped"])
        r = {"ms_per_step": ms, "create_s": t_create, "ex": st["ex"],
             "skipped_pair_points_fraction": st["pair_points_skipped"] / max(1.0, ints),
             "fp32_pair_points_fraction": st["pair_points_lowprec"] / max(1.0, ints),
             "skipped_energy_estimate": st["skipped_bound"], "effective_rate": ints / (ms * 1e-3),
             "tile_functions": st["tile_functions"], "tile_f_rows": st["tile_frows"], "tile_g_rows": st["tile_grows"],
             "phases_ms": {"collocate": st["t_collocate_ms"], "fgemm": st["t_fgemm_ms"], "screen": st["t_screen_ms"],
                           "afg": st["t_afg_ms"], "kgemm": st["t_kgemm_ms"], "finish": st["t_finish_ms"]}}
        if K0 is None:
            K0, ms0, ex0 = K, ms, st["ex"]
            r["shell_pair_points"] = ints
        else:
            r["speedup_vs_fp64"] = ms0 / ms
            r["dE_x_vs_fp64"] = st["ex"] - ex0
            r["max_dK_vs_fp64"] = float((K - K0).abs().max().item())
            if name != "fp64+bound":
                r["speedup_vs_fp64_bound"] = res["fp64+bound"]["ms_per_step"] / ms
        log("config %d %s: %.1f ms/step, E_x %.10f" % (config, name, ms, st["ex"]))
        res[name] = r
    if not args.no_xc:
        # the XC potential of the same density over the same tiles (basis-screened, PBE)
        ctx = snk.Context(s, flags=R, stream=stream.cuda_stream, device=0, eps_basis=1e-9)
        V = torch.empty_like(P)
        ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
        torch.cuda.synchronize()
        t = time.perf_counter()
        for i in range(args.large_steps):
            ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE)
        torch.cuda.synchronize()
        ms = 1000.0 * (time.perf_counter() - t) / args.large_steps
        exc, nel = ctx.vxc_device(P.data_ptr(), V.data_ptr(), snk.SNK_XC_PBE, scalars=True)
        ctx.close()
        res["xc_pbe"] = {"ms_per_build": ms, "exc": exc, "nel": nel}
        log("config %d XC PBE: %.1f ms/build, E_xc %.10f, N_el %.6f" % (config, ms, exc, nel))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision + learned-screen comparison")
    ap.add_argument("--no-xc", action="store_true", help="skip the exchange-correlation potential timings")
    ap.add_argument("--eps", type=float, default=5e-6,
                    help="estimate budget (Eh) of the learned screen's skipped blocks and of the FP32 blocks")
    ap.add_argument("--large", default="4,5",
                    help="comma-separated large configurations (4: 500 atoms, 5: 1000 atoms) to time with basis "
                         "and density screening, or 'none'")
    ap.add_argument("--large-steps", type=int, default=3)
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

    import numpy as np
    import torch
    from paper_2303_14280_amd import flops, snk, synth

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    log("generating config %d" % args.config)
    s = synth.make_system(args.config)
    stream = torch.cuda.Stream(device=dev)          # default priority
    torch.cuda.set_stream(stream)
    # FP64 reference build: the library's A.F kernels, the dense GEMMs through rocBLAS dgemm
    ctx = snk.Context(s, flags=snk.SNK_DEVICE_PTRS, stream=stream.cuda_stream, device=0)
    P = torch.tensor(s.P, dtype=torch.float64, device=dev)
    K = torch.empty_like(P)
    torch.cuda.synchronize()
    log("nbf %d npts %d batches %d" % (ctx.nbf, s.npts, ctx.nbatches))

    for i in range(args.warmup):
        ctx.build_device(P.data_ptr(), K.data_ptr())
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for i in range(args.steps):
        ctx.build_device(P.data_ptr(), K.data_ptr())
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_gpu = e0.elapsed_time(e1) / args.steps
    ms_wall = 1000.0 * wall / args.steps
    ms = max(ms_gpu, ms_wall)
    log("timed %d steps: %.3f ms/step (events %.3f, wall %.3f)" % (args.steps, ms, ms_gpu, ms_wall))

    # per-phase and per-kernel times from the library's HIP events (separate, untimed builds)
    reps = 3
    acc = None
    for i in range(reps):
        st = ctx.build_device(P.data_ptr(), K.data_ptr(), stats=True)
        if acc is None:
            acc = {k: (np.array(v, float) if isinstance(v, list) else float(v)) for k, v in st.items()}
        else:
            for k, v in st.items():
                acc[k] = acc[k] + (np.array(v, float) if isinstance(v, list) else float(v))
    st = {k: v / reps for k, v in acc.items()}
    pair_points = np.array(st["pair_points"])
    prim_points = np.array(st["prim_pair_points"])
    t_cls = np.array(st["t_afg_class_ms"])
    ints = float(pair_points.sum())
    cls_flops = [flops.class_flops(c, pair_points[c], prim_points[c]) for c in range(6)]
    dom = int(np.argmax(t_cls))
    # each batch group launches every class once; the per-launch figures are averages over them
    launches = max(1, int(round(st["n_groups"])))
    launch_ms = float(t_cls[dom]) / launches
    launch_flops = cls_flops[dom] / launches
    achieved = launch_flops / (launch_ms * 1e-3) / 1e12
    dom_name = "afg_kernel<%d,%d>" % flops.CLASS_L[dom]
    traffic, traffic_src = measured_traffic(dom_name)
    afg_total = sum(cls_flops) / (st["t_afg_ms"] * 1e-3) / 1e12

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
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "config%d: %d-atom water-like cluster, %d Cartesian s/p/d functions, "
                               "%d grid points in %d batches of 256, FP64 (dense GEMMs via rocBLAS), no screening"
                               % (args.config, len(s.atom_Z), ctx.nbf, s.npts, ctx.nbatches),
                   "atoms": int(len(s.atom_Z)), "nbf": ctx.nbf, "grid_points": s.npts,
                   "shell_pair_points": ints, "precision": "fp64", "screen": "none",
                   "parallelism": "single GPU"},
        "roofline": {"bound": "alu", "kernel": "afg_kernel<%d,%d> (%s)" % (flops.CLASS_L[dom] + (CLASSES[dom],)),
                     "achieved": achieved, "peak": flops.PEAK_FP64_VALU_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / flops.PEAK_FP64_VALU_TFLOPS, "traffic": traffic,
                     "traffic_unit": "bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
                     "traffic_source": traffic_src,
                     "launch_ms": launch_ms, "algorithmic_flops": launch_flops, "launches_per_build": launches},
        "phases_ms": {"collocate": st["t_collocate_ms"], "fgemm": st["t_fgemm_ms"], "afg": st["t_afg_ms"],
                      "kgemm": st["t_kgemm_ms"], "finish": st["t_finish_ms"]},
        "afg_classes": {CLASSES[c]: {"ms": float(t_cls[c]), "pair_points": float(pair_points[c]),
                                     "tflops": (cls_flops[c] / (t_cls[c] * 1e-3) / 1e12) if t_cls[c] > 0 else 0.0}
                        for c in range(6)},
        "afg_tflops_all_classes": afg_total,
        "ex": st["ex"],
    }
    if not args.no_mixed:
        out["mixed_learned"] = mixed_learned(s, P, K, stream, args, ms, st["ex"], ints)
        out["local_density"] = local_density_comparison(s, stream, args)
    if not args.no_xc:
        out["xc_potential"] = xc_potential(s, P, stream, args, ms)
    if args.large and args.large != "none":
        out["large_systems"] = {}
        for c in args.large.split(","):
            out["large_systems"]["config%d" % int(c)] = large_system(int(c), stream, args)
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        out["cpu_baseline"] = cpu_baseline(s)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
