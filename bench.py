"""Benchmark of the layered multiple-scattering operator on one MI355X.

A step is one application of the whole operator y = x - S (T_free + T_refl) x
(free-space Graf translations: near-field sums and FMM; Sommerfeld aggregate
-> reflection -> disaggregate; S-matrix combine) to one synthetic coefficient
vector of the 20000-particle cloud ([0,600] x [1,150], one third each circles,
ellipses and five-arm stars with GPU-generated S-matrices, p = 15, omega = 8).
value = FP64 operator applies per second with the inputs resident in HBM; the
same line carries the mixed form (FP32 contractions) on the same input and
its error against FP64, preconditioned GMRES on this cloud within an
iteration budget (the time to 1e-9 is reported only when reached), GMRES to
1e-9 on the 2000-particle cloud for both forms, and the oracle timed on the
host (measured on the 16-particle workload, extrapolated to 20000).

Prints one JSON line (rank 0, N = 1 only).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

PEAK_FP64 = 78.6e12      # MI355X FP64 vector and FP64 MFMA, FLOP/s
PEAK_FP32 = 157.3e12
PEAK_HBM = 8.0e12


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c2", choices=["c0", "c1", "c2", "c3", "c4"],
                    help="c2: the headline single-vector apply; c3: 64-RHS block applies at "
                         "three frequencies; c4: misfit + gradient at 5000 particles")
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"])
    ap.add_argument("--solve-its", type=int, default=None,
                    help="GMRES iteration budget on the timed cloud (default 200, 0 switches "
                         "the solve off; 300 for the gradient workload)")
    ap.add_argument("--nrhs", type=int, default=64, help="block size of the c3 measurement")
    ap.add_argument("--block-its", type=int, default=40,
                    help="c3: block GMRES steps per frequency (preconditioned, to 1e-9; 0 skips)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-shapes", action="store_true",
                    help="circles with closed-form S instead of the mixed-shape cloud")
    ap.add_argument("--no-c1-solve", action="store_true",
                    help="skip the 2000-particle GMRES solves to 1e-9")
    ap.add_argument("--c1-its", type=int, default=10000,
                    help="iteration budget of the 2000-particle solves")
    ap.add_argument("--cpu-rows", type=int, default=2)
    ap.add_argument("--fmm-leaf", type=int, default=0, help="particles per FMM leaf (0 = library default)")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device copy of this many bytes (counter calibration)")
    return ap.parse_args()


def workload(name):
    import workloads as W
    if name == "c0":
        return W.c0_circles()
    if name == "c1":
        return W.c1_cloud()
    return W.c2_cloud()


def section8d_flops(kernel, w, info):
    """Algorithmic flops of one launch by the scope table's per-unit figures
    (complex multiply-add = 8): a cross-check of the library's own count."""
    import numpy as np
    if kernel in ("somm_aggregate", "somm_disaggregate"):
        # one complex MAC per (node, coefficient), over the fraction of
        # (node, particle) pairs the depth truncation keeps
        return 8.0 * info["q"] * float(w.n_coeff) * info["somm_kept"]
    if kernel == "combine_s_apply":
        return 8.0 * float(np.sum((4 * w.p.astype(np.int64) + 2) ** 2))
    return None


def kernel_unit(kernel, mixed):
    """(bound, peak FLOP/s) of the unit a kernel runs on."""
    if kernel in ("somm_aggregate", "somm_disaggregate"):
        return "mfma", (PEAK_FP32 if mixed else PEAK_FP64)      # 16x16x4 MFMA
    if kernel.startswith("graf") and mixed:
        return "alu", PEAK_FP32
    return "alu", PEAK_FP64


def source_hash(*names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_2608_26875_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


KERNEL_SRC = {"graf_direct": ("graf.hip",), "somm_aggregate": ("somm.hip",),
              "somm_disaggregate": ("somm.hip",), "combine_s_apply": ("linalg.hip",)}


def traffic_from_profiles(kernel, workload_name, mixed=False):
    """HBM bytes per launch from the committed rocprofv3 counter summary, or
    None when there is none or the kernel source changed since it was taken."""
    suffix = "_mixed" if mixed else ""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload_name}{suffix}_pmc.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("source_hash") != source_hash(*KERNEL_SRC.get(kernel, ())):
        return None
    return d.get("hbm_bytes_per_launch")


def _cpu_time():
    t = os.times()
    return t.user + t.system


def _oracle_apply_full(w, x):
    """One full apply of the oracle (dense Graf + adaptive Sommerfeld)."""
    from oracle import media, operator, smatrix
    m = media.Media.from_workload(w)
    S = smatrix.workload_blocks(w, m)
    return operator.apply(w, m, S, x, tol=1e-13)


def cpu_baseline(w, rows, n_eval=4):
    """The CPU oracle as it stands, timed on this host in the same run.

    Measured: full oracle applies of the 16-particle workload (median of 3).
    The 20000-particle apply is extrapolated from a bounded sample (the oracle
    would need hours): the dense Graf sum for ``rows`` targets (all sources)
    scaled by n / rows (the sum is row-separable), plus ``n_eval``
    evaluations of the oracle's full-apply Sommerfeld integrand scaled by the
    number of evaluations its adaptive quadrature used on this cloud (stored
    by tests/golden/make_goldens.py).  cores = CPU seconds / wall seconds of
    the timed oracle work (the oracle is numpy: Python loops plus BLAS)."""
    import numpy as np
    import workloads as W
    from oracle import graf, interface, media, smatrix, sommerfeld
    w0 = W.c0_circles()
    x0 = W.random_coeffs(w0.n_coeff, 1000)[0]
    c0_t = []
    cpu0, wall0 = _cpu_time(), time.perf_counter()
    for _ in range(3):
        t0 = time.perf_counter()
        _oracle_apply_full(w0, x0)
        c0_t.append(time.perf_counter() - t0)
    c0_cores = (_cpu_time() - cpu0) / (time.perf_counter() - wall0)
    c0_med = sorted(c0_t)[1]
    m = media.Media.from_workload(w)
    x = W.random_coeffs(w.n_coeff, 1002)[0]
    tg = list(np.linspace(0, w.n - 1, rows).astype(int))
    cpu1, wall1 = _cpu_time(), time.perf_counter()
    t0 = time.perf_counter()
    graf.apply_free(w, m, x, targets=tg)
    t_free = (time.perf_counter() - t0) * w.n / rows
    # one S block of the right size stands for every particle: the timing
    # depends only on the amount of arithmetic, not on the values
    S0 = smatrix.disk(m, float(w.radius[0]), int(w.p[0]), int(w.bc[0]))
    Sb = [S0] * w.n
    f, _, _ = sommerfeld._integrand_factory(w, m, x, list(range(w.n)), Sb,
                                            lambda xi, sv: interface.reflection(xi, m, sv))
    xis = np.linspace(-20.0, 20.0, n_eval) + 0.0123
    t0 = time.perf_counter()
    for xi in xis:
        f(float(xi))
    t_eval = (time.perf_counter() - t0) / n_eval
    c2_cores = (_cpu_time() - cpu1) / (time.perf_counter() - wall1)
    g = os.path.join(ROOT, "tests", "golden", "c2_sampled.npz")
    neval = int(np.load(g)["refl_neval"]) if os.path.exists(g) else None
    out = {"value": None, "unit": "applies/s", "kind": "oracle",
           "cores": round(max(c0_cores, c2_cores), 1),
           "measured_c0": {"workload": "16 rigid circles, p=10 (full apply, median of 3)",
                           "seconds_per_apply": c0_med, "applies_per_s": 1.0 / c0_med,
                           "runs_s": c0_t, "cores": round(c0_cores, 2)}}
    if neval is None:
        out["sample"] = "no stored evaluation count for the 20000-particle cloud"
        return out
    t_full = t_free + neval * t_eval
    out.update({"value": 1.0 / t_full, "extrapolated": True, "seconds_per_apply": t_full,
                "sample": f"20000 particles: dense Graf rows of {rows} of {w.n} targets "
                          f"({t_free * rows / w.n:.1f} s, x{w.n / rows:.0f}); reflected part: "
                          f"{n_eval} full-apply integrand evaluations ({t_eval:.2f} s each) x "
                          f"{neval} evaluations of the oracle's adaptive rule at tol 1e-12"})
    return out


def copy_calibration(nbytes):
    """A plain device copy of nbytes (reference for the HBM byte counters)."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    torch.cuda.synchronize()
    b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes}), flush=True)


def bench_c3(args):
    """Block applies of 64 right-hand sides (the 64 incident directions) at the
    three frequencies of the uneven-order cloud; tile shapes autotuned."""
    import numpy as np
    import torch
    import paper_2608_26875_amd as E
    import workloads as W
    mixed = args.precision == "mixed"
    flags = E.EMS_APPLY_ALL | (E.EMS_MIXED if mixed else 0)
    per = []
    tot_ms = 0.0
    for f in range(3):
        w = W.c3_cloud(f)
        op = E.Operator(w.xy, w.radius, w.p, E.make_media(w.host, w.substrate, w.omega), bc=w.bc)
        info = op.build()
        tune = op.autotune(args.nrhs)
        x = op.incident(w.incidence[:args.nrhs])
        y = torch.empty_like(x)
        for _ in range(args.warmup):
            op.apply(x, y, flags=flags)
        torch.cuda.synchronize()
        op.profile(True)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(args.steps):
            op.apply(x, y, flags=flags)
        e1.record()
        torch.cuda.synchronize()
        op.profile(False)
        ms = e0.elapsed_time(e1) / args.steps
        kt = op.profile_read()
        tot_ms += ms
        per.append({"omega": w.omega, "p_range": [int(w.p.min()), int(w.p.max())],
                    "n_coeff": int(w.n_coeff), "q_nodes": info["q"], "ms_per_block_apply": ms,
                    "tiles": tune,
                    "kernels": {k: {"avg_ms": v[1] / v[0],
                                    "tflops": (v[2] / (v[1] * 1e-3) / 1e12) if v[2] else None}
                                for k, v in kt.items()}})
        if args.block_its > 0 and not mixed:
            # block GMRES over the 64 right-hand sides (one Krylov space),
            # cluster preconditioner; the time counts only when 1e-9 is reached
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _, si = op.solve(x, tol=1e-9, restart=0, maxit=args.block_its, precond=1, block=True)
            torch.cuda.synchronize()
            per[-1]["block_gmres"] = dict(si, wall_s=time.perf_counter() - t0,
                                          solve_s=si["seconds"] if si["converged"] else None)
        print(json.dumps({"c3_frequency": f, **per[-1]}), file=sys.stderr, flush=True)
        del op
        torch.cuda.empty_cache()
    nrhs = args.nrhs
    out = {"metric": "block applies/s (64 RHS, 3 frequencies), 20000 particles, uneven p",
           "value": 3.0 * 1e3 / tot_ms, "unit": "block applies/s", "n_gpus": 1,
           "steps": args.steps, "warmup": args.warmup, "ms_per_step": tot_ms / 3.0,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "c64+c128" if mixed else "c128", "data": "synthetic",
           "config": {"workload": f"c3: 20000 particles, p_i = ceil(ks a_i) + 8, {nrhs} RHS x "
                                  f"omega 2/4/8, {'mixed' if mixed else 'FP64'} block apply",
                      "parallelism": "single GPU"},
           "rhs_applies_per_s": 3.0 * nrhs * 1e3 / tot_ms, "per_frequency": per,
           "block_gmres_solve_s": (sum(p["block_gmres"]["solve_s"] for p in per)
                                   if all(p.get("block_gmres", {}).get("solve_s") for p in per)
                                   else None)}
    print(json.dumps(out), flush=True)


def bench_c4(args):
    """Misfit and gradient (centres + substrate Lame parameters) at 5000
    particles, 32 P waves, 1024 receivers: forward solves, field, adjoint
    right-hand side, adjoint solves, vector-Jacobian product."""
    import numpy as np
    import torch
    import paper_2608_26875_amd as E
    import workloads as W
    w = W.c4_cloud()
    pts = W.c4_receivers()
    waves = w.incidence
    its = args.solve_its or 300
    # observed data from the true configuration
    op = E.Operator(w.xy, w.radius, w.p, E.make_media(w.host, w.substrate, w.omega), bc=w.bc)
    op.build()
    b = op.incident(waves)
    g, i0 = op.solve(b, tol=1e-9, restart=0, maxit=its, precond=1)
    u_obs = op.scattered_field(g, pts)
    torch.cuda.synchronize()
    del op
    ws, sub = W.c4_start(w)
    op = E.Operator(ws.xy, ws.radius, ws.p, E.make_media(ws.host, sub, ws.omega), bc=ws.bc)
    t0 = time.perf_counter()
    op.build()
    t_build = time.perf_counter() - t0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    try:
        J, gxy, gl, info = op.misfit_gradient(waves, pts, u_obs, tol=1e-9, restart=0, maxit=its,
                                              precision=1 if args.precision == "mixed" else 0,
                                              precond=1)
    except E.NotConvergedError as exc:
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        print(json.dumps({"metric": "misfit + gradient seconds, 5000 particles, 32 P waves, "
                                    "1024 receivers", "value": None, "unit": "s",
                          "not_converged": str(exc), "solve": exc.info, "wall_s": secs,
                          "true_data_solve": i0}), flush=True)
        return
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    out = {"metric": "misfit + gradient seconds, 5000 particles, 32 P waves, 1024 receivers",
           "value": secs, "unit": "s", "n_gpus": 1, "steps": 1, "warmup": 0, "ms_per_step": secs * 1e3,
           "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
           "dtype": "c128" if args.precision == "fp64" else "c64+c128", "data": "synthetic",
           "config": {"workload": "c4: 5000 particles, p=15, omega=8, gradient w.r.t. 10000 centre "
                                  "coordinates + substrate lambda, mu", "parallelism": "single GPU",
                      "gmres_budget": its},
           "J": J, "grad_norm_centres": float(np.linalg.norm(gxy)), "grad_lame": list(gl),
           "true_data_solve": i0, "solves": info, "build_s": t_build}
    print(json.dumps(out), flush=True)


def shapes_operator(w, with_time=False):
    """Operator of a mixed-shape cloud (one third each circles, ellipses and
    five-arm stars) with S-matrices generated on the GPU; the wall clock of
    the generation (after an untimed call on 64 particles) when asked."""
    import numpy as np
    import torch
    import paper_2608_26875_amd as E
    media = E.make_media(w.host, w.substrate, w.omega)
    gen = None
    if with_time:
        n0 = 64
        small = E.Operator(w.xy[:n0], w.radius[:n0], w.p[:n0], media, bc=w.bc[:n0])
        small.shape_smatrices(w.shape[:n0], w.a[:n0], w.theta0[:n0], w.bc[:n0])
        del small
    op = E.Operator(w.xy, w.radius, w.p, media, bc=w.bc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = op.shape_smatrices(w.shape, w.a, w.theta0, w.bc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    if with_time:
        gen = {"ms": ms, "us_per_particle": ms * 1e3 / w.n, "particles": int(w.n),
               "kinds": np.bincount(w.shape, minlength=3).tolist(), "npts": 256,
               "p": int(w.p.max())}
    op.set_smatrices_packed(S)
    del S
    return op, gen


def time_applies(op, x, y, flags, steps, warmup):
    """(ms per apply, per-kernel table) over `steps` applies after `warmup`."""
    import torch
    for _ in range(warmup):
        op.apply(x, y, flags=flags)
    torch.cuda.synchronize()
    op.profile(True)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(steps):
        op.apply(x, y, flags=flags)
    e1.record(st)
    torch.cuda.synchronize()
    op.profile(False)
    return e0.elapsed_time(e1) / steps, op.profile_read()


def kernel_table(kt, mixed):
    per_kernel = {}
    for k, (nl, tot_ms, fl) in kt.items():
        bound, peak = kernel_unit(k, mixed)
        d = {"launches": nl, "avg_ms": tot_ms / max(nl, 1)}
        if fl > 0:
            d["flops_per_launch"] = fl / nl
            d["tflops"] = fl / (tot_ms * 1e-3) / 1e12
            d["frac_of_peak"] = d["tflops"] * 1e12 / peak
        per_kernel[k] = d
    return per_kernel


def roofline_of(kt, kernel, w, info, mixed, workload_name):
    nl, tot_ms, fl = kt[kernel]
    avg_s = tot_ms / nl / 1e3
    fl_launch = fl / nl
    check = section8d_flops(kernel, w, info)
    if check is not None and abs(check - fl_launch) > 1e-9 * check:
        raise SystemExit(f"flop count mismatch for {kernel}: library {fl_launch} vs {check}")
    bound, peak = kernel_unit(kernel, mixed)
    return {"bound": bound, "achieved": fl_launch / avg_s / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": fl_launch / avg_s / peak,
            "traffic": traffic_from_profiles(kernel, workload_name, mixed),
            "kernel": kernel, "flops_per_launch": fl_launch, "avg_ms": avg_s * 1e3}


def solve_run(op, b, maxit, precision, precond, tol=1e-9):
    """GMRES to tol within maxit; the time counts only when it gets there."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, si = op.solve(b, tol=tol, restart=0, maxit=maxit, precision=precision, precond=precond)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    out = dict(si)
    out["wall_s"] = wall
    out["solve_s"] = si["seconds"] if si["converged"] else None
    out["s_per_iteration"] = si["seconds"] / max(si["iters"], 1)
    return out


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "decomposition is described, not built", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if args.copy_bytes:
        copy_calibration(args.copy_bytes)
        return
    import paper_2608_26875_amd as E
    import workloads as W

    torch.cuda.set_device(0)
    if args.workload == "c3":
        return bench_c3(args)
    if args.workload == "c4":
        return bench_c4(args)
    shapes = args.workload in ("c1", "c2") and not args.no_shapes
    w = {"c0": W.c0_circles, "c1": lambda: W.c1_cloud(shapes=shapes),
         "c2": lambda: W.c2_cloud(shapes=shapes)}[args.workload]()
    t0 = time.perf_counter()
    if shapes:
        op, gen = shapes_operator(w, with_time=(args.workload == "c2"))
    else:
        op = E.Operator(w.xy, w.radius, w.p, E.make_media(w.host, w.substrate, w.omega), bc=w.bc)
        gen = None
    if args.fmm_leaf:
        op.set_fmm(mode=0, leaf=args.fmm_leaf)
    info = op.build()
    tiles = op.autotune(1)
    setup_s = time.perf_counter() - t0
    x = torch.from_numpy(W.random_coeffs(w.n_coeff, 1002)).cuda()
    y = torch.empty_like(x)
    y32 = torch.empty_like(x)
    print(json.dumps({"step": "built", "workload": w.name, "setup_s": setup_s}), file=sys.stderr,
          flush=True)
    # FP64 form: the headline value
    ms, kt = time_applies(op, x, y, E.EMS_APPLY_ALL, args.steps, args.warmup)
    dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
    roof = roofline_of(kt, dom, w, info, False, w.name)
    # mixed form on the same input
    ms32, kt32 = time_applies(op, x, y32, E.EMS_APPLY_ALL | E.EMS_MIXED, args.steps, args.warmup)
    z64 = x - y
    z32 = x - y32
    err_y = float(torch.linalg.norm(y32 - y) / torch.linalg.norm(y))
    err_z = float(torch.linalg.norm(z32 - z64) / torch.linalg.norm(z64))
    somm32 = "somm_aggregate" if "somm_aggregate" in kt32 else max(kt32.items(), key=lambda kv: kv[1][1])[0]
    print(json.dumps({"step": "applies", "fp64_ms": ms, "mixed_ms": ms32}), file=sys.stderr,
          flush=True)
    shape_txt = "1/3 circles, ellipses, stars (GPU-generated S)" if shapes else "circles"
    out = {
        "metric": "operator applies/s & GMRES solve s at N=20k 2D, FP64 vs mixed @1e-9",
        "value": 1e3 / ms, "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128", "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} particles ({shape_txt}), p={int(w.p.max())}, "
                               f"omega={w.omega}, FP64 apply",
                   "n_coeff": int(w.n_coeff), "q_nodes": info["q"], "somm_kept": info["somm_kept"],
                   "pairs_direct": info["n_pairs"], "parallelism": "single GPU"},
        "roofline": roof,
        "mixed": {"applies_per_s": 1e3 / ms32, "ms_per_step": ms32, "dtype": "c64+c128",
                  "rel_err_vs_fp64_y": err_y, "rel_err_vs_fp64_z": err_z,
                  "roofline": roofline_of(kt32, somm32, w, info, True, w.name),
                  "kernels": kernel_table(kt32, True)},
        "kernels": kernel_table(kt, False),
        "setup_s": setup_s,
        "tiles": tiles,
    }
    if gen is not None:
        out["smatrix_shapes"] = gen
    # right-hand-side builders (once each after one untimed call): the plane
    # wave from the particle side, one sent from the substrate, and a point
    # source in the substrate over the middle of the cloud with the
    # polarisation (cos pi/4, sin pi/4); wall clock, each call synchronizes
    src = [(float(np.mean(w.xy[:, 0])), 3.0, math.cos(math.pi / 4), math.sin(math.pi / 4))]
    rhs_ms = {}
    for name, fn in (("plane_wave_particle_side", lambda: op.incident([w.incidence[0]])),
                     ("plane_wave_from_substrate", lambda: op.incident([(3, 0.3)])),
                     ("point_source", lambda: op.incident_point(src))):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fn()
        torch.cuda.synchronize()
        rhs_ms[name] = (time.perf_counter() - t0) * 1e3
    out["rhs_ms"] = rhs_ms
    solve_its = 200 if args.solve_its is None else args.solve_its
    if solve_its:
        # GMRES to 1e-9 on this cloud within an iteration budget, both forms,
        # cluster block-Jacobi preconditioner; gmres_solve_s exists only when
        # the budget reached 1e-9
        b = op.incident([w.incidence[0]])
        g = {"budget_iterations": solve_its, "tol": 1e-9}
        for name, prec in (("fp64", 0), ("mixed", 1)):
            g[name] = solve_run(op, b, solve_its, prec, 1)
            print(json.dumps({"step": f"gmres {w.name} {name}", **g[name]}), file=sys.stderr,
                  flush=True)
        out["gmres"] = g
        out["gmres_solve_s"] = {"fp64": g["fp64"]["solve_s"], "mixed": g["mixed"]["solve_s"]}
    del op, x, y, y32
    torch.cuda.empty_cache()
    if args.workload == "c2" and not args.no_c1_solve:
        # the 2000-particle cloud: GMRES to 1e-9, both forms, preconditioned
        w1 = W.c1_cloud(shapes=shapes)
        op1 = shapes_operator(w1)[0] if shapes else E.Operator(
            w1.xy, w1.radius, w1.p, E.make_media(w1.host, w1.substrate, w1.omega), bc=w1.bc)
        op1.build()
        op1.autotune(1)
        op1.set_progress(lambda it, rr: print(json.dumps({"c1_gmres_it": it, "relres": rr}),
                                              file=sys.stderr, flush=True), 1000)
        b1 = op1.incident([w1.incidence[0]])
        c1 = {"workload": f"c1: {w1.n} particles ({shape_txt}), p=15, omega=8", "tol": 1e-9}
        for name, prec in (("fp64", 0), ("mixed", 1)):
            c1[name] = solve_run(op1, b1, args.c1_its, prec, 1)
            print(json.dumps({"step": f"gmres c1 {name}", **c1[name]}), file=sys.stderr, flush=True)
        out["gmres_c1"] = c1
        del op1
        torch.cuda.empty_cache()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w if args.workload == "c2" else W.c2_cloud(), args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
