"""Benchmark of the layered multiple-scattering operator on one MI355X.

A step is one application of the whole operator y = x - S (T_free + T_refl) x
(free-space Graf translations, Sommerfeld aggregate -> reflection ->
disaggregate, S-matrix combine) to one synthetic coefficient vector of the
20000-particle cloud ([0,600] x [1,150], p = 15, omega = 8, complex128).
value = operator applies per second with the inputs resident in HBM.  With
--solve the GMRES time to a relative residual of 1e-9 is added.

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
    ap.add_argument("--solve", action="store_true", help="also time a GMRES solve to 1e-9")
    ap.add_argument("--solve-its", type=int, default=None,
                    help="GMRES iteration budget (default: 60 for the apply workload, "
                         "0 switches the solve off; 300 for the gradient workload)")
    ap.add_argument("--nrhs", type=int, default=64, help="block size of the c3 measurement")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-shapes", action="store_true",
                    help="skip timing the S-matrix generation of the shapes cloud")
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


def cpu_baseline(w, rows, n_eval=4):
    """Time the CPU oracle (as it is) on a bounded sample and scale to one apply.

    Free part: the dense Graf sum for ``rows`` target particles (all sources),
    scaled by n / rows (the sum is row-separable).  Reflected part: ``n_eval``
    evaluations of the oracle's Sommerfeld integrand for the full apply (all
    sources aggregated, all targets disaggregated and multiplied by S), scaled
    by the number of integrand evaluations the oracle's adaptive quadrature
    used on this cloud (stored by tests/golden/make_goldens.py)."""
    import numpy as np
    import workloads as W
    from oracle import graf, interface, media, smatrix, sommerfeld
    m = media.Media.from_workload(w)
    x = W.random_coeffs(w.n_coeff, 1002)[0]
    tg = list(np.linspace(0, w.n - 1, rows).astype(int))
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
    g = os.path.join(ROOT, "tests", "golden", f"{w.name}_sampled.npz")
    neval = None
    if os.path.exists(g):
        d = np.load(g)
        if "refl_neval" in d:
            neval = int(d["refl_neval"])
    if neval is None:
        return {"value": None, "unit": "applies/s", "cores": os.cpu_count(), "kind": "oracle",
                "sample": "no stored evaluation count for this cloud"}
    t_full = t_free + neval * t_eval
    import threadpoolctl
    cores = max((i.get("num_threads", 1) for i in threadpoolctl.threadpool_info()), default=1)
    return {"value": 1.0 / t_full, "unit": "applies/s", "cores": int(cores), "kind": "oracle",
            "sample": f"free part: dense Graf rows of {rows} of {w.n} targets ({t_free * rows / w.n:.1f} s, "
                      f"x{w.n / rows:.0f}); reflected part: {n_eval} full-apply integrand evaluations "
                      f"({t_eval:.2f} s each) x {neval} evaluations of the oracle's adaptive rule at tol 1e-12",
            "seconds_per_apply": t_full}


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
           "rhs_applies_per_s": 3.0 * nrhs * 1e3 / tot_ms, "per_frequency": per}
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
    g, i0 = op.solve(b, tol=1e-9, restart=its, maxit=its)
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
    J, gxy, gl, info = op.misfit_gradient(waves, pts, u_obs, tol=1e-9, restart=its, maxit=its,
                                          precision=1 if args.precision == "mixed" else 0)
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


def shape_generation(omega):
    """Scattering matrices of the 20000-particle cloud with one third each of
    circles, ellipses (aspect 2) and five-arm stars, generated on the GPU
    (fundamental solutions, 256 points per particle): wall clock of one call
    after an untimed call on 64 particles."""
    import numpy as np
    import torch
    import paper_2608_26875_amd as E
    import workloads as W
    ws = W.c2_cloud(shapes=True)
    media = E.make_media(ws.host, ws.substrate, omega)
    n0 = 64
    small = E.Operator(ws.xy[:n0], ws.radius[:n0], ws.p[:n0], media, bc=ws.bc[:n0])
    small.shape_smatrices(ws.shape[:n0], ws.a[:n0], ws.theta0[:n0], ws.bc[:n0])
    ops = E.Operator(ws.xy, ws.radius, ws.p, media, bc=ws.bc)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S = ops.shape_smatrices(ws.shape, ws.a, ws.theta0, ws.bc)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3
    del S
    return {"ms": ms, "us_per_particle": ms * 1e3 / ws.n, "particles": int(ws.n),
            "kinds": np.bincount(ws.shape, minlength=3).tolist(), "npts": 256,
            "p": int(ws.p.max())}


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
    w = workload(args.workload)
    media = E.make_media(w.host, w.substrate, w.omega)
    t0 = time.perf_counter()
    op = E.Operator(w.xy, w.radius, w.p, media, bc=w.bc)
    if args.fmm_leaf:
        op.set_fmm(mode=0, leaf=args.fmm_leaf)
    info = op.build()
    tiles = op.autotune(1)
    setup_s = time.perf_counter() - t0
    x = torch.from_numpy(W.random_coeffs(w.n_coeff, 1002)).cuda()
    y = torch.empty_like(x)
    flags = E.EMS_APPLY_ALL | (E.EMS_MIXED if args.precision == "mixed" else 0)
    for _ in range(args.warmup):
        op.apply(x, y, flags=flags)
    torch.cuda.synchronize()
    op.profile(True)
    st = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(st)
    for _ in range(args.steps):
        op.apply(x, y, flags=flags)
    e1.record(st)
    torch.cuda.synchronize()
    op.profile(False)
    ms = e0.elapsed_time(e1) / args.steps
    kt = op.profile_read()
    mixed = args.precision == "mixed"
    per_kernel = {}
    for k, (nl, tot_ms, fl) in kt.items():
        bound, peak = kernel_unit(k, mixed)
        d = {"launches": nl, "avg_ms": tot_ms / max(nl, 1)}
        if fl > 0:
            d["flops_per_launch"] = fl / nl
            d["tflops"] = fl / (tot_ms * 1e-3) / 1e12
            d["frac_of_peak"] = d["tflops"] * 1e12 / peak
        per_kernel[k] = d
    dom = max(kt.items(), key=lambda kv: kv[1][1])[0]
    nl, tot_ms, fl = kt[dom]
    dom_avg_s = tot_ms / nl / 1e3
    fl_launch = fl / nl
    check = section8d_flops(dom, w, info)
    if check is not None and abs(check - fl_launch) > 1e-9 * check:
        raise SystemExit(f"flop count mismatch for {dom}: library {fl_launch} vs {check}")
    bound, peak = kernel_unit(dom, mixed)
    traffic = traffic_from_profiles(dom, w.name, mixed)
    roof = {"bound": bound, "achieved": fl_launch / dom_avg_s / 1e12, "peak": peak / 1e12,
            "unit": "TFLOP/s", "frac": fl_launch / dom_avg_s / peak, "traffic": traffic,
            "kernel": dom, "flops_per_launch": fl_launch}
    out = {
        "metric": "operator applies/s & GMRES solve s at N=20k 2D, FP64 vs mixed @1e-9",
        "value": 1e3 / ms, "unit": "applies/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "c128" if args.precision == "fp64" else "c64+c128",
        "data": "synthetic",
        "config": {"workload": f"{w.name}: {w.n} particles, p={int(w.p.max())}, omega={w.omega}, "
                               f"{'FP64' if args.precision == 'fp64' else 'mixed'} apply",
                   "n_coeff": int(w.n_coeff), "q_nodes": info["q"], "somm_kept": info["somm_kept"],
                   "pairs_direct": info["n_pairs"],
                   "parallelism": "single GPU"},
        "roofline": roof,
        "kernels": per_kernel,
        "setup_s": setup_s,
        "tiles": tiles,
    }
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
    if args.workload == "c2" and not args.no_shapes:
        out["smatrix_shapes"] = shape_generation(w.omega)
    solve_its = 60 if args.solve_its is None else args.solve_its
    if args.solve or solve_its:
        # GMRES to 1e-9 within an iteration budget (restart = min(budget, 300)):
        # the time, the iterations and the residual reached are all reported
        its = 3000 if args.solve else solve_its
        b = op.incident([w.incidence[0]])
        torch.cuda.synchronize()
        xs, sinfo = op.solve(b, tol=1e-9, restart=min(its, 300), maxit=its,
                             precision=0 if args.precision == "fp64" else 1)
        out["gmres"] = sinfo
        # a time to 1e-9 exists only when the solve got there
        out["gmres_solve_s"] = sinfo["seconds"] if sinfo["converged"] else None
        out["gmres_budget_s"] = sinfo["seconds"]
        out["gmres_relres_reached"] = sinfo["relres"]
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_rows)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
