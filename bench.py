"""Benchmark: Dirac-apply HBM GB/s and time to a 1e-10 solve, mixed precision
against plain FP64 BiCGStab, on one MI355X.

Workload (default): 64^3 x 128 lattice, c_SW 1.7, random SU(3) links
exp(0.3 i H), Gaussian source, SAP with 4^4 blocks, 4 Jacobi sweeps, SAP loop
count 4; the mixed-precision solver (FP16 SAP, FP32 BiCGStab, FP64 defect
correction) to a true FP64 relative residual of 1e-10.  kappa = 0.133: with
these random links the operator at kappa = 0.1365 is past the critical point on
this volume (neither the SAP solvers nor plain FP64 BiCGStab reach 1e-10 there;
measured scan in the design notes), while 0.133 keeps the solve near-critical
(hundreds of plain FP64 iterations).  The Dirac apply costs the same at any kappa.

A step is one mixed-precision solve of that system from a zero start: every
part of the path runs in it (FP64 Dirac apply for the outer residual, FP16
SAP half-sweeps, FP32 Dirac apply on the preconditioned directions, BiCGStab
vector kernels).  Inputs are drawn on the device before the timed region.

value: algorithmic bytes of all Dirac-apply launches inside the timed steps
divided by their summed launch time (HIP events on the library's stream).
The roofline object reports the dominant kernel of a step.  The plain FP64
BiCGStab solve of the same system runs once, after the timed steps.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0        # MI355X HBM3E
FP32_VEC_TFLOPS = 157.3      # MI355X vector FP32 (published)
FP64_VEC_TFLOPS = 78.6


def class_kernels(block):
    """Kernel class of the library's timers -> the kernel instantiation rocprofv3 reports.
    With 4^4 blocks the FP64, FP32 and FP16-input Dirac applies run the t-streamed kernel
    (k_dirac_ts), the all-FP16 apply and the packed-FP16 SAP half-sweep their 4^4
    specialisations (template argument 4; the half-sweep of one right-hand side is its <B, true>
    form); other block shapes run the generic kernels (0)."""
    if tuple(block) == (4, 4, 4, 4):
        return {"dirac_f64": "k_dirac_ts<0, 0, 0, 0>", "dirac_f32": "k_dirac_ts<1, 1, 1, 1>",
                "dirac_f16in": "k_dirac_ts<2, 1, 1, 1>", "dirac_f16": "k_dirac<2, 2, 2, 1, 4>",
                "sap": "k_sap_half<2>", "sap_pk": "k_sap_half_pk<4, true>", "blas": "vector kernels"}
    return {"dirac_f64": "k_dirac<0, 0, 0, 0, 0>", "dirac_f32": "k_dirac<1, 1, 1, 1, 0>",
            "dirac_f16in": "k_dirac<2, 1, 1, 1, 0>", "dirac_f16": "k_dirac<2, 2, 2, 1, 0>",
            "sap": "k_sap_half<2>", "sap_pk": "k_sap_half_pk<0, true>", "blas": "vector kernels"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--dims", default="64,64,64,128", help="Lx,Ly,Lz,Lt")
    ap.add_argument("--block", default="4,4,4,4")
    ap.add_argument("--kappa", type=float, default=0.133)
    ap.add_argument("--csw", type=float, default=1.7)
    ap.add_argument("--eps", type=float, default=0.3)
    # the SAP loop count of Alg. 1 (the paper leaves it open; its flop tables fit 4): 6 is the
    # fastest setting that stays convergent at kappa 0.1365 on 32^4, where 9 already slows the
    # solve and 10 or more break it down (a scan of the time to 1e-10 on 64^3 x 128 at kappa 0.133
    # and of both 32^4 solves, N_JAC = 4)
    ap.add_argument("--n-sap", type=int, default=6)
    ap.add_argument("--n-jac", type=int, default=4)
    ap.add_argument("--inner-tol", type=float, default=1e-6)
    ap.add_argument("--sap-fp16-arith", type=int, default=1, help="packed FP16 arithmetic in the FP16 SAP (1) or FP32 (0)")
    ap.add_argument("--tol", type=float, default=1e-10)
    ap.add_argument("--seed", type=int, default=2021)
    ap.add_argument("--apply-reps", type=int, default=20)
    ap.add_argument("--fp64", choices=["on", "off"], default="on")
    ap.add_argument("--fp64-maxiter", type=int, default=4000)
    ap.add_argument("--cpu-baseline", choices=["on", "off"], default="on")
    ap.add_argument("--only-apply", action="store_true", help="time the Dirac applies only (profiling runs)")
    ap.add_argument("--force-dims", default="24,24,24,24",
                    help="lattice of the fermion-force leg (L = |D^-1 phi|^2 and its link derivative); 'off' skips it")
    ap.add_argument("--force-reps", type=int, default=10)
    ap.add_argument("--only-force", action="store_true", help="run the fermion-force leg only (profiling runs)")
    ap.add_argument("--batch-dims", default="32,32,32,64",
                    help="lattice of the batched leg (12 spin-colour point sources); 'off' skips it")
    ap.add_argument("--only-batch", action="store_true", help="run the batched leg only (profiling runs)")
    ap.add_argument("--multi", choices=["on", "off"], default="on",
                    help="the multi-lattice leg: 8^4, 12^4, 16^4, 16^3x32, two each, in one launch")
    ap.add_argument("--single-prec", choices=["on", "off"], default="on",
                    help="the 32^4 leg: FP32 SAP-BiCGStab at kappa 0.1365 to 1e-6 against plain FP64")
    ap.add_argument("--single-prec-fp64-maxiter", type=int, default=6000)
    ap.add_argument("--only-single", action="store_true", help="run the 32^4 single-precision leg only (profiling runs)")
    ap.add_argument("--only-multi", action="store_true", help="run the multi-lattice leg only (profiling runs)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a plain device copy of 4 GiB five times (scale for HBM byte counters) and exit")
    return ap.parse_args()


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("dd_kernels.hip", "dd_sap_fp16.hip", "dd_device.h"):
        with open(os.path.join(ROOT, "paper_2109_10687_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, launches_bytes):
    """HBM bytes per launch from committed rocprofv3 counter runs, when they were
    taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    rec = t.get(kernel)
    if not rec or rec.get("source_hash") != kernel_source_hash():
        return None
    return rec.get("bytes_per_launch")


def measured_hbm(reps=10, nbytes=2 << 30):
    """Device bandwidth the same GPU reaches on plain streaming kernels (torch's copy and
    add over 2 GiB arrays, HIP events): the practical ceiling the Dirac apply is also
    compared with, beside the 8 TB/s HBM peak."""
    import torch
    n = nbytes // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.ones(n, dtype=torch.float32, device="cuda")
    c = torch.empty_like(a)
    out = {}
    for name, fn, moved in (("copy", lambda: c.copy_(a), 2 * nbytes), ("add", lambda: torch.add(a, b, out=c), 3 * nbytes)):
        for _ in range(3):
            fn()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        out[f"{name}_GBps"] = round(moved * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9, 1)
    del a, b, c
    torch.cuda.empty_cache()
    return out


def dirac_microbench(dd, solver, b, reps):
    """Standalone applies on internal-layout fields: FP64 D, FP32 A, FP16 A, and the inner
    solver's A (FP16 input, FP32 links / C_inv / output)."""
    import torch
    out = {}
    for name, prec, op in (("f64_D", dd.DD_F64, dd.DD_OP_D), ("f32_A", dd.DD_F32, dd.DD_OP_A),
                           ("f16_A", dd.DD_F16, dd.DD_OP_A), ("f16in_A", dd.DD_F16, dd.DD_OP_A)):
        fin = solver.pack(b, prec)
        if name == "f16in_A":
            fout = solver.field(dd.DD_F32)
            run = lambda: solver.apply_packed_f16in(fout, fin)  # noqa: E731
        else:
            fout = solver.field(prec)
            run = lambda: solver.apply_packed(fout, fin, op=op, prec=prec)  # noqa: E731
        for _ in range(3):
            run()
        solver.timing(True)
        for _ in range(reps):
            run()
        rep = solver.timing_report()
        solver.timing(False)
        cls = {"f64_D": "dirac_f64", "f32_A": "dirac_f32", "f16_A": "dirac_f16", "f16in_A": "dirac_f16in"}[name]
        r = rep[cls]
        ms = r["ms"] / max(r["launches"], 1)
        out[name] = {"ms": ms, "GBps": r["bytes"] / r["ms"] / 1e6, "GFLOPs": r["flops"] / r["ms"] / 1e6,
                     "bytes_per_site": r["bytes"] / r["launches"] / solver.params.volume}
        del fin, fout
        torch.cuda.synchronize()
    return out


def force_bench(dd, args):
    """The differentiation leg: on its own lattice, psi = D^{-1} phi and chi = D^{-dagger} psi by
    the mixed-precision solver, then `force_reps` timed dd_force calls (su(3) force and
    dL/dc_SW, FP64).  The force is compute-heavy (24 leaves per link): it is reported against
    the FP64 vector peak, with its algorithmic bytes beside."""
    import torch
    import synth
    dims = tuple(int(v) for v in args.force_dims.split(","))
    V = math.prod(dims)
    params = dd.Params(dims=dims, kappa=args.kappa, csw=args.csw, block=tuple(int(v) for v in args.block.split(",")),
                       n_sap=args.n_sap, n_jac=args.n_jac, inner_tol=args.inner_tol,
                       sap_fp16_arith=args.sap_fp16_arith)
    U = synth.su3_links(dims, args.eps, args.seed + 7, device="cuda")
    phi = synth.gaussian_spinor(dims, args.seed + 8, device="cuda")
    s = dd.Solver(params, U)
    t0 = time.perf_counter()
    psi, i1 = s.solve(phi, tol=args.tol, mode=dd.DD_SOLVE_MIXED)
    chi, i2 = s.solve_dagger(psi, tol=args.tol, mode=dd.DD_SOLVE_MIXED)
    t_solves = time.perf_counter() - t0
    F, dcsw = s.force(psi, chi, su3=True)
    torch.cuda.synchronize()
    s.timing(True)
    t0 = time.perf_counter()
    for _ in range(args.force_reps):
        s.force(psi, chi, su3=True, out=F)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    r = s.timing_report()["force"]
    s.timing(False)
    ms = r["ms"] / r["launches"]
    tf = r["flops"] / r["ms"] / 1e9
    out = {"workload": f"fermion force {'x'.join(map(str, dims))}", "dims": list(dims),
           "forward_solve": {"status": i1["status"], "seconds": round(i1["seconds"], 3), "relres_true": i1["relres_true"]},
           "adjoint_solve": {"status": i2["status"], "seconds": round(i2["seconds"], 3), "relres_true": i2["relres_true"]},
           "solves_seconds": round(t_solves, 3), "force_ms": round(ms, 4), "force_wall_ms": round(wall / args.force_reps * 1e3, 4),
           "dL_dcsw": dcsw, "loss": s.norm2(psi),
           "roofline": {"kernel": "k_force_y + k_force_w", "bound": "alu", "achieved": round(tf, 3),
                        "peak": FP64_VEC_TFLOPS, "unit": "TFLOP/s", "frac": round(tf / FP64_VEC_TFLOPS, 4),
                        "bytes_GBps": round(r["bytes"] / r["ms"] / 1e6, 1),
                        "flops_per_site": r["flops"] / r["launches"] / V,
                        "algorithmic_bytes_per_site": r["bytes"] / r["launches"] / V}}
    s.close()
    del U, phi, psi, chi, F
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def batch_bench(dd, args, reps=10):
    """The batched leg: the 12 spin-colour point sources at the origin on their own lattice.
    (1) The FP32 operator A on all 12 at once (matrix-core kernel, autotuned variant) against 12
    single right-hand-side FP32 applies; (2) the batched mixed-precision solve to 1e-10 (lockstep
    FP32 BiCGStab with the FP16 SAP of each right-hand side, FP64 defect correction) against 12
    single right-hand-side mixed solves (FP16 SAP) one after another."""
    import torch
    import synth
    dims = tuple(int(v) for v in args.batch_dims.split(","))
    V = math.prod(dims)
    params = dd.Params(dims=dims, kappa=args.kappa, csw=args.csw, block=tuple(int(v) for v in args.block.split(",")),
                       n_sap=args.n_sap, n_jac=args.n_jac, inner_tol=args.inner_tol,
                       sap_fp16_arith=args.sap_fp16_arith)
    U = synth.su3_links(dims, args.eps, args.seed + 11, device="cuda")
    s = dd.Solver(params, U)
    bs = torch.stack([synth.point_source(dims, c, sp, device="cuda") for c in range(3) for sp in range(4)])
    n = bs.shape[0]
    out = {"workload": f"12 point sources {'x'.join(map(str, dims))}", "dims": list(dims), "nrhs": n}
    # (1) operator: batched (tuned on the first call) against single right-hand sides
    ys = s.apply_batch(bs, op=dd.DD_OP_A, prec=dd.DD_F32)
    tune = s.batch_tuning(12)
    s.timing(True)
    for _ in range(reps):
        s.apply_batch(bs, op=dd.DD_OP_A, prec=dd.DD_F32, out=ys)
    r = s.timing_report()["dirac_mrhs"]
    s.timing(False)
    fin = s.pack(bs[0], dd.DD_F32)
    fout = s.field(dd.DD_F32)
    s.apply_packed(fout, fin, op=dd.DD_OP_A, prec=dd.DD_F32)
    s.timing(True)
    for _ in range(reps):
        s.apply_packed(fout, fin, op=dd.DD_OP_A, prec=dd.DD_F32)
    r1 = s.timing_report()["dirac_f32"]
    s.timing(False)
    ms_b = r["ms"] / r["launches"]
    ms_1 = r1["ms"] / r1["launches"]
    out["apply"] = {"batched_ms": round(ms_b, 4), "single_ms": round(ms_1, 4), "single_x12_ms": round(12 * ms_1, 4),
                    "speedup_vs_12_single": round(12 * ms_1 / ms_b, 2),
                    "batched_GBps": round(r["bytes"] / r["ms"] / 1e6, 1),
                    "batched_TFLOPs": round(r["flops"] / r["ms"] / 1e9, 3),
                    "bytes_per_site": r["bytes"] / r["launches"] / V, "flops_per_site": r["flops"] / r["launches"] / V,
                    "variant": tune["name"], "autotuner_ms": tune["ms"]}
    out["roofline"] = {"kernel": "k_dirac_mrhs", "bound": "hbm", "achieved": out["apply"]["batched_GBps"],
                       "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(out["apply"]["batched_GBps"] / HBM_PEAK_GBS, 4),
                       "mfma_fp32_TFLOPs": out["apply"]["batched_TFLOPs"], "mfma_fp32_peak": 157.3}
    del fin, fout, ys
    # (2) solves
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xb, infos = s.solve_batch(bs, tol=args.tol, inner=dd.DD_BATCH_INNER_SAP)
    torch.cuda.synchronize()
    tb = time.perf_counter() - t0
    t0 = time.perf_counter()
    singles = []
    for k in range(n):
        x1, i1 = s.solve(bs[k], tol=args.tol, mode=dd.DD_SOLVE_MIXED)
        singles.append(i1)
        if k == 0:
            err0 = (torch.linalg.vector_norm(xb[0] - x1) / torch.linalg.vector_norm(x1)).item()
    torch.cuda.synchronize()
    t1 = time.perf_counter() - t0
    out["solve"] = {"batched_seconds": round(tb, 3), "batched_status": sorted({i["status"] for i in infos}),
                    "batched_max_relres_true": max(i["relres_true"] for i in infos),
                    "batched_outer": max(i["iters_outer"] for i in infos),
                    "batched_inner_max": max(i["iters_inner_total"] for i in infos),
                    "single_x12_seconds": round(t1, 3), "single_status": sorted({i["status"] for i in singles}),
                    "single_max_relres_true": max(i["relres_true"] for i in singles),
                    "batched_vs_single_solution_relerr_rhs0": err0}
    s.close()
    del U, bs, xb
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def single_prec_bench(dd, args, reps=3, apply_reps=20):
    """The 32^4 leg at the operator parameters the paper's single-precision runs stand for:
    kappa 0.1365, c_SW 1.7, links exp(0.3 i H), 4^4 blocks, N_JAC = 4, N_SAP as given; FP32 SAP-BiCGStab
    (Alg. 5 on A M_SAP, FP32 SAP) to Alg. 5's single-precision tolerance 1e-6 on its recursive
    residual, against plain FP64 BiCGStab on D to a true residual of 1e-6 on the same GPU.  At this
    kappa plain BiCGStab breaks down before reaching 1e-6 on this ensemble: its time is then a lower
    bound.  The FP32 apply of this lattice (0.7 GB per apply) partly stays in the 256 MB Infinity
    Cache, so its GB/s are reported as such, not as HBM bandwidth."""
    import torch
    import synth
    dims = (32, 32, 32, 32)
    params = dd.Params(dims=dims, kappa=0.1365, csw=1.7, block=(4, 4, 4, 4), n_sap=args.n_sap, n_jac=4)
    U = synth.su3_links(dims, 0.3, args.seed + 60, device="cuda")
    b = synth.gaussian_spinor(dims, args.seed + 61, device="cuda")
    s = dd.Solver(params, U)
    del U
    x, info = s.solve(b, tol=1e-6, maxiter=2000, mode=dd.DD_SOLVE_F32_SAP)  # warm-up
    secs = []
    for _ in range(reps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x, info = s.solve(b, tol=1e-6, maxiter=2000, mode=dd.DD_SOLVE_F32_SAP)
        torch.cuda.synchronize()
        secs.append(time.perf_counter() - t0)
    t32 = sorted(secs)[len(secs) // 2]
    out = {"workload": "32x32x32x32 FP32 SAP-BiCGStab, kappa 0.1365, c_SW 1.7, tol 1e-6", "n_sap": args.n_sap,
           "fp32_sap": {"seconds": round(t32, 4), "iters": info["iters_inner_total"], "status": info["status"],
                        "relres_recursive": info["relres_inner_last"], "relres_true": info["relres_true"],
                        "ms_per_iter": round(t32 / max(info["iters_inner_total"], 1) * 1e3, 3),
                        "a_msap": "A applied to the SAP output"}}
    # the same solve with A M_SAP from the fused tail of Alg. 3: same operator, other rounding
    fus = dd.Solver(dd.Params(dims=dims, kappa=0.1365, csw=1.7, block=(4, 4, 4, 4), n_sap=args.n_sap, n_jac=4,
                              sap_fused_tail=1), synth.su3_links(dims, 0.3, args.seed + 60, device="cuda"))
    fus.solve(b, tol=1e-6, maxiter=2000, mode=dd.DD_SOLVE_F32_SAP)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    _, ifus = fus.solve(b, tol=1e-6, maxiter=2000, mode=dd.DD_SOLVE_F32_SAP)
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["fp32_sap_fused_tail"] = {"seconds": round(ts, 4), "iters": ifus["iters_inner_total"],
                                  "status": ifus["status"], "relres_true": ifus["relres_true"],
                                  "ms_per_iter": round(ts / max(ifus["iters_inner_total"], 1) * 1e3, 3)}
    fus.close()
    # the two mixed-precision outer loops to 1e-10 at this kappa: defect correction (Alg. 4) and
    # flexible GMRES, both around the FP32 BiCGStab with the FP16 SAP
    out["mixed_to_1e-10"] = {}
    for name, mode in (("defect_correction", dd.DD_SOLVE_MIXED), ("fgmres", dd.DD_SOLVE_FGMRES)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _, im = s.solve(b, tol=1e-10, maxiter=12, mode=mode)
        torch.cuda.synchronize()
        out["mixed_to_1e-10"][name] = {"seconds": round(time.perf_counter() - t0, 3), "status": im["status"],
                                       "status_detail": im["status_detail"], "outer": im["iters_outer"],
                                       "inner": im["iters_inner_total"], "relres_true": im["relres_true"]}
    x64, i64 = s.solve(b, tol=1e-6, maxiter=args.single_prec_fp64_maxiter, mode=dd.DD_SOLVE_F64_PLAIN)
    conv = i64["status"] == "DD_OK"
    out["fp64_plain"] = {"seconds": round(i64["seconds"], 3), "iters": i64["iters_inner_total"],
                         "status": i64["status"], "status_detail": i64["status_detail"],
                         "relres_true": i64["relres_true"], "converged": conv}
    out["speedup_fp32_sap_vs_fp64" if conv else "speedup_fp32_sap_vs_fp64_lower_bound"] = round(i64["seconds"] / t32, 2)
    fin = s.pack(b, dd.DD_F32)
    fout = s.field(dd.DD_F32)
    for _ in range(3):
        s.apply_packed(fout, fin, op=dd.DD_OP_A, prec=dd.DD_F32)
    s.timing(True)
    for _ in range(apply_reps):
        s.apply_packed(fout, fin, op=dd.DD_OP_A, prec=dd.DD_F32)
    r = s.timing_report()["dirac_f32"]
    s.timing(False)
    out["apply_f32_A"] = {"ms": round(r["ms"] / r["launches"], 4), "GBps": round(r["bytes"] / r["ms"] / 1e6, 1),
                          "note": "partly Infinity-Cache resident (0.7 GB per apply against 256 MB): not an HBM figure"}
    s.close()
    del b, x, x64, fin, fout
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


MULTI_SET = [((8, 8, 8, 8), (4, 4, 4, 4)), ((12, 12, 12, 12), (2, 2, 2, 2)), ((16, 16, 16, 16), (4, 4, 4, 4)),
             ((16, 16, 16, 32), (4, 4, 4, 4))]


def multi_bench(dd, args, reps=20):
    """The multi-lattice leg: eight independent lattices (two each of MULTI_SET, own links),
    A on all of them in one persistent launch against one launch per lattice, and the lockstep
    mixed-precision solve of all eight against eight solves one after another."""
    import torch
    import synth
    params, Us = [], []
    for k in range(8):
        dims, block = MULTI_SET[k // 2]
        params.append(dd.Params(dims=dims, kappa=args.kappa, csw=args.csw, block=block, n_sap=args.n_sap,
                                n_jac=args.n_jac, inner_tol=args.inner_tol, sap_fp16_arith=args.sap_fp16_arith))
        Us.append(synth.su3_links(dims, args.eps, args.seed + 20 + k, device="cuda"))
    m = dd.Multi(params)
    singles = [dd.Solver(p, U) for p, U in zip(params, Us)]
    for k, U in enumerate(Us):
        m.load_gauge(k, U)
    bs = [synth.gaussian_spinor(p.dims, args.seed + 40 + k, device="cuda") for k, p in enumerate(params)]
    V = sum(math.prod(p.dims) for p in params)
    m.apply(bs)
    m.timing(True)
    for _ in range(reps):
        m.apply(bs)
    r = m.timing_report()["dirac_multi"]
    m.timing(False)
    # one launch per lattice, internal layout, the same FP32 operator
    fins = [s.pack(b, dd.DD_F32) for s, b in zip(singles, bs)]
    fouts = [s.field(dd.DD_F32) for s in singles]
    for s, fi, fo in zip(singles, fins, fouts):
        s.apply_packed(fo, fi, op=dd.DD_OP_A, prec=dd.DD_F32)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        for s, fi, fo in zip(singles, fins, fouts):
            s.apply_packed(fo, fi, op=dd.DD_OP_A, prec=dd.DD_F32)
    ev1.record()
    torch.cuda.synchronize()
    ms_seq = ev0.elapsed_time(ev1) / reps
    ms_multi = r["ms"] / r["launches"]
    out = {"workload": "8 lattices: 8^4, 12^4, 16^4, 16^3x32, two each", "sites": V,
           "apply": {"one_launch_ms": round(ms_multi, 4), "eight_launches_ms": round(ms_seq, 4),
                     "one_launch_GBps": round(r["bytes"] / r["ms"] / 1e6, 1),
                     "speedup": round(ms_seq / ms_multi, 2)}}
    del fins, fouts
    # one untimed solve of each kind first (first-call work: descriptor tables, field set-up)
    m.solve(bs, tol=args.tol)
    for s, b in zip(singles, bs):
        s.solve(b, tol=args.tol, mode=dd.DD_SOLVE_MIXED)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    xs, infos = m.solve(bs, tol=args.tol)
    torch.cuda.synchronize()
    tm = time.perf_counter() - t0
    t0 = time.perf_counter()
    seq = [s.solve(b, tol=args.tol, mode=dd.DD_SOLVE_MIXED)[1] for s, b in zip(singles, bs)]
    torch.cuda.synchronize()
    ts = time.perf_counter() - t0
    out["solve"] = {"lockstep_seconds": round(tm, 4), "sequential_seconds": round(ts, 4),
                    "lockstep_status": sorted({i["status"] for i in infos}),
                    "lockstep_max_relres_true": max(i["relres_true"] for i in infos),
                    "sequential_status": sorted({i["status"] for i in seq})}
    for s in singles:
        s.close()
    m.close()
    del Us, bs, xs
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    return out


def cpu_baseline(gpu_fp64_iters=None, seconds_target=8.0, iter_sample=20):
    """The FP64 oracle on the host cores, on bounded samples of the workload (same c_SW and link
    recipe): its D apply on 32^4 in the metric's unit (algorithmic GB/s at 1536 B/site), and its
    plain FP64 BiCGStab (Alg. 5, M = I): to 1e-10 on the 4^4 correctness lattice and on 16^4 at
    kappa 0.133 (measured), and on 32^4 at kappa 0.133 as `iter_sample` timed iterations.  kappa
    0.133 because at 0.1365 plain BiCGStab does not reach 1e-10 on this ensemble at 32^4 and
    above.  The 32^4 and 64^3 x 128 solve times are estimates, labelled so: the oracle's time per
    iteration (at 64^3 x 128 the 32^4 figure times the volume ratio) times the iteration count
    of the GPU's plain FP64 solve."""
    import numpy as np
    import oracle as O
    import synth
    dims = (32, 32, 32, 32)
    p = O.Params(dims=dims, kappa=0.133, csw=1.7, block=(4, 4, 4, 4))
    U = synth.su3_links(dims, 0.3, 5).numpy()
    C = O.clover_field(p, U)
    x = synth.gaussian_spinor(dims, 6).numpy()
    O.dirac_D(p, U, C, x)
    n, t0 = 0, time.perf_counter()
    while True:
        O.dirac_D(p, U, C, x)
        n += 1
        el = time.perf_counter() - t0
        if el > seconds_target or n >= 50:
            break
    V = math.prod(dims)
    cores = os.environ.get("OMP_NUM_THREADS")
    cores = int(cores) if cores else (len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count())
    solves = {}
    for name, d, kappa, csw, eps in (("4x4x4x4", (4, 4, 4, 4), 0.12, 1.0, 0.5), ("16x16x16x16", (16, 16, 16, 16), 0.133, 1.7, 0.3)):
        q = O.Params(dims=d, kappa=kappa, csw=csw, block=(2, 2, 2, 2))
        Uq = synth.su3_links(d, eps, 7).numpy()
        bq = synth.gaussian_spinor(d, 8).numpy()
        Cq = O.clover_field(q, Uq)
        t1 = time.perf_counter()
        r = O.bicgstab(q, Uq, Cq, None, bq, op=O.OP_D, tol=1e-10, maxiter=20000)
        solves[name] = {"kappa": kappa, "csw": csw, "seconds": round(time.perf_counter() - t1, 3), "iters": r.iters,
                        "relres": r.relres, "kind": "measured"}
    b = synth.gaussian_spinor(dims, 9).numpy()
    t1 = time.perf_counter()
    r = O.bicgstab(p, U, C, None, b, op=O.OP_D, tol=1e-10, maxiter=iter_sample)
    per_iter = (time.perf_counter() - t1) / max(r.iters, 1)
    est = {"kappa": 0.133, "csw": 1.7, "seconds_per_iter": round(per_iter, 4), "sampled_iters": r.iters,
           "kind": "estimate: oracle time per iteration x the GPU plain FP64 iteration count"}
    if gpu_fp64_iters and gpu_fp64_iters.get("32x32x32x32"):
        est["gpu_fp64_iters"] = gpu_fp64_iters["32x32x32x32"]
        est["seconds"] = round(per_iter * est["gpu_fp64_iters"], 1)
    solves["32x32x32x32"] = est
    if gpu_fp64_iters and gpu_fp64_iters.get("64x64x64x128"):
        it = gpu_fp64_iters["64x64x64x128"]
        solves["64x64x64x128"] = {"kappa": 0.133, "csw": 1.7, "gpu_fp64_iters": it,
                                  "seconds": round(per_iter * 32 * it, 1),
                                  "kind": "estimate: 32^4 oracle time per iteration x 32 (volume ratio) x the GPU "
                                          "plain FP64 iteration count; the oracle cannot hold this lattice's clover"}
    return {"value": round(1536.0 * V * n / el / 1e9, 4), "unit": "GB/s", "cores": cores, "kind": "oracle",
            "sample": f"FP64 oracle D apply on a 32^4 lattice (kappa 0.133, c_SW 1.7, eps 0.3), {n} applies in "
                      f"{el:.1f} s; {el / n * 1e3:.0f} ms per apply; clover precomputed",
            "cpu_model": cpu_model(), "solves": solves}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def gpu_plain_iters_32(dd, args):
    """Iterations of the GPU's plain FP64 BiCGStab to 1e-10 on the oracle's 32^4 baseline system
    (kappa 0.133; the same links and source as cpu_baseline), for its labelled estimate."""
    import synth
    dims = (32, 32, 32, 32)
    # drawn by the CPU generator, as the oracle's inputs are
    s = dd.Solver(dd.Params(dims=dims, kappa=0.133, csw=1.7, block=(4, 4, 4, 4)),
                  synth.su3_links(dims, 0.3, 5).cuda())
    _, info = s.solve(synth.gaussian_spinor(dims, 9).cuda(), tol=1e-10, maxiter=4000,
                      mode=dd.DD_SOLVE_F64_PLAIN)
    s.close()
    return info["iters_inner_total"] if info["status"] == "DD_OK" else None


def main():
    args = parse()
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported (the path runs on one "
              "MI355X; the multi-GPU decomposition is a design note, not a measured configuration)", file=sys.stderr)
        sys.exit(2)
    import torch

    if args.copy_calibration:
        n = 4 << 30
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration": {"bytes_read_per_copy": n, "bytes_written_per_copy": n, "copies": 5}}))
        return

    import paper_2109_10687_amd as dd
    import synth

    force = None
    if args.force_dims != "off":
        log(f"fermion-force leg on {args.force_dims}")
        force = force_bench(dd, args)
        log(f"force: {force['force_ms']:.3f} ms per call, {force['roofline']['achieved']:.2f} TFLOP/s FP64, "
            f"{force['roofline']['bytes_GBps']:.0f} GB/s algorithmic; solves {force['solves_seconds']:.2f} s")
        if args.only_force:
            print(json.dumps({"force": force}))
            return

    batch = None
    if args.batch_dims != "off":
        log(f"batched leg on {args.batch_dims}")
        batch = batch_bench(dd, args)
        log(f"batched A: {batch['apply']['batched_ms']:.3f} ms for 12 right-hand sides vs "
            f"{batch['apply']['single_x12_ms']:.3f} ms for 12 single ({batch['apply']['variant']}); batched solve "
            f"{batch['solve']['batched_seconds']:.2f} s vs 12 single solves {batch['solve']['single_x12_seconds']:.2f} s")
        if args.only_batch:
            print(json.dumps({"batch": batch}))
            return

    single = None
    if args.single_prec == "on" and not args.only_apply:
        log("32^4 single-precision leg (kappa 0.1365)")
        single = single_prec_bench(dd, args)
        log(f"32^4: FP32 SAP {single['fp32_sap']['seconds']:.3f} s ({single['fp32_sap']['iters']} it., "
            f"{single['fp32_sap']['status']}); plain FP64 {single['fp64_plain']['seconds']:.2f} s "
            f"({single['fp64_plain']['iters']} it., {single['fp64_plain']['status']})")
        if args.only_single:
            print(json.dumps({"single_prec_32x32x32x32": single}))
            return

    multi = None
    if args.multi == "on" and not args.only_apply:
        log("multi-lattice leg")
        multi = multi_bench(dd, args)
        log(f"multi-lattice A: {multi['apply']['one_launch_ms']:.3f} ms in one launch vs "
            f"{multi['apply']['eight_launches_ms']:.3f} ms in eight; lockstep solve {multi['solve']['lockstep_seconds']:.3f} s "
            f"vs {multi['solve']['sequential_seconds']:.3f} s")
        if args.only_multi:
            print(json.dumps({"multi": multi}))
            return

    dims = tuple(int(v) for v in args.dims.split(","))
    block = tuple(int(v) for v in args.block.split(","))
    CLASS_KERNEL = class_kernels(block)
    V = math.prod(dims)
    params = dd.Params(dims=dims, kappa=args.kappa, csw=args.csw, block=block, n_sap=args.n_sap, n_jac=args.n_jac,
                       inner_tol=args.inner_tol, sap_fp16_arith=args.sap_fp16_arith)
    dev = torch.device("cuda:0")
    t0 = time.time()
    log(f"drawing links and source for {dims} on the device")
    U = synth.su3_links(dims, args.eps, args.seed, device=dev)
    b = synth.gaussian_spinor(dims, args.seed + 1, device=dev)
    torch.cuda.synchronize()
    log(f"inputs ready in {time.time() - t0:.1f} s; creating the context and loading the gauge field")
    solver = dd.Solver(params)
    solver.load_gauge(U)
    del U
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    log(f"setup done at {time.time() - t0:.1f} s")

    micro = dirac_microbench(dd, solver, b, args.apply_reps)
    for k, v in micro.items():
        log(f"apply {k}: {v['ms']:.3f} ms, {v['GBps']:.0f} GB/s, {v['GFLOPs']:.0f} GFLOP/s")
    if args.only_apply:
        print(json.dumps({"dirac_apply": micro}))
        return

    # ---- warm-up and timed mixed-precision solves
    x = solver.new_spinor()
    for w in range(args.warmup):
        x, info = solver.solve(b, tol=args.tol, maxiter=50, mode=dd.DD_SOLVE_MIXED)
        log(f"warm-up solve {w}: {info['status']} {info['seconds']:.2f} s, outer {info['iters_outer']}, "
            f"inner {info['iters_inner_total']}, true residual {info['relres_true']:.2e}")
    torch.cuda.synchronize()
    solver.timing(True)
    infos = []
    t_start = time.perf_counter()
    for s in range(args.steps):
        x, info = solver.solve(b, tol=args.tol, maxiter=50, mode=dd.DD_SOLVE_MIXED)
        infos.append(info)
        log(f"step {s}: {info['status']} {info['seconds']:.2f} s, outer {info['iters_outer']}, "
            f"inner {info['iters_inner_total']}, true residual {info['relres_true']:.2e}")
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    hist = solver.history()  # of the last timed solve
    rep = solver.timing_report()
    solver.timing(False)
    ms_step = wall / args.steps * 1e3

    dirac_names = ("dirac_f64", "dirac_f32", "dirac_f16in", "dirac_f16")
    dbytes = sum(rep[k]["bytes"] for k in dirac_names)
    dms = sum(rep[k]["ms"] for k in dirac_names)
    value = dbytes / dms / 1e6 if dms > 0 else 0.0
    kernels = {k: {"launches": v["launches"], "ms_per_step": v["ms"] / args.steps,
                   "avg_ms": v["ms"] / max(v["launches"], 1),
                   "GBps": v["bytes"] / v["ms"] / 1e6 if v["ms"] else 0.0,
                   "GFLOPs": v["flops"] / v["ms"] / 1e6 if v["ms"] else 0.0}
               for k, v in rep.items() if v["launches"]}
    dominant = max(rep, key=lambda k: rep[k]["ms"])
    d = rep[dominant]
    avg_ms = d["ms"] / d["launches"]
    if dominant == "sap":
        # the half-sweep against the roof its arithmetic intensity selects: counted flops per
        # algorithmic byte below the packed-FP16 ridge (157.3 TFLOP/s / 8 TB/s = 19.7 flop/B) put
        # it under the HBM roof; the ALU figures are kept beside
        tflops = d["flops"] / d["launches"] / (avg_ms * 1e-3) / 1e12
        gbps = d["bytes"] / d["launches"] / (avg_ms * 1e-3) / 1e9
        ai = d["flops"] / d["bytes"]
        ridge = FP32_VEC_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
        alu = {"achieved": round(tflops, 3), "peak": FP32_VEC_TFLOPS, "unit": "TFLOP/s",
               "frac": round(tflops / FP32_VEC_TFLOPS, 4)}
        if ai < ridge:
            roof = {"kernel": CLASS_KERNEL["sap"], "bound": "hbm", "achieved": round(gbps, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(gbps / HBM_PEAK_GBS, 4), "alu": alu}
        else:
            roof = {"kernel": CLASS_KERNEL["sap"], "bound": "alu", **alu, "bytes_GBps": round(gbps, 1)}
        roof["arithmetic_intensity_flop_per_byte"] = round(ai, 2)
        roof["ridge_flop_per_byte"] = round(ridge, 2)
    else:
        achieved = d["bytes"] / d["launches"] / (avg_ms * 1e-3) / 1e9
        roof = {"kernel": CLASS_KERNEL[dominant], "bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4)}
    roof["avg_launch_ms"] = round(avg_ms, 4)
    roof["algorithmic_bytes_per_launch"] = d["bytes"] / d["launches"]
    if dominant == "sap" and args.sap_fp16_arith:
        roof["kernel"] = CLASS_KERNEL["sap_pk"]
    roof["traffic"] = measured_traffic(roof["kernel"], None)
    # the Dirac apply inside the solve, against the HBM roof
    dk = max(dirac_names, key=lambda k: rep[k]["ms"])
    dr = rep[dk]
    roof_dirac = {"kernel": CLASS_KERNEL[dk], "bound": "hbm", "achieved": round(dr["bytes"] / dr["ms"] / 1e6, 1),
                  "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(dr["bytes"] / dr["ms"] / 1e6 / HBM_PEAK_GBS, 4),
                  "avg_launch_ms": round(dr["ms"] / dr["launches"], 4),
                  "bytes_per_site": round(dr["bytes"] / dr["launches"] / V, 1),
                  "algorithmic_bytes_per_launch": dr["bytes"] / dr["launches"]}
    roof_dirac["traffic"] = measured_traffic(roof_dirac["kernel"], None)

    result = {
        "metric": "Dirac-apply HBM GB/s; solve time to 1e-10, mixed-prec vs FP64, one GPU",
        "value": round(value, 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_step, 2),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f16/f32/f64",
        "data": "synthetic: seeded random SU(3) links exp(0.3 i H) and a Gaussian source, drawn on the device",
        "config": {"workload": f"Clover-Wilson solve {dims[0]}x{dims[1]}x{dims[2]}x{dims[3]}",
                   "kappa_note": ("0.1365 is past the critical point for this synthetic ensemble: D's leftmost eigenvalue "
                                  "has Re -0.0066 already on 8^4 (+0.019 at 0.133; oracle + ARPACK, "
                                  "tests/golden/kappa_low_modes.txt); the solve runs at 0.133"),
                   "dims": list(dims), "block": list(block), "kappa": args.kappa, "csw": args.csw, "eps": args.eps,
                   "n_sap": args.n_sap, "n_jac": args.n_jac, "tol": args.tol, "inner_tol": args.inner_tol,
                   "precision": "FP16 SAP / FP32 BiCGStab / FP64 defect correction",
                   "sap_fp16_arith": args.sap_fp16_arith, "parallelism": "single GPU"},
        "solve_mixed": {"seconds": round(ms_step / 1e3, 3), "iters_outer": infos[-1]["iters_outer"],
                        "iters_inner": infos[-1]["iters_inner_total"],
                        "relres_true": infos[-1]["relres_true"], "status": infos[-1]["status"],
                        "history": {k: [float(f"{v:.3e}") for v in h] for k, h in hist.items()}},
        "kernels": {k: {kk: (round(vv, 4) if isinstance(vv, float) else vv) for kk, vv in v.items()}
                    for k, v in kernels.items()},
        "dirac_apply": {k: {kk: round(vv, 3) for kk, vv in v.items()} for k, v in micro.items()},
        "roofline": roof,
        "roofline_dirac": roof_dirac,
    }
    # the flexible outer loop (flexible GMRES around the same inner solver) on the same system,
    # after the timed steps: a first solve allocates its extra fields, the second is reported
    for rep in range(2):
        xf, inf_f = solver.solve(b, tol=args.tol, maxiter=50, mode=dd.DD_SOLVE_FGMRES)
    log(f"flexible GMRES: {inf_f['status']} {inf_f['seconds']:.2f} s, outer {inf_f['iters_outer']}, "
        f"inner {inf_f['iters_inner_total']}, true residual {inf_f['relres_true']:.2e}")
    result["solve_fgmres"] = {"seconds": round(inf_f["seconds"], 3), "iters_outer": inf_f["iters_outer"],
                              "iters_inner": inf_f["iters_inner_total"], "relres_true": inf_f["relres_true"],
                              "status": inf_f["status"],
                              "vs_defect_correction": round(inf_f["seconds"] / (ms_step / 1e3), 3),
                              "solution_relerr_vs_defect_correction":
                                  (torch.linalg.vector_norm(xf - x) / torch.linalg.vector_norm(x)).item()}
    del xf

    # the practical streaming ceiling of this GPU, measured beside the 8 TB/s peak
    hbm = measured_hbm()
    best = max(hbm.values())
    hbm["value_frac_of_best_measured"] = round(value / best, 4)
    hbm["note"] = "torch copy (1 read + 1 write) and add (2 reads + 1 write) over 2 GiB, HIP events"
    result["hbm_measured"] = hbm
    log(f"measured streaming bandwidth: copy {hbm['copy_GBps']} GB/s, add {hbm['add_GBps']} GB/s; "
        f"Dirac value = {hbm['value_frac_of_best_measured']:.3f} of the better")
    if force is not None:
        result["force"] = force
    if batch is not None:
        result["batch"] = batch
    if multi is not None:
        result["multi"] = multi
    if single is not None:
        result["single_prec_32x32x32x32"] = single

    # ---- plain FP64 BiCGStab on the same system (speedup denominator), once
    if args.fp64 == "on":
        log(f"plain FP64 BiCGStab, at most {args.fp64_maxiter} iterations")
        x64, i64 = solver.solve(b, tol=args.tol, maxiter=args.fp64_maxiter, mode=dd.DD_SOLVE_F64_PLAIN)
        log(f"plain FP64: {i64['status']} {i64['seconds']:.1f} s, {i64['iters_inner_total']} iterations, "
            f"true residual {i64['relres_true']:.2e}")
        conv = i64["status"] == "DD_OK"
        # error of the mixed solution against the FP64 one (relative L2)
        err = (torch.linalg.vector_norm(x - x64) / torch.linalg.vector_norm(x64)).item() if conv else None
        result["solve_fp64_plain"] = {"seconds": round(i64["seconds"], 3), "iters": i64["iters_inner_total"],
                                      "relres_true": i64["relres_true"], "status": i64["status"],
                                      "converged": conv}
        sp = i64["seconds"] / (ms_step / 1e3)
        result["speedup_mixed_vs_fp64"] = round(sp, 2) if conv else None
        if not conv:
            result["speedup_mixed_vs_fp64_lower_bound"] = round(sp, 2)
        result["mixed_vs_fp64_solution_relerr"] = err
        del x64

    if args.cpu_baseline == "on":
        log("timing the FP64 CPU oracle on bounded samples (D apply on 32^4, solves on 4^4 and 16^4, "
            "iterations on 32^4)")
        gpu_iters = {}
        if "solve_fp64_plain" in result and result["solve_fp64_plain"]["converged"] and args.kappa == 0.133:
            gpu_iters["64x64x64x128"] = result["solve_fp64_plain"]["iters"]
        gpu_iters["32x32x32x32"] = gpu_plain_iters_32(dd, args)
        result["cpu_baseline"] = cpu_baseline(gpu_iters)
    print(json.dumps(result))


if __name__ == "__main__":
    main()
