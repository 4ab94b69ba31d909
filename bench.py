"""Throughput of the selected density matrix on one MI355X.

    python bench.py [--steps K] [--warmup W] [--workload cubic3d_24x4] [--no-cpu-baseline]

A step is one ndrho_density_matrix call: all poles of the workload through
the whole path (assembly, upward block LDL^T over the dissection tree,
downward selected inversion, pole sum), with H, S, the plan and the poles
already resident on the device and rho written to a device buffer.
Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_MFMA_PEAK_TFLOPS = 78.6   # MI355X dense FP64 matrix peak
FP32_MFMA_PEAK_TFLOPS = 157.3  # MI355X dense FP32 matrix peak
BF16_MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense BF16 matrix peak
# split-BF16 front updates execute 4 real products x 6 slice products of 2
# flops per complex multiply-add, for 8 useful flops
BF16X3_EXEC_PER_USEFUL = 48.0 / 8.0
HBM_PEAK_GBS = 8000.0

WORKLOADS = {
    "multi2d_8x4": "8 uneven 2D lattices {32,40,48,56,64,72,80,96}^2 x 4, nn, one schedule, 100 poles",
    "chain1d_256x4": "1D chain 256 sites x 4 orbitals, nearest neighbours, N=1024, 60 poles",
    "square2d_64x4": "2D square lattice 64x64 sites x 4 orbitals, nn + 2nd neighbours, N=16384, 80 poles",
    "cubic3d_24x4": "3D cubic lattice 24^3 sites x 4 orbitals, nearest neighbours, N=55296, 80 poles",
    "cubic3d_40x4": "3D cubic lattice 40^3 sites x 4 orbitals, nn + 2nd neighbours, N=256000, 100 poles",
}

# Shifts kept in FP64 at each end of the pole list (nearest and farthest from
# the real axis) in the mixed forms, as measured against the complex128 result
# of the same input (bar 1e-7): 24^3 x 4 keeps 4 + 4 (6.6e-8; 2 + 2 leaves
# 8.8e-8, 8 + 8 3.1e-8); 40^3 x 4 needs 12 + 12 (8 + 8 leaves 1.03e-7, 12 + 12
# 8.4e-8); the others meet it with the library default of 8 + 8.
FP64_POLES = {"cubic3d_24x4": 4, "cubic3d_40x4": 12}
HEADLINE_METRIC = "poles/sec (selected inversion) on 3D 24^3x4 at 1e-7 rho error; MFMA TFLOP/s"


def cpu_baseline(sysd, mu, beta, n_poles, budget_s=20.0):
    """The oracle timed on the host's cores (BLAS threads = all cores): its
    per-pole dense route (one complex128 inverse of alpha_p S - H per pole,
    oracle.dense.green_dense) and its eigen route (generalized eigensolve,
    oracle.dense.eigen, at the sizes half the budget allows) are timed on
    lattices of the same kind at n = 1024, 2048, 4096 (one pole each, while
    the budget lasts), fitted as c n^3 and extrapolated to the
    workload's n (the dense matrix of the workload itself does not fit the
    host at the 3D sizes).  poles/s = 1 / (extrapolated seconds per pole)."""
    import platform
    import subprocess
    from oracle import dense, poles
    from synth import lattice
    try:
        import threadpoolctl
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info if i.get("user_api") == "blas"] or [1])
        blas = ", ".join(sorted({"%s %s" % (i.get("internal_api"), i.get("version")) for i in info
                                 if i.get("user_api") == "blas"}))
    except Exception:
        threads, blas = os.cpu_count() or 1, "unknown"
    try:
        model = [l.split(":", 1)[1].strip() for l in subprocess.run(["lscpu"], capture_output=True, text=True,
                                                                   timeout=10).stdout.splitlines()
                 if l.startswith("Model name")][0]
    except Exception:
        model = platform.processor() or "unknown"
    dims = sysd["dims"]
    ndim = sum(1 for d in dims if d > 1)
    shapes = {1: [(256,), (512,), (1024,)], 2: [(16, 16), (32, 16), (32, 32)], 3: [(8, 8, 4), (8, 8, 8), (16, 8, 8)]}
    z, _ = poles.cf_poles(n_poles)
    alpha = mu + 1j * z[0] / beta
    t_pole, t_eig, ns, ns_eig = [], [], [], []
    t0 = time.time()
    for shp in shapes[ndim]:
        small = lattice(shp, sysd.get("neighbours", "nn"), 7)
        h, s = _dense_pair(small)
        a = time.perf_counter()
        dense.green_dense(h, s, alpha)
        ns.append(small["n"])
        t_pole.append(time.perf_counter() - a)
        if time.time() - t0 < 0.5 * budget_s:   # the eigen route at the sizes the budget allows
            a = time.perf_counter()
            dense.eigen(h, s)
            ns_eig.append(small["n"])
            t_eig.append(time.perf_counter() - a)
        if time.time() - t0 > budget_s:
            break
    ns, ns_eig = np.asarray(ns, dtype=float), np.asarray(ns_eig, dtype=float)
    # least squares fit of t = k n^3 on the measured sizes (the largest weigh most)
    k_pole = float(np.sum(np.asarray(t_pole) * ns ** 3) / np.sum(ns ** 6))
    k_eig = float(np.sum(np.asarray(t_eig) * ns_eig ** 3) / np.sum(ns_eig ** 6))
    n_big = float(sysd["n"])
    sec_pole = k_pole * n_big ** 3
    return {"value": 1.0 / sec_pole, "unit": "poles/s", "cores": int(threads), "kind": "oracle",
            "sample": "oracle per-pole dense route (complex128 inverse of alpha S - H, one pole) timed at n = %s "
                      "(%s s) on %d BLAS threads, fitted as k n^3 and extrapolated to n = %d: %.3g s per pole; "
                      "eigen route (generalized eigensolve) %s s at n = %s, extrapolated %.3g s"
                      % ([int(x) for x in ns], [round(x, 3) for x in t_pole], threads, int(n_big), sec_pole,
                         [round(x, 3) for x in t_eig], [int(x) for x in ns_eig], k_eig * n_big ** 3),
            "extrapolated": True, "nproc": os.cpu_count(), "lscpu_model": model, "blas": blas,
            "eigen_route_s_extrapolated": k_eig * n_big ** 3}


def _dense_pair(sysd):
    n = sysd["n"]
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))
    h = np.zeros((n, n))
    s = np.zeros((n, n))
    h[rows, sysd["col"]] = sysd["h"]
    s[rows, sysd["col"]] = sysd["s"]
    return h, s


def measured_traffic(name, precision):
    """HBM bytes per launch of the dominant kernel from the committed counter
    summary (calibrated FETCH_SIZE + WRITE_SIZE), or None when it is missing
    or the kernels have changed since it was taken."""
    import hashlib
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (name, precision))
    if not os.path.exists(path):
        return None
    with open(path) as f:
        t = json.load(f)
    with open(os.path.join(ROOT, "paper_1005_0088_amd", "csrc", "kernels.hip"), "rb") as f:
        sha = hashlib.sha256(f.read()).hexdigest()[:16]
    if sha != t["kernels_hip_sha256_16"]:
        return None
    return t["read_bytes_per_launch"] + t["write_bytes_per_launch"]


def golden_error(name, rho, mu, n_poles):
    path = os.path.join(ROOT, "tests", "golden", "rho_sampled_%s.json" % name)
    if not os.path.exists(path):
        return None
    with open(path) as f:
        g = json.load(f)
    if g["mu"] != mu or g["n_poles"] != n_poles:
        return None
    return float(np.max(np.abs(rho[np.asarray(g["entries"])] - np.asarray(g["values"]))))


def run_form(nd, systems, mu, beta, n_poles, steps, warmup, precision, fp64_poles, autotune=True, gemm_variant=-1,
             tune_cache=None, split_streams=1, energy=False, small_fronts=0, pivot_variant=0):
    """Time one precision form on one system (density_matrix, or with
    energy=True energy_density_matrix: rho and e) or several
    (density_matrix_batch: one schedule); returns (timing dict, rho list)."""
    variant = gemm_variant if precision != "fp64" else -1
    ctx = nd.Context(0, precision=precision, fp64_poles=fp64_poles, fp64_far_poles=fp64_poles, gemm_variant=variant,
                     split_streams=split_streams, verbose=1, small_fronts=small_fronts,
                     pivot_variant=pivot_variant if precision != "fp64" else -1)
    t0 = time.time()
    sids = []
    for sysd in systems:
        sid = ctx.set_structure(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"], sysd["coords"],
                                cell=sysd.get("cell"))
        ctx.set_poles(sid, mu, beta, n_poles)
        sids.append(sid)
    register_s = time.time() - t0   # dissection, symbolic analysis, upload and M0 of every structure
    if precision != "fp64" and autotune and variant < 0:
        ctx.autotune(sids, tune_cache)   # per-launch GEMM variant (untimed set-up, like the plan)
    outs = [ctx.device_buffer(int(sysd["row_ptr"][-1])) for sysd in systems]
    multi = len(systems) > 1
    e_out = ctx.device_buffer(int(systems[0]["row_ptr"][-1])) if energy else None

    def step():
        if multi:
            ctx.density_matrix_batch(sids, outs)
        elif energy:
            ctx.energy_density_matrix(sids[0], outs[0], e_out)
        else:
            ctx.density_matrix(sids[0], outs[0])

    if energy:
        if multi:
            raise SystemExit("--energy runs on single-structure workloads")
        step()   # first call: the first moment M1 of the structure (set-up, like M0)
    setup_s = time.time() - t0

    for i in range(warmup):
        step()
    # every density_matrix call ends with a stream synchronisation (it reads
    # the pivot status), so the host clock brackets complete device work
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    dt = time.perf_counter() - t0
    st = [ctx.stats(s) for s in sids]
    # one instrumented step: per-kind kernel time from HIP events on the library's stream
    ctx.profile(True)
    step()
    prof = ctx.profile_read()
    by_depth = ctx.profile_read_depth()
    phases = ctx.phase_stats()
    ctx.profile(False)
    rho = [o.numpy() for o in outs]
    for o in outs:
        o.free()
    e_vals = None
    if energy:
        e_vals = e_out.numpy()
        e_out.free()
    ctx.close()
    res = {"precision": precision, "setup_s": setup_s, "register_s": register_s, "ms_per_step": 1e3 * dt / steps,
           "e": e_vals,
           "phases": phases,
           "poles_per_s": n_poles * steps / dt, "stats": st, "prof": prof,
           "ms_by_depth": {k: [round(float(x), 3) for x in v] for k, v in by_depth.items() if v.any()},
           "flops_model_per_step": n_poles * sum(x["flops_per_pole"] for x in st)}
    print("bench: %s %.1f ms/step" % (precision, res["ms_per_step"]), file=sys.stderr, flush=True)
    return res, rho


def mu_search(nd, sysd, name, n_poles, args, beta):
    """One chemical-potential search at half filling (N electrons in N basis
    functions) from args.find_mu, in the given precision form; prints one JSON line."""
    fp = args.fp64_poles if args.fp64_poles is not None else FP64_POLES.get(name, 8)
    with nd.Context(0, precision=args.precision, fp64_poles=fp, fp64_far_poles=fp) as ctx:
        sid = ctx.set_structure(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"], sysd["coords"])
        ctx.set_poles(sid, args.find_mu, beta, n_poles)
        if args.precision != "fp64" and not args.no_autotune:
            ctx.autotune([sid], args.tune_cache)
        ctx.density_matrix(sid)   # untimed: workspace allocation and graph capture, as for the other timings
        t0 = time.perf_counter()
        mu, dn, it, rho = ctx.find_mu(sid, float(sysd["n"]), beta, n_poles, mu0=args.find_mu, tol=1e-8,
                                      retarded_step=args.retarded_step)
        dt = time.perf_counter() - t0
    print(json.dumps({"metric": "chemical-potential search", "value": dt, "unit": "s", "higher_is_better": False,
                      "n_gpus": 1, "dtype": {"fp64": "f64", "mixed_fp32": "f64+f32",
                                             "mixed_bf16x3": "f64+bf16x3"}[args.precision],
                      "data": "synthetic",
                      "config": {"workload": name, "n": sysd["n"], "n_poles": n_poles, "n_ideal": sysd["n"],
                                 "mu0_eV": args.find_mu, "tol_electrons": 1e-8, "precision": args.precision,
                                 "retarded_step": bool(args.retarded_step)},
                      "mu_eV": mu, "delta_n": dn, "evaluations": it, "s_per_evaluation": dt / max(1, it)}))


def eigen_run(nd, sysd, name, args):
    """The k eigenpairs nearest args.eigenstates by block shift-invert
    (ndrho_eigenstates, Appendix B), timed once after one untimed call (the
    plan and the kernels warm); prints one JSON line.  At full size no dense
    eigensolve is in reach, so the pairs are checked on the host by properties
    that hold at any size: ||H c - eps S c|| recomputed from the CSR matrices
    and the S-orthonormality of the vectors."""
    k, eta, tol = args.eig_k, 1e-3, 1e-8
    with nd.Context(0, precision="fp64") as ctx:
        sid = ctx.set_structure(sysd["n"], sysd["row_ptr"], sysd["col"], sysd["h"], sysd["s"], sysd["coords"])
        ctx.eigenstates(sid, args.eigenstates, k, eta=eta, max_iter=args.eig_iter, tol=tol, vectors=False)
        t0 = time.perf_counter()
        eps, c, it, res = ctx.eigenstates(sid, args.eigenstates, k, eta=eta, max_iter=args.eig_iter, tol=tol)
        dt = time.perf_counter() - t0
    n = sysd["n"]
    rows = np.repeat(np.arange(n), np.diff(sysd["row_ptr"]))

    def csr_mul(vals, x):   # y = A x for the CSR values of H or S
        y = np.zeros_like(x)
        np.add.at(y, rows, vals[:, None] * x[sysd["col"]])
        return y

    hc, sc = csr_mul(sysd["h"], c), csr_mul(sysd["s"], c)
    host_res = np.linalg.norm(hc - sc * eps[None, :], axis=0)
    ortho = float(np.max(np.abs(c.T @ sc - np.eye(k))))
    print(json.dumps({"metric": "selected eigenstates (block shift-invert)", "value": dt, "unit": "s",
                      "higher_is_better": False, "n_gpus": 1, "dtype": "f64", "data": "synthetic",
                      "config": {"workload": name, "n": n, "xi_eV": args.eigenstates, "eta_eV": eta, "k": k,
                                 "tol": tol, "max_iter": args.eig_iter},
                      "iterations": it, "s_per_iteration": dt / max(1, it),
                      "eigenvalues_eV": [float(x) for x in eps],
                      "max_residual_library": float(np.max(res)), "max_residual_host": float(np.max(host_res)),
                      "max_abs_CtSC_minus_I": ortho}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="cubic3d_24x4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="mixed_bf16x3", choices=["mixed_bf16x3", "mixed_fp32", "fp64"],
                    help="form of the headline number")
    ap.add_argument("--fp64-poles", type=int, default=None,
                    help="shifts kept FP64 at each end of the pole list (default: 8, 12 for cubic3d_40x4)")
    ap.add_argument("--forms", default="all", choices=["all", "both", "head"],
                    help="all: every precision form (FP64 is the complex128 reference of the error); "
                         "both: --precision and FP64; head: only --precision")
    ap.add_argument("--copy-calibration", type=float, default=0.0, metavar="GIB",
                    help="only run the plain copy kernel over GIB gibibytes (HBM counter calibration) and exit")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default per-launch GEMM variants")
    ap.add_argument("--tune-cache", default=None, help="autotuner cache file (read and appended)")
    ap.add_argument("--gemm-variant", type=int, default=-1,
                    help="force one GEMM variant on every low-precision front update (see ndrho_options)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--find-mu", type=float, default=None, metavar="MU0",
                    help="time the chemical-potential search (Tr(rho S) = N, half filling) from MU0 instead")
    ap.add_argument("--retarded-step", action="store_true",
                    help="with --find-mu: take the second trial from the retarded Green function")
    ap.add_argument("--energy", action="store_true",
                    help="time energy_density_matrix (rho and the energy density matrix e of the same poles)")
    ap.add_argument("--split-streams", type=int, default=0,
                    help="mixed forms: launch chains beside the main one (default 0: one captured chain, so that "
                         "the kernels' durations in the timed steps are those of the instrumented step and of "
                         "the profiler's trace; 1 runs the FP64 poles beside, about 1 %% faster on 24^3 x 4)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--pivot-variant", type=int, default=0,
                    help="mixed forms: GEMM variant of the low poles' pivot-inverse products (0: FP64, the "
                         "default; -1: per-launch choice; see ndrho_options.pivot_variant)")
    ap.add_argument("--small-fronts", type=int, default=0, choices=[0, 1],
                    help="1: the small fronts of the deep levels run in fused launches (one per depth and "
                         "direction, one workgroup per front and pole)")
    ap.add_argument("--periodic", action="store_true",
                    help="close the workload's lattice into a periodic cell (Sec. II C 1, step (i)); the stored "
                         "oracle samples are of the open lattices, so the line then carries no oracle error")
    ap.add_argument("--eigenstates", type=float, default=None, metavar="XI",
                    help="time the eigenpairs nearest XI eV by block shift-invert (Appendix B) instead")
    ap.add_argument("--eig-k", type=int, default=8, help="with --eigenstates: number of eigenpairs (1..16)")
    ap.add_argument("--eig-iter", type=int, default=300, help="with --eigenstates: iteration limit")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library runs the whole hot path on a single MI355X "
              "(--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import paper_1005_0088_amd as nd
    from synth import BETA, CONFIGS, config_system

    if args.copy_calibration > 0:
        n = int(args.copy_calibration * (1 << 30)) // 8
        with nd.Context(0) as ctx:
            a, b = ctx.device_buffer(n), ctx.device_buffer(n)
            for _ in range(3):
                t0 = time.perf_counter()
                b.copy_from(a)
                dt = time.perf_counter() - t0
            print(json.dumps({"copy_bytes": 8 * n, "read_bytes": 8 * n, "write_bytes": 8 * n,
                              "launches": 3, "GBs_read_plus_write": 2 * 8 * n / dt / 1e9}))
            a.free()
            b.free()
        return

    name = args.workload
    n_poles = CONFIGS[name]["n_poles"]
    if args.find_mu is not None:
        mu_search(nd, config_system(name), name, n_poles, args, BETA)
        return
    if args.eigenstates is not None:
        if name == "multi2d_8x4":
            raise SystemExit("--eigenstates runs on single-structure workloads")
        eigen_run(nd, config_system(name), name, args)
        return
    if args.fp64_poles is None:
        args.fp64_poles = FP64_POLES.get(name, 8)
    mu = 0.0
    if name == "multi2d_8x4":
        systems = [config_system(name, i, args.periodic) for i in range(len(CONFIGS[name]["dims"]))]
    else:
        systems = [config_system(name, periodic=args.periodic)]
    gname = name + "_periodic" if args.periodic else name   # no stored sample or counters for periodic cells
    n = sum(x["n"] for x in systems)
    nnz = sum(int(x["row_ptr"][-1]) for x in systems)
    print("bench: %s structures=%d n=%d nnz=%d poles=%d" % (name, len(systems), n, nnz, n_poles), file=sys.stderr,
          flush=True)

    # the plain FP64 form is the complex128 reference of the error
    r64 = rho64 = None
    if args.forms != "head" or args.precision == "fp64":
        r64, rho64 = run_form(nd, systems, mu, BETA, n_poles, args.steps, args.warmup, "fp64", 0,
                              energy=args.energy, small_fronts=args.small_fronts)
    others = {}
    if args.forms == "all":
        for form in ("mixed_fp32", "mixed_bf16x3"):
            if form != args.precision:
                r, rr = run_form(nd, systems, mu, BETA, n_poles, args.steps, args.warmup, form, args.fp64_poles,
                                 not args.no_autotune, -1, args.tune_cache, args.split_streams, args.energy,
                                 args.small_fronts, args.pivot_variant)
                others[form] = {
                    "poles_per_s": r["poles_per_s"], "ms_per_step": r["ms_per_step"],
                    "kernel_ms": {k: round(v["ms"], 3) for k, v in r["prof"].items()},
                    "max_abs_err_vs_complex128": max(float(np.max(np.abs(a - b))) for a, b in zip(rr, rho64)),
                    "max_abs_err_vs_oracle_sample": golden_error(gname, rr[0], mu, n_poles) if len(rr) == 1 else None,
                    "max_abs_err_e_vs_complex128": (float(np.max(np.abs(r["e"] - r64["e"]))) if args.energy
                                                    else None)}
    if args.precision == "fp64":
        head, rho = r64, rho64
    else:
        head, rho = run_form(nd, systems, mu, BETA, n_poles, args.steps, args.warmup, args.precision,
                             args.fp64_poles, not args.no_autotune, args.gemm_variant, args.tune_cache,
                             args.split_streams, args.energy, args.small_fronts, args.pivot_variant)
    st, prof = head["stats"][0], head["prof"]
    # dominant kernel: the FP64 front GEMMs in the FP64 form, the FP32-product
    # front GEMMs in the mixed form (peak of their own arithmetic)
    exec_per_useful = 1.0
    if head["precision"] == "fp64":
        g, peak, kname = prof["gemm"], FP64_MFMA_PEAK_TFLOPS, "k_zgemm (complex FP64 front-update GEMMs)"
    elif head["precision"] == "mixed_bf16x3":
        g, peak, kname = (prof["gemm_bf16x3"], BF16_MFMA_PEAK_TFLOPS,
                          "k_cgemm_bf3, k_cgemm_bf3s, k_cgemm_bf3p, k_cgemm_bf3w (complex front-update GEMMs, split-BF16 "
                          "products; achieved on useful flops, executed BF16 flops beside)")
        exec_per_useful = BF16X3_EXEC_PER_USEFUL
    else:
        g, peak, kname = prof["gemm_f32"], FP32_MFMA_PEAK_TFLOPS, "k_cgemm32 (complex front-update GEMMs, FP32 products)"
    useful = g["flops"] / (g["ms"] * 1e-3) / 1e12 if g["ms"] > 0 else 0.0
    gemm_tf = {k: (v["flops"] / (v["ms"] * 1e-3) / 1e12 if v["ms"] > 0 else 0.0)
               for k, v in prof.items() if k.startswith("gemm")}
    alg_bytes_per_launch = g["bytes"] / max(1, g["launches"])
    traffic = measured_traffic(gname, head["precision"])

    line = {
        "metric": (HEADLINE_METRIC if gname == "cubic3d_24x4" else
                   "poles/sec (selected inversion) on %s; MFMA TFLOP/s" % gname),
        "value": head["poles_per_s"],
        "unit": "poles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": {"fp64": "f64", "mixed_fp32": "f64+f32", "mixed_bf16x3": "f64+bf16x3"}[head["precision"]],
        "data": "synthetic",
        "config": {"workload": gname, "description": WORKLOADS[name] + (", periodic cell" if args.periodic else ""),
                   "structures": len(systems), "n": n,
                   "nnz": nnz, "n_poles": n_poles, "kT_eV": 1.0 / BETA, "mu_eV": mu,
                   "mu_rule": "fixed at 0 eV for every workload (H is drawn symmetric about 0; on the 24^3 x 4 "
                              "lattice the half-filling mu from ndrho_find_mu is -0.0037 eV)",
                   "precision": head["precision"],
                   "fp64_poles": st["n_fp64_poles"], "fronts": sum(x["n_fronts"] for x in head["stats"]),
                   "levels": max(x["n_levels"] for x in head["stats"]), "root_j": st["root_j"],
                   "pole_batch": st["pole_batch"], "seeds": [int(x["seed"]) for x in systems],
                   "small_fronts": args.small_fronts, "pivot_variant": args.pivot_variant,
                   "neighbours": systems[0]["neighbours"]},
        "pole_structures_per_s": head["poles_per_s"] * len(systems),
        "tflops_model": head["flops_model_per_step"] / (head["ms_per_step"] * 1e-3) / 1e12,
        "max_abs_err_vs_complex128": (max(float(np.max(np.abs(a - b))) for a, b in zip(rho, rho64))
                                      if rho64 is not None else None),
        "max_abs_err_vs_oracle_sample": golden_error(gname, rho[0], mu, n_poles) if len(rho) == 1 else None,
        # electron count Tr(rho S) (Eq. (40)) from the pattern values, against N (half filling); mu is fixed,
        # so the difference is the distance of that mu from half filling, not an error
        "trace_rho_s_minus_n": [float(np.dot(r, x["s"]) - x["n"]) for r, x in zip(rho, systems)],
        "energy_density": None if not args.energy else {
            "computed": "rho and e (Eq. (10)) from the same poles in every timed step",
            "max_abs_e": float(np.max(np.abs(head["e"]))),
            "max_abs_err_e_vs_complex128": (float(np.max(np.abs(head["e"] - r64["e"])))
                                            if r64 is not None and head is not r64 else None)},
        "fp64_form": None if r64 is None else {
            "poles_per_s": r64["poles_per_s"], "ms_per_step": r64["ms_per_step"],
            "tflops_model": r64["flops_model_per_step"] / (r64["ms_per_step"] * 1e-3) / 1e12,
            "gemm_tflops": r64["prof"]["gemm"]["flops"] / (r64["prof"]["gemm"]["ms"] * 1e-3) / 1e12,
            "kernel_ms": {k: round(v["ms"], 3) for k, v in r64["prof"].items()},
            "max_abs_err_vs_oracle_sample": golden_error(gname, rho64[0], mu, n_poles) if len(rho64) == 1 else None},
        "other_forms": others,
        "kernel_ms": {k: round(v["ms"], 3) for k, v in prof.items()},
        "kernel_ms_by_depth": head["ms_by_depth"],
        "gemm_tflops": gemm_tf,
        "roofline": {"kernel": kname, "bound": "mfma",
                     "achieved": useful, "peak": peak, "unit": "TFLOP/s",
                     "frac": useful / peak,
                     "achieved_counts": "useful complex flops (8 per complex multiply-add) per launch / average "
                                        "launch duration (HIP events on the launching stream)",
                     "executed_tflops": useful * exec_per_useful, "executed_frac": useful * exec_per_useful / peak,
                     "traffic": traffic,
                     "traffic_unit": "bytes per launch (calibrated HBM read + write, timed launch mix)",
                     "algorithmic_bytes_per_launch": alg_bytes_per_launch,
                     "traffic_over_algorithmic": (traffic / alg_bytes_per_launch
                                                  if traffic and alg_bytes_per_launch > 0 else None),
                     "launches": g["launches"], "avg_launch_ms": g["ms"] / max(1, g["launches"]),
                     "flops_per_step": g["flops"]},
        "ms_per_phase": head["phases"]["ms_per_phase"],
        # set-up outside the timed steps: registration (dissection, symbolic analysis, upload, M0) and the
        # whole set-up including the autotuner (and, with --energy, the first moment M1)
        "setup_s": {"register": head["register_s"], "total": head["setup_s"]},
    }
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(systems[-1], mu, BETA, n_poles, args.cpu_seconds)
    print(json.dumps(line))


if __name__ == "__main__":
    main()
