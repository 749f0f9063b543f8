"""Benchmark: Hessian applies per second on the largest single-GPU workload.

Headline workload (mesh1024_nt1000): the 1024 x 1024 mesh (nx = 1,046,529
interior nodes), nt = 1000 implicit-Euler steps, alpha = sigma = 1e-2,
observation box [0.25, 0.75]^2, truncation tolerance 1e-6, factor rank <= 128,
mixed precision (float32 stencil and multigrid, float64 refinement,
projections, truncations and Lanczos matrix).  A step is one pass of the hot
path over it: block-Lanczos iterations for the k = 100 leading eigenpairs of
the prior-preconditioned misfit Hessian, stopped at a fixed budget of Krylov
vectors (--vectors, default 40, i.e. 10 block steps of 4 applies; every
Krylov vector a low-rank space-time vector, every apply a forward and an
adjoint low-rank space-time solve plus a prior solve), then the Ritz pairs
reached and the posterior variance diag(Gamma_post) over all nx * nt = 1.05e9
space-time points from them.  A full 100-pair posterior at this size takes
several minutes, so the step budget is in vectors; value counts the applies
completed.  Inputs are synthetic (seeded start block), generated inside the
library and resident in HBM when the timed region starts.

value = Hessian applies completed in the timed steps / timed seconds.  After
the mixed steps the same step runs in float64; its throughput and the mixed
result's relative error against it (Ritz values and posterior variance) are
reported under "fp64_reference".  "mesh256_posterior" reports a complete
50-pair posterior on the 256 x 256 mesh, nt = 200 workload (applies/s and the
posterior latency).  "cpu_baseline" times the float64 oracle's apply on a
bounded sample of the headline workload.
Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
[--precision mixed|fp64] [--vectors V] [--serving R] [--randomized]
"""
import argparse
import json
import os
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X published HBM3E bandwidth
COPY_BYTES = 256 << 20  # calibration copy for the HBM byte counters, each way
# Kernels timed with HIP events (kind as in the library's LRPOST_KERNEL_*):
# name, description, whether the name takes the precision of the V-cycles
# (float32 in mixed precision), and the matrix-core peak of the kernel's
# contraction dtype in TFLOP/s (None: no contraction).
MFMA_F64_PEAK_TFLOPS = 78.6   # MI355X published dense FP64 matrix throughput
MFMA_F32_PEAK_TFLOPS = 157.3  # MI355X published dense FP32 matrix throughput
KERNELS = {
    0: ("k_cheb", "multigrid Chebyshev smoother step", True, None),
    1: ("k_mg_down", "level-fused pre-smoothing + residual + restriction", True, None),
    2: ("k_mg_up", "level-fused prolongation + post-smoothing", True, None),
    3: ("k_gram_mfma", "float64 matrix-core Gram A^T B, partial products", False, MFMA_F64_PEAK_TFLOPS),
    4: ("k_proj_mfma", "float64 matrix-core projection C = beta C + A Q", False, MFMA_F64_PEAK_TFLOPS),
    5: ("k_stencil_strip", "Q1 stencil SpMM a K x + b M x (+ c z), all columns per launch", True, None),
    6: ("k_gram_f32", "float32 matrix-core Gram A^T B (first Gram-Schmidt sweep), partial products", False,
        MFMA_F32_PEAK_TFLOPS),
    7: ("k_proj_grouped_f32", "float32 matrix-core projection (first Gram-Schmidt sweep)", False,
        MFMA_F32_PEAK_TFLOPS),
}


def measured_rates():
    """The float64 rates this device reaches on one instruction stream with
    operands in registers (the matrix-core instruction of the float64 kernels
    and the vector FMA), measured outside the timed region: context for the
    published peak, not a ceiling (a kernel that keeps more products in
    flight per SIMD can exceed the matrix-core figure)."""
    from paper_1703_05638_amd import lrpost
    return {"register_stream_fp64_TFLOPs": lrpost.measure_fp64_rates()}


def traffic_report(kernel, precision, workload):
    # the multigrid kernels run in float32 in mixed precision, the Gram always in float64
    f32 = precision == "mixed" and KERNELS[[k for k in KERNELS if KERNELS[k][0] == kernel][0]][2]
    tag = "f32_" if f32 else ""
    suffix = "_mixed" if precision == "mixed" else ""
    return os.path.join(ROOT, "profiles", "%s_%s%s%s_traffic.txt" % (kernel, tag, workload, suffix))


def cpu_baseline(desc, sample_steps=16):
    """The FP64 oracle's Hessian apply G (implicit-Euler time stepping with a
    sparse LU of M + tau K, observation, backward adjoint stepping, sparse-LU
    prior solve) on the headline mesh and time step, timed on the host over
    the first sample_steps of the nt time steps (the per-step work does not
    depend on the step) and scaled by nt / sample_steps.  The LU factors are
    computed before the timed region."""
    import dataclasses

    import numpy as np
    from oracle.spacetime import Problem as OracleProblem

    short = dataclasses.replace(desc, nt=sample_steps, T=desc.T * sample_steps / desc.nt)
    ora = OracleProblem.from_desc(short)
    rng = np.random.default_rng(1)
    A = rng.standard_normal((ora.nx, 20))
    B = np.cumsum(rng.standard_normal((ora.nt, 20)), axis=0) / np.sqrt(ora.nt)
    X = A @ B.T
    t0 = time.perf_counter()
    ora.G(X)
    dt = time.perf_counter() - t0
    per_apply = dt * desc.nt / sample_steps
    return {"value": 1.0 / per_apply, "unit": "Hessian applies/s", "cores": 1, "kind": "oracle",
            "sample": "one full FP64 G-apply of the oracle on a rank-20 space-time input over the first %d of "
                      "the %d time steps (same %dx%d mesh and tau), %.1f s, scaled by %d; SuperLU factors "
                      "built beforehand, single-threaded" % (sample_steps, desc.nt, desc.N, desc.N, dt,
                                                             desc.nt // sample_steps)}


def serving(args):
    """Replay the first --serving requests of the seeded Poisson request stream
    (20 req/s; mesh side 64/128/256, nt 50/100/200, k = 30 eigenpairs plus the
    posterior variance, tol 1e-6, rank <= 64) through the serving loop (workers
    with resident problems per size class, memory admission), then run the
    same requests one after another on one stream, each on a new problem in
    float64 (the plain FP64 path), and report latency percentiles, throughput
    and the speedup.  The served requests run in --precision (mixed by
    default)."""
    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    import dataclasses
    reqs = synthetic.serving_stream()[: args.serving]
    srv = lp.Server(hbm_budget_bytes=200 << 30, workers=args.workers)
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(dataclasses.replace(r.desc, precision=args.precision), r.desc.k))
    lat = []
    for i, t in enumerate(tickets):
        lat.append(srv.wait(t)[2])
        print("request %d done (latency %.2f s)" % (i, lat[-1]), file=sys.stderr, flush=True)
    t_serve = time.perf_counter() - t0
    info = srv.info()
    srv.close()
    t1 = time.perf_counter()
    for i, r in enumerate(reqs):
        prob = lp.Problem(r.desc)
        eig = prob.eigensolve(r.desc.k)
        prob.post_variance(eig, on_device=False)
        del eig, prob
        print("sequential request %d done" % i, file=sys.stderr, flush=True)
    t_seq = time.perf_counter() - t1
    lat_sorted = sorted(lat)
    out = {
        "metric": "posterior requests served: p50/p99 latency",
        "value": len(reqs) / t_serve, "unit": "requests/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic", "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "config": {"workload": "poisson20_mesh64-256_nt50-200_k30", "requests": len(reqs), "workers": args.workers,
                   "hbm_budget_gb": 200, "precision": args.precision},
        "latency_s": {"p50": statistics.median(lat),
                      "p99": lat_sorted[min(len(lat) - 1, int(0.99 * len(lat)))]},
        "makespan_s": t_serve, "sequential_fp64_s": t_seq, "speedup_vs_sequential": t_seq / t_serve,
        "peak_running": info["peak_running"], "peak_admitted_gb": info["peak_admitted_bytes"] / 2 ** 30,
        "served_on_resident_problem": info["resident_hits"],
    }
    print(json.dumps(out))


def randomized(args):
    """The randomized two-pass eigensolver on the 512 x 512 mesh, nt = 500
    workload (alpha = 1e-3, sigma = 5e-3, tol 1e-6, rank <= 32): 64 + 10
    Gaussian probes of rank 32 drawn by the library (the same probes in every
    run: a counter-based generator of the problem's seed), applied in batched
    passes as large as device memory allows, mixed precision.  Reports probe
    applies per second, the top eigenvalues and the Ritz residual estimate,
    and, unless --no-fp64-reference, the same solve in float64 on the same
    probes with the mixed result's relative error of the top 64 Ritz values."""
    import dataclasses

    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)

    def solve(precision):
        desc = dataclasses.replace(synthetic.MESH512_NT500_PROBES, precision=precision)
        prob = lp.Problem(desc)
        prob.set_log(1)
        a0 = prob.stats()["applies"]
        t0 = time.perf_counter()
        eig = prob.eigensolve(synthetic.PROBE_COUNT, method=lp.LRPOST_RANDOMIZED,
                              oversample=synthetic.PROBE_OVERSAMPLE, allow_unconverged=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = prob.stats()
        lam = eig.values()
        del eig, prob
        return desc, dt, st, st["applies"] - a0, lam

    desc, dt, st, applies, lam = solve(args.precision)
    out = {
        "metric": "probe Hessian applies/s (randomized two-pass eigensolver)",
        "value": applies / dt, "unit": "Hessian applies/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic", "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "config": {"workload": "mesh512_nt500_probes74_rank32", "N": desc.N, "nt": desc.nt, "nx": (desc.N - 1) ** 2,
                   "probes": synthetic.PROBE_COUNT + synthetic.PROBE_OVERSAMPLE, "probe_rank": 32, "k": synthetic.PROBE_COUNT,
                   "trunc_tol": desc.trunc_tol, "rank_cap": desc.rank_cap, "precision": args.precision},
        "seconds": dt, "applies": applies, "lambda_1_to_3": [float(x) for x in lam[:3]],
        "lambda_64": float(lam[-1]), "max_rel_ritz_residual_estimate": st["ritz_resid"],
        "spacetime_check": {"enriched_batches": st["st_enrichments"], "unresolved_batches": st["st_unresolved"],
                            "direct_second_grams": st["st_direct_grams"]},
    }
    if args.precision == "mixed" and not args.no_fp64_reference:
        _, dt64, _, applies64, lam64 = solve("fp64")
        n = min(len(lam), len(lam64))
        rel = abs(lam[:n] - lam64[:n]) / abs(lam64[:n])
        out["fp64_reference"] = {"applies_per_s": applies64 / dt64, "seconds": dt64,
                                 "top64_max_rel_err": float(rel.max()), "top10_max_rel_err": float(rel[:10].max())}
    print(json.dumps(out))


def initial(args):
    """The paper's own experiment setting (Sec. 6, Sec. 6.2): the initial
    condition as the parameter, the heat equation on the 64 x 64 mesh with
    nt = 30, nine sensors of area 1/256, Gamma_prior = 10 I and a noise weight
    1e4 times the prior's (sigma^2 = 1e-3), truncation tolerance 1e-8 (the
    paper's): the 50 leading eigenpairs of the prior-preconditioned misfit
    Hessian (eq. misfit) and the posterior variance (eq. postvar), float64;
    then the same on the 512 x 512 mesh.  Reports the latency and applies/s
    of each and, unless --no-cpu-baseline, the oracle's ARPACK solve of the
    64 x 64 case on one host core."""
    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    c, k, nt = 10.0, 50, 30
    sigma = (1e-3) ** 0.5
    runs = {}
    for N in (64, 512):
        desc = synthetic.ProblemDesc(N=N, nt=nt, sigma=sigma, trunc_tol=1e-8, rank_cap=32, k=k, precision="fp64")
        prob = lp.Problem(desc)
        prob.set_obs_mask(synthetic.sensor_mask(N))
        prob.ic_eigensolve(4, c, max_vectors=8, allow_unconverged=True)  # warm-up: autotuning, graph capture
        torch.cuda.synchronize()
        a0 = prob.stats()["applies"]
        t0 = time.perf_counter()
        vals, vecs, used = prob.ic_eigensolve(k, c, allow_unconverged=True)
        D = prob.ic_post_variance(vals, vecs, c, on_device=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = prob.stats()
        runs["mesh%d_nt%d" % (N, nt)] = {
            "seconds": dt, "applies": st["applies"] - a0, "applies_per_s": (st["applies"] - a0) / dt,
            "basis_vectors": used, "max_rel_ritz_residual": st["ritz_resid"],
            "lambda_1_to_3": [float(x) for x in vals[:3]], "lambda_50": float(vals[-1]),
            "min_posterior_variance": float(D.min().item())}
        print("initial-condition %dx%d done in %.2f s" % (N, N, dt), file=sys.stderr, flush=True)
        del prob, vecs, D
    out = {"metric": "initial-condition posterior (50 eigenpairs + variance): latency", "value": runs["mesh64_nt30"]["seconds"],
           "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic", "dtype": "f64",
           "config": {"workload": "paper_heat_ic_mesh64_nt30_9sensors", "prior_var": c, "sigma2": sigma ** 2,
                      "trunc_tol": 1e-8, "k": k},
           "runs": runs}
    if not args.no_cpu_baseline:
        import numpy as np

        from oracle.initial import ICProblem
        ora = ICProblem(64, nt, sigma=sigma, prior_var=c, mask=synthetic.sensor_mask(64))
        t0 = time.perf_counter()
        lam, V = ora.eig_arpack(k)
        Dc = ora.post_var_lowrank(lam, V)
        dtc = time.perf_counter() - t0
        out["cpu_baseline"] = {"value": dtc, "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": "the whole 64 x 64 case: ARPACK (scipy eigsh) on the oracle's matrix-free "
                                         "G (sparse-LU time stepping), 50 pairs, then the variance"}
        g = runs["mesh64_nt30"]["lambda_1_to_3"]
        out["cpu_baseline"]["lambda_1_rel_diff"] = float(abs(g[0] - lam[0]) / lam[0])
        out["cpu_baseline"]["min_variance"] = float(np.min(Dc))
    print(json.dumps(out))


def convection(args):
    """The paper's convection-diffusion experiment (Sec. 6.3): the initial
    condition as the parameter, -nu Laplace + (0, 1) . grad with SUPG on the
    32 x 32 mesh, nine sensors, Gamma_prior = 10 I, sigma^2 = 1e-3, truncation
    tolerance 1e-8: the 50 leading eigenpairs of the prior-preconditioned
    misfit Hessian and the posterior variance, float64, for nu = 1e-2 and
    1e-3 with nt = 30 (the eigenvalue study) and nt = 90 (the variance study).
    Then a 512 x 512 mesh (nt = 90, nu = 1e-3, 20 pairs) with the
    convection-diffusion kernels timed: the sine transform on the float64
    matrix cores and the tridiagonal sweeps against HBM.  Unless
    --no-cpu-baseline, the oracle's ARPACK solve of the 32 x 32, nt = 90,
    nu = 1e-3 case on one host core."""
    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    # the calibration copy of the HBM byte counters (as in the main leg)
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    c = 10.0
    sigma = (1e-3) ** 0.5
    runs = {}

    def one(N, nt, nu, k, profile=False):
        desc = synthetic.ProblemDesc(N=N, nt=nt, sigma=sigma, trunc_tol=1e-8, rank_cap=96, k=k, precision="fp64")
        prob = lp.Problem(desc)
        prob.set_obs_mask(synthetic.sensor_mask(N))
        prob.set_convection(nu, 1.0)
        prob.ic_eigensolve(4, c, max_vectors=8, allow_unconverged=True)  # warm-up
        torch.cuda.synchronize()
        if profile:
            prob.profile(True)
            for kind in (lp.LRPOST_KERNEL_SINE, lp.LRPOST_KERNEL_TRIDIAG):
                prob.profile_read(kind)
        a0 = prob.stats()["applies"]
        t0 = time.perf_counter()
        vals, vecs, used = prob.ic_eigensolve(k, c, allow_unconverged=True)
        D = prob.ic_post_variance(vals, vecs, c, on_device=True)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        st = prob.stats()
        r = {"seconds": dt, "applies": st["applies"] - a0, "applies_per_s": (st["applies"] - a0) / dt,
             "basis_vectors": used, "max_rel_ritz_residual": st["ritz_resid"],
             "lambda_1_to_3": [float(x) for x in vals[:3]], "lambda_k": float(vals[-1]),
             "pairs_above_10": int((vals > 10).sum()), "pairs_above_1": int((vals > 1).sum()),
             "min_posterior_variance": float(D.min().item()),
             "spacetime_check": {"enriched_batches": st["st_enrichments"], "unresolved_batches": st["st_unresolved"],
                                 "last_basis": st["last_basis"]}}
        if profile:
            kern = {}
            for kind, name, peak, unit in ((lp.LRPOST_KERNEL_SINE, "k_sine_x1", MFMA_F64_PEAK_TFLOPS, "TFLOP/s"),
                                           (lp.LRPOST_KERNEL_TRIDIAG, "k_tridiag_x2", HBM_PEAK_GBS, "GB/s")):
                n, ms, by, fl = prob.profile_read(kind)
                if n == 0:
                    continue
                ach = (fl / (ms * 1e-3) / 1e12) if unit == "TFLOP/s" else (by / (ms * 1e-3) / 1e9)
                kern[name] = {"launches": n, "avg_us": 1e3 * ms / n, "bytes_per_launch": by / n,
                              "flops_per_launch": fl / n, "achieved": ach, "unit": unit, "peak": peak,
                              "frac": ach / peak}
            prob.profile(False)
            r["kernels"] = kern
        print("convection-diffusion %dx%d nt=%d nu=%g done in %.2f s" % (N, N, nt, nu, dt), file=sys.stderr, flush=True)
        return r

    if not args.convection_large_only:
        for nu in (1e-2, 1e-3):
            for nt in (30, 90):
                runs["mesh32_nt%d_nu%g" % (nt, nu)] = one(32, nt, nu, 50)
    big = one(512, 90, 1e-3, 20, profile=True)
    runs["mesh512_nt90_nu0.001"] = big
    head = runs.get("mesh32_nt90_nu0.001", big)
    out = {"metric": "convection-diffusion initial-condition posterior (50 eigenpairs + variance): latency",
           "value": head["seconds"], "unit": "s", "n_gpus": 1, "higher_is_better": False, "data": "synthetic",
           "dtype": "f64",
           "config": {"workload": "paper_convdiff_ic_mesh32_nt90_nu1e-3_9sensors", "wind": [0.0, 1.0],
                      "prior_var": c, "sigma2": sigma ** 2, "trunc_tol": 1e-8, "k": 50},
           "runs": runs}
    if args.convection_large_only:
        out["metric"] = "convection-diffusion initial-condition posterior (20 eigenpairs + variance): latency"
        out["config"] = {"workload": "convdiff_ic_mesh512_nt90_nu1e-3_9sensors", "wind": [0.0, 1.0],
                         "prior_var": c, "sigma2": sigma ** 2, "trunc_tol": 1e-8, "k": 20}
    sk = big.get("kernels", {}).get("k_sine_x1")
    if sk:
        from paper_1703_05638_amd.profile_summary import read_traffic
        traffic = read_traffic(os.path.join(ROOT, "profiles", "k_sine_x1_convdiff_mesh512_nt90_traffic.txt"))
        out["roofline"] = {"bound": "mfma", "kernel": "k_sine_x1", "achieved": sk["achieved"],
                           "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": sk["frac"], "traffic": traffic,
                           "workload": "mesh512_nt90_nu0.001"}
        out["roofline"].update(measured_rates())
    if not args.no_cpu_baseline and not args.convection_large_only:
        from oracle.convdiff import cd_ic_problem
        ora = cd_ic_problem(32, 90, 1e-3, sigma=sigma, prior_var=c, mask=synthetic.sensor_mask(32))
        t0 = time.perf_counter()
        lam, V = ora.eig_arpack(50)
        ora.post_var_lowrank(lam, V)
        dtc = time.perf_counter() - t0
        g = head["lambda_1_to_3"]
        out["cpu_baseline"] = {"value": dtc, "unit": "s", "cores": 1, "kind": "oracle",
                               "sample": "the whole 32 x 32, nt = 90, nu = 1e-3 case: ARPACK (scipy eigsh) on the "
                                         "oracle's matrix-free G (sparse-LU time stepping, transposed adjoint "
                                         "steps), 50 pairs, then the variance",
                               "lambda_1_rel_diff": float(abs(g[0] - lam[0]) / lam[0])}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="mixed")
    ap.add_argument("--no-fp64-reference", action="store_true",
                    help="in mixed precision, skip the float64 comparison step")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-posterior", action="store_true",
                    help="skip the complete 256 x 256 posterior reported beside the headline")
    ap.add_argument("--vectors", type=int, default=40,
                    help="Krylov vectors per headline step (block-Lanczos budget)")
    ap.add_argument("--serving", type=int, default=0,
                    help="measure the serving loop on this many requests instead of the eigensolve step")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--initial", action="store_true",
                    help="measure the paper's own setting: the initial-condition parameter, 64 x 64, nt = 30, 9 sensors")
    ap.add_argument("--convection", action="store_true",
                    help="measure the paper's convection-diffusion setting: 32 x 32, nt = 30 and 90, nu = 1e-2 and 1e-3")
    ap.add_argument("--convection-large-only", action="store_true",
                    help="with --convection: only the 512 x 512 case whose kernels are timed (for profiling)")
    ap.add_argument("--randomized", action="store_true",
                    help="measure the randomized eigensolver on the 512 x 512, nt = 500 probe workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on %d GPUs are not implemented (one process runs on one GPU)"
              % args.gpus, file=sys.stderr)
        sys.exit(2)
    if args.serving > 0:
        serving(args)
        return
    if args.randomized:
        randomized(args)
        return
    if args.initial:
        initial(args)
        return
    if args.convection:
        convection(args)
        return

    import dataclasses

    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    # A plain elementwise copy of known size (8-byte elements, read once and
    # written once): its FETCH_SIZE / WRITE_SIZE counters scale the kernels'.
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst

    def run(base, precision, warmup, steps, profile, vectors):
        desc = dataclasses.replace(base, precision=precision)
        prob = lp.Problem(desc)
        prob.set_log(1)
        if vectors:
            prob.set_eig_limits(max_vectors=vectors)

        def step():
            eig = prob.eigensolve(desc.k, allow_unconverged=vectors > 0)
            D = prob.post_variance(eig, on_device=True)
            return eig, D

        for w in range(warmup):
            t0 = time.perf_counter()
            eig, D = step()
            del eig, D
            print("%s warmup step %d done in %.1f s" % (precision, w, time.perf_counter() - t0), file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        st0 = prob.stats()
        applies0 = st0["applies"]
        if profile:
            prob.profile(True)
        step_ms = []
        lam = D_last = None
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
            D_last = None
            eig, D = step()
            torch.cuda.synchronize()
            step_ms.append((time.perf_counter() - t0) * 1e3)
            lam = eig.values()
            D_last = D
            del eig
            print("%s timed step done in %.1f s" % (precision, step_ms[-1] / 1e3), file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_all
        prof = {k: prob.profile_read(k) for k in KERNELS} if profile else {}
        prob.profile(False)
        st1 = prob.stats()
        res = {"desc": desc, "applies": st1["applies"] - applies0, "elapsed": elapsed, "step_ms": step_ms,
               "lam": lam, "D": D_last, "prof": prof, "stats": st1,
               "pool": {"device_allocations": st1["pool_mallocs"] - st0["pool_mallocs"],
                        "cache_releases": st1["pool_trims"] - st0["pool_trims"],
                        "host_seconds": st1["pool_malloc_s"] - st0["pool_malloc_s"]}}
        del prob
        return res

    head = synthetic.MESH1024_NT1000
    workload = "mesh1024_nt1000"
    main_run = run(head, args.precision, args.warmup, args.steps, True, args.vectors)
    desc = main_run["desc"]
    # the timed kernel kind with the most device time in the timed steps
    kind = max(main_run["prof"], key=lambda k: main_run["prof"][k][1])
    launches, kern_ms, kern_bytes, kern_flops = main_run["prof"][kind]
    applies, elapsed, step_ms, lam, st = (main_run["applies"], main_run["elapsed"], main_run["step_ms"],
                                          main_run["lam"], main_run["stats"])
    ref = None
    fp64_ref = None
    if args.precision == "mixed" and not args.no_fp64_reference:
        # the same step in float64: its throughput, and the mixed result's error against it
        D_mixed = main_run["D"]
        main_run["D"] = None
        ref = run(head, "fp64", 0, 1, False, args.vectors)
        lam64, D64 = ref["lam"], ref["D"]
        fp64_ref = {
            "applies_per_s": ref["applies"] / ref["elapsed"],
            "step_ms": ref["step_ms"][0],
            "ritz_values_max_rel_err": float(abs(lam - lam64).max() / abs(lam64).max()),
            # the leading pairs, which 40 Krylov vectors resolve (the trailing Ritz
            # values of a truncated Lanczos run move with any perturbation)
            "ritz_values_top10_max_rel_err": float((abs(lam[:10] - lam64[:10]) / abs(lam64[:10])).max()),
            "variance_max_rel_err": float(((D_mixed - D64).abs() / D64.abs()).max().item()),
        }
        del D_mixed, D64, ref
        torch.cuda.empty_cache()
    from paper_1703_05638_amd.profile_summary import read_traffic

    kbase, kdesc, mg_kernel, _ = KERNELS[kind]
    traffic = read_traffic(traffic_report(kbase, args.precision, workload))
    avg_ms = kern_ms / max(launches, 1)
    bytes_per_launch = kern_bytes / max(launches, 1)
    flops_per_launch = kern_flops / max(launches, 1)
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    tflops = flops_per_launch / (avg_ms * 1e-3) / 1e12 if launches else 0.0
    # the tighter of the two ceilings bounds the kernel
    mfma_peak = KERNELS[kind][3]
    mfma_bound = mfma_peak is not None and kern_flops / (mfma_peak * 1e12) > kern_bytes / (HBM_PEAK_GBS * 1e9)
    if mg_kernel:
        kname = kbase + ("<double>" if args.precision == "fp64" else "<float>")
    else:
        kname = kbase
    others = {KERNELS[k][0]: {"launches": v[0], "total_ms": v[1],
                              "achieved_GBs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else 0.0,
                              "achieved_TFLOPs": (v[3] / (v[1] * 1e-3) / 1e12) if v[1] > 0 else 0.0}
              for k, v in main_run["prof"].items() if k != kind and v[0] > 0}
    if mfma_bound:
        roof = {"bound": "mfma", "achieved": tflops, "peak": mfma_peak, "unit": "TFLOP/s",
                "frac": tflops / mfma_peak, "achieved_GBs": gbs}
        if mfma_peak == MFMA_F64_PEAK_TFLOPS:
            roof.update(measured_rates())
    else:
        roof = {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS}
        if kern_flops > 0:
            roof["achieved_TFLOPs"] = tflops
    out = {
        "metric": "Hessian applies/s (fwd+adj space-time) + p50/p99 posterior latency @1e-5 rel",
        "value": applies / elapsed,
        "unit": "Hessian applies/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "%s_lanczos%dvec" % (workload, args.vectors), "N": desc.N, "nt": desc.nt,
                   "nx": (desc.N - 1) ** 2, "k": desc.k, "krylov_vectors_per_step": args.vectors,
                   "trunc_tol": desc.trunc_tol, "rank_cap": desc.rank_cap, "alpha": desc.alpha, "sigma": desc.sigma,
                   "precision": args.precision},
        "step_latency_ms": {"p50": statistics.median(step_ms),
                            "p99": sorted(step_ms)[min(len(step_ms) - 1, int(0.99 * len(step_ms)))]},
        "applies_per_step": applies / args.steps,
        "lanczos_block_steps": st["lanczos_steps"],
        "ritz_values_1_to_3": [float(x) for x in lam[:3]],
        "ritz_resid_estimate": st["ritz_resid"],
        "spacetime_check": {"last_resid": st["last_st_resid"], "last_precond_resid": st["last_st_presid"],
                            "enriched_batches": st["st_enrichments"], "unresolved_batches": st["st_unresolved"],
                            "direct_second_grams": st["st_direct_grams"]},
        "device_pool_in_timed_steps": main_run["pool"],
        "roofline": dict({"kernel": "%s (%s)" % (kname, kdesc)}, **roof,
                         **{"traffic": traffic, "launches": launches, "avg_launch_us": avg_ms * 1e3,
                            "bytes_per_launch": bytes_per_launch, "flops_per_launch": flops_per_launch,
                            "total_ms": kern_ms, "other_timed_kernels": others}),
    }
    if fp64_ref is not None:
        out["fp64_reference"] = fp64_ref
    del main_run
    torch.cuda.empty_cache()
    if not args.no_posterior:
        # a complete posterior (50 pairs, converged) on the 256 x 256 mesh, nt = 200
        post = run(synthetic.MESH256_NT200, args.precision, 1, 1, False, 0)
        out["mesh256_posterior"] = {
            "workload": "mesh256_nt200_lanczos50", "applies_per_s": post["applies"] / post["elapsed"],
            "posterior_latency_ms": post["step_ms"][0], "applies": post["applies"],
            "lanczos_block_steps": post["stats"]["lanczos_steps"], "ritz_resid_estimate": post["stats"]["ritz_resid"]}
        del post
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
