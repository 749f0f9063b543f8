"""Benchmark: Hessian applies per second during a full low-rank posterior
computation on one MI355X.

A step is one pass of the whole hot path on the 256 x 256 mesh, nt = 200
workload (alpha = sigma = 1e-2, observation box [0.25, 0.75]^2, truncation
tolerance 1e-6, factor rank <= 64): block-Lanczos eigensolve for the 50
leading eigenpairs of the prior-preconditioned misfit Hessian (every Krylov
vector a low-rank space-time vector, every apply a forward and an adjoint
low-rank space-time solve plus a prior solve) followed by the posterior
variance diag(Gamma_post,50) over all nx * nt space-time points.  Inputs are
synthetic (seeded start block); they are generated inside the library and
are resident in HBM when the timed region starts.

value = Hessian applies completed in the timed steps / timed seconds.  The
default precision is mixed (float32 multigrid cycles with float64 iterative
refinement of the prior solve; projections, truncations and the Lanczos
matrix in float64); afterwards the same step runs in float64, and its
throughput and the mixed result's relative error against it (eigenvalues and
posterior variance) are reported under "fp64_reference".
Prints one JSON line.  Usage: python bench.py [--gpus 1] [--steps K] [--warmup W]
[--precision mixed|fp64] [--serving R]
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
# Multigrid kernels timed with HIP events (kind as in the library's
# LRPOST_KERNEL_*), their names, and the committed HBM-counter reports.
KERNELS = {
    0: ("k_cheb", "multigrid Chebyshev smoother step", True),
    1: ("k_mg_down", "level-fused pre-smoothing + residual + restriction", True),
    2: ("k_mg_up", "level-fused prolongation + post-smoothing", True),
    3: ("k_gram_mfma", "float64 matrix-core Gram A^T B, partial products", False),
    4: ("k_proj_mfma", "float64 matrix-core projection C = beta C + A Q", False),
}
MFMA_F64_PEAK_TFLOPS = 78.6  # MI355X published dense FP64 matrix throughput


def traffic_report(kernel, precision):
    # the multigrid kernels run in float32 in mixed precision, the Gram always in float64
    f32 = precision == "mixed" and KERNELS[[k for k in KERNELS if KERNELS[k][0] == kernel][0]][2]
    tag = "f32_" if f32 else ""
    suffix = "_mixed" if precision == "mixed" else ""
    return os.path.join(ROOT, "profiles", "%s_%smesh256_nt200%s_traffic.txt" % (kernel, tag, suffix))


def cpu_baseline(desc, budget_s=20.0):
    """The FP64 oracle's Hessian apply (implicit-Euler time stepping with a
    sparse LU of M + tau K) on the same workload, timed on the host."""
    import numpy as np
    from oracle.spacetime import Problem as OracleProblem

    ora = OracleProblem.from_desc(desc)
    rng = np.random.default_rng(1)
    A = rng.standard_normal((ora.nx, 20))
    B = np.cumsum(rng.standard_normal((ora.nt, 20)), axis=0) / np.sqrt(ora.nt)
    X = A @ B.T
    t0 = time.perf_counter()
    n = 0
    while True:
        ora.G(X)
        n += 1
        if time.perf_counter() - t0 > budget_s / 2 or n >= 3:
            break
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "Hessian applies/s", "cores": 1, "kind": "oracle",
            "sample": "%d full FP64 G-applies on a rank-20 space-time input, 256x256 mesh, nt=200 "
                      "(SuperLU factor reused; single-threaded)" % n}


def serving(args):
    """Replay the first --serving requests of the seeded Poisson request stream
    (20 req/s; mesh side 64/128/256, nt 50/100/200, k = 30 eigenpairs plus the
    posterior variance, tol 1e-6, rank <= 64) through the serving loop, then
    run the same requests one after another on one stream (the plain FP64
    path) and report latency percentiles, throughput and the speedup."""
    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    reqs = synthetic.serving_stream()[: args.serving]
    srv = lp.Server(hbm_budget_bytes=200 << 30, workers=args.workers)
    t0 = time.perf_counter()
    tickets = []
    for r in reqs:
        delay = r.arrival_s - (time.perf_counter() - t0)
        if delay > 0:
            time.sleep(delay)
        tickets.append(srv.submit(r.desc, r.desc.k))
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
        "data": "synthetic", "dtype": "f64",
        "config": {"workload": "poisson20_mesh64-256_nt50-200_k30", "requests": len(reqs), "workers": args.workers,
                   "hbm_budget_gb": 200},
        "latency_s": {"p50": statistics.median(lat),
                      "p99": lat_sorted[min(len(lat) - 1, int(0.99 * len(lat)))]},
        "makespan_s": t_serve, "sequential_fp64_s": t_seq, "speedup_vs_sequential": t_seq / t_serve,
        "peak_running": info["peak_running"], "peak_admitted_gb": info["peak_admitted_bytes"] / 2 ** 30,
    }
    print(json.dumps(out))


def randomized(args):
    """The randomized two-pass eigensolver on the 512 x 512 mesh, nt = 500
    workload (alpha = 1e-3, sigma = 5e-3, tol 1e-6, rank <= 32): 64 + 10
    Gaussian probes of rank 32 drawn by the library, probes applied 8 at a time
    with fused multigrid solves, mixed precision.  Reports probe applies per
    second, the top eigenvalues and the Ritz residual certificate."""
    import dataclasses

    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    desc = dataclasses.replace(synthetic.MESH512_NT500_PROBES, precision=args.precision)
    prob = lp.Problem(desc)
    prob.set_log(1)
    a0 = prob.stats()["applies"]
    t0 = time.perf_counter()
    eig = prob.eigensolve(synthetic.PROBE_COUNT, method=lp.LRPOST_RANDOMIZED, oversample=synthetic.PROBE_OVERSAMPLE,
                          allow_unconverged=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = prob.stats()
    lam = eig.values()
    out = {
        "metric": "probe Hessian applies/s (randomized two-pass eigensolver)",
        "value": (st["applies"] - a0) / dt, "unit": "Hessian applies/s", "n_gpus": 1, "higher_is_better": True,
        "data": "synthetic", "dtype": "f64" if args.precision == "fp64" else "f32+f64",
        "config": {"workload": "mesh512_nt500_probes74_rank32", "N": desc.N, "nt": desc.nt, "nx": (desc.N - 1) ** 2,
                   "probes": synthetic.PROBE_COUNT + synthetic.PROBE_OVERSAMPLE, "probe_rank": 32, "k": synthetic.PROBE_COUNT,
                   "trunc_tol": desc.trunc_tol, "rank_cap": desc.rank_cap, "precision": args.precision},
        "seconds": dt, "applies": st["applies"] - a0, "lambda_1_to_3": [float(x) for x in lam[:3]],
        "lambda_64": float(lam[-1]), "max_rel_ritz_residual": st["ritz_resid"],
    }
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
    ap.add_argument("--serving", type=int, default=0,
                    help="measure the serving loop on this many requests instead of the eigensolve step")
    ap.add_argument("--workers", type=int, default=4)
    ap.add_argument("--randomized", action="store_true",
                    help="measure the randomized eigensolver on the 512 x 512, nt = 500 probe workload")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; runs on %d GPUs are not part of this build" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.serving > 0:
        serving(args)
        return
    if args.randomized:
        randomized(args)
        return

    import dataclasses

    import torch

    import synthetic
    from paper_1703_05638_amd import lrpost as lp

    lp.load()
    torch.cuda.set_device(0)
    # A plain elementwise copy of known size (8-byte elements, read once and
    # written once): its FETCH_SIZE / WRITE_SIZE counters scale the smoother's.
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        torch.mul(src, 1.0, out=dst)
    torch.cuda.synchronize()
    del src, dst
    def run(precision, warmup, steps, profile):
        desc = dataclasses.replace(synthetic.MESH256_NT200, precision=precision)
        prob = lp.Problem(desc)
        prob.set_log(1)

        def step():
            eig = prob.eigensolve(desc.k)
            D = prob.post_variance(eig, on_device=True)
            return eig, D

        for w in range(warmup):
            t0 = time.perf_counter()
            eig, D = step()
            del eig, D
            print("%s warmup step %d done in %.1f s" % (precision, w, time.perf_counter() - t0), file=sys.stderr,
                  flush=True)
        torch.cuda.synchronize()
        applies0 = prob.stats()["applies"]
        if profile:
            prob.profile(True)
        step_ms = []
        lam = D_last = None
        t_all = time.perf_counter()
        for _ in range(steps):
            t0 = time.perf_counter()
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
        res = {"desc": desc, "applies": prob.stats()["applies"] - applies0, "elapsed": elapsed, "step_ms": step_ms,
               "lam": lam, "D": D_last, "prof": prof, "stats": prob.stats()}
        del prob
        return res

    main_run = run(args.precision, args.warmup, args.steps, True)
    desc = main_run["desc"]
    # the multigrid kernel with the most device time in the timed steps
    kind = max(main_run["prof"], key=lambda k: main_run["prof"][k][1])
    launches, kern_ms, kern_bytes, kern_flops = main_run["prof"][kind]
    applies, elapsed, step_ms, lam, st = (main_run["applies"], main_run["elapsed"], main_run["step_ms"],
                                          main_run["lam"], main_run["stats"])
    ref = None
    if args.precision == "mixed" and not args.no_fp64_reference:
        # the same step in float64: its throughput, and the mixed result's error against it
        ref = run("fp64", 0, 1, False)
    from paper_1703_05638_amd.profile_summary import read_traffic

    kbase, kdesc, mg_kernel = KERNELS[kind]
    traffic = read_traffic(traffic_report(kbase, args.precision))
    avg_ms = kern_ms / max(launches, 1)
    bytes_per_launch = kern_bytes / max(launches, 1)
    flops_per_launch = kern_flops / max(launches, 1)
    gbs = bytes_per_launch / (avg_ms * 1e-3) / 1e9 if launches else 0.0
    tflops = flops_per_launch / (avg_ms * 1e-3) / 1e12 if launches else 0.0
    # the tighter of the two ceilings bounds the kernel
    mfma_bound = kern_flops / (MFMA_F64_PEAK_TFLOPS * 1e12) > kern_bytes / (HBM_PEAK_GBS * 1e9)
    if mg_kernel:
        kname = kbase + ("<double>" if args.precision == "fp64" else "<float>")
    else:
        kname = kbase
    others = {KERNELS[k][0]: {"launches": v[0], "total_ms": v[1],
                              "achieved_GBs": (v[2] / (v[1] * 1e-3) / 1e9) if v[1] > 0 else 0.0}
              for k, v in main_run["prof"].items() if k != kind and v[0] > 0}
    if mfma_bound:
        roof = {"bound": "mfma", "achieved": tflops, "peak": MFMA_F64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": tflops / MFMA_F64_PEAK_TFLOPS, "achieved_GBs": gbs}
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
        "config": {"workload": "mesh256_nt200_lanczos50", "N": desc.N, "nt": desc.nt, "nx": (desc.N - 1) ** 2,
                   "k": desc.k, "trunc_tol": desc.trunc_tol, "rank_cap": desc.rank_cap,
                   "alpha": desc.alpha, "sigma": desc.sigma, "precision": args.precision},
        "posterior_latency_ms": {"p50": statistics.median(step_ms),
                                 "p99": sorted(step_ms)[min(len(step_ms) - 1, int(0.99 * len(step_ms)))]},
        "applies_per_step": applies / args.steps,
        "lanczos_block_steps": st["lanczos_steps"],
        "lambda_1_to_3": [float(x) for x in lam[:3]],
        "roofline": dict({"kernel": "%s (%s)" % (kname, kdesc)}, **roof,
                         **{"traffic": traffic, "launches": launches, "avg_launch_us": avg_ms * 1e3,
                            "bytes_per_launch": bytes_per_launch, "flops_per_launch": flops_per_launch,
                            "total_ms": kern_ms, "other_timed_kernels": others}),
    }
    if ref is not None:
        lam64 = ref["lam"]
        D64 = ref["D"]
        out["fp64_reference"] = {
            "applies_per_s": ref["applies"] / ref["elapsed"],
            "posterior_latency_ms": ref["step_ms"][0],
            "lambda_max_rel_err": float(abs(lam - lam64).max() / abs(lam64).max()),
            "variance_max_rel_err": float(((main_run["D"] - D64).abs() / D64.abs()).max().item()),
        }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(desc)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
