"""Benchmark: CE factorization + FP64 PCG on one MI355X.

Workload (default): 2D 5-point Dirichlet Laplacian on a 1024 x 1024 grid
(N = 1,048,576), 8 x 8 Morton patches (B = 64), eps = 1e-6, 16 right-hand
sides N(0,1) from default_rng(1), PCG in FP64 to a relative residual of 1e-8.
One step = numeric factorization (all levels, dense remainder) + PCG for the
16 right-hand sides.  The matrix, permutation and right-hand sides are
resident on the GPU before the timed region; the host symbolic analysis is
timed separately (``analysis_ms``) and also inside the step when
``--with-analysis`` is given.

Prints ONE JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)


def _cpu_baseline(side, patch, eps, nrhs_full, full_n):
    """The FP64 oracle as it stands, on a bounded sample of the workload: the
    same stencil, patch size and eps on a side x side grid, factorization and
    PCG for one right-hand side, scaled linearly in N (the method is O(N) on
    tensor grids) and in the number of right-hand sides."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    import oracle
    import problems
    with threadpool_limits(limits=1):
        A = problems.laplacian((side, side))
        ip, ix, dv = problems.to_csr_arrays(A)
        perm, bp, co = oracle.grid_order((side, side), patch)
        t0 = time.perf_counter()
        f = oracle.ce_factor(ip, ix, dv, perm, bp, co, oracle.CEOptions(eps=eps, order="multicolour"))
        t1 = time.perf_counter()
        b = problems.rhs_normal(A.shape[0], 1, seed=1)[:, 0]
        _, it, rel = oracle.pcg(A, b, lambda r: oracle.ce_solve(f, r), tol=1e-8)
        t2 = time.perf_counter()
    scale = full_n / A.shape[0]
    est = (t1 - t0) * scale + (t2 - t1) * scale * nrhs_full
    return {"value": est, "unit": "s", "cores": 1, "kind": "oracle",
            "sample": (f"{side}x{side} grid (N={A.shape[0]}), same patch/eps, factor {t1 - t0:.2f} s + "
                       f"PCG 1 RHS {t2 - t1:.2f} s ({it} it); scaled x{scale:.0f} in N and x{nrhs_full} RHS "
                       f"for the PCG part")}


def _log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _traffic(kernel):
    """HBM bytes per launch of ``kernel`` from the committed counter summary
    (FETCH_SIZE / WRITE_SIZE runs scaled by a plain copy), or None when the
    kernel source changed since the counters were taken."""
    import glob
    import hashlib
    src = os.path.join(ROOT, "paper_1603_09133_amd", "csrc", "factor_kernels.hip")
    h = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "*_traffic.md")):
        fields = {}
        for line in open(path):
            if ":" in line and not line.startswith(("|", "#", " ")):
                k, v = line.split(":", 1)
                fields[k.strip()] = v.strip()
        if fields.get("kernel") == kernel and fields.get("source_sha256") == h:
            return float(fields["traffic_bytes_per_launch"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--side", type=int, default=1024)
    ap.add_argument("--patch", type=int, default=8)
    ap.add_argument("--eps", type=float, default=1e-6)
    ap.add_argument("--nrhs", type=int, default=16)
    ap.add_argument("--precision", choices=["fp32", "fp64"], default="fp32")
    ap.add_argument("--order", choices=["multicolour", "paper"], default="multicolour")
    ap.add_argument("--with-analysis", action="store_true")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-side", type=int, default=128)
    ap.add_argument("--config", choices=["c2", "c3", "c4", "c5"], default="c2",
                    help="c2: 2D Laplacian 1024^2 (default, the headline); c3: 3D Laplacian 128^3, B=64, eps=1e-4, "
                         "1 RHS, BF16 Schur, learned ranks; c4: 2D diffusion with a random coefficient 2048^2, "
                         "eps=1e-5, 64 RHS; c5: 256 independent 2D/3D problems in one factorization, 4 RHS each")
    ap.add_argument("--coarsen", choices=["siblings", "pairs"], default=None,
                    help="3D coarsening (default: pairs for c3, siblings otherwise)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="run one plain device-to-device copy of this size before the timed steps "
                         "(reference dispatch for the HBM byte counters)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; "
              "how the factorization would shard is a design, not code", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import paper_1603_09133_amd as cae
    import problems

    dev = torch.device("cuda:0")
    coarsen = "siblings"
    order = cae.ORDER_MULTICOLOUR if args.order == "multicolour" else cae.ORDER_PAPER
    prec = cae.FP32 if args.precision == "fp32" else cae.FP64
    fkw = {}
    if args.config == "c2":
        dims = (args.side, args.side)
        patch = (args.patch, args.patch)
        A = problems.laplacian(dims)
        B = problems.rhs_normal(A.shape[0], args.nrhs, seed=1)
        workload = (f"2D 5-point Laplacian {args.side}x{args.side} (N={A.shape[0]}), {args.patch}x{args.patch} "
                    f"Morton patches (B={args.patch * args.patch}), eps={args.eps}, {args.nrhs} RHS N(0,1) seed 1, "
                    f"PCG FP64 to 1e-8, {args.order} order")
    elif args.config == "c3":
        dims, patch = (128, 128, 128), (4, 4, 4)
        coarsen = "pairs"
        args.eps, args.nrhs = 1e-4, 1
        A = problems.laplacian(dims)
        B = problems.rhs_normal(A.shape[0], 1, seed=0)
        prec = cae.FP32_BF16
        workload = ("3D 7-point Laplacian 128^3 (N=2097152), 4x4x4 Morton patches (B=64), pairs of blocks along "
                    "the Morton curve per level, eps=1e-4, 1 RHS N(0,1) seed 0, FP32 factor with BF16 Schur products, "
                    "learned ranks (MLP trained on a 48^3 problem before timing), PCG FP64 to 1e-8")
    elif args.config == "c4":
        dims, patch = (2048, 2048), (8, 8)
        args.eps, args.nrhs = 1e-5, 64
        A, rng = problems.grf_diffusion_2d(2048)
        B = rng.standard_normal((64, A.shape[0])).T
        workload = ("2D -div(k grad u), k = exp(GRF, l=0.05, sigma=1, seed 2), 2048^2 (N=4194304), 8x8 patches "
                    "(B=64), eps=1e-5, FP32 factor, 64 RHS N(0,1), PCG FP64 to 1e-8")
    else:
        from paper_1603_09133_amd import batched
        kind, sides, rng = problems.batched_problem_draws(256, seed=3)
        mats, dl, pl = [], [], []
        for k, sd in zip(kind, sides):
            d = (int(sd), int(sd)) if k == 0 else (int(sd),) * 3
            mats.append(problems.laplacian(d))
            dl.append(d)
            pl.append((8, 8) if k == 0 else (2, 2, 4))
        A, perm, bp, co, _ = batched.assemble(mats, dl, pl)
        B = np.concatenate([rng.standard_normal((4, m.shape[0])) for m in mats], axis=1).T
        args.nrhs = 4
        workload = (f"256 independent Laplacians (2D side 64..512 with 8x8 patches, 3D side 16..64 with 2x2x4 "
                    f"patches; draws default_rng(3)), N={A.shape[0]} in one joint factorization, eps=1e-6, FP32 "
                    f"factor, 4 RHS per problem, PCG FP64 to 1e-8")
    if args.coarsen:
        coarsen = args.coarsen
    ip, ix, dv = problems.to_csr_arrays(A)
    N = A.shape[0]
    if args.config != "c5":
        perm, bp, co = cae.grid_order(dims, patch)
    _log(f"{args.config}: N={A.shape[0]}, symbolic analysis")
    t = time.perf_counter()
    an = cae.Analysis(ip, ix, perm, bp, co, order=order, coarsen=coarsen)
    analysis_ms = (time.perf_counter() - t) * 1e3
    _log(f"analysis {analysis_ms:.0f} ms, {an.nlevels()} levels")
    vals = torch.from_numpy(dv).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(B.T)).to(dev)
    x = torch.empty_like(b)
    if args.config == "c3":
        from paper_1603_09133_amd import learned
        d2 = (48, 48, 48)
        A2 = problems.laplacian(d2)
        i2, x2, v2 = problems.to_csr_arrays(A2)
        p2, b2, c2 = cae.grid_order(d2, patch)
        an2 = cae.Analysis(i2, x2, p2, b2, c2, order=order, coarsen=coarsen)
        rec = learned.record(an2, torch.from_numpy(v2).to(dev), args.eps, precision=cae.FP32)
        an2.close()
        params, _ = learned.train(rec, epochs=800, lr=1e-3)
        fkw = dict(rank_mode=cae.RANK_LEARNED, mlp_params=params, seed=1)

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * 2**18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def step():
        a = cae.Analysis(ip, ix, perm, bp, co, order=order, coarsen=coarsen) if args.with_analysis else an
        f = cae.Factor(a, vals, args.eps, precision=prec, timing=True, **fkw)
        if args.config in ("c3", "c5"):   # long steps: the factorization reports its end
            torch.cuda.synchronize()
            _log("factorization done")
        _, it, rel = f.pcg(b, rtol=1e-8, maxit=1000, x=x)
        return f, it, rel

    for k in range(args.warmup):
        tw = time.perf_counter()
        f, it, rel = step()
        f.close()
        torch.cuda.synchronize()
        _log(f"warmup step {k + 1}/{args.warmup}: {(time.perf_counter() - tw) * 1e3:.0f} ms, PCG iterations "
             f"max {int(np.max(it))}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    fac_ms = []
    comp = {"ms": 0.0, "launches": 0, "flops": 0.0}
    for k in range(args.steps):
        f, it, rel = step()
        _log(f"timed step {k + 1}/{args.steps} done")
        st = f.stats()
        fac_ms.append(st["factor_ms"])
        comp["ms"] += st["compress_ms"]
        comp["launches"] += st["compress_launches"]
        comp["flops"] += st["compress_flops"]
        f.close()
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / max(args.steps, 1)
    ok = bool(np.all(rel <= 1.0001e-8))
    # reference FP64 GPU factor iterations (same workload; the headline only)
    it64 = None
    if args.config == "c2":
        f64 = cae.Factor(an, vals, args.eps, precision=cae.FP64)
        _, it64, rel64 = f64.pcg(b, rtol=1e-8, maxit=1000, x=x)
        f64.close()
    dtype = {cae.FP32: "f32 factor + f64 PCG", cae.FP64: "f64",
             cae.FP32_BF16: "f32 factor with bf16-input Schur products + f64 PCG"}[prec]
    out = {
        "metric": "factor+PCG time to 1e-8 residual (2D/3D Laplacian); block-op TFLOP/s vs peak",
        "value": dt,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {"workload": workload,
                   "factor_ms_mean": float(np.mean(fac_ms)), "analysis_ms": analysis_ms,
                   "analysis_in_step": bool(args.with_analysis),
                   "pcg_iters": it.tolist(), "pcg_iters_fp64_factor": None if it64 is None else it64.tolist(),
                   "relres_max": float(np.max(rel)), "converged": ok, "levels": st["nlevels"],
                   "coarse_dim": st["coarse_dim"], "factor_bytes": st["factor_bytes"]},
    }
    # roofline of the far-row compression, from HIP events around its launches
    # on the factor's stream; its arithmetic is FP64 vector work for either
    # factor precision (the FP32 factor's Gram matrix, Cholesky, Jacobi and
    # reflectors run in FP64), so the peak is the FP64 vector rate
    peak = 78.6
    kname = ("k_compress_wg<double> (TSQR, pivoted QR, one-sided Jacobi)" if prec == cae.FP64 else
             "k_compress_rand<float> (learned-rank sketch) + k_compress_gram<float,64|128> fallback" if fkw else
             "k_compress_gram<float,64> (FP64 Gram, pivoted Cholesky, one-sided Jacobi)")
    if comp["launches"]:
        per_launch_s = comp["ms"] / comp["launches"] / 1e3
        flops_per_launch = comp["flops"] / comp["launches"]
        ach = flops_per_launch / per_launch_s / 1e12
        out["roofline"] = {"bound": "alu", "kernel": kname,
                           "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak,
                           "traffic": _traffic(kname.split(" ")[0]), "launches_per_step": comp["launches"] / args.steps,
                           "avg_launch_us": per_launch_s * 1e6, "algorithmic_flops_per_launch": flops_per_launch}
    if fkw:
        out["config"]["sketch_accepted"] = st["sketch_accepted"]
        out["config"]["sketch_rejected"] = st["sketch_rejected"]
    if not args.no_cpu_baseline and args.config == "c2":
        out["cpu_baseline"] = _cpu_baseline(args.cpu_side, patch, args.eps, args.nrhs, N)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
