"""Benchmark: CE factorization + FP64 PCG on one MI355X.

Default workload (``--config c3``): the 3D 7-point Dirichlet Laplacian on a
128^3 grid (N = 2,097,152), 4 x 4 x 4 Morton (octree) patches (B = 64), the
eight Morton siblings joined per level (Section 2.5), eps = 1e-4, one
right-hand side N(0,1) from default_rng(0), PCG in FP64 to a relative
residual of 1e-8.  The configured factor is the mixed-precision one: FP32
blocks, Schur products with BF16 inputs and FP32 accumulation on the matrix
cores, learned ranks (an MLP trained on a 48^3 problem before timing), the
dense remainder, the apply vectors and PCG in FP64.  The same workload with
the FP64 factor (exact ranks) is timed as a second leg in the same line, and
the configured arithmetic with exact ranks as a third (what the learned
ranks gain or lose).
``--config c2``: the 2D Laplacian on 1024^2 with 8 x 8 patches, eps = 1e-6,
16 right-hand sides, FP32 factor and the FP64 leg.  ``--config c4``: the
random-coefficient diffusion on 2048^2, 64 right-hand sides.  ``--config
c5``: 256 independent 2D and 3D Laplacians in one batched factorization
with an independent PCG per problem (``cae_factor_batched`` path; its 3D
problems reach blocks above 512 unknowns at the fourth level).

One step = numeric factorization (all levels, dense remainder) + PCG.  The
matrix, permutation and right-hand sides are resident on the GPU before the
timed region; the host symbolic analysis is timed separately
(``analysis_ms``; ``ms_per_step_with_analysis`` adds it).  Besides the
line's ``roofline`` (the far-row compression, FP64 arithmetic) the line
carries ``roofline_schur`` (the Schur updates against the matrix-core peak
of the configured arithmetic), each with the HBM traffic per launch from the
committed counter summary when it matches the kernel source.  Prints ONE
JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "factor+PCG time to 1e-8 residual (2D/3D Laplacian); block-op TFLOP/s vs peak"
FP64_PEAK = 78.6     # MI355X FP64 vector and FP64 matrix-core peak, TFLOP/s
FP32_PEAK = 157.3    # MI355X FP32 matrix-core (and vector) peak, TFLOP/s
BF16_PEAK = 2500.0   # MI355X dense BF16 matrix-core peak, TFLOP/s


def _log(msg):
    """Progress on stderr (the JSON result is the only stdout line)."""
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return platform.processor() or "unknown"


def _cpu_baseline(work, gpu_level1_steps_per_s, max_steps):
    """The FP64 oracle as it stands on a bounded sample of the same workload:
    the first k block steps of level 1 (Algorithm 2 on the same matrix,
    permutation, blocks, eps, coarsening and elimination order), nothing after
    them.  Measured, not scaled: once with one BLAS thread, once with a pool of
    all host cores on a shorter sample of the same steps (the oracle's step
    loop itself is sequential, and a thread pool only slows its small LAPACK
    calls down)."""
    from threadpoolctl import threadpool_limits

    import oracle
    ip, ix, dv = work["csr"]
    perm, bp, co = work["perm"], work["bp"], work["co"]
    opts = dict(eps=work["eps"], order="multicolour", coarsen=work["coarsen"])
    nproc = os.cpu_count() or 1
    # the steps of the first colour have empty far rows (nothing processed
    # yet: no compression); the sample runs through it and max_steps more
    k = int(min(work["M1"], work["first_colour"] + max_steps))
    k_all = int(min(work["M1"], work["first_colour"] + max(max_steps // 8, 1)))
    runs, setup = {}, {}
    for threads, kk in ((1, k), (nproc, k_all)):
        with threadpool_limits(limits=threads):
            t0 = time.perf_counter()
            f = oracle.ce_factor(ip, ix, dv, perm, bp, co, oracle.CEOptions(max_steps=kk, **opts))
            total = time.perf_counter() - t0
        runs[threads] = f.levels[0].seconds
        setup[threads] = total - runs[threads]
        _log(f"oracle: {kk} level-1 steps in {runs[threads]:.1f} s with {threads} BLAS thread(s)")
    return {
        "value": runs[1], "unit": "s", "cores": 1, "kind": "oracle",
        "sample": (f"the first {k} of the {work['M1']} level-1 block steps of this workload's factorization "
                   f"(the {work['first_colour']} steps of the first colour, whose far rows are empty, and "
                   f"{k - work['first_colour']} compressing steps) "
                   f"(Algorithm 2 in the oracle: gather, SVD compression, rotation, elimination, Schur update; "
                   f"FP64, NumPy/LAPACK), nothing after them; measured, not scaled; the oracle's set-up "
                   f"(permutation, level-1 blocks, symbolic pattern, {setup[1]:.1f} s) is not included"),
        "steps": k,
        "steps_per_s": k / runs[1],
        "all_cores": {"value": runs[nproc], "unit": "s", "cores": nproc, "steps": k_all,
                      "steps_per_s": k_all / runs[nproc],
                      "note": (f"the first {k_all} steps of the same sample with a BLAS pool of all host cores; "
                               "the step loop is sequential")},
        "nproc": nproc,
        "cpu_model": _cpu_model(),
        "gpu_level1_steps_per_s": gpu_level1_steps_per_s,
    }


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


def _workload(args, cae, problems):
    import numpy as np
    w = {"config": args.config}
    if args.config == "c2":
        dims, patch = (1024, 1024), (8, 8)
        A = problems.laplacian(dims)
        w.update(dims=dims, patch=patch, eps=1e-6, nrhs=16, coarsen="siblings", precision=cae.FP32, learned=False,
                 B=problems.rhs_normal(A.shape[0], 16, seed=1),
                 text=("2D 5-point Laplacian 1024x1024 (N=1048576), 8x8 Morton patches (B=64), eps=1e-6, 16 RHS "
                       "N(0,1) seed 1, PCG FP64 to 1e-8, multicolour order; configured leg: FP32 factor"))
    elif args.config == "c3":
        dims, patch = (128, 128, 128), (4, 4, 4)
        A = problems.laplacian(dims)
        w.update(dims=dims, patch=patch, eps=1e-4, nrhs=1, coarsen=args.coarsen or "siblings",
                 precision=cae.FP32_BF16, learned=not args.exact_ranks,
                 B=problems.rhs_normal(A.shape[0], 1, seed=0),
                 text=("3D 7-point Laplacian 128^3 (N=2097152), 4x4x4 octree (Morton) patches (B=64), "
                       f"{args.coarsen or 'siblings'} coarsening, eps=1e-4, 1 RHS N(0,1) seed 0, PCG FP64 to 1e-8, "
                       "multicolour order; configured leg: FP32 factor with BF16-input Schur products"
                       + (", exact ranks" if args.exact_ranks else
                          ", learned ranks (MLP trained on a 48^3 problem before timing)")))
    elif args.config == "c4":
        dims, patch = (2048, 2048), (8, 8)
        A, rng = problems.grf_diffusion_2d(2048)
        w.update(dims=dims, patch=patch, eps=1e-5, nrhs=64, coarsen="siblings", precision=cae.FP32, learned=False,
                 B=rng.standard_normal((64, A.shape[0])).T,
                 text=("2D -div(k grad u), k = exp(GRF, l=0.05, sigma=1, seed 2), 2048^2 (N=4194304), 8x8 patches "
                       "(B=64), eps=1e-5, 64 RHS N(0,1), PCG FP64 to 1e-8; configured leg: FP32 factor"))
    elif args.config == "c5":
        from paper_1603_09133_amd import batched
        kind, sides, rng = problems.batched_problem_draws(256, seed=3)
        mats, dl, pl = [], [], []
        for k, sd in zip(kind, sides):
            d = (int(sd), int(sd)) if k == 0 else (int(sd),) * 3
            mats.append(problems.laplacian(d))
            dl.append(d)
            pl.append((8, 8) if k == 0 else (2, 2, 4))
        mats = [m.tocsr() for m in mats]
        for m in mats:
            m.sort_indices()
        N = int(sum(m.shape[0] for m in mats))
        B = np.concatenate([rng.standard_normal((4, m.shape[0])) for m in mats], axis=1).T
        w.update(dims=None, patch=None, eps=1e-6, nrhs=4, coarsen=args.coarsen or "siblings", precision=cae.FP32,
                 learned=False, B=B, N=N, batch=(mats, dl, pl),
                 text=(f"256 independent Laplacians (2D side 64..512 with 8x8 patches, 3D side 16..64 with 2x2x4 "
                       f"patches; draws default_rng(3)), N={N} in one joint factorization (cae_analyze_batched), "
                       f"eps=1e-6, FP32 factor, exact ranks, 4 RHS per problem, an independent FP64 PCG per "
                       f"problem to 1e-8 (cae_pcg_solve_batched)"))
        return w
    else:
        raise SystemExit(f"unknown config {args.config}")
    w["A"] = A
    w["N"] = A.shape[0]
    w["csr"] = problems.to_csr_arrays(A)
    perm, bp, co = cae.grid_order(w["dims"], w["patch"])
    w.update(perm=perm, bp=bp, co=co, M1=len(bp) - 1)
    return w


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", choices=["c2", "c3", "c4", "c5"], default="c3")
    ap.add_argument("--coarsen", choices=["siblings", "pairs"], default=None)
    ap.add_argument("--exact-ranks", action="store_true", help="c3: exact ranks instead of learned ones")
    ap.add_argument("--fp64-steps", type=int, default=3, help="timed steps of the FP64 leg (at most --steps)")
    ap.add_argument("--no-fp64-leg", action="store_true")
    ap.add_argument("--exact-steps", type=int, default=2,
                    help="learned ranks: timed steps of the same arithmetic with exact ranks (0 = none)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=1024,
                    help="compressing level-1 steps of the oracle baseline sample")
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
    work = _workload(args, cae, problems)
    N = work["N"]
    order = cae.ORDER_MULTICOLOUR
    batch = work.get("batch")
    _log(f"{args.config}: N={N}, symbolic analysis")
    t = time.perf_counter()
    if batch:
        from paper_1603_09133_amd import batched
        an = batched.analyze(*batch, order=order, coarsen=work["coarsen"])
    else:
        ip, ix, dv = work["csr"]
        an = cae.Analysis(ip, ix, work["perm"], work["bp"], work["co"], order=order, coarsen=work["coarsen"])
    analysis_ms = (time.perf_counter() - t) * 1e3
    _log(f"analysis {analysis_ms:.0f} ms, {an.nlevels()} levels")
    wave1 = an.level_arrays(0)["wave"]
    work["first_colour"] = int(np.sum(wave1 == 0))
    work["M1"] = len(wave1)
    vals = batched.stacked_values(batch[0], dev) if batch else torch.from_numpy(dv).to(dev)
    b = torch.from_numpy(np.ascontiguousarray(work["B"].T)).to(dev)
    x = torch.empty_like(b)
    fkw = {}
    train_s = None
    if work["learned"]:
        from paper_1603_09133_amd import learned
        t = time.perf_counter()
        d2 = (48, 48, 48)
        A2 = problems.laplacian(d2)
        i2, x2, v2 = problems.to_csr_arrays(A2)
        p2, b2, c2 = cae.grid_order(d2, work["patch"])
        an2 = cae.Analysis(i2, x2, p2, b2, c2, order=order, coarsen=work["coarsen"])
        rec = learned.record(an2, torch.from_numpy(v2).to(dev), work["eps"], precision=cae.FP32)
        an2.close()
        params, _ = learned.train(rec, epochs=800, lr=1e-3)
        fkw = dict(rank_mode=cae.RANK_LEARNED_CAP, mlp_params=params)
        train_s = time.perf_counter() - t
        _log(f"MLP trained in {train_s:.1f} s on {int(rec.shape[0])} records")

    if args.copy_calibration_mib > 0:
        src = torch.ones(args.copy_calibration_mib * 2**18, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst

    def leg(name, prec, kw, steps, warmup):
        def step():
            f = cae.Factor(an, vals, work["eps"], precision=prec, timing=True, **kw)
            if batch:
                # an independent PCG per problem; per column the most iterations over the problems
                _, it, rel = f.pcg_batched(b, rtol=1e-8, maxit=1000, x=x)
                return f, it.max(axis=0), rel.max(axis=0)
            _, it, rel = f.pcg(b, rtol=1e-8, maxit=1000, x=x)
            return f, it, rel

        for k in range(warmup):
            tw = time.perf_counter()
            f, it, rel = step()
            f.close()
            torch.cuda.synchronize()
            _log(f"{name} warmup step {k + 1}/{warmup}: {(time.perf_counter() - tw) * 1e3:.0f} ms, "
                 f"PCG iterations max {int(np.max(it))}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        res = {"factor_ms": [], "compress_ms": 0.0, "compress_launches": 0, "compress_flops": 0.0,
               "schur_ms": 0.0, "schur_launches": 0, "schur_flops": 0.0}
        for k in range(steps):
            f, it, rel = step()
            st = f.stats()
            res["factor_ms"].append(st["factor_ms"])
            res["compress_ms"] += st["compress_ms"]
            res["compress_launches"] += st["compress_launches"]
            res["compress_flops"] += st["compress_flops"]
            res["schur_ms"] += st["schur_ms"]
            res["schur_launches"] += st["schur_launches"]
            res["schur_flops"] += st["schur_flops"]
            if k + 1 < steps:
                f.close()
            _log(f"{name} timed step {k + 1}/{steps} done")
        torch.cuda.synchronize()
        res["s_per_step"] = (time.perf_counter() - t0) / max(steps, 1)
        res.update(it=it, rel=rel, stats=st, level_ms=f.level_ms(), steps=steps)
        f.close()
        return res

    main_leg = leg("configured", work["precision"], fkw, args.steps, args.warmup)
    exact = None
    if fkw and args.exact_steps > 0:
        exact = leg("exact ranks", work["precision"], {}, min(args.steps, args.exact_steps), min(args.warmup, 1))
    f64 = None
    if not args.no_fp64_leg:
        n64 = min(args.steps, args.fp64_steps)
        f64 = leg("fp64", cae.FP64, {}, n64, min(args.warmup, 1))

    st = main_leg["stats"]
    fac_s = float(np.mean(main_leg["factor_ms"])) / 1e3
    ops = {"compress": st["compress_flops"], "rotate": st["rotate_flops"], "eliminate": st["elim_flops"],
           "schur": st["schur_flops"], "coarse": st["coarse_flops"]}
    tot = float(sum(ops.values()))
    dtype = {cae.FP32: "f32 factor + f64 PCG", cae.FP64: "f64",
             cae.FP32_BF16: "f32 factor with bf16-input Schur products + f64 PCG"}[work["precision"]]
    value = main_leg["s_per_step"]
    out = {
        "metric": METRIC,
        "value": value,
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": value * 1e3,
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": dtype,
        "data": "synthetic",
        "config": {
            "workload": work["text"],
            "factor_ms_mean": fac_s * 1e3,
            "level_ms": main_leg["level_ms"],
            "analysis_ms": analysis_ms,
            "ms_per_step_with_analysis": value * 1e3 + analysis_ms,
            "pcg_iters": main_leg["it"].tolist(),
            "relres_max": float(np.max(main_leg["rel"])),
            "converged": bool(np.all(main_leg["rel"] <= 1.0001e-8)),
            "levels": st["nlevels"],
            "coarse_dim": st["coarse_dim"],
            "factor_bytes": st["factor_bytes"],
            "block_op": {"tflops": tot / fac_s / 1e12, "peak_fp64": FP64_PEAK,
                         "frac_fp64": tot / fac_s / 1e12 / FP64_PEAK, "flops_per_step": ops,
                         "note": "algorithmic flops of compression, rotation, elimination, Schur update and "
                                 "dense remainder (model of cae_stats_t) / factor wall time"},
        },
    }
    if fkw:
        out["config"]["sketch_accepted"] = st["sketch_accepted"]
        out["config"]["sketch_rejected"] = st["sketch_rejected"]
        out["config"]["mlp_training_s"] = train_s
    if exact is not None:
        out["config"]["exact_ranks_leg"] = {
            "s_per_step": exact["s_per_step"], "steps": exact["steps"],
            "factor_ms_mean": float(np.mean(exact["factor_ms"])), "level_ms": exact["level_ms"],
            "pcg_iters": exact["it"].tolist(), "relres_max": float(np.max(exact["rel"])),
            "learned_speedup": exact["s_per_step"] / value,
            "note": "the configured arithmetic with exact ranks: learned_speedup > 1 means the learned ranks save time",
        }
    if f64 is not None:
        s64 = f64["stats"]
        out["config"]["fp64_leg"] = {
            "s_per_step": f64["s_per_step"], "steps": f64["steps"],
            "factor_ms_mean": float(np.mean(f64["factor_ms"])), "level_ms": f64["level_ms"],
            "pcg_iters": f64["it"].tolist(), "relres_max": float(np.max(f64["rel"])),
            "converged": bool(np.all(f64["rel"] <= 1.0001e-8)), "levels": s64["nlevels"],
            "coarse_dim": s64["coarse_dim"], "factor_bytes": s64["factor_bytes"],
            "speedup_of_configured_leg": f64["s_per_step"] / value,
        }
    # roofline of the far-row compression (a2 + a3: the paper's most costly
    # part), from HIP events recorded around its launches on the factor's
    # stream; its arithmetic is FP64 (also for an FP32 factor: FP64 Gram
    # matrices, pivoted Cholesky, Jacobi and reflectors), so the peak is the
    # FP64 rate
    if main_leg["compress_launches"]:
        per_launch_s = main_leg["compress_ms"] / main_leg["compress_launches"] / 1e3
        flops_per_launch = main_leg["compress_flops"] / main_leg["compress_launches"]
        ach = flops_per_launch / per_launch_s / 1e12
        kname = ("compress: one wave's far-row compressions (k_feat_mlp, k_compress_gram<float,64|128>, k_bg_gram, "
                 "k_bg_eig, k_bg_cert, k_bg_full, k_compress)")
        out["roofline"] = {"bound": "alu", "kernel": kname, "achieved": ach, "peak": FP64_PEAK, "unit": "TFLOP/s",
                           "frac": ach / FP64_PEAK, "traffic": _traffic("compress"),
                           "launches_per_step": main_leg["compress_launches"] / args.steps,
                           "avg_launch_us": per_launch_s * 1e6, "algorithmic_flops_per_launch": flops_per_launch}
    # the Schur updates (a7) the same way: products on the matrix cores in the
    # configured arithmetic (BF16 inputs with FP32 accumulation, FP32 or FP64)
    if main_leg["schur_launches"]:
        per_launch_s = main_leg["schur_ms"] / main_leg["schur_launches"] / 1e3
        flops_per_launch = main_leg["schur_flops"] / main_leg["schur_launches"]
        ach = flops_per_launch / per_launch_s / 1e12
        peak = {cae.FP32_BF16: BF16_PEAK, cae.FP32: FP32_PEAK, cae.FP64: FP64_PEAK}[work["precision"]]
        out["roofline_schur"] = {
            "bound": "mfma", "kernel": ("schur: one wave's Schur updates (k_schur_bf16, k_schur_big_bf16, "
                                        "k_schur_big_bf16w, or the FP32 / FP64 forms)"),
            "achieved": ach, "peak": peak, "unit": "TFLOP/s", "frac": ach / peak, "traffic": _traffic("schur"),
            "launches_per_step": main_leg["schur_launches"] / args.steps, "avg_launch_us": per_launch_s * 1e6,
            "algorithmic_flops_per_launch": flops_per_launch}
    if not args.no_cpu_baseline and not batch:
        lv1_s = main_leg["level_ms"][0] / 1e3
        out["cpu_baseline"] = _cpu_baseline(work, work["M1"] / lv1_s if lv1_s > 0 else None, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
