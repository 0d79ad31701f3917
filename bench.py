#!/usr/bin/env python3
"""Benchmark of the adaptive sketching solver on one MI355X.

Step = one complete adaptive PCG solve (SRHT sketch, FP64) of the n = 65536, d = 2048
workload (A = U diag(sigma) V^T with sigma_j = 1/j, nu = 1e-3, Lambda = 1 + U[0, 9],
b = A^T y, m_init = 16, rho = 1/8) to relative error 1e-10: every resketch, factorisation,
H.v pass and vector step is inside the timed region; A and b are resident in HBM before it
starts.  Printed value: seconds per solve (time-to-1e-10).  The solution of the last timed
step is checked against the oracle's refined reference on the host; the line says whether it
met 1e-10.

Extra legs (outside the timed region of the headline value):
  * roofline of the fused H.v kernel: HIP-event time of every launch inside the timed solves;
  * mixed precision vs FP64 on the n = 262144, d = 4096 workload (sigma_j = 0.995^j,
    nu = 1e-2), both validated against the oracle reference (skip with --no-mixed);
  * cpu_baseline: the oracle on the host cores (see cpu_baseline());
  * small_n4096_d256 (skip with --no-small): the n = 4096, d = 256 workload, time per solve and
    per step;
  * batched (skip with --no-batched): 64 uneven problems x 32 right-hand sides (n = 256 U{32..512},
    d = 256 U{1..8}, sigma_j = 0.98^j, nu log-uniform in [1e-4, 1e-1]), every step of all problems
    one replay of the captured grouped step, in FP32 storage + FP64 refinement and in FP64; eight
    problems (the four smallest nu, four spread over n d) validated against the oracle;
  * adjoint (skip with --no-adjoint): forward + backward of the autograd Function on n = 131072,
    d = 1024 (sigma_j = j^-1/2, nu = 1e-2), gradients validated against the dense oracle;
  * variants (skip with --no-variants): the headline workload solved with the Gaussian and
    SJLT sketches, with the transform-reuse SRHT and its nested form (variants), by adaptive
    IHS, by adaptive Polyak-IHS, and by the unpreconditioned CG baseline;
  * --skip-main --paper / --paper-large / --paper-e3: the synthetic nu-sweeps of the paper's
    numerical section (n = 16384 or 131072, d = 7000; n = 524288, d = 14000; sigma_j = 0.995^j)
    with its comparison set (including the direct Cholesky baseline);
  * --skip-main --dual: n < d through the dual problem (the OVA-Lung shape n = 1545, d = 10936,
    c = 2, and n = 8192, d = 32768) next to the primal solve; --dual-wide: the dual solve alone;
    --dual-large: the dual solve at n = 16384, d = 131072 with a primal-residual check.

--hv-only runs just fused H.v launches and a calibration copy (for rocprofv3 counter runs);
--sketch-only M runs just sketches (--sketch kind) of size M of the workload's A.
--factor-only M runs just factorisations (aes_factor) of an M x d Gaussian sketch.
--direct-only N D runs just the direct baseline (aes_solve_direct) on an N x D matrix.
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

METRIC = "time-to-1e-10 rel err per solve (s); Aᵀ(Ax) HBM GB/s; mixed vs FP64 speedup"
HBM_PEAK_GBPS = 8000.0
COUNTERS = os.path.join(ROOT, "profiles", "hv_fused_counters.json")


def log(msg):
    """Progress line on stderr (the JSON result line is the only stdout output)."""
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def sha256_file(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def load_traffic(n, d):
    """Measured HBM bytes per hv launch from the committed counter summary, if it was taken
    on this kernel source and this shape; else None."""
    try:
        with open(COUNTERS) as f:
            c = json.load(f)
    except (OSError, ValueError):
        return None
    src = os.path.join(ROOT, "paper_2104_14101_amd", "csrc", "k_hv.hip")
    if c.get("source_sha256") != sha256_file(src) or c.get("n") != n or c.get("d") != d:
        return None
    return c.get("bytes_per_launch")


def cpu_baseline(P_np, info, m_init):
    """Oracle (numpy FP64) timed on the host on a bounded sample of the workload: three H.v passes
    (median), SRHT sketches at the first, a middle and the final sketch size (the oracle's
    transform costs about the same at every m), and the factorisation of H_S at every sketch size
    of the solve (Woodbury below d, Cholesky from d on; timed on row blocks of the final sketch).
    Per solve = passes x H.v + the sketches interpolated over the solve's m sequence + the
    factorisations."""
    import numpy as np
    from threadpoolctl import threadpool_info

    from oracle import factor as ofac
    from oracle import sketch as osk
    from oracle import solvers

    A, lam, nu = P_np["A"], P_np["lam"], P_np["nu"]
    d = A.shape[1]
    p = np.random.default_rng(0).standard_normal((d, 1))
    t_hv = []
    for _ in range(3):
        t0 = time.perf_counter()
        solvers.hess_apply(A, nu, lam, p)
        t_hv.append(time.perf_counter() - t0)
    t_hv = float(np.median(t_hv))
    K = int(info["resketches"])
    ms = [min(m_init << k, int(info["final_m"])) for k in range(K + 1)]
    picks = sorted({0, K // 2, K})
    t_sk = {}
    SA_hi = None
    for k in picks:
        t0 = time.perf_counter()
        SA = osk.srht(A, ms[k], 1, k)
        t_sk[k] = time.perf_counter() - t0
        if k == K:
            SA_hi = SA
    sk_total = float(np.sum(np.interp(np.arange(K + 1), picks, [t_sk[k] for k in picks])))
    fac_total = 0.0
    for m in ms:
        t0 = time.perf_counter()
        ofac.SketchedHessian(SA_hi[:m], nu, lam)
        fac_total += time.perf_counter() - t0
    est = int(info["a_passes"]) * t_hv + sk_total + fac_total
    threads = max([x.get("num_threads", 1) for x in threadpool_info()] + [1])
    sample = 3 * t_hv + sum(t_sk.values()) + fac_total
    return {"value": est, "unit": "s", "cores": int(threads), "kind": "oracle",
            "sample": (f"3 H.v passes (median {t_hv:.3f} s), SRHT sketches at m = "
                       f"{', '.join(str(ms[k]) for k in picks)} ({', '.join(f'{t_sk[k]:.2f}' for k in picks)} s) and "
                       f"the {len(ms)} factorisations of the solve's m sequence ({fac_total:.2f} s) on the full "
                       f"workload; per solve = {info['a_passes']} passes + {len(ms)} sketches (interpolated) + "
                       f"{len(ms)} factorisations"),
            "sample_seconds": sample}


def reference_error(P_np, x, spectral=None):
    import numpy as np

    from oracle import reference

    xr = reference.reference_solution(P_np["A"], P_np["b"], P_np["nu"], P_np.get("lam"), spectral=spectral)
    return float(np.max(reference.rel_error(x, xr)))


def to_numpy(P):
    out = {}
    for k, v in P.items():
        out[k] = v.detach().cpu().numpy() if hasattr(v, "detach") else v
    return out


def timed_solves(aes, torch, A, b, nu, lam, opts, steps, warmup, profile=False, fn=None):
    fn = fn or aes.solve
    for _ in range(warmup):
        fn(A, b, nu, lam, **opts)
    torch.cuda.synchronize()
    infos = []
    t0 = time.perf_counter()
    x = None
    for _ in range(steps):
        x, info = fn(A, b, nu, lam, profile=profile, **opts)
        infos.append(info)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return x, infos, (t1 - t0) / steps


def hv_only(args):
    import torch

    import paper_2104_14101_amd as aes
    import synth

    w = synth.WORKLOADS[args.workload]
    # traffic does not depend on the values: a plain N(0,1) matrix of the workload's shape
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    A = torch.randn((w.n, w.d), dtype=torch.float64, device="cuda", generator=g)
    lam = 1.0 + 9.0 * torch.rand(w.d, dtype=torch.float64, device="cuda", generator=g)
    p = torch.randn(w.d, dtype=torch.float64, device="cuda", generator=g)
    for _ in range(args.steps):
        aes.hv(A, p, w.nu, lam)
    # calibration copy of known size: 1 GiB read + 1 GiB written
    src = torch.empty(2 ** 27, dtype=torch.float64, device="cuda").fill_(1.0)
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"hv_launches": args.steps, "n": w.n, "d": w.d, "copy_bytes_each_way": 2 ** 30}))


def sketch_only(args):
    import torch

    import paper_2104_14101_amd as aes
    import synth

    w = synth.WORKLOADS[args.workload]
    g = torch.Generator(device="cuda")
    g.manual_seed(5)
    A = torch.randn((w.n, w.d), dtype=torch.float64, device="cuda", generator=g)
    for k in range(args.steps):
        aes.sketch(A, args.sketch_only, kind=args.sketch, seed=1, k=k)
    torch.cuda.synchronize()
    print(json.dumps({"sketches": args.steps, "kind": args.sketch, "m": args.sketch_only, "n": w.n, "d": w.d}))


def factor_only(args):
    """aes_factor (Gram of an m x d sketch, Cholesky factor and its inverse) of a Gaussian sketch of
    the workload's width, with the workload's nu and Lambda = 1 + U[0, 9]; the kernels of the
    factorisation are the ones a solve runs after each resize (this entry point also copies L back)."""
    import torch

    import paper_2104_14101_amd as aes
    import synth

    w = synth.WORKLOADS[args.workload]
    g = torch.Generator(device="cuda")
    g.manual_seed(6)
    m = args.factor_only
    SA = torch.randn((m, w.d), dtype=torch.float64, device="cuda", generator=g) / m ** 0.5
    lam = 1.0 + 9.0 * torch.rand(w.d, dtype=torch.float64, device="cuda", generator=g)
    for _ in range(max(args.warmup, 1)):
        aes.factor(SA, w.nu, lam)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        aes.factor(SA, w.nu, lam)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"factorisations": args.steps, "m": m, "d": w.d, "ms_per_factor": ms}))


def direct_only(args):
    """aes_solve_direct (the direct baseline of Sec. 5: Gram of the whole A with nu^2 Lambda,
    Cholesky and inverse factor, two triangular products) on an N x D matrix of N(0, 1/N)
    entries, nu = 1e-2, Lambda = I, one right-hand side.  Values do not change the kernels' work."""
    import torch

    import paper_2104_14101_amd as aes

    n, d = args.direct_only
    g = torch.Generator(device="cuda")
    g.manual_seed(8)
    A = torch.randn((n, d), dtype=torch.float64, device="cuda", generator=g) / n ** 0.5
    b = torch.randn(d, dtype=torch.float64, device="cuda", generator=g)
    for _ in range(max(args.warmup, 1)):
        aes.solve_direct(A, b, 1e-2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        aes.solve_direct(A, b, 1e-2)
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / args.steps
    print(json.dumps({"direct_solves": args.steps, "n": n, "d": d, "ms_per_solve": ms,
                      "gram_flops": n * d * (d + 1)}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="pcg_n65536_d2048")
    ap.add_argument("--method", default="pcg", choices=["pcg", "ihs"])
    ap.add_argument("--sketch", default="srht", choices=["srht", "gauss", "sjlt", "srht_reuse", "srht_nested"])
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-variants", action="store_true", help="skip the Gaussian / SJLT / IHS / CG solves")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--hv-only", action="store_true")
    ap.add_argument("--sketch-only", type=int, default=0, metavar="M")
    ap.add_argument("--direct-only", type=int, nargs=2, default=None, metavar=("N", "D"),
                    help="only the direct baseline (aes_solve_direct) on an N x D matrix")
    ap.add_argument("--factor-only", type=int, default=0, metavar="M",
                    help="only aes_factor of an M x d sketch of the workload's width")
    ap.add_argument("--batched", action="store_true", help="with --skip-main: the batched leg")
    ap.add_argument("--adjoint", action="store_true", help="with --skip-main: the autograd leg")
    ap.add_argument("--no-batched", action="store_true", help="skip the batched leg of the default line")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the autograd leg of the default line")
    ap.add_argument("--no-small", action="store_true", help="skip the n = 4096, d = 256 leg")
    ap.add_argument("--all", action="store_true")
    ap.add_argument("--skip-main", action="store_true", help="run only the selected extra legs (profiling)")
    ap.add_argument("--mixed", action="store_true", help="with --skip-main: the mixed-precision leg")
    ap.add_argument("--paper", action="store_true",
                    help="with --skip-main: the synthetic nu-sweep of Sec. 5 at n=16384, d=7000")
    ap.add_argument("--paper-large", action="store_true",
                    help="with --skip-main: the same at n=131072, d=7000 (nu = 1e-2, 1e-3)")
    ap.add_argument("--dual", action="store_true",
                    help="with --skip-main: n < d through the dual (n=1545, d=10936, c=2; n=8192, d=32768) "
                         "next to the primal solve")
    ap.add_argument("--dual-wide", action="store_true",
                    help="with --skip-main: only the dual solve at n=8192, d=32768, nu=1e-2 (kernel profiles)")
    ap.add_argument("--dual-large", action="store_true",
                    help="with --skip-main: the dual solve at n=16384, d=131072 (beyond the primal's d limit)")
    ap.add_argument("--paper-e3", action="store_true",
                    help="with --skip-main: the same at n=524288, d=14000 (A is 58.7 GB; nu = 1e-2 .. 1e-4; "
                         "CG capped at 2000 steps; errors against PCG at m = 2d to 1e-12)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py: this build runs on one GPU only; the multi-GPU sharding of the solver is a design "
              "note, not an implemented path (use --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.hv_only:
        return hv_only(args)
    if args.sketch_only:
        return sketch_only(args)
    if args.factor_only:
        return factor_only(args)
    if args.direct_only:
        return direct_only(args)

    import numpy as np
    import torch

    import paper_2104_14101_amd as aes
    import synth

    if args.skip_main:
        out = {}
        if args.paper:
            out["paper_e1"] = paper_leg(aes, torch, synth, 16384, 7000, (1e-1, 1e-2, 1e-3, 1e-4))
        if args.paper_large:
            out["paper_e2"] = paper_leg(aes, torch, synth, 131072, 7000, (1e-2, 1e-3))
        if args.paper_e3:
            out["paper_e3"] = paper_leg(aes, torch, synth, 524288, 14000, (1e-2, 1e-3, 1e-4), cross=True,
                                        cg_iters=2000)
        if args.mixed:
            out["mixed_vs_fp64"] = mixed_leg(aes, torch, synth)
        if args.dual:
            # the OVA-Lung shape of Sec. 5 (n = 1545, d = 10936, c = 2), then a wider one
            out["dual_ova_lung_shape"] = dual_leg(aes, torch, synth, 1545, 10936, (1e-1, 1e-2), nrhs=2)
            out["dual_n8192_d32768"] = dual_leg(aes, torch, synth, 8192, 32768, (1e-1, 1e-2), ref="primal")
        if args.dual_wide:
            out["dual_n8192_d32768"] = dual_leg(aes, torch, synth, 8192, 32768, (1e-2,), ref="none", forms=("dual",))
        if args.dual_large:
            out["dual_n16384_d131072"] = dual_large_leg(aes, torch, synth)
        if args.batched or args.all:
            out["batched"] = batched_leg(aes, torch, synth)
        if args.adjoint or args.all:
            out["adjoint"] = adjoint_leg(aes, torch, synth)
        print(json.dumps(out), flush=True)
        return

    w = synth.WORKLOADS[args.workload]
    P = synth.make_workload(args.workload, seed=0, backend="torch", device="cuda")
    A, b, lam, nu = P["A"], P["b"], P["lam"], P["nu"]
    if w.lam == "identity":
        lam = None
    opts = dict(method=args.method, sketch=args.sketch, m_init=w.m_init, seed=1, tol=1e-10)
    log(f"main leg: {args.workload} {args.method} {args.sketch}, {args.warmup} warmup + {args.steps} timed solves")
    x, infos, sec = timed_solves(aes, torch, A, b, nu, lam, opts, args.steps, args.warmup, profile=True)
    info = infos[-1]
    n, d = w.n, w.d
    hv_ms = sum(i["time_hv_ms"] for i in infos)
    hv_n = sum(i["hv_launches"] for i in infos)
    hv_avg_s = hv_ms / max(hv_n, 1) / 1e3
    alg_bytes = n * d * 8 + 2 * d * 8
    achieved = alg_bytes / hv_avg_s / 1e9 if hv_avg_s > 0 else 0.0

    P_np = to_numpy(P)
    if lam is None:
        P_np["lam"] = None
    err = reference_error(P_np, x.cpu().numpy())

    out = {
        "metric": METRIC, "value": sec, "unit": "s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sec * 1e3, "higher_is_better": False, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": args.workload, "n": n, "d": d, "sigma": w.decay, "nu": nu, "lambda": w.lam,
                   "method": args.method, "sketch": args.sketch, "m_init": w.m_init, "rho": 0.125, "tol": 1e-10,
                   "parallelism": "single GPU"},
        "valid": bool(err <= 1e-10), "rel_err": err,
        "solve": {k: info[k] for k in ("iterations", "attempts", "final_m", "resketches", "a_passes",
                                       "time_sketch_ms", "status")},
        "roofline": {"kernel": "hv_fused (A^T(A p) single pass)", "bound": "hbm", "achieved": achieved,
                     "peak": HBM_PEAK_GBPS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBPS,
                     "traffic": load_traffic(n, d), "alg_bytes_per_launch": alg_bytes,
                     "avg_launch_us": hv_avg_s * 1e6, "launches_timed": hv_n},
    }

    if not args.no_variants:
        log("variants leg")
        out["variants"] = variants_leg(aes, torch, A, b, nu, lam, w, P_np, args)
    if not args.no_mixed:
        log("mixed vs fp64 leg")
        out["mixed_vs_fp64"] = mixed_leg(aes, torch, synth)

    if not args.no_small:
        log("small n=4096 d=256 leg")
        out["small_n4096_d256"] = small_leg(aes, torch, synth)
    if not args.no_batched:
        log("batched 64 x 32 rhs leg")
        out["batched"] = batched_leg(aes, torch, synth)
    if not args.no_adjoint:
        log("adjoint leg")
        out["adjoint"] = adjoint_leg(aes, torch, synth)

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle on the host) leg")
        cb = cpu_baseline(P_np, info, w.m_init)
        cb["gpu_speedup"] = cb["value"] / sec
        out["cpu_baseline"] = cb
    print(json.dumps(out), flush=True)


def variants_leg(aes, torch, A, b, nu, lam, w, P_np, args):
    """The same workload solved with the other sketches and methods (3 timed solves each; srht_reuse
    is the transform-reuse variant and srht_nested its nested form with the incremental Gram, not
    the paper's method; polyak the adaptive heavy-ball IHS of the appendix) and by the
    unpreconditioned CG baseline (one timed solve)."""
    res = {}
    for method, sketch in (("pcg", "gauss"), ("pcg", "sjlt"), ("pcg", "srht_reuse"), ("pcg", "srht_nested"),
                           ("ihs", "srht"), ("ihs", "sjlt"), ("polyak", "srht"), ("cg", None)):
        if method == args.method and sketch == args.sketch:
            continue
        opts = dict(method=method, m_init=w.m_init, seed=1, tol=1e-10, max_iter=2000)
        if sketch:
            opts["sketch"] = sketch
        else:
            opts["max_iter"] = 50000  # the unpreconditioned baseline: one timed solve
        x, infos, sec = timed_solves(aes, torch, A, b, nu, lam, opts, 3 if sketch else 1, 1 if sketch else 0)
        err = reference_error(P_np, x.cpu().numpy())
        i = infos[-1]
        res[f"{method}_{sketch}" if sketch else method] = {
            "s_per_solve": sec, "rel_err": err, "valid": bool(err <= 1e-10), "status": i["status"],
            "iterations": i["iterations"], "final_m": i["final_m"], "a_passes": i["a_passes"],
            "time_sketch_ms": i["time_sketch_ms"]}
    return res


def paper_leg(aes, torch, synth, n, d, nus, cross=False, cg_iters=20000):
    """The synthetic experiments of Sec. 5 (sigma_j = 0.995^j, Lambda = I, b = A^T y) at n x d over
    a sweep of nu, with the paper's comparison set: adaptive PCG and IHS from m = 1 (SRHT and
    SJLT), PCG with the fixed size m = 2d, unpreconditioned CG and the direct Cholesky solve of
    the full H (one untimed and one timed solve); plus adaptive PCG with the
    transform-reuse SRHT (a variant; not with cross=True, to keep E3's footprint).  One timed solve each (the
    first solve of each problem is repeated untimed).  Error against the oracle's refined
    reference; with cross=True (sizes the host oracle cannot take) against a PCG solve at
    m = 2d to 1e-12 instead."""
    import numpy as np

    from oracle import reference

    print(json.dumps({"paper": [n, d, "generating"]}), file=sys.stderr, flush=True)
    P = synth.make_problem(n, d, "geo:0.995", nus[0], seed=0, backend="torch", device="cuda",
                           ortho="cholqr" if cross else "qr")
    A, b = P["A"], P["b"]
    torch.cuda.empty_cache()
    print(json.dumps({"paper": [n, d, "generated"]}), file=sys.stderr, flush=True)
    P_np = None if cross else to_numpy(P)
    runs = [("adaptive_pcg_srht", dict(method="pcg", sketch="srht", m_init=1)),
            ("adaptive_pcg_sjlt", dict(method="pcg", sketch="sjlt", m_init=1)),
            ("adaptive_ihs_srht", dict(method="ihs", sketch="srht", m_init=1)),
            ("adaptive_ihs_sjlt", dict(method="ihs", sketch="sjlt", m_init=1)),
            ("pcg_m2d_srht", dict(method="pcg", sketch="srht", m_init=2 * d, adaptive=False)),
            ("pcg_m2d_sjlt", dict(method="pcg", sketch="sjlt", m_init=2 * d, adaptive=False)),
            ("cg", dict(method="cg", max_iter=cg_iters)),
            ("direct", None)]
    if not cross:
        # the stored transform of the reuse variant would add n' x d doubles (58.7 GB in E3)
        runs.insert(2, ("adaptive_pcg_srht_reuse", dict(method="pcg", sketch="srht_reuse", m_init=1)))
    out = {"n": n, "d": d, "sigma": "0.995^j", "nu": {},
           "reference": "PCG at m = 2d to 1e-12" if cross else "oracle refined reference"}
    for nu in nus:
        if cross:
            xr_t, _ = aes.solve(A, b, nu, None, method="pcg", sketch="srht", m_init=2 * d, adaptive=False, seed=7,
                                tol=1e-12, max_iter=2000)
            xr = xr_t.cpu().numpy()
        else:
            xr = reference.reference_solution(P_np["A"], P_np["b"], nu, None, spectral=(P_np["V"], P_np["sigma"]))
        res = {"d_e": reference.effective_dimension_closed(P["sigma"], nu)}
        for name, kw in runs:
            if name == "direct":
                # the direct baseline: one untimed and one timed Cholesky solve of the full H
                aes.solve_direct(A, b, nu)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                x = aes.solve_direct(A, b, nu)
                torch.cuda.synchronize()
                sec = time.perf_counter() - t0
                err = float(np.max(reference.rel_error(x.cpu().numpy(), xr)))
                res[name] = {"s_per_solve": sec, "rel_err": err, "valid": bool(err <= 1e-10), "status": "ok"}
                print(json.dumps({"paper": [n, d, nu, name, round(sec, 5)]}), file=sys.stderr, flush=True)
                continue
            opts = dict(seed=1, tol=1e-10, max_iter=2000)
            opts.update(kw)
            if kw.get("method") != "cg":
                opts["trace_cap"] = 1024  # the per-attempt series (the axes of the paper's plots)
            x, infos, sec = timed_solves(aes, torch, A, b, nu, None, opts, 1, 1 if name == runs[0][0] else 0)
            err = float(np.max(reference.rel_error(x.cpu().numpy(), xr)))
            i = infos[-1]
            res[name] = {"s_per_solve": sec, "rel_err": err, "valid": bool(err <= 1e-10), "status": i["status"],
                         "iterations": i["iterations"], "final_m": i["final_m"], "a_passes": i["a_passes"],
                         "time_sketch_ms": i["time_sketch_ms"]}
            if i.get("trace"):
                tr = i["trace"]
                res[name]["series"] = {
                    "t": [e["t"] for e in tr], "m": [e["m"] for e in tr], "accept": [int(e["accept"]) for e in tr],
                    "log10_dtilde": [round(math.log10(e["dtilde"]), 3) if e["dtilde"] > 0 else None for e in tr],
                    "time_ms": [round(e["time_ms"], 2) for e in tr]}
            print(json.dumps({"paper": [n, d, nu, name, round(sec, 5), i["iterations"], i["final_m"]]}),
                  file=sys.stderr, flush=True)
        out["nu"][f"{nu:g}"] = res
    return out


def dual_leg(aes, torch, synth, n, d, nus, nrhs=1, ref="oracle", forms=("dual", "primal")):
    """n < d through the dual problem of Sec. 1 (aes_solve_dual) next to the primal solve of the
    same problem, adaptive PCG with the SRHT from m = 1, tol 1e-10, Lambda = I,
    sigma_j = 0.995^j over the n directions, b = A^T y.  Errors of x against the oracle's
    refined reference (ref="oracle"), against a primal PCG solve to 1e-12 (ref="primal"), or
    not at all (ref="none": the dual solve alone, for kernel profiles)."""
    import numpy as np

    from oracle import reference

    P = synth.make_wide_problem(n, d, "geo:0.995", nus[0], nrhs=nrhs, seed=0, backend="torch", device="cuda")
    A, b = P["A"], P["b"]
    P_np = to_numpy(P) if ref == "oracle" else None
    out = {"n": n, "d": d, "c": nrhs, "sigma": "0.995^j", "nu": {},
           "reference": {"oracle": "oracle refined reference", "primal": "primal PCG to 1e-12", "none": None}[ref]}
    for nu in nus:
        xr = None
        if ref == "primal":
            xr_t, _ = aes.solve(A, b, nu, None, method="pcg", sketch="srht", m_init=1, seed=7, tol=1e-12)
            xr = xr_t.cpu().numpy()
        elif ref == "oracle":
            xr = reference.reference_solution(P_np["A"], P_np["b"], nu, None)
        res = {"d_e": reference.effective_dimension_closed(P["sigma"], nu)}
        for name in forms:
            fn = aes.solve_dual if name == "dual" else aes.solve
            opts = dict(method="pcg", sketch="srht", m_init=1, seed=1, tol=1e-10)
            x, infos, sec = timed_solves(aes, torch, A, b, nu, None, opts, 3, 1, fn=fn)
            i = infos[-1]
            err = float(np.max(reference.rel_error(x.cpu().numpy(), xr))) if xr is not None else None
            res[name] = {"s_per_solve": sec, "rel_err": err, "status": i["status"], "iterations": i["iterations"],
                         "final_m": i["final_m"], "a_passes": i["a_passes"], "time_sketch_ms": i["time_sketch_ms"]}
            print(json.dumps({"dual_leg": [n, d, nu, name, round(sec, 5), i["iterations"], i["final_m"], err]}),
                  file=sys.stderr, flush=True)
        if len(forms) == 2:
            res["primal_over_dual"] = res["primal"]["s_per_solve"] / res["dual"]["s_per_solve"]
        out["nu"][f"{nu:g}"] = res
    return out


def dual_large_leg(aes, torch, synth):
    """The dual solve at n = 16384, d = 131072 (A and B = Lambda^{-1/2} A^T are 17 GB each), where
    the primal path does not apply (d > 32768) and the host oracle is too slow: the check is the
    relative primal residual ||b - A^T (A x) - nu^2 x|| / ||b||, formed with torch in FP64 after the
    timed solves (a check only, outside the timed region)."""
    n, d, nu = 16384, 131072, 1e-2
    P = synth.make_wide_problem(n, d, "geo:0.995", nu, seed=0, backend="torch", device="cuda")
    A, b = P["A"], P["b"]
    torch.cuda.empty_cache()
    print(json.dumps({"dual_large": [n, d, "generated"]}), file=sys.stderr, flush=True)
    opts = dict(method="pcg", sketch="srht", m_init=1, seed=1, tol=1e-10)
    x, infos, sec = timed_solves(aes, torch, A, b, nu, None, opts, 2, 1, fn=aes.solve_dual)
    r = b - A.T @ (A @ x) - nu * nu * x
    res = float(torch.linalg.norm(r) / torch.linalg.norm(b))
    i = infos[-1]
    return {"n": n, "d": d, "nu": nu, "sigma": "0.995^j", "s_per_solve": sec, "rel_residual": res,
            "status": i["status"], "iterations": i["iterations"], "final_m": i["final_m"],
            "a_passes": i["a_passes"], "time_sketch_ms": i["time_sketch_ms"]}


def mixed_leg(aes, torch, synth):
    name = "mixed_n262144_d4096"
    w = synth.WORKLOADS[name]
    P = synth.make_workload(name, seed=0, backend="torch", device="cuda")
    A, b, nu = P["A"], P["b"], P["nu"]
    res = {"workload": name, "n": w.n, "d": w.d}
    xs = {}
    for prec in ("fp64", "mixed"):
        opts = dict(method="pcg", sketch="srht", m_init=w.m_init, seed=1, tol=1e-10, precision=prec)
        x, infos, sec = timed_solves(aes, torch, A, b, nu, None, opts, 2, 1)
        xs[prec] = x.cpu().numpy()
        res[prec] = {"s_per_solve": sec, "iterations": infos[-1]["iterations"], "final_m": infos[-1]["final_m"],
                     "refine_sweeps": infos[-1]["refine_sweeps"], "status": infos[-1]["status"]}
    P_np = to_numpy(P)
    P_np["lam"] = None
    import numpy as np

    from oracle import reference

    xr = reference.reference_solution(P_np["A"], P_np["b"], nu, None, spectral=(P_np["V"], P_np["sigma"]))
    for prec in ("fp64", "mixed"):
        e = float(np.max(reference.rel_error(xs[prec], xr)))
        res[prec]["rel_err"] = e
        res[prec]["valid"] = bool(e <= 1e-10)
    res["speedup"] = res["fp64"]["s_per_solve"] / res["mixed"]["s_per_solve"]
    # the same mixed solves when the caller declares A unchanged (the FP32 copy of the first solve
    # reused); reported beside the comparison above, which casts A in every solve
    opts = dict(method="pcg", sketch="srht", m_init=w.m_init, seed=1, tol=1e-10, precision="mixed",
                keep_fp32_copy=True)
    _, infos, sec = timed_solves(aes, torch, A, b, nu, None, opts, 2, 1)
    res["mixed_keep_fp32_copy"] = {"s_per_solve": sec, "status": infos[-1]["status"],
                                   "speedup_vs_fp64": res["fp64"]["s_per_solve"] / sec}
    return res


def spectral_error(P_np, x):
    """Per-column ||x - x*|| / ||x|| of a synthetic problem A = U diag(sigma) V^T (Lambda = I):
    the oracle's extended-precision residual r = b - H x mapped by the spectral inverse
    V diag(1 / (sigma^2 + nu^2)) V^T (x* - x = H^{-1} r)."""
    import numpy as np

    from oracle import reference

    r = reference.residual_extended(P_np["A"], P_np["b"], P_np["nu"], None, x, threads=16).astype(np.float64)
    w = 1.0 / (np.asarray(P_np["sigma"], dtype=np.float64) ** 2 + P_np["nu"] ** 2)
    V = P_np["V"]
    e = V @ (w[:, None] * (V.T @ r))
    return np.linalg.norm(e, axis=0) / np.linalg.norm(x, axis=0)


def batched_leg(aes, torch, synth, nvalidate=8):
    """64 uneven problems x 32 right-hand sides, every step of all problems one replay of the
    captured grouped step; FP32 storage + FP64 refinement, then FP64.  The 4 worst-conditioned
    problems (smallest nu) and 4 spread over n d are validated with the oracle's
    extended-precision residual (all 64 are validated by the GPU test suite)."""
    import numpy as np

    specs = synth.batched_specs(64, seed=0)
    probs, keep = [], []
    for i, sp in enumerate(specs):
        P = synth.make_problem(sp["n"], sp["d"], sp["decay"], sp["nu"], nrhs=32, seed=1000 + i, backend="torch",
                               device="cuda")
        probs.append(dict(A=P["A"], b=P["b"], nu=P["nu"]))
        keep.append(P)
    torch.cuda.synchronize()
    nd = [sp["n"] * sp["d"] for sp in specs]
    res = {"problems": 64, "rhs": 32, "sum_nd": int(sum(nd))}
    outs = {}
    for prec, steps in (("mixed_fp32", 2), ("fp64", 1)):
        aes.solve_batched(probs, tol=1e-10, precision=prec, m_init=16, seed=7)  # warmup
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            r = aes.solve_batched(probs, tol=1e-10, precision=prec, m_init=16, seed=7)
        torch.cuda.synchronize()
        sec = (time.perf_counter() - t0) / steps
        outs[prec] = r
        infos = [i for _, i in r]
        # useful work of the grouped products: 4 n d flops per column per step attempt
        flops = sum(4.0 * nd[p] * 32 * infos[p]["attempts"] for p in range(64))
        res[prec] = {"s_per_batch": sec, "statuses_ok": sum(1 for i in infos if i["status"] == "ok"),
                     "max_final_m": max(i["final_m"] for i in infos),
                     "max_attempts": max(i["attempts"] for i in infos),
                     "sum_attempts": sum(i["attempts"] for i in infos),
                     "sum_sketch_ms": sum(i["time_sketch_ms"] for i in infos),
                     "sum_resketches": sum(i["resketches"] for i in infos),
                     "sum_refine_sweeps": sum(i["refine_sweeps"] for i in infos),
                     "step_products_tflop": flops / 1e12}
    by_nu = sorted(range(64), key=lambda i: specs[i]["nu"])[:nvalidate // 2]
    order = sorted(range(64), key=lambda i: nd[i])
    spread = [order[0], order[21], order[42], order[63]]
    pick = sorted(set(by_nu) | set(spread))
    log(f"batched: validating problems {pick} against the oracle residual")
    for prec in ("mixed_fp32", "fp64"):
        res[prec]["per_problem_max_err"] = {}
    for i in pick:
        Pn = to_numpy(keep[i])
        for prec in ("mixed_fp32", "fp64"):
            e = float(np.max(spectral_error(Pn, outs[prec][i][0].cpu().numpy())))
            res[prec]["per_problem_max_err"][str(i)] = e
        log(f"batched: problem {i} checked")
    for prec in ("mixed_fp32", "fp64"):
        errs = list(res[prec]["per_problem_max_err"].values())
        res[prec]["validated_problems"] = pick
        res[prec]["max_rel_err"] = max(errs)
        res[prec]["valid"] = bool(max(errs) <= 1e-10 and res[prec]["statuses_ok"] == 64)
    res["speedup_mixed_vs_fp64"] = res["fp64"]["s_per_batch"] / res["mixed_fp32"]["s_per_batch"]
    return res


def small_leg(aes, torch, synth, steps=20):
    """The n = 4096, d = 256 workload (A of 8.4 MB, resident in cache): time per solve and per
    attempted step, validated against the oracle's refined reference."""
    P = synth.make_workload("pcg_n4096_d256", seed=0, backend="torch", device="cuda")
    opts = dict(m_init=8, seed=1, tol=1e-10)
    x, infos, sec = timed_solves(aes, torch, P["A"], P["b"], P["nu"], None, opts, steps, 3)
    info = infos[-1]
    P_np = to_numpy(P)
    P_np["lam"] = None
    err = reference_error(P_np, x.cpu().numpy())
    return {"workload": "pcg_n4096_d256", "s_per_solve": sec, "us_per_attempted_step": sec * 1e6 / info["attempts"],
            "us_per_iteration": sec * 1e6 / max(info["iterations"], 1), "iterations": info["iterations"],
            "attempts": info["attempts"], "final_m": info["final_m"], "rel_err": err, "valid": bool(err <= 1e-10)}


def adjoint_leg(aes, torch, synth):
    import numpy as np

    from oracle import adjoint, reference

    P = synth.make_workload("adjoint_n131072_d1024", seed=0, backend="torch", device="cuda", with_xt=True)
    opts = dict(m_init=16, seed=3, tol=1e-12)

    def step():
        A = P["A"].detach().requires_grad_(True)
        b = P["b"].detach().requires_grad_(True)
        ln = torch.tensor(np.log(P["nu"]), dtype=torch.float64, device="cuda", requires_grad=True)
        x = aes.SketchSolve.apply(A, b, ln, None, opts)
        loss = 0.5 * torch.sum((x - P["xt"]) ** 2)
        loss.backward()
        return A, b, ln

    step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    A, b, ln = step()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    Pn = to_numpy(P)
    xs = reference.reference_solution(Pn["A"], Pn["b"], Pn["nu"], None, spectral=(Pn["V"], Pn["sigma"]))
    _, adj, db, dA, dln = adjoint.gradients(Pn["A"], Pn["b"], Pn["nu"], xs - Pn["xt"], x=xs)
    e = {"db": float(np.max(np.abs(b.grad.cpu().numpy() - db)) / np.max(np.abs(db))),
         "dA": float(np.max(np.abs(A.grad.cpu().numpy() - dA)) / np.max(np.abs(dA))),
         "dlognu": float(abs(ln.grad.item() - dln) / abs(dln))}
    return {"workload": "adjoint_n131072_d1024", "s_forward_backward": sec, "grad_rel_err": e,
            "valid": bool(max(e.values()) <= 1e-9)}


if __name__ == "__main__":
    main()
