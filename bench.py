"""Benchmark of the RS-S hot path on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W]

Workload: Helmholtz kappa = 50 on the 512 x 512 cell-centre grid of [0,1]^2
(N = 262144), A_ij = h^2 (i/4) H0^(1)(kappa |x_i - x_j|), A_ii = 1, leaf 64,
ID tolerance 1e-6, 128 proxy points, 16 complex N(0,1) right-hand sides
(seed 2).  Synthetic inputs; everything resident on the GPU before timing.

One step = the whole hot path, both precision forms:
  1. factor in complex64 (FP64 pivot/rank decisions)          -> t_fact32
  2. solve 16 RHS, FP64-refined to relres <= 1e-10              -> t_solve32
  3. factor in complex128                                       -> t_fact64
  4. solve 16 RHS in complex128, FP64-refined to relres <= 1e-10 -> t_solve64
  5. SOLVE_REPS single applications of each factorization (latency samples)

The headline value is factor unknowns/s of the FP32+refine form,
N * K / sum(t_fact32); the FP64 figure, times to 1e-10 and solve p50/p99 are
reported beside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

SOLVE_REPS = 20
# HBM bytes per k_residual launch at this workload: rocprofv3 FETCH_SIZE and
# WRITE_SIZE, each scaled by the counts of a 1 GiB elementwise copy.  Valid for
# the kernel as measured; None when the kernel changes until measured again.
RESIDUAL_TRAFFIC_B = 1.074e+10
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TF = 78.6
FP32_MFMA_PEAK_TF = 157.3


def host_description():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return {"nproc": os.cpu_count(), "model": model}


def host_threads():
    """the host cores this process may use (the GPU machine grants a share of them)"""
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count() or 1
    cap = int(os.environ.get("OMP_NUM_THREADS", n) or n)
    return max(1, min(n, cap))


def cpu_baseline():
    """The oracle, as it stands, on a bounded sample of the same workload: the
    128 x 128 corner of the 512^2 grid (same h, kappa, weight, tol, leaf, proxy
    count), FP64 factorization, timed with BLAS limited to one thread and with
    all the host threads this process may use."""
    import threadpoolctl
    from oracle import rss as orss
    from paper_2310_15458_amd import workloads as W
    w = W.helmholtz_512()
    P = W.grid_points(w.n)
    side = 128
    ix = np.arange(w.n * w.n) % w.n
    iy = np.arange(w.n * w.n) // w.n
    sel = (ix < side) & (iy < side)
    Ps = P[sel]
    res = {}
    for nt in (1, host_threads()):
        with threadpoolctl.threadpool_limits(nt):
            t0 = time.perf_counter()
            orss.factor(Ps, w.kernel, w.tol, w.leaf, orss.Options(n_proxy=w.n_proxy),
                        root=(0.0, 0.0, side / w.n))
            res[nt] = time.perf_counter() - t0
    nt_all = max(res)
    best = min(res, key=lambda k: res[k])
    return {"value": Ps.shape[0] / res[best], "unit": "unknowns/s", "cores": best, "kind": "oracle",
            "sample": f"FP64 factorization of the {side}x{side} corner of the 512^2 grid "
                      f"({Ps.shape[0]} unknowns, same h/kappa/tol/leaf)",
            "threads": {str(k): {"seconds": v, "unknowns_per_s": Ps.shape[0] / v} for k, v in res.items()},
            "host": host_description(), "blas_threads_all": nt_all}


def paper_matrices(torch, rss, W, n=512, eps=1e-6):
    """The paper's own matrices (Sec. 5) at N = n^2: first-kind Laplace
    (eqs. e:a1, e:a1i) solved by CG and Lippmann-Schwinger Helmholtz kappa = 25
    (eqs. e:b1, e:b2) by GMRES, each preconditioned by its FP64 factorization,
    to relres 1e-12 (Tab. t:notations n_it), uniform random b (seed 0)."""
    out = {}
    for name, kern, method in (("laplace_first_kind", W.paper_laplace(n), "cg"),
                               ("lippmann_schwinger_k25", W.paper_helmholtz(n, 25.0), "gmres")):
        P = W.grid_points(n)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rss.Factorization(P, kern, eps, 64, n_proxy=64 if kern.kind == "laplace" else 128)
        t_fact = time.perf_counter() - t0
        op = rss.GridOperator(kern, n)
        b = W.uniform_rhs(n * n, 1, 0)
        x1 = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
        F.apply(x1)
        relres1 = float(np.linalg.norm(op.residual(x1, torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t())
                                       .cpu().numpy()) / np.linalg.norm(b))
        Bd = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
        st = rss.krylov(F, op, Bd, method=method, tol=1e-12, maxit=100)
        out[name] = {"N": n * n, "eps": eps, "method": method, "t_factor_ms": t_fact * 1e3,
                     "relres_one_apply": relres1, "n_it": st["iters"], "relres": st["relres"],
                     "t_krylov_ms": st["t_ms"]}
        op.close()
        F.close()
    return out


def _ls_case(torch, rss, W, n, kappa, eps, unprec_maxit=0):
    """One LS Helmholtz problem (eqs. e:b1, e:b2) at N = n^2: FP64
    factorization (timed after an untimed one of the same problem), the
    relres of one application, GMRES preconditioned by it to 1e-12 (n_it), and
    optionally GMRES(20) without a preconditioner (Tab. t:h2's last column)."""
    P = W.grid_points(n)
    kern = W.paper_helmholtz(n, kappa)
    # untimed first factorization: the factor tuner meets this size's box buckets
    rss.Factorization(P, kern, eps, 64).close()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    F = rss.Factorization(P, kern, eps, 64)
    t_fact = time.perf_counter() - t0
    info = F.info()
    op = rss.GridOperator(kern, n)
    b = W.uniform_rhs(n * n, 1, 0)
    B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
    x1 = B.clone()
    F.apply(x1)
    relres1 = float(torch.linalg.norm(op.residual(x1, B)) / torch.linalg.norm(B))
    X = B.clone()
    st = rss.krylov(F, op, X, method="gmres", tol=1e-12, maxit=100)
    out = {"N": n * n, "kappa": kappa, "eps": eps, "t_factor_ms": t_fact * 1e3,
           "ranks": [round(a / c, 1) for a, c in zip(info["rank_sum"], info["box_count"]) if c],
           "device_GB": info["device_bytes"] / 1e9, "relres_one_apply": relres1,
           "n_it": st["iters"], "relres": st["relres"], "t_solve_ms": st["t_ms"]}
    F.close()
    if unprec_maxit:
        X = B.clone()
        s0 = rss.krylov(None, op, X, method="gmres", tol=1e-12, maxit=unprec_maxit, restart=20)
        out.update({"n_it_unpreconditioned": s0["iters"], "relres_unpreconditioned": s0["relres"],
                    "t_unpreconditioned_ms": s0["t_ms"]})
    op.close()
    return out


def tolerance_and_frequency(torch, rss, W):
    """Tab. t:cpp's tolerance sweep (LS Helmholtz kappa = 25, eps 1e-3 ...
    1e-12) at N = 512^2, and Tab. t:h2's rising frequency kappa = pi sqrt(N) / 16
    (32 points per wavelength) at N = 256^2, 512^2, 1024^2 with eps = 1e-6,
    including the GMRES(20) count without a preconditioner."""
    sweep = [_ls_case(torch, rss, W, 512, 25.0, eps) for eps in (1e-3, 1e-6, 1e-9, 1e-12)]
    freq = [_ls_case(torch, rss, W, n, math.pi * n / 16, 1e-6, unprec_maxit=3000) for n in (256, 512, 1024)]
    return {"tolerance_sweep_ls_k25_n512": sweep, "rising_frequency_eps1e-6": freq}


def batched_sweep(torch, rss, W, reps=4):
    """256 independent problems (n uniform over {32,48,64,96,128}, Laplace or
    Helmholtz kappa ~ U[5,40], leaf 64, tol 1e-6, FP64, one RHS each, seed 3),
    factored in one batched sweep and solved in one batched apply."""
    probs = W.batched_problems()
    Ps = [W.grid_points(p.n) for p in probs]
    Ks = [p.kernel for p in probs]
    Bs = [torch.from_numpy(np.ascontiguousarray(p.rhs.T)).cuda().t() for p in probs]
    tot = sum(P.shape[0] for P in Ps)
    tf, ta = [], []
    for r in range(reps + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rss.factor_batch(Ps, Ks, 1e-6, 64)
        t1 = time.perf_counter()
        X = [B.clone() for B in Bs]
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        rss.apply_batch(F, X)
        t3 = time.perf_counter()
        for f in F[::-1]:
            f.close()
        if r > 0:
            tf.append(t1 - t0)
            ta.append(t3 - t2)
    tab = [e for e in rss.factor_tuning() if e["precision_bytes"] == 8]
    return {"problems": len(probs), "unknowns": tot,
            "factor_ms": float(np.median(tf) * 1e3), "factor_unknowns_per_s": tot / float(np.median(tf)),
            "factor_ms_min": float(np.min(tf) * 1e3),
            "apply_ms": float(np.median(ta) * 1e3), "apply_unknowns_per_s": tot / float(np.median(ta)),
            "reps": reps,
            "factor_tuning": {"buckets": len(tab),
                              "targets": sorted({e["target_workgroups"] for e in tab}),
                              "table": tab}}


def serving(torch, rss, W, count=300, sides=(128, 256, 512), max_nrhs=256, load=0.7, budget=32e9):
    """A request stream through the solve server (rss_server_*) with the
    serving workload's mix and size classes: Poisson arrivals, 20% factor
    jobs on n x n grids, n in {128, 256, 512}, Helmholtz kappa ~ U[10,60],
    solves with nrhs ~ U{1..256}, FP32+refine to 1e-10 with the FFT grid
    residual, LRU eviction.  Fewer requests than the full stream (300) and a
    32 GB budget (24 GB of resident factorizations, 8 GB of solve buffers)
    so that it runs in under a minute and the LRU policy evicts.  The
    right-hand sides are drawn on the device.  The arrival rate is ``load``
    times the capacity measured on one factor job and one solve of nrhs 128
    per side.  Before that, one solve per side and right-hand-side bucket
    lets the solve-tile autotuner settle its one-time choices for those
    level shapes, as a long-running server would have done."""
    from paper_2310_15458_amd import serve
    t_f, t_s = [], []
    for n in sides:
        P = W.grid_points(n)
        k = W.grid_kernel("helmholtz", n, 35.0)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F = rss.Factorization(P, k, 1e-6, 64, precision="fp32")
        op = rss.GridOperator(k, n)
        rss.set_residual_op(F, op)
        t1 = time.perf_counter()
        nb = 1
        while nb <= max_nrhs:  # the autotuner's one-time tuning for this side
            F.solve(serve.device_normals(torch, 6, n * n, nb))
            nb *= 2
        B = serve.device_normals(torch, 5, n * n, max_nrhs // 2)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        F.solve(B)
        t3 = time.perf_counter()
        F.close()
        op.close()
        t_f.append(t1 - t0)
        t_s.append(t3 - t2)
    mean_service = 0.2 * float(np.mean(t_f)) + 0.8 * float(np.mean(t_s))
    rate = load / mean_service
    reqs = W.request_stream(count, rate, seed=4, sides=sides, max_nrhs=max_nrhs)
    res, *_ = serve.run_stream(reqs, budget, precision="fp32", grid_residual=True, device_rhs=True)
    res["rate_per_s"] = rate
    res["stream"] = (f"{count} requests, Poisson rate {rate:.2f}/s (= {load} x measured capacity), "
                     f"sides {list(sides)}, nrhs U{{1..{max_nrhs}}}, 20% factor jobs, seed 4, "
                     f"FP32+refine to 1e-10 with the FFT residual, budget {budget / 1e9:.0f} GB, "
                     f"solve tiles tuned before the stream")
    return res


def four_colour_schedule(torch, rss, W, w, P, B, gop, reps=2):
    """The four-colour schedule (rss_options.colours = 4; Sec. 3's coloured
    variant) beside the default nine colours on the headline workload: FP32
    and FP64 factor times, one application, and the time to relres <= 1e-10
    with the FFT residual (FP32: refinement; FP64: one application and its
    check), medians of ``reps`` after a warm-up factorization of each."""
    out = {}
    for col in (9, 4):
        res = {}
        for prec in ("fp32", "fp64"):
            F = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision=prec, n_proxy=w.n_proxy, colours=col)
            F.close()
            tf, ta, ts, steps, rr = [], [], [], 0, 0.0
            for _ in range(reps):
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision=prec, n_proxy=w.n_proxy,
                                      colours=col, max_refine=10, refine_tol=1e-10)
                torch.cuda.synchronize()
                tf.append(time.perf_counter() - t0)
                X = B.clone()
                F.apply(X)  # first use: the solve-tile tuning of this shape
                X = B.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F.apply(X)
                torch.cuda.synchronize()
                ta.append(time.perf_counter() - t0)
                rss.set_residual_op(F, gop)
                X = B.clone()
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                F.solve(X)
                torch.cuda.synchronize()
                ts.append(time.perf_counter() - t0)
                info = F.info()
                steps, rr = info["last_iters"], info["last_relres"]
                rss.set_residual_op(F, None)
                F.close()
            tfm, tsm = float(np.median(tf)), float(np.median(ts))
            res[prec] = {"t_factor_ms": tfm * 1e3, "factor_unknowns_per_s": w.N / tfm,
                         "apply_ms": float(np.median(ta)) * 1e3, "t_solve_to_1e-10_ms": tsm * 1e3,
                         "time_to_solution_unknowns_per_s": w.N / (tfm + tsm), "refine_steps": steps,
                         "relres": rr}
        res["fp32_over_fp64_time_to_solution"] = (res["fp32"]["time_to_solution_unknowns_per_s"]
                                                  / res["fp64"]["time_to_solution_unknowns_per_s"])
        out[f"colours_{col}"] = res
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-paper", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the library runs on one GPU only (the path is single-device); "
              "use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2310_15458_amd import rss, workloads as W

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    rss.load()
    w = W.helmholtz_512()
    P = W.grid_points(w.n)
    nrhs = w.nrhs[0]
    B_host = W.rhs(w.N, nrhs, w.seed)
    B = torch.from_numpy(np.ascontiguousarray(B_host.T)).to(dev).t()
    work = torch.empty_like(B)
    single = torch.empty_like(B)

    gop = rss.GridOperator(w.kernel, w.n)  # the FFT product on the grid (residual variant)

    def step(record, keep=False):
        t = {}
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F32 = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision="fp32", n_proxy=w.n_proxy)
        t["fact32"] = time.perf_counter() - t0
        work.copy_(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc32 = F32.solve(work)
        t["solve32"] = time.perf_counter() - t0
        i32 = F32.info()
        x32 = work.cpu().numpy() if keep else None
        # the same solve with the refinement residual by FFT
        rss.set_residual_op(F32, gop)
        work.copy_(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F32.solve(work)
        t["solve32_fft"] = time.perf_counter() - t0
        i32f = F32.info()
        rss.set_residual_op(F32, None)
        lat32 = []
        for _ in range(SOLVE_REPS):
            single.copy_(B)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F32.apply(single)
            lat32.append(time.perf_counter() - t0)
        F32.close()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F64 = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision="fp64", n_proxy=w.n_proxy,
                                max_refine=10, refine_tol=1e-10)
        t["fact64"] = time.perf_counter() - t0
        work.copy_(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        rc64 = F64.solve(work)
        t["solve64"] = time.perf_counter() - t0
        i64 = F64.info()
        x64 = work.cpu().numpy() if keep else None
        rss.set_residual_op(F64, gop)
        work.copy_(B)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        F64.solve(work)
        t["solve64_fft"] = time.perf_counter() - t0
        i64f = F64.info()
        rss.set_residual_op(F64, None)
        lat64 = []
        for _ in range(SOLVE_REPS):
            single.copy_(B)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            F64.apply(single)
            lat64.append(time.perf_counter() - t0)
        F64.close()
        if record is not None:
            record.append({"t": t, "i32": i32, "i64": i64, "i32f": i32f, "i64f": i64f, "rc": (rc32, rc64),
                           "lat32": lat32, "lat64": lat64, "x32": x32, "x64": x64})

    for _ in range(args.warmup):
        step(None)
    recs = []
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for i in range(args.steps):
        step(recs, keep=(i == args.steps - 1))
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start

    schedules = four_colour_schedule(torch, rss, W, w, P, B, gop)
    gop.close()
    # relres of the last step's results by the oracle's exact FFT product (host)
    from oracle import matvec as omv
    orr32 = omv.relres(omv.fft_matvec(w.kernel, w.n, recs[-1]["x32"]), B_host)
    orr64 = omv.relres(omv.fft_matvec(w.kernel, w.n, recs[-1]["x64"]), B_host)
    for r in recs:
        del r["x32"], r["x64"]
    N = w.N
    f32 = sum(r["t"]["fact32"] for r in recs)
    f64 = sum(r["t"]["fact64"] for r in recs)
    s32 = [r["t"]["solve32"] for r in recs]
    s64 = [r["t"]["solve64"] for r in recs]
    s32f = [r["t"]["solve32_fft"] for r in recs]
    s64f = [r["t"]["solve64_fft"] for r in recs]
    lat32 = np.array([x for r in recs for x in r["lat32"]]) * 1e3  # ms
    lat64 = np.array([x for r in recs for x in r["lat64"]]) * 1e3
    i32, i64 = recs[-1]["i32"], recs[-1]["i64"]

    # live per-kernel-class times (HIP events on the library's stream = torch's
    # current stream), from one profiled factorization of each form
    prof = {}
    for prec in ("fp32", "fp64"):
        Fp = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision=prec, n_proxy=w.n_proxy, profile=True)
        prof[prec] = Fp.info()
        Fp.close()
    # the dominant kernel: the FP64 on-the-fly residual r = b - A x of the refinement,
    # timed with torch events on the stream it is launched on
    Pd = torch.from_numpy(P).to(dev)
    R = None
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    rss.residual(w.kernel, Pd, B, B)  # warm
    torch.cuda.synchronize()
    nres = 2
    ev0.record()
    for _ in range(nres):
        R = rss.residual(w.kernel, Pd, B, B)
    ev1.record()
    torch.cuda.synchronize()
    t_res = ev0.elapsed_time(ev1) / nres / 1e3
    res_flops = 8.0 * N * N * nrhs          # the complex multiply-adds of A x (8 flops each)
    roofline = {"kernel": "k_residual (FP64 on-the-fly b - A x, 16 RHS)", "bound": "alu",
                "achieved": res_flops / t_res / 1e12, "peak": FP64_PEAK_TF, "unit": "TFLOP/s",
                "frac": res_flops / t_res / 1e12 / FP64_PEAK_TF, "traffic": RESIDUAL_TRAFFIC_B,
                "t_launch_ms": t_res * 1e3, "pair_evals_per_s": N * N / t_res,
                "algorithmic": "8 N^2 nrhs flops per launch (kernel evaluations not counted)"}

    def cls_t(info, name):
        return info["t_class_ms"][rss.KERNEL_CLASSES.index(name)] / 1e3

    steps_roof = {}
    for prec, peak in (("fp32", FP32_MFMA_PEAK_TF), ("fp64", FP64_PEAK_TF)):
        info = prof[prec]
        t_id, t_sc = cls_t(info, "id"), cls_t(info, "schur")
        steps_roof[prec] = {
            "id": {"bound": "alu", "achieved": info["flops_id"] / t_id / 1e12,
                   "peak": FP64_PEAK_TF if prec == "fp64" else 78.6, "unit": "TFLOP/s",
                   "t_ms": t_id * 1e3},
            "schur": {"bound": "mfma", "achieved": info["flops_schur"] / t_sc / 1e12, "peak": peak,
                      "unit": "TFLOP/s", "frac": info["flops_schur"] / t_sc / 1e12 / peak,
                      "t_ms": t_sc * 1e3},
            "class_ms": {n: round(info["t_class_ms"][i], 3) for i, n in enumerate(rss.KERNEL_CLASSES)},
        }
    for prec, lat, i in (("fp32", lat32, recs[-1]["i32"]), ("fp64", lat64, recs[-1]["i64"])):
        t = float(np.percentile(lat, 50)) / 1e3
        steps_roof[prec]["solve"] = {"bound": "hbm", "achieved": i["factor_bytes"] / t / 1e9,
                                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": i["factor_bytes"] / t / 1e9 / HBM_PEAK_GBS}

    out = {
        "metric": "RS-S factor unknowns/s at N=512^2 (FP32+refine vs FP64); solve p50/p99",
        "value": N * len(recs) / f32,
        "unit": "unknowns/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": total / len(recs) * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "c64 factor + f64 refine",
        "data": "synthetic: 512x512 cell-centre grid, complex N(0,1) RHS seed 2",
        "config": {"workload": "helmholtz kappa=50 N=512^2 tol=1e-6 leaf=64 n_proxy=128 nrhs=16",
                   "N": N, "nrhs": nrhs, "parallelism": "single GPU"},
        "fp32_refine": {
            "factor_unknowns_per_s": N * len(recs) / f32,
            "t_factor_ms": f32 / len(recs) * 1e3,
            "t_solve_to_1e-10_ms": float(np.median(s32) * 1e3),
            "time_to_solution_unknowns_per_s": N / (f32 / len(recs) + float(np.median(s32))),
            "relres": i32["last_relres"], "relres_oracle_fft": orr32, "refine_steps": i32["last_iters"],
            "apply_p50_ms": float(np.percentile(lat32, 50)), "apply_p99_ms": float(np.percentile(lat32, 99)),
            "device_GB": i32["device_bytes"] / 1e9,
            "fft_residual": {"t_solve_to_1e-10_ms": float(np.median(s32f) * 1e3),
                             "time_to_solution_unknowns_per_s": N / (f32 / len(recs) + float(np.median(s32f))),
                             "relres": recs[-1]["i32f"]["last_relres"],
                             "refine_steps": recs[-1]["i32f"]["last_iters"]},
        },
        "fp64": {
            "factor_unknowns_per_s": N * len(recs) / f64,
            "t_factor_ms": f64 / len(recs) * 1e3,
            "t_solve_to_1e-10_ms": float(np.median(s64) * 1e3),
            "time_to_solution_unknowns_per_s": N / (f64 / len(recs) + float(np.median(s64))),
            "relres": i64["last_relres"], "relres_oracle_fft": orr64, "refine_steps": i64["last_iters"],
            "apply_p50_ms": float(np.percentile(lat64, 50)), "apply_p99_ms": float(np.percentile(lat64, 99)),
            "device_GB": i64["device_bytes"] / 1e9,
            "fft_residual": {"t_solve_to_1e-10_ms": float(np.median(s64f) * 1e3),
                             "time_to_solution_unknowns_per_s": N / (f64 / len(recs) + float(np.median(s64f))),
                             "relres": recs[-1]["i64f"]["last_relres"],
                             "refine_steps": recs[-1]["i64f"]["last_iters"]},
        },
        "schedules_fft_residual": schedules,
        "ranks_fp32": [round(i32["rank_sum"][d] / max(1, i32["box_count"][d]), 2) for d in range(2, i32["depth"] + 1)],
        "ranks_fp64": [round(i64["rank_sum"][d] / max(1, i64["box_count"][d]), 2) for d in range(2, i64["depth"] + 1)],
        "ledger_fp32": {k: i32[k] for k in ("flops_id", "flops_lu", "flops_y", "flops_schur",
                                            "factor_bytes", "kernel_evals")},
        "roofline": roofline,
        "roofline_steps": steps_roof,
        "cpu_baseline": None,
    }
    out["batched"] = batched_sweep(torch, rss, W)
    # a different class of workload follows: hand the batched sweep's ~100 GB
    # of cached blocks back (rss_trim_cache) so that its frees do not stall
    out["batched"]["trimmed_GB"] = rss.trim_cache() / 1e9
    if not args.no_paper:
        out["paper_matrices"] = paper_matrices(torch, rss, W)
        out["tolerance_and_frequency"] = tolerance_and_frequency(torch, rss, W)
    if not args.no_serving:
        out["serving"] = serving(torch, rss, W)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
