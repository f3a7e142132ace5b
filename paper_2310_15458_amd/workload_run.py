"""Run the N = 512^2 Helmholtz workload (kappa = 50, tol 1e-6, leaf 64, 128
proxies, 16 right-hand sides) once: one factorization and a given number of
applications, for profiling a single step under rocprofv3.

    python paper_2310_15458_amd/workload_run.py [--precision fp32|fp64]
        [--applies K] [--no-autotune]

--no-autotune keeps the default solve tiles, so that counters collected over
the run cover exactly one factorization and K applications (the autotuner
otherwise times extra applications on first use).
"""
from __future__ import annotations

import argparse
import os
import sys

if __package__ in (None, ""):  # run as a file: the repository root holds the package
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--precision", default="fp32", choices=("fp32", "fp64"))
    ap.add_argument("--applies", type=int, default=1)
    ap.add_argument("--no-autotune", action="store_true")
    args = ap.parse_args(argv)
    import numpy as np
    import torch

    from paper_2310_15458_amd import rss, workloads as W

    rss.load()
    if args.no_autotune:
        rss.set_autotune(0)
    w = W.helmholtz_512()
    P = W.grid_points(w.n)
    B = torch.from_numpy(np.ascontiguousarray(W.rhs(w.N, w.nrhs[0], w.seed).T)).cuda().t()
    F = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision=args.precision, n_proxy=w.n_proxy)
    for _ in range(args.applies):
        X = B.clone()
        F.apply(X)
    torch.cuda.synchronize()
    F.close()
    print(f"workload_run: {args.precision} factorization and {args.applies} application(s) done", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
