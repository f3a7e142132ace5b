"""Write the oracle's reference results for the full-size parity tests.

    python tests/golden/make_golden.py [case ...]

Calls only the CPU oracle (oracle/) on the seeded inputs of
paper_2310_15458_amd/workloads.py and stores, per case, a JSON file here:

* for every compressed depth and box: the skeleton count k (Def. 1) and the
  CRC-32 of the box's ascending skeleton ids (little-endian int64), so a GPU
  factorization can be checked box by box for identical skeleton sets;
* the FP64 solution of Sec. 2.6 (oracle.rss.solve) at seeded sample rows, all
  right-hand-side columns, full precision;
* the relative residual of that solution by the exact FFT product.

Cases:
  helmholtz-k25-n256   kappa = 25, N = 256^2, leaf 64, tol 1e-6, 128 proxies,
                       nrhs 1 and 64 (each from a fresh default_rng(1))
  helmholtz-k50-n512   kappa = 50, N = 512^2, leaf 64, tol 1e-6, 128 proxies,
                       nrhs 16 (seed 2), the FP64 form of the benchmark
  batch-helmholtz-n128 the first Helmholtz problem of side 128 in the
                       256-problem batched workload (seed 3)
"""
from __future__ import annotations

import json
import os
import sys
import time
import zlib

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from oracle import matvec, rss  # noqa: E402
from paper_2310_15458_amd import workloads as W  # noqa: E402

SAMPLE_SEED = 12345


def skeleton_crc(ids) -> int:
    return zlib.crc32(np.asarray(ids, dtype="<i8").tobytes()) & 0xFFFFFFFF


def sample_rows(N: int, count: int) -> np.ndarray:
    rng = np.random.default_rng(SAMPLE_SEED)
    return np.sort(rng.choice(N, size=min(count, N), replace=False))


def skeleton_table(F) -> dict:
    out = {}
    for d in range(F.tree.D, 1, -1):
        ks, crcs = [], []
        for b in range(4 ** d):
            s = F.skeletons.get((d, b))
            if s is None:
                ks.append(-1)
                crcs.append(0)
            else:
                ks.append(int(s.size))
                crcs.append(skeleton_crc(s))
        out[str(d)] = {"k": ks, "crc": crcs}
    return out


def solution_sample(F, kern, n, B, rows) -> dict:
    X = rss.solve(F, B)
    rr = matvec.relres(matvec.fft_matvec(kern, n, X), B)
    xs = X[rows]
    return {"nrhs": int(B.shape[1]), "rows": [int(r) for r in rows],
            "re": xs.real.tolist(), "im": xs.imag.tolist(), "relres_fft": float(rr)}


def run_grid(name, n, kern, tol, leaf, npx, solves, out):
    P = W.grid_points(n)
    t0 = time.perf_counter()
    F = rss.factor(P, kern, tol, leaf, rss.Options(n_proxy=npx))
    t1 = time.perf_counter()
    res = {"case": name, "n": n, "kind": kern.kind, "kappa": kern.kappa, "weight": kern.weight,
           "diag": kern.diag, "tol": tol, "leaf": leaf, "n_proxy": npx, "depth": F.tree.D,
           "n_root": int(F.root_idx.size), "skeletons": skeleton_table(F), "solves": []}
    for B, rows in solves:
        res["solves"].append(solution_sample(F, kern, n, B, rows))
    res["oracle_factor_s"] = t1 - t0
    with open(out, "w") as f:
        json.dump(res, f, separators=(",", ":"))
    print(f"{name}: D={F.tree.D} factor {t1 - t0:.1f} s, "
          f"relres {[s['relres_fft'] for s in res['solves']]}", flush=True)


def case_c2():
    w = W.helmholtz_256()
    solves = []
    for nrhs, count in ((1, 64), (64, 24)):
        solves.append((W.rhs(w.N, nrhs, w.seed), sample_rows(w.N, count)))
    run_grid(w.name, w.n, w.kernel, w.tol, w.leaf, w.n_proxy, solves,
             os.path.join(HERE, "parity_helmholtz_k25_n256.json"))


def case_c3():
    w = W.helmholtz_512()
    solves = [(W.rhs(w.N, 16, w.seed), sample_rows(w.N, 48))]
    run_grid(w.name, w.n, w.kernel, w.tol, w.leaf, w.n_proxy, solves,
             os.path.join(HERE, "parity_helmholtz_k50_n512.json"))


def batch_index():
    """index of the first Helmholtz problem of side 128 in the batched workload"""
    for i, p in enumerate(W.batched_problems(256, 3)):
        if p.n == 128 and p.kernel.kind == W.HELMHOLTZ:
            return i, p
    raise RuntimeError("no Helmholtz n = 128 problem in the batched workload")


def case_batch():
    i, p = batch_index()
    solves = [(p.rhs, sample_rows(p.n * p.n, 64))]
    out = os.path.join(HERE, "parity_batch_helmholtz_n128.json")
    run_grid(f"batch-problem-{i}", p.n, p.kernel, 1e-6, 64, p.n_proxy, solves, out)
    with open(out) as f:
        res = json.load(f)
    res["batch_index"] = i
    with open(out, "w") as f:
        json.dump(res, f, separators=(",", ":"))


CASES = {"helmholtz-k25-n256": case_c2, "helmholtz-k50-n512": case_c3,
         "batch-helmholtz-n128": case_batch}

if __name__ == "__main__":
    for name in sys.argv[1:] or list(CASES):
        CASES[name]()
