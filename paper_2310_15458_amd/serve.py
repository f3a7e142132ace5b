"""Drive the solve server with a Poisson request stream and report latency.

The stream comes from workloads.request_stream (seeded): factor jobs on
n x n grids (Helmholtz, kappa ~ U[10, 60]) and solves with nrhs ~ U{1..max}
against earlier factor jobs.  Requests are submitted at their arrival times
(wall clock); each solve's right-hand sides are the counter-based normals
keyed by (seed, request id).  Latency = completion time - arrival time.
"""
from __future__ import annotations

import time

import numpy as np

from . import rss
from . import workloads as W


def device_normals(torch, key: int, N: int, nrhs: int, device="cuda"):
    """N x nrhs complex normals (real and imaginary parts N(0,1)) drawn on the
    device by torch's generator seeded with ``key``, column-major: for
    streams whose right-hand sides are too large to draw on the host."""
    g = torch.Generator(device=device)
    g.manual_seed(int(key))
    z = torch.randn((nrhs, N, 2), dtype=torch.float64, device=device, generator=g)
    return torch.view_as_complex(z).t()


def run_stream(reqs, budget_bytes: float, tol=1e-6, leaf=64, precision="fp32", max_batch=64,
               seed=4, keep_results=False, device="cuda", grid_residual=False, device_rhs=False):
    """Submit ``reqs`` at their arrival times and collect completions.
    device_rhs: draw right-hand sides on the device (torch generator keyed
    by (seed, request id)) instead of the host counter-based normals; the
    inputs are then not kept."""
    import torch
    srv = rss.Server(budget_bytes, precision=precision, tol=tol, leaf=leaf, max_batch=max_batch,
                     grid_residual=grid_residual)
    fid = {}        # factor request rid -> server id
    rid_of = {}     # server request id -> stream rid
    arrive = {}
    inputs, outputs = {}, {}
    kinds = {}
    done = {}
    rejected = []
    t0 = time.perf_counter()
    pending = 0
    i = 0
    while i < len(reqs) or pending:
        now = time.perf_counter() - t0
        while i < len(reqs) and reqs[i].t_arrive <= now:
            r = reqs[i]
            if r.kind == "factor":
                P = W.grid_points(r.n)
                k = W.grid_kernel("helmholtz", r.n, r.kappa)
                sid = srv.factor(P, k)
                fid[r.rid] = sid
            else:
                N = r.n * r.n
                if device_rhs:
                    B = device_normals(torch, (seed << 24) | r.rid, N, r.nrhs, device)
                else:
                    b = W.counter_normals((seed << 24) | r.rid, N * r.nrhs).reshape(r.nrhs, N).T
                    B = torch.from_numpy(np.ascontiguousarray(b.T)).to(device).t()
                    if keep_results:
                        inputs[r.rid] = b.copy()
                        outputs[r.rid] = B
                try:
                    sid = srv.solve(fid[r.target], B)
                except rss.RSSError as e:  # the target's factorization failed
                    rejected.append((r.rid, r.target, str(e)))
                    i += 1
                    continue
            rid_of[sid] = r.rid
            arrive[r.rid] = r.t_arrive
            kinds[r.rid] = r.kind
            pending += 1
            i += 1
        wait = 0 if i < len(reqs) else 50
        if i < len(reqs):
            wait = max(0, int((reqs[i].t_arrive - (time.perf_counter() - t0)) * 1000))
            wait = min(wait, 20)
        for c in srv.poll(wait_ms=wait):
            rr = rid_of[c["req"]]
            c["t_done_wall"] = time.perf_counter() - t0
            done[rr] = c
            pending -= 1
    wall = time.perf_counter() - t0
    st = srv.stats()
    lat = {"factor": [], "solve": []}
    for rr, c in done.items():
        lat[kinds[rr]].append(c["t_done_wall"] - arrive[rr])
    res = {"requests": len(reqs), "wall_s": wall, "server": st,
           "failed": sum(1 for c in done.values() if c["status"] not in (0,)),
           "rejected": len(rejected)}
    bad = [(rr, kinds[rr], c["status"]) for rr, c in done.items() if c["status"] != 0]
    if bad or rejected:
        res["failures"] = {"completions": bad[:10], "rejected": rejected[:10]}
    for k, v in lat.items():
        if v:
            a = np.array(v) * 1e3
            res[f"{k}_p50_ms"] = float(np.percentile(a, 50))
            res[f"{k}_p99_ms"] = float(np.percentile(a, 99))
            res[f"{k}_count"] = len(v)
    res["solved_unknowns_per_s"] = st["solved_unknowns"] / wall
    res["mean_batch"] = st["batched_solves"] / max(1, st["batches"])
    if keep_results:
        res["completions"] = {rr: dict(c, kind_name=kinds[rr]) for rr, c in done.items()}
    out = (res, srv, fid, inputs, outputs) if keep_results else (res, None, None, None, None)
    if not keep_results:
        srv.close()
    return out
