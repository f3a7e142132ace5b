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


def run_stream(reqs, budget_bytes: float, tol=1e-6, leaf=64, precision="fp32", max_batch=64,
               seed=4, keep_results=False, device="cuda"):
    import torch
    srv = rss.Server(budget_bytes, precision=precision, tol=tol, leaf=leaf, max_batch=max_batch)
    fid = {}        # factor request rid -> server id
    rid_of = {}     # server request id -> stream rid
    arrive = {}
    inputs, outputs = {}, {}
    kinds = {}
    done = {}
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
                b = W.counter_normals((seed << 24) | r.rid, N * r.nrhs).reshape(r.nrhs, N).T
                B = torch.from_numpy(np.ascontiguousarray(b.T)).to(device).t()
                if keep_results:
                    inputs[r.rid] = b.copy()
                    outputs[r.rid] = B
                sid = srv.solve(fid[r.target], B)
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
           "failed": sum(1 for c in done.values() if c["status"] not in (0,))}
    for k, v in lat.items():
        if v:
            a = np.array(v) * 1e3
            res[f"{k}_p50_ms"] = float(np.percentile(a, 50))
            res[f"{k}_p99_ms"] = float(np.percentile(a, 99))
            res[f"{k}_count"] = len(v)
    res["solved_unknowns_per_s"] = st["solved_unknowns"] / wall
    res["mean_batch"] = st["batched_solves"] / max(1, st["batches"])
    out = (res, srv, fid, inputs, outputs) if keep_results else (res, None, None, None, None)
    if not keep_results:
        srv.close()
    return out
