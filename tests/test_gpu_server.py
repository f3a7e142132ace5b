"""GPU tests of the solve server (continuous batching, resident factorizations,
device-memory budget with LRU eviction).  Bar: every solve served in the mix
equals the same solve done alone within 1e-10 relative (both are refined to
relres <= 1e-10; the per-problem arithmetic does not depend on which other
solves share a step), and reaches relres <= 1e-10 measured with the oracle's
exact FFT product.  The mix must really be mixed: at least two solves share a
step (max_batch_seen >= 2), solves join while others are in flight, and a
factorization runs while solves do (their [start, end] intervals overlap)."""
import time

import numpy as np
import pytest

from oracle import matvec as omv
from paper_2310_15458_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2310_15458_amd import rss
    rss.load()
    return torch


def test_server_alone_vs_mix(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss, serve
    reqs = W.request_stream(count=48, rate=40.0, seed=4, sides=(32, 48), max_nrhs=6)
    nf = sum(r.kind == "factor" for r in reqs)
    print(f"{len(reqs)} requests, {nf} factor jobs", flush=True)
    res, srv, fid, inputs, outputs = serve.run_stream(reqs, budget_bytes=8e9, keep_results=True)
    print({k: v for k, v in res.items() if k != "server"}, res["server"], flush=True)
    assert res["failed"] == 0
    assert res["server"]["batches"] >= 1
    solves = [r for r in reqs if r.kind == "solve"]
    for r in solves:
        x = outputs[r.rid].cpu().numpy()
        k = W.grid_kernel("helmholtz", r.n, r.kappa)
        assert omv.relres(omv.fft_matvec(k, r.n, x), inputs[r.rid]) <= 1e-10, r.rid
    for r in solves[:: max(1, len(solves) // 6)]:
        k = W.grid_kernel("helmholtz", r.n, r.kappa)
        F = rss.Factorization(W.grid_points(r.n), k, 1e-6, 64, precision="fp32")
        B = torch.from_numpy(np.ascontiguousarray(inputs[r.rid].T)).cuda().t()
        assert F.solve(B) == 0
        xa, xm = B.cpu().numpy(), outputs[r.rid].cpu().numpy()
        assert np.linalg.norm(xa - xm) / np.linalg.norm(xa) <= 1e-10, r.rid
        F.close()
    srv.close()


def test_server_evicts_under_budget(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    # budget for about two resident factorizations of a 32 x 32 grid
    probe = rss.Factorization(W.grid_points(32), W.grid_kernel("helmholtz", 32, 20.0), 1e-6, 16)
    one = probe.info()["device_bytes"]
    probe.close()
    srv = rss.Server(budget_bytes=2.5 * one, precision="fp64", leaf=16)
    ids, outs, bs = [], [], []
    for i in range(5):
        k = W.grid_kernel("helmholtz", 32, 15.0 + 5 * i)
        fid = srv.factor(W.grid_points(32), k)
        b = W.rhs(1024, 2, 30 + i)
        B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
        srv.solve(fid, B)
        ids.append((fid, k))
        outs.append(B)
        bs.append(b)
    got = 0
    while got < 10:
        got += len(srv.poll(wait_ms=200))
    st = srv.stats()
    print(st, flush=True)
    assert st["evictions"] >= 2 and st["peak_bytes"] <= 2.5 * one * 1.2
    for (fid, k), B, b in zip(ids, outs, bs):
        x = B.cpu().numpy()
        assert omv.relres(omv.fft_matvec(k, 32, x), b) < 1e-9
    # a solve against an evicted factorization refactors it first
    fid, k = ids[0]
    b = W.rhs(1024, 1, 77)
    B = torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()
    sid = srv.solve(fid, B)
    cs = []
    while not any(c["req"] == sid for c in cs):
        cs += srv.poll(wait_ms=200)
    assert [c["kind"] for c in cs] == [1] and cs[0]["status"] == 0  # no factor completion
    assert srv.stats()["refactors"] == 1
    assert omv.relres(omv.fft_matvec(k, 32, B.cpu().numpy()), b) < 1e-9
    srv.close()


def _wait_all(srv, reqs, done, timeout_s=120.0):
    t0 = time.perf_counter()
    while not set(reqs) <= set(done):
        for c in srv.poll(wait_ms=50):
            done[c["req"]] = c
        assert time.perf_counter() - t0 < timeout_s, "server did not complete"


def test_server_continuous_batching_overlap_and_grid_residual(torch_cuda):
    """Solves keep arriving while a factorization runs and while other solves
    refine; the FFT residual (grid_residual) serves the grid problems."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, kap = 64, 30.0
    kA = W.grid_kernel("helmholtz", n, kap)
    srv = rss.Server(8e9, precision="fp32", leaf=64, grid_residual=True, max_batch=16)
    fa = srv.factor(W.grid_points(n), kA)
    done = {}
    _wait_all(srv, [fa], done)
    assert done[fa]["status"] == 0
    # right-hand sides ready on the device before the stream starts
    pool = []
    for i in range(64):
        b = W.rhs(n * n, 1 + (7 * i) % 12, 100 + i)
        pool.append((b, torch.from_numpy(np.ascontiguousarray(b.T)).cuda().t()))
    torch.cuda.synchronize()
    # a larger factorization, with solves against A arriving every half
    # millisecond meanwhile (each is in flight for several steps)
    fb = srv.factor(W.grid_points(256), W.grid_kernel("helmholtz", 256, 40.0))
    rhs, outs, sids = {}, {}, []
    for b, B in pool:
        sid = srv.solve(fa, B)
        rhs[sid], outs[sid] = b, B
        sids.append(sid)
        time.sleep(5e-4)
        for c in srv.poll(wait_ms=0):
            done[c["req"]] = c
    _wait_all(srv, sids + [fb], done)
    st = srv.stats()
    print(len(sids), "solves;", st, flush=True)
    assert all(done[s]["status"] == 0 for s in sids + [fb])
    assert st["max_batch_seen"] >= 2
    # continuous admission: some solve started while another was in flight
    iv = sorted((done[s]["t_start"], done[s]["t_end"]) for s in sids)
    assert any(b0 < a1 and a0 < b0 for (a0, a1), (b0, _) in zip(iv, iv[1:]))
    # factorization B overlapped solve work
    f0, f1 = done[fb]["t_start"], done[fb]["t_end"]
    assert any(s0 < f1 and f0 < s1 for s0, s1 in iv), (f0, f1, iv[:3], iv[-3:])
    for s in sids:
        x = outs[s].cpu().numpy()
        assert omv.relres(omv.fft_matvec(kA, n, x), rhs[s]) <= 1e-10, s
    # the same right-hand sides again, one at a time: identical to the mix
    for s in sids[:: max(1, len(sids) // 8)]:
        B = torch.from_numpy(np.ascontiguousarray(rhs[s].T)).cuda().t()
        sid = srv.solve(fa, B)
        _wait_all(srv, [sid], done)
        assert done[sid]["batch"] == 1 and done[sid]["status"] == 0
        xa, xm = B.cpu().numpy(), outs[s].cpu().numpy()
        assert np.linalg.norm(xa - xm) / np.linalg.norm(xa) <= 1e-10, s
    srv.close()
