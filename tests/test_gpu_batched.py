"""GPU parity of the batched multi-problem sweep (rss_factor_batch /
rss_apply_batch): every problem of a batch must give the same result as when
it is factored and solved alone (<= 1e-12 relative; the schedule of each
problem is identical, only launches are shared), the oracle's skeleton sets,
and the oracle's solution (<= 1e-10)."""
import numpy as np
import pytest

from oracle import matvec as omv, rss as orss
from paper_2310_15458_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2310_15458_amd import rss
    rss.load()
    return torch


def _dev(torch, A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, np.complex128).T)).cuda().t()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def test_small_mixed_batch(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    specs = [("laplace", 0.0, 16), ("helmholtz", 20.0, 24), ("helmholtz", 35.0, 32),
             ("laplace", 0.0, 24), ("helmholtz", 10.0, 4)]   # the last has D < 2 (dense root only)
    leaf, tol = 9, 1e-6
    Ps = [W.grid_points(n) for _, _, n in specs]
    Ks = [W.grid_kernel(k, n, kap) for k, kap, n in specs]
    Bs = [W.rhs(n * n, 2, 10 + i) for i, (_, _, n) in enumerate(specs)]
    print("batch of", len(specs), "problems", flush=True)
    Fb = rss.factor_batch(Ps, Ks, tol, leaf)
    Db = [_dev(torch, B) for B in Bs]
    rss.apply_batch(Fb, Db)
    for i, (kind, kap, n) in enumerate(specs):
        F1 = rss.Factorization(Ps[i], Ks[i], tol, leaf)
        D1 = _dev(torch, Bs[i])
        F1.apply(D1)
        xb, x1 = Db[i].cpu().numpy(), D1.cpu().numpy()
        assert _rel(xb, x1) <= 1e-12, (i, _rel(xb, x1))
        Fo = orss.factor(Ps[i], Ks[i], tol, leaf)
        for d in range(Fo.tree.D, 1, -1):
            got = Fb[i].skeletons(d)
            for (dd, b), sk in Fo.skeletons.items():
                if dd == d:
                    assert np.array_equal(got[b], sk), (i, d, b)
        assert _rel(xb, orss.solve(Fo, Bs[i])) < 1e-10
        F1.close()
    for F in Fb[::-1]:
        F.close()


def test_batched_workload_256(torch_cuda):
    """256 problems: n uniform over {32, 48, 64, 96, 128}, Laplace or Helmholtz
    (kappa ~ U[5, 40]), leaf 64, tol 1e-6, one real RHS each (seed 3)."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    probs = W.batched_problems()
    Ps = [W.grid_points(p.n) for p in probs]
    Ks = [p.kernel for p in probs]
    print("factoring 256 problems", flush=True)
    Fb = rss.factor_batch(Ps, Ks, 1e-6, 64)
    Db = [_dev(torch, p.rhs) for p in probs]
    rss.apply_batch(Fb, Db)
    torch.cuda.synchronize()
    worst = 0.0
    for i, p in enumerate(probs):
        x = Db[i].cpu().numpy()
        rr = omv.relres(omv.fft_matvec(p.kernel, p.n, x), p.rhs)
        worst = max(worst, rr)
    print(f"worst relres over 256 problems {worst:.3e}", flush=True)
    assert worst < 1e-8
    # a sample of problems against their solo factorization
    for i in (0, 7, 100, 255):
        p = probs[i]
        F1 = rss.Factorization(Ps[i], Ks[i], 1e-6, 64)
        D1 = _dev(torch, p.rhs)
        F1.apply(D1)
        assert _rel(Db[i].cpu().numpy(), D1.cpu().numpy()) <= 1e-12
        F1.close()
    for F in Fb[::-1]:
        F.close()


def test_trim_cache_returns_freed_blocks(torch_cuda):
    """Blocks of a closed factorization stay cached for reuse until
    rss_trim_cache hands them back: free device memory grows by what it
    reports, a second call releases nothing, and a factorization after the
    trim (blocks from the driver again) gives the same solution bit for bit."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 128
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 30.0)
    B = W.rhs(n * n, 1, 2)
    print("factor, close, trim", flush=True)
    F = rss.Factorization(P, k, 1e-6, 64)
    X1 = _dev(torch, B)
    F.apply(X1)
    F.close()
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    got = rss.trim_cache()
    free1 = torch.cuda.mem_get_info()[0]
    assert got > 0
    assert free1 - free0 >= 0.9 * got
    assert rss.trim_cache() == 0
    F = rss.Factorization(P, k, 1e-6, 64)
    X2 = _dev(torch, B)
    F.apply(X2)
    F.close()
    assert torch.equal(X1, X2)
