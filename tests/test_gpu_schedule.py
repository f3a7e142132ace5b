"""GPU parity of the four-colour schedule (rss_options.colours = 4; Sec. 3's
coloured variant, where only neighbours must differ in colour).

Bars: an FP64 factorization has the four-colour oracle's skeleton sets at
every depth (both take a colour's IDs before its first elimination; the Schur
updates of a colour meet on shared blocks only additively and the library
applies them in four ordered passes, so the factorization is deterministic)
and the oracle's solution to 1e-10; two applications agree to 1e-13 (the
forward sweep's neighbour updates are atomic adds, so not bit for bit); an
FP32 solve refined with the oracle-pinned FFT residual reaches relres 1e-10;
a batch of problems equals the problems factored alone.
"""
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
    A = np.asarray(A, dtype=np.complex128)
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


@pytest.mark.parametrize("kind,kappa,n,leaf", [("helmholtz", 40.0, 48, 36), ("laplace", 0.0, 64, 64),
                                               ("helmholtz", 25.0, 64, 64)])
def test_four_colours_match_oracle(torch_cuda, kind, kappa, n, leaf):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    print(f"four colours: {kind} n={n} leaf={leaf}", flush=True)
    Fo = orss.factor(P, k, 1e-6, leaf, orss.Options(colours=4))
    F = rss.Factorization(P, k, 1e-6, leaf, colours=4)
    for d in range(Fo.tree.D, 1, -1):
        got = F.skeletons(d)
        for (dd, b), sk in Fo.skeletons.items():
            if dd == d:
                assert np.array_equal(got[b], sk), (d, b)
    B = W.rhs(n * n, 3, 7)
    X1, X2 = _dev(torch, B), _dev(torch, B)
    F.apply(X1)
    F.apply(X2)
    x1, x2 = X1.cpu().numpy(), X2.cpu().numpy()
    xo = orss.solve(Fo, B)
    assert np.linalg.norm(x1 - xo) / np.linalg.norm(xo) <= 1e-10
    assert np.linalg.norm(x1 - x2) / np.linalg.norm(x1) <= 1e-13
    F.close()


def test_four_colours_fp32_refined_and_batched(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 96
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 50.0)
    B = W.rhs(n * n, 4, 9)
    F = rss.Factorization(P, k, 1e-6, 64, precision="fp32", n_proxy=128, colours=4)
    op = rss.GridOperator(k, n)
    rss.set_residual_op(F, op)
    X = _dev(torch, B)
    assert F.solve(X) == rss.RSS_OK
    rr = omv.relres(omv.fft_matvec(k, n, X.cpu().numpy()), B)
    print(f"FP32 four colours: relres {rr:.2e} in {F.info()['last_iters']} steps", flush=True)
    assert rr <= 1e-10
    rss.set_residual_op(F, None)
    op.close()
    F.close()
    # a batch equals the problems alone (skeletons; applications to 1e-13)
    sides = (48, 64, 32)
    Ps = [W.grid_points(m) for m in sides]
    Ks = [W.grid_kernel("helmholtz", m, 20.0 + m / 4) for m in sides]
    Fb = rss.factor_batch(Ps, Ks, 1e-6, 36, colours=4)
    for m, Pm, km, fb in zip(sides, Ps, Ks, Fb):
        fa = rss.Factorization(Pm, km, 1e-6, 36, colours=4)
        for d in range(fa.info()["depth"], 1, -1):
            assert all(np.array_equal(a, b) for a, b in zip(fa.skeletons(d), fb.skeletons(d))), (m, d)
        Bm = W.rhs(m * m, 2, m)
        Xa, Xb = _dev(torch, Bm), _dev(torch, Bm)
        fa.apply(Xa)
        fb.apply(Xb)
        xa, xb = Xa.cpu().numpy(), Xb.cpu().numpy()
        assert np.linalg.norm(xa - xb) / np.linalg.norm(xa) <= 1e-13
        fa.close()
    for f in Fb:
        f.close()
    # one batch may not mix schedules
    with pytest.raises(rss.RSSError):
        rss.factor_batch([Ps[0]], [Ks[0]], 1e-6, 36, colours=5)
