"""Captured solve sweeps (rss_set_graphs): an apply of one handle replays a HIP
graph of its launches, with the right-hand-side vectors reached through
descriptor tables that each call rewrites.

Bar: every replay equals the direct launches bit for bit (the same kernels
in the same order, every reduction in a fixed order), for several replays in
a row with the program's own eager work and synchronisations between them, on
fresh buffers each time (so the descriptor rewrite is exercised), for both
precision forms, for changes of nrhs (more captured graphs than a handle keeps,
so the least recently used one is dropped and captured again), and through
the refined solve.
"""
import numpy as np
import pytest

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


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_graph_replays_equal_direct_launches(torch_cuda, precision):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 48
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 30.0)
    f = rss.Factorization(P, k, 1e-6, 36, precision=precision, max_refine=-1)
    prev = rss.set_graphs(True)
    try:
        # five widths: the handle keeps four captures, so the last 3 is captured again
        for nrhs, seed in ((3, 11), (5, 12), (1, 14), (2, 15), (4, 16), (3, 13)):
            B0 = W.rhs(n * n, nrhs, seed)
            rss.set_graphs(False)
            E = _dev(torch, B0)
            f.apply(E)
            ref = E.cpu().numpy()
            rss.set_graphs(True)
            for rep in range(4):
                X = _dev(torch, B0)  # a fresh buffer: new addresses in the descriptors
                f.apply(X)
                torch.cuda.synchronize()
                got = X.cpu().numpy()
                assert np.array_equal(got, ref), (precision, nrhs, rep)
                # the program's own eager work between replays
                rss.set_graphs(False)
                Y = _dev(torch, W.rhs(n * n, nrhs, 100 + rep))
                f.apply(Y)
                torch.cuda.synchronize()
                rss.set_graphs(True)
    finally:
        rss.set_graphs(prev)
        f.close()


def test_graph_refined_solve_equals_direct(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 48
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 30.0)
    f = rss.Factorization(P, k, 1e-6, 36, precision="fp32")
    B0 = W.rhs(n * n, 4, 21)
    prev = rss.set_graphs(False)
    try:
        E = _dev(torch, B0)
        assert f.solve(E) == rss.RSS_OK
        it_direct = f.info()["last_iters"]
        ref = E.cpu().numpy()
        rss.set_graphs(True)
        for rep in range(3):
            X = _dev(torch, B0)
            assert f.solve(X) == rss.RSS_OK
            assert f.info()["last_iters"] == it_direct
            assert np.array_equal(X.cpu().numpy(), ref), rep
    finally:
        rss.set_graphs(prev)
        f.close()


def test_autotuned_tiles_agree_with_default(torch_cuda):
    """The tile autotuner (rss_set_autotune) only changes how the sweeps are
    split over workgroups: an FP64 apply with tuned tiles equals the default
    tiles' result to rounding (1e-13 relative), and a refined FP32 solve with
    tuned tiles still reaches relres <= 1e-10 by the oracle's exact product."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    from oracle import matvec as omv
    n = 64
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 40.0)
    B0 = W.rhs(n * n, 7, 31)
    prev_t, prev_g = rss.set_autotune(False), rss.set_graphs(False)
    try:
        f = rss.Factorization(P, k, 1e-6, 64, precision="fp64", max_refine=-1)
        E = _dev(torch, B0)
        f.apply(E)
        ref = E.cpu().numpy()
        f.close()
        rss.set_autotune(True)
        f = rss.Factorization(P, k, 1e-6, 64, precision="fp64", max_refine=-1)
        X = _dev(torch, B0)
        f.apply(X)  # tunes this shape, then applies with the chosen tiles
        got = X.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
        f.close()
        g = rss.Factorization(P, k, 1e-6, 64, precision="fp32")
        Y = _dev(torch, B0)
        assert g.solve(Y) == rss.RSS_OK
        assert omv.relres(omv.fft_matvec(k, n, Y.cpu().numpy()), B0) <= 1e-10
        g.close()
    finally:
        rss.set_autotune(prev_t)
        rss.set_graphs(prev_g)


@pytest.mark.parametrize("kappa,n,leaf", [(40.0, 64, 64), (30.0, 48, 36)])
def test_fused_tiles_agree_with_default(torch_cuda, kappa, n, leaf):
    """The fused solve tile (each sweep step in one launch per box;
    rss_set_autotune(2) forces it wherever its LDS fits) does the arithmetic of
    one slice: an FP64 apply equals the default tiles' to 1e-13, and a refined
    FP32 solve reaches relres <= 1e-10 by the oracle's exact product, directly
    and through a captured graph (two replays, equal bit for bit)."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    from oracle import matvec as omv
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, kappa)
    B0 = W.rhs(n * n, 5, 41)
    prev_t, prev_g = rss.set_autotune(0), rss.set_graphs(False)
    try:
        f = rss.Factorization(P, k, 1e-6, leaf, precision="fp64", max_refine=-1)
        E = _dev(torch, B0)
        f.apply(E)
        ref = E.cpu().numpy()
        f.close()
        rss.set_autotune(2)
        f = rss.Factorization(P, k, 1e-6, leaf, precision="fp64", max_refine=-1)
        X = _dev(torch, B0)
        f.apply(X)
        got = X.cpu().numpy()
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-13
        f.close()
        g = rss.Factorization(P, k, 1e-6, leaf, precision="fp32")
        Y = _dev(torch, B0)
        assert g.solve(Y) == rss.RSS_OK
        y = Y.cpu().numpy()
        assert omv.relres(omv.fft_matvec(k, n, y), B0) <= 1e-10
        rss.set_graphs(True)
        for rep in range(2):
            Z = _dev(torch, B0)
            assert g.solve(Z) == rss.RSS_OK
            assert np.array_equal(Z.cpu().numpy(), y), rep
        g.close()
        assert rss.set_autotune(0) == 2
    finally:
        rss.set_autotune(prev_t)
        rss.set_graphs(prev_g)


def test_factor_tuner_buckets_and_agreement(torch_cuda):
    """The factor-side tuner (rss_factor_tuning): a factorization with tuning
    on fills the table with one entry per bucket it meets, each a candidate
    target; the chunking changes only the summation order of the Gram partial
    matrices, so the skeleton sets equal an untuned factorization's and the
    applies agree to 1e-12; the next factorization reuses the table."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 128
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 40.0)
    B0 = W.rhs(n * n, 3, 32)
    rss.factor_tuning_clear()
    prev = rss.set_autotune(False)
    try:
        f0 = rss.Factorization(P, k, 1e-6, 64, precision="fp64")
        assert rss.factor_tuning() == []
        X0 = _dev(torch, B0)
        f0.apply(X0)
        rss.set_autotune(True)
        f1 = rss.Factorization(P, k, 1e-6, 64, precision="fp64")
        tab = rss.factor_tuning()
        print(tab, flush=True)
        assert len(tab) >= 2  # several depths, several buckets
        for e in tab:
            assert e["target_workgroups"] in (512, 1024, 2048, 4096, 8192)
            assert e["chunks"] >= 1 and e["us"] > 0 and e["precision_bytes"] == 8
        D = f1.info()["depth"]
        for d in range(D, 1, -1):
            a, b = f0.skeletons(d), f1.skeletons(d)
            assert all(np.array_equal(x, y) for x, y in zip(a, b)), d
        X1 = _dev(torch, B0)
        f1.apply(X1)
        x0, x1 = X0.cpu().numpy(), X1.cpu().numpy()
        assert np.linalg.norm(x1 - x0) / np.linalg.norm(x0) <= 1e-12
        f2 = rss.Factorization(P, k, 1e-6, 64, precision="fp64")
        assert rss.factor_tuning() == tab
        for f in (f0, f1, f2):
            f.close()
    finally:
        rss.set_autotune(prev)
