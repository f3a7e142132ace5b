"""The allocation-free residual (rss_residual_static) against rss_residual:
same inputs, identical results (same kernels; the partial sums of its source
slices fit the static scratch at these sizes, so the summation order is the
same), on two calls in a row, the second with fewer points, and with more
than 16 right-hand sides (several column chunks)."""
import numpy as np
import pytest

from paper_2310_15458_amd import workloads as W

pytestmark = pytest.mark.gpu


def _dev(torch, A):
    return torch.from_numpy(np.ascontiguousarray(np.asarray(A, np.complex128).T)).cuda().t()


@pytest.mark.parametrize("kind,kappa", [("helmholtz", 30.0), ("laplace", 0.0)])
def test_static_residual_matches_allocating_one(kind, kappa):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2310_15458_amd import rss
    rss.load()
    for n, nrhs, seed in ((56, 19, 3), (24, 3, 4)):
        print(f"static residual {kind} n={n} nrhs={nrhs}", flush=True)
        P = torch.from_numpy(W.grid_points(n)).cuda()
        k = W.grid_kernel(kind, n, kappa)
        X = _dev(torch, W.rhs(n * n, nrhs, seed))
        B = _dev(torch, W.rhs(n * n, nrhs, seed + 10))
        ref = rss.residual(k, P, X, B).cpu().numpy()
        got = rss.residual_static(k, P, X, B).cpu().numpy()
        assert got.shape == ref.shape
        assert np.array_equal(got, ref), np.abs(got - ref).max()
        assert np.all(np.isfinite(got))
