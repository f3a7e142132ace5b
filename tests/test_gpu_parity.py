"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bars (stated per test):
* kernel entries: relative 2e-14 (FP64 evaluation on both sides);
* FP64 factorization: identical skeleton sets per box and depth (integer
  decisions, bit-exact), solution within 1e-10 relative of the oracle's;
* FP32 + refinement: relres <= 1e-10 measured by the oracle's FFT product,
  and the refined solution within 1e-10 of the oracle's refined solution;
* at the full workload sizes, where the oracle's factorization is too slow to
  rerun, the relative residual of the GPU solution is measured with the
  oracle's exact FFT product (a property that holds at any size).
"""
import numpy as np
import pytest
import scipy.linalg

from oracle import kernels as okern, matvec as omv, rss as orss
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
    """numpy (N x m) -> column-major complex128 CUDA tensor"""
    A = np.asarray(A, dtype=np.complex128)
    if A.ndim == 1:
        return torch.from_numpy(A.copy()).cuda()
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


def _host(T):
    return T.cpu().numpy()


def _rel(a, b):
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


@pytest.mark.parametrize("kind,kappa,q", [("laplace", 0.0, 0), ("helmholtz", 25.0, 0),
                                          ("helmholtz", 200.0, 0), ("degenerate", 0.0, 3)])
def test_kernel_entries(torch_cuda, kind, kappa, q):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    rng = np.random.default_rng(5)
    P = rng.random((700, 2))
    k = W.Kernel(kind, kappa=kappa, weight=0.37, diag=1.25, q=q or 2)
    I = rng.integers(0, 700, 300).astype(np.int32)
    J = rng.integers(0, 700, 310).astype(np.int32)
    I[:5] = J[:5]  # a few diagonal entries
    got = _host(rss.kernel_block(k, torch.from_numpy(P).cuda(), torch.from_numpy(I).cuda(),
                                 torch.from_numpy(J).cuda()))
    ref = okern.entries(k, P, I, J)
    scale = np.abs(ref).max()
    # both sides form the same FP64 argument x = kappa r (correctly rounded
    # square root); the bar's x-growing term is the phase error of SciPy's
    # hankel1 at large x, not the device's (test_h0_large_argument pins the
    # device against 30-digit values at the same x without it)
    x = kappa * np.hypot(P[I, 0][:, None] - P[J, 0][None, :], P[I, 1][:, None] - P[J, 1][None, :])
    bar = (2e-14 + 2.5e-16 * x) * np.abs(ref) + 1e-16 * scale
    ratio = np.max(np.abs(got - ref) / bar)
    assert ratio <= 1.0, ratio


def test_h0_large_argument(torch_cuda):
    """Device H0^(1)(x) against a 30-digit evaluation (mpmath) at the same FP64
    argument, x from 0.01 to ~280: points (0, 0) and (a, 0), so r = a exactly
    and x = fl(kappa a) on both sides; relative error of the complex value
    <= 1e-14 everywhere, including the far range of Hankel's expansion."""
    import mpmath
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    kappa = 200.0
    a = np.concatenate([np.geomspace(5e-5, 1.4, 300), np.linspace(0.3, 1.4, 200)])
    P = np.zeros((a.size + 1, 2))
    P[1:, 0] = a
    k = W.Kernel("helmholtz", kappa=kappa, weight=4.0, diag=1.0)   # w/4 = 1: entries are i H0
    I = np.zeros(1, np.int32)
    J = np.arange(1, a.size + 1, dtype=np.int32)
    got = _host(rss.kernel_block(k, torch.from_numpy(P).cuda(), torch.from_numpy(I).cuda(),
                                 torch.from_numpy(J).cuda()))[0]
    mpmath.mp.dps = 30
    worst = 0.0
    for j, aj in enumerate(a):
        x = kappa * float(np.sqrt(aj * aj))
        h = mpmath.hankel1(0, mpmath.mpf(x))
        ref = complex(1j * complex(h))
        worst = max(worst, abs(got[j] - ref) / abs(ref))
    print(f"H0 worst relative error {worst:.2e} up to x = {kappa * a.max():.0f}", flush=True)
    assert worst <= 1e-14


def test_residual_matches_fft(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 40
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 30.0)
    X = W.rhs(n * n, 5, 3)
    B = W.rhs(n * n, 5, 4)
    R = _host(rss.residual(k, torch.from_numpy(P).cuda(), _dev(torch, X), _dev(torch, B)))
    ref = B - omv.fft_matvec(k, n, X)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


CASES = [
    ("laplace", 0.0, 64, 64, 1e-6),      # Laplace N = 64^2, leaf 64 (the small workload)
    ("helmholtz", 25.0, 32, 16, 1e-6),
    ("helmholtz", 50.0, 48, 36, 1e-6),   # ragged: 36-point leaves
    ("laplace", 0.0, 48, 9, 1e-6),       # three compressed depths
    ("helmholtz", 40.0, 40, 25, 1e-9),
]


@pytest.mark.parametrize("kind,kappa,n,leaf,tol", CASES)
def test_fp64_factorization_parity(torch_cuda, kind, kappa, n, leaf, tol):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    P = W.grid_points(n)
    k = W.grid_kernel(kind, n, kappa)
    print(f"case {kind} kappa={kappa} n={n} leaf={leaf} tol={tol}", flush=True)
    Fo = orss.factor(P, k, tol, leaf)
    F = rss.Factorization(P, k, tol, leaf, precision="fp64")
    info = F.info()
    assert info["depth"] == Fo.tree.D
    for d in range(Fo.tree.D, 1, -1):
        got = F.skeletons(d)
        for b in range(4 ** d):
            if (d, b) in Fo.skeletons:
                assert np.array_equal(got[b], Fo.skeletons[(d, b)]), (d, b)
    B = W.rhs(n * n, 3, 7)
    Bd = _dev(torch, B)
    F.apply(Bd)
    x = _host(Bd)
    xo = orss.solve(Fo, B)
    assert _rel(x, xo) < 1e-10
    assert omv.relres(omv.fft_matvec(k, n, x), B) < max(10 * tol, 1e-9)
    F.close()


def test_degenerate_kernel_exact(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.Kernel("degenerate", weight=1.0 / n ** 2, diag=1.0, q=2)
    F = rss.Factorization(P, k, 1e-6, leaf)
    info = F.info()
    assert max(info["rank_sum"][d] / max(1, info["box_count"][d]) for d in range(2, info["depth"] + 1)) <= 6
    B = W.rhs(n * n, 2, 1)
    Bd = _dev(torch, B)
    F.apply(Bd)
    xd = scipy.linalg.solve(okern.dense_matrix(k, P), B)
    assert _rel(_host(Bd), xd) < 1e-12


@pytest.mark.parametrize("tol", [1e-15, 1.0])
def test_rank_edges(torch_cuda, tol):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 16, 4
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 20.0)
    Fo = orss.factor(P, k, tol, leaf)
    F = rss.Factorization(P, k, tol, leaf)
    assert F.info()["n_root"] == Fo.root_idx.size
    B = W.rhs(n * n, 1, 2)
    Bd = _dev(torch, B)
    F.apply(Bd)
    assert _rel(_host(Bd), orss.solve(Fo, B)) < 1e-10


def test_shallow_tree_dense(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 12
    P = W.grid_points(n)
    k = W.grid_kernel("laplace", n)
    F = rss.Factorization(P, k, 1e-6, 64)
    assert F.info()["depth"] == 1 and F.info()["n_root"] == n * n
    B = W.rhs(n * n, 2, 3)
    Bd = _dev(torch, B)
    F.apply(Bd)
    assert _rel(_host(Bd), scipy.linalg.solve(okern.dense_matrix(k, P), B)) < 1e-13


def test_scattered_points_empty_boxes(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    rng = np.random.default_rng(9)
    P = np.vstack([0.05 + 0.3 * rng.random((300, 2)), 0.6 + 0.35 * rng.random((200, 2))])
    k = W.Kernel("helmholtz", kappa=10.0, weight=1.0 / 500, diag=1.0)
    Fo = orss.factor(P, k, 1e-8, 12)
    F = rss.Factorization(P, k, 1e-8, 12)
    for d in range(Fo.tree.D, 1, -1):
        got = F.skeletons(d)
        for (dd, b), s in Fo.skeletons.items():
            if dd == d:
                assert np.array_equal(got[b], s)
    B = W.rhs(500, 2, 4)
    Bd = _dev(torch, B)
    F.apply(Bd)
    assert _rel(_host(Bd), orss.solve(Fo, B)) < 1e-10


def test_large_boxes_tight_tolerance(torch_cuda):
    """Boxes of more than 255 active points (Helmholtz kappa=25 at tol 1e-12):
    the sparsification then reads T from the factor record rather than LDS.
    One application of the FP64 factors leaves relres near the tolerance."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, kappa, tol = 256, 25.0, 1e-12
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, kappa)
    print(f"case helmholtz kappa={kappa} n={n} tol={tol}", flush=True)
    F = rss.Factorization(P, k, tol, 64, precision="fp64")
    depth = F.info()["depth"]
    # active points of a box at depth d - 1: its four children's skeletons
    nbig = 0
    for d in range(depth, 2, -1):
        nb = 2 ** d
        act = {}
        for b, s in F.skeletons(d).items():
            par = (b // nb // 2) * (nb // 2) + (b % nb) // 2
            act[par] = act.get(par, 0) + len(s)
        nbig = max([nbig] + list(act.values()))
    print(f"largest box: {nbig} active points", flush=True)
    assert nbig > 255
    B = W.rhs(n * n, 2, 5)
    Bd = _dev(torch, B)
    F.apply(Bd)
    assert omv.relres(omv.fft_matvec(k, n, _host(Bd)), B) < 1e-9


def test_multi_rhs_columns(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 35.0)
    F = rss.Factorization(P, k, 1e-6, leaf)
    B = W.rhs(n * n, 12, 6)
    Bd = _dev(torch, B)
    F.apply(Bd)
    X = _host(Bd)
    for j in (0, 5, 11):
        bj = _dev(torch, B[:, j])
        F.apply(bj)
        assert np.abs(_host(bj) - X[:, j]).max() <= 1e-14 * np.abs(X).max()


def test_fp32_refinement_matches_oracle(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf, tol = 48, 36, 1e-6
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 40.0)
    B = W.rhs(n * n, 4, 2)
    F = rss.Factorization(P, k, tol, leaf, precision="fp32")
    Bd = _dev(torch, B)
    rc = F.solve(Bd)
    x = _host(Bd)
    info = F.info()
    assert rc == 0 and info["last_relres"] <= 1e-10
    assert omv.relres(omv.fft_matvec(k, n, x), B) <= 1e-10
    Fo = orss.factor(P, k, tol, leaf)
    xo, hist = omv.refine(Fo, lambda v: omv.fft_matvec(k, n, v), B, tol=1e-13)
    assert _rel(x, xo) <= 1e-10


def test_fp32_factor_accuracy(torch_cuda):
    """The complex64 form's factors: one application leaves relres <= 2e-4 on
    Helmholtz kappa=50, n=96 (leaf 64), and refinement reaches 1e-10 within 3
    steps (the redundant-block and root inverses are formed in FP64)."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 96, 64
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 50.0)
    B = W.rhs(n * n, 4, 0)
    F = rss.Factorization(P, k, 1e-6, leaf, precision="fp32", n_proxy=128)
    Bd = _dev(torch, B)
    F.apply(Bd)
    rr = omv.relres(omv.fft_matvec(k, n, _host(Bd)), B)
    print(f"single application relres {rr:.2e}", flush=True)
    assert rr <= 2e-4
    Bd = _dev(torch, B)
    assert F.solve(Bd) == 0
    info = F.info()
    assert info["last_relres"] <= 1e-10 and info["last_iters"] <= 3, info["last_iters"]


def test_residual_column_chunks(torch_cuda):
    """nrhs = 21 runs as column chunks of 16, 4 and 1; every column equals the
    FFT product to 1e-13."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n = 24
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 20.0)
    X = W.rhs(n * n, 21, 5)
    B = W.rhs(n * n, 21, 6)
    R = _host(rss.residual(k, torch.from_numpy(P).cuda(), _dev(torch, X), _dev(torch, B)))
    ref = B - omv.fft_matvec(k, n, X)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


def test_fp64_refinement(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.grid_kernel("laplace", n)
    F = rss.Factorization(P, k, 1e-4, leaf, precision="fp64", max_refine=8, refine_tol=1e-12)
    B = W.rhs(n * n, 2, 9)
    Bd = _dev(torch, B)
    assert F.solve(Bd) == 0
    assert omv.relres(omv.fft_matvec(k, n, _host(Bd)), B) <= 1e-12
    assert F.info()["last_iters"] >= 1


def test_nan_right_hand_side_never_converges(torch_cuda):
    """A NaN in one column makes the refinement's relres NaN: the solve runs
    to max_refine and reports RSS_ENOCONV instead of convergence."""
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    n, leaf = 32, 16
    P = W.grid_points(n)
    k = W.grid_kernel("helmholtz", n, 20.0)
    F = rss.Factorization(P, k, 1e-6, leaf, precision="fp32", max_refine=2)
    B = W.rhs(n * n, 3, 4)
    B[5, 1] = np.nan
    Bd = _dev(torch, B)
    assert F.solve(Bd) == rss.RSS_ENOCONV
    info = F.info()
    assert np.isnan(info["last_relres"]) and info["last_iters"] == 2
    F.close()


def test_invalid_arguments(torch_cuda):
    from paper_2310_15458_amd import rss
    P = W.grid_points(8)
    with pytest.raises(rss.RSSError) as e:
        rss.Factorization(P, W.grid_kernel("laplace", 8), -1.0, 16)
    assert e.value.code == rss.RSS_EINVAL
    with pytest.raises(rss.RSSError) as e:
        rss.Factorization(P, W.Kernel("helmholtz", kappa=0.0), 1e-6, 16)
    assert e.value.code == rss.RSS_EINVAL
    Pn = P.copy()
    Pn[3, 0] = np.nan
    with pytest.raises(rss.RSSError):
        rss.Factorization(Pn, W.grid_kernel("laplace", 8), 1e-6, 16)


@pytest.mark.parametrize("name", ["helmholtz-k25-n256"])
def test_full_size_fp64_relres(torch_cuda, name):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    w = W.WORKLOADS[name]
    P = W.grid_points(w.n)
    F = rss.Factorization(P, w.kernel, w.tol, w.leaf, n_proxy=w.n_proxy)
    B = W.rhs(w.N, 1, w.seed)
    Bd = _dev(torch, B)
    F.apply(Bd)
    rr = omv.relres(omv.fft_matvec(w.kernel, w.n, _host(Bd)), B)
    print(f"{name}: FP64 relres {rr:.3e}, info {F.info()['t_factor_ms']:.1f} ms", flush=True)
    assert rr < 1e-8


def test_full_size_fp32_refined(torch_cuda):
    torch = torch_cuda
    from paper_2310_15458_amd import rss
    w = W.helmholtz_512()
    P = W.grid_points(w.n)
    F = rss.Factorization(P, w.kernel, w.tol, w.leaf, precision="fp32", n_proxy=w.n_proxy)
    B = W.rhs(w.N, 2, w.seed)
    Bd = _dev(torch, B)
    rc = F.solve(Bd)
    info = F.info()
    rr = omv.relres(omv.fft_matvec(w.kernel, w.n, _host(Bd)), B)
    print(f"{w.name}: FP32+refine relres {rr:.3e} (library {info['last_relres']:.3e}, "
          f"{info['last_iters']} steps)", flush=True)
    assert rc == 0 and rr <= 1e-10


_HOUSEHOLDER_CHILD = r"""
import json, sys
import numpy as np
sys.path.insert(0, sys.argv[1])
from oracle import rss as orss
from paper_2310_15458_amd import rss, workloads as W
import torch
rss.load()
n, leaf = 48, 9
P = W.grid_points(n)
k = W.grid_kernel("laplace", n)
Fo = orss.factor(P, k, 1e-6, leaf)
F = rss.Factorization(P, k, 1e-6, leaf)
bad = 0
for d in range(Fo.tree.D, 1, -1):
    got = F.skeletons(d)
    for (dd, b), sk in Fo.skeletons.items():
        if dd == d and not np.array_equal(got[b], sk):
            bad += 1
B = W.rhs(n * n, 1, 7)
Bd = torch.from_numpy(B.T.copy()).cuda().t()
F.apply(Bd)
x = Bd.cpu().numpy()
xo = orss.solve(Fo, B)
print(json.dumps({"bad": bad, "err": float(np.linalg.norm(x - xo) / np.linalg.norm(xo)),
                  "retries": F.info()["id_retries"]}))
"""


@pytest.mark.parametrize("spin", [None, "1"])
def test_householder_id_and_forced_barrier_timeout(torch_cuda, spin):
    """Boxes above the Gram path's limit take column-pivoted Householder QR,
    with several workgroups per box in phases with few boxes.  RSS_GRAM_NMAX=0
    sends every box there; RSS_MG_SPIN_LIMIT=1 makes the multi-workgroup
    barriers give up at once (forced from the host: every kernel still ends),
    and the factorization must be redone with the single-workgroup QR and
    still give the oracle's skeletons and solution."""
    import json
    import os
    import subprocess
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    env = dict(os.environ, RSS_GRAM_NMAX="0")
    if spin:
        env["RSS_MG_SPIN_LIMIT"] = spin
    print(f"child: Householder ID, spin limit {spin}", flush=True)
    res = subprocess.run([sys.executable, "-c", _HOUSEHOLDER_CHILD, root], env=env, capture_output=True,
                         text=True, timeout=240)
    assert res.returncode == 0, res.stderr[-3000:]
    out = json.loads(res.stdout.strip().splitlines()[-1])
    print(out, flush=True)
    assert out["bad"] == 0 and out["err"] < 1e-10
    assert out["retries"] == (1 if spin else 0)


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
def test_zero_matrix_is_singular(torch_cuda, precision):
    """A zero matrix (weight 0, diagonal 0): the ID keeps no skeletons, every
    redundant block X_RR is exactly zero, and the inverse's pivot search
    reports it: the factorization fails with RSS_ESINGULAR instead of
    returning factors."""
    from paper_2310_15458_amd import rss
    n = 32
    P = W.grid_points(n)
    k = W.Kernel("helmholtz", kappa=10.0, weight=0.0, diag=0.0)
    print(f"case zero matrix n={n} {precision}", flush=True)
    with pytest.raises(rss.RSSError) as e:
        rss.Factorization(P, k, 1e-6, 16, precision=precision)
    assert e.value.code == rss.RSS_ESINGULAR
